"""Pins for the CPU oracle: checks against what the paper and the mathematics fix,
never against the oracle's own formulas retyped.

Each test names the property it pins and the passage it comes from.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ---------------------------------------------------------------------------------------
# primitives: prediction (Sec. 2.3, 4th-order central interpolation) and FD (Sec. 3)
# ---------------------------------------------------------------------------------------

def test_prediction_exact_on_cubics_and_fourth_order():
    """The 4-point central midpoint rule reproduces every cubic exactly and misses
    x^4 by -9 (coarse spacing 2): the interpolation is 4th order (Sec. 3)."""
    rng = np.random.default_rng(0)
    for _ in range(200):
        a = rng.integers(-50, 50, 4).astype(float)
        x0 = float(rng.integers(-20, 20))
        f = lambda x: ((a[3] * x + a[2]) * x + a[1]) * x + a[0]
        assert oracle.p4(f(x0 - 3), f(x0 - 1), f(x0 + 1), f(x0 + 3)) == f(x0)
    assert oracle.p4(81.0, 1.0, 1.0, 81.0) - 0.0 == -9.0


def test_fd_exact_up_to_degree_four():
    """(8(u1-u-1) - (u2-u-2))/(12h) is exact for polynomials of degree <= 4 (4th-order central FD)."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        a = rng.integers(-9, 9, 5).astype(float)
        x0 = float(rng.integers(-10, 10))
        f = lambda x: (((a[4] * x + a[3]) * x + a[2]) * x + a[1]) * x + a[0]
        df = (((4 * a[4] * x0 + 3 * a[3]) * x0 + 2 * a[2]) * x0 + a[1])
        got = oracle.d4(f(x0 - 2), f(x0 - 1), f(x0 + 1), f(x0 + 2), 1.0 / 12.0)
        assert abs(got - df) <= 1e-9 * max(1.0, abs(df))
    # degree 5 is not reproduced
    assert oracle.d4(-32.0, -1.0, 1.0, 32.0, 1.0 / 12.0) != 0.0


def _uniform(cfg, level):
    o = oracle.Oracle(cfg)
    lv, co = W.uniform_forest(cfg, level)
    o.init_forest(lv, co)
    return o


def test_fd_modified_wavenumber_on_block_forest():
    """On a uniform periodic block forest, the RHS of constant advection applied to
    sin(2 pi k x) equals -c kappa cos(2 pi k x), kappa = (8 sin(th) - sin(2 th))/(6h):
    ghost synchronisation across blocks and the periodic wrap add nothing."""
    cfg = W.C1(jmax=3).replace(phys=(1.0, 0.0, 0.0))
    o = _uniform(cfg, 3)
    lv, co = o.read_forest()
    k = 5
    fn = lambda x, y: np.sin(2 * np.pi * k * x)
    o.load_blocks(W.sample(cfg, lv, co, fn=fn))
    r = o.rhs()
    n = (2 ** 3) * (cfg.bs - 1)
    h = 1.0 / n
    th = 2 * np.pi * k * h
    kappa = (8 * np.sin(th) - np.sin(2 * th)) / (6 * h)
    x, y = W.node_coords(cfg, lv, co)
    want = -kappa * np.cos(2 * np.pi * k * x)
    assert np.max(np.abs(r[:, 0, :] - want)) < 1e-11 * kappa


def test_rk4_amplification_factor():
    """Classic RK4 on the semi-discrete mode exp(i 2pi(kx+my)) multiplies it by
    G(z) = 1+z+z^2/2+z^3/6+z^4/24 per step, z = -i dt (cx kx_mod + cy ky_mod)."""
    cfg = W.C1(jmax=2)
    o = _uniform(cfg, 2)
    lv, co = o.read_forest()
    kx, ky = 2, 3
    fn = lambda x, y: np.sin(2 * np.pi * (kx * x + ky * y))
    o.load_blocks(W.sample(cfg, lv, co, fn=fn))
    n = 4 * (cfg.bs - 1)
    h = 1.0 / n
    kap = lambda k: (8 * np.sin(2 * np.pi * k * h) - np.sin(4 * np.pi * k * h)) / (6 * h)
    dt = 0.5 * h
    z = -1j * dt * (1.0 * kap(kx) + 0.5 * kap(ky))
    G = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    nsteps = 20
    for s in range(nsteps):
        o.rk4(s * dt, dt)
    x, y = W.node_coords(cfg, lv, co)
    want = np.imag(G ** nsteps * np.exp(2j * np.pi * (kx * x + ky * y)))
    got = o.read_blocks()[:, 0, :]
    assert np.max(np.abs(got - want)) < 1e-12


# ---------------------------------------------------------------------------------------
# ghost synchronisation across levels (Sec. 2.2 conditional ghost nodes, Sec. 2.3 prediction)
# ---------------------------------------------------------------------------------------

def _two_level_forest():
    # level-2 blocks everywhere except the block (1,1) refined into four level-3 blocks
    keys = [(2, x, y) for x in range(4) for y in range(4) if (x, y) != (1, 1)]
    keys += [(3, 2 + bx, 2 + by) for bx in range(2) for by in range(2)]
    keys.sort()
    lv = np.array([k[0] for k in keys], dtype=np.int8)
    co = np.array([k[1:] for k in keys], dtype=np.int32)
    return lv, co


def test_ghosts_exact_for_cubic_data_across_levels():
    """Data that is a tensor cubic in the middle of the domain is reproduced exactly
    (to rounding) in every ghost node of blocks next to a level jump, whether the
    ghost is copied, injected from a finer block or predicted from a coarser one."""
    cfg = W.C1(jmax=3)
    o = oracle.Oracle(cfg)
    lv, co = _two_level_forest()
    o.init_forest(lv, co)
    lv, co = o.read_forest()
    f = lambda x, y: (1 + x * (0.3 - x * (2 - 1.5 * x))) * (0.7 + y * (1 - y * (0.4 + y)))
    o.load_blocks(W.sample(cfg, lv, co, fn=f))
    checked = 0
    for bi in range(len(lv)):
        l = int(lv[bi])
        cx, cy = co[bi]
        for H in (2, 4):
            T = o.tile(bi, H)[0]
            n = (2 ** l) * (cfg.bs - 1)
            g = np.arange(-H, cfg.bs + H)
            xs = (cx * (cfg.bs - 1) + g) / n
            ys = (cy * (cfg.bs - 1) + g) / n
            # only where no interpolation stencil can reach the periodic wrap
            mx = (xs > 0.1) & (xs < 0.9)
            my = (ys > 0.1) & (ys < 0.9)
            X, Y = np.meshgrid(xs, ys)
            want = f(X, Y)
            m = np.outer(my, mx)
            if m.any():
                assert np.max(np.abs(T[m] - want[m])) < 1e-13, (bi, H)
                checked += 1
    assert checked > 10


def test_interface_ghost_error_is_fourth_order():
    """For smooth non-polynomial data the predicted ghosts converge at order 4."""
    cfg = W.C1(jmax=6)
    errs = []
    for base in (3, 4):
        keys = [(base, x, y) for x in range(2 ** base) for y in range(2 ** base)
                if not (x == 2 ** (base - 1) and y == 2 ** (base - 1))]
        keys += [(base + 1, 2 ** base + bx, 2 ** base + by) for bx in range(2) for by in range(2)]
        lv = np.array([k[0] for k in keys], dtype=np.int8)
        co = np.array([k[1:] for k in keys], dtype=np.int32)
        o = oracle.Oracle(cfg.replace(jmax=base + 1))
        o.init_forest(lv, co)
        lv, co = o.read_forest()
        # refined patch sits at (0.5, 0.5), where |f| and its 4th derivatives are maximal
        f = lambda x, y: np.cos(2 * np.pi * x) * np.cos(2 * np.pi * y)
        o.load_blocks(W.sample(o.cfg, lv, co, fn=f))
        e = 0.0
        for bi in np.nonzero(lv == base + 1)[0]:
            T = o.tile(int(bi), 2)[0]
            n = (2 ** (base + 1)) * (cfg.bs - 1)
            g = np.arange(-2, cfg.bs + 2)
            X, Y = np.meshgrid((co[bi][0] * (cfg.bs - 1) + g) / n, (co[bi][1] * (cfg.bs - 1) + g) / n)
            e = max(e, np.max(np.abs(T - f(X, Y))))
        errs.append(e)
    order = math.log2(errs[0] / errs[1])
    assert 3.6 < order < 4.6, (errs, order)


def test_restriction_of_prediction_is_identity():
    """R(P(B)) = B bitwise: refining a forest and coarsening every family returns the
    original values (nested lattices, injection restriction; Sec. 2.3)."""
    cfg = W.C1(jmax=4)
    o = oracle.Oracle(cfg)
    lv, co = _two_level_forest()
    o.init_forest(lv, co)
    lv, co = o.read_forest()
    o.load_blocks(W.sample(cfg, lv, co))
    before = o.read_blocks()
    o.refine_all()
    assert o.num_blocks() == 4 * len(lv)
    o.coarsen(np.full(o.num_blocks(), -1, dtype=np.int8))
    lv2, co2 = o.read_forest()
    assert np.array_equal(lv, lv2) and np.array_equal(co, co2)
    assert np.array_equal(o.read_blocks().view(np.uint64), before.view(np.uint64))


# ---------------------------------------------------------------------------------------
# details and flags (Sec. 2.3, detail equation and flag rule)
# ---------------------------------------------------------------------------------------

def test_details_closed_form_for_sinusoid_and_exact_flag_flip():
    """For sin(kx+phi), d = f (1 - 9/8 cos(kh) + 1/8 cos(3kh)) at odd nodes; for a
    separable product d = f (1 - Wx Wy) at (odd, odd).  The flag flips exactly when eps
    crosses the block maximum (strict '<')."""
    cfg = W.C2(jmax=3)
    o = _uniform(cfg, 3)
    lv, co = o.read_forest()
    kx, ky = 3, 2
    f = lambda x, y: np.sin(2 * np.pi * kx * x + 0.3) * np.sin(2 * np.pi * ky * y + 1.1)
    o.load_blocks(W.sample(cfg, lv, co, fn=f))
    fl, md = o.mr_pass()
    n = 8 * (cfg.bs - 1)
    h = 1.0 / n
    Wf = lambda k: 9 / 8 * np.cos(2 * np.pi * k * h) - 1 / 8 * np.cos(6 * np.pi * k * h)
    x, y = W.node_coords(cfg, lv, co)
    ix = np.rint(x * n).astype(int) % 2
    iy = np.rint(y * n).astype(int) % 2
    fx = np.where(ix == 1, Wf(kx), 1.0)
    fy = np.where(iy == 1, Wf(ky), 1.0)
    d = f(x, y) * (1 - fx * fy)
    want = np.max(np.abs(d), axis=1)
    assert np.allclose(md[:, 0], want, rtol=1e-9, atol=0)
    # exact flip around the block maximum
    m = float(md[5, 0])
    for eps, flag in ((m * (1 + 1e-12), -1), (m, 0), (m * (1 - 1e-12), 0)):
        o2 = _uniform(cfg.replace(eps=eps), 3)
        o2.load_blocks(W.sample(cfg, lv, co, fn=f))
        fl2, md2 = o2.mr_pass()
        assert md2[5, 0] == m
        assert fl2[5] == flag


def test_details_closed_form_in_3d_for_every_odd_parity_class():
    """3D (Sec. 2.3, detail equation; prediction is the tensor product of the 1D midpoint
    rule): for f = sin(kx x+a) sin(ky y+b) sin(kz z+c) the detail at a node whose odd axes
    form the set A is f (1 - prod_{a in A} W(k_a)), W(k) = 9/8 cos(kh) - 1/8 cos(3kh), and 0
    at all-even nodes.  Checked node by node in each of the seven odd classes, with a
    different wavenumber per axis so that every axis' stencil shows; then the flag flips
    exactly when eps crosses the block maximum (strict '<')."""
    cfg = W.C4(jmax=3, eps=1e-3)
    o = _uniform(cfg, 2)
    lv, co = o.read_forest()
    k = (3, 2, 5)
    ph = (0.3, 1.1, -0.7)
    f = lambda x, y, z: (np.sin(2 * np.pi * k[0] * x + ph[0]) * np.sin(2 * np.pi * k[1] * y + ph[1])
                         * np.sin(2 * np.pi * k[2] * z + ph[2]))
    o.load_blocks(W.sample(cfg, lv, co, fn=f))
    fl, md = o.mr_pass()
    d = o.details()[:, 0]
    n = 4 * (cfg.bs - 1)
    h = 1.0 / n
    Wk = [9 / 8 * np.cos(2 * np.pi * kk * h) - 1 / 8 * np.cos(6 * np.pi * kk * h) for kk in k]
    xs = W.node_coords(cfg, lv, co)
    odd = [np.rint(xa * n).astype(int) % 2 for xa in xs]
    prod = np.ones_like(xs[0])
    for a in range(3):
        prod = prod * np.where(odd[a] == 1, Wk[a], 1.0)
    want = f(*xs) * (1 - prod)
    cls = odd[0] + 2 * odd[1] + 4 * odd[2]
    assert np.all(d[cls == 0] == 0.0)
    for c in range(1, 8):
        sel = cls == c
        assert np.max(np.abs(want[sel])) > 1e-4, c       # every class carries a visible detail
        assert np.max(np.abs(d[sel] - want[sel])) < 1e-13, c
    assert np.array_equal(md[:, 0], np.max(np.abs(d), axis=1))
    # exact flip around one block's maximum
    b = 37
    m = float(md[b, 0])
    for eps, flag in ((m * (1 + 1e-12), -1), (m, 0), (m * (1 - 1e-12), 0)):
        o2 = _uniform(cfg.replace(eps=eps), 2)
        o2.load_blocks(W.sample(cfg, lv, co, fn=f))
        fl2, md2 = o2.mr_pass()
        assert md2[b, 0] == m
        assert fl2[b] == flag


def test_level_one_never_coarsens_and_eps_limits():
    cfg = W.C1(jmax=3, eps=1e300)
    o = _uniform(cfg, 1)
    lv, co = o.read_forest()
    o.load_blocks(W.sample(cfg, lv, co))
    fl, _ = o.mr_pass()
    assert np.all(fl == 0)           # level 1 has no coarser level
    # eps = +inf: a uniform level-3 forest collapses to level 1 within jmax-1 passes
    o = _uniform(cfg, 3)
    lv, co = o.read_forest()
    o.load_blocks(W.sample(cfg, lv, co))
    passes = o.adapt()
    assert passes <= cfg.jmax
    assert np.all(o.read_forest()[0] == 1)
    # eps = 0: details are never < 0, nothing coarsens
    o = _uniform(cfg.replace(eps=0.0), 3)
    o.load_blocks(W.sample(cfg, lv, co))
    assert o.adapt() == 1
    assert o.num_blocks() == 64


# ---------------------------------------------------------------------------------------
# completeness + gradedness, checked by brute force (Sec. 2.3 last paragraph, Sec. 2.2 graded grid)
# ---------------------------------------------------------------------------------------

def _touch(a, b, dim):
    """Closed regions of leaves a=(l, c...) and b touch (periodic unit domain)."""
    L = max(a[0], b[0])
    n = 2 ** L
    for ax in range(dim):
        a0 = a[1 + ax] << (L - a[0]); a1 = (a[1 + ax] + 1) << (L - a[0])
        b0 = b[1 + ax] << (L - b[0]); b1 = (b[1 + ax] + 1) << (L - b[0])
        if not any(b0 + s <= a1 and a0 <= b1 + s for s in (-n, 0, n)):
            return False
    return True


def _brute_force(leaves, flags, dim):
    """Largest set of families that can coarsen together, by enumerating subsets."""
    fl = dict(zip(leaves, flags))
    par = lambda k: (k[0] - 1,) + tuple(c >> 1 for c in k[1:])
    kids = lambda p: [(p[0] + 1,) + tuple(2 * p[1 + a] + ((b >> a) & 1) for a in range(dim))
                      for b in range(2 ** dim)]
    cands = sorted({par(k) for k in leaves if k[0] >= 2 and fl[k] == -1
                    and all(fl.get(c) == -1 for c in kids(par(k)))})
    need = {}
    for p in cands:
        req = set()
        for m in kids(p):
            for nb in leaves:
                if nb[0] == m[0] + 1 and _touch(m, nb, dim):
                    req.add(par(nb))
        need[p] = req
    best = set()
    for r in range(len(cands) + 1):
        for S in itertools.combinations(cands, r):
            S = set(S)
            if all(need[p] <= S for p in S):
                best |= S
    return best, len(cands)


@pytest.mark.parametrize("dim,jmax,seed", [(2, 3, s) for s in range(12)] + [(3, 3, s) for s in range(4)])
def test_coarsening_fixed_point_matches_brute_force(dim, jmax, seed):
    lv, co = W.random_graded_forest(dim, jmax, seed, p_refine=0.55)
    leaves = [(int(l),) + tuple(int(c) for c in cc) for l, cc in zip(lv, co)]
    cfg = (W.C1(jmax=jmax) if dim == 2 else W.C4(jmax=jmax))
    o = oracle.Oracle(cfg)
    o.init_forest(lv, co)
    lv2, co2 = o.read_forest()
    leaves = [(int(l),) + tuple(int(c) for c in cc) for l, cc in zip(lv2, co2)]
    rng = np.random.default_rng(100 + seed)
    tried = 0
    for trial in range(6):
        flags = np.where(rng.random(len(leaves)) < 0.85, -1, 0).astype(np.int8)
        flags[lv2 == 1] = 0
        want, ncand = _brute_force(leaves, flags, dim)
        if ncand > 12:
            continue
        tried += 1
        assert o.coarsenable(flags) == want
    assert tried > 0


def test_forest_validation():
    cfg = W.C1(jmax=3)
    o = oracle.Oracle(cfg)
    lv, co = W.uniform_forest(cfg, 2)
    with pytest.raises(oracle.OracleError):
        o.init_forest(lv[1:], co[1:])                      # hole
    with pytest.raises(oracle.OracleError):
        o.init_forest(np.r_[lv, 1], np.r_[co, [[0, 0]]])   # overlap
    keys = [(1, 1, 0), (1, 0, 1), (1, 1, 1)] + [(2, 0, 1), (2, 1, 0), (2, 1, 1)] + \
           [(3, x, y) for x in range(2) for y in range(2)]
    with pytest.raises(oracle.OracleError):                 # level 1 next to level 3
        o.init_forest([k[0] for k in keys], [k[1:] for k in keys])


# ---------------------------------------------------------------------------------------
# whole MR loop (Sec. 2.1) reduces to the uniform solver at eps = 0; order 4 (Sec. 3, Fig. 4B)
# ---------------------------------------------------------------------------------------

def _uniform_solver(u, c, r, dt, nsteps):
    """Plain periodic-array FD4 + RK4 for constant advection on a uniform grid ([y, x])."""
    D = lambda v, ax: (8.0 * (np.roll(v, -1, ax) - np.roll(v, 1, ax)) - (np.roll(v, -2, ax) - np.roll(v, 2, ax))) * r
    N = lambda v: -(c[0] * D(v, 1) + c[1] * D(v, 0))
    h2, h6 = dt * 0.5, dt / 6.0
    for _ in range(nsteps):
        k1 = N(u)
        k2 = N(u + h2 * k1)
        k3 = N(u + h2 * k2)
        k4 = N(u + dt * k3)
        u = u + h6 * ((k1 + k4) + 2.0 * (k2 + k3))
    return u


def test_eps_zero_adaptive_run_equals_uniform_solver_bitwise():
    cfg = W.C1(jmax=3, eps=0.0)
    o = oracle.Oracle(cfg)
    o.init_grid()
    lv, co = o.read_forest()
    assert np.all(lv == cfg.jmax) and len(lv) == 4 ** cfg.jmax
    nsteps = 6
    for s in range(nsteps):
        o.step(s * cfg.dt, cfg.dt)
    lv, co = o.read_forest()
    assert np.all(lv == cfg.jmax)
    n = (2 ** cfg.jmax) * (cfg.bs - 1)
    g = np.arange(n) / n
    U0 = W.blob_field(cfg, [g, g])
    U = _uniform_solver(U0, cfg.phys, n / 12.0, cfg.dt, nsteps)
    got = o.read_blocks()[:, 0, :].reshape(len(lv), cfg.bs, cfg.bs)
    for b in range(len(lv)):
        ys = (co[b][1] * (cfg.bs - 1) + np.arange(cfg.bs)) % n
        xs = (co[b][0] * (cfg.bs - 1) + np.arange(cfg.bs)) % n
        want = U[np.ix_(ys, xs)]
        assert np.array_equal(got[b].view(np.uint64), want.view(np.uint64)), b


def _exact_translated(cfg, T, x, y):
    c = cfg.phys
    return W.blob_at(cfg, [np.mod(x - c[0] * T, 1.0), np.mod(y - c[1] * T, 1.0)])


@pytest.mark.slow
def test_exact_translation_error_converges_at_order_four():
    """Gaussian advected by c=(1, 0.5) on uniform forests: the max error against the
    exact periodic translation decays with order 4 (Sec. 3: 4th-order FD and RK4)."""
    errs = []
    T = 0.125
    for J in (2, 3, 4):
        cfg = W.C1(jmax=J).replace(blob_beta=2 * 0.1 ** 2)
        o = _uniform(cfg, J)
        lv, co = o.read_forest()
        o.load_blocks(W.sample(cfg, lv, co))
        nsteps = int(round(T / cfg.dt))
        for s in range(nsteps):
            o.rk4(s * cfg.dt, cfg.dt)
        x, y = W.node_coords(cfg, lv, co)
        errs.append(np.max(np.abs(o.read_blocks()[:, 0, :] - _exact_translated(cfg, T, x, y))))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-5
    assert 3.7 < orders[-1] < 4.5, (errs, orders)


def test_adaptive_error_tracks_eps_and_compression_goes_to_one():
    """Thresholding error grows with eps (Fig. 4A) and the block count approaches the
    uniform one as eps -> 0 (Fig. 4C)."""
    res = []
    for eps in (1e-2, 1e-4, 0.0):
        cfg = W.C1(jmax=3, eps=eps)
        o = oracle.Oracle(cfg)
        o.init_grid()
        T = 10 * cfg.dt
        for s in range(10):
            o.step(s * cfg.dt, cfg.dt)
        lv, co = o.read_forest()
        x, y = W.node_coords(cfg, lv, co)
        err = np.max(np.abs(o.read_blocks()[:, 0, :] - _exact_translated(cfg, T, x, y)))
        res.append((err, len(lv)))
    assert res[0][0] > res[1][0] >= res[2][0] * 0.999
    assert res[0][1] < res[1][1] <= res[2][1] == 4 ** 3


def test_redundant_nodes_agree_after_adaptive_steps():
    """Same-level neighbours hold identical values at shared nodes (Sec. 2.5): the
    oracle raises if its highest-level lookup ever finds two that differ."""
    cfg = W.C1(jmax=4)
    o = oracle.Oracle(cfg)
    o.init_grid()
    for s in range(8):
        o.step(s * cfg.dt, cfg.dt)
    assert len(np.unique(o.read_forest()[0])) >= 2
    o.read_blocks()


# ---------------------------------------------------------------------------------------
# Navier-Stokes right-hand side (formulation is a reading): free stream, mass
# ---------------------------------------------------------------------------------------

def test_ns_free_stream_is_steady():
    """A uniform state has zero right-hand side: exactly zero where no prediction is
    involved, and zero to rounding across a level jump (where P reproduces a constant
    only up to one rounding of 9(b+c))."""
    cfg = W.C3(jmax=3)
    fn = lambda x, y: (np.full_like(x, 1.3), np.full_like(x, 0.2), np.full_like(x, -0.1), np.full_like(x, 0.9))
    o = _uniform(cfg, 2)
    lv, co = o.read_forest()
    o.load_blocks(W.sample(cfg, lv, co, fn=fn))
    assert np.all(o.rhs() == 0.0)
    o = oracle.Oracle(cfg)
    lv, co = _two_level_forest()
    o.init_forest(lv, co)
    lv, co = o.read_forest()
    o.load_blocks(W.sample(cfg, lv, co, fn=fn))
    assert np.max(np.abs(o.rhs())) < 1e-11


def test_ns_mass_is_conserved_on_uniform_grid():
    cfg = W.C3(jmax=2)
    o = _uniform(cfg, 2)
    lv, co = o.read_forest()
    o.load_blocks(W.sample(cfg, lv, co))
    uniq = lambda d: d[:, 0, :].reshape(len(lv), cfg.bs, cfg.bs)[:, :-1, :-1].sum()
    m0 = uniq(o.read_blocks())
    for s in range(3):
        o.rk4(s * cfg.dt, cfg.dt)
    m1 = uniq(o.read_blocks())
    assert abs(m1 - m0) < 1e-12 * m0
    assert not np.allclose(o.read_blocks()[:, 2], W.sample(cfg, lv, co)[:, 2], atol=0, rtol=0)


# ---------------------------------------------------------------------------------------
# golden fixtures from the paper
# ---------------------------------------------------------------------------------------

def _golden(name):
    import os
    p = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = []
    for line in open(p):
        line = line.split("#")[0].strip()
        if line:
            rows.append(line.split())
    return rows


def test_fig2_example_grid_is_valid_and_level_is_treecode_length():
    rows = _golden("fig2_forest.txt")
    lv = np.array([int(r[0]) for r in rows], dtype=np.int8)
    co = np.array([[int(r[1]), int(r[2])] for r in rows], dtype=np.int32)
    assert len(lv) == 7 and np.sum(lv == 1) == 3 and np.sum(lv == 2) == 4
    for r in rows:
        l, cx, cy, code = int(r[0]), int(r[1]), int(r[2]), r[3]
        assert len(code) == l
        digits = [((cx >> (l - 1 - i)) & 1) + 2 * ((cy >> (l - 1 - i)) & 1) for i in range(l)]
        assert "".join(str(d) for d in digits) == code
    o = oracle.Oracle(W.C1(jmax=2))
    o.init_forest(lv, co)
    assert o.num_blocks() == 7


def test_swirl_reverses_to_the_initial_state():
    """The swirl velocity times cos(pi t/t_a) brings the blob back at t = t_a (Sec. 3);
    the paper's constants (centre (0.5, 0.75), beta = 0.01) are used, with a short t_a."""
    g = {r[0]: float(r[1]) for r in _golden("paper_constants.txt")}
    ta = 0.25
    cfg = W.C2(jmax=3, eps=1e-5).replace(bs=17, phys=(ta,), blob_beta=g["swirl_beta"],
                                         blob_centers=np.array([[g["swirl_center_x"], g["swirl_center_y"]]]))
    cfg = cfg.replace(dt=0.5 / ((2 ** cfg.jmax) * (cfg.bs - 1)))
    o = oracle.Oracle(cfg)
    o.init_grid()
    nsteps = int(round(ta / cfg.dt))
    mid = None
    for s in range(nsteps):
        o.step(s * cfg.dt, cfg.dt)
        if s + 1 == nsteps // 2:
            lv, co = o.read_forest()
            mid = np.max(np.abs(o.read_blocks()[:, 0] - W.sample(cfg, lv, co)[:, 0]))
    lv, co = o.read_forest()
    end = np.max(np.abs(o.read_blocks()[:, 0] - W.sample(cfg, lv, co)[:, 0]))
    assert mid > 0.3
    assert end < 0.02 * mid


def test_3d_fd_wavenumber_and_cubic_ghosts():
    """3D: the advection RHS of a plane wave along z matches the modified wavenumber,
    and tensor-cubic data is reproduced in ghosts next to a level jump."""
    cfg = W.C4(jmax=2).replace(phys=(0.0, 0.0, 1.0))
    o = _uniform(cfg, 2)
    lv, co = o.read_forest()
    k = 3
    o.load_blocks(W.sample(cfg, lv, co, fn=lambda x, y, z: np.sin(2 * np.pi * k * z)))
    n = 4 * (cfg.bs - 1)
    h = 1.0 / n
    kappa = (8 * np.sin(2 * np.pi * k * h) - np.sin(4 * np.pi * k * h)) / (6 * h)
    x, y, z = W.node_coords(cfg, lv, co)
    assert np.max(np.abs(o.rhs()[:, 0] + kappa * np.cos(2 * np.pi * k * z))) < 1e-11 * kappa
    # two-level 3D forest: block (1,1,1) of level 2 refined
    keys = [(2, x_, y_, z_) for x_ in range(4) for y_ in range(4) for z_ in range(4) if (x_, y_, z_) != (1, 1, 1)]
    keys += [(3, 2 + a, 2 + b, 2 + c) for a in range(2) for b in range(2) for c in range(2)]
    o = oracle.Oracle(cfg.replace(jmax=3))
    o.init_forest([q[0] for q in keys], [q[1:] for q in keys])
    lv, co = o.read_forest()
    f = lambda x, y, z: (1 + x * (0.3 - x)) * (0.7 + y * y * y) * (1 - z * (0.4 + z * z))
    o.load_blocks(W.sample(o.cfg, lv, co, fn=f))
    for bi in np.nonzero(lv == 3)[0][:2]:
        T = o.tile(int(bi), 2)[0]
        nn = 8 * (cfg.bs - 1)
        g = np.arange(-2, cfg.bs + 2)
        ax = [(co[bi][a] * (cfg.bs - 1) + g) / nn for a in range(3)]
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        assert np.max(np.abs(T - f(X, Y, Z))) < 1e-13


def test_finer_block_owns_redundant_nodes():
    """Sec. 2.5: at nodes shared across a level jump the finer block's value wins.
    Coarse blocks are loaded with f + 1, fine blocks with f; after synchronisation every
    node a coarse block shares with a fine block reads f, all its other nodes f + 1."""
    cfg = W.C1(jmax=3)
    o = oracle.Oracle(cfg)
    lv, co = _two_level_forest()
    o.init_forest(lv, co)
    lv, co = o.read_forest()
    f = lambda x, y: np.sin(2 * np.pi * x + 0.2) * np.cos(2 * np.pi * y)
    data = W.sample(cfg, lv, co, fn=f)
    data[lv == 2] += 1.0
    o.load_blocks(data)
    got = o.read_blocks()[:, 0]
    x, y = W.node_coords(cfg, lv, co)
    # fine region: [0.25, 0.5]^2 (level-2 block (1,1) refined)
    on_fine = (x >= 0.25) & (x <= 0.5) & (y >= 0.25) & (y <= 0.5)
    want = f(x, y) + np.where((lv[:, None] == 2) & ~on_fine, 1.0, 0.0)
    assert np.array_equal(got, want)
    assert np.any((lv[:, None] == 2) & on_fine)


def test_swirl_rhs_closed_form():
    """Swirl RHS -(u, v).grad(phi) with u = sin^2(pi x) sin(2 pi y), v = -sin^2(pi y) sin(2 pi x)
    (Sec. 3 velocity field, t_a factor = 1): for phi = sin(2 pi k x) + cos(2 pi m y) the FD
    derivatives are kappa(k) cos(2 pi k x) and -kappa(m) sin(2 pi m y)."""
    cfg = W.C2(jmax=2)
    o = _uniform(cfg, 2)
    lv, co = o.read_forest()
    k, m = 3, 2
    o.load_blocks(W.sample(cfg, lv, co, fn=lambda x, y: np.sin(2 * np.pi * k * x) + np.cos(2 * np.pi * m * y)))
    n = 4 * (cfg.bs - 1)
    h = 1.0 / n
    kap = lambda q: (8 * np.sin(2 * np.pi * q * h) - np.sin(4 * np.pi * q * h)) / (6 * h)
    x, y = W.node_coords(cfg, lv, co)
    u = np.sin(np.pi * x) ** 2 * np.sin(2 * np.pi * y)
    v = -np.sin(np.pi * y) ** 2 * np.sin(2 * np.pi * x)
    want = -(u * kap(k) * np.cos(2 * np.pi * k * x) - v * kap(m) * np.sin(2 * np.pi * m * y))
    assert np.max(np.abs(o.rhs()[:, 0] - want)) < 1e-10 * kap(k)


def _ns_rhs_uniform(fn, mu=1e-2):
    cfg = W.C3(jmax=2).replace(phys=(1.4, mu, 0.71))
    o = _uniform(cfg, 2)
    lv, co = o.read_forest()
    o.load_blocks(W.sample(cfg, lv, co, fn=fn))
    x, y = W.node_coords(cfg, lv, co)
    n = 4 * (cfg.bs - 1)
    h = 1.0 / n
    kap = lambda q: (8 * np.sin(2 * np.pi * q * h) - np.sin(4 * np.pi * q * h)) / (6 * h)
    return o.rhs(), x, y, kap, cfg


def test_ns_rhs_single_mode_closed_forms():
    """Each term of the Navier-Stokes RHS (formulation of our own, primitive variables)
    against its value for single Fourier modes, with D(D(sin)) = -kappa^2 sin:
    shear wave (tau_xy, viscous heating), pressure wave (grad p, heat conduction),
    longitudinal wave (convection, mass flux, gamma p div u, tau_xx with 4/3)."""
    g, mu, pr = 1.4, 1e-2, 0.71
    kc = mu * g / ((g - 1) * pr)
    A, p0, k = 0.01, 1.2, 3
    one = lambda x: np.ones_like(x)
    # shear wave u = A sin(2 pi k y)
    r, x, y, kap, cfg = _ns_rhs_uniform(lambda x, y: (one(x), A * np.sin(2 * np.pi * k * y), 0 * x, p0 * one(x)), mu)
    K = kap(k)
    s, c = np.sin(2 * np.pi * k * y), np.cos(2 * np.pi * k * y)
    tol = 1e-9
    assert np.max(np.abs(r[:, 0])) < tol
    assert np.max(np.abs(r[:, 1] - (-mu * K * K * A * s))) < tol
    assert np.max(np.abs(r[:, 2])) < tol
    assert np.max(np.abs(r[:, 3] - (g - 1) * mu * (K * A * c) ** 2)) < tol
    # pressure wave p = p0 + A sin(2 pi k x), rho = 1 (temperature p/rho follows p)
    r, x, y, kap, cfg = _ns_rhs_uniform(lambda x, y: (one(x), 0 * x, 0 * x, p0 + A * np.sin(2 * np.pi * k * x)), mu)
    s, c = np.sin(2 * np.pi * k * x), np.cos(2 * np.pi * k * x)
    assert np.max(np.abs(r[:, 0])) < tol
    assert np.max(np.abs(r[:, 1] - (-K * A * c))) < tol
    assert np.max(np.abs(r[:, 2])) < tol
    assert np.max(np.abs(r[:, 3] - (-(g - 1) * kc * K * K * A * s))) < 1e-7
    # longitudinal wave u = A sin(2 pi k x)
    r, x, y, kap, cfg = _ns_rhs_uniform(lambda x, y: (one(x), A * np.sin(2 * np.pi * k * x), 0 * x, p0 * one(x)), mu)
    s, c = np.sin(2 * np.pi * k * x), np.cos(2 * np.pi * k * x)
    assert np.max(np.abs(r[:, 0] - (-K * A * c))) < tol
    assert np.max(np.abs(r[:, 1] - (-K * A * A * s * c - 4.0 / 3.0 * mu * K * K * A * s))) < tol
    assert np.max(np.abs(r[:, 2])) < tol
    want_p = -g * p0 * K * A * c + (g - 1) * (4.0 / 3.0) * mu * (K * A * c) ** 2
    assert np.max(np.abs(r[:, 3] - want_p)) < tol


def _touch(a, b, dim):
    """Closed regions of leaves a=(l, c...) and b touch (periodic unit domain)."""
    la, lb = a[0], b[0]
    L = max(la, lb)
    n = 1 << L
    for ax in range(dim):
        sa, sb = 1 << (L - la), 1 << (L - lb)
        lo_a, lo_b = a[1 + ax] * sa, b[1 + ax] * sb
        ok = False
        for s in (-n, 0, n):
            if max(lo_a, lo_b + s) <= min(lo_a + sa, lo_b + s + sb):
                ok = True
        if not ok:
            return False
    return True


@pytest.mark.parametrize("dim,seed", [(2, 0), (2, 1), (2, 2), (3, 3)])
def test_refine_marked_is_graded_minimal_and_matches_refine_all(dim, seed):
    """Partial refinement (the 'arbitrary indicator' refinement of Sec. 2.3 under the
    gradedness of Sec. 2.2): every marked leaf below jmax refines; every other leaf that
    refines touches a finer refining leaf (minimal closure); the result is a valid
    graded forest; children values equal those refine-all computes from the same grid."""
    jmax = 4 if dim == 2 else 3
    cfg = W.Config(name="t", dim=dim, bs=9, hw=2, nf=1, jmax=jmax, eps=1e-3, physics=W.ADV_CONST,
                   phys=(1.0, 0.5, 0.25), dt=1e-3, steps=1, max_blocks=4 * 4 ** jmax if dim == 2 else 8 ** jmax)
    lv, co = W.random_graded_forest(dim, jmax - 1, seed)
    a = oracle.Oracle(cfg)
    a.init_forest(lv, co)
    lv, co = a.read_forest()             # forest order
    data = W.sample(cfg, lv, co, fn=lambda *x: np.cos(2 * np.pi * x[0]) * np.sin(2 * np.pi * x[1])
                    + 0.3 * np.sin(4 * np.pi * x[-1]))
    rng = np.random.default_rng(100 + seed)
    mask = (rng.random(len(lv)) < 0.15).astype(np.int8)
    a.load_blocks(data)
    k = a.refine_marked(mask)
    lv2, co2 = a.read_forest()
    oracle.Oracle(cfg).init_forest(lv2, co2)   # raises unless the result tiles and is graded
    before = {(int(l),) + tuple(int(v) for v in c) for l, c in zip(lv, co)}
    after = {(int(l),) + tuple(int(v) for v in c) for l, c in zip(lv2, co2)}
    refined = before - after
    assert len(refined) == k
    marked = {(int(lv[i]),) + tuple(int(v) for v in co[i]) for i in range(len(lv)) if mask[i] and lv[i] < jmax}
    assert marked <= refined
    for r in refined - marked:
        assert any(q[0] == r[0] + 1 and _touch(q, r, dim) for q in refined), r
    # children of each refined leaf exist and hold the refine-all values
    b = oracle.Oracle(cfg)
    b.init_forest(lv, co)
    b.load_blocks(data)
    b.refine_all()
    lv3, co3 = b.read_forest()
    full = {(int(l),) + tuple(int(v) for v in c): i for i, (l, c) in enumerate(zip(lv3, co3))}
    da, db = a.read_stored(), b.read_stored()
    for i, (l, c) in enumerate(zip(lv2, co2)):
        key = (int(l),) + tuple(int(v) for v in c)
        if key not in before:
            assert np.array_equal(da[i], db[full[key]])
    # all-ones mask is refine-all
    c_ = oracle.Oracle(cfg)
    c_.init_forest(lv, co)
    c_.load_blocks(data)
    c_.refine_marked(np.ones(len(lv), np.int8))
    l4, c4 = c_.read_forest()
    assert np.array_equal(l4, lv3) and np.array_equal(c4, co3)
    assert np.array_equal(c_.read_stored(), db)


# ---------------------------------------------------------------------------------------
# the solution on a uniform lattice of any level (Sec. 2.2 synchronised values, Sec. 2.3
# prediction inside coarser blocks; Sec. 4 takes spectra after refining to a fixed level)
# ---------------------------------------------------------------------------------------

def _inject(cfg, lv, co, data, L):
    """Uniform level-L array from block values at the points the blocks hold (L <= every
    block's level): each block's nodes that lie on the level-L lattice."""
    nl = (2 ** L) * (cfg.bs - 1)
    out = np.full((cfg.nf,) + (nl,) * cfg.dim, np.nan)
    loc = np.indices((cfg.bs,) * cfg.dim)[::-1].reshape(cfg.dim, -1)
    for b in range(len(lv)):
        sh = int(lv[b]) - L
        g = [int(co[b][a]) * (cfg.bs - 1) + loc[a] for a in range(cfg.dim)]
        on = np.ones(loc.shape[1], bool)
        for a in range(cfg.dim):
            on &= (g[a] % (1 << sh)) == 0
        idx = tuple(((g[a][on] >> sh) % nl) for a in range(cfg.dim))[::-1]
        for f in range(cfg.nf):
            out[(f,) + idx] = data[b, f][on]
    return out


def test_read_uniform_at_or_below_the_coarsest_leaf_is_injection():
    cfg = W.C1(jmax=4)
    o = oracle.Oracle(cfg)
    o.init_forest(*_two_level_forest())
    lv, co = o.read_forest()
    o.load_blocks(W.sample(cfg, lv, co, fn=lambda x, y: np.sin(2 * np.pi * x) * np.cos(4 * np.pi * y)))
    for L in (1, 2):
        want = _inject(cfg, lv, co, o.read_blocks(), L)
        assert not np.isnan(want).any()
        assert np.array_equal(o.read_uniform(L).view(np.uint64), want.view(np.uint64))


def test_read_uniform_reproduces_cubics_through_several_prediction_levels():
    """Tensor-cubic data on a two-level 2D forest read on the level-5 lattice: points inside
    the level-2 blocks are predicted through three levels, which the 4-point rule does
    exactly for cubics (away from the periodic seam, where the data is not periodic)."""
    cfg = W.C1(jmax=5)
    o = oracle.Oracle(cfg)
    o.init_forest(*_two_level_forest())
    lv, co = o.read_forest()
    p = lambda x: (x - 0.3) * (x - 0.55) * (x + 0.2)
    q = lambda y: 1.0 + y * (0.5 - y * y)
    o.load_blocks(W.sample(cfg, lv, co, fn=lambda x, y: p(x) * q(y)))
    L = 5
    U = o.read_uniform(L)[0]
    n = (2 ** L) * (cfg.bs - 1)
    g = np.arange(n) / n
    Y, X = np.meshgrid(g, g, indexing="ij")
    inner = (X > 0.12) & (X < 0.88) & (Y > 0.12) & (Y < 0.88)
    assert np.max(np.abs(U - p(X) * q(Y))[inner]) < 1e-13
    # and the data is really predicted there: sin data is not reproduced exactly
    o.load_blocks(W.sample(cfg, lv, co, fn=lambda x, y: np.sin(6 * np.pi * x)))
    U = o.read_uniform(L)[0]
    assert np.max(np.abs(U - np.sin(6 * np.pi * X))[inner]) > 1e-9


@pytest.mark.parametrize("dim", [2, 3])
def test_read_uniform_is_unchanged_by_the_safety_zone_refinement(dim):
    """Refinement gives the children the synchronised finer values (Sec. 2.1 item 1, Sec. 2.3
    prediction), so the solution read on any finer uniform lattice is the same before and
    after refine_all, bit for bit: the level-by-level read agrees with the point-by-point
    ghost values that refinement uses."""
    if dim == 2:
        cfg = W.C1(jmax=5)
        lv, co = W.random_graded_forest(2, 4, 5, p_refine=0.5)
        fn = lambda x, y: np.sin(2 * np.pi * x + 0.4) * np.cos(2 * np.pi * (x + 2 * y))
    else:
        cfg = W.C4(jmax=4).replace(max_blocks=8 ** 4)
        lv, co = W.random_graded_forest(3, 3, 2, p_refine=0.4)
        fn = lambda x, y, z: np.sin(2 * np.pi * (x + 0.2 * z)) * np.cos(2 * np.pi * y)
    o = oracle.Oracle(cfg)
    o.init_forest(lv, co)
    lv, co = o.read_forest()
    o.load_blocks(W.sample(cfg, lv, co, fn=fn))
    L = int(lv.max()) + 1
    before = o.read_uniform(L)
    o.refine_all()
    after = o.read_uniform(L)
    assert np.array_equal(before.view(np.uint64), after.view(np.uint64))


# ---------------------------------------------------------------------------------------
# the shear-layer test's shock-capturing filter (Sec. 4; the formulation is our own)
# ---------------------------------------------------------------------------------------

def _ns_uniform(level=3, fn=None):
    cfg = W.DSL(jmax=4)
    o = oracle.Oracle(cfg)
    lv, co = W.uniform_forest(cfg, level)
    o.init_forest(lv, co)
    lv, co = o.read_forest()
    o.load_blocks(W.sample(cfg, lv, co, fn=fn))
    return cfg, o, lv, co


def test_filter_leaves_constant_and_sub_threshold_states_unchanged():
    cfg, o, lv, co = _ns_uniform(fn=lambda x, y: (np.full_like(x, 1.5), np.full_like(x, 0.25),
                                                  np.full_like(x, -0.5), np.full_like(x, 2.5)))
    before = o.read_blocks()
    o.filter(1e-5)
    assert np.array_equal(o.read_blocks().view(np.uint64), before.view(np.uint64))
    smooth = lambda x, y: (1.0 + 0.1 * np.sin(2 * np.pi * x), 0.2 * np.cos(2 * np.pi * y),
                           0.1 * np.sin(2 * np.pi * (x + y)), 2.5 + 1e-3 * np.sin(2 * np.pi * x))
    cfg, o, lv, co = _ns_uniform(fn=smooth)
    before = o.read_blocks()
    o.filter(1e-5)    # relative pressure curvature ~1e-12 << 1e-5: the sensor stays off
    assert np.array_equal(o.read_blocks().view(np.uint64), before.view(np.uint64))


def test_filter_removes_the_odd_even_mode_where_the_sensor_saturates():
    """With every s = 1 the flux-form filter is q + (q_{i+1} - 2 q_i + q_{i-1})/4 per axis,
    which maps an alternating mode to zero: dyadic data make it exact."""
    n = 8 * 32
    alt = lambda x: np.where(np.rint(x * n).astype(int) % 2 == 0, 1.0, -1.0)
    fn = lambda x, y: (1.5 + 0.25 * alt(x), 0.5 * alt(x), -0.25 * alt(x), 2.5 + 0.25 * alt(x))
    cfg, o, lv, co = _ns_uniform(fn=fn)
    o.filter(1e-30)
    got = o.read_blocks()
    for f, c in enumerate((1.5, 0.0, 0.0, 2.5)):
        assert np.all(got[:, f] == c), f


def test_filter_conserves_every_field_on_a_uniform_periodic_grid():
    """Flux form: the filter's contributions telescope, so the sum over the unique lattice
    points is unchanged (to rounding); a steep pressure bump switches the sensor on."""
    bump = lambda x, y: 2.5 + 0.5 * np.exp(-((x - 0.4) ** 2 + (y - 0.6) ** 2) / 2e-5)
    fn = lambda x, y: (1.0 + 0.3 * np.exp(-((x - 0.5) ** 2) / 1e-3), 0.1 * np.sin(2 * np.pi * y),
                       0.2 * np.cos(2 * np.pi * x), bump(x, y))
    cfg, o, lv, co = _ns_uniform(fn=fn)
    before = o.read_uniform(3)
    o.filter(1e-5)
    after = o.read_uniform(3)
    assert np.max(np.abs(after - before)) > 1e-6          # the filter acted
    for f in range(4):
        s0, s1 = before[f].sum(), after[f].sum()
        assert abs(s1 - s0) <= 1e-12 * np.abs(before[f]).sum(), f
