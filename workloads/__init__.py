"""Seeded synthetic workloads for the block-based multiresolution solver.

This module is shared by the CPU oracle and the GPU library's harness.  It holds
only problem set-up: the configuration records (block size, levels, threshold,
physics constants, time step), the analytic initial conditions sampled at block
nodes, and the velocity tables of the swirl test.  It contains none of the
method's arithmetic (no ghost synchronisation, no prediction/restriction, no
finite differences, no Runge-Kutta, no details).

Geometry used to place samples (the block lattice of Sec. 2.2): a block at
level l with integer coordinates c covers the level-l node indices
g = c*(Bs-1) + i, i = 0..Bs-1, on a periodic unit domain with N_l = 2**l*(Bs-1)
unique nodes per direction, so the node sits at x = (g mod N_l) / N_l.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence

import numpy as np

ADV_CONST = 0
ADV_SWIRL = 1
NS2D = 2

FP64 = 0
MIXED = 1

FORM_PLAIN = 0
FORM_FUSED = 1


@dataclasses.dataclass
class Config:
    """One workload.  Field names mirror the C configuration record."""
    name: str
    dim: int
    bs: int                 # points per block and direction (odd)
    hw: int                 # ghost (halo) width used by the right-hand side
    nf: int                 # number of fields
    jmax: int               # finest level (level 1 is the coarsest)
    eps: float              # detail threshold
    physics: int
    phys: Sequence[float]   # ADV_CONST: c vector; ADV_SWIRL: (t_a,) (0 = steady); NS2D: (gamma, mu, Pr)
    dt: float
    steps: int
    max_blocks: int
    precision: int = FP64
    form: int = FORM_FUSED
    field_scale: Optional[Sequence[float]] = None
    field_offset: Optional[Sequence[float]] = None
    ic: str = "blobs"
    blob_centers: Optional[np.ndarray] = None
    blob_beta: float = 0.01
    ns_seed: int = 3

    @property
    def npts(self) -> int:
        return self.bs ** self.dim

    def n_finest(self) -> int:
        return (2 ** self.jmax) * (self.bs - 1)

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


def swirl_tables(cfg: Config):
    """sin^2(pi x) and sin(2 pi x) on the finest lattice x_i = i / N_jmax (Sec. 3 velocity field)."""
    n = cfg.n_finest()
    x = np.arange(n, dtype=np.float64) / n
    s = np.sin(np.pi * x)
    return np.ascontiguousarray(s * s), np.ascontiguousarray(np.sin(2.0 * np.pi * x))


def _dt_from_cfl(bs: int, jmax: int, speed: float, cfl: float = 0.5) -> float:
    h = 1.0 / ((2 ** jmax) * (bs - 1))
    return cfl * h / speed


def C1(jmax: int = 4, eps: float = 1e-3, steps: int = 100, **kw) -> Config:
    """2D constant advection c=(1,0.5), one Gaussian blob sigma=0.05 at the centre, Bs=17."""
    cfg = Config(name="C1", dim=2, bs=17, hw=2, nf=1, jmax=jmax, eps=eps,
                 physics=ADV_CONST, phys=(1.0, 0.5, 0.0),
                 dt=_dt_from_cfl(17, jmax, 1.0), steps=steps,
                 max_blocks=3 * 4 ** jmax, form=FORM_PLAIN,
                 blob_centers=np.array([[0.5, 0.5]]), blob_beta=2 * 0.05 ** 2)
    return cfg.replace(**kw)


def C2(jmax: int = 7, eps: float = 1e-4, steps: int = 500, **kw) -> Config:
    """2D steady swirl, three seeded blobs (beta=0.01), Bs=33."""
    centers = np.random.default_rng(2).uniform(0.25, 0.75, (3, 2))
    cfg = Config(name="C2", dim=2, bs=33, hw=2, nf=1, jmax=jmax, eps=eps,
                 physics=ADV_SWIRL, phys=(0.0,),
                 dt=_dt_from_cfl(33, jmax, 1.0), steps=steps,
                 max_blocks=min(3 * 4 ** jmax, 65536),
                 blob_centers=centers, blob_beta=0.01)
    return cfg.replace(**kw)


def C3(jmax: int = 8, eps: float = 1e-3, steps: int = 500, **kw) -> Config:
    """2D compressible Navier-Stokes temporal mixing layer (rho, u, v, p), Bs=33."""
    gamma, pr = 1.4, 0.71
    c0 = 1.25                     # Mach 0.4 on the velocity difference 1
    p0 = c0 * c0 / gamma
    mu = 1.0 * 1.0 * 0.02 / 1000.0  # Re = rho0 dU delta / mu = 1000
    cfg = Config(name="C3", dim=2, bs=33, hw=4, nf=4, jmax=jmax, eps=eps,
                 physics=NS2D, phys=(gamma, mu, pr),
                 dt=_dt_from_cfl(33, jmax, 0.5 + c0), steps=steps,
                 max_blocks=min(3 * 4 ** jmax, 3 * 65536), ic="mixing_layer",
                 field_offset=(1.0, 0.0, 0.0, p0))
    return cfg.replace(**kw)


# The double shear layer of Sec. 4 lives on [0, 8]^2; the solver's domain is the unit
# square, so coordinates are scaled by L = 8 (x = L x', t = L t'): velocities, density and
# pressure are unchanged and the viscosity becomes mu / L (second derivatives carry one more
# factor 1/L than the first ones).
DSL_L = 8.0


def DSL(jmax: int = 7, eps: float = 1e-3, t_end: float = 4.0, rth: float = 1e-5, **kw) -> Config:
    """2D compressible Navier-Stokes double shear layer (Sec. 4): L = 8, layers at L/2 +- 0.25,
    rho 2 / u 1 between them and rho 1 / u -1 outside, tanh jumps of width L/240, p = 2.5,
    v = 0.1 sin(2 pi (x - L/2)), mu = 1e-6, gamma 1.4, Pr 0.71, shock-capturing filter with
    threshold rth after every step, Bs = 33.  dt from CFL 0.5 on the finest level with
    |u| + c <= 3; `steps` reaches t_end (in the paper's time units)."""
    gamma, pr, mu = 1.4, 0.71, 1e-6
    dt = _dt_from_cfl(33, jmax, 3.0)
    cfg = Config(name="DSL", dim=2, bs=33, hw=4, nf=4, jmax=jmax, eps=eps,
                 physics=NS2D, phys=(gamma, mu / DSL_L, pr, rth),
                 dt=dt, steps=int(math.ceil(t_end / DSL_L / dt)),
                 max_blocks=min(3 * 4 ** jmax + 64, 3 * 65536), ic="double_shear_layer",
                 field_offset=(1.5, 0.0, 0.0, 2.5))
    return cfg.replace(**kw)


def C4(jmax: int = 6, eps: float = 1e-4, steps: int = 200, **kw) -> Config:
    """3D constant advection c=(1,0.5,0.25), four seeded blobs sigma=0.04, Bs=17."""
    centers = np.random.default_rng(4).uniform(0.25, 0.75, (4, 3))
    cfg = Config(name="C4", dim=3, bs=17, hw=2, nf=1, jmax=jmax, eps=eps,
                 physics=ADV_CONST, phys=(1.0, 0.5, 0.25),
                 dt=_dt_from_cfl(17, jmax, 1.0), steps=steps,
                 max_blocks=min(3 * 8 ** jmax, 400000),
                 blob_centers=centers, blob_beta=2 * 0.04 ** 2)
    return cfg.replace(**kw)


# --------------------------------------------------------------------------------------
# sampling
# --------------------------------------------------------------------------------------

def node_coords(cfg: Config, levels: np.ndarray, coords: np.ndarray):
    """Physical coordinates of every node of every block: list of arrays (one per axis),
    each shaped [n, bs**dim] with x fastest (node index i + bs*j + bs*bs*k)."""
    levels = np.asarray(levels, dtype=np.int64)
    coords = np.asarray(coords, dtype=np.int64).reshape(len(levels), cfg.dim)
    bs = cfg.bs
    loc = np.indices((bs,) * cfg.dim)[::-1]          # loc[0] = x index (fastest)
    loc = [a.reshape(-1) for a in loc]
    nl = (2 ** levels) * (bs - 1)
    out = []
    for a in range(cfg.dim):
        g = coords[:, a:a + 1] * (bs - 1) + loc[a][None, :]
        g = np.mod(g, nl[:, None])
        out.append(g.astype(np.float64) / nl[:, None].astype(np.float64))
    return out


def _axis_coords(cfg: Config, levels, coords):
    """Per block and axis, the physical coordinates of the bs node positions: list of
    dim arrays [n, bs]."""
    levels = np.asarray(levels, dtype=np.int64)
    coords = np.asarray(coords, dtype=np.int64).reshape(len(levels), cfg.dim)
    nl = (2 ** levels) * (cfg.bs - 1)
    i = np.arange(cfg.bs, dtype=np.int64)
    return [np.mod(coords[:, a:a + 1] * (cfg.bs - 1) + i[None, :], nl[:, None]).astype(np.float64)
            / nl[:, None].astype(np.float64) for a in range(cfg.dim)]


def _blob_axis_factor(cfg: Config, c_a: float, x):
    """G(x) = sum_{n in {-1,0,1}} exp(-(x - c_a - n)^2 / beta), evaluated once per distinct
    value of x (so equal coordinates get bitwise equal factors)."""
    u, inv = np.unique(x, return_inverse=True)
    g = np.zeros_like(u)
    for m in (-1.0, 0.0, 1.0):
        dd = u - c_a - m
        g = g + np.exp(-(dd * dd) / cfg.blob_beta)
    return g[inv.reshape(np.shape(x))]


def blob_field(cfg: Config, axes):
    """Sum of periodic Gaussian blobs exp(-|x-c-n|^2/beta) over the images n in {-1,0,1}^d on
    the tensor grid of the 1D coordinate arrays axes[a] ([..., len(axes[1]), len(axes[0])],
    x fastest).  The images form a Cartesian product and the Gaussian factorises over axes,
    so each blob is the product over axes of its 1D factors, x factor first."""
    d = cfg.dim
    shape = [len(axes[a]) for a in reversed(range(d))]
    val = np.zeros(shape)
    for c in cfg.blob_centers:
        prod = None
        for a in range(d):
            sh = [1] * d
            sh[d - 1 - a] = len(axes[a])
            ga = _blob_axis_factor(cfg, c[a], np.asarray(axes[a], dtype=np.float64)).reshape(sh)
            prod = ga if prod is None else prod * ga
        val = val + prod
    return val


def blob_at(cfg: Config, xs):
    """The blob sum at arbitrary points (xs[a]: arrays of one shape), images n in {-1,0,1}^d."""
    val = np.zeros(np.shape(xs[0]))
    for c in cfg.blob_centers:
        prod = None
        for a in range(cfg.dim):
            g = np.zeros(np.shape(xs[a]))
            for m in (-1.0, 0.0, 1.0):
                dd = np.asarray(xs[a]) - c[a] - m
                g = g + np.exp(-(dd * dd) / cfg.blob_beta)
            prod = g if prod is None else prod * g
        val = val + prod
    return val


def _blobs(cfg: Config, levels, coords):
    """blob_field at the nodes of each block: [n, bs^dim], x fastest."""
    ax = _axis_coords(cfg, levels, coords)
    n, bs, d = len(ax[0]), cfg.bs, cfg.dim
    val = np.zeros((n,) + (bs,) * d)
    for c in cfg.blob_centers:
        prod = None
        for a in range(d):
            shape = [n] + [1] * d
            shape[d - a] = bs                                 # axis a varies along array dim d - a
            ga = _blob_axis_factor(cfg, c[a], ax[a]).reshape(shape)
            prod = ga if prod is None else prod * ga
        val = val + prod
    return val.reshape(n, bs ** d)


def mixing_layer_fields(cfg: Config, x, y):
    """rho, u, v, p of the temporally developing mixing layer (delta = 0.02)."""
    gamma = cfg.phys[0]
    delta = 0.02
    c0 = 1.25
    p0 = c0 * c0 / gamma
    rho = np.ones_like(x)
    u = 0.5 * (np.tanh(2.0 * (y - 0.25) / delta) - np.tanh(2.0 * (y - 0.75) / delta) - 1.0)
    theta = np.random.default_rng(cfg.ns_seed).uniform(0.0, 2.0 * math.pi, 8)
    env = np.exp(-((y - 0.25) / (4 * delta)) ** 2) + np.exp(-((y - 0.75) / (4 * delta)) ** 2)
    s = np.zeros_like(x)
    for k in range(1, 9):
        s = s + np.sin(2.0 * math.pi * k * x + theta[k - 1])
    v = 1e-3 * (s / 8.0) * env
    p = np.full_like(x, p0)
    return rho, u, v, p


def double_shear_layer_fields(cfg: Config, x, y):
    """rho, u, v, p of the double shear layer at unit-square coordinates (x, y) (Sec. 4; the
    text names the jumping velocity 'y-velocity' and perturbs the 'x-velocity' along y; read
    as the shear layer it describes: u jumps across the layers normal to y, v is perturbed
    along x)."""
    L = DSL_L
    X, Y = L * x, L * y
    lam_w = L / 240.0
    y1, y2 = L / 2 - 0.25, L / 2 + 0.25
    step = 0.5 * (np.tanh((Y - y1) / lam_w) - np.tanh((Y - y2) / lam_w))   # 1 between the layers
    rho = 1.0 + (2.0 - 1.0) * step
    u = -1.0 + (1.0 - (-1.0)) * step
    v = 0.1 * np.sin(2.0 * math.pi * (X - L / 2))
    p = np.full_like(X, 2.5)
    return rho, u, v, p


def sample(cfg: Config, levels, coords, fn: Optional[Callable] = None) -> np.ndarray:
    """Initial-condition values at every node of the given blocks: float64 [n, nf, bs**dim]."""
    n = len(np.asarray(levels))
    out = np.empty((n, cfg.nf, cfg.npts), dtype=np.float64)
    if fn is None and cfg.ic == "blobs":
        out[:, 0, :] = _blobs(cfg, levels, coords)
        return out
    xs = node_coords(cfg, levels, coords)
    if fn is not None:
        vals = fn(*xs)
        vals = vals if isinstance(vals, (tuple, list)) else (vals,)
        for f in range(cfg.nf):
            out[:, f, :] = vals[f]
    elif cfg.ic == "mixing_layer":
        for f, v in enumerate(mixing_layer_fields(cfg, xs[0], xs[1])):
            out[:, f, :] = v
    elif cfg.ic == "double_shear_layer":
        for f, v in enumerate(double_shear_layer_fields(cfg, xs[0], xs[1])):
            out[:, f, :] = v
    else:
        raise ValueError(cfg.ic)
    return out


def uniform_forest(cfg: Config, level: int):
    """All blocks of one level, as (levels, coords)."""
    nb = 2 ** level
    idx = np.indices((nb,) * cfg.dim)[::-1].reshape(cfg.dim, -1).T
    return np.full(len(idx), level, dtype=np.int8), np.ascontiguousarray(idx.astype(np.int32))


def random_graded_forest(dim: int, jmax: int, seed: int, p_refine: float = 0.45, jmin: int = 1):
    """A random forest: start from uniform `jmin`, refine leaves at random, then add
    refinements until every pair of touching leaves differs by at most one level.
    Returns (levels int8 [n], coords int32 [n, dim]).  Topology only: no method arithmetic."""
    rng = np.random.default_rng(seed)
    leaves = set()
    nb = 2 ** jmin
    for c in np.indices((nb,) * dim).reshape(dim, -1).T:
        leaves.add((jmin,) + tuple(int(v) for v in c))
    for lev in range(jmin, jmax):
        for key in sorted(k for k in leaves if k[0] == lev):
            if rng.random() < p_refine:
                leaves.remove(key)
                for b in np.indices((2,) * dim).reshape(dim, -1).T:
                    leaves.add((lev + 1,) + tuple(2 * key[1 + a] + int(b[a]) for a in range(dim)))
    # grading: refine any leaf touched by a leaf two or more levels finer
    def touching(a, b):
        la, lb = a[0], b[0]
        L = max(la, lb)
        for ax in range(dim):
            n = 2 ** L
            a0 = a[1 + ax] << (L - la); a1 = (a[1 + ax] + 1) << (L - la)
            b0 = b[1 + ax] << (L - lb); b1 = (b[1 + ax] + 1) << (L - lb)
            ok = False
            for s in (-n, 0, n):
                if b0 + s <= a1 and a0 <= b1 + s:
                    ok = True
            if not ok:
                return False
        return True
    changed = True
    while changed:
        changed = False
        lst = sorted(leaves)
        for a in lst:
            if a not in leaves:
                continue
            for b in lst:
                if b in leaves and b[0] >= a[0] + 2 and touching(a, b):
                    leaves.remove(a)
                    for bb in np.indices((2,) * dim).reshape(dim, -1).T:
                        leaves.add((a[0] + 1,) + tuple(2 * a[1 + ax] + int(bb[ax]) for ax in range(dim)))
                    changed = True
                    break
    lst = sorted(leaves)
    levels = np.array([k[0] for k in lst], dtype=np.int8)
    coords = np.array([k[1:] for k in lst], dtype=np.int32).reshape(len(lst), dim)
    return levels, coords


# --------------------------------------------------------------------------------------
# learned predictor: seeded inputs (initial weights, class weights, batch order)
# --------------------------------------------------------------------------------------

MLP_HIDDEN = 64
MLP_OUT = 3


def mlp_init_params(nin: int, seed: int) -> np.ndarray:
    """Initial parameters of the nin -> 64 -> 64 -> 3 MLP, uniform in +-1/sqrt(fan_in),
    packed W1[nin][64], b1, W2[64][64], b2, W3[64][3], b3 (float32)."""
    rng = np.random.default_rng(seed)
    h, o = MLP_HIDDEN, MLP_OUT
    parts = [rng.uniform(-1, 1, (nin, h)) / math.sqrt(nin), rng.uniform(-1, 1, h) / math.sqrt(nin),
             rng.uniform(-1, 1, (h, h)) / math.sqrt(h), rng.uniform(-1, 1, h) / math.sqrt(h),
             rng.uniform(-1, 1, (h, o)) / math.sqrt(h), rng.uniform(-1, 1, o) / math.sqrt(h)]
    return np.concatenate([q.ravel() for q in parts]).astype(np.float32)


def class_weights(labels, ncls: int = 3) -> np.ndarray:
    """Inverse-frequency weights n / (ncls * n_c) (1 for absent classes)."""
    labels = np.asarray(labels)
    n = len(labels)
    w = np.ones(ncls, dtype=np.float32)
    for c in range(ncls):
        k = int(np.sum(labels == c))
        if k:
            w[c] = n / (ncls * k)
    return w


def epoch_order(n: int, seed: int, epoch: int) -> np.ndarray:
    """Seeded permutation of the training samples for one epoch."""
    return np.random.default_rng([seed, epoch]).permutation(n)
