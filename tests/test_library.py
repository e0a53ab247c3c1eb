"""The C-ABI library: exports (CPU) and parity against the CPU oracle (GPU).

FP64 results are compared bit for bit (the tolerance the method allows is 1e-12
relative per field; the design reaches exact equality because both sides round
every operation in the same order).  Flags and forests must match exactly.
"""
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W
import paper_1902_00088_amd as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mrb.h")).read()
    return sorted(set(re.findall(r"\b(mrb_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    import ctypes
    if not os.path.exists(M.LIB_PATH):
        M.build()
    L = ctypes.CDLL(M.LIB_PATH)
    names = _declared()
    assert set(names) == set(M.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_build_entry_reaches_the_hip_build(monkeypatch):
    """build() goes through the package's build() to the hipcc driver module
    (the stubs stand in for the compilers so the test stays fast)."""
    import importlib
    import __graft_entry__ as G
    hb = importlib.import_module("paper_1902_00088_amd.hipbuild")
    calls = []
    monkeypatch.setattr(hb, "build", lambda verbose=False: calls.append("hip") or M.LIB_PATH)
    monkeypatch.setattr(oracle, "build", lambda *a, **k: calls.append("oracle"))
    G.build()
    assert calls == ["hip", "oracle"]
    assert callable(M.build)


def test_solver_refuses_to_run_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        M.Solver(W.C1())


# ------------------------------------------------------------------------------------------
# GPU parity
# ------------------------------------------------------------------------------------------

def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def assert_same(s, o, what=""):
    lv1, co1 = s.read_forest()
    lv2, co2 = o.read_forest()
    assert np.array_equal(lv1, lv2) and np.array_equal(co1, co2), f"forest differs {what}"
    a, b = s.read_blocks(), o.read_blocks()
    if not np.array_equal(_bits(a), _bits(b)):
        den = np.maximum(np.max(np.abs(b), axis=(0, 2)), 1e-300)
        rel = np.max(np.abs(a - b), axis=(0, 2)) / den
        bad = np.argwhere(_bits(a) != _bits(b))
        raise AssertionError(f"values differ {what}: rel per field {rel}, first {bad[:5].tolist()}, n={len(bad)}")


def _pair(cfg, levels=None, coords=None, fn=None):
    s = M.Solver(cfg)
    o = oracle.Oracle(cfg)
    if levels is None:
        s.init_grid(fn=fn)
        o.init_grid(fn=fn)
    else:
        for x in (s, o):
            x.init_forest(levels, coords)
            x.load_blocks(W.sample(cfg, *x.read_forest(), fn=fn))
    return s, o


def oracle_flags_on_state(cfg, lv, co, data):
    """The oracle's analysis (Sec. 2.3) applied to a given state: the flag function checked
    on the GPU's own (mixed-precision) state.  The data here is the GPU's, so this is a
    check of the analysis alone, not a parity case for the fields."""
    o = oracle.Oracle(cfg.replace(precision=W.FP64))
    o.init_forest(lv, co)
    o.load_blocks(data)
    return o.mr_pass()


def assert_own_flags(s, cfg, fs, ms):
    """The GPU's flags and detail maxima from its own mr_pass equal the oracle's analysis of
    the state the GPU holds after that pass (bitwise: the analysis is FP64 in both forms)."""
    lv, co = s.read_forest()
    fo, mo = oracle_flags_on_state(cfg, lv, co, s.read_blocks())
    assert np.array_equal(fs, fo), f"{int(np.sum(fs != fo))} flags differ"
    assert np.array_equal(_bits(ms), _bits(mo))


def _two_level():
    keys = [(2, x, y) for x in range(4) for y in range(4) if (x, y) != (1, 1)]
    keys += [(3, 2 + bx, 2 + by) for bx in range(2) for by in range(2)]
    return np.array([k[0] for k in keys], np.int8), np.array([k[1:] for k in keys], np.int32)


SMOOTH2 = lambda x, y: np.sin(2 * np.pi * x + 0.3) * np.cos(4 * np.pi * y) + 0.5 * np.cos(2 * np.pi * (x - y))
SMOOTH3 = lambda x, y, z: np.sin(2 * np.pi * x + 0.3) * np.cos(2 * np.pi * y) + 0.3 * np.sin(2 * np.pi * (z - x))


@pytest.mark.gpu
@pytest.mark.parametrize("form,nsub", [(W.FORM_FUSED, 1), (W.FORM_FUSED, 2), (W.FORM_PLAIN, 0)])
def test_rk4_on_two_level_forest_is_bitwise(form, nsub):
    cfg = W.C1(jmax=3, form=form)
    lv, co = _two_level()
    s, o = _pair(cfg, lv, co, fn=SMOOTH2)
    if nsub:
        assert s.tune(nsub=nsub) == nsub
    assert_same(s, o, "after load")
    s.rk4(0.0, cfg.dt)
    o.rk4(0.0, cfg.dt)
    assert_same(s, o, "after rk4")


@pytest.mark.gpu
@pytest.mark.parametrize("seed", range(6))
def test_random_graded_forest_refine_rk4_mr(seed):
    lv, co = W.random_graded_forest(2, 4, seed, p_refine=0.5)
    cfg = W.C2(jmax=5, eps=3e-3).replace(bs=17 if seed % 2 == 0 else 33, max_blocks=3 * 4 ** 5)
    s, o = _pair(cfg, lv, co, fn=SMOOTH2)
    s.tune(nsub=[1, 2, 1, 4, 2, 2][seed])
    s.rk4(0.0, cfg.dt)
    o.rk4(0.0, cfg.dt)
    assert_same(s, o, "rk4")
    fs, ms = s.mr_pass()
    fo, mo = o.mr_pass()
    assert np.array_equal(fs, fo) and np.array_equal(_bits(ms), _bits(mo))
    assert_same(s, o, "after mr sync")
    ns, no = s.coarsen(fs), o.coarsen(fo)
    assert ns == no
    assert_same(s, o, "coarsen")
    s.refine_all()
    o.refine_all()
    assert_same(s, o, "refine")


@pytest.mark.gpu
@pytest.mark.parametrize("form", [W.FORM_PLAIN, W.FORM_FUSED])
def test_c1_full_run_is_bitwise(form):
    """C1: 2D advection, Bs=17, Jmax=4, eps=1e-3, 100 steps, FP64."""
    cfg = W.C1(form=form)
    s, o = _pair(cfg)
    assert_same(s, o, "initial grid")
    t = 0.0
    for n in range(cfg.steps):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
        if n % 25 == 24:
            assert_same(s, o, f"step {n + 1}")
    assert_same(s, o, "end")


@pytest.mark.gpu
def test_c2_full_size_sampled_steps():
    """C2 at its full configuration (Bs=33, Jmax=7, eps=1e-4) in the benchmark's launch
    configuration (fused FP64): 40 steps, every 10th compared."""
    cfg = W.C2(form=W.FORM_FUSED)
    s, o = _pair(cfg)
    assert_same(s, o, "initial grid")
    t = 0.0
    for n in range(40):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
        if n % 10 == 9:
            assert_same(s, o, f"step {n + 1}")
    # the forest cycles through the same refine / coarsen transitions every step:
    # from the second step on the library replays memoised plans, and the first
    # coarsening of each adapt is speculated (and confirmed) before the flags are read
    st = s.stats()
    assert st["memo_hits"] >= 2 * 38
    assert st["spec_hits"] >= 35 and st["spec_misses"] == 0


@pytest.mark.gpu
def test_c2_narrow_blobs_deep_forest():
    """Swirl with narrow blobs: a deep, ragged forest (levels 2..6) that changes each step."""
    cfg = W.C2(jmax=6, eps=1e-4, blob_beta=4e-4, form=W.FORM_FUSED)
    s, o = _pair(cfg)
    lv, _ = s.read_forest()
    assert len(np.unique(lv)) >= 3
    t = 0.0
    for n in range(6):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    assert_same(s, o, "after 6 steps")


@pytest.mark.gpu
def test_3d_random_forest_rk4_mr_refine():
    lv, co = W.random_graded_forest(3, 3, 1, p_refine=0.4)
    cfg = W.C4(jmax=4, eps=1e-3, form=W.FORM_FUSED).replace(max_blocks=3 * 8 ** 4)
    s, o = _pair(cfg, lv, co, fn=SMOOTH3)
    assert len(np.unique(lv)) >= 2
    s.rk4(0.0, cfg.dt)
    o.rk4(0.0, cfg.dt)
    assert_same(s, o, "rk4")
    fs, ms = s.mr_pass()
    fo, mo = o.mr_pass()
    assert np.array_equal(fs, fo) and np.array_equal(_bits(ms), _bits(mo))
    assert s.coarsen(fs) == o.coarsen(fo)
    s.refine_all()
    o.refine_all()
    assert_same(s, o, "coarsen + refine")


@pytest.mark.gpu
def test_3d_small_run_is_bitwise():
    cfg = W.C4(jmax=3, eps=1e-3, form=W.FORM_FUSED).replace(max_blocks=3 * 8 ** 3)
    s, o = _pair(cfg)
    assert_same(s, o, "initial grid")
    t = 0.0
    for n in range(3):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    assert_same(s, o, "after 3 steps")


@pytest.mark.gpu
def test_mixed_precision_within_1e5_on_replayed_topology():
    """Mixed form (FP32 stencil and slopes, FP64 state): per-field relative error
    against the FP64 oracle <= 1e-5, with the oracle's coarsening flags replayed."""
    cfg = W.C2(jmax=6, eps=1e-4, blob_beta=4e-4)
    s = M.Solver(cfg.replace(precision=W.MIXED, form=W.FORM_FUSED))
    o = oracle.Oracle(cfg)
    o.init_grid()
    s.init_forest(*o.read_forest())
    s.load_blocks(W.sample(cfg, *o.read_forest()))
    t = 0.0
    worst = 0.0
    for n in range(20):
        for x in (s, o):
            x.refine_all()
            x.rk4(t, cfg.dt)
        while True:
            fo, _ = o.mr_pass()
            fs, ms = s.mr_pass()
            if n % 5 == 0:
                assert_own_flags(s, cfg, fs, ms)
            if o.coarsen(fo) == 0:
                assert s.coarsen(fo) == 0
                break
            s.coarsen(fo)
        t += cfg.dt
        a, b = s.read_blocks(), o.read_blocks()
        assert np.array_equal(s.read_forest()[0], o.read_forest()[0])
        rel = np.max(np.abs(a - b)) / np.max(np.abs(b))
        worst = max(worst, rel)
    assert worst <= 1e-5, worst
    assert worst > 0.0


@pytest.mark.gpu
def test_runs_are_deterministic():
    cfg = W.C2(jmax=5, eps=1e-4, blob_beta=1e-3, form=W.FORM_FUSED)
    outs = []
    for _ in range(2):
        s = M.Solver(cfg)
        s.init_grid()
        s.step(0.0, cfg.dt, 5)
        outs.append((s.read_forest(), s.read_blocks()))
        s.close()
    assert np.array_equal(outs[0][0][0], outs[1][0][0])
    assert np.array_equal(_bits(outs[0][1]), _bits(outs[1][1]))


@pytest.mark.gpu
def test_error_paths_leave_state_unchanged():
    cfg = W.C1(jmax=3)
    s = M.Solver(cfg.replace(max_blocks=64))
    with pytest.raises(M.MrbError) as e:
        s.step(0.0, cfg.dt)
    assert e.value.code == -4                            # no forest yet
    lv, co = W.uniform_forest(cfg, 2)
    with pytest.raises(M.MrbError) as e:
        s.init_forest(lv[1:], co[1:])
    assert e.value.code == -3                            # hole
    s.init_forest(lv, co)
    s.load_blocks(W.sample(cfg, lv, co))
    before = s.read_blocks()
    with pytest.raises(M.MrbError) as e:
        s.refine_all()                                   # 16 + 64 > 64 slots
    assert e.value.code == -2
    assert s.num_blocks() == 16
    assert np.array_equal(_bits(s.read_blocks()), _bits(before))
    keys = [(1, 1, 0), (1, 0, 1), (1, 1, 1), (2, 0, 1), (2, 1, 0), (2, 1, 1)] + \
           [(3, x, y) for x in range(2) for y in range(2)]
    with pytest.raises(M.MrbError) as e:
        s.init_forest([k[0] for k in keys], [k[1:] for k in keys])
    assert e.value.code == -3                            # not graded
    assert s.num_blocks() == 16
    with pytest.raises(M.MrbError):
        M.Solver(cfg.replace(bs=16))                     # even block size


@pytest.mark.gpu
@pytest.mark.parametrize("form", [W.FORM_FUSED, W.FORM_PLAIN])
def test_ns_mixing_layer_fp64_is_bitwise(form):
    """C3 set-up (compressible NS mixing layer) at Jmax 4 with eps = 1e-4, so that the
    grid has two levels (at eps = 1e-3 it is uniform on level 3): initial grid, 3 steps,
    in the fused form and in the plain form (ghosts stored, per-level launches)."""
    cfg = W.C3(jmax=4, eps=1e-4, form=form)
    s, o = _pair(cfg)
    lv, _ = s.read_forest()
    assert len(np.unique(lv)) >= 2
    assert_same(s, o, "initial grid")
    t = 0.0
    for n in range(3):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    assert_same(s, o, "after 3 steps")


@pytest.mark.gpu
@pytest.mark.parametrize("nsub", [2, 4])
def test_ns_tilings_agree_bitwise(nsub):
    cfg = W.C3(jmax=4, form=W.FORM_FUSED)
    lv, co = _two_level()
    s, o = _pair(cfg.replace(jmax=3), lv, co)
    s.tune(nsub=nsub)
    s.rk4(0.0, cfg.dt)
    o.rk4(0.0, cfg.dt)
    assert_same(s, o, "rk4")


@pytest.mark.gpu
@pytest.mark.parametrize("form", [(1, 512), (1, 1024), (2, 512)])
def test_ns_stage_workgroup_sizes_agree_bitwise(form):
    """The Navier-Stokes stage kernel with larger workgroups performs the same operations
    as with 256 threads: mixed, its steps equal the 256-thread ones bit for bit; FP64
    (compiled for quarter blocks), they equal the oracle."""
    nsub, tpb = form
    cfg = W.C3(jmax=4, eps=1e-4, form=W.FORM_FUSED)
    ref = M.Solver(cfg.replace(precision=W.MIXED))
    ref.init_grid()
    lv, co = ref.read_forest()
    data = ref.read_blocks()
    ref.tune(nsub=nsub)
    s = M.Solver(cfg.replace(precision=W.MIXED))
    s.init_forest(lv, co)
    s.load_blocks(data)
    s.tune(nsub=nsub, reps=-tpb)
    assert s.stats()["stage_threads"] == tpb and s.stats()["analysis_threads"] == tpb
    t = 0.0
    for _ in range(3):
        s.step(t, cfg.dt)
        ref.step(t, cfg.dt)
        t += cfg.dt
    a, b = s.read_forest(), ref.read_forest()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(_bits(s.read_blocks()), _bits(ref.read_blocks()))
    s.close()
    ref.close()
    if nsub == 2:
        s, o = _pair(cfg)
        s.tune(nsub=nsub, reps=-tpb)
        t = 0.0
        for _ in range(2):
            s.step(t, cfg.dt)
            o.step(t, cfg.dt)
            t += cfg.dt
        assert_same(s, o, f"FP64 stage, {tpb} threads")
        s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("tpb", [512, 1024])
def test_analysis_workgroup_sizes_match_oracle(tpb):
    """The analysis of whole one-field blocks with larger workgroups, on a forest on two
    levels (coarse-to-fine prediction and finer-owned redundant nodes in play): steps,
    flags and detail maxima equal the oracle's bit for bit."""
    cfg = W.C2(jmax=4, form=W.FORM_FUSED)
    lv, co = _two_level()
    s, o = _pair(cfg, lv, co)
    s.set_graph(0)
    s.tune(nsub=1, reps=-tpb)
    assert s.stats()["analysis_threads"] == tpb
    t = 0.0
    for _ in range(3):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    assert_same(s, o, f"analysis with {tpb} threads")
    fs, ms = s.mr_pass()
    fo, mo = o.mr_pass()
    assert np.array_equal(fs, fo) and np.array_equal(_bits(ms), _bits(mo))
    s.close()


@pytest.mark.gpu
def test_ns_mixed_within_1e5():
    cfg = W.C3(jmax=4, eps=1e-4)
    s = M.Solver(cfg.replace(precision=W.MIXED, form=W.FORM_FUSED))
    o = oracle.Oracle(cfg)
    o.init_grid()
    s.init_forest(*o.read_forest())
    s.load_blocks(W.sample(cfg, *o.read_forest()))
    t = 0.0
    for n in range(4):
        for x in (s, o):
            x.refine_all()
            x.rk4(t, cfg.dt)
        while True:
            fo, _ = o.mr_pass()
            fs, ms = s.mr_pass()
            assert_own_flags(s, cfg, fs, ms)
            if o.coarsen(fo) == 0:
                assert s.coarsen(fo) == 0
                break
            s.coarsen(fo)
        t += cfg.dt
    a, b = s.read_blocks(), o.read_blocks()
    rel = np.max(np.abs(a - b), axis=(0, 2)) / np.max(np.abs(b), axis=(0, 2))
    assert np.all(rel <= 1e-5), rel
    assert np.any(rel > 0)


@pytest.mark.gpu
def test_autotune_picks_a_compiled_tiling_and_keeps_state():
    cfg = W.C2(form=W.FORM_FUSED)
    s = M.Solver(cfg)
    s.init_grid()
    before = s.read_blocks()
    ch = s.tune(reps=3)
    assert ch in (1, 2, 4)
    st = s.stats()
    assert len([k for k in st["tune_ms"] if k.isdigit()]) == 3 and len(st["tune_ms"]["mr"]) == 3
    assert np.array_equal(_bits(s.read_blocks()), _bits(before))


@pytest.mark.gpu
def test_graph_replay_matches_direct_launches():
    """Steps replayed from the captured graph equal directly launched steps bit for bit,
    across topology changes (narrow blobs: the forest changes every few steps)."""
    cfg = W.C2(jmax=6, eps=1e-4, blob_beta=4e-4, form=W.FORM_FUSED)
    outs = []
    for graph in (1, 0, 2):
        s = M.Solver(cfg)
        s.set_graph(graph)
        s.init_grid()
        s.step(0.0, cfg.dt, 24)
        st = s.stats()
        assert (st["graph_launches"] > 0) == (graph != 0)
        if graph == 2:   # automatic: ten steps each way, then the faster one
            assert st["graph_launches"] >= 10 and st["graph_mode"] == 2
        outs.append((s.read_forest(), s.read_blocks()))
        s.close()
    for o in outs[1:]:
        assert np.array_equal(outs[0][0][0], o[0][0]) and np.array_equal(outs[0][0][1], o[0][1])
        assert np.array_equal(_bits(outs[0][1]), _bits(o[1]))
    with pytest.raises(M.MrbError):
        M.Solver(cfg).set_graph(3)


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["C1", "C4", "C3"])
def test_read_uniform_matches_oracle_at_every_level(which):
    """read_uniform at every level 1..jmax equals the oracle's level-by-level V bit for
    bit (injection at or below the coarsest leaf, prediction through several levels above
    it), leaves the solver's state unchanged, and the next step still equals the oracle's."""
    if which == "C1":
        cfg = W.C1(jmax=5, form=W.FORM_FUSED)
        s, o = _pair(cfg)
        for n in range(3):
            s.step(n * cfg.dt, cfg.dt)
            o.step(n * cfg.dt, cfg.dt)
    elif which == "C4":
        cfg = W.C4(jmax=4, form=W.FORM_FUSED).replace(max_blocks=8 ** 4 + 600)
        s, o = _pair(cfg, *W.random_graded_forest(3, 3, 7), fn=SMOOTH3)
    else:
        cfg = W.C3(jmax=5, eps=1e-4, form=W.FORM_FUSED)
        s, o = _pair(cfg)
    lv, co = o.read_forest()
    assert len(np.unique(lv)) >= 2
    before = s.read_blocks()
    for L in range(1, cfg.jmax + 1):
        got = s.read_uniform(L)
        want = o.read_uniform(L)
        assert np.array_equal(_bits(got), _bits(want)), (which, L)
    assert_same(s, o, "after the reads")
    assert np.array_equal(_bits(s.read_blocks()), _bits(before))
    for bad in (0, cfg.jmax + 1):
        with pytest.raises(M.MrbError):
            s.read_uniform(bad)
    s.step(0.5, cfg.dt)
    o.step(0.5, cfg.dt)
    assert_same(s, o, "step after the reads")
    s.close()


@pytest.mark.gpu
def test_speculative_coarsening_rolls_back_when_flags_change():
    """The first coarsening of an adapt is speculated from the previous step; a
    perturbation that changes the flags makes the speculation miss, and the step
    must still equal the oracle's bit for bit."""
    cfg = W.C2(form=W.FORM_FUSED)
    s, o = _pair(cfg)
    t = 0.0
    for _ in range(4):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    assert s.stats()["spec_hits"] >= 2
    # a narrow bump in one block: its refined children keep large details
    lv, co = o.read_forest()
    bump = W.sample(cfg, lv, co, fn=lambda x, y: 0.5 * np.exp(-((x - 0.3) ** 2 + (y - 0.6) ** 2) / 4e-5))
    data = o.read_blocks() + bump
    s.load_blocks(data)
    o.load_blocks(data)
    miss0 = s.stats()["spec_misses"]
    for n in range(3):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
        assert_same(s, o, f"step {n + 1} after the perturbation")
    assert s.stats()["spec_misses"] > miss0


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["c2", "c4", "c3"])
def test_one_launch_sweep_matches_oracle(case):
    """The whole RK4 sweep as one cooperative launch with grid barriers between the
    stages equals the oracle bit for bit: 2D swirl at full size, a 3D forest, and the
    Navier-Stokes shape (two levels)."""
    if case == "c2":
        cfg, n = W.C2(form=W.FORM_FUSED), 6
    elif case == "c4":
        cfg, n = W.C4(jmax=3, eps=1e-3, form=W.FORM_FUSED).replace(max_blocks=3 * 8 ** 3), 3
    else:
        cfg, n = W.C3(jmax=4, eps=1e-4, form=W.FORM_FUSED), 2
    s, o = _pair(cfg)
    s.set_graph(0)
    s.set_sweep(1)
    t = 0.0
    for _ in range(n):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
        assert s.stats()["sweep_launch"] == "one"
    assert_same(s, o, f"{case}: {n} steps")
    st = s.stats()
    assert st["sweep_grid"] >= 8 and st["sweep_grid"] % 8 == 0
    s.set_sweep(0)
    assert s.stats()["sweep_launch"] == "four"
    with pytest.raises(M.MrbError):
        s.set_sweep(4)
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["c2_fp64_1", "c2_fp64_2", "c2_fp64_4", "c2_reversal_4", "c1_uniform"])
def test_overlapped_tile_rk4_matches_oracle(case):
    """One launch per RK4 step over overlapped tiles (every leaf on one level) equals the
    oracle bit for bit, for each compiled tiling: the 2D swirl at full size (its forest is
    16 blocks on level 2, 64 after refine-all), the swirl with the time-reversal factor
    cos(pi t / t_a) (a different factor per stage), and constant advection with Bs 17 on
    a uniform grid (eps = 0)."""
    if case.startswith("c2_fp64"):
        cfg, n, nsub = W.C2(form=W.FORM_FUSED), 5, int(case[-1])
    elif case == "c2_reversal_4":
        cfg, n, nsub = W.C2(form=W.FORM_FUSED).replace(phys=(5.0,)), 5, 4
    else:
        cfg, n, nsub = W.C1(jmax=3, eps=0.0, form=W.FORM_FUSED), 4, 1
    s, o = _pair(cfg)
    s.set_graph(0)
    s.set_sweep(3)
    s.tune(nsub=nsub)
    s.timing(True)
    t = 0.0
    for k in range(n):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    st = s.stats()
    assert st["sweep_launch"] == "rk4_tile" and st["rk4_tile_tiles"] == nsub
    assert st["kernels"]["rk4_tile"]["launches"] == n and st["kernels"]["stage"]["launches"] == 0
    # the first analysis of every adapt runs inside the tile launch, and so does the
    # swirl's refine-all (16 blocks on level 2); where the swirl's coarsening is
    # speculated (every step once the memo knows the forest's cycle) it merges every
    # block, so its second analysis runs inside the tile launch as well; the uniform
    # eps = 0 grid takes one pass per adapt
    if case == "c1_uniform":
        assert st["kernels"]["mr"]["launches"] == 0
    else:
        assert st["spec_hits"] >= n - 1 and st["kernels"]["mr"]["launches"] <= 1
    assert st["kernels"]["refine"]["launches"] == 0
    assert_same(s, o, f"{case}: {n} steps")
    # the last analysis (the folded second pass, for the swirl) equals the oracle's
    # analysis of the final state
    fs, ms = s.get_flags()
    assert_own_flags(s, cfg, fs, ms)
    s.close()


@pytest.mark.gpu
def test_overlapped_tile_rk4_with_device_topology_matches_oracle():
    """The tile step on a uniform grid planned on the device (eps = 0: every step's
    analysis leaves the grid as it is) equals the oracle bit for bit."""
    cfg = W.C2(jmax=4, eps=0.0, form=W.FORM_FUSED).replace(phys=(5.0,))
    s, o = _pair(cfg)
    s.set_graph(0)
    s.set_topology(1)
    s.set_sweep(3)
    s.timing(True)
    t = 0.0
    for _ in range(4):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    st = s.stats()
    assert st["topology"] == "device" and st["kernels"]["rk4_tile"]["launches"] == 4
    assert_same(s, o, "device topology, tile step")
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("sweep", [2, 3])
@pytest.mark.parametrize("case", ["2d_at_jmax", "2d_level1_below_jmax", "3d_level1_below_jmax"])
def test_smallest_forests_match_oracle(case, sweep):
    """Edge cases on the smallest forests (the library takes Jmax >= 2): the uniform
    grid at Jmax 2 (nothing refines), and two blocks per direction (level 1, where the
    neighbour across either face is the same block through a periodic image) one level
    below Jmax (every block refines; in mode 3 the refinement folds into the tile step),
    several steps per call, 2D and 3D."""
    if case == "2d_at_jmax":
        cfg = W.C2(jmax=2, form=W.FORM_FUSED).replace(phys=(5.0,))
        lv, co = W.uniform_forest(cfg, 2)
    elif case == "2d_level1_below_jmax":
        cfg = W.C2(jmax=2, eps=1e-2, form=W.FORM_FUSED).replace(phys=(5.0,))
        lv, co = W.uniform_forest(cfg, 1)
    else:
        cfg = W.C4(jmax=2, eps=1e-3, form=W.FORM_FUSED)
        lv, co = W.uniform_forest(cfg, 1)
    s, o = _pair(cfg, lv, co)
    s.set_graph(0)
    s.set_sweep(sweep)
    t = 0.0
    s.step(t, cfg.dt, 4)
    for _ in range(4):
        o.step(t, cfg.dt)
        t += cfg.dt
    assert_same(s, o, f"{case}, 4 steps")
    fs, ms = s.get_flags()
    assert_own_flags(s, cfg, fs, ms)
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("nsub", [1, 4])
def test_overlapped_tile_rk4_alone_matches_oracle(nsub):
    """mrb_rk4 in mode 3 (the tile step without the analysis folded in), then an
    analysis pass: values, flags and detail maxima equal the oracle's."""
    cfg = W.C2(form=W.FORM_FUSED).replace(phys=(5.0,))
    s, o = _pair(cfg)
    s.set_sweep(3)
    s.tune(nsub=nsub)
    for x in (s, o):
        x.refine_all()
        x.rk4(0.25, cfg.dt)
    assert_same(s, o, "refine-all + rk4")
    fs, ms = s.mr_pass()
    fo, mo = o.mr_pass()
    assert np.array_equal(fs, fo) and np.array_equal(_bits(ms), _bits(mo))
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotuned_tile_step_matches_oracle(prec):
    """The headline workload's step loop with the autotuner's choices (the tile step and,
    where faster, the first analysis folded into it, with the tuned threads per
    workgroup): FP64 equals the oracle bit for bit, mixed stays within 1e-5 with the
    oracle's forest."""
    cfg = W.C2(form=W.FORM_FUSED, precision=W.FP64 if prec == "fp64" else W.MIXED)
    s = M.Solver(cfg)
    o = oracle.Oracle(cfg.replace(precision=W.FP64))
    for x in (s, o):
        x.init_grid()
    s.refine_all()
    s.tune(reps=2)
    lv, co = o.read_forest()
    s.init_forest(lv, co)
    s.load_blocks(o.read_blocks())
    s.set_graph(0)
    t = 0.0
    for _ in range(6):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    st = s.stats()
    print(st["sweep_launch"], st["rk4_tile_tiles"], st["rk4_tile_analysis"], st["tune_ms"].get("rk4_tile_analysis"))
    if prec == "fp64":
        assert_same(s, o, "autotuned step loop")
    else:
        lv1, co1 = s.read_forest()
        lv2, co2 = o.read_forest()
        assert np.array_equal(lv1, lv2) and np.array_equal(co1, co2)
        ref = o.read_blocks()
        assert np.max(np.abs(s.read_blocks() - ref)) / np.max(np.abs(ref)) <= 1e-5
    s.close()


@pytest.mark.gpu
def test_overlapped_tile_rk4_mixed_equals_stage_launches():
    """In the mixed form the overlapped-tile step performs the stage kernels' operations
    in the same order, so it equals the four stage launches bit for bit, and both stay
    within 1e-5 of the FP64 oracle."""
    cfg = W.C2(form=W.FORM_FUSED, precision=W.MIXED)
    a = M.Solver(cfg)
    b = M.Solver(cfg)
    o = oracle.Oracle(cfg.replace(precision=W.FP64))
    for x in (a, b, o):
        x.init_grid()
    for x in (a, b):
        x.set_graph(0)
    a.set_sweep(3)
    a.tune(nsub=2)
    b.set_sweep(0)
    t = 0.0
    for _ in range(6):
        for x in (a, b, o):
            x.step(t, cfg.dt)
        t += cfg.dt
    assert a.stats()["sweep_launch"] == "rk4_tile" and b.stats()["sweep_launch"] == "four"
    assert np.array_equal(_bits(a.read_blocks()), _bits(b.read_blocks()))
    lv1, co1 = a.read_forest()
    lv2, co2 = o.read_forest()
    assert np.array_equal(lv1, lv2) and np.array_equal(co1, co2)
    ref = o.read_blocks()
    assert np.max(np.abs(a.read_blocks() - ref)) / np.max(np.abs(ref)) <= 1e-5
    a.close()
    b.close()


@pytest.mark.gpu
def test_overlapped_tile_rk4_falls_back_on_several_levels():
    """Mode 3 on a forest with two levels takes the four stage launches (and stays exact)."""
    cfg = W.C1(jmax=4, eps=1e-3, form=W.FORM_FUSED)
    s, o = _pair(cfg)
    lv, _ = s.read_forest()
    assert len(set(lv.tolist())) > 1
    s.set_graph(0)
    s.set_sweep(3)
    s.timing(True)
    t = 0.0
    for _ in range(3):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    assert s.stats()["kernels"]["stage"]["launches"] == 12
    assert_same(s, o, "two levels, mode 3")
    s.close()


@pytest.mark.gpu
def test_autotuner_times_both_sweep_launch_forms():
    cfg = W.C2(jmax=5, eps=1e-4, form=W.FORM_FUSED)
    s = M.Solver(cfg)
    s.init_grid()
    before = s.read_blocks()
    s.tune(reps=2)
    st = s.stats()
    sw = st["tune_ms"]["sweep"]
    assert sw["four"] > 0 and sw["one"] > 0
    # the initial grid is on one level, so the overlapped-tile step is timed as well
    rt = st["tune_ms"]["rk4_tile"]
    assert set(rt) == {"1", "2", "4", "stages"} and all(v > 0 for v in rt.values())
    best = min(rt[k] for k in ("1", "2", "4"))
    if best < rt["stages"]:
        assert st["sweep_launch"] == "rk4_tile" and rt[str(st["rk4_tile_tiles"])] == best
    else:
        assert st["sweep_launch"] == ("one" if sw["one"] < sw["four"] else "four")
    assert np.array_equal(_bits(s.read_blocks()), _bits(before))
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("sweep", [2, 3])
def test_multi_step_calls_match_oracle(sweep):
    """The library's own step loop (several steps per call, direct launches) equals
    single oracle steps bit for bit: with the default launches, and with the one-launch
    tile step, where the swirl's forest cycles and each step's launch is queued before
    the previous step's flags are read."""
    cfg = W.C2(form=W.FORM_FUSED).replace(phys=(5.0,))
    s, o = _pair(cfg)
    s.set_graph(0)
    s.set_sweep(sweep)
    t = 0.0
    for chunk in range(3):
        s.step(t, cfg.dt, 10)
        for _ in range(10):
            o.step(t, cfg.dt)
            t += cfg.dt
        assert_same(s, o, f"after {10 * (chunk + 1)} steps")
    st = s.stats()
    assert st["spec_hits"] >= 25
    if sweep == 3:
        assert st["queued_steps"] >= 25 and st["queued_taken_back"] == 0
    else:
        assert st["queued_steps"] == 0
    fs, ms = s.get_flags()
    assert_own_flags(s, cfg, fs, ms)


@pytest.mark.gpu
@pytest.mark.parametrize("form", [(1, 1024), (2, 256), (2, 1024), (4, 256)])
def test_queued_tile_steps_with_each_form_match_oracle(form):
    """The queued one-launch steps with the tile step's folded forms forced to each
    tiling and workgroup size: whole blocks write their flags, sub-tiles leave partial
    detail maxima that the host combines; either way the run equals the oracle bit for
    bit and the last analysis is the oracle's analysis of the final state."""
    nsub, tpb = form
    cfg = W.C2(form=W.FORM_FUSED).replace(phys=(5.0,))
    s, o = _pair(cfg)
    s.set_graph(0)
    s.set_sweep(3)
    s.tune(nsub=nsub, reps=-tpb)
    t = 0.0
    s.step(t, cfg.dt, 30)
    for _ in range(30):
        o.step(t, cfg.dt)
        t += cfg.dt
    st = s.stats()
    assert st["rk4_tile_mothers"] == [nsub, tpb] and st["rk4_tile_tiles"] == nsub
    assert st["queued_steps"] >= 25 and st["queued_taken_back"] == 0
    assert_same(s, o, f"tile form {form}: 30 steps")
    fs, ms = s.get_flags()
    assert_own_flags(s, cfg, fs, ms)
    with pytest.raises(M.MrbError):
        s.tune(nsub=4, reps=-768)    # no form has that workgroup size
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("tpb", [256, 512, 1024])
def test_queued_tile_steps_bs17_match_oracle(tpb):
    """The queued one-launch steps on 17-point blocks (constant advection): a smooth field on
    16 level-2 blocks whose refine-all and coarsening cycle (eps between the details of the
    two levels), with each compiled workgroup size; bitwise equal to the oracle."""
    fn = lambda x, y: 0.5 + 0.1 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    cfg = W.C1(jmax=4, eps=3e-6, form=W.FORM_FUSED)
    lv = np.full(16, 2, np.int8)
    co = np.array([[x, y] for y in range(4) for x in range(4)], np.int32)
    s, o = _pair(cfg, lv, co, fn=fn)
    s.set_graph(0)
    s.set_sweep(3)
    s.tune(nsub=1, reps=-tpb)
    t = 0.0
    s.step(t, cfg.dt, 20)
    for _ in range(20):
        o.step(t, cfg.dt)
        t += cfg.dt
    st = s.stats()
    assert st["rk4_tile_mothers"] == [1, tpb] and st["blocks"] == 16
    assert st["queued_steps"] >= 15 and st["queued_taken_back"] == 0
    assert_same(s, o, f"Bs 17, {tpb} threads: 20 steps")
    fs, ms = s.get_flags()
    assert_own_flags(s, cfg, fs, ms)
    s.close()


@pytest.mark.gpu
def test_graph_steps_after_autotuning_match_oracle():
    """Regression: the autotuner times the tile step's sub-tiled analyses, whose partial
    maxima are combined by the host only after a tile launch of its own; graph-replayed
    steps afterwards (their first analysis pass is the analysis kernel, which writes its
    flags itself) must keep those flags: the run equals the oracle bit for bit."""
    cfg = W.C2(form=W.FORM_FUSED)
    s, o = _pair(cfg)
    lv, co = o.read_forest()
    data = o.read_blocks()
    s.refine_all()
    s.tune(reps=2)
    s.init_forest(lv, co)
    s.load_blocks(data)
    s.set_graph(1)
    t = 0.0
    for _ in range(4):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    assert s.stats()["graph_launches"] >= 4
    assert_same(s, o, "graph steps after autotuning")
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("sweep", [2, 3])
def test_multi_step_call_after_a_perturbation_matches_oracle(sweep):
    """A perturbation between calls makes the first adapt of the next call miss its
    speculation (the host state is put back; with the one-launch tile step the step
    queued behind it is taken back as well); the run must equal the oracle's."""
    cfg = W.C2(form=W.FORM_FUSED)
    s, o = _pair(cfg)
    s.set_graph(0)
    s.set_sweep(sweep)
    t = 0.0
    s.step(t, cfg.dt, 4)
    for _ in range(4):
        o.step(t, cfg.dt)
        t += cfg.dt
    assert_same(s, o, "before the perturbation")
    lv, co = o.read_forest()
    bump = W.sample(cfg, lv, co, fn=lambda x, y: 0.5 * np.exp(-((x - 0.3) ** 2 + (y - 0.6) ** 2) / 4e-5))
    data = o.read_blocks() + bump
    s.load_blocks(data)
    o.load_blocks(data)
    miss0 = s.stats()["spec_misses"]
    s.step(t, cfg.dt, 3)
    for _ in range(3):
        o.step(t, cfg.dt)
        t += cfg.dt
    assert_same(s, o, "3 steps after the perturbation")
    assert s.stats()["spec_misses"] > miss0
    if sweep == 3:
        assert s.stats()["queued_taken_back"] >= 1


@pytest.mark.gpu
def test_headline_configuration_mixed_step_path_within_1e5():
    """The benchmark's headline run: 2D swirl at full size (Bs 33, Jmax 7, eps 1e-4),
    mixed form, autotuned tilings, the library's own step loop (memoised plans,
    speculated coarsening, automatic graph choice).  Against FP64 oracle steps: same
    forest every step, per-field error <= 1e-5 relative."""
    cfg = W.C2()
    o = oracle.Oracle(cfg)
    o.init_grid()
    lv, co = o.read_forest()
    s = M.Solver(cfg.replace(precision=W.MIXED, form=W.FORM_FUSED))
    s.init_forest(lv, co)
    s.load_blocks(o.read_blocks())
    s.refine_all()
    s.tune(reps=2)
    s.init_forest(lv, co)
    s.load_blocks(o.read_blocks())
    t, worst = 0.0, 0.0
    for n in range(30):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
        assert np.array_equal(s.read_forest()[0], o.read_forest()[0]), n
        a, b = s.read_blocks(), o.read_blocks()
        worst = max(worst, float(np.max(np.abs(a - b)) / np.max(np.abs(b))))
    st = s.stats()
    print("worst rel", worst, "spec", st["spec_hits"], "memo", st["memo_hits"], "graph", st["graph_in_use"])
    assert 0.0 < worst <= 1e-5
    assert st["spec_hits"] > 20
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("eps", [0.0, 1e30])
def test_degenerate_thresholds_match_oracle(eps):
    """eps = 0: nothing ever coarsens, the forest fills up to Jmax; eps = 1e30:
    everything coarsens down to level 1 (level-1 blocks never coarsen)."""
    cfg = W.C1(jmax=4, eps=eps)
    lv, co = W.uniform_forest(cfg, 2)
    s, o = _pair(cfg, lv, co)
    t = 0.0
    for n in range(4):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
        assert_same(s, o, f"eps {eps} step {n + 1}")
    lv, _ = s.read_forest()
    if eps == 0.0:
        assert (lv == cfg.jmax).all()
    else:
        assert (lv == 1).all()
    s.close()


def test_hip_build_flags():
    """gfx950 code objects, no FMA contraction (the FP64 path rounds as written), and
    the packed-FP32 instructions switched off."""
    from paper_1902_00088_amd import hipbuild
    f = hipbuild.HIPFLAGS
    assert "--offload-arch=gfx950" in f and "-ffp-contract=off" in f
    i = f.index("-packed-fp32-ops")
    assert f[i - 3:i] == ["-Xclang", "-target-feature", "-Xclang"]


# ------------------------------------------------------------------------------------------
# device-resident topology: plans and neighbour entries built on the GPU (mrb_set_topology)
# ------------------------------------------------------------------------------------------

@pytest.mark.gpu
@pytest.mark.parametrize("case", ["c1", "c2_deep", "c3", "c4_small"])
def test_device_topology_steps_match_oracle(case):
    """mrb_step with every refinement and coarsening planned on the device (mode 1): the
    forest, the slots' values and every step equal the oracle's bit for bit, on forests
    that change every step (narrow swirl blobs), a 3D forest and the 4-field shape."""
    if case == "c1":
        cfg, n = W.C1(form=W.FORM_FUSED), 12
    elif case == "c2_deep":
        cfg, n = W.C2(jmax=6, eps=1e-4, blob_beta=4e-4, form=W.FORM_FUSED), 8
    elif case == "c3":
        cfg, n = W.C3(jmax=5, eps=1e-4, form=W.FORM_FUSED), 3
    else:
        cfg, n = W.C4(jmax=4, eps=1e-4, form=W.FORM_FUSED).replace(max_blocks=8 ** 4 + 2000), 3
    s, o = _pair(cfg)
    s.set_topology(1)
    t = 0.0
    for k in range(n):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
        assert s.stats()["topology"] == "device"
        if k % 4 == 3 or k == n - 1:
            assert_same(s, o, f"{case}: step {k + 1}")     # pulls the forest back
    st = s.stats()
    assert st["device_topology"]["steps"] == n and st["device_topology"]["pushes"] >= 1
    s.close()


@pytest.mark.gpu
def test_device_and_host_topology_agree_and_hand_over():
    """Steps alternate between device and host planning (each switch moves the forest
    across); the result equals a run planned on the host only, slots and flags included."""
    cfg = W.C2(jmax=6, eps=1e-4, blob_beta=4e-4, form=W.FORM_FUSED)
    a, b = M.Solver(cfg), M.Solver(cfg)
    for s in (a, b):
        s.init_grid()
        s.set_graph(0)
    a.set_topology(0)
    t = 0.0
    for k in range(8):
        b.set_topology(1 if k % 3 != 2 else 0)
        a.step(t, cfg.dt)
        b.step(t, cfg.dt)
        t += cfg.dt
    la, lb = a.read_forest(), b.read_forest()
    assert np.array_equal(la[0], lb[0]) and np.array_equal(la[1], lb[1])
    assert np.array_equal(_bits(a.read_blocks()), _bits(b.read_blocks()))
    fa, ma = a.get_flags()
    fb, mb = b.get_flags()
    assert np.array_equal(fa, fb) and np.array_equal(_bits(ma), _bits(mb))
    st = b.stats()
    assert st["device_topology"]["pushes"] >= 2 and st["device_topology"]["pulls"] >= 2
    with pytest.raises(M.MrbError):
        b.set_topology(3)
    a.close()
    b.close()


@pytest.mark.gpu
def test_device_topology_capacity_error_leaves_state():
    """A refinement that does not fit the pool fails with MRB_E_CAPACITY before any
    device write; the forest and values are unchanged."""
    cfg = W.C1(jmax=4, eps=0.0, form=W.FORM_FUSED).replace(max_blocks=80)
    s = M.Solver(cfg)
    lv, co = W.uniform_forest(cfg, 2)
    s.init_forest(lv, co)
    s.load_blocks(W.sample(cfg, *s.read_forest()))
    s.set_topology(1)
    s.step(0.0, cfg.dt)                                  # 16 -> 64 blocks on level 3
    before = s.read_blocks()
    lvb, cob = s.read_forest()
    with pytest.raises(M.MrbError) as e:
        s.step(cfg.dt, cfg.dt)                           # 64 -> 256 does not fit in 80
    assert e.value.code == -2
    assert np.array_equal(s.read_forest()[0], lvb) and np.array_equal(s.read_forest()[1], cob)
    assert np.array_equal(_bits(s.read_blocks()), _bits(before))
    s.close()
