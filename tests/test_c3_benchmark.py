"""Parity of the Navier-Stokes mixing layer at the benchmark's size (C3: Bs 33, four
fields, halo 4, Jmax 8, eps 1e-3, Re 1000, Mach 0.4, the benchmark's time step): the
oracle's initial grid (64 blocks on level 3, 256 on level 4 after the safety-zone
refinement, all of them coarsened back by the adapt), advanced through the step of
Sec. 2.1 piece by piece and by the library's own step loop.

FP64 (fused and plain forms): bit for bit (fields, flags, detail maxima, forests).  Mixed
form (FP64 tile, FP32 after the neighbour differences, FP64 state): per-field error
against the FP64 oracle <= 1e-5 relative on the oracle's topology, for whole blocks with
the workgroup sizes the autotuner chooses between; the flags of the mixed state's own
analysis are checked against the oracle's analysis of that state.

The oracle's reference states take about a second of host time.
"""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_1902_00088_amd as M

from test_library import _bits, assert_own_flags

CFG = W.C3()


@pytest.fixture(scope="module")
def ref():
    """The oracle's states along two steps from its initial grid."""
    o = oracle.Oracle(CFG)
    o.init_grid()
    r = {"lv0": o.read_forest()[0], "co0": o.read_forest()[1], "u0": o.read_blocks()}
    o.refine_all()
    r["lvR"], r["coR"] = o.read_forest()
    r["uR"] = o.read_blocks()
    o.rk4(0.0, CFG.dt)
    r["uK"] = o.read_blocks()
    r["f1"], r["m1"] = o.mr_pass()
    r["uA"] = o.read_blocks()
    flags = [r["f1"]]
    while o.coarsen(flags[-1]) > 0:
        f, _ = o.mr_pass()
        flags.append(f)
    r["flags"] = flags
    r["lv1"], r["co1"] = o.read_forest()
    r["u1"] = o.read_blocks()
    o.step(CFG.dt, CFG.dt)
    r["lv2"], r["co2"] = o.read_forest()
    r["u2"] = o.read_blocks()
    return r


def _start(cfg, r):
    s = M.Solver(cfg)
    s.init_forest(r["lv0"], r["co0"])
    s.load_blocks(r["u0"])
    return s


def _same_forest(s, lv, co, what):
    a, b = s.read_forest()
    assert np.array_equal(a, lv) and np.array_equal(b, co), f"forest differs {what}"


def _bitwise(s, want, what):
    got = s.read_blocks()
    if not np.array_equal(_bits(got), _bits(want)):
        bad = np.argwhere(_bits(got) != _bits(want))
        raise AssertionError(f"values differ {what}: max abs {np.max(np.abs(got - want))}, n={len(bad)}")


def _rel_per_field(got, want):
    """Max relative error of each field (arrays [block][field][node])."""
    return [float(np.max(np.abs(got[:, f] - want[:, f])) / np.max(np.abs(want[:, f]))) for f in range(got.shape[1])]


@pytest.mark.gpu
def test_c3_forest_shape(ref):
    assert len(ref["lv0"]) == 64 and len(ref["lvR"]) == 256
    assert sorted(np.unique(ref["lvR"]).tolist()) == [4]
    assert len(ref["lv1"]) == 64


@pytest.mark.gpu
@pytest.mark.parametrize("form", [W.FORM_FUSED, W.FORM_PLAIN])
def test_c3_fp64_step_pieces_are_bitwise(ref, form):
    """Safety-zone refinement, RK4 sweep, first analysis and the adapt, each compared."""
    cfg = CFG.replace(form=form)
    s = _start(cfg, ref)
    s.refine_all()
    _same_forest(s, ref["lvR"], ref["coR"], "after refine_all")
    _bitwise(s, ref["uR"], "after refine_all")
    s.rk4(0.0, cfg.dt)
    _bitwise(s, ref["uK"], "after rk4")
    f, m = s.mr_pass()
    assert np.array_equal(f, ref["f1"]) and np.array_equal(_bits(m), _bits(ref["m1"]))
    _bitwise(s, ref["uA"], "after the first analysis")
    s.adapt()
    _same_forest(s, ref["lv1"], ref["co1"], "after adapt")
    _bitwise(s, ref["u1"], "after adapt")
    s.close()


@pytest.mark.gpu
def test_c3_fp64_library_step_loop_autotuned_is_bitwise(ref):
    """The benchmark's path: autotuned tilings and workgroup sizes, the library's step
    loop (graph replay or direct launches, whichever it picks), two steps."""
    cfg = CFG.replace(form=W.FORM_FUSED)
    s = _start(cfg, ref)
    s.refine_all()
    s.tune(reps=1)
    s.init_forest(ref["lv0"], ref["co0"])
    s.load_blocks(ref["u0"])
    s.step(0.0, cfg.dt, 2)
    _same_forest(s, ref["lv2"], ref["co2"], "after two steps")
    _bitwise(s, ref["u2"], "after two steps")
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("threads", [256, 1024])
def test_c3_mixed_within_1e5_on_oracle_topology(ref, threads):
    """Mixed form at the benchmark size, whole blocks with 256 or 1,024 threads (the
    benchmark's autotuner takes 1,024), per field."""
    cfg = CFG.replace(precision=W.MIXED, form=W.FORM_FUSED)
    s = _start(cfg, ref)
    assert s.tune(nsub=1, reps=-threads) == 1
    s.refine_all()
    _same_forest(s, ref["lvR"], ref["coR"], "after refine_all")
    _bitwise(s, ref["uR"], "after refine_all (FP64 in both forms)")
    s.rk4(0.0, cfg.dt)
    rel = _rel_per_field(s.read_blocks(), ref["uK"])
    assert max(rel) <= 1e-5 and max(rel) > 0.0, rel
    for i, fo in enumerate(ref["flags"]):
        fs, ms = s.mr_pass()
        assert_own_flags(s, cfg, fs, ms)
        n = s.coarsen(fo)
        assert (n == 0) == (i == len(ref["flags"]) - 1)
    _same_forest(s, ref["lv1"], ref["co1"], "after the replayed adapt")
    rel = _rel_per_field(s.read_blocks(), ref["u1"])
    assert max(rel) <= 1e-5 and max(rel) > 0.0, rel
    s.close()
