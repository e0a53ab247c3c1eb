"""The paper's swirl test (Sec. 3, Fig. 4) on the GPU path: the time-dependent field with
t_a = 5 (factor cos(pi t/t_a) per RK stage).

Parity: the set-up equals the oracle bit for bit.  Study (reduced to Jmax 3-4, reference
on a uniform Jmax-6 grid): at t_a/2 the error decreases as eps decreases (Fig. 4A), the
compression rate grows as eps -> 0 (Fig. 4C), at eps = 1e-7 the error falls by more than
a factor 8 from Jmax 3 to 4 (Fig. 4B: order ~4), and at t_a the solution is back at the
initial condition within the threshold's error (reversal).
"""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_1902_00088_amd as M
from paper_1902_00088_amd import swirl_study as S


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def test_swirl_study_configuration():
    cfg = S.swirl_config(4, 1e-3, 1e-2)
    assert cfg.bs == 33 and cfg.phys[0] == 5.0 and cfg.physics == W.ADV_SWIRL
    assert np.allclose(cfg.blob_centers, [[0.5, 0.75]]) and cfg.blob_beta == 1e-2
    assert cfg.steps * cfg.dt == 5.0     # binary-exact dt: the run ends exactly at t_a


@pytest.mark.gpu
def test_reversal_setup_matches_oracle():
    cfg = S.swirl_config(3, 1e-3, 1e-2)
    s, o = M.Solver(cfg), oracle.Oracle(cfg)
    s.set_graph(0)
    s.init_grid()
    o.init_grid()
    t = 0.0
    for k in range(60):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    lv1, co1 = s.read_forest()
    lv2, co2 = o.read_forest()
    assert np.array_equal(lv1, lv2) and np.array_equal(co1, co2)
    assert np.array_equal(_bits(s.read_blocks()), _bits(o.read_blocks()))
    s.close()


@pytest.mark.gpu
def test_swirl_study_trends():
    out = S.study(M, quick=True)
    runs = {(r["jmax"], r["eps"]): r for r in out["runs"]}
    for j in (3, 4):
        assert runs[(j, 1e-2)]["rel_err_half"] > runs[(j, 1e-4)]["rel_err_half"]
        assert runs[(j, 1e-7)]["compression_mean"] >= runs[(j, 1e-2)]["compression_mean"]
        assert runs[(j, 1e-7)]["rel_err_reversal"] < 1e-4
    assert runs[(3, 1e-7)]["rel_err_half"] > 8 * runs[(4, 1e-7)]["rel_err_half"]
    print(out["fits"])
