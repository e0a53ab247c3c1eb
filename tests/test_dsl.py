"""The paper's double shear layer (Sec. 4): set-up, shock-capturing filter parity, spectra.

The filter and the mapping of the paper's [0, 8]^2 onto the solver's unit square are
readings (the cited filter is not available; see the oracle's pins for the filter)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
import paper_1902_00088_amd as M
from paper_1902_00088_amd import dsl_study as D


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def test_dsl_configuration_and_initial_state():
    cfg = W.DSL(jmax=7)
    assert cfg.physics == W.NS2D and cfg.nf == 4 and cfg.hw == 4 and cfg.bs == 33
    assert cfg.phys[0] == 1.4 and cfg.phys[2] == 0.71 and cfg.phys[3] == 1e-5
    assert cfg.phys[1] == 1e-6 / 8.0                       # mu / L on the unit square
    assert cfg.steps * cfg.dt * W.DSL_L >= 4.0 > (cfg.steps - 1) * cfg.dt * W.DSL_L
    y = np.linspace(0.0, 1.0, 2001)
    rho, u, v, p = W.double_shear_layer_fields(cfg, np.full_like(y, 0.3), y)
    assert abs(rho[0] - rho[-1]) < 1e-12 and abs(u[0] - u[-1]) < 1e-12     # periodic in y
    mid = np.argmin(np.abs(y - 0.5))
    assert abs(rho[mid] - 2.0) < 1e-5 and abs(u[mid] - 1.0) < 1e-5         # between the layers
    assert abs(rho[0] - 1.0) < 1e-12 and abs(u[0] + 1.0) < 1e-12           # outside
    assert np.all(p == 2.5)
    x = np.linspace(0.0, 1.0, 9)
    _, _, v, _ = W.double_shear_layer_fields(cfg, x, np.full_like(x, 0.1))
    assert np.allclose(v, 0.1 * np.sin(2 * math.pi * (8 * x - 4)), atol=1e-15)


def test_spectrum_of_a_single_mode():
    """One Fourier mode of amplitude 1 in u carries E = 1/4 at its shell and nothing else."""
    n, k0 = 64, 5
    i = np.arange(n)
    u = np.cos(2 * np.pi * k0 * i / n)[None, :].repeat(n, 0)
    e = D.spectrum(np.stack([u, np.zeros_like(u)]))
    assert abs(e[k0] - 0.25) < 1e-14 and abs(e.sum() - 0.25) < 1e-14


@pytest.mark.gpu
@pytest.mark.parametrize("rth", [1e-5, 1e-11])
def test_dsl_steps_with_filter_match_oracle(rth):
    """FP64 steps of the shear layer with the filter after every RK4 step (the small
    threshold switches the sensor on across the layers) equal the oracle bit for bit."""
    cfg = W.DSL(jmax=4, eps=1e-3, rth=rth, form=W.FORM_FUSED)
    s, o = M.Solver(cfg), oracle.Oracle(cfg)
    s.set_graph(0)
    s.init_grid()
    o.init_grid()
    lv, co = s.read_forest()
    assert np.array_equal(lv, o.read_forest()[0])
    t = 0.0
    for k in range(4):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    assert np.array_equal(s.read_forest()[0], o.read_forest()[0])
    a, b = s.read_blocks(), o.read_blocks()
    assert np.array_equal(_bits(a), _bits(b)), np.max(np.abs(a - b))
    s.close()


@pytest.mark.gpu
def test_dsl_quick_study_spectra_agree_on_resolved_scales():
    out = D.study(M, quick=True)
    fixed, ad1, ad2 = out["runs"]
    assert fixed["kind"] == "fixed" and ad1["kind"] == "adaptive"
    assert fixed["compression_final"] == 1.0
    e0, e1, e2 = (np.array(r["spectrum"]) for r in (fixed, ad1, ad2))
    n = len(e0)
    low = slice(1, n // 4)
    # adaptive and fixed grids carry the same energy on the well-resolved scales
    assert np.all(np.abs(e1[low] - e0[low]) <= 0.05 * e0[low] + 1e-12)
    assert np.all(np.abs(e2[low] - e0[low]) <= 0.05 * e0[low] + 1e-12)
    # no blow-up: the density stays near its initial range [1, 2] (Gibbs overshoot of the
    # under-resolved jumps aside)
    for r in out["runs"]:
        assert 0.8 < r["rho_range"][0] and r["rho_range"][1] < 2.3, r["rho_range"]
