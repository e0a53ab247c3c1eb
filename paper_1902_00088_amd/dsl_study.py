"""The paper's double shear layer (Sec. 4, Figs. 5-6) on the GPU path.

Compressible Navier-Stokes on [0, 8]^2 (scaled to the solver's unit square: x = 8 x',
t = 8 t', viscosity mu/8), two shear layers at L/2 +- 0.25 with tanh jumps of width L/240,
rho 2 and u 1 between them, rho 1 and u -1 outside, p = 2.5, a sinusoidal v disturbance of
amplitude 0.1, mu = 1e-6, gamma 1.4, Pr 0.71, 4th-order FD, RK4, and a shock-capturing
filter with threshold r_th = 1e-5 after every step (the formulation is ours: the cited
filter is not available).  Runs to t = 4 on a fixed grid and on adaptive grids (eps 1e-3),
then reads the solution on the uniform lattice of a fixed level -- leaves coarser than that
level are refined for the read, as the paper does before taking spectra -- and returns the
kinetic-energy spectrum E(k) = sum over |k'| in [k - 1/2, k + 1/2) of (|u^(k')|^2 +
|v^(k')|^2) / 2 (velocity Fourier coefficients normalised by the number of points, k in
units of 2 pi / L), and the compression rate over time (blocks relative to the uniform grid
on Jmax).  Every step runs in the library's kernels; the spectrum is post-processing of the
read-back field.

Usage: python -m paper_1902_00088_amd.dsl_study [--quick] > dsl.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

import workloads as W


def spectrum(uv: np.ndarray):
    """E(k), k = 0..N/2, from the velocity components uv[0] = u, uv[1] = v on an N x N lattice."""
    n = uv.shape[-1]
    e2 = np.zeros((n, n))
    for c in uv:
        f = np.fft.fft2(c) / (n * n)
        e2 += 0.5 * np.abs(f) ** 2
    k = np.fft.fftfreq(n, 1.0 / n)
    kk = np.sqrt(k[None, :] ** 2 + k[:, None] ** 2)
    shell = np.rint(kk).astype(int)
    return np.bincount(shell.ravel(), weights=e2.ravel(), minlength=n // 2 + 1)[: n // 2 + 1]


def run(M, cfg, read_level: int, chunk: int = 64):
    """From the initial grid to the configuration's end time; spectrum on the uniform
    lattice of read_level and the compression rate sampled every chunk steps."""
    import torch
    s = M.Solver(cfg)
    s.set_graph(0)
    s.init_grid()
    counts = [s.num_blocks()]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < cfg.steps:
        k = min(chunk, cfg.steps - done)
        s.step(done * cfg.dt, cfg.dt, k)
        done += k
        counts.append(s.num_blocks())
        if done % 2048 == 0:
            print(json.dumps({"jmax": cfg.jmax, "steps_done": done, "of": cfg.steps, "blocks": counts[-1],
                              "s": round(time.perf_counter() - t0, 1)}), flush=True, file=sys.stderr)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fields = s.read_uniform(read_level)
    s.close()
    spec = spectrum(fields[1:3])
    return {"jmax": cfg.jmax, "eps": cfg.eps, "steps": cfg.steps, "t_end": cfg.steps * cfg.dt * W.DSL_L,
            "read_level": read_level, "gpu_wall_s": wall, "ms_per_step": 1e3 * wall / cfg.steps,
            "compression": [c / 4 ** cfg.jmax for c in counts], "compression_final": counts[-1] / 4 ** cfg.jmax,
            "rho_range": [float(fields[0].min()), float(fields[0].max())],
            "spectrum": spec.tolist()}


def study(M, quick: bool = False, precision: int = W.MIXED):
    """Fixed grid on level J = 7 and adaptive grids (eps 1e-3) with Jmax 7 and 8, to t = 4
    (Fig. 6); the quick form takes J = 4 to t = 0.5."""
    j, t_end = (4, 0.5) if quick else (7, 4.0)
    out = {"set_up": "Sec. 4 double shear layer, L = 8, filter r_th = 1e-5, t = %g" % t_end, "runs": []}
    cases = [("fixed", W.DSL(jmax=j, eps=0.0, t_end=t_end)),
             ("adaptive", W.DSL(jmax=j, eps=1e-3, t_end=t_end)),
             ("adaptive", W.DSL(jmax=j + 1, eps=1e-3, t_end=t_end))]
    for name, cfg in cases:
        # each run steps with the time step of its own finest level (global time stepping)
        r = run(M, cfg.replace(precision=precision, form=W.FORM_FUSED), j)
        r["kind"] = name
        out["runs"].append(r)
        print(json.dumps({k: v for k, v in r.items() if k not in ("spectrum", "compression")}), flush=True,
              file=sys.stderr)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    import paper_1902_00088_amd as M
    print(json.dumps(study(M, quick=args.quick)), flush=True)


if __name__ == "__main__":
    main()
