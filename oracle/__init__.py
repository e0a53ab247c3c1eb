"""CPU oracle for the block-based multiresolution solver (arXiv 1902.00088).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The GPU library never imports this
package and this package never imports the GPU library; the two share only the
seeded input generators in ``workloads``.

The arithmetic lives in ``oracle.cpp`` (FP64, pointwise definitions, see its
header for the passages each part follows).  This module is a ctypes wrapper
plus the initial-grid procedure (Sec. 2.1, initialisation): start from the
uniform level-1 forest, then repeat {refine all, resample the analytic initial
condition, adapt, resample} until the forest stops changing.

parity unpinned: the Navier-Stokes right-hand side (a formulation of our own;
free-stream preservation, mass conservation and single-mode closed forms of each
term pin it, nothing beyond them).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "oracle.cpp")

_dp = ctypes.POINTER(ctypes.c_double)
_i8p = ctypes.POINTER(ctypes.c_int8)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no FMA contraction, so every product and sum
    is rounded exactly as written)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", LIB_PATH + ".tmp", SRC]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int] * 5 + [ctypes.c_double, ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, _dp]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_error.restype = ctypes.c_char_p
        L.orc_error.argtypes = [ctypes.c_void_p]
        for name, args in [
            ("orc_init_forest", [ctypes.c_void_p, ctypes.c_int, _i8p, _i32p]),
            ("orc_num_blocks", [ctypes.c_void_p]),
            ("orc_read_forest", [ctypes.c_void_p, _i8p, _i32p]),
            ("orc_load", [ctypes.c_void_p, _dp]),
            ("orc_read_blocks", [ctypes.c_void_p, _dp]),
            ("orc_read_stored", [ctypes.c_void_p, _dp]),
            ("orc_tile", [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp]),
            ("orc_rhs", [ctypes.c_void_p, ctypes.c_double, _dp]),
            ("orc_rk4", [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]),
            ("orc_refine_all", [ctypes.c_void_p]),
            ("orc_refine_marked", [ctypes.c_void_p, _i8p]),
            ("orc_mr_pass", [ctypes.c_void_p, _i8p, _dp]),
            ("orc_details", [ctypes.c_void_p, _dp]),
            ("orc_read_uniform", [ctypes.c_void_p, ctypes.c_int, _dp]),
            ("orc_filter", [ctypes.c_void_p, ctypes.c_double]),
            ("orc_coarsen", [ctypes.c_void_p, _i8p]),
            ("orc_coarsenable", [ctypes.c_void_p, _i8p, _i8p, _i32p]),
            ("orc_adapt", [ctypes.c_void_p, ctypes.c_int]),
        ]:
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = args
        L.orc_p4.restype = ctypes.c_double
        L.orc_p4.argtypes = [ctypes.c_double] * 4
        L.orc_d4.restype = ctypes.c_double
        L.orc_d4.argtypes = [ctypes.c_double] * 5
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def p4(a, b, c, d) -> float:
    return lib().orc_p4(a, b, c, d)


def d4(um2, um1, up1, up2, r) -> float:
    return lib().orc_d4(um2, um1, up1, up2, r)


class OracleError(RuntimeError):
    pass


class Oracle:
    """Same method names as the GPU library's Python binding."""

    def __init__(self, cfg: W.Config):
        self.cfg = cfg
        L = lib()
        phys = np.ascontiguousarray(np.asarray(cfg.phys, dtype=np.float64))
        s2 = s = None
        if cfg.physics == W.ADV_SWIRL:
            s2, s = W.swirl_tables(cfg)
        scale = None if cfg.field_scale is None else np.ascontiguousarray(np.asarray(cfg.field_scale, dtype=np.float64))
        self._keep = (phys, s2, s, scale)
        self.h = L.orc_create(cfg.dim, cfg.bs, cfg.hw, cfg.nf, cfg.jmax, cfg.eps, cfg.physics,
                              _ptr(phys, _dp), len(phys), _ptr(s2, _dp), _ptr(s, _dp), _ptr(scale, _dp))
        self.t = 0.0

    def __del__(self):
        try:
            if self.h:
                lib().orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _chk(self, rc):
        if rc < 0:
            raise OracleError(lib().orc_error(self.h).decode())
        return rc

    # ---- forest and data -------------------------------------------------------------
    def init_forest(self, levels, coords):
        levels = np.ascontiguousarray(np.asarray(levels, dtype=np.int8))
        coords = np.ascontiguousarray(np.asarray(coords, dtype=np.int32).reshape(len(levels), self.cfg.dim))
        self._chk(lib().orc_init_forest(self.h, len(levels), _ptr(levels, _i8p), _ptr(coords, _i32p)))

    def num_blocks(self) -> int:
        return lib().orc_num_blocks(self.h)

    def read_forest(self):
        n = self.num_blocks()
        lv = np.zeros(n, dtype=np.int8)
        co = np.zeros((n, self.cfg.dim), dtype=np.int32)
        self._chk(lib().orc_read_forest(self.h, _ptr(lv, _i8p), _ptr(co, _i32p)))
        return lv, co

    def load_blocks(self, data):
        data = np.ascontiguousarray(np.asarray(data, dtype=np.float64))
        assert data.shape == (self.num_blocks(), self.cfg.nf, self.cfg.npts), data.shape
        self._chk(lib().orc_load(self.h, _ptr(data, _dp)))

    def read_blocks(self):
        out = np.zeros((self.num_blocks(), self.cfg.nf, self.cfg.npts))
        self._chk(lib().orc_read_blocks(self.h, _ptr(out, _dp)))
        return out

    def read_stored(self):
        out = np.zeros((self.num_blocks(), self.cfg.nf, self.cfg.npts))
        self._chk(lib().orc_read_stored(self.h, _ptr(out, _dp)))
        return out

    def read_uniform(self, level: int):
        """The synchronised solution on the uniform level-`level` lattice: [nf][N]*dim, x fastest."""
        nl = (2 ** level) * (self.cfg.bs - 1)
        out = np.zeros((self.cfg.nf,) + (nl,) * self.cfg.dim)
        self._chk(lib().orc_read_uniform(self.h, level, _ptr(out, _dp)))
        return out

    def filter(self, rth: float):
        """The shock-capturing filter (Navier-Stokes) alone on the current state."""
        self._chk(lib().orc_filter(self.h, rth))

    def tile(self, bi: int, halo: int):
        w = self.cfg.bs + 2 * halo
        out = np.zeros((self.cfg.nf,) + (w,) * self.cfg.dim)
        self._chk(lib().orc_tile(self.h, bi, halo, _ptr(out, _dp)))
        return out

    def rhs(self, t: float = 0.0):
        out = np.zeros((self.num_blocks(), self.cfg.nf, self.cfg.npts))
        self._chk(lib().orc_rhs(self.h, t, _ptr(out, _dp)))
        return out

    # ---- the method ------------------------------------------------------------------
    def refine_all(self):
        self._chk(lib().orc_refine_all(self.h))

    def refine_marked(self, mask) -> int:
        """Refine the marked leaves (forest order) and every coarser leaf that must
        follow for the grid to stay graded; returns the number refined."""
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.int8))
        assert len(m) == self.num_blocks()
        return self._chk(lib().orc_refine_marked(self.h, _ptr(m, _i8p)))

    def rk4(self, t: float, dt: float):
        self._chk(lib().orc_rk4(self.h, t, dt))

    def mr_pass(self):
        n = self.num_blocks()
        fl = np.zeros(n, dtype=np.int8)
        md = np.zeros((n, self.cfg.nf))
        self._chk(lib().orc_mr_pass(self.h, _ptr(fl, _i8p), _ptr(md, _dp)))
        return fl, md

    def details(self):
        """Per-node details d = u - P(R(u)) of the last mr_pass: [n][nf][bs^dim] (0 at all-even nodes)."""
        out = np.zeros((self.num_blocks(), self.cfg.nf, self.cfg.npts))
        self._chk(lib().orc_details(self.h, _ptr(out, _dp)))
        return out

    def coarsen(self, flags) -> int:
        fl = np.ascontiguousarray(np.asarray(flags, dtype=np.int8))
        assert len(fl) == self.num_blocks()
        return self._chk(lib().orc_coarsen(self.h, _ptr(fl, _i8p)))

    def coarsenable(self, flags):
        fl = np.ascontiguousarray(np.asarray(flags, dtype=np.int8))
        n = self.num_blocks()
        lv = np.zeros(n, dtype=np.int8)
        co = np.zeros((n, self.cfg.dim), dtype=np.int32)
        k = self._chk(lib().orc_coarsenable(self.h, _ptr(fl, _i8p), _ptr(lv, _i8p), _ptr(co, _i32p)))
        return {(int(lv[i]),) + tuple(int(c) for c in co[i]) for i in range(k)}

    def adapt(self, max_passes: int = 0) -> int:
        return self._chk(lib().orc_adapt(self.h, max_passes))

    def step(self, t: float, dt: float) -> int:
        """One MR time step (Sec. 2.1): refine all, RK4 on the refined grid, coarsen."""
        self.refine_all()
        self.rk4(t, dt)
        return self.adapt()

    def init_grid(self, fn=None, max_iter: int = 0):
        """Initial adaptive grid for the analytic initial condition of the workload."""
        cfg = self.cfg
        lv, co = W.uniform_forest(cfg, 1)
        self.init_forest(lv, co)
        self.load_blocks(W.sample(cfg, *self.read_forest(), fn=fn))
        prev = None
        for _ in range(max_iter or cfg.jmax + 1):
            self.refine_all()
            self.load_blocks(W.sample(cfg, *self.read_forest(), fn=fn))
            self.adapt()
            lv, co = self.read_forest()
            self.load_blocks(W.sample(cfg, lv, co, fn=fn))
            key = (lv.tobytes(), co.tobytes())
            if key == prev:
                break
            prev = key
