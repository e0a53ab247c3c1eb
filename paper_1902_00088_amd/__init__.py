"""MI355X block-multiresolution solver (arXiv 1902.00088): Python binding.

A thin ctypes layer over the C ABI in ``include/mrb.h`` (``libmrb.so``, built
in-tree for gfx950 by :func:`paper_1902_00088_amd.build`, which drives
:mod:`paper_1902_00088_amd.hipbuild`).  PyTorch supplies the
device pool arrays and the stream; every step of the method runs in the HIP
kernels of the library.  There is no CPU fallback: importing works anywhere,
but creating a :class:`Solver` needs the built library and a GPU, and raises
otherwise.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrb.so")

MRB_OK = 0
STATUS = {0: "MRB_OK", -1: "MRB_E_ARG", -2: "MRB_E_CAPACITY", -3: "MRB_E_TOPOLOGY",
          -4: "MRB_E_STATE", -5: "MRB_E_DEVICE", -6: "MRB_E_NONFINITE"}

# entry points declared in include/mrb.h
EXPORTS = ("mrb_create", "mrb_destroy", "mrb_last_error", "mrb_init_forest", "mrb_load_blocks",
           "mrb_refine_all", "mrb_rk4", "mrb_mr_pass", "mrb_coarsen", "mrb_adapt", "mrb_step",
           "mrb_num_blocks", "mrb_read_forest", "mrb_read_blocks", "mrb_get_flags", "mrb_stats",
           "mrb_timing", "mrb_tune", "mrb_set_graph", "mrb_set_sweep", "mrb_mlp_init", "mrb_mlp_get_params", "mrb_mlp_features",
           "mrb_mlp_forward", "mrb_mlp_grad", "mrb_mlp_train", "mrb_mlp_predict", "mrb_refine_marked",
           "mrb_step_predicted", "mrb_horizon_labels", "mrb_read_uniform", "mrb_mr_pass_noalloc",
           "mrb_set_topology")


class MrbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class mrb_config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("bs", ctypes.c_int), ("hw", ctypes.c_int), ("nfields", ctypes.c_int),
                ("jmax", ctypes.c_int), ("max_blocks", ctypes.c_int), ("eps", ctypes.c_double),
                ("physics", ctypes.c_int), ("phys", ctypes.c_double * 8),
                ("swirl_s2", ctypes.POINTER(ctypes.c_double)), ("swirl_s", ctypes.POINTER(ctypes.c_double)),
                ("field_scale", ctypes.POINTER(ctypes.c_double)), ("field_offset", ctypes.POINTER(ctypes.c_double)),
                ("precision", ctypes.c_int), ("form", ctypes.c_int)]


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i8p = ctypes.POINTER(ctypes.c_int8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p
_lib = None


def build(verbose: bool = False) -> str:
    from . import hipbuild as _b
    return _b.build(verbose=verbose)


def lib():
    """Load libmrb.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it with paper_1902_00088_amd.build()")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "mrb_create": [ctypes.POINTER(mrb_config), _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)],
            "mrb_destroy": [_vp],
            "mrb_init_forest": [_vp, ctypes.c_int, _i8p, _i32p],
            "mrb_load_blocks": [_vp, _vp, ctypes.c_int],
            "mrb_refine_all": [_vp],
            "mrb_rk4": [_vp, ctypes.c_double, ctypes.c_double],
            "mrb_mr_pass": [_vp, _i8p, _dp],
            "mrb_mr_pass_noalloc": [_vp, _i8p, _dp],
            "mrb_coarsen": [_vp, _i8p, ctypes.POINTER(ctypes.c_int)],
            "mrb_adapt": [_vp, ctypes.POINTER(ctypes.c_int)],
            "mrb_step": [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_int],
            "mrb_num_blocks": [_vp, ctypes.POINTER(ctypes.c_int)],
            "mrb_read_forest": [_vp, _i8p, _i32p],
            "mrb_read_blocks": [_vp, _vp, ctypes.c_int],
            "mrb_read_uniform": [_vp, ctypes.c_int, _vp, ctypes.c_int],
            "mrb_get_flags": [_vp, _i8p, _dp],
            "mrb_stats": [_vp, ctypes.c_char_p, ctypes.c_int],
            "mrb_timing": [_vp, ctypes.c_int],
            "mrb_tune": [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_int)],
            "mrb_set_graph": [_vp, ctypes.c_int],
            "mrb_set_sweep": [_vp, ctypes.c_int],
            "mrb_set_topology": [_vp, ctypes.c_int],
            "mrb_mlp_init": [_vp, ctypes.c_int, _fp, _fp, _fp],
            "mrb_mlp_get_params": [_vp, _fp],
            "mrb_mlp_features": [_vp, _fp],
            "mrb_mlp_forward": [_vp, _fp, ctypes.c_int, _fp],
            "mrb_mlp_grad": [_vp, _fp, _i8p, _fp, ctypes.c_int, _fp, _fp],
            "mrb_mlp_train": [_vp, _fp, _i8p, _fp, ctypes.c_int, ctypes.c_int, ctypes.c_float, _fp],
            "mrb_mlp_predict": [_vp, _i8p, _fp],
            "mrb_refine_marked": [_vp, _i8p, ctypes.POINTER(ctypes.c_int)],
            "mrb_step_predicted": [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_float, ctypes.c_float,
                                   ctypes.POINTER(ctypes.c_int)],
            "mrb_horizon_labels": [ctypes.c_int, ctypes.c_int, _i8p, _i32p, ctypes.c_int, _i8p, _i32p, _i8p],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.mrb_last_error.argtypes = [_vp]
        L.mrb_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


class Solver:
    """One solver context on the current CUDA (HIP) stream of ``device``."""

    def __init__(self, cfg: W.Config, device: str = "cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the solver runs only on the HIP device")
        L = lib()
        self.cfg = cfg
        self.torch = torch
        self.device = torch.device(device)
        n = cfg.max_blocks * cfg.nf * cfg.npts
        kdt = torch.float64 if cfg.precision == W.FP64 else torch.float32
        with torch.cuda.device(self.device):
            # a stream of its own (default priority): graph capture needs a non-default stream
            self.stream = torch.cuda.Stream(self.device)
            self.u = torch.zeros(n, dtype=torch.float64, device=self.device)
            self.u_new = torch.zeros(n, dtype=torch.float64, device=self.device)
            self.k = [torch.zeros(n, dtype=kdt, device=self.device) for _ in range(3)]
            torch.cuda.synchronize(self.device)
        c = mrb_config()
        c.dim, c.bs, c.hw, c.nfields, c.jmax, c.max_blocks = cfg.dim, cfg.bs, cfg.hw, cfg.nf, cfg.jmax, cfg.max_blocks
        c.eps = cfg.eps
        c.physics = cfg.physics
        for i, v in enumerate(list(cfg.phys)[:8]):
            c.phys[i] = float(v)
        keep = []
        if cfg.physics == W.ADV_SWIRL:
            s2, s = W.swirl_tables(cfg)
            keep += [s2, s]
            c.swirl_s2, c.swirl_s = _ptr(s2, _dp), _ptr(s, _dp)
        if cfg.field_scale is not None:
            a = np.ascontiguousarray(np.asarray(cfg.field_scale, dtype=np.float64))
            keep.append(a)
            c.field_scale = _ptr(a, _dp)
        if cfg.field_offset is not None:
            a = np.ascontiguousarray(np.asarray(cfg.field_offset, dtype=np.float64))
            keep.append(a)
            c.field_offset = _ptr(a, _dp)
        c.precision, c.form = cfg.precision, cfg.form
        h = _vp()
        rc = L.mrb_create(ctypes.byref(c), self.u.data_ptr(), self.u_new.data_ptr(), self.k[0].data_ptr(),
                          self.k[1].data_ptr(), self.k[2].data_ptr(), _vp(self.stream.cuda_stream), ctypes.byref(h))
        self.h = h
        if rc != MRB_OK:
            msg = L.mrb_last_error(h).decode() if h.value else "mrb_create failed"
            if h.value:
                L.mrb_destroy(h)
            self.h = None
            raise MrbError(rc, msg)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().mrb_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != MRB_OK:
            raise MrbError(rc, lib().mrb_last_error(self.h).decode())
        return rc

    # ---- forest and data ----------------------------------------------------------------
    def init_forest(self, levels, coords):
        lv = np.ascontiguousarray(np.asarray(levels, dtype=np.int8))
        co = np.ascontiguousarray(np.asarray(coords, dtype=np.int32).reshape(len(lv), self.cfg.dim))
        self._chk(lib().mrb_init_forest(self.h, len(lv), _ptr(lv, _i8p), _ptr(co, _i32p)))

    def num_blocks(self) -> int:
        n = ctypes.c_int()
        self._chk(lib().mrb_num_blocks(self.h, ctypes.byref(n)))
        return n.value

    def read_forest(self):
        n = self.num_blocks()
        lv = np.zeros(n, dtype=np.int8)
        co = np.zeros((n, self.cfg.dim), dtype=np.int32)
        self._chk(lib().mrb_read_forest(self.h, _ptr(lv, _i8p), _ptr(co, _i32p)))
        return lv, co

    def load_blocks(self, data):
        if hasattr(data, "data_ptr"):
            t = data.to(device=self.device, dtype=self.torch.float64).contiguous()
            assert t.numel() == self.num_blocks() * self.cfg.nf * self.cfg.npts
            self.torch.cuda.current_stream(self.device).synchronize()
            self._chk(lib().mrb_load_blocks(self.h, _vp(t.data_ptr()), 1))
            self.stream.synchronize()
            return
        a = np.ascontiguousarray(np.asarray(data, dtype=np.float64))
        assert a.shape == (self.num_blocks(), self.cfg.nf, self.cfg.npts), a.shape
        self._chk(lib().mrb_load_blocks(self.h, _vp(a.ctypes.data), 0))

    def read_uniform(self, level: int):
        """Solution on the uniform level-`level` lattice: [nf][N]*dim (x fastest), numpy."""
        nl = (2 ** level) * (self.cfg.bs - 1)
        out = np.zeros((self.cfg.nf,) + (nl,) * self.cfg.dim)
        self._chk(lib().mrb_read_uniform(self.h, level, _vp(out.ctypes.data), 0))
        return out

    def read_blocks(self, on_device: bool = False):
        n = self.num_blocks()
        if on_device:
            t = self.torch.empty((n, self.cfg.nf, self.cfg.npts), dtype=self.torch.float64, device=self.device)
            self._chk(lib().mrb_read_blocks(self.h, _vp(t.data_ptr()), 1))
            return t
        out = np.zeros((n, self.cfg.nf, self.cfg.npts))
        self._chk(lib().mrb_read_blocks(self.h, _vp(out.ctypes.data), 0))
        return out

    # ---- the method -------------------------------------------------------------------
    def refine_all(self):
        self._chk(lib().mrb_refine_all(self.h))

    def rk4(self, t: float, dt: float):
        self._chk(lib().mrb_rk4(self.h, t, dt))

    def mr_pass(self):
        n = self.num_blocks()
        fl = np.zeros(n, dtype=np.int8)
        md = np.zeros((n, self.cfg.nf))
        self._chk(lib().mrb_mr_pass(self.h, _ptr(fl, _i8p), _ptr(md, _dp)))
        return fl, md

    def mr_pass_noalloc(self):
        """mr_pass through the entry point that allocates nothing (library scratch)."""
        n = self.num_blocks()
        fl = np.zeros(n, dtype=np.int8)
        md = np.zeros((n, self.cfg.nf))
        self._chk(lib().mrb_mr_pass_noalloc(self.h, _ptr(fl, _i8p), _ptr(md, _dp)))
        return fl, md

    def coarsen(self, flags) -> int:
        fl = np.ascontiguousarray(np.asarray(flags, dtype=np.int8))
        assert len(fl) == self.num_blocks()
        nc = ctypes.c_int()
        self._chk(lib().mrb_coarsen(self.h, _ptr(fl, _i8p), ctypes.byref(nc)))
        return nc.value

    def adapt(self) -> int:
        p = ctypes.c_int()
        self._chk(lib().mrb_adapt(self.h, ctypes.byref(p)))
        return p.value

    def step(self, t: float, dt: float, nsteps: int = 1):
        self._chk(lib().mrb_step(self.h, t, dt, nsteps))

    def get_flags(self):
        n = self.num_blocks()
        fl = np.zeros(n, dtype=np.int8)
        md = np.zeros((n, self.cfg.nf))
        self._chk(lib().mrb_get_flags(self.h, _ptr(fl, _i8p), _ptr(md, _dp)))
        return fl, md

    def tune(self, nsub: int = 0, reps: int = 0) -> int:
        """Force (nsub > 0), autotune (reps > 0) or reset the stage tiling; returns the tiling in use."""
        ch = ctypes.c_int()
        self._chk(lib().mrb_tune(self.h, nsub, reps, self.cfg.dt, ctypes.byref(ch)))
        return ch.value

    def set_graph(self, mode):
        """Graph replay in step(): False/0 off, True/1 on, 2 automatic (the default)."""
        m = int(mode) if not isinstance(mode, bool) else (1 if mode else 0)
        self._chk(lib().mrb_set_graph(self.h, m))

    def set_sweep(self, mode):
        """Stage launches of the fused form: 0 four launches, 1 one launch with grid
        barriers, 2 the autotuner's choice (default), 3 one launch per RK4 step over
        overlapped tiles where every leaf is on one level (2D advection shapes)."""
        self._chk(lib().mrb_set_sweep(self.h, int(mode)))

    def set_topology(self, mode: int):
        """Topology planning in step(): 0 host, 1 device, 2 device above 1,024 refined leaves (default)."""
        self._chk(lib().mrb_set_topology(self.h, int(mode)))

    def timing(self, enable: bool):
        self._chk(lib().mrb_timing(self.h, 1 if enable else 0))

    def stats(self) -> dict:
        buf = ctypes.create_string_buffer(8192)
        self._chk(lib().mrb_stats(self.h, buf, len(buf)))
        return json.loads(buf.value.decode())

    # ---- learned predictor -------------------------------------------------------------
    def mlp_init(self, params, mean, std):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        m = np.ascontiguousarray(np.asarray(mean, dtype=np.float32))
        s = np.ascontiguousarray(np.asarray(std, dtype=np.float32))
        self.mlp_nin = self.cfg.nf * 64
        self._chk(lib().mrb_mlp_init(self.h, self.mlp_nin, _ptr(p, _fp), _ptr(m, _fp), _ptr(s, _fp)))
        self.mlp_np = len(p)

    def mlp_params(self):
        out = np.zeros(self.mlp_np, dtype=np.float32)
        self._chk(lib().mrb_mlp_get_params(self.h, _ptr(out, _fp)))
        return out

    def mlp_features(self):
        out = np.zeros((self.num_blocks(), self.cfg.nf * 64), dtype=np.float32)
        self._chk(lib().mrb_mlp_features(self.h, _ptr(out, _fp)))
        return out

    def mlp_forward(self, x):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
        out = np.zeros((len(x), 3), dtype=np.float32)
        self._chk(lib().mrb_mlp_forward(self.h, _ptr(x, _fp), len(x), _ptr(out, _fp)))
        return out

    def mlp_grad(self, x, y, classw):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
        y = np.ascontiguousarray(np.asarray(y, dtype=np.int8))
        cw = np.ascontiguousarray(np.asarray(classw, dtype=np.float32))
        g = np.zeros(self.mlp_np, dtype=np.float32)
        loss = ctypes.c_float()
        self._chk(lib().mrb_mlp_grad(self.h, _ptr(x, _fp), _ptr(y, _i8p), _ptr(cw, _fp), len(x), _ptr(g, _fp),
                                     ctypes.byref(loss)))
        return loss.value, g

    def mlp_train_epoch(self, x, y, classw, batch=1024, lr=1e-3):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
        y = np.ascontiguousarray(np.asarray(y, dtype=np.int8))
        cw = np.ascontiguousarray(np.asarray(classw, dtype=np.float32))
        loss = ctypes.c_float()
        self._chk(lib().mrb_mlp_train(self.h, _ptr(x, _fp), _ptr(y, _i8p), _ptr(cw, _fp), len(x), batch, lr,
                                      ctypes.byref(loss)))
        return loss.value

    def mlp_predict(self):
        n = self.num_blocks()
        pred = np.zeros(n, dtype=np.int8)
        prob = np.zeros(n, dtype=np.float32)
        self._chk(lib().mrb_mlp_predict(self.h, _ptr(pred, _i8p), _ptr(prob, _fp)))
        return pred, prob

    def refine_marked(self, mask) -> int:
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.int8))
        assert len(m) == self.num_blocks()
        k = ctypes.c_int()
        self._chk(lib().mrb_refine_marked(self.h, _ptr(m, _i8p), ctypes.byref(k)))
        return k.value

    def step_predicted(self, t, dt, tau=0.9, guard=0.0) -> int:
        k = ctypes.c_int()
        self._chk(lib().mrb_step_predicted(self.h, t, dt, tau, guard, ctypes.byref(k)))
        return k.value

    def init_grid(self, fn=None, max_iter: int = 0):
        """Initial adaptive grid: uniform level 1, then {refine all, resample the
        analytic initial condition, adapt, resample} until the forest is unchanged."""
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


def horizon_labels(dim, lv_now, co_now, lv_later, co_later):
    """Labels (0 refine, 1 keep, 2 coarsen) of the blocks of one grid from a later grid."""
    a = np.ascontiguousarray(np.asarray(lv_now, dtype=np.int8))
    ca = np.ascontiguousarray(np.asarray(co_now, dtype=np.int32).reshape(len(a), dim))
    b = np.ascontiguousarray(np.asarray(lv_later, dtype=np.int8))
    cb = np.ascontiguousarray(np.asarray(co_later, dtype=np.int32).reshape(len(b), dim))
    out = np.zeros(len(a), dtype=np.int8)
    rc = lib().mrb_horizon_labels(dim, len(a), _ptr(a, _i8p), _ptr(ca, _i32p), len(b), _ptr(b, _i8p), _ptr(cb, _i32p),
                                  _ptr(out, _i8p))
    if rc != MRB_OK:
        raise MrbError(rc, "mrb_horizon_labels")
    return out

