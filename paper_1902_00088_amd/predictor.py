"""Learned refinement predictor: data recording, training and guided runs.

The paper's refinement flag accepts a +1 from indicators other than the detail test
(Sec. 2.3, flag rule); the safety zone (Sec. 2.1 item 1) refines every block by one
level before each step so that the step cannot outrun the grid.  Here a per-block MLP
(features, forward, backward and Adam run in the library's kernels) predicts which
blocks that refinement is needed for, a few steps ahead:

* labels come from the plain method's own grids: block b of G^n at level l is
  'refine' (0) if G^{n+H} has a finer block overlapping it, 'coarsen' (2) if it lies
  inside a coarser block of G^{n+H}, else 'keep' (1);
* a guided step refines only blocks predicted 'refine' or predicted with softmax
  probability below tau (the safety zone stays the fallback), closed under
  gradedness; the exact detail threshold still decides every coarsening;
* every K-th step a shadow plain step runs from the same state: where the two grids
  differ the step counts as mispredicted and the plain result is adopted.

Global time stepping: the step size is set by the finest level the step can reach
(Sec. 4, global time stepping), i.e. one level above the finest leaf of G^n.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import horizon_labels

REFINE, KEEP, COARSEN = 0, 1, 2


def step_size(cfg, levels) -> float:
    """Time step of a grid: the configured CFL step at level jmax, scaled to the
    finest level a step from this grid can reach (finest leaf + 1, at most jmax)."""
    top = min(cfg.jmax, int(np.max(levels)) + 1)
    return cfg.dt * float(2 ** (cfg.jmax - top))


@dataclass
class Recording:
    feats: list = field(default_factory=list)     # per step: [n_blocks][nin] float32
    forests: list = field(default_factory=list)   # per step: (levels, coords)
    times: list = field(default_factory=list)
    dts: list = field(default_factory=list)
    block_updates: list = field(default_factory=list)
    wall_s: float = 0.0

    def labels(self, horizon: int, dim: int):
        """Labels of the steps n with n + horizon recorded."""
        out = []
        for n in range(len(self.forests) - horizon):
            lv, co = self.forests[n]
            lv2, co2 = self.forests[n + horizon]
            out.append(horizon_labels(dim, lv, co, lv2, co2))
        return out

    def dataset(self, steps, horizon: int, dim: int):
        ys = self.labels(horizon, dim)
        steps = [n for n in steps if n < len(ys)]
        X = np.concatenate([self.feats[n] for n in steps])
        Y = np.concatenate([ys[n] for n in steps])
        return X, Y


def record(solver, nsteps: int, t0: float = 0.0, adaptive_dt: bool = True) -> Recording:
    """Run the plain method for nsteps, recording the features and the forest of every
    grid G^0 .. G^nsteps (features of the last one included)."""
    cfg = solver.cfg
    rec = Recording()
    t = t0
    bu0 = solver.stats()["block_updates"]
    for n in range(nsteps + 1):
        lv, co = solver.read_forest()
        rec.forests.append((lv, co))
        rec.feats.append(solver.mlp_features())
        if n == nsteps:
            break
        dt = step_size(cfg, lv) if adaptive_dt else cfg.dt
        tw = time.perf_counter()
        solver.step(t, dt)
        rec.wall_s += time.perf_counter() - tw
        bu = solver.stats()["block_updates"]
        rec.block_updates.append(bu - bu0)
        bu0 = bu
        rec.times.append(t)
        rec.dts.append(dt)
        t += dt
    return rec


def normalisation(X, nf: int):
    """Per-field mean and standard deviation of raw features (FP64, returned float32)."""
    X = np.asarray(X, dtype=np.float64)
    mean = np.array([X[:, f * 64:(f + 1) * 64].mean() for f in range(nf)])
    std = np.array([X[:, f * 64:(f + 1) * 64].std() for f in range(nf)])
    std = np.where(std > 0, std, 1.0)
    return mean.astype(np.float32), std.astype(np.float32)


def class_weights(y, ncls: int = 3):
    y = np.asarray(y)
    n = len(y)
    w = np.ones(ncls, dtype=np.float32)
    for c in range(ncls):
        k = int(np.sum(y == c))
        if k:
            w[c] = n / (ncls * k)
    return w


def train(solver, X, y, params0, epochs: int, batch: int = 1024, lr: float = 1e-3, seed: int = 5,
          classw=None, log=None):
    """Train the solver's predictor from params0 on (X, y) with the library's kernels.
    Normalisation is fitted on X.  Returns the mean loss of every epoch."""
    nf = solver.cfg.nf
    mean, std = normalisation(X, nf)
    solver.mlp_init(params0, mean, std)
    cw = class_weights(y) if classw is None else np.asarray(classw, np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.int8)
    losses = []
    for e in range(epochs):
        perm = np.random.default_rng([seed, e]).permutation(len(y))
        losses.append(solver.mlp_train_epoch(X[perm], y[perm], cw, batch=batch, lr=lr))
        if log:
            log(f"epoch {e}: loss {losses[-1]:.4f}")
    return losses


def evaluate(solver, X, y):
    """Confusion matrix [true][pred] and accuracy of the current predictor on (X, y)."""
    logits = solver.mlp_forward(np.ascontiguousarray(X, dtype=np.float32))
    pred = np.argmax(logits, axis=1)
    cm = np.zeros((3, 3), dtype=np.int64)
    np.add.at(cm, (np.asarray(y, dtype=np.int64), pred), 1)
    return cm, float(np.trace(cm)) / max(1, len(y))


def _forest_key(lv, co):
    return lv.tobytes() + co.tobytes()


@dataclass
class GuidedRun:
    steps: int = 0
    block_updates: int = 0          # RK4 block updates of the guided steps
    shadow_block_updates: int = 0    # of the shadow plain steps
    refined: int = 0
    shadowed: int = 0
    mispredicted_steps: int = 0
    mispredicted_blocks: int = 0
    wall_s: float = 0.0
    blocks: list = field(default_factory=list)


def run_guided(solver, nsteps: int, tau: float = 0.9, shadow_every: int = 10, t0: float = 0.0,
               adaptive_dt: bool = True, guard: float = 0.0) -> GuidedRun:
    """Advance nsteps with predictor-guided refinement.  Every shadow_every-th step
    (0 = never) a plain step from the same state decides: where the grids differ the
    plain result is adopted and the step counts as mispredicted."""
    cfg = solver.cfg
    r = GuidedRun()
    t = t0
    torch = solver.torch
    for n in range(nsteps):
        lv, co = solver.read_forest()
        dt = step_size(cfg, lv) if adaptive_dt else cfg.dt
        shadow = shadow_every > 0 and n % shadow_every == 0
        if shadow:
            snap = solver.read_blocks(on_device=True)
            bu = solver.stats()["block_updates"]
            solver.step(t, dt)
            r.shadow_block_updates += solver.stats()["block_updates"] - bu
            plv, pco = solver.read_forest()
            pdata = solver.read_blocks(on_device=True)
            solver.init_forest(lv, co)
            solver.load_blocks(snap)
        bu = solver.stats()["block_updates"]
        torch.cuda.synchronize()
        tw = time.perf_counter()
        r.refined += solver.step_predicted(t, dt, tau, guard)
        torch.cuda.synchronize()
        r.wall_s += time.perf_counter() - tw
        r.block_updates += solver.stats()["block_updates"] - bu
        if shadow:
            r.shadowed += 1
            glv, gco = solver.read_forest()
            if _forest_key(glv, gco) != _forest_key(plv, pco):
                a = {(int(l),) + tuple(int(v) for v in c) for l, c in zip(glv, gco)}
                b = {(int(l),) + tuple(int(v) for v in c) for l, c in zip(plv, pco)}
                r.mispredicted_steps += 1
                r.mispredicted_blocks += len(a ^ b)
                solver.init_forest(plv, pco)
                solver.load_blocks(pdata)
        r.blocks.append(solver.num_blocks())
        r.steps += 1
        t += dt
    return r


def compare_grids(cfg, a, b):
    """Max abs difference per field of two adaptive solutions at the nodes both grids
    hold on their own lattices.  a, b: (levels, coords, data [n][nf][bs^dim])."""
    J = cfg.jmax
    bs = cfg.bs
    loc = np.indices((bs,) * cfg.dim)[::-1].reshape(cfg.dim, -1)   # x fastest
    NJ = (2 ** J) * (bs - 1)

    def keys(lv, co):
        lv = np.asarray(lv, np.int64)
        co = np.asarray(co, np.int64).reshape(len(lv), cfg.dim)
        s = (2 ** (J - lv))[:, None]
        k = np.zeros((len(lv), loc.shape[1]), np.int64)
        for ax in range(cfg.dim - 1, -1, -1):
            g = (co[:, ax:ax + 1] * (bs - 1) + loc[ax][None, :]) * s
            k = k * NJ + np.mod(g, NJ)
        return k.reshape(-1)

    ka, kb = keys(a[0], a[1]), keys(b[0], b[1])
    da = np.asarray(a[2]).transpose(0, 2, 1).reshape(-1, cfg.nf)
    db = np.asarray(b[2]).transpose(0, 2, 1).reshape(-1, cfg.nf)
    ua, ia = np.unique(ka, return_index=True)
    ub, ib = np.unique(kb, return_index=True)
    _, xa, xb = np.intersect1d(ua, ub, assume_unique=True, return_indices=True)
    d = np.abs(da[ia[xa]] - db[ib[xb]])
    return d.max(axis=0), np.abs(db[ib[xb]]).max(axis=0), len(xa)


def _state(solver):
    lv, co = solver.read_forest()
    return lv, co, solver.read_blocks(on_device=True)


def _restore(solver, st):
    solver.init_forest(st[0], st[1])
    solver.load_blocks(st[2])


def run_plain(solver, nsteps: int, t0: float = 0.0, adaptive_dt: bool = True):
    """Plain method for nsteps; returns (wall seconds, block updates)."""
    cfg = solver.cfg
    torch = solver.torch
    bu0 = solver.stats()["block_updates"]
    t = t0
    torch.cuda.synchronize()
    tw = time.perf_counter()
    for _ in range(nsteps):
        dt = step_size(cfg, solver.read_forest()[0]) if adaptive_dt else cfg.dt
        solver.step(t, dt)
        t += dt
    torch.cuda.synchronize()
    return time.perf_counter() - tw, solver.stats()["block_updates"] - bu0


def gain_study(solver, params0, nsteps: int = 2000, train_frac: float = 0.8, horizon: int = 5, epochs: int = 60,
               batch: int = 1024, lr: float = 1e-3, seed: int = 5, tau: float = 0.97, shadow_every: int = 10,
               adaptive_dt: bool = True, guard: float = 0.0, log=None):
    """Record the plain method, train the predictor on the first part of the run, test
    it on the rest, then rerun from the same initial grid with guided refinement (once
    per detail guard if `guard` is a list) and compare cost and solution with the
    plain run.  The solver must hold the initial grid on entry."""
    cfg = solver.cfg
    say = log or (lambda *_: None)
    init = _state(solver)
    say(f"record {nsteps} plain steps")
    tr0 = time.perf_counter()
    rec = record(solver, nsteps, adaptive_dt=adaptive_dt)
    t_rec = time.perf_counter() - tr0
    ntrain = int(round(train_frac * nsteps))
    last = nsteps - horizon
    Xtr, ytr = rec.dataset(range(0, ntrain), horizon, cfg.dim)
    Xte, yte = rec.dataset(range(ntrain, last + 1), horizon, cfg.dim)
    say(f"train on {len(ytr)} samples, labels {np.bincount(ytr, minlength=3).tolist()}")
    tt0 = time.perf_counter()
    losses = train(solver, Xtr, ytr, params0, epochs, batch=batch, lr=lr, seed=seed)
    solver.torch.cuda.synchronize()
    t_train = time.perf_counter() - tt0
    cm_tr, acc_tr = evaluate(solver, Xtr, ytr)
    cm_te, acc_te = evaluate(solver, Xte, yte)
    # plain run, timed without recording
    _restore(solver, init)
    wall_p, bu_p = run_plain(solver, nsteps, adaptive_dt=adaptive_dt)
    plain_end = _state(solver)
    plain_end = (plain_end[0], plain_end[1], plain_end[2].cpu().numpy())
    guided = {}
    for gd in (guard,) if not isinstance(guard, (list, tuple)) else guard:
        say(f"guided run, detail guard {gd}")
        _restore(solver, init)
        g = run_guided(solver, nsteps, tau=tau, shadow_every=shadow_every, adaptive_dt=adaptive_dt, guard=gd)
        lv, co = solver.read_forest()
        dmax, ref, npts = compare_grids(cfg, (lv, co, solver.read_blocks()), plain_end)
        rel = [float(d / r) if r > 0 else float(d) for d, r in zip(dmax, ref)]
        guided[gd] = {
            "block_updates_per_step": g.block_updates / nsteps,
            "shadow_block_updates_per_step": g.shadow_block_updates / nsteps,
            "ms_per_step": 1e3 * g.wall_s / nsteps, "refined_per_step": g.refined / nsteps,
            "shadowed": g.shadowed, "mispredicted_steps": g.mispredicted_steps,
            "mispredicted_blocks": g.mispredicted_blocks, "blocks_end": int(len(lv)),
            "block_updates_saved": 1.0 - g.block_updates / max(1, bu_p),
            "rel_err_vs_plain": rel, "compared_nodes": int(npts),
            "within_bound": bool(max(rel) <= 10.0 * cfg.eps),
        }
    first = guided[next(iter(guided))]
    return {
        "steps": nsteps, "horizon": horizon, "epochs": epochs, "tau": tau, "shadow_every": shadow_every,
        "adaptive_dt": adaptive_dt,
        "labels_train": np.bincount(ytr, minlength=3).tolist(), "labels_test": np.bincount(yte, minlength=3).tolist(),
        "loss_first_last": [float(losses[0]), float(losses[-1])],
        "train_accuracy": acc_tr, "test_accuracy": acc_te, "test_confusion": cm_te.tolist(),
        "record_s": t_rec, "train_s": t_train,
        "plain": {"block_updates_per_step": bu_p / nsteps, "ms_per_step": 1e3 * wall_p / nsteps,
                  "blocks_end": int(len(plain_end[0]))},
        "bound": 10.0 * cfg.eps,
        # the first (or only) guard's results at top level, every guard under "guards"
        "guided": first, "block_updates_saved": first["block_updates_saved"],
        "rel_err_vs_plain": first["rel_err_vs_plain"], "within_bound": first["within_bound"],
        "guards": {str(k): v for k, v in guided.items()},
    }
