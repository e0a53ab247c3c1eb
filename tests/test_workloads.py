"""The seeded synthetic inputs (no GPU): configurations as the input recipe states them,
time steps from the CFL reading (dt = 0.5 h_Jmax / U), reproducible samples and
random forests that the oracle accepts as graded tilings."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.mark.parametrize("make,dim,bs,jmax,eps,speed", [
    (W.C1, 2, 17, 4, 1e-3, 1.0),
    (W.C2, 2, 33, 7, 1e-4, 1.0),
    (W.C3, 2, 33, 8, 1e-3, 1.75),
    (W.C4, 3, 17, 6, 1e-4, 1.0),
])
def test_configurations_and_cfl_time_step(make, dim, bs, jmax, eps, speed):
    cfg = make()
    assert (cfg.dim, cfg.bs, cfg.jmax, cfg.eps) == (dim, bs, jmax, eps)
    h = 1.0 / ((1 << jmax) * (bs - 1))
    assert cfg.dt == pytest.approx(0.5 * h / speed, rel=1e-15)
    # the pool fits the kernels' 32-bit offsets
    assert cfg.max_blocks * cfg.nf * bs ** dim < 2 ** 31


def test_blob_centres_come_from_the_stated_seeds():
    assert np.array_equal(W.C2().blob_centers, np.random.default_rng(2).uniform(0.25, 0.75, (3, 2)))
    assert np.array_equal(W.C4().blob_centers, np.random.default_rng(4).uniform(0.25, 0.75, (4, 3)))


def test_samples_are_reproducible_and_periodic():
    cfg = W.C2(jmax=3)
    lv, co = W.uniform_forest(cfg, 2)
    a = W.sample(cfg, lv, co)
    b = W.sample(cfg, lv, co)
    assert np.array_equal(a, b)
    # node coordinates wrap: the last node of a block equals the first node of its x-neighbour
    n = 1 << 2
    first = {(int(c[0]), int(c[1])): i for i, c in enumerate(co)}
    bs = cfg.bs
    for i, c in enumerate(co):
        j = first[((int(c[0]) + 1) % n, int(c[1]))]
        left = a[i, 0].reshape(bs, bs)[:, bs - 1]
        right = a[j, 0].reshape(bs, bs)[:, 0]
        assert np.array_equal(left, right)


@pytest.mark.parametrize("dim,seed", [(2, 0), (2, 5), (3, 1)])
def test_random_graded_forests_are_valid(dim, seed):
    jmax = 4 if dim == 2 else 3
    lv, co = W.random_graded_forest(dim, jmax, seed)
    cfg = (W.C2(jmax=jmax) if dim == 2 else W.C4(jmax=jmax)).replace(max_blocks=4 ** jmax if dim == 2 else 8 ** jmax)
    o = oracle.Oracle(cfg)
    o.init_forest(lv, co)          # raises unless the leaves tile the domain and are graded
    assert o.num_blocks() == len(lv)
    lv2, _ = W.random_graded_forest(dim, jmax, seed)
    assert np.array_equal(lv, lv2)
