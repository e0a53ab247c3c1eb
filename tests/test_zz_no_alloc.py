"""The analysis entry point that allocates nothing (mrb_mr_pass_noalloc) against
mrb_mr_pass, through the C ABI: two calls in a row on twin solvers, the second on a
smaller grid.  Flags, detail maxima and the state after the pass (redundant nodes
written back) must be bitwise equal."""
import numpy as np
import pytest

import workloads as W
import paper_1902_00088_amd as M


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["2d", "3d", "ns"])
def test_mr_pass_noalloc_matches_mr_pass(which):
    if which == "2d":
        cfg = W.C2(jmax=6, eps=1e-4, blob_beta=4e-4, form=W.FORM_FUSED)
    elif which == "3d":
        cfg = W.C4(jmax=4, eps=1e-4, form=W.FORM_FUSED).replace(max_blocks=8000)
    else:
        cfg = W.C3(jmax=4, eps=1e-4, form=W.FORM_FUSED)
    a, b = M.Solver(cfg), M.Solver(cfg)
    for s in (a, b):
        s.init_grid()
        s.refine_all()
        s.rk4(0.0, cfg.dt)
    sizes = []
    for call in range(2):
        n = a.num_blocks()
        sizes.append(n)
        fa, ma = a.mr_pass()
        fb, mb = b.mr_pass_noalloc()
        assert np.array_equal(fa, fb), (which, call)
        assert np.array_equal(_bits(ma), _bits(mb)), (which, call)
        assert np.array_equal(_bits(a.read_blocks()), _bits(b.read_blocks())), (which, call)
        if call == 0:
            # the next call runs on the coarsened, smaller grid
            assert a.coarsen(fa) == b.coarsen(fb) > 0
    assert sizes[1] < sizes[0]
    a.close()
    b.close()
