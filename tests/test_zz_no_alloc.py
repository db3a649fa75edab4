"""mwns_tree_eval_noalloc (the evaluation entry point that allocates nothing, for callers that
cannot allocate) against mwns_tree_eval on the same trees and points: two calls in a row, the
second on a smaller tree and fewer points, so that the fixed scratch array is reused."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_noalloc_eval_matches_eval_on_two_calls():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_0706_0747_amd as M
    ctx = M.Context(0)
    big = workloads.small_adaptive(8, k=8, eps=1e-5, jmax=5)
    small = workloads.small_adaptive(11, k=6, eps=1e-3, jmax=4)
    for w, npts, seed in ((big, 20000, 71), (small, 3000, 72)):
        f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
        pts = workloads.points(npts, seed=seed)
        pts[:4] = [[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.5, 0.5, 0.5], [1.0, 0.25, 0.0]]   # corners, faces
        ref = M.mwns_tree_eval(ctx, f, pts)
        xyz = torch.from_numpy(pts).to("cuda")
        out = torch.full((npts,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        M.mwns_tree_eval_noalloc(ctx, f, npts, xyz.data_ptr(), out.data_ptr())
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print("nodes %d, points %d, max |diff| %.3e" % (M.mwns_tree_get_info(f)["nnodes"], npts, np.abs(got - ref).max()))
        assert np.array_equal(got, ref)
    # a point outside the cube gets NaN, the others their values
    bad = torch.tensor([[0.5, 0.5, 1.5], [0.25, 0.75, 0.5]], dtype=torch.float64, device="cuda")
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    M.mwns_tree_eval_noalloc(ctx, f, 2, bad.data_ptr(), out.data_ptr())
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.isnan(o[0]) and o[1] == M.mwns_tree_eval(ctx, f, [[0.25, 0.75, 0.5]])[0]
    from paper_0706_0747_amd import _lib
    with pytest.raises(M.MwnsError) as e:
        M.mwns_tree_eval_noalloc(ctx, f, -1, bad.data_ptr(), out.data_ptr())
    assert e.value.status == _lib.MWNS_EINVAL
