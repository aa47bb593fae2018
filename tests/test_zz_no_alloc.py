"""fmmhp_eval_noalloc (the evaluation for callers that cannot allocate: its per-vector workspace
lives in the library's static device scratch) against fmmhp_eval on the same plan, through the
C-ABI: bitwise equal results (the same kernels in the same order), on two calls in a row, the
second on a smaller plan, with eight-vector and single-vector passes, real and complex impedances
and a forest; a plan whose one-vector workspace exceeds the scratch is rejected before any launch.
"""
import numpy as np
import pytest
import torch

import paper_2507_21913_amd as F
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _both(plan, q):
    """(fmmhp_eval result, fmmhp_eval_noalloc result) for charges q [nv, n] as float64 arrays."""
    nv, n = q.shape
    a = torch.full((nv, n, 2), np.nan, dtype=torch.float64, device=DEV)
    b = torch.full((nv, n, 2), np.nan, dtype=torch.float64, device=DEV)
    s = torch.cuda.current_stream().cuda_stream
    F.fmmhp_eval(plan._plan, nv, q.data_ptr(), a.data_ptr(), s)
    F.fmmhp_eval_noalloc(plan._plan, nv, q.data_ptr(), b.data_ptr(), s)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j])
def test_noalloc_equals_eval_twice_second_smaller(Z):
    big = workloads.plain_small(seed=11, n=6000)
    small = workloads.plain_small(seed=12, n=900)
    for w, nv in ((big, 9), (small, 3)):
        plan = F.HalfPlaneFMM(_t(w.x), _t(w.y), Z, p=20, leaf_size=32)
        rng = np.random.default_rng(5)
        q = _t(rng.uniform(-1.0, 1.0, (nv, w.n)))
        a, b = _both(plan, q)
        plan.close()
        print(f"n={w.n} nv={nv} Z={Z}: max |noalloc - eval| = {np.max(np.abs(a - b)):.1e}", flush=True)
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b)


def test_noalloc_forest():
    sizes = [2500, 700, 1800]
    imps = [0.5, 3.0, 1.0]
    xs, ys = [], []
    for k, m in enumerate(sizes):
        w = workloads.plain_small(seed=20 + k, n=m)
        xs.append(w.x)
        ys.append(w.y)
    off = np.concatenate([[0], np.cumsum(sizes)])
    plan = F.HalfPlaneFMM.batched(_t(np.concatenate(xs)), _t(np.concatenate(ys)), off, imps, p=15, leaf_size=24)
    q = _t(np.random.default_rng(6).standard_normal((8, off[-1])))
    a, b = _both(plan, q)
    plan.close()
    assert np.all(np.isfinite(b))
    assert np.array_equal(a, b)


def test_noalloc_rejects_plan_beyond_scratch():
    w = workloads.uniform_1m(seed=1)
    plan = F.HalfPlaneFMM(_t(w.x), _t(w.y), 1.0 + 0.5j, p=30, leaf_size=40)
    q = _t(w.q[:1])
    out = torch.empty((1, w.n, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(F.FMMHPError) as ei:
        F.fmmhp_eval_noalloc(plan._plan, 1, q.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    plan.close()
    assert ei.value.status == 1
    assert "scratch" in str(ei.value)
