"""Plan creation with explicit image arrays, and the errors plan creation reports for bad inputs,
through the C-ABI on the GPU (every kernel still runs to completion; the checks are reductions
whose result the host reads):

* image arrays that are the exact mirror (x, -y) give bitwise the same potentials as a plan that
  mirrors the points itself; an image array off by one ulp in one entry is FMMHP_EDOMAIN;
* a source with y <= 0 is FMMHP_EDOMAIN, a non-finite coordinate FMMHP_EINVAL; a separate target
  with y < 0 is FMMHP_EDOMAIN while y = 0 is accepted;
* an allocation failure forced by the FMMHP_TEST_FAIL_ALLOC hook (the k-th plan allocation fails)
  returns FMMHP_ENOMEM, leaves no plan behind and releases the device memory the plan had taken.
"""
import os

import numpy as np
import pytest
import torch

import paper_2507_21913_amd as F
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EINVAL, EDOMAIN, ENOMEM = 1, 2, 3


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _status_of(fn):
    with pytest.raises(F.FMMHPError) as ei:
        fn()
    return ei.value.status


def test_explicit_images_equal_implicit_ones():
    w = workloads.plain_small(seed=3)
    x, y, q = _t(w.x), _t(w.y), _t(w.q[0])
    for Z in (1.0, 1.0 + 0.5j):
        a = F.HalfPlaneFMM(x, y, Z, p=20, leaf_size=40)
        b = F.HalfPlaneFMM(x, y, Z, p=20, leaf_size=40, pass_images=True)
        pa, pb = a(q).cpu().numpy(), b(q).cpu().numpy()
        ta, tb = a.export_tree(), b.export_tree()
        a.close()
        b.close()
        assert np.array_equal(pa.view(np.float64), pb.view(np.float64))
        for k in ("level", "first", "count", "perm", "U_ent", "V_ent", "W_ent", "X_ent"):
            assert np.array_equal(ta[k], tb[k]), k


def _create_with_images(x, y, ix, iy):
    opts = F.Opts(20, 40, 0, 0)
    return F.fmmhp_plan_create(x.numel(), x.data_ptr(), y.data_ptr(), ix.data_ptr(), iy.data_ptr(), 1.0, 0.0,
                               opts, torch.cuda.current_stream().cuda_stream)


def test_perturbed_images_are_rejected():
    w = workloads.plain_small(seed=3)
    x, y = _t(w.x), _t(w.y)
    good = _create_with_images(x, y, x.clone(), -y)
    F.fmmhp_plan_destroy(good)
    for which in ("x", "y"):
        ix, iy = x.clone(), -y
        t = ix if which == "x" else iy
        t[777] = float(np.nextafter(t[777].item(), np.inf))
        st = _status_of(lambda: _create_with_images(x, y, ix, iy))
        assert st == EDOMAIN, which
        assert "mirror" in F.lib().fmmhp_last_error_message().decode()


@pytest.mark.parametrize("bad", ["y0", "yneg", "nan_x", "nan_y", "inf_x"])
def test_bad_source_coordinates(bad):
    w = workloads.plain_small(seed=4)
    xs, ys = w.x.copy(), w.y.copy()
    k = 1234
    if bad == "y0":
        ys[k] = 0.0
    elif bad == "yneg":
        ys[k] = -1e-3
    elif bad == "nan_x":
        xs[k] = np.nan
    elif bad == "nan_y":
        ys[k] = np.nan
    else:
        xs[k] = np.inf
    st = _status_of(lambda: F.HalfPlaneFMM(_t(xs), _t(ys), 1.0, p=10, leaf_size=40))
    assert st == (EDOMAIN if bad in ("y0", "yneg") else EINVAL), bad


def test_target_on_boundary_accepted_below_rejected():
    w = workloads.plain_small(seed=5)
    xt = np.array([0.25, 0.5, 0.75])
    yt = np.array([0.0, 0.3, 0.0])
    plan = F.HalfPlaneFMM.with_targets(_t(w.x), _t(w.y), _t(xt), _t(yt), 1.0, p=10, leaf_size=40)
    assert np.all(np.isfinite(plan(_t(w.q[0])).cpu().numpy()))
    plan.close()
    yt[1] = -1e-12
    st = _status_of(lambda: F.HalfPlaneFMM.with_targets(_t(w.x), _t(w.y), _t(xt), _t(yt), 1.0, p=10,
                                                        leaf_size=40))
    assert st == EDOMAIN


@pytest.mark.parametrize("k", [1, 4, 9, 16])
def test_forced_allocation_failure_releases_memory(k):
    w = workloads.plain_small(seed=6)
    x, y, q = _t(w.x), _t(w.y), _t(w.q[0])
    ref = F.HalfPlaneFMM(x, y, 1.0, p=20, leaf_size=40)
    phi_ref = ref(q).cpu().numpy()
    ref.close()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    os.environ["FMMHP_TEST_FAIL_ALLOC"] = str(k)
    try:
        st = _status_of(lambda: F.HalfPlaneFMM(x, y, 1.0, p=20, leaf_size=40))
        msg = F.lib().fmmhp_last_error_message().decode()
    finally:
        del os.environ["FMMHP_TEST_FAIL_ALLOC"]
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    print(f"FMMHP_TEST_FAIL_ALLOC={k}: {msg}; free device memory change {free1 - free0} B", flush=True)
    assert st == ENOMEM
    assert "test hook" in msg
    # the failed plan returned what it had allocated (allow the allocator's own granularity)
    assert free0 - free1 < (2 << 20)
    # and the library still works afterwards
    plan = F.HalfPlaneFMM(x, y, 1.0, p=20, leaf_size=40)
    phi = plan(q).cpu().numpy()
    plan.close()
    assert np.array_equal(phi.view(np.float64), phi_ref.view(np.float64))
