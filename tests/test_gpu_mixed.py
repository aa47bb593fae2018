"""GPU parity of the mixed-precision M2L (FMMHP_FLAG_M2L_FP32): the upper-source M2L on the FP32
matrix cores with FP64 folding per offset slot, everything else FP64.

Bar: rel-l2 <= 1e-6 against the oracle's direct sum (the mode's stated tolerance; FP32 operands
and sums give ~1e-7), on the same cases as the FP64 path (small, adaptive with W/X lists, complex
impedance, forest with several vectors, full 1M sample); and the FP64 and FP32 plans agree to the
same bar.
"""
import os
import sys

import numpy as np
import pytest
import torch

import paper_2507_21913_amd as F
import workloads
from oracle import direct as D

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
from golden_io import load  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-6


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j])
@pytest.mark.parametrize("p", [10, 20, 30])
def test_m2l_fp32_small_vs_oracle(Z, p):
    w = workloads.plain_small()
    ref = D.potential(w.x, w.y, w.q[0], Z, workers=8)
    plan = F.HalfPlaneFMM(_t(w.x), _t(w.y), Z, p=p, leaf_size=16, m2l_fp32=True)
    got = plan(_t(w.q[0])).cpu().numpy()
    err = D.rel_l2(got, ref)
    plan64 = F.HalfPlaneFMM(_t(w.x), _t(w.y), Z, p=p, leaf_size=16)
    err64 = D.rel_l2(plan64(_t(w.q[0])).cpu().numpy(), ref)
    print(f"p={p} Z={Z}: FP32-M2L rel-l2 {err:.2e} (FP64 {err64:.2e})", flush=True)
    assert err < max(TOL, 10 * err64)
    plan.close()
    plan64.close()


def test_m2l_fp32_adaptive_curve_vs_oracle():
    w = workloads.curve_4m(seed=3, n=12000)
    ref = D.potential(w.x, w.y, w.q[0], w.impedance, workers=8)
    plan = F.HalfPlaneFMM(_t(w.x), _t(w.y), w.impedance, p=30, leaf_size=12, m2l_fp32=True)
    info = plan.info()
    assert info["list_len"][2] > 0 and info["list_len"][3] > 0
    err = D.rel_l2(plan(_t(w.q[0])).cpu().numpy(), ref)
    print(f"curve 12k FP32-M2L rel-l2 {err:.2e}", flush=True)
    assert err < TOL
    plan.close()


def test_m2l_fp32_forest_multivector_vs_oracle():
    rng = np.random.default_rng(8)
    sizes = [900, 2500, 60]
    imps = [0.5, 6.0, 1.0]
    xs = [rng.uniform(0, 1, n) for n in sizes]
    ys = [rng.uniform(0.01, 1.01, n) for n in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)])
    x, y = np.concatenate(xs), np.concatenate(ys)
    q = rng.standard_normal((10, off[-1]))
    plan = F.HalfPlaneFMM.batched(_t(x), _t(y), off, imps, p=20, leaf_size=20, m2l_fp32=True)
    phi = plan(_t(q)).cpu().numpy()
    for k in range(len(sizes)):
        a, b = off[k], off[k + 1]
        ref = D.potential(x[a:b], y[a:b], q[:, a:b], imps[k], workers=8)
        for v in (0, 7, 9):
            assert D.rel_l2(phi[v, a:b], ref[v]) < TOL, (k, v)
    plan.close()


def test_m2l_fp32_uniform_1m_sample():
    w = workloads.uniform_1m(seed=1)
    plan = F.HalfPlaneFMM(_t(w.x), _t(w.y), 1.0, p=20, leaf_size=32, m2l_fp32=True)
    phi = plan(_t(w.q[0])).cpu().numpy()
    idx, ref = load("uniform_1m")
    err = D.rel_l2(phi[idx], ref)
    print(f"uniform_1m p=20 leaf 32 FP32-M2L: rel-l2 at 256 targets {err:.2e}", flush=True)
    assert err < TOL
    im = D.imag_part_real_impedance(w.x, w.y, w.q[0], 1.0)
    assert float(np.max(np.abs(phi.imag - im)) / np.max(np.abs(im))) < 1e-12  # Im needs no M2L
    plan.close()
