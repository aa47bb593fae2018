"""GPU parity of the configurations the benchmark times, through the C-ABI:

* the uniform 1,048,576-point workload at the plan the benchmark runs (p = 20, leaf 32, prefetching
  near walk on two workgroups per CU): rel-l2 <= 1e-10 against the oracle's stored direct-sum
  sample, and the exact imaginary part at every target;
* the autotuner: the plan it returns for tolerances 1e-8 and 1e-10 (p, leaf size, near-field shape
  and M2L form) meets that tolerance against the oracle's stored sample (not only against its own
  GPU direct-sum estimate), and its JSON cache returns the same choice on a second call;
* the full batched workload (512 instances, 18.3 M points, 64 charge vectors, one forest plan with
  a recorded graph): every stored oracle sample (4 instances x 2 vectors x 32 targets) within 1e-10
  for the FP64 path and 1e-6 for the FP32 matrix-core M2L.
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
from golden_io import load, load_forest  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.fixture(scope="module")
def uniform():
    w = workloads.uniform_1m(seed=1)
    return w, _t(w.x), _t(w.y), _t(w.q[0])


def test_uniform_1m_bench_plan_vs_oracle(uniform):
    w, x, y, q = uniform
    plan = F.HalfPlaneFMM(x, y, 1.0, p=20, leaf_size=32, near_walk=1, near_groups=2)
    info = plan.info()
    assert (info["p"], info["leaf_size"], info["near_walk"], info["near_groups"]) == (20, 32, 1, 2)
    phi = plan(q).cpu().numpy()
    plan.close()
    idx, ref = load("uniform_1m")
    err = D.rel_l2(phi[idx], ref)
    im = D.imag_part_real_impedance(w.x, w.y, w.q[0], 1.0)
    err_im = float(np.max(np.abs(phi.imag - im)) / np.max(np.abs(im)))
    print(f"uniform_1m p=20 leaf=32 near (1,2): rel-l2 at 256 targets {err:.3e}; Im part max rel {err_im:.3e}",
          flush=True)
    assert np.all(np.isfinite(phi))
    assert err <= 1e-10
    assert err_im < 1e-12


@pytest.mark.parametrize("tol", [1e-8, 1e-10])
def test_tuned_plan_meets_tolerance_vs_oracle(uniform, tol):
    w, x, y, q = uniform
    r = F.tune(x, y, q, 1.0, tol=tol, use_cache=False)
    print(f"tune tol={tol:g}: {r}", flush=True)
    assert r["rel_l2"] <= tol and not r["cached"]
    plan = F.HalfPlaneFMM(x, y, 1.0, p=r["p"], leaf_size=r["leaf_size"], near_walk=r["near_walk"],
                          near_groups=r["near_groups"], m2l_fp32=r["m2l_fp32"])
    phi = plan(q).cpu().numpy()
    plan.close()
    idx, ref = load("uniform_1m")
    err = D.rel_l2(phi[idx], ref)
    print(f"tuned plan (p={r['p']}, leaf={r['leaf_size']}): rel-l2 vs oracle sample {err:.3e}", flush=True)
    assert err <= tol


def test_tune_cache_roundtrip(uniform, tmp_path, monkeypatch):
    w, x, y, q = uniform
    monkeypatch.setenv("FMMHP_TUNE_CACHE", str(tmp_path / "tune.json"))
    a = F.tune(x, y, q, 1.0, tol=1e-6)
    b = F.tune(x, y, q, 1.0, tol=1e-6)
    assert not a["cached"] and b["cached"] and a["cache_key"] == b["cache_key"]
    for k in ("p", "leaf_size", "near_walk", "near_groups", "m2l_fp32", "rel_l2"):
        assert a[k] == b[k], k
    c = F.tune(x, y, q, 1.0 + 0.5j, tol=1e-6, use_cache=True)  # another impedance class: a new entry
    assert not c["cached"] and c["cache_key"] != a["cache_key"]


@pytest.fixture(scope="module")
def forest():
    g = load_forest()
    assert g is not None, "tests/golden/batched_forest_direct_sample.txt is missing"
    x, y, off, lams, q = workloads.batched_forest(seed=1)
    return g, off, lams, _t(x), _t(y), _t(q)


@pytest.mark.parametrize("fp32,tol", [(False, 1e-10), (True, 1e-6)])
def test_batched_forest_full_vs_oracle(forest, fp32, tol):
    (ks, vs, idx, ref), off, lams, x, y, q = forest
    nv, n = q.shape
    assert (nv, len(lams)) == (64, 512)
    st = torch.cuda.Stream(DEV)
    with torch.cuda.stream(st):
        plan = F.HalfPlaneFMM.batched(x, y, off, lams.tolist(), p=20, leaf_size=32, graph=True, m2l_fp32=fp32)
        out = torch.empty((nv, n), dtype=torch.complex128, device=DEV)
        plan(q, out=out)   # records the graph
        out.zero_()
        plan(q, out=out)   # replays it
        st.synchronize()
        pos = torch.as_tensor(off[ks] + idx, device=DEV)
        got = out[torch.as_tensor(vs, device=DEV), pos].cpu().numpy()
        plan.close()
        del out
    err = D.rel_l2(got, ref)
    per = {}
    for k in np.unique(ks):
        for v in np.unique(vs):
            m = (ks == k) & (vs == v)
            per[(int(k), int(v))] = D.rel_l2(got[m], ref[m])
    worst = max(per.values())
    print(f"batched forest (fp32 M2L={fp32}): rel-l2 over {ref.size} samples {err:.3e}; worst "
          f"(instance, vector) {worst:.3e}", flush=True)
    assert np.all(np.isfinite(got))
    assert err <= tol
    assert worst <= 10 * tol
