"""GPU parity of batched plans (forests of independent instances) and of multi-vector evaluation.

* the forest's tree and lists are bit-exact against the reference forest (oracle/tree.py);
* every instance's potentials match the oracle's direct sum over that instance alone
  (rel-l2 <= 1e-10 at p = 30), for all-real impedances (surface term per instance) and for mixed
  real and complex ones;
* a forest evaluates each instance exactly as a plain plan of that instance would (same boxes,
  same summation order): equal to 1e-14;
* n_vec vectors in one call (eight at a time plus a remainder) equal one call per vector;
* the adjoint of a forest gives each instance's impedance gradient.
"""
import numpy as np
import pytest
import torch

import paper_2507_21913_amd as F
from oracle import direct as D
from oracle import grad as GR
from oracle import tree as T

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def _forest(sizes, seed, nvec=1):
    """Instances of the batched workload's shape: uniform in [x0, x0 + 1] x [0.01, 1.01]."""
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for n in sizes:
        x0 = rng.uniform(-3, 3)
        xs.append(x0 + rng.uniform(0, 1, n))
        ys.append(rng.uniform(0.01, 1.01, n))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    q = rng.standard_normal((nvec, off[-1]))
    return np.concatenate(xs), np.concatenate(ys), off, q


def _compare_trees(got, ref):
    assert got["nbox"] == ref["nbox"]
    for k in ("level", "bx", "by", "first", "count", "parent", "leaf", "child_first", "nchild", "perm"):
        assert np.array_equal(got[k], ref[k]), k
    for name in "UVWX":
        assert np.array_equal(got[name + "_off"], ref[name + "_off"]), name
        assert np.array_equal(got[name + "_ent"], ref[name + "_ent"]), name


@pytest.mark.parametrize("sizes,leaf", [([900, 40, 2500, 3, 700], 16), ([200] * 12, 8), ([1, 5000], 30)])
def test_forest_tree_bitexact(sizes, leaf):
    x, y, off, _ = _forest(sizes, 1)
    plan = F.HalfPlaneFMM.batched(_t(x), _t(y), off, [1.0] * len(sizes), p=10, leaf_size=leaf)
    assert plan.info()["n_inst"] == len(sizes)
    _compare_trees(plan.export_tree(), T.build_forest(x, y, off, leaf))
    plan.close()


@pytest.mark.parametrize("imps", [[1.0, 2.5, 0.3, 4.0], [1.0, 1.0 + 0.5j, 0.3 + 1.1j, 2.0]])
def test_forest_potentials_vs_oracle(imps):
    sizes = [1500, 300, 2000, 800]
    x, y, off, q = _forest(sizes, 5)
    plan = F.HalfPlaneFMM.batched(_t(x), _t(y), off, imps, p=30, leaf_size=20)
    phi = plan(_t(q[0])).cpu().numpy()
    for k in range(len(sizes)):
        a, b = off[k], off[k + 1]
        ref = D.potential(x[a:b], y[a:b], q[0, a:b], imps[k], workers=8)
        err = D.rel_l2(phi[a:b], ref)
        print(f"instance {k} (n={b - a}, Z={imps[k]}): rel-l2 {err:.2e}", flush=True)
        assert err < 1e-10, k
    plan.close()


@pytest.mark.parametrize("imps", [[1.0, 0.5, 3.0], [0.5 + 0.25j, 1.0 + 1.0j, 2.0 + 0.1j]])
def test_forest_equals_plain_plans(imps):
    """All-real or all-complex impedances (a mixed forest evaluates its real instances in the
    general two-local form, whose truncation error differs from the plain real-impedance form)."""
    sizes = [1200, 350, 2600]
    x, y, off, q = _forest(sizes, 9)
    plan = F.HalfPlaneFMM.batched(_t(x), _t(y), off, imps, p=20, leaf_size=24)
    phi = plan(_t(q[0])).cpu().numpy()
    for k in range(len(sizes)):
        a, b = off[k], off[k + 1]
        pk = F.HalfPlaneFMM(_t(x[a:b]), _t(y[a:b]), imps[k], p=20, leaf_size=24)
        ref = pk(_t(q[0, a:b])).cpu().numpy()
        pk.close()
        err = D.rel_l2(phi[a:b], ref)
        print(f"instance {k}: forest vs plain rel-l2 {err:.2e}", flush=True)
        assert err <= 1e-14, (k, err)
    plan.close()


@pytest.mark.parametrize("imp", [2.0, 1.0 + 0.5j])
def test_multivector_equals_single(imp):
    x, y, off, q = _forest([3000], 13, nvec=11)
    plan = F.HalfPlaneFMM(_t(x), _t(y), imp, p=20, leaf_size=24)
    many = plan(_t(q)).cpu().numpy()
    for v in range(11):
        one = plan(_t(q[v])).cpu().numpy()
        assert D.rel_l2(many[v], one) < 1e-14, v
    plan.close()


def test_forest_multivector_vs_oracle():
    sizes = [700, 1600, 90]
    imps = [0.2, 5.0, 1.0]
    x, y, off, q = _forest(sizes, 17, nvec=9)
    plan = F.HalfPlaneFMM.batched(_t(x), _t(y), off, imps, p=30, leaf_size=16)
    phi = plan(_t(q)).cpu().numpy()
    for k in range(len(sizes)):
        a, b = off[k], off[k + 1]
        ref = D.potential(x[a:b], y[a:b], q[:, a:b], imps[k], workers=8)
        for v in (0, 5, 8):
            assert D.rel_l2(phi[v, a:b], ref[v]) < 1e-10, (k, v)
    plan.close()


def test_forest_backward_per_instance_impedance_gradient():
    sizes = [600, 900]
    imps = [2.0, 1.0 + 0.5j]
    x, y, off, q = _forest(sizes, 21)
    rng = np.random.default_rng(4)
    g = rng.standard_normal(off[-1]) + 1j * rng.standard_normal(off[-1])
    plan = F.HalfPlaneFMM.batched(_t(x), _t(y), off, imps, p=30, leaf_size=16)
    r = plan.backward(_t(q[0]), _t(g))
    for k in range(len(sizes)):
        a, b = off[k], off[k + 1]
        ref = GR.sampled_gradients(x[a:b], y[a:b], q[0, a:b], imps[k], g[a:b], np.arange(b - a), workers=8,
                                   want_Z=True)
        assert D.rel_l2(r["q"].cpu().numpy()[a:b], ref["grad_q"]) < 1e-10
        assert D.rel_l2(r["x"].cpu().numpy()[a:b], ref["grad_x"]) < 1e-10
        assert D.rel_l2(r["y"].cpu().numpy()[a:b], ref["grad_y"]) < 1e-10
        assert abs(r["lambda"][k] - ref["grad_Z"]) < 1e-10 * abs(ref["grad_Z"]), k
    plan.close()


@pytest.mark.parametrize("imps", [[10.0, 7.5, 0.1], [10.0, 8.0 + 2.0j, 6.0]])
def test_large_impedance_instances_vs_oracle(imps):
    """The batched workload's largest impedances (|Z| up to 10 on a root square of side 2.02): the
    coarse-level reaction M2L coefficients need |Z| * distance up to ~21, where the upward I_n
    recursion amplifies rounding by ~1e8 (extended-precision tables)."""
    sizes = [2000, 1200, 700]
    x, y, off, q = _forest(sizes, 31)
    plan = F.HalfPlaneFMM.batched(_t(x), _t(y), off, imps, p=30, leaf_size=20)
    phi = plan(_t(q[0])).cpu().numpy()
    for k in range(len(sizes)):
        a, b = off[k], off[k + 1]
        ref = D.potential(x[a:b], y[a:b], q[0, a:b], imps[k], workers=8)
        err = D.rel_l2(phi[a:b], ref)
        print(f"instance {k} (n={b - a}, Z={imps[k]}): rel-l2 {err:.2e}", flush=True)
        assert err < 1e-10, k
    plan.close()


def test_graph_replays_match_eager():
    """FMMHP_FLAG_GRAPH: the first call records, later calls replay; every replay (with eager work
    and synchronisations in between) equals the eager evaluation bitwise; new buffers re-record."""
    sizes = [1500, 900, 2500]
    imps = [2.0, 5.0, 0.7]
    x, y, off, q = _forest(sizes, 41, nvec=10)
    eager = F.HalfPlaneFMM.batched(_t(x), _t(y), off, imps, p=20, leaf_size=24)
    ref = eager(_t(q)).cpu().numpy()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        plan = F.HalfPlaneFMM.batched(_t(x), _t(y), off, imps, p=20, leaf_size=24, graph=True)
        qt = _t(q)
        out = torch.empty((10, off[-1]), dtype=torch.complex128, device=DEV)
        for rep in range(4):
            out.zero_()
            plan(qt, out=out)
            st.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), rep
            eager(_t(q[0]))  # unrelated eager work between replays
            torch.cuda.synchronize()
        # new buffers: a new recording (2 q: every operation scales exactly, so 2 phi bitwise)
        q2 = _t(2.0 * q)
        out2 = torch.empty_like(out)
        plan(q2, out=out2)
        st.synchronize()
        assert np.array_equal(out2.cpu().numpy(), 2.0 * ref)
        # a graph plan needs an output buffer of its own (else every call would re-record)
        with pytest.raises(ValueError):
            plan(qt)
    # the null stream runs eagerly
    plan_null = F.HalfPlaneFMM.batched(_t(x), _t(y), off, imps, p=20, leaf_size=24, graph=True)
    out3 = torch.empty_like(out)
    plan_null(_t(q), out=out3)
    assert np.array_equal(out3.cpu().numpy(), ref)
    plan.close()
    plan_null.close()
    eager.close()
