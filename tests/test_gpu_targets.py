"""GPU parity of plans with separate targets (fmmhp_plan_create_targets) against the oracle's direct
sum at the same targets: the paper's Example 2 (Section 5; eight charged unit circles, a field
mesh on [-4.4, 4.4] x [0, 4.2] that includes y = 0), its error decay in p, targets that coincide
with sources, a complex impedance, several and complex charge vectors, and the field (potential and
gradient, fmmhp_eval_field).  Tolerance: rel-l2 1e-10 at p = 30.
"""
import numpy as np
import pytest
import torch

import paper_2507_21913_amd as F
import workloads
from oracle import direct as D

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


@pytest.fixture(scope="module")
def ex2():
    d = workloads.example2_sized(4000)
    d["ref"] = D.potential(d["src_x"], d["src_y"], d["q"], d["impedance"], xt=d["tgt_x"], yt=d["tgt_y"],
                           workers=8)
    return d


def _plan(d, p, leaf=24, Z=None, **kw):
    return F.HalfPlaneFMM.with_targets(_t(d["src_x"]), _t(d["src_y"]), _t(d["tgt_x"]), _t(d["tgt_y"]),
                                       d["impedance"] if Z is None else Z, p=p, leaf_size=leaf, **kw)


def test_example2_vs_oracle(ex2):
    plan = _plan(ex2, 30)
    info = plan.info()
    assert info["n_sources"] == ex2["src_x"].size and info["n"] == ex2["src_x"].size + ex2["tgt_x"].size
    phi = plan(_t(ex2["q"])).cpu().numpy()
    plan.close()
    assert phi.shape == ex2["ref"].shape and np.all(np.isfinite(phi))
    err = D.rel_l2(phi, ex2["ref"])
    on_y0 = ex2["tgt_y"] == 0.0
    err0 = D.rel_l2(phi[on_y0], ex2["ref"][on_y0])
    print(f"Example 2 (N_field + 8 N_source = 4000) p=30: rel-l2 {err:.2e}, on y = 0 {err0:.2e}", flush=True)
    assert err < 1e-10 and err0 < 1e-10
    im = D.imag_part_real_impedance(ex2["src_x"], ex2["src_y"], ex2["q"], 1.0, xt=ex2["tgt_x"], yt=ex2["tgt_y"])
    assert np.max(np.abs(phi.imag - im)) < 1e-10 * np.max(np.abs(im))


def test_example2_error_decays_with_p(ex2):
    errs = {}
    for p in (5, 10, 15, 20, 25):
        plan = _plan(ex2, p)
        errs[p] = D.rel_l2(plan(_t(ex2["q"])).cpu().numpy(), ex2["ref"])
        plan.close()
    print("Example 2 rel-l2 vs p:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    ps = sorted(errs)
    for a, b in zip(ps, ps[1:]):
        assert errs[b] < errs[a] / 4, (a, b, errs)
    assert errs[25] < 1e-8


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j])
def test_targets_on_sources_and_boundary(Z):
    rng = np.random.default_rng(8)
    ns = 3000
    xs = rng.uniform(0.0, 1.0, ns)
    ys = rng.uniform(1e-3, 0.3, ns)
    q = rng.standard_normal(ns)
    xt = np.concatenate([rng.uniform(0.0, 1.0, 1500), xs[:200], rng.uniform(0, 1, 300)])
    yt = np.concatenate([rng.uniform(0.0, 0.5, 1500), ys[:200], np.zeros(300)])
    plan = F.HalfPlaneFMM.with_targets(_t(xs), _t(ys), _t(xt), _t(yt), Z, p=30, leaf_size=16)
    phi = plan(_t(q)).cpu().numpy()
    plan.close()
    ref = D.potential(xs, ys, q, Z, xt=xt, yt=yt, workers=8)
    err = D.rel_l2(phi, ref)
    print(f"Z={Z}: targets on sources and on y = 0: rel-l2 {err:.2e}", flush=True)
    assert err < 1e-10


def test_multivector_and_complex_charges():
    rng = np.random.default_rng(9)
    ns, nt = 2500, 1800
    xs, ys = rng.uniform(0, 1, ns), rng.uniform(0.01, 1.0, ns)
    xt, yt = rng.uniform(-0.2, 1.2, nt), rng.uniform(0.0, 1.0, nt)
    Q = rng.standard_normal((3, ns))
    plan = F.HalfPlaneFMM.with_targets(_t(xs), _t(ys), _t(xt), _t(yt), 2.0, p=30, leaf_size=20)
    many = plan(_t(Q)).cpu().numpy()
    assert many.shape == (3, nt)
    ref = D.potential(xs, ys, Q, 2.0, xt=xt, yt=yt, workers=8)
    for v in range(3):
        assert D.rel_l2(many[v], ref[v]) < 1e-10, v
    qc = Q[0] + 1j * Q[1]
    got = plan(_t(qc)).cpu().numpy()
    assert D.rel_l2(got, ref[0] + 1j * ref[1]) < 1e-10
    with pytest.raises(F.FMMHPError):
        plan.backward(_t(Q[0]), _t(np.ones(ns, dtype=complex)))
    plan.close()


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j])
def test_field_at_targets_vs_oracle(ex2, Z):
    """fmmhp_eval_field on a plan with separate targets: potential and gradient at the Example 2
    mesh (boundary row included), and the Robin condition d_y phi + Z phi = 0 on y = 0."""
    from oracle import grad as GR
    plan = _plan(ex2, 30, Z=Z)
    phi, gx, gy = (t.cpu().numpy() for t in plan.field(_t(ex2["q"])))
    plan.close()
    ref = ex2["ref"] if Z == 1.0 else D.potential(ex2["src_x"], ex2["src_y"], ex2["q"], Z, xt=ex2["tgt_x"],
                                                  yt=ex2["tgt_y"], workers=8)
    rx, ry = GR.field_at(ex2["src_x"], ex2["src_y"], ex2["q"], Z, ex2["tgt_x"], ex2["tgt_y"], workers=8)
    e = (D.rel_l2(phi, ref), D.rel_l2(gx, rx), D.rel_l2(gy, ry))
    print(f"Z={Z} field at Example 2 mesh: rel-l2 phi {e[0]:.2e} d_x {e[1]:.2e} d_y {e[2]:.2e}", flush=True)
    assert max(e) < 1e-10
    b = ex2["tgt_y"] == 0.0
    res = np.abs(gy[b] + complex(Z) * phi[b])
    assert np.max(res) < 1e-9 * np.max(np.abs(gy[b]))


def test_field_sources_as_targets_vs_oracle():
    from oracle import grad as GR
    rng = np.random.default_rng(21)
    n = 3000
    x, y, q = rng.uniform(0, 1, n), rng.uniform(0.01, 1.01, n), rng.uniform(-1, 1, n)
    plan = F.HalfPlaneFMM(_t(x), _t(y), 1.0 + 0.5j, p=30, leaf_size=20)
    phi, gx, gy = (t.cpu().numpy() for t in plan.field(_t(q)))
    ref_phi = plan(_t(q)).cpu().numpy()
    plan.close()
    rx, ry = GR.potential_gradient(x, y, q, 1.0 + 0.5j)
    assert np.array_equal(phi, ref_phi) or D.rel_l2(phi, ref_phi) < 1e-14
    assert D.rel_l2(gx, rx) < 1e-10 and D.rel_l2(gy, ry) < 1e-10
