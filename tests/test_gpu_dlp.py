"""GPU parity of the double-layer potential (fmmhp_eval_double_layer) against the oracle's direct
sum of mu_j n_j . grad_{r_j} G: the three boundary conditions, a complex impedance, coincident points
and points close to y = 0 (near-field, image and reaction terms), complex and several densities,
both near-field walks, the FP32 M2L, a forest, separate targets on the paper's Example 2 mesh
(Section 5) with the circles' outward normals, where unit density also gives the classical jump
values -1 inside a circle and 0 outside, and the error decay in p.  Tolerance: rel-l2 1e-10 at
p = 30 (the expansions are those of the potential, differentiated in the source).
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


def _problem(n, seed):
    """Half the points in a band near y = 0, the rest uniform, a few coincident pairs; random
    unit normals and densities."""
    rng = np.random.default_rng(seed)
    m = n // 2
    x = np.concatenate([rng.uniform(0.0, 1.0, m), rng.uniform(0.0, 1.0, n - m)])
    y = np.concatenate([rng.uniform(1e-3, 0.05, m), rng.uniform(1e-3, 1.0, n - m)])
    x[10:20] = x[0:10]
    y[10:20] = y[0:10]
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    return x, y, np.cos(th), np.sin(th), rng.standard_normal(n)


@pytest.mark.parametrize("bc,Z", [("robin", 1.0), ("robin", 1.0 + 0.5j), ("robin", 4.0),
                                  ("dirichlet", 1.0), ("neumann", 1.0)])
def test_double_layer_vs_oracle(bc, Z):
    x, y, nx, ny, mu = _problem(5000, 3)
    ref = D.double_layer(x, y, nx, ny, mu, Z, bc=bc, workers=8)
    for walk in (1, 2):
        plan = F.HalfPlaneFMM(_t(x), _t(y), Z, p=30, leaf_size=16, near_walk=walk, bc=bc)
        got = plan.double_layer(_t(mu), _t(nx), _t(ny)).cpu().numpy()
        plan.close()
        err = D.rel_l2(got, ref)
        print(f"bc={bc} Z={Z} walk={walk}: double layer rel-l2 {err:.2e}", flush=True)
        assert np.all(np.isfinite(got)) and err < 1e-10


def test_complex_and_several_densities():
    x, y, nx, ny, _ = _problem(4000, 5)
    rng = np.random.default_rng(6)
    M = rng.standard_normal((3, x.size))
    Z = 2.0
    plan = F.HalfPlaneFMM(_t(x), _t(y), Z, p=30, leaf_size=24)
    many = plan.double_layer(_t(M), _t(nx), _t(ny)).cpu().numpy()
    mc = M[0] + 1j * M[1]
    got_c = plan.double_layer(_t(mc), _t(nx), _t(ny)).cpu().numpy()
    # the single layer on the same plan is unchanged by a double-layer call
    phi = plan(_t(M[2])).cpu().numpy()
    plan.close()
    ref = D.double_layer(x, y, nx, ny, M, Z, workers=8)
    assert many.shape == (3, x.size)
    for v in range(3):
        assert D.rel_l2(many[v], ref[v]) < 1e-10, v
    assert D.rel_l2(got_c, ref[0] + 1j * ref[1]) < 1e-10
    assert D.rel_l2(phi, D.potential(x, y, M[2], Z, workers=8)) < 1e-10


def test_fp32_m2l_and_forest():
    x, y, nx, ny, mu = _problem(4000, 9)
    ref = D.double_layer(x, y, nx, ny, mu, 1.0, workers=8)
    plan = F.HalfPlaneFMM(_t(x), _t(y), 1.0, p=20, leaf_size=24, m2l_fp32=True)
    e32 = D.rel_l2(plan.double_layer(_t(mu), _t(nx), _t(ny)).cpu().numpy(), ref)
    plan.close()
    print(f"FP32 M2L double layer rel-l2 {e32:.2e}", flush=True)
    assert e32 < 1e-6
    # two instances with different impedances in one forest
    h = x.size // 2
    Zs = [1.0, 1.0 + 0.5j]
    plan = F.HalfPlaneFMM.batched(_t(x), _t(y), [0, h, x.size], Zs, p=30, leaf_size=24)
    got = plan.double_layer(_t(mu), _t(nx), _t(ny)).cpu().numpy()
    plan.close()
    for k, (a, b) in enumerate(((0, h), (h, x.size))):
        r = D.double_layer(x[a:b], y[a:b], nx[a:b], ny[a:b], mu[a:b], Zs[k], workers=8)
        assert D.rel_l2(got[a:b], r) < 1e-10, k


@pytest.fixture(scope="module")
def ex2():
    d = workloads.example2_sized(4000)
    ns = d["src_x"].size // 8
    cx = np.repeat([-3.3 + 2.2 * (k % 4) for k in range(8)], ns)
    cy = np.repeat([1.01] * 4 + [3.2] * 4, ns)
    d["nx"], d["ny"] = d["src_x"] - cx, d["src_y"] - cy  # outward unit normals of the unit circles
    d["cx"], d["cy"] = cx, cy
    return d


@pytest.mark.parametrize("bc,Z", [("robin", 1.0), ("robin", 1.0 + 0.5j), ("neumann", 1.0)])
def test_example2_targets_vs_oracle_and_jump(ex2, bc, Z):
    d = ex2
    plan = F.HalfPlaneFMM.with_targets(_t(d["src_x"]), _t(d["src_y"]), _t(d["tgt_x"]), _t(d["tgt_y"]), Z,
                                       p=30, leaf_size=24, bc=bc)
    got = plan.double_layer(_t(d["q"]), _t(d["nx"]), _t(d["ny"])).cpu().numpy()
    plan.close()
    ref = D.double_layer(d["src_x"], d["src_y"], d["nx"], d["ny"], d["q"], Z, xt=d["tgt_x"], yt=d["tgt_y"],
                         bc=bc, workers=8)
    err = D.rel_l2(got, ref)
    # unit density (the weights are the arc lengths): -1 inside a circle, 0 outside, for targets
    # well away from every circle (the midpoint rule's error decays like exp(-N dist))
    xs8, ys8 = d["cx"][::d["src_x"].size // 8], d["cy"][::d["src_x"].size // 8]
    r = np.hypot(d["tgt_x"][:, None] - xs8[None, :], d["tgt_y"][:, None] - ys8[None, :])
    far = np.all(np.abs(r - 1.0) > 0.1, axis=1)
    inside = np.any(r < 1.0, axis=1)
    want = np.where(inside, -1.0, 0.0)
    jump = np.max(np.abs(got[far] - want[far]))
    print(f"Example 2 double layer bc={bc} Z={Z}: rel-l2 {err:.2e}, jump identity {jump:.2e} "
          f"({far.sum()} targets)", flush=True)
    assert err < 1e-10 and jump < 1e-9


def test_error_decays_with_p():
    x, y, nx, ny, mu = _problem(4000, 13)
    ref = D.double_layer(x, y, nx, ny, mu, 1.0, workers=8)
    errs = {}
    for p in (5, 10, 15, 20, 25, 40):
        plan = F.HalfPlaneFMM(_t(x), _t(y), 1.0, p=p, leaf_size=24)
        errs[p] = D.rel_l2(plan.double_layer(_t(mu), _t(nx), _t(ny)).cpu().numpy(), ref)
        plan.close()
    print("double layer rel-l2 vs p:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    ps = sorted(errs)
    for a, b in zip(ps[:-2], ps[1:-1]):
        assert errs[b] < errs[a] / 4, (a, b, errs)
    assert errs[25] < 1e-8 and errs[40] < 1e-11


def test_invalid_arguments():
    x, y, nx, ny, mu = _problem(500, 1)
    plan = F.HalfPlaneFMM(_t(x), _t(y), 1.0, p=10, leaf_size=24)
    raw = torch.empty((1, x.size, 2), dtype=torch.float64, device=DEV)
    m, a, b = _t(mu), _t(nx), _t(ny)
    st = F.lib().fmmhp_eval_double_layer(plan._plan, 1, m.data_ptr(), 2, a.data_ptr(), b.data_ptr(),
                                         raw.data_ptr(), None)
    assert st != 0
    st = F.lib().fmmhp_eval_double_layer(plan._plan, 0, m.data_ptr(), 0, a.data_ptr(), b.data_ptr(),
                                         raw.data_ptr(), None)
    assert st != 0
    with pytest.raises(ValueError):
        plan.double_layer(m, a[:-1], b)
    plan.close()


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j])
def test_normal_derivative_at_targets(ex2, Z):
    """fmmhp_eval_normal_derivative at the Example 2 mesh with seeded target normals, against the
    oracle's field at the same targets projected on the normals."""
    from oracle import grad as GR
    d = ex2
    th = np.random.default_rng(17).uniform(0.0, 2.0 * np.pi, d["tgt_x"].size)
    tnx, tny = np.cos(th), np.sin(th)
    plan = F.HalfPlaneFMM.with_targets(_t(d["src_x"]), _t(d["src_y"]), _t(d["tgt_x"]), _t(d["tgt_y"]), Z,
                                       p=30, leaf_size=24)
    got = plan.normal_derivative(_t(d["q"]), _t(tnx), _t(tny)).cpu().numpy()
    plan.close()
    gx, gy = GR.field_at(d["src_x"], d["src_y"], d["q"], Z, d["tgt_x"], d["tgt_y"], workers=8)
    ref = tnx * gx + tny * gy
    err = D.rel_l2(got, ref)
    print(f"Z={Z} normal derivative at the Example 2 mesh: rel-l2 {err:.2e}", flush=True)
    assert err < 1e-10


def test_normal_derivative_sources_as_targets():
    from oracle import grad as GR
    x, y, nx, ny, mu = _problem(3000, 23)
    plan = F.HalfPlaneFMM(_t(x), _t(y), 2.0, p=30, leaf_size=20)
    got = plan.normal_derivative(_t(mu), _t(nx), _t(ny)).cpu().numpy()
    plan.close()
    rx, ry = GR.potential_gradient(x, y, mu, 2.0)
    assert D.rel_l2(got, nx * rx + ny * ry) < 1e-10


def test_degenerate_sizes_and_zero_normals():
    """One source, two coincident sources, leaf size 1, and zero normals (an exactly zero layer)."""
    rng = np.random.default_rng(31)
    cases = [(np.array([0.4]), np.array([0.2])),
             (np.array([0.4, 0.4, 0.7]), np.array([0.2, 0.2, 0.05])),
             (rng.uniform(0, 1, 50), rng.uniform(1e-3, 1, 50))]
    for leaf, (x, y) in zip((40, 40, 1), cases):
        th = rng.uniform(0, 2 * np.pi, x.size)
        nx, ny, mu = np.cos(th), np.sin(th), rng.standard_normal(x.size)
        for Z in (1.0, 1.0 + 0.5j):
            plan = F.HalfPlaneFMM(_t(x), _t(y), Z, p=30, leaf_size=leaf)
            got = plan.double_layer(_t(mu), _t(nx), _t(ny)).cpu().numpy()
            zero = plan.double_layer(_t(mu), _t(np.zeros_like(nx)), _t(np.zeros_like(ny))).cpu().numpy()
            plan.close()
            ref = D.double_layer(x, y, nx, ny, mu, Z, workers=1)
            assert np.all(np.isfinite(got)) and D.rel_l2(got, ref) < 1e-12, (x.size, Z)
            assert np.all(zero == 0.0)
