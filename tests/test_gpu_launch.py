"""GPU checks of the near-field launch shapes (fmmhp_opts.near_walk, near_groups): every shape
computes the same sums (only the order of additions differs), for the potential, several charge
vectors at once and the adjoint; the defaults depend on p; the autotuner returns a valid shape.
Walks 3 and 4 (symmetric leaf pairs; walk 4 with the pairs blocked in registers) are also checked on
leaves of more than 64 points, forests, separate targets, the Dirichlet and Neumann kernels,
coincident points, and two evaluations in a row.
"""
import numpy as np
import pytest
import torch

import paper_2507_21913_amd as F
from oracle import direct as D

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SHAPES = [(1, 1), (1, 2), (1, 16), (2, 4), (2, 8), (3, 1), (3, 2), (3, 16), (4, 1), (4, 2), (4, 16), (0, 0)]


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def _problem(n, seed, nvec=1):
    """Most points in a band near y = 0 (image U entries, adaptive leaves), the rest uniform,
    with a few coincident pairs."""
    rng = np.random.default_rng(seed)
    m = n // 2
    xb = rng.uniform(0.0, 1.0, m)
    yb = rng.uniform(1e-3, 0.05, m)
    x = np.concatenate([xb, rng.uniform(0.0, 1.0, n - m)])
    y = np.concatenate([yb, rng.uniform(1e-3, 1.0, n - m)])
    x[10:20] = x[0:10]
    y[10:20] = y[0:10]
    return x, y, rng.standard_normal((nvec, n))


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j])
def test_shapes_agree_and_match_oracle(Z):
    x, y, q = _problem(6000, 3)
    ref = D.potential(x, y, q[0], Z, workers=8)
    out = {}
    for w, g in SHAPES:
        plan = F.HalfPlaneFMM(_t(x), _t(y), Z, p=30, leaf_size=16, near_walk=w, near_groups=g)
        info = plan.info()
        if w:
            assert (info["near_walk"], info["near_groups"]) == (w, g)
        out[(w, g)] = plan(_t(q[0])).cpu().numpy()
        plan.close()
        err = D.rel_l2(out[(w, g)], ref)
        print(f"Z={Z} shape {(w, g)}: rel-l2 vs oracle {err:.2e}", flush=True)
        assert err < 1e-10
    base = out[(1, 2)]
    for k, v in out.items():
        assert D.rel_l2(v, base) < 1e-13, k


def test_shapes_agree_multivector_and_adjoint():
    x, y, q = _problem(5000, 7, nvec=9)
    rng = np.random.default_rng(1)
    g = rng.standard_normal(x.size) + 1j * rng.standard_normal(x.size)
    res = {}
    for w, gr in [(1, 2), (2, 4), (3, 2), (4, 2)]:
        plan = F.HalfPlaneFMM(_t(x), _t(y), 2.0, p=20, leaf_size=24, near_walk=w, near_groups=gr)
        phi = plan(_t(q)).cpu().numpy()
        b = plan.backward(_t(q[0]), _t(g))
        res[w] = (phi, {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in b.items()})
        plan.close()
    for w in (2, 3, 4):
        for v in range(9):
            assert D.rel_l2(res[1][0][v], res[w][0][v]) < 1e-13, (w, v)
        for k in ("q", "x", "y"):
            assert D.rel_l2(res[1][1][k], res[w][1][k]) < 1e-12, (w, k)
        assert abs(res[1][1]["lambda"] - res[w][1]["lambda"]) < 1e-12 * abs(res[w][1]["lambda"])


def test_default_shape_by_order():
    x, y, _ = _problem(3000, 11)
    for p, want in ((20, (1, 2)), (30, (2, 4))):
        plan = F.HalfPlaneFMM(_t(x), _t(y), 1.0, p=p, leaf_size=16)
        info = plan.info()
        assert (info["near_walk"], info["near_groups"]) == want, (p, info["near_walk"], info["near_groups"])
        plan.close()


def test_tune_returns_a_shape():
    x, y, q = _problem(20000, 5)
    r = F.tune(_t(x), _t(y), _t(q[0]), 1.0, tol=1e-8, leaf_sizes=[24, 40])
    print("tune:", r, flush=True)
    assert r["near_walk"] in (1, 2, 3, 4) and 1 <= r["near_groups"] <= 16
    plan = F.HalfPlaneFMM(_t(x), _t(y), 1.0, p=r["p"], leaf_size=r["leaf_size"], near_walk=r["near_walk"],
                          near_groups=r["near_groups"])
    info = plan.info()
    assert (info["near_walk"], info["near_groups"]) == (r["near_walk"], r["near_groups"])
    plan.close()


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j])
def test_serial_schedule_same_results(Z):
    """FMMHP_FLAG_SERIAL (every kernel on the eval stream) computes the same sums: bitwise equal
    potentials, and the k_m2l launch timing counts two launches per evaluation."""
    x, y, q = _problem(20000, 17)
    out = {}
    for serial in (False, True):
        plan = F.HalfPlaneFMM(_t(x), _t(y), Z, p=20, leaf_size=16, serial=serial)
        plan.set_timing(True)
        out[serial] = plan(_t(q[0])).cpu().numpy()
        ms, n = plan.m2l_kernel_times()
        plan.set_timing(False)
        plan.close()
        assert ms > 0.0 and n >= 1
    assert np.array_equal(out[False], out[True])


@pytest.mark.parametrize("n,groups", [(1500, 2), (70001, 1), (70001, 2)])
def test_xcd_chunk_mapping_covers_every_target(n, groups):
    """The prefetching walk's workgroups take 256-target chunks by XCD (one contiguous range of
    chunks per XCD): with fewer chunks than eight workgroups (n = 1500), more chunks than
    workgroups with a remainder (70,001 targets, 274 chunks, 256 workgroups) and more workgroups
    than chunks, every target's near-field sums must equal the plain walk's (which takes targets
    by plain grid stride), so no chunk is skipped or taken twice."""
    x, y, q = _problem(n, 11)
    res = {}
    for w, g in ((1, groups), (2, 4)):
        plan = F.HalfPlaneFMM(_t(x), _t(y), 1.0 + 0.25j, p=20, leaf_size=32, near_walk=w, near_groups=g)
        res[w] = plan(_t(q[0])).cpu().numpy()
        plan.close()
    diff = np.abs(res[1] - res[2])
    scale = np.max(np.abs(res[2]))
    print(f"n={n} groups={groups}: max |walk1 - walk2| / max|phi| {diff.max() / scale:.2e}", flush=True)
    assert np.all(np.isfinite(res[1]))
    assert diff.max() <= 1e-12 * scale


@pytest.mark.parametrize("walk", [3, 4])
@pytest.mark.parametrize("bc", ["robin", "dirichlet", "neumann"])
def test_symmetric_walk_large_leaves_and_conditions(bc, walk):
    """Walks 3 and 4 with leaves of up to 96 points (chunks of 64 targets share one lane layout), with
    max_level 4 (leaves far above leaf_size, many coincident-free pairs), and the three boundary
    conditions (image sign), against the oracle and walk 1."""
    x, y, q = _problem(8000, 23, nvec=2)
    Z = 1.0 + 0.5j if bc == "robin" else 1.0
    ref = D.potential(x, y, q[1], Z, workers=8, bc=bc)
    for leaf, lmax in ((96, 0), (32, 4)):
        res = {}
        for w in (1, walk):
            plan = F.HalfPlaneFMM(_t(x), _t(y), Z, p=20, leaf_size=leaf, max_level=lmax, near_walk=w,
                                  near_groups=2, bc=bc)
            res[w] = plan(_t(q)).cpu().numpy()
            plan(_t(q))  # a second evaluation reuses the partial sums' workspace
            res[w] = plan(_t(q)).cpu().numpy()
            plan.close()
        err = D.rel_l2(res[walk][1], ref)
        print(f"{bc} leaf {leaf} max_level {lmax}: walk {walk} rel-l2 vs oracle {err:.2e}, vs walk 1 "
              f"{D.rel_l2(res[walk], res[1]):.2e}", flush=True)
        assert err < 1e-9 and D.rel_l2(res[walk], res[1]) < 1e-13


@pytest.mark.parametrize("walk", [3, 4])
def test_symmetric_walk_forest_and_targets(walk):
    """Walks 3 and 4 on a forest (pairs never cross instances) and on a plan with separate targets (the
    target-only points carry no charge) against walk 1 and the oracle."""
    sizes = [1800, 600, 2500]
    imps = [0.5, 3.0, 1.0 + 0.4j]
    xs, ys, qs = [], [], []
    for k, m in enumerate(sizes):
        x, y, q = _problem(m, 40 + k, nvec=8)
        xs.append(x)
        ys.append(y)
        qs.append(q)
    off = np.concatenate([[0], np.cumsum(sizes)])
    X, Y, Q = np.concatenate(xs), np.concatenate(ys), np.concatenate(qs, axis=1)
    res = {}
    for w in (1, walk):
        plan = F.HalfPlaneFMM.batched(_t(X), _t(Y), off, imps, p=20, leaf_size=24, near_walk=w, near_groups=2)
        res[w] = plan(_t(Q)).cpu().numpy()
        plan.close()
    assert D.rel_l2(res[walk], res[1]) < 1e-13
    for k in range(3):
        ref = D.potential(xs[k], ys[k], qs[k][5], imps[k], workers=8)
        assert D.rel_l2(res[walk][5, off[k]:off[k + 1]], ref) < 1e-10, k
    x, y, q = _problem(3000, 51)
    rng = np.random.default_rng(2)
    xt, yt = rng.uniform(0.0, 1.0, 900), rng.uniform(0.0, 0.3, 900)
    yt[:30] = 0.0
    out = {}
    for w in (1, walk):
        plan = F.HalfPlaneFMM.with_targets(_t(x), _t(y), _t(xt), _t(yt), 1.0, p=20, leaf_size=16, near_walk=w,
                                           near_groups=2)
        out[w] = plan(_t(q[0])).cpu().numpy()
        plan.close()
    ref = D.potential(x, y, q[0], 1.0, xt=xt, yt=yt, workers=8)
    assert D.rel_l2(out[walk], ref) < 1e-10 and D.rel_l2(out[walk], out[1]) < 1e-13
