"""GPU parity of the Dirichlet and Neumann half-plane kernels (FMMHP_FLAG_DIRICHLET / _NEUMANN,
eq. (ddd1.2)) against the oracle: potentials on an adaptive point set near y = 0 (W and X lists,
image U entries) at p = 30 (rel-l2 1e-10), the boundary condition of each on y = 0 through separate
targets and the field, several vectors, a forest, and the adjoint (dl/dq against the oracle, zero
impedance gradient).  The impedance argument is ignored for these plans.
"""
import numpy as np
import pytest
import torch

import paper_2507_21913_amd as F
from oracle import direct as D
from oracle import grad as GR

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def _band(n, seed):
    rng = np.random.default_rng(seed)
    m = (3 * n) // 4
    xb = rng.uniform(0.0, 1.0, m)
    yb = 0.05 + 0.03 * np.sin(6 * np.pi * xb) + rng.uniform(-1e-3, 1e-3, m)
    x = np.concatenate([xb, rng.uniform(0.0, 1.0, n - m)])
    y = np.concatenate([yb, rng.uniform(1e-3, 1.0, n - m)])
    return x, y, rng.standard_normal((3, n))


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_potential_vs_oracle(bc):
    x, y, q = _band(4000, 1)
    plan = F.HalfPlaneFMM(_t(x), _t(y), 0.0, p=30, leaf_size=8, bc=bc)
    info = plan.info()
    assert info["list_len"][2] > 0 and info["list_len"][3] > 0
    phi = plan(_t(q)).cpu().numpy()
    plan.close()
    ref = D.potential(x, y, q, 1.0, workers=8, bc=bc)
    for v in range(3):
        err = D.rel_l2(phi[v], ref[v])
        print(f"{bc} vector {v}: rel-l2 {err:.2e}", flush=True)
        assert err < 1e-10
    assert np.max(np.abs(phi.imag)) < 1e-12 * np.max(np.abs(phi.real))


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_boundary_condition_at_targets(bc):
    x, y, q = _band(3000, 2)
    xt = np.concatenate([np.linspace(0, 1, 200), np.linspace(0, 1, 200)])
    yt = np.concatenate([np.zeros(200), np.full(200, 0.02)])
    plan = F.HalfPlaneFMM.with_targets(_t(x), _t(y), _t(xt), _t(yt), 1.0, p=30, leaf_size=12, bc=bc)
    phi, gx, gy = (t.cpu().numpy() for t in plan.field(_t(q[0])))
    plan.close()
    ref = D.potential(x, y, q[0], 1.0, xt=xt, yt=yt, workers=8, bc=bc)
    rx, ry = GR.field_at(x, y, q[0], 1.0, xt, yt, workers=8, bc=bc)
    e = (D.rel_l2(phi, ref), D.rel_l2(gx, rx), D.rel_l2(gy, ry))
    print(f"{bc} at targets: rel-l2 phi {e[0]:.2e} d_x {e[1]:.2e} d_y {e[2]:.2e}", flush=True)
    assert max(e) < 1e-10
    b = yt == 0.0
    if bc == "dirichlet":
        assert np.max(np.abs(phi[b])) < 1e-10 * np.max(np.abs(phi[~b]))
    else:
        assert np.max(np.abs(gy[b])) < 1e-10 * np.max(np.abs(gx[b]))


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_forest_and_adjoint(bc):
    rng = np.random.default_rng(5)
    sizes = [1200, 700]
    x = np.concatenate([rng.uniform(0, 1, n) for n in sizes])
    y = np.concatenate([rng.uniform(0.01, 1.01, n) for n in sizes])
    off = np.concatenate([[0], np.cumsum(sizes)])
    q = rng.standard_normal(off[-1])
    forest = F.HalfPlaneFMM.batched(_t(x), _t(y), off, [0.0, 0.0], p=30, leaf_size=16, bc=bc)
    phi = forest(_t(q)).cpu().numpy()
    forest.close()
    for k in range(2):
        a, b = off[k], off[k + 1]
        ref = D.potential(x[a:b], y[a:b], q[a:b], 1.0, workers=8, bc=bc)
        assert D.rel_l2(phi[a:b], ref) < 1e-10, k
    a, b = off[0], off[1]
    g = rng.standard_normal(b - a) + 1j * rng.standard_normal(b - a)
    plan = F.HalfPlaneFMM(_t(x[a:b]), _t(y[a:b]), 3.0, p=30, leaf_size=16, bc=bc)
    r = plan.backward(_t(q[a:b]), _t(g))
    plan.close()
    ref_q = np.real(D.potential(x[a:b], y[a:b], np.conj(g), 1.0, workers=8, bc=bc))
    assert D.rel_l2(r["q"].cpu().numpy(), ref_q) < 1e-10
    assert r["lambda"] == 0
