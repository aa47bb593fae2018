"""Pins of the oracle's gradients (oracle/grad.py) against central finite differences of the
oracle's direct-sum potential, and of the homogeneity identity the GPU adjoint uses for dL/dZ.

Loss: l = sum_i Re(conj(g_i) phi_i) with a fixed complex g (the form every real loss of the complex
potential takes to first order).  Finite differences use h = 1e-6 (relative where it matters);
central differences are then accurate to ~1e-9 relative, so a dropped term, a wrong sign or a wrong
index in any derivative shows up at O(1).
"""
import numpy as np
import pytest

from oracle import direct as D
from oracle import grad as GR
from oracle import kernel as K


def _problem(n=48, seed=3, dup=False):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, n)
    y = rng.uniform(0.02, 0.6, n)
    q = rng.uniform(-1.0, 1.0, n)
    g = rng.normal(size=n) + 1j * rng.normal(size=n)
    if dup:
        x[5], y[5] = x[9], y[9]
        x[17], y[17] = x[30], y[30]
    return x, y, q, g


def _loss(x, y, q, Z, g):
    return float(np.real(np.sum(np.conj(g) * D.potential_loops(x, y, q, Z))))


@pytest.mark.parametrize("Z", [1.0, 2.5, 1.0 + 0.5j, 0.3 + 1.1j])
def test_grad_q_and_positions_vs_finite_differences(Z):
    x, y, q, g = _problem()
    gr = GR.direct_gradients(x, y, q, Z, g)
    h = 1e-6
    for k in (0, 7, 21, 40):
        # q: the loss is linear in q, so the difference quotient is exact up to rounding
        e = np.zeros_like(q)
        e[k] = 1.0
        fd = (_loss(x, y, q + e, Z, g) - _loss(x, y, q - e, Z, g)) / 2.0
        assert abs(fd - gr["grad_q"][k]) <= 1e-10 * max(1.0, abs(fd))
        e = np.zeros_like(x)
        e[k] = h
        fdx = (_loss(x + e, y, q, Z, g) - _loss(x - e, y, q, Z, g)) / (2 * h)
        fdy = (_loss(x, y + e, q, Z, g) - _loss(x, y - e, q, Z, g)) / (2 * h)
        scale = 1.0 + abs(gr["grad_x"][k]) + abs(gr["grad_y"][k])
        assert abs(fdx - gr["grad_x"][k]) <= 2e-7 * scale, (k, fdx, gr["grad_x"][k])
        assert abs(fdy - gr["grad_y"][k]) <= 2e-7 * scale, (k, fdy, gr["grad_y"][k])


@pytest.mark.parametrize("Z", [1.0, 2.5, 1.0 + 0.5j, 0.3 + 1.1j])
def test_grad_impedance_vs_finite_differences(Z):
    x, y, q, g = _problem()
    gz = GR.direct_gradients(x, y, q, Z, g)["grad_Z"]
    h = 1e-6 * abs(Z)
    d_re = (_loss(x, y, q, Z + h, g) - _loss(x, y, q, Z - h, g)) / (2 * h)
    d_im = (_loss(x, y, q, Z + 1j * h, g) - _loss(x, y, q, Z - 1j * h, g)) / (2 * h)
    assert abs(gz - (d_re + 1j * d_im)) <= 1e-7 * (1.0 + abs(gz))


def test_kernel_derivatives_vs_finite_differences():
    """d_x I_0 = i I_1, d_y I_0 = -I_1 and d_Z I_0 = -w I_0 - 1/(2 pi Z): the three facts the
    gradient formulas rest on."""
    h = 1e-6
    for Z in (1.0, 1.0 + 0.5j, 3.0 + 0.2j):
        for X, Y in ((0.3, 0.2), (-1.1, 0.05), (2.0, 1.5)):
            I = K.reaction_In(1, X, Y, Z)
            dx = (K.reaction_I0(X + h, Y, Z) - K.reaction_I0(X - h, Y, Z)) / (2 * h)
            dy = (K.reaction_I0(X, Y + h, Z) - K.reaction_I0(X, Y - h, Z)) / (2 * h)
            dZ = (K.reaction_I0(X, Y, Z + h) - K.reaction_I0(X, Y, Z - h)) / (2 * h)
            w = Y - 1j * X
            assert abs(dx - 1j * I[1]) <= 1e-8 * (1 + abs(I[1]))
            assert abs(dy + I[1]) <= 1e-8 * (1 + abs(I[1]))
            assert abs(dZ - (-w * I[0] - 1.0 / (K.TWO_PI * Z))) <= 1e-8 * (1 + abs(dZ))


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j])
@pytest.mark.parametrize("dup", [False, True])
def test_homogeneity_identity_for_impedance_gradient(Z, dup):
    """G_Z(s r, s r') = G_{sZ}(r, r') + (1/2pi) log s [free term skipped]: the log parts are scale
    invariant in pairs and the reaction part depends on Z and the coordinates only through
    Z (y - i x).  Differentiating at s = 1,

        Z dl_c/dZ = sum_k [ (x_k - x0) d l_c/dx_k + y_k d l_c/dy_k ] - (1/2pi) sum_{r_i == r_j} conj(g_i) q_j

    with l_c = sum_i conj(g_i) phi_i (complex) and any x0 (translation invariance in x).  The
    right-hand side is built from the oracle's position derivatives, the left from its d/dZ."""
    x, y, q, g = _problem(dup=dup)
    cg = np.conj(g)
    qx, qy = GR.potential_gradient(x, y, q, Z)
    gx, gy = GR.potential_gradient(x, y, cg, Z)
    Dx = cg * qx + q * gx
    Dy = cg * qy + q * gy
    same = (x[:, None] == x[None, :]) & (y[:, None] == y[None, :])
    coinc = np.sum(cg[:, None] * q[None, :] * same)
    for x0 in (0.0, 0.5):
        rhs = np.sum((x - x0) * Dx + y * Dy) - coinc / K.TWO_PI
        lhs = complex(Z) * np.sum(cg * GR.potential_dZ(x, y, q, Z))
        assert abs(lhs - rhs) <= 1e-11 * (1 + np.sum(np.abs((x - x0) * Dx) + np.abs(y * Dy))), (lhs, rhs)


def test_direct_gradients_subset_matches_full():
    x, y, q, g = _problem(n=40)
    full = GR.direct_gradients(x, y, q, 1.0 + 0.5j, g)
    idx = np.array([3, 11, 29])
    sub = GR.direct_gradients(x, y, q, 1.0 + 0.5j, g, idx=idx)
    for k in ("grad_q", "grad_x", "grad_y"):
        assert np.allclose(sub[k], full[k][idx], rtol=1e-14, atol=1e-14)
    assert sub["grad_Z"] == pytest.approx(full["grad_Z"], rel=1e-14)


def test_sampled_gradients_matches_direct():
    x, y, q, g = _problem(n=200, seed=5)
    Z = 1.0 + 0.5j
    ref = GR.direct_gradients(x, y, q, Z, g)
    idx = np.array([0, 17, 99, 150, 199])
    got = GR.sampled_gradients(x, y, q, Z, g, idx, workers=2, want_Z=True)
    for k in ("grad_q", "grad_x", "grad_y"):
        assert np.allclose(got[k], ref[k][idx], rtol=1e-12, atol=1e-12)
    assert abs(got["grad_Z"] - ref["grad_Z"]) <= 1e-12 * abs(ref["grad_Z"])
