"""Pins for the oracle's Green's function (oracle/kernel.py) and direct sum.

Each test checks the oracle against something other than its own formula:
quadrature of the defining Fourier integral, the PDE and the Robin condition,
closed forms printed in the paper, limits, and a brute-force loop.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import kernel as K
from oracle import direct as D

TWO_PI = 2.0 * math.pi


def _fourier(fr, fi, x, a, b=np.inf):
    """int_a^b (fr + i fi)(lam) e^{i lam x} dlam for real-valued fr, fi."""
    if b == np.inf and x != 0.0:
        kw = dict(limlst=200)
        rc = integrate.quad(fr, a, b, weight="cos", wvar=x, **kw)[0]
        rs = integrate.quad(fr, a, b, weight="sin", wvar=x, **kw)[0]
        ic = integrate.quad(fi, a, b, weight="cos", wvar=x, **kw)[0]
        is_ = integrate.quad(fi, a, b, weight="sin", wvar=x, **kw)[0]
    else:
        kw = dict(limit=400, epsabs=1e-15, epsrel=1e-13)
        rc = integrate.quad(lambda t: fr(t) * math.cos(x * t), a, b, **kw)[0]
        rs = integrate.quad(lambda t: fr(t) * math.sin(x * t), a, b, **kw)[0]
        ic = integrate.quad(lambda t: fi(t) * math.cos(x * t), a, b, **kw)[0]
        is_ = integrate.quad(lambda t: fi(t) * math.sin(x * t), a, b, **kw)[0]
    return complex(rc - is_, rs + ic)


def In_quadrature(n, x, y, Z):
    """I_n from its definition (eq. (generalintegral)) by adaptive quadrature.

    eps > 0: the integrand is smooth on [0, inf).  eps = 0: limiting absorption,
    i.e. the principal value plus i*pi times the residue at lam = Z (the
    Sokhotski-Plemelj rule behind eq. (aaa1.5)).
    """
    Z = complex(Z)
    nf = math.factorial(n)
    if Z.imag > 0:
        g = lambda t: math.exp(-t * y) * t ** n / (t - Z)
        val = _fourier(lambda t: g(t).real, lambda t: g(t).imag, x, 0.0)
    else:
        z = Z.real
        # principal value on [0, 2z] (scipy's Cauchy weight 1/(lam - z))
        hr = lambda t: math.exp(-t * y) * t ** n * math.cos(x * t)
        hi = lambda t: math.exp(-t * y) * t ** n * math.sin(x * t)
        pv = complex(integrate.quad(hr, 0.0, 2 * z, weight="cauchy", wvar=z)[0],
                     integrate.quad(hi, 0.0, 2 * z, weight="cauchy", wvar=z)[0])
        g = lambda t: math.exp(-t * y) * t ** n / (t - z)
        tail = _fourier(g, lambda t: 0.0, x, 2 * z)
        res = 1j * math.pi * z ** n * complex(math.cos(x * z), math.sin(x * z)) * math.exp(-z * y)
        val = pv + tail + res
    return val / (TWO_PI * nf)


POINTS = [(2.0, 1.0), (-1.3, 0.4), (0.3, 0.2), (0.7, 0.6), (-0.2, 1.7), (0.0, 0.5)]


@pytest.mark.parametrize("Z", [1.0 + 0.5j, 2.0 + 0.1j, 0.7 + 1.2j])
@pytest.mark.parametrize("xy", POINTS)
def test_I0_matches_fourier_quadrature_dissipative(Z, xy):
    x, y = xy
    ref = In_quadrature(0, x, y, Z)
    got = complex(K.reaction_I0(x, y, Z))
    assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref))


@pytest.mark.parametrize("Z", [1.0, 2.0, 0.5])
@pytest.mark.parametrize("xy", POINTS)
def test_I0_matches_limiting_absorption_lossless(Z, xy):
    x, y = xy
    ref = In_quadrature(0, x, y, Z)
    got = complex(K.reaction_I0(x, y, Z))
    assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref))


def test_I0_is_limit_of_dissipative():
    # limiting absorption (eq. (dzGreensfunimplossless)): eps -> 0+ from above
    for x, y in POINTS:
        a = complex(K.reaction_I0(x, y, 1.3))
        b = complex(K.reaction_I0(x, y, 1.3 + 1e-9j))
        assert abs(a - b) < 1e-7


@pytest.mark.parametrize("Z", [1.0 + 0.5j, 1.0])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_In_recursion_matches_quadrature(Z, n):
    for x, y in [(0.9, 0.7), (-0.4, 1.1), (0.25, 0.45)]:
        ref = In_quadrature(n, x, y, Z)
        got = complex(K.reaction_In(n, x, y, Z)[n])
        assert abs(got - ref) <= 1e-9 * max(1e-3, abs(ref)), (n, x, y)


@pytest.mark.parametrize("Z", [1.0 + 0.5j, 2.0, 0.3 + 0.05j])
def test_In_derivative_identities(Z):
    # Differentiating eq. (generalintegral) under the integral sign:
    # d/dx I_n = i (n+1) I_{n+1},  d/dy I_n = -(n+1) I_{n+1}.
    h = 1e-5
    for x, y in [(0.6, 0.8), (-1.1, 0.5), (0.05, 0.3)]:
        I = K.reaction_In(12, x, y, Z)
        Ixp = K.reaction_In(11, x + h, y, Z)
        Ixm = K.reaction_In(11, x - h, y, Z)
        Iyp = K.reaction_In(11, x, y + h, Z)
        Iym = K.reaction_In(11, x, y - h, Z)
        for n in range(11):
            dx = (Ixp[n] - Ixm[n]) / (2 * h)
            dy = (Iyp[n] - Iym[n]) / (2 * h)
            scale = max(abs(I[n + 1]) * (n + 1), 1e-8)
            assert abs(dx - 1j * (n + 1) * I[n + 1]) < 1e-5 * scale, (n, x, y)
            assert abs(dy + (n + 1) * I[n + 1]) < 1e-5 * scale, (n, x, y)


def _rand_pairs(rng, m):
    xt = rng.uniform(-1, 1, m)
    yt = rng.uniform(0.05, 1.5, m)
    xs = rng.uniform(-1, 1, m)
    ys = rng.uniform(0.05, 1.5, m)
    return xt, yt, xs, ys


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j, 3.0 + 0.2j])
def test_G_symmetry(Z):
    rng = np.random.default_rng(3)
    xt, yt, xs, ys = _rand_pairs(rng, 200)
    a = K.green(xt, yt, xs, ys, Z)
    b = K.green(xs, ys, xt, yt, Z)
    assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j, 2.5 + 1.0j])
def test_G_harmonic_in_target(Z):
    # Eq. (0.0): Laplacian of G in the target vanishes away from the source.
    rng = np.random.default_rng(4)
    h = 2e-3
    w = np.array([-1.0 / 12, 4.0 / 3, -5.0 / 2, 4.0 / 3, -1.0 / 12])  # 4th-order stencil
    for _ in range(20):
        xt, yt = rng.uniform(-1, 1), rng.uniform(0.3, 1.5)
        xs, ys = rng.uniform(-1, 1), rng.uniform(0.3, 1.5)
        if math.hypot(xt - xs, yt - ys) < 0.3:
            continue
        offs = np.arange(-2, 3) * h
        gxx = np.sum(w * K.green(xt + offs, yt, xs, ys, Z)) / h ** 2
        gyy = np.sum(w * K.green(xt, yt + offs, xs, ys, Z)) / h ** 2
        scale = abs(np.sum(w * K.green(xt + offs, yt, xs, ys, Z))) / h ** 2 + 1.0
        assert abs(gxx + gyy) < 1e-5 * scale


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j, 0.4, 5.0 + 2.0j])
def test_G_robin_boundary_condition(Z):
    # Eq. (1.0) with the Robin operator d/dn - Z, n = -y_hat:  dG/dy + Z G = 0 on y = 0.
    rng = np.random.default_rng(5)
    h = 1e-4
    for _ in range(20):
        xt = rng.uniform(-2, 2)
        xs, ys = rng.uniform(-1, 1), rng.uniform(0.1, 1.5)
        gp = K.green(xt, h, xs, ys, Z)
        gm = K.green(xt, -h, xs, ys, Z)
        gp2 = K.green(xt, 2 * h, xs, ys, Z)
        gm2 = K.green(xt, -2 * h, xs, ys, Z)
        dgy = (8 * (gp - gm) - (gp2 - gm2)) / (12 * h)
        g0 = K.green(xt, 0.0, xs, ys, Z)
        resid = dgy + complex(Z) * g0
        assert abs(resid) < 1e-8 * (abs(dgy) + abs(complex(Z) * g0) + 1.0)
        # the opposite sign convention must fail at O(1)
        assert abs(dgy - complex(Z) * g0) > 1e-3


@pytest.mark.parametrize("Z", [1.0, 2.0, 0.3])
def test_imag_part_lossless_closed_form(Z):
    # Lossless closed form (Section 2.1, after Hein et al.): the only imaginary
    # part of G is i exp(-Z (y + y')) cos(Z (x - x')).
    rng = np.random.default_rng(6)
    xt, yt, xs, ys = _rand_pairs(rng, 300)
    G = K.green(xt, yt, xs, ys, Z)
    ref = np.exp(-Z * (yt + ys)) * np.cos(Z * (xt - xs))
    assert np.max(np.abs(G.imag - ref)) < 1e-13


def _hein(X, Y, Z):
    from scipy.special import expi
    return -np.exp(-Z * Y) / TWO_PI * (np.exp(1j * Z * X) * expi(Z * (Y - 1j * X))
                                      + np.exp(-1j * Z * X) * expi(Z * (Y + 1j * X)))


def test_hein_lossless_closed_form():
    # Printed lossless closed form of G_Z (Section 2.1), real Z.
    rng = np.random.default_rng(7)
    for Z in (1.0, 2.0, 0.7):
        X = rng.uniform(-2, 2, 100)
        Y = rng.uniform(0.05, 2, 100)
        ref = _hein(X, Y, Z) + 1j * np.exp(-Z * Y) * np.cos(Z * X)
        got = K.reaction_GZ(X, Y, Z)
        assert np.max(np.abs(got - ref)) < 1e-13


def test_hein_dissipative_form_misses_surface_term():
    # Reading of the printed dissipative closed form: with the principal Ei it
    # differs from the integral (eq. (dzGreensfunimp)) by exactly
    # i exp(-Z Y) cos(Z X), the term its lossless counterpart carries.
    rng = np.random.default_rng(8)
    for Z in (1.0 + 0.5j, 2.0 + 0.3j):
        X = rng.uniform(-2, 2, 50)
        Y = rng.uniform(0.05, 2, 50)
        diff = K.reaction_GZ(X, Y, Z) - _hein(X, Y, Z)
        assert np.max(np.abs(diff - 1j * np.exp(-Z * Y) * np.cos(Z * X))) < 1e-13
        # and one quadrature spot check that the oracle, not the printed form, is the integral
        ref = In_quadrature(0, X[0], Y[0], Z) + In_quadrature(0, -X[0], Y[0], Z)
        assert abs(K.reaction_GZ(X[0], Y[0], Z) - ref) < 1e-9


def test_large_impedance_tends_to_dirichlet():
    # Z -> infinity: the Robin condition becomes G = 0 on y = 0 (eq. (ddd1.2)).
    rng = np.random.default_rng(9)
    xt, yt, xs, ys = _rand_pairs(rng, 50)
    gd = K.green_dirichlet(xt, yt, xs, ys)
    # (the closed form over/underflows once Z (y + y') exceeds ~700; stay below)
    for Z in (50.0, 200.0):
        g = K.green(xt, yt, xs, ys, Z)
        Y = yt + ys
        X = xt - xs
        # leading correction -Y / (pi Z (X^2 + Y^2)); the remainder is O(1/Z^2)
        corr = -Y / (math.pi * Z * (X * X + Y * Y))
        assert np.all(np.abs(g.real - gd - corr) * Z ** 2 * Y ** 3 < 2.0)
        assert np.max(np.abs(g.imag)) < 1e-6


def test_direct_sum_matches_python_loops_with_duplicates():
    rng = np.random.default_rng(10)
    n = 40
    x = rng.uniform(0, 1, n)
    y = rng.uniform(0.01, 1, n)
    x[5], y[5] = x[3], y[3]        # coincident distinct points
    q = rng.uniform(-1, 1, n)
    for Z in (1.0, 1.0 + 0.5j):
        a = D.potential(x, y, q, Z, workers=1)
        b = D.potential_loops(x, y, q, Z)
        assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


def test_direct_sum_multiprocess_equals_serial():
    rng = np.random.default_rng(11)
    n = 300
    x = rng.uniform(0, 1, n)
    y = rng.uniform(0.01, 1, n)
    q = rng.uniform(-1, 1, (2, n))
    a = D.potential(x, y, q, 1.0 + 0.5j, workers=1)
    b = D.potential(x, y, q, 1.0 + 0.5j, workers=3, target_block=32)
    assert np.array_equal(a, b)


def test_imag_part_closed_form_matches_direct():
    rng = np.random.default_rng(12)
    n = 400
    x = rng.uniform(0, 1, n)
    y = rng.uniform(0.01, 1, n)
    q = rng.uniform(-1, 1, n)
    phi = D.potential(x, y, q, 1.5, workers=1)
    im = D.imag_part_real_impedance(x, y, q, 1.5)
    assert np.max(np.abs(phi.imag - im)) < 1e-12 * np.max(np.abs(im))


def test_In_multiprecision_agrees_with_float64_and_quadrature():
    # the mpmath variant follows the same definitions; at small |Z w| the float64 recursion is
    # accurate, so the two agree, and both match quadrature of eq. (generalintegral)
    for Z in (1.0, 1.0 + 0.5j):
        for x, y in ((0.3, 0.4), (-0.7, 0.2)):
            a = K.reaction_In_mp(8, x, y, Z)
            b = K.reaction_In(8, x, y, Z)
            assert np.max(np.abs(a - b) / np.abs(a)) < 1e-12
            assert abs(a[3] - In_quadrature(3, x, y, Z)) < 1e-9 * abs(a[3])
