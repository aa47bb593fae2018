"""Pins of the oracle's Dirichlet and Neumann half-plane kernels (eq. (ddd1.2)): the boundary
condition each satisfies on y = 0, the limits of the Robin kernel (Z -> infinity gives Dirichlet,
Z -> 0 gives Neumann up to a constant), the vectorised sum against the term-by-term loops, and the
field against differences of the potential.
"""
import numpy as np
import pytest

from oracle import direct as D
from oracle import grad as GR


def _problem(n=40, seed=1):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, n), rng.uniform(0.02, 1.0, n), rng.uniform(-1.0, 1.0, n)


def test_dirichlet_vanishes_and_neumann_flux_vanishes_on_boundary():
    xs, ys, q = _problem()
    xt = np.linspace(-1.5, 1.5, 11)
    yt = np.zeros_like(xt)
    phd = D.potential(xs, ys, q, 1.0, xt=xt, yt=yt, workers=1, bc="dirichlet")
    scale = np.max(np.abs(D.potential(xs, ys, q, 1.0, xt=xt, yt=yt + 0.3, workers=1, bc="dirichlet")))
    assert np.max(np.abs(phd)) <= 1e-14 * scale
    _, gy = GR.field_at(xs, ys, q, 1.0, xt, yt, workers=1, bc="neumann")
    gx, _ = GR.field_at(xs, ys, q, 1.0, xt, yt, workers=1, bc="neumann")
    assert np.max(np.abs(gy)) <= 1e-14 * np.max(np.abs(gx))
    # and the other way round they do not vanish
    phn = D.potential(xs, ys, q, 1.0, xt=xt, yt=yt, workers=1, bc="neumann")
    assert np.max(np.abs(phn)) > 0.1 * scale


def test_robin_limits():
    # Z -> infinity: Dirichlet, with an error that falls like 1/Z (points away from y = 0; the
    # Ei closed form overflows float64 for |Z| (y + y') beyond ~700)
    rng = np.random.default_rng(2)
    xs, ys, q = rng.uniform(-1, 1, 40), rng.uniform(0.3, 1.0, 40), rng.uniform(-1, 1, 40)
    xt, yt = rng.uniform(-1, 1, 12), rng.uniform(0.3, 1.0, 12)
    phd = D.potential(xs, ys, q, 1.0, xt=xt, yt=yt, workers=1, bc="dirichlet")
    errs = [np.max(np.abs(D.potential(xs, ys, q, Z, xt=xt, yt=yt, workers=1) - phd)) / np.max(np.abs(phd))
            for Z in (50.0, 100.0, 200.0)]
    assert errs[2] < 0.01 and 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2, errs
    xs, ys, q = _problem(seed=2)
    rng = np.random.default_rng(3)
    xt, yt = rng.uniform(-1, 1, 12), rng.uniform(0.0, 1.0, 12)
    # Z -> 0: Neumann up to a target-independent constant
    phn = D.potential(xs, ys, q, 1.0, xt=xt, yt=yt, workers=1, bc="neumann")
    small = D.potential(xs, ys, q, 1e-6, xt=xt, yt=yt, workers=1)
    d = small - phn
    assert np.max(np.abs(d - d.mean())) <= 1e-4 * np.max(np.abs(phn - phn.mean()))


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_sum_matches_loops_and_field_matches_differences(bc):
    xs, ys, q = _problem(30, 4)
    rng = np.random.default_rng(5)
    xt = np.concatenate([rng.uniform(-1, 1, 8), xs[:2]])
    yt = np.concatenate([rng.uniform(0.05, 1.0, 8), ys[:2]])
    a = D.potential(xs, ys, q, 1.0, xt=xt, yt=yt, workers=1, bc=bc)
    b = D.potential_loops(xs, ys, q, 1.0, xt=xt, yt=yt, bc=bc)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))
    assert np.all(a.imag == 0.0)
    gx, gy = GR.field_at(xs, ys, q, 1.0, xt[:8], yt[:8], workers=1, bc=bc)
    h = 1e-5

    def phi(dx, dy):
        return D.potential(xs, ys, q, 1.0, xt=xt[:8] + dx, yt=yt[:8] + dy, workers=1, bc=bc)

    fdx = (phi(h, 0) - phi(-h, 0)) / (2 * h)
    fdy = (phi(0, h) - phi(0, -h)) / (2 * h)
    sc = 1.0 + np.abs(gx) + np.abs(gy)
    assert np.all(np.abs(fdx - gx) <= 1e-6 * sc) and np.all(np.abs(fdy - gy) <= 1e-6 * sc)
