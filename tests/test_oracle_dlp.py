"""Pins of the oracle's double-layer potential sum_j mu_j n_j . grad_{r_j} G(r_i, r_j)
(``direct.double_layer``, the boundary-integral use of the Green's function the paper motivates):

* against central differences of the single-layer direct sum with the sources moved along their
  normals (all three boundary conditions);
* the classical jump identity: with unit density on a closed circle in the upper half plane the
  double layer is -1 inside and 0 outside, because every part of G but the free-space log is
  harmonic in the source point for y' > 0 (the image and reaction terms, Section 2.1) and the
  free-space part gives Gauss's integral; the trapezoidal rule on the circle makes this exact to
  rounding for targets away from it, for all three boundary conditions.
"""
import numpy as np
import pytest

from oracle import direct as D


def _curve(n, cx=0.3, cy=0.8, r=0.5):
    th = (np.arange(n) + 0.5) * 2 * np.pi / n
    return cx + r * np.cos(th), cy + r * np.sin(th), np.cos(th), np.sin(th), np.full(n, 2 * np.pi * r / n)


@pytest.mark.parametrize("bc,Z", [("robin", 1.0), ("robin", 0.7 + 0.4j), ("dirichlet", 1.0), ("neumann", 1.0)])
def test_double_layer_vs_moved_sources(bc, Z):
    rng = np.random.default_rng(1)
    n = 30
    xs, ys = rng.uniform(-1, 1, n), rng.uniform(0.05, 1.0, n)
    th = rng.uniform(0, 2 * np.pi, n)
    nx, ny = np.cos(th), np.sin(th)
    mu = rng.standard_normal(n)
    xt, yt = rng.uniform(-1, 1, 9), np.concatenate([[0.0], rng.uniform(0.0, 1.0, 8)])
    got = D.double_layer(xs, ys, nx, ny, mu, Z, xt=xt, yt=yt, bc=bc)
    h = 1e-5
    fd = (D.potential(xs + h * nx, ys + h * ny, mu, Z, xt=xt, yt=yt, workers=1, bc=bc)
          - D.potential(xs - h * nx, ys - h * ny, mu, Z, xt=xt, yt=yt, workers=1, bc=bc)) / (2 * h)
    assert np.max(np.abs(fd - got)) <= 1e-6 * (1.0 + np.max(np.abs(got)))


@pytest.mark.parametrize("bc,Z", [("dirichlet", 1.0), ("neumann", 1.0), ("robin", 1.0), ("robin", 2.0 + 1.0j)])
def test_unit_density_circle_jump(bc, Z):
    xs, ys, nx, ny, wt = _curve(400)
    xt = np.array([0.3, 0.45, 0.1, 1.2, -0.6, 0.3, 0.3])
    yt = np.array([0.8, 0.9, 0.6, 0.8, 0.5, 0.0, 1.6])
    inside = np.hypot(xt - 0.3, yt - 0.8) < 0.5
    v = D.double_layer(xs, ys, nx, ny, wt, Z, xt=xt, yt=yt, bc=bc)
    assert np.allclose(v[inside], -1.0, rtol=0, atol=1e-12) and np.allclose(v[~inside], 0.0, rtol=0, atol=1e-12)
