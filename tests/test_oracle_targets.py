"""Pins of the oracle's direct sum at separate targets, including targets on the boundary y = 0
(the field mesh of the paper's Example 2, Section 5, reaches y = 0):

* the vectorised sum equals the term-by-term double loop (targets on y = 0, a target on a source);
* the potential satisfies the Robin condition d_y phi + Z phi = 0 on y = 0 (Section 2.1: every
  term of G does), checked by one-sided second-order differences in y;
* for a real impedance its imaginary part equals the exact O(N) closed form at every target;
* the Example 2 geometry: eight unit circles, the lowest charge 0.01 above the boundary, total
  charge 2 pi per circle;
* the field (gradient of the potential) at separate targets against differences of the potential,
  and the Robin condition d_y phi + Z phi = 0 that it satisfies exactly on the boundary.
"""
import numpy as np
import pytest

import workloads
from oracle import direct as D


def _sources(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, n), rng.uniform(0.02, 1.0, n), rng.uniform(-1.0, 1.0, n)


@pytest.mark.parametrize("Z", [1.0, 0.7 + 0.4j])
def test_targets_on_boundary_match_loops(Z):
    xs, ys, q = _sources(40, 1)
    rng = np.random.default_rng(2)
    xt = np.concatenate([rng.uniform(-1, 1, 12), xs[:3]])
    yt = np.concatenate([np.zeros(6), rng.uniform(0.0, 1.0, 6), ys[:3]])  # boundary, interior, on sources
    a = D.potential(xs, ys, q, Z, xt=xt, yt=yt, workers=1)
    b = D.potential_loops(xs, ys, q, Z, xt=xt, yt=yt)
    assert np.all(np.isfinite(a))
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("Z", [1.0, 2.5, 1.0 + 0.5j])
def test_direct_sum_satisfies_robin_condition_on_boundary(Z):
    xs, ys, q = _sources(30, 3)
    x0 = np.linspace(-0.9, 0.9, 7)
    h = 1e-4
    phi = [D.potential(xs, ys, q, Z, xt=x0, yt=np.full(x0.size, k * h), workers=1) for k in range(3)]
    dy = (-3.0 * phi[0] + 4.0 * phi[1] - phi[2]) / (2.0 * h)
    res = dy + complex(Z) * phi[0]
    scale = np.abs(dy) + np.abs(complex(Z) * phi[0])
    assert np.all(np.abs(res) <= 1e-6 * scale), (res, scale)
    # the opposite sign of the condition fails at O(1)
    assert np.max(np.abs(dy - complex(Z) * phi[0]) / scale) > 0.1


def test_imag_part_closed_form_at_targets():
    xs, ys, q = _sources(50, 5)
    rng = np.random.default_rng(6)
    xt = rng.uniform(-1, 1, 20)
    yt = np.concatenate([np.zeros(5), rng.uniform(0, 1, 15)])
    for Z in (1.0, 3.0):
        phi = D.potential(xs, ys, q, Z, xt=xt, yt=yt, workers=1)
        im = D.imag_part_real_impedance(xs, ys, q, Z, xt=xt, yt=yt)
        assert np.max(np.abs(phi.imag - im)) <= 1e-12 * (1.0 + np.max(np.abs(im)))


def test_example2_geometry():
    d = workloads.example2(64, 9, 5)
    sx, sy, q = d["src_x"], d["src_y"], d["q"]
    assert sx.size == 8 * 64 and d["tgt_x"].size == 45
    # the lowest midpoint of the lower circles: 1.01 - cos(pi / 64)
    assert sy.min() == pytest.approx(1.01 - np.cos(np.pi / 64), abs=1e-15)
    assert sy.min() > 0.01
    for k in range(8):
        assert np.sum(q[64 * k:64 * (k + 1)]) == pytest.approx(2.0 * np.pi, rel=1e-14)
    cx = [-3.3 + 2.2 * (k % 4) for k in range(8)]
    cy = [1.01] * 4 + [3.2] * 4
    for k in range(8):
        r = np.hypot(sx[64 * k:64 * (k + 1)] - cx[k], sy[64 * k:64 * (k + 1)] - cy[k])
        assert np.allclose(r, 1.0, rtol=0, atol=1e-14)
    assert d["tgt_y"].min() == 0.0 and d["tgt_y"].max() == pytest.approx(4.2)
    assert d["tgt_x"].min() == pytest.approx(-4.4) and d["tgt_x"].max() == pytest.approx(4.4)
    s = workloads.example2_sized(4000)
    assert s["src_x"].size + s["tgt_x"].size <= 4000 and s["src_x"].size == 8 * 250


@pytest.mark.parametrize("Z", [1.0, 0.7 + 0.4j])
def test_field_at_targets_vs_differences(Z):
    """The oracle's field at separate targets (grad.field_at) against central differences of its
    direct-sum potential (one-sided in y on the boundary)."""
    from oracle import grad as GR
    xs, ys, q = _sources(40, 12)
    rng = np.random.default_rng(13)
    xt = rng.uniform(-1, 1, 10)
    yt = np.concatenate([np.zeros(3), rng.uniform(0.05, 1.0, 7)])
    gx, gy = GR.field_at(xs, ys, q, Z, xt, yt, workers=1)
    h = 1e-5

    def phi(dx, dy):
        return D.potential(xs, ys, q, Z, xt=xt + dx, yt=yt + dy, workers=1)

    fdx = (phi(h, 0.0) - phi(-h, 0.0)) / (2 * h)
    inner = yt > 0
    fdy = np.empty_like(fdx)
    fdy[inner] = ((phi(0.0, h) - phi(0.0, -h)) / (2 * h))[inner]
    fdy[~inner] = ((-3 * phi(0.0, 0.0) + 4 * phi(0.0, h) - phi(0.0, 2 * h)) / (2 * h))[~inner]
    scale = 1.0 + np.abs(gx) + np.abs(gy)
    assert np.all(np.abs(fdx - gx) <= 1e-6 * scale)
    assert np.all(np.abs(fdy - gy) <= 1e-6 * scale)
    # on the boundary the field satisfies the Robin condition d_y phi + Z phi = 0 exactly
    p0 = phi(0.0, 0.0)
    assert np.all(np.abs(gy[~inner] + complex(Z) * p0[~inner]) <= 1e-12 * (np.abs(gy[~inner]) + 1.0))
