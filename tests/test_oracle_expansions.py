"""Pins for the oracle's expansion operators (oracle/expansions.py).

The paper's Example 1 (Section 5) fixes a source/target pair and four expansion
centres but prints its errors only as plots; what the text fixes is that the
ME, the LE and the chain S2M -> M2M -> M2L -> L2L converge exponentially in p
(Theorems 3.3-3.7).  These tests check exactly that against the directly
evaluated I_0, plus the textbook log-kernel expansions against direct sums.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import expansions as E
from oracle import kernel as K


def _chain(Z, mirror, p):
    e = workloads.example1()
    s = -1.0 if mirror else 1.0
    xt, yt = e["target"]
    xs, ys = e["source"]
    ys_im = -ys
    sc, spc = e["source_centre"], e["source_parent_centre"]
    tc, tpc = e["target_centre"], e["target_parent_centre"]
    exact = complex(K.reaction_I0(s * xt - s * xs, yt - ys_im, Z))
    a = E.s2m([s * xs], [ys_im], [1.0], s * sc[0], sc[1], p)
    me = complex(E.me_eval(a, s * sc[0], sc[1], s * xt, yt, Z))
    b = E.s2l([s * xs], [ys_im], [1.0], s * tc[0], tc[1], p, Z)
    le = complex(E.le_eval(b, s * tc[0], tc[1], s * xt, yt))
    a2 = E.m2m(a, s * sc[0], sc[1], s * spc[0], spc[1])
    bl = E.m2l(a2, s * spc[0], spc[1], s * tpc[0], tpc[1], Z)
    b2 = E.l2l(bl, s * tpc[0], tpc[1], s * tc[0], tc[1])
    chain = complex(E.le_eval(b2, s * tc[0], tc[1], s * xt, yt))
    return exact, me, le, chain


@pytest.mark.parametrize("Z", [1.0, 1.0 + 0.5j, 2.0])
@pytest.mark.parametrize("mirror", [False, True])
def test_example1_exponential_convergence(Z, mirror):
    errs = {p: [abs(v - _chain(Z, mirror, p)[0]) for v in _chain(Z, mirror, p)[1:]]
            for p in (4, 8, 12, 16, 30)}
    for k in range(3):
        seq = [errs[p][k] for p in (4, 8, 12)]
        # geometric decay: each +4 in p gains well over a decade at these ratios
        assert seq[1] < 0.1 * seq[0] and seq[2] < 0.1 * seq[1], (k, seq)
        assert errs[30][k] < 1e-14
    # M2M is exact (Theorem 3.5): shifting the truncated ME changes nothing
    # beyond the truncation of the shifted expansion itself.


def test_m2m_is_exact_for_all_orders():
    # alpha~ from M2M equals S2M taken directly about the parent centre.
    rng = np.random.default_rng(1)
    xs = rng.uniform(0.0, 0.1, 7)
    ys_im = -rng.uniform(0.3, 0.4, 7)
    q = rng.uniform(-1, 1, 7)
    a = E.s2m(xs, ys_im, q, 0.05, -0.35, 25)
    a2 = E.m2m(a, 0.05, -0.35, 0.1, -0.3)
    ref = E.s2m(xs, ys_im, q, 0.1, -0.3, 25)
    assert np.max(np.abs(a2 - ref)) < 1e-13 * np.max(np.abs(ref))


def test_me_error_within_theorem_rate():
    # Theorem 3.3: |error| <= C C_max Q_s q^{p+1} / (p+1), q = sqrt(2) d_s / (2 |r_i - r'_c|).
    e = workloads.example1()
    xs, ys = e["source"]
    xt, yt = e["target"]
    xc, yc = e["source_centre"]
    d_s = 2 * max(abs(xs - xc), abs(-ys - yc))  # smallest box around the image, centred at r'_c
    qrate = math.sqrt(2) * d_s / (2 * math.hypot(xt - xc, yt - yc))
    exact = complex(K.reaction_I0(xt - xs, yt + ys, 1.0))
    ratios = []
    for p in range(2, 14):
        a = E.s2m([xs], [-ys], [1.0], xc, yc, p)
        err = abs(complex(E.me_eval(a, xc, yc, xt, yt, 1.0)) - exact)
        ratios.append(err * (p + 1) / qrate ** (p + 1))
    assert max(ratios) < 10 * min(ratios[:3]) + 1.0


def _cluster(rng, n, c, r):
    return c + r * (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n))


def test_log_expansion_chain_matches_direct():
    rng = np.random.default_rng(2)
    zs = _cluster(rng, 30, 0.1 + 0.1j, 0.05)
    q = rng.uniform(-1, 1, 30)
    zt = _cluster(rng, 20, 0.65 + 0.15j, 0.05)
    zc, zp = 0.1 + 0.1j, 0.125 + 0.125j      # child / parent source centres
    tc, tp = 0.65 + 0.15j, 0.625 + 0.125j    # child / parent target centres
    direct = np.array([np.sum(q * np.log(np.abs(z - zs))) for z in zt])
    for p, tol in ((10, 1e-6), (20, 1e-10), (30, 1e-13)):
        a = E.log_p2m(zs, q, zc, p)
        me = E.log_me_eval(a, zc, zt).real
        a2 = E.log_m2m(a, zc, zp)
        b = E.log_m2l(a2, zp, tp)
        b2 = E.log_l2l(b, tp, tc)
        le = E.log_le_eval(b2, tc, zt).real
        bl = E.log_p2l(zs, q, tc, p)
        le2 = E.log_le_eval(bl, tc, zt).real
        scale = np.max(np.abs(direct))
        assert np.max(np.abs(me - direct)) < tol * scale
        assert np.max(np.abs(le - direct)) < tol * scale
        assert np.max(np.abs(le2 - direct)) < tol * scale


def test_dirichlet_remark_reduces_to_log_series():
    # Remark after Theorem 2.1: with the pole-free kernel int_0^inf e^{-lam w}
    # lam^{n-1} dlam / (2 pi n!) = 1 / (2 pi n w^n) in place of I_n (n >= 1), the
    # ME (reactfieldME) reproduces the textbook series of -(1/2pi) ln|r - r~'|
    # up to the n = 0 (log) term, with w = y - i x = -i z.
    rng = np.random.default_rng(3)
    xs, ys = 0.02, 0.03            # image point r~' below the axis: (xs, -ys)
    for _ in range(5):
        x, y = rng.uniform(-1, 1), rng.uniform(0.5, 1.5)
        z = complex(x, y)
        zim = complex(xs, -ys)
        series = sum((1j ** -n) * complex(xs, -ys) ** n * (1.0 / (2 * math.pi * n * (y - 1j * x) ** n))
                     for n in range(1, 60))
        # -(1/2pi) Re[ln z - sum (zim/z)^n / n] minus the n = 0 term -(1/2pi) Re ln z
        ref = -(1 / (2 * math.pi)) * (-sum((zim / z) ** n / n for n in range(1, 60)))
        assert abs(series.real - ref.real) < 1e-14
