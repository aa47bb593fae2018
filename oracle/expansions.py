"""Far-field expansions and translation operators -- CPU oracle.

Test infrastructure only (see ``oracle/__init__``).

Reaction field Phi_2^+ (Section 2.2), for image sources r_j^im = (x_j, -y_j) in a
source box B_s below y = 0 with centre r'_c, and targets above y = 0:

  S2M  alpha_n = sum_j Q_j i^n [(x'_c - x_j) + i (y'_c - y_j^im)]^n          (MEcoefficients)
  ME   Phi ~ sum_{n<=p} alpha_n I_n(x_i - x'_c, y_i - y'_c)                  (truncatedME)
  M2M  alpha~_n = sum_{m<=n} n!/((n-m)! m!) i^{n-m} [(x~'_c - x'_c) + i (y~'_c - y'_c)]^{n-m} alpha_m
                                                                             (metome)
  S2L  beta_n = sum_j Q_j i^{-n} I_n(x_c - x_j, y_c - y_j^im)                (LEcoefficients)
  LE   Phi ~ sum_{n<=p} beta_n [(x_c - x_i) + i (y_c - y_i)]^n               (truncatedLE)
  L2L  beta_m = sum_{n=m..p} n!/((n-m)! m!) [(x_c - x~_c) + i (y_c - y~_c)]^{n-m} beta_n
                                                                             (truncatedL2L)
  M2L  beta_n = sum_{m<=p} i^{-n} (n+m)!/(n! m!) I_{n+m}(x_c - x'_c, y_c - y'_c) alpha_m
                                                                             (truncatedM2Lcoef)

Phi_2^- is the same algorithm run on x-mirrored coordinates (Algorithm 2):
image sources at (-x_j, y_j^im) and targets at (-x_i, y_i).

Log kernel: the paper hands Phi_free and Phi_1 to "the classic FMM" without
printing its formulas.  The textbook (Greengard-Rokhlin) complex-log expansions
of u(z) = sum_j q_j log(z - z_j) are written out here; Phi_free = -(1/2pi) Re u
over the sources, Phi_1 = +(1/2pi) Re u over the image sources.
"""
from __future__ import annotations

from math import comb, factorial

import numpy as np

from .kernel import reaction_In

# ----------------------------------------------------------------------------
# Reaction field (paper, Section 2.2)
# ----------------------------------------------------------------------------


def s2m(x_src, y_src_im, q, xc, yc, p):
    d = (xc - np.asarray(x_src)) + 1j * (yc - np.asarray(y_src_im))
    return np.array([np.sum(np.asarray(q) * (1j ** n) * d ** n) for n in range(p + 1)])


def me_eval(alpha, xc, yc, x, y, Z):
    p = len(alpha) - 1
    In = reaction_In(p, x - xc, y - yc, Z)
    return np.tensordot(alpha, In, axes=(0, 0))


def m2m(alpha, xc, yc, xc_new, yc_new):
    p = len(alpha) - 1
    t = (xc_new - xc) + 1j * (yc_new - yc)
    out = np.zeros(p + 1, dtype=np.complex128)
    for n in range(p + 1):
        for m in range(n + 1):
            out[n] += comb(n, m) * (1j ** (n - m)) * t ** (n - m) * alpha[m]
    return out


def s2l(x_src, y_src_im, q, xc, yc, p, Z):
    In = reaction_In(p, xc - np.asarray(x_src), yc - np.asarray(y_src_im), Z)
    return np.array([np.sum(np.asarray(q) * (1j ** (-n)) * In[n]) for n in range(p + 1)])


def le_eval(beta, xc, yc, x, y):
    d = (xc - np.asarray(x)) + 1j * (yc - np.asarray(y))
    return sum(beta[n] * d ** n for n in range(len(beta)))


def l2l(beta, xc, yc, xc_new, yc_new):
    p = len(beta) - 1
    t = (xc - xc_new) + 1j * (yc - yc_new)
    out = np.zeros(p + 1, dtype=np.complex128)
    for m in range(p + 1):
        for n in range(m, p + 1):
            out[m] += comb(n, m) * t ** (n - m) * beta[n]
    return out


def m2l(alpha, xs_c, ys_c, xt_c, yt_c, Z):
    p = len(alpha) - 1
    In = reaction_In(2 * p, xt_c - xs_c, yt_c - ys_c, Z)
    out = np.zeros(p + 1, dtype=np.complex128)
    for n in range(p + 1):
        for m in range(p + 1):
            out[n] += (1j ** (-n)) * comb(n + m, n) * In[n + m] * alpha[m]
    return out


# ----------------------------------------------------------------------------
# Log kernel u(z) = sum_j q_j log(z - z_j)  (textbook expansions)
# ----------------------------------------------------------------------------


def log_p2m(z_src, q, zc, p):
    d = np.asarray(z_src) - zc
    q = np.asarray(q)
    a = np.zeros(p + 1, dtype=np.complex128)
    a[0] = np.sum(q)
    for k in range(1, p + 1):
        a[k] = -np.sum(q * d ** k) / k
    return a


def log_me_eval(a, zc, z):
    d = np.asarray(z) - zc
    return a[0] * np.log(d) + sum(a[k] / d ** k for k in range(1, len(a)))


def log_m2m(a, zc, zc_new):
    p = len(a) - 1
    z0 = zc - zc_new
    b = np.zeros(p + 1, dtype=np.complex128)
    b[0] = a[0]
    for l in range(1, p + 1):
        b[l] = -a[0] * z0 ** l / l
        for k in range(1, l + 1):
            b[l] += a[k] * z0 ** (l - k) * comb(l - 1, k - 1)
    return b


def log_m2l(a, zs, zt):
    p = len(a) - 1
    z0 = zs - zt
    b = np.zeros(p + 1, dtype=np.complex128)
    b[0] = a[0] * np.log(-z0) + sum(a[k] * (-1) ** k / z0 ** k for k in range(1, p + 1))
    for l in range(1, p + 1):
        s = sum(a[k] / z0 ** k * comb(l + k - 1, k - 1) * (-1) ** k for k in range(1, p + 1))
        b[l] = -a[0] / (l * z0 ** l) + s / z0 ** l
    return b


def log_l2l(b, zc, zc_new):
    p = len(b) - 1
    t = zc_new - zc
    out = np.zeros(p + 1, dtype=np.complex128)
    for m in range(p + 1):
        for l in range(m, p + 1):
            out[m] += b[l] * comb(l, m) * t ** (l - m)
    return out


def log_le_eval(b, zc, z):
    d = np.asarray(z) - zc
    return sum(b[l] * d ** l for l in range(len(b)))


def log_p2l(z_src, q, zc, p):
    """Local expansion about zc of sum_j q_j log(z - z_j) for sources far from zc."""
    d = np.asarray(z_src) - zc
    q = np.asarray(q)
    b = np.zeros(p + 1, dtype=np.complex128)
    b[0] = np.sum(q * np.log(-d))
    for l in range(1, p + 1):
        b[l] = -np.sum(q / (l * d ** l))
    return b


__all__ = ["s2m", "me_eval", "m2m", "s2l", "le_eval", "l2l", "m2l",
           "log_p2m", "log_me_eval", "log_m2m", "log_m2l", "log_l2l",
           "log_le_eval", "log_p2l", "factorial"]
