"""Green's function of the 2-D Laplace equation in the half plane y > 0 with the
Robin condition dG/dn - Z_eps G = 0 on y = 0 (n = -y_hat) -- CPU oracle.

Test infrastructure only (see ``oracle/__init__``).

Notation (Section 2.1):
  Z          complex impedance Z_eps = Z + i eps, Re Z > 0, Im Z >= 0 (eps = 0 is
             the lossless case, taken by limiting absorption).
  I_n(x, y)  = 1/(2 pi n!) int_0^inf exp(-lam y + i lam x) lam^n / (lam - Z) dlam
             (eq. (generalintegral)).
  G_Z        = I_0(x - x', y + y') + I_0(x' - x, y + y')   (eq. (reactdecomposition)).
  G          = -(1/2pi) ln|r - r'| + (1/2pi) ln|r - r'_im| + G_Z (eq. (ddGreensfunimp)).

Reading of the initial value (the paper's printed closed form for I_0 next to
eq. (integralrecursion) has the sign of x flipped and drops the -i pi that its
own lossless limit (aaa1.5) carries): with w = y - i x and P = Z w,

  I_0(x, y) = (1/2pi) exp(-P) (i pi - Ei(P)),

with the principal-branch exponential integral Ei(z) = gamma + ln z + sum z^k/(k k!)
(``scipy.special.expi``).  The same expression holds for eps > 0 and eps = 0; it is
pinned against quadrature of the defining integral in the tests.
"""
from __future__ import annotations

import numpy as np
from scipy.special import expi

TWO_PI = 2.0 * np.pi


def reaction_P(x, y, Z):
    """P = Z_eps (y - i x), the pole of the integrand after t = (y - i x) lam."""
    return complex(Z) * (np.asarray(y, dtype=np.float64) - 1j * np.asarray(x, dtype=np.float64))


def reaction_I0(x, y, Z):
    """I_0(x, y) for y > 0 (eq. (generalintegral), n = 0), closed form via Ei."""
    P = reaction_P(x, y, Z)
    return np.exp(-P) * (1j * np.pi - expi(P)) / TWO_PI


def reaction_In(nmax: int, x, y, Z):
    """I_0 .. I_nmax by the upward recursion of eq. (integralrecursion):

        I_n = 1 / (2 pi n (y - i x)^n) + (Z / n) I_{n-1}.

    Returns an array of shape (nmax + 1,) + shape(x).
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = y - 1j * x
    Z = complex(Z)
    out = np.empty((nmax + 1,) + np.broadcast(x, y).shape, dtype=np.complex128)
    out[0] = reaction_I0(x, y, Z)
    for n in range(1, nmax + 1):
        out[n] = 1.0 / (TWO_PI * n * w ** n) + (Z / n) * out[n - 1]
    return out


def reaction_GZ(X, Y, Z):
    """G_Z at X = x - x', Y = y + y' (eq. (reactdecomposition))."""
    return reaction_I0(X, Y, Z) + reaction_I0(-np.asarray(X, dtype=np.float64), Y, Z)


def green(xt, yt, xs, ys, Z, skip_self: bool = True, bc: str = "robin"):
    """Full Green's function G(r_t, r_s) (eq. (ddGreensfunimp)), broadcasting.

    With skip_self the free-space log term is dropped where r_t == r_s bitwise
    (the j != i rule of eq. (1.2)); the image and reaction terms are kept.
    bc = "dirichlet" / "neumann" gives the half-plane functions of eq. (ddd1.2)
    instead: no reaction term, the image log term with + / - (Z is ignored).
    """
    xt = np.asarray(xt, dtype=np.float64)
    yt = np.asarray(yt, dtype=np.float64)
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    dx = xt - xs
    r2 = dx * dx + (yt - ys) ** 2
    r2_im = dx * dx + (yt + ys) ** 2
    with np.errstate(divide="ignore"):
        lr2 = np.log(r2)
    free = -lr2 / (2.0 * TWO_PI)
    if skip_self:
        free = np.where(r2 == 0.0, 0.0, free)
    image = np.log(r2_im) / (2.0 * TWO_PI)
    if bc == "dirichlet":
        return free + image
    if bc == "neumann":
        return free - image
    if bc != "robin":
        raise ValueError(f"unknown boundary condition {bc!r}")
    return free + image + reaction_GZ(dx, yt + ys, Z)


def green_dlp(xt, yt, xs, ys, nx, ny, Z, bc: str = "robin"):
    """Double-layer kernel n_s . grad_{r_s} G(r_t, r_s) for a unit normal (nx, ny) at the source,
    broadcasting, from the derivatives of each term of G with respect to the source point:

      free      -(1/2pi) ln|r_t - r_s|         ->  (1/2pi) (nx dx + ny dy) / r^2   (dx = x_t - x_s)
      image     (1/2pi) ln|r_t - r_s^im|       ->  (1/2pi) (-nx dx + ny Y) / r_im^2   (Y = y_t + y_s)
      reaction  I_0(X, Y) + I_0(-X, Y), X = dx ->  nx (-i I_1(X, Y) + i I_1(-X, Y)) - ny (I_1(X, Y) + I_1(-X, Y))

    (d_X I_0 = i I_1 and d_Y I_0 = -I_1, eq. (integralrecursion) with n = 1).  The free term is
    skipped where r_t == r_s; bc = "dirichlet" / "neumann" as in ``green``.
    """
    xt = np.asarray(xt, dtype=np.float64)
    yt = np.asarray(yt, dtype=np.float64)
    dx = xt - xs
    dy = yt - ys
    Y = yt + ys
    r2 = dx * dx + dy * dy
    ri2 = dx * dx + Y * Y
    same = r2 == 0.0
    inv = np.where(same, 0.0, 1.0 / np.where(same, 1.0, r2))
    free = (nx * dx + ny * dy) * inv / TWO_PI
    image = (-nx * dx + ny * Y) / ri2 / TWO_PI
    if bc == "dirichlet":
        return (free + image).astype(np.complex128)
    if bc == "neumann":
        return (free - image).astype(np.complex128)
    if bc != "robin":
        raise ValueError(f"unknown boundary condition {bc!r}")
    Ip = reaction_In(1, dx, Y, Z)[1]
    Im = reaction_In(1, -dx, Y, Z)[1]
    return free + image + nx * (-1j * Ip + 1j * Im) - ny * (Ip + Im)


def green_dirichlet(xt, yt, xs, ys):
    """Dirichlet half-plane Green's function (eq. (ddd1.2), image term with '+'):

    -(1/2pi) ln|r - r'| + (1/2pi) ln|r - r'_im|, the Z -> infinity limit of G.
    """
    dx = np.asarray(xt) - np.asarray(xs)
    r2 = dx * dx + (np.asarray(yt) - np.asarray(ys)) ** 2
    r2_im = dx * dx + (np.asarray(yt) + np.asarray(ys)) ** 2
    return (np.log(r2_im) - np.log(r2)) / (2.0 * TWO_PI)


def reaction_In_mp(nmax: int, x: float, y: float, Z, dps: int = 50):
    """I_0 .. I_nmax at one point in multiple precision (mpmath), same definitions as
    ``reaction_In``: the Ei closed form for I_0 and the recursion of eq. (integralrecursion)
    carried out with ``dps`` digits, so that the upward recursion's growth of rounding error
    (about exp(|Z w|) at orders near |Z w|) does not reach float64 precision.
    Returns complex128 [nmax + 1].
    """
    import mpmath as mp
    with mp.workdps(dps):
        Zm = mp.mpc(complex(Z).real, complex(Z).imag)
        w = mp.mpc(float(y), -float(x))
        P = Zm * w
        I = mp.exp(-P) * (1j * mp.pi - mp.ei(P)) / (2 * mp.pi)
        out = [complex(I)]
        for n in range(1, nmax + 1):
            I = 1 / (2 * mp.pi * n * w ** n) + Zm / n * I
            out.append(complex(I))
    return np.array(out)
