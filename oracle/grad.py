"""Gradients of the half-plane Robin potential by direct summation -- CPU oracle.

Test infrastructure only (see ``oracle/__init__``).

Convention (complex outputs, real inputs, as autograd frameworks use it): for an incoming
gradient g_i = dl/dRe(phi_i) + i dl/dIm(phi_i) of a real loss l, the loss behaves locally as
l = sum_i Re(conj(g_i) phi_i), and

  dl/dq_j  = Re sum_i conj(g_i) G(r_i, r_j)
  dl/dx_k  = Re[ conj(g_k) d_x Phi[q](r_k) + q_k d_x Phi[conj g](r_k) ]      (same for y)
  dl/dZ    = conj( sum_i conj(g_i) dphi_i/dZ )   (dl/dRe Z + i dl/dIm Z; phi is holomorphic in Z)

with Phi[c](r) = sum_j c_j G(r, r_j) and d_x acting on the target argument.  The position formula
uses the symmetry G(r, r') = G(r', r) (eq. (greensfunsymm)) to turn source-side derivatives into
target-side ones; the j = k image and reaction self terms are counted on both sides, as the chain
rule requires.

Kernel derivatives (target side), from the definitions:
  free   -(1/2pi) ln|r - r'|:       d_x = -(1/2pi) dx / r^2,          d_y = -(1/2pi) dy / r^2
  image  (1/2pi) ln|r - r'_im|:     d_x = (1/2pi) dx / r_im^2,        d_y = (1/2pi) (y + y') / r_im^2
  reaction I_0(X, Y), X = x - x', Y = y + y':  d_x = i I_1(X, Y), d_y = -I_1(X, Y)
           I_0(-X, Y):                          d_x = -i I_1(-X, Y), d_y = -I_1(-X, Y)
  (differentiating eq. (generalintegral) under the integral sign), and
  d/dZ I_0(x, y) = -(y - i x) I_0(x, y) - 1/(2 pi Z), from the closed form of I_0.
"""
from __future__ import annotations

import numpy as np

from .kernel import reaction_I0, reaction_In, green, TWO_PI


def _grad_green(xt, yt, xs, ys, Z, bc="robin"):
    """(d_x G, d_y G) at the target, arrays broadcasting like ``green``; free term skipped
    where r_t == r_s.  bc = "dirichlet" / "neumann": the kernels of eq. (ddd1.2)."""
    xt = np.asarray(xt, dtype=np.float64)
    yt = np.asarray(yt, dtype=np.float64)
    dx = xt - xs
    dy = yt - ys
    Y = yt + ys
    r2 = dx * dx + dy * dy
    ri2 = dx * dx + Y * Y
    same = r2 == 0.0
    inv = np.where(same, 0.0, 1.0 / np.where(same, 1.0, r2))
    isg = -1.0 if bc == "neumann" else 1.0
    gx = -dx * inv / TWO_PI + isg * dx / ri2 / TWO_PI
    gy = -dy * inv / TWO_PI + isg * Y / ri2 / TWO_PI
    if bc != "robin":
        return gx.astype(np.complex128), gy.astype(np.complex128)
    Ip = reaction_In(1, dx, Y, Z)[1]
    Im = reaction_In(1, -dx, Y, Z)[1]
    gx = gx + 1j * Ip - 1j * Im
    gy = gy - Ip - Im
    return gx, gy


def _dZ_green(xt, yt, xs, ys, Z):
    """dG/dZ (only the reaction term depends on Z)."""
    Z = complex(Z)
    dx = np.asarray(xt, dtype=np.float64) - xs
    Y = np.asarray(yt, dtype=np.float64) + ys
    out = 0.0
    for X in (dx, -dx):
        w = Y - 1j * X
        out = out + (-w * reaction_I0(X, Y, Z) - 1.0 / (TWO_PI * Z))
    return out


def potential_gradient(xs, ys, c, Z, idx=None, block=64):
    """(d_x Phi[c], d_y Phi[c]) at targets idx (default all), Phi[c](r) = sum_j c_j G(r, r_j)."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    c = np.asarray(c)
    if idx is None:
        idx = np.arange(xs.shape[0])
    gx = np.zeros(len(idx), dtype=np.complex128)
    gy = np.zeros(len(idx), dtype=np.complex128)
    for b0 in range(0, len(idx), block):
        ii = idx[b0:b0 + block]
        kx, ky = _grad_green(xs[ii, None], ys[ii, None], xs[None, :], ys[None, :], Z)
        gx[b0:b0 + block] = kx @ c
        gy[b0:b0 + block] = ky @ c
    return gx, gy


def direct_gradients(xs, ys, q, Z, g, idx=None):
    """Oracle gradients of l = sum_i Re(conj(g_i) phi_i) w.r.t. q, x, y (at indices idx) and Z.

    xs, ys, q : [N] real;  g : [N] complex.  Returns dict with grad_q, grad_x, grad_y (real,
    [len(idx)]) and grad_Z (complex).
    """
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    g = np.asarray(g, dtype=np.complex128)
    n = xs.shape[0]
    if idx is None:
        idx = np.arange(n)
    cg = np.conj(g)
    # dl/dq_j = Re sum_i conj(g_i) G(r_i, r_j) = Re Phi[conj g](r_j)
    G = green(xs[idx, None], ys[idx, None], xs[None, :], ys[None, :], Z)  # rows: r_j (symmetric)
    grad_q = np.real(G @ cg)
    qx, qy = potential_gradient(xs, ys, q, Z, idx)
    gx, gy = potential_gradient(xs, ys, cg, Z, idx)
    grad_x = np.real(cg[idx] * qx + q[idx] * gx)
    grad_y = np.real(cg[idx] * qy + q[idx] * gy)
    # dl/dZ over all pairs
    s = 0.0 + 0.0j
    for b0 in range(0, n, 64):
        D = _dZ_green(xs[b0:b0 + 64, None], ys[b0:b0 + 64, None], xs[None, :], ys[None, :], Z)
        s += np.sum(cg[b0:b0 + 64] * (D @ q))
    return {"grad_q": grad_q, "grad_x": grad_x, "grad_y": grad_y, "grad_Z": np.conj(s)}


def potential_dZ(xs, ys, q, Z, idx=None):
    """dphi/dZ at targets idx by direct summation."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    if idx is None:
        idx = np.arange(xs.shape[0])
    out = np.zeros(len(idx), dtype=np.complex128)
    for b0 in range(0, len(idx), 64):
        ii = idx[b0:b0 + 64]
        out[b0:b0 + 64] = _dZ_green(xs[ii, None], ys[ii, None], xs[None, :], ys[None, :], Z) @ q
    return out


# --- multiprocess sampling at large N (the same formulas, blocked over targets and sources) ----

_SRC = {}


def _grad_block(xt, yt, xs, ys, C, Z, chunk, bc="robin"):
    """[2, n_vec, len(xt)] gradient of Phi[C_v] at a block of targets."""
    nv = C.shape[0]
    acc = np.zeros((2, nv, xt.shape[0]), dtype=np.complex128)
    for s0 in range(0, xs.shape[0], chunk):
        s1 = min(xs.shape[0], s0 + chunk)
        kx, ky = _grad_green(xt[:, None], yt[:, None], xs[None, s0:s1], ys[None, s0:s1], Z, bc)
        acc[0] += C[:, s0:s1] @ kx.T
        acc[1] += C[:, s0:s1] @ ky.T
    return acc


def _dZ_block(xt, yt, xs, ys, C, Z, chunk):
    nv = C.shape[0]
    acc = np.zeros((nv, xt.shape[0]), dtype=np.complex128)
    for s0 in range(0, xs.shape[0], chunk):
        s1 = min(xs.shape[0], s0 + chunk)
        acc += C[:, s0:s1] @ _dZ_green(xt[:, None], yt[:, None], xs[None, s0:s1], ys[None, s0:s1], Z).T
    return acc


def _init_worker(xs, ys, C, Z, bc="robin"):
    _SRC.update(xs=xs, ys=ys, C=C, Z=Z, bc=bc)


def _work(args):
    kind, xt, yt, chunk = args
    if kind == "grad":
        return _grad_block(xt, yt, _SRC["xs"], _SRC["ys"], _SRC["C"], _SRC["Z"], chunk, _SRC["bc"])
    return _dZ_block(xt, yt, _SRC["xs"], _SRC["ys"], _SRC["C"], _SRC["Z"], chunk)


def _run(kind, xs, ys, C, Z, xt, yt, workers, target_block=8, chunk=1 << 14, bc="robin"):
    import os
    from concurrent.futures import ProcessPoolExecutor
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    blocks = [(kind, xt[i:i + target_block], yt[i:i + target_block], chunk)
              for i in range(0, xt.shape[0], target_block)]
    if workers <= 1 or len(blocks) <= 1:
        _init_worker(xs, ys, C, complex(Z), bc)
        parts = [_work(b) for b in blocks]
    else:
        with ProcessPoolExecutor(max_workers=workers, initializer=_init_worker,
                                 initargs=(xs, ys, C, complex(Z), bc)) as ex:
            parts = list(ex.map(_work, blocks))
    return np.concatenate(parts, axis=-1)


def field_at(xs, ys, q, Z, xt, yt, workers=None, bc="robin"):
    """(d_x phi, d_y phi) at separate targets (xt, yt), y >= 0, for real or complex charges q [ns]:
    the target-side kernel derivatives above summed over all sources, over a process pool."""
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    ys = np.ascontiguousarray(ys, dtype=np.float64)
    xt = np.ascontiguousarray(xt, dtype=np.float64)
    yt = np.ascontiguousarray(yt, dtype=np.float64)
    C = np.ascontiguousarray(np.asarray(q, dtype=np.complex128)[None, :])
    g = _run("grad", xs, ys, C, Z, xt, yt, workers, bc=bc)
    return g[0, 0], g[1, 0]


def sampled_gradients(xs, ys, q, Z, g, idx, workers=None, want_Z=False):
    """direct_gradients at the indices idx against ALL sources, over a process pool.  grad_Z
    (an all-pairs sum) only when want_Z."""
    from . import direct as D
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    ys = np.ascontiguousarray(ys, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    cg = np.conj(np.asarray(g, dtype=np.complex128))
    idx = np.asarray(idx)
    xt, yt = xs[idx], ys[idx]
    grad_q = np.real(D.potential(xs, ys, cg, Z, xt=xt, yt=yt, workers=workers))
    C = np.ascontiguousarray(np.stack([q.astype(np.complex128), cg]))
    gr = _run("grad", xs, ys, C, Z, xt, yt, workers)
    out = {"grad_q": grad_q,
           "grad_x": np.real(cg[idx] * gr[0, 0] + q[idx] * gr[0, 1]),
           "grad_y": np.real(cg[idx] * gr[1, 0] + q[idx] * gr[1, 1])}
    if want_Z:
        dphi = _run("dZ", xs, ys, np.ascontiguousarray(q[None, :].astype(np.complex128)), Z, xs, ys, workers)[0]
        out["grad_Z"] = np.conj(np.sum(cg * dphi))
    return out
