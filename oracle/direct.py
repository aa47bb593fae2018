"""O(N^2) direct summation of the half-plane Robin potential -- CPU oracle.

Test infrastructure only (see ``oracle/__init__``).

phi_i = sum_j q_j G(r_i, r_j)                                  (eq. (potential1))
      = Phi_free + Phi_1 + Phi_2                               (eqs. (1.2), (reactioncomp1))

The free-space term skips j with r_j == r_i bitwise (the j != i rule of
eq. (1.2), applied to coincident points too); the image and reaction terms keep
every j, including j = i.  Sources are summed in float64 chunks (a matrix
product per chunk).  Large target sets are split over a process pool.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from .kernel import green, green_dlp, reaction_I0, TWO_PI

_SRC = {}


def _block(xt, yt, xs, ys, q, Z, chunk, bc="robin", normals=None):
    """phi for a block of targets against all sources, q shape [n_vec, ns]; with normals = (nx, ny)
    the double-layer kernel ``green_dlp`` replaces G."""
    nv = q.shape[0]
    acc = np.zeros((nv, xt.shape[0]), dtype=np.complex128)
    for s0 in range(0, xs.shape[0], chunk):
        s1 = min(xs.shape[0], s0 + chunk)
        if normals is None:
            G = green(xt[:, None], yt[:, None], xs[None, s0:s1], ys[None, s0:s1], Z, bc=bc)
        else:
            G = green_dlp(xt[:, None], yt[:, None], xs[None, s0:s1], ys[None, s0:s1],
                          normals[0][None, s0:s1], normals[1][None, s0:s1], Z, bc=bc)
        acc += q[:, s0:s1] @ G.T
    return acc


def _init_worker(xs, ys, q, Z, bc="robin", normals=None):
    _SRC["xs"], _SRC["ys"], _SRC["q"], _SRC["Z"], _SRC["bc"] = xs, ys, q, Z, bc
    _SRC["normals"] = normals


def _work(args):
    xt, yt, chunk = args
    return _block(xt, yt, _SRC["xs"], _SRC["ys"], _SRC["q"], _SRC["Z"], chunk, _SRC["bc"], _SRC["normals"])


def potential(xs, ys, q, Z, xt=None, yt=None, workers: int | None = None,
              target_block: int = 16, chunk: int = 1 << 16, bc: str = "robin", normals=None):
    """Direct-sum potential at targets (default: targets = sources).

    xs, ys  : [ns] float64 source coordinates (ys > 0)
    q       : [ns] or [n_vec, ns] charges (real or complex)
    Z       : complex impedance (ignored for bc = "dirichlet" / "neumann", eq. (ddd1.2))
    normals : None, or (nx, ny) [ns] unit normals: then q are dipole densities and the sum is the
              double layer sum_j q_j n_j . grad_{r_j} G(r_i, r_j) (``kernel.green_dlp``)
    Returns complex128 [nt] (or [n_vec, nt]).
    """
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    ys = np.ascontiguousarray(ys, dtype=np.float64)
    q = np.asarray(q)
    squeeze = q.ndim == 1
    q2 = np.ascontiguousarray(q[None, :] if squeeze else q)
    if xt is None:
        xt, yt = xs, ys
    xt = np.ascontiguousarray(xt, dtype=np.float64)
    yt = np.ascontiguousarray(yt, dtype=np.float64)
    if normals is not None:
        normals = (np.ascontiguousarray(normals[0], dtype=np.float64),
                   np.ascontiguousarray(normals[1], dtype=np.float64))
    nt = xt.shape[0]
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    chunk = max(1, min(chunk, (1 << 20) // max(1, target_block)))
    blocks = [(xt[i:i + target_block], yt[i:i + target_block], chunk)
              for i in range(0, nt, target_block)]
    if workers <= 1 or len(blocks) <= 1:
        parts = [_block(b[0], b[1], xs, ys, q2, complex(Z), chunk, bc, normals) for b in blocks]
    else:
        with ProcessPoolExecutor(max_workers=workers, initializer=_init_worker,
                                 initargs=(xs, ys, q2, complex(Z), bc, normals)) as ex:
            parts = list(ex.map(_work, blocks))
    out = np.concatenate(parts, axis=1) if parts else np.zeros((q2.shape[0], 0), np.complex128)
    return out[0] if squeeze else out


def double_layer(xs, ys, nx, ny, mu, Z, xt=None, yt=None, bc: str = "robin", workers: int | None = None):
    """Double-layer potential sum_j mu_j n_j . grad_{r_j} G(r_i, r_j) (``kernel.green_dlp``) at
    the targets (default: the sources), mu real or complex [ns] or [n_vec, ns]."""
    return potential(xs, ys, mu, Z, xt=xt, yt=yt, workers=workers, chunk=1 << 12, bc=bc, normals=(nx, ny))


def potential_loops(xs, ys, q, Z, xt=None, yt=None, bc: str = "robin"):
    """Pure-Python double loop over (target, source) pairs; small inputs only.

    Written term by term from eqs. (1.2) and (reactioncomp1) as an independent
    check of the vectorised ``potential``.
    """
    import math
    if xt is None:
        xt, yt = xs, ys
    out = np.zeros(len(xt), dtype=np.complex128)
    for i in range(len(xt)):
        s = 0j
        for j in range(len(xs)):
            dx = float(xt[i]) - float(xs[j])
            dy = float(yt[i]) - float(ys[j])
            if not (dx == 0.0 and dy == 0.0):
                s += -float(q[j]) * math.log(math.hypot(dx, dy)) / TWO_PI
            image = float(q[j]) * math.log(math.hypot(dx, float(yt[i]) + float(ys[j]))) / TWO_PI
            if bc == "neumann":
                s -= image
                continue
            s += image
            if bc == "dirichlet":
                continue
            s += float(q[j]) * complex(reaction_I0(dx, float(yt[i]) + float(ys[j]), Z)
                                       + reaction_I0(-dx, float(yt[i]) + float(ys[j]), Z))
        out[i] = s
    return out


def imag_part_real_impedance(xs, ys, q, Z, xt=None, yt=None):
    """Exact Im(phi) for real impedance Z and real charges, in O(N).

    For real Z the lossless closed form printed in Section 2.1 (after Hein et
    al.) gives Im G = exp(-Z (y + y')) cos(Z (x - x')), and the log terms are
    real, so Im phi_i = exp(-Z y_i) [cos(Z x_i) C + sin(Z x_i) S] with
    C = sum_j q_j exp(-Z y_j) cos(Z x_j), S = sum_j q_j exp(-Z y_j) sin(Z x_j).
    """
    Z = float(np.real(Z))
    if xt is None:
        xt, yt = xs, ys
    q = np.asarray(q, dtype=np.float64)
    e = np.exp(-Z * np.asarray(ys))
    C = np.sum(q * e * np.cos(Z * np.asarray(xs)), axis=-1)
    S = np.sum(q * e * np.sin(Z * np.asarray(xs)), axis=-1)
    et = np.exp(-Z * np.asarray(yt))
    C = np.asarray(C)[..., None]
    S = np.asarray(S)[..., None]
    return et * (np.cos(Z * np.asarray(xt)) * C + np.sin(Z * np.asarray(xt)) * S)


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2 over complex vectors (b is the reference)."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
