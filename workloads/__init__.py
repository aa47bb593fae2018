"""Seeded synthetic inputs for the half-plane Robin FMM.

This module only draws random numbers and lays out arrays; it holds none of the
method's arithmetic.  Both the CPU oracle's tests and the GPU path's tests and
benchmark take their inputs from here, so that the two sides see bit-identical
coordinates and charges.

Every generator uses ``numpy.random.default_rng(seed)`` and draws in a fixed
order (x, then y, then the charge vectors).  The point sets follow the shapes
the paper's experiments and the workload list describe:

* ``plain_small``    N=2,000, sources = targets uniform in [0,1]x[0.05,1.05],
                     charges U[-1,1], real impedance 1.0.
* ``uniform_1m``     N=1,048,576 uniform in [0,1]x[1e-3,1.001], charges U[-1,1],
                     real impedance 1.0.
* ``curve_4m``       N=4,194,304: 80% within 1e-3 (vertical offset) of the
                     curve y = 0.3 + 0.1 sin(6 pi x), x in [0,4]; 20% uniform in
                     [0,4]x[1e-4,1]; charges N(0,1); impedance 1+0.5i.
* ``batched_forest`` 512 instances, N_k log-uniform in [1e3, 2e5], each uniform
                     in [0,1]x[0.01,1.01], impedance_k log-uniform in [0.1,10],
                     64 charge vectors N(0,1) per instance.
* ``diff_1m``        N=1,048,576 uniform in [0,1]x[0.01,1.01], charges U[-1,1],
                     impedance 2.0, loss weights w ~ N(0,1).
* ``example1``       the single source/target pair and expansion centres of the
                     paper's Example 1 (Section 5).
* ``example2``       eight charged unit circles plus a Cartesian grid of field
                     points (Section 5, Example 2).

The paper evaluates on no public dataset; these synthetic sets stand in for
its point distributions.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload", "plain_small", "uniform_1m", "curve_4m", "diff_1m",
    "batched_forest", "batched_forest_spec", "batched_forest_instance", "example1", "example2", "example2_sized", "uniform", "sample_targets",
]


@dataclass
class Workload:
    name: str
    x: np.ndarray              # float64 [N]
    y: np.ndarray              # float64 [N], > 0
    q: np.ndarray              # float64 [n_vec, N]
    impedance: complex         # Z_eps, Re > 0, Im >= 0
    p: int                     # truncation order (coefficients 0..p)
    leaf_size: int
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def uniform(n: int, seed: int, x_range=(0.0, 1.0), y_range=(0.05, 1.05),
            charge="uniform", n_vec: int = 1, impedance: complex = 1.0,
            p: int = 20, leaf_size: int = 40, name: str = "uniform") -> Workload:
    rng = np.random.default_rng(seed)
    x = rng.uniform(x_range[0], x_range[1], n)
    y = rng.uniform(y_range[0], y_range[1], n)
    if charge == "uniform":
        q = rng.uniform(-1.0, 1.0, (n_vec, n))
    elif charge == "normal":
        q = rng.standard_normal((n_vec, n))
    else:
        raise ValueError(charge)
    return Workload(name, x, y, q, complex(impedance), p, leaf_size)


def plain_small(seed: int = 1, n: int = 2000) -> Workload:
    return uniform(n, seed, (0.0, 1.0), (0.05, 1.05), "uniform", 1, 1.0, 20, 40,
                   name="plain_small_2k")


def uniform_1m(seed: int = 1, n: int = 1 << 20, p: int = 30,
               leaf_size: int = 40) -> Workload:
    return uniform(n, seed, (0.0, 1.0), (1e-3, 1.001), "uniform", 1, 1.0, p,
                   leaf_size, name="uniform_1m")


def diff_1m(seed: int = 1, n: int = 1 << 20, p: int = 30,
            leaf_size: int = 40) -> Workload:
    w = uniform(n, seed, (0.0, 1.0), (0.01, 1.01), "uniform", 1, 2.0, p,
                leaf_size, name="diff_1m")
    rng = np.random.default_rng(seed + 1000)
    w.extra["loss_w"] = rng.standard_normal(n)
    w.extra["loss_w_im"] = rng.standard_normal(n)
    return w


def curve_4m(seed: int = 1, n: int = 1 << 22, p: int = 30,
             leaf_size: int = 40) -> Workload:
    rng = np.random.default_rng(seed)
    n_band = int(round(0.8 * n))
    n_uni = n - n_band
    xb = rng.uniform(0.0, 4.0, n_band)
    off = rng.uniform(-1e-3, 1e-3, n_band)
    xu = rng.uniform(0.0, 4.0, n_uni)
    yu = rng.uniform(1e-4, 1.0, n_uni)
    yb = 0.3 + 0.1 * np.sin(6.0 * np.pi * xb) + off
    x = np.concatenate([xb, xu])
    y = np.concatenate([yb, yu])
    q = rng.standard_normal((1, n))
    return Workload("curve_4m", x, y, q, complex(1.0, 0.5), p, leaf_size)


def batched_forest_spec(seed: int = 1, n_inst: int = 512, n_min: float = 1e3, n_max: float = 2e5):
    """Sizes N_k = round(exp U[ln n_min, ln n_max)) and real impedances exp U[ln 0.1, ln 10] of the
    batched workload's instances."""
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_inst))).astype(np.int64)
    lams = np.exp(rng.uniform(np.log(0.1), np.log(10.0), n_inst))
    return sizes, lams


def batched_forest_instance(seed: int, k: int, size: int, n_vec: int):
    """Instance k: points uniform in [0, 1] x [0.01, 1.01] and n_vec charge vectors q ~ N(0, 1),
    from a generator of its own (seed, k), so any instance can be rebuilt alone."""
    rng = np.random.default_rng([seed, k])
    x = rng.uniform(0.0, 1.0, size)
    y = rng.uniform(0.01, 1.01, size)
    q = rng.standard_normal((n_vec, size))
    return x, y, q


def batched_forest(seed: int = 1, n_inst: int = 512, n_vec: int = 64,
                   n_min: float = 1e3, n_max: float = 2e5):
    """All instances concatenated: (x, y, offsets [n_inst + 1], impedances [n_inst],
    q [n_vec, sum N_k])."""
    sizes, lams = batched_forest_spec(seed, n_inst, n_min, n_max)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = np.empty(off[-1])
    y = np.empty(off[-1])
    q = np.empty((n_vec, off[-1]))
    for k in range(n_inst):
        a, b = off[k], off[k + 1]
        x[a:b], y[a:b], q[:, a:b] = batched_forest_instance(seed, k, int(sizes[k]), n_vec)
    return x, y, off, lams, q


def example1():
    """Example 1 of Section 5: one target/source pair and the expansion centres."""
    return dict(
        target=(0.625, 1.25), source=(0.0, 0.375),
        target_centre=(0.65625, 1.09375), target_parent_centre=(0.8125, 0.9375),
        source_centre=(0.03125, -0.46875), source_parent_centre=(0.1875, -0.3125),
        charge=1.0,
    )


def example2(n_source: int, n_field_x: int, n_field_y: int):
    """Example 2 of Section 5: eight unit circles with uniform line charge.

    Source points are the midpoints of n_source equal arcs on each circle, each
    carrying charge 2*pi/n_source; field points form a uniform Cartesian mesh on
    [-4.4, 4.4] x [0, 4.2] (the mesh includes points on y = 0).
    """
    centres = [(-3.3 + 2.2 * k, 1.01) for k in range(4)] + \
              [(-3.3 + 2.2 * k, 3.2) for k in range(4)]
    th = (np.arange(n_source) + 0.5) * (2.0 * np.pi / n_source)
    sx = np.concatenate([cx + np.cos(th) for cx, _ in centres])
    sy = np.concatenate([cy + np.sin(th) for _, cy in centres])
    q = np.full(sx.shape, 2.0 * np.pi / n_source)
    gx, gy = np.meshgrid(np.linspace(-4.4, 4.4, n_field_x),
                         np.linspace(0.0, 4.2, n_field_y), indexing="xy")
    return dict(src_x=sx, src_y=sy, q=q, tgt_x=gx.ravel(), tgt_y=gy.ravel(),
                impedance=1.0)


def example2_sized(n_total: int):
    """Example 2 with N_field + 8 N_source = n_total, split evenly between sources and field
    points (the paper fixes only the sum): N_source = n_total // 16 per circle, and a field mesh of
    about n_total / 2 points whose spacing is the same in x and y on [-4.4, 4.4] x [0, 4.2]."""
    n_source = max(1, n_total // 16)
    n_field = max(4, n_total - 8 * n_source)
    ny = max(2, int(round(np.sqrt(n_field * 4.2 / 8.8))))
    nx = max(2, n_field // ny)
    return example2(n_source, nx, ny)


def source_normals(n: int, seed: int = 7):
    """Unit normals (nx, ny) at n source points, angles uniform on [0, 2 pi) (double-layer inputs)."""
    th = np.random.default_rng(seed).uniform(0.0, 2.0 * np.pi, n)
    return np.cos(th), np.sin(th)


def sample_targets(n: int, k: int, seed: int = 12345) -> np.ndarray:
    """Fixed-seed sorted subset of k target indices out of n."""
    rng = np.random.default_rng(seed)
    if k >= n:
        return np.arange(n)
    return np.sort(rng.choice(n, size=k, replace=False))
