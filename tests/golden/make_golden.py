"""Write the stored oracle values used by the full-size GPU parity tests and bench.py.

Calls only the CPU oracle (``oracle.direct``, ``oracle.grad``) and the seeded generators
(``workloads``): for each full-size workload, the direct-sum potential at a fixed-seed sample of
targets against ALL sources, written as text (index, Re phi, Im phi); for the differentiation
workload also the direct-sum gradients at a sample of indices (index, dl/dq, dl/dx, dl/dy).

    python tests/golden/make_golden.py [name ... | grad:name ... | dlp:name ... | forest | example2]

The readers (load, load_grad, load_forest) live in golden_io.py, which imports no oracle code.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import direct as D  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from golden_io import HERE, N_SAMPLE, forest_path, grad_path_for, load, load_grad, path_for  # noqa: E402,F401

GOLDEN = {
    "uniform_1m": lambda: workloads.uniform_1m(seed=1),
    "curve_4m": lambda: workloads.curve_4m(seed=1),
    "diff_1m": lambda: workloads.diff_1m(seed=1),
}


def write(name: str) -> str:
    w = GOLDEN[name]()
    idx = workloads.sample_targets(w.n, N_SAMPLE)
    t0 = time.time()
    phi = D.potential(w.x, w.y, w.q[0], w.impedance, xt=w.x[idx], yt=w.y[idx])
    dt = time.time() - t0
    p = path_for(name)
    with open(p, "w") as f:
        f.write(f"# oracle direct sum, workload {name} (seed 1, N={w.n}, impedance {w.impedance}), "
                f"{N_SAMPLE} sampled targets x all sources; columns: index re im\n")
        for i, v in zip(idx, phi):
            f.write(f"{int(i)} {v.real:.17e} {v.imag:.17e}\n")
    print(f"{name}: {dt:.1f} s -> {p}", flush=True)
    return p


GRAD_GOLDEN = {
    # incoming gradient g = w + i w' of the differentiation workload (loss l = Re sum conj(g) phi)
    "diff_1m": lambda: workloads.diff_1m(seed=1),
}


def write_grad(name: str) -> str:
    from oracle import grad as GR
    w = GRAD_GOLDEN[name]()
    g = w.extra["loss_w"] + 1j * w.extra["loss_w_im"]
    idx = workloads.sample_targets(w.n, N_SAMPLE, seed=4242)
    t0 = time.time()
    r = GR.sampled_gradients(w.x, w.y, w.q[0], w.impedance, g, idx)
    dt = time.time() - t0
    p = grad_path_for(name)
    with open(p, "w") as f:
        f.write(f"# oracle direct-sum gradients, workload {name} (seed 1, N={w.n}, impedance "
                f"{w.impedance}), g = loss_w + i loss_w_im, {N_SAMPLE} sampled indices x all "
                f"sources; columns: index dl/dq dl/dx dl/dy\n")
        for k, i in enumerate(idx):
            f.write(f"{int(i)} {r['grad_q'][k]:.17e} {r['grad_x'][k]:.17e} {r['grad_y'][k]:.17e}\n")
    print(f"{name} gradients: {dt:.1f} s -> {p}", flush=True)
    return p


def write_dlp(name: str) -> str:
    """The double-layer potential of the workload's charges as dipole densities, with the seeded
    normals of ``workloads.source_normals(N, seed=7)``, at the sampled targets against all sources."""
    from golden_io import dlp_path_for
    w = GOLDEN[name]()
    nx, ny = workloads.source_normals(w.n, seed=7)
    idx = workloads.sample_targets(w.n, N_SAMPLE)
    t0 = time.time()
    phi = D.double_layer(w.x, w.y, nx, ny, w.q[0], w.impedance, xt=w.x[idx], yt=w.y[idx])
    dt = time.time() - t0
    p = dlp_path_for(name)
    with open(p, "w") as f:
        f.write(f"# oracle double layer, workload {name} (seed 1, N={w.n}, impedance {w.impedance}), densities "
                f"= charges, normals source_normals(N, seed=7), {N_SAMPLE} sampled targets x all sources; "
                f"columns: index re im\n")
        for i, v in zip(idx, phi):
            f.write(f"{int(i)} {v.real:.17e} {v.imag:.17e}\n")
    print(f"{name} double layer: {dt:.1f} s -> {p}", flush=True)
    return p


FOREST_SAMPLE = {"instances": (0, 137, 300, 511), "vectors": (0, 63), "targets": 32}


def write_forest() -> str:
    """The batched workload (seed 1): direct sums over single instances at a few sampled targets
    (instances and vectors of FOREST_SAMPLE), from each instance's own generator."""
    sizes, lams = workloads.batched_forest_spec(seed=1)
    p = forest_path()
    t0 = time.time()
    rows = []
    for k in FOREST_SAMPLE["instances"]:
        x, y, q = workloads.batched_forest_instance(1, k, int(sizes[k]), 64)
        idx = workloads.sample_targets(x.size, FOREST_SAMPLE["targets"], seed=100 + k)
        for v in FOREST_SAMPLE["vectors"]:
            phi = D.potential(x, y, q[v], lams[k], xt=x[idx], yt=y[idx])
            rows += [(k, v, int(i), c) for i, c in zip(idx, phi)]
    with open(p, "w") as f:
        f.write("# oracle direct sums over single instances of the batched workload (seed 1); "
                "columns: instance vector index_in_instance re im\n")
        for k, v, i, c in rows:
            f.write(f"{k} {v} {i} {c.real:.17e} {c.imag:.17e}\n")
    print(f"batched_forest: {time.time() - t0:.1f} s -> {p}", flush=True)
    return p


def write_example2() -> str:
    """Example 2 of Section 5 with N_field + 8 N_source = 4000: the direct sum at every field point."""
    from golden_io import example2_path
    d = workloads.example2_sized(4000)
    t0 = time.time()
    phi = D.potential(d["src_x"], d["src_y"], d["q"], d["impedance"], xt=d["tgt_x"], yt=d["tgt_y"])
    p = example2_path()
    with open(p, "w") as f:
        f.write(f"# oracle direct sum, Example 2 (N_field + 8 N_source = 4000: {d['src_x'].size} sources, "
                f"{d['tgt_x'].size} field points, impedance {d['impedance']}); columns: target index re im\n")
        for i, v in enumerate(phi):
            f.write(f"{i} {v.real:.17e} {v.imag:.17e}\n")
    print(f"example2: {time.time() - t0:.1f} s -> {p}", flush=True)
    return p


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(GOLDEN) + ["grad:" + k for k in GRAD_GOLDEN]
                 + ["dlp:uniform_1m", "forest", "example2"]):
        if name.startswith("grad:"):
            write_grad(name[5:])
        elif name.startswith("dlp:"):
            write_dlp(name[4:])
        elif name == "forest":
            write_forest()
        elif name == "example2":
            write_example2()
        else:
            write(name)
