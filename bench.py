#!/usr/bin/env python
"""Throughput of the half-plane Robin FMM evaluation on one MI355X.

One step = one fmmhp_eval (Algorithm 2: P2M, M2M, M2L, P2L, L2L, L2P + M2P + near field and
the surface term) over the 1,048,576-point uniform workload (x ~ U[0,1], y ~ U[1e-3, 1.001],
charges U[-1,1], impedance 1.0) with the plan (tree, lists, tables) already built and all
inputs resident in device memory.  Prints ONE JSON line.  Extra fields: the p = 30 rate, the
forward + adjoint rate (fmmhp_backward), plan time, per-phase times.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--tol 1e-10 | --p P --leaf L]

By default the truncation order p and the leaf size come from the library's autotuner
(fmmhp_tune) for a target relative l2 error of 1e-10, measured against the GPU direct sum at 256
targets; the bench output is then checked against the CPU oracle's stored direct-sum sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X fp64 vector (and matrix) peak
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MATRIX_TFLOPS = 157.3  # MI355X fp32 matrix peak

# HBM bytes of k_m2l per evaluation measured with rocprofv3 counter runs (2.00 x FETCH_SIZE + 1.00 x
# WRITE_SIZE, the factors a plain 256 MiB copy gives), keyed by a hash of the evaluation sources and
# (p, leaf size): reported (per launch) only while the kernels are the ones that were measured.
# (k_m2l runs as two launches per evaluation, deep and coarse levels; the figures are their sum.)
M2L_TRAFFIC = {("40e128ed52690a09", 20, 32): 160.0e6}
# k_near per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled as above), same key
NEAR_TRAFFIC = {("40e128ed52690a09", 20, 32): 52.4e6}


def NEAR_ALG_BYTES(info):
    """Algorithmic HBM bytes of the near field per evaluation: every point's coordinates and charge
    read once (24 bytes) and its near-field sum written once (16 bytes)."""
    return 40.0 * info["n"]


def M2L_ALG_BYTES(info):
    """Algorithmic HBM bytes of k_m2l per evaluation: every box's multipole read once and its local
    written once (16 (p + 1) bytes each)."""
    return 2.0 * 16.0 * (info["p"] + 1) * info["nbox"]


def eval_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("fmm.hip", "internal.hpp", "special.hpp", "cplx.hpp"):
        with open(os.path.join(ROOT, "paper_2507_21913_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--p", type=int, default=0, help="truncation order (0: autotune for --tol)")
    ap.add_argument("--leaf", type=int, default=0, help="leaf size (0: autotune, or 40 with --p)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--near-walk", type=int, default=0,
                    help="near-field launch shape with --p (0: library default; see fmmhp_opts)")
    ap.add_argument("--near-groups", type=int, default=0)
    ap.add_argument("--no-p30", action="store_true", help="skip the extra p=30 measurement")
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=128,
                    help="targets of the oracle's direct sum timed for the CPU baseline")
    ap.add_argument("--quiet-extra", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-workload measurement")
    ap.add_argument("--only", choices=("curve", "batched", "fwd_bwd"), default=None,
                    help="run only that workload's measurement (for profiling it) and print its record")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def host_cpu():
    """(logical CPUs of the host, CPUs this process may run on, CPU model)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    if not model:
        import platform
        model = platform.processor() or platform.machine()
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return os.cpu_count() or 1, avail, model


def cpu_baseline(w, k):
    """Time the CPU oracle (plain float64 direct sum) on k sampled targets x all sources, one worker
    process per host core this process may use, at most 16 (the host-core share of one GPU on the
    machines this runs on)."""
    import workloads
    from oracle import direct as D
    nproc, avail, model = host_cpu()
    workers = max(1, min(16, avail))
    idx = workloads.sample_targets(w.n, k, seed=777)
    t0 = time.perf_counter()
    D.potential(w.x, w.y, w.q[0], w.impedance, xt=w.x[idx], yt=w.y[idx], workers=workers)
    dt = time.perf_counter() - t0
    return {"value": k / dt / 1e6, "unit": "Mpts/s", "cores": workers, "kind": "oracle",
            "sample": f"{k} targets x {w.n} sources (direct sum, float64), {dt:.1f} s",
            "extrapolated_full_s": dt * w.n / k, "host_nproc": nproc, "host_cpus_available": avail,
            "cpu_model": model}


def example2_extra(dev, sizes=(4000, 1 << 16, 1 << 20), p=10, leaf=32, reps=10):
    """The paper's Example 2 (eight charged circles, a field mesh reaching y = 0) with separate
    targets: eval time against N_field + 8 N_source at p = 10 (the paper's O(N) timing), and the
    rel-l2 error against the stored oracle values at N = 4000 for p = 5..30."""
    import numpy as np
    import torch

    import paper_2507_21913_amd as F
    import workloads
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden"))
    from golden_io import load_example2
    out = {"p": p, "leaf_size": leaf, "timing": []}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for n_total in sizes:
        d = workloads.example2_sized(n_total)
        t = {k: torch.as_tensor(d[k], device=dev) for k in ("src_x", "src_y", "tgt_x", "tgt_y", "q")}
        plan = F.HalfPlaneFMM.with_targets(t["src_x"], t["src_y"], t["tgt_x"], t["tgt_y"], d["impedance"],
                                           p=p, leaf_size=leaf)
        res = torch.empty(d["tgt_x"].size, dtype=torch.complex128, device=dev)
        for _ in range(2):
            plan(t["q"], out=res)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            plan(t["q"], out=res)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        n_pts = d["src_x"].size + d["tgt_x"].size
        out["timing"].append({"n_field_plus_8n_source": n_pts, "n_source": d["src_x"].size,
                              "n_field": d["tgt_x"].size, "ms": ms, "mpts_s": n_pts / (ms * 1e-3) / 1e6})
        plan.close()
    ref = load_example2()
    if ref is not None:
        d = workloads.example2_sized(4000)
        t = {k: torch.as_tensor(d[k], device=dev) for k in ("src_x", "src_y", "tgt_x", "tgt_y", "q")}
        errs = {}
        for pp in (5, 10, 15, 20, 25, 30):
            plan = F.HalfPlaneFMM.with_targets(t["src_x"], t["src_y"], t["tgt_x"], t["tgt_y"], d["impedance"],
                                               p=pp, leaf_size=leaf)
            phi = plan(t["q"]).cpu().numpy()
            plan.close()
            errs[pp] = float(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
        out["rel_l2_vs_oracle_n4000"] = errs
    return out


def curve_extra(dev, steps):
    """The nonuniform workload with a complex impedance (N = 4,194,304: 80% within 1e-3 of the curve
    y = 0.3 + 0.1 sin(6 pi x), 20% uniform; impedance 1 + 0.5i; p = 30, leaf 40): evaluation time and
    rel-l2 against the stored oracle sample."""
    import numpy as np
    import torch

    import paper_2507_21913_amd as F
    import workloads
    from golden_io import load

    w = workloads.curve_4m(seed=1)
    x, y, q = (torch.as_tensor(v, device=dev) for v in (w.x, w.y, w.q[0]))
    t0 = time.perf_counter()
    plan = F.HalfPlaneFMM(x, y, w.impedance, p=w.p, leaf_size=w.leaf_size)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    out = torch.empty(w.n, dtype=torch.complex128, device=dev)
    for _ in range(2):
        plan(q, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan(q, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res = {"workload": "curve_4m: N=4,194,304, 80% within 1e-3 of y = 0.3 + 0.1 sin(6 pi x), impedance 1+0.5i",
           "p": w.p, "leaf_size": w.leaf_size, "ms_per_step": ms, "mpts_s": w.n / (ms * 1e-3) / 1e6,
           "plan_ms": plan_ms, "depth": plan.info()["depth"]}
    g = load("curve_4m")
    if g is not None:
        got = out.cpu().numpy()[g[0]]
        res["rel_l2_vs_oracle_sample"] = float(np.linalg.norm(got - g[1]) / np.linalg.norm(g[1]))
    plan.close()
    return res


def fwd_bwd_extra(dev, p, leaf, shape, steps):
    """The differentiation workload (N = 1,048,576 uniform in [0,1] x [0.01,1.01], charges U[-1,1],
    impedance 2, loss l = Re sum_i conj(g_i) phi_i with g = w + i w', w, w' ~ N(0, 1)) on the plan the
    benchmark times: the plain FP64 forward, and forward + fmmhp_backward_device (dl/dq, dl/dx, dl/dy
    and dl/dZ, the impedance gradient left on the device) in one timed loop; gradients against the
    oracle's stored direct-sum sample at 256 indices, dl/dZ against a central difference of the GPU
    forward."""
    import numpy as np
    import torch

    import paper_2507_21913_amd as F
    import workloads
    from golden_io import load_grad

    w = workloads.diff_1m(seed=1)
    g = w.extra["loss_w"] + 1j * w.extra["loss_w_im"]
    x, y, q = (torch.as_tensor(v, device=dev) for v in (w.x, w.y, w.q[0]))
    gg = torch.as_tensor(g, device=dev)
    plan = F.HalfPlaneFMM(x, y, w.impedance, p=p, leaf_size=leaf, **shape)
    out = torch.empty(w.n, dtype=torch.complex128, device=dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_f = timed(lambda: plan(q, out=out))

    def fb():
        plan(q, out=out)
        return plan.backward(q, gg, lambda_on_device=True)

    ms_fb = timed(fb)
    r = fb()
    torch.cuda.synchronize()
    res = {"workload": "diff_1m: N=1,048,576 uniform in [0,1]x[0.01,1.01], charges U[-1,1], impedance 2.0, "
                       "g = w + i w' (standard normal)",
           "p": plan.info()["p"], "leaf_size": leaf, "fwd_ms": ms_f, "ms_per_step": ms_fb,
           "mpts_s": w.n / (ms_fb * 1e-3) / 1e6, "bwd_over_fwd": (ms_fb - ms_f) / ms_f,
           "outputs": "phi; dl/dq, dl/dx, dl/dy, dl/dZ (on the device, no host synchronisation)"}
    gr = load_grad("diff_1m")
    if gr is not None:
        idx, ref = gr
        res["grad_rel_l2_vs_oracle_sample"] = {
            k: float(np.linalg.norm(r[k].cpu().numpy()[idx] - ref[:, j]) / np.linalg.norm(ref[:, j]))
            for j, k in enumerate(("q", "x", "y"))}
    dlz = r["lambda"].cpu().numpy()[0, 0]
    plan.close()
    # one autograd step as a training loop runs it: potential() builds its plan, evaluates phi, and
    # the loss's backward gives dl/dx, dl/dy, dl/dq and dl/dZ (the impedance gradient to the host)
    xr, yr, qr = (v.clone().requires_grad_(True) for v in (x, y, q))
    lam = torch.tensor(complex(w.impedance).real, dtype=torch.float64, requires_grad=True)  # real impedance 2

    def step(reuse):
        for t in (xr, yr, qr, lam):
            t.grad = None
        ph = F.potential(xr, yr, qr, lam, p=p, leaf_size=leaf, reuse_plan=reuse)
        loss = torch.sum(torch.view_as_real(ph) * torch.view_as_real(gg))
        loss.backward()

    for key, reuse, n_ag, what in (
            ("autograd_step", False, 3,
             "plan build + forward + backward (dl/dx, dl/dy, dl/dq, dl/dZ to the host), as when the points move"),
            ("autograd_step_same_points", True, 10,
             "forward + backward on the plan potential() keeps for unchanged points (dl/dZ to the host)")):
        step(reuse)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_ag):
            step(reuse)
        torch.cuda.synchronize()
        ms_ag = (time.perf_counter() - t0) * 1e3 / n_ag
        res[key] = {"ms": ms_ag, "mpts_s": w.n / (ms_ag * 1e-3) / 1e6, "includes": what,
                    "launch_shape": "library default"}
    F.clear_potential_plans()
    hz = 1e-5 * w.impedance
    ls = []
    for Zs in (w.impedance + hz, w.impedance - hz):
        p2 = F.HalfPlaneFMM(x, y, Zs, p=p, leaf_size=leaf, **shape)
        ls.append(float(torch.sum(torch.view_as_real(p2(q)) * torch.view_as_real(gg)).item()))
        p2.close()
    fd = (ls[0] - ls[1]) / (2 * hz)
    res["dl_dReZ"] = float(dlz)
    res["dl_dReZ_rel_vs_central_difference"] = float(abs(dlz - fd) / abs(fd))
    return res


def batched_extra(dev, p, leaf, steps):
    """The batched workload (512 instances, N_k log-uniform in [1e3, 2e5], impedances log-uniform
    in [0.1, 10], 64 charge vectors): one forest plan evaluating all instances and vectors in the
    same launches (recorded into a HIP graph), against plain plans evaluated one instance and one
    vector at a time."""
    import numpy as np
    import torch

    import paper_2507_21913_amd as F
    import workloads
    from golden_io import load_forest

    t0 = time.perf_counter()
    x, y, off, lams, q = workloads.batched_forest(seed=1)
    gen_s = time.perf_counter() - t0
    n, nv = int(off[-1]), q.shape[0]
    xt = torch.as_tensor(x, device=dev)
    yt = torch.as_tensor(y, device=dev)
    qt = torch.as_tensor(q, device=dev)
    del q
    st = torch.cuda.Stream(dev)
    res = {"workload": f"batched_forest: {len(lams)} instances, N={n}, {nv} vectors, impedances "
                       "log-uniform [0.1, 10]", "p": p, "leaf_size": leaf, "generate_s": gen_s}
    with torch.cuda.stream(st):
        t0 = time.perf_counter()
        plan = F.HalfPlaneFMM.batched(xt, yt, off, lams.tolist(), p=p, leaf_size=leaf, graph=True)
        st.synchronize()
        res["plan_ms"] = (time.perf_counter() - t0) * 1e3
        out = torch.empty((nv, n), dtype=torch.complex128, device=dev)
        plan(qt, out=out)  # records the graph
        st.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            plan(qt, out=out)
        e1.record(st)
        st.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res["batched_ms_per_step"] = ms
        res["batched_mpts_s"] = n * nv / (ms * 1e-3) / 1e6
        g = load_forest()
        if g is not None:
            ks, vs, idx, ref = g
            got = np.array([out[v, off[k] + i].item() for k, v, i in zip(ks, vs, idx)])
            res["rel_l2_vs_oracle_sample"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        del out
        info = plan.info()
        res["tree"] = {"nbox": info["nbox"], "depth": info["depth"], "device_bytes": info["device_bytes"]}
        plan.close()
        # the same forest with the upper-source M2L on the FP32 matrix cores
        plan = F.HalfPlaneFMM.batched(xt, yt, off, lams.tolist(), p=p, leaf_size=leaf, graph=True, m2l_fp32=True)
        out = torch.empty((nv, n), dtype=torch.complex128, device=dev)
        plan(qt, out=out)
        st.synchronize()
        e0.record(st)
        for _ in range(steps):
            plan(qt, out=out)
        e1.record(st)
        st.synchronize()
        ms32 = e0.elapsed_time(e1) / steps
        r32 = {"ms_per_step": ms32, "mpts_s": n * nv / (ms32 * 1e-3) / 1e6, "over_fp64": ms / ms32}
        if g is not None:
            got = np.array([out[v, off[k] + i].item() for k, v, i in zip(ks, vs, idx)])
            r32["rel_l2_vs_oracle_sample"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        res["m2l_fp32"] = r32
        del out
        plan.close()
    # plain: one plan per instance, one vector at a time (vector 0 timed; the others are the same work)
    plans = [F.HalfPlaneFMM(xt[off[k]:off[k + 1]], yt[off[k]:off[k + 1]], float(lams[k]), p=p, leaf_size=leaf)
             for k in range(len(lams))]
    out1 = torch.empty(n, dtype=torch.complex128, device=dev)
    q0 = qt[0].contiguous()
    for k, pk in enumerate(plans):
        pk(q0[off[k]:off[k + 1]], out=out1[off[k]:off[k + 1]])
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for k, pk in enumerate(plans):
        pk(q0[off[k]:off[k + 1]], out=out1[off[k]:off[k + 1]])
    e1.record()
    torch.cuda.synchronize()
    ms1 = e0.elapsed_time(e1)
    for pk in plans:
        pk.close()
    res["plain_ms_per_vector"] = ms1
    res["plain_mpts_s"] = n / (ms1 * 1e-3) / 1e6
    res["batched_over_plain"] = res["batched_mpts_s"] / res["plain_mpts_s"]
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {a.gpus} is not supported (the path has "
              "no multi-GPU code)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2507_21913_amd as F
    import workloads

    dev = torch.device("cuda:0")
    if a.only is not None:
        sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))  # the stored oracle samples
        # one secondary workload alone, on the plan the full run gives it (p = 20, leaf 32 and the
        # library's default near-field shape for the differentiation workload, unless --p/--leaf)
        if a.only == "curve":
            r = curve_extra(dev, max(2, a.steps // 2))
        elif a.only == "batched":
            r = batched_extra(dev, 20, 32, 3)
        else:
            r = fwd_bwd_extra(dev, a.p or 20, a.leaf or 32, {}, max(2, a.steps // 2))
        print(json.dumps({"only": a.only, "result": r}), flush=True)
        return
    w = workloads.uniform_1m(seed=1, n=a.n, p=a.p, leaf_size=a.leaf)
    x = torch.as_tensor(w.x, device=dev)
    y = torch.as_tensor(w.y, device=dev)
    q = torch.as_tensor(w.q[0], device=dev)

    tuned = None
    p_use, leaf_use = a.p, a.leaf
    shape = {}  # near-field launch shape (library default unless tuned)
    if a.p == 0:
        t0 = time.perf_counter()
        tuned = F.tune(x, y, q, w.impedance, tol=a.tol)
        tuned["tune_s"] = time.perf_counter() - t0
        p_use, leaf_use = tuned["p"], tuned["leaf_size"]
        shape = {"near_walk": tuned["near_walk"], "near_groups": tuned["near_groups"],
                 "m2l_fp32": tuned["m2l_fp32"], "m2l_form": tuned.get("m2l_form")}
    else:
        if a.leaf == 0:
            leaf_use = 40
        shape = {"near_walk": a.near_walk, "near_groups": a.near_groups}

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = F.HalfPlaneFMM(x, y, w.impedance, p=p_use, leaf_size=leaf_use, **shape)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info()
    out = torch.empty(w.n, dtype=torch.complex128, device=dev)
    for _ in range(a.warmup):
        plan(q, out=out)
    torch.cuda.synchronize()

    # timed region: K evals bracketed by events on the eval stream
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.steps):
        plan(q, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.steps
    # the same K evals again with per-phase HIP events on every stream the phases run on (the
    # events themselves cost ~5-10% here, so they stay out of the first timed region)
    plan.set_timing(True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(a.steps):
        plan(q, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms_instrumented = e0.elapsed_time(e1) / a.steps
    phases, nev = plan.phase_times()
    m2l_ms_sum, m2l_launches = plan.m2l_kernel_times()
    plan.set_timing(False)
    phase_avg = {k: v / max(1, nev) for k, v in phases.items()}

    if a.calibrate_copy:
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # accuracy against the stored oracle sample (direct sum at 256 targets x all sources)
    rel = None
    g = None
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    try:
        from golden_io import load
        g = load("uniform_1m") if a.n == (1 << 20) else None
        if g is not None:
            idx, ref = g
            got = out.cpu().numpy()[idx]
            rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    except Exception as ex:  # noqa: BLE001
        print(f"accuracy check skipped: {ex}", file=sys.stderr)

    # roofline of the dominant kernel, from algorithmic work per launch / measured launch time
    P1 = info["p"] + 1
    # k_m2l: the upper-source pairs, (p + 1)^2 complex FMA (8 flops) each; image pairs are k_m2l_img's
    m2l_flops = 8.0 * P1 * P1 * info["m2l_pairs"][0]
    # dominant kernel: the one with the most algorithmic work per evaluation (the near field runs
    # concurrently on its own stream, so phase durations overlap)
    near_flops = 27.0 * (info["p2p_pairs"][0] + info["p2p_pairs"][1])
    dom = "m2l" if m2l_flops >= near_flops else "near"
    if dom == "m2l" and m2l_launches > 0:
        # k_m2l runs as up to two launches per evaluation (deep levels on a second stream, coarse
        # levels on the eval stream), each bracketed by HIP events on its own stream
        per_eval = m2l_launches / max(1, nev)
        fl = m2l_flops / per_eval
        avg_ms = m2l_ms_sum / m2l_launches
        achieved = fl / (avg_ms * 1e-3) / 1e12
        traffic = M2L_TRAFFIC.get((eval_source_hash(), info["p"], leaf_use))
        roof = {"kernel": "k_m2l", "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": None if traffic is None else traffic / per_eval,
                "schedule": "concurrent: the launches share the GPU with the near field (the kernel alone: "
                            "roofline_alone)",
                "flops_per_launch": fl, "launches_per_eval": per_eval, "avg_launch_us": avg_ms * 1e3}
        if traffic is not None:
            roof["traffic_over_algorithmic"] = traffic / M2L_ALG_BYTES(info)
    else:
        # near field (k_near): 27 float64 flops per pair, counted from its compiled inner loop
        # (12 FMA incl. the table-assisted log, 2 add, 1 mul); image-source pairs counted alike
        pairs = info["p2p_pairs"][0] + info["p2p_pairs"][1]
        fl = 27.0 * pairs
        achieved = fl / (phase_avg["near"] * 1e-3) / 1e12
        roof = {"kernel": "k_near", "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                "flops_per_launch": fl}

    # the same evaluation with every kernel on one stream: each k_m2l launch's duration is its own
    # (the concurrent schedule above shares the CUs with the near field)
    alone = None
    roof_near = None
    if dom == "m2l":
        plan_s = F.HalfPlaneFMM(x, y, w.impedance, p=p_use, leaf_size=leaf_use, serial=True, **shape)
        for _ in range(2):
            plan_s(q, out=out)
        plan_s.set_timing(True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(a.steps):
            plan_s(q, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms_s = e0.elapsed_time(e1) / a.steps
        m2l_ms_s, n_s = plan_s.m2l_kernel_times()
        ph_s, nev_s = plan_s.phase_times()
        plan_s.set_timing(False)
        plan_s.close()
        # the near field alone (its phase on the one stream: k_near, the reaction pairs and the surface
        # sums), 27 flops per pair as in the dominant-kernel fallback below
        near_ms = ph_s["near"] / max(1, nev_s)
        near_fl = 27.0 * (info["p2p_pairs"][0] + info["p2p_pairs"][1])
        roof_near = {"kernel": "k_near (+ k_near_reaction, surface sums)", "bound": "alu",
                     "schedule": "every kernel on one stream (FMMHP_FLAG_SERIAL)",
                     "achieved": near_fl / (near_ms * 1e-3) / 1e12, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": near_fl / (near_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                     "phase_us": near_ms * 1e3, "flops": near_fl, "pairs": info["p2p_pairs"]}
        nt = NEAR_TRAFFIC.get((eval_source_hash(), info["p"], leaf_use))
        roof_near["traffic"] = nt
        roof_near["traffic_kernel"] = "k_near (bytes per launch)"
        if nt is not None:
            roof_near["traffic_over_algorithmic"] = nt / NEAR_ALG_BYTES(info)
        if n_s > 0:
            per_eval_s = n_s / max(1, a.steps)
            avg_s = m2l_ms_s / n_s
            ach_s = (m2l_flops / per_eval_s) / (avg_s * 1e-3) / 1e12
            alone = {"kernel": "k_m2l", "schedule": "every kernel on one stream (FMMHP_FLAG_SERIAL)",
                     "achieved": ach_s, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach_s / PEAK_FP64_TFLOPS, "avg_launch_us": avg_s * 1e3,
                     "launches_per_eval": per_eval_s, "ms_per_step_serial": ms_s}

    res = {
        "metric": "Mpts/s FMM eval at 1M pts, rel-l2 1e-10 vs direct; fwd+bwd and batched vs plain",
        "value": w.n / (ms * 1e-3) / 1e6,
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "uniform_1m: N=1,048,576 uniform in [0,1]x[1e-3,1.001], charges U[-1,1], "
                               "impedance 1.0, sources=targets, 1 charge vector",
                   "n": w.n, "p": info["p"], "leaf_size": leaf_use, "impedance": 1.0,
                   "tolerance": a.tol if tuned else None,
                   "near_walk": info["near_walk"], "near_groups": info["near_groups"]},
        "roofline": roof,
    }
    if alone is not None:
        res["roofline_alone"] = alone
        res["roofline_near_alone"] = roof_near
    if tuned:
        res["autotune"] = tuned
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, a.cpu_sample)
    if not a.quiet_extra:
        res["rel_l2_vs_oracle_sample"] = rel
        if not a.no_p30 and not (p_use == 30 and leaf_use == 40):
            plan30 = F.HalfPlaneFMM(x, y, w.impedance, p=30, leaf_size=40)
            for _ in range(2):
                plan30(q, out=out)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(10):
                plan30(q, out=out)
            e1.record()
            torch.cuda.synchronize()
            ms30 = e0.elapsed_time(e1) / 10
            rel30 = None
            if g is not None:
                rel30 = float(np.linalg.norm(out.cpu().numpy()[g[0]] - g[1]) / np.linalg.norm(g[1]))
            res["p30_leaf40"] = {"mpts_s": w.n / (ms30 * 1e-3) / 1e6, "ms_per_step": ms30,
                                 "rel_l2_vs_oracle_sample": rel30}
            plan30.close()
        # the same evaluation with the upper-source M2L on the FP32 matrix cores
        plan32 = F.HalfPlaneFMM(x, y, w.impedance, p=p_use, leaf_size=leaf_use, m2l_fp32=True,
                                **{k: v for k, v in shape.items() if k != "m2l_fp32"})
        for _ in range(2):
            plan32(q, out=out)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(a.steps):
            plan32(q, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms32 = e0.elapsed_time(e1) / a.steps
        plan32.set_timing(True)
        for _ in range(5):
            plan32(q, out=out)
        ph32, nev32 = plan32.phase_times()
        rel32 = None
        if g is not None:
            rel32 = float(np.linalg.norm(out.cpu().numpy()[g[0]] - g[1]) / np.linalg.norm(g[1]))
        plan32.close()
        # the matrix-core M2L alone (serial plan): its launches' time against the FP32 matrix peak
        plan32s = F.HalfPlaneFMM(x, y, w.impedance, p=p_use, leaf_size=leaf_use, m2l_fp32=True, serial=True)
        for _ in range(2):
            plan32s(q, out=out)
        plan32s.set_timing(True)
        for _ in range(10):
            plan32s(q, out=out)
        torch.cuda.synchronize()
        k32_ms, k32_n = plan32s.m2l_kernel_times()
        plan32s.close()
        k32_eval_ms = k32_ms / 10.0
        res["m2l_fp32"] = {"mpts_s": w.n / (ms32 * 1e-3) / 1e6, "ms_per_step": ms32, "over_fp64": ms / ms32,
                           "m2l_phase_ms": ph32["m2l"] / max(1, nev32), "rel_l2_vs_oracle_sample": rel32,
                           "kernel_alone_us_per_eval": k32_eval_ms * 1e3,
                           "kernel_alone_frac_fp32_matrix_peak": m2l_flops / (k32_eval_ms * 1e-3) / 1e12
                           / PEAK_FP32_MATRIX_TFLOPS,
                           "kernel_alone_note": "algorithmic flops 8 (p+1)^2 per upper V pair over the summed "
                                                "duration of the FP32 row conversion and matrix-core M2L launches"}
        nb = max(1, a.steps // 4)
        res["fwd_bwd"] = fwd_bwd_extra(dev, p_use, leaf_use, shape, max(2, a.steps // 2))
        # the double-layer potential of the same densities with seeded unit normals, same plan
        nxh, nyh = workloads.source_normals(w.n, seed=7)
        nxd, nyd = (torch.as_tensor(v, device=dev) for v in (nxh, nyh))
        for _ in range(2):
            dl = plan.double_layer(q, nxd, nyd)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(nb):
            dl = plan.double_layer(q, nxd, nyd)
        e1.record()
        torch.cuda.synchronize()
        ms_dl = e0.elapsed_time(e1) / nb
        rel_dl = None
        if g is not None:
            from golden_io import load_dlp
            gd = load_dlp("uniform_1m")
            if gd is not None:
                rel_dl = float(np.linalg.norm(dl.cpu().numpy()[gd[0]] - gd[1]) / np.linalg.norm(gd[1]))
        res["double_layer"] = {"mpts_s": w.n / (ms_dl * 1e-3) / 1e6, "ms_per_step": ms_dl,
                               "normals": "workloads.source_normals(N, seed=7)",
                               "rel_l2_vs_oracle_sample": rel_dl}
        del dl
        res["example2"] = example2_extra(dev)
        res["curve_4m"] = curve_extra(dev, max(2, a.steps // 2))
        if not a.no_batched:
            plan.close()
            del out
            torch.cuda.empty_cache()
            res["batched"] = batched_extra(dev, 20, 32, 3)
        res["plan_ms"] = plan_ms
        res["plan_plus_eval_mpts_s"] = w.n / ((plan_ms + ms) * 1e-3) / 1e6
        res["phase_ms"] = {k: round(v, 5) for k, v in phase_avg.items()}
        res["ms_per_step_instrumented"] = ms_instrumented
        res["tree"] = {"nbox": info["nbox"], "nleaf": info["nleaf"], "depth": info["depth"],
                       "list_len": info["list_len"], "p2p_pairs": info["p2p_pairs"],
                       "m2l_pairs": info["m2l_pairs"], "device_bytes": info["device_bytes"]}
    print(json.dumps(res), flush=True)
    if a.quiet_extra or a.no_batched:
        plan.close()


if __name__ == "__main__":
    main()
