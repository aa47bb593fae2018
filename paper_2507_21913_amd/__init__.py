"""Half-plane Robin Laplace FMM on AMD MI355X (gfx950): Python binding.

Argument marshalling over the C-ABI library ``libfmmhp.so`` (declared in
``include/fmmhp.h``); every step of the computation runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream only.  There is
no CPU fallback: the functions raise if the library is missing or a tensor is
not on a GPU.

Function names mirror the C entry points (``fmmhp_plan_create``, ``fmmhp_eval``,
...); ``HalfPlaneFMM`` wraps a plan for convenience.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmmhp.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "fmmhp.h")

STATUS = {0: "FMMHP_OK", 1: "FMMHP_EINVAL", 2: "FMMHP_EDOMAIN", 3: "FMMHP_ENOMEM",
          4: "FMMHP_EHIP", 5: "FMMHP_ESTATE", 6: "FMMHP_EUNSUPPORTED"}
MAX_P = 40
FLAG_GRAPH = 1   # fmmhp_opts.flags: record evaluations into a HIP graph and replay them
FLAG_M2L_FP32 = 2  # fmmhp_opts.flags: upper-source M2L on the FP32 matrix cores (~1e-7 relative)
FLAG_DIRICHLET = 4  # fmmhp_opts.flags: Dirichlet half-plane kernel (eq. (ddd1.2), image term +)
FLAG_NEUMANN = 8    # fmmhp_opts.flags: Neumann half-plane kernel (eq. (ddd1.2), image term -)
FLAG_SERIAL = 16    # fmmhp_opts.flags: every kernel on the eval stream (profiling aid)
FLAG_M2L_VECTOR = 32  # fmmhp_opts.flags: FP64 M2L on the vector ALUs (the default form)
FLAG_M2L_MFMA = 64    # fmmhp_opts.flags: FP64 M2L on the matrix cores


def _m2l_flag(form):
    """fmmhp_opts.flags bits of an M2L form: None (the library default), "vector" or "mfma"."""
    if form is None:
        return 0
    if form == "vector":
        return FLAG_M2L_VECTOR
    if form == "mfma":
        return FLAG_M2L_MFMA
    raise ValueError("m2l_form must be None, 'vector' or 'mfma'")
_BC_FLAGS = {"robin": 0, "dirichlet": FLAG_DIRICHLET, "neumann": FLAG_NEUMANN}


def _bc_flag(bc: str) -> int:
    if bc not in _BC_FLAGS:
        raise ValueError(f"bc must be one of {sorted(_BC_FLAGS)}")
    return _BC_FLAGS[bc]


class FMMHPError(RuntimeError):
    def __init__(self, func: str, status: int, message: str):
        super().__init__(f"{func}: {STATUS.get(status, status)}: {message}")
        self.status = status
        self.func = func


class Opts(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("leaf_size", ctypes.c_int),
                ("max_level", ctypes.c_int), ("flags", ctypes.c_uint),
                ("near_walk", ctypes.c_int), ("near_groups", ctypes.c_int)]


class PlanStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("p", ctypes.c_int), ("leaf_size", ctypes.c_int),
                ("max_level", ctypes.c_int), ("depth", ctypes.c_int),
                ("nbox", ctypes.c_int64), ("nleaf", ctypes.c_int64),
                ("list_len", ctypes.c_int64 * 4), ("x_lo", ctypes.c_double),
                ("S", ctypes.c_double), ("scale", ctypes.c_double),
                ("lambda_re", ctypes.c_double), ("lambda_im", ctypes.c_double),
                ("real_impedance", ctypes.c_int), ("device_bytes", ctypes.c_int64),
                ("p2p_pairs", ctypes.c_int64 * 2), ("m2l_pairs", ctypes.c_int64 * 2),
                ("n_inst", ctypes.c_int32), ("near_walk", ctypes.c_int32),
                ("near_groups", ctypes.c_int32), ("n_sources", ctypes.c_int64)]


PHASES = ("p2m", "m2m", "m2l", "p2l", "l2l", "surface", "leaf", "near")


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double
_INT = ctypes.c_int

_SIGNATURES = {
    "fmmhp_plan_create": [_I64, _P, _P, _P, _P, _D, _D, ctypes.POINTER(Opts), _P,
                          ctypes.POINTER(_P)],
    "fmmhp_batch_plan_create": [_INT, _P, _P, _P, _P, ctypes.POINTER(Opts), _P, ctypes.POINTER(_P)],
    "fmmhp_plan_create_targets": [_I64, _P, _P, _I64, _P, _P, _D, _D, ctypes.POINTER(Opts), _P,
                                  ctypes.POINTER(_P)],
    "fmmhp_eval": [_P, _INT, _P, _P, _P],
    "fmmhp_eval_noalloc": [_P, _INT, _P, _P, _P],
    "fmmhp_eval_complex": [_P, _INT, _P, _P, _P],
    "fmmhp_backward": [_P, _P, _P, _P, _P, _P, _P, _P],
    "fmmhp_backward_device": [_P, _P, _P, _P, _P, _P, _P, _P],
    "fmmhp_eval_field": [_P, _P, _P, _P, _P, _P],
    "fmmhp_eval_double_layer": [_P, _INT, _P, _INT, _P, _P, _P, _P],
    "fmmhp_eval_normal_derivative": [_P, _P, _P, _P, _P, _P],
    "fmmhp_plan_info": [_P, ctypes.POINTER(PlanStats)],
    "fmmhp_plan_export_tree": [_P] + [_P] * 18,
    "fmmhp_plan_destroy": [_P],
    "fmmhp_direct_eval": [_I64, _P, _P, _INT, _P, _I64, _P, _P, _D, _D, _P, _P],
    "fmmhp_reaction_integrals": [_I64, _P, _P, _INT, _D, _D, _P, _P],
    "fmmhp_plan_set_timing": [_P, _INT],
    "fmmhp_plan_phase_times": [_P, ctypes.POINTER(_D), ctypes.POINTER(_I64)],
    "fmmhp_plan_m2l_kernel_times": [_P, ctypes.POINTER(_D), ctypes.POINTER(_I64)],
    "fmmhp_tune": [_I64, _P, _P, _P, _D, _D, _D, _INT, _P, _INT, _INT, ctypes.POINTER(Opts),
                   ctypes.POINTER(_D), ctypes.POINTER(_D), _P],
    "fmmhp_status_string": [_INT],
    "fmmhp_last_error_message": [],
}


def lib() -> ctypes.CDLL:
    """Load libfmmhp.so (built in-tree by ``python -m paper_2507_21913_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2507_21913_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name in ("fmmhp_status_string",
                                                    "fmmhp_last_error_message") else ctypes.c_int
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions include/fmmhp.h declares."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fmmhp_\w+)\s*\(", txt)))


def _check(func: str, status: int):
    if status != 0:
        msg = lib().fmmhp_last_error_message().decode(errors="replace")
        raise FMMHPError(func, status, msg)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor (no CPU path exists)")
    return t.to(torch.float64).contiguous()


# --- C entry points, same names --------------------------------------------------------------

def fmmhp_plan_create(n, x_ptr, y_ptr, img_x_ptr, img_y_ptr, lambda_re, lambda_im, opts, stream):
    h = _P()
    st = lib().fmmhp_plan_create(n, x_ptr, y_ptr, img_x_ptr, img_y_ptr, lambda_re, lambda_im,
                                 ctypes.byref(opts) if opts is not None else None, stream,
                                 ctypes.byref(h))
    _check("fmmhp_plan_create", st)
    return h


def fmmhp_plan_create_targets(n_src, xs_ptr, ys_ptr, n_tgt, xt_ptr, yt_ptr, lambda_re, lambda_im, opts,
                              stream):
    h = _P()
    st = lib().fmmhp_plan_create_targets(n_src, xs_ptr, ys_ptr, n_tgt, xt_ptr, yt_ptr, lambda_re, lambda_im,
                                         ctypes.byref(opts) if opts is not None else None, stream,
                                         ctypes.byref(h))
    _check("fmmhp_plan_create_targets", st)
    return h


def fmmhp_batch_plan_create(n_inst, offsets, x_ptr, y_ptr, lambdas, opts, stream):
    """offsets: sequence of n_inst + 1 ints; lambdas: sequence of n_inst complex impedances."""
    h = _P()
    off = (_I64 * (n_inst + 1))(*[int(v) for v in offsets])
    lam = (_D * (2 * n_inst))(*[v for z in lambdas for v in (complex(z).real, complex(z).imag)])
    st = lib().fmmhp_batch_plan_create(n_inst, ctypes.cast(off, _P), x_ptr, y_ptr, ctypes.cast(lam, _P),
                                       ctypes.byref(opts) if opts is not None else None, stream,
                                       ctypes.byref(h))
    _check("fmmhp_batch_plan_create", st)
    return h


def fmmhp_eval(plan, n_vec, q_ptr, phi_ptr, stream):
    _check("fmmhp_eval", lib().fmmhp_eval(plan, n_vec, q_ptr, phi_ptr, stream))


def fmmhp_eval_noalloc(plan, n_vec, q_ptr, phi_ptr, stream):
    """fmmhp_eval with its workspace in the library's static device scratch (no allocation)."""
    _check("fmmhp_eval_noalloc", lib().fmmhp_eval_noalloc(plan, n_vec, q_ptr, phi_ptr, stream))


NOALLOC_SCRATCH_BYTES = 128 << 20  # FMMHP_NOALLOC_SCRATCH_BYTES


def fmmhp_backward(plan, q_ptr, grad_phi_ptr, grad_q_ptr, grad_x_ptr, grad_y_ptr, want_lambda,
                   stream, n_inst=1):
    """Returns [(dl/dRe Z_k, dl/dIm Z_k)] per instance when want_lambda, else None."""
    gl = (_D * (2 * n_inst))() if want_lambda else None
    _check("fmmhp_backward", lib().fmmhp_backward(plan, q_ptr, grad_phi_ptr, grad_q_ptr, grad_x_ptr,
                                                  grad_y_ptr, gl, stream))
    return [(gl[2 * k], gl[2 * k + 1]) for k in range(n_inst)] if want_lambda else None


def fmmhp_eval_complex(plan, n_vec, q_ptr, phi_ptr, stream):
    _check("fmmhp_eval_complex", lib().fmmhp_eval_complex(plan, n_vec, q_ptr, phi_ptr, stream))


def fmmhp_plan_info(plan) -> dict:
    s = PlanStats()
    _check("fmmhp_plan_info", lib().fmmhp_plan_info(plan, ctypes.byref(s)))
    d = {k: getattr(s, k) for k, _ in PlanStats._fields_}
    for k in ("list_len", "p2p_pairs", "m2l_pairs"):
        d[k] = list(getattr(s, k))
    return d


def fmmhp_plan_set_timing(plan, enable: bool):
    _check("fmmhp_plan_set_timing", lib().fmmhp_plan_set_timing(plan, int(bool(enable))))


def fmmhp_plan_phase_times(plan) -> tuple[dict, int]:
    ms = (_D * len(PHASES))()
    n = _I64()
    _check("fmmhp_plan_phase_times", lib().fmmhp_plan_phase_times(plan, ms, ctypes.byref(n)))
    return {k: ms[i] for i, k in enumerate(PHASES)}, n.value


def fmmhp_plan_m2l_kernel_times(plan) -> tuple[float, int]:
    ms = _D()
    n = _I64()
    _check("fmmhp_plan_m2l_kernel_times", lib().fmmhp_plan_m2l_kernel_times(plan, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def fmmhp_plan_export_tree(plan) -> dict:
    info = fmmhp_plan_info(plan)
    nb, n = info["nbox"], info["n"]
    out = {k: np.zeros(nb, np.int32) for k in
           ("level", "bx", "by", "first", "count", "parent", "leaf", "child_first", "nchild")}
    out["perm"] = np.zeros(n, np.int64)
    args = [out[k] for k in ("level", "bx", "by", "first", "count", "parent", "leaf",
                             "child_first", "nchild", "perm")]
    for j, name in enumerate("UVWX"):
        out[name + "_off"] = np.zeros(nb + 1, np.int64)
        out[name + "_ent"] = np.zeros(max(1, info["list_len"][j]), np.int32)
        args += [out[name + "_off"], out[name + "_ent"]]
    _check("fmmhp_plan_export_tree",
           lib().fmmhp_plan_export_tree(plan, *[a.ctypes.data_as(_P) for a in args]))
    for j, name in enumerate("UVWX"):
        out[name + "_ent"] = out[name + "_ent"][: info["list_len"][j]]
    out["nbox"] = nb
    out["x_lo"], out["S"], out["scale"] = info["x_lo"], info["S"], info["scale"]
    return out


def fmmhp_plan_destroy(plan):
    _check("fmmhp_plan_destroy", lib().fmmhp_plan_destroy(plan))


def fmmhp_direct_eval(n_src, sx, sy, n_vec, q, n_tgt, tx, ty, lambda_re, lambda_im, phi, stream):
    _check("fmmhp_direct_eval", lib().fmmhp_direct_eval(n_src, sx, sy, n_vec, q, n_tgt, tx, ty,
                                                        lambda_re, lambda_im, phi, stream))


def fmmhp_reaction_integrals(m, x, y, nmax, lambda_re, lambda_im, out, stream):
    _check("fmmhp_reaction_integrals",
           lib().fmmhp_reaction_integrals(m, x, y, nmax, lambda_re, lambda_im, out, stream))


def fmmhp_tune(n, x_ptr, y_ptr, q_ptr, lambda_re, lambda_im, tol, n_vec, leaf_sizes, sample,
               stream):
    best = Opts()
    err = _D()
    ms = _D()
    if leaf_sizes:
        arr = (_INT * len(leaf_sizes))(*leaf_sizes)
        la, nl = ctypes.cast(arr, _P), len(leaf_sizes)
    else:
        la, nl = None, 0
    _check("fmmhp_tune", lib().fmmhp_tune(n, x_ptr, y_ptr, q_ptr, lambda_re, lambda_im, tol, n_vec,
                                          la, nl, sample, ctypes.byref(best), ctypes.byref(err),
                                          ctypes.byref(ms), stream))
    return {"p": best.p, "leaf_size": best.leaf_size, "near_walk": best.near_walk,
            "near_groups": best.near_groups, "m2l_fp32": bool(best.flags & FLAG_M2L_FP32),
            "m2l_form": ("vector" if best.flags & FLAG_M2L_VECTOR else
                         "mfma" if best.flags & FLAG_M2L_MFMA else None),
            "rel_l2": err.value, "eval_ms": ms.value}


# --- autotuner cache --------------------------------------------------------------------------
# The tuner's choices persist in a JSON file keyed by the GPU, the point count (power-of-two bucket),
# the impedance class, the tolerance, the number of vectors and a hash of the library sources, so a
# second run on the same kind of problem skips the search.  Default file: tune_cache.json beside
# this module; FMMHP_TUNE_CACHE names another (an empty value disables the cache).
TUNE_CACHE_PATH = os.path.join(_HERE, "tune_cache.json")


def _source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(_HERE, "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def tune_cache_key(n, impedance, tol, n_vec, device=None) -> str:
    import math
    z = complex(impedance)
    name = torch.cuda.get_device_name(device)
    nb = int(round(math.log2(max(1, int(n)))))
    zc = f"{'complex' if z.imag != 0 else 'real'}:1e{int(math.floor(math.log10(abs(z)) * 2)) / 2:g}"
    return f"{name}|n~2^{nb}|Z {zc}|tol {tol:g}|nvec {int(n_vec)}|src {_source_hash()}"


def _cache_path():
    p = os.environ.get("FMMHP_TUNE_CACHE")
    if p is None:
        return TUNE_CACHE_PATH
    return p or None


def _cache_load(path) -> dict:
    import json
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _cache_store(path, key, value):
    import json
    d = _cache_load(path)
    d[key] = value
    tmp = f"{path}.{os.getpid()}.tmp"
    try:
        with open(tmp, "w") as fh:
            json.dump(d, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune(x, y, q, impedance, tol=1e-10, n_vec=1, leaf_sizes=None, sample=0, use_cache=True) -> dict:
    """Pick (p, leaf_size) for these points and impedance at a target rel-l2 error, the near-field
    launch shape (near_walk, near_groups) and the M2L form (m2l_form: None for the default,
    "vector" or "mfma"; m2l_fp32) by timing the chosen plan.
    With use_cache the choice is read from (and written to) the tuner's JSON cache; "cached" in the
    result says which."""
    x = _dev_f64(x, "x")
    y = _dev_f64(y, "y")
    q = _dev_f64(q, "q")
    lr, li = _split_impedance(impedance)
    path = _cache_path() if use_cache and not leaf_sizes and not sample else None
    key = tune_cache_key(x.shape[0], complex(lr, li), tol, n_vec, x.device) if path else None
    if path:
        hit = _cache_load(path).get(key)
        if hit is not None:
            return dict(hit, cached=True, cache_key=key)
    with torch.cuda.device(x.device):
        r = fmmhp_tune(x.shape[0], x.data_ptr(), y.data_ptr(), q.data_ptr(), lr, li, tol, n_vec,
                       leaf_sizes, sample, _stream())
    if path:
        _cache_store(path, key, r)
    return dict(r, cached=False, cache_key=key)


# --- tensor-level helpers --------------------------------------------------------------------

def _split_impedance(lam):
    lam = complex(lam)
    return lam.real, lam.imag


class HalfPlaneFMM:
    """A plan over fixed points; call it with charges to get the complex potential.

    x, y        GPU tensors [N] (float64), y > 0
    impedance   Z_eps (complex or real), Re > 0, Im >= 0
    p, leaf_size, max_level   see fmmhp_opts in include/fmmhp.h
    pass_images pass the image arrays (x, -y) explicitly to the library
    graph       record each evaluation into a HIP graph and replay it (needs a non-default
                stream: run under ``torch.cuda.stream(...)``)
    m2l_fp32    run the upper-source M2L on the FP32 matrix cores (relative error ~1e-7)
    near_walk, near_groups   near-field launch shape (0: default; see fmmhp_opts)
    bc          "robin" (the impedance condition), "dirichlet" or "neumann" (eq. (ddd1.2); the
                impedance is then ignored)
    serial      every kernel on the eval stream, one after another (profiling aid; slower)
    m2l_form    FP64 M2L form: None (the default: vector ALUs), "vector" or "mfma" (the same sums
                in another order)
    """

    def __init__(self, x, y, impedance, p=20, leaf_size=40, max_level=0, pass_images=False,
                 graph=False, m2l_fp32=False, near_walk=0, near_groups=0, bc="robin", serial=False,
                 m2l_form=None):
        x = _dev_f64(x, "x")
        y = _dev_f64(y, "y")
        self.n = int(x.shape[0])
        self.device = x.device
        self._x, self._y = x, y
        lr, li = _split_impedance(impedance)
        opts = Opts(int(p), int(leaf_size), int(max_level),
                    (FLAG_GRAPH if graph else 0) | (FLAG_M2L_FP32 if m2l_fp32 else 0) | _bc_flag(bc)
                    | (FLAG_SERIAL if serial else 0) | _m2l_flag(m2l_form),
                    int(near_walk), int(near_groups))
        with torch.cuda.device(self.device):
            if pass_images:
                ix, iy = x.clone(), -y
                self._plan = fmmhp_plan_create(self.n, x.data_ptr(), y.data_ptr(), ix.data_ptr(),
                                               iy.data_ptr(), lr, li, opts, _stream())
            else:
                self._plan = fmmhp_plan_create(self.n, x.data_ptr(), y.data_ptr(), None, None,
                                               lr, li, opts, _stream())
        self.impedance = complex(lr, li)
        self.n_inst = 1
        self.n_out = self.n
        self._graph = bool(graph)

    @classmethod
    def with_targets(cls, xs, ys, xt, yt, impedance, p=20, leaf_size=40, max_level=0, graph=False,
                     m2l_fp32=False, near_walk=0, near_groups=0, bc="robin"):
        """A plan whose potential is evaluated at separate targets (xt, yt), y >= 0: calling it
        with charges q [N_src] (or [n_vec, N_src]) returns phi at the N_tgt targets."""
        self = cls.__new__(cls)
        xs = _dev_f64(xs, "xs")
        ys = _dev_f64(ys, "ys")
        xt = _dev_f64(xt, "xt")
        yt = _dev_f64(yt, "yt")
        self.n = int(xs.shape[0])
        self.n_out = int(xt.shape[0])
        self.device = xs.device
        self._x, self._y = xs, ys
        lr, li = _split_impedance(impedance)
        opts = Opts(int(p), int(leaf_size), int(max_level),
                    (FLAG_GRAPH if graph else 0) | (FLAG_M2L_FP32 if m2l_fp32 else 0) | _bc_flag(bc),
                    int(near_walk), int(near_groups))
        with torch.cuda.device(self.device):
            self._plan = fmmhp_plan_create_targets(self.n, xs.data_ptr(), ys.data_ptr(), self.n_out,
                                                   xt.data_ptr(), yt.data_ptr(), lr, li, opts, _stream())
        self.impedance = complex(lr, li)
        self.n_inst = 1
        self._graph = bool(graph)
        return self

    @classmethod
    def batched(cls, x, y, offsets, impedances, p=20, leaf_size=40, max_level=0, graph=False,
                m2l_fp32=False, near_walk=0, near_groups=0, bc="robin", m2l_form=None, serial=False):
        """A forest plan over n_inst independent instances: points offsets[k]..offsets[k+1]-1 of
        (x, y) form instance k with impedance impedances[k].  Evaluation takes charges for all
        points (instance after instance) and runs every instance in the same launches."""
        self = cls.__new__(cls)
        x = _dev_f64(x, "x")
        y = _dev_f64(y, "y")
        self.n = int(x.shape[0])
        self.device = x.device
        self._x, self._y = x, y
        offsets = [int(v) for v in offsets]
        if len(offsets) < 2 or offsets[-1] != self.n:
            raise ValueError("offsets must have n_inst + 1 entries ending at the point count")
        self.n_inst = len(offsets) - 1
        self.offsets = offsets
        imps = [complex(z) for z in impedances]
        if len(imps) != self.n_inst:
            raise ValueError("one impedance per instance")
        opts = Opts(int(p), int(leaf_size), int(max_level),
                    (FLAG_GRAPH if graph else 0) | (FLAG_M2L_FP32 if m2l_fp32 else 0) | _bc_flag(bc)
                    | _m2l_flag(m2l_form) | (FLAG_SERIAL if serial else 0),
                    int(near_walk), int(near_groups))
        with torch.cuda.device(self.device):
            self._plan = fmmhp_batch_plan_create(self.n_inst, offsets, x.data_ptr(), y.data_ptr(), imps,
                                                 opts, _stream())
        self.impedance = imps[0] if self.n_inst == 1 else imps
        self.n_out = self.n
        self._graph = bool(graph)
        return self

    def info(self) -> dict:
        return fmmhp_plan_info(self._plan)

    def export_tree(self) -> dict:
        return fmmhp_plan_export_tree(self._plan)

    def set_timing(self, enable: bool):
        fmmhp_plan_set_timing(self._plan, enable)

    def phase_times(self) -> tuple[dict, int]:
        """(ms per phase summed since set_timing(True), number of vectors evaluated)."""
        return fmmhp_plan_phase_times(self._plan)

    def m2l_kernel_times(self) -> tuple[float, int]:
        """(summed ms of the upper-source M2L kernel's launches since set_timing(True), launches)."""
        return fmmhp_plan_m2l_kernel_times(self._plan)

    def __call__(self, q: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """phi = A q.  q: [N] or [n_vec, N], real or complex.  Returns complex128 [n_out] or
        [n_vec, n_out] (n_out = N unless the plan has separate targets)."""
        if not isinstance(q, torch.Tensor) or not q.is_cuda:
            raise TypeError("q must be a GPU tensor (no CPU path exists)")
        squeeze = q.dim() == 1
        q2 = q.reshape(1, -1) if squeeze else q
        if q2.shape[-1] != self.n:
            raise ValueError(f"q has {q2.shape[-1]} points, plan has {self.n}")
        nv = q2.shape[0]
        if q2.is_complex():
            parts = torch.view_as_real(q2.to(torch.complex128).contiguous())
        else:
            parts = q2.to(torch.float64).contiguous()
        direct_out = (out is not None and out.dtype == torch.complex128 and out.is_contiguous()
                      and out.device == self.device and out.numel() == nv * self.n_out)
        if getattr(self, "_graph", False) and not direct_out:
            # the recorded graph is keyed on the charge and output pointers: a fresh output tensor per
            # call would re-record it every time
            raise ValueError("a plan built with graph=True needs out= (a contiguous complex128 tensor with "
                             f"{nv * self.n_out} elements on {self.device}) so that replays reuse one graph")
        if direct_out:
            raw = torch.view_as_real(out)
        else:
            raw = torch.empty((nv, self.n_out, 2), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            if q2.is_complex():
                fmmhp_eval_complex(self._plan, nv, parts.data_ptr(), raw.data_ptr(), _stream())
            else:
                fmmhp_eval(self._plan, nv, parts.data_ptr(), raw.data_ptr(), _stream())
        if direct_out:
            return out
        phi = torch.view_as_complex(raw)
        if out is not None:
            out.copy_(phi.reshape(out.shape))
            return out
        return phi[0] if squeeze else phi

    def field(self, q: torch.Tensor):
        """(phi, d phi/dx, d phi/dy) at the targets for one real charge vector q [N]: three
        complex128 tensors [n_out]."""
        if not isinstance(q, torch.Tensor) or not q.is_cuda or q.is_complex():
            raise TypeError("q must be a real GPU tensor")
        if q.numel() != self.n:
            raise ValueError(f"q has {q.numel()} points, plan has {self.n}")
        qd = q.reshape(-1).to(torch.float64).contiguous()
        raw = torch.empty((3, self.n_out, 2), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check("fmmhp_eval_field", lib().fmmhp_eval_field(self._plan, qd.data_ptr(), raw[0].data_ptr(),
                                                               raw[1].data_ptr(), raw[2].data_ptr(), _stream()))
        c = torch.view_as_complex(raw)
        return c[0], c[1], c[2]

    def normal_derivative(self, q: torch.Tensor, nx: torch.Tensor, ny: torch.Tensor) -> torch.Tensor:
        """n . grad phi at the targets for one real charge vector q [N] and target normals nx, ny
        [n_out]: complex128 [n_out]."""
        for name, t in (("q", q), ("nx", nx), ("ny", ny)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.is_complex():
                raise TypeError(f"{name} must be a real GPU tensor")
        if q.numel() != self.n:
            raise ValueError(f"q has {q.numel()} points, plan has {self.n}")
        if nx.numel() != self.n_out or ny.numel() != self.n_out:
            raise ValueError(f"nx, ny must have {self.n_out} entries (one per target)")
        qd = q.reshape(-1).to(torch.float64).contiguous()
        nxd = nx.reshape(-1).to(torch.float64).contiguous()
        nyd = ny.reshape(-1).to(torch.float64).contiguous()
        raw = torch.empty((self.n_out, 2), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check("fmmhp_eval_normal_derivative",
                   lib().fmmhp_eval_normal_derivative(self._plan, qd.data_ptr(), nxd.data_ptr(), nyd.data_ptr(),
                                                      raw.data_ptr(), _stream()))
        return torch.view_as_complex(raw)

    def double_layer(self, mu: torch.Tensor, nx: torch.Tensor, ny: torch.Tensor) -> torch.Tensor:
        """Double-layer potential sum_j mu_j n_j . grad_{r_j} G(r_i, r_j) at the targets for dipole
        densities mu [N] or [n_vec, N] (real or complex) and source normals nx, ny [N].  Returns
        complex128 [n_out] or [n_vec, n_out]."""
        for name, t in (("mu", mu), ("nx", nx), ("ny", ny)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda:
                raise TypeError(f"{name} must be a GPU tensor (no CPU path exists)")
        if nx.is_complex() or ny.is_complex() or nx.numel() != self.n or ny.numel() != self.n:
            raise ValueError(f"nx, ny must be real with {self.n} entries")
        squeeze = mu.dim() == 1
        m2 = mu.reshape(1, -1) if squeeze else mu
        if m2.shape[-1] != self.n:
            raise ValueError(f"mu has {m2.shape[-1]} points, plan has {self.n}")
        nv = m2.shape[0]
        cpx = m2.is_complex()
        parts = (torch.view_as_real(m2.to(torch.complex128).contiguous()) if cpx
                 else m2.to(torch.float64).contiguous())
        nxd = nx.reshape(-1).to(torch.float64).contiguous()
        nyd = ny.reshape(-1).to(torch.float64).contiguous()
        raw = torch.empty((nv, self.n_out, 2), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check("fmmhp_eval_double_layer",
                   lib().fmmhp_eval_double_layer(self._plan, nv, parts.data_ptr(), int(cpx), nxd.data_ptr(),
                                                 nyd.data_ptr(), raw.data_ptr(), _stream()))
        phi = torch.view_as_complex(raw)
        return phi[0] if squeeze else phi

    def backward(self, q: torch.Tensor, grad_phi: torch.Tensor, want_q=True, want_x=True,
                 want_y=True, want_lambda=True, lambda_on_device=False) -> dict:
        """Gradients of a real loss l given g = dl/dRe phi + i dl/dIm phi (complex [N]) for real
        charges q [N]: {"q", "x", "y": float64 [N], "lambda": complex dl/dRe Z + i dl/dIm Z}.
        With lambda_on_device the impedance gradient stays on the GPU (fmmhp_backward_device, no
        host synchronisation): "lambda" is then a float64 tensor [n_inst, 2] of (dl/dRe Z, dl/dIm Z)."""
        if not isinstance(q, torch.Tensor) or not q.is_cuda or q.is_complex():
            raise TypeError("q must be a real GPU tensor")
        if q.numel() != self.n or grad_phi.numel() != self.n:
            raise ValueError("q and grad_phi must have one entry per point")
        qd = q.reshape(-1).to(torch.float64).contiguous()
        gr = torch.view_as_real(grad_phi.reshape(-1).to(torch.complex128).contiguous())
        out = {}
        ptr = {}
        for k, want in (("q", want_q), ("x", want_x), ("y", want_y)):
            if want:
                out[k] = torch.empty(self.n, dtype=torch.float64, device=self.device)
                ptr[k] = out[k].data_ptr()
            else:
                ptr[k] = None
        if want_lambda and lambda_on_device:
            dl = torch.empty((self.n_inst, 2), dtype=torch.float64, device=self.device)
            with torch.cuda.device(self.device):
                _check("fmmhp_backward_device",
                       lib().fmmhp_backward_device(self._plan, qd.data_ptr(), gr.data_ptr(), ptr["q"], ptr["x"],
                                                   ptr["y"], dl.data_ptr(), _stream()))
            out["lambda"] = dl
            return out
        with torch.cuda.device(self.device):
            gl = fmmhp_backward(self._plan, qd.data_ptr(), gr.data_ptr(), ptr["q"], ptr["x"],
                                ptr["y"], bool(want_lambda), _stream(), self.n_inst)
        if want_lambda:
            lam = [complex(a, b) for a, b in gl]
            out["lambda"] = lam[0] if self.n_inst == 1 else lam
        return out

    def close(self):
        if getattr(self, "_plan", None):
            fmmhp_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# potential(): the last plan per device, reused while the same point tensors (unchanged in place:
# torch's version counter), impedance and options come back.  The cached plan holds the point
# tensors, so their memory cannot be reused by other tensors while it is cached; a replaced plan
# closes once no autograd context holds it any more.
_POT_PLANS: dict = {}


def _potential_plan(x, y, lam, p, leaf_size, reuse):
    key = (x.data_ptr(), y.data_ptr(), x._version, y._version, tuple(x.shape), lam, p, leaf_size)
    hit = _POT_PLANS.get(x.device) if reuse else None
    if hit is not None and hit[0] == key:
        return hit[1]
    plan = HalfPlaneFMM(x, y, lam, p=p, leaf_size=leaf_size)
    if reuse:
        _POT_PLANS[x.device] = (key, plan)
    return plan


def clear_potential_plans():
    """Drop the plans potential() keeps for reuse (each closes once no autograd context holds it)."""
    _POT_PLANS.clear()


class _PotentialFn(torch.autograd.Function):
    """phi = A(x, y, Z) q with the adjoint of fmmhp_backward."""

    @staticmethod
    def forward(ctx, x, y, q, lam, p, leaf_size, reuse):
        plan = _potential_plan(x.detach(), y.detach(), complex(lam.detach().cpu().item()), p, leaf_size, reuse)
        phi = plan(q.detach())
        ctx.plan = plan
        ctx.lam_dtype = lam.dtype
        ctx.save_for_backward(q)
        return phi

    @staticmethod
    def backward(ctx, g):
        (q,) = ctx.saved_tensors
        nx, ny, nq, nl = ctx.needs_input_grad[:4]
        r = ctx.plan.backward(q.detach(), g, want_q=nq, want_x=nx, want_y=ny, want_lambda=nl)
        gl = None
        if nl:
            v = r["lambda"] if ctx.lam_dtype.is_complex else r["lambda"].real
            gl = torch.tensor(v, dtype=ctx.lam_dtype)
        return r.get("x"), r.get("y"), r.get("q"), gl, None, None, None


def potential(x, y, q, impedance, p=20, leaf_size=40, reuse_plan=True) -> torch.Tensor:
    """Differentiable phi_i = sum_j q_j G(r_i, r_j) over the points (x, y) for real charges q:
    gradients flow to x, y, q and, when it is a tensor, to the impedance (real or complex).
    The plan (tree, lists, tables) is built for the points and reused by later calls with the same
    x and y tensors, not modified in place since, and the same impedance, p and leaf size (one plan
    per device; reuse_plan=False builds a new one every call).  Changes to the points that bypass
    torch's version counter (through .data, or by other libraries writing the memory) are not seen:
    pass reuse_plan=False then."""
    if q.is_complex():
        raise TypeError("potential() takes real charges; use HalfPlaneFMM for complex ones")
    if not isinstance(impedance, torch.Tensor):
        impedance = torch.tensor(complex(impedance) if isinstance(impedance, complex) else float(impedance),
                                 dtype=torch.complex128 if isinstance(impedance, complex) else torch.float64)
    return _PotentialFn.apply(x, y, q, impedance, int(p), int(leaf_size), bool(reuse_plan))


def direct(xs, ys, q, impedance, xt=None, yt=None) -> torch.Tensor:
    """GPU direct sum phi_i = sum_j q_j G(r_i, r_j) (all pairs)."""
    xs = _dev_f64(xs, "xs")
    ys = _dev_f64(ys, "ys")
    if xt is None:
        xt, yt = xs, ys
    xt = _dev_f64(xt, "xt")
    yt = _dev_f64(yt, "yt")
    squeeze = q.dim() == 1
    q2 = _dev_f64(q.reshape(1, -1) if squeeze else q, "q")
    nv = q2.shape[0]
    raw = torch.empty((nv, xt.shape[0], 2), dtype=torch.float64, device=xs.device)
    lr, li = _split_impedance(impedance)
    with torch.cuda.device(xs.device):
        fmmhp_direct_eval(xs.shape[0], xs.data_ptr(), ys.data_ptr(), nv, q2.data_ptr(),
                          xt.shape[0], xt.data_ptr(), yt.data_ptr(), lr, li, raw.data_ptr(),
                          _stream())
    phi = torch.view_as_complex(raw)
    return phi[0] if squeeze else phi


def reaction_integrals(x, y, nmax: int, impedance) -> torch.Tensor:
    """I_0..I_nmax at points (x, y) on the GPU: complex128 [m, nmax + 1]."""
    x = _dev_f64(x, "x")
    y = _dev_f64(y, "y")
    m = x.shape[0]
    raw = torch.empty((m, nmax + 1, 2), dtype=torch.float64, device=x.device)
    lr, li = _split_impedance(impedance)
    with torch.cuda.device(x.device):
        fmmhp_reaction_integrals(m, x.data_ptr(), y.data_ptr(), nmax, lr, li, raw.data_ptr(),
                                 _stream())
    return torch.view_as_complex(raw)


__all__ = ["HalfPlaneFMM", "direct", "reaction_integrals", "lib", "header_functions",
           "FMMHPError", "Opts", "PlanStats", "fmmhp_plan_create", "fmmhp_plan_create_targets", "fmmhp_eval",
           "fmmhp_plan_info", "fmmhp_plan_export_tree", "fmmhp_plan_destroy",
           "fmmhp_direct_eval", "fmmhp_reaction_integrals", "MAX_P",
           "fmmhp_plan_set_timing", "fmmhp_plan_phase_times", "PHASES", "fmmhp_tune", "tune",
           "fmmhp_backward", "potential", "clear_potential_plans", "fmmhp_batch_plan_create", "fmmhp_eval_complex",
           "fmmhp_eval_noalloc", "NOALLOC_SCRATCH_BYTES"]
