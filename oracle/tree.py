"""ctypes wrapper of ``tree_ref.c`` (the reference quadtree) -- CPU oracle.

Test infrastructure only (see ``oracle/__init__``).  ``build_lib()`` compiles the
C file with gcc (``-ffp-contract=off``) into ``oracle/libtree_ref.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tree_ref.c")
_LIB = os.path.join(_HERE, "libtree_ref.so")
_lib = None

LIST_NAMES = ("U", "V", "W", "X")


def build_lib(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_lib()
        lib = ctypes.CDLL(_LIB)
        lib.tree_ref_build.restype = ctypes.c_void_p
        lib.tree_ref_build.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int, ctypes.c_int]
        lib.tree_ref_free.argtypes = [ctypes.c_void_p]
        lib.tree_ref_info.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 5
        lib.tree_ref_export.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 18
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def build(x, y, leaf_size: int, max_level: int = 30) -> dict:
    """Reference tree and lists as a dict of numpy arrays (see tree_ref.c)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = x.shape[0]
    h = lib.tree_ref_build(n, _ptr(x), _ptr(y), int(leaf_size), int(max_level))
    if not h:
        raise MemoryError("tree_ref_build failed")
    try:
        nbox = np.zeros(1, np.int64)
        xlo = np.zeros(1)
        S = np.zeros(1)
        scale = np.zeros(1)
        lens = np.zeros(4, np.int64)
        lib.tree_ref_info(h, _ptr(nbox), _ptr(xlo), _ptr(S), _ptr(scale), _ptr(lens))
        nb = int(nbox[0])
        out = {k: np.zeros(nb, np.int32) for k in
               ("level", "bx", "by", "first", "count", "parent", "leaf", "child_first", "nchild")}
        out["perm"] = np.zeros(n, np.int64)
        offs = [np.zeros(nb + 1, np.int64) for _ in range(4)]
        ents = [np.zeros(max(1, int(lens[j])), np.int32) for j in range(4)]
        args = [out[k] for k in ("level", "bx", "by", "first", "count", "parent", "leaf",
                                 "child_first", "nchild", "perm")]
        for j in range(4):
            args += [offs[j], ents[j]]
        lib.tree_ref_export(h, *[_ptr(a) for a in args])
        for j, name in enumerate(LIST_NAMES):
            out[name + "_off"] = offs[j]
            out[name + "_ent"] = ents[j][: int(lens[j])]
        out["nbox"] = nb
        out["x_lo"] = float(xlo[0])
        out["S"] = float(S[0])
        out["scale"] = float(scale[0])
        return out
    finally:
        lib.tree_ref_free(h)
