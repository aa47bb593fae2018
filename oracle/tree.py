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
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.tree_ref_free.argtypes = [ctypes.c_void_p]
        lib.tree_ref_info.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 5
        lib.tree_ref_export.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 18
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def build(x, y, leaf_size: int, max_level: int = 30, lbits: int = 30) -> dict:
    """Reference tree and lists as a dict of numpy arrays (see tree_ref.c)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = x.shape[0]
    h = lib.tree_ref_build(n, _ptr(x), _ptr(y), int(leaf_size), int(max_level), int(lbits))
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


FOREST_LBITS = 27


def build_forest(x, y, offsets, leaf_size: int, max_level: int | None = None) -> dict:
    """Reference forest: instance k = points offsets[k]..offsets[k+1]-1, each built by ``build``
    with 27-bit cells (its own root square), then merged into one numbering.

    Box order: by level, then instance, then each instance's own order (Morton prefix).  Point
    order: instance after instance, each in its own sorted order.  List entries are renumbered
    and sorted ascending per target box, as for one tree.  A forest of one instance is ``build``
    with 30-bit cells.
    """
    offsets = [int(v) for v in offsets]
    if len(offsets) == 2:
        return build(x, y, leaf_size, 30 if max_level is None else max_level)
    max_level = FOREST_LBITS if max_level is None else max_level
    trees = [build(x[a:b], y[a:b], leaf_size, max_level, FOREST_LBITS)
             for a, b in zip(offsets[:-1], offsets[1:])]
    depth = max(int(t["level"].max()) for t in trees)
    newidx = [np.full(t["nbox"], -1, np.int64) for t in trees]
    order = []  # (instance, old index) in new order
    for l in range(1, depth + 1):
        for k, t in enumerate(trees):
            for b in np.nonzero(t["level"] == l)[0]:
                newidx[k][b] = len(order)
                order.append((k, int(b)))
    nb = len(order)
    out = {f: np.zeros(nb, np.int32) for f in
           ("level", "bx", "by", "first", "count", "parent", "leaf", "child_first", "nchild")}

    def remap(k, v):
        return -1 if v < 0 else int(newidx[k][v])

    for i, (k, b) in enumerate(order):
        t = trees[k]
        for f in ("level", "bx", "by", "count", "leaf", "nchild"):
            out[f][i] = t[f][b]
        out["first"][i] = t["first"][b] + offsets[k]
        out["parent"][i] = remap(k, t["parent"][b])
        out["child_first"][i] = remap(k, t["child_first"][b])
    out["perm"] = np.concatenate([t["perm"] + offsets[k] for k, t in enumerate(trees)])
    for name in LIST_NAMES:
        off = np.zeros(nb + 1, np.int64)
        ents = []
        for i, (k, b) in enumerate(order):
            t = trees[k]
            e = t[name + "_ent"][t[name + "_off"][b]:t[name + "_off"][b + 1]]
            e = np.sort(2 * newidx[k][e >> 1] + (e & 1))
            ents.append(e)
            off[i + 1] = off[i] + len(e)
        out[name + "_off"] = off
        out[name + "_ent"] = (np.concatenate(ents) if ents else np.zeros(0, np.int64)).astype(np.int32)
    out["nbox"] = nb
    out["x_lo"] = [t["x_lo"] for t in trees]
    out["S"] = [t["S"] for t in trees]
    return out
