"""Pins for the reference quadtree and interaction lists (oracle/tree_ref.c).

* every (target leaf, source leaf) pair -- source leaves in the upper half and
  their images -- is reached by exactly one list path (U at the leaf, V at the
  leaf or an ancestor onto the source leaf or an ancestor, W at the leaf onto
  the source or an ancestor, X at the leaf or an ancestor);
* the lists equal a brute-force evaluation of their defining predicates over
  ALL boxes (no search-region pruning);
* V entries satisfy the paper's M2L separation condition (Section 2.2, M2L:
  |r_c - r'_c| > sqrt(2)(d_s + d_t)/2), W entries the S2M condition and X
  entries the S2L condition, measured on the actual coordinates;
* box ranges partition the sorted points and every point lies in its boxes.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import tree as T

L = 30


def _lists(t):
    nb = t["nbox"]
    out = {}
    for name in "UVWX":
        off, ent = t[name + "_off"], t[name + "_ent"]
        out[name] = [set(ent[off[b]:off[b + 1]].tolist()) for b in range(nb)]
    return out


def _anc(t, b):
    out = []
    while b >= 0:
        out.append(b)
        b = int(t["parent"][b])
    return out


def _coverage_failures(t):
    lists = _lists(t)
    leaves = [b for b in range(t["nbox"]) if t["leaf"][b]]
    bad = 0
    for b in leaves:
        ab = _anc(t, b)
        for c in leaves:
            ac = _anc(t, c)
            for img in (0, 1):
                code = 2 * c + img
                cnt = int(code in lists["U"][b])
                cnt += sum((2 * d + img) in lists["V"][a] for a in ab for d in ac)
                cnt += sum((2 * d + img) in lists["W"][b] for d in ac)
                cnt += sum(code in lists["X"][a] for a in ab)
                bad += cnt != 1
    return bad


def _clustered(n, seed):
    return workloads.curve_4m(seed=seed, n=n)


CASES = [
    ("plain_small", lambda: workloads.plain_small(), 40),
    ("curve_6k_leaf20", lambda: _clustered(6000, 1), 20),
    ("curve_3k_leaf8", lambda: _clustered(3000, 2), 8),
    ("uniform_small_leaf1", lambda: workloads.uniform(300, 5, (0, 1), (1e-3, 0.5)), 1),
]


@pytest.mark.parametrize("name,gen,leaf", CASES)
def test_lists_cover_every_pair_exactly_once(name, gen, leaf):
    w = gen()
    t = T.build(w.x, w.y, leaf)
    assert _coverage_failures(t) == 0


def _spans(t, img):
    lev = t["level"].astype(np.int64)
    w = np.left_shift(np.int64(1), L - lev)
    by = t["by"].astype(np.int64)
    if img:
        by = np.left_shift(np.int64(1), lev) - 1 - by
    x0 = t["bx"].astype(np.int64) * w
    y0 = by * w
    return x0, x0 + w, y0, y0 + w


def _brute_lists(t):
    nb = t["nbox"]
    lev = t["level"]
    leaf = t["leaf"].astype(bool)
    par = t["parent"]
    S = [_spans(t, 0), _spans(t, 1)]
    full = np.int64(1) << L

    def adj(sa, ia, sb, ib):
        ax0, ax1, ay0, ay1 = sa
        bx0, bx1, by0, by1 = sb
        return (ax0[ia] <= bx1[ib]) & (bx0[ib] <= ax1[ia]) & (ay0[ia] <= by1[ib]) & (by0[ib] <= ay1[ia])

    out = {k: [set() for _ in range(nb)] for k in "UVWX"}
    allc = np.arange(nb)
    for b in range(nb):
        pb = par[b]
        for img in (0, 1):
            sc = S[img]
            a_cb = adj(sc, allc, S[0], np.full(nb, b))
            pc = par[allc]
            # parent adjacency (level-1 parents are the root: adjacent to everything)
            if pb < 0:
                a_pc_pb = np.ones(nb, bool)
            else:
                a_pc_pb = np.where(pc < 0, True, adj(sc, np.maximum(pc, 0), S[0], np.full(nb, pb)))
            a_pc_b = np.where(pc < 0, True, adj(sc, np.maximum(pc, 0), S[0], np.full(nb, b)))
            if pb < 0:
                a_c_pb = np.ones(nb, bool)
            else:
                a_c_pb = adj(sc, allc, S[0], np.full(nb, pb))
            V = (lev == lev[b]) & ~a_cb & a_pc_pb
            X = leaf & (lev < lev[b]) & ~a_cb & a_c_pb
            for c in np.nonzero(V)[0]:
                out["V"][b].add(2 * int(c) + img)
            for c in np.nonzero(X)[0]:
                out["X"][b].add(2 * int(c) + img)
            if leaf[b]:
                U = leaf & a_cb
                Wl = (lev > lev[b]) & ~a_cb & a_pc_b
                for c in np.nonzero(U)[0]:
                    out["U"][b].add(2 * int(c) + img)
                for c in np.nonzero(Wl)[0]:
                    out["W"][b].add(2 * int(c) + img)
    return out


@pytest.mark.parametrize("name,gen,leaf", CASES)
def test_lists_equal_bruteforce_predicates(name, gen, leaf):
    w = gen()
    t = T.build(w.x, w.y, leaf)
    ref = _brute_lists(t)
    got = _lists(t)
    for k in "UVWX":
        assert got[k] == ref[k], k
        off, ent = t[k + "_off"], t[k + "_ent"]
        for b in range(t["nbox"]):
            seg = ent[off[b]:off[b + 1]]
            assert np.all(np.diff(seg) > 0)


def _geometry(t):
    S, xlo = t["S"], t["x_lo"]
    size = S / 2.0 ** t["level"]
    cx = xlo + (t["bx"] + 0.5) * size
    cy = -S / 2 + (t["by"] + 0.5) * size
    return cx, cy, size


@pytest.mark.parametrize("name,gen,leaf", CASES)
def test_admissibility_conditions(name, gen, leaf):
    w = gen()
    t = T.build(w.x, w.y, leaf)
    cx, cy, size = _geometry(t)
    perm = t["perm"]
    xs, ys = w.x[perm], w.y[perm]
    for b in range(t["nbox"]):
        for name_, cond in (("V", None), ("W", None), ("X", None)):
            off, ent = t[name_ + "_off"], t[name_ + "_ent"]
            for code in ent[off[b]:off[b + 1]]:
                c, img = int(code) >> 1, int(code) & 1
                ccy = -cy[c] if img else cy[c]
                if name_ == "V":
                    d = math.hypot(cx[b] - cx[c], cy[b] - ccy)
                    assert d > math.sqrt(2) * (size[b] + size[c]) / 2
                elif name_ == "W":
                    f, n = t["first"][b], t["count"][b]
                    d = np.hypot(xs[f:f + n] - cx[c], ys[f:f + n] - ccy)
                    assert np.all(d > math.sqrt(2) / 2 * size[c])
                else:
                    f, n = t["first"][c], t["count"][c]
                    sy = -ys[f:f + n] if img else ys[f:f + n]
                    d = np.hypot(xs[f:f + n] - cx[b], sy - cy[b])
                    assert np.all(d > math.sqrt(2) / 2 * size[b])


@pytest.mark.parametrize("name,gen,leaf", CASES)
def test_boxes_partition_points(name, gen, leaf):
    w = gen()
    t = T.build(w.x, w.y, leaf)
    n = w.n
    perm = t["perm"]
    assert np.array_equal(np.sort(perm), np.arange(n))
    leaves = np.nonzero(t["leaf"])[0]
    cover = np.zeros(n, int)
    for b in leaves:
        cover[t["first"][b]:t["first"][b] + t["count"][b]] += 1
        assert t["count"][b] <= leaf or t["level"][b] == 30
    assert np.all(cover == 1)
    cx, cy, size = _geometry(t)
    for b in range(t["nbox"]):
        f, c = t["first"][b], t["count"][b]
        px, py = w.x[perm[f:f + c]], w.y[perm[f:f + c]]
        tol = 1e-12 * t["S"]
        assert np.all(np.abs(px - cx[b]) <= size[b] / 2 + tol)
        assert np.all(np.abs(py - cy[b]) <= size[b] / 2 + tol)
        if t["parent"][b] >= 0:
            p = t["parent"][b]
            assert t["first"][p] <= f and f + c <= t["first"][p] + t["count"][p]


def test_degenerate_inputs():
    # one point; duplicates beyond leaf size stop at max_level; N below leaf size
    t = T.build(np.array([0.5]), np.array([0.25]), 4)
    assert t["nbox"] == 1 and t["leaf"][0] == 1
    x = np.full(10, 0.3)
    y = np.full(10, 0.2)
    t = T.build(x, y, 2, max_level=6)
    assert t["level"].max() == 6
    assert _coverage_failures(t) == 0
    w = workloads.uniform(30, 3)
    t = T.build(w.x, w.y, 40)
    assert np.all(t["level"] == 1) and _coverage_failures(t) == 0
