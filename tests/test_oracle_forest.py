"""Pins for the reference forest (oracle/tree.py build_forest): several independent instances in
one box numbering, each quantised on its own root square with 27-bit cells.

* a forest of one instance is the plain tree;
* within every instance each (target leaf, source leaf) pair -- sources and their images -- is
  reached by exactly one list path, and no list entry crosses instances;
* box point ranges partition each instance's points; boxes are ordered by (level, instance);
* with 27-bit cells the tree of an instance equals the 30-bit tree whenever no box reaches a
  level where the cells differ (shallow trees), box for box.
"""
import numpy as np
import pytest

from oracle import tree as T
from tests.test_oracle_tree import _coverage_failures


def _instances(sizes, seed):
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for k, n in enumerate(sizes):
        x0 = rng.uniform(-5, 5)
        xs.append(x0 + rng.uniform(0, 1 + k % 3, n))
        ys.append(rng.uniform(1e-3, 0.7 + 0.2 * (k % 4), n))
    off = np.concatenate([[0], np.cumsum(sizes)])
    return np.concatenate(xs), np.concatenate(ys), off


def _inst_of_box(f, off):
    return np.searchsorted(off, f["first"], side="right") - 1


def test_single_instance_forest_is_plain_tree():
    x, y, off = _instances([700], 1)
    a = T.build_forest(x, y, off, 16)
    b = T.build(x, y, 16)
    for k in ("level", "bx", "by", "first", "count", "parent", "leaf", "child_first", "nchild", "perm"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("sizes,leaf", [([300, 50, 900, 7, 400], 12), ([60, 60, 60], 4), ([1, 2, 1500], 20)])
def test_forest_lists_cover_pairs_within_instances(sizes, leaf):
    x, y, off = _instances(sizes, 3)
    f = T.build_forest(x, y, off, leaf)
    inst = _inst_of_box(f, off)
    # no list entry crosses instances
    for name in "UVWX":
        o, e = f[name + "_off"], f[name + "_ent"]
        for b in range(f["nbox"]):
            assert np.all(inst[e[o[b]:o[b + 1]] >> 1] == inst[b]), name
    # exactly-once coverage inside each instance: run the single-tree check on each instance's
    # sub-forest (boxes renumbered in forest order)
    for k in range(len(sizes)):
        boxes = np.nonzero(inst == k)[0]
        ren = {int(b): i for i, b in enumerate(boxes)}
        sub = {"nbox": len(boxes), "leaf": f["leaf"][boxes],
               "parent": np.array([ren.get(int(p), -1) for p in f["parent"][boxes]])}
        for name in "UVWX":
            o, e = f[name + "_off"], f[name + "_ent"]
            offs, ents = [0], []
            for b in boxes:
                seg = e[o[b]:o[b + 1]]
                ents.extend(2 * ren[int(c >> 1)] + (c & 1) for c in seg)
                offs.append(len(ents))
            sub[name + "_off"] = np.array(offs)
            sub[name + "_ent"] = np.array(ents, dtype=np.int64)
        assert _coverage_failures(sub) == 0, k


def test_forest_partitions_points_and_orders_boxes():
    sizes = [500, 30, 1200]
    x, y, off = _instances(sizes, 7)
    f = T.build_forest(x, y, off, 10)
    inst = _inst_of_box(f, off)
    key = f["level"].astype(np.int64) * 1000 + inst
    assert np.all(np.diff(key) >= 0)  # level-major, then instance
    assert sorted(f["perm"].tolist()) == list(range(off[-1]))
    for k in range(len(sizes)):
        assert np.all((f["perm"][off[k]:off[k + 1]] >= off[k]) & (f["perm"][off[k]:off[k + 1]] < off[k + 1]))
        leaves = np.nonzero((inst == k) & (f["leaf"] == 1))[0]
        cover = np.zeros(off[k + 1] - off[k], np.int64)
        for b in leaves:
            cover[f["first"][b] - off[k]: f["first"][b] - off[k] + f["count"][b]] += 1
        assert np.all(cover == 1)


def test_27_bit_cells_match_30_bit_tree_when_shallow():
    x, y, off = _instances([400, 400], 11)
    f = T.build_forest(x, y, off, 50)
    for k in range(2):
        a = T.build(x[off[k]:off[k + 1]], y[off[k]:off[k + 1]], 50, 27, 27)
        b = T.build(x[off[k]:off[k + 1]], y[off[k]:off[k + 1]], 50, 27, 30)
        assert a["nbox"] == b["nbox"]
        for key in ("level", "bx", "by", "count", "perm"):
            assert np.array_equal(a[key], b[key]), key
