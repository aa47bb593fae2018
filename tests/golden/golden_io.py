"""Readers of the stored oracle values under tests/golden (plain text; no oracle code).

The files are written by make_golden.py, which calls the CPU oracle; bench.py and the GPU tests
read them through these functions.
"""
from __future__ import annotations

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLE = 256


def path_for(name: str) -> str:
    return os.path.join(HERE, f"{name}_direct_sample{N_SAMPLE}.txt")


def grad_path_for(name: str) -> str:
    return os.path.join(HERE, f"{name}_grad_sample{N_SAMPLE}.txt")


def dlp_path_for(name: str) -> str:
    return os.path.join(HERE, f"{name}_dlp_sample{N_SAMPLE}.txt")


def load_dlp(name: str):
    """(indices, complex values) from a stored double-layer file, or None if absent."""
    p = dlp_path_for(name)
    if not os.path.exists(p):
        return None
    a = np.loadtxt(p, comments="#")
    return a[:, 0].astype(np.int64), a[:, 1] + 1j * a[:, 2]


def forest_path() -> str:
    return os.path.join(HERE, "batched_forest_direct_sample.txt")


def example2_path() -> str:
    return os.path.join(HERE, "example2_4000_direct.txt")


def load_example2():
    """complex values of the Example 2 direct sum at every field point (N_field + 8 N_source =
    4000), or None if absent."""
    p = example2_path()
    if not os.path.exists(p):
        return None
    a = np.loadtxt(p, comments="#")
    return a[:, 1] + 1j * a[:, 2]


def load(name: str):
    """(indices, complex values) from a stored potential file, or None if absent."""
    p = path_for(name)
    if not os.path.exists(p):
        return None
    a = np.loadtxt(p, comments="#")
    return a[:, 0].astype(np.int64), a[:, 1] + 1j * a[:, 2]


def load_grad(name: str):
    """(indices, [n, 3] array of dl/dq, dl/dx, dl/dy) from a stored file, or None if absent."""
    p = grad_path_for(name)
    if not os.path.exists(p):
        return None
    a = np.loadtxt(p, comments="#")
    return a[:, 0].astype(np.int64), a[:, 1:4]


def load_forest():
    """(instance, vector, index within the instance, complex value) arrays, or None if absent."""
    p = forest_path()
    if not os.path.exists(p):
        return None
    a = np.loadtxt(p, comments="#")
    return (a[:, 0].astype(np.int64), a[:, 1].astype(np.int64), a[:, 2].astype(np.int64),
            a[:, 3] + 1j * a[:, 4])
