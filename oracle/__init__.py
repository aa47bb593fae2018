"""CPU oracle for the half-plane Robin Laplace FMM -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations of what the GPU
library computes, written from the paper (Xiang, Wang, Zhang, Cai, "Fast
multipole method for the Laplace equation in half plane with Robin boundary
condition").  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute anything
under ``oracle/``.  The oracle shares no code with the GPU library and neither
imports the other; the only shared module is the seeded input generator
``workloads``.

Modules
-------
kernel      Green's function pieces: I_0, the I_n recursion, G_Z, full G
            (Section 2.1, eqs. (ddGreensfunimp), (generalintegral),
            (reactdecomposition), (integralrecursion)).
direct      O(N^2) direct summation of the potential (eq. (potential1)).
expansions  S2M/M2M/S2L/L2L/M2L for the reaction field (Section 2.2) and the
            textbook log-kernel expansions the paper defers to.
tree        ctypes wrapper of ``tree_ref.c``: the reference adaptive quadtree
            over targets plus image sources and its U/V/W/X lists.

Every function here is pinned by a ``-m "not gpu"`` test against something other
than itself (quadrature of the defining Fourier integral, the PDE and boundary
condition, closed forms printed in the paper, brute force); see the test files.
"""
