"""Plain, slow CPU oracle for the MPS-trajectory simulator (arXiv 2508.05745).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import anything from here.  The HIP product path never calls it and
shares no code with it; the two meet only in ``paper_2508_05745_amd.inputs`` (seeded
problem descriptions, no arithmetic of the method).

Everything here is NumPy (complex128 / float64) with library primitives (eigh, svd, qr,
einsum) as single steps, following the paper's definitions in the paper's order:

* ``rng``        counter-based uniform draws (SplitMix64, Steele-Lea-Flood 2014)
* ``unravel``    locally entanglement-optimal Kraus mixing (Sec. "Locally
                 entanglement-optimal unraveling" and the appendix on Wootters' decomposition)
* ``dm``         exact density-matrix evolution of a noisy circuit (tiny widths)
* ``sv``         statevector trajectories (Alg. 1 applied to every noise event)
* ``mps``        MPS trajectories with SVD truncation (Sec. "Details of MPS-based
                 trajectory sampling")
* ``kraus_tree`` exact enumeration of the Kraus tree (Sec. "Class of Truncated Trajectory
                 Sampling Algorithms")
* ``cost``       expected linear / Renyi-2 entropy of an unravelling and its gradient

Parity status of each function is stated in its docstring.
"""
