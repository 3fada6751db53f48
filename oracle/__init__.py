"""FP64 CPU oracle for the lossy-GBS matrix-product-operator hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or executes this package; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

It is a plain, slow, dense implementation written from the paper
(Liu, Oh, Liu, Jiang, Alexeev, "Simulating lossy Gaussian boson sampling with
matrix product operators", arXiv 2301.12814):

* ``states``   single-mode squeezed vacuum (App. C, input wavefunction) and the
               pure-loss Kraus channel (App. B, Kraus operators), giving the
               per-mode input density matrices.
* ``fock``     two-mode Fock-space beam-splitter matrix from the explicit
               binomial expansion of the creation-operator transform
               (App. B, creation-operator transform and Eq. kun).
* ``clements`` Haar interferometer -> rectangular mesh of beam splitters plus
               an output phase screen (App. A, M-layer array).
* ``mpo``      dense Vidal-form MPO of the vectorised density operator (Sec. II,
               Eq. MPS and the vectorisation map; App. D, two-site update and
               the truncated SVD), with **no charge blocking**; charges are
               only carried as labels for bookkeeping and for the mirror-pair
               truncation rule.
* ``brute``    full density-matrix evolution and the U(1) operator
               entanglement entropy by definition, for M <= 4.

Every function states the passage it follows.  Pins (closed forms, brute
force, invariants) live in ``tests/test_oracle_*.py``.
"""
