"""Reference oracle for the preconditioned, restarted and shifted block FOM
(PSBFOM-DR) computation of Z = e^{tA} B (Wu, Pang, Sun, arXiv:1405.0707).

THIS PACKAGE IS TEST INFRASTRUCTURE.  It is a plain, slow, CPU-only, FP64
implementation written from the paper, used only to check the HIP library.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product library (``paper_1405_0707_amd``)
never imports, links or calls anything here, and nothing here imports the
product: the two share only the seeded input generators in ``workloads``.

Modules
  cf        Caratheodory-Fejer rational approximation of e^x on (-inf, 0]
            (paper Section 2), computed in mpmath, plus an FP64 numpy twin.
  psbfom    Algorithm 1 (SBFOM-DR) and Algorithm 2 (PSBFOM-DR), Sections 3-4.
  inverses  ways to apply A^{-1} (sparse LU, DST fast Poisson solve,
            Gohberg-Semencul for Toeplitz, Krylov inner solves), Section 4.1.
  exact     plain definitions of r(tA)B and e^{tA}B used as pins.

Every function that has no independent pin says "parity unpinned" in its
docstring.
"""
