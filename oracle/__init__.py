"""FP64 CPU oracle for the sketching hot path of adaptive HSS construction.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check in
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import
or run it.  The product (``paper_2302_01977_amd``) never imports it, and it never
imports the product; the two share no code.  Both sides take their inputs from
the seeded generators in ``workloads``, which hold none of the method's arithmetic.

Contents (each function cites the passage of the paper it follows):
  philox     Philox4x32-10 counter-based generator (replaces the paper's
             std::minstd_rand so that every operator entry is a pure function of
             (seed, counter)).
  operators  explicit FP64 blocks of the Gaussian, SJLT (block construction) and
             SRHT operators of section 2.4, the SRHT element formula of
             section 7.2, the SJLT B+/B- split of section 6.1.
  sketch     S = A R, S' = A^T R, sampled columns, the adjoint dS R^T, the
             matrix-free Gaussian-kernel sketch and its closed-form gradient.
  hss        reference adaptive HSS compression (Algorithm 1), interpolative
             decomposition, dense reconstruction.

Parity status: every function is pinned by a CPU test in ``tests/`` against a
value or property fixed by the paper or by mathematics (published Philox
vectors, the section 6.1 worked example, Hadamard orthogonality, brute-force
products by the paper's own CRS/CCS formulations, an explicit fast
Walsh-Hadamard transform, finite differences, exact-HSS recovery).  Nothing here
is "parity unpinned".
"""
from . import hss, operators, philox, sketch  # noqa: F401
