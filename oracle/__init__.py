"""Independent FP64 CPU oracle for the Krylov CT-HYB local trace.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the
CPU-baseline leg of the benchmark do.  It shares no code with the HIP library:
it builds its own Fock space, its own operator matrices and its own
Hamiltonian, and evaluates the trace by plain dense eigendecomposition of
each quantum-number block and matrix products, in float64.

Modules
-------
fock        occupation-number basis, Jordan-Wigner operator matrices,
            (n_up, n_dn) blocks                        (Sec. III, Sec. IV.C)
hamiltonian Kanamori H_loc of Eq.(4) from operator products, block spectra,
            retained set                               (Sec. III steps 1-2)
trace       Tr_R(c) by eigendecomposition and matrix products
                                                       (Eq.(2), Sec. III steps 3-8)

Every function cites the passage of the paper it follows.  No function here
is "parity unpinned": the tests under tests/ pin each one against values
the paper prints, closed forms, invariants or brute force.
"""
