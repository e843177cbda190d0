"""Reference oracle for the chromatic-polynomial strip transfer matrix.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links anything in this directory; only the test suite, the smoke check and
the benchmark's CPU-baseline leg may use it.

Everything here is plain, slow and written to be checked by eye against
J. L. Jacobsen, "Bulk, surface and corner free energy series for the
chromatic polynomial on the square and triangular lattices" (arXiv 1005.3609):

* ``graphs``      -- the m x n rectangles (Sec. 3, eq. Z_from_T and the
                     triangular-lattice subsection), the definition of P_G(q)
                     as a count of proper colourings (Sec. 1) and the FK
                     subset expansion (Sec. 2, eqs. Z1/Z2), plus a
                     colour-class dynamic programme over the same rectangles.
* ``partitions``  -- set partitions of a layer, Catalan/Motzkin counts
                     (Sec. 3.2) and the NCNNN ordering (Sec. 3.4, eq. M_recurs).
* ``transfer``    -- the FK transfer matrix: the generic product of single-edge
                     operators (Sec. 3.2, any v) and the projected sparse
                     factorisation at v = -1 (eqs. T_sq_decomp, T_sq_proj,
                     T_last, T_last_i and the triangular factors), with weights
                     either exact integer polynomials in q, exact polynomials in
                     1/q (the paper's normalised Z-tilde, eq. Z_modified), or
                     residues modulo 31-bit primes (Sec. 3.5).

Pins (tests/test_oracle_*.py) tie each function to something other than
itself: brute-force colouring counts, closed forms, invariants, the state
lists the paper prints, and agreement between independent methods.
"""
