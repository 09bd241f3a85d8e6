"""CPU oracle for recursive bilinear fast matrix multiplication.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute anything
in this package.  The product (``paper_1409_2908_amd``) never imports it, and
it imports nothing from the product: the two share no code, headers, tables or
generators.  Inputs come from the separate seeded generator module
``fmm_inputs``, which holds none of the method's arithmetic.

Contents (each function cites the passage of Benson and Ballard, "A Framework
for Practical Parallel Fast Matrix Multiplication", PPoPP 2015, that it
follows):

* ``classical``  -- O1, the classical product C = A*B in binary64 (C code,
  OpenMP over rows, no contraction), plus a row-sampled and a compensated
  (Dot2) variant.  Section 2.1 and Equation (1).
* ``tensor``     -- the matrix-multiplication tensor from the membership rule
  of Section 2.2, the exact Brent-equation check (Equation (2)), and the
  permutation transforms of Propositions 2.1 and 2.2.
* ``algorithms`` -- the oracle's own copies of the base-case decompositions
  [[U,V,W]] (Strassen from the formulas of Section 2.1; the others from text
  tables in ``oracle/tables``).
* ``recursive``  -- O2, the recursive fast algorithm written from the steps of
  Section 3.1 (form S_r and T_r, recurse, combine with W) with dynamic peeling
  (Section 3.5), plus flop counting for the closed forms of Section 2.1.
* ``bf16x3``     -- an emulated split-precision reference, tolerance only.

Parity status: O1 is pinned by brute force on rationals and by integer inputs;
O2 is pinned by exact equality with O1 on rationals and by the flop closed
forms; the tables are pinned by the exact Brent check.  The BF16x3 emulation
is "parity unpinned" beyond its exact-integer special case (its tolerances are
derived, not printed in the paper).
"""
