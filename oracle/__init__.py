"""CPU oracle for the f-circulant matrix-vector product (Rosowski, "On Fast
Computation of a Circulant Matrix-Vector Product", arXiv 2103.02605).

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct CPU
statement of what the GPU library computes. Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the library itself never does, and it
shares no code, tables or constants with the HIP path.

Modules:
  ring      -- Z/p helpers (inverse, square roots, primitive roots, n-th roots).
  fcirc     -- the product itself: the dense definition (Definition 2) and the
               recursion of Algorithm 1 (section 2), in a literal recursive form and a
               level-by-level numpy form, over Z/p and over complex numbers.
  polymul   -- integer polynomial products (section 3.1): schoolbook, Kronecker
               substitution, and residues + CRT through the f-circulant product.
  bigint    -- large-integer products (section 3.2 application) and carry propagation.
  grad      -- FP64 reference gradients of the real/complex circulant layer.

Every function states the passage it follows. Functions without a pin of their own are
marked "parity unpinned" in their docstring.
"""
