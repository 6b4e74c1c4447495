"""FP64 CPU oracle for the MACT hot path (Celebi, Kingravi & Celiker,
"Fast Color Space Transformations Using Minimax Approximations").

THIS PACKAGE IS TEST INFRASTRUCTURE.  It is a plain, slow, obviously correct
numpy implementation of what the GPU library computes (and a scalar C one of
its CIELAB and tetrahedral-LUT parts), written from the paper
and used only to check it: by the tests, by the smoke check and by the
``cpu_baseline`` leg of the benchmark.  The product (the HIP library and its
Python binding) never imports, calls or links anything in here, and nothing in
here imports the product.

Modules
-------
colour   exact RGB->CIELAB / HSI / SCT / CIELUV transforms, their inverses
         (the definitions solved for R, G, B; the SCT one is the paper's own) and
         the error metrics (Sec. 3.2.1, 3.3.1, 3.4.1 and the metric of
         Sec. 3.4.1).
tables   the coefficient tables printed in the paper (Tables 1-7).
mact     FP64 evaluation of the minimax-approximated transforms (Sec. 3.2.2,
         3.3.2, 3.4.2-3.4.3) exactly as the GPU kernels evaluate them, and of
         the inverses with sine, cosine and the BT.709 encoding power replaced
         by minimax approximations in the same way.
remez    Remez exchange for minimax polynomials and rationals (Sec. 3.1),
         optionally under a positive weight (max |w (p/q - f)|), and a
         linear-programming discrete minimax used as an independent check.
lut      3-D LUT packing and the trilinear, prism, pyramidal and tetrahedral
         interpolators, with angular channels (Sec. 3.5.3), in the standard
         form and in the caching form (per-cell edge differences).
grad     analytic Jacobian of the minimax CIELAB transform and central finite
         differences.
cbase    ctypes binding of cbase.c: the exact and MACT RGB->CIELAB transforms
         and the packed LUT with tetrahedral interpolation, scalar FP64 C, one
         pixel at a time (built with gcc -O2 by ``cbase.build()``); the
         benchmark's CPU baseline times it.

Pins (what checks this oracle against something other than itself) live in
``tests/test_oracle_*.py``.  Two functions have no pin against a value the
paper prints and are marked "parity unpinned" in their docstrings: the
pyramidal interpolator and the angular (HSI/SCT) LUT channels; they are held
only to invariants (node hits, affine precision, continuity).
"""
