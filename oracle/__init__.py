"""CPU oracle for the Stream-K GEMM -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this package.  The
GPU library never does: the product path fails loudly when its HIP extension
is missing instead of falling back here.

Contents (each function cites the passage of the report it follows):

* ``gemm``      -- plain FP64 definition of C = alpha*A*B + beta*C (C code),
                   exact decoders of the bf16 / f16 / e4m3fn input encodings,
                   relative Frobenius error.
* ``schedule``  -- simulator of the Stream-K iteration-to-workgroup schedule
                   and the invariant checker that pins it.

The oracle shares no code with the HIP path: no common header, kernel,
helper, constant or table generator, and neither imports the other.
"""
