"""CPU oracle for products in F2[X] and F2[X]/(X^n - 1), and for inverses in
F2[X]/(X^n - 1).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.
It shares no code with the GPU library.  See ``gf2x_oracle.c`` for what each
function computes and which passage of the paper it follows.
"""
from .oracle import (  # noqa: F401
    build,
    clmul64,
    fold,
    inv_cyclic,
    load,
    mul,
    mul_cyclic,
    mul_batched,
    mul_cyclic_many,
    mul_cyclic_many_pclmul,
    REF_ITEM_DTYPE,
    words,
)
