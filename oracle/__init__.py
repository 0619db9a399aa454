"""CPU FP64 oracle for Hessenberg-triangular reduction (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and the two share no
code: the oracle is written from the paper (Algorithm 2 of Appendix A,
BasicHouseHT) and from the textbook Givens HT reduction of Moler and Stewart
that the paper compares against (Sec. 1).

The C part lives in ``ht_oracle.c``; ``build_oracle()`` compiles it with gcc
into ``_build/liboracle.so``.  ``checks`` holds the comparison helpers (sign
normalisation, invariants, a Krylov-basis reference for tiny n).
"""
from .core import basic_ht, ms_ht, fast_ht, fast_flops, house, normal, build_oracle, oracle_lib_path  # noqa: F401
