"""FLINNG CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of FLINNG's query path
("Practical Near Neighbor Search via Group Testing", Engels, Coleman and
Shrivastava, 2021), written in C (``flinng_oracle.c``) and driven from here
through ctypes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library in ``paper_2106_11565_amd``; both follow the same
written hashing specification independently.

Every function names the passage of the paper it follows; each is pinned by
``tests/test_oracle_*.py`` (closed forms, invariants, brute force, statistics).
"""
from .core import (  # noqa: F401
    build_lib, lib, sm64, mix64, hyperplanes, srp_codes, exact_dot_sign,
    minhash_codes, text_items, permute, groups, stream_groups, members, build_lists, counts,
    counts_brute, decode, query_fixed_t, set_threads, get_threads, OracleIndex,
    bf16_to_f64, SRP_F32, SRP_BF16, MINHASH_U32, MINHASH_U64,
)
