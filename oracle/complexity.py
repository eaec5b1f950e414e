"""Operation counts of the decoders (Section IV-B): floating-point additions
and comparisons per received vector, as the paper's per-function formulas
(Tables 1 and 2) summed over the nodes that Alg. 2 visits.

Test infrastructure, like the rest of the oracle; nothing in the GPU path
uses it.

Pinned (tests/test_oracle_pins.py): p-FHT-FSCL-1-M reproduces Table 5 for
RM(2,8) with M = 25 and RM(2,9) with M = 100.  Parity unpinned elsewhere:
for RM(3,8) and RM(4,8) at L = 1, and for every list decoder (L > 1), the
sums of the per-function formulas differ from the printed totals; the tests
record the computed values beside the printed ones.
"""
from __future__ import annotations

import math

from . import schedule  # Alg. 2's node schedule, pinned to Fig. 4


def node_ops(kind: str, m: int, L: int) -> int:
    """Operations of one function on a sub-code of length 2^m: Table 2 for
    L = 1, Table 1 for L > 1 (tau = min(L, 2^m - 1) splits at an SPC node).
    kind: 'perm' or 'internal' (f for the left child and g for the right;
    the tables price no permutation-domain selection), 'fhtl' (RM(1, m)) or
    'spcl' (RM(m-1, m))."""
    n = 1 << m
    if kind in ("perm", "internal"):  # f and g, each L 2^(m-1)
        return 2 * L * (n // 2)
    lg = int(math.log2(L))
    if kind == "fhtl":
        if L == 1:
            return n * (m + 1)
        return L * m * n + min(L * m * n, L * L * n) + 2 * L * L * (n // 2 + lg)
    if kind == "spcl":
        if L == 1:
            return n
        tau = min(L, n - 1)
        return min(L * m * n, L * L * n) + L * (2 * tau * (2 + lg) + 1)
    raise ValueError(kind)


def ops_per_decoder(r: int, m: int, L: int) -> int:
    """Operations of one decoder (list size L) over the whole tree."""
    return sum(node_ops(kind, s, L) for kind, _, s in schedule(m, r))


def ops_per_frame(r: int, m: int, L: int, M: int) -> int:
    """p-FHT-FSCL-L-M: M decoders per received vector."""
    return M * ops_per_decoder(r, m, L)
