"""Complexity C, latency T and memory M of the decoders, as Section III-B
counts them (quantitative complexity analysis; Tables 1-5, Fig. 6).

TEST INFRASTRUCTURE, like the rest of the oracle: only tests/ and bench.py's
context figures use it; nothing in the GPU path does.

C counts floating-point additions and comparisons per received vector.  T
counts idealised time steps: hard decisions and binary operations are free,
independent operations run in parallel, and a sort of n items takes log2 n
steps.  M counts bits, with Q bits per LLR or path metric (the published
KB figures are KiB at Q = 32).

Readings (each reproduces the printed values listed beside it; the pins are
in tests/test_oracle_pins.py):

* L = 1 (Table 2, with the first-order node priced as its transform alone,
  s 2^s additions: the maximum search that Table 2 adds as 2^s comparisons is
  not in Fig. 6's figures).  An internal node costs 2^s for f and g, an SPC
  node RM(s-1, s) costs 2^s, and a node of the permutation domain adds its
  selection: 2L candidate LM sums of 2^(s-1) terms each plus a sort of the
  2L sums at 2L log2(2L) comparisons (the n log2 n that Table 1 charges for
  its path-metric sorts).  Reproduces all six L = 1 points of Fig. 6
  (FHT-FSCL-1 and p-FHT-FSCL-1 on RM(2,9), RM(3,9), RM(4,9)) to the three
  digits printed.
* Latency at L = 1: f and g one step each, the FHT s steps, an SPC node
  s + 1 steps (the log2 n of its reliability sort plus the parity
  decision), a permutation node 1 + log2(2L) more (its LM sums, then the
  sort of the 2L candidates).  Reproduces Fig. 6's six L = 1 latencies
  exactly (49/51, 130/134, 209/215).
* M decoders in parallel (Alg. 5): M times one decoder's operations plus the
  M - 1 comparisons of the final minimum, and ceil(log2 M) more steps for
  that minimum.  Reproduces Table 5's p-FHT-FSCL-1-M column (C to the two
  digits printed, T exactly) for RM(2,8), RM(3,8), RM(4,8) and RM(2,9).
* The permutation node's cost at any L: Fig. 6 prints p-FHT-FSCL-L and
  FHT-FSCL-L side by side, and their difference is the permutation
  domain's selection alone.  The latency differences are exactly
  n_perm (1 + log2(2L)) at every printed L, and the operation differences
  fall within the printed rounding of n_perm-node sums above.
* Memory: Table 3's four formulas, which give every published figure of the
  proposed decoders (Fig. 6's six, Table 4's three, Table 5's twelve).

Parity unpinned: the operations and latency of the list nodes at L > 1.  No
reading of Table 1 found here reproduces Fig. 6's list figures (the
per-function formulas summed over Alg. 2's schedule overshoot them by up to
5x); `ops_per_decoder` at L > 1 uses an approximate model of the list nodes
(FHT: L s 2^s additions, one 2^s maximum scan, L min(L, 2^s) candidate
metrics and an L^2 log2 L candidate sort; SPC: L 2^s plus Table 1's
L(2 tau (2 + log2 L) + 1)), which lies within 6% (5.4% at worst) of all 30 list points of
Fig. 6.  It serves only to price configurations the paper prints no figure
for.
"""
from __future__ import annotations

import math

from . import schedule  # Alg. 2's node schedule, pinned to Fig. 4


def _nodes(m: int, r: int, permuted: bool):
    from . import PERM_NONE, PERM_PFHT
    return [(kind, s) for kind, _, s in schedule(m, r, PERM_PFHT if permuted else PERM_NONE)]


def perm_node_ops(s: int, L: int) -> int:
    """Selection at a permutation-domain node of length 2^s (Alg. 2): 2L LM
    sums of 2^(s-1) terms, then the 2L sums sorted (n log2 n)."""
    return 2 * L * (1 << (s - 1)) + int(2 * L * math.log2(2 * L))


def perm_node_steps(L: int) -> int:
    """Time steps the permutation-domain selection adds at one node."""
    return 1 + int(math.log2(2 * L))


def node_ops(kind: str, s: int, L: int) -> float:
    """Operations of one node of length n = 2^s for a list of L paths.
    Exact reading at L = 1; an approximate model at L > 1 (parity unpinned)."""
    n = 1 << s
    if kind in ("perm", "internal"):
        c = L * n  # f and g, L 2^(s-1) each (Table 1-2)
        return c + (perm_node_ops(s, L) if kind == "perm" else 0)
    if kind == "fhtl":
        if L == 1:
            return s * n
        k = min(L, n)
        return L * s * n + n + L * k + L * L * math.log2(L)
    if kind == "spcl":
        if L == 1:
            return n
        tau = min(L, n - 1)
        return L * n + L * (2 * tau * (2 + math.log2(L)) + 1)
    raise ValueError(kind)


def node_steps_l1(kind: str, s: int) -> int:
    """Time steps of one node at L = 1."""
    if kind in ("perm", "internal"):
        return 2 + (perm_node_steps(1) if kind == "perm" else 0)
    if kind == "fhtl":
        return s
    if kind == "spcl":
        return s + 1
    raise ValueError(kind)


def ops_per_decoder(r: int, m: int, L: int, permuted: bool = True) -> float:
    """Operations of one decoder over the whole tree (exact at L = 1)."""
    return sum(node_ops(kind, s, L) for kind, s in _nodes(m, r, permuted))


def steps_per_decoder_l1(r: int, m: int, permuted: bool = True) -> int:
    """Latency of one L = 1 decoder in time steps."""
    return sum(node_steps_l1(kind, s) for kind, s in _nodes(m, r, permuted))


def n_perm_nodes(r: int, m: int) -> int:
    return sum(1 for kind, _ in _nodes(m, r, True) if kind == "perm")


def ops_per_frame(r: int, m: int, L: int, M: int, permuted: bool = True) -> float:
    """p-FHT-FSCL-L-M: M decoders, then the minimum of their M metrics."""
    return M * ops_per_decoder(r, m, L, permuted) + (M - 1)


def steps_per_frame_l1(r: int, m: int, M: int) -> int:
    """p-FHT-FSCL-1-M latency: the decoders run in parallel, then a
    ceil(log2 M)-step minimum."""
    return steps_per_decoder_l1(r, m, True) + (math.ceil(math.log2(M)) if M > 1 else 0)


def memory_bits(N: int, L: int = 1, M: int = 1, Q: int = 32) -> int:
    """Table 3: bits of LLR, path-metric and codeword storage."""
    if L == 1 and M == 1:
        return (2 * N + 1) * Q + N
    if L == 1:
        return (N + M * (N + 1)) * Q + M * N
    if M == 1:
        return N * (L + 1) * Q + 2 * L * Q + 2 * N * L
    return N * (L * M + 1) * Q + 2 * M * L * Q + 2 * M * N * L


def memory_kib(N: int, L: int = 1, M: int = 1, Q: int = 32) -> float:
    return memory_bits(N, L, M, Q) / 8.0 / 1024.0
