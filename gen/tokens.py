"""Seeded token stream whose greedy parse has one 16-byte match per token.

The first block holds T = 1024 distinct random 16-byte tokens in order (token
j starts with byte j mod 256).  Every later token is drawn so that its first
byte differs from the first byte of every token that followed the same
predecessor token anywhere earlier in the stream.  A match found at a token
start therefore copies exactly that token: the source's next byte never
equals the destination's next byte, so no match extends past 16 bytes, and a
16 KiB block after the first holds 1024 sequences (LL = 0, ML = 16), the most
that 16-byte minimum matches allow.  Many tokens repeat inside their own
block, so a block also holds chains of matches whose sources are earlier
matches of the same block.

Input generator only: no codec arithmetic.
"""
from __future__ import annotations

import numpy as np

TOKEN = 16
N_TOKENS = 1024


def token_stream(n_blocks: int, seed: int = 11) -> bytes:
    rng = np.random.default_rng(seed)
    tok = rng.integers(0, 256, (N_TOKENS, TOKEN), dtype=np.uint8)
    tok[:, 0] = np.arange(N_TOKENS) & 255
    first = tok[:, 0].astype(np.int64)
    # succ[j]: first bytes of tokens that followed token j so far
    succ = [set() for _ in range(N_TOKENS)]
    order = list(range(N_TOKENS))
    for j in range(N_TOKENS - 1):
        succ[j].add(int(first[j + 1]))
    prev = N_TOKENS - 1
    per_block = (1 << 14) // TOKEN
    for _ in range((n_blocks - 1) * per_block):
        while True:
            k = int(rng.integers(0, N_TOKENS))
            if int(first[k]) not in succ[prev]:
                break
        succ[prev].add(int(first[k]))
        order.append(k)
        prev = k
    return tok[np.asarray(order)].tobytes()
