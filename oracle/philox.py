"""Philox4x32-10 counter-based generator and the draws the sampler takes from it.

TEST INFRASTRUCTURE ONLY (see the package header).

Philox4x32 with 10 rounds is implemented from its published definition
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11): a 128-bit counter is mixed by ten rounds, each of which takes two
32x32->64-bit products of counter words with fixed multipliers and xors the
high halves with the other counter words and the round key; the 64-bit key is
bumped by two Weyl constants between rounds.

The paper draws its randomness from JAX's splittable keys (listings in
Appendix E).  Here every draw is a pure function of (seed; chain, iteration,
purpose, block), so any subset of chains can be replayed exactly.

Stream layout (the HIP library implements the same layout independently):
  key   = (seed mod 2^32, seed div 2^32)
  ctr   = (global chain id, HMC iteration t, tag, block j)
  tag 1 = momentum refresh: block j gives coordinates 2j and 2j+1
  tag 2 = Metropolis accept: block 0, first two words
  tag 3 = block-shuffle benchmark
  tag 4 = predictive draws of the test rows (DSS)
  tag 5 = starting draw of each chain from the full-data draws
Uniform from two words (w0, w1):
  u = ((w0 * 2^32 + w1) >> 12) * 2^-52 + 2^-53, strictly inside (0, 1), exact in fp64.
Normal pair by Box-Muller from block words (w0,w1) -> u1 and (w2,w3) -> u2:
  r = sqrt(-2 ln u1);  z_even = r cos(2 pi u2);  z_odd = r sin(2 pi u2).

Pins: published known-answer vectors of Philox4x32-10 and distribution tests
(tests/test_oracle_philox.py).
"""
from __future__ import annotations

import numpy as np

TAG_MOMENTUM = 1
TAG_ACCEPT = 2
TAG_SHUFFLE = 3
TAG_PREDICT = 4      # predictive draws of the test rows (DSS)
TAG_INIT = 5         # starting draw of each chain from the full-data draws (workflow Step 2)

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Apply the ten-round Philox4x32 bijection.

    ctr: tuple of four uint32-valued arrays (broadcastable), key: (k0, k1).
    Returns four uint64 arrays holding 32-bit words.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK32 for c in ctr)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK32
            k1 = (k1 + _W1) & _MASK32
        prod0 = _M0 * c0                       # < 2^64, exact in uint64
        prod1 = _M1 * c2
        hi0, lo0 = prod0 >> _S32, prod0 & _MASK32
        hi1, lo1 = prod1 >> _S32, prod1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def seed_key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def uniform_from_words(w0, w1) -> np.ndarray:
    """Map two 32-bit words to a double strictly inside (0, 1)."""
    bits = ((np.asarray(w0, dtype=np.uint64) << _S32) | np.asarray(w1, dtype=np.uint64))
    top52 = (bits >> np.uint64(12)).astype(np.float64)
    return top52 * 2.0 ** -52 + 2.0 ** -53


def momentum_normals(seed: int, chains, t: int, d: int) -> np.ndarray:
    """Standard normal z[c, j] for the momentum refresh of iteration t.

    chains: array of global chain ids.  Returns [len(chains), d] float64.
    """
    chains = np.asarray(chains, dtype=np.uint64)
    nb = (d + 1) // 2
    key = seed_key(seed)
    cc = chains[:, None]
    jj = np.arange(nb, dtype=np.uint64)[None, :]
    w0, w1, w2, w3 = philox4x32_10((cc, np.uint64(t), np.uint64(TAG_MOMENTUM), jj), key)
    u1 = uniform_from_words(w0, w1)
    u2 = uniform_from_words(w2, w3)
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty((chains.shape[0], 2 * nb))
    z[:, 0::2] = r * np.cos(2.0 * np.pi * u2)
    z[:, 1::2] = r * np.sin(2.0 * np.pi * u2)
    return z[:, :d]


def accept_uniforms(seed: int, chains, t: int) -> np.ndarray:
    """Uniform u[c] used by the Metropolis test of iteration t."""
    chains = np.asarray(chains, dtype=np.uint64)
    w0, w1, _, _ = philox4x32_10((chains, np.uint64(t), np.uint64(TAG_ACCEPT), np.uint64(0)),
                                 seed_key(seed))
    return uniform_from_words(w0, w1)


def shuffle_indices(seed: int, fold: int, replicate: int, L: int, D: int) -> np.ndarray:
    """Chain index drawn with replacement for each (chain slot, block) of one
    block-shuffle replicate (benchmark of Rhat_max, Section 4.2 / Algorithm A2).

    Returns [L, D] ints in [0, L).  ctr = (fold, replicate, TAG_SHUFFLE, slot*D + block),
    chain = floor(u * L) with u from the first two words.
    """
    key = seed_key(seed)
    jj = np.arange(L * D, dtype=np.uint64)
    w0, w1, _, _ = philox4x32_10((np.uint64(fold), np.uint64(replicate),
                                  np.uint64(TAG_SHUFFLE), jj), key)
    u = uniform_from_words(w0, w1)
    idx = np.minimum(np.floor(u * L).astype(np.int64), L - 1)
    return idx.reshape(L, D)


def predictive_words(seed: int, chains, t: int, v: int):
    """Philox words for the predictive draws of iteration t: one block per
    (chain, test-row slot j), counter (chain, t, TAG_PREDICT, j).  Returns four
    [len(chains), v] uint64 arrays."""
    chains = np.asarray(chains, dtype=np.uint64)
    jj = np.arange(v, dtype=np.uint64)[None, :]
    return philox4x32_10((chains[:, None], np.uint64(t), np.uint64(TAG_PREDICT), jj), seed_key(seed))


def init_draw_indices(seed: int, chains, n_draws: int) -> np.ndarray:
    """Index of the full-data draw each chain starts from (workflow Step 2):
    counter (chain, 0, TAG_INIT, 0), index = floor(u * n_draws) with u from the
    first two words (clamped to n_draws - 1)."""
    chains = np.asarray(chains, dtype=np.uint64)
    w0, w1, _, _ = philox4x32_10((chains, np.uint64(0), np.uint64(TAG_INIT), np.uint64(0)), seed_key(seed))
    u = uniform_from_words(w0, w1)
    return np.minimum(np.floor(u * n_draws).astype(np.int64), n_draws - 1)
