"""Seeded synthetic operands shared by the tests, the smoke check and the bench.

This module holds no polynomial arithmetic: it only draws words.  Random words
come from SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014): the state advances by the golden-ratio
increment 0x9E3779B97F4A7C15 and each state is passed through the published
two-multiply finaliser.

Stream keying: the words of operand ``role`` of item ``p`` under ``seed`` are
the SplitMix64 outputs for the states ``key + (k + 1) * GAMMA``, k = 0, 1, ...,
with ``key = (seed << 24) ^ (p << 2) ^ role``.  Roles: 0 = operand a,
1 = operand b, 2 = sparse positions.

Operands follow the packing of the library: bit i is bit i % 64 of word
i // 64 (little-endian); bits >= n are zero.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# The six ring sizes of the HQC / BIKE parameter sets the library targets.
RING_SIZES = (12323, 17669, 24659, 35851, 40973, 57637)
# Config seeds: 220110473 * 1000 + k for workload k.
SEED_BASE = 220110473 * 1000


def words(n):
    return (int(n) + 63) // 64


def _finalise(z):
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed, item, role):
    return ((int(seed) << 24) ^ (int(item) << 2) ^ int(role)) & 0xFFFFFFFFFFFFFFFF


def splitmix_words(key, count):
    """First ``count`` SplitMix64 outputs of the stream starting at ``key``."""
    with np.errstate(over="ignore"):
        k = np.arange(1, count + 1, dtype=np.uint64)
        states = np.uint64(key) + k * GAMMA
        return _finalise(states)


def splitmix_scalar(state):
    """Reference scalar SplitMix64 step: returns (new_state, output) as ints."""
    m = 0xFFFFFFFFFFFFFFFF
    state = (state + 0x9E3779B97F4A7C15) & m
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return state, z ^ (z >> 31)


def top_mask(n):
    s = int(n) % 64
    return np.uint64(0xFFFFFFFFFFFFFFFF if s == 0 else (1 << s) - 1)


def dense(n, seed, item=0, role=0):
    """Uniform dense operand of n bits (bits >= n zero), words(n) uint64 words."""
    w = splitmix_words(stream_key(seed, item, role), words(n))
    w[-1] &= top_mask(n)
    return w


def dense_batch(n, count, seed, role=0, first_item=0):
    """(count, words(n)) array; row p is ``dense(n, seed, first_item + p, role)``."""
    W = words(n)
    out = np.empty((count, W), dtype=np.uint64)
    with np.errstate(over="ignore"):
        items = np.arange(first_item, first_item + count, dtype=np.uint64)
        keys = (np.uint64(int(seed) << 24 & 0xFFFFFFFFFFFFFFFF) ^ (items << np.uint64(2))) ^ np.uint64(role)
        k = np.arange(1, W + 1, dtype=np.uint64)
        states = keys[:, None] + k[None, :] * GAMMA
        out[:] = _finalise(states)
    out[:, -1] &= top_mask(n)
    return out


def dense_items(n, item_ids, seed, role=0):
    """(len(item_ids), words(n)); row r is ``dense(n, seed, item_ids[r], role)``."""
    W = words(n)
    ids = np.asarray(item_ids, dtype=np.uint64)
    with np.errstate(over="ignore"):
        keys = (np.uint64(int(seed) << 24 & 0xFFFFFFFFFFFFFFFF) ^ (ids << np.uint64(2))) ^ np.uint64(role)
        k = np.arange(1, W + 1, dtype=np.uint64)
        out = _finalise(keys[:, None] + k[None, :] * GAMMA)
    out[:, -1] &= top_mask(n)
    return out


def sparse_positions(n, weight, seed, item=0, role=2):
    """``weight`` distinct positions in [0, n), uniform, by rejection sampling.

    A 64-bit draw z is accepted when z < floor(2^64 / n) * n (so z mod n is
    unbiased) and z mod n is not already chosen."""
    n = int(n)
    if weight > n:
        raise ValueError("weight exceeds n")
    limit = (1 << 64) // n * n
    key = stream_key(seed, item, role)
    chosen = []
    seen = set()
    state = key
    while len(chosen) < weight:
        state, z = splitmix_scalar(state)
        if z >= limit:
            continue
        pos = z % n
        if pos in seen:
            continue
        seen.add(pos)
        chosen.append(pos)
    return sorted(chosen)


def from_positions(n, positions):
    """Pack a set of bit positions into words(n) uint64 words."""
    w = np.zeros(words(n), dtype=np.uint64)
    for p in positions:
        w[p // 64] |= np.uint64(1) << np.uint64(p % 64)
    return w


def sparse(n, weight, seed, item=0, role=2):
    return from_positions(n, sparse_positions(n, weight, seed, item, role))


def sparse_weight_for(n):
    """Hamming weight of the sparse operand in the mixed workload, by level:
    the two smallest ring sizes take 66, the middle two 100, the largest two 131."""
    n = int(n)
    if n <= 17669:
        return 66
    if n <= 35851:
        return 100
    return 131
