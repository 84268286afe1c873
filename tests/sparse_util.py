"""Dense x sparse items for the tests: position arrays packed into a uint64
buffer (uint32 positions, two per word) and the oracle's view of a sparse
operand (the dense polynomial sum_t X^(p_t mod n), equal positions
cancelling).  Test infrastructure only."""
import numpy as np

import oracle


def dense_of_positions(pos, n):
    """words(n) uint64 words of sum_t X^(pos[t] mod n) over F2."""
    s = np.zeros(oracle.words(n), dtype=np.uint64)
    for p in np.asarray(pos, dtype=np.uint64).tolist():
        p = int(p) % n
        s[p // 64] ^= np.uint64(1) << np.uint64(p % 64)
    return s


def pack_positions(pos_lists):
    """(buffer of uint64 words, word offset of each list): list i occupies
    ceil(len/2) words from its offset, positions as uint32 little-endian."""
    offs, total = [], 0
    for pos in pos_lists:
        offs.append(total)
        total += (len(pos) + 1) // 2 or 1
    buf = np.zeros(total, dtype=np.uint64)
    view = buf.view(np.uint32)
    for o, pos in zip(offs, pos_lists):
        view[2 * o:2 * o + len(pos)] = np.asarray(pos, dtype=np.uint32)
    return buf, np.asarray(offs, dtype=np.uint64)
