"""Helpers shared by the GPU tests: device buffers for uint64 words."""
import numpy as np


def to_dev(x):
    import torch

    a = np.ascontiguousarray(x, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).cuda()


def from_dev(t):
    return t.cpu().numpy().view(np.uint64)


def empty_dev(nwords, fill=0x5A5A5A5A5A5A5A5A):
    """Device buffer pre-filled with a non-zero pattern so that unwritten words show."""
    import torch

    return torch.full((int(nwords),), np.int64(np.uint64(fill).view(np.int64)), dtype=torch.int64, device="cuda")


def parity_rows(x):
    """Parity of each row of a (count, words) uint64 array."""
    return (np.bitwise_count(x).sum(axis=1) & 1).astype(np.uint8)
