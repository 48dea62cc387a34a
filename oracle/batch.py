"""Minibatch selection without replacement (Sec. 3.2: N/n minibatches per epoch).

Each epoch e of chain c visits the observations in the order of a keyed
bijection pi_{c,e} of [0, N): a four-round Feistel network on b =
bitlength(N - 1) bits (left half floor(b/2) bits, right half the rest), whose
round function is the first output word of Philox4x32-10, with cycle walking
back into [0, N).  Minibatch j of the epoch is pi(j*n), ..., pi(j*n + n - 1);
B = floor(N/n) minibatches per epoch, the N - B*n left-over positions are
skipped.  Step t uses epoch t // B and minibatch t % B.
"""
from __future__ import annotations

import numpy as np

from .philox import TAG_PERM, key_of, philox4x32_10

MAX_WALK = 4096   # cycle-walk cap; reaching it is reported as an error


def split_bits(N: int):
    b = max(1, int(N - 1).bit_length())
    bl = b // 2
    return b, bl, b - bl


def feistel(x, N: int, seed: int, stream: int, chain: int, epoch: int):
    """One pass of the four-round Feistel bijection on [0, 2^b)."""
    b, bl, br = split_bits(N)
    k0, k1 = key_of(seed)
    x = np.asarray(x, np.uint64)
    left = x >> np.uint64(br)
    right = x & np.uint64((1 << br) - 1)
    mask_l = np.uint64((1 << bl) - 1)
    mask_r = np.uint64((1 << br) - 1)
    for rnd in range(4):
        tag = TAG_PERM | (stream << 4) | rnd
        if rnd % 2 == 0:
            f = philox4x32_10(right, epoch & 0xFFFFFFFF, chain, tag, k0, k1)[0]
            left = left ^ (f & mask_l)
        else:
            f = philox4x32_10(left, epoch & 0xFFFFFFFF, chain, tag, k0, k1)[0]
            right = right ^ (f & mask_r)
    return (left << np.uint64(br)) | right


def permute(k, N: int, seed: int, stream: int, chain: int, epoch: int) -> np.ndarray:
    """pi_{chain,epoch}(k) for positions k in [0, N), by cycle walking."""
    y = feistel(k, N, seed, stream, chain, epoch)
    for _ in range(MAX_WALK):
        out = y >= np.uint64(N)
        if not out.any():
            return y.astype(np.int64)
        y[out] = feistel(y[out], N, seed, stream, chain, epoch)
    raise RuntimeError("cycle walk did not return to [0, N)")


def batch_indices(seed: int, stream: int, chain: int, step: int, N: int, n: int) -> np.ndarray:
    """Observation indices of the minibatch of `chain` at global step `step`."""
    if not 0 < n <= N:
        raise ValueError("need 0 < n <= N")
    B = N // n
    epoch, j = divmod(step, B)
    k = np.arange(j * n, j * n + n, dtype=np.uint64)
    return permute(k, N, seed, stream, chain, epoch)
