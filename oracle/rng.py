"""Counter-based Gaussian generator for the random sketches (oracle side).

The compression draws Gaussian test matrices (Algorithm A.1).  So that the
oracle and the HIP library sketch with the same matrices without sharing
code, both implement Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11) from its published definition,
followed by the Box-Muller transform.

Entry (i, j) of the sketch of compression instance (seed, instance):
    key     = (seed, instance)             instance = 4*tree_node + kind
    counter = (i, j, 0, 0)
    (x0, x1, _, _) = Philox4x32-10(counter, key)
    u1 = (x0 + 0.5) / 2^32,  u2 = (x1 + 0.5) / 2^32
    g  = sqrt(-2 ln u1) * cos(2 pi u2)
"""
import numpy as np

__all__ = ["philox4x32", "gaussian_block", "instance_key"]

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=10):
    """Vectorised Philox4x32 on uint64 arrays holding 32-bit values."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & _MASK for v in (c0, c1, c2, c3))
    k0 = np.uint64(k0) & _MASK
    k1 = np.uint64(k1) & _MASK
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def instance_key(tree_node, kind):
    """Second key word of a compression instance (kind 0: Schur complement of
    the node, kind 1: the inner Schur complement of its interior block)."""
    return (int(tree_node) << 2) | int(kind)


def gaussian_block(seed, instance, rows, col0, ncols):
    """rows x ncols float64 block of standard normals, columns col0.."""
    i = np.repeat(np.arange(rows, dtype=np.uint64), ncols)
    j = np.tile(np.arange(col0, col0 + ncols, dtype=np.uint64), rows)
    zero = np.zeros_like(i)
    x0, x1, _, _ = philox4x32(i, j, zero, zero, seed, instance)
    u1 = (x0.astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = (x1.astype(np.float64) + 0.5) * 2.0 ** -32
    g = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return g.reshape(rows, ncols)
