"""Boolean matrix operators of the paper (Section 2), on dense 0/1 arrays.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Addition is element-wise OR, multiplication is the OR of ANDs
``(AB)_ij = OR_k A_ik AND B_kj`` (over k = 0..n-1), transpose swaps the
arguments of a relation, negation flips every bit of the n x n matrix.  The
product uses an integer matrix product followed by ``> 0``: the count of
witnesses k is positive exactly when the OR of ANDs is true.

``to_bits`` / ``from_bits`` convert between dense 0/1 arrays and row-major
uint64 bit rows with column j at bit (j & 63) of word (j >> 6).
"""
from __future__ import annotations

import numpy as np


def words(n: int) -> int:
    return (n + 63) // 64


def to_bits(dense, ld=None) -> np.ndarray:
    d = np.asarray(dense).astype(bool)
    if d.ndim == 1:
        d = d[None, :]
    rows, n = d.shape
    ld = ld or max(words(n), 1)
    padded = np.zeros((rows, ld * 64), dtype=bool)
    padded[:, :n] = d
    b = np.packbits(padded, axis=1, bitorder="little")
    return b.view("<u8").reshape(rows, ld).astype(np.uint64)


def from_bits(bits, n: int) -> np.ndarray:
    b = np.ascontiguousarray(bits, dtype="<u8")
    rows = b.shape[0]
    u8 = b.view(np.uint8).reshape(rows, -1)
    d = np.unpackbits(u8, axis=1, bitorder="little")
    return d[:, :n].astype(np.uint8)


def dense_from_edges(n: int, src, dst) -> np.ndarray:
    a = np.zeros((n, n), dtype=np.uint8)
    a[np.asarray(src, dtype=np.int64), np.asarray(dst, dtype=np.int64)] = 1
    return a


def add(a, b):
    return (np.asarray(a, bool) | np.asarray(b, bool)).astype(np.uint8)


def land(a, b):
    return (np.asarray(a, bool) & np.asarray(b, bool)).astype(np.uint8)


def mul(a, b):
    ai = np.asarray(a, dtype=np.int64)
    bi = np.asarray(b, dtype=np.int64)
    return ((ai @ bi) > 0).astype(np.uint8)


def transp(a):
    return np.ascontiguousarray(np.asarray(a, np.uint8).T)


def neg(a):
    return (1 - np.asarray(a, np.uint8)).astype(np.uint8)


def identity(n: int):
    return np.eye(n, dtype=np.uint8)
