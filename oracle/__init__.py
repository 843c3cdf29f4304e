"""CPU oracle for the BMLP hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library and never imports it.

Contents
--------
* ``two_sided_rows``: the least P = B | L P R (a linear program with a
  relation on each side of its recursive atom) by Kleene iteration from B,
  each step two dense numpy products of 0/1 matrices; n up to a few thousand.
* ``closure_rows``, ``smp``, ``compose_rows``, ``warshall``: the C oracle
  (``bmlp_oracle.c``): per-source breadth-first search, i.e. the plain
  definition of the transitive closure R1+ (Eq. 1), of the selection v R1+
  (Eq. 5) and of the linear composition P = Rs* Rb (Theorem 1), plus
  Warshall's algorithm as an independent brute force.
* ``algorithms``: Algorithms 1 and 2 of the paper stepped literally on dense
  0/1 matrices (numpy), for small sizes and iteration counts.
* ``datalog``: a pure-Python semi-naive bottom-up evaluator over sets of
  pairs, for the paper's programs (P2, the linear composition, and the
  stratified P3 u P4 u P5 example).
* ``boolops``: Boolean matrix addition, multiplication, transpose and
  negation (Section 2) on dense 0/1 arrays, and the oracle's own conversion
  between dense 0/1 arrays and the LSB-first uint64 bit rows.
* ``mlp``: FP64 forward pass, masked MSE loss and its gradient for the
  dispatcher network (the reference its GPU training kernels are checked
  against).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bmlp_oracle.c")
_LIB = os.path.join(_HERE, "libbmlp_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        i64, ip, i32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        L.bmlp_oracle_closure_rows.argtypes = [i64, i64, ip, ip, ip, i64, ip, i64, i32, ip]
        L.bmlp_oracle_smp.argtypes = [i64, i64, ip, ip, ip, i64, i64, ip, i32, i32, ip]
        L.bmlp_oracle_compose_rows.argtypes = [i64, i64, ip, ip, i64, ip, ip, ip, i64, ip, i64, i32, ip]
        L.bmlp_oracle_warshall.argtypes = [i64, ip, i64]
        for f in (L.bmlp_oracle_closure_rows, L.bmlp_oracle_smp,
                  L.bmlp_oracle_compose_rows, L.bmlp_oracle_warshall):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def words(n: int) -> int:
    return (n + 63) // 64


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _edges(src, dst):
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    assert s.shape == d.shape
    return s, d


last_threads = 0


def closure_rows(n, src, dst, rows=None, ld=None, threads=0):
    """Rows of R1+ (all rows when ``rows`` is None) as uint64 bit rows."""
    global last_threads
    s, d = _edges(src, dst)
    ld = ld or max(words(n), 1)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = n if r is None else len(r)
    out = np.zeros((nr, ld), dtype=np.uint64)
    used = ctypes.c_int(0)
    rc = lib().bmlp_oracle_closure_rows(n, len(s), _p(s), _p(d), _p(r), nr,
                                        _p(out), ld, threads, ctypes.byref(used))
    if rc:
        raise RuntimeError("oracle closure failed: %d" % rc)
    last_threads = used.value
    return out


def smp(n, src, dst, V, reflexive=False, threads=0):
    """``V R1+`` row by row (``V R1*`` when reflexive); V is uint64 bit rows."""
    global last_threads
    s, d = _edges(src, dst)
    V = np.ascontiguousarray(V, dtype=np.uint64)
    k, ldv = V.shape
    out = np.zeros((k, ldv), dtype=np.uint64)
    used = ctypes.c_int(0)
    rc = lib().bmlp_oracle_smp(n, len(s), _p(s), _p(d), _p(V), k, ldv, _p(out),
                               1 if reflexive else 0, threads, ctypes.byref(used))
    if rc:
        raise RuntimeError("oracle smp failed: %d" % rc)
    last_threads = used.value
    return out


def compose_rows(n, bsrc, bdst, ssrc, sdst, rows=None, ld=None, threads=0):
    """Rows of P = Rs* Rb."""
    global last_threads
    bs, bd = _edges(bsrc, bdst)
    ss, sd = _edges(ssrc, sdst)
    ld = ld or max(words(n), 1)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = n if r is None else len(r)
    out = np.zeros((nr, ld), dtype=np.uint64)
    used = ctypes.c_int(0)
    rc = lib().bmlp_oracle_compose_rows(n, len(bs), _p(bs), _p(bd), len(ss), _p(ss), _p(sd),
                                        _p(r), nr, _p(out), ld, threads, ctypes.byref(used))
    if rc:
        raise RuntimeError("oracle compose failed: %d" % rc)
    last_threads = used.value
    return out


def warshall(bits, n):
    """R1+ of an n x n bit matrix by Warshall's algorithm (copy returned)."""
    R = np.array(bits, dtype=np.uint64, copy=True, order="C")
    rc = lib().bmlp_oracle_warshall(n, _p(R), R.shape[1])
    if rc:
        raise RuntimeError("oracle warshall failed: %d" % rc)
    return R


from . import boolops, algorithms, datalog, mlp  # noqa: E402,F401


def is_foreign_rows(n, contains, adjoins, location=None, threads=0):
    """P3 u P4 u P5 of Section 3.4 on bit rows; returns (hasPlace, indirectlyPartOf, isForeign).

    hasPlace is the closure of contains (its rows by breadth-first search);
    indirectlyPartOf is the least model of the linear recursion whose base is
    adjoins together with its inverse and whose step is the inverse of
    hasPlace (Theorem 1, P = Rs* Rb); isForeign holds between two locations
    unless indirectlyPartOf does (negation of a finished lower stratum).
    ``location`` defaults to every constant.  Inverses are taken on the pair
    lists, the negation and the location mask on the bit rows with numpy.
    """
    cs, cd = _edges(*contains)
    as_, ad = _edges(*adjoins)
    ld = max(words(n), 1)
    has_place = closure_rows(n, cs, cd, ld=ld, threads=threads)
    hp_src, hp_dst = _bits_pairs(has_place, n)
    base_src = np.concatenate([as_, ad])
    base_dst = np.concatenate([ad, as_])
    ipo = compose_rows(n, base_src, base_dst, hp_dst, hp_src, ld=ld, threads=threads)
    loc = np.zeros(n, dtype=bool)
    if location is None:
        loc[:] = True
    else:
        loc[np.asarray(location, dtype=np.int64)] = True
    mask = np.zeros(ld * 64, dtype=np.uint8)
    mask[:n] = loc
    row_mask = np.packbits(mask, bitorder="little").view(np.uint64)
    foreign = np.where(loc[:, None], ~ipo & row_mask[None, :], np.uint64(0))
    return has_place, ipo, foreign


def _bits_pairs(bits, n):
    """(row, col) pairs of the set bits of uint64 bit rows (LSB first)."""
    dense = np.unpackbits(np.ascontiguousarray(bits).view(np.uint8), axis=1, bitorder="little")[:, :n]
    r, c = np.nonzero(dense)
    return r.astype(np.int32), c.astype(np.int32)


def two_sided_rows(n, base, left, right, ld=None, max_rounds=None):
    """Bit rows of the least P with P = B | L . P . R, by iterating P <- B | L . P . R from P = B until
    nothing changes (the operator is monotone, so this reaches the least fixpoint).  base, left,
    right: (src, dst) pairs.  Dense float32 products of 0/1 matrices, each thresholded at > 0 (the
    counts stay below n <= 2**24, so they are exact)."""
    def dense(pairs):
        s, d = _edges(*pairs)
        a = np.zeros((n, n), np.float32)
        a[s, d] = 1.0
        return a
    B, L, R = dense(base), dense(left), dense(right)
    P = B.copy()
    rounds = 0
    while True:
        nxt = np.maximum(B, (((L @ P) > 0).astype(np.float32) @ R > 0).astype(np.float32))
        rounds += 1
        if np.array_equal(nxt, P):
            break
        P = nxt
        if max_rounds is not None and rounds > max_rounds:
            raise RuntimeError("two-sided oracle did not converge")
    ld = ld or max(words(n), 1)
    bits = np.zeros((n, ld * 64), np.uint8)
    bits[:, :n] = P > 0
    return np.packbits(bits, axis=1, bitorder="little").view(np.uint64)
