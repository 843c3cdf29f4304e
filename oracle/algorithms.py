"""Algorithms 1 and 2 of the paper, stepped literally on dense 0/1 matrices.

TEST INFRASTRUCTURE ONLY (see the package docstring).  For small matrices;
they report how many products they took, which pins the loop logic of the
fixpoint drivers (not only their results).

Algorithm 1 (BMLP-RMS, Section 4): R = I + R1; repeat R' = R R until R' = R;
the answer is the last square times R1.

Algorithm 2 (BMLP-SMP, Section 4): v' = v; repeat v* = v' + v' R1 until
v* = v'; the answer is v* R1.

``rms_squaring_or`` is the variant the hot path runs by default: R = R1;
repeat R' = R + R R until R' = R (the fixpoint of Eq. 1, reached by doubling
the path length each product).  It needs no final product.
"""
from __future__ import annotations

import numpy as np

from .boolops import add, identity, mul


def rms_paper(R1):
    """Algorithm 1.  Returns (R2*, squarings, products including the final)."""
    R1 = np.asarray(R1, np.uint8)
    n = R1.shape[0]
    R = add(identity(n), R1)
    squarings = 0
    while True:
        R2 = mul(R, R)
        squarings += 1
        if np.array_equal(R2, R):
            break
        R = R2
    return mul(R2, R1), squarings, squarings + 1


def rms_squaring_or(R1):
    """R <- R + R R until unchanged.  Returns (R1+, products)."""
    R = np.asarray(R1, np.uint8).copy()
    products = 0
    while True:
        R2 = add(R, mul(R, R))
        products += 1
        if np.array_equal(R2, R):
            return R, products
        R = R2


def smp_paper(v, R1):
    """Algorithm 2 on a 1 x n (or k x n, row-wise) selection.

    Returns (v*, loop iterations, products including the final)."""
    v = np.asarray(v, np.uint8)
    if v.ndim == 1:
        v = v[None, :]
    vp = v.copy()
    it = 0
    while True:
        vs = add(vp, mul(vp, R1))
        it += 1
        if np.array_equal(vs, vp):
            break
        vp = vs
    return mul(vs, R1), it, it + 1
