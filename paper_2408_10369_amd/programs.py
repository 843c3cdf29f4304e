"""Whole programs built from the library's C-ABI operators (no computation here).

``is_foreign`` is the stratified program of Section 3.4 (P3, P4 and P5):

    hasPlace          = contains+                          (BMLP-RMS)
    indirectlyPartOf  = (hasPlace^T)* . (adjoins | adjoins^T)  (linear recursion, Theorem 1)
    isForeign         = (location . location^T) & NEG(indirectlyPartOf)

``hasPlace`` is a lower stratum: it is finished before the recursion that uses
it, so that recursion is linear.  ``location`` is the monadic predicate, a set of
constants; the product of its column and its row is the relation that holds
between any two locations.
"""
from __future__ import annotations


def is_foreign(ctx, n: int, contains, adjoins, location, opts=None, stream=None, stats=None):
    """Returns the device bit matrices (hasPlace, indirectlyPartOf, isForeign), each n x n.

    contains, adjoins: (src, dst) pairs of int32 tensors of constant indices; location: int32 tensor
    of the constants that are locations.  ``stats`` (a dict) receives the composition's statistics.
    """
    import torch

    dev = f"cuda:{ctx.device}"
    cs, cd = contains
    as_, ad = adjoins
    loc = torch.as_tensor(location).to(device=dev, dtype=torch.int32)
    Rc = ctx.pack_coo(cs, cd, n, n, stream=stream)
    Ra = ctx.pack_coo(as_, ad, n, n, stream=stream)
    has_place = ctx.rms(Rc, n, opts=opts, stream=stream)
    base = ctx.or_(Ra, ctx.transpose(Ra, n, stream=stream), n, stream=stream)
    step = ctx.transpose(has_place, n, stream=stream)
    ipo = ctx.compose_linear(base, step, n, opts=opts, stream=stream, stats=stats)
    zeros = torch.zeros_like(loc)
    loc_col = ctx.pack_coo(loc, zeros, n, 1, stream=stream)   # n x 1
    loc_row = ctx.pack_coo(zeros, loc, 1, n, stream=stream)   # 1 x n
    both = ctx.product(loc_col, loc_row, 1, n, stream=stream)  # location(X), location(Y)
    foreign = ctx.andnot(both, ipo, n, stream=stream)
    return has_place, ipo, foreign
