"""GPU parity of the closure under insertions (bmlp_closure_insert): the
closure of a relation, updated in place with a batch of new edges, must be
bit-for-bit the closure of the enlarged relation as the oracle computes it
from scratch (per-source BFS over the union of the edge lists)."""
import numpy as np
import pytest

import gen
import oracle
from oracle import boolops

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2408_10369_amd as B  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = B.Context(0)
    yield c
    c.close()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def t32(a):
    return torch.as_tensor(np.asarray(a, np.int32))


def closure_of(ctx, n, s, d, opts=None):
    R = ctx.pack_coo(t32(s), t32(d), n, n)
    return ctx.rms(R, n, opts=opts)


@pytest.mark.parametrize("n,p,b", [(1, 0.0, 1), (2, 0.0, 1), (65, 0.02, 3), (200, 0.005, 17), (1000, 0.001, 64),
                                   (1100, 0.0005, 200), (3000, 0.0003, 700)])
def test_insert_matches_recomputed_closure(ctx, n, p, b):
    rng = np.random.default_rng(n * 13 + b)
    s, d = gen.er_digraph(n, p, int(rng.integers(1 << 30)))
    T = closure_of(ctx, n, s, d)
    es = rng.integers(0, n, b).astype(np.int32)
    ed = rng.integers(0, n, b).astype(np.int32)
    print(f"closure_insert n={n} m={len(s)} b={b}", flush=True)
    st = {}
    ctx.closure_insert(T, n, es, ed, stats=st)
    want = oracle.closure_rows(n, np.concatenate([s, es]), np.concatenate([d, ed]))
    assert np.array_equal(host(T), want)


@pytest.mark.parametrize("arm", [B.ARM_PRODUCT_VALU, B.ARM_PRODUCT_MFMA])
def test_insert_product_arms_and_batches(ctx, arm):
    """Several batches in a row, each product on one forced arm; the padding words stay zero."""
    n = 1500
    rng = np.random.default_rng(7 + arm)
    s, d = gen.er_digraph(n, 0.0006, 77)
    ld = boolops.words(n) + 2
    R = ctx.pack_coo(t32(s), t32(d), n, n, ld=ld)
    o = B.make_opts(dispatch=B.DISPATCH_FORCED, product_arm=arm)
    T = ctx.rms(R, n, opts=o)
    alls, alld = list(s), list(d)
    for b in (1, 40, 9, 600):
        es = rng.integers(0, n, b).astype(np.int32)
        ed = rng.integers(0, n, b).astype(np.int32)
        ctx.closure_insert(T, n, es, ed, opts=o)
        alls += list(es)
        alld += list(ed)
        assert np.array_equal(host(T), oracle.closure_rows(n, alls, alld, ld=ld)), (arm, b)


def test_insert_special_edges(ctx):
    n = 130
    # a path 0 -> 1 -> ... -> 129
    s, d = np.arange(n - 1, dtype=np.int32), np.arange(1, n, dtype=np.int32)
    T = closure_of(ctx, n, s, d)
    before = host(T).copy()
    # no edges: unchanged
    ctx.closure_insert(T, n, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert np.array_equal(host(T), before)
    # edges already implied, and duplicates: unchanged
    ctx.closure_insert(T, n, [0, 0, 5, 5], [7, 7, 129, 129])
    assert np.array_equal(host(T), before)
    # a self-loop puts the node on a cycle of length one
    ctx.closure_insert(T, n, [64], [64])
    want = oracle.closure_rows(n, np.concatenate([s, [64]]), np.concatenate([d, [64]]))
    assert np.array_equal(host(T), want)
    # closing the path into a cycle: everything reaches everything
    ctx.closure_insert(T, n, [129], [0])
    assert np.array_equal(host(T), boolops.to_bits(np.ones((n, n), np.uint8)))
    # an endpoint outside [0, n) is an error and leaves the closure alone
    cur = host(T).copy()
    with pytest.raises(B.BmlpError):
        ctx.closure_insert(T, n, [3, n], [4, 5])
    with pytest.raises(B.BmlpError):
        ctx.closure_insert(T, n, [3], [-1])
    assert np.array_equal(host(T), cur)


def test_insert_at_sweep_size(ctx):
    """n = 16,384 (the sparsest graph of the density sweep), 256 new edges; rows sampled for the oracle."""
    n, s, d = gen.c2(0)
    T = closure_of(ctx, n, s, d)
    old = host(T).copy()
    rng = np.random.default_rng(99)
    es = rng.integers(0, n, 256).astype(np.int32)
    ed = rng.integers(0, n, 256).astype(np.int32)
    ctx.closure_insert(T, n, es, ed)
    got = host(T)
    assert np.array_equal(got & old, old)  # closures only grow
    rows = np.sort(np.concatenate([rng.choice(n, 96, replace=False), es[:16], ed[:16]]))
    want = oracle.closure_rows(n, np.concatenate([s, es]), np.concatenate([d, ed]), rows=rows)
    assert np.array_equal(got[rows], want)
