"""The allocation-free selection (bmlp_smp_noalloc) against the allocating one (bmlp_smp with the same
one-launch sparse arm), bit for bit, on two calls in a row (the second smaller), and against the
oracle; its size limits."""
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


def case(ctx, n, deg, k, seed):
    s, d = gen.er_digraph(n, deg / n, seed)
    rng = np.random.default_rng(seed)
    Vd = np.zeros((k, n), np.uint8)
    Vd[np.arange(k), rng.integers(0, n, k)] = 1
    Vd[: k // 4] |= (rng.random((k // 4, n)) < 0.002).astype(np.uint8)
    R = ctx.pack_coo(torch.as_tensor(s), torch.as_tensor(d), n, n)
    V = torch.from_numpy(boolops.to_bits(Vd).view(np.int64)).cuda()
    return s, d, R, V


@pytest.mark.parametrize("refl", [0, 1])
def test_noalloc_matches_smp_twice(ctx, refl):
    sparse = B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_SPARSE, smp_reflexive=refl)
    # first call: a relation of mean degree 6 (edge index with in-edges) and 700 query rows; second call:
    # smaller, mean degree 2 (no in-edges), 90 rows -- the array keeps the first call's contents
    for (n, deg, k, seed) in [(20000, 6.0, 700, 11), (3000, 2.0, 90, 12)]:
        s, d, R, V = case(ctx, n, deg, k, seed)
        out = ctx.zeros(k, n)
        out.fill_(-1)  # every word is written
        got = host(ctx.smp_noalloc(R, n, V, out, reflexive=bool(refl)))
        want = host(ctx.smp(R, n, V, opts=sparse))
        assert np.array_equal(got, want), (n, deg, k, refl)
        assert np.array_equal(got, oracle.smp(n, s, d, host(V), reflexive=bool(refl))), (n, deg, k, refl)


def test_noalloc_limits(ctx):
    n = 1000
    s, d, R, V = case(ctx, n, 3.0, 5, 3)
    out = ctx.zeros(5, n)
    ctx.smp_noalloc(R, n, V[:0], out[:0])  # k = 0: nothing to do
    with pytest.raises(B.BmlpError) as e:
        ctx.smp_noalloc(R, n, V, V)  # the answer overlaps the query rows
    assert e.value.status == B.EALIAS
    # n beyond the one-launch kernel is refused on the host, before any device work
    import ctypes
    big = 140000
    small = ctx.zeros(1, 64)
    p = ctypes.c_void_p(small.data_ptr())
    q = ctypes.c_void_p(out.data_ptr())
    rc = B.lib().bmlp_smp_noalloc(ctx._h, p, big, B.words(big), p, q, 1, B.words(big), 0, None)
    assert rc == B.EINVAL and b"n <= 131072" in B.lib().bmlp_last_error()
    # an edge index larger than the array: an all-ones relation of 8,192 nodes has 67 M edges
    n = 8192
    Rf = torch.full((n, n // 64), -1, dtype=torch.int64, device="cuda")
    Vf = ctx.zeros(2, n)
    outf = ctx.zeros(2, n)
    outf.fill_(7)
    with pytest.raises(B.BmlpError) as e:
        ctx.smp_noalloc(Rf, n, Vf, outf)
    assert e.value.status == B.ENOMEM
    assert (host(outf) == 7).all()  # nothing written
