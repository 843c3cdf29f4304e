"""The autotuner and its candidates: every candidate tile code of the matrix-core and VALU products
gives the oracle's bits (products of ragged shapes, with and without C_old, in place, saturated tiles,
skipped words; closures by BMLP-RMS, including a relabelled block-structured one), the tuner keeps the
fastest candidate it measured per bucket, and its JSON cache round-trips and refuses another device's."""
import json
import os

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


def dev(bits, ld=None):
    b = np.ascontiguousarray(bits, dtype=np.uint64)
    if ld is not None and ld > b.shape[1]:
        b = np.concatenate([b, np.zeros((b.shape[0], ld - b.shape[1]), np.uint64)], axis=1)
    return torch.from_numpy(b.view(np.int64)).cuda()


def even(w):
    return w + (w & 1)


def forced(**kw):
    return B.make_opts(dispatch=B.DISPATCH_FORCED, **kw)


KERNELS = [(B.TUNE_MFMA_PRODUCT, B.ARM_PRODUCT_MFMA), (B.TUNE_VALU_PRODUCT, B.ARM_PRODUCT_VALU)]


def candidates():
    out = []
    for kern, arm in KERNELS:
        for v in range(B.Context.tune_candidates(kern)):
            out.append((kern, arm, v))
    return out


@pytest.mark.parametrize("kern,arm,v", candidates())
def test_candidate_products(ctx, kern, arm, v):
    ctx.tune_set(kern, -1, v)
    try:
        for (m, k, n) in [(1, 1, 1), (65, 129, 200), (300, 77, 4100), (513, 1000, 777), (1000, 2100, 1000)]:
            rng = np.random.default_rng(m + 3 * k + 7 * n + v)
            for pa, pb in ((0.02, 0.05), (0.5, 0.5), (0.0005, 0.3)):
                A = (rng.random((m, k)) < pa).astype(np.uint8)
                Bm = (rng.random((k, n)) < pb).astype(np.uint8)
                Co = (rng.random((m, n)) < 0.01).astype(np.uint8)
                Co[: min(m, 256), : min(n, 256)] = 1  # a saturated corner tile
                lda, ldb, ldc = even(boolops.words(k)), even(boolops.words(n)), even(boolops.words(n))
                ba, bb, bc = dev(boolops.to_bits(A), lda), dev(boolops.to_bits(Bm), ldb), dev(boolops.to_bits(Co), ldc)
                want = boolops.to_bits(boolops.mul(A, Bm), ldc)
                got = host(ctx.product(ba, bb, k, n, out=ctx.zeros(m, n, ldc), opts=forced(product_arm=arm)))
                assert np.array_equal(got, want), (m, k, n, pa, v)
                want_c = boolops.to_bits(boolops.add(Co, boolops.mul(A, Bm)), ldc)
                ctx.product(ba, bb, k, n, Cold=bc, out=bc, opts=forced(product_arm=arm))  # in place
                assert np.array_equal(host(bc), want_c), (m, k, n, pa, v, "in place")
    finally:
        ctx.tune_set(kern, -1, -1)


@pytest.mark.parametrize("kern,arm,v", candidates())
def test_candidate_closures(ctx, kern, arm, v):
    ctx.tune_set(kern, -1, v)
    try:
        for n, p in ((1100, 3.0 / 1100), (2000, 1.2 / 2000), (2048, 0.01)):
            s, d = gen.er_digraph(n, p, n + v)
            R = ctx.pack_coo(torch.as_tensor(s), torch.as_tensor(d), n, n)
            got = host(ctx.rms(R, n, opts=forced(product_arm=arm)))
            assert np.array_equal(got, oracle.closure_rows(n, s, d)), (n, p, v)
        if kern == B.TUNE_MFMA_PRODUCT:
            # the sparsest sweep graph: relabelled, block-structured squarings
            n, s, d = gen.c2(0)
            R = ctx.pack_coo(torch.as_tensor(s), torch.as_tensor(d), n, n)
            got = host(ctx.rms(R, n))
            rows = np.sort(np.random.default_rng(v).choice(n, 256, replace=False))
            assert np.array_equal(got[rows], oracle.closure_rows(n, s, d, rows=rows)), v
    finally:
        ctx.tune_set(kern, -1, -1)


def test_autotune_picks_fastest_and_cache_round_trip(ctx, tmp_path):
    path = str(tmp_path / "cache.json")
    rep = ctx.autotune(kernel_mask=1, reps=1, cache_out=path)
    nb = B.Context.tune_buckets(B.TUNE_MFMA_PRODUCT)
    nc = B.Context.tune_candidates(B.TUNE_MFMA_PRODUCT)
    chosen = []
    for b in range(nb):
        times = rep[B.TUNE_MFMA_PRODUCT][b][:nc]
        assert all(t > 0 for t in times), (b, times)
        v, ms = ctx.tune_get(B.TUNE_MFMA_PRODUCT, b)
        assert v == int(np.argmin(times)) and abs(ms - min(times)) < 1e-6
        chosen.append(v)
    # the VALU kernel was not in the mask: not measured, left at its default
    assert all(t == -1 for t in rep[B.TUNE_VALU_PRODUCT][0])
    doc = json.load(open(path))
    assert doc["format"] == "bmlp-autotune" and doc["kernels"][0]["choice"] == chosen
    # a fresh handle reads the cache back
    with B.Context(0) as c2:
        c2.tune_set(B.TUNE_MFMA_PRODUCT, -1, -1)
        c2.tune_load(path)
        assert [c2.tune_get(B.TUNE_MFMA_PRODUCT, b)[0] for b in range(nb)] == chosen
        # a cache written on another kind of device is refused and leaves the handle as it was
        doc["arch"] = "gfx000"
        other = str(tmp_path / "other.json")
        json.dump(doc, open(other, "w"))
        c2.tune_set(B.TUNE_MFMA_PRODUCT, -1, 0)
        with pytest.raises(B.BmlpError) as e:
            c2.tune_load(other)
        assert e.value.status == B.EMODEL
        assert all(c2.tune_get(B.TUNE_MFMA_PRODUCT, b)[0] == 0 for b in range(nb))


def test_shipped_cache_matches_device(ctx):
    """The cache shipped beside the library loads on this device (it is loaded by bmlp_create)."""
    path = os.path.join(os.path.dirname(B.LIB_PATH), "autotune_cache.json")
    if not os.path.exists(path):
        pytest.skip("no shipped tuning cache")
    with B.Context(0) as c2:
        c2.tune_load(path)
