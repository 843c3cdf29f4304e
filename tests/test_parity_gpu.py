"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
bit-exact, on seeded inputs.  Sizes span several tiles and ragged tails; the
n = 16,384 density-sweep graphs are checked on sampled rows."""
import math
import os

import numpy as np
import pytest

import gen
import oracle
from oracle import boolops

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2408_10369_amd as B  # noqa: E402

ARMS_SMP = [B.ARM_SMP_DENSE, B.ARM_SMP_SPARSE, B.ARM_SMP_CLOSURE, B.ARM_SMP_CLOSURE_SELECT]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = B.Context(0)
    yield c
    c.close()


def dev(bits):
    return torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint64).view(np.int64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def gpu_pack(ctx, n, s, d, ld=None):
    return ctx.pack_coo(torch.as_tensor(np.asarray(s, np.int32)), torch.as_tensor(np.asarray(d, np.int32)), n, n, ld)


def rand_graph(rng, n, p):
    A = (rng.random((n, n)) < p).astype(np.uint8)
    s, d = np.nonzero(A)
    return A, s.astype(np.int32), d.astype(np.int32)


def forced(**kw):
    return B.make_opts(dispatch=B.DISPATCH_FORCED, **kw)


SIZES = [1, 2, 3, 63, 64, 65, 127, 129, 200, 513, 1000, 1100]


# ----------------------------------------------------------------- packing and operators
@pytest.mark.parametrize("n", [1, 63, 64, 65, 130, 1000])
def test_pack_coo_and_u8(ctx, n):
    rng = np.random.default_rng(n)
    A, s, d = rand_graph(rng, n, 0.05)
    for ld in (max(boolops.words(n), 1), boolops.words(n) + 3):
        want = boolops.to_bits(A, ld=ld)
        assert np.array_equal(host(gpu_pack(ctx, n, s, d, ld)), want)
        got = host(ctx.pack_u8(torch.from_numpy(A).cuda(), ld=ld))
        assert np.array_equal(got, want)
        unp = ctx.unpack_u8(dev(want), n)
        assert np.array_equal(unp.cpu().numpy(), A)


@pytest.mark.parametrize("n", [1, 64, 65, 200, 1000])
def test_elementwise_and_transpose(ctx, n):
    rng = np.random.default_rng(10 + n)
    rows = n + 7
    X = (rng.random((rows, n)) < 0.3).astype(np.uint8)
    Y = (rng.random((rows, n)) < 0.3).astype(np.uint8)
    ld = boolops.words(n) + 1
    bx, by = dev(boolops.to_bits(X, ld)), dev(boolops.to_bits(Y, ld))
    assert np.array_equal(host(ctx.or_(bx, by, n)), boolops.to_bits(boolops.add(X, Y), ld))
    assert np.array_equal(host(ctx.and_(bx, by, n)), boolops.to_bits(boolops.land(X, Y), ld))
    assert np.array_equal(host(ctx.andnot(bx, by, n)), boolops.to_bits(X & (1 - Y), ld))
    assert np.array_equal(host(ctx.not_(bx, n)), boolops.to_bits(boolops.neg(X), ld))
    for ldt in (boolops.words(rows), boolops.words(rows) + 2):
        got = host(ctx.transpose(bx, n, ldat=ldt))
        assert np.array_equal(got, boolops.to_bits(boolops.transp(X), ldt))


@pytest.mark.parametrize("rows,cols", [(1, 1), (1, 5000), (5000, 1), (511, 1025), (513, 1023), (1500, 3000),
                                       (4100, 70), (33, 9000), (2048, 2048)])
def test_transpose_tiles(ctx, rows, cols):
    """Transposes spanning several 512-row x 1,024-column tiles, ragged in both directions."""
    rng = np.random.default_rng(rows * 31 + cols)
    X = (rng.random((rows, cols)) < 0.2).astype(np.uint8)
    ld = boolops.words(cols) + (cols % 3)
    bx = dev(boolops.to_bits(X, ld))
    for ldt in (boolops.words(rows), boolops.words(rows) + 1):
        got = host(ctx.transpose(bx, cols, ldat=ldt))
        assert np.array_equal(got, boolops.to_bits(boolops.transp(X), ldt)), (rows, cols, ldt)


@pytest.mark.parametrize("arm", [B.ARM_PRODUCT_VALU, B.ARM_PRODUCT_MFMA])
@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 70, 3), (64, 64, 64), (65, 129, 200), (130, 1000, 70),
                                   (300, 77, 4100), (1000, 1000, 1000)])
def test_product(ctx, arm, shape):
    m, k, n = shape
    rng = np.random.default_rng(m * 7 + k * 3 + n)
    A = (rng.random((m, k)) < 0.02).astype(np.uint8)
    Bm = (rng.random((k, n)) < 0.05).astype(np.uint8)
    Co = (rng.random((m, n)) < 0.01).astype(np.uint8)
    o = forced(product_arm=arm)
    ba, bb = dev(boolops.to_bits(A)), dev(boolops.to_bits(Bm))
    got = host(ctx.product(ba, bb, k, n, opts=o))
    assert np.array_equal(got, boolops.to_bits(boolops.mul(A, Bm)))
    bc = dev(boolops.to_bits(Co))
    got = host(ctx.product(ba, bb, k, n, Cold=bc, opts=o))
    assert np.array_equal(got, boolops.to_bits(boolops.add(Co, boolops.mul(A, Bm))))
    # in place: C = Cold
    ctx.product(ba, bb, k, n, Cold=bc, out=bc, opts=o)
    assert np.array_equal(host(bc), got)
    # dense operands
    A2 = (rng.random((m, k)) < 0.5).astype(np.uint8)
    B2 = (rng.random((k, n)) < 0.5).astype(np.uint8)
    got = host(ctx.product(dev(boolops.to_bits(A2)), dev(boolops.to_bits(B2)), k, n, opts=o))
    assert np.array_equal(got, boolops.to_bits(boolops.mul(A2, B2)))


def test_product_mfma_skipped_words(ctx):
    # k-words that are zero in every row of a 128-row block are skipped by the matrix-core arm;
    # a pattern that differs per row block and per word exercises mixed skip masks
    m, k, n = 600, 64 * 40, 300
    rng = np.random.default_rng(4242)
    A = (rng.random((m, k)) < 0.05).astype(np.uint8)
    for r in range(m):
        for w in range(k // 64):
            if (w + r // 128) % 3 != 0 or (w % 8 == 7 and r // 128 == 1):
                A[r, 64 * w:64 * w + 64] = 0
    Bm = (rng.random((k, n)) < 0.05).astype(np.uint8)
    want = boolops.to_bits(boolops.mul(A, Bm))
    for arm in (B.ARM_PRODUCT_VALU, B.ARM_PRODUCT_MFMA):
        got = host(ctx.product(dev(boolops.to_bits(A)), dev(boolops.to_bits(Bm)), k, n, opts=forced(product_arm=arm)))
        assert np.array_equal(got, want), arm


@pytest.mark.parametrize("inplace", [False, True])
def test_product_mfma_saturated_tiles(ctx, inplace):
    # output tiles whose C_old bits are all set are copied without a product; a tile one bit short
    # of full, and a full ragged corner tile, sit beside them
    m, k, n = 700, 300, 600
    rng = np.random.default_rng(99)
    A = (rng.random((m, k)) < 0.02).astype(np.uint8)
    Bm = (rng.random((k, n)) < 0.02).astype(np.uint8)
    Co = (rng.random((m, n)) < 0.01).astype(np.uint8)
    Co[0:256, 0:256] = 1
    Co[256:512, 256:512] = 1
    Co[300, 400] = 0
    Co[512:, 512:] = 1
    Co[0:256, 512:] = 1
    want = boolops.to_bits(boolops.add(Co, boolops.mul(A, Bm)))
    bc = dev(boolops.to_bits(Co))
    o = forced(product_arm=B.ARM_PRODUCT_MFMA)
    got = host(ctx.product(dev(boolops.to_bits(A)), dev(boolops.to_bits(Bm)), k, n, Cold=bc,
                           out=bc if inplace else None, opts=o))
    assert np.array_equal(got, want)


def test_product_mfma_longest_k(ctx):
    # all-ones operands at the largest K the matrix-core arm accepts (65,536 words): every fp32 sum
    # takes its largest value and must still be exact and read as "> 0"; one word more is refused
    kw = 65536
    k = 64 * kw
    A = torch.full((256, kw), -1, dtype=torch.int64, device="cuda")
    Bm = torch.full((k, 4), -1, dtype=torch.int64, device="cuda")
    got = host(ctx.product(A, Bm, k, 256, opts=forced(product_arm=B.ARM_PRODUCT_MFMA)))
    assert (got == np.uint64(0xFFFFFFFFFFFFFFFF)).all()
    # a single witness at the far end of k
    A.zero_()
    Bm.zero_()
    A[5, kw - 1] = -(1 << 63)  # bit 63 of the last word
    Bm[k - 1, 2] = 1 << 7
    got = host(ctx.product(A, Bm, k, 256, opts=forced(product_arm=B.ARM_PRODUCT_MFMA)))
    want = np.zeros((256, 4), np.uint64)
    want[5, 2] = np.uint64(1 << 7)
    assert np.array_equal(got, want)
    del A, Bm
    A1 = torch.zeros((256, kw + 1), dtype=torch.int64, device="cuda")
    B1 = torch.zeros((k + 64, 4), dtype=torch.int64, device="cuda")
    with pytest.raises(B.BmlpError) as e:
        ctx.product(A1, B1, k + 64, 256, opts=forced(product_arm=B.ARM_PRODUCT_MFMA))
    assert e.value.status == B.EINVAL


# ----------------------------------------------------------------- RMS
@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("n", SIZES)
def test_rms_random(ctx, n, variant):
    rng = np.random.default_rng(1000 + n)
    for p in (1.5 / n, 4.0 / n, 0.3):
        A, s, d = rand_graph(rng, n, min(p, 1.0))
        R = gpu_pack(ctx, n, s, d)
        st = {}
        got = host(ctx.rms(R, n, opts=B.make_opts(rms_variant=variant), stats=st))
        want = oracle.closure_rows(n, s, d)
        assert np.array_equal(got, want), (n, p, variant)
        assert 1 <= st["iterations"] <= math.ceil(math.log2(max(n, 2))) + 2


def test_rms_first_config(ctx):
    n, s, d, _ = gen.c1()
    R = gpu_pack(ctx, n, s, d)
    want = oracle.closure_rows(n, s, d)
    for variant in (0, 1):
        for parm in (B.ARM_PRODUCT_VALU, B.ARM_PRODUCT_MFMA):
            got = host(ctx.rms(R, n, opts=B.make_opts(rms_variant=variant, product_arm=parm)))
            assert np.array_equal(got, want), (variant, parm)


@pytest.mark.parametrize("n", [1, 65, 257, 700, 2100])
def test_rms_mfma_arm(ctx, n):
    rng = np.random.default_rng(4000 + n)
    for p in (1.5 / n, 0.05):
        A, s, d = rand_graph(rng, n, min(p, 1.0))
        R = gpu_pack(ctx, n, s, d)
        st = {}
        got = host(ctx.rms(R, n, opts=B.make_opts(product_arm=B.ARM_PRODUCT_MFMA), stats=st))
        assert np.array_equal(got, oracle.closure_rows(n, s, d)), (n, p)


def test_rms_dense_relation_early_votes(ctx):
    """A dense relation (a quarter or more of its bits set): its matrix-core squarings vote on saturation
    right after the first chunk of k.  Tiles saturated there stop; rows empty over the first 640 columns get
    nothing from that chunk and go on through the pipeline (saturated at the next vote); columns with no
    edge into them never saturate and run the whole of k.  The closure is compared with Warshall's
    algorithm."""
    n = 2048
    rng = np.random.default_rng(5)
    A = (rng.random((n, n)) < 0.9).astype(np.uint8)
    A[:, :256] = 0
    A[1024:, :640] = 0
    s, d = np.nonzero(A)
    R = gpu_pack(ctx, n, s.astype(np.int32), d.astype(np.int32))
    st = {}
    got = host(ctx.rms(R, n, stats=st))
    assert np.array_equal(got, oracle.warshall(boolops.to_bits(A), n))
    assert st["iterations"] == 2


def test_rms_stops_at_all_ones(ctx):
    """An all-ones relation is its own square: once a squaring leaves R full, the fixpoint is reached
    without the squaring that would only confirm it."""
    n = 2048
    rng = np.random.default_rng(6)
    A = (rng.random((n, n)) < 0.5).astype(np.uint8)
    s, d = np.nonzero(A)
    R = gpu_pack(ctx, n, s.astype(np.int32), d.astype(np.int32))
    st = {}
    got = host(ctx.rms(R, n, stats=st))
    want = oracle.warshall(boolops.to_bits(A), n)
    assert np.array_equal(got, want)
    assert np.array_equal(boolops.from_bits(want, n), np.ones((n, n), np.uint8))
    assert st["iterations"] == 1


@pytest.mark.parametrize("n", [2, 3, 5, 9, 17, 100, 1000, 1025])
def test_rms_path_graph_loop_counts(ctx, n):
    s, d = gen.path_graph(n)
    R = gpu_pack(ctx, n, s, d)
    st = {}
    got = host(ctx.rms(R, n, stats=st))
    assert np.array_equal(got, oracle.closure_rows(n, s, d))
    # squarings (by the product kernels or, while R is sparse, by row gathers)
    assert st["iterations"] == math.ceil(math.log2(n - 1)) + 1
    assert st["products"] + st["arm_trace"].count(B.ARM_PRODUCT_GATHER) == st["iterations"]
    # the timed gather squarings and their algorithmic bytes: squaring t reads the n rows of R_t = R + ..
    # + R^(2^t), whose bits are the paths of length 1 .. 2^t, one source row per bit, and writes n rows
    bits = [sum(n - j for j in range(1, min(2 ** t, n - 1) + 1)) for t in range(st["iterations"])]
    want = sum((2 * n + bits[t]) * ((n + 7) // 8) for t, a in enumerate(st["arm_trace"]) if a == B.ARM_PRODUCT_GATHER)
    assert st["gathers"] == st["arm_trace"].count(B.ARM_PRODUCT_GATHER)
    assert st["gather_bytes"] == want, (st["gather_bytes"], want)
    assert (st["gather_ms"] > 0) == (st["gathers"] > 0)
    st1 = {}
    ctx.rms(R, n, opts=B.make_opts(rms_variant=1), stats=st1)
    assert st1["iterations"] == math.ceil(math.log2(n - 1)) + 1
    # plus Algorithm 1's final product by R1
    assert st1["products"] + st1["arm_trace"].count(B.ARM_PRODUCT_GATHER) == st1["iterations"] + 1
    for parm in (B.ARM_PRODUCT_VALU, B.ARM_PRODUCT_MFMA):
        st2 = {}
        ctx.rms(R, n, opts=B.make_opts(product_arm=parm), stats=st2)
        assert st2["products"] == st2["iterations"] == math.ceil(math.log2(n - 1)) + 1


def test_rms_seminaive_squaring(ctx):
    """A sparse random digraph at n = 8,192 (mean degree 1.6): its last squaring adds 3,684 bits spread
    over 159 rows, so the next is done from them (R | D.R | R.D) with R.D = (D^T . R^T)^T by a second
    gather, rather than as a dense product.  Whole closure checked."""
    n = 8192
    s, d = gen.er_digraph(n, 2e-4, 5)
    R = gpu_pack(ctx, n, s, d)
    st = {}
    got = host(ctx.rms(R, n, stats=st))
    tr = st["arm_trace"]
    assert B.ARM_PRODUCT_SEMINAIVE_T in tr, tr
    assert st["products"] + tr.count(B.ARM_PRODUCT_GATHER) + tr.count(B.ARM_PRODUCT_SEMINAIVE_T) == st["iterations"]
    assert np.array_equal(got, oracle.closure_rows(n, s, d))
    # the same closure with every squaring a dense product
    got2 = host(ctx.rms(R, n, opts=B.make_opts(product_arm=B.ARM_PRODUCT_MFMA)))
    assert np.array_equal(got, got2)


def test_rms_seminaive_both_routes(ctx):
    """A chain of 200 nodes into a strongly connected core of 3,000 (n = 8,192): late squarings add the
    whole core to a few chain rows, so R.D goes through the nonempty rows of D (a product with K = those
    rows), while an earlier squaring whose new bits are spread thin takes the transposed gather.  Whole
    closure checked against the oracle and against all-dense squarings."""
    n = 8192
    s, d = gen.tail_core(n, 3000, 200, 3.0, 11)
    R = gpu_pack(ctx, n, s, d)
    st = {}
    got = host(ctx.rms(R, n, stats=st))
    tr = st["arm_trace"]
    print("tail_core arm trace", tr, flush=True)
    assert B.ARM_PRODUCT_SEMINAIVE in tr and B.ARM_PRODUCT_SEMINAIVE_T in tr, tr
    assert np.array_equal(got, oracle.closure_rows(n, s, d))
    assert np.array_equal(got, host(ctx.rms(R, n, opts=B.make_opts(product_arm=B.ARM_PRODUCT_MFMA))))
    # with a leading dimension beyond the words of a row (padding words must stay zero)
    ld = boolops.words(n) + 3
    R2 = ctx.pack_coo(torch.as_tensor(s), torch.as_tensor(d), n, n, ld)
    got2 = host(ctx.rms(R2, n))
    assert np.array_equal(got2[:, :boolops.words(n)], got) and not got2[:, boolops.words(n):].any()


def test_rms_special_graphs(ctx):
    for n in (1, 64, 65, 300):
        cs, cd = gen.cycle_graph(n)
        got = host(ctx.rms(gpu_pack(ctx, n, cs, cd), n))
        assert np.array_equal(got, boolops.to_bits(np.ones((n, n), np.uint8)))
        got = host(ctx.rms(ctx.zeros(n, n), n))
        assert not got.any()
        i = n // 2
        got = host(ctx.rms(gpu_pack(ctx, n, [i], [i]), n))
        want = np.zeros((n, n), np.uint8)
        want[i, i] = 1
        assert np.array_equal(got, boolops.to_bits(want))


def test_rms_padding_words_zeroed(ctx):
    n = 100
    rng = np.random.default_rng(3)
    A, s, d = rand_graph(rng, n, 0.03)
    ld = boolops.words(n) + 5
    R = gpu_pack(ctx, n, s, d, ld)
    out = torch.full((n, ld), -1, dtype=torch.int64, device="cuda")
    ctx.rms(R, n, out=out)
    assert np.array_equal(host(out), oracle.closure_rows(n, s, d, ld=ld))


# ----------------------------------------------------------------- SMP
@pytest.mark.parametrize("parm", [B.ARM_PRODUCT_VALU, B.ARM_PRODUCT_MFMA])
@pytest.mark.parametrize("reflexive", [0, 1])
@pytest.mark.parametrize("arm", ARMS_SMP)
@pytest.mark.parametrize("n", [1, 2, 63, 65, 129, 700, 2000])
def test_smp_random(ctx, n, arm, reflexive, parm):
    if parm == B.ARM_PRODUCT_MFMA and arm in (B.ARM_SMP_SPARSE, B.ARM_SMP_CLOSURE_SELECT):
        pytest.skip("the arm launches no product")
    rng = np.random.default_rng(2000 + n)
    for p in (1.2 / n, 5.0 / n):
        A, s, d = rand_graph(rng, n, min(p, 1.0))
        k = int(rng.integers(1, 40))
        V = np.zeros((k, n), np.uint8)
        V[np.arange(k), rng.integers(0, n, k)] = 1
        V[: k // 3] |= (rng.random((k // 3, n)) < 0.02).astype(np.uint8)  # some multi-source rows
        Vb = boolops.to_bits(V)
        R = gpu_pack(ctx, n, s, d)
        st = {}
        got = host(ctx.smp(R, n, dev(Vb), opts=forced(smp_arm=arm, smp_reflexive=reflexive, product_arm=parm),
                           stats=st))
        want = oracle.smp(n, s, d, Vb, reflexive=bool(reflexive))
        assert np.array_equal(got, want), (n, p, arm, reflexive)
        assert st["arm"] == arm


@pytest.mark.parametrize("n", [1, 2, 64, 65, 1000, 5000])
def test_rms_closure_by_selection(ctx, n):
    """bmlp_rms forced to the closure by selection, and under the learned schedule (which may pick either
    route): the oracle's closure, padding words zeroed."""
    rng = np.random.default_rng(777 + n)
    for p in (1.2 / max(n, 1), 4.0 / max(n, 1)):
        A, s, d = rand_graph(rng, n, min(p, 1.0))
        ld = (n + 63) // 64 + 3
        R = gpu_pack(ctx, n, s, d, ld)
        want = oracle.closure_rows(n, s, d, ld=ld)
        st = {}
        out = torch.full_like(R, -1)
        got = host(ctx.rms(R, n, out=out, opts=forced(smp_arm=B.ARM_SMP_CLOSURE_SELECT), stats=st))
        assert np.array_equal(got, want), (n, p)
        assert st["arm"] == B.ARM_SMP_CLOSURE_SELECT
        out.fill_(-1)
        assert np.array_equal(host(ctx.rms(R, n, out=out, opts=B.make_opts(dispatch=B.DISPATCH_LEARNED))), want)


@pytest.mark.parametrize("n", [1, 64, 65, 1000, 5000])
def test_closure_by_selection_is_the_closure(ctx, n):
    """The selection from every source (V = I) under the closure-by-selection arm returns R1+ itself,
    and the read-off of I, R1+ and R1* rows agrees with the oracle's closure."""
    rng = np.random.default_rng(4242 + n)
    for p in (1.5 / max(n, 1), 4.0 / max(n, 1)):
        A, s, d = rand_graph(rng, n, min(p, 1.0))
        R = gpu_pack(ctx, n, s, d)
        eye_bits = boolops.to_bits(boolops.identity(n))
        eye = dev(eye_bits)
        want = oracle.closure_rows(n, s, d)
        for refl in (0, 1):
            got = host(ctx.smp(R, n, eye, opts=forced(smp_arm=B.ARM_SMP_CLOSURE_SELECT, smp_reflexive=refl)))
            w = want | eye_bits if refl else want
            assert np.array_equal(got, w), (n, p, refl)


@pytest.mark.parametrize("reflexive", [0, 1])
@pytest.mark.parametrize("n", [700, 3000, 16384])
def test_smp_closure_heavy_query_rows(ctx, n, reflexive):
    """Query rows from empty to full read off the closure: rows with more than 64 set bits are split over
    several waves (the first 64 bits in place, the rest queued and ORed in with atomics)."""
    rng = np.random.default_rng(77 + n)
    s, d = gen.er_digraph(n, 2.5 / n, n)
    dens = [0.0, 1.0 / n, 0.01, 0.05, 0.3, 0.9, 1.0]
    k = 3 * len(dens)
    V = np.zeros((k, n), np.uint8)
    for i in range(k):
        V[i] = rng.random(n) < dens[i % len(dens)]
    Vb = boolops.to_bits(V)
    R = gpu_pack(ctx, n, s, d)
    got = host(ctx.smp(R, n, dev(Vb), opts=forced(smp_arm=B.ARM_SMP_CLOSURE, smp_reflexive=reflexive)))
    want = oracle.smp(n, s, d, Vb, reflexive=bool(reflexive))
    assert np.array_equal(got, want), (n, reflexive)


@pytest.mark.parametrize("n,deg", [(4096, 5.0), (4096, 12.0), (9000, 40.0), (16384, 82.0)])
def test_smp_bottom_up_rounds(ctx, n, deg):
    """The one-launch arm turns bottom-up (in-edges of the unvisited nodes) once the frontier is large;
    its in-edge index is built from the CSR with atomics for a sparse relation (n = 4,096, degree 5) and
    through R^T otherwise.  Single sources, hubs of a skewed degree sequence and a reflexive call."""
    rng = np.random.default_rng(int(n + deg))
    s, d = gen.er_digraph(n, deg / n, int(deg * 100) + n)
    # a few hubs with a quarter of the nodes as successors
    hubs = rng.choice(n, 3, replace=False)
    hs = np.repeat(hubs, n // 4).astype(np.int32)
    hd = rng.integers(0, n, hs.size).astype(np.int32)
    s, d = np.r_[s, hs].astype(np.int32), np.r_[d, hd].astype(np.int32)
    k = 40
    V = np.zeros((k, n), np.uint8)
    V[np.arange(k), rng.integers(0, n, k)] = 1
    V[-5:] |= (rng.random((5, n)) < 0.01).astype(np.uint8)
    Vb = boolops.to_bits(V)
    R = gpu_pack(ctx, n, s, d)
    for refl in (0, 1):
        st = {}
        got = host(ctx.smp(R, n, dev(Vb), opts=forced(smp_arm=B.ARM_SMP_SPARSE, smp_reflexive=refl), stats=st))
        want = oracle.smp(n, s, d, Vb, reflexive=bool(refl))
        assert np.array_equal(got, want), (n, deg, refl, st.get("iterations"))


def test_smp_first_config(ctx):
    n, s, d, srcs = gen.c1()
    R = gpu_pack(ctx, n, s, d)
    r, c = gen.query_lists(srcs)
    V = ctx.pack_coo(torch.as_tensor(r), torch.as_tensor(c), len(srcs), n)
    want = oracle.smp(n, s, d, host(V))
    for arm in ARMS_SMP:
        assert np.array_equal(host(ctx.smp(R, n, V, opts=forced(smp_arm=arm))), want), arm


def test_smp_path_rounds(ctx):
    n = 300
    s, d = gen.path_graph(n)
    R = gpu_pack(ctx, n, s, d)
    V = ctx.pack_coo(torch.tensor([0], dtype=torch.int32), torch.tensor([0], dtype=torch.int32), 1, n)
    for arm in (B.ARM_SMP_DENSE, B.ARM_SMP_SPARSE):
        st = {}
        got = host(ctx.smp(R, n, V, opts=forced(smp_arm=arm), stats=st))
        want = np.r_[0, np.ones(n - 1, np.uint8)][None, :]
        assert np.array_equal(got, boolops.to_bits(want))
        # Algorithm 2 from node 0 of a path runs n rounds; the semi-naive form reaches the same
        # fixpoint in n - 1 expansions plus the empty one
        assert st["iterations"] == n


def test_smp_hub_node(ctx):
    # a star with a high out-degree centre exercises the cooperative (hub) expansion and the
    # dense-row path of the sparse kernel
    n = 5000
    hub_s = np.zeros(n - 1, np.int32)
    hub_d = np.arange(1, n, dtype=np.int32)
    chain_s = np.arange(1, 200, dtype=np.int32)
    chain_d = chain_s + 1
    s = np.r_[hub_s, chain_s, [4999]].astype(np.int32)
    d = np.r_[hub_d, chain_d, [0]].astype(np.int32)
    R = gpu_pack(ctx, n, s, d)
    V = ctx.pack_coo(torch.tensor([0, 1, 2], dtype=torch.int32), torch.tensor([0, 7, 4999], dtype=torch.int32), 3, n)
    want = oracle.smp(n, s, d, host(V))
    for arm in ARMS_SMP:
        assert np.array_equal(host(ctx.smp(R, n, V, opts=forced(smp_arm=arm))), want), arm


# ----------------------------------------------------------------- composition
@pytest.mark.parametrize("parm", [B.ARM_PRODUCT_VALU, B.ARM_PRODUCT_MFMA])
@pytest.mark.parametrize("arm", [B.ARM_COMPOSE_RMS, B.ARM_COMPOSE_SEMINAIVE, B.ARM_COMPOSE_ROWWISE])
@pytest.mark.parametrize("n", [1, 3, 64, 65, 300, 1000])
def test_compose_random(ctx, n, arm, parm):
    rng = np.random.default_rng(3000 + n)
    for pb, ps in ((0.01, 1.5 / n), (0.002, 3.0 / n), (0.2, 0.01)):
        Bm, bs, bd = rand_graph(rng, n, min(pb, 1.0))
        S, ss, sd = rand_graph(rng, n, min(ps, 1.0))
        got = host(ctx.compose_linear(gpu_pack(ctx, n, bs, bd), gpu_pack(ctx, n, ss, sd), n,
                                      opts=forced(compose_arm=arm, product_arm=parm)))
        assert np.array_equal(got, oracle.compose_rows(n, bs, bd, ss, sd)), (n, pb, ps, arm)


@pytest.mark.parametrize("sarm", [B.ARM_SMP_DENSE, B.ARM_SMP_SPARSE, B.ARM_SMP_CLOSURE, B.ARM_SMP_SPARSE_ROUNDS])
def test_compose_rowwise_selection_arms(ctx, sarm):
    # the row-wise route under every selection arm; a padded leading dimension, rows of the step
    # relation without edges (copied from the base), a hub row and a long chain
    rng = np.random.default_rng(515)
    n, ld = 777, 16
    _, bs, bd = rand_graph(rng, n, 0.004)
    _, ss, sd = rand_graph(rng, n, 0.0008)
    ss = np.r_[ss, np.zeros(300, np.int32), np.arange(400, 700, dtype=np.int32)].astype(np.int32)
    sd = np.r_[sd, rng.choice(n, 300, replace=False).astype(np.int32), np.arange(401, 701, dtype=np.int32)]
    keep = np.unique(ss.astype(np.int64) * n + sd, return_index=True)[1]
    ss, sd = ss[keep], sd[keep]
    out = ctx.zeros(n, n, ld)
    out.fill_(-1)  # every word of the output is written, padding words included
    P = host(ctx.compose_linear(gpu_pack(ctx, n, bs, bd, ld), gpu_pack(ctx, n, ss, sd, ld), n, out=out,
                                opts=forced(compose_arm=B.ARM_COMPOSE_ROWWISE, smp_arm=sarm)))
    nw = (n + 63) // 64
    assert not P[:, nw:].any()
    assert np.array_equal(P[:, :nw], oracle.compose_rows(n, bs, bd, ss, sd)), sarm


def test_compose_rowwise_empty_step(ctx):
    rng = np.random.default_rng(516)
    n = 300
    _, bs, bd = rand_graph(rng, n, 0.01)
    got = host(ctx.compose_linear(gpu_pack(ctx, n, bs, bd), ctx.zeros(n, n), n,
                                  opts=forced(compose_arm=B.ARM_COMPOSE_ROWWISE)))
    none = np.zeros(0, np.int32)
    assert np.array_equal(got, oracle.compose_rows(n, bs, bd, none, none))


def test_compose_of_same_relation_is_closure(ctx):
    n, s, d, _ = gen.c1()
    R = gpu_pack(ctx, n, s, d)
    for arm in (B.ARM_COMPOSE_RMS, B.ARM_COMPOSE_SEMINAIVE, B.ARM_COMPOSE_ROWWISE):
        got = host(ctx.compose_linear(R, R, n, opts=forced(compose_arm=arm)))
        assert np.array_equal(got, oracle.closure_rows(n, s, d))


def test_isforeign_pipeline(ctx, golden_dir):
    """The paper's composition example, run entirely through the GPU operators."""
    path = os.path.join(golden_dir, "isforeign_example.txt")
    consts, facts = None, {"contains": [], "adjoins": [], "false": []}
    for line in open(path):
        line = line.split("#", 1)[0].split()
        if not line:
            continue
        if line[0] == "constants":
            consts = line[1:]
        else:
            facts[line[0]].append(line[1:])
    idx = {c: i for i, c in enumerate(consts)}
    n = len(consts)

    def pack(pairs):
        s = [idx[a] for a, b in pairs]
        d = [idx[b] for a, b in pairs]
        return gpu_pack(ctx, n, s, d)

    has_place = ctx.rms(pack(facts["contains"]), n)
    adj = pack(facts["adjoins"])
    base = ctx.or_(adj, ctx.transpose(adj, n), n)
    step = ctx.transpose(has_place, n)
    for arm in (B.ARM_COMPOSE_RMS, B.ARM_COMPOSE_SEMINAIVE, B.ARM_COMPOSE_ROWWISE):
        ipo = ctx.compose_linear(base, step, n, opts=forced(compose_arm=arm))
        foreign = ctx.unpack_u8(ctx.not_(ipo, n), n).cpu().numpy()
        want = np.ones((n, n), np.uint8)
        for a, b in facts["false"]:
            want[idx[a], idx[b]] = 0
        assert np.array_equal(foreign, want)


# ----------------------------------------------------------------- full-size density sweep (sampled)
@pytest.mark.parametrize("parm", [B.ARM_AUTO, B.ARM_PRODUCT_VALU, B.ARM_PRODUCT_MFMA])
@pytest.mark.parametrize("pi", [0, 2, 4])
def test_density_sweep_rms_sampled_rows(ctx, pi, parm):
    n, s, d = gen.c2(pi)
    R = gpu_pack(ctx, n, s, d)
    got = host(ctx.rms(R, n, opts=B.make_opts(product_arm=parm)))
    rng = np.random.default_rng(77 + pi)
    rows = np.sort(rng.choice(n, 96, replace=False))
    assert np.array_equal(got[rows], oracle.closure_rows(n, s, d, rows=rows))
    # R1 is contained in R1+ on every row
    r1 = host(R)
    assert not np.any(r1 & ~got)


@pytest.mark.parametrize("case", ["sweep_p1e-4", "tail_core", "n20000", "n66000"])
def test_rms_relabelled_closure_whole(ctx, case):
    """Relations with a tenth or more empty rows at n >= 16,384 are relabelled (nodes grouped by heavy /
    light row and column classes) before their dense squarings and mapped back at the end: the whole
    closure must equal the one squared in the given order (every squaring forced onto the matrix cores,
    which never relabels) and, on sampled rows, the oracle's."""
    if case == "tail_core":
        n = 16384
        s, d = gen.tail_core(n, 5000, 300, 2.5, 13)
    elif case == "n20000":  # rows of 313 words: the relabelling stages four rows per workgroup
        n = 20000
        s, d = gen.er_digraph(n, 1.7 / n, 20000)
    elif case == "n66000":  # rows of 1,032 words: one staged row per workgroup
        n = 66000
        s, d = gen.er_digraph(n, 1.7 / n, 66000)
    else:
        n, s, d = gen.c2(0)
    R = gpu_pack(ctx, n, s, d)
    got = host(ctx.rms(R, n))
    plain = host(ctx.rms(R, n, opts=B.make_opts(product_arm=B.ARM_PRODUCT_MFMA)))
    assert np.array_equal(got, plain)
    rows = np.sort(np.random.default_rng(5).choice(n, 64, replace=False))
    assert np.array_equal(got[rows], oracle.closure_rows(n, s, d, rows=rows))


@pytest.mark.parametrize("pi", [0, 2, 4])
def test_density_sweep_smp(ctx, pi):
    n, s, d = gen.c2(pi)
    R = gpu_pack(ctx, n, s, d)
    srcs = gen.c2_sources(pi, 1)
    r, c = gen.query_lists(srcs)
    V = ctx.pack_coo(torch.as_tensor(r), torch.as_tensor(c), len(srcs), n)
    want = oracle.smp(n, s, d, host(V))
    for arm in (B.ARM_SMP_DENSE, B.ARM_SMP_SPARSE):
        assert np.array_equal(host(ctx.smp(R, n, V, opts=forced(smp_arm=arm))), want), arm


# ----------------------------------------------------------------- boundary behaviour
def test_errors(ctx):
    n = 100
    R = ctx.zeros(n, n)
    with pytest.raises(B.BmlpError) as e:
        ctx.rms(R, n, out=R)
    assert e.value.status == B.EALIAS
    bad = torch.zeros((n, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(B.BmlpError) as e:
        ctx.rms(bad, n, out=torch.zeros_like(bad))
    assert e.value.status == B.EINVAL
    P = ctx.zeros(n, n)
    P[0, 1] = 1 << 40  # column 104 >= n: a padding bit
    with pytest.raises(B.BmlpError) as e:
        ctx.rms(P, n, opts=B.make_opts(check_padding=1))
    assert e.value.status == B.EPAD
    with pytest.raises(B.BmlpError) as e:
        ctx.pack_coo(torch.tensor([0, 5], dtype=torch.int32), torch.tensor([1, n], dtype=torch.int32), n, n)
    assert e.value.status == B.EINVAL
    with pytest.raises(B.BmlpError) as e:
        ctx.smp(R, n, ctx.zeros(2, n), opts=forced(smp_arm=B.ARM_COMPOSE_RMS))
    assert e.value.status == B.EINVAL
    with pytest.raises(B.BmlpError) as e:
        ctx.compose_linear(R, R, n, opts=forced(compose_arm=B.ARM_SMP_DENSE))
    assert e.value.status == B.EINVAL
    with pytest.raises(B.BmlpError) as e:
        ctx.compose_linear(R, R, n, opts=forced(compose_arm=B.ARM_COMPOSE_ROWWISE, smp_arm=B.ARM_COMPOSE_RMS))
    assert e.value.status == B.EINVAL


def test_empty_sizes(ctx):
    z = torch.zeros((0, 1), dtype=torch.int64, device="cuda")
    ctx.rms(z, 0, out=torch.zeros_like(z))
    R = ctx.zeros(10, 10)
    out = ctx.smp(R, 10, ctx.zeros(0, 10))
    assert out.shape == (0, 1)
    V = ctx.zeros(3, 10)
    assert not host(ctx.smp(R, 10, V)).any()
