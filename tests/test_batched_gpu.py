"""GPU parity of the batched launch (many graphs of uneven sizes, one hipGraph
launch): every closure and every query answer against the CPU oracle."""
import numpy as np
import pytest

import gen
import oracle

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


def make_batch(ctx, specs, with_closure=True):
    graphs, refs = [], []
    for (n, s, d, srcs) in specs:
        R = ctx.pack_coo(torch.as_tensor(np.asarray(s, np.int32)), torch.as_tensor(np.asarray(d, np.int32)), n, n)
        g = {"n": n, "R1": R}
        if with_closure:
            g["closure"] = torch.full_like(R, -1)
        if len(srcs):
            r, c = gen.query_lists(np.asarray(srcs, np.int32))
            g["V"] = ctx.pack_coo(torch.as_tensor(r), torch.as_tensor(c), len(srcs), n)
            g["Vstar"] = torch.full_like(g["V"], -1)
        graphs.append(g)
        refs.append((n, np.asarray(s), np.asarray(d)))
    return graphs, refs


def check(graphs, refs):
    for g, (n, s, d) in zip(graphs, refs):
        if "closure" in g:
            assert np.array_equal(host(g["closure"]), oracle.closure_rows(n, s, d, ld=g["closure"].shape[1])), n
        if "V" in g:
            assert np.array_equal(host(g["Vstar"]), oracle.smp(n, s, d, host(g["V"]))), n


MODES = {"plain": None, "learned": "learned", "closure": "closure"}


def mode_opts(mode):
    if mode == "learned":
        return B.make_opts(dispatch=B.DISPATCH_LEARNED)
    if mode == "closure":
        return B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_CLOSURE)
    return None


@pytest.mark.parametrize("mode", list(MODES))
def test_batched_mixed_sizes(ctx, mode):
    rng = np.random.default_rng(11)
    specs = []
    for n in [1, 2, 63, 64, 65, 129, 300, 700, 1100, 2049, 5, 40]:
        A = (rng.random((n, n)) < min(2.5 / n, 1.0)).astype(np.uint8)
        s, d = np.nonzero(A)
        k = int(rng.integers(0, min(n, 70) + 1))
        specs.append((n, s, d, rng.choice(n, k, replace=False) if k else []))
    graphs, refs = make_batch(ctx, specs)
    st = {}
    ctx.batched(graphs, opts=mode_opts(mode), stats=st)
    check(graphs, refs)
    assert st["iterations"] >= 1 and st["bool_ops"] > 0


@pytest.mark.parametrize("mode", ["plain", "closure"])
def test_batched_dense_blocks(ctx, mode):
    """Dense graphs (30% of the pairs) square on the matrix cores.  No edge enters the first 128 columns,
    so those outputs never saturate and their tiles run the whole of k; rows of the lower half are empty
    over the first 384 columns, so the first chunks of k add nothing to them; a 700-node graph has partial
    tiles, which never vote on saturation."""
    rng = np.random.default_rng(21)
    specs = []
    for n in (1024, 1536, 1024, 700):
        A = (rng.random((n, n)) < 0.3).astype(np.uint8)
        A[:, :128] = 0
        A[n // 2:, :384] = 0
        s, d = np.nonzero(A)
        specs.append((n, s, d, rng.choice(n, 40, replace=False)))
    graphs, refs = make_batch(ctx, specs)
    ctx.batched(graphs, opts=mode_opts(mode))
    check(graphs, refs)


@pytest.mark.parametrize("mode", ["plain", "learned"])
def test_batched_matrix_core_graphs(ctx, mode):
    # graphs at and above the matrix-core size: dense from the first round, ragged (n not a multiple
    # of 256 or 64), and one whose first 256-row block is empty while the others are dense, so row
    # blocks of one graph take different kernels in the same round; small graphs beside them
    rng = np.random.default_rng(21)
    specs = []
    for n, p in ((1024, 0.03), (1300, 0.02), (2049, 1.5 / 2049), (1500, 0.0)):
        A = (rng.random((n, n)) < p).astype(np.uint8)
        if p == 0.0:
            A = (rng.random((n, n)) < 0.01).astype(np.uint8)
            A[:256, :] = 0
            A[300, 5] = 1  # a path into the empty block's columns
        s, d = np.nonzero(A)
        specs.append((n, s, d, rng.choice(n, 40, replace=False)))
    for n in (70, 500, 1023):
        ss, dd = gen.er_digraph(n, 3.0 / n, int(rng.integers(1 << 30)))
        specs.append((n, ss, dd, rng.choice(n, 10, replace=False)))
    graphs, refs = make_batch(ctx, specs)
    ctx.batched(graphs, opts=mode_opts(mode))
    check(graphs, refs)


def test_batched_reuses_and_rereads_inputs(ctx):
    rng = np.random.default_rng(12)
    specs = []
    for n in (100, 500, 70):
        s, d = gen.er_digraph(n, 2.0 / n, int(rng.integers(1 << 30)))
        specs.append((n, s, d, rng.choice(n, 9, replace=False)))
    graphs, refs = make_batch(ctx, specs)
    ctx.batched(graphs)
    check(graphs, refs)
    # same descriptors, new contents in place: the cached launch reads the new relation
    n = 500
    s2, d2 = gen.path_graph(n)
    ctx.pack_coo(torch.as_tensor(s2), torch.as_tensor(d2), n, n, out=graphs[1]["R1"])
    refs[1] = (n, s2, d2)
    for g in graphs:
        g["closure"].fill_(-1)
        if "Vstar" in g:
            g["Vstar"].fill_(-1)
    ctx.batched(graphs)
    check(graphs, refs)


def test_batched_edge_cases(ctx):
    graphs = [{"n": 0, "R1": torch.zeros((0, 1), dtype=torch.int64, device="cuda")}]
    specs = [(50, [0, 1], [1, 2], []), (64, [], [], [0, 5])]
    g2, refs = make_batch(ctx, specs)
    g2[0].pop("closure")  # answers only / closure only mixes
    graphs += g2
    ctx.batched(graphs)
    assert np.array_equal(host(g2[1]["closure"]), np.zeros((64, 1), np.uint64))
    assert not host(g2[1]["Vstar"]).any()


@pytest.mark.parametrize("mode", ["plain", "learned"])
def test_batched_512_graph_workload(ctx, mode):
    """All 512 graphs (n log-uniform in [64, 4096], mean degree U(2, 8), 64 queries each)."""
    bg = gen.batch_graphs()
    specs = [(g.n, g.src, g.dst, g.srcs) for g in bg]
    graphs, refs = make_batch(ctx, specs)
    st = {}
    ctx.batched(graphs, opts=mode_opts(mode), stats=st)
    check(graphs, refs)
    assert st["iterations"] <= 14
    if mode == "learned":
        # every closure is an output, so every graph reads its answers off it
        assert st["arm_trace"][0] == len(bg) and st["arm_trace"][1] == 0, st["arm_trace"][:2]


@pytest.mark.parametrize("mode", list(MODES) + ["selection"])
def test_batched_queries_only(ctx, mode):
    """Graphs whose closure is not an output: the plain schedule answers every query row by per-row
    selection (and squares nothing), the forced closure squares every graph, and the learned schedule
    lets the model choose per graph on the device; every answer is the oracle's."""
    rng = np.random.default_rng(12)
    specs = []
    for n in [1, 64, 65, 300, 700, 1100, 2049, 4096, 40]:
        A = (rng.random((n, n)) < min(3.0 / n, 1.0)).astype(np.uint8)
        s, d = np.nonzero(A)
        k = int(rng.integers(1, min(n, 64) + 1))
        specs.append((n, s, d, rng.choice(n, k, replace=False)))
    graphs, refs = make_batch(ctx, specs, with_closure=False)
    opts = mode_opts(mode) if mode != "selection" else B.make_opts(dispatch=B.DISPATCH_FORCED,
                                                                   smp_arm=B.ARM_SMP_SPARSE)
    st = {}
    ctx.batched(graphs, opts=opts, stats=st)
    check(graphs, refs)
    by_closure, by_selection = st["arm_trace"][0], st["arm_trace"][1]
    assert by_closure + by_selection == len(specs)
    if mode in ("plain", "selection"):
        assert by_selection == len(specs) and st["products"] == 0  # nothing squared
    if mode == "closure":
        assert by_closure == len(specs)
    # a second call reuses the captured launch and gives the same answers
    ctx.batched(graphs, opts=opts)
    check(graphs, refs)


@pytest.mark.parametrize("mode", ["plain", "selection"])
def test_batched_selection_chunks_and_sizes(ctx, mode):
    """Per-row selection inside the batch: 64 query rows at a time for n <= 4,096 (k = 1, 64, 65, 130 and
    200 rows, multi-source rows, a hub, self-loops), one row at a time above that (n = 4,097 and 5,000)."""
    rng = np.random.default_rng(31)
    specs = []
    for n, k, deg in ((64, 64, 2.0), (65, 65, 3.0), (700, 130, 1.5), (4096, 200, 4.0), (1000, 1, 6.0),
                      (257, 64, 40.0), (4097, 70, 3.0), (5000, 20, 2.5)):
        A = (rng.random((n, n)) < min(deg / n, 1.0)).astype(np.uint8)
        A[n // 2, :] = rng.random(n) < 0.5  # a hub row
        A[np.arange(0, n, 7), np.arange(0, n, 7)] = 1  # self-loops
        s, d = np.nonzero(A)
        specs.append((n, s, d, rng.choice(n, k, replace=k > n)))
    graphs, refs = make_batch(ctx, specs, with_closure=False)
    # a few query rows with several sources
    for g, (n, s, d) in zip(graphs, refs):
        Vh = host(g["V"]).copy()
        extra = rng.integers(0, n, (min(5, Vh.shape[0]), 3))
        for i, cols in enumerate(extra):
            for c in cols:
                Vh[i, c // 64] |= np.uint64(1) << np.uint64(c % 64)
        g["V"].copy_(torch.from_numpy(Vh.view(np.int64)))
    opts = None if mode == "plain" else B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_SPARSE)
    ctx.batched(graphs, opts=opts)
    check(graphs, refs)


def _host_batch_features(specs):
    """The dispatcher's features of each graph of a queries-only batch, from counts taken on the host (the
    same formula as the library's: edges, largest row, nonempty rows, query bits; context 0, call level,
    round 0, delta = previous = query bits, nothing visited)."""
    F = np.zeros((len(specs), 16), np.float64)
    for i, (n, s, d, srcs) in enumerate(specs):
        A = np.zeros((n, n), bool)
        A[s, d] = True
        rowdeg = A.sum(axis=1)
        m = float(A.sum())
        k = float(len(srcs))
        vb = float(len(set(int(x) for x in srcs)))
        nn = max(float(n), 1.0)
        deg = m / nn
        F[i, 0] = np.log2(1 + nn) / 16
        F[i, 1] = np.log2(1 + m) / 24
        F[i, 2] = np.log2(1 + deg) / 8
        F[i, 3] = np.log2(1 + rowdeg.max() / (1 + deg)) / 8
        F[i, 4] = (rowdeg > 0).sum() / nn
        F[i, 5] = np.log2(1 + k) / 16
        F[i, 6] = min(k / nn, 4.0)
        F[i, 8] = 1.0
        F[i, 10] = vb / (max(k, 1.0) * nn)
        F[i, 12] = np.log2(1 + vb) / 32
        F[i, 13] = min(vb / max(vb, 1.0), 16.0) / 16
        F[i, 14] = np.log2(1 + vb * deg) / 40
    return F.astype(np.float32)


def test_batched_learned_choice_from_exact_statistics():
    """The learned batch decides per graph on the device from statistics that a two-pass reduction takes
    over 64-row groups of every graph (set bits, largest row, nonempty rows, query bits).  With a model
    whose choice flips across the batch, every graph's decision must be the one the same model makes from
    the host's counts: alone (one graph per batch) and, as a count, in one batch of all the graphs."""
    c = B.Context(0)
    try:
        rng = np.random.default_rng(31)
        specs = []
        for _ in range(40):
            n = int(np.exp(rng.uniform(np.log(64), np.log(4096))))
            m = int(rng.uniform(0.3, 10.0) * n)
            s = rng.integers(0, n, m)
            d = rng.integers(0, n, m)
            if rng.random() < 0.3:  # a hub row: the largest row count differs from the mean
                hub = rng.integers(0, n, n // 2)
                s = np.concatenate([s, np.zeros(len(hub), np.int64)])
                d = np.concatenate([d, hub])
            k = int(rng.integers(1, 65))
            specs.append((n, s, d, rng.choice(n, min(k, n), replace=False)))
        F = _host_batch_features(specs)
        # a network fitted to random targets around these graphs' features: its choices are arbitrary
        # functions of every statistic
        X = np.repeat(F, 20, axis=0) + rng.normal(0, 0.02, (len(F) * 20, 16)).astype(np.float32)
        T = rng.normal(0, 1, (len(X), 4)).astype(np.float32)
        c.dispatcher_train(X, T, np.ones_like(T), epochs=300, lr=1e-2, seed=4)
        Y = c.dispatcher_forward(F)
        want = Y[:, 3] < Y[:, 2]
        sure = np.abs(Y[:, 3] - Y[:, 2]) > 1e-5
        assert want[sure].any() and (~want[sure]).any(), "the model's choices do not vary"
        learned = B.make_opts(dispatch=B.DISPATCH_LEARNED)
        for i, spec in enumerate(specs):
            graphs, refs = make_batch(c, [spec], with_closure=False)
            st = {}
            c.batched(graphs, opts=learned, stats=st)
            check(graphs, refs)
            if sure[i]:
                assert st["arm_trace"][1] == int(want[i]), (i, spec[0], Y[i])
        graphs, refs = make_batch(c, specs, with_closure=False)
        st = {}
        c.batched(graphs, opts=learned, stats=st)
        check(graphs, refs)
        lo = int((want & sure).sum())
        assert lo <= st["arm_trace"][1] <= lo + int((~sure).sum())
    finally:
        c.close()
