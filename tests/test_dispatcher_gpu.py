"""GPU tests of the learned dispatcher.

* The GPU forward/backward kernels against the FP64 reference (tolerance,
  not bit-exact: the network is the only floating-point step).
* Training reduces the loss; the model file round-trips; a corrupt file is
  rejected and leaves the plain schedule in force.
* Whatever the model chooses, results stay bit-exact: a model trained on
  random targets makes arbitrary per-round choices, and every selection,
  composition and session answer is checked against the oracle.
"""
import os

import numpy as np
import pytest

import gen
import oracle
from oracle import boolops, mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2408_10369_amd as B  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    os.environ["BMLP_DISPATCHER_MODEL"] = ""
    c = B.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def random_model(ctx, tmp_path_factory):
    """A model fitted to random targets: its per-round choices are arbitrary mixes."""
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (400, 16)).astype(np.float32)
    X[:, 8] = rng.integers(0, 2, 400)
    T = rng.normal(0, 1, (400, 4)).astype(np.float32)
    M = np.ones((400, 4), np.float32)
    ctx.dispatcher_train(X, T, M, epochs=300, lr=1e-2, seed=3)
    path = str(tmp_path_factory.mktemp("model") / "m.bin")
    ctx.dispatcher_save(path)
    return path


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def pack(ctx, n, s, d):
    return ctx.pack_coo(torch.as_tensor(np.asarray(s, np.int32)), torch.as_tensor(np.asarray(d, np.int32)), n, n)


# ----------------------------------------------------------------- network kernels vs FP64 reference
@pytest.mark.parametrize("rows", [1, 7, 300])
def test_gpu_loss_and_gradient_match_reference(ctx, rows):
    rng = np.random.default_rng(rows)
    p = rng.normal(0, 0.2, mlp.N_PARAMS).astype(np.float32)
    mu = rng.normal(0, 1, 16).astype(np.float32)
    sd = rng.uniform(0.5, 2.0, 16).astype(np.float32)
    X = rng.normal(0, 1, (rows, 16)).astype(np.float32)
    T = rng.normal(0, 1, (rows, 4)).astype(np.float32)
    M = (rng.random((rows, 4)) < 0.7).astype(np.float32)
    M[0, 0] = 1
    L, G = ctx.mlp_loss_grad(p, mu, sd, X, T, M)
    Lr, Gr = mlp.loss_grad(p, mu, sd, X, T, M)
    assert abs(L - Lr) <= 1e-4 * abs(Lr) + 1e-6
    assert np.all(np.abs(G - Gr) <= 1e-3 * np.abs(Gr) + 1e-5), np.max(np.abs(G - Gr))


def test_training_reduces_loss_and_forward_matches_reference(ctx, tmp_path):
    rng = np.random.default_rng(9)
    X = rng.normal(0, 1, (2000, 16)).astype(np.float32)
    w = rng.normal(0, 1, (16, 4))
    T = (np.tanh(X @ w) + 0.1 * rng.normal(0, 1, (2000, 4))).astype(np.float32)
    M = (rng.random((2000, 4)) < 0.8).astype(np.float32)
    base = float((M * (T - (T * M).sum(0) / M.sum(0)) ** 2).sum() / M.sum())
    loss = ctx.dispatcher_train(X, T, M, epochs=400, lr=3e-3, seed=1)
    assert loss < 0.3 * base
    Y = ctx.dispatcher_forward(X[:50])
    path = str(tmp_path / "m.bin")
    ctx.dispatcher_save(path)
    raw = np.fromfile(path, dtype=np.uint8)
    body = raw[:-4].tobytes()
    hdr = 8 + 6 * 4
    fl = np.frombuffer(body[hdr:], dtype=np.float32)
    mu, sd, params = fl[:16], fl[16:32], fl[32:]
    Yr, _ = mlp.forward(params, mu, sd, X[:50])
    assert np.allclose(Y, Yr, rtol=1e-4, atol=1e-4)


def test_model_file_roundtrip_and_corruption(ctx, tmp_path, random_model):
    ctx.dispatcher_load(random_model)
    X = np.random.default_rng(1).normal(0, 1, (5, 16)).astype(np.float32)
    Y0 = ctx.dispatcher_forward(X)
    bad = tmp_path / "bad.bin"
    raw = bytearray(open(random_model, "rb").read())
    raw[100] ^= 0xFF
    bad.write_bytes(bytes(raw))
    with pytest.raises(B.BmlpError) as e:
        ctx.dispatcher_load(str(bad))
    assert e.value.status == B.EMODEL
    with pytest.raises(B.BmlpError) as e:
        ctx.dispatcher_load(str(tmp_path / "missing.bin"))
    assert e.value.status == B.EMODEL
    assert np.array_equal(ctx.dispatcher_forward(X), Y0)  # unchanged


def test_no_model_falls_back_to_plain(tmp_path):
    os.environ["BMLP_DISPATCHER_MODEL"] = str(tmp_path / "none.bin")
    c = B.Context(0)
    try:
        assert not c.dispatcher_loaded()
        n = 300
        s, d = gen.er_digraph(n, 3.0 / n, 1)
        R = pack(c, n, s, d)
        V = c.pack_coo(torch.tensor([0], dtype=torch.int32), torch.tensor([5], dtype=torch.int32), 1, n)
        st = {}
        out = c.smp(R, n, V, opts=B.make_opts(dispatch=B.DISPATCH_LEARNED), stats=st)
        assert np.array_equal(host(out), oracle.smp(n, s, d, host(V)))
        assert st["arm"] in (B.ARM_SMP_SPARSE, B.ARM_SMP_DENSE)
    finally:
        c.close()
        os.environ["BMLP_DISPATCHER_MODEL"] = ""


# ----------------------------------------------------------------- bit-exact whatever the choices
@pytest.mark.parametrize("n,deg,k", [(200, 1.5, 9), (1000, 4.0, 33), (3000, 12.0, 5), (700, 60.0, 70)])
def test_adaptive_and_learned_selection_bit_exact(ctx, random_model, n, deg, k):
    ctx.dispatcher_load(random_model)
    rng = np.random.default_rng(n)
    s, d = gen.er_digraph(n, deg / (n - 1), n + 1)
    R = pack(ctx, n, s, d)
    V = np.zeros((k, n), np.uint8)
    V[np.arange(k), rng.integers(0, n, k)] = 1
    V[: k // 4] |= (rng.random((k // 4, n)) < 0.01).astype(np.uint8)
    Vd = torch.from_numpy(boolops.to_bits(V).view(np.int64)).cuda()
    for refl in (0, 1):
        want = oracle.smp(n, s, d, boolops.to_bits(V), reflexive=bool(refl))
        tr = B.Trace()
        ctx.set_trace(tr)
        st = {}
        got = ctx.smp(R, n, Vd, opts=B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_ADAPTIVE,
                                                  smp_reflexive=refl), stats=st)
        ctx.set_trace(None)
        assert np.array_equal(host(got), want)
        t = tr.as_dict()
        assert t["rounds"] == min(st["iterations"], 64) and t["features"].shape == (t["rounds"], 16)
        assert set(t["arm"]) <= {B.ARM_SMP_DENSE, B.ARM_SMP_SPARSE}
        for arm in (B.ARM_SMP_SPARSE_ROUNDS, B.ARM_SMP_DENSE):
            got = ctx.smp(R, n, Vd, opts=B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=arm, smp_reflexive=refl))
            assert np.array_equal(host(got), want), arm
        got = ctx.smp(R, n, Vd, opts=B.make_opts(dispatch=B.DISPATCH_LEARNED, smp_reflexive=refl))
        assert np.array_equal(host(got), want)


def test_learned_composition_bit_exact(ctx, random_model):
    ctx.dispatcher_load(random_model)
    mr = gen.multirel(n=1500, nrel=40, total=9000, seed=11)
    for (b, st) in gen.programs(mr, count=6, base_seed=123):
        Rb = pack(ctx, mr.n, mr.rel_src[b], mr.rel_dst[b])
        Rs = pack(ctx, mr.n, mr.rel_src[st], mr.rel_dst[st])
        want = oracle.compose_rows(mr.n, mr.rel_src[b], mr.rel_dst[b], mr.rel_src[st], mr.rel_dst[st])
        got = ctx.compose_linear(Rb, Rs, mr.n, opts=B.make_opts(dispatch=B.DISPATCH_LEARNED))
        assert np.array_equal(host(got), want)
        for sarm in (B.ARM_SMP_SPARSE_ROUNDS, B.ARM_SMP_ADAPTIVE):
            got = ctx.compose_linear(Rb, Rs, mr.n, opts=B.make_opts(dispatch=B.DISPATCH_FORCED,
                                                                     compose_arm=B.ARM_COMPOSE_SEMINAIVE,
                                                                     smp_arm=sarm))
            assert np.array_equal(host(got), want), sarm


# ----------------------------------------------------------------- sessions
def test_sessions_plain_learned_and_cached_closure(ctx, random_model):
    ctx.dispatcher_load(random_model)
    n = 2000
    s, d = gen.scalefree_digraph(n=n, m=8000, seed=3)
    R = pack(ctx, n, s, d)
    queries = gen.query_stream(n=n, count=12, kmax=64, base_seed=77)
    closure = oracle.closure_rows(n, s, d)
    for mode, expect_cache in ((B.DISPATCH_PLAIN, False), (B.DISPATCH_LEARNED, None)):
        with ctx.graph(R, n) as g:
            for q in queries:
                V = ctx.pack_coo(*map(torch.as_tensor, gen.query_lists(q)), len(q), n)
                st = {}
                out = g.query(V, opts=B.make_opts(dispatch=mode), stats=st)
                want = np.zeros((len(q), boolops.words(n)), np.uint64)
                for r, src in enumerate(q):
                    want[r] = closure[src]
                assert np.array_equal(host(out), want)
            if expect_cache is not None:
                assert g.has_closure == expect_cache
    with ctx.graph(R, n) as g:
        V = ctx.pack_coo(*map(torch.as_tensor, gen.query_lists(queries[0])), len(queries[0]), n)
        g.query(V, opts=B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_CLOSURE))
        assert g.has_closure
        st = {}
        g.query(V, stats=st)
        assert st["arm"] == B.ARM_SMP_CLOSURE


@pytest.mark.parametrize("n", [1, 130, 3000, 20000])
def test_call_features_match_graph_statistics(ctx, n):
    """The call-level features come from the library's device counts (edges, largest row, nonempty
    rows, source bits); they must equal the counts taken on the host, also for rows of more than
    256 words and for a degree table scanned in several segments."""
    rng = np.random.default_rng(n + 3)
    m_target = max(1, n * 3)
    s = rng.integers(0, n, m_target).astype(np.int32)
    d = rng.integers(0, n, m_target).astype(np.int32)
    hub = 0
    extra = np.arange(min(n, 700), dtype=np.int32)
    s = np.concatenate([s, np.full(len(extra), hub, np.int32)])
    d = np.concatenate([d, extra])
    A = np.zeros((n, n), np.uint8)
    A[s, d] = 1
    m = int(A.sum())
    rowdeg = A.sum(axis=1)
    k = min(n, 37)
    V = np.zeros((k, n), np.uint8)
    V[np.arange(k), rng.integers(0, n, k)] = 1
    V[0, : min(n, 90)] = 1
    R = pack(ctx, n, s, d)
    Vd = torch.from_numpy(boolops.to_bits(V).view(np.int64)).cuda()
    tr = B.Trace()
    ctx.set_trace(tr)
    got = ctx.smp(R, n, Vd, opts=B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_SPARSE))
    ctx.set_trace(None)
    assert np.array_equal(host(got), oracle.smp(n, s, d, boolops.to_bits(V)))
    f = tr.as_dict()["call_features"]
    deg = m / n
    want = {0: np.log2(1 + n) / 16, 1: np.log2(1 + m) / 24, 2: np.log2(1 + deg) / 8,
            3: np.log2(1 + rowdeg.max() / (1 + deg)) / 8, 4: (rowdeg > 0).sum() / n, 5: np.log2(1 + k) / 16,
            12: np.log2(1 + V.sum()) / 32}
    for i, v in want.items():
        assert abs(float(f[i]) - v) <= 1e-6 * max(1.0, abs(v)), (i, float(f[i]), v)
