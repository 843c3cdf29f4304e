"""GPU parity at the full sizes of the benchmark workloads, bit-exact against the CPU oracle.

* The n = 16,384 density sweep: every closure row and every answer row of the k = 1, 64 and 1,024
  selections, for all five edge probabilities, under the plain and the learned schedule.
* The n = 65,536 scale-free relation (mean out-degree 4) of the query stream: 2,048 sampled closure
  rows, and every answer row of the first 24 stream queries (three of them with k > 2,048, which the
  one-launch selection serves with its one-slot bottom-up rounds) through a session, under the plain,
  learned and forced-closure schedules.
* The 100 linear-recursion programs over the 14,951-entity multi-relational graph: 512 random rows
  and 512 rows with a step edge of every program, under the plain and learned schedules.
* The one-slot bottom-up selection on its own (k of 2,100 .. 3,000 rows, mean degree >= 4, forced
  one-launch arm, strict and reflexive answers).
"""
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


def dev(bits):
    return torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint64).view(np.int64)).cuda()


def gpu_pack(ctx, n, s, d):
    return ctx.pack_coo(torch.as_tensor(np.asarray(s, np.int32)), torch.as_tensor(np.asarray(d, np.int32)), n, n)


def first_diff(got, want):
    bad = np.nonzero((got != want).any(axis=1))[0]
    return None if bad.size == 0 else (int(bad.size), int(bad[0]))


# ----------------------------------------------------------------- n = 16,384 density sweep, every row
@pytest.mark.parametrize("pi", range(len(gen.C2_PROBS)))
def test_density_sweep_every_row(ctx, pi):
    n, s, d = gen.c2(pi)
    print("density sweep p=%g m=%d" % (gen.C2_PROBS[pi], len(s)), flush=True)
    R = gpu_pack(ctx, n, s, d)
    want = oracle.closure_rows(n, s, d)
    for mode in (B.DISPATCH_PLAIN, B.DISPATCH_LEARNED):
        got = host(ctx.rms(R, n, opts=B.make_opts(dispatch=mode)))
        assert first_diff(got, want) is None, ("rms", pi, mode, first_diff(got, want))
    for ki in range(len(gen.C2_KS)):
        srcs = gen.c2_sources(pi, ki)
        r, c = gen.query_lists(srcs)
        V = ctx.pack_coo(torch.as_tensor(r), torch.as_tensor(c), len(srcs), n)
        vw = oracle.smp(n, s, d, host(V))
        # the answers to one-hot queries are the closure rows of their sources
        assert np.array_equal(vw, want[np.asarray(srcs, np.int64)])
        for mode in (B.DISPATCH_PLAIN, B.DISPATCH_LEARNED):
            st = {}
            got = host(ctx.smp(R, n, V, opts=B.make_opts(dispatch=mode), stats=st))
            assert first_diff(got, vw) is None, ("smp", pi, len(srcs), mode, st.get("arm"), first_diff(got, vw))


# ----------------------------------------------------------------- n = 65,536 scale-free stream
@pytest.fixture(scope="module")
def scalefree():
    n = 65536
    s, d = gen.scalefree_digraph()
    return n, s, d


def test_scalefree_closure_sampled_rows(ctx, scalefree):
    n, s, d = scalefree
    R = gpu_pack(ctx, n, s, d)
    rows = np.sort(np.random.default_rng(65536).choice(n, 2048, replace=False))
    want = oracle.closure_rows(n, s, d, rows=rows)
    got = host(ctx.rms(R, n))
    assert first_diff(got[rows], want) is None, first_diff(got[rows], want)
    assert not np.any(host(R) & ~got)


STREAM_QUERIES = 24


def test_scalefree_closure_by_selection_sampled_rows(ctx, scalefree):
    """R1+ of the stream's relation by the selection from every source: the same sampled rows as the
    oracle, and bit for bit the closure BMLP-RMS reaches."""
    n, s, d = scalefree
    R = gpu_pack(ctx, n, s, d)
    eye = ctx.pack_coo(torch.arange(n, dtype=torch.int32), torch.arange(n, dtype=torch.int32), n, n)
    got = ctx.smp(R, n, eye, opts=B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_CLOSURE_SELECT))
    rows = np.sort(np.random.default_rng(65537).choice(n, 2048, replace=False))
    want = oracle.closure_rows(n, s, d, rows=rows)
    gh = host(got)
    assert first_diff(gh[rows], want) is None, first_diff(gh[rows], want)
    del eye
    assert np.array_equal(gh, host(ctx.rms(R, n)))


@pytest.mark.parametrize("mode", ["plain", "learned", "forced_closure", "forced_closure_select"])
def test_scalefree_stream_every_answer(ctx, scalefree, mode):
    n, s, d = scalefree
    queries = gen.query_stream(count=STREAM_QUERIES)
    ks = [len(q) for q in queries]
    assert sum(k > 2048 for k in ks) >= 3  # the one-slot bottom-up kernel serves these under every schedule
    opts = {"plain": B.make_opts(dispatch=B.DISPATCH_PLAIN),
            "learned": B.make_opts(dispatch=B.DISPATCH_LEARNED),
            "forced_closure": B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_CLOSURE),
            "forced_closure_select": B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_CLOSURE_SELECT)}[mode]
    R = gpu_pack(ctx, n, s, d)
    arms = []
    with ctx.graph(R, n) as g:
        for qi, q in enumerate(queries):
            r, c = gen.query_lists(q)
            V = ctx.pack_coo(torch.as_tensor(r).cuda(), torch.as_tensor(c).cuda(), len(q), n)
            st = {}
            got = host(g.query(V, opts=opts, stats=st))
            arms.append(st["arm"])
            want = oracle.smp(n, s, d, host(V))
            assert first_diff(got, want) is None, (mode, qi, len(q), st["arm"], first_diff(got, want))
    if mode == "plain":
        # the plain schedule answers every query of 64 or more rows with the one-launch selection
        assert all(a == B.ARM_SMP_SPARSE for a, k in zip(arms, ks) if k >= 64)
    if mode == "forced_closure":
        assert all(a == B.ARM_SMP_CLOSURE for a in arms)
    if mode == "forced_closure_select":
        # the first query builds the closure by selection, the others read it off
        assert arms[0] == B.ARM_SMP_CLOSURE_SELECT and all(a == B.ARM_SMP_CLOSURE for a in arms[1:]), arms


@pytest.mark.parametrize("n,deg,k", [(4096, 4.4, 2100), (9000, 6.0, 2500), (16384, 4.6, 3000)])
def test_one_slot_bottom_up_selection(ctx, n, deg, k):
    """More than 2,048 rows in one launch take the one-slot kernel; from mean degree 4 on the relation's
    in-edge index is built and rounds with a large frontier run bottom-up."""
    s, d = gen.er_digraph(n, deg / n, int(10 * deg) + n + k)
    assert len(s) >= 4 * n
    rng = np.random.default_rng(n + k)
    V = np.zeros((k, n), np.uint8)
    V[np.arange(k), rng.integers(0, n, k)] = 1
    V[-7:] |= (rng.random((7, n)) < 0.003).astype(np.uint8)  # a few multi-source rows
    Vb = boolops.to_bits(V)
    R = gpu_pack(ctx, n, s, d)
    for refl in (0, 1):
        st = {}
        got = host(ctx.smp(R, n, dev(Vb), opts=B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_SPARSE,
                                                            smp_reflexive=refl), stats=st))
        want = oracle.smp(n, s, d, Vb, reflexive=bool(refl))
        assert first_diff(got, want) is None, (n, deg, k, refl, first_diff(got, want))
        assert st["arm"] == B.ARM_SMP_SPARSE


# ----------------------------------------------------------------- the 100 programs at n = 14,951
@pytest.fixture(scope="module")
def multirel():
    mr = gen.multirel()
    return mr, gen.programs(mr, count=100, base_seed=4000)


@pytest.mark.parametrize("half", [0, 1])
def test_programs_all_hundred_sampled_rows(ctx, multirel, half):
    mr, progs = multirel
    n = mr.n
    packed = {}
    out = ctx.zeros(n, n)
    for i in range(50 * half, 50 * half + 50):
        b, s = progs[i]
        for rel in (b, s):
            if rel not in packed:
                packed[rel] = gpu_pack(ctx, n, mr.rel_src[rel], mr.rel_dst[rel])
        # 512 random rows and 512 of the rows where the step relation has an edge (where the recursion
        # can add facts beyond the base relation's)
        rng = np.random.default_rng(4000 + i)
        heads = np.unique(mr.rel_src[s])
        rows = np.unique(np.r_[rng.choice(n, 512, replace=False),
                               rng.choice(heads, min(512, heads.size), replace=False)]).astype(np.int64)
        want = oracle.compose_rows(n, mr.rel_src[b], mr.rel_dst[b], mr.rel_src[s], mr.rel_dst[s], rows=rows)
        for mode in (B.DISPATCH_PLAIN, B.DISPATCH_LEARNED):
            st = {}
            got = host(ctx.compose_linear(packed[b], packed[s], n, out=out, opts=B.make_opts(dispatch=mode),
                                          stats=st))
            assert first_diff(got[rows], want) is None, (i, b, s, mode, st.get("arm"), first_diff(got[rows], want))
