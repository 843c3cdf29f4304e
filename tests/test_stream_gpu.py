"""The stream path without host waits: asynchronous packing (out-of-range facts skipped and reported by
bmlp_deferred_error), session queries without statistics, and the session's last arm."""
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


def test_pack_coo_async_and_deferred_error(ctx):
    n, rows = 300, 77
    rng = np.random.default_rng(5)
    r = rng.integers(0, rows, 2000).astype(np.int32)
    c = rng.integers(0, n, 2000).astype(np.int32)
    R, C = torch.as_tensor(r).cuda(), torch.as_tensor(c).cuda()
    out = ctx.zeros(rows, n)
    out.fill_(-1)  # every word is rewritten
    ctx.pack_coo_async(R, C, rows, n, out=out)
    assert np.array_equal(host(out), host(ctx.pack_coo(R, C, rows, n)))
    ctx.deferred_error()  # nothing latched
    # out-of-range facts: skipped, latched, reported once, then cleared
    r2, c2 = r.copy(), c.copy()
    r2[7], c2[9] = rows, -1
    ctx.pack_coo_async(torch.as_tensor(r2).cuda(), torch.as_tensor(c2).cuda(), rows, n, out=out)
    keep = np.ones(len(r), bool)
    keep[[7, 9]] = False
    want = host(ctx.pack_coo(torch.as_tensor(r[keep]).cuda(), torch.as_tensor(c[keep]).cuda(), rows, n))
    assert np.array_equal(host(out), want)
    with pytest.raises(B.BmlpError) as e:
        ctx.deferred_error()
    assert e.value.status == B.EINVAL
    ctx.deferred_error()


@pytest.mark.parametrize("mode", ["plain", "learned", "forced_closure", "forced_closure_select"])
def test_session_without_stats(ctx, mode):
    n = 20000
    s, d = gen.er_digraph(n, 3.0 / n, 20000)
    R = ctx.pack_coo(torch.as_tensor(s), torch.as_tensor(d), n, n)
    opts = {"plain": B.make_opts(dispatch=B.DISPATCH_PLAIN), "learned": B.make_opts(dispatch=B.DISPATCH_LEARNED),
            "forced_closure": B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_CLOSURE),
            "forced_closure_select": B.make_opts(dispatch=B.DISPATCH_FORCED,
                                                 smp_arm=B.ARM_SMP_CLOSURE_SELECT)}[mode]
    rng = np.random.default_rng(77)
    V = ctx.zeros(600, n)
    Vs = ctx.zeros(600, n)
    with ctx.graph(R, n) as g:
        assert g.last_arm == -1
        for q in range(12):
            k = int(rng.integers(1, 600))
            srcs = rng.choice(n, k, replace=False).astype(np.int32)
            rr, cc = gen.query_lists(srcs)
            ctx.pack_coo_async(torch.as_tensor(rr).cuda(), torch.as_tensor(cc).cuda(), k, n, out=V[:k])
            g.query(V[:k], out=Vs[:k], opts=opts)
            arm = g.last_arm
            assert arm in (B.ARM_SMP_SPARSE, B.ARM_SMP_CLOSURE, B.ARM_SMP_DENSE, B.ARM_SMP_ADAPTIVE,
                           B.ARM_SMP_CLOSURE_SELECT)
            if mode == "forced_closure":
                assert arm == B.ARM_SMP_CLOSURE
            if mode == "forced_closure_select":
                assert arm == (B.ARM_SMP_CLOSURE_SELECT if q == 0 else B.ARM_SMP_CLOSURE), (q, arm)
            if arm == B.ARM_SMP_CLOSURE_SELECT:
                assert g.has_closure
            want = oracle.smp(n, s, d, host(V[:k]))
            assert np.array_equal(host(Vs[:k]), want), (mode, q, k, arm)
    ctx.deferred_error()


@pytest.mark.parametrize("mode", ["plain", "learned", "forced_closure"])
@pytest.mark.parametrize("refl", [0, 1])
def test_session_query_by_sources(ctx, mode, refl):
    """One-hot queries given by their source indices equal the same queries given as bit rows; an index out
    of range gives a zero row and is reported by bmlp_deferred_error."""
    n = 9000
    s, d = gen.er_digraph(n, 2.5 / n, 9000)
    R = ctx.pack_coo(torch.as_tensor(s), torch.as_tensor(d), n, n)
    base = {"plain": dict(dispatch=B.DISPATCH_PLAIN), "learned": dict(dispatch=B.DISPATCH_LEARNED),
            "forced_closure": dict(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_CLOSURE)}[mode]
    opts = B.make_opts(smp_reflexive=refl, **base)
    rng = np.random.default_rng(9 + refl)
    out = ctx.zeros(700, n)
    with ctx.graph(R, n) as g:
        for q in range(10):
            k = int(rng.integers(1, 700))
            srcs = rng.choice(n, k, replace=False).astype(np.int32)
            out.fill_(-1)
            g.query_sources(torch.as_tensor(srcs).cuda(), out[:k], opts=opts)
            V = np.zeros((k, n), np.uint8)
            V[np.arange(k), srcs] = 1
            from oracle import boolops
            want = oracle.smp(n, s, d, boolops.to_bits(V), reflexive=bool(refl))
            assert np.array_equal(host(out[:k]), want), (mode, refl, q, k, g.last_arm)
        ctx.deferred_error()
        bad = np.array([3, n, 5], np.int32)
        g.query_sources(torch.as_tensor(bad).cuda(), out[:3], opts=opts)
        got = host(out[:3])
        assert not got[1].any()
        with pytest.raises(B.BmlpError):
            ctx.deferred_error()


def test_batched_rejects_closure_by_selection(ctx):
    n = 100
    s, d = gen.er_digraph(n, 0.03, 3)
    R = ctx.pack_coo(torch.as_tensor(s), torch.as_tensor(d), n, n)
    V = ctx.zeros(4, n)
    desc = [{"n": n, "R1": R, "V": V, "Vstar": ctx.zeros(4, n), "closure": None}]
    with pytest.raises(B.BmlpError) as e:
        ctx.batched(desc, opts=B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_CLOSURE_SELECT))
    assert e.value.status == B.EINVAL
