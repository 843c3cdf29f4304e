"""GPU parity of the stratified program P3 u P4 u P5 (Section 3.4), composed
from the C-ABI operators, against the oracle's bit-row pipeline: bit-exact
hasPlace, indirectlyPartOf and isForeign, at the knowledge-graph size
(14,541 constants) under every schedule, and on small ragged and degenerate
instances."""
import numpy as np
import pytest

import gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2408_10369_amd as B  # noqa: E402
from paper_2408_10369_amd.programs import is_foreign  # noqa: E402


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


def run(ctx, n, cs, cd, as_, ad, loc, opts=None, st=None):
    return [host(t) for t in is_foreign(ctx, n, (t32(cs), t32(cd)), (t32(as_), t32(ad)), t32(loc),
                                        opts=opts, stats=st)]


SCHEDULES = {
    "plain": B.make_opts(dispatch=B.DISPATCH_PLAIN),
    "learned": B.make_opts(dispatch=B.DISPATCH_LEARNED),
    "cols_dense": B.make_opts(dispatch=B.DISPATCH_FORCED, compose_arm=B.ARM_COMPOSE_SEMINAIVE,
                              smp_arm=B.ARM_SMP_DENSE),
    "cols_one_launch": B.make_opts(dispatch=B.DISPATCH_FORCED, compose_arm=B.ARM_COMPOSE_SEMINAIVE,
                                   smp_arm=B.ARM_SMP_SPARSE),
    "rows": B.make_opts(dispatch=B.DISPATCH_FORCED, compose_arm=B.ARM_COMPOSE_ROWWISE),
    "closure": B.make_opts(dispatch=B.DISPATCH_FORCED, compose_arm=B.ARM_COMPOSE_RMS),
}


@pytest.fixture(scope="module")
def kg():
    g = gen.geo()
    want = oracle.is_foreign_rows(g.n, (g.contains_src, g.contains_dst), (g.adjoins_src, g.adjoins_dst))
    return g, want


@pytest.mark.parametrize("schedule", list(SCHEDULES))
def test_isforeign_full_size(ctx, kg, schedule):
    g, want = kg
    print(f"isForeign n={g.n} schedule={schedule}", flush=True)
    st = {}
    got = run(ctx, g.n, g.contains_src, g.contains_dst, g.adjoins_src, g.adjoins_dst, np.arange(g.n),
              opts=SCHEDULES[schedule], st=st)
    for name, a, b in zip(("hasPlace", "indirectlyPartOf", "isForeign"), got, want):
        assert a.shape == b.shape, name
        assert np.array_equal(a, b), (name, schedule, st.get("arm"))


@pytest.mark.parametrize("n,levels,seed", [(65, (2, 5, 12, 30), 1), (420, (4, 20, 60, 150), 2),
                                           (1000, (6, 40, 200, 500), 3), (3000, (10, 100, 500, 1500), 4)])
def test_isforeign_location_subset(ctx, n, levels, seed):
    """Only the hierarchy's constants are locations; ragged sizes, second parents."""
    g = gen.geo(n=n, levels=levels, seed=seed, extra_parent=0.2)
    want = oracle.is_foreign_rows(n, (g.contains_src, g.contains_dst), (g.adjoins_src, g.adjoins_dst), g.location)
    for schedule in ("plain", "rows", "closure"):
        got = run(ctx, n, g.contains_src, g.contains_dst, g.adjoins_src, g.adjoins_dst, g.location,
                  opts=SCHEDULES[schedule])
        for a, b in zip(got, want):
            assert np.array_equal(a, b), (n, schedule)


def test_isforeign_degenerate(ctx):
    e = np.zeros(0, np.int32)
    # one constant, no facts: the only pair is foreign
    got = run(ctx, 1, e, e, e, e, [0])
    assert [int(x[0, 0]) for x in got] == [0, 0, 1]
    # no adjoins facts: nothing is part of anything, every pair of locations is foreign
    n = 130
    cs, cd = np.arange(n - 1, dtype=np.int32), np.arange(1, n, dtype=np.int32)
    want = oracle.is_foreign_rows(n, (cs, cd), (e, e))
    got = run(ctx, n, cs, cd, e, e, np.arange(n))
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    assert not got[1].any()
    # no contains facts: indirectlyPartOf is adjoins with its inverse
    as_, ad = np.array([0, 5, 64, 129], np.int32), np.array([1, 64, 5, 3], np.int32)
    want = oracle.is_foreign_rows(n, (e, e), (as_, ad))
    got = run(ctx, n, e, e, as_, ad, np.arange(n))
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    # no locations: isForeign is empty whatever the other relations hold
    got = run(ctx, n, cs, cd, as_, ad, e)
    assert not got[2].any()
