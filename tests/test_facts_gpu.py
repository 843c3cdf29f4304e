"""GPU side of the fact <-> matrix pipeline: decoding bit matrices into
(row, column) pairs on the device (bmlp_unpack_coo) against numpy, and whole
programs from Prolog fact text to named facts, checked against the results
the paper prints for its worked examples."""
import ctypes

import numpy as np
import pytest

import gen
from oracle import boolops

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2408_10369_amd as B  # noqa: E402
from paper_2408_10369_amd import facts  # noqa: E402
from paper_2408_10369_amd.programs import is_foreign  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = B.Context(0)
    yield c
    c.close()


def dev(bits):
    return torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint64).view(np.int64)).cuda()


@pytest.mark.parametrize("rows,n,p", [(1, 1, 1.0), (3, 5, 0.5), (70, 64, 0.1), (129, 65, 0.3), (500, 1000, 0.01),
                                      (1000, 130, 0.9), (3000, 4100, 0.002)])
def test_unpack_coo_matches_numpy(ctx, rows, n, p):
    rng = np.random.default_rng(rows + n)
    X = (rng.random((rows, n)) < p).astype(np.uint8)
    for ld in (boolops.words(n), boolops.words(n) + 3):
        r, c = ctx.unpack_coo(dev(boolops.to_bits(X, ld)), n)
        wr, wc = np.nonzero(X)  # row-major order: sorted by row, then column
        assert np.array_equal(r.cpu().numpy(), wr) and np.array_equal(c.cpu().numpy(), wc), (rows, n, ld)


def test_unpack_coo_empty_and_capacity(ctx):
    r, c = ctx.unpack_coo(ctx.zeros(40, 300), 300)
    assert r.numel() == 0 and c.numel() == 0
    X = np.ones((4, 70), np.uint8)
    bits = dev(boolops.to_bits(X))
    cnt = ctypes.c_int64(-1)
    small = torch.zeros(10, dtype=torch.int32, device="cuda")
    rc = B.lib().bmlp_unpack_coo(ctx._h, ctypes.c_void_p(bits.data_ptr()), 4, 70, bits.shape[1],
                                 ctypes.c_void_p(small.data_ptr()), None, 10, ctypes.byref(cnt), None)
    assert rc != 0 and cnt.value == 280
    assert not small.any()  # nothing written


def test_roundtrip_at_sweep_size(ctx):
    n, s, d = gen.c2(2)
    R = ctx.pack_coo(torch.as_tensor(s), torch.as_tensor(d), n, n)
    r, c = ctx.unpack_coo(R, n)
    key = np.unique(s.astype(np.int64) * n + d)
    assert np.array_equal(r.cpu().numpy().astype(np.int64) * n + c.cpu().numpy(), key)


def test_appendix_b_example_from_text(ctx):
    """Example 1 / Appendix B: edge(a,b), edge(b,c); the RMS result decodes to exactly the facts the
    paper prints, path(a,b), path(a,c), path(b,c), and its rows are the codes 011, 001, 000."""
    f = facts.parse_facts("node(a). node(b). node(c). edge(a,b). edge(b,c).")
    t = facts.SymbolTable.from_facts(f, ["node"])
    P = ctx.rms(facts.compile_relation(ctx, t, f["edge"]), len(t))
    assert facts.relation_facts(ctx, t, P, "path") == ["path(a,b)", "path(a,c)", "path(b,c)"]
    assert facts.row_codes(ctx, P, len(t)) == ["011", "001", "000"]


def test_isforeign_example_from_text(ctx):
    """The worked example of Section 3.4 from its facts: every grounding of isForeign over the seven
    constants holds except isForeign(t1,g4), isForeign(g2,g4), isForeign(g3,g4), isForeign(g4,g3)."""
    text = """location(g1). location(g2). location(g3). location(g4). location(t1). location(t2). location(t3).
              contains(t1,g2). contains(g3,t1). adjoins(g3,g4)."""
    f = facts.parse_facts(text)
    t = facts.SymbolTable.from_facts(f, ["location"])
    n = len(t)
    cs, cd = (t.index([p[i] for p in f["contains"]]) for i in (0, 1))
    as_, ad = (t.index([p[i] for p in f["adjoins"]]) for i in (0, 1))
    loc = t.index([p[0] for p in f["location"]])
    T = lambda a: torch.as_tensor(a)  # noqa: E731
    _, _, foreign = is_foreign(ctx, n, (T(cs), T(cd)), (T(as_), T(ad)), T(loc))
    got = set(facts.relation_facts(ctx, t, foreign, "isForeign"))
    names = t.names(range(n))
    false = {"isForeign(t1,g4)", "isForeign(g2,g4)", "isForeign(g3,g4)", "isForeign(g4,g3)"}
    assert got == {f"isForeign({x},{y})" for x in names for y in names} - false
    assert len(got) == 45
