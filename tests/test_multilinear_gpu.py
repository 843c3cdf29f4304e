"""GPU parity of the two-sided linear recursion (bmlp_compose_two_sided):
p <- b; p <- l, p, r.  Bit-exact against the oracle's Kleene iteration on
random relations of ragged sizes, on every product arm, against the
composition when one side is the identity, and against the closed form of
same-generation on a forest at n = 16,384."""
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


def pack(ctx, n, pairs, ld=None):
    s, d = pairs
    return ctx.pack_coo(torch.as_tensor(np.asarray(s, np.int32)), torch.as_tensor(np.asarray(d, np.int32)), n, n, ld)


def rand_pairs(rng, n, p):
    A = rng.random((n, n)) < p
    s, d = np.nonzero(A)
    return s.astype(np.int32), d.astype(np.int32)


ARMS = {"auto": None,
        "valu": B.make_opts(dispatch=B.DISPATCH_FORCED, product_arm=B.ARM_PRODUCT_VALU),
        "mfma": B.make_opts(dispatch=B.DISPATCH_FORCED, product_arm=B.ARM_PRODUCT_MFMA)}


@pytest.mark.parametrize("n,pb,pl,pr", [(1, 1.0, 1.0, 1.0), (2, 0.5, 0.5, 0.5), (65, 0.02, 0.03, 0.03),
                                        (300, 0.004, 0.006, 0.005), (1000, 0.001, 0.0015, 0.0012),
                                        (1500, 0.0005, 0.001, 0.001)])
@pytest.mark.parametrize("arm", list(ARMS))
def test_two_sided_random(ctx, n, pb, pl, pr, arm):
    rng = np.random.default_rng(n * 7 + int(pl * 1e4))
    b, l, r = rand_pairs(rng, n, pb), rand_pairs(rng, n, pl), rand_pairs(rng, n, pr)
    ld = boolops.words(n) + (n % 2)
    print(f"two_sided n={n} arm={arm}", flush=True)
    st = {}
    got = ctx.compose_two_sided(pack(ctx, n, b, ld), pack(ctx, n, l, ld), pack(ctx, n, r, ld), n, opts=ARMS[arm],
                                stats=st)
    assert np.array_equal(host(got), oracle.two_sided_rows(n, b, l, r, ld=ld)), (n, arm, st.get("iterations"))


def test_two_sided_one_sided_cases(ctx):
    """Rright = I gives compose_linear(Rbase, Rleft); empty sides give Rbase."""
    n = 700
    rng = np.random.default_rng(21)
    b, l = rand_pairs(rng, n, 0.003), rand_pairs(rng, n, 0.002)
    eye = (np.arange(n, dtype=np.int32),) * 2
    Rb, Rl, I = pack(ctx, n, b), pack(ctx, n, l), pack(ctx, n, eye)
    got = host(ctx.compose_two_sided(Rb, Rl, I, n))
    assert np.array_equal(got, host(ctx.compose_linear(Rb, Rl, n)))
    assert np.array_equal(got, oracle.compose_rows(n, *b, *l))
    Z = ctx.zeros(n, n)
    assert np.array_equal(host(ctx.compose_two_sided(Rb, Z, Rl, n)), host(Rb))
    assert np.array_equal(host(ctx.compose_two_sided(Rb, Rl, Z, n)), host(Rb))
    E = ctx.zeros(n, n)
    assert not host(ctx.compose_two_sided(E, Rl, Rl, n)).any()


def test_two_sided_errors(ctx):
    n = 64
    R = ctx.zeros(n, n)
    with pytest.raises(B.BmlpError):
        ctx.compose_two_sided(R, R, R, n, out=R)


@pytest.mark.parametrize("n,trees", [(2000, 3), (16384, 8)])
def test_same_generation_forest(ctx, n, trees):
    """sg on a forest: flat on each root, up = child -> parent, down = its inverse.  sg(x, y) holds
    exactly when x and y are in the same tree at the same depth (checked on every row)."""
    f = gen.forest(n=n, trees=trees, seed=n)
    roots = np.unique(f.root).astype(np.int32)
    st = {}
    got = host(ctx.compose_two_sided(pack(ctx, n, (roots, roots)), pack(ctx, n, (f.child, f.parent)),
                                     pack(ctx, n, (f.parent, f.child)), n, stats=st))
    key = f.root * (int(f.depth.max()) + 1) + f.depth
    order = np.argsort(key, kind="stable")
    want = np.zeros((n, boolops.words(n) * 64), np.uint8)
    ks = key[order]
    starts = np.flatnonzero(np.r_[True, ks[1:] != ks[:-1]])
    ends = np.r_[starts[1:], n]
    for a, e in zip(starts, ends):
        members = order[a:e]
        want[np.ix_(members, members)] = 1
    want_bits = np.packbits(want, axis=1, bitorder="little").view(np.uint64)
    assert np.array_equal(got, want_bits)
    assert st["iterations"] == int(f.depth.max()) + 1
