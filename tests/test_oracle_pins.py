"""Pins for the CPU oracle: checks it against facts fixed by the paper and by
mathematics, never against itself.

* the paper's worked examples (golden fixtures with their citations);
* closed forms (empty, cycle, complete, path, self-loop, disjoint union);
* exhaustive brute force on every digraph with n <= 3 and on all 2^16
  digraphs with n = 4 (powers of the integer adjacency matrix);
* cross-checks between three independent routes (BFS, Warshall, pure-Python
  semi-naive datalog) and the paper's Algorithms 1 and 2 stepped literally;
* the algebraic invariants of a closure;
* loop counts of Algorithms 1 and 2 on path graphs (closed forms).
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from oracle import algorithms, boolops, datalog


def _parse(path):
    out = {"edge": [], "row": [], "contains": [], "adjoins": [], "false": []}
    consts = None
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *rest = line.split()
            if key == "constants":
                consts = rest
            else:
                out[key].append(rest)
    return consts, out


def dense_closure(n, s, d):
    return boolops.from_bits(oracle.closure_rows(n, s, d), n)


def brute_closure(A):
    """Sum_{k=1..n} A^k > 0 with integer matrix powers (paths of length 1..n
    suffice: a shortest path never repeats a node)."""
    n = A.shape[-1]
    A = A.astype(np.int64)
    P = A.copy()
    acc = A.copy()
    for _ in range(max(n - 1, 0)):
        P = np.minimum(P @ A, 1)
        acc = acc | P
    return (acc > 0).astype(np.uint8)


# ---------------------------------------------------------------- worked examples
def test_example1_path_matrix(golden_dir):
    consts, g = _parse(os.path.join(golden_dir, "example1_path.txt"))
    idx = {c: i for i, c in enumerate(consts)}
    s = [idx[a] for a, b in g["edge"]]
    d = [idx[b] for a, b in g["edge"]]
    want = np.array([[int(x) for x in r] for r in g["row"]], dtype=np.uint8)
    n = len(consts)
    assert np.array_equal(dense_closure(n, s, d), want)
    R1 = boolops.dense_from_edges(n, s, d)
    assert np.array_equal(algorithms.rms_paper(R1)[0], want)
    assert np.array_equal(algorithms.rms_squaring_or(R1)[0], want)
    pairs = datalog.closure(set(zip(s, d)))
    assert pairs == {(i, j) for i in range(n) for j in range(n) if want[i, j]}
    assert np.array_equal(boolops.from_bits(oracle.warshall(boolops.to_bits(R1), n), n), want)


def test_isforeign_example(golden_dir):
    consts, g = _parse(os.path.join(golden_dir, "isforeign_example.txt"))
    idx = {c: i for i, c in enumerate(consts)}
    n = len(consts)
    cs = [idx[a] for a, b in g["contains"]]
    cd = [idx[b] for a, b in g["contains"]]
    As = [idx[a] for a, b in g["adjoins"]]
    Ad = [idx[b] for a, b in g["adjoins"]]
    want = np.ones((n, n), np.uint8)
    for a, b in g["false"]:
        want[idx[a], idx[b]] = 0
    assert want.sum() == 45

    # matrix route: hasPlace = RMS(contains); IPO = (hasPlace^T)* (adj + adj^T);
    # isForeign = NEG(IPO) (every constant is a location)
    has_place = dense_closure(n, cs, cd)
    adj = boolops.dense_from_edges(n, As, Ad)
    base = boolops.add(adj, boolops.transp(adj))
    step = boolops.transp(has_place)
    bs, bd = np.nonzero(base)
    ss, sd = np.nonzero(step)
    ipo = boolops.from_bits(oracle.compose_rows(n, bs, bd, ss, sd), n)
    foreign = boolops.neg(ipo)
    assert np.array_equal(foreign, want)

    # clause route: pure-Python semi-naive evaluation of P3 u P4 u P5
    hp, ipo2, f2 = datalog.is_foreign(range(n), set(zip(cs, cd)), set(zip(As, Ad)))
    assert f2 == {(i, j) for i in range(n) for j in range(n) if want[i, j]}
    assert ipo2 == {(i, j) for i in range(n) for j in range(n) if ipo[i, j]}


@pytest.mark.parametrize("seed,all_locations", [(1, True), (2, False), (3, True)])
def test_isforeign_bit_pipeline_matches_clauses(seed, all_locations):
    """The oracle's bit-row pipeline for P3 u P4 u P5 (closure, composition,
    negation, location mask) against the clause-by-clause evaluator, on a
    small hierarchy shaped like the knowledge-graph workload."""
    import gen
    g = gen.geo(n=420, levels=(4, 20, 60, 150), seed=seed, extra_parent=0.15)
    n = g.n
    loc = None if all_locations else g.location
    hp, ipo, fr = oracle.is_foreign_rows(n, (g.contains_src, g.contains_dst),
                                         (g.adjoins_src, g.adjoins_dst), loc)
    hp2, ipo2, fr2 = datalog.is_foreign(range(n), set(zip(g.contains_src.tolist(), g.contains_dst.tolist())),
                                        set(zip(g.adjoins_src.tolist(), g.adjoins_dst.tolist())),
                                        None if loc is None else loc.tolist())
    as_set = lambda bits: {(int(i), int(j)) for i, j in zip(*np.nonzero(boolops.from_bits(bits, n)))}
    assert as_set(hp) == hp2
    assert as_set(ipo) == ipo2
    assert as_set(fr) == fr2
    assert len(ipo2) > len(g.adjoins_src)          # the recursion derived new facts
    # padding bits of the negated rows stay zero
    assert boolops.to_bits(boolops.from_bits(fr, n), ld=fr.shape[1]).tolist() == fr.tolist()


def _pairs(A):
    s, d = np.nonzero(A)
    return s.astype(np.int32), d.astype(np.int32)


def _bitset(bits, n):
    return {(int(i), int(j)) for i, j in zip(*np.nonzero(boolops.from_bits(bits, n)))}


@pytest.mark.parametrize("seed", range(12))
def test_two_sided_oracle_against_clauses(seed):
    """The Kleene iteration of P = B | L P R against the clause-by-clause evaluator."""
    rng = np.random.default_rng(400 + seed)
    n = int(rng.integers(1, 30))
    b, l, r = (_pairs(rng.random((n, n)) < q) for q in (0.08, 0.12, 0.12))
    want = datalog.two_sided(set(zip(*b)), set(zip(*l)), set(zip(*r)))
    assert _bitset(oracle.two_sided_rows(n, b, l, r), n) == want


@pytest.mark.parametrize("seed", range(6))
def test_two_sided_reduces_to_one_sided(seed):
    """With R = I the program is p <- b; p <- l, p, whose least model is L* B (the composition
    oracle); with L = I it is B R*, the transpose of the composition over the transposes."""
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(2, 70))
    B = rng.random((n, n)) < 0.05
    S = rng.random((n, n)) < 0.04
    eye = _pairs(np.eye(n, dtype=bool))
    got = oracle.two_sided_rows(n, _pairs(B), _pairs(S), eye)
    assert np.array_equal(got, oracle.compose_rows(n, *_pairs(B), *_pairs(S)))
    got = oracle.two_sided_rows(n, _pairs(B), eye, _pairs(S))
    want_t = boolops.from_bits(oracle.compose_rows(n, *_pairs(B.T), *_pairs(S.T)), n)
    assert np.array_equal(boolops.from_bits(got, n), want_t.T)
    # no left or right relation: P is B
    none = (np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert np.array_equal(oracle.two_sided_rows(n, _pairs(B), none, _pairs(S)), boolops.to_bits(B.astype(np.uint8)))


def test_same_generation_closed_form():
    """Same-generation on a forest: flat holds on each root, up maps a node to its parent, down is its
    inverse.  Then sg(x, y) holds exactly when x and y lie in the same tree at the same depth."""
    import gen
    g = gen.forest(n=300, trees=4, seed=3)
    n = g.n
    depth, root = g.depth, g.root
    want = {(x, y) for x in range(n) for y in range(n) if depth[x] == depth[y] and root[x] == root[y]}
    roots = np.unique(root)
    flat = (roots.astype(np.int32), roots.astype(np.int32))
    up = (g.child, g.parent)
    down = (g.parent, g.child)
    assert _bitset(oracle.two_sided_rows(n, flat, up, down), n) == want
    assert datalog.two_sided(set(zip(*flat)), set(zip(*up)), set(zip(*down))) == want


@pytest.mark.parametrize("seed", range(8))
def test_quadratic_closure_is_the_squaring_closure(seed):
    """The non-linear program p <- e; p <- p, p has the same least model as the linear P2, and it is
    what the squaring R <- R | R.R computes: the clause evaluator, the linear evaluator, the oracle's
    BFS closure and Algorithm 1's squaring all agree."""
    rng = np.random.default_rng(600 + seed)
    n = int(rng.integers(1, 24))
    A = (rng.random((n, n)) < 0.1).astype(np.uint8)
    e = set(zip(*[x.tolist() for x in np.nonzero(A)]))
    q = datalog.quadratic_closure(e)
    assert q == datalog.closure(e)
    assert q == {(int(i), int(j)) for i, j in zip(*np.nonzero(dense_closure(n, *np.nonzero(A))))}
    assert q == {(int(i), int(j)) for i, j in zip(*np.nonzero(algorithms.rms_squaring_or(A)[0]))}


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 130])
def test_closed_forms(n):
    # empty graph
    assert dense_closure(n, [], []).sum() == 0
    # directed n-cycle: every node reaches every node (itself included)
    s = np.arange(n)
    assert dense_closure(n, s, (s + 1) % n).all()
    # path 0 -> 1 -> ... -> n-1: strictly upper triangular ones
    ps, pd = np.arange(n - 1), np.arange(1, n)
    assert np.array_equal(dense_closure(n, ps, pd), np.triu(np.ones((n, n), np.uint8), 1))
    # complete digraph without loops, n >= 2: all ones
    if n >= 2:
        ii, jj = np.nonzero(1 - np.eye(n, dtype=np.uint8))
        assert dense_closure(n, ii, jj).all()
    # single self-loop at i: e_i e_i^T
    i = n // 2
    want = np.zeros((n, n), np.uint8)
    want[i, i] = 1
    assert np.array_equal(dense_closure(n, [i], [i]), want)


def test_disjoint_union_is_block_diagonal():
    rng = np.random.default_rng(7)
    n1, n2 = 40, 70
    a = (rng.random((n1, n1)) < 0.05).astype(np.uint8)
    b = (rng.random((n2, n2)) < 0.03).astype(np.uint8)
    u = np.zeros((n1 + n2, n1 + n2), np.uint8)
    u[:n1, :n1] = a
    u[n1:, n1:] = b
    cu = dense_closure(n1 + n2, *np.nonzero(u))
    assert np.array_equal(cu[:n1, :n1], dense_closure(n1, *np.nonzero(a)))
    assert np.array_equal(cu[n1:, n1:], dense_closure(n2, *np.nonzero(b)))
    assert cu[:n1, n1:].sum() == 0 and cu[n1:, :n1].sum() == 0


# ---------------------------------------------------------------- brute force
def test_exhaustive_n_le_3():
    for n in (1, 2, 3):
        for code in range(1 << (n * n)):
            A = np.array([(code >> b) & 1 for b in range(n * n)], np.uint8).reshape(n, n)
            want = brute_closure(A)
            s, d = np.nonzero(A)
            assert np.array_equal(dense_closure(n, s, d), want), (n, code)
            assert datalog.closure(set(zip(s.tolist(), d.tolist()))) == \
                {(i, j) for i in range(n) for j in range(n) if want[i, j]}
            assert np.array_equal(algorithms.rms_paper(A)[0], want)
            v = np.zeros((n, n), np.uint8)
            np.fill_diagonal(v, 1)
            assert np.array_equal(algorithms.smp_paper(v, A)[0], want)


def test_exhaustive_n4_bfs_and_warshall():
    n = 4
    codes = np.arange(1 << 16)
    A = ((codes[:, None] >> np.arange(16)[None, :]) & 1).astype(np.int64).reshape(-1, 4, 4)
    P = A.copy()
    acc = A.copy()
    for _ in range(3):
        P = np.minimum(P @ A, 1)
        acc |= P
    want = acc.astype(np.uint8)
    wbits = np.packbits(np.pad(want, ((0, 0), (0, 0), (0, 60))).astype(bool),
                        axis=2, bitorder="little").view("<u8")[..., 0]
    for c in range(1 << 16):
        s, d = np.nonzero(A[c])
        got = oracle.closure_rows(n, s, d)[:, 0]
        assert np.array_equal(got, wbits[c]), c
        bits = np.zeros((4, 1), np.uint64)
        for i in range(4):
            bits[i, 0] = sum(int(A[c, i, j]) << j for j in range(4))
        assert np.array_equal(oracle.warshall(bits, 4)[:, 0], wbits[c]), c


@pytest.mark.parametrize("seed", range(60))
def test_random_small_three_routes(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 65))
    p = float(rng.choice([0.01, 0.03, 0.08, 0.2]))
    A = (rng.random((n, n)) < p).astype(np.uint8)
    s, d = np.nonzero(A)
    got = dense_closure(n, s, d)
    assert np.array_equal(got, brute_closure(A))
    assert np.array_equal(boolops.from_bits(oracle.warshall(boolops.to_bits(A), n), n), got)
    assert np.array_equal(algorithms.rms_paper(A)[0], got)
    assert np.array_equal(algorithms.rms_squaring_or(A)[0], got)
    if n <= 40:
        assert datalog.closure(set(zip(s.tolist(), d.tolist()))) == \
            {(i, j) for i in range(n) for j in range(n) if got[i, j]}


# ---------------------------------------------------------------- selection and composition
@pytest.mark.parametrize("seed", range(20))
def test_smp_matches_alg2_and_row_or(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(2, 90))
    A = (rng.random((n, n)) < 0.04).astype(np.uint8)
    s, d = np.nonzero(A)
    k = int(rng.integers(1, 8))
    V = (rng.random((k, n)) < 0.05).astype(np.uint8)
    V[0] = 0
    V[0, rng.integers(n)] = 1
    got = boolops.from_bits(oracle.smp(n, s, d, boolops.to_bits(V)), n)
    C = dense_closure(n, s, d)
    assert np.array_equal(got, boolops.mul(V, C))  # Eq. 5: v* = v R2*
    for r in range(k):
        assert np.array_equal(algorithms.smp_paper(V[r], A)[0][0], got[r])
    refl = boolops.from_bits(oracle.smp(n, s, d, boolops.to_bits(V), reflexive=True), n)
    assert np.array_equal(refl, boolops.add(V, got))


def test_smp_strictness():
    # 0 -> 1 -> 2, 2 -> 1: source 0 is not on a cycle, 1 is
    n = 3
    s, d = [0, 1, 2], [1, 2, 1]
    V = boolops.to_bits(np.eye(3, dtype=np.uint8))
    got = boolops.from_bits(oracle.smp(n, s, d, V), n)
    assert got.tolist() == [[0, 1, 1], [0, 1, 1], [0, 1, 1]]


@pytest.mark.parametrize("seed", range(20))
def test_compose_definitions(seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(1, 70))
    B = (rng.random((n, n)) < 0.05).astype(np.uint8)
    S = (rng.random((n, n)) < 0.05).astype(np.uint8)
    P = boolops.from_bits(oracle.compose_rows(n, *np.nonzero(B), *np.nonzero(S)), n)
    Splus = brute_closure(S)
    assert np.array_equal(P, boolops.add(B, boolops.mul(Splus, B)))   # Rb + Rs+ Rb
    assert np.array_equal(P, boolops.add(B, boolops.mul(S, P)))       # least fixpoint eq.
    if n <= 30:
        pairs = datalog.linear(set(zip(*map(list, np.nonzero(B)))), set(zip(*map(list, np.nonzero(S)))))
        assert pairs == {(i, j) for i in range(n) for j in range(n) if P[i, j]}
    # compose(R, R) = R+
    Q = boolops.from_bits(oracle.compose_rows(n, *np.nonzero(S), *np.nonzero(S)), n)
    assert np.array_equal(Q, Splus)


def test_rows_subset_matches_full():
    rng = np.random.default_rng(3)
    n = 300
    A = (rng.random((n, n)) < 0.01).astype(np.uint8)
    s, d = np.nonzero(A)
    full = oracle.closure_rows(n, s, d)
    rows = rng.choice(n, 17, replace=False)
    assert np.array_equal(oracle.closure_rows(n, s, d, rows=rows), full[rows])
    B = (rng.random((n, n)) < 0.01).astype(np.uint8)
    fullc = oracle.compose_rows(n, *np.nonzero(B), s, d)
    assert np.array_equal(oracle.compose_rows(n, *np.nonzero(B), s, d, rows=rows), fullc[rows])


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("seed", range(10))
def test_closure_invariants(seed):
    rng = np.random.default_rng(1300 + seed)
    n = int(rng.integers(20, 200))
    A = (rng.random((n, n)) < 1.5 / n).astype(np.uint8)
    s, d = np.nonzero(A)
    C = dense_closure(n, s, d)
    assert (A <= C).all()                                            # R subset R+
    assert (boolops.mul(C, C) <= C).all()                            # R+ R+ subset R+
    assert np.array_equal(dense_closure(n, *np.nonzero(C)), C)      # idempotent
    assert np.array_equal(C, boolops.add(A, boolops.mul(A, C)))     # Eq. 1 fixed point
    assert np.array_equal(dense_closure(n, d, s), C.T)              # (R^T)+ = (R+)^T
    A2 = A.copy()
    A2[rng.integers(n), rng.integers(n)] = 1
    assert (C <= dense_closure(n, *np.nonzero(A2))).all()           # monotone


def test_dag_zero_diagonal():
    rng = np.random.default_rng(4)
    n = 120
    A = np.triu((rng.random((n, n)) < 0.05).astype(np.uint8), 1)
    perm = rng.permutation(n)
    A = A[perm][:, perm]
    assert np.diagonal(dense_closure(n, *np.nonzero(A))).sum() == 0


# ---------------------------------------------------------------- loop logic
@pytest.mark.parametrize("n", [2, 3, 5, 9, 17, 100])
def test_path_graph_loop_counts(n):
    A = np.eye(n, k=1, dtype=np.uint8)
    R, sq, prods = algorithms.rms_paper(A)
    assert sq == math.ceil(math.log2(n - 1)) + 1 and prods == sq + 1
    R2, p2 = algorithms.rms_squaring_or(A)
    assert p2 == math.ceil(math.log2(n - 1)) + 1
    v = np.zeros(n, np.uint8)
    v[0] = 1
    vs, it, _ = algorithms.smp_paper(v, A)
    assert it == n
    assert np.array_equal(vs[0], np.r_[0, np.ones(n - 1, np.uint8)])


# ---------------------------------------------------------------- operators and layout
def test_boolean_product_is_or_of_ands():
    rng = np.random.default_rng(5)
    for _ in range(30):
        m, k, n = rng.integers(1, 7, size=3)
        A = (rng.random((m, k)) < 0.4).astype(np.uint8)
        B = (rng.random((k, n)) < 0.4).astype(np.uint8)
        want = np.array([[int(any(A[i, t] and B[t, j] for t in range(k))) for j in range(n)]
                         for i in range(m)], np.uint8)
        assert np.array_equal(boolops.mul(A, B), want)


def test_bit_layout_lsb_first():
    d = np.zeros((1, 130), np.uint8)
    d[0, [0, 63, 64, 129]] = 1
    b = boolops.to_bits(d)
    assert b.shape == (1, 3)
    assert int(b[0, 0]) == (1 | (1 << 63)) and int(b[0, 1]) == 1 and int(b[0, 2]) == 2
    assert np.array_equal(boolops.from_bits(b, 130), d)
    assert boolops.to_bits(d, ld=8).shape == (1, 8)


def test_oracle_threads_reported():
    s, d = np.arange(99), np.arange(1, 100)
    oracle.closure_rows(100, s, d, threads=2)
    assert oracle.last_threads == 2
    # a later call with the default does not inherit the fixed count
    oracle.closure_rows(100, s, d, threads=1)
    oracle.closure_rows(100, s, d)
    expect = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    assert oracle.last_threads == expect
