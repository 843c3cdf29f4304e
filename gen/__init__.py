"""Seeded synthetic inputs for the BMLP hot path.

This module only draws random graphs, query sources and programs.  It holds
none of the method's arithmetic: no bit packing, no products, no closures.
Both the oracle and the HIP path take their inputs from here, so a workload
is identical on the two sides by construction.

Every graph is returned as a COO edge list (``src``, ``dst``: int32 arrays,
sorted by ``(src, dst)``, no duplicates) over node indices ``0..n-1``.  Node
indices stand for the constants of a datalog program after the bijection onto
the naturals that the paper's matrix encoding uses (Section 3.2); edge
``(i, j)`` is the fact ``r1(c_i, c_j)``.

Workload recipes (shapes follow the paper's benchmarks, Section 6.1 and
Table 1; the sizes are those of the five benchmark configurations):

* ``er_digraph``: directed Erdos-Renyi graph, every ordered pair ``i != j``
  an edge independently with probability ``p`` (the DG / DG+partial graphs of
  Section 6.3).  Sampled exactly: ``m ~ Binomial(n(n-1), p)`` and then ``m``
  distinct ordered pairs uniformly, which is the same distribution.
* ``sources``: ``k`` distinct source nodes drawn uniformly (the constants of
  the partially grounded queries ``r2(c, Y)``).
* ``batch_graphs``: 512 uneven random graphs, ``n`` log-uniform in
  [64, 4096], mean out-degree uniform in [2, 8].
* ``multirel``: a multi-relational graph shaped like Freebase 15K (the paper's
  third benchmark; the dataset itself is not used): 14,951 entities, 1,345
  relations with Zipf(1.1) triple counts summing to 592,000, power-law entity
  degrees; plus seeded two-relation linear programs over it.
* ``scalefree_digraph``: directed Chung-Lu graph with power-law weights,
  ``n = 65,536``, exactly ``m = 262,144`` edges.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "er_digraph", "sources", "query_lists", "c1", "c2", "C2_PROBS", "C2_KS",
    "batch_graphs", "BatchGraph", "multirel", "MultiRel", "programs",
    "scalefree_digraph", "query_stream", "path_graph", "cycle_graph", "tail_core",
]


def _dedupe_sorted(src: np.ndarray, dst: np.ndarray, n: int):
    key = src.astype(np.int64) * n + dst.astype(np.int64)
    key = np.unique(key)
    return (key // n).astype(np.int32), (key % n).astype(np.int32)


def er_digraph(n: int, p: float, seed: int):
    """Directed ER graph: each ordered pair (i, j), i != j, w.p. ``p``."""
    rng = np.random.default_rng(seed)
    npairs = n * (n - 1)
    if n < 2 or p <= 0.0:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    m = int(rng.binomial(npairs, min(p, 1.0)))
    idx = rng.choice(npairs, size=m, replace=False) if m < npairs else np.arange(npairs)
    idx = np.sort(idx.astype(np.int64))
    i = idx // (n - 1)
    jj = idx % (n - 1)
    j = jj + (jj >= i)
    return i.astype(np.int32), j.astype(np.int32)


def sources(n: int, k: int, seed: int) -> np.ndarray:
    """``k`` distinct source nodes, uniform without replacement."""
    rng = np.random.default_rng(seed)
    return rng.choice(n, size=k, replace=False).astype(np.int32)


def query_lists(srcs: np.ndarray):
    """One one-hot query row per source: returns (row_index, column) COO pairs."""
    k = len(srcs)
    return np.arange(k, dtype=np.int32), np.asarray(srcs, dtype=np.int32)


def path_graph(n: int):
    s = np.arange(max(n - 1, 0), dtype=np.int32)
    return s, s + 1


def cycle_graph(n: int):
    s = np.arange(n, dtype=np.int32)
    return s, ((s + 1) % n).astype(np.int32)


def tail_core(n: int, core: int, tail: int, deg: float, seed: int):
    """A strongly connected random core (nodes 0..core-1: a random Hamiltonian cycle plus ER edges of mean
    out-degree ``deg``) and a chain of ``tail`` nodes (core .. core+tail-1) whose last node points into the
    core; the remaining nodes are isolated.  Row c of the chain reaches the whole core at a distance that
    grows along the chain, so late closure rounds add many bits to few rows."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(core).astype(np.int32)
    s = [perm, np.zeros(0, np.int32)]
    d = [np.roll(perm, -1), np.zeros(0, np.int32)]
    es, ed = er_digraph(core, deg / max(core - 1, 1), seed + 1)
    s.append(es)
    d.append(ed)
    ch = np.arange(core, core + tail, dtype=np.int32)
    s.append(ch)
    d.append(np.r_[ch[1:], np.int32(perm[0])].astype(np.int32))
    src, dst = np.concatenate(s), np.concatenate(d)
    return _dedupe_sorted(src, dst, n)


# --- first configuration: one small ER graph ---------------------------------
def c1():
    """n=1,000, p=0.002, seed 1; 10 sources (seed 11)."""
    n = 1000
    s, d = er_digraph(n, 0.002, 1)
    return n, s, d, sources(n, 10, 11)


# --- second configuration: n=16,384 density sweep ----------------------------
C2_PROBS = (1e-4, 5e-4, 1e-3, 5e-3, 1e-2)
C2_KS = (1, 64, 1024)


def c2(pi: int):
    """Graph ``pi`` of the sweep: n=16,384, p=C2_PROBS[pi], seed 2000+pi."""
    n = 16384
    s, d = er_digraph(n, C2_PROBS[pi], 2000 + pi)
    return n, s, d


def c2_sources(pi: int, ki: int):
    return sources(16384, C2_KS[ki], 2100 + 10 * pi + ki)


# --- third configuration: 512 uneven graphs ----------------------------------
@dataclass
class BatchGraph:
    n: int
    src: np.ndarray
    dst: np.ndarray
    srcs: np.ndarray  # 64 query sources


def batch_graphs(count: int = 512, base_seed: int = 3000, k: int = 64,
                 nmin: int = 64, nmax: int = 4096):
    out = []
    for g in range(count):
        rng = np.random.default_rng(base_seed + g)
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        n = min(max(n, nmin), nmax)
        deg = rng.uniform(2.0, 8.0)
        p = deg / (n - 1)
        s, d = er_digraph(n, p, int(rng.integers(1 << 31)))
        srcs = rng.choice(n, size=min(k, n), replace=False).astype(np.int32)
        out.append(BatchGraph(n, s, d, srcs))
    return out


# --- fourth configuration: multi-relational graph + linear programs ----------
@dataclass
class MultiRel:
    n: int
    rel_src: list  # per relation: int32 array of heads
    rel_dst: list  # per relation: int32 array of tails
    counts: np.ndarray


def _zipf_counts(nrel: int, total: int, s: float) -> np.ndarray:
    w = np.arange(1, nrel + 1, dtype=np.float64) ** (-s)
    c = np.maximum(1, np.floor(w / w.sum() * total)).astype(np.int64)
    # distribute the remainder to the most frequent relations, deterministically
    rem = total - int(c.sum())
    i = 0
    while rem > 0:
        c[i % nrel] += 1
        rem -= 1
        i += 1
    return c


def multirel(n: int = 14951, nrel: int = 1345, total: int = 592000,
             s: float = 1.1, ent_exp: float = 0.8, seed: int = 4) -> MultiRel:
    """Synthetic stand-in shaped like Freebase 15K (not its data)."""
    rng = np.random.default_rng(seed)
    counts = _zipf_counts(nrel, total, s)
    perm = rng.permutation(n)
    w = np.empty(n)
    w[perm] = np.arange(1, n + 1, dtype=np.float64) ** (-ent_exp)
    w /= w.sum()
    rs, rd = [], []
    for r in range(nrel):
        want = int(counts[r])
        want = min(want, n * (n - 1))
        hs = np.zeros(0, np.int32)
        ts = np.zeros(0, np.int32)
        while len(hs) < want:
            need = want - len(hs)
            h = rng.choice(n, size=need + 8, p=w)
            t = rng.choice(n, size=need + 8, p=w)
            keep = h != t
            hs2, ts2 = _dedupe_sorted(np.concatenate([hs, h[keep]]),
                                      np.concatenate([ts, t[keep]]), n)
            hs, ts = hs2, ts2
        if len(hs) > want:
            sel = np.sort(rng.choice(len(hs), size=want, replace=False))
            hs, ts = hs[sel], ts[sel]
        rs.append(hs.astype(np.int32))
        rd.append(ts.astype(np.int32))
    return MultiRel(n, rs, rd, counts)


def programs(mr: MultiRel, count: int = 100, base_seed: int = 4000):
    """Programs ``p <- r_base; p <- r_step, p`` as (base, step) relation ids.

    Both relations are drawn with probability proportional to their triple
    count; ``base == step`` is allowed (it is the plain transitive closure).
    """
    pr = mr.counts / mr.counts.sum()
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        base = int(rng.choice(len(pr), p=pr))
        step = int(rng.choice(len(pr), p=pr))
        out.append((base, step))
    return out


# --- fifth configuration: large scale-free graph + query stream --------------
def scalefree_digraph(n: int = 65536, m: int = 262144, exp: float = 0.8,
                      seed: int = 5):
    """Directed Chung-Lu graph: P(u->v) ~ w_out(u) w_in(v), power-law weights."""
    rng = np.random.default_rng(seed)
    ranks = np.arange(1, n + 1, dtype=np.float64) ** (-exp)
    wout = np.empty(n)
    win = np.empty(n)
    wout[rng.permutation(n)] = ranks
    win[rng.permutation(n)] = ranks
    wout /= wout.sum()
    win /= win.sum()
    s = np.zeros(0, np.int32)
    d = np.zeros(0, np.int32)
    while len(s) < m:
        need = m - len(s)
        a = rng.choice(n, size=need + 64, p=wout)
        b = rng.choice(n, size=need + 64, p=win)
        keep = a != b
        s, d = _dedupe_sorted(np.concatenate([s, a[keep]]),
                              np.concatenate([d, b[keep]]), n)
    if len(s) > m:
        sel = np.sort(rng.choice(len(s), size=m, replace=False))
        s, d = s[sel], d[sel]
    return s.astype(np.int32), d.astype(np.int32)


def query_stream(n: int = 65536, count: int = 10000, kmax: int = 4096,
                 base_seed: int = 50000):
    """``count`` queries; query q has k ~ log-uniform integer in [1, kmax]."""
    out = []
    for q in range(count):
        rng = np.random.default_rng(base_seed + q)
        k = int(math.floor(math.exp(rng.uniform(0.0, math.log(kmax + 1)))))
        k = min(max(k, 1), kmax)
        out.append(rng.choice(n, size=k, replace=False).astype(np.int32))
    return out


# --- the composition benchmark of Section 3.4 at knowledge-graph scale --------
@dataclass
class Geo:
    n: int
    contains_src: np.ndarray
    contains_dst: np.ndarray
    adjoins_src: np.ndarray
    adjoins_dst: np.ndarray
    location: np.ndarray      # indices of the constants that are locations


def geo(n: int = 14541, levels=(20, 200, 1000, 2780), seed: int = 6,
        extra_parent: float = 0.05, adjoin_p: float = 0.73) -> Geo:
    """Synthetic geography shaped like the FB15K-237 location facts.

    Locations are a random subset of the n constants arranged in levels
    (countries, regions, counties, cities).  contains(parent, child): each
    location below the top level has a parent one level up, and with
    probability ``extra_parent`` a second one (a place inside two regions).
    adjoins(x, y): each location makes two tries, each succeeding with
    probability ``adjoin_p``, at adjoining another location of the same parent
    (a sibling).  The defaults give 4,172 contains and 3,811 adjoins facts,
    7,983 in all (the paper's table lists 7,991 over 14,541 constants).
    ``location`` lists the constants of the hierarchy; the paper's reading
    makes every constant a location, which callers get by passing all n.
    """
    rng = np.random.default_rng(seed)
    total = int(sum(levels))
    loc = rng.permutation(n)[:total].astype(np.int32)
    lv = []
    off = 0
    for c in levels:
        lv.append(loc[off:off + c])
        off += c
    cs, cd, parent = [], [], {}
    for li in range(1, len(lv)):
        up = lv[li - 1]
        for x in lv[li]:
            p = int(up[rng.integers(len(up))])
            parent[int(x)] = p
            cs.append(p)
            cd.append(int(x))
            if rng.random() < extra_parent:
                q = int(up[rng.integers(len(up))])
                if q != p:
                    cs.append(q)
                    cd.append(int(x))
    sib = {}
    for x, p in parent.items():
        sib.setdefault(p, []).append(x)
    sib[-1] = [int(x) for x in lv[0]]
    as_, ad = [], []
    for group in sib.values():
        if len(group) < 2:
            continue
        for x in group:
            for _ in range(2):
                if rng.random() < adjoin_p:
                    y = group[rng.integers(len(group))]
                    if y != x:
                        as_.append(x)
                        ad.append(y)
    cs, cd = _dedupe_sorted(np.asarray(cs, np.int32), np.asarray(cd, np.int32), n)
    as_, ad = _dedupe_sorted(np.asarray(as_, np.int32), np.asarray(ad, np.int32), n)
    return Geo(n, cs, cd, as_, ad, np.sort(loc))


# --- forests for the two-sided (same-generation) program ----------------------
@dataclass
class Forest:
    n: int
    child: np.ndarray    # edge child -> parent, as (child, parent) pairs
    parent: np.ndarray
    depth: np.ndarray    # depth of every node (roots 0)
    root: np.ndarray     # root of every node's tree


def forest(n: int = 16384, trees: int = 8, seed: int = 8, max_children: int = 4) -> Forest:
    """A random forest: nodes 0..trees-1 are roots; every later node picks a random parent among the
    nodes before it whose child count is below ``max_children`` (shapes vary from bushy to deep)."""
    rng = np.random.default_rng(seed)
    parent = np.full(n, -1, np.int64)
    depth = np.zeros(n, np.int64)
    root = np.arange(n, dtype=np.int64)
    kids = np.zeros(n, np.int64)
    open_ = list(range(min(trees, n)))
    for v in range(min(trees, n), n):
        i = int(rng.integers(len(open_)))
        p = open_[i]
        parent[v] = p
        depth[v] = depth[p] + 1
        root[v] = root[p]
        kids[p] += 1
        if kids[p] >= max_children:
            open_[i] = open_[-1]
            open_.pop()
        open_.append(v)
    ch = np.nonzero(parent >= 0)[0]
    return Forest(n, ch.astype(np.int32), parent[ch].astype(np.int32), depth, root)
