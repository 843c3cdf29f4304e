"""Pure-Python semi-naive bottom-up evaluation over sets of pairs.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Tiny inputs only.

These evaluate the paper's datalog programs directly from their clauses,
without matrices, so they pin the matrix formulations from outside:

* ``linear`` evaluates  p(X,Y) <- b(X,Y).  p(X,Y) <- s(X,Z), p(Z,Y).
  (the program P2 of Section 3.3 when b = s = r1; the general linear
  recursion of Section 3.4 otherwise).  Semi-naive: each round joins the
  step relation only with the facts that were new in the previous round.
* ``is_foreign`` evaluates P3 u P4 u P5 of Section 3.4 stratum by stratum:
  hasPlace, then indirectlyPartOf, then isForeign with negation against the
  finished lower stratum.
* ``quadratic_closure`` evaluates the non-linear transitive closure
  p(X,Y) <- e(X,Y).  p(X,Y) <- p(X,Z), p(Z,Y).  (two recursive atoms).
* ``two_sided`` evaluates  p(X,Y) <- b(X,Y).  p(X,Y) <- l(X,X1), p(X1,Y1), r(Y1,Y).
  (same-generation when l = up and r = down), a linear program whose
  recursive atom has a relation on each side.
"""
from __future__ import annotations


def linear(base, step):
    """Least model of p <- b; p <- s, p (sets of (x, y) pairs)."""
    base = set(base)
    succ_inv = {}
    for (x, z) in step:
        succ_inv.setdefault(z, []).append(x)
    p = set(base)
    delta = set(base)
    while delta:
        new = set()
        for (z, y) in delta:
            for x in succ_inv.get(z, ()):
                if (x, y) not in p:
                    new.add((x, y))
        p |= new
        delta = new
    return p


def closure(edges):
    """P2: r2 <- r1; r2 <- r1, r2."""
    return linear(edges, edges)


def is_foreign(constants, contains, adjoins, location=None):
    """The P3 u P4 u P5 program of Section 3.4; returns the four relations."""
    location = set(constants) if location is None else set(location)
    has_place = linear(contains, contains)
    # indirectlyPartOf(X,Y) <- adjoins(X,Y) | adjoins(Y,X)
    #                        | hasPlace(Z,X), indirectlyPartOf(Z,Y)
    base = set(adjoins) | {(y, x) for (x, y) in adjoins}
    step = {(x, z) for (z, x) in has_place}  # s(X,Z) := hasPlace(Z,X)
    ipo = linear(base, step)
    foreign = {(x, y) for x in location for y in location if (x, y) not in ipo}
    return has_place, ipo, foreign


def two_sided(base, left, right):
    """Least model of p <- b; p <- l, p, r (sets of (x, y) pairs), semi-naive."""
    pre = {}
    for (x, x1) in left:
        pre.setdefault(x1, []).append(x)
    post = {}
    for (y1, y) in right:
        post.setdefault(y1, []).append(y)
    p = set(base)
    delta = set(base)
    while delta:
        new = set()
        for (x1, y1) in delta:
            for x in pre.get(x1, ()):
                for y in post.get(y1, ()):
                    if (x, y) not in p:
                        new.add((x, y))
        p |= new
        delta = new
    return p


def quadratic_closure(edges):
    """Least model of p <- e; p <- p, p (non-linear transitive closure), semi-naive: a new fact is
    joined with every known fact on either side."""
    p = set(edges)
    delta = set(edges)
    while delta:
        succ, pred = {}, {}
        for (x, y) in p:
            succ.setdefault(x, set()).add(y)
            pred.setdefault(y, set()).add(x)
        new = set()
        for (x, z) in delta:
            for y in succ.get(z, ()):
                if (x, y) not in p:
                    new.add((x, y))
            for w in pred.get(x, ()):
                if (w, z) not in p:
                    new.add((w, z))
        p |= new
        delta = new
    return p
