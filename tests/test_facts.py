"""Host side of the fact <-> matrix pipeline (Section 3.2): the Prolog fact
reader and the symbol table.  No GPU."""
import numpy as np
import pytest

from paper_2408_10369_amd.facts import SymbolTable, parse_facts

EXAMPLE = """% Example 1 of Section 3.2: edge facts over a, b, c
node(a). node(b). node(c).
edge(a,b).
edge(b, c).   /* a block comment. with a full stop */
path(X,Y) :- edge(X,Y).
path(X,Y) :- edge(X,Z), path(Z,Y).
"""


def test_parse_example():
    f = parse_facts(EXAMPLE)
    assert f == {"node": [("a",), ("b",), ("c",)], "edge": [("a", "b"), ("b", "c")]}
    t = SymbolTable.from_facts(f, ["node"])
    assert len(t) == 3 and list(t.index(["a", "b", "c"])) == [0, 1, 2] and t.names([2, 0]) == ["c", "a"]


def test_parse_quotes_numbers_and_atoms():
    f = parse_facts("w('x y', \"q.r\"). n(1, 2.5). flag.\ncontains('New York', 'Brooklyn').")
    assert f == {"w": [("x y", "q.r")], "n": [("1", "2.5")], "flag": [()],
                 "contains": [("New York", "Brooklyn")]}


@pytest.mark.parametrize("bad", ["edge(X,b).", "edge(a,b)", "edge(f(a),b).", "edge(a,,b).", "Edge(a,b)."])
def test_parse_errors(bad):
    with pytest.raises(ValueError):
        parse_facts(bad)


def test_symbol_table_order_and_reuse():
    t = SymbolTable(["g1", "g2"])
    assert t.add("t1") == 2 and t.add("g1") == 0 and len(t) == 3
    f = parse_facts("contains(t1,g2). contains(g3,t1). adjoins(g3,g4).")
    t = SymbolTable.from_facts(f)
    assert t.names(range(len(t))) == ["t1", "g2", "g3", "g4"]
    assert np.array_equal(t.index(["g4", "t1"]), np.array([3, 0], np.int32))
