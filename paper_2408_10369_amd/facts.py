"""Facts to matrices and back (Section 3.2), around the device path.

* ``parse_facts`` reads ground facts written in Prolog syntax (``edge(a,b).``,
  ``node(a).``; ``%`` comments; clauses with a body are skipped) into a dict
  predicate -> list of argument tuples.
* ``SymbolTable`` is the bijection of Section 3.2 between constants and the
  indices 0..n-1, in the order the constants are first added.
* ``compile_relation`` / ``compile_set`` pack a dyadic predicate into an
  n x n bit matrix and a monadic one into a 1 x n row on the device
  (``bmlp_pack_coo``); ``relation_facts`` decodes a matrix back into facts on
  the device (``bmlp_unpack_coo``) and names them through the table;
  ``row_codes`` gives the paper's row encoding v(i, b_i), one binary code per
  row with bit j first for column j.

Only the symbol table and the text live on the host; packing and decoding run
in the library's kernels.
"""
from __future__ import annotations

import re

import numpy as np


def _statements(text: str):
    """Split Prolog text into clauses at the full stops outside quotes, parentheses and comments."""
    out, cur, depth, quote, i = [], [], 0, None, 0
    while i < len(text):
        ch = text[i]
        if quote:
            cur.append(ch)
            if ch == "\\" and i + 1 < len(text):
                cur.append(text[i + 1])
                i += 1
            elif ch == quote:
                quote = None
        elif ch == "%":
            while i < len(text) and text[i] != "\n":
                i += 1
            continue
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = len(text) if j < 0 else j + 2
            cur.append(" ")
            continue
        elif ch in "'\"":
            quote = ch
            cur.append(ch)
        elif ch == "(":
            depth += 1
            cur.append(ch)
        elif ch == ")":
            depth -= 1
            cur.append(ch)
        elif ch == "." and depth == 0 and (i + 1 == len(text) or text[i + 1].isspace()):
            out.append("".join(cur).strip())
            cur = []
        else:
            cur.append(ch)
        i += 1
    if "".join(cur).strip():
        raise ValueError(f"clause without a final full stop: {''.join(cur).strip()!r}")
    return out


_HEAD = re.compile(r"([a-z][A-Za-z0-9_]*)\s*(?:\((.*)\))?", re.S)


def _split_args(args: str):
    out, cur, quote = [], [], None
    for ch in args:
        if quote:
            cur.append(ch)
            if ch == quote:
                quote = None
        elif ch in "'\"":
            quote = ch
            cur.append(ch)
        elif ch == ",":
            out.append("".join(cur).strip())
            cur = []
        else:
            cur.append(ch)
    out.append("".join(cur).strip())
    return out


def parse_facts(text: str) -> dict:
    """Ground facts of a Prolog text: {predicate: [tuple of argument names, ...]} in text order.
    Clauses with a body (``:-``) and directives are skipped."""
    out: dict = {}
    for stmt in _statements(text):
        if not stmt or ":-" in stmt or stmt.startswith("?-"):
            continue
        m = _HEAD.fullmatch(stmt)
        if not m:
            raise ValueError(f"not a ground fact: {stmt!r}")
        pred, args = m.group(1), m.group(2)
        names = []
        if args is not None:
            for tok in _split_args(args):
                if not tok:
                    raise ValueError(f"empty argument in {stmt!r}")
                if tok[0] in "'\"":
                    tok = tok[1:-1]
                elif tok[0].isupper() or tok[0] == "_":
                    raise ValueError(f"variable in a fact: {stmt!r}")
                elif not re.fullmatch(r"[A-Za-z0-9_.+-]+", tok):
                    raise ValueError(f"compound or bad argument in {stmt!r}")
                names.append(tok)
        out.setdefault(pred, []).append(tuple(names))
    return out


class SymbolTable:
    """Constants <-> indices 0..n-1 (first-added order)."""

    def __init__(self, names=()):
        self._index: dict = {}
        self._names: list = []
        for x in names:
            self.add(x)

    def add(self, name: str) -> int:
        i = self._index.get(name)
        if i is None:
            i = len(self._names)
            self._index[name] = i
            self._names.append(name)
        return i

    def __len__(self) -> int:
        return len(self._names)

    def index(self, names) -> np.ndarray:
        return np.fromiter((self._index[x] for x in names), dtype=np.int32, count=len(names))

    def names(self, idx) -> list:
        return [self._names[int(i)] for i in idx]

    @classmethod
    def from_facts(cls, facts: dict, predicates=None) -> "SymbolTable":
        """Every constant of the given predicates (all by default), in order of appearance."""
        t = cls()
        for pred, rows in facts.items():
            if predicates is not None and pred not in predicates:
                continue
            for args in rows:
                for x in args:
                    t.add(x)
        return t


def compile_relation(ctx, table: SymbolTable, pairs, ld=None):
    """n x n bit matrix of a dyadic predicate's facts (a list of (x, y) name pairs) on the device."""
    import torch
    n = len(table)
    src = table.index([p[0] for p in pairs])
    dst = table.index([p[1] for p in pairs])
    return ctx.pack_coo(torch.as_tensor(src), torch.as_tensor(dst), n, n, ld)


def compile_set(ctx, table: SymbolTable, names, ld=None):
    """1 x n bit row of a monadic predicate's facts (a list of names) on the device."""
    import torch
    n = len(table)
    idx = table.index(list(names))
    return ctx.pack_coo(torch.zeros(len(idx), dtype=torch.int32), torch.as_tensor(idx), 1, n, ld)


def relation_facts(ctx, table: SymbolTable, bits, pred: str) -> list:
    """The facts pred(x, y) of a bit matrix, decoded on the device, sorted by (x, y) index."""
    r, c = ctx.unpack_coo(bits, len(table))
    rs = table.names(r.cpu().numpy())
    cs = table.names(c.cpu().numpy())
    return [f"{pred}({a},{b})" for a, b in zip(rs, cs)]


def row_codes(ctx, bits, n: int) -> list:
    """Section 3.2's encoding of a matrix as facts v(i, b_i): the binary code of each row, column j at
    position j."""
    dense = ctx.unpack_u8(bits, n).cpu().numpy()
    return ["".join("1" if v else "0" for v in row) for row in dense]
