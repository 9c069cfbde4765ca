"""Process compiler for tree-level QCD processes with several quark lines
(build time): the two-jet channels of p p -> t tbar (q qbar -> t tbar g g,
q g -> t tbar q g, g g -> t tbar q qbar, the four-quark channels).

Diagrams.  Every diagram contains the top line, whose outgoing top (leg 2,
a row spinor ubar) sits at exactly one vertex: the diagram is that vertex
closing a gluon sub-diagram and a column-ended top sub-diagram over the other
legs.  Sub-diagrams are built bottom-up over bitmasks of legs, each one a
HELAS-style call joining smaller sub-diagrams:
    column current + gluon        -> column current     (ffv_fin)
    row current + gluon           -> row current        (ffv_fout)
    row + column of one flavour   -> gluon              (ffv_v0)
    gluon + gluon                 -> gluon              (vvv_v)
    gluon + gluon + gluon         -> gluon, one call per colour structure
                                     of the four-gluon vertex (vvvv_v)
(column ends: incoming quarks u, outgoing antiquarks v; row ends: outgoing
quarks ubar, incoming antiquarks vbar).  Equal sub-diagrams are one value,
so the schedule computes each once per helicity.

Colour.  Each diagram's colour factor is the explicit tensor over the
colours of all external legs, contracted numerically from the Gell-Mann
generators: t^a_{new,old} at a column vertex, t^a_{old,new} at a row vertex,
t^x_{row,column} where a line closes into a gluon x, f^{x a b} at a
three-gluon vertex and f^{x y e} f^{e z w} for the four-gluon structure
(y; z, w).  With quark lines present every tree colour factor is a
combination of products of open strings (t^{a..} ... t^{a..})_{row, column},
one per line, over all ways of joining row ends to column ends and of
ordering the gluons on the strings: a linearly independent subset of those
products that spans the diagrams is the colour basis, the coordinates of
each diagram in it (rationals, made integer by a common scale) its jamp
coefficients, and sum_colours conj(b_k) b_l the colour matrix.

Fermi statistics.  With several fermion lines a diagram carries the sign of
the permutation that takes the external fermions, in leg order, to (row end,
column end) of each of its lines in turn.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from functools import lru_cache
from math import gcd

import numpy as np

from .program import Op, Program, _incoming_count, add_kinematics, share_half_contractions  # noqa: F401

LIGHT = ("u", "d")


def _anti(x):
    return x[:-1] if x.endswith("~") else x + "~"


def _legs(process):
    a, b = process.split(">")
    return [(x, True) for x in a.split()] + [(x, False) for x in b.split()]


# ------------------------------------------------------------ SU(3) numerics
@lru_cache(maxsize=None)
def _gen():
    """t^a = lambda^a / 2 and f^{abc} from [t^a, t^b] = i f^{abc} t^c."""
    lam = np.zeros((8, 3, 3), dtype=complex)
    pairs = [(0, 1), (0, 2), (1, 2)]
    k = 0
    for (i, j) in pairs:                       # symmetric and antisymmetric off-diagonal
        lam[k][i, j] = lam[k][j, i] = 1
        lam[k + 1][i, j], lam[k + 1][j, i] = -1j, 1j
        k += 2
    lam[6] = np.diag([1, -1, 0])
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    t = lam / 2
    f = np.zeros((8, 8, 8))
    for a, b, c in itertools.product(range(8), repeat=3):
        f[a, b, c] = (-2j * np.trace(t[a] @ (t[b] @ t[c] - t[c] @ t[b]))).real
    return t, f


class _Sub:
    """A sub-diagram over the legs in `mask`: kind 'g', 'col' or 'row'
    (flavour `flav` for fermion currents), its value name, its colour
    tensor (axes: legs of mask in order, then its own index), its open
    fermion end and completed fermion lines; extra: how many of its
    four-gluon vertices use their second or third colour structure (the
    Feynman diagrams are the sub-diagrams with none)."""
    __slots__ = ("kind", "flav", "mask", "name", "colour", "end", "lines", "extra")

    def __init__(self, kind, flav, mask, name, colour, end=None, lines=(), extra=0):
        self.kind, self.flav, self.mask, self.name, self.colour = kind, flav, mask, name, colour
        self.end, self.lines, self.extra = end, lines, extra


def _sign(lines):
    seq = [i for ln in sorted(lines) for i in ln]
    inv = sum(1 for a in range(len(seq)) for b in range(a + 1, len(seq)) if seq[a] > seq[b])
    return -1 if inv % 2 else 1


def _mask_legs(m):
    return [i for i in range(m.bit_length()) if m >> i & 1]


def general_program(name: str, process: str, share_half: bool = False) -> Program:
    legs = _legs(process)
    n = len(legs)
    if [x for x, _ in legs[2:4]] != ["t", "t~"]:
        raise ValueError("legs 2 and 3 must be t t~")
    field = [x if (not inc or x == "g") else _anti(x) for x, inc in legs]
    dims = [8 if f == "g" else 3 for f in field]
    iden = 1
    for x, inc in legs:
        if inc:
            iden *= 2 * (8 if x == "g" else 3)
    finals = [x for x, inc in legs if not inc]
    for x in set(finals):
        for k in range(2, finals.count(x) + 1):
            iden *= k
    prog = Program(name=name, process=process, npar=n, leg_sign=[1, 1] + [-1] * (n - 2), ncolor=0,
                   colour_num=[], colour_den=1, iden=iden, n_diagrams=0)
    t, f = _gen()
    L = "abcdefgh"                           # leg axes in the colour tensors

    def define(nm, ops):
        ops = [add_kinematics(prog, op) for op in ops]
        prog.values[nm] = ops
        deps = []
        for op in ops:
            for v in op.ins:
                if v != nm and v not in deps:
                    deps.append(v)
        prog.deps[nm] = deps
        return nm

    def axes(m):
        return "".join(L[i] for i in _mask_legs(m))

    def fkind(flav, m):
        if flav in LIGHT:
            return "quark"
        return "top_t" if _incoming_count(m) == 1 else "top_s"

    # external wavefunctions
    subs = {}
    for i, (x, inc) in enumerate(legs):
        m = 1 << i
        if field[i] == "g":
            nm = define(f"w{i}", [Op("ext_eps", f"w{i}", [], {"leg": i, "conj": not inc})])
            subs[m] = [_Sub("g", None, m, nm, np.eye(8))]
            continue
        light = x.rstrip("~") in LIGHT
        is_anti = x.endswith("~")
        if field[i].endswith("~"):           # column end: incoming quark u or outgoing antiquark v
            kind = "ext_v" if is_anti else "ext_u"
            nm = define(f"w{i}", [Op(kind, f"w{i}", [], {"leg": i, "light": light})])
            subs[m] = [_Sub("col", field[i][:-1], m, nm, np.eye(3), end=i)]
        else:                                # row end: outgoing quark ubar or incoming antiquark vbar
            kind = "ext_vbar" if is_anti else "ext_ubar"
            nm = define(f"w{i}", [Op(kind, f"w{i}", [], {"leg": i, "light": light})])
            subs[m] = [_Sub("row", field[i], m, nm, np.eye(3), end=i)]

    counter = itertools.count()
    root = 2
    full = ((1 << n) - 1) & ~(1 << root)

    def splits2(m):
        low = m & -m
        rest = m & ~low
        s = rest
        while True:                          # A = low | s' for every s' < rest
            a = low | (rest & ~s)
            b = m & ~a
            if b:
                yield a, b
            if s == 0:
                break
            s = (s - 1) & rest

    def splits3(m):
        for a, bc in splits2(m):
            for b, c in splits2(bc):
                yield a, b, c

    def build(m):
        if m in subs:
            return subs[m]
        out = []
        for a, b in splits2(m):
            for x, y in itertools.product(build(a), build(b)):
                lines = x.lines + y.lines
                extra = x.extra + y.extra
                for p, q in ((x, y), (y, x)):
                    if p.kind == "col" and q.kind == "g":
                        prog.dens[m] = fkind(p.flav, m)
                        nm = f"C{next(counter)}"
                        define(nm, [Op("ffv_fin", nm, [p.name, q.name],
                                       {"m": m, "light": p.flav in LIGHT})])
                        col = np.einsum(f"{axes(p.mask)}Y,{axes(q.mask)}A,AXY->{axes(m)}X", p.colour, q.colour, t)
                        out.append(_Sub("col", p.flav, m, nm, col, end=p.end, lines=lines, extra=extra))
                    if p.kind == "row" and q.kind == "g":
                        prog.dens[m] = fkind(p.flav, m)
                        nm = f"R{next(counter)}"
                        define(nm, [Op("ffv_fout", nm, [p.name, q.name],
                                       {"m": m, "light": p.flav in LIGHT})])
                        col = np.einsum(f"{axes(p.mask)}Y,{axes(q.mask)}A,AYX->{axes(m)}X", p.colour, q.colour, t)
                        out.append(_Sub("row", p.flav, m, nm, col, end=p.end, lines=lines, extra=extra))
                    if p.kind == "row" and q.kind == "col" and p.flav == q.flav:
                        prog.dens[m] = "gluon"
                        nm = f"J{next(counter)}"
                        define(nm, [Op("ffv_v0", nm, [p.name, q.name], {"m": m})])
                        col = np.einsum(f"{axes(p.mask)}Y,{axes(q.mask)}Z,XYZ->{axes(m)}X", p.colour, q.colour, t)
                        out.append(_Sub("g", None, m, nm, col, lines=lines + ((p.end, q.end),), extra=extra))
                if x.kind == "g" and y.kind == "g":
                    prog.dens[m] = "gluon"
                    nm = f"J{next(counter)}"
                    define(nm, [Op("vvv_v", nm, [x.name, y.name], {"mA": a, "mB": b, "m": m})])
                    col = np.einsum(f"{axes(a)}Y,{axes(b)}Z,XYZ->{axes(m)}X", x.colour, y.colour, f)
                    out.append(_Sub("g", None, m, nm, col, lines=lines, extra=extra))
        for a, b, c in splits3(m):
            for x, y, z in itertools.product(build(a), build(b), build(c)):
                if not (x.kind == y.kind == z.kind == "g"):
                    continue
                prog.dens[m] = "gluon"
                for piece, (p, q, r) in enumerate(((x, y, z), (y, x, z), (z, x, y))):
                    nm = f"J{next(counter)}"
                    define(nm, [Op("vvvv_v", nm, [p.name, q.name, r.name], {"m": m})])
                    col = np.einsum(f"{axes(p.mask)}Y,{axes(q.mask)}Z,{axes(r.mask)}W,XYE,EZW->{axes(m)}X",
                                    p.colour, q.colour, r.colour, f, f)
                    out.append(_Sub("g", None, m, nm, col, lines=x.lines + y.lines + z.lines,
                                    extra=x.extra + y.extra + z.extra + (piece > 0)))
        subs[m] = out
        return out

    # the diagrams: leg 2 (ubar of the top) closes a gluon and a top column current
    wt = subs[1 << root][0]
    diagrams = []
    for a, b in splits2(full):
        for x, y in itertools.product(build(a), build(b)):
            for g_, c_ in ((x, y), (y, x)):
                if g_.kind != "g" or c_.kind != "col" or c_.flav != "t":
                    continue
                col = np.einsum(f"{L[root]}Y,{axes(g_.mask)}A,{axes(c_.mask)}Z,AYZ->{L[root]}{axes(g_.mask)}"
                                f"{axes(c_.mask)}", wt.colour, g_.colour, c_.colour, t)
                cur = L[root] + axes(g_.mask) + axes(c_.mask)
                col = np.einsum(f"{cur}->{''.join(sorted(cur))}", col)
                lines = g_.lines + c_.lines + ((root, c_.end),)
                diagrams.append((g_, c_, col.reshape(-1) * _sign(lines), g_.extra + c_.extra))
    # Feynman diagrams: the three colour structures of a four-gluon vertex
    # are one diagram
    prog.n_diagrams = sum(1 for d in diagrams if d[3] == 0)

    # ------------------------------------------------------- colour basis
    rows = [i for i in range(n) if field[i] != "g" and not field[i].endswith("~")]
    cols = [i for i in range(n) if field[i].endswith("~")]
    gls = [i for i in range(n) if field[i] == "g"]

    cands = []
    for perm in itertools.permutations(cols):
        for assign in itertools.product(range(len(rows)), repeat=len(gls)):
            groups = [[g for g, a in zip(gls, assign) if a == k] for k in range(len(rows))]
            for orders in itertools.product(*[list(itertools.permutations(gr)) for gr in groups]):
                # tensor over all legs: product of strings (rows[k] -> perm[k])
                ops, names = [], []
                for k, seq in enumerate(orders):
                    st = np.eye(3, dtype=complex)
                    for _ in seq:      # (t^{a1} ... t^{aj})_{ik}: gluon axes in string order
                        st = np.einsum("...ij,Ajk->...Aik", st, t)
                    # axes: gluons of seq (in seq order), then row, column
                    ops.append(st)
                    names.append("".join(L[g] for g in seq) + L[rows[k]] + L[perm[k]])
                out = "".join(sorted("".join(names)))
                cands.append((np.einsum(",".join(names) + "->" + out, *ops).reshape(-1), (perm, orders)))
    D = np.stack([d[2] for d in diagrams])
    chosen, basis = [], []
    for vec, key in cands:
        trial = np.stack(basis + [vec])
        if np.linalg.matrix_rank(trial, tol=1e-9) == len(basis) + 1:
            basis.append(vec)
            chosen.append(key)
    B = np.stack(basis)
    # coordinates of every diagram in the basis (exactly representable)
    X, res, _, _ = np.linalg.lstsq(B.T, D.T, rcond=None)
    if np.abs(B.T @ X - D.T).max() > 1e-9:
        raise ValueError(f"{name}: the string basis does not span the diagrams")
    used = [k for k in range(B.shape[0]) if np.abs(X[k]).max() > 1e-9]
    B, X = B[used], X[used]
    X, _, _, _ = np.linalg.lstsq(B.T, D.T, rcond=None)
    coef = [[Fraction(v.real).limit_denominator(720) if abs(v.real) > 1e-9 else Fraction(0) for v in row] +
            [Fraction(v.imag).limit_denominator(720) if abs(v.imag) > 1e-9 else Fraction(0) for v in row]
            for row in X]
    scale = 1
    for row in coef:
        for q in row:
            scale = scale * q.denominator // gcd(scale, q.denominator)
    ncolor = B.shape[0]
    jams = []
    for d in range(len(diagrams)):
        jam = []
        for k in range(ncolor):
            re_, im_ = coef[k][d] * scale, coef[k][d + len(diagrams)] * scale
            if re_ != 0 and im_ != 0:
                raise ValueError(f"{name}: complex colour coefficient")
            if re_ != 0 or im_ != 0:
                jam.append((k, complex(int(re_), int(im_))))
        jams.append(jam)
    G = np.conj(B) @ B.T
    Gq = [[Fraction(v.real).limit_denominator(10 ** 6) for v in row] for row in G]
    if np.abs(np.array([[float(q) for q in r] for r in Gq]) - G.real).max() > 1e-9 or np.abs(G.imag).max() > 1e-9:
        raise ValueError(f"{name}: colour matrix is not rational")
    den = 1
    for r in Gq:
        for q in r:
            den = den * q.denominator // gcd(den, q.denominator)
    # jamps carry `scale` x the coordinates: |M|^2 = J^H (G / scale^2) J
    cden = den * scale * scale
    prog.ncolor = ncolor
    prog.colour_num = [[int(q * den) for q in r] for r in Gq]
    prog.colour_den = cden
    g = 0
    for r in prog.colour_num:
        for v in r:
            g = gcd(g, v)
    g = gcd(g, cden)
    if g > 1:
        prog.colour_num = [[v // g for v in r] for r in prog.colour_num]
        prog.colour_den = cden // g

    # ---------------------------------------------------- amplitude items
    for k, (g_, c_, _, _) in enumerate(diagrams):
        if not jams[k]:
            continue
        a = f"a{k}"
        ops = [add_kinematics(prog, Op("amp_ffv", a, [wt.name, g_.name, c_.name], {})),
               Op("jamp", None, [a], {"jam": jams[k]})]
        prog.items.append(ops)
    if share_half:
        share_half_contractions(prog, define)
    items = []
    for ops in prog.items:
        amps = {op.out for op in ops if op.kind.startswith("amp")}
        deps = []
        for op in ops:
            for v in op.ins:
                if v not in amps and v not in deps:
                    deps.append(v)
        items.append((ops, deps))
    prog.items = items
    return prog


# the two-jet channels of p p -> t tbar built by the general compiler
TWO_JET = {
    "uuttgg": "u u~ > t t~ g g",
    "uxuttgg": "u~ u > t t~ g g",
    "ugttug": "u g > t t~ u g",
    "guttug": "g u > t t~ u g",
    "uxgttuxg": "u~ g > t t~ u~ g",
    "guxttuxg": "g u~ > t t~ u~ g",
    "ggttuux": "g g > t t~ u u~",
    "uuttuux": "u u~ > t t~ u u~",
    "uuttddx": "u u~ > t t~ d d~",
    "uuttuu": "u u > t t~ u u",
    "udttud": "u d > t t~ u d",
    "uxuxttuxux": "u~ u~ > t t~ u~ u~",
}
