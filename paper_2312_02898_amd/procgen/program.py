"""Process compiler: straight-line helicity-amplitude programs (build time).

A program is the list of HELAS-style vertex calls that evaluates, for one
event and one helicity configuration, every Feynman diagram of a process and
accumulates the colour-flow amplitudes jamp_k (the matrix-element evaluation
that the paper offloads, Sec. 2 and Sec. 3).  Sub-diagrams are computed once
and shared between all diagrams that contain them.

Conventions
  * legs in the order of the process string; legs 0 and 1 incoming.  The
    momentum a leg carries INTO the diagram is k_i = +p_i (incoming) or -p_i
    (outgoing); an internal line fed by the legs in mask S carries
    K_S = sum_{i in S} k_i into the vertex it feeds.
  * helicity configuration h: leg i has helicity +1 iff bit i of h is set.
  * the top line runs from the outgoing top (row spinor ubar) to the outgoing
    antitop (column spinor v).  A diagram of t tbar + n gluons is an ordered
    sequence of gluon trees T1..Tk hanging off that line (top side first).
  * gluon trees are canonical binary trees (children ordered by smallest
    leaf).  The four-gluon vertex never needs a tree of its own: each of its
    three colour structures f^{xbe} f^{ecd} has the colour of the binary tree
    (b, (c, d)) and is added to that tree's current.
  * a propagator is "t-channel" when its mask holds exactly one incoming leg;
    the top width used there is a run-time parameter (zero in the paper's
    zero-width t-channel mode, Sec. 3).

The builder produces a DAG (values = wavefunctions, items = amplitudes with
their jamp updates).  ``schedule`` turns it into straight-line code for one
lane: amplitudes in a locality-friendly order, every wavefunction computed
just before it is needed and kept in a cache of at most ``budget``
wavefunctions; when the cache is full the value whose next use is furthest
away is dropped and recomputed later (Belady's rule).  That bounds the
registers a lane needs at the cost of some recomputation.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from functools import lru_cache

from . import colour

# Static flop counts of the device functions (add/mul = 1, FMA = 2, complex
# mul = 6, complex add = 2, real*complex = 2), used for the algorithmic flop
# count of a helicity.  sqrt and division are counted as 1 each.
FLOPS = {
    "ext_u": 40, "ext_v": 40, "ext_ubar": 40, "ext_vbar": 40, "ext_eps": 30,
    "ffv_fin": 154, "ffv_fout": 154, "ffv_v0": 144, "ffv_vm": 170,
    "vvv_v": 158, "vvvv_acc": 132, "vvvv_v": 124,
    "amp_ffv": 98, "amp_vvv": 168, "amp_vvvv_acc": 150,
    "ffv_half_row": 64, "ffv_half_col": 64, "amp_dot": 30,
    "ffv_v0_ew": 144, "ffv_vm_ew": 170, "amp_ffv_ew": 98, "amp_ffv_ew_acc": 100,
}
# momentum sum per extra leg, and the propagator factor per kind
DEN_FLOPS = {"top_t": 12, "top_s": 12, "gluon": 8, "z": 12, "photon": 8, "quark": 8}


def _zero_saving(op, eps) -> int:
    """Flops of a vertex call that the device functions skip because an
    external massless vector operand has a zero time component and a real z
    component, or because a fermion line is massless (same counting rules as
    FLOPS).  Per wavefunction-wavefunction product: 12 with one such vector,
    14 with two; per momentum-vector product: 6; per fermion-vector vertex
    with the vector external: 20; massless fermion propagator (zero mass,
    real 1/K^2): 32."""
    k = op.kind
    isv = [v.split("_r")[0] in eps for v in op.ins]

    def wdot(a, b):
        return 14 if a and b else (12 if a or b else 0)
    if k in ("ffv_fin", "ffv_fout", "ffv_half_row", "amp_ffv"):
        return 20 * isv[1] + (32 if k in ("ffv_fin", "ffv_fout") and op.prm.get("light") else 0)
    if k == "ffv_half_col":
        return 20 * isv[0]
    if k == "vvv_v":
        a, b = isv[0], isv[1]
        return 50 if a and b else (30 if a or b else 0)
    if k == "amp_vvv":
        x, a, b = isv[:3]
        return wdot(x, a) + wdot(a, b) + wdot(b, x) + 6 * (x + a + b)
    if k in ("vvvv_acc", "amp_vvvv_acc", "vvvv_v"):
        j = {"vvvv_acc": 1, "amp_vvvv_acc": 2, "vvvv_v": 0}[k]
        b, c, d = isv[j:j + 3]
        f = wdot(b, d) + wdot(b, c) + (22 if c and d else (12 if c or d else 0))
        if k == "amp_vvvv_acc":
            f += 12 * isv[1]
        return f
    return 0


@dataclass
class Op:
    kind: str
    out: str | None          # value written (None for jamp updates)
    ins: list                # value names read
    prm: dict = field(default_factory=dict)


@dataclass
class Program:
    name: str
    process: str
    npar: int
    leg_sign: list            # +1 incoming, -1 outgoing
    ncolor: int
    colour_num: list          # integer colour matrix
    colour_den: int
    iden: int
    n_diagrams: int
    values: dict = field(default_factory=dict)   # name -> list[Op] defining it
    deps: dict = field(default_factory=dict)     # name -> list of value names
    items: list = field(default_factory=list)    # (list[Op] amplitude ops + jamp op, deps)
    dens: dict = field(default_factory=dict)     # mask -> propagator kind
    ops: list = field(default_factory=list)      # scheduled straight-line code (last schedule)
    ops_f64: list = field(default_factory=list)  # schedule for the FP64 form
    ops_f32: list = field(default_factory=list)  # schedule for the FP32 form

    def value_masks(self, op: Op):
        return [v for k, v in op.prm.items() if k.startswith("m")]

    def flops_of(self, ops) -> int:
        f = 0
        for op in ops:
            if op.kind == "jamp":
                f += 2 * len(op.prm["jam"])
            elif op.kind in ("jadd", "jflush"):
                f += 2
            elif op.kind == "jset":
                pass
            elif op.kind == "kmom":
                f += 4 * (bin(op.prm["mk"]).count("1") - 1)
            elif op.kind == "den":
                f += 4 * (bin(op.prm["mk"]).count("1") - 1) + DEN_FLOPS[op.prm["kind"]]
            else:
                f += FLOPS.get(op.kind, 0)
        return f

    def flops_per_helicity(self) -> int:
        """Algorithmic flops of one helicity: every distinct vertex call,
        momentum sum and propagator factor once (no recomputation), jamp
        updates, colour quadratic form; the terms that the structurally zero
        components of external massless vectors and massless fermion masses
        remove are not counted."""
        eps = {v for v, ops in self.values.items() if ops and ops[0].kind == "ext_eps"}
        f = 0
        for ops in list(self.values.values()) + [ops for ops, _ in self.items]:
            f += self.flops_of(ops) - sum(_zero_saving(op, eps) for op in ops)
        n = self.ncolor
        f += 2 * n * (n + 1) + 4 * n
        return f

    def executed_flops_per_helicity(self) -> int:
        """Flops of the scheduled code including recomputation."""
        f = self.flops_of(self.ops)
        n = self.ncolor
        return f + 2 * n * (n + 1) + 4 * n

    def counts(self) -> dict:
        c = {}
        for op in self.ops:
            c[op.kind] = c.get(op.kind, 0) + 1
        return c


def _incoming_count(mask):
    return (mask & 1) + ((mask >> 1) & 1)


# register footprint of a value in FP64 dwords (the FP32 form needs about half)
def value_size(name: str) -> int:
    if name.startswith("K"):      # momentum sum (4 reals)
        return 8
    if name.startswith("D"):      # complex propagator factor
        return 4
    if name.startswith("I"):      # real propagator factor 1/K^2
        return 2
    if name.startswith("Q"):      # complex jamp accumulator (workspace-backed)
        return 4
    return 16                     # complex 4-component wavefunction


def add_kinematics(prog: "Program", op: "Op") -> "Op":
    """Make the momentum sums (K<mask>) and propagator factors (D<mask> for
    massive, I<mask> for massless lines) an op needs explicit inputs, so the
    scheduler bounds their live ranges like any other value."""
    extra = []
    for key in ("mA", "mB", "mX"):
        if key in op.prm:
            extra.append(kmom(prog, op.prm[key]))
    m = op.prm.get("m")
    if m is not None:
        kind = prog.dens[m]
        if op.kind in ("ffv_fin", "ffv_fout", "ffv_vm_ew"):
            extra.append(kmom(prog, m))
        if kind in ("top_t", "top_s", "quark"):
            extra.append(den(prog, m, "D"))
        elif kind == "z":
            extra.append(den(prog, m, "D"))
            extra.append(den(prog, m, "I"))
        else:
            extra.append(den(prog, m, "I"))
    for v in extra:
        if v not in op.ins:
            op.ins.append(v)
    return op


def kmom(prog, m):
    name = f"K{m}"
    if name not in prog.values:
        prog.values[name] = [Op("kmom", name, [], {"mk": m})]
        prog.deps[name] = []
    return name


def den(prog, m, tag):
    name = f"{tag}{m}"
    if name not in prog.values:
        prog.values[name] = [Op("den", name, [], {"mk": m, "kind": prog.dens[m], "tag": tag})]
        prog.deps[name] = []
    return name


# ------------------------------------------------------------------ QCD
def feynman_diagram_count(ng: int) -> int:
    """Tree diagrams of g g > t t~ + (ng-2) g with 3- and 4-gluon vertices:
    a top line carrying an ordered sequence of gluon subtrees."""
    from math import comb

    @lru_cache(maxsize=None)
    def D(k):   # sub-diagrams of a k-gluon subtree hanging off one line
        if k == 1:
            return 1
        tot = 0
        for a in range(1, k):                      # binary: A holds gluon 1
            tot += comb(k - 1, a - 1) * D(a) * D(k - a)
        for a in range(1, k - 1):                  # ternary: A holds gluon 1,
            for b in range(1, k - a):              # B the smallest of the rest
                c = k - a - b
                tot += comb(k - 1, a - 1) * comb(k - a - 1, b - 1) * D(a) * D(b) * D(c)
        return tot

    @lru_cache(maxsize=None)
    def L(k):   # ordered sequences of subtrees covering k labelled gluons
        if k == 0:
            return 1
        return sum(comb(k, a) * D(a) * L(k - a) for a in range(1, k + 1))
    return L(ng)


@lru_cache(maxsize=None)
def _trees(S):
    """Canonical binary trees over a sorted tuple of gluon labels."""
    if len(S) == 1:
        return (S[0],)
    first, rest = S[0], S[1:]
    out = []
    for r in range(len(rest)):
        for extra in itertools.combinations(rest, r):
            A = (first,) + extra
            B = tuple(x for x in rest if x not in extra)
            for ta in _trees(A):
                for tb in _trees(B):
                    out.append((ta, tb))
    return tuple(out)


def _ordered_partitions(S):
    if not S:
        yield ()
        return
    for r in range(1, len(S) + 1):
        for block in itertools.combinations(S, r):
            rest = tuple(x for x in S if x not in block)
            for tail in _ordered_partitions(rest):
                yield (block,) + tail


def qcd_program(ng: int, share_half: bool = True) -> Program:
    """g g > t t~ + (ng-2) g.  Gluon g sits on leg 0, 1, 4, 5, ... ."""
    gl = [0, 1] + [4 + i for i in range(ng - 2)]
    T, TB = 2, 3
    npar = ng + 2
    name = {2: "ggtt", 3: "ggttg", 4: "ggttgg", 5: "ggttggg"}[ng]
    order = colour.basis(ng)
    index = {s: i for i, s in enumerate(order)}
    cnum, cden = colour.colour_matrix(ng)
    iden = 256
    for k in range(2, ng - 2 + 1):
        iden *= k
    prog = Program(name=name, process="g g > t t~" + " g" * (ng - 2), npar=npar,
                   leg_sign=[1, 1] + [-1] * (npar - 2), ncolor=len(order), colour_num=cnum,
                   colour_den=cden, iden=iden, n_diagrams=feynman_diagram_count(ng))

    def define(name, ops):
        ops = [add_kinematics(prog, op) for op in ops]
        prog.values[name] = ops
        deps = []
        for op in ops:
            for v in op.ins:
                if v != name and v not in deps:
                    deps.append(v)
        prog.deps[name] = deps
        return name

    def gmask(tree):
        m = 0
        for g in colour.leaves(tree):
            m |= 1 << gl[g]
        return m

    ext = {}
    for g in range(ng):
        leg = gl[g]
        ext[g] = define(f"w{leg}", [Op("ext_eps", f"w{leg}", [], {"leg": leg, "conj": leg >= 2})])
    define("wT", [Op("ext_ubar", "wT", [], {"leg": T})])
    define("wTB", [Op("ext_v", "wTB", [], {"leg": TB})])

    tree_name = {}

    def tree(t):
        if isinstance(t, int):
            return ext[t]
        if t in tree_name:
            return tree_name[t]
        A, B = t
        na, nb = tree(A), tree(B)
        out = f"J{len(tree_name)}"
        tree_name[t] = out
        m = gmask(t)
        prog.dens[m] = "gluon"
        ops = [Op("vvv_v", out, [na, nb], {"mA": gmask(A), "mB": gmask(B), "m": m})]
        if not isinstance(B, int):      # f^{x A e} f^{e B0 B1}
            ops.append(Op("vvvv_acc", out, [out, tree(A), tree(B[0]), tree(B[1])], {"sgn": 1, "m": m}))
        if not isinstance(A, int):      # tree (A, B) = -(B, A): f^{x B e} f^{e A0 A1}
            ops.append(Op("vvvv_acc", out, [out, tree(B), tree(A[0]), tree(A[1])], {"sgn": -1, "m": m}))
        return define(out, ops)

    def top_mask(m):
        prog.dens[m] = "top_t" if _incoming_count(m) == 1 else "top_s"
        return m

    rows, cols = {(): "wT"}, {(): "wTB"}

    def row(prefix):
        if prefix in rows:
            return rows[prefix]
        r_in, J = row(prefix[:-1]), tree(prefix[-1])
        m = 1 << T
        for t in prefix:
            m |= gmask(t)
        out = f"R{len(rows)}"
        rows[prefix] = out
        return define(out, [Op("ffv_fout", out, [r_in, J], {"m": top_mask(m)})])

    def col(suffix):
        if suffix in cols:
            return cols[suffix]
        c_in, J = col(suffix[1:]), tree(suffix[0])
        m = 1 << TB
        for t in suffix:
            m |= gmask(t)
        out = f"C{len(cols)}"
        cols[suffix] = out
        return define(out, [Op("ffv_fin", out, [c_in, J], {"m": top_mask(m)})])

    sequences = []
    for part in _ordered_partitions(tuple(range(ng))):
        for trees in itertools.product(*[_trees(b) for b in part]):
            sequences.append(trees)

    def new_currents(seq, j):
        n = sum(1 for m in range(1, j) if seq[:m] not in rows)
        return n + sum(1 for m in range(j, len(seq)) if seq[m:] not in cols)

    mtt = (1 << T) | (1 << TB)
    namp = 0
    # longest sequences first: they fix the shared row/column currents
    for seq in sorted(sequences, key=lambda s: -len(s)):
        coeffs = colour.expand_line(seq)
        jam = [(index[s], c) for s, c in sorted(coeffs.items(), key=lambda kv: index[kv[0]])]
        a = f"a{namp}"
        namp += 1
        k = len(seq)
        if k == 1:
            A, B = seq[0]
            if "JTT" not in prog.values:
                prog.dens[mtt] = "gluon"
                define("JTT", [Op("ffv_v0", "JTT", ["wT", "wTB"], {"m": mtt})])
            ops = [Op("amp_vvv", a, ["JTT", tree(A), tree(B)], {"mX": mtt, "mA": gmask(A), "mB": gmask(B)})]
            if not isinstance(B, int):
                ops.append(Op("amp_vvvv_acc", a, [a, "JTT", tree(A), tree(B[0]), tree(B[1])], {"sgn": 1}))
            if not isinstance(A, int):
                ops.append(Op("amp_vvvv_acc", a, [a, "JTT", tree(B), tree(A[0]), tree(A[1])], {"sgn": -1}))
        else:
            j = min(range(1, k + 1), key=lambda jj: (new_currents(seq, jj), abs(2 * jj - (k + 1))))
            ops = [Op("amp_ffv", a, [row(seq[:j - 1]), tree(seq[j - 1]), col(seq[j:])], {})]
        ops = [add_kinematics(prog, op) for op in ops]
        ops.append(Op("jamp", None, [a], {"jam": jam}))
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


def share_half_contractions(prog, define):
    """Amplitudes rbar (gamma.J) psi that share (rbar, J) or (J, psi) compute
    the shared half contraction once (64 flop) and finish with a 4-component
    dot (30 flop) instead of a full vertex (98 flop) each."""
    amps = [ops[0] for ops in prog.items if ops[0].kind == "amp_ffv"]
    by_rj, by_jc = {}, {}
    for o in amps:
        by_rj[(o.ins[0], o.ins[1])] = by_rj.get((o.ins[0], o.ins[1]), 0) + 1
        by_jc[(o.ins[1], o.ins[2])] = by_jc.get((o.ins[1], o.ins[2]), 0) + 1
    names = {}
    groups = {}     # half contraction -> position of its merged item
    merged = []
    for ops in prog.items:
        o = ops[0]
        if o.kind != "amp_ffv":
            merged.append(ops)
            continue
        r, J, c = o.ins[:3]
        n_rj, n_jc = by_rj[(r, J)], by_jc[(J, c)]
        if max(n_rj, n_jc) < 2:
            merged.append(ops)
            continue
        if n_rj >= n_jc:
            key = ("row", r, J)
            if key not in names:
                names[key] = define(f"H{len(names)}", [Op("ffv_half_row", f"H{len(names)}", [r, J], {})])
            ops[0] = Op("amp_dot", o.out, [names[key], c], {})
        else:
            key = ("col", J, c)
            if key not in names:
                names[key] = define(f"H{len(names)}", [Op("ffv_half_col", f"H{len(names)}", [J, c], {})])
            ops[0] = Op("amp_dot", o.out, [r, names[key]], {})
        # amplitudes sharing a half contraction form one scheduling item
        if key in groups:
            merged[groups[key]] = merged[groups[key]] + ops
        else:
            groups[key] = len(merged)
            merged.append(ops)
    prog.items = merged


# --------------------------------------------------------------- ee -> mumu
def eemumu_program() -> Program:
    """e+ e- > mu+ mu- through s-channel photon and Z (2 diagrams)."""
    prog = Program(name="eemumu", process="e+ e- > mu+ mu-", npar=4, leg_sign=[1, 1, -1, -1],
                   ncolor=1, colour_num=[[1]], colour_den=1, iden=4, n_diagrams=2)
    m = 0b0011
    prog.dens[m] = "z"

    def define(name, ops):
        ops = [add_kinematics(prog, op) for op in ops]
        prog.values[name] = ops
        prog.deps[name] = [v for op in ops for v in op.ins if v != name]

    define("w0", [Op("ext_vbar", "w0", [], {"leg": 0})])    # incoming e+
    define("w1", [Op("ext_u", "w1", [], {"leg": 1})])       # incoming e-
    define("w2", [Op("ext_v", "w2", [], {"leg": 2})])       # outgoing mu+
    define("w3", [Op("ext_ubar", "w3", [], {"leg": 3})])    # outgoing mu-
    define("JA", [Op("ffv_v0_ew", "JA", ["w0", "w1"], {"m": m})])
    define("JZ", [Op("ffv_vm_ew", "JZ", ["w0", "w1"], {"m": m})])
    ops = [Op("amp_ffv_ew", "a0", ["w3", "JA", "w2"], {}),
           Op("amp_ffv_ew_acc", "a0", ["a0", "w3", "JZ", "w2"], {}),
           Op("jamp", None, ["a0"], {"jam": [(0, 1 + 0j)]})]
    prog.items.append((ops, ["w3", "JA", "w2", "JZ"]))
    return prog


# ------------------------------------------------------- q qbar -> t tbar
def qqtt_program(quark_first: bool = True) -> Program:
    """u u~ > t t~ (quark_first) or u~ u > t t~: the light-quark channels of
    p p > t t~.  One diagram, the s-channel gluon between the light line and
    the top line.  Its colour structure (t^a)_{c_qbar c_q} (t^a)_{c_t c_tbar}
    is the single colour flow; summed over colours it gives
    Tr(t^a t^b) Tr(t^a t^b) = 2, the 1x1 colour matrix."""
    name, proc = ("uutt", "u u~ > t t~") if quark_first else ("uxutt", "u~ u > t t~")
    q, qb = (0, 1) if quark_first else (1, 0)
    prog = Program(name=name, process=proc, npar=4, leg_sign=[1, 1, -1, -1],
                   ncolor=1, colour_num=[[2]], colour_den=1, iden=36, n_diagrams=1)
    m = 0b0011
    prog.dens[m] = "gluon"

    def define(nm, ops):
        ops = [add_kinematics(prog, op) for op in ops]
        prog.values[nm] = ops
        prog.deps[nm] = [v for op in ops for v in op.ins if v != nm]

    define(f"w{q}", [Op("ext_u", f"w{q}", [], {"leg": q})])          # incoming quark
    define(f"w{qb}", [Op("ext_vbar", f"w{qb}", [], {"leg": qb})])    # incoming antiquark
    define("wT", [Op("ext_ubar", "wT", [], {"leg": 2})])
    define("wTB", [Op("ext_v", "wTB", [], {"leg": 3})])
    define("JQ", [Op("ffv_v0", "JQ", [f"w{qb}", f"w{q}"], {"m": m})])
    ops = [Op("amp_ffv", "a0", ["wT", "JQ", "wTB"], {}),
           Op("jamp", None, ["a0"], {"jam": [(0, 1 + 0j)]})]
    prog.items.append((ops, ["wT", "JQ", "wTB"]))
    return prog


# ---------------------------------- light-quark line + t tbar + one gluon
QQG_CHANNELS = {
    # name: (process, column leg, row leg, gluon leg); legs 2, 3 are t, t~
    "uuttg": ("u u~ > t t~ g", 0, 1, 4),
    "uxuttg": ("u~ u > t t~ g", 1, 0, 4),
    "ugttu": ("u g > t t~ u", 0, 4, 1),
    "guttu": ("g u > t t~ u", 1, 4, 0),
    "uxgttux": ("u~ g > t t~ u~", 4, 0, 1),
    "guxttux": ("g u~ > t t~ u~", 4, 1, 0),
}


def qqg_program(name: str) -> Program:
    """One light-quark line, the top line and one gluon (the one-jet
    channels of p p > t t~ with a quark).  The light line runs along the
    fermion arrow from its column end (u of an incoming quark or v of an
    outgoing antiquark) to its row end (ubar of an outgoing quark or vbar of
    an incoming antiquark).  Five diagrams: the gluon on the light line at
    its column (D1) or row (D2) end, on the top line at the t (D3) or t~ (D4)
    end, or on the exchanged gluon (D5).

    Colour, in the flow basis F1 = (t^b)_{t c} d_{r tb}, F2 = (t^b)_{r tb} d_{t c},
    F3 = (t^b)_{t tb} d_{r c}, F4 = (t^b)_{r c} d_{t tb} (r, c: the light
    line's row and column colours; t, tb: the top line's; b: the gluon), by
    t^a_ij t^a_kl = (d_il d_kj - d_ij d_kl / 3) / 2 and f^{abx} t^x = -i[t^a, t^b]:
      D1 (t^a t^b)_rc (t^a)_ttb = F1/2 - F4/6,   D2 (t^b t^a)_rc (t^a)_ttb = F2/2 - F4/6,
      D3 (t^a)_rc (t^b t^a)_ttb = F1/2 - F3/6,   D4 (t^a)_rc (t^a t^b)_ttb = F2/2 - F3/6,
      D5 f^{x a b} (t^a)_rc (t^x)_ttb = i (F1 - F2)/2.
    The jamps carry 6 x these coefficients; sum_colours conj(F_k) F_l gives
    the matrix below, and the colour denominator is 36."""
    process, col, row, glu = QQG_CHANNELS[name]
    leg_sign = [1, 1, -1, -1, -1]
    iden = 36 if glu == 4 else 96
    C = [[12, 0, 4, 4], [0, 12, 4, 4], [4, 4, 12, 0], [4, 4, 0, 12]]
    prog = Program(name=name, process=process, npar=5, leg_sign=leg_sign, ncolor=4, colour_num=C,
                   colour_den=36, iden=iden, n_diagrams=5)
    col_in, row_in, glu_in = col < 2, row < 2, glu < 2

    def define(nm, ops):
        ops = [add_kinematics(prog, op) for op in ops]
        prog.values[nm] = ops
        prog.deps[nm] = [v for op in ops for v in op.ins if v != nm]
        return nm

    def top_kind(m):
        return "top_t" if _incoming_count(m) == 1 else "top_s"

    mc, mr, mg, mt, mtb = 1 << col, 1 << row, 1 << glu, 1 << 2, 1 << 3
    wc = define("wC", [Op("ext_u" if col_in else "ext_v", "wC", [], {"leg": col, "light": True})])
    wr = define("wR", [Op("ext_vbar" if row_in else "ext_ubar", "wR", [], {"leg": row, "light": True})])
    wg = define("wG", [Op("ext_eps", "wG", [], {"leg": glu, "conj": not glu_in})])
    wt = define("wT", [Op("ext_ubar", "wT", [], {"leg": 2})])
    wtb = define("wTB", [Op("ext_v", "wTB", [], {"leg": 3})])
    # gluon currents of the two lines and the three-gluon current
    prog.dens[mc | mr] = "gluon"
    prog.dens[mt | mtb] = "gluon"
    prog.dens[mc | mr | mg] = "gluon"
    jl = define("JL", [Op("ffv_v0", "JL", [wr, wc], {"m": mc | mr})])
    jtt = define("JTT", [Op("ffv_v0", "JTT", [wt, wtb], {"m": mt | mtb})])
    j5 = define("J5", [Op("vvv_v", "J5", [jl, wg], {"mA": mc | mr, "mB": mg, "m": mc | mr | mg})])
    # fermion currents with the gluon absorbed
    prog.dens[mc | mg] = "quark"
    prog.dens[mr | mg] = "quark"
    prog.dens[mt | mg] = top_kind(mt | mg)
    prog.dens[mtb | mg] = top_kind(mtb | mg)
    c1 = define("C1", [Op("ffv_fin", "C1", [wc, wg], {"m": mc | mg, "light": True})])
    r2 = define("R2", [Op("ffv_fout", "R2", [wr, wg], {"m": mr | mg, "light": True})])
    r3 = define("R3", [Op("ffv_fout", "R3", [wt, wg], {"m": mt | mg})])
    c4 = define("C4", [Op("ffv_fin", "C4", [wtb, wg], {"m": mtb | mg})])
    diagrams = [
        ([wr, jtt, c1], [(0, 3), (3, -1)]),    # D1
        ([r2, jtt, wc], [(1, 3), (3, -1)]),    # D2
        ([r3, jl, wtb], [(0, 3), (2, -1)]),    # D3
        ([wt, jl, c4], [(1, 3), (2, -1)]),     # D4
        ([wt, j5, wtb], [(0, 3j), (1, -3j)]),  # D5
    ]
    for k, (ins, jam) in enumerate(diagrams):
        a = f"a{k}"
        ops = [Op("amp_ffv", a, list(ins), {}), Op("jamp", None, [a], {"jam": [(i, complex(c)) for i, c in jam]})]
        prog.items.append((ops, list(ins)))
    return prog


# --------------------------------------------------------------- scheduling
def _closure(prog, names):
    seen = []
    stack = list(names)
    while stack:
        v = stack.pop()
        if v in seen:
            continue
        seen.append(v)
        stack.extend(prog.deps.get(v, []))
    return seen


def schedule(prog: Program, budget: int, iters: int = 4) -> Program:
    """Best of ``iters`` greedy passes, each starting from the amplitude
    order the previous pass chose (fewest executed flops wins)."""
    items = prog.items
    best = None
    start = list(range(len(items)))
    for _ in range(max(1, iters)):
        prog.items = [items[i] for i in start]
        _schedule_once(prog, budget)
        order = [start[i] for i in prog.order]
        f = prog.executed_flops_per_helicity()
        if best is None or f < best[0]:
            best = (f, prog.ops, order)
        start = order
    prog.items = items
    prog.ops, prog.order = best[1], best[2]
    return prog


def _schedule_once(prog: Program, budget: int) -> Program:
    """Linearise the DAG for one lane with at most ``budget`` live register
    dwords of cached values (FP64 sizes; recomputing evicted ones).
    Amplitudes are taken greedily:
    next is the one whose missing wavefunctions are cheapest to compute given
    the current cache.  Recomputed copies get a new name '<v>_r<k>' and are
    marked so the code generator can keep the compiler from merging them
    with the first copy."""
    items = list(prog.items)
    closures = [set(_closure(prog, deps)) for _, deps in items]
    vcost = {v: max(1, prog.flops_of(ops)) for v, ops in prog.values.items()}
    remaining = set(range(len(items)))
    # next-use is evaluated against the items still to come, in their
    # original order, as a proxy for the greedy order chosen on the fly
    uses = {}
    for i in range(len(items)):
        for v in closures[i]:
            uses.setdefault(v, []).append(i)
    # workspace-backed jamps: accumulator Q<k> is a cached value whose
    # eviction writes it back to memory (store or read-add-store)
    jmem = getattr(prog, "jamps_in_memory", False)
    item_jamps = [set() for _ in items]
    if jmem:
        for i, (ops, _) in enumerate(items):
            for op in ops:
                if op.kind == "jamp":
                    item_jamps[i] |= {f"Q{k}" for k, _ in op.prm["jam"]}
            for q in sorted(item_jamps[i]):
                uses.setdefault(q, []).append(i)
                vcost[q] = JFLUSH_COST

    def next_use(v):
        best = len(items) + 1
        for i in uses.get(v, []):
            if i in remaining:
                # distance in "remaining" order: the number of remaining items before it
                best = i
                break
        return best

    cache = {}          # value -> current emitted name
    version = {}
    out = []

    def rename(op, names):
        ins = [names.get(v, cache.get(v, v)) for v in op.ins]
        return Op(op.kind, names.get(op.out, op.out) if op.out else None, ins, dict(op.prm))

    jcap = getattr(prog, "jamp_capacity", None)

    def evict(pinned):
        # jamp accumulators: their own capacity when one is set, else they
        # share the register budget with the wavefunctions
        while jcap is not None and sum(1 for v in cache if v.startswith("Q")) > jcap:
            cands = [v for v in cache if v.startswith("Q") and v not in pinned]
            if not cands:
                break
            victim = max(cands, key=next_use)
            out.append(Op("jflush", None, [cache[victim]], {"k": int(victim[1:])}))
            del cache[victim]

        def held(v):
            return jcap is None or not v.startswith("Q")
        while sum(value_size(v) for v in cache if held(v)) > budget:
            cands = [v for v in cache if v not in pinned and held(v)]
            if not cands:
                return
            # furthest next use, weighted by footprint over recompute cost
            victim = max(cands, key=lambda v: (next_use(v) - cur[0] + 1) * value_size(v) / vcost[v])
            if victim.startswith("Q"):
                out.append(Op("jflush", None, [cache[victim]], {"k": int(victim[1:])}))
            del cache[victim]

    def ensure(v, pinned):
        if v in cache:
            return cache[v]
        pinned = pinned | {v}
        for d in prog.deps.get(v, []):
            ensure(d, pinned)
            pinned = pinned | {d}
        k = version.get(v, 0)
        version[v] = k + 1
        nm = v if k == 0 else f"{v}_r{k}"
        names = {v: nm}
        for op in prog.values[v]:
            o = rename(op, names)
            if k > 0:
                o.prm["recompute"] = True
            out.append(o)
        cache[v] = nm
        evict(pinned | set(prog.deps.get(v, [])))
        return nm

    def missing_cost(i):
        c = sum(vcost[v] for v in closures[i] if v not in cache)
        if jcap is not None and len([v for v in cache if v.startswith("Q")]) < jcap:
            return c
        return c + sum(JFLUSH_COST for q in item_jamps[i] if q not in cache)

    order = []
    item_end = []
    cur = [0]
    while remaining:
        i = _pick[0](remaining, lambda j: (missing_cost(j), j))
        cur[0] = i
        remaining.discard(i)
        order.append(i)
        ops, deps = items[i]
        pinned = set()
        for d in deps:
            ensure(d, pinned)
            pinned.add(d)
        for op in ops:
            if op.kind == "jamp" and jmem:
                held = set()
                for k, c in op.prm["jam"]:
                    q = f"Q{k}"
                    if q in cache:
                        out.append(Op("jadd", None, [cache[q], op.ins[0]], {"k": k, "c": c}))
                    else:
                        nm = f"Q{k}_{version.get(q, 0)}"
                        version[q] = version.get(q, 0) + 1
                        out.append(Op("jset", nm, [op.ins[0]], {"k": k, "c": c}))
                        cache[q] = nm
                    held.add(q)
                    evict(held)
                out.append(Op("jsync", None, [], {}))
            else:
                out.append(rename(op, {}))
        evict(set())
        item_end.append(len(out))
    if jmem:
        for q in sorted((v for v in cache if v.startswith("Q")), key=lambda v: int(v[1:])):
            out.append(Op("jflush", None, [cache[q]], {"k": int(q[1:])}))
    # prog.items keeps the builder's order so that every schedule starts from
    # the same point; the chosen order is kept separately
    prog.order = order
    prog.item_end = item_end
    prog.ops = out
    return prog


def schedule_parts(prog: Program, budget: int, nparts: int, iters: int = 4) -> list:
    """Kernel splitting for workspace-backed jamps: schedule the whole
    program, cut the chosen amplitude order into ``nparts`` contiguous runs
    of about equal executed cost, and schedule each run on its own (fresh
    register cache; every part writes its jamp contributions back).  Returns
    one op list per part and leaves their concatenation in prog.ops."""
    assert getattr(prog, "jamps_in_memory", False)
    schedule(prog, budget, iters)
    if nparts <= 1:
        prog.parts = [prog.ops]
        return prog.parts
    order = list(prog.order)
    _schedule_once_in_order(prog, budget, order)
    prog.order = order
    cost, prev = [], 0
    for end in prog.item_end:
        cost.append(prog.flops_of(prog.ops[prev:end]))
        prev = end
    total = sum(cost)
    cuts, acc, j = [], 0, 1
    for i, c in enumerate(cost):
        acc += c
        if j < nparts and acc >= total * j / nparts:
            cuts.append(i + 1)
            j += 1
    bounds = [0] + cuts + [len(prog.order)]
    items = prog.items
    parts = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        sub = [items[i] for i in order[a:b]]
        prog.items = sub
        schedule(prog, budget, iters)
        parts.append(prog.ops)
        prog.items = items
    prog.parts = parts
    prog.order = order
    prog.ops = [op for part in parts for op in part]
    return parts


def _schedule_once_in_order(prog: Program, budget: int, order) -> None:
    """_schedule_once with the amplitude order fixed (used to measure the
    cost of each amplitude in a given order)."""
    items = prog.items
    prog.items = [items[i] for i in order]
    saved = _pick[0]
    _pick[0] = lambda remaining, key: min(remaining)
    try:
        _schedule_once(prog, budget)
    finally:
        _pick[0] = saved
        prog.items = items


# item selection rule of _schedule_once (replaceable to fix the order)
_pick = [lambda remaining, key: min(remaining, key=key)]
# write-back cost of a jamp accumulator in flop equivalents (memory round trip)
JFLUSH_COST = 48


def peak_live(prog: Program) -> int:
    """Peak FP64 dwords of simultaneously live cached values in prog.ops."""
    last = {}
    for i, op in enumerate(prog.ops):
        for v in op.ins:
            last[v] = i
    live, peak = set(), 0
    for i, op in enumerate(prog.ops):
        if op.out and not op.out.startswith("a"):
            live.add(op.out)
        peak = max(peak, sum(value_size(v.split("_r")[0]) for v in live))
        for v in op.ins:
            if last.get(v) == i:
                live.discard(v)
    return peak


def all_programs(budget=None):
    """Programs with one register schedule per arithmetic type.  Budgets are
    in FP64 dwords; an FP32 value takes half the registers, so the FP32
    schedule gets the same register count as twice the FP64 budget."""
    progs = [eemumu_program()] + [qcd_program(ng, share_half=SHARE_HALF.get(n, True))
                                  for ng, n in ((2, "ggtt"), (3, "ggttg"), (4, "ggttgg"), (5, "ggttggg"))]
    progs += [qqtt_program(True), qqtt_program(False)]
    progs += [qqg_program(n) for n in QQG_CHANNELS]
    from .general import TWO_JET, general_program
    progs += [general_program(n, proc) for n, proc in TWO_JET.items()]
    for p in progs:
        if p.name in SPLIT:
            split_program(p, SPLIT[p.name], budget)
            continue
        p.fp64_lds_jamps = p.name in FP64_LDS_JAMPS
        p.f32_lds_jamps = p.name in F32_LDS_JAMPS
        p.mixed_mfma = p.name in MIXED_MFMA
        p.den_cache_f32 = p.name in DEN_CACHE_F32
        p.den_cache_f64 = p.name in DEN_CACHE_F64 and not p.fp64_lds_jamps
        p.mom_cache_f32 = p.name in MOM_CACHE_F32 and p.den_cache_f32
        p.f32_kc_waves = F32_KC_WAVES if p.mom_cache_f32 else 1
        p.mom_cache_f64 = p.name in MOM_CACHE_F64 and p.den_cache_f64 and not p.fp64_lds_jamps
        p.f64_kcw_waves = F64_KCW_WAVES if p.mom_cache_f64 else 1
        b64, i64 = DEFAULT_SCHEDULE_F64.get(p.name, SCHEDULE_F64_OTHERS)
        b32, i32 = DEFAULT_SCHEDULE_F32.get(p.name, SCHEDULE_F32_OTHERS)
        schedule(p, budget if budget is not None else b32, i32)
        p.ops_f32 = p.ops
        schedule(p, budget if budget is not None else b64, i64)
        p.ops_f64 = p.ops
    return progs


# (budget in FP64 dwords, greedy passes) per process and arithmetic type,
# and whether amplitudes share half contractions; chosen by measurement on
# gfx950 (2^20 gg -> t tbar gg events)
# (with the momentum sums and spinors in the per-event cache, registers that
# the schedule can use grew: budgets of 1024 (no eviction) for the FP32 forms
# and 512 for the FP64 ones measured fastest, except where noted)
DEFAULT_SCHEDULE_F64 = {"eemumu": (512, 4), "ggtt": (512, 4), "ggttg": (512, 4), "ggttgg": (250, 4)}
DEFAULT_SCHEDULE_F32 = {"eemumu": (1024, 4), "ggtt": (1024, 4), "ggttg": (1024, 1), "ggttgg": (1024, 2),
                        # the q g > t t~ q g channels ran 40 % slower at 1024
                        "ugttug": (512, 4), "guttug": (512, 4), "uxgttuxg": (512, 4), "guxttuxg": (512, 4)}
SCHEDULE_F64_OTHERS = (512, 4)
SCHEDULE_F32_OTHERS = (1024, 4)
SHARE_HALF = {"ggttg": False, "ggttgg": True, "ggttggg": True}
# FP64 forms that keep their jamps in LDS (frees 4 registers per colour flow
# for the wavefunction schedule; none since the momentum sums and spinors
# left the registers for the per-event cache)
FP64_LDS_JAMPS = set()
# the same for the mixed form's vector-ALU kernel
F32_LDS_JAMPS = set()
# mixed forms whose vector-ALU kernel forms the propagator factors once per
# event into LDS instead of once per helicity
DEN_CACHE_F32 = {"eemumu", "ggtt", "ggttg", "ggttgg", "uutt", "uxutt", "uuttg", "uxuttg", "ugttu", "guttu",
                 "uxgttux", "guxttux", "uuttgg", "uxuttgg", "ugttug", "guttug", "uxgttuxg", "guxttuxg", "ggttuux",
                 "uuttuux", "uuttddx", "uuttuu", "udttud", "uxuxttuxux"}
# the same for the FP64 forms whose jamps stay in registers
DEN_CACHE_F64 = {"ggttgg", "eemumu", "ggtt", "ggttg", "uutt", "uxutt", "uuttg", "uxuttg", "ugttu", "guttu", "uxgttux",
                 "guxttux", "uuttgg", "uxuttgg", "ugttug", "guttug", "uxgttuxg", "guxttuxg", "ggttuux",
                 "uuttuux", "uuttddx", "uuttuu", "udttud", "uxuxttuxux"}
# mixed forms whose vector-ALU kernel also caches the momentum sums and both
# helicity states of the external spinors per event (their helicities spread
# over F32_KC_WAVES waves that share the cache); measured faster for all but
# the q g > t t~ q g channels and g g > t t~ u u~, where it made no gain
MOM_CACHE_F32 = DEN_CACHE_F32 - {"ugttug", "guttug", "uxgttuxg", "guxttuxg", "ggttuux"}
F32_KC_WAVES = 2
# the same for the FP64 forms whose jamps stay in registers (FP64 entries
# take twice the LDS: F64_KCW_WAVES waves share one cache; gg -> t tbar gg
# FP64 54.2 -> 41.3 ms per 2^20 events against jamps in LDS)
MOM_CACHE_F64 = set(DEN_CACHE_F64)
F64_KCW_WAVES = 4
# processes whose default mixed form (ME_MIXED) sums colours on FP16 hi+lo
# MFMA; the others use the vector ALU (chosen by measurement on 2^20 events
# of each process's configuration)
MIXED_MFMA = {"uuttgg", "uxuttgg", "uuttuu", "uuttuux", "uxuxttuxux"}

# Split form (jamps in a workspace, amplitudes in several kernels) for the
# processes whose colour flows do not fit in registers: per arithmetic type
# the wavefunction budget (FP64 dwords), the number of jamp accumulators a
# lane holds at once, the number of parts and (optional) whether the
# accumulators live in LDS instead of registers.
SPLIT = {"ggttggg": {"f64": (288, 36, 12, True), "f32": (384, 56, 8)}}


def split_program(p: Program, cfg: dict, budget=None) -> Program:
    p.split = True
    p.jamps_in_memory = True
    for tag in ("f32", "f64"):
        b, jcap, nparts = cfg[tag][:3]
        # optional fourth entry: the jamp accumulators live in LDS (jcap
        # slots per lane) instead of registers
        setattr(p, f"qlds_{tag}", jcap if len(cfg[tag]) > 3 and cfg[tag][3] else 0)
        p.jamp_capacity = jcap
        parts = schedule_parts(p, budget if budget is not None else b, nparts, iters=2)
        setattr(p, f"parts_{tag}", parts)
    p.ops_f64 = [op for part in p.parts_f64 for op in part]
    p.ops_f32 = [op for part in p.parts_f32 for op in part]
    return p
