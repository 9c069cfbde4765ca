"""Colour algebra for one quark line with n gluons (build time).

Basis (colour-flow / trace basis along the top line):
    c_sigma = (t^{a_sigma1} ... t^{a_sigman})_{i_t j_tbar},  sigma in S_n,
enumerated in lexicographic order of sigma.

Gluon subtrees.  A tree node (L, R) stands for the colour tensor f^{x L R}
(x the index towards the quark line); attaching it to the quark line with
t^x and using  t^x f^{x b c} = -i [t^b, t^c]  expands every tree into a sum
of ordered strings of its leaves with coefficients in {+-1, +-i}:
    E(leaf a)  = t^a
    E((L, R))  = -i (E(L) E(R) - E(R) E(L)).
A quark line carrying trees T1..Tk (from the top end to the antitop end) has
colour E(T1) E(T2) ... E(Tk): its coordinates in the basis above are the
coefficients of each full-length string.

Colour matrix C[sigma][tau] = sum_colours conj(c_sigma) c_tau
    = sum_a Tr(t^{a_sn}...t^{a_s1} t^{a_t1}...t^{a_tn}),
evaluated exactly with the Fierz identity
    sum_a (t^a)_{ij} (t^a)_{kl} = 1/2 [d_il d_kj - d_ij d_kl / N],  Tr(1) = N,
applied to one label at a time (within one trace or joining two traces), in
rational arithmetic.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from functools import lru_cache

N_C = 3


def leaves(tree):
    if isinstance(tree, int):
        return (tree,)
    return leaves(tree[0]) + leaves(tree[1])


def expand(tree):
    """dict: tuple of gluon labels -> complex coefficient (Gaussian integer)."""
    if isinstance(tree, int):
        return {(tree,): 1 + 0j}
    el, er = expand(tree[0]), expand(tree[1])
    out = {}
    for sl, cl in el.items():
        for sr, cr in er.items():
            out[sl + sr] = out.get(sl + sr, 0) + (-1j) * cl * cr
            out[sr + sl] = out.get(sr + sl, 0) - (-1j) * cl * cr
    return {k: v for k, v in out.items() if v != 0}


def expand_line(trees):
    res = {(): 1 + 0j}
    for t in trees:
        et = expand(t)
        nxt = {}
        for s0, c0 in res.items():
            for s1, c1 in et.items():
                nxt[s0 + s1] = nxt.get(s0 + s1, 0) + c0 * c1
        res = {k: v for k, v in nxt.items() if v != 0}
    return res


def basis(n):
    """Orderings sigma of gluons 0..n-1 in lexicographic order."""
    return list(itertools.permutations(range(n)))


@lru_cache(maxsize=None)
def _traces(words):
    """sum over repeated adjoint labels of prod_w Tr(t^{w_1} ... t^{w_k}).
    Every label occurs exactly twice in total.  Returns a Fraction."""
    for wi, w in enumerate(words):
        if w:
            a = w[0]
            break
    else:
        return Fraction(N_C) ** len(words)
    rest = words[:wi] + words[wi + 1:]
    w = words[wi]
    if a in w[1:]:
        # Tr(t^a Y t^a Z) = 1/2 [Tr(Y) Tr(Z) - Tr(Y Z)/N]
        j = w.index(a, 1)
        y, z = w[1:j], w[j + 1:]
        return Fraction(1, 2) * (_traces(_canon(rest + (y, z))) - _traces(_canon(rest + (y + z,))) / N_C)
    # a appears in another trace: Tr(t^a X) Tr(t^a Y) = 1/2 [Tr(X Y) - Tr(X) Tr(Y)/N]
    for vi, v in enumerate(rest):
        if a in v:
            break
    k = v.index(a)
    x = w[1:]
    y = v[k + 1:] + v[:k]
    rest2 = rest[:vi] + rest[vi + 1:]
    return Fraction(1, 2) * (_traces(_canon(rest2 + (x + y,))) - _traces(_canon(rest2 + (x, y))) / N_C)


def _canon(words):
    """Rename labels by first appearance (keeps the cache small); empty
    traces stay and contribute a factor N each."""
    m = {}
    out = []
    for w in words:
        ow = []
        for a in w:
            if a not in m:
                m[a] = len(m)
            ow.append(m[a])
        out.append(tuple(ow))
    return tuple(out)


def colour_matrix(n):
    """Return (integer matrix as list of lists, common denominator)."""
    orders = basis(n)
    entries = []
    for s in orders:
        row = []
        for t in orders:
            word = tuple(reversed(s)) + tuple(t)
            row.append(_traces(_canon((word,))))
        entries.append(row)
    den = 1
    for row in entries:
        for v in row:
            den = den * v.denominator // _gcd(den, v.denominator)
    mat = [[int(v * den) for v in row] for row in entries]
    return mat, den


def _gcd(a, b):
    while b:
        a, b = b, a % b
    return a
