"""Pins of the CPU oracle against results that do not come from the oracle.

Each test checks the oracle against something the mathematics fixes: closed
forms, trace-technique spin sums with explicit gamma matrices, gauge and
Lorentz invariance, Bose symmetry, helicity-selection rules, the literal
colour-dressed Feynman rules, colour identities and a total cross section.
A plausible mistake anywhere in the oracle (a dropped diagram, a wrong
sign, index or coupling, a transposed operand, a missing symmetry factor)
fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest

from paper_2312_02898_amd.inputs import config_events, rambo

G = np.diag([1.0, -1.0, -1.0, -1.0])
ALPHA = 1.0 / 132.507
ALPHA_S = 0.118
MT = 173.0
MZ, WZ = 91.188, 2.441
SW2 = 0.2222


def mdot(a, b):
    return a[..., 0] * b[..., 0] - (a[..., 1:] * b[..., 1:]).sum(-1)


# ----------------------------------------------------------- closed forms
def ee_closed_form(p):
    """e+(p1) e-(p2) -> mu+(p3) mu-(p4) via photon and Z, massless leptons:
    (e^4/4)[(|A_LL|^2+|A_RR|^2)(1+cos)^2 + (|A_LR|^2+|A_RL|^2)(1-cos)^2],
    A_ij = Q_e Q_mu + c_i c_j s/(s - MZ^2 + i MZ GZ)."""
    s = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1])
    e2 = 4 * np.pi * ALPHA
    sw, cw = np.sqrt(SW2), np.sqrt(1 - SW2)
    cl, cr = (-0.5 + SW2) / (sw * cw), SW2 / (sw * cw)
    chi = s / (s - MZ ** 2 + 1j * MZ * WZ)
    onepc = -2 * mdot(p[:, 1] - p[:, 2], p[:, 1] - p[:, 2]) / s
    onemc = -2 * mdot(p[:, 1] - p[:, 3], p[:, 1] - p[:, 3]) / s

    def A(ci, cj):
        return 1 + ci * cj * chi
    return e2 ** 2 / 4 * ((abs(A(cl, cl)) ** 2 + abs(A(cr, cr)) ** 2) * onepc ** 2
                          + (abs(A(cl, cr)) ** 2 + abs(A(cr, cl)) ** 2) * onemc ** 2)


def ggtt_closed_form(p, m=MT):
    """Combridge / Glueck-Owens-Reya: g^4 (1/(6 t1 t2) - 3/8)(t1^2 + t2^2 + rho
    - rho^2/(4 t1 t2)), t1 = 2 p1.p3/s, t2 = 2 p2.p3/s, rho = 4 m^2/s."""
    s = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1])
    g2 = 4 * np.pi * ALPHA_S
    t1 = 2 * mdot(p[:, 0], p[:, 2]) / s
    t2 = 2 * mdot(p[:, 1], p[:, 2]) / s
    rho = 4 * m * m / s
    return g2 ** 2 * (1 / (6 * t1 * t2) - 3 / 8) * (t1 ** 2 + t2 ** 2 + rho - rho ** 2 / (4 * t1 * t2))


def test_eemumu_closed_form(oracle_lib):
    p = config_events("eemumu", 4096)
    o = oracle_lib.me("e+ e- > mu+ mu-", p)
    rel = np.abs(o / ee_closed_form(p) - 1)
    # the closed form's (p2-p3)^2 loses digits at near-collinear points
    assert np.median(rel) < 1e-15 and rel.max() < 1e-11, rel.max()


def test_ggtt_closed_form(oracle_lib):
    p = config_events("ggtt", 4096)
    o = oracle_lib.me("g g > t t~", p)
    rel = np.abs(o / ggtt_closed_form(p) - 1)
    assert np.median(rel) < 1e-14 and rel.max() < 1e-11, rel.max()


def test_ggtt_massless_limit(oracle_lib):
    """m -> 0: g^4 [(t^2+u^2)/(6tu) - 3(t^2+u^2)/(8 s^2)]."""
    p = rambo(512, 1500.0, [0.0, 0.0], seed=11)
    o = oracle_lib.me("g g > t t~", p, oracle_lib.default_params(mt=0.0, wt=0.0))
    s = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1])
    t = mdot(p[:, 0] - p[:, 2], p[:, 0] - p[:, 2])
    u = mdot(p[:, 0] - p[:, 3], p[:, 0] - p[:, 3])
    g4 = (4 * np.pi * ALPHA_S) ** 2
    ref = g4 * ((t * t + u * u) / (6 * t * u) - 3 * (t * t + u * u) / (8 * s * s))
    assert np.abs(o / ref - 1).max() < 1e-11


def test_ggtt_threshold(oracle_lib):
    """At threshold every angle gives 7 g^4 / 48."""
    p = rambo(64, 2 * MT * (1 + 1e-9), [MT, MT], seed=12)
    o = oracle_lib.me("g g > t t~", p)
    ref = 7 * (4 * np.pi * ALPHA_S) ** 2 / 48
    assert np.abs(o / ref - 1).max() < 1e-6


# --------------------------------------------------------- trace technique
def _gammas():
    """Chiral representation (the oracle itself uses the Dirac one)."""
    s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]),
         np.array([[1, 0], [0, -1]], complex)]
    z, one = np.zeros((2, 2), complex), np.eye(2, dtype=complex)
    g = [np.block([[z, one], [one, z]])] + [np.block([[z, si], [-si, z]]) for si in s]
    g5 = np.block([[-one, z], [z, one]])
    return np.array(g), g5


GAM, G5 = _gammas()


def slash(p):
    return np.einsum("m,mij->ij", G @ p, GAM)


def gbar(M):
    return GAM[0] @ M.conj().T @ GAM[0]


def ggtt_trace(p1, p2, p3, p4, m=MT, width=0.0):
    """sum over spins, physical gluon polarisations and colours of |M|^2 / 256,
    from Tr[(p3/+m) Gamma (p4/-m) Gamma-bar] with the three diagrams written
    as 4x4 matrices and the two colour structures t^a t^b, t^b t^a."""
    g2 = 4 * np.pi * ALPHA_S
    I4 = np.eye(4)
    t = mdot(p3 - p1, p3 - p1)
    u = mdot(p3 - p2, p3 - p2)
    s = mdot(p1 + p2, p1 + p2)
    Tm = np.zeros((4, 4, 4, 4), complex)
    Um = np.zeros_like(Tm)
    Sm = np.zeros_like(Tm)
    prop_t = slash(p3 - p1) + m * I4
    prop_u = slash(p3 - p2) + m * I4
    k, pp, q = p1, p2, -p1 - p2
    for mu in range(4):
        for nu in range(4):
            Tm[mu, nu] = -1j * g2 * GAM[mu] @ prop_t @ GAM[nu] / (t - m * m + 1j * m * width)
            Um[mu, nu] = -1j * g2 * GAM[nu] @ prop_u @ GAM[mu] / (u - m * m + 1j * m * width)
            # V^{mu nu rho} = g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu
            Vr = np.array([G[mu, nu] * (k - pp)[r] + G[nu, r] * (pp - q)[mu] + G[r, mu] * (q - k)[nu]
                           for r in range(4)])
            Sm[mu, nu] = g2 / s * np.einsum("r,rij->ij", G @ Vr, GAM)
    Gam = [Tm - 1j * Sm, Um + 1j * Sm]
    CF, N = 4.0 / 3.0, 3.0
    Cmat = np.array([[N * CF * CF, -CF / 2], [-CF / 2, N * CF * CF]])

    def polsum(kk, n):
        kl, nl = G @ kk, G @ n
        return -G + (np.outer(kl, nl) + np.outer(nl, kl)) / mdot(kk, n)
    P1, P2 = polsum(p1, p2), polsum(p2, p1)
    A = slash(p3) + m * I4
    B = slash(p4) - m * I4
    tot = 0.0
    for a in range(2):
        for b in range(2):
            Gb = np.array([[gbar(Gam[b][m1, n1]) for n1 in range(4)] for m1 in range(4)])
            tr = np.einsum("ij,mnjk,kl,MNli->mnMN", A, Gam[a], B, Gb)
            tot += Cmat[a, b] * np.einsum("mM,nN,mnMN->", P1, P2, tr)
    return tot.real / 256.0


def eemumu_trace(p1, p2, p3, p4):
    e = math.sqrt(4 * math.pi * ALPHA)
    sw, cw = math.sqrt(SW2), math.sqrt(1 - SW2)
    cl, cr = (-0.5 + SW2) / (sw * cw), SW2 / (sw * cw)
    PL, PR = (np.eye(4) - G5) / 2, (np.eye(4) + G5) / 2
    q = p1 + p2
    s = mdot(q, q)
    verts = {
        "a": [-1j * e * (-1) * GAM[mu] for mu in range(4)],
        "z": [-1j * e * GAM[mu] @ (cl * PL + cr * PR) for mu in range(4)],
    }
    ql = G @ q
    props = {"a": -1j * G / s,
             "z": -1j * (G - np.outer(ql, ql) / MZ ** 2) / (s - MZ ** 2 + 1j * MZ * WZ)}
    tot = 0.0
    for V in "az":
        for W in "az":
            L1 = np.array([[np.trace(verts[V][mu] @ slash(p2) @ gbar(verts[W][nu]) @ slash(p1))
                            for nu in range(4)] for mu in range(4)])
            L2 = np.array([[np.trace(verts[V][mu] @ slash(p3) @ gbar(verts[W][nu]) @ slash(p4))
                            for nu in range(4)] for mu in range(4)])
            tot += np.einsum("mn,MN,mM,nN->", props[V], props[W].conj(), L1, L2)
    return tot.real / 4.0


def test_ggtt_trace_bruteforce(oracle_lib):
    """Spin sums without spinors, for both settings of the t-channel width."""
    p = config_events("ggtt", 6)
    for flag in (0, 1):
        o = oracle_lib.me("g g > t t~", p, oracle_lib.default_params(tchan_zero_width=flag))
        ref = np.array([ggtt_trace(*ev, width=0.0 if flag else 1.49) for ev in p])
        assert np.abs(o / ref - 1).max() < 1e-12


def test_eemumu_trace_bruteforce(oracle_lib):
    p = config_events("eemumu", 6)
    o = oracle_lib.me("e+ e- > mu+ mu-", p)
    ref = np.array([eemumu_trace(*ev) for ev in p])
    assert np.abs(o / ref - 1).max() < 1e-12


# ------------------------------------------------------------- invariances
QCD = [("ggtt", "g g > t t~"), ("ggttg", "g g > t t~ g"), ("ggttgg", "g g > t t~ g g"),
       ("ggttggg", "g g > t t~ g g g")]


@pytest.mark.parametrize("cfg,proc", QCD)
def test_gauge_invariance(oracle_lib, cfg, proc):
    """Replacing one gluon's polarisation by k/k^0 makes every colour-ordered
    partial amplitude vanish (zero top width: a fixed width breaks gauge
    invariance at order Gamma/m)."""
    prm = oracle_lib.default_params(wt=0.0)
    npar = oracle_lib.npar(proc)
    p = config_events(cfg, 3)
    gluon_legs = [0, 1] + list(range(4, npar))
    rng = np.random.default_rng(7)
    for ev in p:
        hels = rng.choice(1 << npar, size=4, replace=False)
        scale = max(np.abs(oracle_lib.partial_amps(proc, ev, int(h), params=prm)).max()
                    for h in range(1 << npar))
        for h in hels:
            for leg in gluon_legs:
                a = oracle_lib.partial_amps(proc, ev, int(h), gauge_leg=leg, params=prm)
                assert np.abs(a).max() < 1e-12 * scale


def _boost(p, beta_vec):
    b2 = beta_vec @ beta_vec
    gam = 1 / np.sqrt(1 - b2)
    bp = p[..., 1:] @ beta_vec
    out = np.empty_like(p)
    out[..., 0] = gam * (p[..., 0] + bp)
    out[..., 1:] = p[..., 1:] + ((gam - 1) * bp / b2 + gam * p[..., 0])[..., None] * beta_vec
    return out


def _rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


ALL = [("eemumu", "e+ e- > mu+ mu-")] + QCD


@pytest.mark.parametrize("cfg,proc", ALL)
def test_lorentz_and_parity_invariance(oracle_lib, cfg, proc):
    """Random rotation + boost (beta = 0.9) and spatial parity leave the
    helicity-summed |M|^2 unchanged.  Zero top width: with a fixed width the
    amplitude is not gauge invariant, so the sum over the two physical
    polarisations depends on the frame at order Gamma/m."""
    n = 16 if cfg != "ggttggg" else 4
    p = config_events(cfg, n)
    prm = oracle_lib.default_params(wt=0.0)
    ref = oracle_lib.me(proc, p, prm)
    rng = np.random.default_rng(3)
    beta = rng.normal(size=3)
    beta *= 0.9 / np.linalg.norm(beta)
    R = _rotation(rng)
    q = p.copy()
    q[..., 1:] = q[..., 1:] @ R.T
    q = _boost(q, beta)
    assert np.abs(oracle_lib.me(proc, q, prm) / ref - 1).max() < 1e-11
    par = p.copy()
    par[..., 1:] *= -1
    assert np.abs(oracle_lib.me(proc, par, prm) / ref - 1).max() < 1e-12


@pytest.mark.parametrize("cfg,proc", QCD)
def test_bose_symmetry(oracle_lib, cfg, proc):
    n = 16 if cfg != "ggttggg" else 4
    p = config_events(cfg, n)
    ref = oracle_lib.me(proc, p)
    sw = p[:, [1, 0] + list(range(2, p.shape[1]))]
    assert np.abs(oracle_lib.me(proc, sw) / ref - 1).max() < 1e-12
    npar = p.shape[1]
    if npar >= 6:
        perm = list(range(npar))
        perm[4], perm[npar - 1] = perm[npar - 1], perm[4]
        assert np.abs(oracle_lib.me(proc, p[:, perm]) / ref - 1).max() < 1e-12


# ---------------------------------------------------- helicity selection
@pytest.mark.parametrize("cfg,proc,nlive", [("eemumu", "e+ e- > mu+ mu-", 4),
                                             ("ggtt", "g g > t t~", 4),
                                             ("ggttg", "g g > t t~ g", 12),
                                             ("ggttgg", "g g > t t~ g g", 28),
                                             ("ggttggg", "g g > t t~ g g g", 60)])
def test_massless_helicity_count(oracle_lib, cfg, proc, nlive):
    """Massless quarks: helicity is conserved along each fermion line and a
    tree amplitude with all gluon helicities equal (or all but one) vanishes,
    leaving 2(2^n - 2) live configurations for ttbar + n gluons; ee->mumu has 4."""
    npar = oracle_lib.npar(proc)
    masses = [0.0] * (npar - 2)
    p = rambo(3, 1500.0, masses, seed=21)
    prm = oracle_lib.default_params(mt=0.0, wt=0.0)
    mh = oracle_lib.me_hel(proc, p, prm)
    live = (mh / mh.sum(axis=1, keepdims=True)).max(axis=0) > 1e-20
    assert live.sum() == nlive


def test_ggtt_massive_cm_helicities(oracle_lib):
    """With m_t = 173 in the CM frame exactly the 4 configurations with equal
    gluon helicities and opposite t/tbar helicities vanish; the zeros are a
    property of the frame (they come back to life after a transverse boost)."""
    p = config_events("ggtt", 8)
    mh = oracle_lib.me_hel("g g > t t~", p)
    r = mh / mh.sum(axis=1, keepdims=True)
    dead = sorted(np.nonzero(r.max(axis=0) < 1e-24)[0].tolist())
    # bit i = leg i helicity: legs (g, g, t, tbar)
    assert dead == [4, 7, 8, 11]
    q = _boost(p, np.array([0.5, 0.0, 0.0]))
    mq = oracle_lib.me_hel("g g > t t~", q)
    assert (mq / mq.sum(axis=1, keepdims=True)).max(axis=0).min() > 1e-6


# ------------------------------------------------------------- rounding
@pytest.mark.parametrize("cfg,proc", ALL)
def test_long_double_agrees(oracle_lib, cfg, proc):
    n = 32 if cfg != "ggttggg" else 4
    p = config_events(cfg, n)
    d = oracle_lib.me(proc, p)
    ld = oracle_lib.me(proc, p, long_double=True)
    assert np.median(np.abs(d / ld - 1)) < 5e-14
    assert np.abs(d / ld - 1).max() < 1e-12


# ------------------------------------------------------------------ colour
@pytest.mark.parametrize("proc,ng", [("g g > t t~", 2), ("g g > t t~ g", 3),
                                     ("g g > t t~ g g", 4), ("g g > t t~ g g g", 5)])
def test_colour_ordered_matches_colour_dressed(oracle_lib, proc, ng):
    """Full amplitude from literal f^{abc}, t^a rules with explicit colours
    equals sum_sigma c_sigma A(sigma) from the colour-ordered recursion."""
    cfg = {2: "ggtt", 3: "ggttg", 4: "ggttgg", 5: "ggttggg"}[ng]
    p = config_events(cfg, 2)
    rng = np.random.default_rng(ng)
    npar = oracle_lib.npar(proc)
    checked = 0
    tries = 0
    while checked < (6 if ng < 5 else 2) and tries < 5000:
        tries += 1
        # colours 0..2 (lambda_1..3) and 7 (lambda_8) keep most strings non-zero
        col = list(rng.choice([0, 1, 2, 3, 4, 7], size=ng)) + list(rng.integers(0, 3, size=2))
        c = oracle_lib.colour_basis(ng, col)
        if np.abs(c).max() == 0:
            continue
        ev = p[checked % 2]
        h = int(rng.integers(0, 1 << npar))
        A = oracle_lib.partial_amps(proc, ev, h)
        m1 = (c * A).sum()
        m2 = oracle_lib.dressed_amp(proc, ev, h, col)
        amax = max(np.abs(oracle_lib.partial_amps(proc, ev, hh)).max() for hh in range(1 << npar))
        scale = np.abs(c).max() * amax
        assert abs(m1 - m2) < 1e-12 * scale
        checked += 1
    assert checked >= 2


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_colour_matrix_identities(oracle_lib, n):
    """C_ss = N C_F^n (t^a t^a = C_F 1); C real, symmetric, positive definite;
    C_{sigma tau} depends only on sigma^-1 tau (renaming summed indices);
    entries are rationals with a small common denominator."""
    import itertools
    C = oracle_lib.colour_matrix(n)
    N, CF = 3.0, 4.0 / 3.0
    assert np.allclose(np.diag(C), N * CF ** n, rtol=1e-13)
    assert np.array_equal(C, C.T)
    assert np.linalg.eigvalsh(C).min() > 0.5
    perms = list(itertools.permutations(range(n)))
    index = {pp: i for i, pp in enumerate(perms)}
    for s_i, s in enumerate(perms[:3]):
        inv = [0] * n
        for k, v in enumerate(s):
            inv[v] = k
        for t_i, t in enumerate(perms):
            rel = tuple(inv[t[k]] for k in range(n))
            assert abs(C[s_i, t_i] - C[0, index[rel]]) < 1e-11
    den = {1: 1, 2: 3, 3: 9, 4: 54, 5: 324}[n]
    assert np.abs(C * den - np.round(C * den)).max() < 1e-9
    if n == 2:
        # Tr(t^b t^a t^b t^a) = -C_F/2 (t^b t^a t^b = -t^a / (2N))
        assert abs(C[0, 1] + CF / 2) < 1e-14


# ------------------------------------------------------ total cross section
def test_ggtt_cross_section(oracle_lib):
    """RAMBO Monte-Carlo integral of the oracle over 2-body phase space equals
    sigma = pi alpha_s^2/(3s) [(1 + rho + rho^2/16) ln((1+beta)/(1-beta))
    - beta (7/4 + 31 rho/16)] (pins RAMBO and the overall normalisation)."""
    sqs = 1500.0
    p = rambo(1 << 15, sqs, [MT, MT], seed=31)
    me = oracle_lib.me("g g > t t~", p)
    s = sqs * sqs
    rho = 4 * MT * MT / s
    beta = math.sqrt(1 - rho)
    flux_ps = beta / (8 * math.pi) / (2 * s)
    mc = flux_ps * me.mean()
    err = flux_ps * me.std() / math.sqrt(me.size)
    ref = math.pi * ALPHA_S ** 2 / (3 * s) * ((1 + rho + rho * rho / 16) * math.log((1 + beta) / (1 - beta))
                                              - beta * (7 / 4 + 31 * rho / 16))
    assert abs(mc - ref) < 4 * err
    assert err / ref < 0.01


# ------------------------------------------------------------------ RAMBO
@pytest.mark.parametrize("cfg", ["eemumu", "ggtt", "ggttg", "ggttgg", "ggttggg"])
def test_rambo_kinematics(cfg):
    p = config_events(cfg, 2000)
    sqs = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1]) ** 0.5
    bal = p[:, 0] + p[:, 1] - p[:, 2:].sum(axis=1)
    assert np.abs(bal).max() < 1e-12 * sqs.max()
    m2 = mdot(p, p)
    masses = np.array([0, 0, 173.0, 173.0, 0, 0, 0][:p.shape[1]]) if cfg != "eemumu" else np.zeros(4)
    assert np.abs(m2 - masses ** 2).max() < 1e-9 * sqs.max() ** 2
    assert (p[..., 0] > 0).all()
    # isotropy of the final state: <cos theta> ~ 0
    c = p[:, 2:, 3] / np.linalg.norm(p[:, 2:, 1:], axis=-1)
    assert abs(c.mean()) < 5 / math.sqrt(c.size)
    assert np.array_equal(config_events(cfg, 10), p[:10])


def test_max_weight_bruteforce(oracle_lib):
    """The unweighting step's definition checked element by element with a
    plain loop on a small batch (including a negative factor and a NaN)."""
    me = [1.5, 2.0, float("nan"), 0.25, 7.0]
    f = [2.0, -1.0, 3.0, 8.0, 0.5]
    w, m = oracle_lib.max_weight(me, f)
    expect = []
    for a, b in zip(me, f):
        x = a * b
        expect.append(x if x > 0 else 0.0)
    assert list(w) == expect and m == max(expect) == 3.5
    assert oracle_lib.max_weight([], [])[1] == 0.0


# ------------------------------------------------- device phase-space pins
class _FixedUniforms:
    """numpy.random.Generator stand-in that hands out given uniforms."""

    def __init__(self, u):
        self.u = u

    def random(self, shape):
        assert tuple(shape) == self.u.shape
        return self.u


@pytest.mark.parametrize("masses,sqs", [([0.0, 0.0], 500.0), ([173.0, 173.0], 1500.0),
                                        ([173.0, 173.0, 0.0], 1500.0), ([173.0, 173.0, 0.0, 0.0], 1500.0),
                                        ([173.0, 173.0, 0.0, 0.0, 0.0], 1500.0)])
def test_philox_rambo_matches_extended_precision_rambo(oracle_lib, masses, sqs):
    """The oracle's double-precision RAMBO equals the extended-precision RAMBO
    of the input module fed with the same uniforms."""
    n = 4000
    u = oracle_lib.uniforms(n, len(masses), seed=9)
    ref = rambo(n, sqs, masses, seed=0, rng=_FixedUniforms(u))
    got = oracle_lib.rambo(n, masses, sqs, seed=9)
    rel = np.abs(got - ref).max(axis=(1, 2)) / sqs
    assert np.median(rel) < 1e-15 and rel.max() < 1e-11


def test_philox_uniformity(oracle_lib):
    """Philox4x32-10 stream: uniform on [0,1) (chi-square over 64 bins for
    each of the four draws per particle) and uncorrelated across draws."""
    u = oracle_lib.uniforms(1 << 14, 5, seed=123).reshape(-1, 4)
    assert u.min() >= 0 and u.max() < 1
    for k in range(4):
        h, _ = np.histogram(u[:, k], bins=64, range=(0, 1))
        exp = u.shape[0] / 64
        chi2 = ((h - exp) ** 2 / exp).sum()
        assert chi2 < 63 + 5 * math.sqrt(2 * 63)
    c = np.corrcoef(u.T)
    assert np.abs(c - np.eye(4)).max() < 0.03
    # different seeds and counters give different streams
    assert not np.array_equal(oracle_lib.uniforms(8, 2, 1), oracle_lib.uniforms(8, 2, 2))


def test_qqbar_ttbar_closed_form(oracle_lib):
    """q qbar -> t tbar through one s-channel gluon: spin- and colour-averaged
    |M|^2 = (4/9) g_s^4 [(m^2 - t)^2 + (m^2 - u)^2 + 2 m^2 s] / s^2
    (Combridge 1979; Gluck, Owens, Reya 1978).  This fixes the light-quark
    spinors, the gluon propagator, the colour factor Tr(t^a t^b) Tr(t^a t^b) = 2
    and the averaging 1/36.  The channel with the incoming legs swapped gives
    the same values with swapped momenta."""
    mom = config_events("ggtt", 400)
    g2 = 4 * np.pi * 0.118
    m2 = 173.0 ** 2

    def mdot(a, b):
        return a[..., 0] * b[..., 0] - (a[..., 1:] * b[..., 1:]).sum(axis=-1)
    s = mdot(mom[:, 0] + mom[:, 1], mom[:, 0] + mom[:, 1])
    t = mdot(mom[:, 0] - mom[:, 2], mom[:, 0] - mom[:, 2])
    u = mdot(mom[:, 0] - mom[:, 3], mom[:, 0] - mom[:, 3])
    ref = 4.0 / 9.0 * g2 ** 2 * ((m2 - t) ** 2 + (m2 - u) ** 2 + 2 * m2 * s) / s ** 2
    got = oracle_lib.me("u u~ > t t~", mom)
    assert np.abs(got / ref - 1).max() <= 1e-12
    swapped = np.ascontiguousarray(mom[:, [1, 0, 2, 3]])
    assert np.abs(oracle_lib.me("u~ u > t t~", swapped) / got - 1).max() <= 1e-14
    # massless quarks: only opposite q and qbar helicities couple to the gluon
    hel = oracle_lib.me_hel("u u~ > t t~", mom[:8])
    for h in range(16):
        if ((h >> 0) & 1) == ((h >> 1) & 1):
            assert np.abs(hel[:, h]).max() <= 1e-12 * hel.sum(axis=1).max()


QQG = ["u u~ > t t~ g", "u~ u > t t~ g", "u g > t t~ u", "g u > t t~ u", "u~ g > t t~ u~", "g u~ > t t~ u~"]


@pytest.mark.parametrize("name", QQG)
def test_one_jet_quark_channels_gauge_invariant(oracle_lib, name):
    """One light-quark line, t tbar and a gluon (five diagrams incl. the
    three-gluon vertex): with the gluon polarisation replaced by k/k^0 the
    colour-summed |M|^2 vanishes (top width 0: a fixed width breaks gauge
    invariance at O(Gamma/m)).  This fixes the relative signs and colour
    factors of the five diagrams."""
    mom = config_events("ggttg", 24)
    p0 = oracle_lib.default_params(wt=0.0)
    me = oracle_lib.me(name, mom, p0)
    g = oracle_lib.me_gauge(name, mom, p0)
    assert (me > 0).all()
    assert np.abs(g / me).max() <= 1e-12


def test_one_jet_quark_channels_leg_swap_and_helicity(oracle_lib):
    """The channels with the incoming legs swapped give the same |M|^2 with
    swapped momenta; the massless light line conserves helicity, so half of
    the helicity configurations vanish."""
    mom = config_events("ggttg", 16)
    sw = np.ascontiguousarray(mom[:, [1, 0, 2, 3, 4]])
    for a, b in (("u u~ > t t~ g", "u~ u > t t~ g"), ("u g > t t~ u", "g u > t t~ u"),
                 ("u~ g > t t~ u~", "g u~ > t t~ u~")):
        assert np.abs(oracle_lib.me(b, sw) / oracle_lib.me(a, mom) - 1).max() <= 1e-13
    # u u~ > t t~ g: incoming q and qbar must have opposite helicities;
    # u g > t t~ u: incoming and outgoing quark the same helicity
    for name, legs, same in (("u u~ > t t~ g", (0, 1), True), ("u g > t t~ u", (0, 4), False)):
        hel = oracle_lib.me_hel(name, mom)
        tot = hel.sum(axis=1).max()
        for h in range(32):
            bit_a, bit_b = (h >> legs[0]) & 1, (h >> legs[1]) & 1
            if (bit_a == bit_b) == same:
                assert np.abs(hel[:, h]).max() <= 1e-12 * tot, (name, h)


def _gell_mann():
    """t^a = lambda^a / 2 (numpy, independent of the oracle's tables)."""
    l = np.zeros((8, 3, 3), dtype=complex)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return l / 2


def test_one_jet_soft_gluon_limit(oracle_lib):
    """q qbar -> t tbar g as the gluon energy goes to zero: the colour-summed
    |M|^2 tends to  -g^2 sum_{i,j} (p_i.p_j)/((p_i.k)(p_j.k)) <T_i.T_j>/<1> x
    |M|^2(q qbar -> t tbar)  (eikonal factorisation; i = j terms give the
    m_i^2/(p_i.k)^2 C_F of the massive tops).  The colour correlators of the
    Born colour tensor sum_A (t^A)_{b a} (t^A)_{t tb} are computed here by
    brute force, with colour conservation sum_i T_i = 0 checked.  This pins
    the normalisation of the one-jet amplitude (couplings, colour sums,
    averaging) to the closed-form-pinned zero-jet process.  Both sides run
    at zero top width: for a soft gluon the top propagators are off shell by
    2 p_t.k, far below m_t Gamma_t, so a finite width would switch the
    emission from the tops off and the eikonal limit would not hold."""
    t = _gell_mann()
    # Born colour tensor c[a, b, t, tb]: a incoming quark, b incoming antiquark
    c = np.einsum("Aba,Atu->abtu", t, t)
    # colour charges (all legs read as outgoing): incoming quark -> -t^T on a,
    # incoming antiquark -> t on b, outgoing top -> t on t, outgoing antitop -> -t^T on tb
    def charge(i, A, x):
        if i == 0:
            return -np.einsum("ya,ybtu->abtu", t[A], x)
        if i == 1:
            return np.einsum("by,aytu->abtu", t[A], x)
        if i == 2:
            return np.einsum("ty,abyu->abtu", t[A], x)
        return -np.einsum("yu,abty->abtu", t[A], x)
    for A in range(8):
        assert np.abs(sum(charge(i, A, c) for i in range(4))).max() < 1e-14
    norm = np.vdot(c, c).real
    TT = np.array([[sum(np.vdot(charge(i, A, c), charge(j, A, c)) for A in range(8)).real / norm
                    for j in range(4)] for i in range(4)])

    g2 = 4 * np.pi * 0.118
    mt = 173.0
    prm = oracle_lib.default_params(wt=0.0)
    born = config_events("ggtt", 4)

    def mdot(a, b):
        return a[0] * b[0] - a[1:] @ b[1:]

    def boost(p, beta):
        b2 = beta @ beta
        if b2 == 0:
            return p.copy()
        gam = 1 / np.sqrt(1 - b2)
        bp = beta @ p[1:]
        e = gam * (p[0] + bp)
        v = p[1:] + ((gam - 1) * bp / b2 + gam * p[0]) * beta
        return np.concatenate([[e], v])

    rng = np.random.default_rng(3)
    for ev in born:
        p0, p1, p2, p3 = ev
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        dirt = p2[1:] / np.linalg.norm(p2[1:])
        errs = []
        for lam in (1e-2, 1e-3):
            k = lam * np.concatenate([[1.0], n])
            P = p0 + p1 - k
            mp = np.sqrt(mdot(P, P))
            es = mp / 2
            ps = np.sqrt(es * es - mt * mt)
            q2 = boost(np.concatenate([[es], ps * dirt]), P[1:] / P[0])
            q3 = boost(np.concatenate([[es], -ps * dirt]), P[1:] / P[0])
            five = np.array([[p0, p1, q2, q3, k]])
            four = np.array([[p0, p1, q2 + 0.5 * k, q3 + 0.5 * k]])   # on the Born surface up to O(k)
            legs = [p0, p1, q2, q3]
            eik = 0.0
            for i in range(4):
                for j in range(4):
                    eik += mdot(legs[i], legs[j]) / (mdot(legs[i], k) * mdot(legs[j], k)) * TT[i, j]
            pred = -g2 * eik * oracle_lib.me("u u~ > t t~", four, prm)[0]
            errs.append(abs(oracle_lib.me("u u~ > t t~ g", five, prm)[0] / pred - 1))
        print(f"  soft-gluon limit: |ratio - 1| = {errs[0]:.2e} (k0 = 1e-2 GeV), {errs[1]:.2e} (k0 = 1e-3 GeV)")
        # next-to-soft corrections are O(k): the error falls tenfold with the gluon energy
        assert errs[1] < 1e-4 and errs[1] < errs[0] / 5, errs


def _gluon_basis(t, n):
    """Colour-flow tensors c_sigma[a_0..a_{n-1}, i_t, j_tbar] =
    (t^{a_sigma1} ... t^{a_sigman})_{i_t j_tbar}, sigma in lexicographic order."""
    out = []
    for s in itertools.permutations(range(n)):
        m = np.ones((1,) * n + (3, 3), dtype=complex) * np.eye(3)
        for g in s:
            sh = [1] * n + [3, 3]
            sh[g] = 8
            m = np.einsum("...ij,...jk->...ik", m, t.reshape(sh))
        out.append(m)
    return np.array(out)


def _apply_on_axis(b, ax, mat):
    """mat[x, y] acting on tensor axis ax of every basis tensor (axis 0 = basis index)."""
    return np.moveaxis(np.tensordot(mat, b, axes=([1], [ax + 1])), 0, ax + 1)


def _soft_event(born, k, masses):
    """Add the soft momentum k to a Born event given in its centre-of-mass
    frame: the final-state 3-momenta are scaled by one factor so that their
    energies add up to sqrt((P_in - k)^2), then boosted to the frame of P_in - k."""
    pin = born[0] + born[1]
    assert np.abs(pin[1:]).max() < 1e-9 * pin[0]
    q = pin - k
    mq = np.sqrt(q[0] ** 2 - q[1:] @ q[1:])
    pv = born[2:, 1:]
    m = np.asarray(masses)
    lo, hi = 0.0, 1.0
    for _ in range(200):
        xi = 0.5 * (lo + hi)
        if np.sqrt(m * m + xi * xi * (pv * pv).sum(1)).sum() > mq:
            hi = xi
        else:
            lo = xi
    beta = q[1:] / q[0]
    gam = 1 / np.sqrt(1 - beta @ beta)
    out = [born[0], born[1]]
    for mi, p in zip(m, xi * pv):
        e = np.sqrt(mi * mi + p @ p)
        bp = beta @ p
        out.append(np.concatenate([[gam * (e + bp)], p + ((gam - 1) * bp / (beta @ beta) + gam * e) * beta]))
    out.append(k)
    return np.array(out)


@pytest.mark.parametrize("nglu", [0, 1, 2])
def test_gluon_channels_soft_gluon_limit(oracle_lib, nglu):
    """g g -> t tbar + (n+1) g with the last gluon soft factorises onto
    g g -> t tbar + n g: the colour- and helicity-summed |M|^2 tends to
    -g^2 sum_{i,j} (p_i.p_j)/((p_i.k)(p_j.k)) <A| T_i.T_j |A>, summed over the
    Born helicities, with |A> the Born's partial amplitudes in the colour-flow
    basis.  The basis tensors and the colour charges of every leg (adjoint
    -i f for gluons, t for the top, -t^T for the antitop) are built here from
    Gell-Mann matrices, with colour conservation checked and the Born colour
    sum compared with the Born |M|^2.  Chained from the closed-form-pinned
    g g -> t tbar, this pins the absolute normalisation of each extra gluon
    (coupling, three- and four-gluon vertices, colour factors, averaging and
    identical-particle factors).  Zero top width on both sides, as for the
    quark channel."""
    t = _gell_mann()
    f = np.array([[[(-2j * np.trace(t[a] @ (t[b] @ t[c] - t[c] @ t[b]))).real for c in range(8)]
                   for b in range(8)] for a in range(8)])
    adj = np.array([-1j * f[c] for c in range(8)])
    n = nglu + 2                       # gluons in the Born
    basis = _gluon_basis(t, n)
    nb = basis.shape[0]
    # legs 0, 1 -> gluon axes 0, 1; leg 2 (top) -> axis n; leg 3 (antitop) -> axis n + 1;
    # leg 4 + m -> gluon axis 2 + m
    axes = [0, 1, n, n + 1] + [2 + m for m in range(n - 2)]
    tt = np.zeros((n + 2, n + 2, nb, nb), dtype=complex)
    for col in range(8):
        q = []
        for leg, ax in enumerate(axes):
            if leg == 2:
                q.append(_apply_on_axis(basis, ax, t[col]))
            elif leg == 3:
                q.append(-_apply_on_axis(basis, ax, t[col].T))
            else:
                q.append(_apply_on_axis(basis, ax, adj[col]))
        assert np.abs(sum(q)).max() < 1e-13
        qf = [x.reshape(nb, -1) for x in q]
        for i in range(n + 2):
            for j in range(n + 2):
                tt[i, j] += qf[i].conj() @ qf[j].T
    bf = basis.reshape(nb, -1)
    gmat = bf.conj() @ bf.T

    names = ["g g > t t~", "g g > t t~ g", "g g > t t~ g g", "g g > t t~ g g g"]
    born_p, real_p = names[nglu], names[nglu + 1]
    prm = oracle_lib.default_params(wt=0.0)
    g2 = 4 * np.pi * 0.118

    def mdot(a, b):
        return a[0] * b[0] - a[1:] @ b[1:]

    rng = np.random.default_rng(5)
    for ev in config_events(["ggtt", "ggttg", "ggttgg"][nglu], 2):
        nhat = rng.normal(size=3)
        nhat /= np.linalg.norm(nhat)
        born_sum = 0.0
        errs = []
        for lam in (1e-2, 1e-3):
            k = lam * np.concatenate([[1.0], nhat])
            real = _soft_event(ev, k, [173.0, 173.0] + [0.0] * nglu)
            legs = real[:-1]
            eik = np.array([[mdot(legs[i], legs[j]) / (mdot(legs[i], k) * mdot(legs[j], k))
                             for j in range(n + 2)] for i in range(n + 2)])
            corr = 0.0
            born_sum = 0.0
            for h in range(2 ** (n + 2)):
                a = oracle_lib.partial_amps(born_p, ev, h, params=prm)
                born_sum += np.vdot(a, gmat @ a).real
                corr += np.einsum("ij,ij->", eik, np.einsum("s,ijst,t->ij", a.conj(), tt, a)).real
            real_me = oracle_lib.me(real_p, real[None], prm)[0] * oracle_lib.iden(real_p)
            errs.append(abs(real_me / (-g2 * corr) - 1))
        born_me = oracle_lib.me(born_p, ev[None], prm)[0] * oracle_lib.iden(born_p)
        assert abs(born_sum / born_me - 1) < 1e-12
        print(f"  {real_p}: soft-gluon limit |ratio - 1| = {errs[0]:.2e}, {errs[1]:.2e}")
        assert errs[1] < 1e-4 and errs[1] < errs[0] / 5, errs


def _qqbar_ttbar_g_trace(p1, p2, p3, p4, k, mt, t, f, pol_sum):
    """sum over spins, colours and gluon polarisations of |M|^2 / g_s^6 for
    q(p1) qbar(p2) -> t(p3) tbar(p4) g(k), zero widths, by the trace
    technique: each diagram is a 16x16 matrix on (light-line spinor) x
    (top-line spinor) space for each gluon index mu, and the spin sum is
    Tr[K_d (p1-slash x (p4-slash - m)) Kbar_e (p2-slash x (p3-slash + m))].
    Feynman rules: vertex i g gamma^mu t^a, fermion propagator
    i(p-slash + m)/(p^2 - m^2), gluon propagator -i g_{mu nu}/q^2, three-gluon
    vertex g f^{abc}[g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu]
    with all momenta incoming.  pol_sum(mu, mu') is the gluon polarisation
    sum.  Momenta may be crossed (negative energies): nothing here needs a
    spinor."""
    i2, z2 = np.eye(2), np.zeros((2, 2))
    sig = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]),
           np.array([[1, 0], [0, -1]], complex)]
    g0 = np.block([[i2, z2], [z2, -i2]]).astype(complex)
    gam = [g0] + [np.block([[z2, s], [-s, z2]]) for s in sig]     # Dirac representation
    eta = np.array([1.0, -1.0, -1.0, -1.0])
    one = np.eye(4)

    def sl(p):
        return sum(eta[m] * p[m] * gam[m] for m in range(4))

    def msq(p):
        return p[0] ** 2 - p[1:] @ p[1:]

    # colour tensors c_d[j, i, t, u, a]: j incoming antiquark, i incoming quark,
    # t top, u antitop, a emitted gluon
    col = np.zeros((5, 3, 3, 3, 3, 8), complex)
    for a in range(8):
        for b in range(8):
            col[0, ..., a] += np.einsum("ji,tu->jitu", t[b] @ t[a], t[b])
            col[1, ..., a] += np.einsum("ji,tu->jitu", t[a] @ t[b], t[b])
            col[2, ..., a] += np.einsum("ji,tu->jitu", t[b], t[a] @ t[b])
            col[3, ..., a] += np.einsum("ji,tu->jitu", t[b], t[b] @ t[a])
            for c in range(8):
                if f[a, b, c] != 0:
                    col[4, ..., a] += f[a, b, c] * np.einsum("ji,tu->jitu", t[b], t[c])
    cf = col.reshape(5, -1)
    cmat = cf @ cf.conj().T

    s, q = msq(p1 + p2), p3 + p4
    q2 = msq(q)
    s1 = sl(p1 - k) / msq(p1 - k)
    s2 = sl(k - p2) / msq(k - p2)
    s3 = (sl(p3 + k) + mt * one) / (msq(p3 + k) - mt * mt)
    s4 = (-sl(p4 + k) + mt * one) / (msq(p4 + k) - mt * mt)
    kd = np.zeros((5, 4, 16, 16), complex)
    # diagrams 1-4 carry (i g)^3 i (-i) = -i g^3; diagram 5 (i g)^2 (-i)^2 g = g^3
    for mu in range(4):
        for nu in range(4):
            kd[0, mu] += -1j * eta[nu] * np.kron(gam[nu] @ s1 @ gam[mu], gam[nu]) / q2
            kd[1, mu] += -1j * eta[nu] * np.kron(gam[mu] @ s2 @ gam[nu], gam[nu]) / q2
            kd[2, mu] += -1j * eta[nu] * np.kron(gam[nu], gam[mu] @ s3 @ gam[nu]) / s
            kd[3, mu] += -1j * eta[nu] * np.kron(gam[nu], gam[nu] @ s4 @ gam[mu]) / s
    # gluons at the three-gluon vertex: (mu, a, -k), (nu, b, p1 + p2), (rho, c, -q)
    ka, kb, kc = -k, p1 + p2, -q
    g = np.diag(eta)
    v = (np.einsum("mn,r->mnr", g, ka - kb) + np.einsum("nr,m->mnr", g, kb - kc)
         + np.einsum("rm,n->mnr", g, kc - ka))
    for mu, nu, rho in itertools.product(range(4), repeat=3):
        if v[mu, nu, rho] != 0:
            kd[4, mu] += eta[nu] * eta[rho] * v[mu, nu, rho] * np.kron(gam[nu], gam[rho]) / (s * q2)
    gg0 = np.kron(g0, g0)
    kbar = np.einsum("ab,dmcb,cx->dmax", gg0, kd.conj(), gg0)
    pr = np.kron(sl(p1), sl(p4) - mt * one)
    pl = np.kron(sl(p2), sl(p3) + mt * one)
    tot = 0.0
    for d, e in itertools.product(range(5), repeat=2):
        for mu, mp in itertools.product(range(4), repeat=2):
            w = pol_sum(mu, mp)
            if w != 0:
                tot += cmat[d, e] * w * np.trace(kd[d, mu] @ pr @ kbar[e, mp] @ pl)
    return tot


def test_one_jet_trace_technique_and_crossing(oracle_lib):
    """All six one-jet light-quark channels against one independent
    evaluation of q qbar -> t tbar g: literal Feynman rules, spin sums as
    Dirac traces (no spinors, no helicities), colour by brute force over
    explicit colour tensors, polarisation sum -g_{mu nu} (valid with a single
    external gluon, which the k_mu k_nu sum checks).  The q g and qbar g
    channels follow by crossing: an outgoing quark of momentum p becomes an
    incoming antiquark of momentum -p (one fermion crossed: overall sign -1),
    an incoming gluon of momentum p an outgoing one of momentum -p.
    Averaging: 36 for q qbar, 96 for q g (2 x 2 spins, 3 x 8 colours)."""
    t = _gell_mann()
    f = np.array([[[(-2j * np.trace(t[a] @ (t[b] @ t[c] - t[c] @ t[b]))).real for c in range(8)]
                   for b in range(8)] for a in range(8)])
    eta = np.array([1.0, -1.0, -1.0, -1.0])
    mt = 173.0
    prm = oracle_lib.default_params(wt=0.0)
    gs6 = (4 * np.pi * 0.118) ** 3

    def tr(p1, p2, p3, p4, k, pol=None):
        ps = pol or (lambda m, n: -eta[m] if m == n else 0.0)
        return _qqbar_ttbar_g_trace(p1, p2, p3, p4, k, mt, t, f, ps)

    for ev in config_events("ggttg", 4):
        pa, pb, p3, p4, p5 = ev
        direct = tr(pa, pb, p3, p4, p5)
        kl = eta * p5
        gauge = tr(pa, pb, p3, p4, p5, lambda m, n: kl[m] * kl[n])
        assert abs(gauge) <= 1e-12 * p5[0] ** 2 * abs(direct)
        assert abs(direct.imag) <= 1e-14 * abs(direct.real)
        want = {
            "u u~ > t t~ g": direct,
            "u~ u > t t~ g": tr(pb, pa, p3, p4, p5),
            "u g > t t~ u": -tr(pa, -p5, p3, p4, -pb),
            "g u > t t~ u": -tr(pb, -p5, p3, p4, -pa),
            "u~ g > t t~ u~": -tr(-p5, pa, p3, p4, -pb),
            "g u~ > t t~ u~": -tr(-p5, pb, p3, p4, -pa),
        }
        for name, w in want.items():
            got = oracle_lib.me(name, ev[None], prm)[0]
            expect = w.real * gs6 / oracle_lib.iden(name)
            assert abs(got / expect - 1) <= 1e-12, (name, got, expect)
