"""Seeded synthetic inputs: RAMBO phase-space points.

This module only generates momenta.  It holds none of the matrix-element
arithmetic and imports nothing else from the package, so the tests can feed
the same events to the GPU path and to the CPU oracle.

RAMBO (Kleiss, Stirling, Ellis, Comput. Phys. Commun. 40 (1986) 359) is the
flat multi-particle generator the paper's standalone test-bed uses to make
batches of test events for throughput measurements (Sec. 2).  Readings where
the paper is silent:
  * random numbers: ``numpy.random.Generator(PCG64(seed))`` uniform doubles,
    drawn event-major, final-particle-major, 4 per particle; a uniform u in
    [0,1) enters the logarithm as 1-u (so it lies in (0,1]);
  * incoming legs are massless and lie on the beam axis in the centre-of-mass
    frame: p1 = (sqrt(s)/2)(1,0,0,1), p2 = (sqrt(s)/2)(1,0,0,-1);
  * massive final states: the massless momenta are rescaled by xi solving
    sum_i sqrt(m_i^2 + xi^2 p0_i^2) = sqrt(s) with Newton's method from
    xi0 = sqrt(1 - (sum m / sqrt s)^2), stopping at |residual| <= 4 eps sqrt(s)
    (extended precision) or after 50 steps;
  * all arithmetic in extended precision, one rounding to double at the end.
"""
from __future__ import annotations

import numpy as np

# Leg masses of the benchmark processes (GeV): top = 173, everything else 0.
PROCESS_LEGS = {
    "e+ e- > mu+ mu-": (0.0, 0.0, 0.0, 0.0),
    "g g > t t~": (0.0, 0.0, 173.0, 173.0),
    "g g > t t~ g": (0.0, 0.0, 173.0, 173.0, 0.0),
    "g g > t t~ g g": (0.0, 0.0, 173.0, 173.0, 0.0, 0.0),
    "g g > t t~ g g g": (0.0, 0.0, 173.0, 173.0, 0.0, 0.0, 0.0),
    "u u~ > t t~": (0.0, 0.0, 173.0, 173.0),
    "u~ u > t t~": (0.0, 0.0, 173.0, 173.0),
    "u u~ > t t~ g": (0.0, 0.0, 173.0, 173.0, 0.0),
    "u~ u > t t~ g": (0.0, 0.0, 173.0, 173.0, 0.0),
    "u g > t t~ u": (0.0, 0.0, 173.0, 173.0, 0.0),
    "g u > t t~ u": (0.0, 0.0, 173.0, 173.0, 0.0),
    "u~ g > t t~ u~": (0.0, 0.0, 173.0, 173.0, 0.0),
    "g u~ > t t~ u~": (0.0, 0.0, 173.0, 173.0, 0.0),
}
# two-jet channels of p p > t t~: t t~ and two massless partons
for _p in ("u u~ > t t~ g g", "u~ u > t t~ g g", "u g > t t~ u g", "g u > t t~ u g", "u~ g > t t~ u~ g",
           "g u~ > t t~ u~ g", "g g > t t~ u u~", "u u~ > t t~ u u~", "u u~ > t t~ d d~", "u u > t t~ u u",
           "u d > t t~ u d", "u~ u~ > t t~ u~ u~"):
    PROCESS_LEGS[_p] = (0.0, 0.0, 173.0, 173.0, 0.0, 0.0)


def rambo(nevt: int, sqrt_s: float, final_masses, seed: int, rng=None) -> np.ndarray:
    """Return float64 momenta [nevt][2 + nfinal][4] as (E, px, py, pz).

    The arithmetic runs in x87 extended precision (numpy longdouble) and is
    rounded to double once at the end, and the invariant mass of the massless
    seeds is formed as sum_{i<j} q0_i q0_j |n_i - n_j|^2 (no cancellation), so
    the events are on shell and balanced to a few ulps of double even for
    nearly collinear seeds.  Plain double RAMBO leaves ~1e-11 relative
    off-shell noise on such events, which different spinor constructions
    turn into different |M|^2 at that level."""
    L = np.longdouble
    masses = np.asarray(final_masses, dtype=np.float64)
    n = masses.size
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.random((nevt, n, 4)).astype(L)
    one, two = L(1), L(2)
    c = two * r[..., 0] - one
    phi = two * np.arccos(L(-1)) * r[..., 1]
    q0 = -np.log((one - r[..., 2]) * (one - r[..., 3]))
    st = np.sqrt(np.maximum(L(0), one - c * c))
    nhat = np.empty((nevt, n, 3), dtype=L)
    nhat[..., 0] = st * np.cos(phi)
    nhat[..., 1] = st * np.sin(phi)
    nhat[..., 2] = c
    q = np.empty((nevt, n, 4), dtype=L)
    q[..., 0] = q0
    q[..., 1:] = q0[..., None] * nhat
    Q = q.sum(axis=1)
    M2 = np.zeros(nevt, dtype=L)
    for i in range(n):
        for j in range(i + 1, n):
            d = nhat[:, i] - nhat[:, j]
            M2 += q0[:, i] * q0[:, j] * (d * d).sum(axis=-1)
    M = np.sqrt(M2)
    b = -Q[:, 1:] / M[:, None]
    gamma = Q[:, 0] / M
    a = one / (one + gamma)
    x = L(sqrt_s) / M
    bq = (b[:, None, :] * q[..., 1:]).sum(axis=-1)
    p = np.empty_like(q)
    p[..., 0] = x[:, None] * (gamma[:, None] * q[..., 0] + bq)
    p[..., 1:] = x[:, None, None] * (q[..., 1:] + b[:, None, :] * q[..., 0:1]
                                     + a[:, None, None] * bq[..., None] * b[:, None, :])
    if n == 2:
        # two bodies: the event is fixed by one direction; rebuild the
        # back-to-back pair from RAMBO's direction so it is exactly on shell
        # and balanced (the conformal boost loses ~gamma^2 eps of accuracy for
        # nearly collinear seeds)
        nd = p[:, 0, 1:] / np.sqrt((p[:, 0, 1:] ** 2).sum(axis=-1))[:, None]
        sq = L(sqrt_s)
        m1, m2 = L(masses[0]), L(masses[1])
        e1 = (sq * sq + m1 * m1 - m2 * m2) / (two * sq)
        e2 = sq - e1
        pabs = np.sqrt(np.maximum(L(0), e1 * e1 - m1 * m1))
        p[:, 0, 0], p[:, 1, 0] = e1, e2
        p[:, 0, 1:] = pabs * nd
        p[:, 1, 1:] = -pabs * nd
    elif np.any(masses > 0):
        p = _rescale_massive(p, masses.astype(L), L(sqrt_s))
    out = np.empty((nevt, n + 2, 4))
    e = 0.5 * sqrt_s
    out[:, 0] = (e, 0.0, 0.0, e)
    out[:, 1] = (e, 0.0, 0.0, -e)
    out[:, 2:] = p.astype(np.float64)
    return out


def _rescale_massive(p, masses, sqrt_s):
    if masses.sum() >= sqrt_s:
        raise ValueError("sqrt(s) below the production threshold")
    m2 = masses[None, :] ** 2
    p02 = p[..., 0] ** 2
    xi = np.full(p.shape[0], np.sqrt(1 - (masses.sum() / sqrt_s) ** 2))
    tol = 4 * np.finfo(np.longdouble).eps * sqrt_s
    for _ in range(50):
        e = np.sqrt(m2 + (xi[:, None] ** 2) * p02)
        f = e.sum(axis=1) - sqrt_s
        todo = np.abs(f) > tol      # per event, so a batch's prefix is reproducible
        if not np.any(todo):
            break
        df = (xi[:, None] * p02 / e).sum(axis=1)
        xi = np.where(todo, xi - f / df, xi)
    k = np.empty_like(p)
    k[..., 1:] = xi[:, None, None] * p[..., 1:]
    k[..., 0] = np.sqrt(m2 + (xi[:, None] ** 2) * p02)
    return k


def process_events(process: str, nevt: int, sqrt_s: float, seed: int) -> np.ndarray:
    """RAMBO events for one of the benchmark processes (leg order of the
    process string, legs 0 and 1 incoming)."""
    masses = PROCESS_LEGS[process]
    if any(m != 0 for m in masses[:2]):
        raise ValueError("massive incoming legs are not supported")
    return rambo(nevt, sqrt_s, masses[2:], seed)


# The benchmark configurations: process, sqrt(s) in GeV, number of events, seed.
CONFIGS = {
    "eemumu": ("e+ e- > mu+ mu-", 500.0, 16384, 1),
    "ggtt": ("g g > t t~", 1500.0, 1 << 19, 2),
    "ggttg": ("g g > t t~ g", 1500.0, 1 << 20, 3),
    "ggttgg": ("g g > t t~ g g", 1500.0, 1 << 20, 4),
    "ggttggg": ("g g > t t~ g g g", 1500.0, 1 << 20, 5),
    # light-quark channels of p p > t t~ (same kinematics as g g > t t~)
    "uutt": ("u u~ > t t~", 1500.0, 1 << 19, 6),
    "uxutt": ("u~ u > t t~", 1500.0, 1 << 19, 7),
    # one-jet channels of p p > t t~ with a light quark (same kinematics as g g > t t~ g)
    "uuttg": ("u u~ > t t~ g", 1500.0, 1 << 20, 8),
    "uxuttg": ("u~ u > t t~ g", 1500.0, 1 << 20, 9),
    "ugttu": ("u g > t t~ u", 1500.0, 1 << 20, 10),
    "guttu": ("g u > t t~ u", 1500.0, 1 << 20, 11),
    "uxgttux": ("u~ g > t t~ u~", 1500.0, 1 << 20, 12),
    "guxttux": ("g u~ > t t~ u~", 1500.0, 1 << 20, 13),
    # two-jet channels of p p > t t~ (same kinematics as g g > t t~ g g)
    "uuttgg": ("u u~ > t t~ g g", 1500.0, 1 << 20, 14),
    "uxuttgg": ("u~ u > t t~ g g", 1500.0, 1 << 20, 15),
    "ugttug": ("u g > t t~ u g", 1500.0, 1 << 20, 16),
    "guttug": ("g u > t t~ u g", 1500.0, 1 << 20, 17),
    "uxgttuxg": ("u~ g > t t~ u~ g", 1500.0, 1 << 20, 18),
    "guxttuxg": ("g u~ > t t~ u~ g", 1500.0, 1 << 20, 19),
    "ggttuux": ("g g > t t~ u u~", 1500.0, 1 << 20, 20),
    "uuttuux": ("u u~ > t t~ u u~", 1500.0, 1 << 20, 21),
    "uuttddx": ("u u~ > t t~ d d~", 1500.0, 1 << 20, 22),
    "uuttuu": ("u u > t t~ u u", 1500.0, 1 << 20, 23),
    "udttud": ("u d > t t~ u d", 1500.0, 1 << 20, 24),
    "uxuxttuxux": ("u~ u~ > t t~ u~ u~", 1500.0, 1 << 20, 25),
}


def config_events(name: str, nevt: int | None = None) -> np.ndarray:
    """Events of a named benchmark configuration.  A prefix of the full batch
    when nevt is smaller (the draws are event-major, so prefixes agree)."""
    process, sqrt_s, n_full, seed = CONFIGS[name]
    return process_events(process, n_full if nevt is None else nevt, sqrt_s, seed)
