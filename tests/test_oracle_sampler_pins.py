"""Pins of the oracle's importance-sampled phase-space generator
(oracle_sample: sequential two-body splitting with beam-peaked angles and
soft-favouring remainder masses, each event with its phase-space weight).

Its Monte-Carlo average of the weight must reproduce the phase-space volume
(closed form for massless particles; the exact two-body value; for massive
tops RAMBO's independently weighted estimate), its points must balance and
sit on shell, and sampler x oracle |M|^2 must integrate to the closed-form
total cross section of g g -> t tbar.
"""
import math

import numpy as np
import pytest

ALPHA_S = 0.118
MT = 173.0
SQS = 1500.0


def _massless_volume(n, s):
    """RAMBO's closed form: (2pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!)."""
    return ((2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) * s ** (n - 2)
            / (math.factorial(n - 1) * math.factorial(n - 2)))


def _rambo_weight(mom, masses, sqrt_s):
    """RAMBO's massive weight (Kleiss, Stirling, Ellis): the massless volume
    times (sum|k|/sqrt s)^(2n-3) prod(|k|/E) sqrt s / sum(|k|^2/E)."""
    n = len(masses)
    p = mom[:, 2:]
    k = np.sqrt((p[..., 1:] ** 2).sum(-1))
    E = p[..., 0]
    return (_massless_volume(n, sqrt_s ** 2) * (k.sum(1) / sqrt_s) ** (2 * n - 3) * (k / E).prod(1)
            * sqrt_s / (k ** 2 / E).sum(1))


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_massless_volume(oracle_lib, n):
    """(The mapping favours soft and beam-collinear points, so for a flat
    integrand the weights spread widely at five bodies.)"""
    mom, w = oracle_lib.sample(400000, [0.0] * n, SQS, 11)
    est, err = w.mean(), w.std() / math.sqrt(w.size)
    assert abs(est - _massless_volume(n, SQS ** 2)) < 4 * err
    assert err / est < 0.05


def test_massive_two_body_exact(oracle_lib):
    """Two bodies: the weight divided by the polar-angle Jacobian is the
    exact density lambda^1/2 / (8 pi s) / (4 pi) for every point, and the
    weights average to the volume lambda^1/2 / (8 pi s)."""
    mom, w = oracle_lib.sample(200000, [MT, MT], SQS, 12)
    s = SQS * SQS
    vol = math.sqrt(s * (s - 4 * MT * MT)) / (8 * math.pi * s)
    c = mom[:, 2, 3] / np.sqrt((mom[:, 2, 1:] ** 2).sum(-1))
    eps = 0.01
    jac = 2 * math.atanh(1 / math.sqrt(1 + eps)) * (1 + eps - c * c) / math.sqrt(1 + eps) * 2 * math.pi
    assert np.abs(w / jac / (vol / (4 * math.pi)) - 1).max() < 1e-9
    assert abs(w.mean() - vol) < 4 * w.std() / math.sqrt(w.size)


@pytest.mark.parametrize("masses", [[MT, MT, 0.0], [MT, MT, 0.0, 0.0]])
def test_massive_volume_against_rambo(oracle_lib, masses):
    mom, w = oracle_lib.sample(200000, masses, SQS, 13)
    wr = _rambo_weight(oracle_lib.rambo(200000, masses, SQS, 13), masses, SQS)
    d = w.mean() - wr.mean()
    err = math.hypot(w.std(), wr.std()) / math.sqrt(w.size)
    assert abs(d) < 4 * err and err / wr.mean() < 0.02


@pytest.mark.parametrize("masses", [[MT, MT], [MT, MT, 0.0], [MT, MT, 0.0, 0.0], [MT, MT, 0.0, 0.0, 0.0]])
def test_points_balance_and_on_shell(oracle_lib, masses):
    mom, w = oracle_lib.sample(5000, masses, SQS, 14)
    assert (w > 0).all() and np.isfinite(w).all()
    bal = mom[:, 2:].sum(axis=1) - np.array([SQS, 0, 0, 0])
    assert np.abs(bal).max() < 1e-11 * SQS
    m2 = mom[:, 2:, 0] ** 2 - (mom[:, 2:, 1:] ** 2).sum(-1)
    assert np.abs(m2 - np.array(masses) ** 2).max() < 1e-12 * SQS ** 2
    # the beams
    assert np.array_equal(mom[:, 0], np.broadcast_to([SQS / 2, 0, 0, SQS / 2], (5000, 4)))
    assert np.array_equal(mom[:, 1], np.broadcast_to([SQS / 2, 0, 0, -SQS / 2], (5000, 4)))


def test_ggtt_cross_section_with_sampler(oracle_lib):
    """sigma = 1/(2s) <W |M|^2> over the sampler's points equals the closed
    form pi alpha_s^2/(3s) [(1 + rho + rho^2/16) ln((1+beta)/(1-beta))
    - beta (7/4 + 31 rho/16)] (top width 0 in the t-channel as in the
    closed form)."""
    mom, w = oracle_lib.sample(1 << 15, [MT, MT], SQS, 15)
    me = oracle_lib.me("g g > t t~", mom)
    s = SQS * SQS
    f = w * me / (2 * s)
    mc, err = f.mean(), f.std() / math.sqrt(f.size)
    rho = 4 * MT * MT / s
    beta = math.sqrt(1 - rho)
    ref = math.pi * ALPHA_S ** 2 / (3 * s) * ((1 + rho + rho * rho / 16) * math.log((1 + beta) / (1 - beta))
                                              - beta * (7 / 4 + 31 * rho / 16))
    assert abs(mc - ref) < 4 * err and err / ref < 0.01
