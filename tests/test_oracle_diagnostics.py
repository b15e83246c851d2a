"""Pins of the oracle's particle diagnostics (Sec. 4.2: energy distribution, kinetic pressure):
brute force on small inputs, exact placements, and the closed forms of the Maxwell-Juttner
distribution (<gamma> = K1(1/theta)/K2(1/theta) + 3 theta; ideal-gas pressure n theta)."""
import math

import numpy as np
from scipy.special import kn

import oracle


def brute_histogram(u, edges):
    counts = [0] * (len(edges) + 1)
    for ux, uy, uz in u:
        uu = ux * ux + uy * uy + uz * uz
        k = uu / (math.sqrt(1.0 + uu) + 1.0)
        if k != k:
            counts[-1] += 1
            continue
        slot = 0
        for e in edges:
            if e <= k:
                slot += 1
        counts[slot] += 1
    return counts


def test_histogram_matches_brute_force():
    rng = np.random.default_rng(5)
    u = (rng.standard_normal((300, 3)) * rng.choice([0.01, 0.3, 3.0, 30.0], (300, 1))).astype(np.float32)
    edges = [1e-4, 1e-3, 0.01, 0.1, 1.0, 10.0, 100.0]
    got = oracle.energy_histogram(u[:, 0], u[:, 1], u[:, 2], edges)
    assert list(got) == brute_histogram(u.astype(np.float64), edges)
    assert got.sum() == 300


def test_histogram_exact_placements():
    # at rest: energy 0, in the bin [-1, 1e-6); u = sqrt(3) and sqrt(120) (energies 1 and 10 up
    # to rounding) land in the bins that hold 1 and 10; NaN goes to the last slot
    u = np.array([[0, 0, 0], [0, math.sqrt(3.0), 0], [math.sqrt(120.0), 0, 0], [np.nan, 0, 0]])
    edges = [-1.0, 1e-6, 0.5, 5.0, 50.0]
    assert list(oracle.energy_histogram(u[:, 0], u[:, 1], u[:, 2], edges)) == [0, 1, 0, 1, 1, 1]
    # a particle at rest (energy exactly 0) below the first edge, and on the last edge
    z = np.zeros(1)
    assert list(oracle.energy_histogram(z, z, z, [0.5, 1.0])) == [1, 0, 0]
    assert list(oracle.energy_histogram(z, z, z, [-1.0, 0.0])) == [0, 0, 1]


def juttner_quantiles(theta, n):
    """|u| at the midpoint quantiles of f(u) ~ u^2 exp(-gamma/theta), CDF by the trapezoid
    rule on a fine grid (independent of the oracle's inverse-CDF table)."""
    umax = math.sqrt((1 + 60 * theta) ** 2 - 1)
    ug = np.linspace(0.0, umax, 400001)
    f = ug * ug * np.exp(-(np.sqrt(1 + ug * ug) - 1) / theta)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(ug))])
    cdf /= cdf[-1]
    return np.interp((np.arange(n) + 0.5) / n, cdf, ug)


def test_juttner_mean_energy_and_pressure():
    theta = 0.3
    r = juttner_quantiles(theta, 20000)
    # the six axis directions: <u_x^2> = |u|^2 / 3 exactly
    u = np.zeros((3, 6 * len(r)))
    for a in range(3):
        u[a, (2 * a) * len(r):(2 * a + 1) * len(r)] = r
        u[a, (2 * a + 1) * len(r):(2 * a + 2) * len(r)] = -r
    n = u.shape[1]
    mean_gamma = kn(1, 1 / theta) / kn(2, 1 / theta) + 3 * theta
    assert abs(oracle.kinetic_energy(*u).mean() - (mean_gamma - 1)) < 2e-5
    P = oracle.kinetic_stress(*u, m=2.0) / n  # per particle, m = 2
    assert np.all(np.abs(P - 2.0 * theta) < 2e-5 * 2.0), P
    # one particle: u = (3, 0, 0), gamma = sqrt(10)
    assert np.allclose(oracle.kinetic_stress([3.0], [0.0], [0.0]), [9 / math.sqrt(10), 0, 0], rtol=1e-15)
