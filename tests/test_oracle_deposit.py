"""Pins of the oracle's charge-conserving deposit and of the Gauss-law consistency of a full step.

  * discrete continuity rho^{n+1} - rho^n + dt div J = 0 to roundoff (Esirkepov's identity);
  * the total current equals sum q dx/dt;
  * for moves that stay inside one cell the current equals the exact line integral
    q int v S(x(s)) ds (Villasenor-Buneman, the deposit cited in Sec. 2.2);
  * Gauss's law div E - 4 pi rho is preserved by the full plain step, and in primed
    variables (div' E' - 4 pi rho') by the expanding-box step (Sec. 3.2: the deposit of the
    primed displacement is l J').
"""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle


def div_J(box, J):
    """backward-difference divergence of J (Yee: J on the E lattice) at the nodes"""
    d = J[0] - np.roll(J[0], 1, axis=2)
    d = d + J[1] - np.roll(J[1], 1, axis=1)
    if box.dim == 3:
        d = d + J[2] - np.roll(J[2], 1, axis=0)
    return d


@pytest.mark.parametrize("dim,maxmove", [(2, 0.45), (3, 0.45), (2, 1.2), (3, 1.2)])
def test_continuity(dim, maxmove):
    rng = np.random.default_rng(20 + dim)
    n = (7, 6, 5) if dim == 3 else (9, 8)
    box = oracle.make_box(dim, n, dt=0.45)
    N = 400
    x0 = [rng.uniform(0, n[d], N) for d in range(dim)]
    mv = [rng.uniform(-maxmove, maxmove, N) for d in range(dim)]
    x1 = [x0[d] + mv[d] for d in range(dim)]
    q = -0.7
    z0 = x0[2] if dim == 3 else None
    z1 = x1[2] if dim == 3 else None
    Jext = oracle.deposit(box, q, x0[0], x0[1], x1[0], x1[1], z0, z1)
    J = oracle.finalize_current(box, Jext, 0.0)
    w1 = [np.mod(x1[d], n[d]) for d in range(dim)]
    rho0 = oracle.charge(box, q, x0[0], x0[1], z0)
    rho1 = oracle.charge(box, q, w1[0], w1[1], w1[2] if dim == 3 else None)
    gross = oracle.charge(box, abs(q), x0[0], x0[1], z0).max()
    res = rho1 - rho0 + box.dt * div_J(box, J)
    assert np.abs(res).max() <= 1e-13 * gross


@pytest.mark.parametrize("dim", [2, 3])
def test_total_current(dim):
    rng = np.random.default_rng(30 + dim)
    n = (6, 5, 4) if dim == 3 else (8, 7)
    box = oracle.make_box(dim, n, dt=0.45)
    N = 100
    x0 = [rng.uniform(0, (list(n) + [1])[d], N) for d in range(3)]
    mv = [rng.uniform(-0.45, 0.45, N) for d in range(3)]
    q = 1.3
    dz = mv[2] if dim == 2 else None
    Jext = oracle.deposit(box, q, x0[0], x0[1], x0[0] + mv[0], x0[1] + mv[1],
                          x0[2], x0[2] + mv[2], dz=dz)
    J = oracle.finalize_current(box, Jext, 0.0)
    for c in range(3):
        assert abs(J[c].sum() - q * mv[c].sum() / box.dt) < 1e-12 * (1 + np.abs(mv[c]).sum())


def S(r):
    return max(0.0, 1.0 - abs(r))


@pytest.mark.parametrize("dim", [2, 3])
def test_single_cell_move_is_line_integral(dim):
    """Inside one cell CIC weights are linear along the path, and Esirkepov equals the line
    integral of q v S over the path (Villasenor-Buneman)."""
    rng = np.random.default_rng(40 + dim)
    n = (6, 6, 6) if dim == 3 else (6, 6)
    box = oracle.make_box(dim, n, dt=0.45)
    q, dt = 0.9, 0.45
    for _ in range(20):
        cell = rng.integers(1, 4, 3)
        a = cell + rng.uniform(0.05, 0.95, 3)
        b = cell + rng.uniform(0.05, 0.95, 3)
        dz = rng.uniform(-0.4, 0.4)
        if dim == 2:
            a[2] = b[2] = 0.0
        Jext = oracle.deposit(box, q, [a[0]], [a[1]], [b[0]], [b[1]], [a[2]], [b[2]], dz=[dz])
        J = oracle.finalize_current(box, Jext, 0.0)
        path = lambda s: a + s * (b - a)
        i, j, k = cell
        # J_x on the edge (i+1/2) at nodes (j', k')
        for jj in (j, j + 1):
            for kk in ((k, k + 1) if dim == 3 else (0,)):
                f = lambda s: S(jj - path(s)[1]) * (S(kk - path(s)[2]) if dim == 3 else 1.0)
                ref = q * (b[0] - a[0]) / dt * quad(f, 0, 1, epsabs=1e-14)[0]
                assert abs(J[0][kk, jj, i] - ref) < 1e-12
        for ii in (i, i + 1):
            for kk in ((k, k + 1) if dim == 3 else (0,)):
                f = lambda s: S(ii - path(s)[0]) * (S(kk - path(s)[2]) if dim == 3 else 1.0)
                ref = q * (b[1] - a[1]) / dt * quad(f, 0, 1, epsabs=1e-14)[0]
                assert abs(J[1][kk, j, ii] - ref) < 1e-12
        for ii in (i, i + 1):
            for jj in (j, j + 1):
                f = lambda s: S(ii - path(s)[0]) * S(jj - path(s)[1])
                vz = (b[2] - a[2]) / dt if dim == 3 else dz / dt
                ref = q * vz * quad(f, 0, 1, epsabs=1e-14)[0]
                kk = k if dim == 3 else 0
                assert abs(J[2][kk, jj, ii] - ref) < 1e-12


def yee_div_E(box, E):
    d = E[0] - np.roll(E[0], 1, axis=2) + E[1] - np.roll(E[1], 1, axis=1)
    if box.dim == 3:
        d = d + E[2] - np.roll(E[2], 1, axis=0)
    return d


def thermal_pairs(rng, box, ppc, uth, q):
    n = [box.n[d] for d in range(box.dim)]
    N = ppc * int(np.prod(n))
    pos = [rng.uniform(0, n[d], N) for d in range(box.dim)]
    z = pos[2] if box.dim == 3 else None
    sp = []
    for sgn in (-1.0, 1.0):
        u = rng.normal(0, uth, (3, N))
        sp.append(oracle.SpeciesState(pos[0], pos[1], z, u[0], u[1], u[2], sgn, sgn * q))
    return sp


@pytest.mark.parametrize("dim", [2, 3])
def test_gauss_law_preserved_plain(dim):
    rng = np.random.default_rng(50 + dim)
    n = (8, 8, 8) if dim == 3 else (16, 12)
    box = oracle.make_box(dim, n, dt=0.45)
    E, B, J = oracle.zeros_fields(box)
    B[2][:] = 0.2
    E[0][:] = rng.normal(0, 1e-3, E[0].shape)  # arbitrary initial divergence, carried along
    sp = thermal_pairs(rng, box, 4, 0.5, 0.05)
    g0 = yee_div_E(box, E) - 4 * np.pi * sum(
        oracle.charge(box, s.q, s.x, s.y, s.z if dim == 3 else None) for s in sp)
    for _ in range(12):
        oracle.step(box, E, B, J, sp)
    g1 = yee_div_E(box, E) - 4 * np.pi * sum(
        oracle.charge(box, s.q, s.x, s.y, s.z if dim == 3 else None) for s in sp)
    scale = 4 * np.pi * 0.05 * 8
    assert np.abs(g1 - g0).max() < 1e-12 * scale
    assert np.abs(J).max() > 1e-3  # the plasma did move current


def test_gauss_law_preserved_expanding_primed():
    """div' E' - 4 pi rho' is preserved with E' = l L^-1 E (Sec. 3.1) and rho' the density per
    primed cell of the x' positions."""
    rng = np.random.default_rng(61)
    box = oracle.make_box(2, (12, 10), dt=0.45, frame=oracle.EXPAND, adot=5e-3, axis_mask=0b110)
    E, B, J = oracle.zeros_fields(box)
    B[0][:] = 0.2
    sp = thermal_pairs(rng, box, 4, 0.5, 0.05)

    def gauss():
        t = box.step * box.dt
        l = [oracle.scale(box, d, t) for d in range(3)]
        ell = l[0] * l[1] * l[2]
        Ep = np.stack([ell / l[c] * E[c] for c in range(3)])
        return yee_div_E(box, Ep) - 4 * np.pi * sum(oracle.charge(box, s.q, s.x, s.y) for s in sp)

    g0 = gauss()
    for _ in range(15):
        oracle.step(box, E, B, J, sp)
    assert np.abs(gauss() - g0).max() < 1e-12 * 4 * np.pi * 0.05 * 8
    assert np.abs(E).max() > 1e-5
