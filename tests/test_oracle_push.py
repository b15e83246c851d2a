"""Pins of the oracle's particle pushers against what the paper and the mathematics fix.

Boris (the alpha = 0 / Lambda = 0 limits of Secs. 2.2 and 3.2), the shearing-box push
(eq. OAu_disc and its closed-form solution, Sec. 2.2) and the expanding-box push
(eq. EBu_disc and the modified Boris operator, Sec. 3.2).  Each pin is chosen so that a
dropped term, a flipped sign or a transposed operand fails it:
  * brute-force linear solves of the discrete equations;
  * consistency with the continuous equations (eq. OAu, eq. EBu) integrated by a generic
    ODE solver: the local error of a consistent second-order scheme falls 8x per halving;
  * closed forms: gyration angle, E x B drift, epicyclic frequency and invariant, the
    scale-factor invariant of the expanding box.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def cross_mat(t):
    """matrix X with X v = v x t"""
    return np.array([[0.0, t[2], -t[1]], [-t[2], 0.0, t[0]], [t[1], -t[0], 0.0]])


def rand_inputs(rng, n, emax=0.05, bmax=0.3, umax=2.0):
    E = rng.uniform(-emax, emax, (n, 3))
    B = rng.uniform(-bmax, bmax, (n, 3))
    u = rng.uniform(-umax, umax, (n, 3))
    return E, B, u


# ---------------------------------------------------------------- Boris

def test_boris_equals_linear_solve():
    rng = np.random.default_rng(11)
    E, B, u = rand_inputs(rng, 400)
    qm, dt = -1.0, 0.45
    got = oracle.push_boris(qm, dt, E, B, u)
    for p in range(len(u)):
        eps = qm * dt * E[p] / 2
        um = u[p] + eps
        gb = np.sqrt(1 + um @ um)
        tau = qm * dt * B[p] / (2 * gb)
        X = cross_mat(tau)
        up = np.linalg.solve(np.eye(3) - X, (np.eye(3) + X) @ um)
        np.testing.assert_allclose(got[p], up + eps, rtol=0, atol=1e-13 * (1 + np.abs(up).max()))


def test_boris_rotation_preserves_norm_and_gyro_angle():
    """E = 0: |u| is preserved and u turns by 2 atan(|tau|) per step about B."""
    rng = np.random.default_rng(3)
    n = 200
    u = rng.normal(size=(n, 3))
    Bz = rng.uniform(0.01, 1.0, n)
    B = np.zeros((n, 3))
    B[:, 2] = Bz
    E = np.zeros((n, 3))
    qm, dt = 1.0, 0.45
    got = oracle.push_boris(qm, dt, E, B, u)
    np.testing.assert_allclose(np.linalg.norm(got, axis=1), np.linalg.norm(u, axis=1), rtol=1e-14)
    gam = np.sqrt(1 + (u * u).sum(1))
    ang = np.arctan2(got[:, 1], got[:, 0]) - np.arctan2(u[:, 1], u[:, 0])
    ang = (ang + np.pi) % (2 * np.pi) - np.pi
    expect = -2 * np.arctan(qm * dt * Bz / (2 * gam))  # positive charge gyrates clockwise about +z
    np.testing.assert_allclose(ang, expect, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(got[:, 2], u[:, 2], rtol=1e-14, atol=1e-16)


def test_boris_exb_drift():
    """Time-averaged velocity over many gyroperiods equals c E x B / B^2."""
    qm, dt = 1.0, 0.1
    B = np.array([[0.0, 0.0, 1.0]])
    E = np.array([[0.0, 0.01, 0.0]])  # v_E = E x B / B^2 = (0.01, 0, 0)
    u = np.array([[0.0, 0.0, 0.0]])
    vs = []
    nsteps = int(200 * 2 * np.pi / dt)  # about 200 gyroperiods
    for _ in range(nsteps):
        u = oracle.push_boris(qm, dt, E, B, u)
        vs.append(u[0] / np.sqrt(1 + u[0] @ u[0]))
    v = np.mean(vs, axis=0)
    vE = np.cross(E[0], B[0]) / (B[0] @ B[0])
    assert abs(v[0] - vE[0]) < 1e-3 * abs(vE[0]) + 2e-6
    assert abs(v[1]) < 2e-5 and abs(v[2]) < 1e-12


# ---------------------------------------------------------------- shearing box

def shear_disc_solve(qm, dt, s, om, xr, E, B, u, gbar):
    """Brute force: solve eq. OAu_disc as a 3x3 linear system for u+."""
    eps = qm * dt * E / 2
    um = u + eps
    et = eps / gbar
    tt = qm * dt * B / 2 / gbar + dt * np.array([0, 0, om])
    a1, a2 = s * om * dt / 2, s * om * xr
    X = cross_mat(tt)
    ey = np.array([0.0, 1.0, 0.0])
    S = np.outer(ey, np.array([a1 + a2 * et[0], a2 * et[1], a2 * et[2]]))
    up = np.linalg.solve(np.eye(3) - X - S, (np.eye(3) + X + S) @ um)
    return up + eps


def test_shear_closed_form_equals_linear_solve():
    rng = np.random.default_rng(5)
    n = 300
    E, B, u = rand_inputs(rng, n)
    xr = rng.uniform(-128, 128, n)
    qm, dt, s, om = 1.0, 0.45, 1.5, 0.01
    got, gb = oracle.push_shear(qm, dt, s, om, xr, E, B, u, return_gbar=True)
    for p in range(n):
        ref = shear_disc_solve(qm, dt, s, om, xr[p], E[p], B[p], u[p], gb[p])
        np.testing.assert_allclose(got[p], ref, rtol=0, atol=2e-13 * (1 + np.abs(ref).max()))


def test_shear_reduces_to_boris():
    """alpha1 = alpha2 = 0 and Omega0 = 0: S = 0 and the push is Boris (Sec. 2.2)."""
    rng = np.random.default_rng(6)
    E, B, u = rand_inputs(rng, 200)
    a = oracle.push_shear(-1.0, 0.45, 1.5, 0.0, np.full(200, 30.0), E, B, u)
    b = oracle.push_boris(-1.0, 0.45, E, B, u)
    np.testing.assert_allclose(a, b, rtol=1e-15, atol=1e-15)


def test_shear_gamma_bar_root():
    """gamma-bar is the largest real root of g^3 - (1+A) g - K (numpy.roots); with
    alpha = 0 it is sqrt(1 + (u-)^2)."""
    rng = np.random.default_rng(7)
    for _ in range(500):
        A = rng.uniform(0, 20)
        K = rng.uniform(-0.5, 0.5)
        g = oracle.shear_gamma_bar(A, K)
        r = np.roots([1.0, 0.0, -(1 + A), -K])
        rr = r[np.abs(r.imag) < 1e-9].real.max()
        assert abs(g - rr) <= 1e-12 * rr
    for A in (0.0, 0.3, 7.0):
        assert abs(oracle.shear_gamma_bar(A, 0.0) - np.sqrt(1 + A)) < 1e-15 * np.sqrt(1 + A)


def test_shear_gamma_bar_first_order_approximation():
    """The printed approximation of gamma-bar (small Omega0) differs from the root at second
    order in Omega0: halving Omega0 divides the difference by about 4."""
    rng = np.random.default_rng(8)
    E, B, u = rand_inputs(rng, 50, emax=0.05)
    xr = rng.uniform(-100, 100, 50)
    qm, dt, s = 1.0, 0.45, 1.5
    errs = []
    for om in (0.02, 0.01, 0.005):
        _, gb = oracle.push_shear(qm, dt, s, om, xr, E, B, u, return_gbar=True)
        eps = qm * dt * E / 2
        um = u + eps
        gm = np.sqrt(1 + (um * um).sum(1))
        a1, a2 = s * om * dt / 2, s * om * xr
        approx = gm + (a1 * um[:, 0] * um[:, 1] * gm + a2 * (um * eps).sum(1) * um[:, 1]) / gm**2
        errs.append(np.abs(gb - approx).max())
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


@pytest.mark.parametrize("xr", [25.0, -60.0])
def test_shear_consistent_with_eq_OAu(xr):
    """Local error of one push against eq. OAu integrated from t^{n-1/2} to t^{n+1/2} (x frozen
    at x^n, where the scheme evaluates it) falls ~8x per halving of dt."""
    qm, s, om = -1.0, 1.5, 0.05
    E = np.array([0.03, -0.02, 0.04])
    B = np.array([0.1, 0.05, 0.2])
    u0 = np.array([0.5, -0.3, 0.7])
    vs = np.array([0.0, -s * om * xr, 0.0])

    def rhs(t, u):
        g = np.sqrt(1 + u @ u)
        return (qm * (E + np.cross(u / g, B)) + 2 * np.cross(u, [0, 0, om]) +
                s * om * u[0] * np.array([0, 1, 0]) - qm * (u @ E / g) * vs)

    errs = []
    for dt in (0.4, 0.2, 0.1):
        ue = solve_ivp(rhs, [0, dt], u0, rtol=1e-13, atol=1e-15).y[:, -1]
        ud = oracle.push_shear(qm, dt, s, om, [xr], E[None], B[None], u0[None])[0]
        errs.append(np.abs(ud - ue).max())
    assert 6.5 < errs[0] / errs[1] < 9.5 and 6.5 < errs[1] / errs[2] < 9.5


@pytest.mark.parametrize("s", [0.0, 0.5, 1.5])
def test_shear_epicycles(s):
    """E = B = 0: du_x/dt = 2 Omega0 u_y, du_y/dt = -(2-s) Omega0 u_x (from eq. OAu).  The
    discrete rotation angle per step is 2 atan(kappa dt/2), kappa^2 = 2(2-s) Omega0^2, and
    (2-s) u_x^2 + 2 u_y^2 is invariant."""
    om, dt, n = 0.01, 0.45, 3000
    u = np.array([[0.01, 0.0, 0.003]])
    Z = np.zeros((1, 3))
    inv0 = (2 - s) * u[0, 0] ** 2 + 2 * u[0, 1] ** 2
    for _ in range(n):
        u = oracle.push_shear(1.0, dt, s, om, [10.0], Z, Z, u)
    inv = (2 - s) * u[0, 0] ** 2 + 2 * u[0, 1] ** 2
    assert abs(inv - inv0) <= 1e-13 * inv0
    kappa = np.sqrt(2 * (2 - s)) * om
    v = u[0, 1] * np.sqrt(2 / (2 - s))
    ang = np.arctan2(-v, u[0, 0])  # (u_x, v) rotates as (cos, -sin) of kappa t
    expect = (n * 2 * np.arctan(kappa * dt / 2) + np.pi) % (2 * np.pi) - np.pi
    d = (ang - expect + np.pi) % (2 * np.pi) - np.pi
    assert abs(d) < 1e-10
    assert u[0, 2] == 0.003


# ---------------------------------------------------------------- expanding box

def expand_solve(qm, dt, lam, E, B, u):
    eps = qm * dt * E / 2
    um = u + eps
    gb = np.sqrt(1 + ((1 + lam) * um) @ ((1 + lam) * um))
    tau = qm * dt * B / (2 * gb)
    X = cross_mat(tau)
    up = np.linalg.solve(np.diag(1 - lam) - X, np.diag(1 + lam) @ um + X @ um)
    return up + eps


def test_expand_isotropic_equals_linear_solve():
    rng = np.random.default_rng(9)
    E, B, u = rand_inputs(rng, 300)
    for p in range(300):
        lam = np.full(3, rng.uniform(-0.05, 0.05))
        got = oracle.push_expand(1.0, 0.45, lam, E[p:p + 1], B[p:p + 1], u[p:p + 1])[0]
        ref = expand_solve(1.0, 0.45, lam, E[p], B[p], u[p])
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * (1 + np.abs(ref).max()))


def test_expand_anisotropic_deviation_bound():
    """For anisotropic diagonal Lambda the printed operator differs from the exact solve of
    eq. EBu_disc by at most ~2 |Lambda| |tau| |u-| per step (a reading recorded in the design)."""
    rng = np.random.default_rng(10)
    E, B, u = rand_inputs(rng, 300)
    worst = 0.0
    for p in range(300):
        lam = rng.uniform(-1e-3, 1e-3) * np.array([1.0, 1.0, 0.0])
        qm, dt = 1.0, 0.45
        got = oracle.push_expand(qm, dt, lam, E[p:p + 1], B[p:p + 1], u[p:p + 1])[0]
        ex = oracle.push_expand(qm, dt, lam, E[p:p + 1], B[p:p + 1], u[p:p + 1], exact=True)[0]
        np.testing.assert_allclose(ex, expand_solve(qm, dt, lam, E[p], B[p], u[p]), rtol=0,
                                   atol=1e-13)
        um = u[p] + qm * dt * E[p] / 2
        gb = np.sqrt(1 + ((1 + lam) * um) @ ((1 + lam) * um))
        tau = np.linalg.norm(qm * dt * B[p] / (2 * gb))
        worst = max(worst, np.linalg.norm(got - ex) / (np.abs(lam).max() * tau * np.linalg.norm(um)))
    assert worst < 2.2


@pytest.mark.parametrize("rates,order", [([0.05, 0.05, 0.05], 3), ([0.05, 0.05, 0.0], 2)])
def test_expand_consistent_with_eq_EBu(rates, order):
    """Local error against eq. EBu (du/dt = q/m (E + u x B/gamma) - L^-1 dL/dt u): third order
    for isotropic expansion; the printed operator is second order for anisotropic
    expansion, while the exact solve of eq. EBu_disc stays third order."""
    qm = 1.0
    E = np.array([0.03, -0.02, 0.04])
    B = np.array([0.1, 0.05, 0.2])
    u0 = np.array([0.5, -0.3, 0.7])
    r = np.array(rates)

    def rhs(t, u):
        return qm * (E + np.cross(u / np.sqrt(1 + u @ u), B)) - r * u

    errs, errx = [], []
    for dt in (0.4, 0.2, 0.1):
        ue = solve_ivp(rhs, [0, dt], u0, rtol=1e-13, atol=1e-15).y[:, -1]
        lam = -0.5 * dt * r
        errs.append(np.abs(oracle.push_expand(qm, dt, lam, E[None], B[None], u0[None])[0] - ue).max())
        errx.append(np.abs(oracle.push_expand(qm, dt, lam, E[None], B[None], u0[None],
                                              exact=True)[0] - ue).max())
    lo, hi = (6.5, 9.5) if order == 3 else (3.2, 4.8)
    assert lo < errs[0] / errs[1] < hi and lo < errs[1] / errs[2] < hi
    assert 6.5 < errx[0] / errx[1] < 9.5


def test_expand_reduces_to_boris():
    rng = np.random.default_rng(12)
    E, B, u = rand_inputs(rng, 100)
    a = oracle.push_expand(-1.0, 0.45, np.zeros(3), E, B, u)
    b = oracle.push_boris(-1.0, 0.45, E, B, u)
    np.testing.assert_allclose(a, b, rtol=1e-15, atol=1e-15)


def test_expand_momentum_scales_with_inverse_scale_factor():
    """E = B = 0, a(t) = 1 + adot t on x and y: with Lambda taken at t^n the factor
    (1+Lambda)/(1-Lambda) equals a(t^{n-1/2})/a(t^{n+1/2}), so u_perp a(t^{n+1/2}) is invariant
    to roundoff and u_z is constant, through the full step of the expanding frame."""
    dt, adot = 0.45, 2.5e-3
    box = oracle.make_box(2, (8, 8), dt=dt, frame=oracle.EXPAND, adot=adot, axis_mask=0b011)
    E, B, J = oracle.zeros_fields(box)
    sp = oracle.SpeciesState([3.3], [4.1], None, [0.4], [-0.2], [0.3], 1.0, 0.0)  # test particle
    for _ in range(400):
        oracle.step(box, E, B, J, [sp])
        a_half = 1 + adot * (box.step - 0.5) * dt
        a_init = 1 - adot * 0.5 * dt  # the loaded momentum is u^{-1/2}
        np.testing.assert_allclose([sp.ux[0] * a_half, sp.uy[0] * a_half],
                                   [0.4 * a_init, -0.2 * a_init], rtol=1e-13)
        assert sp.uz[0] == 0.3
