"""Pins of the oracle's combined shearing and expanding frame (the extension the conclusion,
Sec. 5, names; the reading composes Sec. 2.2 and Sec. 3.2).

Particle push, (1 - Lambda) u+ - u+ x tau~ - S u+ = (1 + Lambda) u- + u- x tau~ + S u-:
  * the exact mode equals a brute-force linear solve of that equation, and gbar is the largest
    real root of the combined cubic;
  * the printed-style closed form (Sherman-Morrison on the expanding frame's operator) equals
    the exact solve for isotropic Lambda;
  * Lambda = 0 gives the shearing push of Sec. 2.2, s = Omega0 = 0 the expanding push of
    Sec. 3.2;
  * consistency with the continuous equation (eq. OAu plus the -L^-1 dL/dt u' force of
    eq. EBu): local error third order, second for the printed form under anisotropic
    expansion (the same property as the expanding push alone).
Field step, implicit midpoint of Sec. 2.2 on the expanding-frame fields with the curl factors
of eqs. EBB/EBE:
  * no expansion reproduces the shearing-box step bit for bit;
  * uniform fields follow the closed form: B'' = (l/l_c) B is frozen except for the tidal
    term, B''_y(t) = B''_y(0) - s Omega0 B''_x t, and E stays zero;
  * without shear the right-hand side is the shearing-box one on the scaled fields d_c F_c;
    the kz factor multiplies the z transport of E'_y only, against the analytic derivative;
  * a converged step satisfies the implicit-midpoint equation of the scaled fields.
"""
import ctypes as C

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

QM, DT, S_KEP = -1.0, 0.45, 1.5


def rand_inputs(rng, n, emax=0.05, bmax=0.3, umax=2.0):
    return (rng.uniform(-emax, emax, (n, 3)), rng.uniform(-bmax, bmax, (n, 3)),
            rng.uniform(-umax, umax, (n, 3)))


def cross_mat(t):
    """matrix X with X v = v x t"""
    return np.array([[0.0, t[2], -t[1]], [-t[2], 0.0, t[0]], [t[1], -t[0], 0.0]])


def combined_solve(qm, dt, s, om, lam, xr, E, B, u, gbar):
    """u^{n+1/2} from the combined discrete equation, solved by numpy for the given gbar"""
    eps = qm * dt * E / 2
    um = u + eps
    tt = qm * dt * B / (2 * gbar) + np.array([0, 0, dt * om])
    a1, a2 = s * om * dt / 2, s * om * xr
    s2 = np.array([a1, 0, 0]) + a2 * eps / gbar
    Sm = np.zeros((3, 3))
    Sm[1] = s2
    X = cross_mat(tt)
    M = np.diag(1 - lam) - X - Sm
    r = (1 + lam) * um + X @ um + Sm @ um
    return np.linalg.solve(M, r) + eps


def largest_root(qm, dt, s, om, lam, xr, E, u):
    """largest real root of g^3 - (1 + A) g - K with A, K of the combined gbar"""
    eps = qm * dt * E / 2
    um = u + eps
    A = ((1 + lam) * um) @ ((1 + lam) * um) + 2 * (s * om * dt / 2) * um[0] * um[1]
    K = 2 * (s * om * xr) * (um @ eps) * um[1]
    roots = np.roots([1.0, 0.0, -(1.0 + A), -K])
    return max(r.real for r in roots if abs(r.imag) < 1e-9)


# ---------------------------------------------------------------- push

def test_exact_mode_equals_linear_solve_and_gbar_is_the_cubic_root():
    rng = np.random.default_rng(501)
    E, B, u = rand_inputs(rng, 200)
    for p in range(200):
        lam = rng.uniform(-0.02, 0.02, 3)
        om = rng.uniform(-0.03, 0.03)
        xr = rng.uniform(-60, 60)
        got, gb = oracle.push_shear_expand(QM, DT, S_KEP, om, lam, [xr], E[p:p + 1], B[p:p + 1],
                                           u[p:p + 1], exact=True, return_gbar=True)
        g = largest_root(QM, DT, S_KEP, om, lam, xr, E[p], u[p])
        assert abs(gb[0] - g) <= 1e-12 * g
        ref = combined_solve(QM, DT, S_KEP, om, lam, xr, E[p], B[p], u[p], gb[0])
        np.testing.assert_allclose(got[0], ref, rtol=0, atol=1e-12 * (1 + np.abs(ref).max()))


def test_printed_form_is_exact_for_isotropic_expansion():
    rng = np.random.default_rng(502)
    E, B, u = rand_inputs(rng, 300)
    for p in range(300):
        lam = np.full(3, rng.uniform(-0.03, 0.03))
        om = rng.uniform(-0.03, 0.03)
        xr = rng.uniform(-60, 60)
        args = (QM, DT, S_KEP, om, lam, [xr], E[p:p + 1], B[p:p + 1], u[p:p + 1])
        a = oracle.push_shear_expand(*args)[0]
        b = oracle.push_shear_expand(*args, exact=True)[0]
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * (1 + np.abs(b).max()))


def test_reduces_to_each_frame():
    rng = np.random.default_rng(503)
    n = 400
    E, B, u = rand_inputs(rng, n)
    xr = rng.uniform(-60, 60, n)
    # no expansion: the shearing-box push of Sec. 2.2
    sh = oracle.push_shear(QM, DT, S_KEP, 0.02, xr, E, B, u)
    for exact in (False, True):
        got = oracle.push_shear_expand(QM, DT, S_KEP, 0.02, np.zeros(3), xr, E, B, u, exact=exact)
        np.testing.assert_allclose(got, sh, rtol=0, atol=1e-13)
    # no shear, no rotation: the expanding-box push of Sec. 3.2 (printed and exact)
    lam = np.array([-4e-3, -4e-3, 0.0])
    for exact in (False, True):
        ex = oracle.push_expand(QM, DT, lam, E, B, u, exact=exact)
        got = oracle.push_shear_expand(QM, DT, 0.0, 0.0, lam, xr, E, B, u, exact=exact)
        np.testing.assert_allclose(got, ex, rtol=0, atol=1e-13)


@pytest.mark.parametrize("rates,printed_order", [([0.05, 0.05, 0.05], 3), ([0.0, 0.0, 0.06], 2),
                                                 ([0.05, 0.05, 0.0], 2)])
def test_consistent_with_the_continuous_equation(rates, printed_order):
    """One step from u^{n-1/2} against the ODE du'/dt = q/m (E' + u' x B/gamma') + 2 u' x Omega0
    + s Omega0 u'_x e_y + q/m (u'.E'/gamma') s Omega0 x e_y - L^-1 dL/dt u' (eq. OAu with
    v_s = -s Omega0 x e_y, plus eq. EBu's expansion force) at fixed fields and x: the local
    error falls 8x per halving of dt (4x for the printed form under anisotropic expansion)."""
    E = np.array([0.03, -0.02, 0.04])
    B = np.array([0.1, 0.05, 0.2])
    u0 = np.array([0.5, -0.3, 0.7])
    r = np.array(rates)
    om, xr = 0.04, 6.0

    def rhs(t, u):
        g = np.sqrt(1 + u @ u)
        f = QM * (E + np.cross(u / g, B)) + 2 * np.cross(u, [0, 0, om]) - r * u
        f[1] += S_KEP * om * u[0] + QM * (u @ E / g) * S_KEP * om * xr
        return f

    err = {False: [], True: []}
    for dt in (0.4, 0.2, 0.1):
        ue = solve_ivp(rhs, [0, dt], u0, rtol=1e-13, atol=1e-15).y[:, -1]
        lam = -0.5 * dt * r
        for exact in (False, True):
            got = oracle.push_shear_expand(QM, dt, S_KEP, om, lam, [xr], E[None], B[None],
                                           u0[None], exact=exact)[0]
            err[exact].append(np.abs(got - ue).max())
    for exact, order in ((True, 3), (False, printed_order)):
        e = err[exact]
        lo, hi = (6.5, 9.5) if order == 3 else (3.0, 5.0)
        assert lo < e[0] / e[1] < hi and lo < e[1] / e[2] < hi, (exact, e)


# ---------------------------------------------------------------- fields

def _box(frame, n, mask=0b111, adot=0.0, om=0.01, s=S_KEP, step=0, iters=8, tol=0.0):
    return oracle.make_box(len(n), n, frame=frame, shear_s=s, omega0=om, adot=adot,
                           axis_mask=mask, step=step, maxwell_iters=iters, maxwell_tol=tol)


def _rand_fields(n, seed):
    rng = np.random.default_rng(seed)
    shp = (3, n[2] if len(n) == 3 else 1, n[1], n[0])
    return (rng.uniform(-0.05, 0.05, shp), rng.uniform(-0.2, 0.2, shp),
            rng.uniform(-0.01, 0.01, shp))


def test_no_expansion_is_the_shearing_box_step():
    n = (12, 10, 8)
    E, B, J = _rand_fields(n, 511)
    a = _box(oracle.SHEAR, n, step=3)
    b = _box(oracle.SHEAR_EXPAND, n, adot=0.0, step=3)
    Ea, Ba, Eb, Bb = E.copy(), B.copy(), E.copy(), B.copy()
    oracle.maxwell(a, Ea, Ba, J)
    oracle.maxwell(b, Eb, Bb, J)
    np.testing.assert_array_equal(Ea, Eb)
    np.testing.assert_array_equal(Ba, Bb)


@pytest.mark.parametrize("mask", [0b111, 0b100, 0b011])
def test_uniform_field_follows_the_closed_form(mask):
    n = (8, 6, 6)
    adot, om = 2e-3, 0.02
    b = _box(oracle.SHEAR_EXPAND, n, mask=mask, adot=adot, om=om, iters=3)
    shp = (3, n[2], n[1], n[0])
    B0 = np.array([0.3, -0.1, 0.2])
    E = np.zeros(shp)
    B = np.broadcast_to(B0[:, None, None, None], shp).copy()
    J = np.zeros(shp)
    for step in range(1, 41):
        oracle.maxwell(b, E, B, J)
        b.step = step
    t = 40 * DT
    l = np.array([1 + adot * t if (mask >> c) & 1 else 1.0 for c in range(3)])
    sc = l.prod() / l  # B''_c = (l/l_c) B_c, and s_c(0) = 1
    Bpp = B0.copy()
    Bpp[1] = B0[1] - S_KEP * om * B0[0] * t
    want = Bpp / sc
    for c in range(3):
        np.testing.assert_allclose(B[c], want[c], rtol=1e-12, atol=1e-14)
    assert np.abs(E).max() <= 1e-15  # the face interpolation of a uniform field rounds


def test_rhs_factors_without_shear_scale_the_curls():
    n = (10, 8, 6)
    E, B, J = _rand_fields(n, 512)
    b = _box(oracle.SHEAR_EXPAND, n, s=0.0, om=0.0)
    d = np.array([0.9, 1.1, 1.3])
    got = oracle.ksb_rhs_f(b, E, B, J, d, kz=1.7)
    ref = oracle.ksb_rhs(b, d[:, None, None, None] * E, d[:, None, None, None] * B, J)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-15)


def test_kz_multiplies_the_z_transport_of_Ey():
    """E'_y = sin(2 pi z / n_z) alone: kz changes only dE'z/dt, by -v (kz - 1) dE'y/dz, with
    the central difference within O(h^2) of the analytic derivative."""
    n = (16, 4, 32)
    b = _box(oracle.SHEAR_EXPAND, n, om=0.01)
    shp = (3, n[2], n[1], n[0])
    E, B, J = np.zeros(shp), np.zeros(shp), np.zeros(shp)
    z = np.arange(n[2])
    k = 2 * np.pi / n[2]
    E[1] = np.sin(k * z)[:, None, None]
    d = np.ones(3)
    a = oracle.ksb_rhs_f(b, E, B, J, d, kz=1.0)
    c = oracle.ksb_rhs_f(b, E, B, J, d, kz=2.5)
    diff = c - a
    assert np.abs(diff[:5]).max() == 0.0
    x = np.arange(n[0])
    v = -S_KEP * 0.01 * (x - 0.5 * n[0])                       # v at the E'z node x = i
    dEy_dz = k * np.cos(k * (z + 0.5))                          # at z + 1/2 (E'z)
    want = -v[None, None, :] * 1.5 * dEy_dz[:, None, None]
    want = np.broadcast_to(want, diff[5].shape)
    np.testing.assert_allclose(diff[5], want, rtol=0, atol=1.5 * np.abs(want).max() * k * k / 6)


def test_converged_step_solves_the_implicit_midpoint_equation():
    n = (12, 10, 6)
    E, B, J = _rand_fields(n, 513)
    step, adot, om, mask = 4, 3e-3, 0.012, 0b100
    b = _box(oracle.SHEAR_EXPAND, n, mask=mask, adot=adot, om=om, step=step, iters=400, tol=1e-14)
    E1, B1 = E.copy(), B.copy()
    oracle.maxwell(b, E1, B1, J)
    tn = step * DT
    th, t1 = tn + DT / 2, tn + DT
    l = lambda t: np.array([1 + adot * t if (mask >> c) & 1 else 1.0 for c in range(3)])
    sn, s1, lh = l(tn).prod() / l(tn), l(t1).prod() / l(t1), l(th)
    d = lh * lh / lh.prod()
    kz = (lh[1] / lh[2]) ** 2
    col = lambda a: a[:, None, None, None]
    Fn = (col(sn) * E, col(sn) * B)
    F1 = (col(s1) * E1, col(s1) * B1)
    dys = lambda t: oracle.shear_offset(b, t)
    r = 0.5 * (oracle.ksb_rhs_f(b, Fn[0], Fn[1], J, d, kz, dys(tn)) +
               oracle.ksb_rhs_f(b, F1[0], F1[1], J, d, kz, dys(t1)))
    lhs = np.concatenate([F1[1] - Fn[1], F1[0] - Fn[0]])
    np.testing.assert_allclose(lhs, DT * r, rtol=0, atol=1e-12)


def test_combined_frame_rejects_masks_that_separate_x_and_y():
    for mask in (0b001, 0b010, 0b101, 0b110):
        with pytest.raises(ValueError):
            oracle.make_box(3, (8, 8, 8), frame=oracle.SHEAR_EXPAND, axis_mask=mask)
