"""Pins of oracle parts that no other test fixes against the paper or the mathematics.

  * Delta y_s (Sec. 2.1): a field f(y + s Omega0 x t) solves the advection part of eq. OAB and
    obeys the shearing-periodic identity exactly when Delta y_s = s Omega0 L_x t.  Through the
    discrete right-hand side of eqs. OAB/OAE with the oracle's own Delta y_s(t), the columns
    next to the x faces (whose stencils read the shifted images) converge at first order with
    the same error as the interior; an offset of the wrong size or sign leaves an O(1) jump;
  * the staggered gather (Sec. 1, fields interpolated to the particles): each of the six Yee
    components set to its own multilinear function of its own staggered coordinates is
    reproduced at random points to roundoff; a wrong staggering offset shifts a value by its
    gradient;
  * the energy diagnostics (field energy E^2/8pi per component, kinetic energy m(gamma-1),
    momentum m u, live count; Sec. 2.3 and 3.3 observables): closed forms for uniform fields
    and momenta with rational Lorentz factors, escaped particles excluded;
  * the implicit-midpoint step of Sec. 2.2 at the shearing-periodic faces, s != 0 and a
    fractional Delta y_s: the converged step solves F^{n+1} = F^n + dt [L(F^n) + L(F^{n+1})]/2
    - 4 pi dt J' with the images of F^n at Delta y_s(t^n) and those of F^{n+1} at
    Delta y_s(t^{n+1}), whatever iterate the fixed point starts from, and its local error
    against an accurate integration of the semi-discrete equations with the time-dependent
    offset is third order in dt (images of F^{n+1} taken at t^n would make it second order).
"""
import numpy as np
import pytest

import oracle

STAG_E = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5]])
STAG_B = np.array([[0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


def grid_coords(box, st):
    nz, ny, nx = box.n[2], box.n[1], box.n[0]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i + st[0], j + st[1], k + st[2]


# ---------------------------------------------------------------- sheared waves
MODES = {  # amplitude, integer wave numbers (x, y, z), phase
    "Ex": (0.7, (1, 1, 1), 0.1), "Ey": (-0.4, (2, 1, -1), 0.7), "Ez": (0.5, (1, -2, 1), 1.3),
    "Bx": (0.3, (-1, 1, 2), 0.4), "By": (0.6, (1, 2, 1), 2.1), "Bz": (-0.8, (2, -1, 1), 0.9),
}


def sheared_wave(box, t):
    """F_c = a sin(kx x + ky (y + s Omega0 x t) + kz z + ph) on each component's own lattice, and
    its exact gradient; periodic in y and z, and F(x + L_x, y) = F(x, y + s Omega0 L_x t)."""
    nx, ny, nz = box.n
    sO = box.shear_s * box.omega0
    k0 = [2 * np.pi / nx, 2 * np.pi / ny, 2 * np.pi / nz if box.dim == 3 else 0.0]

    def val_grad(name, X, Y, Z):
        a, m, ph = MODES[name]
        kx, ky, kz = (m[d] * k0[d] for d in range(3))
        arg = kx * X + ky * (Y + sO * X * t) + kz * Z + ph
        c = a * np.cos(arg)
        return a * np.sin(arg), np.stack([(kx + ky * sO * t) * c, ky * c, kz * c])

    return val_grad


def exact_rhs(box, t):
    """eqs. OAB/OAE with J' = 0 at every component's own lattice points"""
    val_grad = sheared_wave(box, t)
    nx = box.n[0]
    sO = box.shear_s * box.omega0
    out = []
    for c in range(6):
        st = STAG_B[c] if c < 3 else STAG_E[c - 3]
        X, Y, Z = grid_coords(box, st)
        gE = [val_grad("E" + nm, X, Y, Z)[1] for nm in "xyz"]
        gB = [val_grad("B" + nm, X, Y, Z)[1] for nm in "xyz"]
        curlE = np.stack([gE[2][1] - gE[1][2], gE[0][2] - gE[2][0], gE[1][0] - gE[0][1]])
        curlB = np.stack([gB[2][1] - gB[1][2], gB[0][2] - gB[2][0], gB[1][0] - gB[0][1]])
        divE = gE[0][0] + gE[1][1] + gE[2][2]
        vs = np.stack([0 * X, -sO * (X - nx / 2), 0 * X])
        if c < 3:
            bx = val_grad("Bx", X, Y, Z)[0]
            out.append(-curlE[c] - vs[1] * gB[c][1] - (sO * bx if c == 1 else 0.0))
        else:
            cc = c - 3
            out.append(curlB[cc] - np.cross(vs, curlE, axis=0)[cc] - vs[cc] * divE)
    return out


def set_fields(box, t):
    val_grad = sheared_wave(box, t)
    E, B, J = oracle.zeros_fields(box)
    for c, nm in enumerate("xyz"):
        E[c][:] = val_grad("E" + nm, *grid_coords(box, STAG_E[c]))[0]
        B[c][:] = val_grad("B" + nm, *grid_coords(box, STAG_B[c]))[0]
    return E, B, J


def shear_box(dim, N, omega0, dt=0.45, **kw):
    n = (N, N, N) if dim == 3 else (N, N)
    return oracle.make_box(dim, n, dt=dt, frame=oracle.SHEAR, shear_s=1.5, omega0=omega0, **kw)


def rhs_errors(dim, N, tau, dys_fn=None):
    """(face, interior) max errors of the discrete RHS, relative to max |exact|, for a sheared
    wave at t = tau N on an N^dim box with Omega0 = 0.3/N (the same continuous problem at every
    N); dys_fn(box, t) overrides the offset handed to the RHS."""
    box = shear_box(dim, N, 0.3 / N)
    t = tau * N
    E, B, J = set_fields(box, t)
    dys = oracle.shear_offset(box, t) if dys_fn is None else dys_fn(box, t)
    got = oracle.ksb_rhs(box, E, B, J, dys=dys)
    ex = exact_rhs(box, t)
    face = np.zeros(box.n[0], bool)
    face[[0, 1, box.n[0] - 2, box.n[0] - 1]] = True  # columns whose stencils reach the images
    ef = max(np.abs(got[c] - ex[c])[..., face].max() for c in range(6))
    ei = max(np.abs(got[c] - ex[c])[..., ~face].max() for c in range(6))
    scale = max(np.abs(ex[c]).max() for c in range(6))
    return ef / scale, ei / scale, dys


@pytest.mark.parametrize("dim", [2, 3])
def test_shear_offset_pinned_by_sheared_wave_across_the_x_faces(dim):
    tau = 0.457  # Delta y_s = 0.45 tau N before the reduction mod n_y: fractional at N = 16, 32
    sizes = (16, 32) if dim == 3 else (32, 64)
    ef1, ei1, dys1 = rhs_errors(dim, sizes[0], tau)
    ef2, ei2, dys2 = rhs_errors(dim, sizes[1], tau)
    for d in (dys1, dys2):
        assert 0.05 < d % 1.0 < 0.95  # the images need the fractional interpolation
    # first order everywhere, faces included; the faces no worse than the interior
    assert max(ef1, ei1) / max(ef2, ei2) > 1.7
    assert ef1 < 3 * ei1 and ef2 < 3 * ei2
    # the pin fails on the plausible mistakes: an offset of half the size, the wrong sign, or
    # one taken from the radial coordinate of a face instead of the box length
    for wrong in (lambda b, t: 0.5 * oracle.shear_offset(b, t),
                  lambda b, t: (-oracle.shear_offset(b, t)) % b.n[1],
                  lambda b, t: (b.shear_s * b.omega0 * (b.n[0] / 2) * t) % b.n[1]):
        ef, ei, _ = rhs_errors(dim, sizes[1], tau, dys_fn=wrong)
        assert ef > 20 * ei, (ef, ei)


# ---------------------------------------------------------------- staggered gather
@pytest.mark.parametrize("dim", [2, 3])
def test_gather_reproduces_multilinear_fields_on_every_staggered_lattice(dim):
    rng = np.random.default_rng(4100 + dim)
    n = (9, 11, 10) if dim == 3 else (9, 11)
    box = oracle.make_box(dim, n, dt=0.45)
    E, B, J = oracle.zeros_fields(box)
    coef = rng.normal(size=(6, 5))

    def f(c, X, Y, Z):
        a = coef[c]
        return a[0] + a[1] * X + a[2] * Y + a[3] * Z * (dim == 3) + a[4] * X * Y

    for c in range(3):
        E[c][:] = f(c, *grid_coords(box, STAG_E[c]))
        B[c][:] = f(3 + c, *grid_coords(box, STAG_B[c]))
    # points whose stencils stay inside one period on every lattice (no wrap of the linear
    # functions): coordinates in [1, n - 2]
    m = 400
    x = rng.uniform(1, box.n[0] - 2, m)
    y = rng.uniform(1, box.n[1] - 2, m)
    z = rng.uniform(1, box.n[2] - 2, m) if dim == 3 else np.zeros(m)
    Eo, Bo = oracle.gather(box, E, B, x, y, z)
    for c in range(3):
        np.testing.assert_allclose(Eo[:, c], f(c, x, y, z), rtol=0, atol=1e-13)
        np.testing.assert_allclose(Bo[:, c], f(3 + c, x, y, z), rtol=0, atol=1e-13)
    # nodes carry their own values: a particle at a lattice point of B_y reads that value
    i, j, k = 4, 5, 3 if dim == 3 else 0
    X, Y, Z = i + STAG_B[1][0], j + STAG_B[1][1], (k + STAG_B[1][2]) if dim == 3 else 0.0
    _, Bo = oracle.gather(box, E, B, [X], [Y], [Z])
    assert abs(Bo[0, 1] - B[1][k, j, i]) < 1e-13


# ---------------------------------------------------------------- energies
def test_energies_closed_forms():
    box = oracle.make_box(3, (4, 5, 6), dt=0.45)
    E, B, J = oracle.zeros_fields(box)
    e, b = (0.1, -0.2, 0.3), (0.5, 0.25, -0.125)
    for c in range(3):
        E[c][:] = e[c]
        B[c][:] = b[c]
    ncell = 4 * 5 * 6
    # momenta with rational Lorentz factors: |u| = 3/4 -> gamma = 5/4, 4/3 -> 5/3, 12/5 -> 13/5
    u1 = np.array([[0.75, 0, 0], [0, 4 / 3, 0], [0, 0, 2.4], [0.45, 0.6, 0.0]])  # last: 3/4
    u2 = np.array([[0, -0.75, 0], [2.4 * 0.6, 0, -2.4 * 0.8], [0, 0, -4 / 3]])
    alive1 = np.array([1, 1, 1, 0], np.uint8)  # the last one escaped
    alive2 = np.array([1, 1, 1], np.uint8)
    sp = []
    for u, q, qm, alive in ((u1, -2e-3, -1.0, alive1), (u2, 3e-3, 0.5, alive2)):
        n = len(u)
        sp.append(oracle.SpeciesState(np.ones(n), np.ones(n), np.ones(n), u[:, 0], u[:, 1], u[:, 2],
                                      qm, q, alive=alive))
    out = oracle.energies(box, E, B, J, sp)
    for c in range(3):
        assert abs(out[c] - ncell * e[c] ** 2 / (8 * np.pi)) < 1e-15
        assert abs(out[3 + c] - ncell * b[c] ** 2 / (8 * np.pi)) < 1e-15
    m1, m2 = 2e-3, 6e-3  # |q / (q/m)|
    ke = m1 * (0.25 + 2 / 3 + 1.6) + m2 * (0.25 + 1.6 + 2 / 3)
    assert abs(out[6] - ke) < 1e-16
    mom = m1 * np.array([0.75, 4 / 3, 2.4]) + m2 * np.array([1.44, -0.75, -1.92 - 4 / 3])
    np.testing.assert_allclose(out[7:10], mom, rtol=0, atol=1e-16)
    assert out[10] == 6


# ---------------------------------------------------------------- implicit midpoint at the faces
def _F(E, B):
    return np.concatenate([B, E])  # (6, nz, ny, nx): Bx By Bz Ex Ey Ez as the RHS orders them


def _L(box, F, dys):
    """the linear part of the discrete RHS (J' = 0) with the images at offset dys"""
    J = np.zeros((3,) + F.shape[1:])
    return oracle.ksb_rhs(box, np.ascontiguousarray(F[3:]), np.ascontiguousarray(F[:3]), J, dys=dys)


def _converged_step(box, E, B):
    E1, B1, J = E.copy(), B.copy(), np.zeros_like(E)
    oracle.maxwell(box, E1, B1, J)
    return _F(E1, B1)


@pytest.mark.parametrize("dim", [2, 3])
def test_converged_ksb_step_solves_the_midpoint_equation_at_the_faces(dim):
    N = 12 if dim == 3 else 24
    box = shear_box(dim, N, 0.02, maxwell_iters=400, maxwell_tol=1e-15)
    box.step = 57
    dt = box.dt
    tn = box.step * dt
    d0, d1 = oracle.shear_offset(box, tn), oracle.shear_offset(box, tn + dt)
    assert 0.05 < d0 % 1 < 0.95 and 0.05 < d1 % 1 < 0.95
    E, B, _ = set_fields(box, tn)
    Fn = _F(E, B)
    F1 = _converged_step(box, E, B)
    assert box.last_iters < 400
    res = F1 - Fn - 0.5 * dt * (_L(box, Fn, d0) + _L(box, F1, d1))
    assert np.abs(res).max() < 1e-13 * np.abs(Fn).max()
    # the fixed point does not depend on the iterate it starts from: started from F^n with its
    # images at t^{n+1} instead of t^n it reaches the same fields
    Fk = Fn.copy()
    for _ in range(400):
        Fk_new = Fn + 0.5 * dt * (_L(box, Fn, d0) + _L(box, Fk, d1))
        done = np.abs(Fk_new - Fk).max() <= 1e-15 * np.abs(Fk_new).max()
        Fk = Fk_new
        if done:
            break
    np.testing.assert_allclose(Fk, F1, rtol=0, atol=1e-13 * np.abs(Fn).max())


def _rk4_reference(box, F0, t0, T, nsub):
    """the semi-discrete equations dF/dt = L(F; Delta y_s(t)) integrated by RK4"""
    h = T / nsub
    F, t = F0.copy(), t0
    for _ in range(nsub):
        k1 = _L(box, F, oracle.shear_offset(box, t))
        k2 = _L(box, F + 0.5 * h * k1, oracle.shear_offset(box, t + 0.5 * h))
        k3 = _L(box, F + 0.5 * h * k2, oracle.shear_offset(box, t + 0.5 * h))
        k4 = _L(box, F + h * k3, oracle.shear_offset(box, t + h))
        F = F + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        t += h
    return F


def test_converged_ksb_step_is_third_order_locally_with_moving_images():
    dim, N = 2, 16
    dt0, m = 0.45, 20
    errs, errs_wrong = [], []
    for dt in (dt0, dt0 / 2):
        box = shear_box(dim, N, 0.02, dt=dt, maxwell_iters=400, maxwell_tol=1e-15)
        box.step = int(round(m * dt0 / dt))  # the same t^n for both step sizes
        tn = box.step * dt
        d0, d1 = oracle.shear_offset(box, tn), oracle.shear_offset(box, tn + dt)
        # the images move by a fraction of a cell inside the step without crossing a lattice
        # line, so the semi-discrete equations are smooth in time there
        assert int(d0) == int(d1) and d1 > d0
        E, B, _ = set_fields(box, tn)
        Fn = _F(E, B)
        F1 = _converged_step(box, E, B)
        ref = _rk4_reference(box, Fn, tn, dt, 64)
        errs.append(np.abs(F1 - ref).max())
        # the other reading of the time levels, images of F^{n+1} at t^n: the same fixed point
        # with d0 for both members
        Fk = Fn.copy()
        for _ in range(400):
            Fk = Fn + 0.5 * dt * (_L(box, Fn, d0) + _L(box, Fk, d0))
        errs_wrong.append(np.abs(Fk - ref).max())
    assert errs[0] / errs[1] > 6.0, errs  # local error O(dt^3)
    assert errs_wrong[0] / errs_wrong[1] < 5.0, errs_wrong  # O(dt^2): told apart
    assert errs_wrong[0] > 3 * errs[0]
