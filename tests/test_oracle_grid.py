"""Pins of the oracle's grid operators: Maxwell solvers of the three frames, the shearing-box
current finalisation and the shearing-periodic boundary.

  * Yee leapfrog: a standing wave evolves as cos(n w dt) with
    sin^2(w dt/2) = dt^2 sum sin^2(k_d/2) (c = dx = 1), to roundoff;
  * shearing-box implicit midpoint with s = 0 (no shear): the Cayley rotation angle
    2 atan(dt K/2), K = 2 sqrt(sum sin^2(k_d/2)), once the fixed point has converged;
  * uniform fields in the shearing box: B_y(t) = B_y0 - s Omega0 B_x0 t exactly (eq. OAB);
  * the discrete right-hand side of eqs. OAB/OAE converges at first order to the continuous
    one evaluated in vector form (curl, v_s x curl E', v_s div E');
  * expanding box: uniform fields obey flux freezing B'=const, i.e. B_i = (l_i/l) B'_i;
  * the shearing-periodic identity F(x_i, y) = F(x_o, y - dys) (Sec. 2.1) for the field
    remap, the current fold as its exact transpose, and the J' transport of Sec. 2.2 moving
    the y centroid by v_{s,y} dt/2.
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


@pytest.mark.parametrize("dim", [2, 3])
def test_yee_standing_wave(dim):
    n = (16, 12, 10) if dim == 3 else (16, 12)
    box = oracle.make_box(dim, n, dt=0.45)
    E, B, J = oracle.zeros_fields(box)
    m = (3, 0, 2) if dim == 3 else (3, 2, 0)
    k = [2 * np.pi * m[d] / box.n[d] for d in range(3)]
    # dim 3: E_y(x, z) (div-free, independent of y); dim 2: E_z(x, y)
    c = 1 if dim == 3 else 2
    X, Y, Z = grid_coords(box, STAG_E[c])
    E0 = np.cos(k[0] * X + k[1] * Y + k[2] * Z)
    E[c][:] = E0
    nsteps = 57
    for _ in range(nsteps):
        oracle.maxwell(box, E, B, J)
        box.step += 1
    K2 = 4 * sum(np.sin(kk / 2) ** 2 for kk in k)
    w = 2 * np.arcsin(np.sqrt(box.dt**2 * K2 / 4)) / box.dt
    np.testing.assert_allclose(E[c], np.cos(nsteps * w * box.dt) * E0, atol=2e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_implicit_midpoint_standing_wave_no_shear(dim):
    n = (12, 10, 8) if dim == 3 else (16, 12)
    box = oracle.make_box(dim, n, dt=0.45, frame=oracle.SHEAR, shear_s=0.0, omega0=0.01,
                          maxwell_iters=400, maxwell_tol=1e-15)
    E, B, J = oracle.zeros_fields(box)
    m = (2, 0, 1) if dim == 3 else (2, 1, 0)
    k = [2 * np.pi * m[d] / box.n[d] for d in range(3)]
    c = 1 if dim == 3 else 2
    X, Y, Z = grid_coords(box, STAG_E[c])
    E0 = np.cos(k[0] * X + k[1] * Y + k[2] * Z)
    E[c][:] = E0
    nsteps = 20
    for _ in range(nsteps):
        oracle.maxwell(box, E, B, J)
        box.step += 1
    K = 2 * np.sqrt(sum(np.sin(kk / 2) ** 2 for kk in k))
    theta = 2 * np.arctan(box.dt * K / 2)
    np.testing.assert_allclose(E[c], np.cos(nsteps * theta) * E0, atol=1e-11)


@pytest.mark.parametrize("dim", [2, 3])
def test_shear_uniform_field_stretching(dim):
    n = (8, 8, 4) if dim == 3 else (8, 8)
    s, om = 1.5, 0.02
    box = oracle.make_box(dim, n, dt=0.45, frame=oracle.SHEAR, shear_s=s, omega0=om,
                          maxwell_iters=3)
    E, B, J = oracle.zeros_fields(box)
    B[0][:], B[1][:], B[2][:] = 0.03, -0.01, 0.2
    for _ in range(25):
        oracle.maxwell(box, E, B, J)
        box.step += 1
    t = 25 * box.dt
    np.testing.assert_allclose(B[1], -0.01 - s * om * 0.03 * t, rtol=1e-13)
    np.testing.assert_allclose(B[0], 0.03, rtol=1e-14)
    np.testing.assert_allclose(B[2], 0.2, rtol=1e-14)
    assert np.abs(E).max() < 1e-15


def analytic_fields(kx, ky, kz):
    """smooth periodic test fields and their exact gradients"""
    modes = {
        "Ex": (0.7, (kx, ky, kz), 0.1), "Ey": (-0.4, (2 * kx, ky, -kz), 0.7),
        "Ez": (0.5, (kx, -2 * ky, kz), 1.3), "Bx": (0.3, (-kx, ky, 2 * kz), 0.4),
        "By": (0.6, (kx, 2 * ky, kz), 2.1), "Bz": (-0.8, (2 * kx, -ky, kz), 0.9),
        "Jx": (0.02, (kx, ky, -kz), 0.3), "Jy": (-0.01, (kx, -ky, kz), 1.1),
        "Jz": (0.015, (-kx, ky, kz), 2.0),
    }

    def val(name, X, Y, Z):
        a, (qx, qy, qz), ph = modes[name]
        return a * np.sin(qx * X + qy * Y + qz * Z + ph)

    def grad(name, X, Y, Z):
        a, (qx, qy, qz), ph = modes[name]
        cc = a * np.cos(qx * X + qy * Y + qz * Z + ph)
        return np.stack([qx * cc, qy * cc, qz * cc])

    return val, grad


def ksb_rhs_error(dim, N):
    nx, ny, nz = (N, N, N) if dim == 3 else (N, N, 1)
    box = oracle.make_box(dim, (nx, ny, nz)[:dim], dt=0.45, frame=oracle.SHEAR, shear_s=1.5,
                          omega0=0.3 / N)
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    kz = 2 * np.pi / nz if dim == 3 else 0.0
    val, grad = analytic_fields(kx, ky, kz)
    E, B, J = oracle.zeros_fields(box)
    for c, nm in enumerate("xyz"):
        E[c][:] = val("E" + nm, *grid_coords(box, STAG_E[c]))
        B[c][:] = val("B" + nm, *grid_coords(box, STAG_B[c]))
        J[c][:] = val("J" + nm, *grid_coords(box, STAG_E[c]))
    out = oracle.ksb_rhs(box, E, B, J, dys=0.0)
    sO = box.shear_s * box.omega0
    errs, scale = [], 0.0
    for c in range(6):
        st = STAG_B[c] if c < 3 else STAG_E[c - 3]
        X, Y, Z = grid_coords(box, st)
        gE = [grad("E" + nm, X, Y, Z) for nm in "xyz"]
        gB = [grad("B" + nm, X, Y, Z) for nm in "xyz"]
        if dim == 2:
            for g in gE + gB:
                g[2] = 0.0
        curlE = np.stack([gE[2][1] - gE[1][2], gE[0][2] - gE[2][0], gE[1][0] - gE[0][1]])
        curlB = np.stack([gB[2][1] - gB[1][2], gB[0][2] - gB[2][0], gB[1][0] - gB[0][1]])
        divE = gE[0][0] + gE[1][1] + gE[2][2]
        vs = np.stack([0 * X, -sO * (X - nx / 2), 0 * X])
        if c < 3:
            Bv = [val("B" + nm, X, Y, Z) for nm in "xyz"]
            adv = vs[1] * gB[c][1]  # (v_s . grad) B_c
            exact = -curlE[c] - adv - (sO * Bv[0] if c == 1 else 0.0)
        else:
            cc = c - 3
            vxc = np.cross(vs, curlE, axis=0)
            Jv = val("J" + "xyz"[cc], X, Y, Z)
            exact = curlB[cc] - 4 * np.pi * Jv - vxc[cc] - vs[cc] * divE
        d = out[c] - exact
        # stay away from the x faces, where v_s jumps by s Omega0 Lx between images
        interior = (X > 2) & (X < nx - 2)
        errs.append(np.abs(d[interior]).max())
        scale = max(scale, np.abs(exact).max())
    return np.array(errs) / scale


@pytest.mark.parametrize("dim", [2, 3])
def test_ksb_rhs_consistent_with_eqs_OAB_OAE(dim):
    sizes = (16, 32) if dim == 3 else (32, 64)
    e1 = ksb_rhs_error(dim, sizes[0])
    e2 = ksb_rhs_error(dim, sizes[1])
    assert e2.max() < 0.08
    assert np.all(e1 / e2 > 1.7)  # at least first-order convergence of every component


def test_keb_flux_freezing_uniform_fields():
    adot, dt = 4e-3, 0.45
    box = oracle.make_box(3, (6, 6, 6), dt=dt, frame=oracle.EXPAND, adot=adot, axis_mask=0b011)
    E, B, J = oracle.zeros_fields(box)
    B[0][:], B[2][:] = 0.05, 0.3
    E[0][:], E[2][:] = 0.01, -0.02
    for _ in range(30):
        oracle.maxwell(box, E, B, J)
        box.step += 1
    a = 1 + adot * 30 * dt
    # B' = l L^-1 B is constant: l = a^2, L = diag(a, a, 1)
    np.testing.assert_allclose(B[2], 0.3 / a**2, rtol=1e-13)
    np.testing.assert_allclose(B[0], 0.05 / a, rtol=1e-13)
    np.testing.assert_allclose(E[0], 0.01 / a, rtol=1e-13)
    np.testing.assert_allclose(E[2], -0.02 / a**2, rtol=1e-13)


def test_shearing_periodic_field_identity():
    """Interpolating at the x guards reproduces F(x_i, y) = F(x_o, y - dys) for a field that is
    linear in y, for which linear interpolation is exact."""
    box = oracle.make_box(2, (8, 10), dt=0.45, frame=oracle.SHEAR, shear_s=1.5, omega0=0.01)
    E, B, J = oracle.zeros_fields(box)
    # Ez at nodes: linear in y inside one period, read far from the wrap of y
    X, Y, Z = grid_coords(box, STAG_E[2])
    E[2][:] = 0.1 * Y + 0.01 * X
    dys = 2.37
    # the gather of Ez at a point just beyond x_o (x = 8.0 exactly, the node of column 8)
    Eo, _ = oracle.gather(box, E, B, [8.0], [3.0], dys=dys)
    # column 8 is column 0 at y + dys
    assert abs(Eo[0, 2] - (0.1 * (3.0 + dys) + 0.0)) < 1e-14
    # below x_i: column -1 is column nx-1 at y - dys
    Eo, _ = oracle.gather(box, E, B, [-1.0], [6.0], dys=dys)
    assert abs(Eo[0, 2] - (0.1 * (6.0 - dys) + 0.01 * 7)) < 1e-14


def test_current_fold_is_transpose_of_field_remap():
    rng = np.random.default_rng(70)
    box = oracle.make_box(2, (8, 10), dt=0.45, frame=oracle.SHEAR, shear_s=1.5, omega0=0.01)
    nx, ny, G = 8, 10, oracle.JG
    t_half = 37.3
    dys = oracle.shear_offset(box, t_half)
    assert 0 < dys < ny and abs(dys - round(dys)) > 0.05
    Jext = rng.normal(size=oracle.jext_shape(box))
    F = rng.normal(size=oracle.field_shape(box))
    J = oracle.finalize_current(box, Jext, t_half)
    lhs = (J * F).sum()
    # the same pairing computed on the extended grid: extend F by the boundary condition
    # (guard column i >= nx is column i - nx at y + dys; i < 0 is column i + nx at y - dys),
    # then apply the transpose of the J' transport (a shift by -d along y)
    ext = np.zeros_like(Jext)
    y = np.arange(ny)
    for c in range(3):
        for ie in range(nx + 2 * G):
            i = ie - G
            if 0 <= i < nx:
                col = F[c][0, :, i]
            else:
                ii, sh = (i - nx, dys) if i >= nx else (i + nx, -dys)
                col = np.interp(np.mod(y + sh, ny), np.arange(ny + 1),
                                np.append(F[c][0, :, ii], F[c][0, 0, ii]))
            xc = i + STAG_E[c][0] - nx / 2
            d = -box.shear_s * box.omega0 * xc * box.dt / 2
            ext[c][0, :, ie] = np.interp(np.mod(y + d, ny), np.arange(ny + 1), np.append(col, col[0]))
    rhs = (Jext * ext).sum()
    assert abs(lhs - rhs) < 1e-12 * abs(Jext).sum()
    np.testing.assert_allclose(J.sum(axis=(1, 2, 3)), Jext.sum(axis=(1, 2, 3)), rtol=1e-13)


def test_current_transport_moves_centroid_by_half_step_shear():
    box = oracle.make_box(2, (16, 32), dt=0.45, frame=oracle.SHEAR, shear_s=1.5, omega0=0.2)
    Jext = np.zeros(oracle.jext_shape(box))
    G = oracle.JG
    cols = [1, 5, 12]
    for i in cols:
        for c in range(3):
            Jext[c][0, 16, i + G] = 1.0
    J = oracle.finalize_current(box, Jext, 0.0)
    y = np.arange(32)
    for i in cols:
        for c in range(3):
            xc = i + STAG_E[c][0] - 8
            d = -1.5 * 0.2 * xc * 0.45 / 2  # v_{s,y} dt/2 at the component's x
            cen = (J[c][0, :, i] * y).sum() / J[c][0, :, i].sum()
            assert abs(cen - (16 + d)) < 1e-12
