"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Sizes span several tiles with ragged tails (3D 20x12x16 on 8^3 tiles, 2D 40x36 on 16^2 tiles).
Bars: integer work bit-exact (sort permutation and offsets, escape masks, survivor counts);
single-step push 2e-6 relative (|du| / max(|u|, 0.01)); positions 2e-6 cells; deposited J
1e-5 of max|J|; continuity residual 1e-6 of the gross charge density; fields after the Maxwell
step 1e-5 of their maximum; 200- and 1000-step energy histories within 1%.
"""
import numpy as np
import pytest
import torch

import oracle
from _cases import Case, cell_coords, compare_particles, positions_f64, random_fields
from paper_2602_15939_amd import _lib as L

pytestmark = pytest.mark.gpu

SIZE = {2: (40, 36), 3: (20, 12, 16)}
TILE = {2: (16, 16, 1), 3: (8, 8, 8)}


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("dim", [2, 3])
def test_tile_sort_bit_exact(dim):
    c = Case(dim, SIZE[dim], "plain", ppc=5, seed=11)
    try:
        c.gpu.sort()
        for s in range(2):
            perm, off = c.gpu.get_sort(s)
            i, j, k = cell_coords(c.parts[s]["cell"], c.n)
            keys = oracle.tile_keys(c.box, TILE[dim], i, j, k if dim == 3 else None)
            nt = len(off) - 1
            ref, roff = oracle.stable_sort(keys, nt)
            np.testing.assert_array_equal(perm.cpu().numpy(), ref)
            np.testing.assert_array_equal(off.cpu().numpy(), roff[: nt + 1])
    finally:
        c.close()


FRAME_CASES = [(d, f) for f in ("plain", "shear", "expand", "leaky") for d in (2, 3)]


@pytest.mark.parametrize("mem", ["caller", "library"])
@pytest.mark.parametrize("dim,frame", FRAME_CASES)
def test_one_step_parity(dim, frame, mem):
    """One whole step against the oracle, for a box on torch memory (pic_box_mem) and for a box
    on memory the library allocates."""
    c = Case(dim, SIZE[dim], frame, ppc=4, seed=20 + dim, mem=mem)
    try:
        c.gpu.step()
        c.oracle_step()
        for s in range(2):
            st = compare_particles(c, s, c.gpu_species(s))
            assert st["n"] == len(c.parts[s]["cell"])
            assert st["err_u"] < 2e-6, st["err_u"]
            assert st["err_x"] < 2e-6, st["err_x"]
        J = c.gpu.get_current().cpu().numpy()
        assert rel(J, c.J) < 1e-5
        E, B = (t.cpu().numpy() for t in c.gpu.get_fields())
        assert rel(E, c.E) < 1e-5 and rel(B, c.B) < 1e-5
        info = c.gpu.info()
        assert info.errors & ~L.DERR_ORDER == 0 and info.n_slow == 0
    finally:
        c.close()


def div_J(J, dim):
    d = J[0] - np.roll(J[0], 1, axis=2) + J[1] - np.roll(J[1], 1, axis=1)
    if dim == 3:
        d = d + J[2] - np.roll(J[2], 1, axis=0)
    return d


@pytest.mark.parametrize("dim", [2, 3])
def test_continuity(dim):
    """rho^{n+1} - rho^n + dt div J = 0 with rho from the GPU's own old and new positions."""
    c = Case(dim, SIZE[dim], "plain", ppc=6, seed=30 + dim)
    try:
        c.gpu.sort()
        c.gpu.push(fuse=True)
        c.gpu.remap(L.REMAP_CURRENT)
        J = c.gpu.get_current().cpu().numpy().astype(np.float64)
        rho0 = np.zeros(J.shape[1:])
        rho1 = np.zeros(J.shape[1:])
        gross = np.zeros(J.shape[1:])
        for s in range(2):
            q = c.qms[s] * c.q
            p = c.parts[s]
            x, y, z = positions_f64(p["cell"], p["off"], c.n, dim)
            oracle.charge(c.box, q, x, y, z if dim == 3 else None, rho0)
            oracle.charge(c.box, abs(q), x, y, z if dim == 3 else None, gross)
            g = c.gpu_species(s)
            x, y, z = positions_f64(g["cell"], g["off"], c.n, dim)
            oracle.charge(c.box, q, x, y, z if dim == 3 else None, rho1)
        res = rho1 - rho0 + c.box.dt * div_J(J, dim)
        assert np.abs(res).max() <= 1e-6 * gross.max()
        assert np.abs(J).max() > 0
    finally:
        c.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_unfused_deposit_matches_fused(dim):
    a = Case(dim, SIZE[dim], "shear", ppc=4, seed=40 + dim)
    b = Case(dim, SIZE[dim], "shear", ppc=4, seed=40 + dim)
    try:
        a.gpu.sort()
        a.gpu.push(fuse=True)
        b.gpu.sort()
        b.gpu.push(fuse=False)
        b.gpu.deposit()
        for s in range(2):
            ga, gb = a.gpu_species(s), b.gpu_species(s)
            for k in ("cell", "off", "u", "id"):
                np.testing.assert_array_equal(ga[k], gb[k])
        Ja = a.gpu.get_current().cpu().numpy()
        Jb = b.gpu.get_current().cpu().numpy()
        assert rel(Ja, Jb) < 1e-6
    finally:
        a.close()
        b.close()


def frozen_parts(n, gamma_hot, gamma_cold, seed, dims):
    rng = np.random.default_rng(seed)
    out = []
    for g in (gamma_hot, gamma_cold):
        um = np.sqrt(g * g - 1)
        v = rng.normal(size=(n, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        cell = rng.integers(0, int(np.prod(dims)), n).astype(np.int32)
        off = rng.uniform(0, 1, (len(dims), n)).astype(np.float32)
        out.append(dict(cell=torch.from_numpy(cell), off=torch.from_numpy(off),
                        u=torch.from_numpy((um * v.T).astype(np.float32))))
    return out


def test_probabilistic_escape_masks_bit_exact():
    """E = B = 0, test particles: the push leaves u bit-unchanged, so the gamma test sees identical
    inputs; the escape masks (from the same Philox counters) and survivor counts must agree
    exactly at every step."""
    dims = (32, 32)
    dt = 0.45
    zero = (np.zeros((3, 1, 32, 32), np.float32), np.zeros((3, 1, 32, 32), np.float32))
    parts = frozen_parts(6000, 20.0, 5.0, 50, dims)
    c = Case(2, dims, "leaky", parts=parts, fields=zero, q=0.0,
             leaky_mode=L.LEAKY_PROBABILISTIC, t_esc=dt / 0.1, gamma_thr=10.0)
    try:
        for step in range(6):
            c.gpu.escape_compact()  # compaction (sort with the dead bin)
            c.gpu.push(fuse=True)
            c.gpu.remap(L.REMAP_CURRENT)
            c.gpu.maxwell()
            c.oracle_step()
            for s in range(2):
                g = c.gpu_species(s)
                dead_gpu = set(int(v) for v in g["id"][g["cell"] < 0])
                o = c.sp[s]
                newly = set(int(v) for v in o.id[o.alive == 0]) - getattr(c, f"_dead{s}", set())
                assert dead_gpu == newly, f"step {step} species {s}"
                setattr(c, f"_dead{s}", set(int(v) for v in o.id[o.alive == 0]))
        c.gpu.escape_compact()
        info = c.gpu.info()
        for s in range(2):
            assert info.n_particles[s] == int(c.sp[s].alive.sum())
        assert info.n_particles[1] == 6000
        assert info.n_particles[0] < 6000
        # the escape counter (summed per wave on the GPU) equals the oracle's escapes
        assert info.n_escaped == sum(int((c.sp[s].alive == 0).sum()) for s in range(2))
    finally:
        c.close()


@pytest.mark.parametrize("dim,use_3vec", [(2, 0), (3, 0), (3, 1)])
def test_displacement_escape_and_reinjection(dim, use_3vec):
    """Sec. 4.1: escape when the in-plane displacement (or, with use_3vec, the 3-vector
    displacement) reaches l_esc; the particle keeps its position and gets a Maxwell-Juttner
    momentum from its Philox words."""
    dims = (32, 32) if dim == 2 else (12, 12, 12)
    shape = (3, 1, 32, 32) if dim == 2 else (3, 12, 12, 12)
    zero = (np.zeros(shape, np.float32), np.zeros(shape, np.float32))
    parts = frozen_parts(4000, 1.3, 1.05, 60 + dim + use_3vec, dims)
    c = Case(dim, dims, "leaky", parts=parts, fields=zero, q=0.0,
             leaky_mode=L.LEAKY_DISPLACEMENT, l_esc=1.5, theta_inj=0.3, use_3vec=use_3vec)
    ncomp = 3 if use_3vec else 2
    try:
        nesc = 0
        for step in range(10):
            c.gpu.step()
            c.oracle_step()
            for s in range(2):
                g = c.gpu_species(s)
                st = compare_particles(c, s, g)
                o = c.sp[s]
                dr_o = o.dr[:, st["sel"]]
                # escape decisions are FP32 on the GPU and FP64 in the oracle: only a particle
                # within rounding of l_esc may differ, and none should here
                assert np.abs(g["dr"][:ncomp] - dr_o[:ncomp]).max() < 1e-5
                # re-drawn momenta (FP32 table interpolation and sincos, measured 4e-7) within
                # the push bar
                assert st["err_u"] < 2e-6, (step, s, st["err_u"])
                nesc += int((dr_o[0] == 0).sum())
        assert nesc > 100
    finally:
        c.close()


def test_displacement_drift_over_1000_steps():
    """The tracked displacement of Sec. 4.1 accumulates in FP32: over n steps its distance from
    the FP64 sum is bounded by the rounding of the n additions, n 2^-24 max|dr|, plus the FP32
    error of the increments (~1e-7 cells each).  Frozen fields (straight lines), l_esc beyond
    reach; measured 4.8e-3 cells at |dr| = 351 after 1000 steps (bound 2.1e-2), i.e. escape
    decisions at l_esc ~ 10^3 can differ from FP64 for particles within ~1e-2 cells of l_esc."""
    dims = (32, 32)
    zero = (np.zeros((3, 1, 32, 32), np.float32),) * 2
    parts = frozen_parts(4000, 1.6, 1.2, 77, dims)
    c = Case(2, dims, "leaky", parts=parts, fields=zero, q=0.0, leaky_mode=L.LEAKY_DISPLACEMENT,
             l_esc=1024.0, theta_inj=0.3)
    try:
        nsteps = 1000
        for _ in range(nsteps):
            c.gpu.step()
            c.oracle_step(nthreads=8)
        err = big = 0.0
        for s in range(2):
            g = c.gpu_species(s)
            st = compare_particles(c, s, g)
            o = c.sp[s]
            err = max(err, float(np.abs(g["dr"][:2, st["live"]] - o.dr[:2, st["sel"]]).max()))
            big = max(big, float(np.abs(o.dr[:2]).max()))
        assert big > 300
        assert err <= nsteps * (2.0 ** -24 * big + 1e-7), err
    finally:
        c.close()


def test_energy_history_config0_200_steps():
    """The 2D shearing box of the parity configuration (64x64, 16 ppc per species, theta 0.1,
    skin depth 4 cells, sigma 0.1, q = 1.5, Omega0 = 0.1 omega_c): field and kinetic energy
    histories within 1% over 200 steps."""
    from paper_2602_15939_amd import synth
    dims = (64, 64)
    ppc = 16
    wp, q, B0 = synth.plasma_params(ppc, 4.0, 0.1)
    E, B = synth.uniform_field(dims, 2, B0)
    fields = (E.astype(np.float32), B.astype(np.float32))
    c = Case(2, dims, "shear", ppc=ppc, theta=0.1, seed=2026, fields=fields, q=q,
             shear_s=1.5, omega0=0.1 * B0, maxwell_iters=8)
    try:
        hist_g, hist_o = [], []
        for step in range(200):
            c.gpu.step()
            c.oracle_step(nthreads=8)
            if (step + 1) % 20 == 0:
                info = c.gpu.info()
                eg = sum(info.field_energy_B) + sum(info.field_energy_E)
                eo = oracle.energies(c.box, c.E, c.B, c.J, c.sp)
                hist_g.append((eg, info.kinetic_energy))
                hist_o.append((eo[0:6].sum(), eo[6]))
        hg, ho = np.array(hist_g), np.array(hist_o)
        assert np.all(np.abs(hg - ho) <= 0.01 * np.abs(ho)), (hg, ho)
    finally:
        c.close()


@pytest.mark.parametrize("dim,frame", [(2, "shear"), (2, "expand"), (2, "leaky"), (3, "shear"),
                                       (2, "shear_expand")])
def test_energy_history_1000_steps(dim, frame):
    """Field and kinetic energy histories within 1% of the FP64 oracle over 1000 steps, sampled
    every 50 steps, at the size of the parity configuration (64x64 cells, 16 ppc per species;
    3D: 16^3 cells, 8 ppc per species; theta 0.1, skin depth 4 cells, sigma 0.1, B0 along z):
    the shearing box (q = 1.5, Omega0 = 0.1 omega_c), the expanding box (x and y, perpendicular
    to B0, grow as a = 1 + adot t with adot = 1e-3 omega_p) and the leaky box in the paper's
    displacement mode (escape at |dr| = L/2, Maxwell-Juttner reinjection at the plasma
    temperature: every particle crosses that distance many times in 1000 steps), and the
    combined frame (the shearing box's parameters with x and y expanding as above).  The magnetic
    energy per component (the observable of the shearing-box application, Sec. 2.3) within 1%
    of the total magnetic energy.  Live particle counts equal."""
    import os

    from paper_2602_15939_amd import synth
    dims = (64, 64) if dim == 2 else (16, 16, 16)
    ppc = 16 if dim == 2 else 8
    wp, q, B0 = synth.plasma_params(ppc, 4.0, 0.1)
    E, B = synth.uniform_field(dims, 2, B0)  # B0 along z
    fields = (E.astype(np.float32), B.astype(np.float32))
    kw = dict(shear=dict(shear_s=1.5, omega0=0.1 * B0, maxwell_iters=8),
              expand=dict(adot=1e-3 * wp, axis_mask=0b011),
              leaky=dict(leaky_mode=L.LEAKY_DISPLACEMENT, l_esc=32.0, theta_inj=0.1),
              shear_expand=dict(shear_s=1.5, omega0=0.1 * B0, maxwell_iters=8, adot=1e-3 * wp,
                                axis_mask=0b011))[frame]
    c = Case(dim, dims, frame, ppc=ppc, theta=0.1, seed=4051, fields=fields, q=q, **kw)
    nthreads = min(16, len(os.sched_getaffinity(0)))
    try:
        hist_g, hist_o, bc_g, bc_o = [], [], [], []
        for step in range(1000):
            c.gpu.step()
            c.oracle_step(nthreads=nthreads)
            if (step + 1) % 50 == 0:
                info = c.gpu.info()
                assert info.errors & ~L.DERR_ORDER == 0, info.errors
                eg = sum(info.field_energy_B) + sum(info.field_energy_E)
                eo = oracle.energies(c.box, c.E, c.B, c.J, c.sp)
                hist_g.append((eg, info.kinetic_energy))
                hist_o.append((eo[0:6].sum(), eo[6]))
                bc_g.append(list(info.field_energy_B))
                bc_o.append(list(eo[3:6]))
                assert int(info.n_particles[0] + info.n_particles[1]) == int(eo[10])
        hg, ho = np.array(hist_g), np.array(hist_o)
        assert np.all(np.abs(hg - ho) <= 0.01 * np.abs(ho)), (frame, np.abs(hg - ho) / np.abs(ho))
        bg, bo = np.array(bc_g), np.array(bc_o)
        tot = bo.sum(axis=1, keepdims=True)
        assert np.all(np.abs(bg - bo) <= 0.01 * tot), (frame, np.abs(bg - bo) / tot)
    finally:
        c.close()
