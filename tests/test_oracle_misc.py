"""Pins of the oracle's integer and sampling layers and of the leaky-box and shearing-box
particle boundaries.

  * Philox4x32-10 against rocRAND's independent implementation (host build of its header);
  * the Maxwell-Juttner inverse-CDF table against the CDF integrated by quadrature and the
    closed-form mean <gamma> = K1(1/theta)/K2(1/theta) + 3 theta;
  * the stable counting sort against numpy.argsort(kind="stable");
  * FP32 offset renormalisation: offsets in [0,1), exact in the s >= 1 branch, position kept;
  * probabilistic escape: survivors of a frozen gamma > gamma_thr population within 5 sigma of
    Binomial(N, (1-p)^n); particles below the threshold never escape;
  * displacement escape (Sec. 4.1, eq. escape): a free particle escapes at the first step
    where |Delta x| >= l_esc, is resampled and its displacement reset;
  * shearing-periodic particle mapping consistent with the field identity of Sec. 2.1.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import special
from scipy.integrate import quad

import oracle

ROCRAND_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Eng : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Eng e;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.run(make_uint4(c0, c1, c2, c3), make_uint2(k0, k1));
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc (rocRAND headers) not available")
def test_philox_matches_rocrand(tmp_path):
    src = tmp_path / "kat.cpp"
    src.write_text(ROCRAND_PROG)
    exe = tmp_path / "kat"
    subprocess.check_call(["hipcc", "-O1", "--offload-arch=gfx950", "-o", str(exe), str(src)],
                          stderr=subprocess.DEVNULL)
    rng = np.random.default_rng(80)
    ctr = rng.integers(0, 2**32, (300, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, (300, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0], key[0] = 0, 0
    ctr[1], key[1] = 0xFFFFFFFF, 0xFFFFFFFF
    inp = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctr, key))
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                   dtype=np.uint64).astype(np.uint32)
    got = oracle.philox(ctr, key)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("theta", [0.05, 0.3, 1.0])
def test_mj_table_quantiles(theta):
    tab = oracle.mj_table(theta)
    nb, nt = oracle.MJ_BINS, oracle.MJ_TAIL
    dens = lambda u: u * u * np.exp(-(np.sqrt(1 + u * u) - 1) / theta)
    Z = quad(dens, 0, np.inf, epsabs=0, epsrel=1e-13, limit=400)[0]
    for i in (1, 7, 512, 2048, 3500, 4000, 4095):
        F = quad(dens, 0, tab[i], epsabs=0, epsrel=1e-13, limit=400)[0] / Z
        assert abs(F - i / nb) < 1e-9
    for k in (1, 20, 63, 64):  # tail: 1 - F = 2^-(12 + 20 k/64)
        tail = quad(dens, tab[nb - 1 + k], np.inf, epsabs=0, epsrel=1e-12, limit=400)[0] / Z
        assert abs(np.log2(tail) + 12 + 20 * k / nt) < 1e-6
    assert tab[0] == 0.0 and np.all(np.diff(tab) > 0)


@pytest.mark.parametrize("theta", [0.1, 0.3])
def test_mj_sampler_mean_gamma_closed_form(theta):
    """<gamma> over quantile-stratified table samples matches K1(1/theta)/K2(1/theta) + 3 theta,
    and the bulk bins (all but the top one) the conditional mean from quadrature."""
    nb = oracle.MJ_BINS
    tab = oracle.mj_table(theta)
    M = 1 << 16
    w0 = ((np.arange(M, dtype=np.uint64) << 16) + (1 << 15)).astype(np.uint32)
    words = np.zeros((M, 4), dtype=np.uint32)
    words[:, 0] = w0
    words[:, 1] = 0x80000000
    u = oracle.mj_sample(tab, words)
    g = np.sqrt(1 + (u * u).sum(1))
    exact = special.kv(1, 1 / theta) / special.kv(2, 1 / theta) + 3 * theta
    assert abs(g.mean() - exact) < 1e-5 * exact
    bulk = (w0 >> 20) < nb - 1
    dens = lambda v: v * v * np.exp(-(np.sqrt(1 + v * v) - 1) / theta)
    Z = quad(dens, 0, np.inf, epsabs=0, epsrel=1e-13, limit=400)[0]
    num = quad(lambda v: np.sqrt(1 + v * v) * dens(v), 0, tab[nb - 1], epsabs=0, epsrel=1e-13,
               limit=400)[0]
    cond = num / Z / (1 - 1 / nb)
    assert abs(g[bulk].mean() - cond) < 1e-5 * cond


def test_mj_sampler_isotropy():
    tab = oracle.mj_table(0.3)
    rng = np.random.default_rng(81)
    words = rng.integers(0, 2**32, (20000, 4), dtype=np.uint64).astype(np.uint32)
    u = oracle.mj_sample(tab, words)
    m2 = (u * u).sum(1).mean()
    for c in range(3):
        assert abs(u[:, c].mean()) < 5 * np.sqrt(m2 / 3 / len(u))
        assert abs((u[:, c] ** 2).mean() - m2 / 3) < 0.05 * m2 / 3


def test_stable_sort_matches_numpy():
    rng = np.random.default_rng(82)
    nkeys = 37
    keys = rng.integers(0, nkeys + 1, 5000).astype(np.int32)  # includes the dead bin
    perm, off = oracle.stable_sort(keys, nkeys)
    live = np.nonzero(keys < nkeys)[0]
    ref = live[np.argsort(keys[live], kind="stable")]
    np.testing.assert_array_equal(perm, ref)
    np.testing.assert_array_equal(np.diff(off)[:nkeys], np.bincount(keys, minlength=nkeys + 1)[:nkeys])
    assert off[nkeys + 1] == len(keys)


def test_tile_keys():
    box = oracle.make_box(3, (10, 7, 9))
    rng = np.random.default_rng(83)
    ci, cj, ck = rng.integers(0, 10, 500), rng.integers(0, 7, 500), rng.integers(0, 9, 500)
    ci[:5] = -1
    keys = oracle.tile_keys(box, (4, 4, 4), ci, cj, ck)
    ntx, nty, ntz = 3, 2, 3
    for p in range(500):
        if ci[p] < 0:
            assert keys[p] == ntx * nty * ntz
        else:
            assert keys[p] == ci[p] // 4 + ntx * (cj[p] // 4 + nty * (ck[p] // 4))


def test_f32_normalize_properties():
    rng = np.random.default_rng(84)
    n = 200000
    cell = rng.integers(0, 1000, n).astype(np.int32)
    off = rng.uniform(0, 1, n).astype(np.float32)
    off[:1000] = np.float32(0.0)
    off[1000:2000] = np.nextafter(np.float32(1), np.float32(0))
    delta = rng.uniform(-0.99, 0.99, n).astype(np.float32)
    delta[2000:3000] = -np.float32(1e-12)
    co, oo = oracle.f32_normalize(cell, off, delta)
    assert np.all(oo >= 0) and np.all(oo < 1)
    s = (off + delta).astype(np.float32)
    up = s >= 1
    np.testing.assert_array_equal(oo[up], (s[up].astype(np.float64) - 1).astype(np.float32))
    exact = cell.astype(np.float64) + off.astype(np.float64) + delta.astype(np.float64)
    assert np.abs(co + oo.astype(np.float64) - exact).max() < 2 ** -23
    assert np.all(np.abs(co - cell) <= 1)


def frozen_population(n, gamma, rng):
    um = np.sqrt(gamma**2 - 1)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    return um * v


def test_probabilistic_escape_statistics():
    rng = np.random.default_rng(85)
    dt, p = 0.45, 0.05
    box = oracle.make_box(2, (16, 16), dt=dt, frame=oracle.LEAKY,
                          leaky_mode=oracle.LEAKY_PROBABILISTIC, t_esc=dt / p, gamma_thr=10.0,
                          seed=0x1234ABCD5678, box_id=3)
    E, B, J = oracle.zeros_fields(box)
    N = 4000
    u_hot = frozen_population(N, 20.0, rng)
    u_cold = frozen_population(N, 5.0, rng)
    x, y = rng.uniform(0, 16, N), rng.uniform(0, 16, N)
    hot = oracle.SpeciesState(x, y, None, *u_hot.T, 1.0, 0.0)
    cold = oracle.SpeciesState(x, y, None, *u_cold.T, 1.0, 0.0, ids=np.arange(N, 2 * N))
    nsteps = 40
    for _ in range(nsteps):
        oracle.step(box, E, B, J, [hot, cold])
    surv = hot.alive.sum()
    mean = N * (1 - p) ** nsteps
    sd = np.sqrt(N * (1 - p) ** nsteps * (1 - (1 - p) ** nsteps))
    assert abs(surv - mean) < 5 * sd
    assert cold.alive.all()
    np.testing.assert_array_equal(hot.ux[hot.alive == 1], u_hot[hot.alive == 1, 0])


def test_displacement_escape_free_particle():
    dt, lesc = 0.45, 10.0
    tab = oracle.mj_table(0.3)
    box = oracle.make_box(2, (32, 32), dt=dt, frame=oracle.LEAKY,
                          leaky_mode=oracle.LEAKY_DISPLACEMENT, l_esc=lesc, seed=77, box_id=5,
                          mj_table=tab)
    E, B, J = oracle.zeros_fields(box)
    ux = 1 / np.sqrt(3)  # v_x = 0.5
    sp = oracle.SpeciesState([3.0], [5.0], None, [ux], [0.0], [0.0], 1.0, 0.0, ids=[42])
    vx = ux / np.sqrt(1 + ux * ux)
    n_esc = int(np.ceil(lesc / (vx * dt) - 1e-12))  # first n with n v dt >= l_esc
    for n in range(1, n_esc):
        oracle.step(box, E, B, J, [sp])
        assert abs(sp.dr[0, 0] - n * vx * dt) < 1e-12
        assert sp.ux[0] == ux
    oracle.step(box, E, B, J, [sp])
    assert sp.dr[0, 0] == 0.0 and sp.dr[1, 0] == 0.0
    w = oracle.philox([[42, n_esc - 1, 1, 5]], [77 & 0xFFFFFFFF, 77 >> 32])
    np.testing.assert_allclose([sp.ux[0], sp.uy[0], sp.uz[0]], oracle.mj_sample(tab, w)[0],
                               rtol=1e-15)


def test_shear_particle_crossing_matches_field_image():
    """A particle just beyond x_o is the image of one at x_i shifted by +dys in y: it
    re-enters there, and (for an integer dys, where the interpolations commute) both see
    the same field."""
    rng = np.random.default_rng(86)
    nx, ny = 16, 20
    s, om, dt = 1.5, 0.01, 0.45
    box = oracle.make_box(2, (nx, ny), dt=dt, frame=oracle.SHEAR, shear_s=s, omega0=om)
    E, B, J = oracle.zeros_fields(box)
    for c in range(3):
        E[c][:] = rng.normal(size=E[c].shape)
        B[c][:] = rng.normal(size=B[c].shape)
    for dys in (3.0, 7.0):
        for yy in (2.3, 11.7):
            a = oracle.gather(box, E, B, [nx + 0.3], [yy], dys=dys)
            b = oracle.gather(box, E, B, [0.3], [yy + dys], dys=dys)
            np.testing.assert_allclose(a[0], b[0], rtol=1e-14, atol=1e-14)
            np.testing.assert_allclose(a[1], b[1], rtol=1e-14, atol=1e-14)
    # a test particle crossing x_o during step n re-enters at x_i with y + dys(t^{n+1})
    E0, B0, J0 = oracle.zeros_fields(box)
    box.step = 1000
    u = np.array([0.9, 0.1, 0.0])
    sp = oracle.SpeciesState([nx - 0.1], [4.0], None, [u[0]], [u[1]], [u[2]], 1.0, 0.0)
    upush = oracle.push_shear(1.0, dt, s, om, [nx - 0.1 - nx / 2], np.zeros((1, 3)),
                              np.zeros((1, 3)), u[None])[0]
    g = np.sqrt(1 + upush @ upush)
    x1 = nx - 0.1 + dt * upush[0] / g
    y1 = 4.0 + dt * upush[1] / g - s * om * ((x1 - nx / 2) + (nx - 0.1 - nx / 2)) / 2 * dt
    oracle.step(box, E0, B0, J0, [sp])
    dys1 = oracle.shear_offset(box, 1001 * dt)
    assert x1 >= nx
    assert abs(sp.x[0] - (x1 - nx)) < 1e-12
    assert abs(sp.y[0] - np.mod(y1 + dys1, ny)) < 1e-12
