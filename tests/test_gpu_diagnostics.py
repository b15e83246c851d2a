"""Particle diagnostics of the leaky-box application (Sec. 4.2) on the GPU: the energy
histogram equals the oracle's histogram of the same FP32 momenta bit for bit (FP64 energies on
both sides), and the kinetic-pressure, kinetic-energy and momentum sums equal the oracle's FP64
sums within summation-order rounding, all over the particles that have not escaped (an escaped
particle keeps its slot, with cell -1, until the next sort); after steps of a leaky box, both
follow the oracle's own particles."""
import math

import numpy as np
import pytest
import torch

import oracle
from _cases import Case, compare_particles
from paper_2602_15939_amd import _lib as L

pytestmark = pytest.mark.gpu

EDGES = list(np.concatenate([[0.0], np.logspace(-4, 2, 49)]))


@pytest.mark.parametrize("frame,kw", [
    ("leaky", dict(leaky_mode=L.LEAKY_DISPLACEMENT, l_esc=2.0, theta_inj=0.3)),
    ("leaky", dict(leaky_mode=L.LEAKY_PROBABILISTIC, t_esc=20.0, gamma_thr=1.5)),
    ("shear", {}),
])
def test_histogram_and_pressure_after_steps(frame, kw):
    c = Case(2, (48, 40), frame, ppc=6, theta=0.5, seed=77, **kw)
    try:
        for _ in range(4):
            c.gpu.step()
            c.oracle_step()
        info = c.gpu.info()
        assert info.errors & ~L.DERR_ORDER == 0
        P, Po, mom, mom_abs = np.zeros(3), np.zeros(3), np.zeros(3), 0.0
        ke = 0.0
        for s in range(2):
            g = c.gpu_species(s)
            h = c.gpu.energy_histogram(s, EDGES)
            # bit for bit against the oracle's definition on the GPU's momenta
            ug = g["u"][:, g["cell"] >= 0]
            assert h == list(oracle.energy_histogram(ug[0], ug[1], ug[2], EDGES))
            assert sum(h) == int((g["cell"] >= 0).sum())  # escaped particles excluded
            # the oracle's own momenta of the same particles (matched by id, so that an escape
            # decided differently within rounding of the threshold cannot enter): only
            # energies within FP32 rounding of an edge may fall on the other side
            o = c.sp[s]
            sel = compare_particles(c, s, g)["sel"]
            ho = oracle.energy_histogram(o.ux[sel], o.uy[sel], o.uz[sel], EDGES)
            assert np.abs(np.array(h) - ho).sum() <= 2, (h, list(ho))
            m = abs(c.q)  # |q|/m = 1 per species: macro mass = |q|
            P += oracle.kinetic_stress(*ug, m=m)
            ke += m * oracle.kinetic_energy(*ug).sum()
            mom += m * ug.astype(np.float64).sum(axis=1)
            mom_abs += m * np.abs(ug.astype(np.float64)).sum()
            Po += oracle.kinetic_stress(o.ux[sel], o.uy[sel], o.uz[sel], m=m)
        # the info reductions cover the same particles (none that escaped in the last step)
        assert abs(info.kinetic_energy - ke) <= 1e-12 * ke
        assert np.abs(np.array(info.momentum) - mom).max() <= 1e-12 * mom_abs
        got = np.array(info.pressure)
        assert np.allclose(got, P, rtol=1e-12, atol=0), (got, P)
        assert np.allclose(got, Po, rtol=1e-5, atol=0), (got, Po)
    finally:
        c.close()


def test_histogram_edge_cases():
    rng = np.random.default_rng(3)
    n = 5000
    u = (rng.standard_normal((3, n)) * 2.0).astype(np.float32)
    u[:, 0] = 0.0  # at rest: energy exactly 0
    u[0, 1] = np.nan  # non-finite energy: the last slot
    u[:, 2] = [0.0, 0.0, 1e-3]
    parts = [dict(cell=torch.from_numpy(rng.integers(0, 256, n).astype(np.int32)),
                  off=torch.from_numpy(rng.uniform(0, 1, (2, n)).astype(np.float32)),
                  u=torch.from_numpy(u))] * 2
    c = Case(2, (16, 16), "plain", parts=parts, q=0.0)
    try:
        for edges in ([0.0, 1e30], [-1.0, 0.0], [0.5, 0.6], EDGES,
                      list(np.linspace(0.0, 50.0, L.HIST_MAX_BINS + 1))):
            h = c.gpu.energy_histogram(0, edges)
            assert len(h) == len(edges) + 1
            assert h == list(oracle.energy_histogram(u[0], u[1], u[2], edges)), edges
            assert sum(h) == n
        with pytest.raises(L.PicError):
            c.gpu.energy_histogram(0, [1.0, 1.0])
        with pytest.raises(L.PicError):
            c.gpu.energy_histogram(0, list(range(L.HIST_MAX_BINS + 2)))
        with pytest.raises(L.PicError):
            c.gpu.energy_histogram(0, [0.0, math.inf])
        with pytest.raises(L.PicError):
            c.gpu.energy_histogram(2, [0.0, 1.0])
    finally:
        c.close()


def test_empty_box_histogram():
    c = Case(2, (16, 16), "plain", ppc=0)
    try:
        assert c.gpu.energy_histogram(1, EDGES) == [0] * (len(EDGES) + 1)
        assert list(c.gpu.info().pressure) == [0.0, 0.0, 0.0]
    finally:
        c.close()
