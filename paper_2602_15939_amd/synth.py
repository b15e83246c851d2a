"""Seeded synthetic inputs shaped like the paper's setups (pair plasma, uniform guide field,
random-phase magnetic fluctuations).  These generators hold none of the method's arithmetic;
both the HIP path and the CPU oracle consume what they produce.

Recipes (code units c = 1, dx = 1, Gaussian 4 pi):
  * positions: an independent uniform cell index per axis and a uniform FP32 offset in [0,1);
    electrons and positrons share positions (zero net charge, so E = 0 satisfies Gauss's law);
  * momenta: isotropic Maxwell-Juttner of temperature theta, |u| by inverse transform of a
    fine FP64 CDF table (numpy), direction uniform on the sphere;
  * plasma frequency from the total density of both species, omega_p^2 = 4 pi n_tot q^2/m
    with |q|/m = 1, so q_macro = omega_p^2 / (4 pi n_tot); B0 = omega_p sqrt(sigma);
  * fluctuations: random-phase Fourier modes built from a scalar potential psi (B = curl(psi e)),
    which keeps the discrete divergence of B zero on the Yee lattice.
"""
from __future__ import annotations

import math

import numpy as np
import torch

FOUR_PI = 4.0 * math.pi


def plasma_params(ppc_per_species: int, skin_depth: float = 4.0, sigma: float = 0.1):
    """(omega_p, q_macro, B0) for an e+/e- plasma with ppc_per_species of each species."""
    n_tot = 2.0 * ppc_per_species
    wp = 1.0 / skin_depth
    q = wp * wp / (FOUR_PI * n_tot)
    return wp, q, wp * math.sqrt(sigma)


def _mj_cdf(theta: float, npts: int = 20001):
    gmax = 1.0 + 50.0 * theta
    umax = math.sqrt(gmax * gmax - 1.0)
    u = np.linspace(0.0, umax, npts)
    f = u * u * np.exp(-(np.sqrt(1.0 + u * u) - 1.0) / theta)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(u))])
    return u, cdf / cdf[-1]


def mj_momenta(n: int, theta: float, gen: torch.Generator, device) -> torch.Tensor:
    """(3, n) float32 isotropic Maxwell-Juttner momenta."""
    ugrid, cdf = _mj_cdf(theta)
    ug = torch.as_tensor(ugrid, dtype=torch.float64, device=device)
    cg = torch.as_tensor(cdf, dtype=torch.float64, device=device)
    p = torch.rand(n, generator=gen, device=device, dtype=torch.float64)
    k = torch.searchsorted(cg, p).clamp(1, len(cdf) - 1)
    c0, c1 = cg[k - 1], cg[k]
    w = ((p - c0) / (c1 - c0).clamp_min(1e-300)).clamp(0, 1)
    um = ug[k - 1] + w * (ug[k] - ug[k - 1])
    mu = 2.0 * torch.rand(n, generator=gen, device=device, dtype=torch.float64) - 1.0
    phi = 2.0 * math.pi * torch.rand(n, generator=gen, device=device, dtype=torch.float64)
    st = torch.sqrt((1.0 - mu * mu).clamp_min(0.0))
    u = torch.stack([um * st * torch.cos(phi), um * st * torch.sin(phi), um * mu])
    return u.to(torch.float32)


def uniform_positions(n_cells, count: int, gen: torch.Generator, device):
    """linear cell index (int32) and (dim, count) float32 offsets of uniform positions"""
    dim = len(n_cells)
    cell = torch.zeros(count, dtype=torch.int64, device=device)
    stride = 1
    for d in range(dim):
        c = torch.randint(0, n_cells[d], (count,), generator=gen, device=device)
        cell += c * stride
        stride *= n_cells[d]
    off = torch.rand((dim, count), generator=gen, device=device, dtype=torch.float32)
    return cell.to(torch.int32), off


def pair_plasma(n_cells, ppc_per_species: int, theta: float, seed: int, device="cpu"):
    """Two species (electron first) sharing positions, independent momenta.  Positions are
    uniform random; the particles are stored in order of their cell (as a loader that fills the
    grid cell by cell would lay them out), which only fixes the storage order."""
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    count = ppc_per_species * int(np.prod(n_cells))
    cell, off = uniform_positions(n_cells, count, gen, device)
    order = torch.argsort(cell, stable=True)
    cell, off = cell[order].contiguous(), off[:, order].contiguous()
    del order
    u_e = mj_momenta(count, theta, gen, device)
    u_p = mj_momenta(count, theta, gen, device)
    return [dict(cell=cell, off=off, u=u_e), dict(cell=cell.clone(), off=off.clone(), u=u_p)]


def uniform_field(n_cells, axis: int, value: float):
    """(3, nz, ny, nx) float64 arrays E = 0 and B = value e_axis"""
    shape = (3, n_cells[2] if len(n_cells) == 3 else 1, n_cells[1], n_cells[0])
    E = np.zeros(shape)
    B = np.zeros(shape)
    B[axis] = value
    return E, B


def random_phase_psi(n_cells, kmax_index: float, slope: float, seed: int, kperp_axes=(0, 1)):
    """Real random-phase field psi with |psi_k| proportional to |k|^slope / |k_perp| on integer
    mode vectors 1 <= |n| <= kmax_index (Euclidean), k_perp over kperp_axes; modes with
    k_perp = 0 are left out (they carry no field of this polarisation)."""
    rng = np.random.default_rng(seed)
    dims = list(n_cells)
    shape = tuple(reversed(dims))  # (nz, ny, nx) or (ny, nx)
    ks = [np.fft.fftfreq(nd) * nd for nd in reversed(dims)]  # integer mode numbers per axis
    grids = np.meshgrid(*ks, indexing="ij")
    nvec = list(reversed(grids))  # nvec[d] = mode number along axis d
    kphys = [2 * np.pi * nvec[d] / dims[d] for d in range(len(dims))]
    nmag = np.sqrt(sum(n * n for n in nvec))
    kmag = np.sqrt(sum(k * k for k in kphys))
    kperp = np.sqrt(sum(kphys[d] ** 2 for d in kperp_axes))
    mask = (nmag >= 1) & (nmag <= kmax_index) & (kperp > 0)
    amp = np.zeros(shape)
    amp[mask] = kmag[mask] ** slope / kperp[mask]
    phase = rng.uniform(0, 2 * np.pi, shape)
    spec = amp * np.exp(1j * phase)
    return np.real(np.fft.ifftn(spec))


def curl_of_psi(n_cells, psi, axis: int = 2):
    """B = curl(psi e_axis) on the Yee lattice for axis = 2 (psi at the E_z points):
    B_x = d psi/dy at (i, j+1/2), B_y = -d psi/dx at (i+1/2, j)."""
    assert axis == 2
    shape = (3, n_cells[2] if len(n_cells) == 3 else 1, n_cells[1], n_cells[0])
    B = np.zeros(shape)
    p = psi.reshape(shape[1:])
    B[0] = np.roll(p, -1, axis=1) - p
    B[1] = -(np.roll(p, -1, axis=2) - p)
    return B


def fluctuation_field(n_cells, rms_over_b0: float, b0: float, kmax_index: float, slope: float,
                      seed: int):
    """In-plane (x, y) fluctuation field B = curl(psi e_z), normalised to rms |dB| = rms*b0."""
    psi = random_phase_psi(n_cells, kmax_index, slope, seed)
    dB = curl_of_psi(n_cells, psi)
    rms = math.sqrt(float((dB * dB).sum(axis=0).mean()))
    if rms > 0:
        dB *= rms_over_b0 * b0 / rms
    return dB
