"""Synthetic full-size workloads shaped like the paper's setups (input recipes only; none of the
method's arithmetic).  Code units c = 1, dx = 1; skin depth 4 cells; |q|/m = 1 per species.

  shear3d   3D shearing box, 256^3 cells, 8 ppc per species, Maxwell-Juttner theta = 0.3,
            B0 along z with sigma = 0.05, Keplerian s = 1.5, Omega0 = 0.05 omega_c, dt = 0.45
  shear2d_parity  the small parity configuration: 2D shearing box, 64^2 cells, 16 ppc per
            species (131,072 particles), theta = 0.1, B0 along z with sigma = 0.1, s = 1.5,
            Omega0 = 0.1 omega_c, dt = 0.45, timed over 200 steps with the oracle beside it
  expand3d  3D expanding box, 128 x 128 x 512 cells, 16 ppc per species, theta = 0.05,
            B0 along the long axis (z) with sigma = 0.05 plus random-phase transverse
            fluctuations B = curl(psi e_z), |dB_k| ~ |k|^(-11/6) on 1 <= |n| <= 8,
            rms dB/B0 = 0.5; l_x = l_y = 1 + adot t, adot = 1e-3 omega_p
  leaky2d   2D leaky box, 2048^2 cells, 32 ppc per species, theta = 0.3, B0 along z with
            sigma = 1, in-plane fluctuations with a flat spectrum on |n| <= 128 (|k| <= k_max/8),
            rms dB/B0 = 1; probabilistic escape above gamma = 10 with t_esc = 10 L/c
  leaky2d_stress  the same box with every particle on a gamma = 20 shell and t_esc = 100 dt
            (1 % of the particles escape per step: the escape and compaction path under load)
  leaky2d_paper   the same box with the paper's own escape rule (Sec. 4.1): a particle whose
            in-plane displacement reaches l_esc = L/2 is re-drawn from the Maxwell-Juttner
            distribution at theta in place
  leaky2d_paper_stress  the paper's rule with l_esc = 2 cells, so that the displacement test
            and the Maxwell-Juttner re-draw run under load (a few % of the particles per step)
"""
from __future__ import annotations

import math

import numpy as np

from . import synth


def shear3d(n=256, ppc=8):
    wp, q, B0 = synth.plasma_params(ppc, 4.0, 0.05)
    return dict(name=f"shear3d_{n}^3_ppc{ppc}", kind="shear", dim=3, n=(n, n, n), ppc=ppc,
                theta=0.3, q=q, B0=B0, shear_s=1.5, omega0=0.05 * B0, dt=0.45, maxwell_iters=8)


def shear2d_parity(n=64, ppc=16):
    wp, q, B0 = synth.plasma_params(ppc, 4.0, 0.1)
    return dict(name=f"shear2d_{n}^2_ppc{ppc}", kind="shear", dim=2, n=(n, n), ppc=ppc,
                theta=0.1, q=q, B0=B0, shear_s=1.5, omega0=0.1 * B0, dt=0.45, maxwell_iters=8)


def expand3d(nxy=128, nz=512, ppc=16):
    wp, q, B0 = synth.plasma_params(ppc, 4.0, 0.05)
    return dict(name=f"expand3d_{nxy}x{nxy}x{nz}_ppc{ppc}", kind="expand", dim=3, n=(nxy, nxy, nz),
                ppc=ppc, theta=0.05, q=q, B0=B0, adot=1e-3 * wp, axis_mask=0b011, dB=0.5,
                kmax_index=8, slope=-11.0 / 6.0, dt=0.45, maxwell_iters=8)


def leaky2d(n=2048, ppc=32):
    wp, q, B0 = synth.plasma_params(ppc, 4.0, 1.0)
    return dict(name=f"leaky2d_{n}^2_ppc{ppc}", kind="leaky", dim=2, n=(n, n), ppc=ppc, theta=0.3,
                q=q, B0=B0, dB=1.0, kmax_index=n / 16, slope=0.0, t_esc=10.0 * n, gamma_thr=10.0,
                dt=0.45, maxwell_iters=8)


def leaky2d_stress(n=2048, ppc=32):
    """The leaky box with its escape path under load: every particle on a mono-energetic
    gamma = 20 shell (isotropic directions) above the gamma = 10 threshold, t_esc = 100 dt, so
    that 1 % of the particles escape (and are compacted away by the next sort) every step."""
    w = leaky2d(n, ppc)
    w.update(name=f"leaky2d_stress_{n}^2_ppc{ppc}", shell_gamma=20.0, t_esc=100 * 0.45)
    return w


def leaky2d_paper(n=2048, ppc=32, l_esc=None):
    w = leaky2d(n, ppc)
    w.update(name=f"leaky2d_paper_{n}^2_ppc{ppc}", escape="displacement",
             l_esc=float(n // 2) if l_esc is None else l_esc)
    return w


def leaky2d_paper_stress(n=2048, ppc=32):
    w = leaky2d_paper(n, ppc, l_esc=2.0)
    w.update(name=f"leaky2d_paper_stress_{n}^2_ppc{ppc}")
    return w


WORKLOADS = {"shear3d": shear3d, "shear2d_parity": shear2d_parity, "expand3d": expand3d,
             "leaky2d": leaky2d,
             "leaky2d_stress": leaky2d_stress, "leaky2d_paper": leaky2d_paper,
             "leaky2d_paper_stress": leaky2d_paper_stress}


def fields(w, seed):
    """(E, B) float64 arrays (3, nz, ny, nx): E = 0, B = B0 e_z (+ fluctuations)."""
    E, B = synth.uniform_field(w["n"], 2, w["B0"])
    if "dB" in w:
        B += synth.fluctuation_field(w["n"], w["dB"], w["B0"], w["kmax_index"], w["slope"], seed)
    return E, B


def make_box(w, seed, device="cuda", track_ids=False):
    """The box on the GPU with its synthetic plasma; returns (box, particle count)."""
    import torch

    from . import _lib as L
    from .box import Box

    count = w["ppc"] * math.prod(w["n"])
    species = [(-1.0, -w["q"], count), (1.0, w["q"], count)]
    kw = dict(dt=w["dt"], species=species, seed=seed, maxwell_iters=w["maxwell_iters"],
              track_ids=track_ids)
    if w["kind"] == "shear":
        box = Box(w["dim"], w["n"], frame=L.FRAME_SHEAR, shear_s=w["shear_s"],
                  shear_omega0=w["omega0"], **kw)
    elif w["kind"] == "expand":
        box = Box(w["dim"], w["n"], frame=L.FRAME_EXPAND, expand_adot=w["adot"],
                  expand_axis_mask=w["axis_mask"], **kw)
    elif w.get("escape") == "displacement":
        box = Box(w["dim"], w["n"], frame=L.FRAME_LEAKY, leaky_mode=L.LEAKY_DISPLACEMENT,
                  leaky_l_esc=w["l_esc"], leaky_theta_inj=w["theta"], **kw)
    else:
        box = Box(w["dim"], w["n"], frame=L.FRAME_LEAKY, leaky_mode=L.LEAKY_PROBABILISTIC,
                  leaky_t_esc=w["t_esc"], leaky_gamma_thr=w["gamma_thr"], **kw)
    E, B = fields(w, seed)
    box.set_fields(torch.from_numpy(E).float(), torch.from_numpy(B).float())
    del E, B
    parts = synth.pair_plasma(w["n"], w["ppc"], w["theta"], seed, device=device)
    if "shell_gamma" in w:  # momenta on a sphere |u| = sqrt(gamma^2 - 1), isotropic
        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed) + 17)
        for p in parts:
            d = torch.randn(p["u"].shape, generator=gen, device=device, dtype=torch.float64)
            d *= math.sqrt(w["shell_gamma"] ** 2 - 1.0) / torch.linalg.vector_norm(d, dim=0)
            p["u"] = d.float().contiguous()
    for s, p in enumerate(parts):
        box.set_particles(s, p["cell"], p["off"], p["u"])
    del parts
    torch.cuda.synchronize()
    return box, 2 * count
