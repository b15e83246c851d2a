"""Shared construction of matching inputs for the HIP path and the CPU oracle.

Inputs are generated once (seeded, ``paper_2602_15939_amd.synth``) in the FP32 layout of the
C ABI; the oracle receives the exact FP64 values of the same numbers (positions cell + offset,
momenta, fields), so any difference in the outputs comes from the two implementations.
"""
from __future__ import annotations

import math

import numpy as np
import torch

import oracle
from paper_2602_15939_amd import _lib as L
from paper_2602_15939_amd import synth

FRAMES = {"plain": L.FRAME_PLAIN, "shear": L.FRAME_SHEAR, "expand": L.FRAME_EXPAND,
          "leaky": L.FRAME_LEAKY, "shear_expand": L.FRAME_SHEAR_EXPAND}


def cell_coords(cell, n):
    cell = np.asarray(cell, dtype=np.int64)
    i = cell % n[0]
    r = cell // n[0]
    return i, r % n[1], r // n[1]


def positions_f64(cell, off, n, dim):
    i, j, k = cell_coords(cell, n)
    off = np.asarray(off, dtype=np.float64)
    x = i + off[0]
    y = j + off[1]
    z = k + off[2] if dim == 3 else np.zeros_like(x)
    return x, y, z


def random_fields(n3, seed, e_amp=0.03, b_amp=0.2, b0=(0.0, 0.0, 0.1)):
    rng = np.random.default_rng(seed)
    shape = (3, n3[2], n3[1], n3[0])
    E = rng.uniform(-e_amp, e_amp, shape).astype(np.float32)
    B = rng.uniform(-b_amp, b_amp, shape).astype(np.float32)
    for c in range(3):
        B[c] += np.float32(b0[c])
    return E, B


class Case:
    """A box built twice: on the GPU through the C ABI and in the oracle."""

    def __init__(self, dim, n, frame="plain", ppc=4, theta=0.3, seed=1, dt=0.45, fields=None,
                 tile=(0, 0, 0), shear_s=1.5, omega0=0.02, adot=2e-3, axis_mask=0b011,
                 leaky_mode=L.LEAKY_DISPLACEMENT, l_esc=3.0, t_esc=9.0, gamma_thr=10.0,
                 theta_inj=0.3, maxwell_iters=4, maxwell_tol=0.0, q=None, parts=None, track_ids=True,
                 use_3vec=0, box_seed=0x5EED1234ABCDEF01, box_id=7, stream=None,
                 count_superluminal=False, escape=False, mem="caller"):
        self.dim = dim
        self.n = tuple(list(n) + [1] * (3 - len(n)))
        self.frame = FRAMES[frame]
        if parts is None:
            parts = synth.pair_plasma(tuple(n), ppc, theta, seed)
        self.parts = [{k: v.cpu().numpy() for k, v in p.items()} for p in parts]
        if q is None:
            q = synth.plasma_params(max(ppc, 1))[1]  # an empty box keeps the 1-ppc charge
        self.q = q
        self.qms = (-1.0, 1.0)
        if fields is None:
            fields = random_fields(self.n, seed + 100)
        self.E32, self.B32 = fields
        cap = max(len(p["cell"]) for p in self.parts) + 16
        mj = None
        if (self.frame == L.FRAME_LEAKY or escape) and leaky_mode == L.LEAKY_DISPLACEMENT:
            mj = oracle.mj_table(theta_inj)
        common = dict(dt=dt)
        self.gpu = None
        from paper_2602_15939_amd.box import Box
        self.gpu = Box(dim, self.n, dt=dt, frame=self.frame,
                       species=[(qm, qm * q, cap) for qm in self.qms], shear_s=shear_s,
                       shear_omega0=omega0, expand_adot=adot, expand_axis_mask=axis_mask,
                       leaky_mode=leaky_mode, leaky_l_esc=l_esc, leaky_use_3vec=use_3vec,
                       leaky_theta_inj=theta_inj, leaky_t_esc=t_esc, leaky_gamma_thr=gamma_thr,
                       seed=box_seed, box_id=box_id, tile=tile, maxwell_iters=maxwell_iters,
                       maxwell_tol=maxwell_tol,
                       track_ids=track_ids, stream=stream,
                       count_superluminal=count_superluminal, escape=escape, mem=mem,
                       unfused=True)
        self.gpu.set_fields(torch.from_numpy(self.E32), torch.from_numpy(self.B32))
        for s, p in enumerate(self.parts):
            ids = np.arange(len(p["cell"])) + s * 10_000_000
            p["id"] = ids
            self.gpu.set_particles(s, torch.from_numpy(p["cell"]), torch.from_numpy(p["off"]),
                                   torch.from_numpy(p["u"]), ids=torch.from_numpy(ids))
        self.box = oracle.make_box(dim, self.n[:dim], frame=self.frame, shear_s=shear_s,
                                   omega0=omega0, adot=adot, axis_mask=axis_mask,
                                   leaky_mode=leaky_mode, l_esc=l_esc, use_3vec=use_3vec,
                                   t_esc=t_esc, gamma_thr=gamma_thr, seed=box_seed, box_id=box_id,
                                   mj_table=mj, maxwell_iters=maxwell_iters,
                                   maxwell_tol=maxwell_tol, escape=escape, **common)
        self.E = self.E32.astype(np.float64)
        self.B = self.B32.astype(np.float64)
        self.J = np.zeros_like(self.E)
        self.sp = []
        for s, p in enumerate(self.parts):
            x, y, z = positions_f64(p["cell"], p["off"], self.n, dim)
            u = p["u"].astype(np.float64)
            self.sp.append(oracle.SpeciesState(x, y, z, u[0], u[1], u[2], self.qms[s],
                                               self.qms[s] * q, ids=p["id"]))

    # ---- GPU state in the oracle's order
    def gpu_species(self, s):
        """GPU particles (slot order) and, per slot, the input index it came from."""
        g = {k: v.cpu().numpy() for k, v in self.gpu.get_particles(s).items()}
        return g

    def oracle_step(self, nthreads=1):
        oracle.step(self.box, self.E, self.B, self.J, self.sp, nthreads=nthreads)

    def close(self):
        if self.gpu is not None:
            self.gpu.close()


def wrap_diff(a, b, n):
    d = np.asarray(a) - np.asarray(b)
    return d - n * np.round(d / n)


def compare_particles(case, s, g, tol_u=2e-6, tol_x=2e-6):
    """GPU particles g (with ids) against the oracle species s (same ids); returns stats."""
    o = case.sp[s]
    idx = {int(v): k for k, v in enumerate(o.id)}
    live = g["cell"] >= 0
    sel = np.array([idx[int(v)] for v in g["id"][live]])
    n = case.n
    x, y, z = positions_f64(g["cell"][live], g["off"][:, live], n, case.dim)
    dx = [wrap_diff(x, o.x[sel], n[0]), wrap_diff(y, o.y[sel], n[1])]
    if case.dim == 3:
        dx.append(wrap_diff(z, o.z[sel], n[2]))
    ex = max(float(np.abs(d).max()) for d in dx) if live.any() else 0.0
    uo = np.stack([o.ux[sel], o.uy[sel], o.uz[sel]])
    ug = g["u"][:, live].astype(np.float64)
    du = np.linalg.norm(ug - uo, axis=0) / np.maximum(np.linalg.norm(uo, axis=0), 1e-2)
    eu = float(du.max()) if live.any() else 0.0
    return dict(err_x=ex, err_u=eu, n=int(live.sum()), sel=sel, live=live)
