"""Parity at the full sizes of the throughput workloads, in the launch configuration bench.py times
(default tiles, fused push, 268,435,456 particles), against the FP64 oracle on what it can
compute one by one:

  * the push of every particle whose cell lies in a sub-block of the grid plus a random sample of
    4096 particles per species from the whole box (the shearing-periodic and periodic wraps
    included): momenta within 2e-6 relative (|du| / max(|u|, 0.01)), positions within 2e-6 cells,
    escape decisions equal, the leaky box's tracked displacement within 2e-6 cells;
  * the deposited current (before the guard fold and the J' transport) inside that sub-block:
    the oracle deposits every particle that can reach it, from x^n to its own deposit endpoint
    (x^n + dt u/gamma; primed coordinates for the expanding box); within 1e-5 of max|J| there.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from _cases import cell_coords, wrap_diff
from paper_2602_15939_amd import workloads

pytestmark = pytest.mark.gpu

SEED = 20260216


def oracle_box(w):
    kw = dict(dt=w["dt"], maxwell_iters=w["maxwell_iters"], seed=SEED)
    if w["kind"] == "shear":
        kw.update(frame=oracle.SHEAR, shear_s=w["shear_s"], omega0=w["omega0"])
    elif w["kind"] == "expand":
        kw.update(frame=oracle.EXPAND, adot=w["adot"], axis_mask=w["axis_mask"])
    elif w.get("escape") == "displacement":
        kw.update(frame=oracle.LEAKY, leaky_mode=oracle.LEAKY_DISPLACEMENT, l_esc=w["l_esc"],
                  mj_table=oracle.mj_table(w["theta"]))
    else:
        kw.update(frame=oracle.LEAKY, leaky_mode=oracle.LEAKY_PROBABILISTIC, t_esc=w["t_esc"],
                  gamma_thr=w["gamma_thr"])
    return oracle.make_box(w["dim"], w["n"], **kw)


def to_np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("name", ["shear3d", "expand3d", "leaky2d", "leaky2d_paper"])
def test_full_size_sampled_parity(name):
    w = workloads.WORKLOADS[name]()
    dim, n = w["dim"], tuple(list(w["n"]) + [1] * (3 - w["dim"]))
    print(f"[fullsize] {w['name']}", flush=True)
    box, npart = workloads.make_box(w, SEED)
    try:
        pre = [box.get_particles(s) for s in range(2)]
        E, B = (to_np(t).astype(np.float64) for t in box.get_fields())
        box.sort()
        perms = [box.get_sort(s)[0] for s in range(2)]
        box.push(fuse=True)
        J = to_np(box.get_current()).astype(np.float64)
        post = [box.get_particles(s) for s in range(2)]
        info = box.info()
        assert info.errors & ~4 == 0 and info.n_slow == 0
    finally:
        box.close()
    torch.cuda.empty_cache()

    # sub-block R (cells [a, a+L) per axis) and the particles that can deposit into it
    L = 24 if dim == 3 else 64
    a = [n[d] // 2 - L // 2 if d < dim else 0 for d in range(3)]
    ob = oracle_box(w)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(SEED)
    Jo = np.zeros(oracle.jext_shape(ob))
    for s in range(2):
        cell = pre[s]["cell"].long()
        i, j, k = cell % n[0], (cell // n[0]) % n[1], cell // (n[0] * n[1])
        near = ((i >= a[0] - 2) & (i < a[0] + L + 2) & (j >= a[1] - 2) & (j < a[1] + L + 2))
        if dim == 3:
            near &= (k >= a[2] - 2) & (k < a[2] + L + 2)
        region = torch.nonzero(near).flatten()
        sample = torch.randint(0, cell.numel(), (4096,), generator=gen, device="cuda")
        idx = torch.cat([region, sample])
        nreg = region.numel()
        # output slot of each input index
        perm = perms[s].long()
        inv = torch.full((cell.numel(),), -1, dtype=torch.long, device="cuda")
        inv[perm] = torch.arange(perm.numel(), device="cuda")
        slot = inv[idx]
        assert (slot >= 0).all()
        old = {k_: to_np(v[..., idx]) for k_, v in pre[s].items() if k_ in ("cell", "off", "u")}
        new = {k_: to_np(v[..., slot]) for k_, v in post[s].items() if k_ in ("cell", "off", "u", "dr")}
        ci, cj, ck = cell_coords(old["cell"], n)
        x0 = ci + old["off"][0].astype(np.float64)
        y0 = cj + old["off"][1].astype(np.float64)
        z0 = ck + old["off"][2].astype(np.float64) if dim == 3 else np.zeros_like(x0)
        u0 = old["u"].astype(np.float64)
        qm = (-1.0, 1.0)[s]
        sp = oracle.SpeciesState(x0, y0, z0, u0[0], u0[1], u0[2], qm, qm * w["q"],
                                 ids=to_np(idx).astype(np.uint32))
        oracle.particles_only(ob, E, B, [sp])

        live_g = new["cell"] >= 0
        np.testing.assert_array_equal(live_g, sp.alive.astype(bool))
        uo = np.stack([sp.ux, sp.uy, sp.uz])[:, live_g]
        ug = new["u"][:, live_g].astype(np.float64)
        du = np.linalg.norm(ug - uo, axis=0) / np.maximum(np.linalg.norm(uo, axis=0), 1e-2)
        assert du.max() < 2e-6, (name, s, du.max())
        gi, gj, gk = cell_coords(new["cell"][live_g], n)
        pos_g = [gi + new["off"][0][live_g], gj + new["off"][1][live_g]]
        pos_o = [sp.x[live_g], sp.y[live_g]]
        if dim == 3:
            pos_g.append(gk + new["off"][2][live_g])
            pos_o.append(sp.z[live_g])
        ex = max(float(np.abs(wrap_diff(g, o, n[d])).max()) for d, (g, o) in enumerate(zip(pos_g, pos_o)))
        assert ex < 2e-6, (name, s, ex)
        if w.get("escape") == "displacement":  # the tracked in-plane displacement (Sec. 4.1)
            ddr = np.abs(new["dr"][:2, live_g] - sp.dr[:2, live_g]).max()
            assert ddr < 2e-6, (name, s, ddr)
        print(f"[fullsize] {name} species {s}: {len(idx)} particles, max du {du.max():.2e}, "
              f"max dx {ex:.2e}", flush=True)

        # oracle deposit of the region's particles from x^n to the deposit endpoint
        ux, uy, uz = sp.ux[:nreg], sp.uy[:nreg], sp.uz[:nreg]
        ig = 1.0 / np.sqrt(1.0 + ux * ux + uy * uy + uz * uz)
        lin = [1.0, 1.0, 1.0]
        if w["kind"] == "expand":
            th = 0.5 * w["dt"]
            lin = [1.0 / oracle.scale(ob, d, th) for d in range(3)]
        dx = w["dt"] * ux * ig * lin[0]
        dy = w["dt"] * uy * ig * lin[1]
        dzv = w["dt"] * uz * ig * lin[2]
        r = slice(0, nreg)
        if dim == 3:
            oracle.deposit(ob, qm * w["q"], x0[r], y0[r], x0[r] + dx, y0[r] + dy, z0[r], z0[r] + dzv,
                           Jext=Jo)
        else:
            oracle.deposit(ob, qm * w["q"], x0[r], y0[r], x0[r] + dx, y0[r] + dy, dz=dzv, Jext=Jo)

    JG = (Jo.shape[3] - n[0]) // 2
    lo = [a[d] + 2 if d < dim else 0 for d in range(3)]
    hi = [a[d] + L - 2 if d < dim else 1 for d in range(3)]
    sub_g = J[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
    sub_o = Jo[:, lo[2]:hi[2], lo[1]:hi[1], lo[0] + JG:hi[0] + JG]
    err = np.abs(sub_g - sub_o).max() / np.abs(sub_o).max()
    print(f"[fullsize] {name} J sub-block {sub_o.shape}: max|dJ|/max|J| = {err:.2e}", flush=True)
    assert err < 1e-5
    assert math.isfinite(err) and np.abs(sub_o).max() > 0
