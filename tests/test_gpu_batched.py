"""The batched step (one launch per kernel over many boxes of different frames and sizes, driven
by box-descriptor tables) against the same boxes stepped one at a time: every box's result in
the mix equals its result alone within the parity tolerances (push 2e-6 relative, positions
2e-6 cells, fields 1e-5 of their maximum) after several steps; integer work (cells, ids, escape
counts) equal."""
import numpy as np
import pytest
import torch

from _cases import Case, wrap_diff, positions_f64
from paper_2602_15939_amd import _lib as L
from paper_2602_15939_amd.box import step_many

pytestmark = pytest.mark.gpu

MIX = [
    dict(dim=2, n=(64, 64), frame="shear", tile=(16, 16, 1), ppc=4, kw=dict(omega0=0.02)),
    dict(dim=2, n=(32, 32), frame="shear", tile=(8, 8, 1), ppc=6, kw=dict(omega0=0.03)),
    dict(dim=2, n=(32, 64), frame="expand", tile=(8, 8, 1), ppc=5, kw=dict(adot=2e-3)),
    dict(dim=2, n=(64, 48), frame="leaky", tile=(16, 16, 1), ppc=4,
         kw=dict(leaky_mode=L.LEAKY_PROBABILISTIC, t_esc=4.0, gamma_thr=1.5)),
    dict(dim=2, n=(48, 64), frame="plain", tile=(16, 16, 1), ppc=3, kw={}),
    dict(dim=3, n=(24, 24, 24), frame="shear", tile=(8, 8, 8), ppc=2, kw=dict(omega0=0.04)),
    dict(dim=2, n=(32, 48), frame="shear_expand", tile=(8, 8, 1), ppc=4,
         kw=dict(omega0=0.02, adot=3e-3, axis_mask=0b011)),
    dict(dim=3, n=(24, 24, 24), frame="shear_expand", tile=(8, 8, 8), ppc=2,
         kw=dict(omega0=0.03, adot=3e-3, axis_mask=0b100)),
]


def make(spec, seed, stream=None, mem="caller"):
    return Case(spec["dim"], spec["n"], spec["frame"], ppc=spec["ppc"], seed=seed, theta=0.4,
                tile=spec["tile"], maxwell_iters=4, stream=stream, mem=mem, **spec["kw"])


def assert_same_state(a, b, tag, by_id=False):
    """Two copies of one box after the same steps: integer work equal, momenta within 2e-6
    relative, positions within 2e-6 cells, fields within 1e-5 of their maximum (the float
    atomics of the tile-halo flush add in a run-dependent order).  by_id: the copies may use
    different tilings, so particles are matched by id instead of slot."""
    ia, ib = a.gpu.info(), b.gpu.info()
    assert ia.errors & ~L.DERR_ORDER == 0 and ib.errors & ~L.DERR_ORDER == 0, tag
    assert ia.step == ib.step, tag
    assert list(ia.n_particles) == list(ib.n_particles), tag
    for s in range(2):
        ga, gb = a.gpu_species(s), b.gpu_species(s)
        if by_id:
            ga = {k: (v[..., np.argsort(ga["id"], kind="stable")] if k != "dr" else v)
                  for k, v in ga.items()}
            gb = {k: (v[..., np.argsort(gb["id"], kind="stable")] if k != "dr" else v)
                  for k, v in gb.items()}
        np.testing.assert_array_equal(ga["id"], gb["id"])
        np.testing.assert_array_equal(ga["cell"] >= 0, gb["cell"] >= 0)
        live = gb["cell"] >= 0
        ua, ub = ga["u"][:, live].astype(np.float64), gb["u"][:, live].astype(np.float64)
        du = np.linalg.norm(ua - ub, axis=0) / np.maximum(np.linalg.norm(ub, axis=0), 1e-2)
        assert du.max() < 2e-6, (tag, s, du.max())
        xa = positions_f64(ga["cell"][live], ga["off"][:, live], a.n, a.dim)
        xb = positions_f64(gb["cell"][live], gb["off"][:, live], b.n, b.dim)
        for d in range(a.dim):
            assert np.abs(wrap_diff(xa[d], xb[d], a.n[d])).max() < 2e-6, (tag, s, d)
    for fa, fb in zip(a.gpu.get_fields(), b.gpu.get_fields()):
        fa, fb = fa.cpu().numpy(), fb.cpu().numpy()
        assert np.abs(fa - fb).max() <= 1e-5 * np.abs(fb).max(), tag


@pytest.mark.parametrize("mem", ["caller", "library"])
def test_batched_equals_alone(mem):
    """Boxes on torch memory step in batches through a pic_batch on torch staging; library-owned
    boxes through the first box's own staging."""
    mix = [make(sp, 300 + i, mem=mem) for i, sp in enumerate(MIX)]
    alone = [make(sp, 300 + i, mem=mem) for i, sp in enumerate(MIX)]
    try:
        for step in range(6):
            step_many([c.gpu for c in mix], batched=True)
            for c in alone:
                step_many([c.gpu], batched=False)
        for i, (a, b) in enumerate(zip(mix, alone)):
            ia, ib = a.gpu.info(), b.gpu.info()
            assert ia.errors & ~L.DERR_ORDER == 0 and ib.errors & ~L.DERR_ORDER == 0
            assert ia.step == ib.step == 6
            assert list(ia.n_particles) == list(ib.n_particles)
            assert ia.n_sort_migrations > 0 and ia.n_sort_fallbacks == 0
            for s in range(2):
                ga, gb = a.gpu_species(s), b.gpu_species(s)
                np.testing.assert_array_equal(ga["id"], gb["id"])
                np.testing.assert_array_equal(ga["cell"] >= 0, gb["cell"] >= 0)
                live = gb["cell"] >= 0
                ua, ub = ga["u"][:, live].astype(np.float64), gb["u"][:, live].astype(np.float64)
                du = np.linalg.norm(ua - ub, axis=0) / np.maximum(np.linalg.norm(ub, axis=0), 1e-2)
                assert du.max() < 2e-6, (i, s, du.max())
                xa = positions_f64(ga["cell"][live], ga["off"][:, live], a.n, a.dim)
                xb = positions_f64(gb["cell"][live], gb["off"][:, live], b.n, b.dim)
                for d in range(a.dim):
                    assert np.abs(wrap_diff(xa[d], xb[d], a.n[d])).max() < 2e-6, (i, s, d)
            for fa, fb in zip(a.gpu.get_fields(), b.gpu.get_fields()):
                fa, fb = fa.cpu().numpy(), fb.cpu().numpy()
                assert np.abs(fa - fb).max() <= 1e-5 * np.abs(fb).max(), i
    finally:
        for c in mix + alone:
            c.close()


def test_graph_replays_equal_eager_batched():
    """The batched step captured as a HIP graph and replayed: after every replay (with eager
    read-backs and synchronisations in between) each box equals the same box stepped by the
    eager batched step; the box set then shrinks (a new graph is captured) and grows back to
    the first set (its cached graph is replayed again)."""
    st = torch.cuda.Stream()  # capture needs a stream other than the null stream
    with torch.cuda.stream(st):
        gr = [make(sp, 500 + i, stream=st) for i, sp in enumerate(MIX)]
        ea = [make(sp, 500 + i, stream=st) for i, sp in enumerate(MIX)]
        try:
            plan = [list(range(len(MIX)))] * 3 + [[0, 2, 3, 5]] * 3 + [list(range(len(MIX)))] * 3
            for k, sel in enumerate(plan):
                step_many([gr[i].gpu for i in sel], batched=True, graph=True)
                step_many([ea[i].gpu for i in sel], batched=True)
                st.synchronize()
                for i in sel:
                    assert_same_state(gr[i], ea[i], (k, i))
        finally:
            for c in gr + ea:
                c.close()
