"""The batched step (one launch per kernel over many boxes of different frames and sizes, driven
by box-descriptor tables) against the same boxes stepped one at a time: every box's result in
the mix equals its result alone within the parity tolerances (push 2e-6 relative, positions
2e-6 cells, fields 1e-5 of their maximum) after several steps; integer work (cells, ids, escape
counts) equal."""
import numpy as np
import pytest

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
]


def make(spec, seed):
    return Case(spec["dim"], spec["n"], spec["frame"], ppc=spec["ppc"], seed=seed, theta=0.4,
                tile=spec["tile"], maxwell_iters=4, **spec["kw"])


def test_batched_equals_alone():
    mix = [make(sp, 300 + i) for i, sp in enumerate(MIX)]
    alone = [make(sp, 300 + i) for i, sp in enumerate(MIX)]
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
