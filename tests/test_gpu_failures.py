"""Failure detection in the batched step: errors latch per box and do not spread.  One box gets a
particle with a NaN momentum (PIC_DERR_NAN), another a time step dt = 0.6 (inside the 2D Yee
limit) and an ultrarelativistic particle whose displacement reaches half a cell (PIC_DERR_CFL);
a clean box stepped in the same launches equals its solo run, with no error bits.  The
conditions are forced from the host; the kernels stay in bounds (a NaN offset keeps the cell, a
long move keeps the deposit's fixed node range, only its values are wrong)."""
import numpy as np
import pytest
import torch

from _cases import Case
from paper_2602_15939_amd import _lib as L
from paper_2602_15939_amd import synth
from paper_2602_15939_amd.box import step_many
from test_gpu_batched import assert_same_state

pytestmark = pytest.mark.gpu


def poisoned(seed, n, u_bad, dt=0.45):
    parts = synth.pair_plasma(n, 4, 0.3, seed)
    u = parts[0]["u"].clone()
    u[:, 5] = torch.tensor(u_bad, dtype=torch.float32)
    parts[0]["u"] = u
    return Case(2, n, "plain", parts=parts, dt=dt, seed=seed, tile=(16, 16, 1))


def test_errors_latch_per_box_and_do_not_spread():
    n = (48, 32)
    clean = Case(2, n, "shear", ppc=4, seed=81, tile=(16, 16, 1), omega0=0.02)
    solo = Case(2, n, "shear", ppc=4, seed=81, tile=(16, 16, 1), omega0=0.02)
    nan_box = poisoned(82, n, [float("nan"), 0.0, 0.0])
    cfl_box = poisoned(83, n, [1000.0, 0.0, 0.0], dt=0.6)
    boxes = [clean, nan_box, cfl_box]
    try:
        for _ in range(3):
            step_many([c.gpu for c in boxes], batched=True)
            step_many([solo.gpu], batched=False)
        assert clean.gpu.info().errors & ~L.DERR_ORDER == 0
        assert_same_state(clean, solo, "clean box in the mix")
        e_nan = nan_box.gpu.info().errors
        e_cfl = cfl_box.gpu.info().errors
        assert e_nan & L.DERR_NAN and not e_nan & L.DERR_CFL, e_nan
        assert e_cfl & L.DERR_CFL and not e_cfl & L.DERR_NAN, e_cfl
        # the rest of a latched box still steps: its fields stay finite
        for c in (nan_box, cfl_box):
            for f in c.gpu.get_fields():
                assert torch.isfinite(f).all()
    finally:
        for c in boxes + [solo]:
            c.close()
