"""Whole steps against the oracle on grids of more cells than one pass of the capped grid-stride
launches covers (4096 blocks x 256 threads = 1,048,576 cells), so that their threads loop: the
shearing box's J' transport and x fold (and its staged Maxwell sweeps, x = 128), the
expanding box's Yee updates, and the combined frame's field scaling around its one-thread-per-
cell sweeps.  Particles within 2e-6, current and fields within 1e-5 of their
maximum, as the small-grid parity tests."""
import numpy as np
import pytest

from _cases import Case, compare_particles
from paper_2602_15939_amd import _lib as L

pytestmark = pytest.mark.gpu

N = (128, 64, 160)  # 1,310,720 cells


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("frame,kw", [("shear", dict(omega0=0.004)), ("expand", dict(adot=2e-3, axis_mask=0b011)),
                                      ("shear_expand", dict(omega0=0.004, adot=2e-3, axis_mask=0b011))])
def test_step_on_a_grid_larger_than_one_stride_pass(frame, kw):
    print(f"[grid-stride] {frame} {N}", flush=True)
    c = Case(3, N, frame, ppc=1, seed=81, maxwell_iters=8, **kw)
    try:
        for step in range(2):
            c.gpu.step()
            c.oracle_step(nthreads=16)
            for s in range(2):
                st = compare_particles(c, s, c.gpu_species(s))
                assert st["err_u"] < 2e-6 and st["err_x"] < 2e-6, (step, s, st)
            assert rel(c.gpu.get_current().cpu().numpy(), c.J) < 1e-5, step
            E, B = (t.cpu().numpy() for t in c.gpu.get_fields())
            assert rel(E, c.E) < 1e-5 and rel(B, c.B) < 1e-5, step
        info = c.gpu.info()
        assert info.errors & ~L.DERR_ORDER == 0 and info.n_slow == 0
    finally:
        c.close()
