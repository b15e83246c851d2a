"""The tile-shape autotuner on the GPU: it leaves the box state unchanged (particles bit-exact,
error bits and step), picks a supported shape that admits the migration sort, reports a
positive time per candidate, and the re-tiled box then steps like an untuned twin (parity
tolerances: momenta 2e-6 relative, positions 2e-6 cells, fields 1e-5 of their maximum)."""
import numpy as np
import pytest

from _cases import Case
from paper_2602_15939_amd import _lib as L
from test_gpu_batched import assert_same_state

pytestmark = pytest.mark.gpu

CASES = [
    dict(dim=3, n=(32, 32, 32), frame="shear", batched=False, kw=dict(omega0=0.04)),
    dict(dim=2, n=(64, 64), frame="expand", batched=True, kw=dict(adot=2e-3)),
    dict(dim=2, n=(64, 32), frame="leaky", batched=False,
         kw=dict(leaky_mode=L.LEAKY_PROBABILISTIC, t_esc=4.0, gamma_thr=1.5)),
]


@pytest.mark.parametrize("spec", CASES, ids=[c["frame"] + str(c["dim"]) for c in CASES])
def test_autotune_keeps_state_and_steps_like_untuned(spec):
    tuned = Case(spec["dim"], spec["n"], spec["frame"], ppc=3, seed=77, theta=0.4, **spec["kw"])
    twin = Case(spec["dim"], spec["n"], spec["frame"], ppc=3, seed=77, theta=0.4, **spec["kw"])
    try:
        for c in (tuned, twin):
            c.gpu.step()
        before = [tuned.gpu_species(s) for s in range(2)]
        info0 = tuned.gpu.info()
        shape, ms = tuned.gpu.autotune(batched=spec["batched"], trials=2)
        flags = L.TUNE_BATCHED if spec["batched"] else 0
        assert shape in L.pic_tile_candidates(spec["dim"], flags)
        assert set(ms) == set(L.pic_tile_candidates(spec["dim"], flags))
        assert all(v > 0 for v in ms.values()), ms
        info1 = tuned.gpu.info()
        assert info1.step == info0.step and info1.errors == info0.errors
        assert info1.n_escaped == info0.n_escaped and info1.n_slow == info0.n_slow
        for s in range(2):
            after = tuned.gpu_species(s)
            for k in ("cell", "off", "u", "id"):
                np.testing.assert_array_equal(after[k], before[s][k])
        for k in range(3):
            tuned.gpu.step()
            twin.gpu.step()
        assert_same_state(tuned, twin, (spec["frame"], shape), by_id=True)
        assert tuned.gpu.info().n_sort_fallbacks == 0
    finally:
        tuned.close()
        twin.close()
