"""The entry point that allocates nothing: pic_energy_histogram_static (static device scratch)
against pic_energy_histogram (the box's own scratch) on the same particles, bit for bit, on two
calls in a row, the second with a smaller input (fewer particles and fewer bins), so that a
count left in the shared scratch by the first call would show.  Also: the size limit of the
scratch is an error, not a fault."""
import numpy as np
import pytest

from _cases import Case
from paper_2602_15939_amd import _lib as L

pytestmark = pytest.mark.gpu


def _edges(nb, hi):
    return list(np.concatenate([[0.0], np.logspace(-4, hi, nb)]))


def test_static_histogram_equals_box_histogram_twice():
    big = Case(2, (64, 48), "leaky", ppc=8, theta=0.5, seed=91, leaky_mode=L.LEAKY_DISPLACEMENT,
               l_esc=2.0, theta_inj=0.5)
    small = Case(2, (16, 16), "shear", ppc=2, theta=0.2, seed=92)
    try:
        for _ in range(3):
            big.gpu.step()
            small.gpu.step()
        e1 = _edges(300, 2)
        for s in range(2):
            ref = big.gpu.energy_histogram(s, e1)
            got = big.gpu.energy_histogram(s, e1, static=True)
            assert got == ref
            assert sum(got) == big.gpu.count(s)
        # second call: a smaller box and fewer bins; the first call's counts stay in the
        # scratch beyond the new bins and must not leak into the result
        e2 = _edges(12, 0)
        for s in range(2):
            ref = small.gpu.energy_histogram(s, e2)
            got = small.gpu.energy_histogram(s, e2, static=True)
            assert got == ref
            assert len(got) == 14 and sum(got) == small.gpu.count(s)
    finally:
        big.close()
        small.close()


def test_static_histogram_rejects_sizes_beyond_the_scratch():
    c = Case(2, (16, 16), "plain", ppc=2, seed=93)
    try:
        too_many = list(np.arange(L.HIST_STATIC_MAX_BINS + 2, dtype=float))
        with pytest.raises(L.PicError):
            c.gpu.energy_histogram(0, too_many, static=True)
        # still usable afterwards, and equal to the box variant
        e = _edges(40, 1)
        assert c.gpu.energy_histogram(1, e, static=True) == c.gpu.energy_histogram(1, e)
    finally:
        c.close()
