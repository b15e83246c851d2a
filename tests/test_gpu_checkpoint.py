"""Checkpoint and resume: a run split at step k (fields, particles with ids and displacements,
and the step counter saved; a new box created from the same descriptor, loaded, pic_set_step)
continues like the unsplit run: same escapes from the same Philox stream (keyed by id and step),
the shearing offset and the scale factor of the same time, and the state after further steps
equal within the tolerances of the batched tests (the float atomics of the tile-halo current
flush add in a run-dependent order)."""
import numpy as np
import pytest
import torch

from _cases import Case
from paper_2602_15939_amd import _lib as L
from test_gpu_batched import assert_same_state

pytestmark = pytest.mark.gpu

CASES = [
    (2, (48, 40), "shear", dict(omega0=0.03)),
    (3, (16, 16, 16), "shear", dict(omega0=0.03)),
    (2, (48, 40), "expand", dict(adot=2e-3)),
    (2, (48, 40), "leaky", dict(leaky_mode=L.LEAKY_PROBABILISTIC, t_esc=4.0, gamma_thr=1.3)),
    (2, (48, 40), "leaky", dict(leaky_mode=L.LEAKY_DISPLACEMENT, l_esc=1.5, theta_inj=0.3)),
]


@pytest.mark.parametrize("dim,n,frame,kw", CASES)
def test_split_run_resumes(dim, n, frame, kw):
    a = Case(dim, n, frame, ppc=4, theta=0.4, seed=61, **kw)
    b = Case(dim, n, frame, ppc=4, theta=0.4, seed=62, **kw)  # other particles, overwritten
    try:
        k = 5
        for _ in range(k):
            a.gpu.step()
        E, B = a.gpu.get_fields()
        saved = []
        for s in range(2):
            p = a.gpu.get_particles(s)
            live = p["cell"] >= 0  # escaped particles are not part of the state
            saved.append({key: v[..., live].clone() for key, v in p.items()})
        b.gpu.set_fields(E, B)
        for s, p in enumerate(saved):
            b.gpu.set_particles(s, p["cell"], p["off"], p["u"], ids=p["id"], dr=p["dr"])
        b.gpu.set_step(k)
        ia, ib = a.gpu.info(), b.gpu.info()
        assert ia.step == ib.step == k and ia.t == ib.t and ia.dys == ib.dys and ia.a == ib.a
        for _ in range(5):
            a.gpu.step()
            b.gpu.step()
        assert_same_state(a, b, (frame, dim), by_id=True)
        if frame == "leaky" and kw["leaky_mode"] == L.LEAKY_DISPLACEMENT:
            for s in range(2):
                ga, gb = a.gpu_species(s), b.gpu_species(s)
                oa, ob = np.argsort(ga["id"]), np.argsort(gb["id"])
                assert np.abs(ga["dr"][:2, oa] - gb["dr"][:2, ob]).max() < 2e-6
    finally:
        a.close()
        b.close()


def test_set_step_argument_checks():
    c = Case(2, (16, 16), "plain", ppc=1)
    try:
        with pytest.raises(L.PicError):
            c.gpu.set_step(-1)
    finally:
        c.close()
