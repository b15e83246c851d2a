"""Pins of the leaky box's escape rule applied in the shearing, expanding and combined frames
(the combination the paper's conclusion suggests; escape on the displacement the deposit uses):
* with s = Omega0 = 0 the shearing box with escape is the leaky box: positions, momenta,
  displacements and escape decisions equal those of the leaky frame;
* the combined frame with escape reduces to the shearing box with escape when the expansion
  rate is 0, and to the expanding box with escape when s = Omega0 = 0 (the same escapes);
* the probabilistic rule in a rotating shearing frame and in an expanding frame removes a
  population far above gamma_thr at the binomial rate (1 - p)^n, p = dt / t_esc, as in the
  leaky frame: rotation and expansion change the momenta but not the escape law."""
import numpy as np
import pytest

import oracle


def population(n, gamma, rng):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    return np.sqrt(gamma ** 2 - 1) * v


def test_degenerate_shear_with_escape_is_the_leaky_box():
    rng = np.random.default_rng(4)
    n, N = (24, 20), 3000
    x, y = rng.uniform(0, 24, N), rng.uniform(0, 20, N)
    u = population(N, 1.3, rng)
    mj = oracle.mj_table(0.3)
    common = dict(dt=0.45, leaky_mode=oracle.LEAKY_DISPLACEMENT, l_esc=1.5, seed=77, box_id=2,
                  mj_table=mj, maxwell_iters=2)
    a = oracle.make_box(2, n, frame=oracle.SHEAR, shear_s=0.0, omega0=0.0, escape=True, **common)
    b = oracle.make_box(2, n, frame=oracle.LEAKY, **common)
    sa = oracle.SpeciesState(x, y, None, *u.T, 1.0, 0.0, ids=np.arange(N))
    sb = oracle.SpeciesState(x, y, None, *u.T, 1.0, 0.0, ids=np.arange(N))
    E, B, J = oracle.zeros_fields(a)
    E2, B2, J2 = oracle.zeros_fields(b)
    for _ in range(12):
        oracle.step(a, E, B, J, [sa])
        oracle.step(b, E2, B2, J2, [sb])
    assert np.abs(sa.x - sb.x).max() < 1e-12 and np.abs(sa.y - sb.y).max() < 1e-12
    assert np.abs(sa.ux - sb.ux).max() < 1e-12 and np.abs(sa.uy - sb.uy).max() < 1e-12
    np.testing.assert_array_equal(sa.dr[0] == 0, sb.dr[0] == 0)  # same escapes
    assert (sb.dr[0] == 0).sum() > 100


@pytest.mark.parametrize("reduce_to", ["shear", "expand"])
def test_combined_frame_with_escape_reduces_to_each_frame(reduce_to):
    rng = np.random.default_rng(12)
    n, N = (24, 20), 3000
    x, y = rng.uniform(0, 24, N), rng.uniform(0, 20, N)
    u = population(N, 1.3, rng)
    mj = oracle.mj_table(0.3)
    common = dict(dt=0.45, leaky_mode=oracle.LEAKY_DISPLACEMENT, l_esc=1.5, seed=78, box_id=2,
                  mj_table=mj, maxwell_iters=2, escape=True)
    if reduce_to == "shear":
        kw = dict(shear_s=1.5, omega0=0.01, adot=0.0)
        b = oracle.make_box(2, n, frame=oracle.SHEAR, shear_s=1.5, omega0=0.01, **common)
    else:
        kw = dict(shear_s=0.0, omega0=0.0, adot=3e-3, axis_mask=0b011)
        b = oracle.make_box(2, n, frame=oracle.EXPAND, adot=3e-3, axis_mask=0b011, **common)
    a = oracle.make_box(2, n, frame=oracle.SHEAR_EXPAND, **kw, **common)
    sa = oracle.SpeciesState(x, y, None, *u.T, 1.0, 0.0, ids=np.arange(N))
    sb = oracle.SpeciesState(x, y, None, *u.T, 1.0, 0.0, ids=np.arange(N))
    E, B, J = oracle.zeros_fields(a)
    E2, B2, J2 = oracle.zeros_fields(b)
    for _ in range(12):
        oracle.step(a, E, B, J, [sa])
        oracle.step(b, E2, B2, J2, [sb])
    assert np.abs(sa.x - sb.x).max() < 1e-11 and np.abs(sa.y - sb.y).max() < 1e-11
    assert np.abs(sa.ux - sb.ux).max() < 1e-11 and np.abs(sa.uy - sb.uy).max() < 1e-11
    assert np.abs(sa.dr - sb.dr).max() < 1e-11
    np.testing.assert_array_equal(sa.dr[0] == 0, sb.dr[0] == 0)  # same escapes
    assert (sb.dr[0] == 0).sum() > 100


FRAME_KW = {"shear": (oracle.SHEAR, dict(shear_s=1.5, omega0=0.01)),
            "expand": (oracle.EXPAND, dict(adot=2e-3, axis_mask=0b011)),
            "shear_expand": (oracle.SHEAR_EXPAND, dict(shear_s=1.5, omega0=0.01, adot=2e-3,
                                                       axis_mask=0b011))}


@pytest.mark.parametrize("frame", ["shear", "expand", "shear_expand"])
def test_probabilistic_escape_law_in_other_frames(frame):
    rng = np.random.default_rng(86)
    dt, p, N, nsteps = 0.45, 0.05, 4000, 40
    fr, kw = FRAME_KW[frame]
    box = oracle.make_box(2, (16, 16), dt=dt, frame=fr,
                          leaky_mode=oracle.LEAKY_PROBABILISTIC, t_esc=dt / p, gamma_thr=10.0,
                          seed=0x1234ABCD5678, box_id=3, escape=True, **kw)
    E, B, J = oracle.zeros_fields(box)
    hot = oracle.SpeciesState(rng.uniform(0, 16, N), rng.uniform(0, 16, N), None,
                              *population(N, 30.0, rng).T, 1.0, 0.0)
    for _ in range(nsteps):
        oracle.step(box, E, B, J, [hot])
    g = np.sqrt(1 + hot.ux ** 2 + hot.uy ** 2 + hot.uz ** 2)
    assert g.min() > 10.0  # the whole population stayed eligible
    mean = N * (1 - p) ** nsteps
    sd = np.sqrt(N * (1 - p) ** nsteps * (1 - (1 - p) ** nsteps))
    assert abs(hot.alive.sum() - mean) < 5 * sd, (hot.alive.sum(), mean, sd)
    # without the flag nothing escapes
    box2 = oracle.make_box(2, (16, 16), dt=dt, frame=box.frame, leaky_mode=oracle.LEAKY_PROBABILISTIC,
                           t_esc=dt / p, gamma_thr=10.0, seed=1, box_id=3, **kw)
    cold = oracle.SpeciesState(rng.uniform(0, 16, 100), rng.uniform(0, 16, 100), None,
                               *population(100, 30.0, rng).T, 1.0, 0.0)
    for _ in range(5):
        oracle.step(box2, E, B, J, [cold])
    assert cold.alive.sum() == 100
