"""Pin of the oracle's superluminal count (Sec. 2.1: the shearing-box effective velocity
u'/gamma' + v_s can exceed c; counted, not corrected).  With E' = B = 0 a particle at rest
stays at rest in the shearing frame (every term of eq. OAu is proportional to u' or to the
fields), so its effective velocity is the background flow v_s = -s Omega0 x alone: exactly the
particles with s Omega0 |x| > 1 count.  Particles moving along y add the closed-form cases
|u_y/gamma + v_s| far above or below 1."""
import math

import numpy as np

import oracle


def run(x, ux, uy, n=(64, 8), s=1.5, omega0=1.0 / 30.0, steps=1):
    box = oracle.make_box(2, n, frame=oracle.SHEAR, shear_s=s, omega0=omega0, dt=0.45,
                          maxwell_iters=2)
    E, B = np.zeros((3, 1, n[1], n[0])), np.zeros((3, 1, n[1], n[0]))
    J = np.zeros_like(E)
    k = len(x)
    sp = oracle.SpeciesState(np.asarray(x, float), np.full(k, 3.5), np.zeros(k), np.asarray(ux, float),
                             np.asarray(uy, float), np.zeros(k), 1.0, 0.0, ids=np.arange(k))
    for _ in range(steps):
        oracle.step(box, E, B, J, [sp])
    return box.n_superluminal


def test_background_flow_beyond_light_cylinder():
    # s Omega0 = 0.05: |v_s| = 1 at |x - 32| = 20
    xs = np.arange(0.25, 64.0, 0.5)
    expect = int((0.05 * np.abs(xs - 32.0) > 1.0).sum())
    assert expect == 2 * 24  # x < 12 or x > 52: 24 positions on each side
    assert run(xs, np.zeros(len(xs)), np.zeros(len(xs))) == expect
    # three steps: at rest the particles stay put, so each step counts them again
    assert run(xs, np.zeros(len(xs)), np.zeros(len(xs)), steps=3) == 3 * expect


def test_moving_particles_add_to_the_flow():
    # at x - 32 = +12 the flow is v_s = -0.6; u_y = -1 (v_y = -1/sqrt 2) makes |v| = 1.31,
    # u_y = +1 makes 0.11; at x - 32 = 0 no speed u'/gamma' < 1 ever counts
    x = [44.0, 44.0, 32.0, 32.0]
    uy = [-1.0, 1.0, 50.0, -50.0]
    assert run(x, [0.0] * 4, uy) == 1
    # a fast particle along x at x - 32 = +12: |v|^2 = v_x^2 + 0.36 with v_x -> 1 exceeds 1
    assert run([44.0], [20.0], [0.0]) == 1
    assert math.isclose(20.0 / math.sqrt(401.0), 0.99875, rel_tol=1e-4)
