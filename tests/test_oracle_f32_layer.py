"""Pins of the oracle's FP32 position-update layer (the integer layer the GPU's cell indices and
offsets are compared with bit for bit).

  * every axis follows the offset renormalisation of the FP32 path (s >= 1 -> next cell, s - 1
    exact; s < 0 -> previous cell, s + 1, or the same cell at 0 when s + 1 rounds to 1), and
    the FP64 position cell + offset moves by the displacement to FP32 rounding;
  * the shearing box adds the shear move of Sec. 2.2, y -= s Omega0 (x' + x^n)/2 dt: particles
    at rest move by -s Omega0 x dt in y, and a move of a whole cell or more is flagged, the
    bound that keeps the renormalisation valid;
  * an x-face crossing re-enters at the opposite face shifted by +Delta y_s(t^{n+1}) (through
    x_o) or -Delta y_s (through x_i), Sec. 2.1, with y wrapped periodically;
  * offsets within one ulp of 0 and 1.
"""
import numpy as np

import oracle


def _ulp_below_one():
    return np.nextafter(np.float32(1), np.float32(0))


def test_plain_move_follows_renormalisation_and_fp64_positions():
    rng = np.random.default_rng(600)
    n = (12, 10, 8)
    box = oracle.make_box(3, n, dt=0.45)
    m = 5000
    cell = rng.integers(0, 12 * 10 * 8, m).astype(np.int32)
    off = rng.uniform(0, 1, (3, m)).astype(np.float32)
    disp = rng.uniform(-0.49, 0.49, (3, m)).astype(np.float32)
    co, oo, err = oracle.f32_move(box, cell, off, disp)
    assert not err.any()
    i, j, k = cell % 12, (cell // 12) % 10, cell // 120
    ci, cj, ck = co % 12, (co // 12) % 10, co // 120
    for ax, (a, b, nn) in enumerate(((i, ci, 12), (j, cj, 10), (k, ck, 8))):
        # the renormalisation of the FP32 path on this axis (no wrap involved away from edges)
        ref_c, ref_o = oracle.f32_normalize(a, off[ax], disp[ax])
        np.testing.assert_array_equal(oo[ax], ref_o)
        np.testing.assert_array_equal(b, np.mod(ref_c, nn))
        assert np.all((oo[ax] >= 0) & (oo[ax] < 1))
        new = b + oo[ax].astype(np.float64)
        old = a + off[ax].astype(np.float64) + disp[ax].astype(np.float64)
        d = (new - old + nn / 2) % nn - nn / 2
        assert np.abs(d).max() < 2e-6


def test_shear_move_of_particles_at_rest_and_the_whole_cell_bound():
    n = (64, 16)
    s, om = 1.5, 0.05 / 1.5  # s Omega0 = 0.05: flows up to 1.6 c at the faces
    box = oracle.make_box(2, n, dt=0.45, frame=oracle.SHEAR, shear_s=s, omega0=om)
    xs = np.arange(0.25, 64.0, 0.5)
    m = len(xs)
    cell = (np.floor(xs) + 64 * 5).astype(np.int32)
    off = np.stack([xs - np.floor(xs), np.full(m, 0.5)]).astype(np.float32)
    disp = np.zeros((3, m), np.float32)
    co, oo, err = oracle.f32_move(box, cell, off, disp)
    dy = -0.45 * 0.05 * (xs - 32.0)  # v_s dt at the particle's own x (it does not move in x)
    y_new = (co // 64) + oo[1].astype(np.float64)
    ok = np.abs(dy) < 1.0
    np.testing.assert_allclose(y_new[ok], (5.5 + dy[ok]) % 16, rtol=0, atol=2e-6)
    np.testing.assert_array_equal(co[ok] % 64, np.floor(xs[ok]).astype(np.int32))
    # flagged exactly where the shear move reaches a whole cell: |x| >= 1/(0.45 * 0.05)
    np.testing.assert_array_equal(err.astype(bool), np.abs(dy) >= 1.0)
    assert err.sum() == 2 * np.sum(xs >= 32 + 1 / 0.0225)


def test_x_face_crossings_shift_y_by_the_shear_offset():
    n = (20, 12)
    box = oracle.make_box(2, n, dt=0.45, frame=oracle.SHEAR, shear_s=1.5, omega0=0.01)
    box.step = 37
    dys = oracle.shear_offset(box, (37 + 1) * 0.45)
    assert 0.1 < dys % 1 < 0.9
    sO = 0.015
    # out through x_o: cell 19, offset 0.9, D_x = 0.3; in through x_i: cell 0, offset 0.1,
    # D_x = -0.3; both at y = 4.25 with D_y = 0.05
    cell = np.array([19 + 20 * 4, 0 + 20 * 4], np.int32)
    off = np.array([[0.9, 0.1], [0.25, 0.25]], np.float32)
    disp = np.array([[0.3, -0.3], [0.05, 0.05], [0, 0]], np.float32)
    co, oo, err = oracle.f32_move(box, cell, off, disp)
    assert not err.any()
    x0 = np.array([19.9, 0.1]) - 10.0
    dy = 0.05 - 0.45 * sO * (x0 + np.array([0.15, -0.15]))  # v_s at the midpoint x
    x_new = (co % 20) + oo[0].astype(np.float64)
    y_new = (co // 20) + oo[1].astype(np.float64)
    np.testing.assert_allclose(x_new, [0.2, 19.8], atol=2e-6)
    np.testing.assert_allclose(y_new, [(4.25 + dy[0] + dys) % 12, (4.25 + dy[1] - dys) % 12],
                               atol=2e-6)


def test_offsets_within_one_ulp_of_the_cell_edges():
    box = oracle.make_box(2, (8, 8), dt=0.45)
    below1 = _ulp_below_one()
    tiny = np.float32(1e-30)
    ulp = np.float32(2.0 ** -24)
    cell = np.array([3 + 8 * 3] * 4, np.int32)
    off = np.array([[below1, below1, 0.0, 0.0], [0.5, 0.5, 0.5, 0.5]], np.float32)
    disp = np.array([[ulp, 0.0, -tiny, 0.0], [0, 0, 0, 0], [0, 0, 0, 0]], np.float32)
    co, oo, err = oracle.f32_move(box, cell, off, disp)
    assert not err.any()
    # 1 - 2^-24 + 2^-24 = 1.0 -> next cell at 0; unmoved stays; 0 - 1e-30 -> s + 1 rounds to 1
    # -> same cell at 0.0 (1.0 is never stored); 0 stays 0
    np.testing.assert_array_equal(co % 8, [4, 3, 3, 3])
    np.testing.assert_array_equal(oo[0], np.array([0.0, below1, 0.0, 0.0], np.float32))
    assert np.all(oo[0] < 1.0)
