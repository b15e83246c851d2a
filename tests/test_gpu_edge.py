"""Edge cases of the HIP path against the FP64 oracle or against the plain frame:
empty boxes (no particles: the fields follow the oracle's vacuum Maxwell steps), boxes smaller
than one tile (a single partial tile), the degenerate frames (shearing box with s = Omega0 = 0,
expanding box with adot = 0, the combined frame with both, which reduce to the plain push), and positions on cell edges (the
FP32 offset renormalisation never stores 1.0 and stays within 2e-6 cells of the oracle)."""
import numpy as np
import pytest
import torch

from _cases import Case, compare_particles, positions_f64, random_fields, wrap_diff
from paper_2602_15939_amd import _lib as L

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("dim,frame", [(2, "plain"), (2, "shear"), (3, "shear"), (3, "expand"),
                                       (2, "shear_expand"), (3, "shear_expand")])
def test_empty_box_fields_follow_oracle(dim, frame):
    n = (24, 20) if dim == 2 else (16, 12, 8)
    c = Case(dim, n, frame, ppc=0, seed=90 + dim)
    try:
        for _ in range(3):
            c.gpu.step()
            c.oracle_step()
        info = c.gpu.info()
        assert info.errors == 0 and list(info.n_particles) == [0, 0]
        E, B = (t.cpu().numpy() for t in c.gpu.get_fields())
        assert rel(E, c.E) < 1e-5 and rel(B, c.B) < 1e-5
        assert np.abs(c.gpu.get_current().cpu().numpy()).max() == 0.0
    finally:
        c.close()


@pytest.mark.parametrize("dim,n,frame", [(2, (10, 6), "shear"), (2, (12, 9), "leaky"),
                                         (3, (5, 6, 7), "plain"), (3, (7, 5, 6), "shear"),
                                         (2, (10, 6), "shear_expand"), (3, (7, 5, 6), "shear_expand")])
def test_box_smaller_than_one_tile(dim, n, frame):
    """Default tiles (16x16, 8^3) larger than the box: one partial tile holds everything."""
    c = Case(dim, n, frame, ppc=4, seed=70 + dim)
    try:
        for _ in range(2):
            c.gpu.step()
            c.oracle_step()
        for s in range(2):
            st = compare_particles(c, s, c.gpu_species(s))
            assert st["err_u"] < 2e-6 * 4 and st["err_x"] < 2e-6 * 4, st  # two steps
        assert rel(c.gpu.get_current().cpu().numpy(), c.J) < 1e-5
        info = c.gpu.info()
        assert info.errors & ~L.DERR_ORDER == 0 and info.n_slow == 0
    finally:
        c.close()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("frame,kw", [("shear", dict(shear_s=0.0, omega0=0.0)),
                                      ("expand", dict(adot=0.0)),
                                      ("shear_expand", dict(shear_s=0.0, omega0=0.0, adot=0.0))])
def test_degenerate_frame_equals_plain(dim, frame, kw):
    """With no shear and no rotation, or no expansion (the combined frame: neither), the
    frame's pusher is the Boris push:
    momenta, positions and the deposited current equal the plain box's after one step (FP32
    rounding of different formulas), and the expanding box's Maxwell step equals Yee's."""
    n = (40, 36) if dim == 2 else (20, 12, 16)
    fields = random_fields(tuple(list(n) + [1] * (3 - len(n))), 123)
    a = Case(dim, n, frame, ppc=4, seed=55, fields=fields, **kw)
    b = Case(dim, n, "plain", ppc=4, seed=55, fields=fields)
    try:
        a.gpu.step()
        b.gpu.step()
        for s in range(2):
            ga, gb = a.gpu_species(s), b.gpu_species(s)
            np.testing.assert_array_equal(ga["id"], gb["id"])
            ua, ub = ga["u"].astype(np.float64), gb["u"].astype(np.float64)
            du = np.linalg.norm(ua - ub, axis=0) / np.maximum(np.linalg.norm(ub, axis=0), 1e-2)
            assert du.max() < 2e-6, du.max()
            xa = positions_f64(ga["cell"], ga["off"], a.n, dim)
            xb = positions_f64(gb["cell"], gb["off"], b.n, dim)
            for d in range(dim):
                assert np.abs(wrap_diff(xa[d], xb[d], a.n[d])).max() < 2e-6, d
        assert rel(a.gpu.get_current().cpu().numpy(), b.gpu.get_current().cpu().numpy()) < 1e-5
        if frame == "expand":
            for fa, fb in zip(a.gpu.get_fields(), b.gpu.get_fields()):
                assert rel(fa.cpu().numpy(), fb.cpu().numpy()) < 1e-5
    finally:
        a.close()
        b.close()


def edge_parts(n_cells, seed):
    """Uncharged particles with offsets on or next to cell edges and momenta that move them by
    nothing, by less than half an FP32 ulp of 1 (so that s + 1 rounds to 1), or by up to 0.45
    cells, in both directions."""
    rng = np.random.default_rng(seed)
    dim = len(n_cells)
    offs = np.array([0.0, np.nextafter(np.float32(1), np.float32(0)), 0.5,
                     np.nextafter(np.float32(0.5), np.float32(0)), 2.0 ** -24, 0.25], np.float32)
    mags = np.array([0.0, 1e-8, 3e-8, 0.1, 0.6, 5.0])
    out = []
    for sp in range(2):
        m = len(offs) ** 2 * len(mags) * 4
        cell = rng.integers(0, int(np.prod(n_cells)), m).astype(np.int32)
        off = offs[rng.integers(0, len(offs), (dim, m))]
        u = (rng.choice([-1.0, 1.0], (3, m)) * mags[rng.integers(0, len(mags), (3, m))]).astype(np.float32)
        out.append(dict(cell=torch.from_numpy(cell), off=torch.from_numpy(off.astype(np.float32)),
                        u=torch.from_numpy(u)))
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_offsets_on_cell_edges(dim):
    n = (16, 16) if dim == 2 else (8, 8, 8)
    zero = (np.zeros((3, n[2] if dim == 3 else 1, n[1], n[0]), np.float32),) * 2
    c = Case(dim, n, "plain", parts=edge_parts(n, 17 + dim), fields=zero, q=0.0)
    try:
        for _ in range(3):
            c.gpu.step()
            c.oracle_step()
            for s in range(2):
                g = c.gpu_species(s)
                assert g["off"].min() >= 0.0 and g["off"].max() < 1.0
                st = compare_particles(c, s, g)
                assert st["err_x"] < 2e-6 and st["err_u"] == 0.0, st
        assert c.gpu.info().errors & ~L.DERR_ORDER == 0
    finally:
        c.close()
