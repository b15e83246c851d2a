"""The tile sort after pushes (the neighbour-migration counting sort) against the oracle's stable
sort of the tile keys of the particles as they stand, bit for bit: permutation and offsets."""
import numpy as np
import pytest
import torch

import oracle
from _cases import Case, cell_coords
from paper_2602_15939_amd import _lib as L

pytestmark = pytest.mark.gpu


def current_keys(c, s, tile, n_upper):
    """tile keys of the particle arrays in slot order; dead (cell < 0) and slots past the live
    count of the last sort go to the dead bin n_tiles"""
    g = c.gpu.get_particles(s)
    cell = g["cell"].cpu().numpy().astype(np.int64)
    nt = 1
    for d in range(c.dim):
        nt *= c.n[d] // tile[d]
    i, j, k = cell_coords(np.maximum(cell, 0), c.n)
    keys = np.asarray(oracle.tile_keys(c.box, tile, i, j, k if c.dim == 3 else None), np.int64)
    keys[cell < 0] = nt
    out = np.full(n_upper, nt, np.int64)
    out[: len(keys)] = keys
    return out, nt


CASES = [
    ("plain3d", 3, (24, 24, 24), "plain", dict(), (8, 8, 8)),
    ("shear3d", 3, (24, 24, 32), "shear", dict(omega0=0.05), (8, 8, 8)),
    ("shear2d", 2, (64, 64), "shear", dict(omega0=0.02), (16, 16, 1)),
    ("expand2d", 2, (48, 64), "expand", dict(), (16, 16, 1)),
]


@pytest.mark.parametrize("name,dim,n,frame,kw,tile", CASES, ids=[c[0] for c in CASES])
def test_sort_after_push_bit_exact(name, dim, n, frame, kw, tile):
    c = Case(dim, n, frame, ppc=3, seed=70 + dim, theta=0.5, **kw)
    try:
        n_upper = [len(p["cell"]) for p in c.parts]
        for step in range(12):
            keys = [current_keys(c, s, tile, n_upper[s]) for s in range(2)]
            c.gpu.sort()
            for s in range(2):
                k, nt = keys[s]
                ref, roff = oracle.stable_sort(k, nt)
                perm, off = c.gpu.get_sort(s)
                np.testing.assert_array_equal(off.cpu().numpy(), roff[: nt + 1], err_msg=f"step {step}")
                np.testing.assert_array_equal(perm.cpu().numpy(), ref[: int(roff[nt])],
                                              err_msg=f"step {step}")
            c.gpu.push(fuse=True)
            c.gpu.remap(L.REMAP_CURRENT)
            c.gpu.maxwell()
        info = c.gpu.info()
        assert info.n_sort_migrations == 2 * 11
        assert info.n_sort_fallbacks == 0
        assert info.errors & ~L.DERR_ORDER == 0 and info.n_slow == 0
    finally:
        c.close()


def test_sort_after_push_with_escapes():
    """probabilistic escape on a 64x64 grid of 16x16 tiles: the particles that died go to the
    dead bin after the survivors, the previous dead bin stays at the end"""
    rng = np.random.default_rng(5)
    dims = (64, 64)
    parts = []
    for g in (20.0, 3.0):
        v = rng.normal(size=(3, 5000))
        v /= np.linalg.norm(v, axis=0)
        parts.append(dict(cell=torch.from_numpy(rng.integers(0, 64 * 64, 5000).astype(np.int32)),
                          off=torch.from_numpy(rng.uniform(0, 1, (2, 5000)).astype(np.float32)),
                          u=torch.from_numpy((np.sqrt(g * g - 1) * v).astype(np.float32))))
    zero = (np.zeros((3, 1, 64, 64), np.float32), np.zeros((3, 1, 64, 64), np.float32))
    c = Case(2, dims, "leaky", parts=parts, fields=zero, q=0.0, leaky_mode=L.LEAKY_PROBABILISTIC,
             t_esc=0.45 / 0.05, gamma_thr=10.0)
    tile = (16, 16, 1)
    try:
        for step in range(8):
            keys = [current_keys(c, s, tile, 5000) for s in range(2)]
            c.gpu.escape_compact()
            for s in range(2):
                k, nt = keys[s]
                ref, roff = oracle.stable_sort(k, nt)
                perm, off = c.gpu.get_sort(s)
                np.testing.assert_array_equal(off.cpu().numpy(), roff[: nt + 1])
                np.testing.assert_array_equal(perm.cpu().numpy(), ref[: int(roff[nt])])
            c.gpu.push(fuse=True)
            c.gpu.remap(L.REMAP_CURRENT)
            c.gpu.maxwell()
        info = c.gpu.info()
        assert info.n_particles[0] < 5000 and info.n_particles[1] == 5000
        assert info.n_sort_migrations == 2 * 7 and info.n_sort_fallbacks == 0
    finally:
        c.close()


@pytest.mark.parametrize("dim,n,frame,kw", [
    (3, (32, 32, 32), "shear", dict(omega0=0.03)),
    (2, (64, 48), "leaky", dict(leaky_mode=L.LEAKY_PROBABILISTIC, t_esc=4.0, gamma_thr=1.3)),
])
def test_overlapped_sort_equals_plain_sort(dim, n, frame, kw):
    """PIC_SORT_OVERLAP (the sort for the next step on the box's second stream, overlapping the
    current fold and Maxwell step) gives the same particles after every push, and the same
    permutation and tile offsets, as the sort queued on the box stream before each push."""
    from test_gpu_batched import assert_same_state

    a = Case(dim, n, frame, ppc=4, theta=0.4, seed=71, **kw)
    b = Case(dim, n, frame, ppc=4, theta=0.4, seed=71, **kw)
    try:
        b.gpu.sort()
        for _ in range(6):
            a.gpu.sort()
            a.gpu.push()
            a.gpu.remap(L.REMAP_CURRENT)
            a.gpu.maxwell()
            b.gpu.push()
            b.gpu.sort(overlap=True)
            b.gpu.remap(L.REMAP_CURRENT)
            b.gpu.maxwell()
        a.gpu.sort()  # b has sorted for its next push already
        for s in range(2):
            pa, oa = a.gpu.get_sort(s)
            pb, ob = b.gpu.get_sort(s)
            assert torch.equal(oa, ob) and torch.equal(pa, pb), s
        assert_same_state(a, b, "overlap")
        assert b.gpu.info().n_sort_migrations > 0
    finally:
        a.close()
        b.close()


def test_overlapped_sort_then_whole_steps_and_batched_step():
    """Calls that sort or step again after an overlapped sort wait for it: a box sorted on its
    second stream and then stepped (alone, then batched with a twin) ends like the box sorted
    on its own stream."""
    from test_gpu_batched import assert_same_state
    from paper_2602_15939_amd.box import step_many

    a = Case(3, (24, 24, 24), "shear", ppc=3, theta=0.4, seed=73, omega0=0.03)
    b = Case(3, (24, 24, 24), "shear", ppc=3, theta=0.4, seed=73, omega0=0.03)
    try:
        a.gpu.sort()
        b.gpu.sort(overlap=True)
        a.gpu.step()
        b.gpu.step()
        a.gpu.sort()
        b.gpu.sort(overlap=True)
        a.gpu.push()
        b.gpu.push()
        a.gpu.sort()
        b.gpu.sort(overlap=True)
        step_many([a.gpu], batched=True)
        step_many([b.gpu], batched=True)
        assert_same_state(a, b, "overlap then step")
    finally:
        a.close()
        b.close()
