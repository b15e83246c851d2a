"""Boxes on caller-owned memory (torch tensors, pic_box_mem): the library allocates nothing for
them through a whole workload of calls (creation, loading, whole and batched steps, graph
replay, unfused pushes with their record, the overlapped sort, the autotuner, histograms,
reductions), the fields and currents sit in the caller's tensors where pic_box_info says, a
batch whose staging is too small refuses the step and leaves every box unchanged, and the
library-owned path holds exactly its boxes' memory until they are destroyed."""
import numpy as np
import pytest
import torch

from _cases import Case
from paper_2602_15939_amd import _lib as L
from paper_2602_15939_amd.box import Batch, step_many

pytestmark = pytest.mark.gpu

EDGES = list(np.concatenate([[0.0], np.logspace(-4, 1, 30)]))


def _mix(mem, stream=None):
    return [
        Case(3, (16, 16, 16), "shear", ppc=2, seed=801, tile=(8, 8, 8), mem=mem, stream=stream),
        Case(2, (32, 32), "leaky", ppc=4, seed=802, tile=(8, 8, 1), mem=mem, stream=stream,
             leaky_mode=L.LEAKY_DISPLACEMENT, l_esc=2.0, theta_inj=0.3),
        Case(2, (32, 48), "expand", ppc=3, seed=803, tile=(16, 16, 1), mem=mem, stream=stream),
    ]


def test_caller_memory_allocates_nothing():
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        batch = Batch(st, nbytes=1 << 20)
        torch.cuda.synchronize()
        before = L.pic_allocated_bytes()
        mix = _mix("caller", st)
        try:
            for c in mix:
                c.gpu.step()
            for k in range(4):
                step_many([c.gpu for c in mix], batched=True, batch=batch, graph=k >= 2)
            for c in mix:
                c.gpu.sort(overlap=True)
                c.gpu.push(fuse=False)
                rec = c.gpu.get_push_record(0)
                assert rec["cell"].numel() == c.gpu.count(0)
                c.gpu.deposit()
                c.gpu.remap()
                c.gpu.maxwell()
                c.gpu.energy_histogram(0, EDGES)
                c.gpu.energy_histogram(1, EDGES, static=True)
            mix[1].gpu.autotune(trials=1)
            mix[1].gpu.step()
            for c in mix:
                info = c.gpu.info()
                assert info.errors & ~L.DERR_ORDER == 0
            torch.cuda.synchronize()
            assert L.pic_allocated_bytes() == before
        finally:
            for c in mix:
                c.close()
            batch.close()
        assert L.pic_allocated_bytes() == before


def test_fields_and_current_are_read_in_place():
    """After steps, the caller's tensors of the field set and current array pic_box_info names
    hold what pic_get_fields / pic_get_current copy out (the shearing box rotates three field
    sets and two current arrays)."""
    c = Case(2, (40, 36), "shear", ppc=3, seed=810)
    try:
        for k in range(5):
            c.gpu.step()
            info = c.gpu.info()
            E, B = (t.cpu() for t in c.gpu.get_fields())
            J = c.gpu.get_current().cpu()
            fs = c.gpu.mem["field"][info.field_set]
            cur = c.gpu.mem["current"][info.current_array]
            for comp in range(3):
                assert torch.equal(c.gpu.interior(fs[comp]).cpu(), B[comp])
                assert torch.equal(c.gpu.interior(fs[3 + comp]).cpu(), E[comp])
                assert torch.equal(c.gpu.interior(cur[comp]).cpu(), J[comp])
        assert c.gpu.info().field_set in (0, 1, 2)
    finally:
        c.close()


def test_too_small_staging_refuses_the_step_and_keeps_the_boxes():
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        mix = _mix("caller", st)
        ref = _mix("caller", st)
        tiny = Batch(st, nbytes=8192)
        big = Batch(st, nbytes=1 << 20)
        try:
            handles = [c.gpu.h for c in mix]
            need = L.pic_step_table_bytes(handles)
            assert need > 4096
            before = [c.gpu.info().step for c in mix]
            rc = L.pic_step_batch(tiny.h, handles, L.STEP_BATCHED)
            assert rc == L.PIC_ENOMEM
            assert [c.gpu.info().step for c in mix] == before
            # the refused step changed nothing: the same boxes now step like an untouched twin
            # (particles bit for bit: the same fields pushed them; fields within the rounding
            # of the float atomics that flush the tile-halo current in a run-dependent order)
            L.check(L.pic_step_batch(big.h, handles, L.STEP_BATCHED), "pic_step_batch")
            L.check(L.pic_step_batch(big.h, [c.gpu.h for c in ref], L.STEP_BATCHED), "pic_step_batch")
            st.synchronize()
            for a, b in zip(mix, ref):
                assert a.gpu.info().step == b.gpu.info().step == 1
                for s in range(2):
                    ga, gb = a.gpu_species(s), b.gpu_species(s)
                    for k in ("cell", "off", "u", "id"):
                        np.testing.assert_array_equal(ga[k], gb[k])
                for fa, fb in zip(a.gpu.get_fields(), b.gpu.get_fields()):
                    fa, fb = fa.cpu().numpy(), fb.cpu().numpy()
                    assert np.abs(fa - fb).max() <= 1e-6 * np.abs(fb).max()
        finally:
            for c in mix + ref:
                c.close()
            tiny.close()
            big.close()


def test_library_owned_boxes_hold_their_memory_until_destroyed():
    torch.cuda.synchronize()
    d0, h0 = L.pic_allocated_bytes()
    mix = _mix("library")
    try:
        d1, _ = L.pic_allocated_bytes()
        assert d1 > d0
        step_many([c.gpu for c in mix], batched=True)  # the first box grows its staging
        d2, h2 = L.pic_allocated_bytes()
        assert d2 > d1 and h2 > h0
    finally:
        for c in mix:
            c.close()
    assert L.pic_allocated_bytes() == (d0, h0)
