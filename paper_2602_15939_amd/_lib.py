"""ctypes binding of the C ABI in include/pic.h (argument marshalling only).

The shared library is the in-tree ``libpic.so`` built by ``build.py``.  There is no
fallback: a missing or unloadable library raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EDEVICE, PIC_ESTATE, PIC_ECAP = 0, -1, -2, -3, -4, -5
FRAME_PLAIN, FRAME_SHEAR, FRAME_EXPAND, FRAME_LEAKY, FRAME_SHEAR_EXPAND = 0, 1, 2, 3, 4
LEAKY_DISPLACEMENT, LEAKY_PROBABILISTIC = 0, 1
FUSE_DEPOSIT = 1
REMAP_FIELDS, REMAP_CURRENT = 1, 2
BOX_TRACK_IDS = 1
BOX_COUNT_SUPERLUMINAL = 2
BOX_ESCAPE = 4
BOX_UNFUSED = 8
SORT_OVERLAP = 1
DERR_CFL, DERR_NAN, DERR_ORDER, DERR_CELL, DERR_SORT, DERR_NOCONVERGE = 1, 2, 4, 8, 16, 32
STEP_BATCHED = 1
STEP_GRAPH = 2
TUNE_BATCHED = 1


class pic_box_desc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32 * 3), ("dt", C.c_double), ("frame", C.c_int32),
        ("shear_s", C.c_double), ("shear_omega0", C.c_double),
        ("expand_adot", C.c_double), ("expand_axis_mask", C.c_int32),
        ("leaky_mode", C.c_int32), ("leaky_l_esc", C.c_double), ("leaky_use_3vec", C.c_int32),
        ("leaky_theta_inj", C.c_double), ("leaky_t_esc", C.c_double),
        ("leaky_gamma_thr", C.c_double),
        ("n_species", C.c_int32), ("q_over_m", C.c_double * 2), ("q_macro", C.c_double * 2),
        ("capacity", C.c_int64 * 2), ("seed", C.c_uint64), ("box_id", C.c_uint32),
        ("tile", C.c_int32 * 3), ("maxwell_iters", C.c_int32), ("maxwell_tol", C.c_double),
        ("flags", C.c_uint32),
        ("stream", C.c_void_p),
    ]


class pic_box_info(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("t", C.c_double), ("dys", C.c_double), ("a", C.c_double),
        ("n_particles", C.c_int64 * 2), ("errors", C.c_uint32), ("n_slow", C.c_int64),
        ("n_escaped", C.c_int64), ("field_energy_E", C.c_double * 3),
        ("field_energy_B", C.c_double * 3), ("kinetic_energy", C.c_double),
        ("momentum", C.c_double * 3),
        ("n_sort_migrations", C.c_int64), ("n_sort_fallbacks", C.c_int64), ("maxwell_sweeps", C.c_int32),
        ("pressure", C.c_double * 3), ("n_superluminal", C.c_int64),
        ("field_set", C.c_int32), ("current_array", C.c_int32), ("particle_copy", C.c_int32 * 2),
    ]


class pic_box_layout_info(C.Structure):
    _fields_ = [
        ("workspace_bytes", C.c_int64), ("field_sets", C.c_int32), ("current_arrays", C.c_int32),
        ("field_pitch_min", C.c_int32 * 2), ("field_rows", C.c_int32), ("field_planes", C.c_int32),
        ("field_elems_min", C.c_int64), ("particle_elems", C.c_int64 * 2), ("has_id", C.c_int32),
        ("has_dr", C.c_int32),
    ]


class pic_box_mem(C.Structure):
    _fields_ = [
        ("field", (C.c_void_p * 6) * 3), ("current", (C.c_void_p * 3) * 2),
        ("field_pitch", C.c_int32 * 2),
        ("cell", (C.c_void_p * 2) * 2), ("off", ((C.c_void_p * 3) * 2) * 2),
        ("u", ((C.c_void_p * 3) * 2) * 2), ("id", (C.c_void_p * 2) * 2),
        ("dr", ((C.c_void_p * 3) * 2) * 2),
        ("workspace", C.c_void_p), ("workspace_bytes", C.c_int64),
    ]


class PicError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libpic.so (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PicError(f"HIP library not built: {LIB_PATH} (run paper_2602_15939_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp, i32, u32, i64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_int64
        boxes = C.POINTER(C.c_void_p)
        sig = {
            "pic_box_create": ([C.POINTER(pic_box_desc), C.POINTER(pic_box_mem), C.POINTER(C.c_void_p)], i32),
            "pic_box_layout": ([C.POINTER(pic_box_desc), C.POINTER(pic_box_layout_info)], i32),
            "pic_workspace_bytes": ([C.POINTER(pic_box_desc), C.POINTER(i64)], i32),
            "pic_allocated_bytes": ([C.POINTER(i64), C.POINTER(i64)], i32),
            "pic_batch_create": ([vp, vp, i64, vp, C.POINTER(C.c_void_p)], i32),
            "pic_batch_destroy": ([vp], i32),
            "pic_step_batch": ([vp, boxes, i32, u32], i32),
            "pic_step_table_bytes": ([boxes, i32, C.POINTER(i64)], i32),
            "pic_box_destroy": ([vp], i32),
            "pic_set_fields": ([vp, vp, vp], i32),
            "pic_get_fields": ([vp, vp, vp], i32),
            "pic_get_current": ([vp, vp], i32),
            "pic_set_particles": ([vp, i32, i64, vp, vp, vp, vp, vp], i32),
            "pic_get_particles": ([vp, i32, C.POINTER(i64), vp, vp, vp, vp, vp], i32),
            "pic_get_sort": ([vp, i32, vp, vp, C.POINTER(i32)], i32),
            "pic_get_push_record": ([vp, i32, C.POINTER(i64), vp, vp, vp], i32),
            "pic_tile_sort": ([boxes, i32, u32], i32),
            "pic_gather_push": ([boxes, i32, u32], i32),
            "pic_deposit": ([boxes, i32, u32], i32),
            "pic_shear_remap": ([boxes, i32, u32], i32),
            "pic_maxwell_step": ([boxes, i32, u32], i32),
            "pic_escape_compact": ([boxes, i32, u32], i32),
            "pic_step": ([boxes, i32, u32], i32),
            "pic_box_get": ([vp, C.POINTER(pic_box_info)], i32),
            "pic_energy_histogram": ([vp, i32, C.POINTER(C.c_double), i32, C.POINTER(C.c_uint64)], i32),
            "pic_energy_histogram_static": ([vp, i32, C.POINTER(C.c_double), i32,
                                             C.POINTER(C.c_uint64)], i32),
            "pic_set_step": ([vp, i64], i32),
            "pic_autotune": ([vp, u32, i32, C.POINTER(i32), C.POINTER(C.c_float), i32,
                              C.POINTER(i32)], i32),
            "pic_tile_candidates": ([i32, u32, C.POINTER(i32), i32], i32),
            "pic_status_str": ([i32], C.c_char_p),
            "pic_device_copy": ([vp, vp, i64, vp], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(rc: int, what: str = "") -> None:
    if rc != PIC_OK:
        msg = lib().pic_status_str(rc).decode()
        raise PicError(f"{what}: {msg} ({rc})")


def box_array(handles):
    arr = (C.c_void_p * len(handles))(*handles)
    return C.cast(arr, C.POINTER(C.c_void_p)), arr


def pic_autotune(h, flags=0, trials=3):
    """(chosen tile shape, {candidate shape: ms}) of the tile-shape autotuner."""
    tile = (C.c_int32 * 3)()
    ms = (C.c_float * 8)()
    n = C.c_int32()
    check(lib().pic_autotune(h, flags, trials, tile, ms, 8, C.byref(n)), "pic_autotune")
    return tuple(tile), list(ms[: n.value])


def pic_tile_candidates(dim, flags=0):
    """Supported tile shapes, in the order pic_autotune reports its times."""
    out = (C.c_int32 * 24)()
    n = lib().pic_tile_candidates(dim, flags, out, 8)
    if n < 0:
        check(n, "pic_tile_candidates")
    return [tuple(out[3 * i: 3 * i + 3]) for i in range(n)]


def pic_device_copy(dst_ptr, src_ptr, nbytes, stream_ptr=None):
    check(lib().pic_device_copy(dst_ptr, src_ptr, nbytes, stream_ptr), "pic_device_copy")


def pic_box_create(desc: pic_box_desc, mem: pic_box_mem | None = None) -> int:
    """mem: caller-owned buffers (pic_box_mem), or None for library-allocated memory."""
    h = C.c_void_p()
    check(lib().pic_box_create(C.byref(desc), C.byref(mem) if mem is not None else None, C.byref(h)),
          "pic_box_create")
    return h.value


def pic_box_layout(desc: pic_box_desc) -> pic_box_layout_info:
    out = pic_box_layout_info()
    check(lib().pic_box_layout(C.byref(desc), C.byref(out)), "pic_box_layout")
    return out


def pic_workspace_bytes(desc: pic_box_desc) -> int:
    v = C.c_int64()
    check(lib().pic_workspace_bytes(C.byref(desc), C.byref(v)), "pic_workspace_bytes")
    return v.value


def pic_allocated_bytes():
    """(device, pinned host) bytes the library holds."""
    d, h = C.c_int64(), C.c_int64()
    check(lib().pic_allocated_bytes(C.byref(d), C.byref(h)), "pic_allocated_bytes")
    return d.value, h.value


def pic_batch_create(dev_ptr, host_ptr, nbytes, stream_ptr) -> int:
    h = C.c_void_p()
    check(lib().pic_batch_create(dev_ptr, host_ptr, nbytes, stream_ptr, C.byref(h)), "pic_batch_create")
    return h.value


def pic_batch_destroy(h) -> None:
    check(lib().pic_batch_destroy(h), "pic_batch_destroy")


def pic_step_batch(batch, handles, flags=0):
    p, keep = box_array(handles)
    rc = lib().pic_step_batch(batch, p, len(handles), flags)
    del keep
    return rc


def pic_step_table_bytes(handles) -> int:
    p, keep = box_array(handles)
    v = C.c_int64()
    check(lib().pic_step_table_bytes(p, len(handles), C.byref(v)), "pic_step_table_bytes")
    del keep
    return v.value


def pic_box_destroy(h) -> None:
    check(lib().pic_box_destroy(h), "pic_box_destroy")


def pic_set_fields(h, E_ptr, B_ptr):
    check(lib().pic_set_fields(h, E_ptr, B_ptr), "pic_set_fields")


def pic_get_fields(h, E_ptr, B_ptr):
    check(lib().pic_get_fields(h, E_ptr, B_ptr), "pic_get_fields")


def pic_get_current(h, J_ptr):
    check(lib().pic_get_current(h, J_ptr), "pic_get_current")


def pic_set_particles(h, species, n, cell, off, u, ids=None, dr=None):
    check(lib().pic_set_particles(h, species, n, cell, off, u, ids, dr), "pic_set_particles")


def pic_get_particles(h, species, cell, off, u, ids=None, dr=None) -> int:
    n = C.c_int64()
    check(lib().pic_get_particles(h, species, C.byref(n), cell, off, u, ids, dr),
          "pic_get_particles")
    return n.value


def pic_get_push_record(h, species, cell, off, disp) -> int:
    n = C.c_int64()
    check(lib().pic_get_push_record(h, species, C.byref(n), cell, off, disp), "pic_get_push_record")
    return n.value


def pic_get_sort(h, species, perm, offsets) -> int:
    nt = C.c_int32()
    check(lib().pic_get_sort(h, species, perm, offsets, C.byref(nt)), "pic_get_sort")
    return nt.value


def _batched(name):
    def call(handles, flags=0):
        p, keep = box_array(handles)
        check(getattr(lib(), name)(p, len(handles), flags), name)
        del keep
    call.__name__ = name
    return call


pic_tile_sort = _batched("pic_tile_sort")
pic_gather_push = _batched("pic_gather_push")
pic_deposit = _batched("pic_deposit")
pic_shear_remap = _batched("pic_shear_remap")
pic_maxwell_step = _batched("pic_maxwell_step")
pic_escape_compact = _batched("pic_escape_compact")
pic_step = _batched("pic_step")


def pic_box_get(h) -> pic_box_info:
    info = pic_box_info()
    check(lib().pic_box_get(h, C.byref(info)), "pic_box_get")
    return info


def pic_set_step(h, step):
    check(lib().pic_set_step(h, int(step)), "pic_set_step")


HIST_MAX_BINS = 4096
HIST_STATIC_MAX_BINS = 4096


def pic_energy_histogram(h, species, edges, static=False):
    """edges: nbins + 1 increasing floats; returns nbins + 2 counts (below, bins, at/above).
    static=True: the variant whose scratch is the library's static device array (no
    allocation)."""
    nb = len(edges) - 1
    e = (C.c_double * (nb + 1))(*[float(v) for v in edges])
    out = (C.c_uint64 * (nb + 2))()
    name = "pic_energy_histogram_static" if static else "pic_energy_histogram"
    check(getattr(lib(), name)(h, species, e, nb, out), name)
    return list(out)
