"""A box of the particle hot path driven through the C ABI (include/pic.h).

PyTorch supplies device memory and the stream; every step of the path runs in the HIP
library.  By default a box lives in torch tensors (pic_box_mem: particle arrays, field and
current arrays, one workspace block), sized by pic_box_layout, and the library allocates
nothing for it; mem="library" lets the library allocate instead.  Field tensors at the
boundary are float32 of shape (3, nz, ny, nx) (x fastest); particle tensors follow the boundary
layout of pic.h: cell int32 (n,), off float32 (dim, n), u float32 (3, n).
"""
from __future__ import annotations

import torch

from . import _lib as L


def describe(dim, n, dt=0.45, frame=L.FRAME_PLAIN, species=((-1.0, -1e-3, 0),),
             shear_s=0.0, shear_omega0=0.0, expand_adot=0.0, expand_axis_mask=0,
             leaky_mode=L.LEAKY_DISPLACEMENT, leaky_l_esc=0.0, leaky_use_3vec=0,
             leaky_theta_inj=0.0, leaky_t_esc=0.0, leaky_gamma_thr=10.0, seed=0, box_id=0,
             tile=(0, 0, 0), maxwell_iters=8, maxwell_tol=0.0, track_ids=False,
             count_superluminal=False, escape=False, unfused=False, stream_ptr=0):
    """The pic_box_desc of a box (arguments as for Box)."""
    n = list(n) + [1] * (3 - len(n))
    d = L.pic_box_desc()
    d.dim = dim
    for k in range(3):
        d.n[k] = int(n[k])
        d.tile[k] = int(tile[k]) if k < len(tile) else 0
    d.dt, d.frame = dt, frame
    d.shear_s, d.shear_omega0 = shear_s, shear_omega0
    d.expand_adot, d.expand_axis_mask = expand_adot, expand_axis_mask
    d.leaky_mode, d.leaky_l_esc, d.leaky_use_3vec = leaky_mode, leaky_l_esc, leaky_use_3vec
    d.leaky_theta_inj, d.leaky_t_esc, d.leaky_gamma_thr = leaky_theta_inj, leaky_t_esc, leaky_gamma_thr
    d.n_species = len(species)
    for s, (qm, q, cap) in enumerate(species):
        d.q_over_m[s], d.q_macro[s], d.capacity[s] = qm, q, int(cap)
    d.seed, d.box_id = int(seed), int(box_id)
    d.maxwell_iters = maxwell_iters
    d.maxwell_tol = maxwell_tol
    d.flags = ((L.BOX_TRACK_IDS if track_ids else 0) |
               (L.BOX_COUNT_SUPERLUMINAL if count_superluminal else 0) |
               (L.BOX_ESCAPE if escape else 0) | (L.BOX_UNFUSED if unfused else 0))
    d.stream = stream_ptr
    return d


def footprint(desc, nsp=None) -> int:
    """Device bytes a box of this descriptor takes on caller memory (pic_box_layout): field
    and current arrays, both particle copies, workspace."""
    lay = L.pic_box_layout(desc)
    nsp = desc.n_species if nsp is None else nsp
    grid = 4 * lay.field_elems_min * (6 * lay.field_sets + 3 * lay.current_arrays)
    per = 4 + 4 * desc.dim + 12 + 4 * lay.has_id + 12 * lay.has_dr
    parts = sum(2 * lay.particle_elems[s] * per for s in range(nsp))
    return grid + parts + lay.workspace_bytes


class Box:
    def __init__(self, dim, n, stream=None, mem="caller", **kw):
        """kw: the descriptor (describe); species: sequence of (q_over_m, q_macro, capacity).
        mem: "caller" (torch tensors) or "library".  unfused=True reserves the record of unfused
        pushes (needed on caller memory for push(fuse=False), deposit() and
        get_push_record())."""
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        d = describe(dim, n, stream_ptr=stream.cuda_stream, **kw)
        n = list(n) + [1] * (3 - len(n))
        species = kw.get("species", ((-1.0, -1e-3, 0),))
        self.desc = d
        self.dim, self.n = dim, tuple(n)
        self.ncell = n[0] * n[1] * n[2]
        self.nsp = len(species)
        self.caller_mem = mem == "caller"
        self._tensors = []
        if self.caller_mem:
            m = self._caller_memory(d)
            # the library clears the field arrays on the box stream; torch made them on its own
            self._wait_for_torch()
            self.h = L.pic_box_create(d, m)
        else:
            self.h = L.pic_box_create(d)

    def _caller_memory(self, d) -> L.pic_box_mem:
        """Every buffer of the box as a torch tensor (pic_box_layout sizes them)."""
        lay = L.pic_box_layout(d)
        m = L.pic_box_mem()
        dev = torch.device("cuda")

        self.mem = {"field": [], "current": []}

        def take(nelem, dtype, role=None):
            t = torch.empty(max(int(nelem), 1), dtype=dtype, device=dev)
            assert t.data_ptr() % 256 == 0
            self._tensors.append(t)
            if role is not None:
                role.append(t)
            return t.data_ptr()

        m.field_pitch[0], m.field_pitch[1] = lay.field_pitch_min[0], lay.field_pitch_min[1]
        self.layout = lay
        for st in range(lay.field_sets):
            self.mem["field"].append([])
            for c in range(6):
                m.field[st][c] = take(lay.field_elems_min, torch.float32, self.mem["field"][-1])
        for a in range(lay.current_arrays):
            self.mem["current"].append([])
            for c in range(3):
                m.current[a][c] = take(lay.field_elems_min, torch.float32, self.mem["current"][-1])
        for sp in range(self.nsp):
            ne = lay.particle_elems[sp]
            for k in range(2):
                m.cell[sp][k] = take(ne, torch.int32)
                for c in range(self.dim):
                    m.off[sp][k][c] = take(ne, torch.float32)
                for c in range(3):
                    m.u[sp][k][c] = take(ne, torch.float32)
                if lay.has_id:
                    m.id[sp][k] = take(ne, torch.int32)
                if lay.has_dr:
                    for c in range(3):
                        m.dr[sp][k][c] = take(ne, torch.float32)
        m.workspace = take(lay.workspace_bytes, torch.uint8)
        m.workspace_bytes = lay.workspace_bytes
        self.device_bytes = sum(t.numel() * t.element_size() for t in self._tensors)
        return m

    # ---- stream ordering of caller buffers
    def _wait_for_torch(self):
        """Inputs made on torch's current stream must be ready before the box stream reads
        them (nothing to do when that is the box stream)."""
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _keep_until_stream(self, *tensors):
        """The library reads caller buffers asynchronously on the box stream: tell torch's
        allocator not to reuse them before that stream has passed this point."""
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)

    def interior(self, t):
        """The interior (nz, ny, nx) of one of this box's guarded field or current tensors (a
        view into the caller-owned memory, no copy)."""
        lay = self.layout
        py, pz = lay.field_pitch_min[0], lay.field_pitch_min[1]
        gz = 2 if self.dim == 3 else 0
        v = t[: pz * lay.field_planes].view(lay.field_planes, pz)[:, : py * (self.n[1] + 4)]
        v = v.reshape(lay.field_planes, self.n[1] + 4, py)
        return v[gz: gz + self.n[2], 2: 2 + self.n[1], 32: 32 + self.n[0]]

    # ---- lifetime
    def close(self):
        if getattr(self, "h", None):
            L.pic_box_destroy(self.h)  # synchronises the box stream: the buffers are free then
            self.h = None
        self._tensors = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state transfer
    def _grid(self):
        return torch.empty((3, self.n[2], self.n[1], self.n[0]), dtype=torch.float32, device="cuda")

    def set_fields(self, E, B):
        E = torch.as_tensor(E, dtype=torch.float32).cuda().contiguous()
        B = torch.as_tensor(B, dtype=torch.float32).cuda().contiguous()
        self._wait_for_torch()
        L.pic_set_fields(self.h, E.data_ptr(), B.data_ptr())
        self._keep_until_stream(E, B)

    def get_fields(self):
        E, B = self._grid(), self._grid()
        L.pic_get_fields(self.h, E.data_ptr(), B.data_ptr())
        return E, B

    def get_current(self):
        J = self._grid()
        L.pic_get_current(self.h, J.data_ptr())
        return J

    def set_particles(self, species, cell, off, u, ids=None, dr=None):
        cell = torch.as_tensor(cell, dtype=torch.int32).cuda().contiguous()
        off = torch.as_tensor(off, dtype=torch.float32).cuda().contiguous()
        u = torch.as_tensor(u, dtype=torch.float32).cuda().contiguous()
        n = cell.numel()
        assert off.shape == (self.dim, n) and u.shape == (3, n)
        ip = dp = None
        if ids is not None:
            ids = torch.as_tensor(ids, dtype=torch.int64).to(torch.int32).cuda().contiguous()
            ip = ids.data_ptr()
        if dr is not None:
            dr = torch.as_tensor(dr, dtype=torch.float32).cuda().contiguous()
            assert dr.shape == (3, n)
            dp = dr.data_ptr()
        self._wait_for_torch()
        L.pic_set_particles(self.h, species, n, cell.data_ptr(), off.data_ptr(), u.data_ptr(), ip, dp)
        self._keep_until_stream(cell, off, u, ids, dr)

    def count(self, species=0) -> int:
        return int(self.info().n_particles[species])

    def get_particles(self, species=0):
        n = self.count(species)
        cell = torch.empty(n, dtype=torch.int32, device="cuda")
        off = torch.empty((self.dim, n), dtype=torch.float32, device="cuda")
        u = torch.empty((3, n), dtype=torch.float32, device="cuda")
        ids = torch.empty(n, dtype=torch.int32, device="cuda")
        dr = torch.zeros((3, n), dtype=torch.float32, device="cuda")
        L.pic_get_particles(self.h, species, cell.data_ptr(), off.data_ptr(), u.data_ptr(),
                            ids.data_ptr(), dr.data_ptr())
        return dict(cell=cell, off=off, u=u, id=ids, dr=dr)

    def get_push_record(self, species=0):
        """Old cell, old offsets and FP32 deposit displacement of every particle of the last
        unfused push, in the slot order of get_particles."""
        n = self.count(species)
        cell = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        off = torch.empty((self.dim, max(n, 1)), dtype=torch.float32, device="cuda")
        disp = torch.empty((3, max(n, 1)), dtype=torch.float32, device="cuda")
        m = L.pic_get_push_record(self.h, species, cell.data_ptr(), off.data_ptr(), disp.data_ptr())
        assert m == n
        if n == 0:
            return dict(cell=cell[:0], off=off[:, :0], disp=disp[:, :0])
        return dict(cell=cell, off=off, disp=disp)

    def get_sort(self, species=0):
        """(perm, offsets) of the last tile sort: perm[i] = pre-sort index of sorted slot i."""
        import ctypes as C
        nt = C.c_int32()
        L.check(L.lib().pic_get_sort(self.h, species, None, None, C.byref(nt)), "pic_get_sort")
        off = torch.empty(nt.value + 1, dtype=torch.int32, device="cuda")
        L.pic_get_sort(self.h, species, None, off.data_ptr())
        n = int(off[-1].item())
        perm = torch.empty(max(1, n), dtype=torch.int32, device="cuda")
        L.pic_get_sort(self.h, species, perm.data_ptr(), None)
        return perm[:n], off

    # ---- the hot path
    def sort(self, overlap=False):
        """overlap: on the box's second stream, joined by the next particle or sort access."""
        L.pic_tile_sort([self.h], L.SORT_OVERLAP if overlap else 0)

    def push(self, fuse=True):
        L.pic_gather_push([self.h], L.FUSE_DEPOSIT if fuse else 0)

    def deposit(self):
        L.pic_deposit([self.h])

    def remap(self, what=L.REMAP_CURRENT | L.REMAP_FIELDS):
        L.pic_shear_remap([self.h], what)

    def maxwell(self):
        L.pic_maxwell_step([self.h])

    def escape_compact(self):
        L.pic_escape_compact([self.h])

    def step(self):
        L.pic_step([self.h])

    def autotune(self, batched=False, trials=3):
        """Pick the tile shape by timing the fused kernel on this machine's particles for every
        supported shape; returns (shape, {shape: ms})."""
        tile, ms = L.pic_autotune(self.h, L.TUNE_BATCHED if batched else 0, trials)
        shapes = L.pic_tile_candidates(self.dim, L.TUNE_BATCHED if batched else 0)
        return tile, dict(zip(shapes, ms))

    def info(self) -> L.pic_box_info:
        return L.pic_box_get(self.h)

    def set_step(self, step):
        """Resume at step n (after loading fields and particles from a checkpoint)."""
        L.pic_set_step(self.h, step)

    def energy_histogram(self, species, edges, static=False):
        """Counts of gamma - 1 over the edges: [below, bin 0 .. bin nbins-1, at/above].
        static=True uses the entry point that allocates nothing (static device scratch)."""
        self._wait_for_torch()
        return L.pic_energy_histogram(self.h, species, edges, static=static)


class Batch:
    """Staging of the batched step's argument tables in torch memory (a device tensor and a
    pinned host tensor): pic_batch.  It grows (a new pic_batch on larger tensors) when a step's
    tables exceed half of it; its HIP graphs are freed then."""

    def __init__(self, stream=None, nbytes=1 << 20):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = None
        self._alloc(nbytes)

    def _alloc(self, nbytes):
        self.close()
        nbytes = int(nbytes + 255) // 256 * 256
        self.dev = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.host = torch.empty(nbytes + 256, dtype=torch.uint8, pin_memory=True)
        hp = self.host.data_ptr()
        hp += (-hp) % 256
        assert self.dev.data_ptr() % 256 == 0
        self.nbytes = nbytes
        self.h = L.pic_batch_create(self.dev.data_ptr(), hp, nbytes, self.stream.cuda_stream)

    def step(self, boxes, graph=False):
        handles = [b.h for b in boxes]
        need = L.pic_step_table_bytes(handles)
        if 2 * need > self.nbytes:
            self._alloc(4 * need)
        flags = L.STEP_BATCHED | (L.STEP_GRAPH if graph else 0)
        L.check(L.pic_step_batch(self.h, handles, flags), "pic_step_batch")

    def close(self):
        if getattr(self, "h", None):
            L.pic_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_DEFAULT_BATCHES: dict = {}


def default_batch(stream) -> Batch:
    """A Batch per stream, kept for the process (its staging grows with the largest step)."""
    key = stream.cuda_stream
    if key not in _DEFAULT_BATCHES:
        _DEFAULT_BATCHES[key] = Batch(stream)
    return _DEFAULT_BATCHES[key]


def step_many(boxes, batched=True, graph=False, batch=None):
    """One whole step of several boxes sharing a stream: batched (one launch per kernel for all
    boxes, through box-descriptor tables; graph=True replays it as a captured HIP graph) or one
    box after another.  Boxes on caller memory take the batched step through a Batch (its
    staging in torch memory); library-owned boxes may use the first box's own staging."""
    if batched and (batch is not None or boxes[0].caller_mem):
        if batch is None:
            batch = default_batch(boxes[0].stream)
        batch.step(boxes, graph=graph)
        return
    flags = (L.STEP_BATCHED if batched else 0) | (L.STEP_GRAPH if graph else 0)
    L.pic_step([b.h for b in boxes], flags)
