"""FP64 CPU oracle of the particle hot path (test infrastructure).

A plain C implementation of the paper's equations (Bacchini et al., arXiv
2602.15939), compiled with gcc and loaded through ctypes.  Only the test suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package; the HIP product path never does and shares no code with it.

Arrays: fields are float64 numpy arrays of shape (3, nz, ny, nx) (x fastest);
particle arrays are float64 of shape (n,).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libpic_oracle.so")

PLAIN, SHEAR, EXPAND, LEAKY, SHEAR_EXPAND = 0, 1, 2, 3, 4
# axis masks of the combined shearing and expanding frame: x and y scale together
SHEAR_EXPAND_MASKS = (0b000, 0b100, 0b011, 0b111)
LEAKY_DISPLACEMENT, LEAKY_PROBABILISTIC = 0, 1
JG = 3  # x guard columns of the extended current grid


def build(force: bool = True) -> str:
    """Compile the oracle library (gcc, FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Box(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n", C.c_int * 3), ("dt", C.c_double), ("frame", C.c_int),
        ("shear_s", C.c_double), ("omega0", C.c_double),
        ("adot", C.c_double), ("axis_mask", C.c_int), ("expand_push", C.c_int),
        ("leaky_mode", C.c_int), ("l_esc", C.c_double), ("use_3vec", C.c_int),
        ("t_esc", C.c_double), ("gamma_thr", C.c_double), ("reinject", C.c_int),
        ("seed", C.c_uint64), ("box_id", C.c_uint32),
        ("mj_table", C.POINTER(C.c_double)), ("mj_bins", C.c_int), ("mj_tail", C.c_int),
        ("maxwell_iters", C.c_int), ("maxwell_tol", C.c_double),
        ("step", C.c_int64), ("last_iters", C.c_int), ("n_superluminal", C.c_int64),
        ("escape", C.c_int),
    ]


class Species(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("q_over_m", C.c_double), ("q", C.c_double),
        ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)), ("z", C.POINTER(C.c_double)),
        ("ux", C.POINTER(C.c_double)), ("uy", C.POINTER(C.c_double)), ("uz", C.POINTER(C.c_double)),
        ("drx", C.POINTER(C.c_double)), ("dry", C.POINTER(C.c_double)), ("drz", C.POINTER(C.c_double)),
        ("id", C.POINTER(C.c_uint32)), ("alive", C.POINTER(C.c_uint8)),
    ]


class Fields(C.Structure):
    _fields_ = [("E", C.POINTER(C.c_double) * 3), ("B", C.POINTER(C.c_double) * 3),
                ("J", C.POINTER(C.c_double) * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.ora_shear_offset.restype = C.c_double
        L.ora_shear_offset.argtypes = [C.POINTER(Box), C.c_double]
        L.ora_scale.restype = C.c_double
        L.ora_scale.argtypes = [C.POINTER(Box), C.c_int, C.c_double]
        L.ora_shear_gamma_bar.restype = C.c_double
        L.ora_shear_gamma_bar.argtypes = [C.c_double, C.c_double]
        L.ora_mj_table.argtypes = [C.c_double, C.c_int, C.c_int, dp]
        L.ora_mj_sample.argtypes = [dp, C.c_int, C.c_int, C.POINTER(C.c_uint32), dp]
        L.ora_step.restype = C.c_int
        _lib = L
    return _lib


def _p(a, ctype=C.c_double):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "array must be contiguous"
    return a.ctypes.data_as(C.POINTER(ctype))


def make_box(dim, n, dt=0.45, frame=PLAIN, shear_s=0.0, omega0=0.0, adot=0.0, axis_mask=0,
             expand_push=0, leaky_mode=LEAKY_DISPLACEMENT, l_esc=0.0, use_3vec=0, t_esc=0.0,
             gamma_thr=10.0, seed=0, box_id=0, mj_table=None, maxwell_iters=8, maxwell_tol=0.0,
             step=0, escape=False) -> Box:
    n = list(n) + [1] * (3 - len(n))
    if frame == SHEAR_EXPAND and axis_mask not in SHEAR_EXPAND_MASKS:
        raise ValueError("the combined frame scales x and y together: axis_mask 0, 4, 3 or 7")
    b = Box()
    b.dim = dim
    for d in range(3):
        b.n[d] = int(n[d])
    b.dt, b.frame = dt, frame
    b.shear_s, b.omega0 = shear_s, omega0
    b.adot, b.axis_mask, b.expand_push = adot, axis_mask, expand_push
    b.leaky_mode, b.l_esc, b.use_3vec = leaky_mode, l_esc, use_3vec
    b.t_esc, b.gamma_thr, b.reinject = t_esc, gamma_thr, 0
    b.seed, b.box_id = seed, box_id
    if mj_table is not None:
        tab = np.ascontiguousarray(mj_table, dtype=np.float64)
        b._mj_keep = tab  # keep alive
        b.mj_table = _p(tab)
        b.mj_bins, b.mj_tail = MJ_BINS, len(tab) - MJ_BINS
    b.maxwell_iters, b.maxwell_tol = maxwell_iters, maxwell_tol
    b.step = step
    b.escape = 1 if escape else 0
    return b


def shear_offset(box: Box, t: float) -> float:
    return lib().ora_shear_offset(C.byref(box), t)


def scale(box: Box, axis: int, t: float) -> float:
    return lib().ora_scale(C.byref(box), axis, t)


def field_shape(box: Box):
    return (3, box.n[2], box.n[1], box.n[0])


def zeros_fields(box: Box):
    return (np.zeros(field_shape(box)), np.zeros(field_shape(box)), np.zeros(field_shape(box)))


def _fields(E, B, J):
    f = Fields()
    for c in range(3):
        f.E[c] = _p(E[c])
        f.B[c] = _p(B[c])
        f.J[c] = _p(J[c])
    return f


class SpeciesState:
    """One species in FP64 for the oracle: global positions and momenta."""

    def __init__(self, x, y, z, ux, uy, uz, q_over_m, q, ids=None, dr=None, alive=None):
        n = len(x)
        f64 = lambda a: np.array(a, dtype=np.float64, copy=True)  # never alias the caller's arrays
        self.x, self.y = f64(x), f64(y)
        self.z = f64(z if z is not None else np.zeros(n))
        self.ux, self.uy, self.uz = f64(ux), f64(uy), f64(uz)
        self.q_over_m, self.q = float(q_over_m), float(q)
        self.id = np.array(ids if ids is not None else np.arange(n), dtype=np.uint32, copy=True)
        self.dr = f64(dr if dr is not None else np.zeros((3, n)))
        self.alive = np.array(alive if alive is not None else np.ones(n), dtype=np.uint8, copy=True)

    def cstruct(self) -> Species:
        s = Species()
        s.n = len(self.x)
        s.q_over_m, s.q = self.q_over_m, self.q
        s.x, s.y, s.z = _p(self.x), _p(self.y), _p(self.z)
        s.ux, s.uy, s.uz = _p(self.ux), _p(self.uy), _p(self.uz)
        s.drx, s.dry, s.drz = _p(self.dr[0]), _p(self.dr[1]), _p(self.dr[2])
        s.id = _p(self.id, C.c_uint32)
        s.alive = _p(self.alive, C.c_uint8)
        return s

    def copy(self):
        return SpeciesState(self.x.copy(), self.y.copy(), self.z.copy(), self.ux.copy(),
                            self.uy.copy(), self.uz.copy(), self.q_over_m, self.q, self.id.copy(),
                            self.dr.copy(), self.alive.copy())


def step(box: Box, E, B, J, species, nthreads: int = 1) -> None:
    """One full step of the box frame (updates E, B, J, species and box.step in place)."""
    f = _fields(E, B, J)
    arr = (Species * len(species))(*[s.cstruct() for s in species])
    rc = lib().ora_step(C.byref(box), C.byref(f), arr, len(species), nthreads)
    assert rc == 0


def particles_only(box: Box, E, B, species) -> None:
    """gather + push + move (+ leaky escape) of the species, without deposit or Maxwell"""
    J = np.zeros(field_shape(box))
    f = _fields(E, B, J)
    arr = (Species * len(species))(*[s.cstruct() for s in species])
    rc = lib().ora_particles_only(C.byref(box), C.byref(f), arr, len(species))
    assert rc == 0


def gather(box: Box, E, B, x, y, z=None, dys=0.0):
    n = len(x)
    Eo, Bo = np.zeros((n, 3)), np.zeros((n, 3))
    J = np.zeros(field_shape(box))
    f = _fields(E, B, J)
    x, y = np.ascontiguousarray(x, float), np.ascontiguousarray(y, float)
    z = np.ascontiguousarray(z if z is not None else np.zeros(n), float)
    lib().ora_gather(C.byref(box), C.byref(f), C.c_double(dys), C.c_int64(n), _p(x), _p(y), _p(z),
                     _p(Eo), _p(Bo))
    return Eo, Bo


def push_boris(qm, dt, E, B, u):
    u = np.ascontiguousarray(u, float).copy()
    E, B = np.ascontiguousarray(E, float), np.ascontiguousarray(B, float)
    lib().ora_push_boris(C.c_int64(len(u)), C.c_double(qm), C.c_double(dt), _p(E), _p(B), _p(u))
    return u


def push_shear(qm, dt, s, omega0, xr, E, B, u, return_gbar=False):
    u = np.ascontiguousarray(u, float).copy()
    E, B = np.ascontiguousarray(E, float), np.ascontiguousarray(B, float)
    xr = np.ascontiguousarray(xr, float)
    gb = np.zeros(len(u))
    lib().ora_push_shear(C.c_int64(len(u)), C.c_double(qm), C.c_double(dt), C.c_double(s),
                         C.c_double(omega0), _p(xr), _p(E), _p(B), _p(u), _p(gb))
    return (u, gb) if return_gbar else u


def push_expand(qm, dt, lam, E, B, u, exact=False):
    u = np.ascontiguousarray(u, float).copy()
    E, B = np.ascontiguousarray(E, float), np.ascontiguousarray(B, float)
    lam = np.ascontiguousarray(lam, float)
    lib().ora_push_expand(C.c_int64(len(u)), C.c_double(qm), C.c_double(dt), _p(lam),
                          C.c_int(1 if exact else 0), _p(E), _p(B), _p(u))
    return u


def push_shear_expand(qm, dt, s, omega0, lam, xr, E, B, u, exact=False, return_gbar=False):
    u = np.ascontiguousarray(u, float).copy()
    E, B = np.ascontiguousarray(E, float), np.ascontiguousarray(B, float)
    xr = np.ascontiguousarray(xr, float)
    lam = np.ascontiguousarray(lam, float)
    gb = np.zeros(len(u))
    lib().ora_push_shear_expand(C.c_int64(len(u)), C.c_double(qm), C.c_double(dt), C.c_double(s),
                                C.c_double(omega0), _p(lam), C.c_int(1 if exact else 0), _p(xr),
                                _p(E), _p(B), _p(u), _p(gb))
    return (u, gb) if return_gbar else u


def shear_gamma_bar(A, K):
    return lib().ora_shear_gamma_bar(float(A), float(K))


def jext_shape(box: Box):
    return (3, box.n[2], box.n[1], box.n[0] + 2 * JG)


def deposit(box: Box, q, x0, y0, x1, y1, z0=None, z1=None, dz=None, Jext=None):
    n = len(x0)
    if Jext is None:
        Jext = np.zeros(jext_shape(box))
    arrs = [np.ascontiguousarray(a if a is not None else np.zeros(n), float)
            for a in (x0, y0, z0, x1, y1, z1, dz)]
    lib().ora_deposit(C.byref(box), C.c_int64(n), C.c_double(q), *[_p(a) for a in arrs], _p(Jext))
    return Jext


def finalize_current(box: Box, Jext, t_half):
    J = np.zeros(field_shape(box))
    Jext = np.ascontiguousarray(Jext, float)
    lib().ora_finalize_current(C.byref(box), _p(Jext), _p(J), C.c_double(t_half))
    return J


def maxwell(box: Box, E, B, J):
    f = _fields(E, B, J)
    lib().ora_maxwell(C.byref(box), C.byref(f))


def ksb_rhs(box: Box, E, B, J, dys=0.0):
    out = np.zeros((6,) + field_shape(box)[1:])
    Ea = (C.POINTER(C.c_double) * 3)(*[_p(E[c]) for c in range(3)])
    Ba = (C.POINTER(C.c_double) * 3)(*[_p(B[c]) for c in range(3)])
    Ja = (C.POINTER(C.c_double) * 3)(*[_p(J[c]) for c in range(3)])
    Oa = (C.POINTER(C.c_double) * 6)(*[_p(out[c]) for c in range(6)])
    lib().ora_ksb_rhs(C.byref(box), Ea, Ba, C.c_double(dys), Ja, Oa)
    return out


def ksb_rhs_f(box: Box, E, B, J, d, kz, dys=0.0):
    """The shearing-box right-hand side with the combined frame's factors: the curls act on
    d_c F_c, kz multiplies v dE'y/dz in dE'z/dt."""
    out = np.zeros((6,) + field_shape(box)[1:])
    Ea = (C.POINTER(C.c_double) * 3)(*[_p(E[c]) for c in range(3)])
    Ba = (C.POINTER(C.c_double) * 3)(*[_p(B[c]) for c in range(3)])
    Ja = (C.POINTER(C.c_double) * 3)(*[_p(J[c]) for c in range(3)])
    Oa = (C.POINTER(C.c_double) * 6)(*[_p(out[c]) for c in range(6)])
    dd = np.ascontiguousarray(d, float)
    lib().ora_ksb_rhs_f(C.byref(box), Ea, Ba, C.c_double(dys), Ja, _p(dd), C.c_double(kz), Oa)
    return out


def charge(box: Box, q, x, y, z=None, rho=None):
    if rho is None:
        rho = np.zeros(field_shape(box)[1:])
    n = len(x)
    x, y = np.ascontiguousarray(x, float), np.ascontiguousarray(y, float)
    z = np.ascontiguousarray(z if z is not None else np.zeros(n), float)
    lib().ora_charge(C.byref(box), C.c_int64(n), C.c_double(q), _p(x), _p(y), _p(z), _p(rho))
    return rho


def philox(ctr, key):
    """Philox4x32-10 of counters (n,4) under keys (n,2) -> (n,4) uint32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(np.broadcast_to(np.asarray(key, np.uint32), (len(ctr), 2)))
    out = np.zeros_like(ctr)
    lib().ora_philox_many(C.c_int64(len(ctr)), _p(ctr, C.c_uint32), _p(key, C.c_uint32),
                          _p(out, C.c_uint32))
    return out


MJ_BINS, MJ_TAIL = 4096, 64


def mj_table(theta):
    """bulk inverse-CDF table (MJ_BINS values) followed by the tail table (MJ_TAIL more)"""
    tab = np.zeros(MJ_BINS + MJ_TAIL)
    lib().ora_mj_table(float(theta), MJ_BINS, MJ_TAIL, _p(tab))
    return tab


def mj_sample(table, words):
    words = np.ascontiguousarray(words, dtype=np.uint32).reshape(-1, 4)
    table = np.ascontiguousarray(table, float)
    out = np.zeros((len(words), 3))
    for p in range(len(words)):
        lib().ora_mj_sample(_p(table), MJ_BINS, len(table) - MJ_BINS, _p(words[p], C.c_uint32),
                            _p(out[p]))
    return out


def stable_sort(keys, nkeys):
    keys = np.ascontiguousarray(keys, dtype=np.int32)
    perm = np.zeros(len(keys), dtype=np.int64)
    off = np.zeros(nkeys + 2, dtype=np.int64)
    lib().ora_stable_sort(C.c_int64(len(keys)), _p(keys, C.c_int32), C.c_int32(nkeys),
                          _p(perm, C.c_int64), _p(off, C.c_int64))
    return perm[: off[nkeys]], off


def tile_keys(box: Box, tile, ci, cj, ck=None):
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    cj = np.ascontiguousarray(cj, dtype=np.int32)
    ckp = _p(np.ascontiguousarray(ck, dtype=np.int32), C.c_int32) if ck is not None else None
    t = (C.c_int * 3)(*list(tile) + [1] * (3 - len(tile)))
    keys = np.zeros(len(ci), dtype=np.int32)
    lib().ora_tile_keys(C.byref(box), t, C.c_int64(len(ci)), _p(ci, C.c_int32), _p(cj, C.c_int32),
                        ckp, _p(keys, C.c_int32))
    return keys


def f32_normalize(cell, off, delta):
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    off = np.ascontiguousarray(off, dtype=np.float32)
    delta = np.ascontiguousarray(delta, dtype=np.float32)
    co = np.zeros_like(cell)
    oo = np.zeros_like(off)
    lib().ora_f32_normalize(C.c_int64(len(cell)), _p(cell, C.c_int32), _p(off, C.c_float),
                            _p(delta, C.c_float), _p(co, C.c_int32), _p(oo, C.c_float))
    return co, oo


def f32_move(box: Box, cell, off, disp):
    """FP32 position update of the integer layer: (cell, off) moved by the FP32 deposit
    displacement disp (3, n) with the frame's shear move and boundaries at t^{n+1} =
    (box.step + 1) dt.  Returns (cell_out, off_out, err)."""
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    n = len(cell)
    off = np.ascontiguousarray(off, dtype=np.float32).reshape(box.dim, n)
    disp = np.ascontiguousarray(disp, dtype=np.float32).reshape(3, n)
    co = np.zeros_like(cell)
    oo = np.zeros_like(off)
    err = np.zeros(n, dtype=np.uint8)
    lib().ora_f32_move(C.byref(box), C.c_int64(n), _p(cell, C.c_int32), _p(off, C.c_float),
                       _p(disp, C.c_float), _p(co, C.c_int32), _p(oo, C.c_float),
                       _p(err, C.c_uint8))
    return co, oo, err


def energies(box: Box, E, B, J, species):
    f = _fields(E, B, J)
    arr = (Species * len(species))(*[s.cstruct() for s in species])
    out = np.zeros(11)
    lib().ora_energies(C.byref(box), C.byref(f), arr, len(species), _p(out))
    return out


# ---- particle diagnostics of the leaky-box application (Sec. 4.2): the energy distribution
# and the kinetic pressure behind the plasma beta.  Plain numpy in FP64.

def kinetic_energy(ux, uy, uz):
    """gamma - 1 per particle (units of m c^2) from FP32 or FP64 momenta, in FP64:
    u.u / (1 + sqrt(1 + u.u)), which equals sqrt(1 + u.u) - 1 without its cancellation."""
    x, y, z = (np.asarray(v, np.float64) for v in (ux, uy, uz))
    uu = x * x + y * y + z * z
    return uu / (np.sqrt(1.0 + uu) + 1.0)


def energy_histogram(ux, uy, uz, edges):
    """Counts over nbins + 2 slots: slot = number of edges <= gamma - 1 (0: below the first
    edge, 1 + b: in [edges[b], edges[b+1]), nbins + 1: at or above the last edge); a
    non-finite energy goes to the last slot."""
    edges = np.asarray(edges, np.float64)
    nb = len(edges) - 1
    k = kinetic_energy(ux, uy, uz)
    slot = np.searchsorted(edges, k, side="right")
    slot[np.isnan(k)] = nb + 1
    return np.bincount(slot, minlength=nb + 2).astype(np.int64)


def kinetic_stress(ux, uy, uz, m=1.0):
    """Diagonal of the kinetic stress, m * sum u_c^2 / gamma for c = x, y, z (FP64).  For an
    ideal gas the pressure is its trace over 3 per unit volume: n k T."""
    x, y, z = (np.asarray(v, np.float64) for v in (ux, uy, uz))
    g = np.sqrt(1.0 + x * x + y * y + z * z)
    return np.array([m * (x * x / g).sum(), m * (y * y / g).sum(), m * (z * z / g).sum()])
