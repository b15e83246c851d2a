"""Served mode: a request loop that keeps many independent 2D box runs resident on the GPU and
advances all of them together with the batched step (one launch per kernel for every active box,
box-descriptor tables).  Runs arrive over time; each is admitted as soon as its HBM footprint
fits the budget, stepped until it has done its steps, and retired (its memory freed for the next
arrivals).  Completion is timed after the GPU has finished the run's last step.

Workload of a served batch (seeded): box sizes uniform over {32^2, 64^2, 128^2, 256^2} cells,
particles per cell per species uniform in [4, 32], variant uniform over shearing box
(s uniform in [0, 1.5]), expanding box (adot uniform in [1e-4, 1e-3] omega_p) and leaky box
(t_esc uniform in [5, 50] L/c, probabilistic escape above gamma = 10), Maxwell-Juttner
theta uniform in [0.05, 0.5], skin depth 4 cells, sigma = 0.1.
Tile shapes (hence particles per workgroup) come from the library's autotuner, per box size
and ppc class, measured on proxy boxes before the runs start (tune_tiles).
Readings: B0 along z (shearing and leaky boxes) and along x for the expanding box, which
expands in y and z (l_y = l_z = a(t), the expansion perpendicular to B0); Omega0 = 0.1 omega_c,
reduced on boxes wider than 64 cells so that the shear flow stays at most 0.38 c at the x faces
(s Omega0 L/2 <= 1.5 * 0.1 * 0.079 * 32).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from . import synth
from .box import Batch, Box, describe, footprint as box_footprint, step_many

SIZES = (32, 64, 128, 256)
KINDS = ("shear", "expand", "leaky")


@dataclass
class RunSpec:
    rid: int
    n: int
    ppc: int
    kind: str
    theta: float
    param: float  # s (shear), adot (expand), t_esc in units of L/c (leaky)
    steps: int
    seed: int
    arrival: float = 0.0

    @property
    def particles(self) -> int:
        return 2 * self.ppc * self.n * self.n


def make_specs(n_runs=512, steps=500, seed=20260217):
    rng = np.random.default_rng(seed)
    wp = 0.25
    out = []
    for r in range(n_runs):
        kind = KINDS[int(rng.integers(0, 3))]
        if kind == "shear":
            param = float(rng.uniform(0.0, 1.5))
        elif kind == "expand":
            param = float(rng.uniform(1e-4, 1e-3)) * wp
        else:
            param = float(rng.uniform(5.0, 50.0))
        out.append(RunSpec(r, int(SIZES[int(rng.integers(0, 4))]), int(rng.integers(4, 33)), kind,
                           float(rng.uniform(0.05, 0.5)), param, steps, seed * 1000 + r))
    return out


def poisson_arrivals(specs, rate, seed=7):
    """Arrival times of a Poisson process of the given rate (runs per second), in order."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, len(specs)))
    for s, a in zip(specs, t):
        s.arrival = float(a)
    return specs


PPC_CLASSES = ((4, 11, 8), (12, 21, 16), (22, 32, 27))  # (low, high, proxy ppc)
_TILES: dict = {}


def ppc_class(ppc: int) -> int:
    return next(i for i, (lo, hi, _) in enumerate(PPC_CLASSES) if lo <= ppc <= hi)


SETTLE_STEPS = 30


def tune_tiles(sizes=SIZES, log=None):
    """Tile shape per (box size, ppc class) from the library's autotuner (pic_autotune, batched
    shapes only) on a proxy box of that size and particle load (a shearing box at theta 0.3);
    the choice sets the particles per workgroup.  Cached for the process."""
    for n in sizes:
        for k, (_, _, ppc) in enumerate(PPC_CLASSES):
            if (n, k) in _TILES:
                continue
            spec = RunSpec(-1, n, ppc, "shear", 0.3, 1.5, 1, 99)
            box = build_box(spec, tile=(0, 0, 0))
            # the fused kernel's speed depends on the particles' order inside a tile, which
            # settles within some tens of steps from the loader's cell-by-cell order: time the
            # shapes on the settled order that a run spends its steps in
            for _ in range(SETTLE_STEPS):
                box.step()
            shape, ms = box.autotune(batched=True, trials=2)
            box.close()
            _TILES[(n, k)] = shape
            if log:
                log(f"[tune] {n}^2 ppc~{ppc}: {shape} " +
                    " ".join(f"{t[0]}x{t[1]}={v:.3f}ms" for t, v in ms.items()))
    return dict(_TILES)


def tile_for(n: int, ppc: int):
    """Tile shape of a run: the autotuner's choice for its size and ppc class."""
    if (n, ppc_class(ppc)) not in _TILES:
        tune_tiles((n,))
    return _TILES[(n, ppc_class(ppc))]


def box_args(spec: RunSpec, tile=None):
    """(descriptor arguments of the run's box, axis of B0)"""
    wp, q, B0 = synth.plasma_params(spec.ppc, 4.0, 0.1)
    count = spec.ppc * spec.n * spec.n
    species = [(-1.0, -q, count), (1.0, q, count)]
    kw = dict(dt=0.45, species=species, seed=spec.seed, box_id=max(spec.rid, 0),
              tile=tile if tile is not None else tile_for(spec.n, spec.ppc), maxwell_iters=4)
    axis = 2
    if spec.kind == "shear":
        kw.update(frame=L.FRAME_SHEAR, shear_s=spec.param,
                  shear_omega0=0.1 * B0 * min(1.0, 64.0 / spec.n))
    elif spec.kind == "expand":
        kw.update(frame=L.FRAME_EXPAND, expand_adot=spec.param, expand_axis_mask=0b110)
        axis = 0
    else:
        kw.update(frame=L.FRAME_LEAKY, leaky_mode=L.LEAKY_PROBABILISTIC,
                  leaky_t_esc=spec.param * spec.n, leaky_gamma_thr=10.0)
    return kw, axis


_FOOTPRINTS: dict = {}


def footprint(spec: RunSpec) -> int:
    """Device bytes of one run, exactly: its box on torch memory as pic_box_layout sizes it
    (fields and currents with guards, both particle copies, the workspace)."""
    key = (spec.n, spec.ppc, spec.kind)
    if key not in _FOOTPRINTS:
        kw, _ = box_args(spec, tile=(0, 0, 0))
        _FOOTPRINTS[key] = box_footprint(describe(2, (spec.n, spec.n), **kw))
    return _FOOTPRINTS[key]


def build_box(spec: RunSpec, tile=None, track_ids=False) -> Box:
    """track_ids: carry particle ids (to match final states by id)."""
    wp, q, B0 = synth.plasma_params(spec.ppc, 4.0, 0.1)
    n = (spec.n, spec.n)
    kw, axis = box_args(spec, tile)
    box = Box(2, n, track_ids=track_ids, **kw)
    E, B = synth.uniform_field(n, axis, B0)
    box.set_fields(torch.from_numpy(E).float(), torch.from_numpy(B).float())
    for s, p in enumerate(synth.pair_plasma(n, spec.ppc, spec.theta, spec.seed, device="cuda")):
        box.set_particles(s, p["cell"], p["off"], p["u"])
    return box


@dataclass
class RunResult:
    spec: RunSpec
    admitted: float
    done: float
    energies: tuple = field(default_factory=tuple)
    state: dict = field(default_factory=dict)  # keep_state: final particles (by id) and fields

    @property
    def latency(self) -> float:
        return self.done - self.spec.arrival


def _state(box: Box):
    """Final particles of each species ordered by id, and the fields, on the host."""
    out = {}
    for sp in range(box.nsp):
        g = {k: v.cpu().numpy() for k, v in box.get_particles(sp).items()}
        order = np.argsort(g["id"], kind="stable")
        out[sp] = {k: (v[..., order] if k != "dr" else v[:, order]) for k, v in g.items()}
    E, B = box.get_fields()
    out["E"], out["B"] = E.cpu().numpy(), B.cpu().numpy()
    return out


def _energies(box: Box):
    info = box.info()
    assert info.errors & ~L.DERR_ORDER == 0, f"device error bits {info.errors}"
    return (sum(info.field_energy_E) + sum(info.field_energy_B), info.kinetic_energy,
            int(info.n_particles[0] + info.n_particles[1]))


ADMIT_PER_STEP = 8  # runs built per loop turn: building overlaps the GPU's steps


def serve(specs, budget_bytes, batched=True, keep_energies=False, graph=False,
          clock=time.perf_counter, keep_state=False):
    """Run every spec (arrival times relative to the call) and return the results in
    completion order.  batched=False steps the active boxes one at a time (per-box launches);
    with admission of one run at a time that is the one-box-at-a-time baseline.  graph=True
    replays the batched step as a captured HIP graph while the set of active boxes is unchanged
    (newly admitted runs take their first step, whose sort differs, before joining the set).
    keep_state: each result also holds the run's final particles (ids carried) and fields.
    After the call,
    serve.max_active is the most runs stepped together and serve.waited the runs that arrived
    but waited for memory."""
    if graph:
        st = torch.cuda.Stream()  # graph capture needs a stream other than the null stream
        with torch.cuda.stream(st):
            return _serve(specs, budget_bytes, batched, keep_energies, True, clock, keep_state)
    return _serve(specs, budget_bytes, batched, keep_energies, False, clock, keep_state)


def _serve(specs, budget_bytes, batched, keep_energies, graph, clock, keep_state):
    # the batched step's argument tables are staged in torch memory (pic_batch)
    batch = Batch(torch.cuda.current_stream()) if batched else None
    try:
        return _serve_loop(specs, budget_bytes, batched, keep_energies, graph, clock, batch,
                           keep_state)
    finally:
        if batch is not None:
            batch.close()


def _serve_loop(specs, budget_bytes, batched, keep_energies, graph, clock, batch, keep_state):
    pending = sorted(specs, key=lambda s: s.arrival)
    active = []  # [spec, box, steps_done, admitted]
    used = 0
    out = []
    serve.build_s = serve.step_s = 0.0
    serve.max_active = 0
    waited = set()
    t0 = clock()
    i = 0
    while i < len(pending) or active:
        now = clock() - t0
        admitted = []
        if i < len(pending) and pending[i].arrival <= now and active and \
                used + footprint(pending[i]) > budget_bytes:
            waited.add(pending[i].rid)  # arrived, but the memory is taken
        while i < len(pending) and pending[i].arrival <= now and len(admitted) < ADMIT_PER_STEP and (
                not (active or admitted) or used + footprint(pending[i]) <= budget_bytes):
            sp = pending[i]
            tb = clock()
            admitted.append([sp, build_box(sp, track_ids=keep_state), 0, now])
            serve.build_s += clock() - tb
            used += footprint(sp)
            i += 1
            now = clock() - t0
        if not active and not admitted:
            time.sleep(max(0.0, min(pending[i].arrival - now, 0.01)))
            continue
        ts = clock()
        if batched:
            if graph and admitted:
                step_many([a[1] for a in admitted], batched=True, batch=batch)
                for a in admitted:
                    a[2] += 1
            elif admitted:
                active.extend(admitted)
                admitted = []
            if active:
                step_many([a[1] for a in active], batched=True, graph=graph, batch=batch)
                for a in active:
                    a[2] += 1
            active.extend(admitted)
        else:
            active.extend(admitted)
            for a in active:
                step_many([a[1]], batched=False)
                a[2] += 1
        serve.step_s += clock() - ts
        serve.max_active = max(serve.max_active, len(active))
        finished = [a for a in active if a[2] >= a[0].steps]
        if finished:
            torch.cuda.synchronize()
            t = clock() - t0
            for a in finished:
                e = _energies(a[1]) if keep_energies else ()
                stt = _state(a[1]) if keep_state else {}
                out.append(RunResult(a[0], a[3], t, e, stt))
                a[1].close()
                used -= footprint(a[0])
            active = [a for a in active if a[2] < a[0].steps]
    serve.waited = len(waited)
    return out, clock() - t0


def summarize(results, wall):
    lat = np.array([r.latency for r in results])
    ps = sum(r.spec.particles * r.spec.steps for r in results)
    return dict(runs=len(results), wall_s=wall, particle_steps=ps,
                host_build_s=serve.build_s, host_step_enqueue_s=serve.step_s,
                particle_steps_per_s=ps / wall if wall > 0 else math.nan,
                p50_latency_s=float(np.percentile(lat, 50)) if len(lat) else math.nan,
                p99_latency_s=float(np.percentile(lat, 99)) if len(lat) else math.nan,
                runs_per_s=len(results) / wall if wall > 0 else math.nan)
