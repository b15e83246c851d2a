"""The served mode's request loop (continuous batching) at small scale: 24 box runs of the
served workload's recipe (shearing, expanding and leaky 2D boxes of 32^2 and 64^2 cells, 4-32
ppc per species) arrive as a Poisson stream faster than they finish, under an HBM budget of
about three runs, so that runs wait for memory and are admitted as others retire while the
rest keep stepping together.  Every run's final particles (matched by id) and fields equal its
run alone (one box at a time, per-box launches) within the parity tolerances: momenta 2e-6
relative, positions 2e-6 cells, fields 1e-5 of their maximum, integer work (ids, live
particles) equal."""
import numpy as np
import pytest

from _cases import wrap_diff
from paper_2602_15939_amd import serve

pytestmark = pytest.mark.gpu

STEPS = 12


def _specs():
    specs = serve.make_specs(24, STEPS, seed=4242)
    for k, sp in enumerate(specs):
        sp.n = (32, 64)[k % 2]
    return serve.poisson_arrivals(specs, rate=400.0, seed=11)


def _positions(g, n):
    i = g["cell"] % n
    j = g["cell"] // n
    return i + g["off"][0].astype(np.float64), j + g["off"][1].astype(np.float64)


def _same(a, b, n, tag):
    for sp in (0, 1):
        ga, gb = a[sp], b[sp]
        np.testing.assert_array_equal(ga["id"], gb["id"], err_msg=str(tag))
        live = gb["cell"] >= 0
        np.testing.assert_array_equal(ga["cell"] >= 0, live, err_msg=str(tag))
        ua, ub = ga["u"][:, live].astype(np.float64), gb["u"][:, live].astype(np.float64)
        du = np.linalg.norm(ua - ub, axis=0) / np.maximum(np.linalg.norm(ub, axis=0), 1e-2)
        assert du.max(initial=0.0) < 2e-6, (tag, sp, du.max())
        xa, ya = _positions({k: v[..., live] for k, v in ga.items()}, n)
        xb, yb = _positions({k: v[..., live] for k, v in gb.items()}, n)
        assert np.abs(wrap_diff(xa, xb, n)).max(initial=0.0) < 2e-6, tag
        assert np.abs(wrap_diff(ya, yb, n)).max(initial=0.0) < 2e-6, tag
    for f in ("E", "B"):
        assert np.abs(a[f] - b[f]).max() <= 1e-5 * np.abs(b[f]).max(), (tag, f)


@pytest.mark.parametrize("graph", [False, True])
def test_served_runs_equal_their_solo_runs(graph):
    specs = _specs()
    fp = sorted(serve.footprint(s) for s in specs)
    budget = fp[-1] + fp[-2] + fp[-3]
    res, wall = serve.serve(specs, budget, batched=True, graph=graph, keep_state=True)
    assert len(res) == 24 and sorted(r.spec.rid for r in res) == list(range(24))
    assert serve.serve.max_active >= 2  # runs overlapped on the device
    assert serve.serve.waited >= 3  # and arrivals waited for memory to free up
    for r in res:
        alone, _ = serve.serve([serve.RunSpec(r.spec.rid, r.spec.n, r.spec.ppc, r.spec.kind,
                                              r.spec.theta, r.spec.param, r.spec.steps,
                                              r.spec.seed)],
                               0, batched=False, keep_state=True)
        _same(r.state, alone[0].state, r.spec.n, (r.spec.rid, r.spec.kind, graph))
