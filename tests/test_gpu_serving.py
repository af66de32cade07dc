"""Serving (continuous batching) through the C ABI: requests that arrive while
others run are admitted as slots and memory free up, run concurrently, and
each result equals the result of the same solve alone: bit for bit when it
ran on its own, to rounding when it shared a grouped solve (compatible
requests waiting together are solved as one concatenated block)."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# mixed surfaces, levels, k, shifts, precisions and smoothers; two requests
# share a hierarchy (and run on it concurrently)
REQUESTS = [
    dict(kind="sphere", n_refine=3, k=9, sigma=0.0, m=12, precision="mixed", smoother="jacobi", seed=0),
    dict(kind="sphere", n_refine=4, k=16, sigma=0.0, m=20, precision="fp64", smoother="gs", seed=1),
    dict(kind="ellipsoid", n_refine=3, k=8, sigma=0.0, axes=(1.2, 1.5, 1.9), precision="mixed",
         smoother="jacobi", seed=2),
    dict(kind="sphere", n_refine=4, k=5, sigma=6.0, m=12, precision="mixed", smoother="gs", seed=3),
    dict(kind="ellipsoid", n_refine=4, k=12, sigma=0.0, axes=(1.0, 1.5, 2.0), precision="fp64",
         smoother="jacobi", seed=4),
    dict(kind="sphere", n_refine=3, k=9, sigma=0.0, m=12, precision="mixed", smoother="jacobi", seed=5),
    dict(kind="sphere", n_refine=5, k=25, sigma=0.0, m=32, precision="mixed", smoother="jacobi", seed=6),
    # interior shifts (the shifted scheme) on the three surfaces, and a torus at sigma = 0
    dict(kind="torus", n_refine=1, k=12, sigma=60.0, precision="mixed", smoother="jacobi", seed=7),
    dict(kind="ellipsoid", n_refine=5, k=16, sigma=40.0, axes=(1.0, 1.5, 2.0), precision="mixed",
         smoother="jacobi", seed=8),
    dict(kind="torus", n_refine=1, k=8, sigma=0.0, precision="fp64", smoother="gs", seed=9),
    dict(kind="sphere", n_refine=4, k=10, sigma=150.0, precision="fp64", smoother="jacobi", seed=10),
    dict(kind="ellipsoid", n_refine=4, k=20, sigma=120.0, axes=(1.3, 1.9, 1.1), precision="mixed",
         smoother="gs", seed=11),
]

SURF = ("kind", "n_refine", "axes")
SOLVE = ("m", "precision", "smoother", "seed")


@pytest.fixture(scope="module")
def lib():
    import paper_1511_07042_amd as p
    return p


def _alone(lib, req):
    with lib.Hierarchy(req["kind"], req["n_refine"], axes=req.get("axes", (1.0, 1.0, 1.0))) as h:
        kw = {k: req[k] for k in SOLVE if k in req}
        return h.solve(req["k"], req["sigma"], 1e-8, **kw)


def _submit(lib, srv, req):
    kw = {k: req[k] for k in SOLVE if k in req}
    return srv.submit(req["kind"], req["n_refine"], req["k"], req["sigma"], 1e-8,
                      axes=req.get("axes", (1.0, 1.0, 1.0)), **kw)


def _same(res, alone, what, req=None):
    ev, V, st = alone
    assert res["status"] == 0, (what, res["error"])
    if res["stats"]["group_size"] == 1:
        assert res["stats"]["cycles"] == st["cycles"], what
        assert np.array_equal(res["evals"], ev), (what, np.max(np.abs(res["evals"] - ev)))
        assert np.array_equal(res["evecs"], V), (what, np.max(np.abs(res["evecs"] - V)))
        return
    # grouped: the same iteration up to the grouping of the residual sums
    from oracle import bmg as ob, reference
    assert abs(res["stats"]["cycles"] - st["cycles"]) <= 1, what
    assert np.max(np.abs(res["evals"] - ev) / np.maximum(np.abs(ev), 1.0)) < 1e-9, what
    lv = ob.build_levels(req["kind"], req["n_refine"], axes=req.get("axes", (1.0, 1.0, 1.0)))
    rel, sine = reference.compare(res["evals"], res["evecs"], ev, V, lv[-1].M)
    assert rel < 1e-9 and sine < 2e-7, (what, rel, sine)


@pytest.mark.parametrize("grouping", ["on", "off"])
def test_mix_equals_alone(lib, grouping, monkeypatch):
    if grouping == "off":
        monkeypatch.setenv("BMG_NO_GROUP", "1")  # read when the server is created
    alone = [_alone(lib, r) for r in REQUESTS]
    with lib.Server(8 << 30, max_slots=4) as srv:
        ids = [_submit(lib, srv, r) for r in REQUESTS[:3]]
        # later arrivals: submitted while the first ones are queued or running
        time.sleep(0.002)
        ids += [_submit(lib, srv, r) for r in REQUESTS[3:]]
        res = [srv.wait(i) for i in ids]
    lat = [r["latency_ms"] for r in res]
    print("latencies ms:", [round(x, 1) for x in lat])
    for i, (r, a) in enumerate(zip(res, alone)):
        _same(r, a, i, REQUESTS[i])
        assert r["stats"]["converged"] == 1 and r["latency_ms"] > 0
        if grouping == "off":
            assert r["stats"]["group_size"] == 1


def test_waiting_compatible_requests_are_grouped(lib):
    # one slot, busy with a first request: the compatible requests that arrive
    # meanwhile wait together and then run as one grouped solve (same surface,
    # level and shift; different k, m and seeds), the others on their own
    base = dict(kind="sphere", n_refine=4, sigma=0.0, precision="mixed", smoother="jacobi")
    reqs = [dict(base, k=9, m=12, seed=21), dict(base, k=16, m=20, seed=22),
            dict(base, k=25, m=32, seed=23), dict(base, k=4, m=8, seed=24),
            dict(kind="torus", n_refine=1, k=8, sigma=0.0, precision="mixed", smoother="jacobi", seed=25),
            dict(base, k=9, m=12, seed=26, precision="fp64")]
    alone = [_alone(lib, r) for r in reqs]
    with lib.Server(8 << 30, max_slots=1) as srv:
        first = srv.submit("sphere", 5, 25, 0.0, 1e-8, m=32)
        ids = [_submit(lib, srv, r) for r in reqs]
        srv.wait(first)
        res = [srv.wait(i) for i in ids]
    sizes = [r["stats"]["group_size"] for r in res]
    print("group sizes:", sizes, "latencies ms:", [round(r["latency_ms"], 1) for r in res])
    assert sizes[:4] == [4, 4, 4, 4] and sizes[4] == 1 and sizes[5] == 1, sizes
    for i, (r, a) in enumerate(zip(res, alone)):
        _same(r, a, i, reqs[i])


def test_tight_budget_evicts_and_still_matches(lib):
    # a budget that holds about one problem at a time: requests wait for memory,
    # idle hierarchies and workspaces are freed, results do not change
    reqs = [REQUESTS[0], REQUESTS[2], REQUESTS[0], REQUESTS[1]]
    alone = [_alone(lib, r) for r in reqs]
    with lib.Server(10 << 20, max_slots=3) as srv:
        ids = [_submit(lib, srv, r) for r in reqs]
        res = [srv.wait(i) for i in ids]
    for i, (r, a) in enumerate(zip(res, alone)):
        _same(r, a, i, reqs[i])


def test_cancel_enomem_and_errors(lib):
    with lib.Server(8 << 30, max_slots=1) as srv:
        # the single slot is busy with a long request; a queued one is canceled
        # at once, the running one at the end of its current cycle
        # an unreachable certificate keeps it cycling until canceled
        long_id = srv.submit("sphere", 5, 25, 0.0, 1e-300, m=32, max_cycles=100000,
                             angle_tol=1e-300)
        queued = srv.submit("sphere", 3, 9, 0.0, 1e-8, m=12)
        srv.cancel(queued)
        r = srv.wait(queued)
        assert r["status"] == lib.ECANCELED
        time.sleep(0.05)
        srv.cancel(long_id)
        r = srv.wait(long_id)
        assert r["status"] == lib.ECANCELED and r["stats"]["cycles"] >= 1
        # unknown ids and invalid requests
        with pytest.raises(lib.BMGError) as e:
            srv.cancel(123456)
        assert e.value.status == lib.EINVAL
        with pytest.raises(lib.BMGError) as e:
            srv.submit("sphere", 3, 0)
        assert e.value.status == lib.EINVAL
        # the server still serves after all that
        rid = srv.submit("sphere", 3, 9, 0.0, 1e-8, m=12, seed=0, smoother="jacobi",
                         precision="mixed")
        _same(srv.wait(rid), _alone(lib, REQUESTS[0]), "after-cancel", REQUESTS[0])
    with lib.Server(1 << 20, max_slots=2) as srv:
        with pytest.raises(lib.BMGError) as e:
            srv.submit("sphere", 5, 25, m=32)
        assert e.value.status == lib.ENOMEM


def test_poll_busy_then_done(lib):
    with lib.Server(8 << 30, max_slots=2) as srv:
        rid = srv.submit("sphere", 5, 25, 0.0, 1e-8, m=32)
        assert srv.poll(rid) is None  # still queued or running right after submit
        r = srv.wait(rid)
        assert r["status"] == lib.OK and r["evecs"].shape == (10 * 4 ** 5 + 2, 25)


def test_new_hierarchies_under_eviction_all_succeed(lib):
    # 24 requests, each on a hierarchy of its own (random ellipsoid axes),
    # both schemes and widths the solver chooses, on 8 slots under a budget
    # that holds only a few at a time: workers free hierarchies, workspaces
    # and eigendecompositions (device-wide synchronisations) while others
    # capture their cycle graphs.  Every request must succeed, and a few are
    # checked against their solo solves.
    rs = np.random.default_rng(5)
    reqs = []
    for i in range(24):
        axes = tuple(float(x) for x in rs.uniform(1.0, 2.0, 3))
        sigma = 0.0 if i % 2 == 0 else float(rs.uniform(15.0, 60.0))
        reqs.append(dict(kind="ellipsoid", n_refine=3 + i % 2, k=int(rs.integers(4, 13)), sigma=sigma,
                         axes=axes, precision="mixed", smoother="jacobi", seed=100 + i))
    with lib.Server(512 << 20, max_slots=8) as srv:
        ids = [_submit(lib, srv, r) for r in reqs]
        res = [srv.wait(i) for i in ids]
    for i, r in enumerate(res):
        assert r["status"] == 0, (i, reqs[i], r["error"])
    for i in (0, 1, 7):
        _same(res[i], _alone(lib, reqs[i]), i, reqs[i])
