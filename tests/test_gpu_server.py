"""GPU: the continuous-batching request server.

  * a served request equals the oracle on the same plan (uniform split, budget
    split, seed) within 1e-6 (FP64) / 1e-4 (FP32 form);
  * each request's result is bit-identical alone and in a mix of concurrent
    requests of different lattices, parameters, budgets and precisions;
  * admission by device memory, the pending limit, cancellation and invalid
    requests behave as documented (conditions forced from the host)."""
import time

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture()
def server(bfi, ctx):
    srv = bfi.bfi_server_create(ctx, bfi.server_config(memory_budget=1 << 30, max_requests=64,
                                                        chunks_per_step=16))
    yield srv
    bfi.bfi_server_destroy(srv)


def req(bfi, nx, nt, nu, prec, seed, box, k, budget):
    return bfi.request(bfi.lattice(nx, nt, nu=nu), prec, seed, box, k, budget)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-6), ("fp32", 1e-4)])
def test_served_result_matches_oracle(bfi, server, prec, tol):
    nx, nt, nu, B, k, budget = 4, 2, 0.5, 4.0, 4, 200_003
    t = bfi.bfi_server_submit(server, req(bfi, nx, nt, nu, prec, 7, B, k, budget))
    res, latency = bfi.bfi_server_wait(server, t, 60.0)
    assert latency > 0
    ref = oracle.integrate_uniform(oracle.lattice(nx, nt, nu=nu), 7, -B, B, k, budget)
    assert abs(res["Z"] - ref["Z"]) <= tol * ref["Z"]
    assert np.all(np.abs(res["C"] - ref["C"]) <= tol * abs(ref["C"][0]))
    assert res["n_evals"] == budget


def mixed_requests(bfi, count, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        nx, nt = workloads.SERVING_SHAPES[int(rng.integers(4))]
        nu = float(np.exp(rng.uniform(np.log(0.05), np.log(2.0))))
        budget = int(2 ** rng.uniform(14, 21)) // 16 * 16
        prec = "fp32" if rng.random() < 0.5 else "fp64"
        box = 3.0 if (nx, nt) == (16, 4) else 4.0
        out.append(req(bfi, nx, nt, nu, prec, i + 1, box, 4, budget))
    return out


def test_alone_equals_mix(bfi, ctx, server):
    reqs = mixed_requests(bfi, 40, 3)
    tickets = [bfi.bfi_server_submit(server, r) for r in reqs]
    mixed = [bfi.bfi_server_wait(server, t, 120.0)[0] for t in tickets]
    st = bfi.bfi_server_stats_get(server)
    assert st["completed"] >= 40 and st["steps"] >= 1
    for i in range(0, 40, 3):
        alone_srv = bfi.bfi_server_create(ctx, bfi.server_config(memory_budget=1 << 30))
        try:
            t = bfi.bfi_server_submit(alone_srv, reqs[i])
            alone = bfi.bfi_server_wait(alone_srv, t, 60.0)[0]
        finally:
            bfi.bfi_server_destroy(alone_srv)
        assert alone["Z"] == mixed[i]["Z"], i
        assert np.array_equal(alone["C"], mixed[i]["C"]), i
        assert np.array_equal(alone["C_err"], mixed[i]["C_err"]), i


def test_served_equals_integrate(bfi, ctx, server):
    """The server's result equals the one-shot uniform-split entry with the
    server's launch shape."""
    r = req(bfi, 10, 2, 1.0, "fp64", 5, 4.0, 6, 1 << 22)
    res = bfi.bfi_server_wait(server, bfi.bfi_server_submit(server, r), 60.0)[0]
    ref = bfi.bfi_integrate(ctx, bfi.lattice(10, 2), "fp64", 5, -4.0, 4.0, 6, 1 << 22)
    assert res["log_Z"] == pytest.approx(ref["log_Z"], abs=1e-12)
    assert np.all(np.abs(res["C"] - ref["C"]) <= 1e-12 * abs(ref["C"][0]))


def test_admission_by_memory(bfi, ctx):
    small = req(bfi, 4, 2, 1.0, "fp64", 1, 4.0, 2, 4096)
    big = req(bfi, 10, 2, 1.0, "fp64", 1, 4.0, 12, 1 << 20)
    srv = bfi.bfi_server_create(ctx, bfi.server_config(memory_budget=256 << 10))
    try:
        with pytest.raises(bfi.BfiError) as e:
            bfi.bfi_server_submit(srv, big)
        assert e.value.name == "BFI_EBUSY"
        # requests that fit one or two at a time are queued and all complete
        ts = [bfi.bfi_server_submit(srv, small) for _ in range(12)]
        out = [bfi.bfi_server_wait(srv, t, 60.0) for t in ts]
        assert all(o is not None for o in out)
        assert len({o[0]["Z"] for o in out}) == 1
        assert bfi.bfi_server_stats_get(srv)["rejected"] == 1
    finally:
        bfi.bfi_server_destroy(srv)


def test_pending_limit(bfi, ctx):
    srv = bfi.bfi_server_create(ctx, bfi.server_config(memory_budget=1 << 30, max_requests=1,
                                                        max_pending=2))
    try:
        slow = req(bfi, 16, 4, 0.5, "fp64", 1, 3.0, 4, 1 << 31)
        accepted, busy = [], 0
        for _ in range(8):
            try:
                accepted.append(bfi.bfi_server_submit(srv, slow))
            except bfi.BfiError as e:
                assert e.name == "BFI_EBUSY"
                busy += 1
        assert busy >= 1 and len(accepted) <= 3
        for t in accepted:
            bfi.bfi_server_cancel(srv, t)
        for t in accepted:
            with pytest.raises(bfi.BfiError) as e:
                bfi.bfi_server_wait(srv, t, 120.0)
            assert e.value.name == "BFI_ECANCELLED"
    finally:
        bfi.bfi_server_destroy(srv)


def test_cancel_running_request(bfi, server):
    t = bfi.bfi_server_submit(server, req(bfi, 16, 4, 0.5, "fp32", 1, 3.0, 6, 1 << 31))
    time.sleep(0.01)
    bfi.bfi_server_cancel(server, t)
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_server_wait(server, t, 120.0)
    assert e.value.name == "BFI_ECANCELLED"
    # the server keeps serving
    t2 = bfi.bfi_server_submit(server, req(bfi, 4, 2, 1.0, "fp64", 2, 4.0, 2, 4096))
    assert bfi.bfi_server_wait(server, t2, 60.0) is not None


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nonfinite_request_is_isolated(bfi, ctx, server, prec):
    """A request whose sums come out non-finite (a box of 1e200, where the action
    overflows) fails alone with BFI_EDEVICE; requests served beside it are
    bit-identical to their results alone, and the server keeps serving."""
    good = [req(bfi, 4, 2, 0.5, "fp64", 3, 4.0, 3, 1 << 18),
            req(bfi, 10, 2, 1.0, "fp32", 4, 4.0, 4, 1 << 20)]
    alone = []
    for r in good:
        srv = bfi.bfi_server_create(ctx, bfi.server_config(memory_budget=1 << 30))
        try:
            alone.append(bfi.bfi_server_wait(srv, bfi.bfi_server_submit(srv, r), 60.0)[0])
        finally:
            bfi.bfi_server_destroy(srv)
    bad = bfi.bfi_server_submit(server, req(bfi, 4, 2, 0.5, prec, 5, 1e200, 3, 1 << 18))
    tickets = [bfi.bfi_server_submit(server, r) for r in good]
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_server_wait(server, bad, 60.0)
    assert e.value.name == "BFI_EDEVICE"
    for t, ref in zip(tickets, alone):
        res = bfi.bfi_server_wait(server, t, 60.0)[0]
        assert res["Z"] == ref["Z"]
        assert np.array_equal(res["C"], ref["C"])
    t = bfi.bfi_server_submit(server, good[0])
    assert bfi.bfi_server_wait(server, t, 60.0)[0]["Z"] == alone[0]["Z"]


def test_invalid_requests(bfi, server):
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_server_submit(server, req(bfi, 7, 7, 1.0, "fp64", 1, 4.0, 2, 4096))
    assert e.value.name == "BFI_EUNSUPPORTED"
    for bad in (dict(budget=7), dict(box=0.0), dict(k=30)):
        args = dict(nx=4, nt=2, nu=1.0, prec="fp64", seed=1, box=4.0, k=2, budget=4096)
        args.update(bad)
        with pytest.raises(bfi.BfiError) as e:
            bfi.bfi_server_submit(server, req(bfi, **args))
        assert e.value.name == "BFI_EINVAL"
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_server_poll(server, 123456789)
    assert e.value.name == "BFI_ENOTFOUND"
    # a request far too large is refused before anything is built for it
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_server_submit(server, req(bfi, 10, 2, 1.0, "fp32", 1, 4.0, 2, 1 << 62))
    assert e.value.name in ("BFI_EINVAL", "BFI_EBUSY")
    st = bfi.bfi_server_stats_get(server)
    t = bfi.bfi_server_submit(server, req(bfi, 4, 2, 1.0, "fp64", 1, 4.0, 2, 4096))
    assert bfi.bfi_server_wait(server, t, 60.0) is not None


def test_poisson_burst_latency(bfi, server):
    """A short Poisson stream (200 requests/s) completes with finite latencies."""
    reqs = workloads.serving_requests(200.0, 0.5, seed=2, budget_log2=(16, 20))
    t0 = time.perf_counter()
    tickets = []
    for r in reqs:
        while time.perf_counter() - t0 < r.arrival_s:
            time.sleep(0.0002)
        tickets.append(bfi.bfi_server_submit(server, bfi.request(
            bfi.lattice(r.nx, r.nt, nu=r.nu, D=r.D), "fp32", r.seed, r.box, r.split_log2,
            r.budget)))
    lat = [bfi.bfi_server_wait(server, t, 60.0)[1] for t in tickets]
    assert len(lat) == len(reqs) and all(0 < x < 30 for x in lat)
