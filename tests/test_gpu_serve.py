"""Serving: each request's result is the same alone and in the mix.

A mixed trace (Boolean and uint16 anti-distance closures of uneven sizes,
arriving close together) is replayed through the continuously batched server;
every result must equal the same request closed alone on the device, and the
oracle's closure.  A small budget forces admission control to queue requests.
"""
import numpy as np
import pytest

import oracle
import paper_1705_08743_amd as sr
import synthgen
from gpu_util import set_oracle_threads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    set_oracle_threads()


def make_requests(count, nlo, nhi, seed, spacing):
    from paper_1705_08743_amd.serve import Request
    trace = synthgen.serving_trace(count, nlo=nlo, nhi=nhi, seed=seed)
    kinds = {"bool": sr.SR_BOOL, "u16": sr.SR_ANTIDIST_U16}
    return [Request(i, kinds[k], n, synthgen.serving_request(n, k, s), i * spacing)
            for i, (n, k, s) in enumerate(trace)]


def solo(r):
    if r.kind == sr.SR_BOOL:
        t = sr.to_device(sr.SR_BOOL, r.host, cols=r.n)
        sr.closure(sr.SR_BOOL, t, D=r.n)
    else:
        t = sr.to_device(r.kind, r.host[:, :r.n])
        sr.closure(r.kind, t)
    torch.cuda.synchronize()
    return sr.to_host(t)


def want(r):
    if r.kind == sr.SR_BOOL:
        return oracle.bool_closure_words(r.host, r.n)[:, :(r.n + 63) // 64]
    return oracle.ad_closure(r.host[:, :r.n], 65535)


@pytest.mark.parametrize("budget_mb", [4096, 4])
def test_served_results_equal_solo_and_oracle(budget_mb):
    from paper_1705_08743_amd.serve import ClosureServer
    reqs = make_requests(40, 40, 700, seed=4242, spacing=2e-4)
    server = ClosureServer(budget_bytes=budget_mb << 20, slots=4, batch_n=256)
    stats = server.run(reqs, "served")
    assert stats["requests"] == len(reqs)
    if budget_mb > 100:
        assert stats["batched_requests"] > 0  # small requests were batched
    for r in reqs:
        got = r.result.view(np.uint64) if r.kind == sr.SR_BOOL else r.result
        alone = solo(r)
        if r.kind == sr.SR_BOOL:
            alone = alone[:, :(r.n + 63) // 64]
        assert np.array_equal(got, alone), (r.rid, r.n, r.kind)
        assert np.array_equal(got.astype(np.int64) if r.kind != sr.SR_BOOL else got, want(r)), r.rid


def test_serial_mode_matches_served():
    from paper_1705_08743_amd.serve import ClosureServer, Request
    reqs = make_requests(16, 64, 1500, seed=99, spacing=0.0)
    twin = [Request(r.rid, r.kind, r.n, r.host, r.arrival) for r in reqs]
    server = ClosureServer(budget_bytes=1 << 30)
    a = server.run(reqs, "served")
    b = server.run(twin, "serial")
    for x, y in zip(reqs, twin):
        assert np.array_equal(x.result, y.result)
    assert b["batched_requests"] == 0
    assert a["p99_ms"] > 0 and b["p99_ms"] > 0


def test_budget_too_small_is_refused():
    from paper_1705_08743_amd.serve import ClosureServer
    reqs = make_requests(2, 300, 301, seed=5, spacing=0.0)
    server = ClosureServer(budget_bytes=1024)
    with pytest.raises(ValueError):
        server.run(reqs, "served")


def test_boolean_requests_are_batched():
    """Small Boolean requests that wait together are closed by one batched
    launch ({0, 255} anti-distance working copies), with the same results as
    alone and as the oracle."""
    from paper_1705_08743_amd.serve import ClosureServer, Request
    trace = synthgen.serving_trace(24, nlo=40, nhi=250, seed=321)
    reqs = [Request(i, sr.SR_BOOL, n, synthgen.serving_request(n, "bool", s), 0.0)
            for i, (n, _, s) in enumerate(trace)]
    server = ClosureServer(budget_bytes=1 << 30, slots=2, batch_n=256)
    stats = server.run(reqs, "served")
    assert stats["batched_requests"] > 0
    for r in reqs:
        got = r.result.view(np.uint64)
        assert np.array_equal(got, solo(r)[:, :(r.n + 63) // 64]), (r.rid, r.n)
        assert np.array_equal(got, want(r)), r.rid


def test_failed_request_fails_alone():
    """Two requests marked to fail (their closure call is refused by the
    library): one small enough to be batched with others of its kind, one
    large.  Each fails alone with its error recorded; every other request,
    including those batched with the bad one, equals the oracle."""
    from paper_1705_08743_amd.serve import ClosureServer, Request
    base = make_requests(30, 40, 900, seed=777, spacing=0.0)
    small = min((r for r in base if r.n <= 256), key=lambda r: r.rid)
    large = max(base, key=lambda r: r.n)
    bad = {small.rid, large.rid}
    reqs = [Request(r.rid, r.kind, r.n, r.host, 0.0, inject_fault=r.rid in bad) for r in base]
    server = ClosureServer(budget_bytes=1 << 30, slots=4, batch_n=256)
    stats = server.run(reqs, "served")
    assert stats["failed"] == 2 and stats["requests"] == len(reqs) - 2
    for r in reqs:
        if r.rid in bad:
            assert r.result is None and "SR_EINVAL" in r.error, r.rid
            continue
        assert r.error is None
        got = r.result.view(np.uint64) if r.kind == sr.SR_BOOL else r.result
        assert np.array_equal(got.astype(np.int64) if r.kind != sr.SR_BOOL else got, want(r)), r.rid
    # the server keeps serving afterwards
    again = [Request(r.rid, r.kind, r.n, r.host, 0.0) for r in base[:6]]
    assert server.run(again, "served")["failed"] == 0


def test_queued_request_can_be_cancelled():
    """With a budget that admits one request at a time, a request withdrawn
    while it is queued (its cancel_at passed; or cancel() called from another
    thread, which the serving loop applies at its next pass) is never run;
    the others complete and equal the oracle; a withdrawal time after a
    request's completion changes nothing."""
    import threading
    from paper_1705_08743_amd.serve import ClosureServer, Request, footprint_bytes
    base = make_requests(8, 500, 700, seed=1357, spacing=0.0)
    budget = max(footprint_bytes(r.kind, r.n) for r in base)
    reqs = [Request(r.rid, r.kind, r.n, r.host, 0.0,
                    cancel_at=0.0 if r.rid == 3 else (100.0 if r.rid == 5 else None))
            for r in base]
    server = ClosureServer(budget_bytes=budget, slots=1, batch_n=0)
    stats = server.run(reqs, "served")
    assert stats["cancelled"] == 1 and reqs[3].cancelled and reqs[3].result is None
    assert reqs[3].t_admit is None
    for r in reqs:
        if r.rid == 3:
            continue
        assert not r.cancelled
        got = r.result.view(np.uint64) if r.kind == sr.SR_BOOL else r.result
        assert np.array_equal(got.astype(np.int64) if r.kind != sr.SR_BOOL else got, want(r)), r.rid
    # cancel() from another thread: the last request, queued behind the
    # others for the only slot, is withdrawn when the loop sees the request
    reqs2 = [Request(r.rid, r.kind, r.n, r.host, 0.0) for r in base]
    t = threading.Timer(0.0, server.cancel, args=(reqs2[-1].rid,))
    t.start()
    t.join()
    stats2 = server.run(reqs2, "served")
    assert stats2["cancelled"] == 1 and reqs2[-1].cancelled and reqs2[-1].result is None
    assert all(r.result is not None for r in reqs2[:-1])

