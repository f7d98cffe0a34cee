"""Serving (continuous batching): each event's result is the same alone and in
a mix, admission respects the device budget, and the ticket API behaves."""
import time

import numpy as np
import pytest

from paper_1702_06359_amd import abi, synth

pytestmark = pytest.mark.gpu

FIELDS = ("par", "cov", "hits", "n_hits", "n_holes", "chi2", "status", "ndof")


def _wait(ctx, tickets, timeout=60.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for t in tickets:
            if t in done:
                continue
            r = ctx.serve_poll(t)
            if r is not None:
                done[t] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(tickets) - len(done)} tickets not done after {timeout} s")
        time.sleep(0.0005)
    return done


@pytest.fixture(scope="module")
def ctx(gpu_required):
    c = abi.Context(abi.config_from_geometry(synth.Geometry(), max_cands=6))
    yield c
    c.close()


def test_result_is_the_same_alone_and_in_the_mix(ctx):
    ctx.serve_config(2 << 30, max_in_flight=16)
    evs = [synth.make_event(n, cfg=220, event=i, noise=0.3) for i, n in enumerate((3000, 700, 5000, 1200, 90))]
    print("case serve alone", flush=True)
    t, _ = ctx.serve_submit(evs[0])
    alone = _wait(ctx, [t])[t]
    assert alone[0] == abi.OK
    print("case serve mix", flush=True)
    tickets = []
    for i, e in enumerate(evs * 2):
        t, _ = ctx.serve_submit(e)
        tickets.append(t)
        if i % 3 == 0:
            time.sleep(0.001)
    res = _wait(ctx, tickets)
    for j, t in enumerate(tickets):
        st, lat, out = res[t]
        assert st == abi.OK and lat > 0
        if j % len(evs) == 0:
            for k in FIELDS:
                assert np.array_equal(out[k], alone[2][k]), k
    # and equal to the plain builder of the loaded event
    h = ctx.load_event(evs[0])
    try:
        ref = ctx.build(h, evs[0].n_seeds)
    finally:
        ctx.unload_event(h)
    for k in FIELDS:
        assert np.array_equal(ref[k], alone[2][k]), k


def test_admission_under_a_tight_budget(ctx):
    ev = synth.make_event(4000, cfg=221, event=0, noise=0.3)
    # room for about two such events at a time
    ctx.serve_config(12 << 20, max_in_flight=8)
    print("case serve tight budget", flush=True)
    tickets = [ctx.serve_submit(ev)[0] for _ in range(6)]
    res = _wait(ctx, tickets)
    outs = [res[t][2] for t in tickets]
    for o in outs[1:]:
        for k in FIELDS:
            assert np.array_equal(o[k], outs[0][k]), k
    big = synth.make_event(60000, cfg=221, event=1, noise=0.3)
    with pytest.raises(abi.MkfError) as e:
        ctx.serve_submit(big)
    assert e.value.status == abi.E_NOMEM


def test_ticket_api(ctx):
    ctx.serve_config(1 << 30, max_in_flight=1, max_batch_events=1)
    ev = synth.make_event(20000, cfg=222, event=0, noise=0.1)
    small = synth.make_event(100, cfg=222, event=1, noise=0.1)
    print("case serve tickets", flush=True)
    first = [ctx.serve_submit(ev)[0] for _ in range(3)]
    last, _ = ctx.serve_submit(small)
    try:
        ctx.serve_cancel(last)
        cancelled = True
    except abi.MkfError as e:
        assert e.status == abi.E_STATE     # already admitted
        cancelled = False
    ctx.serve_drain()
    res = _wait(ctx, first)
    assert all(r[0] == abi.OK for r in res.values())
    if cancelled:
        with pytest.raises(abi.MkfError) as e:
            ctx.serve_poll(last)
        assert e.value.status == abi.E_NOTFOUND
    else:
        _wait(ctx, [last])
    with pytest.raises(abi.MkfError) as e:
        ctx.serve_poll(123456789)
    assert e.value.status == abi.E_NOTFOUND
    bad = [h.copy() for h in small.hits]
    bad[0][0, 0] = np.inf
    with pytest.raises(abi.MkfError) as e:
        ctx.serve_submit(abi.EventArrays(bad, small.seed_par, small.seed_cov, small.seed_hits))
    assert e.value.status == abi.E_INVALID
