"""Serving (continuous batching): each event's result is the same alone and in
a mix, and equal to the FP64 oracle under the tie protocol; admission takes
an in-flight slot and budget at submit (MKF_E_AGAIN otherwise); the launch
shapes are the ones serving was configured with; the ticket API behaves."""
import time

import numpy as np
import pytest

import oracle
from conftest import report
from paper_1702_06359_amd import abi, synth
from parity_util import assert_build_parity, compare_build

pytestmark = pytest.mark.gpu

FIELDS = ("par", "cov", "hits", "n_hits", "n_holes", "chi2", "status", "ndof")


def _wait(ctx, tickets, timeout=120.0):
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


def _submit_retry(ctx, ev, timeout=120.0):
    """Submit, waiting while no slot or budget is free."""
    t0 = time.time()
    while True:
        t, out = ctx.serve_submit(ev)
        if t is not None:
            return t
        if time.time() - t0 > timeout:
            raise TimeoutError("no slot or budget became free")
        time.sleep(0.0005)


def _equal(a, b):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k


@pytest.fixture(scope="module")
def ctx(gpu_required):
    c = abi.Context(abi.config_from_geometry(synth.Geometry(), max_cands=6))
    yield c
    c.close()


def test_each_result_is_the_same_alone_in_the_mix_and_against_the_oracle(ctx):
    """A mix of events (500 to 50,000 tracks, 30 % noise) submitted while
    others are in flight, the 50,000-track one in the middle: every ticket
    equals the same event served alone, field by field, and sampled seeds of
    every event agree with the oracle."""
    ctx.serve_config(8 << 30, max_in_flight=16)
    sizes = (3000, 700, 50000, 5000, 1200, 90, 20000)
    evs = [synth.make_event(n, cfg=220, event=i, noise=0.3) for i, n in enumerate(sizes)]
    alone = []
    for i, e in enumerate(evs):
        print(f"case serve alone: event {i} ({e.n_seeds} tracks)", flush=True)
        t = _submit_retry(ctx, e)
        st, lat, out = _wait(ctx, [t])[t]
        assert st == abi.OK and lat > 0
        alone.append(out)
    print("case serve mix: 3 rounds of 7 events", flush=True)
    tickets = []
    for j, e in enumerate(evs * 3):
        tickets.append((j % len(evs), _submit_retry(ctx, e)))
        if j % 4 == 0:
            time.sleep(0.0005)
    res = _wait(ctx, [t for _, t in tickets])
    for i, t in tickets:
        st, lat, out = res[t]
        assert st == abi.OK and lat > 0
        _equal(out, alone[i])
    # sampled seeds of every served event against the oracle
    rng = np.random.default_rng(31)
    for i, (e, out) in enumerate(zip(evs, alone)):
        rows = np.sort(rng.choice(e.n_seeds, min(150, e.n_seeds), replace=False)).astype(np.int32)
        print(f"case serve oracle parity: event {i}, {len(rows)} seeds", flush=True)
        cfg = oracle.config(e.geometry, max_cands=6)
        o = oracle.build_tracks(cfg, e.hits, e.seed_par, e.seed_cov, e.seed_hits, seed_ids=rows, n_threads=16)
        rep = compare_build(out, o, cfg, e.hits, e.seed_par, e.seed_cov, rows=rows)
        report(f"serve_event{i}_{e.n_seeds}", rep)
        assert_build_parity(rep, max_tie_frac=0.05)
    # and the served result equals the plain builder on the loaded event
    h = ctx.load_event(evs[2])
    try:
        ref = ctx.build(h, evs[2].n_seeds)
    finally:
        ctx.unload_event(h)
    _equal(ref, alone[2])


def test_admission_takes_a_slot_and_budget_at_submit(ctx):
    """With one in-flight slot a second submit is refused with MKF_E_AGAIN
    until the first finishes; with a budget of about one event likewise; an
    event larger than the budget is refused with MKF_E_NOMEM; refused events
    are taken once the budget is free again and give identical results."""
    big = synth.make_event(20000, cfg=221, event=0, noise=0.3)
    small = synth.make_event(400, cfg=221, event=1, noise=0.3)
    ctx.serve_config(1 << 30, max_in_flight=1)
    print("case serve admission: one slot", flush=True)
    t1, _ = ctx.serve_submit(big)
    assert t1 is not None
    t2, _ = ctx.serve_submit(small)
    assert t2 is None                                   # MKF_E_AGAIN: the one slot is taken
    assert "slot" in abi.last_error()
    first = _wait(ctx, [t1])[t1]
    t2 = _submit_retry(ctx, small)
    second = _wait(ctx, [t2])[t2]
    assert first[0] == abi.OK and second[0] == abi.OK
    # a budget that holds one 4,000-track event at a time (its hits, seeds,
    # outputs and an index on its own 1024 x 16 grid take about 6 MB)
    ev = synth.make_event(4000, cfg=221, event=2, noise=0.3)
    ctx.serve_config(10 << 20, max_in_flight=8)
    print("case serve admission: tight budget", flush=True)
    ta, _ = ctx.serve_submit(ev)
    assert ta is not None
    tb, _ = ctx.serve_submit(ev)
    refused = tb is None
    if refused:
        assert "budget" in abi.last_error()
    outs = [_wait(ctx, [ta])[ta][2]]
    for _ in range(3):
        t = _submit_retry(ctx, ev)
        outs.append(_wait(ctx, [t])[t][2])
    if not refused:
        outs.append(_wait(ctx, [tb])[tb][2])
    for o in outs[1:]:
        _equal(o, outs[0])
    huge = synth.make_event(60000, cfg=221, event=3, noise=0.3)
    with pytest.raises(abi.MkfError) as e:
        ctx.serve_submit(huge)
    assert e.value.status == abi.E_NOMEM
    report("serve_admission", dict(budget_refused=bool(refused)))
    assert refused


def test_tuning_changes_do_not_reach_serving(ctx):
    """The context's tuning changed while events are in flight: serving
    keeps the launch shapes it was configured with, and the results are
    those of the same events served before the change."""
    ctx.set_tuning(bins_phi=2048, bins_z=32)
    ctx.serve_config(2 << 30, max_in_flight=8)
    evs = [synth.make_event(n, cfg=223, event=i, noise=0.3) for i, n in enumerate((6000, 2500, 800))]
    print("case serve tuning: reference", flush=True)
    ref = [_wait(ctx, [t])[t][2] for t in [_submit_retry(ctx, e) for e in evs]]
    print("case serve tuning: change while in flight", flush=True)
    tickets = [_submit_retry(ctx, e) for e in evs]
    ctx.set_tuning(bins_phi=64, bins_z=4, waves_per_block=2)
    tickets += [_submit_retry(ctx, e) for e in evs]
    res = _wait(ctx, tickets)
    for j, t in enumerate(tickets):
        assert res[t][0] == abi.OK
        _equal(res[t][2], ref[j % 3])
    ctx.set_tuning(bins_phi=2048, bins_z=32, waves_per_block=1)


def test_ticket_api(ctx):
    ctx.serve_config(1 << 30, max_in_flight=4, max_batch_events=1)
    ev = synth.make_event(20000, cfg=222, event=0, noise=0.1)
    small = synth.make_event(100, cfg=222, event=1, noise=0.1)
    print("case serve tickets", flush=True)
    first = [_submit_retry(ctx, ev) for _ in range(3)]
    last = _submit_retry(ctx, small)
    try:
        ctx.serve_cancel(last)
        cancelled = True
    except abi.MkfError as e:
        assert e.status == abi.E_STATE     # already started
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
    # the slots are free again
    t = _submit_retry(ctx, small, timeout=5.0)
    assert _wait(ctx, [t])[t][0] == abi.OK
    with pytest.raises(abi.MkfError) as e:
        ctx.serve_poll(123456789)
    assert e.value.status == abi.E_NOTFOUND
    bad = [h.copy() for h in small.hits]
    bad[0][0, 0] = np.inf
    with pytest.raises(abi.MkfError) as e:
        ctx.serve_submit(abi.EventArrays(bad, small.seed_par, small.seed_cov, small.seed_hits))
    assert e.value.status == abi.E_INVALID
