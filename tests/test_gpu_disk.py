"""GPU building and fitting on endcap disks against the FP64 oracle.

Same protocol as the barrel tests: identical hit lists for every seed the
oracle does not flag as tie-sensitive, states and covariances (in the disk
frame u, r, q/pT, phi, theta) within the frozen FP32 tolerances.
"""
import numpy as np
import pytest

import oracle
from conftest import report
from paper_1702_06359_amd import abi, synth
from parity_util import assert_build_parity, compare_build
from test_gpu_fit import _check

pytestmark = pytest.mark.gpu

FIELDS = ("par", "cov", "hits", "n_hits", "n_holes", "chi2", "status", "ndof")
GEO = synth.Geometry.endcap()


def _ctx(k, **tuning):
    c = abi.Context(abi.config_from_geometry(GEO, max_cands=k))
    if tuning:
        c.set_tuning(**tuning)
    return c


@pytest.fixture(scope="module")
def ctx6(gpu_required):
    c = _ctx(6)
    yield c
    c.close()


def _equal(a, b):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k


def _oracle(ev, k, rows=None, threads=8):
    cfg = oracle.config(ev.geometry, max_cands=k)
    return cfg, oracle.build_tracks(cfg, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits, seed_ids=rows,
                                    n_threads=threads)


def test_disk_best_hit_parity(gpu_required):
    ev = synth.make_event(1000, cfg=230, event=0, geometry=GEO, noise=0.0)
    print("case disk best_hit n=1000 k=1", flush=True)
    c = _ctx(1)
    try:
        h = c.load_event(ev)
        g = c.build_batch([h], [ev.n_seeds])[0]
    finally:
        c.close()
    cfg, o = _oracle(ev, 1)
    rep = compare_build(g, o, cfg, ev.hits, ev.seed_par, ev.seed_cov)
    report("disk_best_hit_1000", rep)
    assert_build_parity(rep)


def test_disk_combinatorial_parity_ragged(ctx6):
    ev = synth.make_event(2003, cfg=231, event=0, geometry=GEO, noise=0.3)
    print("case disk ckf n=2003 k=6 noise=0.3 plain+batched", flush=True)
    h = ctx6.load_event(ev)
    try:
        g = ctx6.build(h, ev.n_seeds)
        gb = ctx6.build_batch([h], [ev.n_seeds])[0]
    finally:
        ctx6.unload_event(h)
    _equal(g, gb)
    cfg, o = _oracle(ev, 6)
    rep = compare_build(g, o, cfg, ev.hits, ev.seed_par, ev.seed_cov)
    report("disk_ckf_2003", rep)
    assert_build_parity(rep)
    assert (g["hits"] == ev.truth_hit).all(1).mean() > 0.85


def test_disk_full_size_events_sampled_seeds(ctx6):
    """The endcap workload the benchmark times (ten events of 10,000 tracks,
    10 % noise; one-block-per-layer index, one batched launch); 60 sampled
    seeds per event."""
    evs = synth.endcap_events(10)
    hs = [ctx6.load_event(e) for e in evs]
    try:
        print("case disk ckf full size 10x10000 batched", flush=True)
        outs = ctx6.build_batch(hs, [e.n_seeds for e in evs], flags=abi.BATCH_REINDEX)
    finally:
        for h in hs:
            ctx6.unload_event(h)
    rng = np.random.default_rng(17)
    for i, (ev, g) in enumerate(zip(evs, outs)):
        rows = np.sort(rng.choice(ev.n_seeds, 60, replace=False)).astype(np.int32)
        cfg, o = _oracle(ev, 6, rows=rows, threads=16)
        rep = compare_build(g, o, cfg, ev.hits, ev.seed_par, ev.seed_cov, rows=rows)
        report(f"disk_ckf_full_event{i}", rep)
        assert_build_parity(rep, max_tie_frac=0.02)


def test_disk_launch_shapes_do_not_change_results(gpu_required):
    ev = synth.make_event(1200, cfg=232, event=0, geometry=GEO, noise=0.3)
    ref = None
    for sh in (dict(), dict(bins_phi=64, bins_z=4), dict(bins_phi=2048, bins_z=128), dict(persistent=1),
               dict(lanes_per_seed=8, waves_per_block=2)):
        c = _ctx(6, **sh)
        try:
            print(f"case disk shapes {sh}", flush=True)
            h = c.load_event(ev)
            a = c.build(h, ev.n_seeds)
            b = c.build_batch([h], [ev.n_seeds])[0]
        finally:
            c.close()
        _equal(a, b)
        if ref is None:
            ref = a
        else:
            _equal(ref, a)


def test_disk_fit_parity_true_hits(ctx6):
    ev = synth.make_event(3001, cfg=233, event=0, geometry=GEO, noise=0.1)
    print("case disk fit n=3001", flush=True)
    h = ctx6.load_event(abi.EventArrays(ev.hits))
    try:
        g = ctx6.fit(h, ev.prior_par, ev.prior_cov, ev.truth_hit)
    finally:
        ctx6.unload_event(h)
    o = oracle.fit(oracle.config(GEO), ev.hits, ev.prior_par, ev.prior_cov, ev.truth_hit, n_threads=8)
    _check("disk_fit_true_hits", g, o, prior_cov=ev.prior_cov, disk=True)


def test_disk_build_then_fit_on_device(gpu_required):
    c = _ctx(6)
    ev = synth.make_event(2500, cfg=234, event=0, geometry=GEO, noise=0.1)
    h = c.load_event(ev)
    try:
        print("case disk build+fit n=2500", flush=True)
        built = c.build_batch([h], [ev.n_seeds], flags=abi.BATCH_REINDEX | abi.BATCH_FIT)[0]
        g = c.fetch_fit(h, ev.n_seeds)
    finally:
        c.close()
    cfg = oracle.config(GEO)
    par, cov, ok = oracle.circle_prior(cfg, ev.hits, built["hits"])
    assert ok.all()
    o = oracle.fit(cfg, ev.hits, par, cov, built["hits"], n_threads=8)
    _check("disk_build_then_fit", g, o, prior_cov=cov, disk=True)


def test_mixed_layer_kinds_are_rejected(gpu_required):
    cfg = abi.config_from_geometry(GEO, max_cands=2)
    cfg.layer_kind[5] = 0
    with pytest.raises(abi.MkfError):
        abi.Context(cfg)
    cfg = abi.config_from_geometry(GEO, max_cands=2)
    cfg.sigma_r = 0.0
    with pytest.raises(abi.MkfError):
        abi.Context(cfg)


def test_disk_edge_cases(ctx6):
    """Empty outer disks (hole, then stop), seeds heading away from the next
    disk (propagation fails: status 2, state kept on the seed's disk), and a
    disk whose extra hits all sit beyond the grid's outer radius (one edge
    bin): parity with the oracle in each."""
    ev = synth.make_event(300, cfg=235, event=0, geometry=GEO, noise=0.2)

    def run(hits, sp):
        h = ctx6.load_event(abi.EventArrays(hits, sp, ev.seed_cov, ev.seed_hits))
        try:
            g = ctx6.build(h, ev.n_seeds)
            b = ctx6.build_batch([h], [ev.n_seeds])[0]
        finally:
            ctx6.unload_event(h)
        _equal(g, b)
        e2 = synth.Event(GEO, hits, sp, ev.seed_cov, ev.seed_hits, ev.truth_hit, ev.truth_par, ev.vertex_par,
                         ev.prior_par, ev.prior_cov, ev.n_noise)
        cfg, o = _oracle(e2, 6)
        assert_build_parity(compare_build(g, o, cfg, hits, sp, ev.seed_cov))
        return g, o

    hits = [x.copy() for x in ev.hits]
    for L in (7, 8, 9):
        hits[L] = np.zeros((0, 3))
    print("case disk edge: empty outer disks", flush=True)
    g, _ = run(hits, ev.seed_par)
    assert (g["status"] == 1).all()
    sp = ev.seed_par.copy()
    sp[::3, 5] = np.pi - sp[::3, 5]          # every third seed heads to -z
    print("case disk edge: seeds heading away", flush=True)
    g, o = run(ev.hits, sp)
    assert (g["status"][::3] == 2).all() and (o["status"][::3] == 2).all()
    assert np.allclose(g["par"][::3, 2], GEO.disk_z[2], atol=1e-4)
    crowd = [x.copy() for x in ev.hits]
    crowd[5] = np.concatenate([crowd[5], np.tile([[100.0, 0.0, GEO.disk_z[5]]], (5000, 1))])
    print("case disk edge: crowded outer edge bin", flush=True)
    run(crowd, ev.seed_par)
