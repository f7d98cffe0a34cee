"""GPU two-step building and fitting on layers of finite thickness, and the
3x3 global-Cartesian measurement, against the FP64 oracle (barrel cylinders
and endcap disks).

Same protocol as the thin-layer tests: identical hit lists for every seed
the oracle does not flag as tie-sensitive, states and covariances within the
frozen FP32 tolerances.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from conftest import report
from paper_1702_06359_amd import abi, synth
from parity_util import assert_build_parity, compare_build
from test_gpu_fit import _check

pytestmark = pytest.mark.gpu

FIELDS = ("par", "cov", "hits", "n_hits", "n_holes", "chi2", "status", "ndof")
BARREL = synth.Geometry(thickness=tuple(0.6 for _ in range(10)))
ENDCAP = dataclasses.replace(synth.Geometry.endcap(), thickness=tuple(1.0 for _ in range(10)))


def _ctx(g, k, **tuning):
    c = abi.Context(abi.config_from_geometry(g, max_cands=k))
    if tuning:
        c.set_tuning(**tuning)
    return c


def _equal(a, b):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k


def _oracle(ev, k, rows=None, threads=8):
    cfg = oracle.config(ev.geometry, max_cands=k)
    return cfg, oracle.build_tracks(cfg, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits, seed_ids=rows,
                                    n_threads=threads)


@pytest.mark.parametrize("name,g", [("barrel", BARREL), ("endcap", ENDCAP)])
def test_thick_best_hit_parity(gpu_required, name, g):
    ev = synth.make_event(1000, cfg=240, event=0, geometry=g, noise=0.0)
    print(f"case thick {name} best_hit n=1000 k=1", flush=True)
    c = _ctx(g, 1)
    try:
        h = c.load_event(ev)
        out = c.build_batch([h], [ev.n_seeds])[0]
    finally:
        c.close()
    cfg, o = _oracle(ev, 1)
    rep = compare_build(out, o, cfg, ev.hits, ev.seed_par, ev.seed_cov)
    report(f"thick_{name}_best_hit_1000", rep)
    assert_build_parity(rep)


@pytest.mark.parametrize("name,g", [("barrel", BARREL), ("endcap", ENDCAP)])
def test_thick_combinatorial_parity_ragged(gpu_required, name, g):
    ev = synth.make_event(2003, cfg=241, event=0, geometry=g, noise=0.3)
    print(f"case thick {name} ckf n=2003 k=6 noise=0.3 plain+batched", flush=True)
    c = _ctx(g, 6)
    try:
        h = c.load_event(ev)
        a = c.build(h, ev.n_seeds)
        b = c.build_batch([h], [ev.n_seeds])[0]
    finally:
        c.close()
    _equal(a, b)
    cfg, o = _oracle(ev, 6)
    rep = compare_build(a, o, cfg, ev.hits, ev.seed_par, ev.seed_cov)
    report(f"thick_{name}_ckf_2003", rep)
    assert_build_parity(rep)


def test_thick_full_size_sampled_seeds(gpu_required):
    """The two-step workload the benchmark times (ten 20,000-track events on
    the 6 mm deep barrel, 10 % noise; one-block-per-layer index, one batched
    launch); 40 sampled seeds per event."""
    evs = [synth.make_event(20000, cfg=5, event=e, geometry=BARREL, noise=0.1) for e in range(10)]
    c = _ctx(BARREL, 6)
    try:
        hs = [c.load_event(e) for e in evs]
        print("case thick barrel ckf full size 10x20000 batched", flush=True)
        outs = c.build_batch(hs, [e.n_seeds for e in evs], flags=abi.BATCH_REINDEX)
    finally:
        c.close()
    rng = np.random.default_rng(27)
    for i, (ev, g) in enumerate(zip(evs, outs)):
        rows = np.sort(rng.choice(ev.n_seeds, 40, replace=False)).astype(np.int32)
        cfg, o = _oracle(ev, 6, rows=rows, threads=16)
        rep = compare_build(g, o, cfg, ev.hits, ev.seed_par, ev.seed_cov, rows=rows)
        report(f"thick_barrel_full_event{i}", rep)
        assert_build_parity(rep, max_tie_frac=0.02)


def test_thick_launch_shapes_do_not_change_results(gpu_required):
    ev = synth.make_event(1200, cfg=243, event=0, geometry=BARREL, noise=0.3)
    ref = None
    for sh in (dict(), dict(bins_phi=64, bins_z=4), dict(bins_phi=2048, bins_z=128), dict(persistent=1),
               dict(lanes_per_seed=8, waves_per_block=2)):
        c = _ctx(BARREL, 6, **sh)
        try:
            print(f"case thick shapes {sh}", flush=True)
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


@pytest.mark.parametrize("name,g", [("barrel", BARREL), ("endcap", ENDCAP)])
def test_thick_fit_parity_true_hits(gpu_required, name, g):
    ev = synth.make_event(3001, cfg=244, event=0, geometry=g, noise=0.1)
    print(f"case thick {name} fit n=3001", flush=True)
    c = _ctx(g, 6)
    try:
        h = c.load_event(abi.EventArrays(ev.hits))
        out = c.fit(h, ev.prior_par, ev.prior_cov, ev.truth_hit)
    finally:
        c.close()
    o = oracle.fit(oracle.config(g), ev.hits, ev.prior_par, ev.prior_cov, ev.truth_hit, n_threads=8)
    _check(f"thick_{name}_fit", out, o, prior_cov=ev.prior_cov, disk=g.is_disk)


def test_thick_build_then_fit_on_device(gpu_required):
    ev = synth.make_event(2500, cfg=245, event=0, geometry=BARREL, noise=0.1)
    c = _ctx(BARREL, 6)
    try:
        h = c.load_event(ev)
        print("case thick build+fit n=2500", flush=True)
        built = c.build_batch([h], [ev.n_seeds], flags=abi.BATCH_REINDEX | abi.BATCH_FIT)[0]
        g = c.fetch_fit(h, ev.n_seeds)
    finally:
        c.close()
    cfg = oracle.config(BARREL)
    par, cov, ok = oracle.circle_prior(cfg, ev.hits, built["hits"])
    assert ok.all()
    o = oracle.fit(cfg, ev.hits, par, cov, built["hits"], n_threads=8)
    _check("thick_build_then_fit", g, o, prior_cov=cov)


def test_mixed_thickness_is_rejected(gpu_required):
    cfg = abi.config_from_geometry(BARREL, max_cands=2)
    cfg.layer_thickness[4] = 0.0
    with pytest.raises(abi.MkfError):
        abi.Context(cfg)
    cfg = abi.config_from_geometry(BARREL, max_cands=2)
    cfg.layer_thickness[0] = 9.0          # deeper than twice the radius
    with pytest.raises(abi.MkfError):
        abi.Context(cfg)


@pytest.mark.parametrize("name,g", [("thin_barrel", synth.Geometry()), ("thick_endcap", ENDCAP)])
def test_update3d_build_parity(gpu_required, name, g):
    """The 3x3 global-Cartesian measurement (MKF_UPDATE_3D) in the build."""
    ev = synth.make_event(2003, cfg=246, event=0, geometry=g, noise=0.3)
    print(f"case update3d {name} ckf n=2003 k=6", flush=True)
    c = abi.Context(abi.config_from_geometry(g, max_cands=6, update3d=True))
    try:
        h = c.load_event(ev)
        a = c.build(h, ev.n_seeds)
        b = c.build_batch([h], [ev.n_seeds])[0]
    finally:
        c.close()
    _equal(a, b)
    cfg = oracle.config(g, max_cands=6, update3d=True)
    o = oracle.build_tracks(cfg, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits, n_threads=8)
    rep = compare_build(a, o, cfg, ev.hits, ev.seed_par, ev.seed_cov)
    report(f"update3d_{name}_ckf_2003", rep)
    assert_build_parity(rep)


@pytest.mark.parametrize("name,g", [("thin_barrel", synth.Geometry()), ("thick_barrel", BARREL)])
def test_update3d_fit_parity(gpu_required, name, g):
    ev = synth.make_event(3001, cfg=247, event=0, geometry=g, noise=0.1)
    print(f"case update3d {name} fit n=3001", flush=True)
    c = abi.Context(abi.config_from_geometry(g, max_cands=6, update3d=True))
    try:
        h = c.load_event(abi.EventArrays(ev.hits))
        out = c.fit(h, ev.prior_par, ev.prior_cov, ev.truth_hit)
    finally:
        c.close()
    o = oracle.fit(oracle.config(g, update3d=True), ev.hits, ev.prior_par, ev.prior_cov, ev.truth_hit, n_threads=8)
    _check(f"update3d_{name}_fit", out, o, prior_cov=ev.prior_cov, disk=g.is_disk)


def test_update3d_needs_sigma_r(gpu_required):
    cfg = abi.config_from_geometry(synth.Geometry(), max_cands=2, update3d=True)
    cfg.sigma_r = 0.0
    with pytest.raises(abi.MkfError):
        abi.Context(cfg)


def test_thick_edge_cases(gpu_required):
    """Empty outer thick layers (hole, then stop on the average surface) and
    a layer with 5,000 extra hits in one edge bin: parity with the oracle."""
    ev = synth.make_event(300, cfg=248, event=0, geometry=BARREL, noise=0.2)
    c = _ctx(BARREL, 6)
    try:
        for name, mod in (("empty outer layers", lambda h: [np.zeros((0, 3)) if L >= 7 else x for L, x in enumerate(h)]),
                          ("crowded edge bin", lambda h: [np.concatenate([x, np.tile([[20.1, 0.0, 1e4]], (5000, 1))])
                                                          if L == 5 else x for L, x in enumerate(h)])):
            hits = mod([x.copy() for x in ev.hits])
            print(f"case thick edge: {name}", flush=True)
            h = c.load_event(abi.EventArrays(hits, ev.seed_par, ev.seed_cov, ev.seed_hits))
            g = c.build(h, ev.n_seeds)
            c.unload_event(h)
            e2 = synth.Event(BARREL, hits, ev.seed_par, ev.seed_cov, ev.seed_hits, ev.truth_hit, ev.truth_par,
                             ev.vertex_par, ev.prior_par, ev.prior_cov, ev.n_noise)
            cfg, o = _oracle(e2, 6)
            assert_build_parity(compare_build(g, o, cfg, hits, ev.seed_par, ev.seed_cov))
            if name == "empty outer layers":
                assert (g["status"] == 1).all()
                r = np.hypot(g["par"][:, 0], g["par"][:, 1])
                assert np.allclose(r, BARREL.radii[8], atol=1e-3)   # hole on 7, stopped on 8
    finally:
        c.close()
