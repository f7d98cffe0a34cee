"""Pins of the oracle's combinatorial track building.

The beam search is checked against an exhaustive enumeration of every
hit/hole path on tiny events, the one-candidate beam against a greedy
minimum-chi2 walk, exact recovery on perfect hits, the hole and stop rules
on hand-made events, and a stored regression fixture.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1702_06359_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _no_material():
    return synth.Geometry(x0=tuple(0.0 for _ in range(10)))


def test_build_exact_recovery_with_perfect_hits():
    geo = _no_material()
    ev = synth.make_event(300, cfg=95, event=0, geometry=geo, smear=False, scatter=False)
    cfg = oracle.config(geo, max_cands=6)
    seed = ev.truth_par[:, 2].copy()
    out = oracle.build_tracks(cfg, ev.hits, seed, ev.seed_cov, ev.seed_hits, n_threads=4)
    assert (out["hits"][:, :10] == ev.truth_hit).all()
    assert (out["n_hits"] == 10).all() and (out["status"] == 0).all()
    d = out["par"] - ev.truth_par[:, 9]
    d[:, 4] = (d[:, 4] + np.pi) % (2 * np.pi) - np.pi
    assert np.abs(d / np.maximum(np.abs(ev.truth_par[:, 9]), 1.0)).max() < 1e-10
    assert np.abs(out["chi2"]).max() < 1e-12


def _enumerate_paths(cfg, hits, sp, sc, sh):
    """Every path the building rules allow, each Kalman-filtered, with no beam limit."""
    nsl, nl = cfg.n_seed_layers, cfg.n_layers
    start = dict(par=np.array(sp), C=synth.unpack_sym(np.asarray(sc)), chi2=0.0,
                 n_hits=int((np.asarray(sh) >= 0).sum()), n_holes=0,
                 hits=list(sh) + [-1] * (nl - nsl), status=0, stopped=False)
    paths = [start]
    max_live = 1
    for L in range(nsl, nl):
        nxt = []
        for pth in paths:
            if pth["stopped"]:
                nxt.append(pth)
                continue
            Cm = oracle.add_ms(pth["par"], pth["C"], cfg.x0[L - 1], cfg.mass)
            ok, pp, F, _, _ = oracle.propagate(pth["par"], cfg.radius[L], cfg.bz)
            if not ok:
                nxt.append(dict(pth, stopped=True, status=2))
                continue
            Cp = oracle.transport(F, Cm)
            acc = []
            for j, h in enumerate(hits[L]):
                if h[0] * pp[0] + h[1] * pp[1] <= 0:
                    continue
                if oracle.chi2(pp, Cp, h, cfg.sigma_rphi, cfg.sigma_z) < cfg.chi2_cut:
                    acc.append(j)
            for j in acc:
                pu, Cu, c2 = oracle.update(pp, Cp, hits[L][j], cfg.sigma_rphi, cfg.sigma_z)
                hl = list(pth["hits"])
                hl[L] = j
                nxt.append(dict(pth, par=pu, C=Cu, chi2=pth["chi2"] + c2, n_hits=pth["n_hits"] + 1,
                                hits=hl))
            if not acc:
                if pth["n_holes"] < cfg.max_holes:
                    nxt.append(dict(pth, par=pp, C=Cp, n_holes=pth["n_holes"] + 1))
                else:
                    nxt.append(dict(pth, par=pp, C=Cp, stopped=True, status=1))
        paths = nxt
        max_live = max(max_live, len(paths))
    paths.sort(key=lambda q: (-q["n_hits"], q["chi2"]))
    return paths, max_live


def _tiny_event(rng_seed, branch_layers=(3, 5, 7), n_tracks=2):
    ev = synth.make_event(n_tracks, cfg=96, event=rng_seed, noise=0.0)
    rng = np.random.default_rng(rng_seed)
    hits = [h.copy() for h in ev.hits]
    for L in branch_layers:
        r = ev.geometry.radii[L]
        h = hits[L][ev.truth_hit[0, L]]
        ph = math.atan2(h[1], h[0]) + rng.choice([-1, 1]) * 0.015 / r
        extra = np.array([[r * math.cos(ph), r * math.sin(ph), h[2] + rng.normal(0, 0.12)]])
        hits[L] = np.concatenate([hits[L], extra])
    return ev, hits


@pytest.mark.parametrize("rng_seed", [0, 1, 2, 3, 4, 5])
def test_beam_equals_exhaustive_enumeration_on_tiny_events(rng_seed):
    ev, hits = _tiny_event(rng_seed)
    cfg = oracle.config(ev.geometry, max_cands=16)
    for s in range(ev.n_seeds):
        paths, max_live = _enumerate_paths(cfg, hits, ev.seed_par[s], ev.seed_cov[s], ev.seed_hits[s])
        assert max_live <= 16
        out = oracle.build_tracks(cfg, hits, ev.seed_par, ev.seed_cov, ev.seed_hits, seed_ids=[s])[0]
        best = paths[0]
        assert list(out["hits"][:10]) == best["hits"]
        assert out["chi2"] == pytest.approx(best["chi2"], rel=1e-12, abs=1e-12)
        assert out["n_final"] == len(paths)
        assert np.allclose(out["par"], best["par"], rtol=1e-12, atol=1e-12)
        if s == 0:
            assert max_live >= 2      # the planted hits really branch the search
        # nothing was pruned (max_live <= 16), so the whole final beam is every
        # path, in the beam order
        _, beam = oracle.build_beam(cfg, hits, ev.seed_par, ev.seed_cov, ev.seed_hits, seed_ids=[s])
        for r in range(16):
            if r < len(paths):
                assert list(beam[0, r]["hits"][:10]) == paths[r]["hits"]
                assert beam[0, r]["chi2"] == pytest.approx(paths[r]["chi2"], rel=1e-12, abs=1e-12)
                assert np.allclose(beam[0, r]["par"], paths[r]["par"], rtol=1e-12, atol=1e-12)
            else:
                assert beam[0, r]["status"] == -1


@pytest.mark.parametrize("rng_seed", [0, 1, 2])
def test_best_hit_equals_greedy_minimum_chi2_walk(rng_seed):
    """With one candidate per seed the beam keeps, per layer, the accepted hit
    of smallest chi2 (lowest index on ties), or a hole."""
    ev, hits = _tiny_event(rng_seed, branch_layers=(3, 4, 6, 8), n_tracks=4)
    cfg = oracle.config(ev.geometry, max_cands=1)
    out = oracle.build_tracks(cfg, hits, ev.seed_par, ev.seed_cov, ev.seed_hits)
    for s in range(ev.n_seeds):
        par = ev.seed_par[s].copy()
        Cm = synth.unpack_sym(ev.seed_cov[s])
        walk = list(ev.seed_hits[s]) + [-1] * 7
        holes = 0
        total = 0.0
        for L in range(3, 10):
            Cm = oracle.add_ms(par, Cm, cfg.x0[L - 1], cfg.mass)
            ok, par, F, _, _ = oracle.propagate(par, cfg.radius[L], cfg.bz)
            assert ok
            Cm = oracle.transport(F, Cm)
            c2 = [(oracle.chi2(par, Cm, h, 0.01, 0.1), j) for j, h in enumerate(hits[L])
                  if h[0] * par[0] + h[1] * par[1] > 0]
            c2 = [c for c in c2 if c[0] < 30.0]
            if c2:
                best = min(c2)
                par, Cm, v = oracle.update(par, Cm, hits[L][best[1]], 0.01, 0.1)
                walk[L] = best[1]
                total += v
            else:
                holes += 1
                if holes > 1:
                    break
        assert list(out[s]["hits"][:10]) == walk
        assert out[s]["chi2"] == pytest.approx(total, rel=1e-12, abs=1e-12)


def test_hole_then_stop_when_layers_are_empty():
    ev = synth.make_event(50, cfg=97, event=0, noise=0.0)
    hits = [h.copy() for h in ev.hits]
    for L in (6, 7, 8, 9):
        hits[L] = np.zeros((0, 3))
    cfg = oracle.config(ev.geometry, max_cands=6, max_holes=1)
    out = oracle.build_tracks(cfg, hits, ev.seed_par, ev.seed_cov, ev.seed_hits)
    assert (out["status"] == 1).all()
    assert (out["n_holes"] == 1).all()
    assert (out["hits"][:, 6:10] == -1).all()
    assert (out["hits"][:, 3:6] == ev.truth_hit[:, 3:6]).all()
    assert (out["n_hits"] == 6).all()
    # the stopped candidate keeps its prediction on the layer where it stopped (layer 7)
    r = np.hypot(out["par"][:, 0], out["par"][:, 1])
    assert np.allclose(r, ev.geometry.radii[7], atol=1e-9)
    # with no hole allowance it stops on layer 6 instead
    cfg0 = oracle.config(ev.geometry, max_cands=6, max_holes=0)
    out0 = oracle.build_tracks(cfg0, hits, ev.seed_par, ev.seed_cov, ev.seed_hits)
    assert (out0["status"] == 1).all() and (out0["n_holes"] == 0).all()
    assert np.allclose(np.hypot(out0["par"][:, 0], out0["par"][:, 1]), ev.geometry.radii[6], atol=1e-9)


def test_propagation_failure_keeps_previous_surface():
    """0.15 GeV tracks curl inside 2R = 26.3 cm: they cross layer 5 (r = 24 cm)
    but never reach layer 6, so every candidate stops there with its state on
    layer 5."""
    ev = synth.make_event(30, cfg=98, event=0, noise=0.0, pt_range=(0.15, 0.15), eta_max=0.5)
    cfg = oracle.config(ev.geometry, max_cands=3)
    out = oracle.build_tracks(cfg, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits)
    assert (out["status"] == 2).all()
    assert (out["hits"][:, 3:6] == ev.truth_hit[:, 3:6]).all()
    assert (out["hits"][:, 6:10] == -1).all()
    r = np.hypot(out["par"][:, 0], out["par"][:, 1])
    assert np.allclose(r, ev.geometry.radii[5], atol=5e-3)   # the update moves along the tangent
    assert (out["m_prop"] > 0).all()


def test_best_hit_efficiency_on_clean_event():
    """1,000 tracks, no noise, one candidate per seed: nearly every track
    collects its own seven hits (a bug catcher; the paper's curve is absent)."""
    ev = synth.best_hit_event(1000)
    cfg = oracle.config(ev.geometry, max_cands=1)
    out = oracle.build_tracks(cfg, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits, n_threads=8)
    good = (out["hits"][:, :10] == ev.truth_hit).all(axis=1)
    assert good.mean() >= 0.95
    per_hit = (out["hits"][:, 3:10] == ev.truth_hit[:, 3:10]).mean()
    assert per_hit >= 0.98


def test_combinatorial_beats_best_hit_with_noise():
    ev = synth.make_event(1500, cfg=99, event=0, noise=0.3)
    eff = {}
    for k in (1, 6):
        cfg = oracle.config(ev.geometry, max_cands=k)
        out = oracle.build_tracks(cfg, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits, n_threads=8)
        eff[k] = (out["hits"][:, :10] == ev.truth_hit).all(axis=1).mean()
        # built covariances are rank 5 and positive on the other five directions
        for i in range(0, 1500, 25):
            w = np.linalg.eigvalsh(synth.unpack_sym(out["cov"][i]))
            assert abs(w[0]) <= 1e-10 * w.sum() and w[1] > 0
    assert eff[6] >= eff[1]


def test_matches_stored_regression_fixture():
    with open(os.path.join(GOLDEN, "oracle_build_small.json")) as f:
        gold = json.load(f)
    ev = synth.make_event(gold["n_tracks"], cfg=gold["cfg"], event=gold["event"], noise=gold["noise"])
    cfg = oracle.config(ev.geometry, max_cands=gold["k"])
    out = oracle.build_tracks(cfg, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits)
    assert out["hits"][:, :10].tolist() == gold["hits"]
    assert np.allclose(out["chi2"], gold["chi2"], rtol=1e-10, atol=1e-10)
    assert np.allclose(out["par"], gold["par"], rtol=1e-10, atol=1e-12)


def test_replay_reproduces_built_chi2():
    """Replaying the hits a build chose gives back its chi2 and passes the cut."""
    ev = synth.make_event(200, cfg=101, event=0, noise=0.2)
    cfg = oracle.config(ev.geometry, max_cands=6)
    out = oracle.build_tracks(cfg, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits, n_threads=4)
    hs = oracle.HitSet(ev.hits)
    for i in range(0, 200, 7):
        if out["status"][i] != 0:
            continue
        tot, per_layer, ok = oracle.replay(cfg, hs, ev.seed_par[i], ev.seed_cov[i], out["hits"][i])
        assert ok
        assert tot == pytest.approx(out["chi2"][i], rel=1e-12, abs=1e-12)
        assert ((per_layer[3:] < 30.0) | (out["hits"][i, 3:10] < 0)).all()
