"""Pins of the oracle's two-step propagation on layers of finite thickness.

The second step (average surface -> the hit's own surface, ahead or behind)
is checked against a Runge-Kutta integration, against the forward
propagation of the time-reversed state, by reversibility and by finite
differences; the build's use of it against an exhaustive enumeration of
every path on tiny thick events; the whole against unit-width pulls of fits
on generated thick events, and against the thin build when every hit lies
on its layer's average surface.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1702_06359_amd import synth
from test_oracle_propagation import random_states, rk4_to_radius

BZ = 3.8


def _wrapdiff(a, b):
    d = a - b
    d[4] = (d[4] + np.pi) % (2 * np.pi) - np.pi
    return d


def _reverse(p):
    r = p.copy()
    r[3] = -p[3]
    r[4] = p[4] + np.pi
    r[5] = np.pi - p[5]
    return r


def test_short_step_forward_matches_rk4_and_forward_propagation():
    rng = np.random.default_rng(31)
    for p in random_states(12, rng, r0=20.0, qpt_max=1.5):
        ok, p20, _, _, _ = oracle.propagate(p, 20.3, BZ, jacobian=False)   # a state moving outward at r = 20.3
        assert ok
        for r in (20.6, 21.0):
            ok, out, _, s = oracle.step_near(p20, 0, r, BZ, jacobian=False)
            assert ok and s > 0
            ref = rk4_to_radius(p20, r, BZ, h=0.005)
            assert np.abs(out[:3] - ref[:3]).max() < 1e-9
            ok2, fwd, _, s2, _ = oracle.propagate(p20, r, BZ, jacobian=False)
            assert ok2 and np.abs(_wrapdiff(out, fwd)).max() < 1e-12 and s == pytest.approx(s2, rel=1e-12)


def test_short_step_backward_equals_reversed_forward_propagation():
    rng = np.random.default_rng(32)
    for p in random_states(40, rng, r0=20.0):
        ok, p20, _, _, _ = oracle.propagate(p, 20.3, BZ, jacobian=False)
        assert ok
        for r in (19.8, 20.0, 20.29):
            ok, back, _, s = oracle.step_near(p20, 0, r, BZ, jacobian=False)
            assert ok and s < 0
            ok2, rev, _, s2, _ = oracle.propagate(_reverse(p20), r, BZ, jacobian=False)
            assert ok2 and s2 == pytest.approx(-s, rel=1e-10)
            assert np.abs(_wrapdiff(_reverse(rev), back)).max() < 1e-10
            # and back again lands on the start
            ok3, again, _, _ = oracle.step_near(back, 0, 20.3, BZ, jacobian=False)
            assert ok3 and np.abs(_wrapdiff(again, p20)).max() < 1e-10


def test_short_step_on_planes_both_directions():
    p = np.array([3.0, -1.0, 40.0, 0.8, 0.4, 0.3])
    for zd in (39.5, 40.0, 40.7):
        ok, out, _, s = oracle.step_near(p, 1, zd, BZ, jacobian=False)
        assert ok and out[2] == zd
        assert s == pytest.approx((zd - 40.0) * math.tan(0.3), rel=1e-14, abs=0.0)
        if zd > 40.0:
            ok2, fwd, _, _, _ = oracle.propagate_plane(p, zd, BZ, jacobian=False)
            assert np.abs(_wrapdiff(out, fwd)).max() < 1e-13


def test_short_step_jacobian_matches_central_differences():
    rng = np.random.default_rng(33)
    steps = np.array([1e-6, 1e-6, 1e-6, 1e-7, 1e-7, 1e-7])
    worst = 0.0
    for p in random_states(30, rng, r0=20.0):
        ok, p20, _, _, _ = oracle.propagate(p, 20.3, BZ, jacobian=False)
        for kind, where, base in ((0, 19.9, p20), (0, 20.8, p20), (1, p20[2] + 0.4, p20), (1, p20[2] - 0.4, p20)):
            ok, out, F, _ = oracle.step_near(base, kind, where, BZ)
            assert ok
            num = np.zeros((6, 6))
            for j in range(6):
                pp, pm = base.copy(), base.copy()
                pp[j] += steps[j]
                pm[j] -= steps[j]
                _, op, _, _ = oracle.step_near(pp, kind, where, BZ, jacobian=False)
                _, om, _, _ = oracle.step_near(pm, kind, where, BZ, jacobian=False)
                num[:, j] = _wrapdiff(op, om) / (2 * steps[j])
            worst = max(worst, float((np.abs(F - num) / np.maximum(np.abs(num), 1.0)).max()))
    assert worst < 1e-6


def _thick_barrel(t=0.6):
    return synth.Geometry(thickness=tuple(t for _ in range(10)))


def _thick_endcap(t=1.0):
    return dataclasses.replace(synth.Geometry.endcap(), thickness=tuple(t for _ in range(10)))


def test_generator_thick_hits_lie_on_the_helix():
    """Zero-noise hits of a thick layer sit on the true helix at their own
    radius (z on disks), spread over the layer's depth."""
    for g in (_thick_barrel(), _thick_endcap()):
        ev = synth.make_event(200, cfg=330, event=0, geometry=g, smear=False, scatter=False)
        for i in range(200):
            p = ev.vertex_par[i].copy()
            for L in range(10):
                h = ev.hits[L][ev.truth_hit[i, L]]
                if g.is_disk:
                    ok, p, _, _, _ = oracle.propagate_plane(p, h[2], g.bz, jacobian=False)
                else:
                    ok, p, _, _, _ = oracle.propagate(p, math.hypot(h[0], h[1]), g.bz, jacobian=False)
                assert ok and np.abs(p[:3] - h).max() < 1e-9
        surf = [np.abs((ev.hits[L][:, 2] - g.disk_z[L]) if g.is_disk else
                       (np.hypot(ev.hits[L][:, 0], ev.hits[L][:, 1]) - g.radii[L])) for L in range(10)]
        assert max(s.max() for s in surf) <= 0.5 * g.thick(0) + 1e-12
        assert min(s.max() for s in surf) > 0.4 * g.thick(0)


def test_thick_build_on_surface_hits_equals_thin_build():
    """With every hit on its layer's average surface the second step has
    zero length: the two-step build equals the one-step build."""
    ev = synth.make_event(400, cfg=331, event=0, noise=0.3)
    thin = oracle.config(ev.geometry, max_cands=6)
    thick = oracle.config(_thick_barrel(), max_cands=6)
    a = oracle.build_tracks(thin, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits, n_threads=8)
    b = oracle.build_tracks(thick, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits, n_threads=8)
    assert (a["hits"] == b["hits"]).all()
    assert np.allclose(a["chi2"], b["chi2"], rtol=1e-9, atol=1e-9)
    assert np.allclose(a["par"], b["par"], rtol=1e-9, atol=1e-9)


def _tiny_thick_event(rng_seed, g, branch_layers=(3, 5, 7)):
    ev = synth.make_event(2, cfg=332, event=rng_seed, geometry=g, noise=0.0)
    rng = np.random.default_rng(rng_seed)
    hits = [h.copy() for h in ev.hits]
    for L in branch_layers:
        h = hits[L][ev.truth_hit[0, L]]
        r = math.hypot(h[0], h[1])
        ph = math.atan2(h[1], h[0]) + rng.choice([-1, 1]) * 0.015 / r
        if g.is_disk:
            r2 = r + rng.normal(0, 0.12)
            extra = [r2 * math.cos(ph), r2 * math.sin(ph), g.disk_z[L] + rng.uniform(-0.5, 0.5) * g.thick(L)]
        else:
            r2 = g.radii[L] + rng.uniform(-0.5, 0.5) * g.thick(L)
            extra = [r2 * math.cos(ph), r2 * math.sin(ph), h[2] + rng.normal(0, 0.12)]
        hits[L] = np.concatenate([hits[L], [extra]])
    return ev, hits


def _enumerate_two_step(cfg, hits, sp, sc, sh):
    nsl, nl = cfg.n_seed_layers, cfg.n_layers
    kind = int(cfg.kind[0])
    s2 = cfg.sigma_r if kind else cfg.sigma_z
    paths = [dict(par=np.array(sp), C=synth.unpack_sym(np.asarray(sc)), chi2=0.0,
                  n_hits=int((np.asarray(sh) >= 0).sum()), n_holes=0, hits=list(sh) + [-1] * (nl - nsl),
                  stopped=False)]
    max_live = 1
    for L in range(nsl, nl):
        nxt = []
        for pth in paths:
            if pth["stopped"]:
                nxt.append(pth)
                continue
            Cm = oracle.add_ms(pth["par"], pth["C"], cfg.x0[L - 1], cfg.mass, kind=kind)
            if kind:
                ok, pp, F, _, _ = oracle.propagate_plane(pth["par"], cfg.zplane[L], cfg.bz)
            else:
                ok, pp, F, _, _ = oracle.propagate(pth["par"], cfg.radius[L], cfg.bz)
            assert ok
            Cp = oracle.transport(F, Cm)
            acc = []
            for j, h in enumerate(hits[L]):
                if h[0] * pp[0] + h[1] * pp[1] <= 0:
                    continue
                where = h[2] if kind else math.hypot(h[0], h[1])
                ok2, ph, F2, _ = oracle.step_near(pp, kind, where, cfg.bz)
                if not ok2:
                    continue
                Ch = oracle.transport(F2, Cp)
                if oracle.chi2(ph, Ch, h, cfg.sigma_rphi, s2, kind=kind) < cfg.chi2_cut:
                    acc.append((j, ph, Ch))
            for j, ph, Ch in acc:
                pu, Cu, c2 = oracle.update(ph, Ch, hits[L][j], cfg.sigma_rphi, s2, kind=kind)
                hl = list(pth["hits"])
                hl[L] = j
                nxt.append(dict(pth, par=pu, C=Cu, chi2=pth["chi2"] + c2, n_hits=pth["n_hits"] + 1, hits=hl))
            if not acc:
                if pth["n_holes"] < cfg.max_holes:
                    nxt.append(dict(pth, par=pp, C=Cp, n_holes=pth["n_holes"] + 1))
                else:
                    nxt.append(dict(pth, par=pp, C=Cp, stopped=True))
        paths = nxt
        max_live = max(max_live, len(paths))
    paths.sort(key=lambda q: (-q["n_hits"], q["chi2"]))
    return paths, max_live


@pytest.mark.parametrize("rng_seed,disk", [(0, False), (1, False), (2, False), (0, True), (1, True)])
def test_two_step_beam_equals_exhaustive_enumeration(rng_seed, disk):
    g = _thick_endcap() if disk else _thick_barrel()
    ev, hits = _tiny_thick_event(rng_seed, g)
    cfg = oracle.config(g, max_cands=16)
    for s in range(ev.n_seeds):
        paths, max_live = _enumerate_two_step(cfg, hits, ev.seed_par[s], ev.seed_cov[s], ev.seed_hits[s])
        out = oracle.build_tracks(cfg, hits, ev.seed_par, ev.seed_cov, ev.seed_hits, seed_ids=[s])[0]
        best = paths[0]
        assert list(out["hits"][:10]) == best["hits"]
        assert out["chi2"] == pytest.approx(best["chi2"], rel=1e-12, abs=1e-12)
        assert out["n_final"] == len(paths)
        assert np.allclose(out["par"], best["par"], rtol=1e-12, atol=1e-12)
        if s == 0:
            assert max_live >= 2


@pytest.mark.parametrize("disk", [False, True])
def test_thick_fit_pulls_and_chi2(disk):
    g = _thick_endcap() if disk else _thick_barrel()
    ev = synth.make_event(20000, cfg=333, event=0, geometry=g, noise=0.0)
    cfg = oracle.config(g)
    res = oracle.fit(cfg, ev.hits, ev.prior_par, ev.prior_cov, ev.truth_hit, n_threads=8, want_hit_chi2=True)
    assert (res["status"] == 0).all()
    d = _wrapdiff(res["par"].T, ev.truth_par[:, 9].T).T
    Cm = synth.unpack_sym(res["cov"])
    ph = np.arctan2(res["par"][:, 1], res["par"][:, 0])
    n = d.shape[0]
    eu = np.stack([-np.sin(ph), np.cos(ph)], 1)
    pulls = [(eu * d[:, :2]).sum(1) / np.sqrt(np.einsum("ni,nij,nj->n", eu, Cm[:, :2, :2], eu))]
    pulls += [d[:, j] / np.sqrt(Cm[:, j, j]) for j in (3, 4, 5)]
    for pl in pulls:
        assert abs(pl.mean()) < 3.0 / math.sqrt(n)
        assert abs(pl.std() - 1.0) < 3.0 / math.sqrt(2 * n)
    c2 = res["hit_chi2"][:, 5:].ravel()
    assert abs(c2.mean() - 2.0) < 3.0 * 2.0 / math.sqrt(c2.size)
    assert stats.kstest(c2[:20000], "chi2", args=(2,)).pvalue > 0.01


def test_thick_build_efficiency_and_replay():
    g = _thick_barrel()
    ev = synth.make_event(1500, cfg=334, event=0, geometry=g, noise=0.3)
    cfg = oracle.config(g, max_cands=6)
    out = oracle.build_tracks(cfg, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits, n_threads=8)
    assert (out["hits"][:, :10] == ev.truth_hit).all(1).mean() > 0.9
    hs = oracle.HitSet(ev.hits)
    for i in range(0, 1500, 37):
        if out["status"][i] != 0:
            continue
        tot, _, ok = oracle.replay(cfg, hs, ev.seed_par[i], ev.seed_cov[i], out["hits"][i])
        assert ok and tot == pytest.approx(out["chi2"][i], rel=1e-12, abs=1e-12)
