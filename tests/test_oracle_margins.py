"""Pins of the oracle's decision margins, on hand-built events.

The tie protocol of the GPU parity tests rests on these numbers: m_cut (the
smallest |chi2 - cut| of a decision whose reversal changes the seed's
result), m_rank (the smallest relative key gap at a k/(k+1) beam boundary or
at the final choice, likewise relevant), m_prop (the smallest distance to
tangency over the seed's propagations, relative to the radius) and the
alternative outcomes.  Each case places hits so that the expected margin is
known in closed form: a hit at chi2 = cut -+ delta, two hits at a known chi2
gap, a helix whose circle is at a known distance from tangency with a layer.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_1702_06359_amd import synth

CUT = 30.0
SRPHI, SZ = 0.01, 0.1


def _one_track(cfg=300, event=0, pt=2.0):
    ev = synth.make_event(1, cfg=cfg, event=event, noise=0.0, pt_range=(pt, pt), eta_max=0.3)
    return ev


def _predict(ev, layer, hits):
    """Predicted state and covariance on `layer` from the seed through the
    given hits on the building layers before it (the building rules written
    out with the oracle's primitives: scattering of the layer left,
    propagation, transport, update)."""
    g = ev.geometry
    p = ev.seed_par[0].copy()
    C = synth.unpack_sym(ev.seed_cov[0:1])[0]
    for L in range(3, layer + 1):
        C = oracle.add_ms(p, C, g.x0[L - 1], g.mass)
        ok, p, F, _, _ = oracle.propagate(p, g.radii[L], g.bz)
        assert ok
        C = oracle.transport(F, C)
        if L < layer and hits[L] is not None:
            p, C, _ = oracle.update(p, C, hits[L], SRPHI, SZ)
    return p, C


def _hit_at_chi2(p, C, r, target, side=1.0):
    """A point on the cylinder of radius r, at the predicted z, whose chi2
    against (p, C) is `target` (bisection in azimuth from the prediction)."""
    phi0 = math.atan2(p[1], p[0])

    def at(dphi):
        a = phi0 + side * dphi
        return np.array([r * math.cos(a), r * math.sin(a), p[2]])
    lo, hi = 0.0, 0.05
    while oracle.chi2(p, C, at(hi), SRPHI, SZ) < target:
        hi *= 2
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if oracle.chi2(p, C, at(mid), SRPHI, SZ) < target:
            lo = mid
        else:
            hi = mid
    h = at(0.5 * (lo + hi))
    return h, oracle.chi2(p, C, h, SRPHI, SZ)


def _build(ev, hits, k=1, max_holes=1):
    cfg = oracle.config(ev.geometry, max_cands=k, max_holes=max_holes)
    return oracle.build_tracks(cfg, hits, ev.seed_par, ev.seed_cov, ev.seed_hits)[0]


def _chi2_before(ev, hits, layer):
    """Accumulated chi2 of the true hits on the building layers before `layer`."""
    g = ev.geometry
    cfg = oracle.config(dataclasses.replace(g, n_layers=layer, radii=g.radii[:layer], x0=g.x0[:layer]),
                        max_cands=1)
    lh = list(ev.truth_hit[0, :layer])
    tot, _, ok = oracle.replay(cfg, [h for h in hits[:layer]], ev.seed_par[0], ev.seed_cov[0], lh)
    assert ok
    return tot


@pytest.mark.parametrize("sign", [-1.0, 1.0])
def test_m_cut_is_the_distance_of_a_relevant_hit_to_the_cut(sign):
    """Layer 5 holds one hit, at chi2 = cut + sign * delta: accepting it makes a
    hit child, rejecting it a hole, so the decision is relevant and m_cut =
    delta; the alternative outcome is the other path."""
    ev = _one_track()
    truth = [ev.hits[L][ev.truth_hit[0, L]] for L in range(10)]
    p, C = _predict(ev, 5, truth)
    for delta in (0.004, 0.02):
        h, c2 = _hit_at_chi2(p, C, ev.geometry.radii[5], CUT + sign * delta)
        assert c2 == pytest.approx(CUT + sign * delta, abs=1e-9)
        hits = [x.copy() for x in ev.hits]
        hits[5] = h[None, :]
        o = _build(ev, hits)
        assert o["m_cut"] == pytest.approx(delta, abs=1e-9)
        assert o["m_cut_raw"] == pytest.approx(delta, abs=1e-9)
        took = o["hits"][5] == 0
        assert took == (sign < 0)
        alt = [a for a in range(o["n_alt"]) if o["alt_kind"][a] == 0]
        assert len(alt) == 1 and o["alt_margin"][alt[0]] == pytest.approx(delta, abs=1e-9)
        # the alternative takes layer 5 the other way after the same start
        assert o["alt_hits"][alt[0]][5] == (-1 if took else 0)
        for L in (3, 4):
            assert o["alt_hits"][alt[0]][L] == o["hits"][L] == ev.truth_hit[0, L]


def test_m_cut_ignores_a_decision_that_cannot_change_the_result():
    """The same near-cut hit beside the true hit, one candidate per seed: the
    true hit's child wins either way, so the near-cut decision is not
    relevant (m_cut_raw = delta, m_cut far larger, no alternative)."""
    ev = _one_track()
    truth = [ev.hits[L][ev.truth_hit[0, L]] for L in range(10)]
    p, C = _predict(ev, 5, truth)
    h, c2 = _hit_at_chi2(p, C, ev.geometry.radii[5], CUT - 0.004)
    hits = [x.copy() for x in ev.hits]
    hits[5] = np.vstack([hits[5], h[None, :]])
    o = _build(ev, hits)
    assert o["hits"][5] == ev.truth_hit[0, 5]
    assert o["m_cut_raw"] == pytest.approx(0.004, abs=1e-9)
    assert o["m_cut"] > 1.0
    assert o["n_alt"] == 0


@pytest.mark.parametrize("gap", [2e-4, 3e-3])
def test_m_rank_is_the_relative_gap_at_the_beam_boundary(gap):
    """Layer 5 holds two hits, at chi2 a and a + gap*(1 + chi2_before + a),
    one candidate per seed: the k/(k+1) boundary separates them, m_rank is
    their relative gap, and the alternative takes the other hit."""
    ev = _one_track(event=1)
    truth = [ev.hits[L][ev.truth_hit[0, L]] for L in range(10)]
    p, C = _predict(ev, 5, truth)
    before = _chi2_before(ev, [x.copy() for x in ev.hits], 5)
    a = 3.0
    b = a + gap * (1.0 + before + a)
    h1, c1 = _hit_at_chi2(p, C, ev.geometry.radii[5], a, side=1.0)
    h2, c2 = _hit_at_chi2(p, C, ev.geometry.radii[5], b, side=-1.0)
    hits = [x.copy() for x in ev.hits]
    hits[5] = np.vstack([h2, h1])            # index 1 is the better one
    o = _build(ev, hits)
    expect = (before + c2 - (before + c1)) / (1.0 + before + c1)
    assert expect == pytest.approx(gap, rel=1e-6)
    assert o["hits"][5] == 1
    assert o["m_rank"] == pytest.approx(expect, rel=1e-9)
    assert o["m_rank_raw"] == pytest.approx(expect, rel=1e-9)
    alt = [j for j in range(o["n_alt"]) if o["alt_kind"][j] == 1]
    assert alt and o["alt_hits"][alt[0]][5] == 0
    assert o["alt_margin"][alt[0]] == pytest.approx(expect, rel=1e-9)


def test_m_rank_is_the_relative_gap_of_the_final_choice():
    """Two hits on the last layer at a known chi2 gap and two candidates per
    seed: both survive, the final rank-0/rank-1 choice is the tie, and the
    alternative is rank 1 (the other hit)."""
    ev = _one_track(event=2)
    truth = [ev.hits[L][ev.truth_hit[0, L]] for L in range(10)]
    p, C = _predict(ev, 9, truth)
    before = _chi2_before(ev, [x.copy() for x in ev.hits], 9)
    a, gap = 2.0, 5e-4
    h1, c1 = _hit_at_chi2(p, C, ev.geometry.radii[9], a, side=1.0)
    h2, c2 = _hit_at_chi2(p, C, ev.geometry.radii[9], a + gap * (1 + before + a), side=-1.0)
    hits = [x.copy() for x in ev.hits]
    hits[9] = np.vstack([h1, h2])
    o = _build(ev, hits, k=2)
    expect = (c2 - c1) / (1.0 + before + c1)
    assert o["hits"][9] == 0 and o["n_final"] == 2
    assert o["m_rank"] == pytest.approx(expect, rel=1e-6)
    alt = [j for j in range(o["n_alt"]) if o["alt_kind"][j] == 2]
    assert len(alt) == 1 and o["alt_hits"][alt[0]][9] == 1
    assert o["m_cut"] > 1.0


def test_m_prop_is_the_distance_to_tangency():
    """A seed on layer 2 whose circle (centre at distance d from the axis,
    radius R) reaches 28.05 cm, on empty building layers with holes allowed:
    the candidate is propagated to r = 16, 20, 24 and 28 cm and fails at 32
    cm.  The margin at radius r is r minus the distance of the two circles'
    radical line from the axis, (d^2 + r^2 - R^2) / (2 d); m_prop is the
    smallest |margin| / r."""
    g = synth.Geometry()
    d, R = 14.0, 14.05
    r2 = g.radii[2]
    cos_a = (d * d + R * R - r2 * r2) / (2 * d * R)       # angle at the centre from the closest point
    alpha = math.acos(cos_a)
    beta = 0.4
    c = d * np.array([math.cos(beta), math.sin(beta)])
    u = -c / d
    v = np.array([-u[1], u[0]])
    p0 = c + R * (math.cos(alpha) * u + math.sin(alpha) * v)
    rad = p0 - c
    t = np.array([-rad[1], rad[0]]) / R                  # tangent, oriented away from the axis below
    if t @ p0 < 0:
        t = -t
    # the centre to the left of the motion is an anticlockwise turn, w > 0
    left = np.array([-t[1], t[0]])
    w = (1.0 / R) * (1.0 if left @ (c - p0) > 0 else -1.0)
    qpt = -w / (0.00299792458 * g.bz)
    seed_par = np.array([[p0[0], p0[1], 0.0, qpt, math.atan2(t[1], t[0]), 1.3]])
    seed_cov = synth.local_cov_to_packed(np.array([math.atan2(p0[1], p0[0])]), synth.SEED_SIGMA)
    hits = [np.array([[r * math.cos(1.0), r * math.sin(1.0), 0.0]]) for r in g.radii[:3]]
    hits += [np.zeros((0, 3)) for _ in range(7)]
    cfg = oracle.config(g, max_cands=1, max_holes=7)
    o = oracle.build_tracks(cfg, hits, seed_par, seed_cov, np.array([[0, 0, 0]], dtype=np.int32))[0]
    assert o["status"] == 2
    margins = [abs(r - (d * d + r * r - R * R) / (2 * d)) / r for r in g.radii[3:8]]
    assert o["m_prop"] == pytest.approx(min(margins), rel=1e-9)
    assert min(margins) < 2e-3
