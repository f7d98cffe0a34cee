"""Pins of the oracle's helix propagation, Jacobian and covariance transport.

Each check compares the oracle with something that does not reuse its
formulas: a Runge-Kutta integration of the Lorentz force, the generator's
independent turning-angle helix, the textbook chord formula, a time-reversed
trajectory, central finite differences and a sigma-point transform.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1702_06359_amd import synth

KAPPA = 0.00299792458
BZ = 3.8
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_states(n, rng, r0=8.0, qpt_max=2.0):
    phi_pos = rng.uniform(-np.pi, np.pi, n)
    x = r0 * np.cos(phi_pos)
    y = r0 * np.sin(phi_pos)
    z = rng.uniform(-5, 5, n)
    qpt = rng.uniform(-qpt_max, qpt_max, n)
    phi = phi_pos + rng.uniform(-0.6, 0.6, n)
    theta = rng.uniform(0.7, 2.4, n)
    return np.stack([x, y, z, qpt, phi, theta], axis=1)


def rk4_to_radius(par, r, bz, h=0.05):
    """Integrate dr/dl = t, dt/dl = (q kappa B / p) t x z-hat (3-D path length l)
    with classical RK4 until the transverse radius reaches r; the last step is
    bisected so the end point lies on the cylinder."""
    x, y, z, qpt, phi, th = par
    pos = np.array([x, y, z], dtype=np.float64)
    t = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
    k = qpt * math.sin(th) * KAPPA * bz          # (q / p) kappa B, 1/cm

    def f(state):
        d = state[3:]
        return np.concatenate([d, k * np.array([d[1], -d[0], 0.0])])

    def step(state, hh):
        k1 = f(state)
        k2 = f(state + 0.5 * hh * k1)
        k3 = f(state + 0.5 * hh * k2)
        k4 = f(state + hh * k3)
        return state + hh / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)

    st = np.concatenate([pos, t])
    for _ in range(200000):
        nxt = step(st, h)
        if math.hypot(nxt[0], nxt[1]) >= r:
            lo, hi = 0.0, h
            for _ in range(80):
                mid = 0.5 * (lo + hi)
                if math.hypot(*step(st, mid)[:2]) >= r:
                    hi = mid
                else:
                    lo = mid
            return step(st, 0.5 * (lo + hi))
        st = nxt
    raise RuntimeError("did not reach radius")


def test_propagation_matches_rk4_lorentz_force():
    rng = np.random.default_rng(11)
    states = random_states(12, rng, qpt_max=1.5)
    for p in states:
        for r in (12.0, 24.0, 40.0):
            ok, out, _, _, _ = oracle.propagate(p, r, BZ, jacobian=False)
            assert ok
            ref = rk4_to_radius(p, r, BZ, h=0.02)
            assert np.abs(out[:3] - ref[:3]).max() < 1e-8
            d = ref[3:]
            phi_ref = math.atan2(d[1], d[0])
            th_ref = math.acos(d[2] / np.linalg.norm(d))
            dphi = (out[4] - phi_ref + np.pi) % (2 * np.pi) - np.pi
            assert abs(dphi) < 1e-10
            assert abs(out[5] - th_ref) < 1e-10


def test_zero_noise_generator_hits_equal_propagated_crossings():
    ev = synth.make_event(300, cfg=90, event=0, smear=False, scatter=False)
    g = ev.geometry
    worst = 0.0
    for i in range(300):
        p = ev.vertex_par[i].copy()
        for L in range(g.n_layers):
            ok, p, _, _, _ = oracle.propagate(p, g.radii[L], g.bz, jacobian=False)
            assert ok
            h = ev.hits[L][ev.truth_hit[i, L]]
            worst = max(worst, float(np.abs(p[:3] - h).max()))
            assert abs(((p[4] - ev.truth_par[i, L, 4]) + np.pi) % (2 * np.pi) - np.pi) < 1e-9
    assert worst < 1e-9


def test_chord_closed_form_golden():
    """A track from the origin reaches radius r after s = 2R asin(r / 2R) (golden values)."""
    with open(os.path.join(GOLDEN, "closed_forms.json")) as f:
        gold = json.load(f)["helix_from_origin"]
    for case in gold["cases"]:
        pt, r, eta = case["pt"], case["r"], case["eta"]
        theta = 2 * math.atan(math.exp(-eta))
        p = np.array([0.0, 0.0, 0.0, 1.0 / pt, 0.3, theta])
        ok, out, _, s, _ = oracle.propagate(p, r, gold["bz"], jacobian=False)
        assert ok
        assert s == pytest.approx(case["s"], abs=5e-3)
        assert out[2] == pytest.approx(case["z"], abs=5e-3)
        R = pt / (KAPPA * gold["bz"])
        assert R == pytest.approx(case["R"], abs=5e-3)


def test_straight_line_limit():
    rng = np.random.default_rng(3)
    for p in random_states(50, rng):
        p = p.copy()
        p[3] = 0.0
        ok, out, _, s, _ = oracle.propagate(p, 30.0, BZ, jacobian=False)
        assert ok
        # |(x, y) + s (cos phi, sin phi)| = r with s > 0, direction unchanged
        xy = p[:2] + s * np.array([math.cos(p[4]), math.sin(p[4])])
        assert np.abs(out[:2] - xy).max() < 1e-12
        assert math.hypot(*out[:2]) == pytest.approx(30.0, abs=1e-12)
        assert abs((out[4] - p[4] + np.pi) % (2 * np.pi) - np.pi) < 1e-15
        # continuity into a tiny but nonzero curvature
        p2 = p.copy()
        p2[3] = 1e-9
        ok2, out2, _, _, _ = oracle.propagate(p2, 30.0, BZ, jacobian=False)
        assert ok2 and np.abs(out2[:3] - out[:3]).max() < 1e-8


def test_time_reversal_returns_to_start():
    rng = np.random.default_rng(5)
    for p in random_states(60, rng):
        ok, out, _, _, _ = oracle.propagate(p, 28.0, BZ, jacobian=False)
        assert ok
        rev = out.copy()
        rev[3] = -out[3]
        rev[4] = out[4] + np.pi
        rev[5] = np.pi - out[5]
        ok2, back, _, _, _ = oracle.propagate(rev, 8.0, BZ, jacobian=False)
        assert ok2
        assert np.abs(back[:3] - p[:3]).max() < 1e-9


def test_unreachable_radius_fails_with_margin_sign():
    # pT = 0.1 GeV: 2R = 17.6 cm, so a track from the origin cannot reach r = 30
    p = np.array([0.0, 0.0, 0.0, 10.0, 0.1, 1.2])
    ok, _, _, _, margin = oracle.propagate(p, 30.0, BZ)
    assert not ok and margin < 0
    ok, _, _, _, margin = oracle.propagate(p, 12.0, BZ)
    assert ok and margin > 0


def _wrapdiff(a, b):
    d = a - b
    d[4] = (d[4] + np.pi) % (2 * np.pi) - np.pi
    return d


def test_jacobian_matches_central_differences():
    rng = np.random.default_rng(7)
    steps = np.array([1e-6, 1e-6, 1e-6, 1e-7, 1e-7, 1e-7])
    worst = 0.0
    for p in random_states(40, rng):
        for r in (12.0, 40.0):
            ok, out, F, _, _ = oracle.propagate(p, r, BZ)
            assert ok
            num = np.zeros((6, 6))
            for j in range(6):
                pp = p.copy()
                pm = p.copy()
                pp[j] += steps[j]
                pm[j] -= steps[j]
                _, op, _, _, _ = oracle.propagate(pp, r, BZ, jacobian=False)
                _, om, _, _, _ = oracle.propagate(pm, r, BZ, jacobian=False)
                num[:, j] = _wrapdiff(op, om) / (2 * steps[j])
            scale = np.maximum(np.abs(num), 1.0)
            worst = max(worst, float((np.abs(F - num) / scale).max()))
    assert worst < 1e-6


def test_jacobian_small_curvature_branch():
    """Series branch (|w s| < 1e-2) and direct branch agree with differences."""
    rng = np.random.default_rng(8)
    for qpt in (1e-7, 1e-4, 0.05, 0.2):
        p = random_states(1, rng)[0]
        p[3] = qpt
        ok, out, F, _, _ = oracle.propagate(p, 30.0, BZ)
        assert ok
        h = 1e-6
        for j in (0, 1, 3, 4):
            pp = p.copy()
            pm = p.copy()
            pp[j] += h
            pm[j] -= h
            _, op, _, _, _ = oracle.propagate(pp, 30.0, BZ, jacobian=False)
            _, om, _, _, _ = oracle.propagate(pm, 30.0, BZ, jacobian=False)
            col = _wrapdiff(op, om) / (2 * h)
            assert np.abs(F[:, j] - col).max() < 1e-6 * max(1.0, np.abs(col).max())


def test_transport_equals_sigma_point_transform():
    """C' = F C F^T against the nonlinear map of the eigen-directions of C."""
    rng = np.random.default_rng(9)
    for p in random_states(20, rng):
        A = rng.normal(size=(6, 6))
        Cm = A @ A.T * 1e-6 + np.diag([1e-6, 1e-6, 1e-5, 1e-6, 1e-7, 1e-7])
        ok, _, F, _, _ = oracle.propagate(p, 36.0, BZ)
        assert ok
        got = oracle.transport(F, Cm)
        lam, V = np.linalg.eigh(Cm)
        ref = np.zeros((6, 6))
        eps = 1e-3
        for i in range(6):
            d = np.sqrt(lam[i]) * V[:, i]
            _, op, _, _, _ = oracle.propagate(p + eps * d, 36.0, BZ, jacobian=False)
            _, om, _, _, _ = oracle.propagate(p - eps * d, 36.0, BZ, jacobian=False)
            col = _wrapdiff(op, om) / (2 * eps)
            ref += np.outer(col, col)
        scale = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
        assert np.abs(got - ref).max() / scale.max() < 1e-6
        assert np.allclose(got, got.T, atol=0)


def test_propagated_covariance_is_tangent_to_layer():
    """F maps onto the cylinder, so C' has zero variance along the layer normal."""
    rng = np.random.default_rng(10)
    for p in random_states(30, rng):
        A = rng.normal(size=(6, 6))
        Cm = A @ A.T * 1e-4
        ok, out, F, _, _ = oracle.propagate(p, 20.0, BZ)
        Cp = oracle.transport(F, Cm)
        n = np.array([out[0], out[1], 0, 0, 0, 0]) / 20.0
        assert abs(n @ Cp @ n) <= 1e-10 * np.trace(Cp)


def rk4_first_crossing(states, r, bz, max_turns=1.05, steps_per_radian=400):
    """Vectorised classical RK4 of the Lorentz force (3-D path length l) for
    many states at once, each with a step of 1/steps_per_radian of its turning
    radius, until its transverse radius first reaches r (the last step
    bisected onto the cylinder) or it has turned max_turns revolutions.
    Returns (reached, end position, end direction, transverse path)."""
    n = states.shape[0]
    x, y, z, qpt, phi, th = states.T
    pos = np.stack([x, y, z], 1)
    d = np.stack([np.sin(th) * np.cos(phi), np.sin(th) * np.sin(phi), np.cos(th)], 1)
    k = qpt * np.sin(th) * KAPPA * bz                         # (q / p) kappa B, 1/cm
    kk = np.maximum(np.abs(k), 1e-6)
    h = np.minimum(0.02, 1.0 / (kk * steps_per_radian))       # 3-D step per state
    n_steps = np.ceil(max_turns * 2 * np.pi / (kk * h)).astype(int)

    def f(st, kv):
        dd = st[:, 3:]
        return np.concatenate([dd, kv[:, None] * np.stack([dd[:, 1], -dd[:, 0], np.zeros(len(dd))], 1)], 1)

    def step(st, hh, kv):
        k1 = f(st, kv)
        k2 = f(st + 0.5 * hh[:, None] * k1, kv)
        k3 = f(st + 0.5 * hh[:, None] * k2, kv)
        k4 = f(st + hh[:, None] * k3, kv)
        return st + hh[:, None] / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)

    st = np.concatenate([pos, d], 1)
    done = np.zeros(n, bool)
    end = np.zeros((n, 6))
    path = np.zeros(n)
    l3 = np.zeros(n)
    for it in range(int(n_steps.max())):
        live = ~done & (it < n_steps)
        if not live.any():
            break
        nxt = st.copy()
        nxt[live] = step(st[live], h[live], k[live])
        cross = live & (np.hypot(nxt[:, 0], nxt[:, 1]) >= r)
        for i in np.flatnonzero(cross):
            lo, hi = 0.0, h[i]
            s0 = st[i:i + 1]
            for _ in range(80):
                mid = 0.5 * (lo + hi)
                e = step(s0, np.array([mid]), k[i:i + 1])[0]
                if math.hypot(e[0], e[1]) >= r:
                    hi = mid
                else:
                    lo = mid
            end[i] = step(s0, np.array([0.5 * (lo + hi)]), k[i:i + 1])[0]
            path[i] = (l3[i] + 0.5 * (lo + hi)) * math.sin(states[i, 5])
            done[i] = True
        l3 = np.where(live & ~cross, l3 + h, l3)
        st = np.where((live & ~cross)[:, None], nxt, st)
    return done, end[:, :3], end[:, 3:], path


def test_propagation_matches_rk4_on_every_kind_of_crossing():
    """Starting states anywhere on three inner cylinders, heading in any
    direction, pT 0.1-3 GeV of both charges, to three outer radii, against
    the integrated Lorentz force: each crossing the oracle finds is the first
    one along the motion (position within 1e-8 cm, direction within 1e-9
    rad), and it fails exactly where the integration never reaches the
    radius within a revolution.  The cases cover tracks heading out, tracks
    heading in (whose first crossing lies beyond the closest approach to the
    axis, half of them after more than half a turn) and loopers whose circle
    stays inside the radius, for both charges."""
    rng = np.random.default_rng(42)
    rows = []
    for r0 in (4.0, 8.0, 16.0):
        n = 60
        phi_pos = rng.uniform(-np.pi, np.pi, n)
        pt = np.exp(rng.uniform(np.log(0.1), np.log(3.0), n))
        q = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
        heading = rng.uniform(-np.pi, np.pi, n)
        st = np.stack([r0 * np.cos(phi_pos), r0 * np.sin(phi_pos), rng.uniform(-5, 5, n), q / pt,
                       phi_pos + heading, rng.uniform(0.7, 2.4, n)], 1)
        for r in (r0 + 4.0, 24.0, 40.0):
            rows.append((st, r))
    # More than half a turn before the first crossing needs a start on the
    # far side of a small circle, heading in, and a radius within the
    # circle's reach below sqrt(2) times the start radius: circles of
    # 9-12 cm from r = 16 cm to r = 20 cm, both turning senses.
    far = []
    for q in (1.0, -1.0):
        for R in (9.0, 10.0, 11.0, 12.0):
            for a1 in np.linspace(0.52, 0.85, 8) * np.pi:
                # centre at distance d with |p0| = 16 at angle a1 from the closest point
                d = (R * math.cos(a1) + math.sqrt(R * R * math.cos(a1) ** 2 - R * R + 256.0))
                if d + R < 20.5:
                    continue
                beta = rng.uniform(-np.pi, np.pi)
                c = d * np.array([math.cos(beta), math.sin(beta)])
                u = -np.array([math.cos(beta), math.sin(beta)])        # centre towards the axis
                v = np.array([-u[1], u[0]])
                sgn = 1.0 if q < 0 else -1.0                            # w > 0 for q < 0: anticlockwise
                p0 = c + R * (math.cos(a1) * u - sgn * math.sin(a1) * v)
                # moving towards the closest point: anticlockwise about c when w > 0
                rad = p0 - c
                t = sgn * np.array([-rad[1], rad[0]]) / R
                pt = R * KAPPA * BZ
                far.append([p0[0], p0[1], 0.0, q / pt, math.atan2(t[1], t[0]), 1.2])
    rows.append((np.array(far), 20.0))
    classes = {}
    worst_pos = worst_dir = 0.0
    for st, r in rows:
        reached, pos, d, path = rk4_first_crossing(st, r, BZ)
        for i, p in enumerate(st):
            ok, out, _, s, margin = oracle.propagate(p, r, BZ, jacobian=False)
            assert ok == bool(reached[i]), (p, r)
            heading_in = math.cos(p[4]) * p[0] + math.sin(p[4]) * p[1] < 0
            charge = "+" if p[3] > 0 else "-"
            if not ok:
                assert margin < 0
                classes[("unreachable", charge)] = classes.get(("unreachable", charge), 0) + 1
                continue
            w = -KAPPA * BZ * p[3]
            far = abs(w * s) > np.pi
            kind = ("in" if heading_in else "out") + ("-far" if far else "-near")
            classes[(kind, charge)] = classes.get((kind, charge), 0) + 1
            assert s == pytest.approx(path[i], abs=1e-7)
            worst_pos = max(worst_pos, float(np.abs(out[:3] - pos[i]).max()))
            phi_ref = math.atan2(d[i, 1], d[i, 0])
            th_ref = math.acos(d[i, 2] / np.linalg.norm(d[i]))
            worst_dir = max(worst_dir, abs((out[4] - phi_ref + np.pi) % (2 * np.pi) - np.pi), abs(out[5] - th_ref))
    assert worst_pos < 1e-8 and worst_dir < 1e-9, (worst_pos, worst_dir)
    for kind in ("out-near", "in-near", "in-far", "unreachable"):
        for charge in "+-":
            assert classes.get((kind, charge), 0) >= 3, classes
    # heading out from inside a cylinder, the first crossing comes before the
    # farthest point of the circle: never more than half a turn
    assert classes.get(("out-far", "+"), 0) == classes.get(("out-far", "-"), 0) == 0


def test_propagation_of_loopers_matches_rk4():
    """Low-pT tracks from near the axis (pT 0.15-0.5 GeV, turning radius
    13-44 cm): crossings within the circle's reach match the integration;
    radii beyond 2R (for a start at the axis) fail."""
    rng = np.random.default_rng(43)
    n = 40
    pt = rng.uniform(0.15, 0.5, n)
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    phi = rng.uniform(-np.pi, np.pi, n)
    st = np.stack([0.01 * np.cos(phi + 0.3), 0.01 * np.sin(phi + 0.3), rng.uniform(-1, 1, n), q / pt, phi,
                   rng.uniform(0.9, 2.2, n)], 1)
    n_fail = n_ok = 0
    for r in (8.0, 20.0, 40.0, 60.0):
        reached, pos, d, path = rk4_first_crossing(st, r, BZ)
        for i, p in enumerate(st):
            ok, out, _, s, margin = oracle.propagate(p, r, BZ, jacobian=False)
            assert ok == bool(reached[i])
            R = pt[i] / (KAPPA * BZ)
            if r > 2 * R + 0.02:
                assert not ok
            if ok:
                n_ok += 1
                assert np.abs(out[:3] - pos[i]).max() < 1e-8
                assert s == pytest.approx(path[i], abs=1e-7)
            else:
                n_fail += 1
    assert n_ok > 40 and n_fail > 20
