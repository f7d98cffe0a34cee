"""Pins of the oracle's endcap-disk surfaces (planes at fixed z).

Independent references: a Runge-Kutta integration of the Lorentz force
stopped on the plane, the generator's turning-angle crossing, the circle
chord from the origin, central finite differences, the information-filter
identities with the disk's own (r*phi, r) projection written out here, the
chi2 of a state with no uncertainty, the Highland angle at the disk's
incidence, exact recovery of true tracks, unit-width pulls, and the beam
search against exhaustive enumeration on tiny disk events.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1702_06359_amd import synth

KAPPA = 0.00299792458
BZ = 3.8
SR, SV = 0.01, 0.1


def forward_states(n, rng, qpt_max=2.0):
    """States near the beam line heading forward (0.1 < theta < 0.6)."""
    phi_pos = rng.uniform(-np.pi, np.pi, n)
    r0 = rng.uniform(0.0, 4.0, n)
    x = r0 * np.cos(phi_pos)
    y = r0 * np.sin(phi_pos)
    z = rng.uniform(-2, 12, n)
    qpt = rng.uniform(-qpt_max, qpt_max, n)
    phi = rng.uniform(-np.pi, np.pi, n)
    theta = rng.uniform(0.1, 0.6, n)
    return np.stack([x, y, z, qpt, phi, theta], axis=1)


def rk4_to_plane(par, zd, bz, h=0.02):
    """Classical RK4 on dr/dl = t, dt/dl = (q kappa B / p) t x z-hat until z
    reaches zd; the last step is bisected onto the plane."""
    x, y, z, qpt, phi, th = par
    t = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
    k = qpt * math.sin(th) * KAPPA * bz

    def f(st):
        d = st[3:]
        return np.concatenate([d, k * np.array([d[1], -d[0], 0.0])])

    def step(st, hh):
        k1 = f(st)
        k2 = f(st + 0.5 * hh * k1)
        k3 = f(st + 0.5 * hh * k2)
        k4 = f(st + hh * k3)
        return st + hh / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)

    st = np.concatenate([[x, y, z], t])
    for _ in range(400000):
        nxt = step(st, h)
        if nxt[2] >= zd:
            lo, hi = 0.0, h
            for _ in range(80):
                mid = 0.5 * (lo + hi)
                if step(st, mid)[2] >= zd:
                    hi = mid
                else:
                    lo = mid
            return step(st, 0.5 * (lo + hi))
        st = nxt
    raise RuntimeError("did not reach the plane")


def _wrapdiff(a, b):
    d = a - b
    d[4] = (d[4] + np.pi) % (2 * np.pi) - np.pi
    return d


def test_plane_propagation_matches_rk4_lorentz_force():
    rng = np.random.default_rng(21)
    for p in forward_states(10, rng, qpt_max=1.5):
        for zd in (20.0, 45.0, 110.0):
            ok, out, _, s, _ = oracle.propagate_plane(p, zd, BZ, jacobian=False)
            assert ok
            ref = rk4_to_plane(p, zd, BZ, h=0.02)
            assert out[2] == zd
            assert np.abs(out[:2] - ref[:2]).max() < 1e-8
            d = ref[3:]
            dphi = (out[4] - math.atan2(d[1], d[0]) + np.pi) % (2 * np.pi) - np.pi
            assert abs(dphi) < 1e-10
            assert abs(out[5] - math.acos(d[2] / np.linalg.norm(d))) < 1e-10
            assert s == pytest.approx((zd - p[2]) * math.tan(p[5]), rel=1e-14)


def test_zero_noise_disk_generator_hits_equal_plane_crossings():
    g = synth.Geometry.endcap()
    ev = synth.make_event(300, cfg=190, event=0, geometry=g, smear=False, scatter=False)
    worst = 0.0
    for i in range(300):
        p = ev.vertex_par[i].copy()
        for L in range(g.n_layers):
            ok, p, _, _, _ = oracle.propagate_plane(p, g.disk_z[L], g.bz, jacobian=False)
            assert ok
            h = ev.hits[L][ev.truth_hit[i, L]]
            worst = max(worst, float(np.abs(p[:3] - h).max()))
            assert abs(((p[4] - ev.truth_par[i, L, 4]) + np.pi) % (2 * np.pi) - np.pi) < 1e-9
    assert worst < 1e-9


def test_chord_from_origin_closed_form():
    """From the origin the transverse distance after path s is the chord
    2R |sin(s / 2R)| of the circle of radius R = pT / (kappa B)."""
    for pt, eta, zd in [(0.5, 2.0, 30.0), (1.0, 2.5, 110.0), (3.0, 1.9, 20.0), (0.4, 2.6, 100.0)]:
        th = 2 * math.atan(math.exp(-eta))
        for q in (1, -1):
            p = np.array([0.0, 0.0, 0.0, q / pt, 0.7, th])
            ok, out, _, s, _ = oracle.propagate_plane(p, zd, BZ, jacobian=False)
            assert ok
            R = pt / (KAPPA * BZ)
            assert s == pytest.approx(zd * math.tan(th), rel=1e-14)
            assert math.hypot(out[0], out[1]) == pytest.approx(2 * R * abs(math.sin(s / (2 * R))), rel=1e-12)
            # the momentum turns by s / R, clockwise for positive charge in +z field
            dphi = (out[4] - p[4] + np.pi) % (2 * np.pi) - np.pi
            assert dphi == pytest.approx(-q * s / R, rel=1e-12)


def test_plane_behind_or_parallel_fails():
    p = np.array([1.0, 0.0, 50.0, 0.5, 0.2, 0.3])
    ok, _, _, _, margin = oracle.propagate_plane(p, 40.0, BZ)      # moving away from z = 40
    assert not ok and margin < 0
    ok, _, _, _, margin = oracle.propagate_plane(p, 60.0, BZ)
    assert ok and margin > 0
    back = p.copy()
    back[5] = math.pi - 0.3                                            # heading to -z
    assert not oracle.propagate_plane(back, 60.0, BZ)[0]
    assert oracle.propagate_plane(back, 40.0, BZ)[0]


def test_plane_jacobian_matches_central_differences():
    rng = np.random.default_rng(22)
    steps = np.array([1e-6, 1e-6, 1e-6, 1e-7, 1e-7, 1e-7])
    worst = 0.0
    for p in forward_states(40, rng):
        for zd in (25.0, 100.0):
            ok, out, F, _, _ = oracle.propagate_plane(p, zd, BZ)
            assert ok
            num = np.zeros((6, 6))
            for j in range(6):
                pp, pm = p.copy(), p.copy()
                pp[j] += steps[j]
                pm[j] -= steps[j]
                _, op, _, _, _ = oracle.propagate_plane(pp, zd, BZ, jacobian=False)
                _, om, _, _, _ = oracle.propagate_plane(pm, zd, BZ, jacobian=False)
                num[:, j] = _wrapdiff(op, om) / (2 * steps[j])
            scale = np.maximum(np.abs(num), 1.0)
            worst = max(worst, float((np.abs(F - num) / scale).max()))
            # the plane fixes z: no variance can leak into it
            assert np.abs(F[2]).max() < 1e-12
    assert worst < 1e-6


def _H_disk(hit):
    ph = math.atan2(hit[1], hit[0])
    H = np.zeros((2, 6))
    H[0, 0], H[0, 1] = -math.sin(ph), math.cos(ph)
    H[1, 0], H[1, 1] = math.cos(ph), math.sin(ph)
    return H


def _disk_state(rng, zd):
    ph = rng.uniform(-np.pi, np.pi)
    r = rng.uniform(5, 35)
    return np.array([r * math.cos(ph), r * math.sin(ph), zd, rng.uniform(-2, 2),
                     rng.uniform(-np.pi, np.pi), rng.uniform(0.1, 0.5)])


def _spd(rng, scale=1e-3):
    A = rng.normal(size=(6, 6))
    return A @ A.T * scale + np.eye(6) * scale * 0.1


def test_disk_update_information_form():
    rng = np.random.default_rng(23)
    V = np.diag([SR ** 2, SV ** 2])
    for _ in range(50):
        p = _disk_state(rng, 40.0)
        Cm = _spd(rng)
        r = math.hypot(p[0], p[1])
        ph = math.atan2(p[1], p[0]) + rng.normal(0, 0.01 / r)
        rh = r + rng.normal(0, 0.1)
        hit = np.array([rh * math.cos(ph), rh * math.sin(ph), 40.0])
        pu, Cu, c2 = oracle.update(p, Cm, hit, SR, SV, kind=1)
        H = _H_disk(hit)
        info = np.linalg.inv(Cm) + H.T @ np.linalg.inv(V) @ H
        assert np.allclose(np.linalg.inv(Cu), info, rtol=1e-9, atol=1e-9 * np.abs(info).max())
        res = H[:, :2] @ (hit[:2] - p[:2])
        dp = Cu @ H.T @ np.linalg.inv(V) @ res
        assert np.allclose(_wrapdiff(pu, p), dp, rtol=1e-8, atol=1e-12)
        assert oracle.chi2(p, Cm, hit, SR, SV, kind=1) == pytest.approx(c2, rel=1e-14)


def test_disk_chi2_of_a_certain_state():
    """With no uncertainty in the state the chi2 is du^2/s_u^2 + dr^2/s_r^2
    for a hit displaced by du along r*phi and dr along r."""
    rng = np.random.default_rng(24)
    for _ in range(20):
        ph = rng.uniform(-np.pi, np.pi)
        rh = rng.uniform(5, 35)
        hit = np.array([rh * math.cos(ph), rh * math.sin(ph), 30.0])
        du, dr = rng.normal(0, 0.02), rng.normal(0, 0.2)
        pos = hit[:2] - du * np.array([-math.sin(ph), math.cos(ph)]) - dr * np.array([math.cos(ph), math.sin(ph)])
        p = np.array([pos[0], pos[1], 30.0, 0.5, 1.0, 0.3])
        c2 = oracle.chi2(p, np.zeros((6, 6)), hit, SR, SV, kind=1)
        assert c2 == pytest.approx(du ** 2 / SR ** 2 + dr ** 2 / SV ** 2, rel=1e-10)
        # the barrel projection of the same pair would measure z instead of r
        assert oracle.chi2(p, np.zeros((6, 6)), hit, SR, SV, kind=0) == pytest.approx(du ** 2 / SR ** 2, rel=1e-10)


def test_disk_scattering_uses_the_angle_to_z():
    """Highland angle with the path x0 / |cos theta| through a disk."""
    x0, mass = 0.002, 0.0
    for th in (0.15, 0.3, 0.5):
        p = np.array([10.0, 0.0, 30.0, 1.0, 0.4, th])
        Q = oracle.add_ms(p, np.zeros((6, 6)), x0, mass, kind=1)
        t = x0 / math.cos(th)
        pinv = abs(p[3]) * math.sin(th)
        th0 = 0.0136 * pinv * math.sqrt(t) * (1 + 0.038 * math.log(t))
        assert Q[5, 5] == pytest.approx(th0 ** 2, rel=1e-12)
        assert Q[4, 4] == pytest.approx(th0 ** 2 / math.sin(th) ** 2, rel=1e-12)
        assert np.abs(Q[:3]).max() == 0.0


def test_disk_fit_exact_recovery_with_perfect_hits():
    g = dataclasses.replace(synth.Geometry.endcap(), x0=tuple(0.0 for _ in range(10)))
    ev = synth.make_event(200, cfg=192, event=0, geometry=g, smear=False, scatter=False)
    cfg = oracle.config(g)
    res = oracle.fit(cfg, ev.hits, ev.truth_par[:, 0].copy(), ev.prior_cov, ev.truth_hit)
    d = _wrapdiff(res["par"].T, ev.truth_par[:, 9].T).T
    assert np.abs(d / np.maximum(np.abs(ev.truth_par[:, 9]), 1.0)).max() < 1e-10
    assert np.abs(res["chi2"]).max() < 1e-12


def test_disk_fit_pulls_and_chi2():
    """Generated disk events (Gaussian r*phi and r resolution, Highland
    scattering at the disk incidence) fit with unit-width pulls and chi2_2
    hit residuals."""
    g = synth.Geometry.endcap()
    ev = synth.make_event(20000, cfg=193, event=0, geometry=g, noise=0.0)
    cfg = oracle.config(g)
    res = oracle.fit(cfg, ev.hits, ev.prior_par, ev.prior_cov, ev.truth_hit, n_threads=8,
                     want_hit_chi2=True)
    assert (res["status"] == 0).all() and (res["ndof"] == 15).all()
    d = _wrapdiff(res["par"].T, ev.truth_par[:, 9].T).T
    Cm = synth.unpack_sym(res["cov"])
    assert np.abs(d[:, 2]).max() == 0.0 and np.abs(Cm[:, 2, :]).max() < 1e-12
    ph = np.arctan2(res["par"][:, 1], res["par"][:, 0])
    n = d.shape[0]
    pulls = []
    for e in (np.stack([-np.sin(ph), np.cos(ph)], 1), np.stack([np.cos(ph), np.sin(ph)], 1)):
        v = (e * d[:, :2]).sum(1)
        pulls.append(v / np.sqrt(np.einsum("ni,nij,nj->n", e, Cm[:, :2, :2], e)))
    pulls += [d[:, j] / np.sqrt(Cm[:, j, j]) for j in (3, 4, 5)]
    for pl in pulls:
        assert abs(pl.mean()) < 3.0 / math.sqrt(n)
        assert abs(pl.std() - 1.0) < 3.0 / math.sqrt(2 * n)
    # from layer 5 on: the first predictions after three disk hits (curvature
    # known to ~0.5/GeV from a few cm of arc) carry a few percent of
    # linearisation excess, which vanishes with finer hits (below)
    c2 = res["hit_chi2"][:, 5:].ravel()
    assert abs(c2.mean() - 2.0) < 3.0 * 2.0 / math.sqrt(c2.size)
    assert stats.kstest(c2[:20000], "chi2", args=(2,)).pvalue > 0.01
    g0 = dataclasses.replace(g, x0=tuple(0.0 for _ in range(10)))
    ev = synth.make_event(20000, cfg=193, event=1, geometry=g0, noise=0.0, scatter=False, smear_scale=0.1)
    cfg = oracle.config(g0)
    cfg.sigma_rphi *= 0.1
    cfg.sigma_r *= 0.1
    res = oracle.fit(cfg, ev.hits, ev.prior_par, ev.prior_cov, ev.truth_hit, n_threads=8, want_hit_chi2=True)
    c2 = res["hit_chi2"][:, 3:].ravel()
    assert abs(c2.mean() - 2.0) < 3.0 * 2.0 / math.sqrt(c2.size)


def test_disk_seed_covariance_covers_the_seed_spread():
    """The disk seed's stated covariance is at least the measured spread of
    the three-hit estimate (chi2 per seed of about 5 or less on average)."""
    g = synth.Geometry.endcap()
    ev = synth.make_event(5000, cfg=194, event=0, geometry=g, noise=0.0)
    d = _wrapdiff(ev.seed_par.T, ev.truth_par[:, 2].T).T
    Cm = synth.unpack_sym(ev.seed_cov)
    keep = [0, 1, 3, 4, 5]
    c2 = np.array([d[i, keep] @ np.linalg.solve(Cm[i][np.ix_(keep, keep)], d[i, keep]) for i in range(5000)])
    assert 2.0 < c2.mean() < 5.0


def test_disk_circle_prior_recovers_exact_helix_and_frame():
    g = synth.Geometry.endcap()
    ev = synth.make_event(500, cfg=195, event=0, geometry=g, noise=0.0, smear=False, scatter=False)
    cfg = oracle.config(g)
    par, cov, ok = oracle.circle_prior(cfg, ev.hits, ev.truth_hit)
    assert ok.all()
    d = _wrapdiff(par.T, ev.truth_par[:, 0].T).T
    assert np.abs(d).max() < 1e-9
    sig = np.asarray(oracle.FIT_PRIOR_SIGMA)
    Cm = synth.unpack_sym(cov)
    for i in range(0, 500, 61):
        a = np.arctan2(par[i, 1], par[i, 0])
        G = np.zeros((6, 5))
        G[:2, 0] = (-np.sin(a), np.cos(a))
        G[:2, 1] = (np.cos(a), np.sin(a))
        G[3, 2] = G[4, 3] = G[5, 4] = 1.0
        assert np.allclose(G.T @ Cm[i] @ G, np.diag(sig ** 2), rtol=1e-12, atol=1e-12)
        assert np.abs(Cm[i, 2]).max() == 0.0
    # the generator's own (independent) disk prior has the same frame
    assert np.allclose(synth.unpack_sym(ev.prior_cov), Cm, rtol=1e-12, atol=1e-15)


def _tiny_disk_event(rng_seed, branch_layers=(3, 5, 7), n_tracks=2):
    g = synth.Geometry.endcap()
    ev = synth.make_event(n_tracks, cfg=196, event=rng_seed, geometry=g, noise=0.0)
    rng = np.random.default_rng(rng_seed)
    hits = [h.copy() for h in ev.hits]
    for L in branch_layers:
        h = hits[L][ev.truth_hit[0, L]]
        r = math.hypot(h[0], h[1])
        ph = math.atan2(h[1], h[0]) + rng.choice([-1, 1]) * 0.015 / r
        r2 = r + rng.normal(0, 0.12)
        hits[L] = np.concatenate([hits[L], [[r2 * math.cos(ph), r2 * math.sin(ph), h[2]]]])
    return ev, hits


def _enumerate_disk_paths(cfg, hits, sp, sc, sh):
    nsl, nl = cfg.n_seed_layers, cfg.n_layers
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
            Cm = oracle.add_ms(pth["par"], pth["C"], cfg.x0[L - 1], cfg.mass, kind=1)
            ok, pp, F, _, _ = oracle.propagate_plane(pth["par"], cfg.zplane[L], cfg.bz)
            assert ok
            Cp = oracle.transport(F, Cm)
            acc = [j for j, h in enumerate(hits[L]) if h[0] * pp[0] + h[1] * pp[1] > 0
                   and oracle.chi2(pp, Cp, h, cfg.sigma_rphi, cfg.sigma_r, kind=1) < cfg.chi2_cut]
            for j in acc:
                pu, Cu, c2 = oracle.update(pp, Cp, hits[L][j], cfg.sigma_rphi, cfg.sigma_r, kind=1)
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


@pytest.mark.parametrize("rng_seed", [0, 1, 2, 3])
def test_disk_beam_equals_exhaustive_enumeration(rng_seed):
    ev, hits = _tiny_disk_event(rng_seed)
    cfg = oracle.config(ev.geometry, max_cands=16)
    for s in range(ev.n_seeds):
        paths, max_live = _enumerate_disk_paths(cfg, hits, ev.seed_par[s], ev.seed_cov[s], ev.seed_hits[s])
        assert max_live <= 16
        out = oracle.build_tracks(cfg, hits, ev.seed_par, ev.seed_cov, ev.seed_hits, seed_ids=[s])[0]
        best = paths[0]
        assert list(out["hits"][:10]) == best["hits"]
        assert out["chi2"] == pytest.approx(best["chi2"], rel=1e-12, abs=1e-12)
        assert out["n_final"] == len(paths)
        assert np.allclose(out["par"], best["par"], rtol=1e-12, atol=1e-12)
        if s == 0:
            assert max_live >= 2


def test_disk_build_efficiency_with_noise():
    g = synth.Geometry.endcap()
    ev = synth.make_event(1500, cfg=197, event=0, geometry=g, noise=0.3)
    eff = {}
    for k in (1, 6):
        cfg = oracle.config(g, max_cands=k)
        out = oracle.build_tracks(cfg, ev.hits, ev.seed_par, ev.seed_cov, ev.seed_hits, n_threads=8)
        eff[k] = (out["hits"][:, :10] == ev.truth_hit).all(axis=1).mean()
        assert (out["status"] == 0).mean() > 0.97
    assert eff[6] >= eff[1] and eff[6] > 0.9
