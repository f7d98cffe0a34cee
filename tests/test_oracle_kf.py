"""Pins of the oracle's measurement update, multiple scattering and fit.

Independent references: the information-filter identities, a Monte-Carlo of
the generator-style scattering kick, the Highland value, weighted least
squares on the stacked linearised problem, exact recovery of the true track,
unit-width pulls and chi2_2 statistics, and Gluckstern's resolution formula.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1702_06359_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SR, SZ = 0.01, 0.1


def _spd(rng, scale=1e-3):
    A = rng.normal(size=(6, 6))
    return A @ A.T * scale + np.eye(6) * scale * 0.1


def _state_on(rng, r):
    ph = rng.uniform(-np.pi, np.pi)
    return np.array([r * math.cos(ph), r * math.sin(ph), rng.uniform(-5, 5),
                     rng.uniform(-2, 2), ph + rng.uniform(-0.3, 0.3), rng.uniform(0.8, 2.3)])


def _hit_near(rng, p, r):
    ph = math.atan2(p[1], p[0]) + rng.normal(0, 0.01 / r)
    return np.array([r * math.cos(ph), r * math.sin(ph), p[2] + rng.normal(0, 0.1)])


def _H(hit):
    ph = math.atan2(hit[1], hit[0])
    H = np.zeros((2, 6))
    H[0, 0], H[0, 1], H[1, 2] = -math.sin(ph), math.cos(ph), 1.0
    return H


def test_update_information_form():
    """(C+)^-1 = C^-1 + H^T V^-1 H and p+ = p + C+ H^T V^-1 r (information filter)."""
    rng = np.random.default_rng(1)
    V = np.diag([SR ** 2, SZ ** 2])
    for _ in range(50):
        p = _state_on(rng, 20.0)
        Cm = _spd(rng)
        hit = _hit_near(rng, p, 20.0)
        pu, Cu, c2 = oracle.update(p, Cm, hit, SR, SZ)
        H = _H(hit)
        info = np.linalg.inv(Cm) + H.T @ np.linalg.inv(V) @ H
        assert np.allclose(np.linalg.inv(Cu), info, rtol=1e-9, atol=1e-9 * np.abs(info).max())
        ph = math.atan2(hit[1], hit[0])
        res = np.array([(hit[0] - p[0]) * -math.sin(ph) + (hit[1] - p[1]) * math.cos(ph), hit[2] - p[2]])
        dp = Cu @ H.T @ np.linalg.inv(V) @ res
        d = pu - p
        d[4] = (d[4] + np.pi) % (2 * np.pi) - np.pi
        assert np.allclose(d, dp, rtol=1e-8, atol=1e-12)
        # filtered chi2 decomposition: r^T S^-1 r = r+^T V^-1 r+ + dp^T C^-1 dp
        res_post = res - H @ dp
        c2_ref = res_post @ np.linalg.inv(V) @ res_post + dp @ np.linalg.inv(Cm) @ dp
        assert c2 == pytest.approx(c2_ref, rel=1e-8)
        assert oracle.chi2(p, Cm, hit, SR, SZ) == pytest.approx(c2, rel=1e-14)


def test_highland_golden_at_normal_incidence():
    with open(os.path.join(GOLDEN, "closed_forms.json")) as f:
        g = json.load(f)["highland"]
    # p = 1 GeV (q/pT = 1 at theta = 90 deg), momentum along the layer normal, beta = 1
    p = np.array([10.0, 0.0, 0.0, 1.0, 0.0, math.pi / 2])
    Q = oracle.add_ms(p, np.zeros((6, 6)), g["x_over_x0"], 0.0)
    assert math.sqrt(Q[5, 5]) == pytest.approx(g["theta0"], rel=1e-6)
    assert math.sqrt(Q[4, 4]) == pytest.approx(g["theta0"], rel=1e-6)
    assert np.count_nonzero(Q[:3]) == 0 and np.count_nonzero(Q[:, :3]) == 0


def test_scattering_noise_matches_kick_monte_carlo():
    """Q on (q/pT, phi, theta) equals the covariance of random kicks of the
    momentum direction at fixed |p| (two Gaussian angles orthogonal to p)."""
    rng = np.random.default_rng(2)
    for qpt, th, dphi in [(1.5, 1.1, 0.2), (-0.3, 2.0, -0.4), (0.8, 0.9, 0.0)]:
        p = np.array([12.0 * math.cos(0.3), 12.0 * math.sin(0.3), 1.0, qpt, 0.3 + dphi, th])
        Q = oracle.add_ms(p, np.zeros((6, 6)), 0.002, 0.13957)
        th0 = math.sqrt(Q[5, 5])
        n = 400000
        a1 = rng.normal(0, th0, n)
        a2 = rng.normal(0, th0, n)
        phi = p[4]
        d = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
        e1 = np.array([-math.sin(phi), math.cos(phi), 0.0])
        e2 = np.array([math.cos(th) * math.cos(phi), math.cos(th) * math.sin(phi), -math.sin(th)])
        dd = d[None] + a1[:, None] * e1 + a2[:, None] * e2
        dd /= np.linalg.norm(dd, axis=1, keepdims=True)
        mom = 1.0 / (abs(qpt) * math.sin(th))
        nphi = np.arctan2(dd[:, 1], dd[:, 0])
        nth = np.arccos(dd[:, 2])
        nq = np.sign(qpt) / (mom * np.sin(nth))
        S = np.cov(np.stack([nq - qpt, nphi - phi, nth - th]))
        ref = Q[3:, 3:]
        scale = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
        assert np.abs(S - ref).max() / scale.max() < 0.01


def test_scattering_commutes_with_update_on_same_surface():
    """H Q = 0: adding Q before or after the update on that layer gives the same result."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        p = _state_on(rng, 16.0)
        Cm = _spd(rng)
        hit = _hit_near(rng, p, 16.0)
        Q = oracle.add_ms(p, np.zeros((6, 6)), 0.002, 0.13957)
        pa, Ca, _ = oracle.update(p, Cm, hit, SR, SZ)
        pb, Cb, _ = oracle.update(p, Cm + Q, hit, SR, SZ)
        assert np.allclose(pa, pb, atol=1e-13)
        assert np.allclose(Ca + Q, Cb, atol=1e-13 * np.abs(Cb).max())


def _local_frame(phi_pos):
    G = np.zeros((6, 5))
    G[0, 0], G[1, 0] = -math.sin(phi_pos), math.cos(phi_pos)
    G[2, 1] = G[3, 2] = G[4, 3] = G[5, 4] = 1.0
    return G


def test_fit_equals_weighted_least_squares_in_linear_limit():
    """Smearing scaled by 1e-3 and no material: the KF estimate at the last
    layer equals batch weighted least squares of the problem linearised about
    the true trajectory (stacked H_L J_L rows plus the prior's information)."""
    geo = synth.Geometry(x0=tuple(0.0 for _ in range(10)))
    ev = synth.make_event(40, cfg=91, event=0, geometry=geo, smear_scale=1e-3, scatter=False)
    cfg = oracle.config(geo)
    res = oracle.fit(cfg, ev.hits, ev.prior_par, ev.prior_cov, ev.truth_hit)
    # the fit uses the nominal sigmas, so the normal equations do too
    V_nom = np.diag([SR ** 2, SZ ** 2])
    for i in range(40):
        tp = ev.truth_par[i]
        G = _local_frame(math.atan2(tp[0, 1], tp[0, 0]))
        J = np.eye(6)
        rows, rhs = [], []
        prior_sig = np.array(synth.PRIOR_SIGMA)
        dq_prior = G.T @ np.r_[ev.prior_par[i][:4] - tp[0][:4],
                               (ev.prior_par[i][4] - tp[0][4] + np.pi) % (2 * np.pi) - np.pi,
                               ev.prior_par[i][5] - tp[0][5]]
        rows.append(np.diag(1.0 / prior_sig))
        rhs.append(dq_prior / prior_sig)
        for L in range(10):
            if L > 0:
                ok, _, F, _, _ = oracle.propagate(tp[L - 1], geo.radii[L], geo.bz)
                J = F @ J
            hit = ev.hits[L][ev.truth_hit[i, L]]
            H = _H(hit)
            ph = math.atan2(hit[1], hit[0])
            r0 = np.array([(hit[0] - tp[L, 0]) * -math.sin(ph) + (hit[1] - tp[L, 1]) * math.cos(ph),
                           hit[2] - tp[L, 2]])
            A = H @ J @ G
            w = 1.0 / np.sqrt(np.diag(V_nom))
            rows.append(A * w[:, None])
            rhs.append(r0 * w)
        Amat = np.vstack(rows)
        bvec = np.concatenate(rhs)
        dq, *_ = np.linalg.lstsq(Amat, bvec, rcond=None)
        N = Amat.T @ Amat
        est = tp[9] + J @ G @ dq
        cov = J @ G @ np.linalg.inv(N) @ G.T @ J.T
        got = res["par"][i]
        gcov = synth.unpack_sym(res["cov"][i])
        d = got - est
        d[4] = (d[4] + np.pi) % (2 * np.pi) - np.pi
        G9 = _local_frame(math.atan2(est[1], est[0]))
        dl = G9.T @ d
        sl = np.sqrt(np.diag(G9.T @ cov @ G9)) * 1e-3   # spread of this scaled-down fit
        assert np.abs(dl / sl).max() < 1e-3
        c5 = G9.T @ cov @ G9
        g5 = G9.T @ gcov @ G9
        assert np.abs(np.diag(g5) / np.diag(c5) - 1).max() < 1e-4


def test_fit_exact_recovery_with_perfect_hits():
    geo = synth.Geometry(x0=tuple(0.0 for _ in range(10)))
    ev = synth.make_event(200, cfg=92, event=0, geometry=geo, smear=False, scatter=False)
    cfg = oracle.config(geo)
    prior = ev.truth_par[:, 0].copy()
    res = oracle.fit(cfg, ev.hits, prior, ev.prior_cov, ev.truth_hit)
    d = res["par"] - ev.truth_par[:, 9]
    d[:, 4] = (d[:, 4] + np.pi) % (2 * np.pi) - np.pi
    scale = np.maximum(np.abs(ev.truth_par[:, 9]), 1.0)
    assert np.abs(d / scale).max() < 1e-10
    assert np.abs(res["chi2"]).max() < 1e-12


def _rank5_ok(par, cov, rel, max_tilt=2e-3):
    """Symmetric, positive definite on the 5-D local frame, and rank 5: the
    null eigenvector is the layer normal at the point where the last update
    linearised, which the update moves by u/r rad at most."""
    Cm = synth.unpack_sym(cov)
    assert np.allclose(Cm, np.swapaxes(Cm, -1, -2))
    ph = np.arctan2(par[:, 1], par[:, 0])
    for i in range(par.shape[0]):
        G = _local_frame(ph[i])
        np.linalg.cholesky(G.T @ Cm[i] @ G)
        w, V = np.linalg.eigh(Cm[i])
        assert abs(w[0]) <= rel * np.trace(Cm[i])
        v = V[:, 0]
        assert np.linalg.norm(v[:2]) > 1 - 1e-6
        n = np.array([math.cos(ph[i]), math.sin(ph[i])])
        assert abs(abs(v[:2] @ n) - 1.0) < max_tilt ** 2


def test_fit_statistics_pulls_chi2_and_rank5():
    ev = synth.make_event(20000, cfg=93, event=0, noise=0.0)
    cfg = oracle.config(ev.geometry)
    res = oracle.fit(cfg, ev.hits, ev.prior_par, ev.prior_cov, ev.truth_hit, n_threads=8,
                     want_hit_chi2=True)
    assert (res["status"] == 0).all() and (res["ndof"] == 15).all()
    _rank5_ok(res["par"][:2000], res["cov"][:2000], 1e-10)
    tp = ev.truth_par[:, 9]
    d = res["par"] - tp
    d[:, 4] = (d[:, 4] + np.pi) % (2 * np.pi) - np.pi
    Cm = synth.unpack_sym(res["cov"])
    ph = np.arctan2(res["par"][:, 1], res["par"][:, 0])
    eu = np.stack([-np.sin(ph), np.cos(ph)], 1)
    u = (eu * d[:, :2]).sum(1)
    vu = np.einsum("ni,nij,nj->n", eu, Cm[:, :2, :2], eu)
    n = d.shape[0]
    pulls = [u / np.sqrt(vu)] + [d[:, j] / np.sqrt(Cm[:, j, j]) for j in (2, 3, 4, 5)]
    for pl in pulls:
        assert abs(pl.mean()) < 3.0 / math.sqrt(n)
        assert abs(pl.std() - 1.0) < 3.0 / math.sqrt(2 * n)
    c2 = res["hit_chi2"][:, 3:].ravel()
    assert abs(c2.mean() - 2.0) < 3.0 * 2.0 / math.sqrt(c2.size)
    assert stats.kstest(c2[:20000], "chi2", args=(2,)).pvalue > 0.01


def test_gluckstern_resolution_at_10_gev():
    with open(os.path.join(GOLDEN, "closed_forms.json")) as f:
        g = json.load(f)["gluckstern"]
    geo = synth.Geometry(x0=tuple(0.0 for _ in range(10)))
    ev = synth.make_event(5000, cfg=94, event=0, geometry=geo, noise=0.0, scatter=False,
                          pt_range=(g["pt"], g["pt"]))
    cfg = oracle.config(geo)
    res = oracle.fit(cfg, ev.hits, ev.prior_par, ev.prior_cov, ev.truth_hit, n_threads=8)
    q = res["par"][:, 3]
    qt = ev.truth_par[:, 9, 3]
    emp = np.std((q - qt) / np.abs(qt))
    own = np.median(np.sqrt(synth.unpack_sym(res["cov"])[:, 3, 3]) / np.abs(qt))
    assert emp == pytest.approx(g["sigma_pt_over_pt"], rel=0.15)
    assert own == pytest.approx(g["sigma_pt_over_pt"], rel=0.15)


def test_circle_prior_recovers_exact_helix_and_frame():
    """Final-fit prior (helix through the hits on layers 0-2): with hits
    exactly on the generator's helix (no smearing, no scattering) it is the
    true state at the first layer; its covariance is diag(sigma)^2 in the
    layer-tangent frame; a missing hit gives no prior."""
    ev = synth.make_event(800, cfg=301, event=0, noise=0.0, smear=False, scatter=False)
    cfg = oracle.config(ev.geometry)
    par, cov, ok = oracle.circle_prior(cfg, ev.hits, ev.truth_hit)
    assert ok.all()
    d = par - ev.truth_par[:, 0]
    d[:, 4] = (d[:, 4] + np.pi) % (2 * np.pi) - np.pi
    assert np.abs(d[:, :3]).max() < 1e-9
    assert np.abs(d[:, 3:]).max() < 1e-9
    sig = np.asarray(oracle.FIT_PRIOR_SIGMA)
    Cm = synth.unpack_sym(cov)
    for i in range(0, 800, 97):
        a = np.arctan2(par[i, 1], par[i, 0])
        G = np.zeros((6, 5))
        G[:2, 0] = (-np.sin(a), np.cos(a))
        G[2, 1] = G[3, 2] = G[4, 3] = G[5, 4] = 1.0
        assert np.allclose(G.T @ Cm[i] @ G, np.diag(sig ** 2), rtol=1e-12, atol=1e-15)
        n = np.array([np.cos(a), np.sin(a), 0, 0, 0, 0])   # no variance along the layer normal
        assert abs(n @ Cm[i] @ n) < 1e-12
    th = ev.truth_hit.copy()
    th[5, 1] = -1
    _, _, ok2 = oracle.circle_prior(cfg, ev.hits, th)
    assert not ok2[5] and ok2[[4, 6]].all()


def test_circle_prior_fit_matches_generator_prior_fit():
    """The fit from the oracle's prior equals the fit from the generator's own
    prior construction (independent code, same reading) on smeared events."""
    ev = synth.make_event(400, cfg=302, event=0, noise=0.0)
    cfg = oracle.config(ev.geometry)
    par, cov, ok = oracle.circle_prior(cfg, ev.hits, ev.truth_hit)
    assert ok.all()
    a = oracle.fit(cfg, ev.hits, par, cov, ev.truth_hit, n_threads=4)
    b = oracle.fit(cfg, ev.hits, ev.prior_par, ev.prior_cov, ev.truth_hit, n_threads=4)
    assert np.allclose(a["par"], b["par"], rtol=1e-9, atol=1e-9)
    assert np.allclose(a["chi2"], b["chi2"], rtol=1e-9, atol=1e-9)
