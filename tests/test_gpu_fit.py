"""GPU KF fit against the FP64 oracle (element by element on seeded inputs)."""
import numpy as np
import pytest

import oracle
from conftest import report
from paper_1702_06359_amd import abi, synth
from parity_util import TOL, local_frame, state_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_required):
    c = abi.Context(abi.config_from_geometry(synth.Geometry(), max_cands=6))
    yield c
    c.close()


def _fit_both(ctx, ev, hits_assign, prior_par=None, prior_cov=None):
    prior_par = ev.prior_par if prior_par is None else prior_par
    prior_cov = ev.prior_cov if prior_cov is None else prior_cov
    h = ctx.load_event(abi.EventArrays(ev.hits))
    try:
        g = ctx.fit(h, prior_par, prior_cov, hits_assign)
    finally:
        ctx.unload_event(h)
    o = oracle.fit(oracle.config(ev.geometry), ev.hits, prior_par, prior_cov, hits_assign, n_threads=8)
    return g, o


def _check(name, g, o, tol=None, prior_cov=None, disk=False):
    """Element-wise parity.  With prior_cov, each covariance component's
    tolerance is max(tau_cov_rel, f R 2^-24), R = prior variance / final
    variance in the local frame (the conditioning of that track's fit)."""
    tol = tol or TOL["fit"]
    assert (g["status"] == o["status"]).all()
    ok = o["status"] == 0
    assert (g["ndof"][ok] == o["ndof"][ok]).all()
    dpar, dcov = state_errors(g["par"][ok], g["cov"][ok], o["par"][ok], o["cov"][ok], disk)
    dchi = np.abs(g["chi2"][ok] - o["chi2"][ok]) / (1.0 + o["chi2"][ok])
    cov_tol = np.full(int(ok.sum()), tol["tau_cov_rel"])
    chi_tol = np.full(int(ok.sum()), tol["eps_chi2_rel"])
    if prior_cov is not None:
        # each chi2 term is r^2/S with S built from that covariance
        R = conditioning(prior_cov[ok], o["par"][ok], o["cov"][ok], disk)
        cov_tol = np.maximum(cov_tol, tol["cov_conditioning_factor"] * R * 2.0 ** -24)
        chi_tol = np.maximum(chi_tol, tol["cov_conditioning_factor"] * R * 2.0 ** -24)
    rep = dict(n=int(ok.sum()), max_dpar_sigma=dpar.max(), p9999_dpar_sigma=np.quantile(dpar, 0.9999),
               p99_dpar_sigma=np.quantile(dpar, 0.99), max_dcov_rel=dcov.max(),
               p9999_dcov_rel=np.quantile(dcov, 0.9999), max_dchi2_rel=dchi.max(),
               p9999_dchi2_rel=np.quantile(dchi, 0.9999), max_dcov_over_tol=(dcov / cov_tol).max(),
               max_dchi2_over_tol=(dchi / chi_tol).max())
    report(name, rep)
    assert rep["max_dpar_sigma"] <= tol["tau_par_sigma"], rep
    assert rep["max_dcov_over_tol"] <= 1.0, rep
    assert rep["max_dchi2_over_tol"] <= 1.0, rep


def conditioning(prior_cov, par, cov, disk=False):
    """Per track, max over the local components of prior variance / final variance."""
    Cp = synth.unpack_sym(prior_cov)
    Cf = synth.unpack_sym(cov)
    R = np.zeros(par.shape[0])
    for i in range(par.shape[0]):
        G = local_frame(np.arctan2(par[i, 1], par[i, 0]), disk)
        R[i] = np.max(np.diag(G.T @ Cp[i] @ G) / np.diag(G.T @ Cf[i] @ G))
    return R


def test_fit_parity_true_hits(ctx):
    ev = synth.make_event(3001, cfg=200, event=0, noise=0.1)
    print("case fit_parity_true_hits n=3001", flush=True)
    g, o = _fit_both(ctx, ev, ev.truth_hit)
    _check("fit_parity_true_hits", g, o)


def test_fit_parity_with_skipped_layers(ctx):
    ev = synth.make_event(2500, cfg=201, event=0, noise=0.0)
    rng = np.random.default_rng(5)
    assign = ev.truth_hit.copy()
    drop = rng.uniform(size=assign.shape) < 0.2
    drop[:, 0] = False
    assign[drop] = -1
    print("case fit_parity_with_skipped_layers n=2500", flush=True)
    g, o = _fit_both(ctx, ev, assign)
    _check("fit_parity_with_skipped_layers", g, o, prior_cov=ev.prior_cov)
    assert (g["n_hits"] == (assign >= 0).sum(1)).all()


def test_fit_propagation_failure_status(ctx):
    ev = synth.make_event(64, cfg=202, event=0, noise=0.0, pt_range=(0.15, 0.15), eta_max=0.5)
    print("case fit_propagation_failure n=64", flush=True)
    g, o = _fit_both(ctx, ev, ev.truth_hit)
    assert (o["status"] == 2).all() and (g["status"] == 2).all()


def test_fit_batch_uneven_equals_single_fits(ctx):
    sizes = [2000, 37, 5001, 1, 640]
    evs = [synth.make_event(n, cfg=203, event=i, noise=0.05) for i, n in enumerate(sizes)]
    hs = [ctx.load_event(abi.EventArrays.from_synth(e, with_seeds=False, with_tracks=True)) for e in evs]
    try:
        print(f"case fit_batch sizes={sizes}", flush=True)
        outs = ctx.fit_batch(hs, sizes)
        for e, h, out in zip(evs, hs, outs):
            single = ctx.fit(h, e.prior_par, e.prior_cov, e.truth_hit)
            for k in ("par", "cov", "chi2", "n_hits", "status", "ndof"):
                assert np.array_equal(out[k], single[k]), k
        o = oracle.fit(oracle.config(evs[2].geometry), evs[2].hits, evs[2].prior_par, evs[2].prior_cov,
                       evs[2].truth_hit, n_threads=8)
        _check("fit_batch_event2", outs[2], o)
    finally:
        for h in hs:
            ctx.unload_event(h)


def test_fit_rejects_bad_input(ctx):
    ev = synth.make_event(10, cfg=204, event=0)
    h = ctx.load_event(abi.EventArrays(ev.hits))
    try:
        bad = ev.truth_hit.copy()
        bad[3, 4] = ev.hits[4].shape[0]
        with pytest.raises(abi.MkfError) as e:
            ctx.fit(h, ev.prior_par, ev.prior_cov, bad)
        assert e.value.status == abi.E_INVALID
        par = ev.prior_par.copy()
        par[2, 1] = np.nan
        with pytest.raises(abi.MkfError):
            ctx.fit(h, par, ev.prior_cov, ev.truth_hit)
        empty = ctx.fit(h, np.zeros((0, 6)), np.zeros((0, 21)), np.zeros((0, 10), np.int32))
        assert empty["par"].shape == (0, 6)
    finally:
        ctx.unload_event(h)


def test_build_then_fit_on_device(gpu_required):
    """Built tracks fitted on the device without leaving it (build_batch with
    BATCH_FIT), against the oracle's fit of the same hit lists from the
    oracle's own prior; a track without its layer-1 hit gets no prior."""
    c = abi.Context(abi.config_from_geometry(synth.Geometry(), max_cands=6))
    ev = synth.make_event(2500, cfg=205, event=0, noise=0.1)
    sh = ev.seed_hits.copy()
    sh[7, 1] = -1
    h = c.load_event(abi.EventArrays(ev.hits, ev.seed_par, ev.seed_cov, sh))
    try:
        print("case build+fit n=2500", flush=True)
        built = c.build_batch([h], [ev.n_seeds], flags=abi.BATCH_REINDEX | abi.BATCH_FIT)[0]
        g = c.fetch_fit(h, ev.n_seeds)
        again = c.fetch_tracks(h, ev.n_seeds)
    finally:
        c.unload_event(h)
        c.close()
    assert np.array_equal(built["hits"], again["hits"]) and np.array_equal(g["hits"], built["hits"])
    cfg = oracle.config(ev.geometry)
    par, cov, ok = oracle.circle_prior(cfg, ev.hits, built["hits"])
    assert not ok[7] and g["status"][7] == 3
    o = oracle.fit(cfg, ev.hits, par, cov, built["hits"], n_threads=8)
    o["status"] = np.where(ok, o["status"], 3)
    keep = ok
    assert (g["n_hits"][keep] == (built["hits"][keep] >= 0).sum(1)).all()
    sub = lambda d: {k: v[keep] for k, v in d.items() if isinstance(v, np.ndarray) and v.shape[:1] == keep.shape}
    _check("build_then_fit", sub(g), sub(o), prior_cov=cov[keep])
