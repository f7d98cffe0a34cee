"""FP64 CPU oracle of the Kalman-filter track builder, barrel and endcap (ctypes binding).

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg use it.  The GPU library never imports, links or
calls anything here, and this module imports nothing from the GPU package
(only the shared synthetic-event generator is used by callers of both).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mkf_oracle.c")
HDR = os.path.join(HERE, "mkf_oracle.h")
LIB = os.path.join(HERE, "liboracle.so")

MAX_LAYERS = 16
MAX_CANDS = 16
MAX_ALT = 4
CUT_CONSIDER = 0.1      # decisions re-run to test their relevance (see mkf_oracle.h)
RANK_CONSIDER = 0.01


class OrcConfig(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32), ("n_seed_layers", C.c_int32), ("max_cands", C.c_int32),
        ("max_holes", C.c_int32), ("hole_always", C.c_int32), ("update3d", C.c_int32),
        ("radius", C.c_double * MAX_LAYERS), ("x0", C.c_double * MAX_LAYERS),
        ("bz", C.c_double), ("sigma_rphi", C.c_double), ("sigma_z", C.c_double),
        ("chi2_cut", C.c_double), ("mass", C.c_double),
        ("kind", C.c_int32 * MAX_LAYERS), ("zplane", C.c_double * MAX_LAYERS), ("sigma_r", C.c_double),
        ("thick", C.c_double * MAX_LAYERS),
    ]


class OrcHits(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("pad_", C.c_int32),
                ("n_hits", C.POINTER(C.c_int32)), ("xyz", C.POINTER(C.POINTER(C.c_double)))]


class OrcTrack(C.Structure):
    _fields_ = [
        ("par", C.c_double * 6), ("cov", C.c_double * 21), ("chi2", C.c_double),
        ("hits", C.c_int32 * MAX_LAYERS), ("n_hits", C.c_int32), ("n_holes", C.c_int32),
        ("status", C.c_int32), ("n_final", C.c_int32),
        ("m_cut", C.c_double), ("m_rank", C.c_double), ("m_prop", C.c_double),
        ("m_cut_raw", C.c_double), ("m_rank_raw", C.c_double),
        ("n_alt", C.c_int32), ("alt_kind", C.c_int32 * MAX_ALT), ("alt_margin", C.c_double * MAX_ALT),
        ("alt_hits", (C.c_int32 * MAX_LAYERS) * MAX_ALT), ("alt_status", C.c_int32 * MAX_ALT),
        ("n_prop", C.c_int64), ("n_accept", C.c_int64), ("n_update", C.c_int64),
    ]


TRACK_DTYPE = np.dtype([
    ("par", np.float64, 6), ("cov", np.float64, 21), ("chi2", np.float64),
    ("hits", np.int32, MAX_LAYERS), ("n_hits", np.int32), ("n_holes", np.int32),
    ("status", np.int32), ("n_final", np.int32),
    ("m_cut", np.float64), ("m_rank", np.float64), ("m_prop", np.float64),
    ("m_cut_raw", np.float64), ("m_rank_raw", np.float64),
    ("n_alt", np.int32), ("alt_kind", np.int32, MAX_ALT), ("alt_margin", np.float64, MAX_ALT),
    ("alt_hits", np.int32, (MAX_ALT, MAX_LAYERS)), ("alt_status", np.int32, MAX_ALT),
    ("n_prop", np.int64), ("n_accept", np.int64), ("n_update", np.int64),
], align=True)
assert TRACK_DTYPE.itemsize == C.sizeof(OrcTrack)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, -O2, scalar double)."""
    fresh = (os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC)
             and os.path.getmtime(LIB) >= os.path.getmtime(HDR))
    if force or not fresh:
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.orc_propagate.argtypes = [dp, C.c_double, C.c_double, dp, dp, dp, dp]
        L.orc_propagate.restype = C.c_int
        L.orc_propagate_plane.argtypes = [dp, C.c_double, C.c_double, dp, dp, dp, dp]
        L.orc_propagate_plane.restype = C.c_int
        L.orc_step_near.argtypes = [dp, C.c_int, C.c_double, C.c_double, dp, dp, dp]
        L.orc_step_near.restype = C.c_int
        L.orc_add_ms.argtypes = [dp, C.c_int, C.c_double, C.c_double, dp]
        L.orc_chi2.argtypes = [dp, dp, dp, C.c_int, C.c_double, C.c_double]
        L.orc_chi2.restype = C.c_double
        L.orc_update.argtypes = [dp, dp, dp, C.c_int, C.c_double, C.c_double, dp, dp]
        L.orc_update.restype = C.c_double
        L.orc_transport.argtypes = [dp, dp]
        L.orc_chi2_3d.argtypes = [dp, dp, dp, C.c_double, C.c_double, C.c_double]
        L.orc_chi2_3d.restype = C.c_double
        L.orc_update_3d.argtypes = [dp, dp, dp, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_update_3d.restype = C.c_double
        L.orc_fit.argtypes = [C.POINTER(OrcConfig), C.POINTER(OrcHits), C.c_int32, dp, dp, ip,
                              dp, dp, dp, ip, ip, dp, C.c_int32]
        L.orc_build.argtypes = [C.POINTER(OrcConfig), C.POINTER(OrcHits), C.c_int32, dp, dp, ip, ip,
                                C.c_int32, C.POINTER(OrcTrack), C.c_int32]
        L.orc_replay.argtypes = [C.POINTER(OrcConfig), C.POINTER(OrcHits), dp, dp, ip, dp, ip]
        L.orc_build_beam.argtypes = [C.POINTER(OrcConfig), C.POINTER(OrcHits), C.c_int32, dp, dp, ip, ip,
                                     C.c_int32, C.POINTER(OrcTrack), C.POINTER(OrcTrack), C.c_int32]
        L.orc_build_beam.restype = None
        L.orc_circle_prior.argtypes = [C.POINTER(OrcConfig), C.POINTER(OrcHits), C.c_int32, ip, dp, dp, dp, ip]
        L.orc_circle_prior.restype = None
        L.orc_replay.restype = C.c_double
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def config(geometry, *, max_cands=1, max_holes=1, chi2_cut=30.0, n_seed_layers=3,
           hole_always=False, update3d=False) -> OrcConfig:
    c = OrcConfig()
    c.n_layers = geometry.n_layers
    c.n_seed_layers = n_seed_layers
    c.max_cands = max_cands
    c.max_holes = max_holes
    c.hole_always = int(bool(hole_always))
    c.update3d = int(bool(update3d))
    for i in range(geometry.n_layers):
        c.radius[i] = geometry.radii[i]
        c.x0[i] = geometry.x0[i]
        if geometry.is_disk:
            c.kind[i] = 1
            c.zplane[i] = geometry.disk_z[i]
        c.thick[i] = geometry.thick(i)
    c.bz = geometry.bz
    c.sigma_rphi = geometry.sigma_rphi
    c.sigma_z = geometry.sigma_z
    c.chi2_cut = chi2_cut
    c.mass = geometry.mass
    c.sigma_r = geometry.sigma_r
    return c


class HitSet:
    """Keeps per-layer hit arrays alive while the oracle holds pointers to them."""

    def __init__(self, hits):
        self.arrays = [np.ascontiguousarray(h, dtype=np.float64).reshape(-1, 3) for h in hits]
        self.counts = np.array([a.shape[0] for a in self.arrays], dtype=np.int32)
        self.ptrs = (C.POINTER(C.c_double) * len(self.arrays))(*[_dp(a) for a in self.arrays])
        self.s = OrcHits()
        self.s.n_layers = len(self.arrays)
        self.s.n_hits = _ip(self.counts)
        self.s.xyz = C.cast(self.ptrs, C.POINTER(C.POINTER(C.c_double)))


def propagate(par, r, bz, jacobian=True):
    """Returns (ok, new_par, F or None, path, margin)."""
    p = _f64(par, (6,))
    out = np.zeros(6)
    F = np.zeros(36) if jacobian else None
    s = C.c_double(0.0)
    m = C.c_double(0.0)
    rc = lib().orc_propagate(_dp(p), float(r), float(bz), _dp(out), _dp(F) if F is not None else None,
                             C.byref(s), C.byref(m))
    return rc == 0, out, (F.reshape(6, 6) if F is not None else None), s.value, m.value


def propagate_plane(par, zd, bz, jacobian=True):
    """Propagation to the plane z = zd; returns (ok, new_par, F or None, path, margin)."""
    p = _f64(par, (6,))
    out = np.zeros(6)
    F = np.zeros(36) if jacobian else None
    s = C.c_double(0.0)
    m = C.c_double(0.0)
    rc = lib().orc_propagate_plane(_dp(p), float(zd), float(bz), _dp(out),
                                   _dp(F) if F is not None else None, C.byref(s), C.byref(m))
    return rc == 0, out, (F.reshape(6, 6) if F is not None else None), s.value, m.value


def step_near(par, kind, where, bz, jacobian=True):
    """Nearest crossing (either direction) of r = where (kind 0) or z = where
    (kind 1); returns (ok, new_par, F or None, signed path)."""
    p = _f64(par, (6,))
    out = np.zeros(6)
    F = np.zeros(36) if jacobian else None
    s = C.c_double(0.0)
    rc = lib().orc_step_near(_dp(p), int(kind), float(where), float(bz), _dp(out),
                             _dp(F) if F is not None else None, C.byref(s))
    return rc == 0, out, (F.reshape(6, 6) if F is not None else None), s.value


def add_ms(par, C6, x0, mass, kind=0):
    p = _f64(par, (6,))
    Cm = _f64(C6, (36,)).copy()
    lib().orc_add_ms(_dp(p), int(kind), float(x0), float(mass), _dp(Cm))
    return Cm.reshape(6, 6)


def transport(F, C6):
    Fm = _f64(F, (36,))
    Cm = _f64(C6, (36,)).copy()
    lib().orc_transport(_dp(Fm), _dp(Cm))
    return Cm.reshape(6, 6)


def chi2(par, C6, hit, sigma_rphi, sigma_2, kind=0):
    """kind 0: (r*phi, z) measurement of a cylinder; kind 1: (r*phi, r) of a disk."""
    return lib().orc_chi2(_dp(_f64(par, (6,))), _dp(_f64(C6, (36,))), _dp(_f64(hit, (3,))),
                          int(kind), sigma_rphi, sigma_2)


def update(par, C6, hit, sigma_rphi, sigma_2, kind=0):
    out_p = np.zeros(6)
    out_C = np.zeros(36)
    c2 = lib().orc_update(_dp(_f64(par, (6,))), _dp(_f64(C6, (36,))), _dp(_f64(hit, (3,))),
                          int(kind), sigma_rphi, sigma_2, _dp(out_p), _dp(out_C))
    return out_p, out_C.reshape(6, 6), c2


def chi2_3d(par, C6, hit, sigma_rphi, sigma_r, sigma_z):
    return lib().orc_chi2_3d(_dp(_f64(par, (6,))), _dp(_f64(C6, (36,))), _dp(_f64(hit, (3,))),
                             sigma_rphi, sigma_r, sigma_z)


def update_3d(par, C6, hit, sigma_rphi, sigma_r, sigma_z):
    out_p = np.zeros(6)
    out_C = np.zeros(36)
    c2 = lib().orc_update_3d(_dp(_f64(par, (6,))), _dp(_f64(C6, (36,))), _dp(_f64(hit, (3,))),
                             sigma_rphi, sigma_r, sigma_z, _dp(out_p), _dp(out_C))
    return out_p, out_C.reshape(6, 6), c2


def fit(cfg: OrcConfig, hits, init_par, init_cov, track_hits, n_threads=1, want_hit_chi2=False):
    hs = hits if isinstance(hits, HitSet) else HitSet(hits)
    n = int(np.asarray(init_par).shape[0])
    nl = cfg.n_layers
    ip_ = _f64(init_par, (n, 6))
    ic = _f64(init_cov, (n, 21))
    th = np.ascontiguousarray(track_hits, dtype=np.int32).reshape(n, nl)
    out_par = np.zeros((n, 6))
    out_cov = np.zeros((n, 21))
    out_chi2 = np.zeros(n)
    out_ndof = np.zeros(n, dtype=np.int32)
    out_status = np.zeros(n, dtype=np.int32)
    hc = np.zeros((n, nl)) if want_hit_chi2 else None
    lib().orc_fit(C.byref(cfg), C.byref(hs.s), n, _dp(ip_), _dp(ic), _ip(th), _dp(out_par),
                  _dp(out_cov), _dp(out_chi2), _ip(out_ndof), _ip(out_status),
                  _dp(hc) if hc is not None else None, int(n_threads))
    res = dict(par=out_par, cov=out_cov, chi2=out_chi2, ndof=out_ndof, status=out_status)
    if hc is not None:
        res["hit_chi2"] = hc
    return res


FIT_PRIOR_SIGMA = (1.0, 10.0, 1.0, 0.1, 0.1)   # (u cm, z cm, q/pT 1/GeV, phi, theta)


def circle_prior(cfg: OrcConfig, hits, track_hits, sig=FIT_PRIOR_SIGMA):
    """Prior of the final fit of built tracks: helix through the hits on
    layers 0-2, at the first hit, loose diagonal local covariance.  Returns
    (par, cov, ok)."""
    hs = hits if isinstance(hits, HitSet) else HitSet(hits)
    th = np.ascontiguousarray(track_hits, dtype=np.int32)
    n = th.shape[0]
    th = th.reshape(n, cfg.n_layers)
    par = np.zeros((n, 6))
    cov = np.zeros((n, 21))
    ok = np.zeros(n, dtype=np.int32)
    sg = np.ascontiguousarray(sig, dtype=np.float64)
    lib().orc_circle_prior(C.byref(cfg), C.byref(hs.s), n, _ip(th), _dp(sg), _dp(par), _dp(cov), _ip(ok))
    return par, cov, ok.astype(bool)


def build_tracks(cfg: OrcConfig, hits, seed_par, seed_cov, seed_hits, seed_ids=None, n_threads=1):
    """Combinatorial KF build; returns a structured array (TRACK_DTYPE), one row per seed."""
    hs = hits if isinstance(hits, HitSet) else HitSet(hits)
    n_total = int(np.asarray(seed_par).shape[0])
    sp = _f64(seed_par, (n_total, 6))
    sc = _f64(seed_cov, (n_total, 21))
    sh = np.ascontiguousarray(seed_hits, dtype=np.int32).reshape(n_total, cfg.n_seed_layers)
    if seed_ids is None:
        ids = None
        n_sel = n_total
    else:
        ids = np.ascontiguousarray(seed_ids, dtype=np.int32)
        n_sel = int(ids.shape[0])
    out = np.zeros(n_sel, dtype=TRACK_DTYPE)
    lib().orc_build(C.byref(cfg), C.byref(hs.s), n_total, _dp(sp), _dp(sc), _ip(sh),
                    _ip(ids) if ids is not None else None, n_sel,
                    out.ctypes.data_as(C.POINTER(OrcTrack)), int(n_threads))
    return out


def build_beam(cfg: OrcConfig, hits, seed_par, seed_cov, seed_hits, seed_ids=None, n_threads=1):
    """As build_tracks, plus the whole final beam: (tracks, beam) with beam of
    shape (n_sel, max_cands) (status -1 beyond the beam)."""
    hs = hits if isinstance(hits, HitSet) else HitSet(hits)
    n_total = int(np.asarray(seed_par).shape[0])
    sp = _f64(seed_par, (n_total, 6))
    sc = _f64(seed_cov, (n_total, 21))
    sh = np.ascontiguousarray(seed_hits, dtype=np.int32).reshape(n_total, cfg.n_seed_layers)
    ids = None if seed_ids is None else np.ascontiguousarray(seed_ids, dtype=np.int32)
    n_sel = n_total if ids is None else int(ids.shape[0])
    k = min(int(cfg.max_cands), MAX_CANDS)
    out = np.zeros(n_sel, dtype=TRACK_DTYPE)
    beam = np.zeros(n_sel * k, dtype=TRACK_DTYPE)
    lib().orc_build_beam(C.byref(cfg), C.byref(hs.s), n_total, _dp(sp), _dp(sc), _ip(sh),
                         _ip(ids) if ids is not None else None, n_sel, out.ctypes.data_as(C.POINTER(OrcTrack)),
                         beam.ctypes.data_as(C.POINTER(OrcTrack)), int(n_threads))
    return out, beam.reshape(n_sel, k)


def replay(cfg: OrcConfig, hits, seed_par, seed_cov, layer_hits):
    """Chi2 along a given hit list; returns (total, per-layer chi2, ok)."""
    hs = hits if isinstance(hits, HitSet) else HitSet(hits)
    lh = np.full(MAX_LAYERS, -1, dtype=np.int32)
    lh[:cfg.n_layers] = np.asarray(layer_hits, dtype=np.int32)[:cfg.n_layers]
    lc = np.zeros(MAX_LAYERS)
    ok = C.c_int32(0)
    tot = lib().orc_replay(C.byref(cfg), C.byref(hs.s), _dp(_f64(seed_par, (6,))),
                           _dp(_f64(seed_cov, (21,))), _ip(lh), _dp(lc), C.byref(ok))
    return tot, lc[:cfg.n_layers], bool(ok.value)
