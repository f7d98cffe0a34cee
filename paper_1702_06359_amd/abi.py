"""ctypes binding of the C ABI in include/mkf.h (argument marshalling only).

Every function of the header is available under its own name through
``lib()``; ``Context`` wraps them for numpy arrays.  The compute path is the
HIP library ``libmkf.so``: if it is missing this module raises, it never
falls back to anything else.  PyTorch, when it sees a GPU, supplies device
memory (its caching allocator) and the stream.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
import re
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmkf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mkf.h")

MAX_LAYERS = 16
MAX_CANDS = 8

OK, E_INVALID, E_NOMEM, E_DEVICE, E_AGAIN, E_NOTFOUND, E_STATE = 0, -1, -2, -3, -4, -5, -6
HOLE_ALWAYS = 0x1
UPDATE_3D = 0x2
BATCH_REINDEX, BATCH_STATS, BATCH_GRAPH, BATCH_ASYNC, BATCH_FIT, BATCH_BEAM = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
TIMER_BUILD, TIMER_INDEX, TIMER_FIT = 0, 1, 2

_STATUS_NAMES = {0: "MKF_OK", -1: "MKF_E_INVALID", -2: "MKF_E_NOMEM", -3: "MKF_E_DEVICE",
                 -4: "MKF_E_AGAIN", -5: "MKF_E_NOTFOUND", -6: "MKF_E_STATE"}


class MkfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Config(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32), ("n_seed_layers", C.c_int32), ("max_cands", C.c_int32),
        ("max_holes", C.c_int32), ("flags", C.c_uint32), ("reserved", C.c_int32),
        ("layer_r", C.c_double * MAX_LAYERS), ("layer_half_z", C.c_double * MAX_LAYERS),
        ("layer_x0", C.c_double * MAX_LAYERS),
        ("bz", C.c_double), ("sigma_rphi", C.c_double), ("sigma_z", C.c_double),
        ("chi2_cut", C.c_double), ("mass", C.c_double),
        ("layer_kind", C.c_int32 * MAX_LAYERS), ("layer_z", C.c_double * MAX_LAYERS),
        ("layer_rmin", C.c_double * MAX_LAYERS), ("sigma_r", C.c_double),
        ("layer_thickness", C.c_double * MAX_LAYERS),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class Event(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32), ("n_seeds", C.c_int32), ("n_tracks", C.c_int32), ("reserved", C.c_int32),
        ("n_hits", C.POINTER(C.c_int32)), ("hit_xyz", C.POINTER(C.POINTER(C.c_double))),
        ("seed_par", C.POINTER(C.c_double)), ("seed_cov", C.POINTER(C.c_double)),
        ("seed_hits", C.POINTER(C.c_int32)),
        ("track_par", C.POINTER(C.c_double)), ("track_cov", C.POINTER(C.c_double)),
        ("track_hits", C.POINTER(C.c_int32)),
    ]


class Tracks(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("reserved", C.c_int32),
        ("par", C.POINTER(C.c_double)), ("cov", C.POINTER(C.c_double)), ("hits", C.POINTER(C.c_int32)),
        ("n_hits", C.POINTER(C.c_int32)), ("n_holes", C.POINTER(C.c_int32)), ("chi2", C.POINTER(C.c_double)),
        ("ndof", C.POINTER(C.c_int32)), ("status", C.POINTER(C.c_int32)),
    ]


class Tuning(C.Structure):
    _fields_ = [("lanes_per_seed", C.c_int32), ("waves_per_block", C.c_int32), ("bins_phi", C.c_int32),
                ("bins_z", C.c_int32), ("persistent", C.c_int32), ("blocks_per_cu", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BuildStats(C.Structure):
    _fields_ = [("cand_layers", C.c_int64), ("chi2_evals", C.c_int64), ("accepted", C.c_int64),
                ("updates", C.c_int64), ("hits_scanned", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_P = C.POINTER
_ctx_p = C.c_void_p
_PROTOS = {
    "mkf_version": (C.c_char_p, []),
    "mkf_create": (C.c_int, [_P(Config), _P(Allocator), C.c_void_p, _P(C.c_void_p)]),
    "mkf_destroy": (None, [_ctx_p]),
    "mkf_last_error": (C.c_char_p, [_ctx_p]),
    "mkf_set_tuning": (C.c_int, [_ctx_p, _P(Tuning)]),
    "mkf_get_tuning": (C.c_int, [_ctx_p, _P(Tuning)]),
    "mkf_load_event": (C.c_int, [_ctx_p, _P(Event), _P(C.c_int32)]),
    "mkf_unload_event": (C.c_int, [_ctx_p, C.c_int32]),
    "mkf_load_events": (C.c_int, [_ctx_p, _P(Event), C.c_int32, _P(C.c_int32)]),
    "mkf_build": (C.c_int, [_ctx_p, C.c_int32, _P(Tracks)]),
    "mkf_build_batch": (C.c_int, [_ctx_p, _P(C.c_int32), C.c_int32, C.c_uint32, _P(Tracks)]),
    "mkf_build_batch_noalloc": (C.c_int, [_ctx_p, _P(C.c_int32), C.c_int32, C.c_uint32, _P(Tracks)]),
    "mkf_fetch_tracks": (C.c_int, [_ctx_p, C.c_int32, _P(Tracks)]),
    "mkf_fetch_fit": (C.c_int, [_ctx_p, C.c_int32, _P(Tracks)]),
    "mkf_fetch_beam": (C.c_int, [_ctx_p, C.c_int32, _P(Tracks)]),
    "mkf_ctx_broken": (C.c_int32, [_ctx_p]),
    "mkf_get_stats": (C.c_int, [_ctx_p, C.c_int32, _P(BuildStats)]),
    "mkf_fetch_index": (C.c_int, [_ctx_p, C.c_int32, C.c_int32, _P(C.c_int32), _P(C.c_int32), _P(C.c_int32)]),
    "mkf_index_grid": (C.c_int, [_ctx_p, C.c_int32, _P(C.c_int32), _P(C.c_int32)]),
    "mkf_fit": (C.c_int, [_ctx_p, C.c_int32, C.c_int32, _P(C.c_double), _P(C.c_double), _P(C.c_int32),
                          _P(Tracks)]),
    "mkf_fit_batch": (C.c_int, [_ctx_p, _P(C.c_int32), C.c_int32, _P(Tracks)]),
    "mkf_timer_read": (C.c_int, [_ctx_p, C.c_int32, _P(C.c_double), _P(C.c_int64)]),
    "mkf_timer_reset": (C.c_int, [_ctx_p]),
    "mkf_sync": (C.c_int, [_ctx_p]),
    "mkf_autotune": (C.c_int, [_ctx_p, _P(C.c_int32), C.c_int32, _P(Tuning)]),
    "mkf_serve_config": (C.c_int, [_ctx_p, C.c_uint64, C.c_int32, C.c_int32]),
    "mkf_serve_submit": (C.c_int, [_ctx_p, _P(Event), _P(Tracks), _P(C.c_uint64)]),
    "mkf_serve_poll": (C.c_int, [_ctx_p, C.c_uint64, _P(C.c_int32), _P(C.c_int32), _P(C.c_double)]),
    "mkf_serve_cancel": (C.c_int, [_ctx_p, C.c_uint64]),
    "mkf_serve_drain": (C.c_int, [_ctx_p]),
    "mkf_calib_copy": (C.c_int, [_ctx_p, C.c_void_p, C.c_void_p, C.c_size_t]),
    "mkf_calib_fma": (C.c_int, [_ctx_p, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                C.POINTER(C.c_double)]),
}

_lib = None


def header_functions() -> List[str]:
    """Names of the functions declared in include/mkf.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mkf_[a-z_0-9]+)\s*\(", text)))


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1702_06359_amd.build.build()")
        # One HIP runtime per process: PyTorch ships its own, and the streams
        # and device memory it hands to the library are only valid in that
        # runtime.  Loaded first, it also serves the library (same soname);
        # loaded after the library, a second runtime would come up beside it
        # and the two contend for the device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    """Message of this thread's last failed call (the library keeps one per thread)."""
    return lib().mkf_last_error(None).decode()


def check(status: int):
    if status != OK:
        raise MkfError(status, last_error())


def _dp(a):
    return a.ctypes.data_as(_P(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(_P(C.c_int32)) if a is not None else None


def config_from_geometry(geometry, *, max_cands=1, max_holes=1, chi2_cut=30.0, n_seed_layers=3,
                         hole_always=False, update3d=False) -> Config:
    c = Config()
    c.n_layers = geometry.n_layers
    c.n_seed_layers = n_seed_layers
    c.max_cands = max_cands
    c.max_holes = max_holes
    c.flags = (HOLE_ALWAYS if hole_always else 0) | (UPDATE_3D if update3d else 0)
    hz = geometry.half_z()
    for i in range(geometry.n_layers):
        c.layer_r[i] = geometry.radii[i]
        c.layer_half_z[i] = hz[i]
        c.layer_x0[i] = geometry.x0[i]
        if geometry.is_disk:
            c.layer_kind[i] = 1
            c.layer_z[i] = geometry.disk_z[i]
            c.layer_rmin[i] = geometry.disk_rmin
        c.layer_thickness[i] = geometry.thick(i)
    c.bz = geometry.bz
    c.sigma_rphi = geometry.sigma_rphi
    c.sigma_z = geometry.sigma_z
    c.sigma_r = geometry.sigma_r
    c.chi2_cut = chi2_cut
    c.mass = geometry.mass
    return c


class EventArrays:
    """Keeps the numpy arrays behind an mkf_event alive for one call."""

    def __init__(self, hits, seed_par=None, seed_cov=None, seed_hits=None, track_par=None, track_cov=None,
                 track_hits=None, n_seed_layers=3):
        self.hits = [np.ascontiguousarray(h, dtype=np.float64).reshape(-1, 3) for h in hits]
        nl = len(self.hits)
        self.counts = np.array([h.shape[0] for h in self.hits], dtype=np.int32)
        self.ptrs = (_P(C.c_double) * nl)(*[_dp(h) for h in self.hits])
        self.seed_par = None if seed_par is None else np.ascontiguousarray(seed_par, dtype=np.float64)
        self.seed_cov = None if seed_cov is None else np.ascontiguousarray(seed_cov, dtype=np.float64)
        self.seed_hits = None if seed_hits is None else np.ascontiguousarray(seed_hits, dtype=np.int32)
        self.track_par = None if track_par is None else np.ascontiguousarray(track_par, dtype=np.float64)
        self.track_cov = None if track_cov is None else np.ascontiguousarray(track_cov, dtype=np.float64)
        self.track_hits = None if track_hits is None else np.ascontiguousarray(track_hits, dtype=np.int32)
        e = Event()
        e.n_layers = nl
        e.n_seeds = 0 if self.seed_par is None else self.seed_par.shape[0]
        e.n_tracks = 0 if self.track_par is None else self.track_par.shape[0]
        e.n_hits = _ip(self.counts)
        e.hit_xyz = C.cast(self.ptrs, _P(_P(C.c_double)))
        e.seed_par, e.seed_cov, e.seed_hits = _dp(self.seed_par), _dp(self.seed_cov), _ip(self.seed_hits)
        e.track_par, e.track_cov, e.track_hits = _dp(self.track_par), _dp(self.track_cov), _ip(self.track_hits)
        self.event = e

    @classmethod
    def from_synth(cls, ev, with_seeds=True, with_tracks=False):
        return cls(ev.hits,
                   ev.seed_par if with_seeds else None, ev.seed_cov if with_seeds else None,
                   ev.seed_hits if with_seeds else None,
                   ev.prior_par if with_tracks else None, ev.prior_cov if with_tracks else None,
                   ev.truth_hit if with_tracks else None)


class TrackArrays:
    """Host output arrays plus the mkf_tracks that points at them."""

    def __init__(self, n: int, n_layers: int, empty=None):
        """empty(shape, dtype) makes each array (default: numpy zeros); a
        factory over page-locked memory lets a caller reuse pinned buffers."""
        mk = empty or (lambda shape, dtype: np.zeros(shape, dtype=dtype))
        self.n = n
        self.par = mk((n, 6), np.float64)
        self.cov = mk((n, 21), np.float64)
        self.hits = mk((n, n_layers), np.int32)
        self.n_hits = mk((n,), np.int32)
        self.n_holes = mk((n,), np.int32)
        self.chi2 = mk((n,), np.float64)
        self.ndof = mk((n,), np.int32)
        self.status = mk((n,), np.int32)
        for a in (self.par, self.cov, self.hits, self.n_hits, self.n_holes, self.chi2, self.ndof, self.status):
            if not a.flags.c_contiguous:
                raise ValueError("track arrays must be C-contiguous")
        t = Tracks()
        t.n = n
        t.par, t.cov, t.hits = _dp(self.par), _dp(self.cov), _ip(self.hits)
        t.n_hits, t.n_holes, t.chi2 = _ip(self.n_hits), _ip(self.n_holes), _dp(self.chi2)
        t.ndof, t.status = _ip(self.ndof), _ip(self.status)
        self.tracks = t

    def as_dict(self) -> Dict[str, np.ndarray]:
        return dict(par=self.par, cov=self.cov, hits=self.hits, n_hits=self.n_hits, n_holes=self.n_holes,
                    chi2=self.chi2, ndof=self.ndof, status=self.status)


def _torch_hooks():
    """Device memory and stream from PyTorch's caching allocator, when a GPU is visible."""
    try:
        import torch
    except ImportError:
        return None, None, None
    if not torch.cuda.is_available():
        return None, None, None
    device = torch.cuda.current_device()
    stream = torch.cuda.current_stream(device).cuda_stream

    def _alloc(nbytes, stream_ptr, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, int(stream_ptr or 0))
        except Exception:
            return None

    delete, finalizing = torch.cuda.caching_allocator_delete, sys.is_finalizing

    def _free(ptr, stream_ptr, user):
        # a context left open until the interpreter exits is destroyed after
        # torch's allocator may be gone; the process's memory goes with it
        if finalizing():
            return
        delete(int(ptr))

    keep = (ALLOC_FN(_alloc), FREE_FN(_free))
    a = Allocator()
    a.alloc, a.free = keep
    a.user = None
    return a, stream, keep


class Context:
    """One mkf context (C ABI: mkf_create ... mkf_destroy)."""

    def __init__(self, config: Config, use_torch: bool = True):
        L = lib()
        self.config = config
        self.n_layers = config.n_layers
        self._keep = None
        alloc, stream = None, None
        if use_torch:
            alloc, stream, self._keep = _torch_hooks()
        h = C.c_void_p()
        check(L.mkf_create(C.byref(config), C.byref(alloc) if alloc is not None else None,
                           C.c_void_p(stream) if stream else None, C.byref(h)))
        self._alloc = alloc
        self.h = h
        self._serving = {}

    # -- lifetime
    def close(self):
        if self.h:
            lib().mkf_destroy(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tuning
    def set_tuning(self, **kw):
        t = self.get_tuning()
        for k, v in kw.items():
            setattr(t, k, int(v))
        check(lib().mkf_set_tuning(self.h, C.byref(t)))
        return self.get_tuning()

    def get_tuning(self) -> Tuning:
        t = Tuning()
        check(lib().mkf_get_tuning(self.h, C.byref(t)))
        return t

    def autotune(self, handles: Sequence[int]) -> Tuning:
        arr = np.ascontiguousarray(handles, dtype=np.int32)
        t = Tuning()
        check(lib().mkf_autotune(self.h, _ip(arr), len(arr), C.byref(t)))
        return t

    # -- events
    def load_event(self, ev) -> int:
        ea = ev if isinstance(ev, EventArrays) else EventArrays.from_synth(ev, with_tracks=True)
        h = C.c_int32()
        check(lib().mkf_load_event(self.h, C.byref(ea.event), C.byref(h)))
        return int(h.value)

    def load_events(self, evs) -> List[int]:
        """mkf_load_events: several events in one pass; returns their handles."""
        eas = [e if isinstance(e, EventArrays) else EventArrays.from_synth(e, with_tracks=True) for e in evs]
        arr = (Event * len(eas))(*[ea.event for ea in eas])
        hs = np.zeros(len(eas), dtype=np.int32)
        check(lib().mkf_load_events(self.h, arr, len(eas), _ip(hs)))
        return [int(h) for h in hs]

    def unload_event(self, handle: int):
        check(lib().mkf_unload_event(self.h, int(handle)))

    # -- building
    def build(self, handle: int, n_seeds: int) -> Dict[str, np.ndarray]:
        out = TrackArrays(n_seeds, self.n_layers)
        check(lib().mkf_build(self.h, int(handle), C.byref(out.tracks)))
        return out.as_dict()

    def build_batch(self, handles: Sequence[int], n_seeds: Optional[Sequence[int]] = None, flags: int = 0,
                    outs: Optional[Sequence["TrackArrays"]] = None):
        """outs: caller-made TrackArrays to fill (their sizes give n_seeds)."""
        arr = np.ascontiguousarray(handles, dtype=np.int32)
        if n_seeds is None and outs is None:
            check(lib().mkf_build_batch(self.h, _ip(arr), len(arr), flags, None))
            return None
        if outs is None:
            outs = [TrackArrays(int(n), self.n_layers) for n in n_seeds]
        tarr = (Tracks * len(outs))(*[o.tracks for o in outs])
        check(lib().mkf_build_batch(self.h, _ip(arr), len(arr), flags, tarr))
        return [o.as_dict() for o in outs]

    def build_batch_noalloc(self, handles: Sequence[int], n_seeds: Optional[Sequence[int]] = None, flags: int = 0):
        """mkf_build_batch_noalloc: the batched build with no allocation in the call."""
        arr = np.ascontiguousarray(handles, dtype=np.int32)
        if n_seeds is None:
            check(lib().mkf_build_batch_noalloc(self.h, _ip(arr), len(arr), flags, None))
            return None
        outs = [TrackArrays(int(n), self.n_layers) for n in n_seeds]
        tarr = (Tracks * len(outs))(*[o.tracks for o in outs])
        check(lib().mkf_build_batch_noalloc(self.h, _ip(arr), len(arr), flags, tarr))
        return [o.as_dict() for o in outs]

    def fetch_tracks(self, handle: int, n_seeds: int):
        out = TrackArrays(n_seeds, self.n_layers)
        check(lib().mkf_fetch_tracks(self.h, int(handle), C.byref(out.tracks)))
        return out.as_dict()

    def fetch_fit(self, handle: int, n_seeds: int):
        """Final fit of the built tracks (after build_batch with BATCH_FIT)."""
        out = TrackArrays(n_seeds, self.n_layers)
        check(lib().mkf_fetch_fit(self.h, int(handle), C.byref(out.tracks)))
        return out.as_dict()

    def broken(self) -> bool:
        """True once a device fault made the GPU's context unusable."""
        return bool(lib().mkf_ctx_broken(self.h))

    def fetch_beam(self, handle: int, n_seeds: int):
        """Every rank of each seed's final beam (after build_batch with
        BATCH_BEAM): arrays of shape (n_seeds, max_cands, ...)."""
        k = int(self.config.max_cands)
        out = TrackArrays(n_seeds * k, self.n_layers)
        check(lib().mkf_fetch_beam(self.h, int(handle), C.byref(out.tracks)))
        return {name: v.reshape((n_seeds, k) + v.shape[1:]) for name, v in out.as_dict().items()}

    def index_grid(self, handle: int):
        """(bins_phi, bins_z) of the event's own index grid."""
        bp, bz = C.c_int32(), C.c_int32()
        check(lib().mkf_index_grid(self.h, int(handle), C.byref(bp), C.byref(bz)))
        return bp.value, bz.value

    def fetch_index(self, handle: int, layer: int, n_hits: int):
        """(bin_off, bin_of, order) of one layer's device hit index."""
        bp, bz = self.index_grid(handle)
        off = np.zeros(bp * bz + 1, dtype=np.int32)
        bin_of = np.zeros(n_hits, dtype=np.int32)
        order = np.zeros(n_hits, dtype=np.int32)
        check(lib().mkf_fetch_index(self.h, int(handle), int(layer), _ip(off), _ip(bin_of), _ip(order)))
        return off, bin_of, order

    def get_stats(self, handle: int) -> Dict[str, int]:
        s = BuildStats()
        check(lib().mkf_get_stats(self.h, int(handle), C.byref(s)))
        return s.as_dict()

    # -- fitting
    def fit(self, handle: int, init_par, init_cov, track_hits):
        par = np.ascontiguousarray(init_par, dtype=np.float64)
        cov = np.ascontiguousarray(init_cov, dtype=np.float64)
        th = np.ascontiguousarray(track_hits, dtype=np.int32)
        n = par.shape[0]
        out = TrackArrays(n, self.n_layers)
        check(lib().mkf_fit(self.h, int(handle), n, _dp(par), _dp(cov), _ip(th), C.byref(out.tracks)))
        return out.as_dict()

    def fit_batch(self, handles: Sequence[int], n_tracks: Optional[Sequence[int]] = None):
        arr = np.ascontiguousarray(handles, dtype=np.int32)
        if n_tracks is None:
            check(lib().mkf_fit_batch(self.h, _ip(arr), len(arr), None))
            return None
        outs = [TrackArrays(int(n), self.n_layers) for n in n_tracks]
        tarr = (Tracks * len(outs))(*[o.tracks for o in outs])
        check(lib().mkf_fit_batch(self.h, _ip(arr), len(arr), tarr))
        return [o.as_dict() for o in outs]

    # -- timing
    def timer_read(self, which: int):
        ms = C.c_double()
        n = C.c_int64()
        check(lib().mkf_timer_read(self.h, which, C.byref(ms), C.byref(n)))
        return ms.value, int(n.value)

    def timer_reset(self):
        check(lib().mkf_timer_reset(self.h))

    def sync(self):
        """Wait for all work queued on the context stream (asynchronous batches)."""
        check(lib().mkf_sync(self.h))

    # -- serving
    def serve_config(self, hbm_budget_bytes: int, max_in_flight: int, max_batch_events: int = 0):
        check(lib().mkf_serve_config(self.h, int(hbm_budget_bytes), int(max_in_flight), int(max_batch_events)))

    def serve_submit(self, ev, ea: Optional[EventArrays] = None, out: Optional[TrackArrays] = None):
        """Returns (ticket, TrackArrays), or (None, None) when no in-flight slot
        or budget is free (MKF_E_AGAIN: submit again later).  out: the arrays
        to fill (made here if None)."""
        ea = ea or (ev if isinstance(ev, EventArrays) else EventArrays.from_synth(ev))
        out = out or TrackArrays(int(ea.event.n_seeds), self.n_layers)
        t = C.c_uint64()
        st = lib().mkf_serve_submit(self.h, C.byref(ea.event), C.byref(out.tracks), C.byref(t))
        if st == E_AGAIN:
            return None, None
        check(st)
        self._serving[int(t.value)] = out
        return int(t.value), out

    def serve_poll(self, ticket: int):
        """Returns None while running, else (status, latency_s, outputs dict)."""
        done = C.c_int32()
        tst = C.c_int32()
        lat = C.c_double()
        check(lib().mkf_serve_poll(self.h, C.c_uint64(ticket), C.byref(done), C.byref(tst), C.byref(lat)))
        if not done.value:
            return None
        out = self._serving.pop(ticket)
        return int(tst.value), float(lat.value), out.as_dict()

    def serve_cancel(self, ticket: int):
        check(lib().mkf_serve_cancel(self.h, C.c_uint64(ticket)))
        self._serving.pop(ticket, None)

    def serve_drain(self):
        check(lib().mkf_serve_drain(self.h))

    def calib_copy(self, src_ptr: int, dst_ptr: int, nbytes: int):
        check(lib().mkf_calib_copy(self.h, C.c_void_p(src_ptr), C.c_void_p(dst_ptr), int(nbytes)))

    def calib_fma(self, dst_ptr: int, n_blocks: int, iters: int):
        """(device ms, FLOP) of the FP32 multiply-add throughput kernel."""
        ms, flop = C.c_double(), C.c_double()
        check(lib().mkf_calib_fma(self.h, C.c_void_p(dst_ptr), int(n_blocks), int(iters), C.byref(ms),
                                  C.byref(flop)))
        return ms.value, flop.value


def version() -> str:
    return lib().mkf_version().decode()
