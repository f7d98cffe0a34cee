"""The no-allocation batched builder (mkf_build_batch_noalloc) against
mkf_build_batch: bit-identical tracks on two calls in a row, the second with
a smaller batch (so the fixed descriptor array keeps stale entries beyond
it), asynchronous calls queued back to back, and the limits it rejects."""
import numpy as np
import pytest

from paper_1702_06359_amd import abi, synth

pytestmark = pytest.mark.gpu

FIELDS = ("par", "cov", "hits", "n_hits", "n_holes", "chi2", "status", "ndof")


def _equal(a, b):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k


def test_noalloc_build_equals_the_allocating_build(gpu_required):
    evs = [synth.make_event(n, cfg=240, event=i, noise=0.2) for i, n in enumerate((6000, 1500, 333, 2600))]
    small = synth.make_event(700, cfg=240, event=9, noise=0.2)
    c = abi.Context(abi.config_from_geometry(synth.Geometry(), max_cands=6))
    try:
        hs = [c.load_event(e) for e in evs]
        hsmall = c.load_event(small)
        counts = [e.n_seeds for e in evs]
        print("case noalloc: first call, 4 events", flush=True)
        ref = c.build_batch(hs, counts, flags=abi.BATCH_REINDEX)
        got = c.build_batch_noalloc(hs, counts, flags=abi.BATCH_REINDEX)
        for a, b in zip(ref, got):
            _equal(a, b)
        print("case noalloc: second call, 2 smaller events", flush=True)
        two = [hsmall, hs[2]]
        ref2 = c.build_batch(two, [small.n_seeds, evs[2].n_seeds])
        got2 = c.build_batch_noalloc(two, [small.n_seeds, evs[2].n_seeds])
        for a, b in zip(ref2, got2):
            _equal(a, b)
        print("case noalloc: asynchronous calls back to back, then fetch", flush=True)
        for _ in range(3):
            assert c.build_batch_noalloc(hs, None, flags=abi.BATCH_REINDEX | abi.BATCH_ASYNC) is None
        c.sync()
        for h, e, a in zip(hs, evs, ref):
            _equal(c.fetch_tracks(h, e.n_seeds), a)
        print("case noalloc: limits", flush=True)
        with pytest.raises(abi.MkfError) as err:
            c.build_batch_noalloc([hs[0]] * 257, None)
        assert err.value.status == abi.E_INVALID and "at most 256" in str(err.value)
        for bad in (abi.BATCH_BEAM, abi.BATCH_GRAPH):
            with pytest.raises(abi.MkfError) as err:
                c.build_batch_noalloc(hs[:1], counts[:1], flags=bad)
            assert err.value.status == abi.E_INVALID
        with pytest.raises(abi.MkfError) as err:
            c.build_batch_noalloc([hs[0], hs[0]], None)
        assert err.value.status == abi.E_INVALID
        # a grid change leaves the events without an index for it: refused
        # until an allocating build has made one, then equal again
        c.set_tuning(bins_phi=512, bins_z=16)
        with pytest.raises(abi.MkfError) as err:
            c.build_batch_noalloc(hs[:1], counts[:1])
        assert err.value.status == abi.E_STATE
        c.build_batch(hs, None, flags=abi.BATCH_REINDEX)
        got3 = c.build_batch_noalloc(hs, counts)
        for a, b in zip(ref, got3):
            _equal(a, b)
    finally:
        c.close()
