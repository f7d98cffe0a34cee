"""The device hit index, checked as integer work (Section 3.2.1: the
structures that select the hit candidates of a layer).

For every layer: the bin the device gave each hit equals the bin computed on
the host from the caller's FP64 coordinates, except for hits within a
rounding error of a bin edge (there either side is correct; such hits are
counted and must be rare); the bin offsets equal a host counting sort of the
device's bin ids, bit for bit; and each bin of the binned order holds
exactly the hits with that bin id (compared as sets: the order inside a bin
is free)."""
import math

import numpy as np
import pytest

from conftest import report
from paper_1702_06359_amd import abi, synth

pytestmark = pytest.mark.gpu


def host_bins(hits, L, geometry, bins_phi, bins_z):
    """Bin of each hit from its FP64 coordinates, and its distance to the
    nearest bin edge in units of a bin (in phi or in the second coordinate)."""
    x, y, z = hits[:, 0], hits[:, 1], hits[:, 2]
    phi = np.arctan2(y, x)
    fp = (phi + math.pi) * bins_phi / (2 * math.pi)
    if geometry.is_disk:
        g2, lo, ext = np.hypot(x, y), geometry.disk_rmin, geometry.radii[L] - geometry.disk_rmin
    else:
        hz = geometry.half_z()[L]
        g2, lo, ext = z, -hz, 2 * hz
    fz = (g2 - lo) * bins_z / ext
    ip = np.clip(np.floor(fp), 0, bins_phi - 1).astype(np.int64)
    iz = np.clip(np.floor(fz), 0, bins_z - 1).astype(np.int64)
    edge = np.minimum(np.abs(fp - np.round(fp)), np.where((fz > 0) & (fz < bins_z), np.abs(fz - np.round(fz)), 1.0))
    return (iz * bins_phi + ip).astype(np.int32), edge


# FP32 rounding of a hit's bin coordinate on the device, in bins: the azimuth
# carries the rounding of the packed (cos, sin) (< 1e-7 rad), the device's
# atan2 (3.8e-7 rad, pinned in test_atan_approximation.py), the sum with the
# FP32 pi (< 2.5e-7 rad, plus the 9e-8 rad by which FP32 pi differs from
# pi): under 1e-6 rad, taken as 1.5e-6, times bins_phi / 2 pi; the scaling
# by bins / extent and the product's own rounding add less than 3 x 2^-24
# of the bin count.
PHI_ERR_RAD = 1.5e-6


def edge_tolerance(bins_phi, bins_z):
    return PHI_ERR_RAD * bins_phi / (2 * math.pi) + 3 * 2.0 ** -24 * max(bins_phi, bins_z)


def check_layer(off, bin_of, order, ref_bins, edge, tol):
    n = len(bin_of)
    nb = len(off) - 1
    # offsets: exactly the counting sort of the device's bin ids
    want = np.zeros(nb + 1, dtype=np.int64)
    want[1:] = np.cumsum(np.bincount(bin_of, minlength=nb))
    assert np.array_equal(off, want)
    # every bin holds exactly its hits
    assert np.array_equal(np.sort(order), np.arange(n))
    in_bin = np.repeat(np.arange(nb), np.diff(off))
    assert np.array_equal(bin_of[order], in_bin)
    # device bins equal the host's FP64 bins away from the edges
    diff = bin_of != ref_bins
    assert (edge[diff] < tol).all(), (np.flatnonzero(diff)[:5], edge[diff][:5], tol)
    return int(diff.sum())


# Cases by the index form the launch takes: one event (bin ranges split over
# many blocks, 16-bit counters), batches of seven uneven and of sixty small
# events (one block per layer, binning included; small events on coarsened
# grids of their own), many events one of which keeps a grid too fine for one
# block's LDS (device-wide counting atomics), a layer of more than 65,535 hits
# (32-bit counters), a disk geometry, and a coarse ragged grid (not halved).
CASES = ["barrel_one_event", "barrel_batch", "many_events", "many_events_fine_grid", "big_layer", "endcap",
         "coarse"]


@pytest.mark.parametrize("case", CASES)
def test_index_is_the_counting_sort_of_the_bins(gpu_required, case):
    g = synth.Geometry.endcap() if case == "endcap" else synth.Geometry()
    if case == "barrel_batch":
        evs = [synth.make_event(n, cfg=230, event=i, noise=0.3) for i, n in enumerate((20000, 3000, 777, 9000,
                                                                                       40, 12000, 500))]
    elif case.startswith("many_events"):
        rng = np.random.default_rng(232)
        sizes = rng.integers(50, 1500, size=60)
        if case == "many_events_fine_grid":
            sizes[7] = 10000   # an event whose own grid stays the full, too fine one
        evs = [synth.make_event(int(n), cfg=232, event=i, noise=0.3) for i, n in enumerate(sizes)]
    elif case == "big_layer":
        evs = [synth.make_event(60000, cfg=233, event=0, noise=0.1)]
    else:
        evs = [synth.make_event(20000 if case != "endcap" else 10000, cfg=231, event=0, noise=0.1, geometry=g)]
    tuning = {"coarse": dict(bins_phi=97, bins_z=13),
              "many_events_fine_grid": dict(bins_phi=1024, bins_z=128)}.get(case, {})
    c = abi.Context(abi.config_from_geometry(g, max_cands=6))
    try:
        if tuning:
            c.set_tuning(**tuning)
        hs = [c.load_event(e) for e in evs]
        if len(evs) > 1:
            print(f"case index {case}: batch re-index of {len(evs)} events", flush=True)
            c.build_batch(hs, None, flags=abi.BATCH_REINDEX)
        t = c.get_tuning()
        n_edge = n_hits = 0
        for e, h in zip(evs, hs):
            bp, bz = c.index_grid(h)
            # the event's grid: the context's, halved on both axes while the
            # fullest layer keeps three bins per hit
            k = 0
            while (t.bins_phi % (2 << k) == 0 and t.bins_z % (2 << k) == 0 and t.bins_phi >> (k + 1) >= 64
                   and t.bins_z >> (k + 1) >= 2
                   and (t.bins_phi >> (k + 1)) * (t.bins_z >> (k + 1)) >= 3 * max(len(x) for x in e.hits)):
                k += 1
            assert (bp, bz) == (t.bins_phi >> k, t.bins_z >> k)
            for L in range(g.n_layers):
                print(f"case index {case}: layer {L}", flush=True)
                off, bin_of, order = c.fetch_index(h, L, len(e.hits[L]))
                ref, edge = host_bins(e.hits[L], L, g, bp, bz)
                n_edge += check_layer(off, bin_of, order, ref, edge, edge_tolerance(bp, bz))
                n_hits += len(bin_of)
    finally:
        c.close()
    report(f"index_{case}", dict(hits=n_hits, edge_differences=n_edge))
    assert n_edge <= 1e-4 * n_hits + 2
