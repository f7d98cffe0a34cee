"""Measures the FP32 error behind the build tolerances eps_cut and eps_rank.

Run on a GPU:  python tests/measure_build_tolerances.py [events] [seeds] [out.npz]

Builds 20,000-track events (10 % noise, six candidates per seed) truncated
to 4..10 layers, keeping every rank of each seed's final beam, and replays
every GPU path through the FP64 oracle.  A path's chi2 error minus that of
its prefix (the same path one layer shorter, which the GPU computes with the
identical FP32 operations) is the error of the last hit's chi2; consecutive
beam ranks of one seed give the error of a rank gap.  Prints the 99.99th
percentiles the tolerances are 4 x of (tests/tolerances.json)."""
import dataclasses, os, sys, time
import numpy as np
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import oracle
from paper_1702_06359_amd import abi, synth

n_ev = int(sys.argv[1]) if len(sys.argv) > 1 else 3
n_sample = int(sys.argv[2]) if len(sys.argv) > 2 else 2000
out_path = sys.argv[3] if len(sys.argv) > 3 else "chi2err.npz"
g = synth.Geometry()
rows_c2, rows_d, rows_tot, rows_dtot, rows_L = [], [], [], [], []
gaps_g, gaps_o = [], []
t0 = time.time()
for e in range(n_ev):
    ev = synth.make_event(20000, cfg=1, event=e, noise=0.10)
    rng = np.random.default_rng(100 + e)
    sel = np.sort(rng.choice(ev.n_seeds, n_sample, replace=False))
    paths = {}   # depth -> dict(path tuple -> (gpu_tot, orc_tot, orc_last_c2))
    for nl in range(4, 11):
        gt = dataclasses.replace(g, n_layers=nl, radii=tuple(g.radii[:nl]), x0=tuple(g.x0[:nl]))
        cfgo = oracle.config(gt, max_cands=6)
        hs = oracle.HitSet(ev.hits[:nl])
        with abi.Context(abi.config_from_geometry(gt, max_cands=6)) as ctx:
            h = ctx.load_event(abi.EventArrays(ev.hits[:nl], ev.seed_par, ev.seed_cov, ev.seed_hits))
            ctx.build_batch([h], [ev.n_seeds], flags=abi.BATCH_BEAM)
            beam = ctx.fetch_beam(h, ev.n_seeds)
            ctx.unload_event(h)
        d = {}
        for s in sel:
            prev = None
            for r in range(6):
                if beam["status"][s, r] < 0:
                    continue
                lh = beam["hits"][s, r]
                tot, per, ok = oracle.replay(cfgo, hs, ev.seed_par[s], ev.seed_cov[s], lh)
                d[(int(s),) + tuple(int(x) for x in lh)] = (float(beam["chi2"][s, r]), tot, float(per[nl - 1]))
                cur = (int(beam["n_hits"][s, r]), float(beam["chi2"][s, r]), tot)
                if prev is not None and prev[0] == cur[0]:
                    gaps_g.append((cur[1] - prev[1]) / (1 + prev[2]))
                    gaps_o.append((cur[2] - prev[2]) / (1 + prev[2]))
                prev = cur
        paths[nl] = d
        print(f"event {e} depth {nl}: {len(d)} paths, {time.time() - t0:.1f} s", flush=True)
    for nl in range(5, 11):
        for key, (gt_, ot, c2) in paths[nl].items():
            if key[nl] < 0:
                continue
            pre = key[:nl]
            if pre not in paths[nl - 1]:
                continue
            gp, op, _ = paths[nl - 1][pre]
            rows_c2.append(c2)
            rows_d.append((gt_ - ot) - (gp - op))
            rows_tot.append(ot)
            rows_dtot.append(gt_ - ot)
            rows_L.append(nl - 1)
os.makedirs(os.path.dirname(out_path) or ".", exist_ok=True)
np.savez(out_path, c2=np.array(rows_c2), dc2=np.array(rows_d), tot=np.array(rows_tot),
         dtot=np.array(rows_dtot), layer=np.array(rows_L), gap_gpu=np.array(gaps_g), gap_orc=np.array(gaps_o))
c2 = np.array(rows_c2); dc = np.abs(np.array(rows_d))
print("pairs", len(c2), "p99.99 |dc2|", np.quantile(dc, 0.9999), "max", dc.max(), flush=True)
for lo, hi in ((0, 1), (1, 5), (5, 15), (15, 30)):
    m = (c2 >= lo) & (c2 < hi)
    if m.any():
        print(f"chi2 in [{lo},{hi}): n={m.sum()} p99.99={np.quantile(dc[m], 0.9999):.3e} max={dc[m].max():.3e}", flush=True)
rel = np.abs(np.array(rows_dtot)) / (1 + np.array(rows_tot))
print("tot rel p99.99", np.quantile(rel, 0.9999), "max", rel.max(), flush=True)
ge = np.abs(np.array(gaps_g) - np.array(gaps_o))
print("rank gaps", len(ge), "p99.99 |gap err|", np.quantile(ge, 0.9999), "max", ge.max(), flush=True)
