"""Benchmark of the MI355X Kalman-filter track builder.

Default (the headline): combinatorial KF building of 10 events x 20,000
tracks (10 % noise hits, up to 6 candidates per seed, chi2 cut 30, one hole),
all events in one batched launch per step, inputs resident on the device.
A step = hit-index build for every event + the batched build.  Prints one
JSON line with throughput, the roofline of the build kernel, the CPU oracle
baseline and serving latencies.

Other workloads (--workload): endcap (10 events x 10,000 tracks on ten
disks), two_step (the headline on 6 mm deep barrel layers), fit (1,000,000 tracks in 64 uneven batches), batched (256 uneven
events, batched vs plain builder), serve (Poisson arrivals, p50/p99 latency).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 operation counts per unit of work, counted from the kernel
# source (fma = 2; add, sub, mul, rcp, sqrt, rsq, sin, cos, log, atan = 1;
# compares, selects and integer work not counted).
FLOP_SCATTER = 40             # Highland angle and the 4 noise terms
FLOP_PROPAGATE = 136          # path root, helix step and the Jacobian's factors P, v, d
FLOP_TRANSPORT = 212          # F C F^T with F = P + v d^T (cylinders)
FLOP_WINDOW = 37              # search window and bin range
FLOP_PER_CAND_LAYER = FLOP_SCATTER + FLOP_PROPAGATE + FLOP_TRANSPORT + FLOP_WINDOW   # 425
FLOP_PER_CHI2 = 39            # window tests, tangent-plane residual, 2x2 innovation, chi2
FLOP_PER_UPDATE = 187         # gain, state and covariance update
FLOP_PER_UPDATE_JOSEPH = 445  # fit update in Joseph form (the first JOSEPH_UPDATES of a fit)
JOSEPH_UPDATES = 3
FLOP_PER_FIT_STEP = FLOP_SCATTER + FLOP_PROPAGATE + FLOP_TRANSPORT   # 388, layers 1..9 of a fit
BYTES_PER_FIT_TRACK = 108 + 40 + 10 * 16 + 232   # prior (f32), hit ids, hits (float4), fit result (f64)
BYTES_PER_SEED_IO = 120 + 276     # seed in (f32 state, cov, hit ids) + track out (f64)
BYTES_PER_HIT = 16                # binned hit read once
BYTES_PER_BIN = 4                 # bin offset read once
PEAK_FP32_VALU_TFLOPS = 157.3     # MI355X vector FP32 (256 CU x 2.4 GHz x 256 FLOP/clk)
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ("paper_1702_06359_amd/csrc/mkf_kernels.hip", "paper_1702_06359_amd/csrc/mkf_device.hpp",
                  "paper_1702_06359_amd/csrc/mkf_internal.hpp")


def fma_ceiling(ctx, n_blocks=2048, iters=4096, reps=5):
    """Measured FP32 multiply-add throughput of the vector ALUs (no packed
    instructions, like the library's kernels): best of `reps` launches of the
    library's calibration kernel, untimed by the benchmark step."""
    import torch
    out = torch.empty(n_blocks * 256, dtype=torch.float32, device="cuda")
    ctx.calib_fma(out.data_ptr(), n_blocks, iters)
    best = min(ctx.calib_fma(out.data_ptr(), n_blocks, iters)[0] for _ in range(reps))
    flop = 2.0 * 8 * iters * 256 * n_blocks
    tf = flop / (best * 1e-3) / 1e12
    return {"tflops": round(tf, 2), "frac_of_peak": round(tf / PEAK_FP32_VALU_TFLOPS, 4),
            "frac_of_nonpacked_peak": round(tf / (PEAK_FP32_VALU_TFLOPS / 2), 4)}


def measured_traffic(kernel):
    """Calibrated bytes per launch of `kernel` (read + written) from the
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs summarised in profiles/traffic.json,
    or None when the kernel sources changed since those runs."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["source_sha256"]:
            return None
        return int(round(rec["kernels"][kernel]["bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_count_guard(n):
    if n != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "detail": "events would shard across GPUs with no exchange between them; "
                                    "no multi-GPU launcher is provided"}))
        sys.exit(2)


def make_ctx(k, tuning=None, geometry=None):
    from paper_1702_06359_amd import abi, synth
    ctx = abi.Context(abi.config_from_geometry(geometry or synth.Geometry(), max_cands=k))
    if tuning:
        ctx.set_tuning(**tuning)
    return ctx


PRIME_S = 0.15


def prime(fn, sync, seconds=PRIME_S):
    """Run the step until `seconds` of wall time have passed: after a load or
    an idle gap the GPU's clocks ramp up over the first ~40 launches (20 ms of
    work), each launch a little faster than the last (measured on MI355X: the
    build kernel takes 0.40 ms, then settles at 0.365 ms), so a few warm-up
    steps leave the timed steps on the ramp.  Untimed; returns the steps run."""
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            fn()
        sync()
        n += 8
    return n


def time_steps(fn, steps, warmup, sync, primed=False):
    if not primed:
        prime(fn, sync)
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return time.perf_counter() - t0


def cpu_baseline_build(ev, k, target_cpu_s=15.0):
    """The FP64 oracle on a bounded sample of seeds of one event."""
    import oracle
    cfg = oracle.config(ev.geometry, max_cands=k)
    threads = max(1, min(16, os.cpu_count() or 1))
    hs = oracle.HitSet(ev.hits)
    probe = np.arange(min(64, ev.n_seeds), dtype=np.int32)
    t0 = time.perf_counter()
    oracle.build_tracks(cfg, hs, ev.seed_par, ev.seed_cov, ev.seed_hits, seed_ids=probe, n_threads=1)
    per_seed = (time.perf_counter() - t0) / len(probe)
    n = int(min(ev.n_seeds, max(threads, target_cpu_s / max(per_seed, 1e-6))))
    rows = np.arange(n, dtype=np.int32)
    t0 = time.perf_counter()
    oracle.build_tracks(cfg, hs, ev.seed_par, ev.seed_cov, ev.seed_hits, seed_ids=rows, n_threads=threads)
    wall = time.perf_counter() - t0
    return {"value": n / wall, "unit": "tracks/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "single_thread_value": 1.0 / per_seed,
            "sample": f"{n} seeds of one 20,000-track event (FP64 oracle, brute-force hit search), "
                      f"{wall:.1f} s wall on {threads} threads; single-thread rate from the first "
                      f"{len(probe)} seeds"}


def _poisson_arrivals(n, rate_hz, seed):
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n)
    return np.cumsum(gaps) - gaps[0], rng.integers(0, 1 << 30, n)


def serve_run(ctx, arrays, sizes, arrivals, picks):
    """Serve events arriving at `arrivals` (seconds from the start; picks[i]
    indexes `arrays`).  One thread submits each event at its arrival time
    (again and again while the server answers MKF_E_AGAIN: no slot or budget
    free); another polls.  Latency of an event = the wait from its scheduled
    arrival to its accepted submit plus the library's own submit-to-completion
    time.  Returns (latencies in s, wall time from the first arrival to the
    last completion)."""
    import threading
    from paper_1702_06359_amd import abi
    n = len(arrivals)
    pending = {}
    lat = np.zeros(n)
    lock = threading.Lock()
    done_all = threading.Event()
    t_last = [0.0]

    def poller():
        left = n
        while left:
            with lock:
                items = list(pending.items())
            for t, (i, waited) in items:
                r = ctx.serve_poll(t)
                if r is None:
                    continue
                assert r[0] == abi.OK, r[0]
                lat[i] = waited + r[1]
                t_last[0] = time.perf_counter()
                with lock:
                    del pending[t]
                left -= 1
            time.sleep(0.0001)
        done_all.set()

    th = threading.Thread(target=poller)
    th.start()
    t0 = time.perf_counter()
    for i in range(n):
        while time.perf_counter() - t0 < arrivals[i]:
            pass
        ea = arrays[picks[i]]
        out = abi.TrackArrays(int(ea.event.n_seeds), len(ea.hits))
        while True:
            t_call = time.perf_counter()
            t, _ = ctx.serve_submit(None, ea=ea, out=out)
            if t is not None:
                break
        with lock:
            pending[t] = (i, t_call - t0 - arrivals[i])
    done_all.wait()
    th.join()
    return lat, t_last[0] - t0


def plain_run(ctx, arrays, n_seeds, arrivals, picks, max_events):
    """The plain per-event builder on the same arrivals, one event at a time
    (load: copy and index; build; tracks to the host; unload).  Latency from
    the scheduled arrival to the event's tracks on the host."""
    from paper_1702_06359_amd import abi
    n = min(len(arrivals), max_events)
    lat = np.zeros(n)
    t0 = time.perf_counter()
    for i in range(n):
        while time.perf_counter() - t0 < arrivals[i]:
            pass
        h = ctx.load_event(arrays[picks[i]])
        ctx.build(h, n_seeds[picks[i]])
        ctx.unload_event(h)
        lat[i] = time.perf_counter() - t0 - arrivals[i]
    return lat, time.perf_counter() - t0


def serving_leg(args, n_events=2048, n_plain=384, budget=16 << 30):
    """Served building (Poisson arrivals, tracks log-uniform in [500, 50,000],
    30 % noise, k = 6) against the plain per-event builder on the same
    arrivals, at 0.5 and 0.8 of the served saturated rate."""
    from paper_1702_06359_amd import abi, synth
    n_pool = 32
    sizes = synth.loguniform_sizes(n_pool, 500, 50000, cfg=4)
    log(f"serving: generating a pool of {n_pool} events")
    pool = [synth.make_event(int(n), cfg=4, event=i, noise=0.3) for i, n in enumerate(sizes)]
    arrays = [abi.EventArrays.from_synth(e) for e in pool]
    n_seeds = [e.n_seeds for e in pool]
    ctx = make_ctx(6, args.tuning)
    ctx.serve_config(budget, max_in_flight=64)
    # saturated: every event arrives at once, the server admits as slots and
    # budget free up
    arr0, pick0 = _poisson_arrivals(256, 1e12, seed=3)
    serve_run(ctx, arrays, sizes, np.zeros(64), pick0[:64] % n_pool)                 # warm-up
    n_sat = 1024
    arr_s, pick_s = _poisson_arrivals(n_sat, 1e12, seed=4)
    _, wall = serve_run(ctx, arrays, sizes, np.zeros(n_sat), pick_s % n_pool)
    sat = n_sat / wall
    mean_tracks = float(np.mean(sizes[pick_s % n_pool]))
    out = {"workload": "served building, Poisson arrivals, tracks log-uniform in [500, 50000] (pool of 32 events), "
                       "30% noise, k=6, 16 GiB budget, 64 events in flight",
           "saturated_events_per_s": round(sat, 1), "saturated_tracks_per_s": round(sat * mean_tracks, 1),
           "hbm_budget_bytes": budget, "rates": []}
    for frac in (0.5, 0.8):
        rate = frac * sat
        arr, pick = _poisson_arrivals(n_events, rate, seed=int(frac * 10))
        pick = pick % n_pool
        log(f"serving: {n_events} events at {rate:.0f} events/s")
        lat, wall = serve_run(ctx, arrays, sizes, arr, pick)
        tracks = float(sizes[pick].sum())
        log(f"plain builder: first {n_plain} of the same arrivals")
        plat, pwall = plain_run(ctx, arrays, n_seeds, arr, pick, n_plain)
        ptracks = float(sizes[pick[:n_plain]].sum())
        out["rates"].append({
            "load": frac, "rate_events_per_s": round(rate, 1), "events": n_events,
            "events_per_s": round(n_events / wall, 1), "tracks_per_s": round(tracks / wall, 1),
            "latency_p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "latency_p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "plain": {"events": n_plain, "events_per_s": round(n_plain / pwall, 1),
                      "tracks_per_s": round(ptracks / pwall, 1),
                      "latency_p50_ms": round(float(np.percentile(plat, 50)) * 1e3, 3),
                      "latency_p99_ms": round(float(np.percentile(plat, 99)) * 1e3, 3)}})
    ctx.close()
    return out


def batched_leg(args, steps=10):
    """256 uneven events (tracks log-uniform in [500, 20,000], noise
    U[0.1, 0.5] per event and layer), indexed and built in one batched launch
    per step with the launch shapes mkf_autotune picks on them, against the
    plain per-event builder on the same resident events."""
    import torch
    from paper_1702_06359_amd import abi, synth
    log("batched: generating 256 uneven events")
    evs = synth.batched_events(256, 500, 20000)
    ctx = make_ctx(6, args.tuning)
    handles = [ctx.load_event(e) for e in evs]
    log("batched: autotune")
    tuned = ctx.autotune(handles).as_dict()

    def sync():
        ctx.sync()
        torch.cuda.synchronize()
    tracks = int(sum(e.n_seeds for e in evs))
    step = lambda: ctx.build_batch(handles, None, flags=abi.BATCH_REINDEX | abi.BATCH_ASYNC)
    prime(step, sync)
    ctx.timer_reset()
    t_batch = time_steps(step, steps, 0, sync, primed=True)
    build_ms, build_n = ctx.timer_read(abi.TIMER_BUILD)
    index_ms, index_n = ctx.timer_read(abi.TIMER_INDEX)
    n_plain = max(1, steps // 5)
    t_plain = time_steps(lambda: [lib_build_plain(ctx, h) for h in handles], n_plain, 1, sync)
    ctx.close()
    rate = tracks * steps / t_batch
    prate = tracks * n_plain / t_plain
    return {"workload": "256 events, tracks log-uniform in [500, 20000], noise U[0.1,0.5] per event and layer, "
                        "k=6, index + one batched build per step",
            "tracks": tracks, "tuning": tuned, "tracks_per_s": round(rate, 1),
            "ms_per_step": round(t_batch / steps * 1e3, 4),
            "build_kernel_ms": round(build_ms / max(build_n, 1), 4),
            "index_ms": round(index_ms / max(index_n, 1), 4),
            "plain_builder_tracks_per_s": round(prate, 1), "speedup_vs_plain": round(rate / prate, 3)}


def workload_ckf(args):
    import torch
    from paper_1702_06359_amd import abi, synth
    n_events, n_tracks, noise, k = 10, 20000, 0.10, 6
    log(f"generating {n_events} events x {n_tracks} tracks")
    evs = synth.ckf_events(n_events, n_tracks, noise)
    ctx = make_ctx(k, args.tuning)
    handles = [ctx.load_event(e) for e in evs]
    if args.tune:
        t = ctx.autotune(handles)
        log("autotuned:", t.as_dict())
    tuning = ctx.get_tuning().as_dict()

    def step():
        # queued without waiting: the steps run back to back on the device
        ctx.build_batch(handles, None, flags=abi.BATCH_REINDEX | abi.BATCH_ASYNC)

    def sync():
        ctx.sync()
        torch.cuda.synchronize()
    log("priming, warmup + timed steps")
    n_prime = prime(step, sync)
    for _ in range(args.warmup):
        step()
    sync()
    ctx.timer_reset()
    elapsed = time_steps(step, args.steps, 0, sync, primed=True)
    build_ms, build_n = ctx.timer_read(abi.TIMER_BUILD)
    index_ms, index_n = ctx.timer_read(abi.TIMER_INDEX)
    tracks = n_events * n_tracks
    value = tracks * args.steps / elapsed
    # work counters of one launch (separate, untimed)
    ctx.build_batch(handles, None, flags=abi.BATCH_REINDEX | abi.BATCH_STATS)
    st = {k2: 0 for k2 in ("cand_layers", "chi2_evals", "accepted", "updates", "hits_scanned")}
    for h in handles:
        for k2, v in ctx.get_stats(h).items():
            st[k2] += v
    flops = (st["cand_layers"] * FLOP_PER_CAND_LAYER + st["chi2_evals"] * FLOP_PER_CHI2 +
             st["updates"] * FLOP_PER_UPDATE)
    avg_ms = build_ms / max(build_n, 1)
    achieved = flops / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VALU_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 5),
                "traffic": measured_traffic("k_build_batch<6,false,0>") if tuning["lanes_per_seed"] == 6 else None,
                "kernel": "k_build_batch", "kernel_avg_ms": round(avg_ms, 4),
                "flop_per_launch": int(flops), "counters": st,
                "fma_ceiling": fma_ceiling(ctx)}
    # the same steps with the final fit of every built track chained on the device
    def step_fit():
        ctx.build_batch(handles, None, flags=abi.BATCH_REINDEX | abi.BATCH_ASYNC | abi.BATCH_FIT)

    prime(step_fit, sync)
    ctx.timer_reset()
    fit_steps = max(1, args.steps // 2)
    fit_elapsed = time_steps(step_fit, fit_steps, 0, sync, primed=True)
    refit_ms, refit_n = ctx.timer_read(abi.TIMER_FIT)
    fit_vs_build = fitted_vs_built(ctx, evs[0], handles[0])
    plain_rate = None
    if not args.quick:
        # the plain per-event builder (one launch per layer) on the same events
        n_plain = max(1, args.steps // 5)
        plain_s = time_steps(lambda: [lib_build_plain(ctx, h) for h in handles], n_plain, 1, sync)
        plain_rate = tracks * n_plain / plain_s
    result = {
        "metric": "tracks built/sec (20k-track events, combinatorial KF) and p50/p99 event latency",
        "value": round(value, 1), "unit": "tracks/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "combinatorial KF building, 10 events x 20,000 tracks, 10% noise hits, "
                               "k=6 candidates/seed, chi2<30, 1 hole, 10-layer barrel, 3.8 T",
                   "events": n_events, "tracks_per_event": n_tracks, "noise": noise, "max_cands": k,
                   "step": "hit index + batched build of all events, steps queued back to back", "tuning": tuning,
                   "priming": f"{n_prime} untimed steps ({PRIME_S} s) before the warmup, so that the timed steps run "
                              "at the GPU's sustained clock"},
        "roofline": roofline,
        "index_build_ms_per_step": round(index_ms / max(index_n, 1), 4),
        "build_and_fit": {"tracks_per_s": round(tracks * fit_steps / fit_elapsed, 1),
                          "ms_per_step": round(fit_elapsed / fit_steps * 1e3, 4),
                          "final_fit_kernel_ms": round(refit_ms / max(refit_n, 1), 4),
                          "fitted_vs_built": fit_vs_build},
        "plain_builder_tracks_per_s": None if plain_rate is None else round(plain_rate, 1),
    }
    if not args.quick:
        log("two batch slots in flight")
        result["two_slots"] = two_slots_leg(args, ctx, handles, evs, sync)
        log("host-inclusive step")
        result["host_inclusive"] = host_inclusive(ctx, evs)
        log("endcap workload")
        result["endcap"] = endcap_leg(args)
        log("two-step workload")
        result["two_step"] = two_step_leg(args)
        log("fit workload")
        fit = workload_fit(argparse.Namespace(steps=5, warmup=1, no_cpu_baseline=True))
        result["fit"] = {"workload": fit["config"]["workload"], "tracks_per_s": fit["value"],
                         "ms_per_step": fit["ms_per_step"], "kernel_avg_ms": fit["roofline"]["kernel_avg_ms"],
                         "frac_of_fp32_peak": fit["roofline"]["frac"], "hbm_frac": fit["roofline"]["hbm_frac"]}
        log("best-hit latency")
        result["best_hit"] = best_hit_latency()
        log("batched workload")
        result["batched"] = batched_leg(args)
        log("serving workload")
        result["serving"] = serving_leg(args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline_build(evs[0], k, args.cpu_seconds)
    ctx.close()
    return result


def best_hit_latency(reps=10):
    """1 event x 1,000 tracks, no noise, one candidate per seed, plain
    per-layer builder: median latency with the event resident on the device,
    and end to end (load + index + build + copy of the tracks to the host)."""
    from paper_1702_06359_amd import synth
    ev = synth.best_hit_event(1000)
    ctx = make_ctx(1)
    h = ctx.load_event(ev)
    lib_build_plain(ctx, h)
    dev = []
    for _ in range(reps):
        t0 = time.perf_counter()
        lib_build_plain(ctx, h)
        dev.append(time.perf_counter() - t0)
    ctx.unload_event(h)
    e2e = []
    for _ in range(reps):
        t0 = time.perf_counter()
        h = ctx.load_event(ev)
        ctx.build(h, ev.n_seeds)
        e2e.append(time.perf_counter() - t0)
        ctx.unload_event(h)
    ctx.close()
    return {"workload": "best-hit building, 1 event x 1,000 tracks, no noise, k=1, plain builder",
            "device_resident_ms_p50": round(float(np.median(dev)) * 1e3, 4),
            "end_to_end_ms_p50": round(float(np.median(e2e)) * 1e3, 4)}


def fitted_vs_built(ctx, ev, h):
    """Final fit against the build's own state on one event (after a build
    with the final fit chained): on tracks whose every hit is the true one and
    that reached the last layer, the RMS pulls of q/pT, phi and theta against
    the true state there, for the built and the fitted parameters, and the
    RMS of their difference over the built sigma."""
    built, fitted = ctx.fetch_tracks(h, ev.n_seeds), ctx.fetch_fit(h, ev.n_seeds)

    def wrap(d, i):   # azimuth differences into (-pi, pi]
        return np.remainder(d + np.pi, 2 * np.pi) - np.pi if i == 4 else d
    good = (built["hits"] == ev.truth_hit).all(1) & (built["status"] == 0) & (fitted["status"] == 0)
    last = ev.truth_par.shape[1] - 1
    out = {"tracks": int(good.sum()), "of": int(ev.n_seeds)}
    for name, d in (("built", built), ("fitted", fitted)):
        out[name + "_pull_rms"] = {}
        for i, k in ((3, "q/pT"), (4, "phi"), (5, "theta")):
            sig = np.sqrt(d["cov"][good, 6 * i - i * (i - 1) // 2])
            pull = wrap(d["par"][good, i] - ev.truth_par[good, last, i], i) / sig
            out[name + "_pull_rms"][k] = round(float(np.sqrt(np.mean(pull ** 2))), 3)
    out["diff_over_built_sigma_rms"] = {}
    for i, k in ((3, "q/pT"), (4, "phi"), (5, "theta")):
        sig = np.sqrt(built["cov"][good, 6 * i - i * (i - 1) // 2])
        dd = wrap(fitted["par"][good, i] - built["par"][good, i], i) / sig
        out["diff_over_built_sigma_rms"][k] = round(float(np.sqrt(np.mean(dd ** 2))), 4)
    return out


def two_slots_leg(args, ctx, handles, evs, sync, steps=200):
    """The headline step with two batches in flight: a second context on a
    stream of its own holds another copy of the ten events, and the steps
    alternate between the two, so that one batch's index and build overlap
    the other's (as a serving pipeline runs consecutive batches).  Reported
    beside `value`, which keeps one stream."""
    import torch
    from paper_1702_06359_amd import abi
    s2 = torch.cuda.Stream()
    with torch.cuda.stream(s2):
        ctx2 = make_ctx(6, args.tuning)
        handles2 = [ctx2.load_event(e) for e in evs]
    flags = abi.BATCH_REINDEX | abi.BATCH_ASYNC
    slots = [(ctx, handles), (ctx2, handles2)]
    k = [0]

    def step():
        c, h = slots[k[0] & 1]
        k[0] += 1
        c.build_batch(h, None, flags=flags)

    def sync2():
        ctx2.sync()
        sync()
    elapsed = time_steps(step, steps, 0, sync2)
    ctx2.close()
    tracks = sum(e.n_seeds for e in evs)
    return {"step": "index + batched build of ten events, two batches (two contexts, two streams) in flight",
            "tracks_per_s": round(tracks * steps / elapsed, 1), "ms_per_step": round(elapsed / steps * 1e3, 4)}


def host_inclusive(ctx, evs, reps=3):
    """The headline workload from host buffers to host buffers: load the
    events in one call (their FP64 hits and seeds checked and narrowed to
    FP32 on host threads, one copy per event, every hit index), one batched
    build, copy of every track to the host, unload.  Median wall time of
    `reps` steps after one warm-up step, with the caller's buffers in
    ordinary (pageable) numpy arrays made per step, and in page-locked
    buffers made once and reused (as a serving caller would)."""
    import torch
    from paper_1702_06359_amd import abi
    counts = [e.n_seeds for e in evs]

    def pinned(shape, dtype):
        return torch.empty(shape, dtype=torch.from_numpy(np.empty(0, dtype)).dtype, pin_memory=True).numpy()

    def pin_copy(a):
        out = pinned(a.shape, a.dtype)
        out[...] = a
        return out

    def run(arrays, outs):
        times = []
        for _ in range(reps + 1):
            t0 = time.perf_counter()
            hs = ctx.load_events(arrays)
            if outs is None:
                ctx.build_batch(hs, counts)
            else:
                ctx.build_batch(hs, outs=outs)
            for h in hs:
                ctx.unload_event(h)
            times.append(time.perf_counter() - t0)
        return float(np.median(times[1:]))

    t_page = run([abi.EventArrays.from_synth(e) for e in evs], None)
    pin_in = [abi.EventArrays([pin_copy(np.ascontiguousarray(h, dtype=np.float64)) for h in e.hits],
                              pin_copy(e.seed_par), pin_copy(e.seed_cov), pin_copy(e.seed_hits)) for e in evs]
    pin_out = [abi.TrackArrays(n, len(evs[0].hits), empty=pinned) for n in counts]
    t_pin = run(pin_in, pin_out)
    return {"step": "load of all events (FP64 hits and seeds narrowed to FP32 on the host, copies, index) + "
                    "batched build + tracks to host + unload",
            "tracks_per_s": round(sum(counts) / t_page, 1), "ms_per_step": round(t_page * 1e3, 3),
            "pinned_reused_buffers": {"tracks_per_s": round(sum(counts) / t_pin, 1),
                                      "ms_per_step": round(t_pin * 1e3, 3)}}


def geometry_leg(args, evs, geometry, workload, steps=None):
    """The headline step (index + batched build, k = 6) on other events."""
    import torch
    from paper_1702_06359_amd import abi
    ctx = make_ctx(6, args.tuning, geometry=geometry)
    handles = [ctx.load_event(e) for e in evs]

    def step():
        ctx.build_batch(handles, None, flags=abi.BATCH_REINDEX | abi.BATCH_ASYNC)

    def sync():
        ctx.sync()
        torch.cuda.synchronize()
    n = steps or args.steps
    prime(step, sync)
    ctx.timer_reset()
    elapsed = time_steps(step, n, 0, sync, primed=True)
    build_ms, build_n = ctx.timer_read(abi.TIMER_BUILD)
    ctx.close()
    tracks = sum(e.n_seeds for e in evs)
    return {"workload": workload, "tracks_per_s": round(tracks * n / elapsed, 1),
            "ms_per_step": round(elapsed / n * 1e3, 4), "build_kernel_ms": round(build_ms / max(build_n, 1), 4)}


def endcap_leg(args, steps=None):
    """10 events x 10,000 tracks on ten disks (1.6 < eta < 2.6), 10 % noise."""
    from paper_1702_06359_amd import synth
    return geometry_leg(args, synth.endcap_events(10, 10000, 0.10), synth.Geometry.endcap(),
                        "combinatorial KF building, 10 events x 10,000 tracks, 10-disk endcap "
                        "(z = 30..120 cm, 1.6 < eta < 2.6), 10% noise hits, k=6, chi2<30, 1 hole", steps)


def two_step_leg(args, steps=None):
    """The headline events' recipe on a barrel whose layers are 6 mm deep:
    two-step propagation, every window hit carried to its own radius."""
    from paper_1702_06359_amd import synth
    g = synth.Geometry(thickness=tuple(0.6 for _ in range(10)))
    evs = [synth.make_event(20000, cfg=5, event=e, noise=0.10, geometry=g) for e in range(10)]
    return geometry_leg(args, evs, g, "combinatorial KF building, 10 events x 20,000 tracks, 10-layer barrel "
                        "of 6 mm deep layers (two-step propagation), 10% noise hits, k=6, chi2<30, 1 hole", steps)


def workload_endcap(args):
    r = endcap_leg(args) if args.workload == "endcap" else two_step_leg(args)
    return {"metric": f"tracks built/sec ({args.workload}, combinatorial KF)", "value": r["tracks_per_s"],
            "unit": "tracks/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic", "config": {"workload": r["workload"]},
            "build_kernel_ms": r["build_kernel_ms"]}


def workload_fit(args):
    """KF fit of 1,000,000 tracks with known hits in 64 uneven batches, one launch."""
    import torch
    from paper_1702_06359_amd import abi, synth
    sizes = synth.fit_batch_sizes(64, 1_000_000, 2000, 30000)
    log("generating 64 fit batches")
    evs = [synth.make_event(int(n), cfg=2, event=i, noise=0.0) for i, n in enumerate(sizes)]
    ctx = make_ctx(6)
    handles = [ctx.load_event(abi.EventArrays.from_synth(e, with_seeds=False, with_tracks=True)) for e in evs]
    sync = torch.cuda.synchronize
    prime(lambda: ctx.fit_batch(handles), sync)
    for _ in range(args.warmup):
        ctx.fit_batch(handles)
    sync()
    ctx.timer_reset()
    elapsed = time_steps(lambda: ctx.fit_batch(handles), args.steps, 0, sync, primed=True)
    fit_ms, fit_n = ctx.timer_read(abi.TIMER_FIT)
    n = int(sizes.sum())
    per_track = np.concatenate([(e.truth_hit >= 0).sum(1) for e in evs])
    joseph = int(np.minimum(per_track, JOSEPH_UPDATES).sum())       # the first updates of each track
    plain = int(per_track.sum()) - joseph
    flops = n * 9 * FLOP_PER_FIT_STEP + joseph * FLOP_PER_UPDATE_JOSEPH + plain * FLOP_PER_UPDATE
    avg_ms = fit_ms / max(fit_n, 1)
    achieved = flops / (avg_ms * 1e-3) / 1e12
    bytes_ = n * BYTES_PER_FIT_TRACK
    gbs = bytes_ / (avg_ms * 1e-3) / 1e9
    res = {
        "metric": "fitted tracks/sec (1,000,000 tracks in 64 uneven batches, one launch)",
        "value": round(n * args.steps / elapsed, 1), "unit": "tracks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "KF fit with known hits, 1,000,000 tracks, batches of 2,000-30,000, 10 layers",
                   "batches": 64},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 5),
                     "traffic": measured_traffic("k_fit"), "kernel": "k_fit", "kernel_avg_ms": round(avg_ms, 4), "flop_per_launch": int(flops),
                     "hbm_algorithmic_GBs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 5)},
    }
    if not args.no_cpu_baseline:
        import oracle
        ev = evs[0]
        threads = max(1, min(16, os.cpu_count() or 1))
        t0 = time.perf_counter()
        oracle.fit(oracle.config(ev.geometry), ev.hits, ev.prior_par, ev.prior_cov, ev.truth_hit, n_threads=threads)
        wall = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": ev.n_seeds / wall, "unit": "tracks/s", "cores": threads, "kind": "oracle",
                               "sample": f"batch 0 ({ev.n_seeds} tracks), {wall:.2f} s wall"}
    ctx.close()
    return res


def workload_batched(args):
    """256 uneven events in one batched launch vs the plain per-event builder."""
    r = batched_leg(args, steps=args.steps)
    return {"metric": "tracks built/sec, 256 uneven events in one batched launch", "value": r["tracks_per_s"],
            "unit": "tracks/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic", "config": {"workload": r["workload"]}, "batched": r}


def workload_serve(args):
    """Poisson arrivals of events (500-50,000 tracks, 30 % noise), served with
    continuous batching; p50/p99 latency against the plain builder serving
    the same arrivals one event at a time."""
    r = serving_leg(args, n_events=args.serve_events)
    return {"metric": "served events/sec and p50/p99 latency (Poisson arrivals)", "unit": "events/s",
            "value": r["rates"][-1]["events_per_s"], "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
            "data": "synthetic", "vs_baseline": None, "config": {"workload": r["workload"]}, "serving": r}


def workload_calib(args):
    """Plain device copy of a known size (calibrates hardware memory counters)."""
    import torch
    nbytes = 256 << 20
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    dst = torch.empty_like(src)
    ctx = make_ctx(1)
    for _ in range(args.steps):
        ctx.calib_copy(src.data_ptr(), dst.data_ptr(), nbytes)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    fma = fma_ceiling(ctx)
    ctx.close()
    return {"metric": "calibration copy", "bytes_per_launch": nbytes, "launches": args.steps, "fma_ceiling": fma}


def lib_build_plain(ctx, h):
    from paper_1702_06359_amd import abi
    abi.check(abi.lib().mkf_build(ctx.h, int(h), None))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ckf",
                    choices=["ckf", "endcap", "two_step", "fit", "batched", "serve", "calib"])
    ap.add_argument("--serve-events", type=int, default=2048)
    ap.add_argument("--tune", action="store_true", help="autotune launch shapes first")
    ap.add_argument("--quick", action="store_true", help="headline number only (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    gpu_count_guard(args.gpus)
    args.tuning = None
    res = {"ckf": workload_ckf, "endcap": workload_endcap, "two_step": workload_endcap, "fit": workload_fit,
           "batched": workload_batched,
           "serve": workload_serve, "calib": workload_calib}[args.workload](args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
