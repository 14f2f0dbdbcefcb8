"""Benchmark of conditional flow-matching sampling on one MI355X.

A step is one fmd_simulate call over the whole batch: the truth encoding with its cross K/V
cache, the Philox noise, and every velocity evaluation and fused state update. The
default workload has 4096 events with N ~ U{20..200} particles. The network is d = 256,
6 blocks, 8 heads, integrated with RK4 over 16 steps (64 evaluations). Inputs are already
resident in HBM when the timed region starts, and outputs stay in HBM.
  value            BF16-path events/s (BF16 MFMA operands, FP32 accumulation/state), timed
                   with per-kernel HIP events on (kernels launched one by one)
  graph_replay     the same steps right after, with timing off (each stage one graph replay)
  fp32             the same workload on the plain FP32 path (median of per-call times)
  fp8              the same workload with FP8 operands for the MLP projections
  error            errors against the FP64 oracle's stored outputs of the first 256 events
                   (normwise per feature and elementwise), BF16 against FP32, pT / eta response
  roofline         the kernel class with the largest device time, timed with HIP events
                   on its launch stream during the timed steps
  cpu_baseline     the FP64 oracle on a bounded sample of the same events, host cores
  reco_multiplicity  the same workload with reco counts drawn on the device (missed truth
                   particles, extra slots); truth_selection and observables: the steps
                   before and after the sampler
  batch_workload   65,536 events with heavy-tailed multiplicities in one call
  latency          the continuous-batching server under open-loop Poisson load, 1k-50k
                   events/s offered, with its saturation throughput and the batch path on the
                   same request mix
Prints one JSON line on stdout.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}    # MI355X dense matrix peaks
WORKLOAD_TEXT = {
    "base": "4096 events, N~U{20..200}, d=256, 6 blocks, 8 heads, RK4 16 steps (64 evaluations)",
    "batch": "65536 events, N~lognormal(median 60, sigma 0.8) in [1, 1000], d=256, 6 blocks, "
             "8 heads, RK4 16 steps (64 evaluations)",
}
PEAK_HBM_GBS = 8000.0
# HBM bytes per launch measured with rocprofv3 byte counters (FETCH_SIZE, WRITE_SIZE), scaled
# by the counts of a 1 GiB copy; valid while the kernel's source is unchanged
TRAFFIC = os.path.join(ROOT, "profiles", "base-4096ev_hbm-traffic.json")


def measured_traffic(kernel):
    import hashlib
    try:
        with open(TRAFFIC) as f:
            rec = json.load(f)["kernels"][kernel]
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                return None
        return rec["hbm_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_path(fmd, torch, cfg, flat, off, feat_d, w, steps, warmup, timing, per_step=False):
    """Times `steps` sampling calls after `warmup` untimed ones; with per_step each call is
    timed on its own (synchronized before and after) and their durations are kept too."""
    m = fmd.Model(cfg, flat)
    out = torch.empty((int(off[-1]), 9), dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        m.simulate(off, feat_d, w.noise_seed, w.schedule, out=out)
    torch.cuda.synchronize()
    if timing:
        m.timing_enable(True)
    step_s = []
    t0 = time.perf_counter()
    for _ in range(steps):
        m.simulate(off, feat_d, w.noise_seed, w.schedule, out=out)
        if per_step:
            torch.cuda.synchronize()
            step_s.append(time.perf_counter() - (t0 + sum(step_s)))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern = {"_step_s": step_s}
    if timing:
        for cls, name in enumerate(fmd.KERNEL_CLASSES):
            ms, n, work, nbytes = m.timing_read(cls)
            kern[name] = {"ms": ms, "launches": n, "work": work, "bytes": nbytes,
                          "kernel": m.kernel_name(cls)}
        m.timing_enable(False)
    table = m.tuning_table()["entries"]
    for e in table:
        log(f"  autotune {e['site']:14s} 2^{e['tokens_log2']} tokens: tile {e['tile']} "
            f"({e['BM']}x{e['BN']}x{e['BK']}, {e['threads']} threads) {e['us']:.0f} us; "
            f"candidates {e['candidates_us']}")
    tiles = {e["site"]: f"{e['BM']}x{e['BN']}x{e['BK']}/{e['threads']}t" for e in table}
    kern["_tiles"] = tiles
    if timing:
        # the same steps with per-kernel timing off: each stage is one graph replay
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            m.simulate(off, feat_d, w.noise_seed, w.schedule, out=out)
        torch.cuda.synchronize()
        kern["_graph_s"] = time.perf_counter() - t1
    m.close()
    return dt, out.cpu().numpy(), kern


def observables_leg(fmd, torch, off, reco, reps):
    """Event observables (Sec. 2.4: H_T, MET, lepton isolation in a Delta R < 0.4 cone) of the
    BF16 sampler's output, resident on the device: wall time per call over `reps` calls
    (each uploads the offsets and ends synchronized), and the cone tests per second counted
    algorithmically (one per lepton and other particle of its event)."""
    reco_d = torch.from_numpy(reco).cuda()
    fmd.event_observables(off, reco_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fmd.event_observables(off, reco_d)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    cls = np.argmax(reco[:, 3:8], axis=1)
    lep = (cls == 1) | (cls == 2)
    n = np.diff(off)
    E = len(off) - 1
    n_lep = np.bincount(np.repeat(np.arange(E), n)[lep], minlength=E)
    tests = float((n_lep * np.maximum(n - 1, 0)).sum())
    return {"kernel": "k_event_observables", "ms_per_call": round(dt * 1e3, 4),
            "events_per_s": round(E / dt, 1), "cone_tests_per_s": round(tests / dt, 1),
            "cone_tests_per_call": tests, "calls": reps}


def select_leg(fmd, torch, off, feat_d, cut, limit, reps):
    """Truth preprocessing (model pT cut and particle limit) on the workload's truth, resident
    on the device: wall time per call over `reps` calls (each ends synchronized)."""
    o2, _ = fmd.truth_select(off, feat_d, cut, limit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fmd.truth_select(off, feat_d, cut, limit)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    E = len(off) - 1
    return {"kernels": ["k_select_count", "k_select_write"], "pt_cut_gev": cut,
            "max_particles": limit, "ms_per_call": round(dt * 1e3, 4),
            "events_per_s": round(E / dt, 1), "particles_in": int(off[-1]),
            "particles_out": int(o2[-1]), "calls": reps}


def batch_leg(fmd, torch, configs, events, params):
    """The batching workload (65,536 events, heavy-tailed multiplicities, BF16, RK4 16) as one
    fmd_simulate call: one warm-up call (which also runs the autotuner for this size), then one
    timed call; the attention and fused-kernel choices of the autotuner for its size bucket."""
    wb = configs.BATCH_BF16
    off, feat = events.for_workload(wb)
    feat_d = torch.from_numpy(feat).cuda()
    m = fmd.Model(wb.model, params.draw(wb.model, wb.weight_seed))
    out = torch.empty((int(off[-1]), 9), dtype=torch.float32, device="cuda")
    m.simulate(off, feat_d, wb.noise_seed, wb.schedule, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.simulate(off, feat_d, wb.noise_seed, wb.schedule, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    table = m.tuning_table()["entries"]
    m.close()
    E, T = len(off) - 1, int(off[-1])
    flops = event_flops(wb.model, np.diff(off), wb.schedule.evals)
    del out, feat_d
    torch.cuda.empty_cache()
    return {"workload": WORKLOAD_TEXT["batch"], "events": E, "particles": T,
            "ms_per_call": round(dt * 1e3, 1), "events_per_s": round(E / dt, 1),
            "mfma_frac": round(flops / dt / (PEAK_TFLOPS["bf16"] * 1e12), 4),
            "tiles": {e["site"]: f"{e['BM']}x{e['BN']}x{e['BK']}/{e['threads']}t" for e in table},
            "tuning": [{k: e[k] for k in ("site", "tokens_log2", "tile", "us", "candidates_us")}
                       for e in table]}


# stand-in reco multiplicity law of the reco leg: 5% of truth particles missed, Binomial(64, 1/4)
# extra slots per event (16 on average)
RECO_LAW = (0.05, 0.25, 64)


def reco_leg(fmd, torch, cfg, flat, off, feat_d, w, steps):
    """The sampler with reco multiplicities that differ from the truth multiplicities, drawn on
    the device (fmd_reco_multiplicity, law RECO_LAW): the draw's wall time per call, and the
    sampler's wall time per step on the same workload, timed like the main path."""
    n = np.diff(off)
    q, p, trials = RECO_LAW
    roff = fmd.reco_multiplicity(off, w.noise_seed, q, p, trials, cfg.n_max)
    t0 = time.perf_counter()
    for _ in range(10):
        fmd.reco_multiplicity(off, w.noise_seed, q, p, trials, cfg.n_max)
    draw_ms = (time.perf_counter() - t0) / 10 * 1e3
    m = fmd.Model(cfg, flat)
    out = torch.empty((int(roff[-1]), 9), dtype=torch.float32, device="cuda")
    m.simulate(off, feat_d, w.noise_seed, w.schedule, out=out, reco_offsets=roff)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        m.simulate(off, feat_d, w.noise_seed, w.schedule, out=out, reco_offsets=roff)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    m.close()
    E = len(n)
    return {"entry": "fmd_reco_multiplicity + fmd_simulate_reco",
            "law": {"loss_prob": q, "fake_prob": p, "fake_trials": trials},
            "reco_slots": int(roff[-1]), "truth_particles": int(off[-1]),
            "count_draw_ms_per_call": round(draw_ms, 3),
            "ms_per_step": round(dt * 1e3, 2), "events_per_s": round(E / dt, 1),
            "reco_slots_per_s": round(int(roff[-1]) / dt, 1), "steps": steps}


def bound_of(k, dtype):
    """The resource that bounds a kernel class at its algorithmic FLOPs and bytes: the one
    whose peak takes longer to serve them."""
    return "hbm" if k["bytes"] / (PEAK_HBM_GBS * 1e9) > k["work"] / (PEAK_TFLOPS[dtype] * 1e12) \
        else "mfma"


def roofline(kern, dtype, traffic_known=True):
    gemm_attn = {k: v for k, v in kern.items() if not k.startswith("_") and k != "other"
                 and v["launches"]}
    name, k = max(gemm_attn.items(), key=lambda kv: kv[1]["ms"])
    avg_s = k["ms"] / k["launches"] * 1e-3
    flops = k["work"] / k["launches"]
    nbytes = k["bytes"] / k["launches"]
    total_ms = sum(v["ms"] for k_, v in kern.items() if not k_.startswith("_"))
    bound = bound_of(k, dtype)
    if bound == "hbm":
        achieved, peak, unit = nbytes / avg_s / 1e9, PEAK_HBM_GBS, "GB/s"
    else:
        achieved, peak, unit = flops / avg_s / 1e12, PEAK_TFLOPS[dtype], "TFLOP/s"
    traffic = measured_traffic(k["kernel"]) if dtype == "bf16" and traffic_known else None
    return {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": k["kernel"],
            "class": name, "avg_launch_ms": round(k["ms"] / k["launches"], 4),
            "flop_per_launch": flops, "bytes_per_launch": nbytes,
            "tflops": round(flops / avg_s / 1e12, 2), "gbps": round(nbytes / avg_s / 1e9, 1),
            "share_of_device_time": round(k["ms"] / total_ms, 3)}


# FP64 oracle outputs of the first 256 base-workload events, written by
# tests/golden/make_oracle_outputs.py (which runs the oracle only)
GOLDEN_BASE = os.path.join(ROOT, "tests", "golden", "oracle_base_rk4x16_first256.npz")


def precision_report(off, feat, out16, out32, label="bf16", resp_frac=0.01):
    """Errors of the BF16 path (and the FP32 one) on the first 256 events against the FP64
    oracle, BF16 against FP32 on all events, and the pT / eta response (slot i of an event
    against truth particle i: pT ratio and eta difference, mean and population width) of
    each source with its agreement with the oracle's at 1%. Normwise per feature:
    max|dy| / max|ref| (the headline, worst feature); elementwise diagnostic: max |dy| /
    (|ref| + rms of the feature)."""
    from workload import errors
    g = np.load(GOLDEN_BASE)
    n = len(g["offsets"]) - 1
    assert np.array_equal(g["offsets"], off[:n + 1]), "golden events differ from the workload"
    rows = int(off[n])
    ref = g["reco"]
    truth = feat[:rows]
    srcs = {label: out16}
    if out32 is not None:
        srcs["fp32"] = out32
    rep = {"events_checked": n, "oracle": "FP64 oracle outputs of the first 256 events"}
    resp_ref = errors.response(ref, truth)
    rep["response_oracle"] = resp_ref
    for name, y in srcs.items():
        rep[f"{name}_vs_oracle"] = float(errors.normwise_rel_err(y[:rows], ref).max())
        rep[f"{name}_vs_oracle_elementwise"] = float(errors.elementwise_rel_err(y[:rows], ref).max())
        resp = errors.response(y[:rows], truth)
        rep[f"response_{name}"] = resp
        frac = resp_frac if name == label else 0.01
        rep[f"response_{name}_within_{round(frac * 100)}pct_of_oracle"] = errors.response_agrees(
            resp, resp_ref, frac)
    if out32 is not None:
        rep["bf16_vs_fp32_all_events"] = float(errors.normwise_rel_err(out16, out32).max())
        rep["bf16_vs_fp32_all_events_elementwise"] = float(errors.elementwise_rel_err(out16, out32).max())
        rep["response_bf16_within_1pct_of_fp32"] = errors.response_agrees(
            rep["response_bf16"], errors.response(out32[:rows], truth))
    return rep


def cpu_baseline(w, flat, off, feat, sample_events, processes):
    from oracle import sample
    ids = list(range(sample_events))
    t0 = time.perf_counter()
    outs = sample.simulate_events(flat, w.model, off, feat, w.schedule, seed=w.noise_seed,
                                  event_ids=ids, processes=processes,
                                  progress=lambda k, n: log(f"oracle: {k}/{n} events"))
    dt = time.perf_counter() - t0
    return dt, np.concatenate(outs)


def event_flops(cfg, n, evals):
    """Algorithmic flops of sampling one event of n particles with `evals` network evaluations:
    per evaluation L (28 d^2 n + 8 d n^2) + 4 F d n (matrix products, both attentions, input
    embedding and output head), plus once per event the truth encoder (2 F d n) and the cross
    K/V cache (4 L d^2 n)."""
    d, L, F = cfg.d_model, cfg.n_blocks, 9
    n = np.asarray(n, dtype=np.float64)
    return float(np.sum(evals * (L * (28 * d * d * n + 8 * d * n * n) + 4 * F * d * n)
                        + 2 * F * d * n + 4 * L * d * d * n))


def run_rate(fmd, srv, reqs, model_cfg):
    """Submits `reqs` at their arrival times (open loop, from a thread) and collects them;
    returns the latency and throughput record."""
    import threading

    n_req = len(reqs)
    ids = [None] * n_req
    t_start = time.perf_counter()

    def submit():
        for i, r in enumerate(reqs):
            dt = r.t_arrive - (time.perf_counter() - t_start)
            if dt > 0:
                time.sleep(dt)
            ids[i] = srv.submit(r.offsets, r.feat, r.seed, r.schedule)

    info0 = srv.info()
    th = threading.Thread(target=submit)
    th.start()
    lat_req, lat_ev, n_events, t_first, t_last, flops = [], [], 0, None, None, 0.0
    for i in range(n_req):
        while ids[i] is None:
            time.sleep(0.0005)
        _, st = srv.wait(ids[i])
        lat = (st["t_done_ns"] - st["t_submit_ns"]) * 1e-6
        ne = len(reqs[i].offsets) - 1
        lat_req.append(lat)
        lat_ev += [lat] * ne
        n_events += ne
        flops += event_flops(model_cfg, np.diff(reqs[i].offsets), reqs[i].schedule.evals)
        t_first = st["t_submit_ns"] if t_first is None else min(t_first, st["t_submit_ns"])
        t_last = st["t_done_ns"] if t_last is None else max(t_last, st["t_done_ns"])
    th.join()
    info1 = srv.info()
    wall = (t_last - t_first) * 1e-9
    rows = info1["rows_processed"] - info0["rows_processed"]
    return {"requests": n_req, "events": n_events,
            "achieved_events_per_s": round(n_events / wall, 1),
            "p50_event_ms": round(float(np.percentile(lat_ev, 50)), 2),
            "p99_event_ms": round(float(np.percentile(lat_ev, 99)), 2),
            "p50_request_ms": round(float(np.percentile(lat_req, 50)), 2),
            "p99_request_ms": round(float(np.percentile(lat_req, 99)), 2),
            "device_busy_frac": round((info1["busy_ns"] - info0["busy_ns"]) * 1e-9 / wall, 3),
            "live_row_frac": round((info1["rows_live"] - info0["rows_live"]) / max(rows, 1), 3),
            "iterations": info1["iterations"] - info0["iterations"],
            "mfma_frac": round(flops / wall / (PEAK_TFLOPS["bf16"] * 1e12), 4)}


def batch_reference(fmd, torch, model, reqs, model_cfg):
    """The batch path on the same events and schedules as `reqs`: one fmd_simulate call per
    schedule over all its events (inputs resident on the device), timed after a warm-up."""
    groups = {}
    for r in reqs:
        groups.setdefault((r.schedule.scheme, r.schedule.n_steps), []).append(r)
    calls = []
    for key, rs in groups.items():
        off = np.r_[0, np.cumsum(np.concatenate([np.diff(r.offsets) for r in rs]))].astype(np.int64)
        feat = torch.from_numpy(np.concatenate([r.feat for r in rs])).cuda()
        out = torch.empty((int(off[-1]), 9), dtype=torch.float32, device="cuda")
        calls.append((off, feat, out, rs[0].schedule))
    for off, feat, out, sch in calls:
        model.simulate(off, feat, 5, sch, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for off, feat, out, sch in calls:
        model.simulate(off, feat, 5, sch, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_ev = sum(len(off) - 1 for off, _, _, _ in calls)
    flops = sum(event_flops(model_cfg, np.diff(r.offsets), r.schedule.evals) for r in reqs)
    return {"events": n_ev, "events_per_s": round(n_ev / dt, 1),
            "mfma_frac": round(flops / dt / (PEAK_TFLOPS["bf16"] * 1e12), 4)}


def serve_leg(fmd, torch, w_serve, flat, rates, n_requests, budget):
    """Open-loop Poisson load on the continuous-batching server, one run per offered rate.

    Requests arrive at exponential gaps (mean = E[events per request] / rate). Each carries
    1..512 events with heavy-tailed multiplicities and asks for Euler 20 or RK4 16 with
    probability 1/2. They are submitted at their arrival times whatever the server's state,
    so queueing counts in the latency. Latency = completion - submission on the server's
    monotonic clock, weighted per event (each event takes its request's latency) and per
    request. A warm-up stream runs first (allocation and tuning of the sizes it meets). The
    saturation throughput is the largest achieved rate; the batch path is timed on the
    request mix of the highest rate for comparison.
    """
    from workload import arrivals

    cfg = w_serve.model
    out = []
    m = fmd.Model(cfg, flat)
    srv = fmd.Server(m, hbm_budget_bytes=budget)
    seed = w_serve.extra["arrival_seed"]
    run_rate(fmd, srv, arrivals.stream(20000.0, max(20, n_requests // 2), seed=seed + 100), cfg)
    last = None
    for i, rate in enumerate(rates):
        reqs = arrivals.stream(rate, n_requests, seed=seed + i)
        rec = {"offered_events_per_s": rate, **run_rate(fmd, srv, reqs, cfg)}
        log(f"serve @ {rate} ev/s offered: {rec}")
        out.append(rec)
        last = reqs
    info = srv.info()
    srv.close()
    batch = batch_reference(fmd, torch, m, last, cfg)
    m.close()
    sat = max(r["achieved_events_per_s"] for r in out)
    log(f"serve: saturation {sat} events/s; batch path on the same mix {batch}")
    return {"rates": out, "saturation_events_per_s": sat,
            "batch_path_same_mix": batch, "saturation_vs_batch": round(sat / batch["events_per_s"], 3),
            "hbm_budget_bytes": budget, "pool_tokens": info["pool_tokens"],
            "requests_per_rate": n_requests}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp32-steps", type=int, default=5, help="FP32 calls timed (median reported)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8-operand leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batching-workload leg")
    ap.add_argument("--fp8-steps", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle events (0: 6 per core)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-reco", action="store_true", help="skip the reco-multiplicity leg")
    ap.add_argument("--serve-rates", default="1000,2000,5000,10000,20000,50000")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests per offered rate")
    ap.add_argument("--workload", choices=["base", "batch"], default="base",
                    help="base: 4096 events, N~U{20..200} (the headline); batch: 65,536 events "
                         "with heavy-tailed N (FP32, reco and serving legs skipped)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB three times "
                         "(reference kernel of known traffic for HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {a.gpus}): events are independent and "
              "shard across GPUs without communication, but this build runs on one device.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2606_26089_amd import fmd
    from workload import configs, errors, events, params

    if a.copy_mib:
        src = torch.ones(a.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {a.copy_mib} MiB three times")
        del src, dst

    w = configs.BASE_BF16
    if a.workload == "batch":
        w = configs.BATCH_BF16
        a.no_fp32 = a.no_reco = a.no_serve = True
    off, feat = events.for_workload(w)
    T = int(off[-1])
    E = len(off) - 1
    feat_d = torch.from_numpy(feat).cuda()
    flat = params.draw(w.model, w.weight_seed)
    log(f"workload {w.name}: {E} events, {T} particles, {w.schedule.evals} evaluations")

    dt16, out16, kern16 = time_path(fmd, torch, w.model, flat, off, feat_d, w, a.steps, a.warmup, True)
    ev16 = E * a.steps / dt16
    log(f"bf16: {dt16 / a.steps * 1e3:.1f} ms/step, {ev16:.1f} events/s")
    graph = {"ms_per_step": round(kern16["_graph_s"] / a.steps * 1e3, 2),
             "events_per_s": round(E * a.steps / kern16["_graph_s"], 2)}
    log(f"bf16 with stage graphs (no per-kernel timing): {graph['ms_per_step']:.1f} ms/step, "
        f"{graph['events_per_s']:.1f} events/s")
    log(f"  tiles chosen by the autotuner: {kern16['_tiles']}")
    for name, k in kern16.items():
        if name.startswith("_"):
            continue
        log(f"  {name:11s} {k['kernel']:14s} {k['ms'] / a.steps:9.1f} ms/step  {k['launches'] // a.steps:5d} "
            f"launches/step  {k['work'] / max(k['ms'], 1e-9) / 1e9:8.1f} TFLOP/s "
            f"{k['bytes'] / max(k['ms'], 1e-9) / 1e6:8.1f} GB/s  ({bound_of(k, 'bf16')}-bound)")
    rl = roofline(kern16, "bf16", traffic_known=a.workload == "base")
    log(f"dominant kernel {rl['kernel']}: {rl['achieved']} {rl['unit']} ({rl['frac']:.3f} of peak), "
        f"HBM traffic {rl['traffic']} bytes/launch (algorithmic {rl['bytes_per_launch']:.0f})")

    selection = select_leg(fmd, torch, off, feat_d, 0.5, 128, 20)
    log(f"truth selection (0.5 GeV, 128 particles): {selection['ms_per_call']:.3f} ms per call, "
        f"{selection['particles_in']} -> {selection['particles_out']} particles")
    obs = observables_leg(fmd, torch, off, out16, 20)
    log(f"event observables: {obs['ms_per_call']:.3f} ms per call, {obs['events_per_s']:.0f} "
        f"events/s, {obs['cone_tests_per_s'] / 1e9:.2f} G cone tests/s")

    reco = None
    if not a.no_reco:
        reco = reco_leg(fmd, torch, w.model, flat, off, feat_d, w, 1)
        log(f"reco multiplicities drawn on the device: {reco['reco_slots']} slots for "
            f"{reco['truth_particles']} truth particles, {reco['ms_per_step']:.1f} ms/step, "
            f"{reco['events_per_s']:.1f} events/s")

    fp32 = None
    out32 = None
    if not a.no_fp32:
        cfg32 = w.model.with_precision(configs.FP32)
        dt32, out32, kern32 = time_path(fmd, torch, cfg32, flat, off, feat_d, w, a.fp32_steps, 1,
                                        True, per_step=True)
        med32 = float(np.median(kern32["_step_s"]))
        ev32 = E / med32
        log(f"fp32: median {med32 * 1e3:.1f} ms/step over {a.fp32_steps}, {ev32:.1f} events/s")
        rl32 = roofline(kern32, "fp32")
        fp32 = {"events_per_s": round(ev32, 2), "ms_per_step": round(med32 * 1e3, 2),
                "steps": a.fp32_steps, "timing": "median of per-call times",
                "roofline": rl32, "tiles": kern32["_tiles"]}

    batch = None
    if not a.no_batch and a.workload == "base":
        batch = batch_leg(fmd, torch, configs, events, params)
        log(f"batching workload: {batch['ms_per_call']:.0f} ms per call, {batch['events_per_s']} "
            f"events/s, tiles {batch['tiles']}")

    fp8 = None
    if not a.no_fp8 and a.workload == "base":
        cfg8 = w.model.with_precision(configs.FP8)
        dt8, out8, kern8 = time_path(fmd, torch, cfg8, flat, off, feat_d, w, a.fp8_steps, 1, True,
                                     per_step=True)
        med8 = float(np.median(kern8["_step_s"]))
        rl8 = roofline(kern8, "bf16", traffic_known=False)
        mlp = kern8["fused_mlp"]
        fp8 = {"events_per_s": round(E / med8, 2), "ms_per_step": round(med8 * 1e3, 2),
               "steps": a.fp8_steps, "timing": "median of per-call times",
               "precision": "fp8 (e4m3) operands for W_up and W_dn, bf16 elsewhere, fp32 "
                            "accumulation and state",
               "mlp_kernel_ms_per_launch": round(mlp["ms"] / max(mlp["launches"], 1), 4),
               "dominant_kernel": {k: rl8[k] for k in ("kernel", "avg_launch_ms", "tflops")},
               "error": precision_report(off, feat, out8, None, label="fp8", resp_frac=0.03)}
        log(f"fp8: median {med8 * 1e3:.1f} ms/step, {fp8['events_per_s']} events/s, "
            f"error {fp8['error']['fp8_vs_oracle']:.3e}")

    cpu = None
    err = None
    if not a.no_cpu_baseline:
        cores = min(os.cpu_count() or 1, 16)
        n = a.cpu_sample or 6 * cores
        dt_cpu, ref = cpu_baseline(w, flat, off, feat, n, cores)
        rows = int(off[n])
        cpu = {"value": round(n / dt_cpu, 4), "unit": "events/s", "cores": cores, "kind": "oracle",
               "sample": f"first {n} events of the workload ({rows} particles), full RK4 16 "
                         f"integration in NumPy float64, {cores} processes, {dt_cpu:.1f} s"}
        log(f"oracle: {cpu['value']} events/s on {cores} cores")
    if a.workload == "base":
        err = precision_report(off, feat, out16, out32)
        log(f"errors: {json.dumps(err)}")

    serve = None
    if not a.no_serve:
        ws = configs.SERVE_BF16
        rates = [float(r) for r in a.serve_rates.split(",") if r]
        serve = serve_leg(fmd, torch, ws, flat, rates, a.serve_requests, ws.extra["hbm_budget_bytes"])

    line = {
        "metric": "sampled events/s, BF16 vs FP32 plain at stated error; p50/p99 event latency",
        "value": round(ev16, 2), "unit": "events/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(dt16 / a.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (seeded truth events and stand-in weights)",
        "config": {"workload": WORKLOAD_TEXT[a.workload], "events": E, "particles": T,
                   "precision": "bf16 operands, fp32 accumulation and state",
                   "tiles": kern16["_tiles"]},
        "graph_replay": graph, "fp32": fp32, "error": err,
        "latency": serve, "truth_selection": selection, "observables": obs,
        "reco_multiplicity": reco, "fp8": fp8, "batch_workload": batch,
        "roofline": rl, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
