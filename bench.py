#!/usr/bin/env python3
"""Throughput of the batched cost-model hot path on one MI355X.

Headline: the bf16 serving path, saturated.  256 search sessions, each over a
pipeline of S stages (log-uniform in [3, 120]); a step is one beam-step query
from every session (candidates uniform in [16, 4096], bf16 schedule features,
float32 cost terms), 256 queries in all, submitted with one call and served
by continuous batching: per-stage rows hoisted once per session ->
persistent bf16 matrix-core evaluation with Kahan stage sums -> per-query
top-32 selection, micro-batches overlapping on several streams.  Three steps
are kept submitted so the device never waits for the client; before the warm-up
steps the device serves saturated for 100 ms, past the ramp of its power
state that follows the light-load latency phase.  Inputs are
resident in HBM before timing (distinct inputs per session and step, several
GB in all, far above the 256 MB last-level cache).

Also reported: p50/p99 latency under an open-loop Poisson load of 2,000
queries/s; the dominant kernel's HBM roofline (algorithmic bytes over the
kernel's own GPU time); the ragged 17-query batch as one step (with parity
against the FP64 oracle); the float32 plain path on a 6,400 x 30 beam step;
the FP64 CPU oracle on a bounded sample.

Prints one JSON line.  --gpus N with N > 1 is refused: this path runs on one
GPU (sessions shard across GPUs with no exchange of features).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cost-model candidates/sec (BF16 vs FP32 plain) at ≥99.9% top-32 agreement; p99"
HBM_PEAK_GBS = 8000.0
BYTES_PER_ROW_BF16 = 40 * 2 + 8 * 4   # schedule features (bf16) + cost terms (fp32)
BYTES_PER_CAND_OUT = 4                # one float32 cost written per candidate
K = 32
SESSIONS = 256
# the step kernel's sources, as paths from the repository root; the public
# header's constants (the stage split among them) shape its work too, so its
# "#define CM_" lines join the hash (its comments do not)
STEP_SOURCES = tuple("paper_2012_07145_amd/csrc/" + f for f in
                     ("k_step.hip", "eval_bf16.h", "eval_fp8.h", "topk_dev.h", "cm_internal.h"))
STEP_HEADER = "include/cm.h"


def step_kernel_hash():
    """sha256 over the step kernel's sources and the public header's constants."""
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    for line in open(os.path.join(ROOT, STEP_HEADER), "rb"):
        if line.startswith(b"#define CM_"):
            h.update(line)
    return h.hexdigest()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed serving steps")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--inputs-per-session", type=int, default=4)
    ap.add_argument("--latency-queries", type=int, default=20000)
    ap.add_argument("--latency-qps", type=float, default=2000.0)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-agreement", action="store_true",
                    help="skip the served-beam agreement with the FP64 oracle")
    ap.add_argument("--no-read-probe", action="store_true",
                    help="skip the measured streaming-read roof")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--serve-tune", action="store_true",
                    help="try a few step configurations of the server on the serving traffic "
                         "and serve with the fastest (default: two workgroups per compute "
                         "unit, one row-tile group per task)")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the 65,536 x 64 bf16 / fp8 comparison")
    ap.add_argument("--settle-ms", type=float, default=100.0,
                    help="saturated serving before the warm-up steps, in ms (0: none)")
    ap.add_argument("--queue-depth", type=int, default=3,
                    help="serving steps the client keeps submitted at a time")
    ap.add_argument("--no-fp8-serving", action="store_true",
                    help="skip the same serving workload in the FP8 form")
    ap.add_argument("--slots", type=int, default=3, help="serving micro-batches in flight")
    ap.add_argument("--serve-graph", type=int, choices=(0, 1), default=None,
                    help="server steps as a replayed HIP graph (1) or plain launches (0); "
                         "default: the library's")
    ap.add_argument("--max-batch-queries", type=int, default=128)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


def traffic_record():
    """HBM bytes per step-kernel launch from committed counter runs, valid
    only while the step kernel's sources are unchanged."""
    path = os.path.join(ROOT, "profiles", "step_bf16_serving_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sha256") != step_kernel_hash():
        return None
    return rec


def draw_request(torch, S, N, seed, device):
    """One request's float32 schedule features exp(N(4, 2^2)) and cost terms
    exp(N(6, 1.5^2)), drawn on the GPU from their own seed, so that the
    float32 originals of a bf16 request can be drawn again for the oracle."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    sched = torch.empty(S * N * 40, device=device).normal_(4.0, 2.0, generator=g).exp_()
    terms = torch.empty(S * N * 8, device=device).normal_(6.0, 1.5, generator=g).exp_()
    return sched, terms


def session_inputs(torch, rng, n_sessions, per_session, device, seed):
    """Stage counts of the sessions and per-session request inputs drawn on
    the GPU: (S, pipe, [(N, sched bf16, terms f32, seed), ...]) per session."""
    import numpy as np
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = []
    for s in range(n_sessions):
        S = int(np.floor(np.exp(rng.uniform(np.log(3), np.log(121)))))
        reqs = []
        for j in range(per_session):
            N = int(rng.integers(16, 4097))
            rseed = seed * 100003 + s * 4099 + j
            sched, terms = draw_request(torch, S, N, rseed, device)
            reqs.append((N, sched.to(torch.bfloat16), terms, rseed))
            del sched
        pipe = torch.poisson(torch.full((S * 56,), 3.0, device=device), generator=g)
        out.append((S, pipe.cpu().numpy().reshape(S, 56), reqs))
    return out


def host_cpu():
    """(threads this process may use, CPU model name) of the host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return len(os.sched_getaffinity(0)), model


def probe_read_gbs(reps=10, gib=4):
    """Median and best streaming-read GB/s of a plain read kernel of the
    library's probe over `gib` GiB (far above the 256 MB last-level cache)."""
    import ctypes
    path = os.path.join(ROOT, "paper_2012_07145_amd", "libcm_probe.so")
    L = ctypes.CDLL(path)
    L.cm_probe_read_gbs.argtypes = [ctypes.c_int64, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    med, best = ctypes.c_double(), ctypes.c_double()
    rc = L.cm_probe_read_gbs(gib << 30, reps, ctypes.byref(med), ctypes.byref(best))
    if rc != 0:
        raise RuntimeError(f"cm_probe_read_gbs failed ({rc})")
    return med.value, best.value


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the cost-model path shards by session across "
              "GPUs with no feature exchange, and the benchmark measures one GPU's share. "
              f"--gpus {args.gpus} is not supported.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2012_07145_amd as cm
    from synth import model_params, workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = "cuda"

    if args.copy_calibration:
        n = 1 << 28  # 1 GiB of float32
        a = torch.ones(n, device=dev)
        b = torch.empty(n, device=dev)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 5}))
        return

    params = model_params()
    model = cm.cm_model_create(params)

    # ------------------------------------------------------------ serving inputs
    rng = np.random.default_rng(5)
    log(f"generating inputs of {SESSIONS} sessions x {args.inputs_per_session} requests")
    sess_in = session_inputs(torch, rng, SESSIONS, args.inputs_per_session, dev, 5005)
    torch.cuda.synchronize()
    in_bytes = sum(S * N * BYTES_PER_ROW_BF16 for S, _, reqs in sess_in for N, *_ in reqs)
    log(f"{in_bytes / 1e9:.2f} GB of request inputs resident")
    srv = cm.cm_server_create(model, k=K, arena_bytes=16 << 30, max_slots=args.slots,
                              max_pending=8192, max_sessions=SESSIONS, max_stages=128,
                              max_batch_queries=args.max_batch_queries, max_batch_cands=1 << 20)
    if args.serve_graph is not None:
        srv.set_step_config(0, 1, args.serve_graph)
    sids = [srv.session_open(pipe) for _, pipe, _ in sess_in]

    # a step's request j of every session, as pre-marshalled arrays
    steps_pre = []
    for j in range(args.inputs_per_session):
        ns = [sess_in[s][2][j][0] for s in range(SESSIONS)]
        sp = np.array([sess_in[s][2][j][1].data_ptr() for s in range(SESSIONS)], np.uint64)
        tp = np.array([sess_in[s][2][j][2].data_ptr() for s in range(SESSIONS)], np.uint64)
        steps_pre.append((np.array(ns, np.int32), sp, tp, sum(ns),
                          sum(n * sess_in[s][0] for s, n in enumerate(ns))))
    sids_arr = np.array(sids, np.int32)

    def submit_step(i):
        ns, sp, tp, _, _ = steps_pre[i % len(steps_pre)]
        return srv.submit_batch(sids_arr, ns, sp, tp, K)

    def run_steps(n):
        """n steps, args.queue_depth of them queued at a time; returns
        (candidates, rows)."""
        depth = max(1, args.queue_depth)
        q = [submit_step(i) for i in range(min(depth, n))]
        cands = rows = 0
        for i in range(n):
            srv.wait_all(q.pop(0), 120000)
            if i + depth < n:
                q.append(submit_step(i + depth))
            cands += steps_pre[i % len(steps_pre)][3]
            rows += steps_pre[i % len(steps_pre)][4]
        return cands, rows

    # ------------------------------------------------------------ latency
    # The open-loop phase runs first, at light load; the saturated phase
    # follows it after a settle period (below).
    latency = None
    if not args.no_latency:
        srv.reset_stats()
        lrng = np.random.default_rng(6)
        n_warm = int(args.latency_qps)  # one second
        n_all = n_warm + args.latency_queries
        gaps = lrng.exponential(1.0 / args.latency_qps, n_all)
        who = lrng.integers(0, SESSIONS, n_all)
        pick = lrng.integers(0, args.inputs_per_session, n_all)
        tickets = []
        t_next = time.perf_counter()
        for i in range(n_all):
            t_next += gaps[i]
            while time.perf_counter() < t_next:
                pass
            if i == n_warm:
                srv.wait_all(np.array(tickets, np.uint64), 120000)
                tickets = []
                srv.reset_stats()
            s = int(who[i])
            N, sched, terms, _ = sess_in[s][2][int(pick[i])]
            tickets.append(srv.submit(sids[s], N, sched, terms, K))
        srv.wait_all(np.array(tickets, np.uint64), 120000)
        ls = srv.stats()
        latency = {"offered_qps": args.latency_qps, "queries": ls["completed"],
                   "achieved_qps": ls["completed"] / (ls["wall_us"] * 1e-6) if ls["wall_us"] else 0,
                   "p50_us": ls["p50_us"], "p99_us": ls["p99_us"], "max_us": ls["max_us"],
                   "micro_batches": ls["micro_batches"]}
        log(f"latency at {args.latency_qps:.0f} q/s: p50 {ls['p50_us']:.0f} us, "
            f"p99 {ls['p99_us']:.0f} us over {ls['completed']} queries")
    # ------------------------------------------------------------ saturated
    # Settle: the open-loop phase keeps the device mostly idle, and the first
    # tens of milliseconds of saturated serving after it run the step kernel
    # about a quarter slower (about 225 us instead of 177 us per launch, the
    # device's power state ramping back up).  A saturated server is past that
    # ramp, so the device serves saturated for at least --settle-ms before the
    # warm-up steps; the JSON line reports how long.
    # for the record, 20 steps timed right after the light-load phase, before
    # the settle period (the same measure as the headline's)
    cold = None
    if not args.no_latency:
        srv.reset_stats()
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        c_cold, _ = run_steps(20)
        torch.cuda.synchronize()
        w_c = time.perf_counter() - t_c
        sc = srv.stats()
        dev_c = sc["kernel_busy_us"] if sc["kernel_busy_launches"] == sc["micro_batches"] else sc["kernel_us"]
        cold = {"steps": 20, "candidates_per_s": c_cold / w_c, "ms_per_step": w_c / 20 * 1e3,
                "roofline_frac": sc["kernel_bytes"] / (dev_c * 1e-6) / 1e9 / HBM_PEAK_GBS if dev_c else None}
        log(f"cold: {cold['candidates_per_s']:.3e} candidates/s, frac {cold['roofline_frac']:.3f}")
    settle = {"ms": 0.0, "steps": 0}
    if args.settle_ms > 0:
        t_s = time.perf_counter()
        while (time.perf_counter() - t_s) * 1e3 < args.settle_ms:
            run_steps(10)
            settle["steps"] += 10
        torch.cuda.synchronize()
        settle["ms"] = (time.perf_counter() - t_s) * 1e3
        log(f"settle: {settle['steps']} saturated steps in {settle['ms']:.1f} ms")
    run_steps(args.warmup)
    torch.cuda.synchronize()
    log(f"warm-up done ({args.warmup} steps)")

    # the server's step configuration: a short trial of a few launch shapes on
    # this traffic (part of the warm-up, outside the timed region).  Only grids
    # that fill every compute unit by themselves are tried: with fewer
    # workgroups, consecutive micro-batches share the device and a launch's own
    # duration no longer measures the kernel.
    tune = None
    if args.serve_tune:
        trials = []
        for grid, gt in ((0, 1), (0, 2), (0, 4), (1024, 1), (1024, 2)):
            srv.set_step_config(grid, gt, 1)
            run_steps(2)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            c_, _ = run_steps(8)
            torch.cuda.synchronize()
            trials.append((c_ / (time.perf_counter() - ta), grid, gt))
        best = max(trials)
        srv.set_step_config(best[1], best[2], 1)
        tune = {"chosen": srv.get_step_config(),
                "trials": [{"grid": g, "group_tiles": t, "candidates_per_s": v} for v, g, t in trials]}
        log(f"serving step configuration: {tune['chosen']}")
    srv.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cands, rows = run_steps(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    st = srv.stats()
    value = cands / wall
    log(f"serving: {args.steps} steps, {cands} candidates in {wall * 1e3:.1f} ms "
        f"({st['micro_batches']} micro-batches)")
    launches = max(1, st["micro_batches"])
    # The step kernel's device time over the timed region: the union of the
    # launches' [first wave start, last wave end] intervals, from the kernel's
    # own clock.  Consecutive micro-batches overlap on the device (the next
    # one's workgroups start on compute units the previous one has left, and
    # early in a run several are queued at once), so the mean of the
    # launches' own spans counts that time twice; it is reported beside, as
    # is the device time left idle between launches.
    own_us = st["kernel_us"] / launches
    if st["kernel_busy_launches"] == st["micro_batches"]:
        avg_us = st["kernel_busy_us"] / launches
        launch_time = ("union of the timed launches' intervals (first wave start to last wave "
                       "end, the kernel's clock) per launch")
    else:  # more launches than the server records: their own spans
        avg_us = own_us
        launch_time = "mean of the timed launches' own spans (first wave start to last wave end)"
    idle_us = max(0.0, st["kernel_span_us"] / launches - avg_us)
    bytes_per_launch = st["kernel_bytes"] / launches
    achieved = bytes_per_launch / (avg_us * 1e-6) / 1e9 if avg_us else 0.0
    tr = traffic_record()
    read_roof = None
    if not args.no_read_probe:
        read_roof = probe_read_gbs()
        log(f"streaming-read probe: {read_roof[0]:.0f} GB/s median, {read_roof[1]:.0f} best; "
            f"k_step_bf16 {achieved:.0f} GB/s = {achieved / read_roof[0]:.3f} of it")

    # served beams of every request of every input set against the FP64
    # oracle, on two readings: the float32 originals the bf16 features were
    # rounded from (the headline reading) and the bf16-rounded features the
    # server reads (its arithmetic alone).  The server's beams do not depend on
    # batching, so these are the beams of the timed steps.
    import oracle
    agree = None
    if not args.no_agreement:
        t_ag = time.perf_counter()
        hits = {"f32": 0, "bf16": 0}
        tot = 0
        worst_bf16 = worst_f32 = 0.0
        n_req = 0
        for j in range(args.inputs_per_session):
            ns, sp, tp, _, _ = steps_pre[j]
            tickets = srv.submit_batch(sids, ns, sp, tp, K)
            beams = srv.wait_all_results(tickets, 120000)
            for s_, (idx, val) in enumerate(beams):
                S, pipe, reqs = sess_in[s_]
                N, sched16, terms, rseed = reqs[j]
                x32, _ = draw_request(torch, S, N, rseed, dev)
                x32 = x32.cpu().numpy().reshape(S, N, 40)
                t_h = terms.cpu().numpy().reshape(S, N, 8)
                x16 = sched16.float().cpu().numpy().reshape(S, N, 40)
                kk = min(K, N)
                sel = idx[:kk].tolist()
                for name, x in (("f32", x32), ("bf16", x16)):
                    ref = oracle.eval_query(params, pipe, x, t_h)
                    top = np.lexsort((np.arange(N), ref))[:kk]
                    hits[name] += len(set(sel) & set(top.tolist()))
                    rel = float(np.max(np.abs(val[:kk].astype(np.float64) - ref[idx[:kk]]) /
                                       np.abs(ref[idx[:kk]])))
                    if name == "f32":
                        worst_f32 = max(worst_f32, rel)
                    else:
                        worst_bf16 = max(worst_bf16, rel)
                tot += kk
                n_req += 1
        agree = {"requests": n_req, "selections": tot,
                 "vs_fp64_f32_inputs": hits["f32"] / tot, "hits_f32_inputs": [hits["f32"], tot],
                 "vs_fp64_bf16_inputs": hits["bf16"] / tot, "hits_bf16_inputs": [hits["bf16"], tot],
                 "max_rel_err_beam_vs_fp64_f32_inputs": worst_f32,
                 "max_rel_err_beam_vs_fp64_bf16_inputs": worst_bf16,
                 "meets_999": hits["f32"] / tot >= 0.999,
                 "seconds": time.perf_counter() - t_ag}
        log(f"served beams ({n_req} requests, {tot} selections) vs FP64: top-32 agreement "
            f"{hits['f32']}/{tot} = {hits['f32'] / tot:.5f} on the float32 originals, "
            f"{hits['bf16']}/{tot} = {hits['bf16'] / tot:.5f} on the bf16 inputs "
            f"({agree['seconds']:.0f} s)")
    # a bounded sample for the CPU baseline: the first request of 8 sessions
    sample = []
    for s_ in range(8):
        S, pipe, reqs = sess_in[s_]
        N, sched, terms, _ = reqs[0]
        sample.append((pipe, sched.float().cpu().numpy().reshape(S, N, 40),
                       terms.cpu().numpy().reshape(S, N, 8)))
    srv.close()

    # ------------------------------------------------------------ ragged step
    ragged = None
    W = workload("ragged_17q")
    if not args.no_ragged:
        batch0, cost_t = cm.pack_queries(W.queries, "bf16", dev)
        nq = len(W.queries)
        n_stages = sum(q.n_stages for q in W.queries)
        step = cm.cm_step_create(model, "bf16", max_queries=nq, max_stages=n_stages,
                                 max_cands=W.n_cands, max_k=K, slots=2)
        idx_t = torch.empty(nq * K, dtype=torch.int32, device=dev)
        val_t = torch.empty(nq * K, device=dev)
        cfg, tuned_us = cm.cm_step_autotune(step, batch0, None, K, cost_t, idx_t, val_t, reps=10)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(100)]
        kern = []
        for a, b in evs:
            a.record()
            cm.cm_step_run(step, batch0, None, K, cost_t, idx_t, val_t)
            b.record()
        torch.cuda.synchronize()
        ms = np.array([a.elapsed_time(b) for a, b in evs])
        for _ in range(20):
            cm.cm_step_run(step, batch0, None, K, cost_t, idx_t, val_t)
            kern.append(cm.cm_step_kernel_time(step))
        cost0 = cost_t.cpu().numpy()
        idx0 = idx_t.cpu().numpy().reshape(-1, K)
        val0 = val_t.cpu().numpy().reshape(-1, K)
        sel_exact, hit, tot, max_rel, off = True, 0, 0, 0.0, 0
        for j, q in enumerate(W.queries):
            c = cost0[off:off + q.n_cands]
            off += q.n_cands
            oi, ov = oracle.select(c.astype(np.float64), K)
            sel_exact &= bool(np.array_equal(oi, idx0[j]) and
                              np.array_equal(ov.astype(np.float32).view(np.uint32),
                                             val0[j].view(np.uint32)))
            r = oracle.eval_query(params, q.pipe, q.sched, q.terms)
            kk = min(K, len(r))
            sg = set(np.lexsort((np.arange(len(r)), c.astype(np.float64)))[:kk].tolist())
            sr = set(np.lexsort((np.arange(len(r)), r))[:kk].tolist())
            hit += len(sg & sr)
            tot += kk
            max_rel = max(max_rel, float(np.max(np.abs(c - r) / r)))
        ragged = {"workload": "ragged_17q", "queries": nq, "candidates": W.n_cands,
                  "rows": W.n_rows, "step_us_p50": float(np.percentile(ms, 50) * 1e3),
                  "step_us_p99": float(np.percentile(ms, 99) * 1e3),
                  "candidates_per_s": W.n_cands / (float(np.median(ms)) * 1e-3),
                  "kernel_us": float(np.median(kern)), "config": cfg, "autotune_us": tuned_us,
                  "selection_bit_exact": sel_exact, "top32_agreement_vs_fp64": hit / tot,
                  "top32_hits": [hit, tot], "max_rel_err_vs_fp64": max_rel}
        log(f"ragged_17q step: p50 {ragged['step_us_p50']:.1f} us (kernel {ragged['kernel_us']:.1f} us), "
            f"selection bit-exact={sel_exact}, top-32 agreement {hit}/{tot}")
        step.close()

    # ------------------------------------------------------------ cpu baseline
    cpu = None
    if not args.no_cpu_baseline:
        # a bounded sample of the serving workload: the first request of 8
        # sessions (bf16 features widened to float32), FP64 evaluation +
        # stable selection, on every thread of this process and on one
        import oracle
        n_s = sum(x[1].shape[1] for x in sample)
        rows_s = sum(x[1].shape[0] * x[1].shape[1] for x in sample)
        nproc, cpu_model = host_cpu()

        def timed_oracle(nthreads, seconds):
            reps, t_start = 0, time.perf_counter()
            while reps == 0 or time.perf_counter() - t_start < seconds:
                for pipe, sched, terms in sample:
                    oracle.select(oracle.eval_query(params, pipe, sched, terms, nthreads=nthreads), K)
                reps += 1
            return reps, time.perf_counter() - t_start

        threads = oracle.lib().max_threads()
        reps_all, dt_all = timed_oracle(0, args.cpu_seconds)
        reps_one, dt_one = timed_oracle(1, args.cpu_seconds)
        cpu = {"value": reps_all * n_s / dt_all, "unit": "candidates/s",
               "cores": threads, "kind": "oracle",
               "sample": f"8 serving requests ({n_s} candidates, {rows_s} rows), FP64 "
                         f"evaluation + stable selection, {reps_all} passes in {dt_all:.1f} s "
                         f"on {threads} threads",
               "single_thread": {"value": reps_one * n_s / dt_one, "unit": "candidates/s",
                                 "cores": 1, "passes": reps_one, "seconds": dt_one},
               "rows_per_s": reps_all * rows_s / dt_all,
               "host": {"nproc": nproc, "cpu_model": cpu_model}}
        log(f"cpu oracle: {cpu['value']:.0f} candidates/s on {threads} threads, "
            f"{cpu['single_thread']['value']:.0f} on 1 ({cpu_model}, nproc {nproc})")

    # ------------------------------------------------------------ bf16 vs fp8
    precision = None
    if not args.no_precision:
        W3 = workload("precision_65536x64")
        q3 = W3.queries[0]
        S3, N3 = q3.n_stages, q3.n_cands
        log("precision_65536x64: FP64 oracle for the agreement figures")
        ref3 = oracle.eval_query(params, q3.pipe, q3.sched, q3.terms)
        top_ref = set(np.lexsort((np.arange(N3), ref3))[:K].tolist())
        s_in, s_h = cm.cm_fp8_calibrate(model, np.repeat(q3.pipe, 256, axis=0),
                                        q3.sched[:, :256].reshape(-1, 40))
        cm.cm_model_prepare_fp8(model, s_in, s_h)
        ws3 = cm.cm_workspace_create(1, S3, N3, S3 * N3, K)
        i3 = torch.empty(K, dtype=torch.int32, device=dev)
        v3 = torch.empty(K, device=dev)

        def timed(fn, reps=30):
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / reps * 1e3  # us

        precision = {"workload": "precision_65536x64", "stages": S3, "candidates": N3,
                     "rows": S3 * N3, "k": K, "fp8_scales": {"s_in": s_in, "s_h": s_h}}
        for pname, row_bytes in (("bf16", 80 + 32), ("fp8", 40 + 32)):
            b3, c3 = cm.pack_queries([q3], pname, dev, in_scale=s_in)
            us_eval = timed(lambda: cm.cm_eval_batch(model, pname, b3, ws3, c3))
            us_call = timed(lambda: (cm.cm_eval_batch(model, pname, b3, ws3, c3),
                                     cm.cm_topk_per_query(c3, b3, K, ws3, i3, v3)))
            g3 = c3.cpu().numpy()[:N3].astype(np.float64)
            top = set(i3.cpu().numpy().tolist())
            precision[pname] = {
                "eval_us": us_eval, "eval_topk_us": us_call,
                "rows_per_s": S3 * N3 / (us_eval * 1e-6),
                "candidates_per_s": N3 / (us_call * 1e-6),
                "eval_gb_per_s": S3 * N3 * row_bytes / (us_eval * 1e3),
                "bytes_per_row": row_bytes,
                "top32_agreement_vs_fp64": len(top & top_ref) / K,
                "median_rel_err_vs_fp64": float(np.median(np.abs(g3 - ref3) / ref3))}
            log(f"precision_65536x64 {pname}: eval {us_eval:.1f} us "
                f"({precision[pname]['eval_gb_per_s']:.0f} GB/s), eval+top-k {us_call:.1f} us, "
                f"top-32 agreement {len(top & top_ref)}/{K}")
            del b3, c3
        x3 = torch.from_numpy(np.ascontiguousarray(q3.sched).ravel()).to(dev)
        codes3 = torch.empty(x3.numel(), dtype=torch.uint8, device=dev)
        us_enc = timed(lambda: cm.cm_fp8_encode(x3, s_in, codes3))
        precision["fp8_encode"] = {"us": us_enc, "gb_per_s": x3.numel() * 5 / (us_enc * 1e3)}
        del x3, codes3
        ws3.close()

    # ------------------------------------------------------------ fp8 serving
    # The same sessions and steps served in the FP8 form (e4m3 features,
    # weights and hidden activations; scales calibrated on a sample of the
    # serving inputs): context for the bf16 headline, whose agreement bar the
    # FP8 form's quantization does not meet (see the precision section).
    fp8_serving = None
    if not args.no_fp8_serving:
        # an auxiliary figure: a failure here is recorded, not fatal to the line
        try:
            t_f8 = time.perf_counter()
            rows_p, rows_x = [], []
            for S_, pipe_, reqs_ in sess_in[:32]:
                x_ = reqs_[0][1].float().reshape(S_, reqs_[0][0], 40)[:, :64].cpu().numpy()
                rows_x.append(x_.reshape(-1, 40))
                rows_p.append(np.repeat(pipe_, x_.shape[1], axis=0))
            f8_in, f8_h = cm.cm_fp8_calibrate(model, np.concatenate(rows_p), np.concatenate(rows_x))
            cm.cm_model_prepare_fp8(model, f8_in, f8_h)
            codes_in = []  # per session: [(N, e4m3 codes, terms), ...]
            for S_, pipe_, reqs_ in sess_in:
                codes_in.append([(N_, cm.cm_fp8_encode(x_.float().contiguous(), f8_in), t_)
                                 for N_, x_, t_, _ in reqs_])
            torch.cuda.synchronize()
            srv8 = cm.cm_server_create(model, k=K, arena_bytes=16 << 30, max_slots=args.slots,
                                       max_pending=8192, max_sessions=SESSIONS, max_stages=128,
                                       max_batch_queries=args.max_batch_queries,
                                       max_batch_cands=1 << 20, precision="fp8")
            sids8 = np.array([srv8.session_open(pipe_) for _, pipe_, _ in sess_in], np.int32)
            pre8 = []
            for j in range(args.inputs_per_session):
                pre8.append((np.array([codes_in[s_][j][0] for s_ in range(SESSIONS)], np.int32),
                             np.array([codes_in[s_][j][1].data_ptr() for s_ in range(SESSIONS)],
                                      np.uint64),
                             np.array([codes_in[s_][j][2].data_ptr() for s_ in range(SESSIONS)],
                                      np.uint64)))

            def run8(n):
                depth = max(1, args.queue_depth)
                q8 = [srv8.submit_batch(sids8, *pre8[i % len(pre8)], K) for i in range(min(depth, n))]
                for i in range(n):
                    srv8.wait_all(q8.pop(0), 120000)
                    if i + depth < n:
                        q8.append(srv8.submit_batch(sids8, *pre8[(i + depth) % len(pre8)], K))

            t_s8 = time.perf_counter()
            while (time.perf_counter() - t_s8) * 1e3 < args.settle_ms:
                run8(10)
            run8(args.warmup)
            torch.cuda.synchronize()
            srv8.reset_stats()
            n8 = max(20, args.steps // 2)
            t0_8 = time.perf_counter()
            run8(n8)
            torch.cuda.synchronize()
            wall8 = time.perf_counter() - t0_8
            st8 = srv8.stats()
            cands8 = sum(steps_pre[i % len(steps_pre)][3] for i in range(n8))
            rows8 = sum(steps_pre[i % len(steps_pre)][4] for i in range(n8))
            bytes8 = rows8 * (40 + 32) + cands8 * BYTES_PER_CAND_OUT
            dev8 = st8["kernel_busy_us"] if st8["kernel_busy_launches"] == st8["micro_batches"] else st8["kernel_us"]
            fp8_serving = {"candidates_per_s": cands8 / wall8, "steps": n8,
                           "ms_per_step": wall8 / n8 * 1e3,
                           "bytes_per_row": 40 + 32,
                           "kernel": "k_step_fp8",
                           "achieved_gb_per_s": bytes8 / (dev8 * 1e-6) / 1e9 if dev8 else None,
                           "frac_of_hbm_peak": bytes8 / (dev8 * 1e-6) / 1e9 / HBM_PEAK_GBS if dev8 else None,
                           "launches": st8["micro_batches"],
                           "algorithmic_bytes_per_launch": bytes8 / max(1, st8["micro_batches"]),
                           "device_us_per_launch": dev8 / max(1, st8["micro_batches"]),
                           "scales": {"s_in": f8_in, "s_h": f8_h},
                           "seconds": time.perf_counter() - t_f8}
            srv8.close()
            del codes_in
            log(f"fp8 serving: {fp8_serving['candidates_per_s']:.3e} candidates/s, "
                f"{fp8_serving['achieved_gb_per_s']:.0f} GB/s of algorithmic bytes")
        except Exception as exc:  # noqa: BLE001
            fp8_serving = {"error": f"{type(exc).__name__}: {exc}"}
            log(f"fp8 serving failed: {exc}")

    # ------------------------------------------------------------ fp32 plain
    fp32 = None
    if not args.no_fp32:
        W2 = workload("beam_6400x30")
        bq, cq = cm.pack_queries(W2.queries, "fp32", dev)
        q2 = W2.queries[0]
        ws2 = cm.cm_workspace_create(1, q2.n_stages, q2.n_cands, q2.n_stages * q2.n_cands, K)
        i2 = torch.empty(K, dtype=torch.int32, device=dev)
        v2 = torch.empty(K, device=dev)
        for _ in range(5):
            cm.cm_eval_batch(model, "fp32", bq, ws2, cq)
            cm.cm_topk_per_query(cq, bq, K, ws2, i2, v2)
            torch.cuda.synchronize()
        reps = 50
        t2 = time.perf_counter()
        for _ in range(reps):
            cm.cm_eval_batch(model, "fp32", bq, ws2, cq)
            cm.cm_topk_per_query(cq, bq, K, ws2, i2, v2)
            torch.cuda.synchronize()
        dt2 = time.perf_counter() - t2
        r2 = oracle.eval_query(params, q2.pipe, q2.sched, q2.terms)
        rel2 = float(np.max(np.abs(cq.cpu().numpy() - r2) / r2))
        fp32 = {"workload": "beam_6400x30", "candidates_per_s": reps * q2.n_cands / dt2,
                "ms_per_call": dt2 / reps * 1e3, "max_rel_err_vs_fp64": rel2}
        log(f"fp32 plain: {fp32['candidates_per_s']:.3e} candidates/s, max rel err {rel2:.1e}")
        ws2.close()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "serving_256_sessions_saturated", "sessions": SESSIONS,
                   "queries_per_step": SESSIONS, "k": K,
                   "stages": "log-uniform [3, 120] per session",
                   "candidates": "uniform [16, 4096] per query",
                   "inputs_per_session": args.inputs_per_session,
                   "input_gb": round(in_bytes / 1e9, 2), "slots": args.slots,
                   "queue_depth_steps": args.queue_depth,
                   "max_batch_queries": args.max_batch_queries},
        "rows_per_s": rows / wall,
        # algorithmic bytes of every timed launch over the timed wall time:
        # the device-level rate, which counts the overlap of consecutive
        # micro-batches that a launch's own duration cannot
        "aggregate_gb_per_s": st["kernel_bytes"] / wall / 1e9,
        "latency": latency,
        "settle_before_warmup": settle,
        "serving_cold": cold,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if tr is None else tr["bytes_per_launch"],
                     "kernel": "k_step_bf16", "avg_launch_us": avg_us, "launch_time": launch_time,
                     "avg_launch_own_span_us": own_us,
                     "frac_of_own_span": bytes_per_launch / (own_us * 1e3) / HBM_PEAK_GBS if own_us else None,
                     "device_idle_us_per_launch": idle_us,
                     "algorithmic_bytes_per_launch": bytes_per_launch, "launches": launches,
                     "measured_read_gbs": None if read_roof is None else read_roof[0],
                     "frac_of_measured_read": None if read_roof is None else achieved / read_roof[0]},
        "cpu_baseline": cpu,
        "fp32_plain": fp32,
        "fp8_serving": fp8_serving,
        "bf16_over_fp32_plain": None if fp32 is None else value / fp32["candidates_per_s"],
        "serving_step_tuning": tune,
        "ragged_step": ragged,
        "precision": precision,
        "serving_agreement": agree,
        "top32_agreement_vs_fp64": None if agree is None else agree["vs_fp64_f32_inputs"],
        "selection_bit_exact": None if ragged is None else ragged["selection_bit_exact"],
    }
    print(json.dumps(out), flush=True)
    model.close()


if __name__ == "__main__":
    main()
