"""Benchmark: decoded windows/s and window latency of sliding-window GDG on
[[144,12,12]] under circuit-level noise, one MI355X.

A step is one pass of the whole decoder over one batch of synthetic shots:
for every (3,1) window in turn, decode (preprocessing BP, ranking and
truncation, peeling, 16 decision paths, path metric) and commit, then the
Eq. 8 / Eq. 9 evaluation. Shots are sampled on the GPU from the circuit-level
DEM before the timed region; every step decodes a fresh batch.

Prints one JSON line: the metric, windows/s over the timed steps, window
latencies, the logical error rate, the decode kernel's LDS roofline (16 B per
edge-iteration against 157.3 TB/s, with the HBM traffic per launch from the
rocprofv3 summary when it matches the kernel source), the LDS rates the probe
kernels reach, and the FP64 oracle's rate on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402


# 256 CUs x 256 B/clk x 2.4 GHz = 157286 GB/s of LDS reads: the LDS probe's 16 KiB
# b64/b128 reads reach 129.5 TB/s, above what 128 B/clk per CU (78.6 TB/s) allows
LDS_PEAK_GBS = 256 * 256 * 2.4
BYTES_PER_EDGE_ITER = 16         # one FP32 message written and read each way


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shots", type=int, default=100000, help="shots per step")
    ap.add_argument("--p", type=float, default=0.002)
    ap.add_argument("--code", default="144")
    ap.add_argument("--rounds", type=int, default=12)
    ap.add_argument("--g", type=int, default=4)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget for the oracle CPU baseline (0 = skip)")
    ap.add_argument("--latency-windows", type=int, default=110,
                    help="single-shot windows timed for the latency figures")
    ap.add_argument("--warm", type=int, default=1,
                    help="also time the same steps with cross-window message reuse (0: skip)")
    ap.add_argument("--lds-probe", type=int, default=1,
                    help="also measure the LDS bandwidth with the probe kernels (0: skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    ap.add_argument("--workload", choices=["c2", "c1", "mixed", "stream", "learned"], default="c2",
                    help="c2: [[144,12,12]] (the headline); mixed: five BB codes in shared "
                         "persistent launches with the autotuner; stream: the streaming "
                         "service over 256 [[144]] + 32 [[288]] blocks; learned: the "
                         "learned proposer against plain GDG on held-out shots")
    ap.add_argument("--stream-sat-s", type=float, default=0.3,
                    help="virtual seconds of the saturated streaming run")
    ap.add_argument("--stream-s", type=float, default=0.6,
                    help="virtual seconds of the 80%%-load streaming run")
    ap.add_argument("--stream-chain", type=int, default=-1,
                    help="windows of one experiment per tick: -1 one per tick with separate "
                         "launches and commits, 0 all decodable (chained launch), n at most n")
    ap.add_argument("--stream-decouple", type=int, default=1,
                    help="1: each code runs its own ticks on its own stream and clock")
    ap.add_argument("--stream-waves", default="4,8",
                    help="wavefronts per workgroup of the streaming launches: one count, "
                         "or one per code ([[144]],[[288]]), e.g. 4,8")
    ap.add_argument("--stream-wpc", default="0",
                    help="persistent workgroups per CU of the streaming launches (0: one "
                         "workgroup per shot): one count, or one per code")
    ap.add_argument("--stream-mem-mib", type=float, default=0.0,
                    help="device memory budget of the streaming service's experiment "
                         "slots in MiB (0: a quarter of the free memory, at most 1 GiB)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the decoder shards "
              "shots across GPUs with no communication (each GPU its own shot range)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "mixed":
        return bench_mixed(args)
    if args.workload == "stream":
        return bench_stream(args)
    if args.workload == "learned":
        return bench_learned(args)
    import torch
    from gdg_inputs.bb import get_code
    from gdg_inputs.dem import circuit_dem, phenomenological_dem
    import paper_2403_18901_amd.gdg as G

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    c1 = args.workload == "c1"
    if c1:
        # [[72,12,6]] phenomenological, p = q = 0.005, 6 noisy rounds: the main
        # path only (plain BPGD, no preprocessing), alpha = 0.625
        code = get_code("72")
        dem = phenomenological_dem(code, 6, 0.005, 0.005)
        low_error = 1
        prm = G.params(alpha=0.625, g=0, pre_iters=0, low_error=1, dmax_main=25)
    else:
        code = get_code(args.code)
        dem = circuit_dem(code, args.rounds, args.p)
        low_error = 1 if args.p <= 0.002 else 0
        prm = G.params(alpha=1.0, g=args.g, pre_iters=8, trunc_factor=2, low_error=low_error,
                       dmax_main=25, extra_steps=10)
    dec = G.SlidingWindowDecoder(dem, prm, W=3)
    ddem = G.DeviceDem(dem)
    B = args.shots
    nwin = dec.n_windows
    n_batches = args.warmup + args.steps
    batches = []
    for i in range(n_batches):
        det, obs = ddem.sample(B, seed=args.seed, stream=0, shot0=i * B, device=dev)
        batches.append((det, obs))
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ehat_bufs = [torch.empty((B, w.n), dtype=torch.uint8, device=dev) for w in dec.windows]
    pm_buf = torch.empty(B, dtype=torch.float64, device=dev)
    fl_buf = torch.empty(B, dtype=torch.int32, device=dev)
    fail_buf = torch.empty(B, dtype=torch.uint8, device=dev)
    edge_buf = torch.empty(B, dtype=torch.int64, device=dev)

    def run_step(det, obs, events=None, edge_sum=None):
        for k, w in enumerate(dec.windows):
            if events is not None:
                events[k][0].record(stream)
            trace = G.Trace(None, None, 0, None, None, G._ptr(edge_buf), None)
            G._check(G.lib().gdg_decode_batch(w.h, B, G._ptr(det, w.row0), det.shape[1],
                                               G._ptr(ehat_bufs[k]), G._ptr(pm_buf),
                                               G._ptr(fl_buf), None, 0, G.C.byref(trace),
                                               G._stream()))
            if events is not None:
                events[k][1].record(stream)
            if edge_sum is not None:
                edge_sum.append(edge_buf.sum())
            w.commit(ehat_bufs[k], det, obs)
            if events is not None:
                events[k][2].record(stream)
        G.evaluate(det, obs, out=fail_buf)
        return fail_buf.sum()

    for i in range(args.warmup):
        run_step(*batches[i])
    torch.cuda.synchronize()

    all_events = []
    edge_sums = []
    fails = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, n_batches):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(nwin)]
        all_events.append(ev)
        fails.append(run_step(*batches[i], events=ev, edge_sum=edge_sums))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    windows = args.steps * B * nwin
    value = windows / elapsed
    dec_ms = [ev[k][0].elapsed_time(ev[k][1]) for ev in all_events for k in range(nwin)]
    win_ms = [ev[k][0].elapsed_time(ev[k][2]) for ev in all_events for k in range(nwin)]
    edge_iters = int(sum(int(x.item()) for x in edge_sums))
    n_fail = int(sum(int(f.item()) for f in fails))
    shots = args.steps * B
    P_L = n_fail / shots
    ler_round = 1.0 - (1.0 - P_L) ** (1.0 / args.rounds) if P_L < 1 else 1.0

    # roofline of the decode kernel: algorithmic LDS bytes per launch / mean launch time
    mean_dec_s = float(np.mean(dec_ms)) / 1e3
    launches = len(dec_ms)
    bytes_per_launch = BYTES_PER_EDGE_ITER * edge_iters / launches
    achieved_gbs = bytes_per_launch / mean_dec_s / 1e9

    # the same steps again with cross-window message reuse (each window's
    # preprocessing BP starts from the messages the previous one handed over)
    warm = None
    if args.warm and not c1:
        for k in range(1, nwin):
            dec.windows[k].link(dec.windows[k - 1])
        slots = max(w.n_msg for w in dec.windows)
        wbuf = [torch.empty((B, slots), dtype=torch.float32, device=dev) for _ in range(2)]
        wb = []
        for i in range(args.warmup, n_batches):   # the timed steps' shots, sampled again
            det, obs = ddem.sample(B, seed=args.seed, stream=0, shot0=i * B, device=dev)
            wb.append((det, obs))

        def warm_step(det, obs, edge_sum):
            for k, w in enumerate(dec.windows):
                trace = G.Trace(None, None, 0, None, None, G._ptr(edge_buf), None)
                win_in = wbuf[(k + 1) % 2] if k > 0 else None
                win_out = wbuf[k % 2] if k + 1 < nwin else None
                G._check(G.lib().gdg_decode_batch_warm(
                    w.h, B, G._ptr(det, w.row0), det.shape[1], G._ptr(win_in), slots,
                    G._ptr(win_out), slots, G._ptr(ehat_bufs[k]), G._ptr(pm_buf),
                    G._ptr(fl_buf), None, 0, G.C.byref(trace), G._stream()))
                edge_sum.append(edge_buf.sum())
                w.commit(ehat_bufs[k], det, obs)
            G.evaluate(det, obs, out=fail_buf)
            return fail_buf.sum()

        warm_step(*batches[0], [])   # first launches of the warm path
        torch.cuda.synchronize()
        w_edges, w_fails = [], []
        tw0 = time.perf_counter()
        for det, obs in wb:
            w_fails.append(warm_step(det, obs, w_edges))
        torch.cuda.synchronize()
        tw = time.perf_counter() - tw0
        w_ei = int(sum(int(x.item()) for x in w_edges))
        warm = {"value": windows / tw, "unit": "windows/s", "ms_per_step": tw * 1e3 / args.steps,
                "failures": int(sum(int(f.item()) for f in w_fails)), "shots": shots,
                "edge_iters_per_window": w_ei / windows,
                "cold_edge_iters_per_window": edge_iters / windows,
                "note": "same shots as the timed steps; Sec. V's message reuse, not the "
                        "paper's decoder"}

    # single-shot window latency (one window of one shot, decode + commit)
    lat = []
    if args.latency_windows > 0:
        det1, obs1 = ddem.sample(max(1, args.latency_windows // nwin + 1), seed=args.seed + 1,
                                 stream=1, device=dev)
        torch.cuda.synchronize()
        for s in range(det1.shape[0]):
            d = det1[s:s + 1].contiguous()
            o = obs1[s:s + 1].contiguous()
            for k, w in enumerate(dec.windows):
                if len(lat) >= args.latency_windows:
                    break
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                eh, _, _ = w.decode(d, syn_offset=w.row0)
                w.commit(eh, d, o)
                e1.record(stream)
                e1.synchronize()
                lat.append(e0.elapsed_time(e1))

    probe = lds_probe(dev) if args.lds_probe else None

    if args.copy_probe:
        # plain copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters
        src = torch.empty(256 * 1024 * 1024, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(dem, args, nwin, c1)

    # LDS accesses the counters saw per edge-iteration (wavefront LDS
    # instructions, at most 64 lanes x 4 B each): the roofline counted from
    # the hardware side, an upper bound on the LDS bytes moved
    lds_counted = None
    lpath = os.path.join(ROOT, "profiles", "decode_lds.txt")
    if not c1 and os.path.exists(lpath):
        with open(lpath) as f:
            t = json.load(f)
        if t.get("kernel_hash") == kernel_hash():
            bpe = t["lds_instr_per_edge_iter"] * t["bytes_per_lds_instr_max"]
            gbs = bpe * edge_iters / launches / mean_dec_s / 1e9
            lds_counted = {"bytes_per_edge_iter_max": bpe, "gbs_max": gbs,
                           "frac_max": gbs / LDS_PEAK_GBS}
            if "valu_instr_per_edge_iter" in t:
                # VALU issue: a wavefront instruction holds a 16-lane SIMD for
                # four clocks; 1024 SIMDs at 2.4 GHz
                ipe = t["valu_instr_per_edge_iter"]
                rate = ipe * edge_iters / launches / mean_dec_s
                lds_counted["valu_instr_per_edge_iter"] = ipe
                lds_counted["valu_issue_frac"] = rate * 4 / (1024 * 2.4e9)

    traffic = None
    tpath = os.path.join(ROOT, "profiles", "decode_traffic.txt")
    if not c1 and os.path.exists(tpath):   # the summary covers the C2 workload
        with open(tpath) as f:
            t = json.load(f)
        if t.get("kernel_hash") == kernel_hash():
            traffic = t["bytes_per_shot"] * B

    out = {
        "metric": ("decoded windows/s and p99 window latency, [[72,12,6]] phenomenological "
                   "BPGD (main path)" if c1 else
                   "decoded windows/s and p99 window latency, [[144,12,12]] GDG at matched LER"),
        "value": value,
        "unit": "windows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"BPGD main path (alpha 0.625), [[72,12,6]] phenomenological "
                         f"p=q=0.005, 6 rounds, (3,1) windows x {nwin} per shot, {B} shots "
                         f"per step, FP32 messages" if c1 else
                         f"GDG g={args.g} ({1 << args.g} paths), [[{code.n},12,12]] "
                         f"circuit-level p={args.p}, {args.rounds} rounds, (3,1) windows "
                         f"x {nwin} per shot, {B} shots per step, FP32 messages"),
            "code": code.name, "p": 0.005 if c1 else args.p, "rounds": 6 if c1 else args.rounds,
            "W": 3, "F": 1, "shots_per_step": B, "windows_per_shot": nwin,
            "low_error_mode": bool(low_error), "pre_iters": 0 if c1 else 8,
            "n_act": dec.windows[1].n_act,
            "waves_per_workgroup": dec.windows[1].info["waves"],
            "lds_bytes": dec.windows[1].info["lds_bytes"],
        },
        "latency_ms": {
            "batch_window_p50": float(np.percentile(win_ms, 50)),
            "batch_window_p99": float(np.percentile(win_ms, 99)),
            "single_window_p50": float(np.percentile(lat, 50)) if lat else None,
            "single_window_p99": float(np.percentile(lat, 99)) if lat else None,
            "single_window_max": float(np.max(lat)) if lat else None,
            "paper_context_worst_case_cpu": 3.0,
        },
        "ler": {"shots": shots, "failures": n_fail, "P_L": P_L, "per_round": ler_round},
        "edge_iters_per_s": edge_iters / (float(np.sum(dec_ms)) / 1e3),
        "roofline": {
            "bound": "lds",
            "achieved": achieved_gbs,
            "peak": LDS_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / LDS_PEAK_GBS,
            "traffic": traffic,
            # the counted HBM bytes as a rate, against HBM's 8 TB/s
            "traffic_gbs": traffic / mean_dec_s / 1e9 if traffic else None,
            "traffic_frac_hbm": traffic / mean_dec_s / 8e12 if traffic else None,
            "lds_counted": lds_counted,
            "kernel": "gdg_decode_kernel",
            "mean_launch_ms": mean_dec_s * 1e3,
            "edge_iters_per_launch": edge_iters / launches,
        },
        "cpu_baseline": cpu,
        "warm_start": warm,
        "lds_probe_gbs": probe,
    }
    print(json.dumps(out))


def bench_mixed(args):
    """Five BB codes ([[72]], [[90]], [[108]], [[144]], [[288]]), circuit-level
    noise, d rounds each, g = 4: every window step decodes all codes still in
    range in shared persistent launches whose shape the autotuner picked.
    Compared with decoding the codes one after another at the default shape."""
    import torch
    from gdg_inputs.bb import CODE_D, get_code
    from gdg_inputs.dem import circuit_dem
    import paper_2403_18901_amd.batched as Bt
    import paper_2403_18901_amd.gdg as G

    dev = torch.device("cuda:0")
    keys = ["72", "90", "108", "144", "288"]
    B = args.shots
    low = 1 if args.p <= 0.002 else 0
    prm = G.params(alpha=1.0, g=args.g, pre_iters=8, trunc_factor=2, low_error=low)
    dems = [circuit_dem(get_code(k), CODE_D[k], args.p) for k in keys]
    # [[288,12,18]] with the paper's N = 288 settings (Sec. IV-C), the others g = args.g
    prms = [prm if k != "288" else G.paper_params(288, args.p) for k in keys]
    md = Bt.MixedDecoder(dems, prms)
    ddems = [G.DeviceDem(d) for d in dems]

    def batch(i):
        out = [dd.sample(B, seed=args.seed, stream=c, shot0=i * B, device=dev)
               for c, dd in enumerate(ddems)]
        return [o[0] for o in out], [o[1] for o in out]

    t = time.perf_counter()
    dets, _ = batch(0)
    plan, timings = md.tune(dets, reps=2)
    tune_s = time.perf_counter() - t
    n_windows = sum(d.n_windows for d in md.decoders) * B
    batches = [batch(i + 1) for i in range(args.warmup + 3 * args.steps)]
    outs = md.alloc(batches[0][0])
    torch.cuda.synchronize()
    for i in range(args.warmup):
        md.decode(*batches[i], outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fails = []
    for i in range(args.warmup, args.warmup + args.steps):
        fails.append(md.decode(*batches[i], outs=outs))
    torch.cuda.synchronize()
    mixed_s = time.perf_counter() - t0
    # baseline: codes one after another, one window per launch, default shape
    t0 = time.perf_counter()
    for i in range(args.warmup + args.steps, args.warmup + 2 * args.steps):
        dets, obss = batches[i]
        for c, dec in enumerate(md.decoders):
            dec.decode(dets[c], obss[c])
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    # alternative: each code's whole window sequence on a stream of its own
    # (default launch shape), the codes running concurrently
    streams = [torch.cuda.Stream(device=dev) for _ in keys]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup + 2 * args.steps, args.warmup + 3 * args.steps):
        dets, obss = batches[i]
        for c, dec in enumerate(md.decoders):
            with torch.cuda.stream(streams[c]):
                dec.decode(dets[c], obss[c])
    torch.cuda.synchronize()
    streams_s = time.perf_counter() - t0
    per_code = {}
    for c, k in enumerate(keys):
        nf = int(sum(int(f[c].sum().item()) for f in fails))
        per_code[get_code(k).name] = {"rounds": CODE_D[k], "windows_per_shot": md.decoders[c].n_windows,
                                      "failures": nf, "shots": args.steps * B}
    out = {
        "metric": "decoded windows/s, mixed BB codes in shared persistent launches",
        "value": n_windows * args.steps / mixed_s,
        "unit": "windows/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": mixed_s * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"[[72]], [[90]], [[108]], [[144]], [[288]] circuit-level p={args.p}, "
                               f"d rounds, (3,1) windows, g={args.g}, {B} shots per code per step",
                   "plan": repr(plan), "autotune_s": tune_s,
                   "autotune_ms": {str(k): v for k, v in timings.items()}},
        "sequential_windows_per_s": n_windows * args.steps / seq_s,
        "per_code_streams_windows_per_s": n_windows * args.steps / streams_s,
        "speedup_vs_sequential": seq_s / mixed_s,
        "per_code": per_code,
    }
    print(json.dumps(out))


def bench_stream(args):
    """Streaming service: 256 [[144,12,12]] blocks (12 noisy rounds) and 32
    [[288,12,18]] blocks (18), circuit-level p, Poisson round arrivals. First at
    one round per microsecond per block (far above capacity: reports the
    sustained rate, backlog growth and admission rejections), then at 80%, 50%
    and 10% of the capacity measured there (reports p50/p99 window latency)."""
    import torch
    from gdg_inputs.bb import get_code
    from gdg_inputs.dem import circuit_dem
    import paper_2403_18901_amd.gdg as G
    import paper_2403_18901_amd.stream as S

    low = 1 if args.p <= 0.002 else 0
    prm = G.params(alpha=1.0, g=args.g, pre_iters=8, trunc_factor=2, low_error=low)
    dems = [(circuit_dem(get_code("144"), 12, args.p), 256), (circuit_dem(get_code("288"), 18, args.p), 32)]
    wins_per_round = sum(nb * (d.n_rounds - 2) / d.n_rounds for d, nb in dems)
    t = time.perf_counter()
    budget = int(args.stream_mem_mib * 2**20) if args.stream_mem_mib > 0 else None
    import paper_2403_18901_amd.batched as BT
    waves = [int(x) for x in str(args.stream_waves).split(",")]
    if len(waves) == 1:
        waves = waves * len(dems)
    if len(waves) != len(dems) or any(w not in (2, 4, 8) for w in waves):
        raise SystemExit("--stream-waves: 2, 4 or 8, once or once per code")
    wpcs = [int(x) for x in str(args.stream_wpc).split(",")]
    if len(wpcs) == 1:
        wpcs = wpcs * len(dems)
    if len(wpcs) != len(dems) or any(not 0 <= x <= 8 for x in wpcs):
        raise SystemExit("--stream-wpc: 0..8, once or once per code")
    chain = dict(chain=args.stream_chain >= 0, chain_max=max(args.stream_chain, 0),
                 plan=[BT.LaunchPlan(waves=w, wg_per_cu=x, split=True)
                       for w, x in zip(waves, wpcs)],
                 decouple=bool(args.stream_decouple))
    sat = S.StreamingService(dems, prm, rate=1e6, n_slots=None, seed=args.seed,
                             mem_budget=budget, **chain)
    rep_sat = sat.run(duration=args.stream_sat_s)
    wall_sat = time.perf_counter() - t
    cap = rep_sat["windows_per_s"]
    loads = {}
    for frac in (0.8, 0.5, 0.1):
        rate = frac * cap / wins_per_round
        t = time.perf_counter()
        svc = S.StreamingService(dems, prm, rate=rate, n_slots=None, seed=args.seed + 1,
                                 mem_budget=budget, **chain)
        rep = svc.run(duration=args.stream_s)
        loads[frac] = dict(rep, rate_rounds_per_s_per_block=rate, wall_s=time.perf_counter() - t)
    rep80, wall80, rate80 = loads[0.8], loads[0.8]["wall_s"], loads[0.8]["rate_rounds_per_s_per_block"]
    out = {
        "metric": "streaming decoded windows/s and p99 window latency at 80% load",
        "value": rep80["windows_per_s"], "unit": "windows/s",
        "n_gpus": 1, "steps": rep80["ticks"], "warmup": 0,
        "ms_per_step": rep80["virtual_s"] * 1e3 / max(rep80["ticks"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"256 x [[144,12,12]] (12 rounds) + 32 x [[288,12,18]] (18 rounds), "
                               f"circuit-level p={args.p}, g={args.g}, Poisson round arrivals, "
                               "virtual time advanced by measured device time",
                   "blocks": 288, "chain": args.stream_chain, "waves": waves, "wg_per_cu": wpcs,
                   "decouple": bool(args.stream_decouple)},
        "saturated_1_round_per_us": dict(rep_sat, wall_s=wall_sat),
        "load_80pct": rep80,
        "load_50pct": loads[0.5],
        "load_10pct": loads[0.1],
    }
    print(json.dumps(out))


def bench_learned(args):
    """Learned proposer (trained weights shipped with the package) against
    plain GDG on held-out [[144,12,12]] shots at p = 0.001, 0.002, 0.003:
    windows/s, batch window latency, BP work (edge-iterations per window) and
    logical failures, and the network's matrix-core throughput on its own."""
    import torch
    from gdg_inputs.bb import get_code
    from gdg_inputs.dem import circuit_dem
    import paper_2403_18901_amd.gdg as G
    import paper_2403_18901_amd.learned as LRN

    params = LRN.load(LRN.default_model_path("144"))
    B = args.shots
    rows = {}
    for p in (0.001, 0.002, 0.003):
        dem = circuit_dem(get_code("144"), 12, p)
        prm = G.params(alpha=1.0, g=args.g, pre_iters=8, trunc_factor=2, low_error=int(p <= 0.002))
        det0, obs0 = G.DeviceDem(dem).sample(B, seed=args.seed + 77, stream=11)
        plain = G.SlidingWindowDecoder(dem, prm)
        learned = LRN.LearnedSlidingWindowDecoder(dem, prm, params)
        row = {}
        for name, dec in (("plain", plain), ("learned", learned)):
            det, obs = det0.clone(), obs0.clone()
            dec.decode(det[:256].clone(), obs[:256].clone())   # warm-up
            torch.cuda.synchronize()
            lat = []
            t0 = time.perf_counter()
            wins = []
            fl_all = []
            ei = torch.zeros((dec.n_windows, B), dtype=torch.int64, device="cuda")
            for k, w in enumerate(dec.windows):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                if name == "plain":
                    eh = torch.empty((B, w.n), dtype=torch.uint8, device="cuda")
                    pm = torch.empty(B, dtype=torch.float64, device="cuda")
                    fl = torch.empty(B, dtype=torch.int32, device="cuda")
                    tr = G.Trace(None, None, 0, None, None, G._ptr(ei[k]), None)
                    G._check(G.lib().gdg_decode_batch(w.h, B, G._ptr(det, w.row0), det.shape[1],
                                                       G._ptr(eh), G._ptr(pm), G._ptr(fl), None,
                                                       0, G.C.byref(tr), G._stream()))
                else:
                    eh, pm, fl = G.decode_learned(w, det, w.row0, dec.cfg(ei[k]), dec.model,
                                                  dec.work)
                w.commit(eh, det, obs)
                e1.record()
                wins.append((e0, e1))
                fl_all.append(fl)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            lat = [a.elapsed_time(b) for a, b in wins]
            fail = int(G.evaluate(det, obs).sum().item())
            fb = float(torch.stack(fl_all).bitwise_and(8).ne(0).float().mean().item())
            row[name] = {"windows_per_s": B * dec.n_windows / dt, "failures": fail,
                         "P_L": fail / B, "batch_window_ms_p50": float(np.percentile(lat, 50)),
                         "batch_window_ms_p99": float(np.percentile(lat, 99)),
                         "fallback_frac": fb,
                         "edge_iters_per_window": float(ei.sum().item()) / (B * dec.n_windows)}
        row["speedup"] = row["learned"]["windows_per_s"] / row["plain"]["windows_per_s"]
        rows[str(p)] = row
    head = rows["0.002"]
    out = {
        "metric": "decoded windows/s, learned proposer vs plain GDG, [[144,12,12]] held-out shots",
        "value": head["learned"]["windows_per_s"], "unit": "windows/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": B * 11 / head["learned"]["windows_per_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": f"[[144,12,12]] circuit-level, 12 rounds, (3,1) windows, {B} "
                               "held-out shots per p; proposer 17-64-64-1 (BF16 inference), "
                               "learned tree of 4 paths (guesses at depths 1-2), plain GDG "
                               "(16 paths) fallback",
                   "value_at_p": 0.002},
        "by_p": rows,
    }
    # the proposer's network alone: BF16 matrix-core inference of 2^20 samples,
    # algorithmic MACs (17x64 + 64x64 + 64 per sample) against the dense BF16
    # peak (2.5 PFLOP/s = 1.25e15 MAC/s)
    model = G.Model(params)
    n = 1 << 20
    x = torch.rand((n, G.MLP_IN), device="cuda")
    model.infer(x)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        model.infer(x)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    macs = n * (G.MLP_IN * G.MLP_H + G.MLP_H * G.MLP_H + G.MLP_H)
    out["mlp_infer"] = {"samples": n, "ms": ms, "mac_per_s": macs / (ms * 1e-3),
                        "peak_mac_per_s": 1.25e15, "frac": macs / (ms * 1e-3) / 1.25e15}
    print(json.dumps(out))


def lds_probe(dev):
    """LDS GB/s of the probe kernels (4, 8, 16-byte reads on 32 and 16 KiB per
    workgroup; 4-byte writes), each timed with HIP events on the stream it is
    launched on, best of three after a first launch."""
    import ctypes as C
    import torch
    lib = C.CDLL(os.path.join(ROOT, "paper_2403_18901_amd", "libgdg_probe.so"))
    lib.lds_probe_launch.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    lib.lds_probe_bytes.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.lds_probe_bytes.restype = C.c_double
    n_blocks, reps = 256 * 20, 256
    sink = torch.empty(n_blocks * 256, dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream()
    out = {}
    for mode, name in ((0, "read_b32"), (1, "read_b64"), (2, "read_b128"), (3, "write_b32"),
                       (4, "read_b32_16k"), (5, "read_b64_16k"), (6, "read_b128_16k")):
        best = None
        for _ in range(4):   # the first launch also loads the code object
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            rc = lib.lds_probe_launch(mode, n_blocks, reps, C.c_void_p(sink.data_ptr()),
                                      C.c_void_p(st.cuda_stream))
            e1.record(st)
            e1.synchronize()
            if rc != 0:
                raise RuntimeError("LDS probe launch failed")
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        nbytes = lib.lds_probe_bytes(mode, n_blocks, reps)
        out[name] = nbytes / (best * 1e-3) / 1e9
    return out


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2403_18901_amd", "csrc", "gdg_kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def cpu_baseline(dem, args, nwin, c1=False):
    """The FP64 oracle on the host cores, on a bounded sample of the same workload."""
    from gdg_inputs.philox import sample_errors, syndromes
    from oracle import oracle as O
    threads = len(os.sched_getaffinity(0))
    if c1:
        op = O.params(alpha=0.625, g=0, pre_iters=0, low_error=1, dmax_main=25)
    else:
        op = O.params(alpha=1.0, g=args.g, pre_iters=8, trunc_factor=2,
                      low_error=1 if args.p <= 0.002 else 0)
    # calibrate on a small sample (large enough that building the windows does
    # not dominate), then size the sample to the time budget
    n0 = max(16 * threads, 256)
    e = sample_errors(dem.thresholds(), n0, seed=args.seed)
    det, obs = syndromes(dem, e)
    t = time.perf_counter()
    O.decode_shots(dem, 3, op, det, obs, n_threads=threads)
    dt = time.perf_counter() - t
    n = int(max(n0, min(20000, n0 * args.cpu_seconds / max(dt, 1e-3))))
    e = sample_errors(dem.thresholds(), n, seed=args.seed)
    det, obs = syndromes(dem, e)
    t = time.perf_counter()
    r = O.decode_shots(dem, 3, op, det, obs, n_threads=threads)
    dt = time.perf_counter() - t
    # single-thread latency of one window decode (the first window, one shot
    # per call, window built once)
    w0 = O.OracleWindow(dem, 0, 3)
    syn0 = np.ascontiguousarray(det[:, w0.row0:w0.row0 + w0.m])
    lat = []
    for i in range(min(200, n)):
        t1 = time.perf_counter()
        w0.decode(op, syn0[i:i + 1], n_threads=1)
        lat.append((time.perf_counter() - t1) * 1e3)
    return {"value": n * nwin / dt, "unit": "windows/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} shots x {nwin} windows of the same workload (first {n} shots of "
                      f"seed {args.seed}), {dt:.1f} s, {int(r['fail'].sum())} failures",
            "window_ms_p50": float(np.percentile(lat, 50)),
            "window_ms_p99": float(np.percentile(lat, 99)),
            "latency_sample": f"first window of the first {len(lat)} shots, one thread, "
                              "one shot per call"}


if __name__ == "__main__":
    main()
