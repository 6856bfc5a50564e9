#!/usr/bin/env python3
"""Benchmark: RZF precoder updates/s, WB-arSVD vs full inverse, K=64 N=256.

Workload: one synthetic LEO channel track, 16x16 half-wavelength UPA (N=256),
K=64 users in a 100 km disk, Rician K-factor 10 dB, SNR 10 dB, 1000 snapshots
10 ms apart, energy threshold eta = 0.999, FP64 drift re-inversion every 100
steps.  A step is one pass of the whole hot path on one snapshot: the update
(Gram correction, arSVD, Woodbury or direct inversion, precoder with power
normalisation) followed by the per-user SINR / sum rate.

Printed: one JSON line with the WB-arSVD throughput as `value`, the
full-inversion RZF baseline on the same GPU and snapshots, p50/p99 per-step
latency of both, the dominant kernel's roofline figure (HIP-event durations
of a second pass over the same steps) and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RZF precoder updates/s, WB-arSVD vs full inverse, K=64 N=256; p99 latency"
FP32_MFMA_PEAK_TFLOPS = 157.3
# FP32 vector peak without packed FP32 instructions (every HIP source is built
# with them off): 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6


def metric_for(cfg):
    """The headline metric string for a single-track configuration."""
    return f"RZF precoder updates/s, WB-arSVD vs full inverse, K={cfg.K} N={cfg.N}; p99 latency"


def kernel_flops(name, K, N):
    """Algorithmic real flops of one track's share of a GEMM-shaped kernel
    (8 per complex multiply-add): the Gram kernel forms A' (4 K^2 N, lower
    half) and Delta A (8 K^2 N, lower half); the precoder 8 K^2 N; the
    sum-rate tiles E = H W, 8 K^2 N."""
    return {"gram": 12.0 * K * K * N, "precoder": 8.0 * K * K * N, "sum_rate": 8.0 * K * K * N}.get(name)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2",
                    help="c2 (default), c1, c5 (K=256 N=1024 track) or mix (multi-track batch)")
    ap.add_argument("--eta", type=float, default=None)
    ap.add_argument("--policy", choices=["fixed", "warm"], default="fixed")
    ap.add_argument("--precision", choices=["fp32", "bf16", "bf16x3"], default="fp32",
                    help="operand format of the Gram and precoder products")
    ap.add_argument("--error-feedback", action="store_true",
                    help="policy: sketch Delta A plus the residual earlier truncations left out")
    ap.add_argument("--early-fallback", action="store_true",
                    help="policy: end Alg. 1 once d passes the Woodbury limit without success")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the oracle CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-switch", action="store_true",
                    help="Alg. 2's switch ratio from rzf_tune_switch (measured costs) instead of 0.5")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the eta sweep of the K=64 track")
    ap.add_argument("--sweep-steps", type=int, default=300)
    ap.add_argument("--batch-tracks", type=int, default=512,
                    help="independent tracks of the same configuration in the batched pass (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--table-v", action="store_true",
                    help="run the Table V / Fig. 2 analog instead (prints its own JSON line)")
    ap.add_argument("--passes", type=int, default=16, help="Monte Carlo passes of --table-v")
    ap.add_argument("--hybrid", action="store_true",
                    help="--table-v through the hybrid front end of eq. (4) (16 RF chains)")
    ap.add_argument("--counters", action="store_true",
                    help="counter target for rocprofv3 --pmc: one 1 GiB elementwise copy (the "
                         "calibration of FETCH_SIZE / WRITE_SIZE), then --steps updates of the "
                         "configuration's track at its eta; prints one line, times nothing")
    ap.add_argument("--serve", action="store_true",
                    help="run the serving experiment instead (prints its own JSON line)")
    ap.add_argument("--serve-tracks", type=int, default=2048)
    ap.add_argument("--serve-ring", type=int, default=8, help="device-resident snapshots per track")
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[1e4, 3e4, 1e5])
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="trace length per rate")
    ap.add_argument("--serve-batch", type=int, default=1024)
    ap.add_argument("--serve-wait-us", type=float, default=1000.0)
    return ap.parse_args()


PRECISIONS = {"fp32": 0, "bf16": 1, "bf16x3": 2}
ECDF_Q = (0.05, 0.25, 0.5, 0.75, 0.95)   # sum-rate quantiles reported for Fig. 2's ECDFs


def d_sequence(iters, k0, p, K):
    out = []
    for _ in range(iters):
        out.append(min(k0 + p, K))
        k0 *= 2
    return out


def measured_traffic(kernel_file_stem):
    """HBM bytes per launch from the committed counter summary
    (profiles/traffic_<stem>.json: FETCH_SIZE and WRITE_SIZE per dispatch,
    scaled by a copy of known size), or None when the kernel sources have
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_file_stem}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, "paper_2512_16543_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return rec["bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def arsvd_flops(K, info, k_init, p):
    """Algorithmic real flops of one arSVD/Woodbury launch: the two sketch
    products (Delta A Omega, Delta A Q: 8 K^2 d each) per iteration, and on
    the Woodbury path A^-1 U, V~^H A^-1 and the rank-r correction (8 K^2 r
    each); a direct inversion of A' (8 K^3) otherwise."""
    ds = d_sequence(info["iters"], k_init, p, K)
    f = sum(16.0 * K * K * d for d in ds)
    if info["path"] == 1:
        f += 24.0 * K * K * info["r"]
    elif info["path"] in (2, 3):
        f += 8.0 * K ** 3
    return f


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path "
              f"(--gpus {a.gpus} requested); independent tracks would shard across GPUs with no "
              f"exchange, see the design notes.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2512_16543_amd import rzf, workload as wl

    if a.counters:
        counters_target(a)
        return 0
    if a.table_v:
        print(json.dumps(table_v(a)), flush=True)
        return 0
    if a.serve:
        print(json.dumps(serve(a)), flush=True)
        return 0
    if a.config == "mix":
        print(json.dumps(mix(a, rzf.KINIT_WARM if a.policy == "warm" else rzf.KINIT_FIXED)), flush=True)
        return 0

    cfg = wl.CONFIGS[a.config]
    eta = cfg.eta if a.eta is None else a.eta
    K_steps, W_steps = a.steps, a.warmup
    tcfg = wl.with_overrides(cfg, steps=max(cfg.steps, K_steps))
    K, N = cfg.K, cfg.N
    dev = torch.device("cuda", 0)

    Hs_np = wl.make_track(tcfg, 0).snapshots(0, K_steps + 1).astype(np.complex64)
    Hw_np = wl.make_track(tcfg, 1).snapshots(0, W_steps + 1).astype(np.complex64)
    Hs = torch.from_numpy(Hs_np).to(dev)
    Hw = torch.from_numpy(Hw_np).to(dev)
    W = torch.empty(N, K, dtype=torch.complex64, device=dev)
    rates = torch.empty(K, dtype=torch.float32, device=dev)

    ctx = rzf.Context(0, 64 << 20)
    policy = rzf.KINIT_WARM if a.policy == "warm" else rzf.KINIT_FIXED

    tuned = ctx.tune_switch(K, N, PRECISIONS[a.precision]) if a.tune_switch else None
    switch_ratio = tuned["switch_ratio"] if tuned else 0.5
    if tuned and switch_ratio <= 0.0:
        switch_ratio = 0.5 / K   # the Woodbury branch never pays: every rank inverts

    def params(track_id):
        return rzf.default_params(k_init=cfg.k_init, p=cfg.p, P=cfg.P, seed=cfg.seed,
                                  track_id=track_id, reset_period=cfg.reset_period,
                                  kinit_policy=policy, early_fallback=int(a.early_fallback),
                                  precision=PRECISIONS[a.precision], error_feedback=int(a.error_feedback),
                                  switch_ratio=switch_ratio)

    def run_wb(H, steps, track_id, want_info=False, per_step_sync=False):
        tr = ctx.init(H[0], cfg.alpha, params(track_id))
        infos, lat, Rs = [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(1, steps + 1):
            ts = time.perf_counter()
            info = tr.update(H[t], eta, W, want_info=want_info)
            if per_step_sync:
                Rs.append(ctx.sum_rate(H[t], W, cfg.P, cfg.sigma2, rates))
                lat.append(time.perf_counter() - ts)
            else:
                ctx.sum_rate_async(H[t], W, cfg.P, cfg.sigma2, rates)
            if info is not None:
                infos.append(info)
        ctx.sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tr.destroy()
        return el, [i.as_dict() for i in infos], lat, Rs

    def run_full(H, steps, per_step_sync=False):
        lat, Rs = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prec = PRECISIONS[a.precision]
        items = [ctx.full_items([H[t]], [cfg.alpha], cfg.P, [W], prec) for t in range(steps + 1)] if prec else None
        for t in range(1, steps + 1):
            ts = time.perf_counter()
            if items is None:
                ctx.full(H[t], cfg.alpha, cfg.P, W)
            else:
                ctx.full_batch_raw(items[t])
            if per_step_sync:
                Rs.append(ctx.sum_rate(H[t], W, cfg.P, cfg.sigma2, rates))
                lat.append(time.perf_counter() - ts)
            else:
                ctx.sum_rate_async(H[t], W, cfg.P, cfg.sigma2, rates)
        ctx.sync()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, lat, Rs

    # two streams of default priority: the updates on one, each step's sum rate
    # on the other, so that step t's sum rate runs beside step t+1's update
    s_main, s_rate = torch.cuda.Stream(dev), torch.cuda.Stream(dev)
    pctx = rzf.Context(0, 64 << 20, stream=s_main)
    rctx = rzf.Context(0, 64 << 20, stream=s_rate)

    def run_pipelined(H, steps, kind, track_id=0):
        """The eager step with its sum rate on a second stream: W alternates
        between two buffers; step t's sum rate waits for step t's update, and
        step t+2's update waits for step t's sum rate (the buffer's reuse)."""
        Wp = [torch.empty_like(W) for _ in range(2)]
        rp = [torch.empty_like(rates) for _ in range(2)]
        sums = torch.zeros(steps + 1, dtype=torch.float64, device=dev)
        e_upd = [torch.cuda.Event() for _ in range(2)]
        e_rate = [torch.cuda.Event() for _ in range(2)]
        rit = [rctx.rate_items([H[t]], [Wp[t % 2]], [rp[t % 2]], sums[t:t + 1]) for t in range(steps + 1)]
        tr = pctx.init(H[0], cfg.alpha, params(track_id)) if kind == "wb" else None
        pctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(1, steps + 1):
            b = t % 2
            if t > 2:
                s_main.wait_event(e_rate[b])
            if kind == "wb":
                tr.update(H[t], eta, Wp[b], want_info=False)
            else:
                pctx.full(H[t], cfg.alpha, cfg.P, Wp[b])
            e_upd[b].record(s_main)
            s_rate.wait_event(e_upd[b])
            rctx.sum_rate_batch_raw(rit[t], cfg.P, cfg.sigma2)
            e_rate[b].record(s_rate)
        pctx.sync()
        rctx.sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if tr is not None:
            tr.destroy()
        return el, sums[1:].cpu().numpy()

    def run_graph(H, steps, kind, track_id=0, per_step_sync=False):
        """The same step captured once (rzf_graph_update / rzf_graph_full,
        the sum rate inside the graph): each step copies H_t into the graph's
        input buffer and launches the graph."""
        Hb = torch.empty_like(H[0])
        Wb = torch.empty_like(W)
        sums = torch.zeros(1, dtype=torch.float64, device=dev)
        Hb.copy_(H[0])
        tr = None
        if kind == "wb":
            tr = ctx.init(H[0], cfg.alpha, params(track_id))
            g = ctx.graph_update([tr], [Hb], [Wb], eta, rate=(cfg.P, cfg.sigma2, sums))
        else:
            g = ctx.graph_full([Hb], [cfg.alpha], cfg.P, [Wb], PRECISIONS[a.precision],
                               rate=(cfg.P, cfg.sigma2, sums))
        lat, Rs = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(1, steps + 1):
            ts = time.perf_counter()
            Hb.copy_(H[t])        # on the context's stream (torch's current one)
            g.launch()
            if per_step_sync:
                Rs.append(sums.item())
                lat.append(time.perf_counter() - ts)
        ctx.sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g.destroy()
        if tr is not None:
            tr.destroy()
        return el, lat, Rs

    # warm-up on a separate track of the same configuration
    run_wb(Hw, W_steps, 1)
    run_full(Hw, W_steps)
    run_graph(Hw, W_steps, "wb", 1)
    run_graph(Hw, W_steps, "full")
    run_pipelined(Hw, W_steps, "wb", 1)
    run_pipelined(Hw, W_steps, "full")
    print(f"[bench] warmup done ({W_steps} steps)", file=sys.stderr, flush=True)

    # timed region: exactly K steps of the WB-arSVD path (update + sum rate),
    # each step's sum rate on a second stream (the headline), then the same
    # steps on one stream, and as captured-graph launches
    torch.cuda.synchronize()
    wb_s, R_pipe = run_pipelined(Hs, K_steps, "wb")
    print(f"[bench] wb timed: {wb_s:.3f}s", file=sys.stderr, flush=True)
    full_s, _ = run_pipelined(Hs, K_steps, "full")
    print(f"[bench] full timed: {full_s:.3f}s", file=sys.stderr, flush=True)
    wb_1, _, _, _ = run_wb(Hs, K_steps, 0)
    full_1, _, _ = run_full(Hs, K_steps)
    print(f"[bench] one stream: wb {wb_1:.3f}s full {full_1:.3f}s", file=sys.stderr, flush=True)
    wb_g, _, _ = run_graph(Hs, K_steps, "wb")
    full_g, _, _ = run_graph(Hs, K_steps, "full")
    print(f"[bench] graph: wb {wb_g:.3f}s full {full_g:.3f}s", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC if a.config == "c2" else metric_for(cfg),
        "value": K_steps / wb_s,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K_steps,
        "warmup": W_steps,
        "ms_per_step": 1e3 * wb_s / K_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32" if a.precision == "fp32" else f"fp32 ({a.precision} Gram/precoder operands)",
        "data": "synthetic (seeded LEO channel track standing in for the paper's simulated pass)",
        "config": {
            "workload": (f"{a.config}: single LEO track, K={K} users, N={N} antennas "
                         f"({cfg.nx}x{cfg.nx} UPA), {tcfg.steps} snapshots of {cfg.dt_s * 1e3:g} ms, "
                         f"eta={eta}, FP64 re-inversion every {cfg.reset_period} steps, "
                         f"k_init={cfg.k_init}, p={cfg.p}, {a.policy} k_init policy"
                         f"{', early fallback' if a.early_fallback else ''}"
                         f"{', error feedback' if a.error_feedback else ''}; "
                         f"step = update + sum rate, batch of 1 track; the sum rate of step t on a "
                         f"second stream beside the update of step t+1"),
            "K": K, "N": N, "eta": eta, "batch_tracks": 1, "reset_period": cfg.reset_period,
            "switch_ratio": switch_ratio,
        },
        "full_inverse": {"value": K_steps / full_s, "unit": "updates/s",
                         "ms_per_step": 1e3 * full_s / K_steps},
        "speedup_vs_full_inverse": full_s / wb_s,
        "one_stream": {"wb": {"value": K_steps / wb_1, "ms_per_step": 1e3 * wb_1 / K_steps},
                       "full": {"value": K_steps / full_1, "ms_per_step": 1e3 * full_1 / K_steps},
                       "note": "the same steps with update and sum rate on one stream"},
        "graph": {"wb": {"value": K_steps / wb_g, "ms_per_step": 1e3 * wb_g / K_steps},
                  "full": {"value": K_steps / full_g, "ms_per_step": 1e3 * full_g / K_steps},
                  "note": "the same steps as one captured-graph launch each (rzf_graph_update / "
                          "rzf_graph_full with the sum rate inside), H_t first copied into the graph's "
                          "input buffer"},
    }

    # per-step latency (submit -> sum rate on the host) and path statistics
    if not a.no_latency:
        _, infos, lat_wb, R_wb = run_wb(Hs, K_steps, 0, want_info=True, per_step_sync=True)
        _, lat_full, R_full = run_full(Hs, K_steps, per_step_sync=True)
        _, lat_wbg, R_wbg = run_graph(Hs, K_steps, "wb", per_step_sync=True)
        _, lat_fullg, _ = run_graph(Hs, K_steps, "full", per_step_sync=True)
        pct = lambda v, q: float(np.percentile(np.array(v) * 1e3, q))
        out["latency_ms"] = {"wb_p50": pct(lat_wbg, 50), "wb_p99": pct(lat_wbg, 99),
                             "full_p50": pct(lat_fullg, 50), "full_p99": pct(lat_fullg, 99),
                             "eager_wb_p50": pct(lat_wb, 50), "eager_wb_p99": pct(lat_wb, 99),
                             "eager_full_p50": pct(lat_full, 50), "eager_full_p99": pct(lat_full, 99),
                             "note": "per step, host submit to sum rate on the host, one step in flight; "
                                     "wb/full: captured graph (input copy included), eager_*: the calls"}
        out["graph_sum_rate_equal"] = bool(np.array_equal(np.array(R_wbg), np.array(R_wb)))
        out["two_stream_sum_rate_equal"] = bool(np.array_equal(np.array(R_pipe), np.array(R_wb)))
        paths = {}
        for i in infos:
            paths[str(i["path"])] = paths.get(str(i["path"]), 0) + 1
        nr = [i for i in infos if i["path"] != 4]
        out["wb_stats"] = {
            "paths": {rzf_name: paths.get(str(code), 0) for code, rzf_name in
                      ((0, "noop"), (1, "wb"), (2, "full_rank"), (3, "full_singular"), (4, "reset"))},
            "r_mean": float(np.mean([i["r"] for i in nr])) if nr else 0.0,
            "iters_mean": float(np.mean([i["iters"] for i in nr])) if nr else 0.0,
            "sum_rate_wb_mean": float(np.mean(R_wb)), "sum_rate_full_mean": float(np.mean(R_full)),
            "sum_rate_loss": float(1.0 - np.mean(R_wb) / np.mean(R_full)),
        }
        print(f"[bench] latency pass done", file=sys.stderr, flush=True)
    else:
        infos = []

    # per-kernel durations with HIP events over a second pass of the same steps
    ctx.profile(True)
    _, infos2, _, _ = run_wb(Hs, K_steps, 0, want_info=True)
    prof = ctx.profile_read()
    ctx.profile(False)
    kern = {k: {"launches": c, "avg_us": 1e3 * ms / c} for k, (c, ms) in prof.items()}
    out["kernels_wb"] = kern
    dom = max(prof, key=lambda k: prof[k][1])
    cnt, tot_ms = prof[dom]
    avg_s = tot_ms / cnt * 1e-3
    if dom == "arsvd_wb":
        fl = [arsvd_flops(K, i, cfg.k_init, cfg.p) for i in infos2 if i["path"] != 4]
        per_launch = float(np.mean(fl))
        unit_note = ("mean over the timed steps of 16 K^2 sum_i d_i (sketch products) + "
                     "24 K^2 r (Woodbury) or 8 K^3 (direct inversion)")
    elif dom == "gram":
        per_launch = 12.0 * K * K * N
        unit_note = "4 K^2 N (A' lower half) + 8 K^2 N (Delta A lower half)"
    elif dom == "precoder":
        per_launch = 8.0 * K * K * N
        unit_note = "8 K^2 N"
    else:
        per_launch = 0.0
        unit_note = "n/a"
    achieved = per_launch / avg_s / 1e12
    traffic = None
    if dom == "arsvd_wb" and (K, N) == (64, 256) and a.config == "c2":
        traffic = measured_traffic("k_arsvd_wb_k64_n256")
    # k_arsvd_wb's instruction mix is VALU (counters: SQ_INSTS_VALU against SQ_INSTS_MFMA): its
    # peak is the FP32 vector rate without packed instructions, 78.6 TFLOP/s
    bound = "alu" if dom == "arsvd_wb" else "mfma"
    peak = FP32_VALU_PEAK_TFLOPS if bound == "alu" else FP32_MFMA_PEAK_TFLOPS
    out["roofline"] = {"kernel": dom, "bound": bound, "achieved": achieved,
                       "peak": peak, "unit": "TFLOP/s",
                       "frac": achieved / peak, "traffic": traffic,
                       "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                       "flops_per_launch": per_launch, "avg_launch_us": avg_s * 1e6,
                       "work": unit_note}
    print(f"[bench] profiled pass done: dominant {dom}", file=sys.stderr, flush=True)

    # batched pass: many independent tracks of the same configuration per launch
    if a.batch_tracks > 0:
        out["batched"] = batched(a, [cfg] * a.batch_tracks, eta, policy)
        print(f"[bench] batched pass done", file=sys.stderr, flush=True)

    if tuned:
        out["switch_tuning"] = tuned   # rzf_tune_switch's fit (cycles after the SVD)
    # FP64 CPU oracle on a bounded sample of the same track
    if not a.no_cpu_baseline:
        kept = []
        out["cpu_baseline"] = cpu_baseline(cfg, eta, Hs_np, a.cpu_seconds, policy, int(a.early_fallback),
                                           int(a.error_feedback), switch_ratio, keep=kept)
        print(f"[bench] cpu baseline done", file=sys.stderr, flush=True)
        out["oracle_error"] = gpu_vs_oracle(ctx, cfg, eta, Hs, kept, params(0), rates)
    if not a.no_sweep and a.config == "c2":
        out["eta_sweep"] = eta_sweep(ctx, cfg, Hs, min(K_steps, a.sweep_steps), params, W, rates)
        print(f"[bench] eta sweep done", file=sys.stderr, flush=True)
    ctx.close()
    pctx.close()
    rctx.close()
    print(json.dumps(out), flush=True)
    return 0


def gpu_vs_oracle(ctx, cfg, eta, Hs, kept, prm, rates):
    """The GPU's error against the FP64 oracle over the steps of the CPU
    sample: a fresh track run over the same snapshots, each side carrying its
    own state (trajectory, no re-seeding); relative Frobenius error of A^-1 and
    W per step, and of the sum rate."""
    import numpy as np
    import torch
    n = len(kept)
    if n == 0:
        return None
    W = torch.empty(cfg.N, cfg.K, dtype=torch.complex64, device=Hs.device)
    tr = ctx.init(Hs[0], cfg.alpha, prm)
    ea, ew, er, paths = [], [], [], []
    for t in range(1, n + 1):
        info = tr.update(Hs[t], eta, W)
        R = ctx.sum_rate(Hs[t], W, cfg.P, cfg.sigma2, rates)
        Wo, Ao, Ro = kept[t - 1]
        Ag = tr.inverse().cpu().numpy().astype(np.complex128)
        Wg = W.cpu().numpy().astype(np.complex128)
        ea.append(float(np.linalg.norm(Ag - Ao) / np.linalg.norm(Ao)))
        ew.append(float(np.linalg.norm(Wg - Wo) / np.linalg.norm(Wo)))
        er.append(abs(R - Ro) / abs(Ro))
        paths.append(info.path)
    tr.destroy()
    return {"steps": n, "ainv_rel_max": max(ea), "w_rel_max": max(ew), "sum_rate_rel_max": max(er),
            "ainv_rel_last": ea[-1], "resets": paths.count(4),
            "note": "GPU (FP32, FP64 capacitance and reset) against the FP64 oracle over the CPU sample's "
                    "steps, each side carrying its own state"}


def eta_sweep(ctx, cfg, Hs, steps, params, W, rates):
    """Single-track throughput of WB-arSVD against full inversion at the paper's
    Table V thresholds (and 0.99), with the fixed and warm-start k_init
    policies: updates/s of each (update + sum rate, one track), the paths and
    ranks taken, and the method's sum-rate loss against full inversion."""
    import numpy as np
    import torch
    from paper_2512_16543_amd import rzf
    rows = []
    Wf = torch.empty_like(W)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        ctx.sync()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def full_pass():
        for t in range(1, steps + 1):
            ctx.full(Hs[t], cfg.alpha, cfg.P, Wf)
            ctx.sum_rate_async(Hs[t], Wf, cfg.P, cfg.sigma2, rates)

    full_s = timed(full_pass)
    R_full = []
    for t in range(1, steps + 1):
        ctx.full(Hs[t], cfg.alpha, cfg.P, Wf)
        R_full.append(ctx.sum_rate(Hs[t], Wf, cfg.P, cfg.sigma2))
    for eta in (0.99, 0.9, 0.8, 0.65):
        for pol, code in (("fixed", rzf.KINIT_FIXED), ("warm", rzf.KINIT_WARM)):
            prm = params(0)
            prm.kinit_policy = code
            tr = ctx.init(Hs[0], cfg.alpha, prm)

            def wb_pass():
                for t in range(1, steps + 1):
                    tr.update(Hs[t], eta, W, want_info=False)
                    ctx.sum_rate_async(Hs[t], W, cfg.P, cfg.sigma2, rates)

            wb_s = timed(wb_pass)
            tr.destroy()
            tr = ctx.init(Hs[0], cfg.alpha, prm)
            infos, R_wb = [], []
            for t in range(1, steps + 1):
                infos.append(tr.update(Hs[t], eta, W))
                R_wb.append(ctx.sum_rate(Hs[t], W, cfg.P, cfg.sigma2))
            tr.destroy()
            nr = [i for i in infos if i.path != rzf.PATH_RESET]
            rows.append({"eta": eta, "policy": pol, "wb_updates_per_s": steps / wb_s,
                         "full_updates_per_s": steps / full_s, "speedup_vs_full_inverse": full_s / wb_s,
                         "sum_rate_loss": float(1.0 - np.mean(R_wb) / np.mean(R_full)),
                         "r_mean": float(np.mean([i.r for i in nr])),
                         "iters_mean": float(np.mean([i.iters for i in nr])),
                         "wb_fraction": float(np.mean([i.path == rzf.PATH_WB for i in nr]))})
            print(f"[bench] sweep eta={eta} {pol}: {rows[-1]['wb_updates_per_s']:.0f} vs "
                  f"{rows[-1]['full_updates_per_s']:.0f} updates/s, loss {rows[-1]['sum_rate_loss']:.2e}",
                  file=sys.stderr, flush=True)
    return {"steps": steps, "rows": rows,
            "note": "one track, batch 1, update + sum rate per step; loss = 1 - mean R(WB) / mean R(full)"}


def batched(a, cfgs, eta, policy):
    """len(cfgs) independent tracks (track ids 0..B-1; each its own size, SNR
    and regularisation) updated together: B x S updates of WB-arSVD, then of
    the full-inversion baseline, each step followed by the batched sum rate.
    Snapshots are resident in HBM before timing starts."""
    import numpy as np
    import torch
    from paper_2512_16543_amd import rzf, workload as wl
    B, S, Wu = len(cfgs), a.batch_steps, 2
    dev = torch.device("cuda", 0)
    T = Wu + S + 2          # snapshot 0 inits; 1..Wu warm up; S timed; the last one is profiled
    Hs = [torch.from_numpy(wl.make_track(c, b).snapshots(0, T).astype(np.complex64)).to(dev)
          for b, c in enumerate(cfgs)]
    Wl = [torch.empty(c.N, c.K, dtype=torch.complex64, device=dev) for c in cfgs]
    rl = [torch.empty(c.K, dtype=torch.float32, device=dev) for c in cfgs]
    sums = torch.empty(B, dtype=torch.float64, device=dev)
    arena = 2 * sum(rzf.track_bytes(c.K, c.N) for c in cfgs) + (256 << 20)   # eager and captured track sets
    ctx = rzf.Context(0, arena)
    trs = [ctx.init(Hs[b][0], c.alpha,
                    rzf.default_params(k_init=c.k_init, p=c.p, P=c.P, seed=c.seed, track_id=b,
                                       reset_period=c.reset_period, kinit_policy=policy,
                                       early_fallback=int(a.early_fallback),
                                       precision=PRECISIONS[a.precision],
                                       error_feedback=int(a.error_feedback)))
           for b, c in enumerate(cfgs)]
    P = cfgs[0].P
    s2 = [c.sigma2 for c in cfgs]
    upd = [ctx.update_items(trs, [Hs[b][t] for b in range(B)], Wl) for t in range(T)]
    full = [ctx.full_items([Hs[b][t] for b in range(B)], [c.alpha for c in cfgs], P, Wl, PRECISIONS[a.precision])
            for t in range(T)]
    rt = [ctx.rate_items([Hs[b][t] for b in range(B)], Wl, rl, sums, s2) for t in range(T)]

    def run(kind, t0, t1):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for t in range(t0, t1):
            if kind == "wb":
                ctx.update_batch_raw(upd[t], eta)
            else:
                ctx.full_batch_raw(full[t])
            ctx.sum_rate_batch_raw(rt[t], P, s2[0])
        ctx.sync()
        torch.cuda.synchronize()
        return time.perf_counter() - s0

    run("wb", 1, 1 + Wu)
    run("full", 1, 1 + Wu)
    wb_e = run("wb", 1 + Wu, 1 + Wu + S)
    full_e = run("full", 1 + Wu, 1 + Wu + S)

    # the same steps captured (rzf_graph_update / rzf_graph_full over one
    # packed input buffer, the batched sum rate inside the graph): each step
    # copies the packed snapshots of all tracks and launches the graph
    sizes = [c.K * c.N for c in cfgs]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    Hpack = [torch.cat([Hs[b][t].reshape(-1) for b in range(B)]) for t in range(T)]
    Hbuf = torch.empty_like(Hpack[0])
    Hv = [Hbuf[offs[b]:offs[b + 1]].view(c.K, c.N) for b, c in enumerate(cfgs)]
    Wg = [torch.empty_like(w) for w in Wl]
    sums_g = torch.empty(B, dtype=torch.float64, device=dev)
    trs_g = [ctx.init(Hs[b][0], c.alpha,
                      rzf.default_params(k_init=c.k_init, p=c.p, P=c.P, seed=c.seed, track_id=b,
                                         reset_period=c.reset_period, kinit_policy=policy,
                                         early_fallback=int(a.early_fallback),
                                         precision=PRECISIONS[a.precision],
                                         error_feedback=int(a.error_feedback)))
             for b, c in enumerate(cfgs)]
    torch.cuda.synchronize()
    g_wb = ctx.graph_update(trs_g, Hv, Wg, eta, rate=(P, s2[0], sums_g))
    g_full = ctx.graph_full(Hv, [c.alpha for c in cfgs], P, Wg, PRECISIONS[a.precision], rate=(P, s2[0], sums_g))

    def run_graph(g, t0, t1):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for t in range(t0, t1):
            Hbuf.copy_(Hpack[t])
            g.launch()
        ctx.sync()
        torch.cuda.synchronize()
        return time.perf_counter() - s0

    run_graph(g_wb, 1, 1 + Wu)
    run_graph(g_full, 1, 1 + Wu)
    wb_s = run_graph(g_wb, 1 + Wu, 1 + Wu + S)
    full_s = run_graph(g_full, 1 + Wu, 1 + Wu + S)
    g_wb.destroy()
    g_full.destroy()
    for tr in trs_g:
        tr.destroy()
    del Hpack
    res = {"tracks": B, "steps": S, "value": B * S / wb_s, "unit": "updates/s",
           "ms_per_batched_step": 1e3 * wb_s / S,
           "full_inverse": {"value": B * S / full_s, "unit": "updates/s",
                            "ms_per_batched_step": 1e3 * full_s / S},
           "speedup_vs_full_inverse": full_s / wb_s,
           "eager": {"value": B * S / wb_e, "ms_per_batched_step": 1e3 * wb_e / S,
                     "full_value": B * S / full_e, "full_ms_per_batched_step": 1e3 * full_e / S},
           "note": "value: one captured-graph launch per batched step (packed snapshots copied into its "
                   "input buffer first); eager: rzf_update_batch / rzf_full_batch and rzf_sum_rate_batch"}
    # dominant kernel of the batched WB pass: HIP events over the next (fresh)
    # snapshot of every track, with each track's info record for its work
    ctx.profile(True)
    infos = ctx.update_batch(trs, [Hs[b][T - 1] for b in range(B)], Wl, eta, want_info=True)
    ctx.sum_rate_batch_raw(rt[T - 1], P, s2[0])
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.sync()
    res["kernels_wb"] = {k: {"launches": c, "avg_us": 1e3 * ms / c} for k, (c, ms) in prof.items()}
    dom = max(prof, key=lambda k: prof[k][1])
    dur = prof[dom][1] / prof[dom][0] * 1e-3
    if dom == "arsvd_wb":
        fl = sum(arsvd_flops(c.K, i.as_dict(), c.k_init, c.p) for c, i in zip(cfgs, infos) if i.path != 4)
    elif dom == "gram":
        fl = sum(12.0 * c.K * c.K * c.N for c in cfgs)
    elif dom == "precoder":
        fl = sum(8.0 * c.K * c.K * c.N for c in cfgs)
    else:
        fl = 0.0
    bpk = FP32_VALU_PEAK_TFLOPS if dom == "arsvd_wb" else FP32_MFMA_PEAK_TFLOPS
    res["roofline"] = {"kernel": dom, "bound": "alu" if dom == "arsvd_wb" else "mfma",
                       "achieved": fl / dur / 1e12,
                       "peak": bpk, "unit": "TFLOP/s",
                       "frac": fl / dur / 1e12 / bpk, "traffic": None,
                       "flops_per_launch": fl, "avg_launch_us": dur * 1e6,
                       "paths": {str(p): sum(1 for i in infos if i.path == p) for p in range(5)}}
    # the GEMM-shaped kernels of the same batched step against the FP32
    # matrix-core peak (their operands at this precision)
    mf = {}
    for name in ("gram", "precoder", "sum_rate"):
        if name not in prof:
            continue
        c, ms = prof[name]
        us = 1e3 * ms / c
        f = sum(kernel_flops(name, cf.K, cf.N) for cf in cfgs)
        if name == "gram":     # reset steps run the FP64 Gram instead
            f = sum(kernel_flops(name, cf.K, cf.N) for cf, i in zip(cfgs, infos) if i.path != 4)
        mf[name] = {"avg_us": us, "flops": f, "achieved_tflops": f / (us * 1e-6) / 1e12,
                    "frac": f / (us * 1e-6) / 1e12 / FP32_MFMA_PEAK_TFLOPS}
    res["mfma_kernels"] = mf
    ctx.close()
    return res


def mix(a, policy):
    """Multi-track mix: B tracks, K uniform on 16..128, N in {64, 256, 1024},
    SNR uniform on 0..20 dB, all updated by one batched call per step."""
    import numpy as np
    from paper_2512_16543_amd import workload as wl
    eta = 0.999 if a.eta is None else a.eta
    cfgs = wl.mix_configs(a.batch_tracks, seed=3, eta=eta)
    res = batched(a, cfgs, eta, policy)
    Ks = np.array([c.K for c in cfgs])
    Ns = np.array([c.N for c in cfgs])
    out = {
        "metric": "RZF precoder updates/s, multi-track mix (K 16..128, N 64/256/1024), WB-arSVD vs full inverse",
        "value": res["value"], "unit": "updates/s", "n_gpus": 1, "steps": res["steps"],
        "warmup": 2, "ms_per_step": res["ms_per_batched_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32" if a.precision == "fp32" else f"fp32 ({a.precision} Gram/precoder operands)",
        "data": "synthetic (seeded LEO channel tracks)",
        "config": {"workload": (f"mix: {len(cfgs)} tracks, K uniform 16..128 (mean {Ks.mean():.1f}, "
                                f"{int((Ks > 64).sum())} above 64), N in {{64, 256, 1024}} "
                                f"(mean {Ns.mean():.0f}), SNR 0..20 dB, eta={eta}, FP64 reset every 100 steps, "
                                f"{a.precision} operands; "
                                f"step = one batched update of every track + batched sum rate"),
                   "tracks": len(cfgs), "eta": eta},
    }
    out.update({k: v for k, v in res.items() if k not in ("value", "unit", "steps")})
    return out


def serve(a):
    """Serving loop: resident tracks of the multi-track size mix receive update
    requests as Poisson arrivals (aggregate rate lambda, each request for a
    uniformly drawn track), replayed on time by the library's request server.
    Each track cycles through a device-resident ring of consecutive snapshots
    (forward, then back).  Per rate: latency percentiles (completion minus
    submission, server clock) and achieved throughput of the WB-arSVD server,
    then of the full-inversion server on the same trace."""
    import numpy as np
    import torch
    from paper_2512_16543_amd import rzf, workload as wl
    B, R = a.serve_tracks, a.serve_ring
    cfgs = wl.mix_configs(B, seed=4, eta=0.999 if a.eta is None else a.eta)
    eta = cfgs[0].eta
    dev = torch.device("cuda", 0)
    Hs = [torch.from_numpy(wl.make_track(c, b).snapshots(0, R).astype(np.complex64)).to(dev)
          for b, c in enumerate(cfgs)]
    Ws = [torch.empty(c.N, c.K, dtype=torch.complex64, device=dev) for c in cfgs]
    ctx = rzf.Context(0, sum(rzf.track_bytes(c.K, c.N) for c in cfgs) + (256 << 20))
    trs = [ctx.init(Hs[b][0], c.alpha,
                    rzf.default_params(k_init=c.k_init, p=c.p, P=c.P, seed=c.seed, track_id=b,
                                       reset_period=c.reset_period))
           for b, c in enumerate(cfgs)]
    print(f"[serve] {B} tracks resident", file=sys.stderr, flush=True)
    period = 2 * (R - 1)
    step = np.zeros(B, dtype=np.int64)

    def ring(k):       # snapshot index of a track's k-th update (k >= 1): 1..R-1, R-2..0, 1..
        m = k % period
        return m if m <= R - 1 else period - m

    rows = []
    rng = np.random.default_rng(np.random.SeedSequence([4, 4242]))
    for lam in a.serve_rates:
        n = int(rng.poisson(lam * a.serve_seconds))
        t_arr = np.cumsum(rng.exponential(1e6 / lam, n))
        who = rng.integers(0, B, n)
        idx = np.empty(n, dtype=np.int64)
        for j in range(n):
            step[who[j]] += 1
            idx[j] = ring(int(step[who[j]]))
        reqs = rzf.Server.requests([trs[b] for b in who], [Hs[b][k] for b, k in zip(who, idx)],
                                   [Ws[b] for b in who], range(n), t_arr)
        row = {"rate_per_s": lam, "requests": n, "seconds": a.serve_seconds}
        for mode, name in ((rzf.SERVE_UPDATE, "wb"), (rzf.SERVE_FULL, "full")):
            srv = rzf.Server(ctx, rzf.server_params(mode=mode, tol=eta, max_batch=a.serve_batch,
                                                    max_wait_us=a.serve_wait_us))
            srv.replay(reqs)
            srv.drain()
            done = []
            while True:
                got = srv.poll(65536)
                if not got:
                    break
                done += got
            srv.close()
            ctx.sync()
            lat = np.array([c.t_done_us - c.t_submit_us for c in done]) * 1e-3
            t_first = min(c.t_submit_us for c in done)
            t_last = max(c.t_done_us for c in done)
            launches = len({c.t_launch_us for c in done})
            row[name] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                         "p999_ms": float(np.percentile(lat, 99.9)), "mean_ms": float(lat.mean()),
                         "achieved_per_s": len(done) / ((t_last - t_first) * 1e-6),
                         "mean_batch": len(done) / max(launches, 1),
                         "errors": int(sum(c.status != 0 for c in done))}
            print(f"[serve] rate {lam:g}/s {name}: p50 {row[name]['p50_ms']:.2f} ms, "
                  f"p99 {row[name]['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
        rows.append(row)
    Ks = np.array([c.K for c in cfgs])
    ctx.close()
    return {"experiment": "serving", "tracks": B, "snapshot_ring": R, "eta": eta,
            "k_mean": float(Ks.mean()), "k_above_64": int((Ks > 64).sum()),
            "max_batch": a.serve_batch, "max_wait_us": a.serve_wait_us,
            "latency": "completion minus submission on the server clock; submission is on the arrival time",
            "rows": rows}


def counters_target(a):
    """Work for a hardware-counter pass: a plain copy of known size first
    (1 GiB in, 1 GiB out, so each counter's scale can be read off it), then
    a.steps updates of one track of the configuration, nothing else."""
    import numpy as np
    import torch
    from paper_2512_16543_amd import rzf, workload as wl
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y
    cfg = wl.CONFIGS[a.config]
    eta = cfg.eta if a.eta is None else a.eta
    Hs = torch.from_numpy(wl.make_track(wl.with_overrides(cfg, steps=max(cfg.steps, a.steps)))
                          .snapshots(0, a.steps + 1).astype(np.complex64)).cuda()
    ctx = rzf.Context(0, 64 << 20)
    tr = ctx.init(Hs[0], cfg.alpha, rzf.default_params(k_init=cfg.k_init, p=cfg.p, P=cfg.P, seed=cfg.seed,
                                                       reset_period=0,
                                                       precision=PRECISIONS[a.precision],
                                                       error_feedback=int(a.error_feedback),
                                                       early_fallback=int(a.early_fallback)))
    W = torch.empty(cfg.N, cfg.K, dtype=torch.complex64, device="cuda")
    for t in range(1, a.steps + 1):
        tr.update(Hs[t], eta, W, want_info=False)
    ctx.sync()
    ctx.close()
    print(f"counters target: 1 GiB copy, {a.steps} updates of {a.config} at eta={eta}", flush=True)


def table_v(a):
    """Analog of the paper's Table V / Fig. 2 on synthetic passes.

    Scenario (the paper's Table IV where it is given): 16x16 half-wavelength
    array, 600 km orbit, Rician K-factor 10 dB, K = 16 users (the Gram matrix
    is 16 x 16 as after the paper's 16 RF chains), precoder updates every 50 ms
    over a 120 s pass, p = 1, k_init = 2, no drift reset.  Users are uniform in
    a 50 km disk and SNR is 10 dB (the paper's link budget is not given in
    full).  Every pass is one track; passes run as one batch.  For each eta:
      * sum-rate degradation against full-inversion RZF on the same snapshots;
      * computational savings by Table III's count K^2 + K^2 r + r^3 + r^2 K
        against K^3 per step, with the observed k_est (steps that fall back
        to direct inversion count K^3);
      * the measured GPU time of the batched passes against full inversion.

    With --hybrid the precoder runs on H_eff = H~ F_RF of eq. (4) (the
    configuration "h1": users spread over a 250 km disk so that most have a
    beam of their own): every snapshot's beams are chosen on the GPU from the
    users' array manifolds, and eq. (15) is scored on H(t) F_RF.  The front
    end runs once per snapshot before the timed passes (it is the same for
    both precoders) and is timed on its own.
    """
    import numpy as np
    import torch
    from paper_2512_16543_amd import rzf, workload as wl
    from paper_2512_16543_amd import opcount as cx    # Table III operation count
    if a.hybrid:
        base = wl.CONFIGS["h1"]
    else:
        base = wl.CONFIGS["tv"]
    B, T = a.passes, base.steps
    K, N = base.K, base.N
    Np = base.n_rf if a.hybrid else N        # columns the precoder sees
    dev = torch.device("cuda", 0)
    ctx = rzf.Context(0, B * rzf.track_bytes(K, Np) + (64 << 20))
    Hs = torch.empty(B, T + 1, K, N, dtype=torch.complex64, device=dev)
    for b in range(B):
        Hs[b] = torch.from_numpy(wl.make_track(base, b).snapshots().astype(np.complex64)).to(dev)
    front = {}
    if a.hybrid:
        Ms = torch.empty(B, T + 1, K, N, dtype=torch.complex64, device=dev)
        for b in range(B):
            Ms[b] = torch.from_numpy(wl.make_track(base, b).snapshots(manifold=True).astype(np.complex64)).to(dev)
        Hp = torch.empty(B, T + 1, K, Np, dtype=torch.complex64, device=dev)   # H~ F_RF
        Hr = torch.empty(B, T + 1, K, Np, dtype=torch.complex64, device=dev)   # H F_RF
        beams = torch.empty(B, T + 1, Np, dtype=torch.int32, device=dev)
        def front_end(b, t):
            ctx.beamspace(Ms[b, t], base.nx, base.nx, beams[b, t], Hp[b, t])
            ctx.beamspace(Hs[b, t], base.nx, base.nx, beams[b, t], Hr[b, t], select=False)

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(B):
            for t in range(T + 1):
                front_end(b, t)
        ctx.sync()
        fe_s = time.perf_counter() - t0
        ctx.profile(True)            # kernel averages over a few hundred repeated snapshots
        for t in range(min(T + 1, 300)):
            front_end(0, t)
        prof = {k: 1e3 * ms / max(n, 1) for k, (n, ms) in ctx.profile_read().items()}   # avg us
        ctx.profile(False)
        del Ms
        bh = beams.cpu().numpy()
        front = {"front_end_ms_per_snapshot": 1e3 * fe_s / (B * (T + 1)),
                 "beam_resp_us": prof.get("beam_resp"), "beam_select_us": prof.get("beam_select"),
                 "beam_switches_per_step": float(np.mean(np.sum(bh[:, 1:] != bh[:, :-1], axis=2))),
                 "n_rf": Np, "N_t": N}
        print(f"[table-v] front end {front}", file=sys.stderr, flush=True)
    else:
        Hp = Hr = Hs
    Wl = [torch.empty(Np, K, dtype=torch.complex64, device=dev) for _ in range(B)]
    sums = torch.empty(T + 1, B, dtype=torch.float64, device=dev)
    full_items = [ctx.full_items([Hp[b, t] for b in range(B)], [base.alpha] * B, base.P, Wl)
                  for t in range(T + 1)]
    rate_items = [ctx.rate_items([Hr[b, t] for b in range(B)], Wl, None, sums[t]) for t in range(T + 1)]
    # full-inversion RZF reference
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(1, T + 1):
        ctx.full_batch_raw(full_items[t])
        ctx.sum_rate_batch_raw(rate_items[t], base.P, base.sigma2)
    ctx.sync()
    full_s = time.perf_counter() - t0
    R_full = sums[1:].cpu().numpy().copy()
    rows = []
    for eta in (0.9, 0.8, 0.65, 0.999):
        trs = [ctx.init(Hp[b, 0], base.alpha,
                        rzf.default_params(k_init=base.k_init, p=base.p, P=base.P, seed=base.seed,
                                           track_id=b, reset_period=0, error_feedback=int(a.error_feedback)))
               for b in range(B)]
        upd = [ctx.update_items(trs, [Hp[b, t] for b in range(B)], Wl) for t in range(T + 1)]
        # timed pass (no info records), then an identical pass that records ranks
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(1, T + 1):
            ctx.update_batch_raw(upd[t], eta)
            ctx.sum_rate_batch_raw(rate_items[t], base.P, base.sigma2)
        ctx.sync()
        wb_s = time.perf_counter() - t0
        R_wb = sums[1:].cpu().numpy().copy()
        for tr in trs:
            tr.destroy()
        trs = [ctx.init(Hp[b, 0], base.alpha,
                        rzf.default_params(k_init=base.k_init, p=base.p, P=base.P, seed=base.seed,
                                           track_id=b, reset_period=0, error_feedback=int(a.error_feedback)))
               for b in range(B)]
        ranks, paths, iters = [], [], []
        for t in range(1, T + 1):
            infos = ctx.update_batch(trs, [Hp[b, t] for b in range(B)], Wl, eta, want_info=True)
            if t % 200 == 0 or t == T:
                ctx.sync()
            ranks.append(infos)
        ctx.sync()
        for infos in ranks:
            for i in infos:
                paths.append(i.path)
                iters.append(i.iters)
        rs = np.array([i.r for infos in ranks for i in infos])
        pa = np.array(paths)
        cost = np.where(pa == rzf.PATH_WB, [cx.wb_arsvd_ops(K, r) for r in rs], float(K) ** 3)
        rows.append({
            "eta": eta,
            "sr_ecdf_quantiles": [float(x) for x in np.quantile(R_wb, ECDF_Q)],
            "sr_degradation": float(1.0 - R_wb.mean() / R_full.mean()),
            "opcount_savings": float(1.0 - cost.mean() / float(K) ** 3),
            "k_est_mean": float(rs.mean()),
            "wb_fraction": float((pa == rzf.PATH_WB).mean()),
            "iters_mean": float(np.mean(iters)),
            "gpu_time_savings": float(1.0 - wb_s / full_s),
            "wb_ms_per_batched_step": 1e3 * wb_s / T,
        })
        for tr in trs:
            tr.destroy()
        print(f"[table-v] eta={eta} done", file=sys.stderr, flush=True)
    ctx.close()
    return {"experiment": "table_v_analog", "hybrid": bool(a.hybrid), **front,
            "error_feedback": bool(a.error_feedback),
            "passes": B, "steps_per_pass": T, "K": K, "N": Np,
            "update_interval_s": base.dt_s, "full_ms_per_batched_step": 1e3 * full_s / T,
            "ecdf_q": list(ECDF_Q), "sr_ecdf_quantiles_full": [float(x) for x in np.quantile(R_full, ECDF_Q)],
            "paper_table_v": [{"eta": 0.90, "savings": 0.306, "sr_degradation": 0.016},
                              {"eta": 0.80, "savings": 0.477, "sr_degradation": 0.058},
                              {"eta": 0.65, "savings": 0.612, "sr_degradation": 0.095}],
            "rows": rows}


def host_cores():
    """Cores this process may run on, the BLAS libraries NumPy uses and their
    thread counts."""
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    blas, threads = [], 1
    try:
        from threadpoolctl import threadpool_info
        for i in threadpool_info():
            if i.get("user_api") == "blas":
                blas.append(f"{i.get('internal_api')} {i.get('version')} ({i.get('num_threads')} threads)")
                threads = max(threads, int(i.get("num_threads") or 1))
    except Exception:
        pass
    return nproc, threads, "; ".join(blas) or "unknown"


def cpu_baseline(cfg, eta, Hs_np, budget_s, policy, early_fallback=0, error_feedback=0, switch_ratio=0.5,
                 keep=None):
    """The FP64 oracle (update + sum rate) on the first steps of the track for
    about budget_s seconds.  keep: a list that receives each step's
    (W, A^-1, sum rate) for the GPU's error against the oracle."""
    import numpy as np
    import oracle.rzf as orz
    nproc, threads, blas = host_cores()
    H = Hs_np.astype(np.complex128)
    prm = orz.TrackParams(alpha=cfg.alpha, P=cfg.P, k_init=cfg.k_init, p=cfg.p,
                          reset_period=cfg.reset_period, seed=cfg.seed, track_id=0,
                          kinit_policy=policy, early_fallback=early_fallback,
                          error_feedback=error_feedback, switch_ratio=switch_ratio)
    ot = orz.OracleTrack(H[0], prm)
    t0 = time.perf_counter()
    n = 0
    for t in range(1, H.shape[0]):
        Wt, _ = ot.update(H[t], eta)
        _, R = orz.sum_rate(H[t], Wt, cfg.P, cfg.sigma2)
        if keep is not None:
            keep.append((Wt, ot.Ainv.copy(), R))
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": "updates/s", "cores": int(threads), "nproc": int(nproc),
            "blas": blas, "kind": "oracle",
            "sample": f"first {n} steps of the same track (update + sum rate, complex128 NumPy, one process; "
                      f"cores = the BLAS threads it used, nproc = cores available)"}


if __name__ == "__main__":
    sys.exit(main())
