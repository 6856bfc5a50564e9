"""Launch-shape autotuner: measures, per track size (K, N), the precoder's rows
per workgroup (single-track and batched launches) and the single-track sum
rate's spread over workgroups, and writes the fastest of each to a JSON table
that Context loads (rzf_tune_table).  Neither knob changes a result bit, so the
table only moves time.

    python -m paper_2512_16543_amd.tune --out paper_2512_16543_amd/tuning.json

Each candidate is timed with the library's HIP-event profile over `reps`
launches (after one untimed launch); the batched precoder over `batch` tracks
of the size.  Needs a GPU.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

GRID_K = (8, 16, 32, 64, 128, 256)
GRID_N = (64, 128, 256, 512, 1024, 2048, 4096)
ROWS = (32, 64, 256)
SPLITS = (1, 2, 4, 8)


def kernel_us(ctx, fn, reps, name):
    """Mean HIP-event duration (us) of kernel `name` over reps calls of fn."""
    fn()
    ctx.sync()
    ctx.profile(True)
    for _ in range(reps):
        fn()
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.sync()
    n, ms = prof[name]
    return 1e3 * ms / n


def tune_size(ctx, K, N, reps, batch):
    import numpy as np
    import torch
    from paper_2512_16543_amd import workload as wl
    H = torch.from_numpy(wl.random_channel(K, N, 7).astype(np.complex64)).cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(K * 10007 + N)
    W = torch.empty(N, K, dtype=torch.complex64, device="cuda")
    rates = torch.empty(K, dtype=torch.float32, device="cuda")
    alpha = K / 10.0
    # the batch's channels drawn on the device (i.i.d. CN(0, 1/N), as random_channel)
    Hb = [torch.randn(K, N, dtype=torch.complex64, device="cuda", generator=g) / N ** 0.5 for _ in range(batch)]
    Wb = [torch.empty(N, K, dtype=torch.complex64, device="cuda") for _ in range(batch)]
    items = ctx.full_items(Hb, [alpha] * batch, 1.0, Wb)
    meas = {"precoder_us": {}, "batch_precoder_us": {}, "sum_rate_us": {}}
    for pb in (ROWS if K <= 64 else tuple(v for v in ROWS if v != 256)):
        ctx.tune_table([{"K": K, "N": N, "precoder_rows": pb, "batch_precoder_rows": pb}])
        meas["precoder_us"][pb] = kernel_us(ctx, lambda: ctx.full(H, alpha, 1.0, W), reps, "precoder")
        meas["batch_precoder_us"][pb] = kernel_us(ctx, lambda: ctx.full_batch_raw(items), max(2, reps // 8),
                                                  "precoder")
    splits = SPLITS if K <= 64 else (1,)
    for ns in splits:
        if ns > 1 and ns > (N + 63) // 64:
            continue
        ctx.tune_table([{"K": K, "N": N, "rate_splits": ns}])
        meas["sum_rate_us"][ns] = kernel_us(ctx, lambda: ctx.sum_rate_async(H, W, 1.0, 0.1, rates), reps,
                                            "sum_rate")
    ctx.tune_table([])
    del Hb, Wb
    torch.cuda.empty_cache()
    best = lambda d: min(d, key=lambda k: (d[k], k))
    entry = {"K": K, "N": N, "precoder_rows": best(meas["precoder_us"]),
             "batch_precoder_rows": best(meas["batch_precoder_us"]),
             "rate_splits": best(meas["sum_rate_us"]) if K <= 64 else 0}
    entry["measured_us"] = {k: {str(a): round(b, 2) for a, b in v.items()} for k, v in meas.items()}
    return entry


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default="tuning.json")
    ap.add_argument("--reps", type=int, default=40)
    ap.add_argument("--batch", type=int, default=512, help="tracks of the batched precoder measurement")
    ap.add_argument("--K", type=int, nargs="*", default=list(GRID_K))
    ap.add_argument("--N", type=int, nargs="*", default=list(GRID_N))
    a = ap.parse_args(argv)
    import torch
    from paper_2512_16543_amd import rzf
    ctx = rzf.Context(0, 1 << 30, tuning=None)
    entries = []
    t0 = time.time()
    for K in a.K:
        for N in a.N:
            if K > N:
                continue
            e = tune_size(ctx, K, N, a.reps, a.batch)
            entries.append(e)
            print(f"[tune] K={K} N={N}: rows {e['precoder_rows']} (batch {e['batch_precoder_rows']}), "
                  f"splits {e['rate_splits']}  {e['measured_us']}", file=sys.stderr, flush=True)
    ctx.close()
    out = {"device": torch.cuda.get_device_name(0), "reps": a.reps, "batch": a.batch,
           "seconds": round(time.time() - t0, 1),
           "note": "per (K, N): the fastest precoder rows per workgroup (single / batched launches) and "
                   "sum-rate spread (single track, K <= 64) by mean HIP-event kernel time; "
                   "written by python -m paper_2512_16543_amd.tune",
           "entries": entries}
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"[tune] {len(entries)} sizes -> {a.out}", file=sys.stderr, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
