"""Benchmark of the hot path on one MI355X.

Workload (batched image coding, Section 3.1's experiment at scale): 1024
uint8 images of 512x512 (first-order Markov field, rho = 0.95), i.e.
1,048,576 tiles of 16x16.  One step codes the whole batch at every zonal
size r in {2, 4, 8, 12, 16}: for each r, the forward transform of every tile
(int32 coefficients to HBM), then zonal retention + inverse + rounding into
a uint8 reconstruction with a per-image exact SSE against the original.

Printed: one JSON line with tiles/s (each tile counted once per r, i.e. per
forward+inverse pair), the HIP-event-timed duration and roofline of the
dominant kernel, the CPU oracle on a bounded sample, and the PSNR per r.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_IMG, SIDE = 1024, 512
RS = (2, 4, 8, 12, 16)
HBM_PEAK_GBS = 8000.0
FWD_BYTES_PER_TILE = 256 + 1024           # u8 tile in, int32 coefficients out


def recon_bytes_per_tile(r: int) -> int:
    # kept r x r int32 coefficients in, reference tile in (SSE), u8 tile out
    return 4 * r * r + 256 + 256


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--images", type=int, default=N_IMG)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-images", type=int, default=32)
    return ap.parse_args()


def cpu_baseline(img: np.ndarray, n_sample: int):
    """The plain C oracle (dense int64 products, OpenMP over tiles) on the
    first n_sample images, every r, timed on the host cores."""
    from tests import oracle_c
    sample = np.ascontiguousarray(img[: n_sample * SIDE])
    H = sample.shape[0]
    t0 = time.perf_counter()
    for r in RS:
        coef = oracle_c.fwd2d_u8(sample)
        oracle_c.zonal_recon_u8(coef, H, SIDE, r, sample, SIDE)
    dt = time.perf_counter() - t0
    tiles = (H // 16) * (SIDE // 16) * len(RS)
    return {"value": tiles / dt, "unit": "16x16 blocks/s", "cores": oracle_c.threads(), "kind": "oracle",
            "sample": f"{n_sample} of the {N_IMG} images, fwd + zonal inverse + SSE at each r in {list(RS)}, "
                      f"C oracle (dense int64 16x16 products), {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_1606_07414_amd import adct
    import synth

    n_img = args.images
    t0 = time.perf_counter()
    img = synth.ar1_batch(n_img, SIDE, SIDE)
    gen_s = time.perf_counter() - t0
    ntiles = n_img * (SIDE // 16) ** 2

    dev = torch.device("cuda:0")
    x = torch.from_numpy(img).to(dev)
    coef = torch.empty((ntiles, 16, 16), dtype=torch.int32, device=dev)
    out = torch.empty_like(x)
    sse = {r: torch.empty(n_img, dtype=torch.int64, device=dev) for r in RS}
    stream = torch.cuda.current_stream()

    ev = {"fwd": [], "recon": {r: [] for r in RS}}

    def step(timed: bool):
        for r in RS:
            if timed:
                e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
                e0.record(stream)
            adct.fwd2d(x, coef, stream=stream)
            if timed:
                e1.record(stream)
            adct.zonal_recon(coef, r, out, ref=x, image_height=SIDE, sse=sse[r], stream=stream)
            if timed:
                e2.record(stream)
                ev["fwd"].append((e0, e1))
                ev["recon"][r].append((e1, e2))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    ms_step = 1000.0 * wall / args.steps
    tiles_per_step = ntiles * len(RS)
    fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in ev["fwd"]]))
    rec_ms = {r: float(np.mean([a.elapsed_time(b) for a, b in ev["recon"][r]])) for r in RS}
    fwd_gbs = FWD_BYTES_PER_TILE * ntiles / (fwd_ms * 1e-3) / 1e9
    psnr = {r: float(np.mean(adct.psnr(sse[r].cpu().numpy(), SIDE * SIDE))) for r in RS}

    result = {
        "metric": "16x16 blocks/s (fwd+inv) and fraction of HBM peak",
        "value": tiles_per_step / (ms_step * 1e-3),
        "unit": "16x16 blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{n_img} uint8 AR(1) rho=0.95 images of {SIDE}x{SIDE} ({ntiles} tiles); "
                               f"per step, for each r in {list(RS)}: fwd2d + zonal r x r + inverse + per-image SSE",
                   "images": n_img, "side": SIDE, "zonal_r": list(RS)},
        "roofline": {"bound": "hbm", "kernel": "fwd2d (k_fwd u8 -> int32)", "achieved": fwd_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fwd_gbs / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_tile": FWD_BYTES_PER_TILE, "tiles_per_launch": ntiles,
                     "avg_launch_ms": fwd_ms},
        "kernels_ms": {"fwd2d": fwd_ms, **{f"zonal_recon_r{r}": rec_ms[r] for r in RS}},
        "kernels_gbs": {"fwd2d": fwd_gbs, **{f"zonal_recon_r{r}": recon_bytes_per_tile(r) * ntiles /
                                             (rec_ms[r] * 1e-3) / 1e9 for r in RS}},
        "psnr_db_mean": psnr,
        "input_gen_s": gen_s,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(img, min(args.cpu_sample_images, n_img))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
