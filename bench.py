"""Benchmark of the hot path on one MI355X.

Workload (batched image coding, Section 3.1's experiment at scale): 1024
uint8 images of 512x512 (first-order Markov field, rho = 0.95), i.e.
1,048,576 tiles of 16x16.  One step codes the whole batch at every zonal
size r in {2, 4, 8, 12, 16}: for each r, one pass of the single-pass encoder
(adct_encode_zonal) reads every tile once, writes its int32 coefficients
Y = T A T^T, keeps the top-left r x r coefficients with S folded in, runs the
inverse, and writes the rounded uint8 reconstruction with an exact per-image
SSE against the original.

Printed: one JSON line with tiles/s (each tile counted once per r, i.e. per
forward+inverse pair), the HIP-event-timed duration and roofline of the
encoder kernel, the two-kernel path (adct_fwd2d + adct_zonal_recon) timed
after the measured region for context, the CPU oracle on the same workload,
and the PSNR per r.
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
ENC_BYTES_PER_TILE = 256 + 1024 + 256     # u8 tile in, int32 coefficients out, u8 reconstruction out
FWD_BYTES_PER_TILE = 256 + 1024           # two-kernel path: forward
CPU_MIN_SECONDS = 10.0


def recon_bytes_per_tile(r: int) -> int:
    # two-kernel path, inverse: kept r x r int32 coefficients in, reference
    # tile in (SSE), u8 tile out
    return 4 * r * r + 256 + 256


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--images", type=int, default=N_IMG)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(img: np.ndarray):
    """The plain C oracle (dense int64 products, OpenMP over tiles): the whole
    workload (every image, every r), repeated until at least CPU_MIN_SECONDS
    of host time (at most 3 passes)."""
    from tests import oracle_c
    H = img.shape[0]
    passes, t0 = 0, time.perf_counter()
    while passes < 3 and (passes == 0 or time.perf_counter() - t0 < CPU_MIN_SECONDS):
        for r in RS:
            coef = oracle_c.fwd2d_u8(img)
            oracle_c.zonal_recon_u8(coef, H, SIDE, r, img, SIDE)
        passes += 1
    dt = time.perf_counter() - t0
    tiles = (H // 16) * (SIDE // 16) * len(RS) * passes
    return {"value": tiles / dt, "unit": "16x16 blocks/s", "cores": oracle_c.threads(), "kind": "oracle",
            "sample": f"the full workload ({H // SIDE} images, fwd + zonal inverse + SSE at each r in "
                      f"{list(RS)}) x {passes} pass(es), C oracle (dense int64 16x16 products, OpenMP), "
                      f"{dt:.1f} s"}


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

    ev = {r: [] for r in RS}

    def step(timed: bool):
        for r in RS:
            if timed:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            adct.encode_zonal(x, r, out, coef=coef, image_height=SIDE, sse=sse[r], stream=stream)
            if timed:
                e1.record(stream)
                ev[r].append((e0, e1))

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
    enc_ms = {r: float(np.mean([a.elapsed_time(b) for a, b in ev[r]])) for r in RS}
    enc_avg_ms = float(np.mean(list(enc_ms.values())))
    enc_gbs = ENC_BYTES_PER_TILE * ntiles / (enc_avg_ms * 1e-3) / 1e9
    psnr = {r: float(np.mean(adct.psnr(sse[r].cpu().numpy(), SIDE * SIDE))) for r in RS}

    # context, after the measured region: the same coding with two kernels
    # (coefficients written to HBM and read back)
    two = {}
    for r in RS:
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        adct.fwd2d(x, coef, stream=stream)
        adct.zonal_recon(coef, r, out, ref=x, image_height=SIDE, sse=sse[r], stream=stream)
        e0.record(stream)
        for _ in range(5):
            adct.fwd2d(x, coef, stream=stream)
        e1.record(stream)
        for _ in range(5):
            adct.zonal_recon(coef, r, out, ref=x, image_height=SIDE, sse=sse[r], stream=stream)
        e2.record(stream)
        e2.synchronize()
        two[r] = (e0.elapsed_time(e1) / 5, e1.elapsed_time(e2) / 5)
    fwd_ms = float(np.mean([v[0] for v in two.values()]))

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
        "roofline": {"bound": "hbm", "kernel": "encode_zonal (k_group fwd + coef + zonal inverse + SSE)",
                     "achieved": enc_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": enc_gbs / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_tile": ENC_BYTES_PER_TILE, "tiles_per_launch": ntiles,
                     "avg_launch_ms": enc_avg_ms},
        "kernels_ms": {f"encode_zonal_r{r}": enc_ms[r] for r in RS},
        "two_kernel_path": {
            "fwd2d_ms": fwd_ms, "fwd2d_gbs": FWD_BYTES_PER_TILE * ntiles / (fwd_ms * 1e-3) / 1e9,
            **{f"zonal_recon_r{r}_ms": two[r][1] for r in RS},
            **{f"zonal_recon_r{r}_gbs": recon_bytes_per_tile(r) * ntiles / (two[r][1] * 1e-3) / 1e9 for r in RS}},
        "psnr_db_mean": psnr,
        "input_gen_s": gen_s,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(img)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
