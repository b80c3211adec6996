"""The benchmark's stdout line: compact enough for a log tail, with every
field of the measurement contract (value, roofline, CPU baseline)."""
import json

import bench


def _full_result():
    rs = bench.RS
    qp_row = {"fused_ms": 0.25, "fused_gbs": 4800.0, "two_kernel_ms": 0.5, "psnr_y_u_v_db": [40.0, 40.0, 40.0],
              "t8": {"ms": 0.26}, "mixed": {"ms": 0.4}}
    serve_row = {m: {"p50_ms": 0.05, "p99_ms": 0.4, "mean_ms": 0.1, "tiles_per_s": 2.4e7} for m in
                 ("persistent", "plain")}
    return {
        "metric": "16x16 blocks/s (fwd+inv) and fraction of HBM peak", "value": 3.5e9, "unit": "16x16 blocks/s",
        "n_gpus": 1, "steps": 20, "warmup": 5, "ms_per_step": 1.5, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "x" * 300, "images": 1024, "side": 512, "zonal_r": list(rs)},
        "roofline": {"bound": "hbm", "kernel": "k" * 80, "achieved": 5600.0, "peak": 8000.0, "unit": "GB/s",
                     "frac": 0.7, "traffic": 1.6e9, "bytes_per_tile": 1536, "tiles_per_launch": 1048576,
                     "avg_launch_ms": 0.28, "median_launch_ms": 0.28, "traffic_note": "n" * 120,
                     "frac_cache_reuse": 0.8, "avg_launch_ms_cache_reuse": 0.24, "copy_probe_gbs": 5200.0},
        "codec_form": {"kernels": "fwd2d then zonal_recon", "ms_per_r": 0.45, "bytes_per_tile_moved": 2200.0,
                       "frac": 0.64, "bytes_per_tile_int32_codec": 2560, "frac_int32_codec_basis": 0.74},
        "kernels_ms": {f"encode_zonal_r{r}": 0.25 for r in rs},
        "psnr_db_mean": {r: 25.0 for r in rs},
        "cpu_baseline": {"value": 3.0e6, "unit": "16x16 blocks/s", "cores": 16, "kind": "oracle", "sample": "s" * 200,
                         "single_thread": {"value": 2e5}, "numpy_oracle": {"value": 1e5}},
        "other_workloads": {
            "video_residuals_64x1920x1088": {"qp": {q: dict(qp_row) for q in (22, 27, 32, 37)}},
            "uneven_batch_4096": {"tiles": 17660000, "ms": 5.3, "frac_of_8tbs": 0.64,
                                  "quant_qp27": {"ms": 4.05, "frac_of_8tbs": 0.56}},
            "serving_poisson": {"rate": {lam: serve_row for lam in (200, 500, 1000, 2000, 5000)},
                                "capacity": {m: {"max_rate_p99_within_bound": 10000, "p99_bound_ms": 1.0,
                                                 "tiles_per_s": 1.2e8, "burst_tiles_per_s": 2.0e8,
                                                 "burst_p99_ms": 50.0,
                                                 "tried": {lam: {"p50_ms": 0.1, "p99_ms": 0.5, "tiles_per_s": 1e8}
                                                           for lam in bench.CAPACITY_RATES}}
                                             for m in ("persistent", "plain")},
                                "dma_policy": {lam: {pol: {"p50_ms": 0.05, "p99_ms": 0.36, "mean_ms": 0.1,
                                                           "dma_copies": 400} for pol in ("adaptive", "by_size")}
                                               for lam in bench.SERVE_POLICY_RATES}},
            "image_experiment_zigzag_1024x512x512": {"r": {r: {"psnr_db": 30.0} for r in bench.ZIGZAG_R}},
            "t32_images_1024x512x512": {"r": {r: {"frac_of_8tbs": 0.7} for r in bench.T32_RS}},
            "t64_images_1024x512x512": {"r": {r: {"frac_of_8tbs": 0.5} for r in bench.T64_RS}},
        },
        "detail_file": "gpurun_out/bench_detail.json",
    }


def test_summary_line_is_compact_and_complete():
    line = bench.summary_line(_full_result())
    text = json.dumps(line)
    assert len(text) < 4096, len(text)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "dtype", "config", "roofline",
              "cpu_baseline", "vs_baseline", "higher_is_better", "scaling", "data"):
        assert k in line, k
    assert "workload" in line["config"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in line["roofline"], k
    assert set(line["cpu_baseline"]) == {"value", "unit", "cores", "kind", "sample"}
    assert "\n" not in text
    assert set(line["other_workloads"]["t64_zonal_frac"]) == {str(r) for r in bench.T64_RS}
    assert set(line["other_workloads"]["serving_p99_ms_dma_adaptive_vs_by_size"]) == \
        {str(lam) for lam in bench.SERVE_POLICY_RATES}


def test_summary_line_without_other_workloads():
    full = _full_result()
    del full["other_workloads"], full["cpu_baseline"]
    line = bench.summary_line(full)
    assert "other_workloads" not in line and len(json.dumps(line)) < 4096
