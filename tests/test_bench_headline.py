"""The benchmark's last stdout line is a compact headline: it must carry the
fields a reader of the run needs (metric, value, timing, config, roofline,
CPU baseline) and stay small whatever the detailed sections hold."""
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def full_result():
    """A result shaped like a full default run, with long detail sections."""
    runs = [{"blocks": 2629311, "label": f"load {i}", "p99_ms": 0.1234567891, "generator_limited": False,
             "extra": "x" * 200} for i in range(30)]
    fine = {"E_dB": -37.95123456, "E_dB_worst_filter": -27.57123, "frac_filters_above_-30dB": 0.01234567,
            "SD_dB_mean": 0.75123, "nnze_mean": 15.9912}
    pipe = {"topk_refit": fine, "l1_nnls_identity": dict(fine, host_s=1.2345),
            "l1_nnls_window_sigma_tuned_at_16_taps": dict(fine, host_s=11.2, sigma_grid=[15.0] * 6)}
    return {
        "metric": "output samples/s, sparse K=16 vs dense 200-tap on 1 GPU; p99 block latency",
        "value": 1.2623456789e12, "unit": "output samples/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "ms_per_step": 2.12712345678, "ms_median": 2.1243456, "ms_min": 2.0761234, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "sparse HRIR render: 64 pink sources x 1,048,576 samples x 20 directions x 2 ears, "
                               "K=16 of a 169-tap reflection filter, 32-tap resonance, 1,250-direction set",
                   "K": 16, "output_samples": 2684864000, "tile": 2048, "tiles": 32832, "grid": 32832,
                   "kernel": "quad", "sources": 64},
        "roofline": {"bound": "hbm", "achieved": 5175.123456, "peak": 8000.0, "unit": "GB/s", "frac": 0.64689123,
                     "traffic": 11053123456.0, "algorithmic_bytes": 11008339968.0, "kernel": "k_render_quad<32,16>"},
        "factorize": {"E_dB_aggregate": -37.95, "E_dB_worst_filter": -27.57, "frac_filters_above_-30dB": 0.012},
        "quality": {"headline_factorization": "x" * 100, "l1_continuation_T2000": pipe, "alg1_lambda0_T50": pipe,
                    "alg1_lambda0_T2000": pipe, "sigma_table_lambda0": {"identity_SD_dB_mean": 0.6}},
        "legs": {"dense_200": {"ms_per_step": 11.0712345, "speedup_sparse": 5.2012345},
                 "fft_ola": {"ms_per_step": 23.331234, "speedup_sparse": 10.9812345, "ms_by_nfft": {"1024": 1.0}},
                 "unfused": {"ms_per_step": 7.1312345, "speedup_fused": 3.3512345}},
        "k_sweep": {"8": {"ms_per_step": 2.0001234}, "32": {"ms_per_step": 3.4471234}},
        "uneven": {"ms_per_step": 0.8912345, "frac_hbm_peak": 0.5112345,
                   "best_any_shape": {"ms_per_step": 0.8312345}},
        "block_latency": {"p50_ms": 0.0240123, "p99_ms": 0.0375123},
        "serving": {"saturation_blocks_per_s": 2823456.789, "p99_ms_realtime": 0.107123, "runs": runs},
        "surrogate": {"heldout_E_dB_vs_factorization": {"frac_below_-30": 0.0}, "fallback_fraction": 1.0,
                      "moving_render": {"ms_per_step": 0.218123}},
        "cpu_baseline": {"value": 2.5012345e9, "unit": "output samples/s", "cores": 16, "kind": "oracle",
                         "host": {"model": "AMD EPYC 9575F 64-Core Processor", "nproc": 256, "affinity": 16},
                         "sample": "y" * 400},
    }


def test_headline_is_small_and_complete():
    bench = load_bench()
    res = full_result()
    assert len(json.dumps(res)) > 10000
    h = bench.headline(res, "gpurun_out/bench_detail.json")
    line = json.dumps(h)
    assert len(line.encode()) < bench.HEADLINE_MAX_BYTES, len(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "dtype", "config", "roofline",
              "cpu_baseline", "higher_is_better", "vs_baseline"):
        assert k in h, k
    assert h["config"]["workload"].startswith("sparse HRIR render")
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in h["roofline"], k
    for k in ("value", "unit", "cores", "kind"):
        assert k in h["cpu_baseline"], k
    assert abs(h["value"] - res["value"]) < 1e-5 * res["value"]
    assert abs(h["roofline"]["frac"] - res["roofline"]["frac"]) < 1e-3


def test_headline_without_optional_sections():
    bench = load_bench()
    res = full_result()
    for k in ("legs", "k_sweep", "uneven", "block_latency", "serving", "surrogate", "quality", "cpu_baseline",
              "factorize"):
        res.pop(k)
    h = bench.headline(res)
    assert "cpu_baseline" not in h and h["summary"] == {}
    assert len(json.dumps(h)) < bench.HEADLINE_MAX_BYTES
