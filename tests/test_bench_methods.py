"""CPU checks of the benchmark's measurement arithmetic: the Section VI
speedup curve and the one-line result that the benchmark prints."""
import json

import pytest

import bench


def test_speedup_curve_hand_trace():
    """Fig. 6 method on a hand-built trace: the level of ALS-NCG iteration k
    is the mean of its norms after k-1 and k; j = first ALS iteration at or
    below it; speedup = j t_ALS / (k t_NCG); a level ALS never reaches gives
    the lower bound len(trace) t_ALS / (k t_NCG)."""
    g_ncg = [1.0, 0.5, 0.1, 0.01]
    g_als = [0.9, 0.7, 0.5, 0.3, 0.2, 0.1, 0.06]
    rows = bench.speedup_vs_gnorm(g_ncg, g_als, ms_als=1.0, ms_ncg=2.0)
    assert [r["ncg_iteration"] for r in rows] == [2, 3, 4]
    # k = 2: level 0.75, ALS reaches 0.7 at j = 2: 2 * 1 / (2 * 2)
    assert rows[0]["gnorm_over_N"] == pytest.approx(0.75)
    assert rows[0]["als_iterations"] == 2 and rows[0]["speedup"] == pytest.approx(0.5)
    # k = 3: level 0.3, reached exactly at j = 4 (<= counts): 4 / 6
    assert rows[1]["als_iterations"] == 4 and rows[1]["speedup"] == pytest.approx(4.0 / 6.0)
    assert rows[1]["speedup_at_least"] is None
    # k = 4: level 0.055, below every ALS norm: lower bound 7 * 1 / (4 * 2)
    assert rows[2]["als_iterations"] is None and rows[2]["speedup"] is None
    assert rows[2]["speedup_at_least"] == pytest.approx(7.0 / 8.0)


def test_speedup_curve_uses_the_moving_average_not_the_last_norm():
    """A non-monotone NCG trace: the level after a spike is the average, so
    ALS needs fewer iterations than the last norm alone would ask for."""
    rows = bench.speedup_vs_gnorm([0.4, 0.2, 0.6], [0.5, 0.35, 0.3, 0.25, 0.2],
                                  ms_als=3.0, ms_ncg=1.0)
    assert rows[0]["gnorm_over_N"] == pytest.approx(0.3) and rows[0]["als_iterations"] == 3
    assert rows[1]["gnorm_over_N"] == pytest.approx(0.4) and rows[1]["als_iterations"] == 2
    assert rows[1]["speedup"] == pytest.approx(2 * 3.0 / (3 * 1.0))


def _full_result():
    """A result of the full benchmark's shape with long traces in it."""
    rates = {str(r): {"requests": 10 * r, "p50_ms": 0.1, "p99_ms": 0.2, "solves_per_s": float(r),
                      "errors": 0} for r in (10_000, 50_000, 200_000)}
    c3 = {"gnorm_over_N_tol": 1e-6, "steps": 20}
    for nf in bench.C3_NF:
        d = {"train_nnz": 1, "held_out": 1}
        for form in ("fp32", "bf16_refined", "bf16"):
            d[form] = {"heldout_rmse_after_5": 0.9, "heldout_rmse_after_25": 0.8,
                       "rel_f_err_vs_fp64": [1e-7] * 5, "max_abs_factor_diff_vs_fp64": 1e-3,
                       "compared_after_iterations": 5, "ms_per_iteration": 10.0,
                       "phase_ms": {"a": 1.0}, "f_after": {}, "iterations_to_g_tol": 50,
                       "final_gnorm_over_N": 1e-7, "seconds_to_g_tol": 0.5}
        c3[str(nf)] = d
    curve = [{"ncg_iteration": k, "gnorm_over_N": 1.0 / k, "als_iterations": 3 * k,
              "speedup": 1.5, "speedup_at_least": None} for k in range(2, 26)]
    tt = {"f_gap_tol": 1e-6, "gnorm_over_N_tol": 1e-6, "f_star": 1.0,
          "speedup_f_tol": 7.0, "speedup_g_tol": 1.4, "speedup_exact_search_f_tol": 8.0,
          "speedup_exact_search_g_tol": 1.5,
          "ranking_accuracy": {"acceleration": {"70%": 0.5, "100%": 7.0},
                               "als": {"accuracy_at": {str(k): 0.5 for k in range(100)}}}}
    for name in ("als", "als_ncg", "als_ncg_exact_search"):
        tt[name] = {"iterations_to_f_tol": 100, "seconds_to_f_tol": 1.0,
                    "iterations_to_g_tol": 50, "seconds_to_g_tol": 0.5}
    return {
        "metric": bench.METRIC, "value": 4.123456789e9, "unit": "ratings/s", "n_gpus": 1,
        "steps": 20, "warmup": 5, "ms_per_step": 9.7, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "w", "n_f": 100},
        "roofline": {"bound": "mfma", "achieved": 57.8, "peak": 157.3, "unit": "TFLOP/s",
                     "frac": 0.367, "traffic": None, "kernel": "k", "flops_per_launch": 2.5e11,
                     "launch_ms": 4.41, "algorithmic_bytes": 3.4e8},
        "cpu_baseline": {"value": 8.5e6, "unit": "ratings/s", "cores": 16, "kind": "oracle",
                         "sample": "s", "cpu": "c",
                         "half_sweep_ratings_per_s": {"threads_16": 1e7, "threads_1": 1e6}},
        "half_sweep_ratings_per_s": {"U": 4.5e9, "M": 7e9},
        "phase_ms": {"sweep_U": 4.4, "sweep_M": 2.8}, "pass_hbm_gbs": {"linesearch": 238.0},
        "f": 1.234567890123e6, "time_to_tol": tt,
        "ranking_accuracy_small": {"acceleration": {"70%": 0.5}},
        "ranking_kernels": {"top_t_ms": 20.0, "accuracy_ms": 25.0},
        "fold_in": {"continuous_batching": {"rates": rates},
                    "one_request_per_launch": {"rates": rates}},
        "reduced_precision": c3,
        "length_bins": {"U": {"dual_max": 78, "split_copy": 1}, "M": {"dual_max": 62, "split_copy": 0}},
        "grad_slices": {"best": {"slices": 8, "ms": 0.7}, "trials": [{"slices": 0, "ms": 1.1}]},
        "split_copy": {"U": 1, "M": 0},
        "scale_1e9": {"als": {"ms_per_sweep": 100.0}, "sweep_U_tflops_eager": 31.5,
                      "tuning": {"U": {"best": {"dual_max": 46, "split_copy": 1}},
                                 "M": {"best": {"dual_max": 0, "split_copy": 0, "grad_slices": 0}}},
                      "als_ncg": {"ms_per_iteration": 280.0, "ratings_per_s": 7e9,
                                  "phase_ms_eager_step": {"sweep_U": 99.0}},
                      "speedup_vs_gnorm": {"curve": curve,
                                           "als_gnorm_over_N": [1e-3] * 100}},
    }


def test_compact_line_keeps_the_headline_and_fits_the_log_tail():
    res = _full_result()
    line = json.dumps(bench.compact(res, "/x/gpurun_out/bench_full.json"), separators=(",", ":"))
    assert len(line) < 4096, len(line)
    d = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config"):
        assert k in d, k
    assert d["roofline"]["frac"] == 0.367 and d["roofline"]["bound"] == "mfma"
    assert d["cpu_baseline"]["kind"] == "oracle" and d["cpu_baseline"]["cores"] == 16
    assert d["time_to_tol"]["speedup_f_tol"] == 7.0
    assert d["fold_in_p99_ms"]["200000"] == 0.2
    assert d["reduced_precision"]["bf16_refined_nf128"]["rmse"] == 0.8
    assert d["scale_1e9"]["als_ncg_ms_per_iteration"] == 280.0
    assert d["value"] == pytest.approx(res["value"], rel=1e-5)
    # the plan choices behind the numbers
    assert d["dual_max"] == {"U": 78, "M": 62}
    assert d["split_copy"] == {"U": 1, "M": 0} and d["grad_slices"] == 8
    assert d["scale_1e9"]["split_copy"] == {"U": 1, "M": 0}
    assert d["scale_1e9"]["grad_slices"] == 0


def test_profiled_traffic_matches_hash_bound_and_split_copy(tmp_path, monkeypatch):
    """The roofline's traffic is taken only from a TRAFFIC line of the same
    kernel sources, length bound and split-copy choice (a line without the
    split-copy key stands for the split in the loop)."""
    (tmp_path / "profiles").mkdir()
    lines = [
        'TRAFFIC {"dual_max": 78, "split_copy": 1, "source_hash": "h1", "bytes": 11}',
        'TRAFFIC {"dual_max": 78, "split_copy": 0, "source_hash": "h1", "bytes": 12}',
        'TRAFFIC {"dual_max": 62, "source_hash": "h1", "bytes": 13}',
        'TRAFFIC {"dual_max": 62, "split_copy": 1, "source_hash": "old", "bytes": 14}',
    ]
    (tmp_path / "profiles" / "sweep_chunks_f32_nf100_ml20m_shape.md").write_text(
        "text\n" + "\n".join("    " + x for x in lines) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h1")
    assert bench.profiled_traffic(78, 1) == 11
    assert bench.profiled_traffic(78, 0) == 12
    assert bench.profiled_traffic(78) == 12
    assert bench.profiled_traffic(62, 0) == 13
    assert bench.profiled_traffic(62, 1) is None  # taken on other sources
    assert bench.profiled_traffic(94, 1) is None
