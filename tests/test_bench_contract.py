"""The bench script's command-line contract, checked without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _stub_detail():
    """A full bench result of realistic size: 64 per-scene adjoint records,
    per-kernel tables in every section."""
    kern = {k: {"launches": 1234, "total_ms": 12.3456789, "avg_us": 9.87654321, "bytes_per_launch": 4.4e6,
                "achieved_GBps": 456.789, "frac_hbm": 0.0571234} for k in ("cg_iter", "p2g", "g2p", "grad_hess")}
    roof = {"bound": "hbm", "kernel": "k_cg_iter", "achieved": 456.789, "peak": 8000.0, "unit": "GB/s",
            "frac": 0.0571234, "traffic": 5.77e6, "avg_us": 9.87654321, "bytes_per_launch": 4.4e6, "launches": 1234}
    return {
        "metric": "m" * 80, "value": 2.8e7, "unit": "particle-steps/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "ms_per_step": 5.4321, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "w" * 120, "N_B": 62308, "N_S": 45244, "M": 2, "path": "mixed",
                   "schwarz_iters_mean": 2.65, "newton_per_frame_mean": 12.3, "cg_per_frame_mean": 432.1,
                   "cg_per_newton_mean": 35.1, "ls_halvings_per_frame_mean": 0.0, "inner_unconverged_total": 0,
                   "inner_ls_failed_total": 0, "tile_B": [8, 8], "tile_S": [8, 8]},
        "particle_updates_per_s_incl_schwarz_iters": 7.4e7,
        "tile_tuning_ms_per_frame": {"B(%d, %d) S(8, 8)" % (i, i): 5.5 for i in range(10)},
        "roofline": roof, "kernels": kern, "profiled_pass_ms_per_step": 6.1,
        "fp64_gpu_path": {"value": 1.8e7, "ms_per_step": 8.5, "schwarz_iters_mean": 2.6, "roofline": roof,
                          "kernels": kern},
        "speedup_vs_fp64_gpu": 1.56,
        "cpu_baseline": {"value": 5.6e4, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
                         "sample": "s" * 100, "host": {"model": "AMD EPYC 9575F 64-Core Processor",
                                                       "logical_cpus": 256, "usable_cpus": 16}},
        "paper_context": {"x": "y" * 200},
        "parity": {"frames": 5, "vs": "FP64 CPU oracle", "path": "mixed", "max_rel_err": 1.2e-7,
                   "u_B": 1e-7, "u_S": 1e-7, "x_B": 1e-9, "x_S": 1e-9},
        "batched": {"workload": "b" * 200, "scenes": 64, "particles": 6000000, "value": 1.33e8,
                    "ms_per_step": 44.4, "schwarz_iters_mean": 2.7, "tile": [16, 8],
                    "tile_tuning_ms_per_frame": {str(i): 50.0 for i in range(5)}, "roofline": roof, "kernels": kern},
        "large": [{"workload": "hertz", "frames": "1-2", "value": 5e8, "ms_per_step": 3.9, "schwarz_iters_mean": 2,
                   "cg_per_frame_mean": 54, "kernels": kern},
                  {"workload": "fold", "frames": "1-1", "value": 1e6, "ms_per_step": 1000.0,
                   "schwarz_iters_mean": 28, "cg_per_frame_mean": 22338, "kernels": kern}],
        "graphs": {"solves": "s" * 80, "frames": "1-10",
                   "direct": {"ms_per_step": 5.0, "schwarz_iters": [30] * 10, "cg_per_frame_mean": 2000.0},
                   "cycle_graphs": {"ms_per_step": 5.1, "schwarz_iters": [30] * 10, "cg_per_frame_mean": 2000.0},
                   "iteration_graphs": {"ms_per_step": 4.9, "schwarz_iters": [30] * 10,
                                        "cg_per_frame_mean": 2000.0},
                   "max_rel_diff_vs_direct": {"cycle_graphs": 1e-9, "iteration_graphs": 1e-9},
                   "iteration_graph_speedup": 1.02},
        "multi_domain": {"multi": {"ms_per_step": 6.14}, "union": {"ms_per_step": 5.85},
                         "max_rel_diff_multi_vs_union": {"B": 3e-8, "S": 3e-8}},
        "adjoint": {"frames": 100, "forward_ms_per_frame": 5.5, "backward_ms_per_frame": 16.1,
                    "dL_dE": [1.0, 2.0], "implicit": {"backward_ms_per_frame": 14.7, "rel_diff_vs_unrolled": 1.8e-8}},
        "adjoint_batched": {"scenes": 64, "frames": 100, "checkpoint_every": 10, "targets_forward_s": 7.5,
                            "forward_s": 7.0, "backward_s": 60.0, "particle_steps_per_s_forward_and_reverse": 8.8e6,
                            "sign_agrees_with_E_minus_E_target": 64,
                            "per_scene": [{"scene": s, "loss": 1e-9, "dL_dE": [1e-10, 1e-13], "E_inclusion": 3e4,
                                           "E_target": 1e5} for s in range(64)]},
    }


def test_summary_line_is_compact_and_keeps_the_contract():
    sys.path.insert(0, ROOT)
    import json

    import bench

    detail = _stub_detail()
    assert len(json.dumps(detail)) > 10000  # the full result is what overflowed a 10 KB tail
    line = bench.compact_summary(detail, "gpurun_out/bench_detail.json")
    text = json.dumps(line, separators=(",", ":"))
    assert len(text) < bench.SUMMARY_MAX_BYTES, len(text)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in line, k
    assert line["config"]["workload"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in line["roofline"], k
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in line["cpu_baseline"], k
    assert json.loads(text)["value"] == detail["value"]


def test_summary_line_stays_under_the_limit_with_a_long_error():
    sys.path.insert(0, ROOT)
    import json

    import bench

    detail = _stub_detail()
    detail["large"][1] = {"workload": "fold", "error": "e" * 6000}
    line = bench.compact_summary(detail, "gpurun_out/bench_detail.json")
    text = json.dumps(line, separators=(",", ":"))
    assert len(text) < bench.SUMMARY_MAX_BYTES, len(text)
    assert line["value"] == detail["value"] and line["roofline"]["frac"] is not None
    assert line["large"] == "in the detail file"
