"""The benchmark's last stdout line is one compact JSON object (the driver keeps only the tail of
stdout): it carries the contract's fields, the roofline and the CPU baseline, and stays well under
4 KB with every section filled; the tables go to the full record."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _method(k=32, c=32):
    return dict(ms_per_step=5.55555, mrays_s=2985.4321, encode_ms=0.1, sort_ms=0.5, trace_ms=5.3,
                trace_ms_mean=5.31, trace_only_mrays_s=3100.0, wall_s=0.1, cut=c, key_bits=k, skip_bits=16,
                trace_opts=dict(block=64, stack=2, xcd_remap=0, persistent=1, refill=32, chunk=64, waves=8192,
                                flags=2))


def _full():
    methods = {m: _method() for m in ("nosort", "twopoint", "hcc", "hcc_paper_exact")}
    methods["hcc_paper_exact"]["skip_bits"] = 0
    rows = [dict(method=f"variant number {i} with a long name", mrays_s=2500.5 + i) for i in range(8)]
    brows = ([dict(method="nosort", mrays_s=2500.0, ms=6.4, tuned=True),
              dict(method="twopoint K=32", mrays_s=2600.0, ms=6.2, tuned=True),
              dict(method="hcc C=16 K=16 skip 8", mrays_s=2400.0, ms=6.7, tuned=True)] + rows)
    fetch = dict(node_fetches_per_ray=26.712, tri_fetches_per_ray=3.123, bytes_per_ray=1859.3, waves_modelled=32400,
                 wave_stride=8, anc64=1.234, anc32=1.111)
    return {
        "metric": bench.METRIC, "workload": "w" * 160, "steps": 20, "warmup": 5, "triangles": 1012012,
        "rays": 16588800, "headline": "hcc", "methods": methods,
        "cut_composition": dict(sorted_nodes=32, leaves=3, distinct_boxes=30),
        "shadow": dict(rays=33177600, **{m: dict(ms=7.9, mrays_s=4158.12) for m in methods}),
        "packets": {name: dict(lane_ms=6.5887, packet_ms=8.4635, lane_opts=methods["hcc"]["trace_opts"],
                               packet_opts=methods["hcc"]["trace_opts"])
                    for name in ("primary nosort", "shadow nosort", "shadow hcc C=32 K=32",
                                 "shadow hcc C=16 K=16 skip 8", "shadow twopoint K=32")},
        "fetches": dict(model={m: fetch for m in methods}, kernel_counted=None),
        "frame_bounces": {b: dict(rays=16588000, rows=brows) for b in ("2", "3")},
        "batched": dict(engine_hcc_mrays_s=1122.5, plain_hcc_mrays_s=353.5, engine_nosort_mrays_s=1138.0,
                        plain_nosort_mrays_s=402.1, tuning=[dict(ms=1.0)] * 50),
        "serve": dict(loads={rho: dict(plain=dict(p50_ms=22.639, p99_ms=75.06, mrays_s=420.0),
                                       continuous=dict(p50_ms=1.806, p99_ms=10.04, mrays_s=425.5))
                             for rho in ("0.5", "0.8", "0.95")}),
        "drift": dict(bounces={b: dict(rows=rows + [dict(method="nosort", mrays_s=500.0),
                                                    dict(method="hcc C=16 K=16", mrays_s=535.0)])
                               for b in ("1", "2")},
                      shadow=dict(rows=[dict(method="nosort", mrays_s=700.0), dict(method="twopoint K=32", mrays_s=820.0),
                                        dict(method="hcc C=16 K=16", mrays_s=735.0),
                                        dict(method="hcc C=32 K=32", mrays_s=742.0),
                                        dict(method="mlhcc32 (16+16)", mrays_s=760.0)])),
        "roofline": dict(bound="hbm", achieved=6924.4, peak=8000.0, unit="GB/s", frac=0.8656, traffic=10334608383,
                         kernel="k_trace_wide<closest>", launch_ms=5.3101, bytes_per_ray=2222.7,
                         numerator="oracle wave model (BVH2 nodes, 64-lane waves)", kernel_counted_bytes_per_ray=2300.1),
        "cpu_baseline": dict(value=3.2354, unit="Mrays/s", cores=16, kind="oracle", sample="s" * 200,
                             prim_agreement_with_gpu=1.0, single_thread=dict(value=0.262, cores=1, sample="x" * 60)),
    }


def test_compact_line_fields_and_size():
    args = bench.parse(["--steps", "20", "--warmup", "5"])
    line = bench.compact_line(_full(), args, "w" * 160)
    text = json.dumps(line, separators=(",", ":"))
    assert len(text) < 4096, len(text)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in line, k
    assert line["config"]["workload"]
    assert set(line["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert set(line["cpu_baseline"]) >= {"value", "unit", "cores", "kind", "sample"}
    assert "hcc_paper_exact" in line["methods"] and line["paper_exact_vs_nosort"] == 1.0
    assert line["sort32"]["bytes_per_key"] == 68 and 0 < line["sort32"]["frac"] < 1
    assert line["shadow_speedup_vs_nosort"] == 1.0
    assert line["packet_vs_lane_ms"]["shadow twopoint K=32"] == [6.5887, 8.4635]
    assert len(line["packet_vs_lane_ms"]) == 5
    assert line["drift_shadow_hcc_vs_nosort"] == 1.06
    assert line["drift_shadow_best_mrays_s"] == [820.0, "twopoint K=32"]
    # three bounces: (16588800 + 2 x 16588000) rays over 5.55555 + 6.4 + 6.4 ms for NoSort
    assert abs(line["frame_3_bounces_mrays_s"]["nosort"] - 49764800 / 18.35555e-3 / 1e6) < 0.1
    assert set(line["frame_3_bounces_mrays_s"]) == {"nosort", "twopoint", "hcc"}
    assert json.loads(text) == line


def test_multi_gpu_refused(capsys):
    import pytest
    with pytest.raises(SystemExit) as e:
        bench.main(["--gpus", "2"])
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
