"""Host-side pieces of bench.py (no GPU): the CPU baseline, the roofline
selection and the --gpus contract."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cpu_baseline_small():
    import bench
    from workloads import lattice, preferential_attachment

    graphs = [lattice(3, 3, lengths=(0.1, 2.0), seed=1), preferential_attachment(20, 1, lengths=(0.1, 2.0), seed=2),
              lattice(4, 5, lengths=(0.1, 2.0), seed=3), preferential_attachment(40, 1, lengths=(0.1, 2.0), seed=4)]
    r = bench.cpu_baseline(graphs, [3.0, 5.0, 7.0, 9.0], 1.0 / 32, "round", 0.75, 40, 8)
    assert r["kind"] == "oracle" and r["unit"] == "DOF-shift-solves/s"
    assert r["value"] > 0 and r["single_core_value"] > 0 and "extrapolated" in r["sample"]
    assert r["cores"] >= 1 and r["nproc"] >= 1 and isinstance(r["cpu_model"], str)


def test_multi_gpu_request_exits_with_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr


def _stats(ms, launches, pcg_ms=None, pcg_launches=None, vit=None, eit=None):
    keys = ["noise", "coeff", "ends_fwd", "ends_bwd", "condense", "pcg", "scatter", "acc_fwd", "acc_bwd", "layout",
            "mixed", "learned", "table"]
    return {"kernel_ms": {k: ms.get(k, 0.0) for k in keys},
            "kernel_launches": {k: launches.get(k, 0) for k in keys},
            "pcg_class_ms": pcg_ms or [0.0] * 7, "pcg_class_launches": pcg_launches or [0] * 7,
            "pcg_class_vertex_its": vit or [0] * 7, "pcg_class_end_its": eit or [0] * 7}


def test_roofline_picks_the_dominant_kernel_and_counts_its_work():
    import bench

    # pass A backward dominates: 2.5 flops per (interior DOF, shift, sample) over 2 launches of 5 ms
    st = _stats({"ends_fwd": 9.0, "ends_bwd": 10.0, "acc_fwd": 8.0, "pcg": 3.0, "noise": 1.0},
                {"ends_fwd": 2, "ends_bwd": 2, "acc_fwd": 2, "pcg": 2, "noise": 1},
                pcg_ms=[0, 0, 0, 3.0, 0, 0, 0], pcg_launches=[0, 0, 0, 2, 0, 0, 0])
    r = bench.roofline(st, n_dof=1000, n_interior=900, n_vertices=100, n_edges=200, L=40, S=64, mode="fp64")
    assert r["kernel_id"] == "ends_bwd" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert abs(r["avg_launch_ms"] - 5.0) < 1e-12
    assert abs(r["work_per_launch"] - 2.5 * 900 * 40 * 64 / 2) < 1e-6
    assert abs(r["achieved"] - r["work_per_launch"] / 5e-3 / 1e12) < 1e-12
    assert abs(r["frac"] - r["achieved"] / 78.6) < 1e-12
    # a PCG size class dominates: 2 flops per edge end + 11 per vertex, per iteration and system
    st = _stats({"ends_fwd": 1.0, "pcg": 30.0}, {"ends_fwd": 2, "pcg": 2},
                pcg_ms=[0, 0, 0, 0, 0, 24.0, 0], pcg_launches=[0, 0, 0, 0, 0, 2, 0],
                vit=[0, 0, 0, 0, 0, 1000, 0], eit=[0, 0, 0, 0, 0, 3000, 0])
    r = bench.roofline(st, 1000, 900, 100, 200, 40, 64, "mixed")
    assert r["kernel_id"] == "pcg_class5" and r["bound"] == "alu" and r["launches_per_step"] == 2
    assert abs(r["work_per_launch"] - (2 * 3000 + 11 * 1000) / 2) < 1e-9
    # the blocked pass A runs both directions in one launch: 5 flops per unit
    st = _stats({"ends_fwd": 12.0, "acc_fwd": 4.0}, {"ends_fwd": 2, "acc_fwd": 2})
    r = bench.roofline(st, 1000, 900, 100, 200, 40, 64, "fp64")
    assert r["kernel_id"] == "ends_fwd" and abs(r["work_per_launch"] - 5.0 * 900 * 40 * 64 / 2) < 1e-6
    assert bench.with_traffic(dict(r), "no such workload")["traffic"] is None
