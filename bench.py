"""Throughput benchmark: sample-shift DOF-solves per second on one MI355X.

One step = one grf_sample call on the 64x64 random-length lattice (4096
vertices, 8064 edges, h = 1/256 rounded mesh, ~2.07M DOFs), kappa = 10,
beta = 0.6, quadrature step 0.3 (116 shifts), 256 samples: noise, every
shift's condensed solve, accumulation and the output layout, with the inputs
(graph, mesh) resident on the device.  value = N_dof * shifts * samples /
seconds per step.

Prints one JSON line (rank 0).  Also reports the roofline of the dominant
kernel (HIP-event durations recorded inside the timed steps), the FP64 CPU
oracle timed on a bounded sample of the same workload, and (unless
--no-forms) the other forms of the method measured in the same run:
  mixed                  the same lattice with FP32 edge sweeps (error vs FP64 reported);
  nn                     the same lattice with the paper's Neumann-Neumann preconditioner;
  and on a batch of 64 uneven graphs (trees and lattices, 100..20000 edges),
  every form with its PCG at tolerance 1e-8 and its error against the FP64
  batch at tolerance 1e-12 reported (the metric counts results within 1e-6):
  batch_plain_per_graph  the plain method: one grf_sample call per graph, FP64, Jacobi,
  batch_plain            one batched call (captured graph replayed), FP64, Jacobi,
  batch_mixed            one batched call, FP32 edge sweeps, Jacobi,
  batch_nn               one batched call, FP64, Neumann-Neumann preconditioner,
  batch_learned_mixed    one batched call, FP32 edge sweeps, learned preconditioner
                         (trained on the GPU in this run on small graphs of the same kinds),
                         with the PCG variant of each size class picked by the autotuner;
  batch_learned_mixed_op the same with the learned operator and initial guess in every class.
--workload rgg100k times the learned preconditioner's held-out graph (98k vertices) instead;
--workload lattice256 the 256x256 lattice (66.7M DOFs) in FP64 and mixed precision.
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

METRIC = "sample-shift DOF-solves/sec at 1e-6 rel err: learned+batched vs plain, 1 GPU"
# PCG tolerance of the batch forms: their samples stay within 1e-6 of the FP64
# result at tolerance 1e-12 (reported with each form)
METRIC_TOL = 1e-8
# Adam phases (steps, learning rate) of the learned preconditioner's training, 16 shifts x 4 samples per step
TRAIN_PHASES = ((3000, 5e-3), (3000, 2e-3), (1000, 5e-4))
TRAIN_STEPS = sum(n for n, _ in TRAIN_PHASES)
BATCH_WORKLOAD = "64 uneven graphs (trees + lattices, 100..20000 edges) h=1/128 beta=0.75 S=32, PCG tol 1e-8"
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64, matrix cores (dense) and vector units alike; FMA = 2 flops
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X FP32 matrix cores, dense

# Algorithmic FP64 flops per (interior DOF, real shift, sample) of each timed
# edge kernel: the Thomas recurrences themselves (forward elimination
# y = r + rho y and the output update x += g y are one FMA each), whatever the
# blocking.  Padding shifts and the blocked form's extra work are not counted.
#   blocked (matrix cores): pass A per direction = elimination + output (4),
#                           pass B = two end-column updates (4)
#   streamed (vector ALU):  end sweeps = elimination (2), recovery sweeps = 4
EDGE_FLOPS = {
    "blocked": {"ends_fwd": 4.0, "ends_bwd": 4.0, "acc_fwd": 4.0},
    "mixed": {"ends_fwd": 4.0, "ends_bwd": 4.0, "acc_fwd": 4.0},
    "streamed": {"ends_fwd": 2.0, "ends_bwd": 2.0, "acc_fwd": 4.0, "acc_bwd": 4.0},
}
HIP_KERNEL = {
    "blocked": {"ends_fwd": "k_sweep_blocked<8, true>", "ends_bwd": "k_sweep_blocked<8, false>",
                "acc_fwd": "k_corr_blocked<8>"},
    "mixed": {"ends_fwd": "k_sweep_blocked32<8, true>", "ends_bwd": "k_sweep_blocked32<8, false>",
              "acc_fwd": "k_corr_blocked32<8>"},
    "streamed": {"ends_fwd": "k_sweep_ends<BL, true>", "ends_bwd": "k_sweep_ends<BL, false>",
                 "acc_fwd": "k_sweep_acc<BL, true>", "acc_bwd": "k_sweep_acc<BL, false>"},
}
# HBM bytes per launch of the blocked edge kernels on this workload (rocprofv3
# FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0 KiB: the factors a 1 GiB plain copy
# reads on these counters), valid only for the kernel source they were taken on.
TRAFFIC_SOURCE = "paper_2605_02670_amd/csrc/blocked.hip"
TRAFFIC_SHA256 = "567b9b8afdc3c9e0fc035d721ca3a88746bc6740cf9ab833f2b62ac144c70747"
TRAFFIC = {  # kernel id: (fetch KiB, write KiB) per launch
    "ends_fwd": (4425197.5625, 5996584.0),
    "ends_bwd": (6568436.125, 5980456.0),
    "acc_fwd": (5662891.1875, 4125736.0),
}
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0


def _traffic(dom: str, mode: str):
    import hashlib

    if mode != "blocked" or dom not in TRAFFIC:
        return None
    with open(os.path.join(ROOT, TRAFFIC_SOURCE), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != TRAFFIC_SHA256:
            return None  # kernel changed since the counters were taken
    fetch, write = TRAFFIC[dom]
    return 1024.0 * (FETCH_FACTOR * fetch + WRITE_FACTOR * write)


def cpu_baseline(cfg, L: int, S: int, n_shift_sample: int = 3, n_samp: int = 4) -> dict:
    """Time the FP64 oracle (numpy Philox noise, one sparse LU per shift) on a
    bounded sample and extrapolate the whole job linearly:
        t_job = S t_noise + L (t_factor + S t_rhs),
    with t_factor and t_rhs fitted from solves with 1 and n_samp right-hand sides."""
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):
        return _cpu_baseline(cfg, L, S, n_shift_sample, n_samp)


def _cpu_baseline(cfg, L: int, S: int, n_shift_sample: int, n_samp: int) -> dict:
    import numpy as np

    from oracle import mesh as omesh
    from oracle import noise as onoise
    from oracle import quadrature as oquad
    from oracle import solve as osolve

    g = cfg["graph"]
    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    ML = omesh.lumped_mass(m)
    t0 = time.perf_counter()
    W = onoise.white_noise(ML, cfg["seed"], n_samp)
    t_noise = (time.perf_counter() - t0) / n_samp
    _, cI, cL = oquad.shifts(cfg["beta"], cfg["quad_step"])
    idx = np.linspace(0, len(cI) - 1, n_shift_sample).round().astype(int)
    times = {}
    for ns in (1, n_samp):
        t0 = time.perf_counter()
        for i in idx:
            osolve.solve_shifted(m, cfg["kappa"], float(cI[i]), float(cL[i]), W[:ns])
        times[ns] = (time.perf_counter() - t0) / n_shift_sample
    t_rhs = max(0.0, (times[n_samp] - times[1]) / (n_samp - 1))
    t_factor = max(0.0, times[1] - t_rhs)
    t_job = S * t_noise + L * (t_factor + S * t_rhs)
    return {"value": m.n_dof * L * S / t_job, "unit": "DOF-shift-solves/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (numpy Philox noise, scipy splu per shift, 1 thread) on the same graph: noise for "
                      f"{n_samp} samples ({t_noise:.2f} s/sample) and {n_shift_sample} shifts solved with 1 and "
                      f"{n_samp} right-hand sides (factor+assemble {t_factor:.2f} s/shift, {t_rhs:.3f} s/rhs); "
                      f"whole job ({S} samples x {L} shifts) extrapolated as S*t_noise + L*(t_factor + S*t_rhs)"}


def _batch_setup():
    import torch

    from paper_2605_02670_amd import grf
    from workloads import config_c3

    cfg = config_c3()
    Gs = [grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"]) for g in cfg["graphs"]]
    outs = [torch.empty((cfg["n_samples"], G.n_dof), dtype=torch.float64, device="cuda") for G in Gs]
    return cfg, Gs, outs


def run_batched(cfg, Gs, outs, steps: int, warmup: int, **kw) -> dict:
    """Times grf_sample_batched over the 64-graph batch (the first call tunes and captures)."""
    import torch

    from paper_2605_02670_amd import grf

    S = cfg["n_samples"]
    t0 = time.perf_counter()
    grf.sample_batched(Gs, cfg["kappas"], cfg["beta"], 0.0, S, cfg["seed"], outs=outs, **kw)
    first = time.perf_counter() - t0
    for _ in range(max(0, warmup - 1)):
        grf.sample_batched(Gs, cfg["kappas"], cfg["beta"], 0.0, S, cfg["seed"], outs=outs, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [grf.sample_batched(Gs, cfg["kappas"], cfg["beta"], 0.0, S, cfg["seed"], outs=outs, timing=True,
                                **kw)[1] for _ in range(steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    L = stats[0]["n_shifts"]
    ndof = sum(G.n_dof for G in Gs)
    return {"value": ndof * L * S / dt, "ms_per_step": dt * 1e3, "first_call_s": first, "n_dof": ndof,
            "shifts": L, "samples": S, "graphs": len(Gs),
            "pcg": {"max_iterations": max(s_["max_iterations"] for s_ in stats),
                    "mean_iterations": stats[0]["total_iterations"] / max(1, stats[0]["n_systems"]),
                    "class_variants": grf.class_modes(stats[0]["pcg_class_modes"])}}


def run_per_graph(cfg, steps: int, **kw):
    """Times the plain method on the batch's graphs: one grf_sample call per
    graph, each graph timed after a warm-up call and released before the next
    (a handle keeps its workspace).  Returns (result dict, outputs)."""
    import torch

    from paper_2605_02670_amd import grf

    S = cfg["n_samples"]
    total, ndof, its, nsys, maxit, L = 0.0, 0, 0, 0, 0, 0
    outs = []
    for g, kap in zip(cfg["graphs"], cfg["kappas"]):
        G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
        o = torch.empty((S, G.n_dof), dtype=torch.float64, device="cuda")
        G.sample(float(kap), cfg["beta"], 0.0, S, cfg["seed"], out=o, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st = G.sample(float(kap), cfg["beta"], 0.0, S, cfg["seed"], out=o, **kw)
        torch.cuda.synchronize()
        total += (time.perf_counter() - t0) / steps
        ndof += G.n_dof
        L = st["n_shifts"]
        its += st["total_iterations"]
        nsys += st["n_systems"]
        maxit = max(maxit, st["max_iterations"])
        outs.append(o)
        G.close()
    return ({"value": ndof * L * S / total, "ms_per_step": total * 1e3, "n_dof": ndof, "shifts": L, "samples": S,
             "graphs": len(outs), "pcg": {"max_iterations": maxit, "mean_iterations": its / max(1, nsys)}}, outs)


def train_network(seed: int = 0):
    """Trains the learned preconditioner on the GPU on small graphs of the batch's kinds
    (preferential-attachment trees and lattices, 100..2000 edges, h = 1/128)."""
    import numpy as np

    from paper_2605_02670_amd import grf
    from workloads import lattice, preferential_attachment
    from workloads.learned_init import init_params

    rng = np.random.default_rng(1000 + seed)
    graphs, kappas = [], []
    for i in range(8):
        n_e = int(np.exp(rng.uniform(np.log(100), np.log(2000))))
        if i % 2 == 0:
            g = preferential_attachment(n_e + 1, 1, lengths=(0.1, 2.0), seed=int(rng.integers(1 << 30)))
        else:
            nx = max(2, int(round(np.sqrt(n_e / 2.0))))
            g = lattice(nx, max(2, int(round(n_e / (2.0 * nx)))), lengths=(0.1, 2.0), seed=int(rng.integers(1 << 30)))
        graphs.append(grf.Graph(g.n_vertices, g.edges, g.lengths, 1.0 / 128, "round"))
        kappas.append(float(rng.uniform(2.0, 20.0)))
    net = grf.Learned(init_params(seed))
    t0 = time.perf_counter()
    losses = np.concatenate([net.train(graphs, kappas, 0.75, 0.0, n_samples=4, seed=seed + 11 + 7 * k, n_steps=n,
                                       shifts_per_step=16, lr=lr) for k, (n, lr) in enumerate(TRAIN_PHASES)])
    t = time.perf_counter() - t0
    for G in graphs:
        G.close()
    return net, t, float(losses[:400].mean()), float(losses[-400:].mean())


def _batch_rel_err(Gs, cfg, outs, ref):
    """max over graphs and samples of ||u - ref||_{M_L} / ||ref||_{M_L}."""
    import numpy as np

    from oracle import mesh as omesh

    worst = 0.0
    for g, a, b in zip(cfg["graphs"], outs, ref):
        ML = omesh.lumped_mass(omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"]))
        r = b.cpu().numpy()
        d = a.cpu().numpy() - r
        worst = max(worst, float(np.max(np.sqrt((d * d * ML).sum(1) / (r * r * ML).sum(1)))))
    return worst


def train_network_rgg(seed: int = 0):
    """Trains the learned preconditioner on the GPU on the held-out graph's kind: 16
    random geometric graphs of 2k..20k points, h = 1/256, kappa ~ U[2, 20]."""
    from paper_2605_02670_amd import grf
    from workloads import config_c5_train
    from workloads.learned_init import init_params

    tr = config_c5_train()
    Gs = [grf.Graph(d["graph"].n_vertices, d["graph"].edges, d["graph"].lengths, 1.0 / 256, "round") for d in tr]
    net = grf.Learned(init_params(seed))
    t0 = time.perf_counter()
    for k, (n, lr) in enumerate(TRAIN_PHASES):
        net.train(Gs, [d["kappa"] for d in tr], 0.75, 0.0, n_samples=4, seed=seed + 11 + 7 * k, n_steps=n,
                  shifts_per_step=16, lr=lr)
    t = time.perf_counter() - t0
    for G in Gs:
        G.close()
    return net, t


def bench_rgg(args) -> int:
    """The held-out random geometric graph (98,129 vertices, 199,826 edges, h =
    1/256, 38.4M DOFs), kappa = 2, beta = 0.75 (229 shifts), 64 samples, PCG
    tol 1e-8: one grf_sample call per step with Jacobi, the learned
    preconditioner (trained first, on the GPU, on 16 smaller graphs of the
    same kind), the Neumann-Neumann preconditioner, and learned + FP32 edge
    sweeps.  value: the learned form."""
    import torch

    from paper_2605_02670_amd import grf
    from workloads import config_c5_eval

    net, t_train = train_network_rgg()
    torch.cuda.empty_cache()
    cfg = config_c5_eval()
    g = cfg["graph"]
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    S = cfg["n_samples"]
    out = torch.empty((S, G.n_dof), dtype=torch.float64, device="cuda")
    steps = max(1, min(args.steps, 2))
    forms, ref = {}, None
    for name, kw in (("jacobi", {}), ("learned", {"learned": net}), ("nn", {"precond": "nn"}),
                     ("learned_mixed", {"learned": net, "precision": "mixed"})):
        G.sample(cfg["kappa"], cfg["beta"], 0.0, S, cfg["seed"], out=out, tol=METRIC_TOL, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = [G.sample(cfg["kappa"], cfg["beta"], 0.0, S, cfg["seed"], out=out, tol=METRIC_TOL, timing=True,
                          **kw)[1] for _ in range(steps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st = stats[0]
        f = {"value": G.n_dof * st["n_shifts"] * S / dt, "ms_per_step": dt * 1e3,
             "pcg_ms": sum(s_["kernel_ms"]["pcg"] for s_ in stats) / steps,
             "learned_ms": sum(s_["kernel_ms"]["learned"] for s_ in stats) / steps,
             "pcg": {"max_iterations": st["max_iterations"],
                     "mean_iterations": st["total_iterations"] / max(1, st["n_systems"])}}
        if ref is None:
            ref = out[:8].clone()
        else:
            f["rel_err_vs_jacobi_8_samples"] = float(((out[:8] - ref).norm(dim=1) / ref.norm(dim=1)).max())
        forms[name] = f
        print(f"# {name}: {dt * 1e3:.0f} ms, PCG {f['pcg_ms']:.0f} ms, mean iterations "
              f"{f['pcg']['mean_iterations']:.2f}", file=sys.stderr, flush=True)
    for k in ("learned", "nn", "learned_mixed"):
        forms[k]["speedup_vs_jacobi"] = forms["jacobi"]["ms_per_step"] / forms[k]["ms_per_step"]
    lf = forms["learned"]
    line = {
        "metric": METRIC, "value": lf["value"], "unit": "DOF-shift-solves/s", "n_gpus": 1, "steps": steps,
        "warmup": 1, "ms_per_step": lf["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"held-out random geometric graph {g.n_vertices} vertices {g.edges.shape[0]} edges "
                               f"h=1/256 kappa=2 beta=0.75 S={S} PCG tol {METRIC_TOL:g} learned",
                   "n_dof": G.n_dof, "shifts": stats[0]["n_shifts"], "samples": S, "parallelism": "1 GPU"},
        "roofline": None, "cpu_baseline": None,
        "training": {"seconds": t_train, "steps": TRAIN_STEPS, "graphs": "16 random geometric graphs, 2k..20k points"},
        "forms": forms,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_lattice256(args) -> int:
    """The 256x256 lattice (65,536 vertices, 130,560 edges, h = 1/512, about 66.7M DOFs),
    kappa = 20, beta = 0.55, step 0.2 with |l| <= 46 (93 shifts, e^{2y} in [1e-8, 1e8]),
    64 samples: one grf_sample call per step in FP64 and with FP32 edge sweeps; the mixed
    sample's error against the FP64 one (8 samples, lumped-mass norm) is reported.
    value: the mixed form."""
    import numpy as np
    import torch

    from oracle import mesh as omesh
    from paper_2605_02670_amd import grf
    from workloads import config_c4

    cfg = config_c4()
    g = cfg["graph"]
    S = cfg["n_samples"]
    steps = max(1, min(args.steps, 3))
    outs, forms = {}, {}
    for name, prec in (("fp64", "fp64"), ("mixed", "mixed")):
        # a handle per form: each plans its shift blocks with the whole memory (a handle keeps its workspace)
        G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
        out = torch.empty((S, G.n_dof), dtype=torch.float64, device="cuda")
        kw = dict(tol=cfg["tol"], precision=prec, k_minus=cfg["k_minus"], k_plus=cfg["k_plus"],
                  shift_block=args.shift_block)
        G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"], out=out, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = [G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"], out=out, timing=True,
                          **kw)[1] for _ in range(steps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st = stats[0]
        forms[name] = {"value": G.n_dof * st["n_shifts"] * S / dt, "ms_per_step": dt * 1e3,
                       "shift_block": st["shift_block"],
                       "kernel_ms_per_step": {k: sum(s_["kernel_ms"][k] for s_ in stats) / steps
                                              for k in st["kernel_ms"] if st["kernel_ms"][k] > 0},
                       "pcg": {"max_iterations": st["max_iterations"],
                               "mean_iterations": st["total_iterations"] / max(1, st["n_systems"])}}
        outs[name] = out[:8].clone()
        n_dof = G.n_dof
        del out
        G.close()
        torch.cuda.empty_cache()
        print(f"# {name}: {dt * 1e3:.1f} ms per call", file=sys.stderr, flush=True)
    ML = omesh.lumped_mass(omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"]))
    d = (outs["mixed"] - outs["fp64"]).cpu().numpy()
    r = outs["fp64"].cpu().numpy()
    forms["mixed"]["rel_err_vs_fp64_8_samples"] = float(np.max(np.sqrt((d * d * ML).sum(1) / (r * r * ML).sum(1))))
    forms["mixed"]["speedup_vs_fp64"] = forms["fp64"]["ms_per_step"] / forms["mixed"]["ms_per_step"]
    mf = forms["mixed"]
    line = {
        "metric": METRIC, "value": mf["value"], "unit": "DOF-shift-solves/s", "n_gpus": 1, "steps": steps,
        "warmup": 1, "ms_per_step": mf["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"lattice256x256 U[0.5,1.5] h=1/512 kappa=20 beta=0.55 k=0.2 |l|<=46 S={S} "
                               f"mixed-fp32sweeps-jacobi", "n_dof": n_dof, "shifts": stats[0]["n_shifts"],
                   "samples": S, "parallelism": "1 GPU"},
        "roofline": None, "cpu_baseline": None, "forms": forms,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_batched(args) -> int:
    """64 uneven graphs (preferential-attachment trees and lattices, 100..20000
    edges, h = 1/128), one kappa per graph, all 176 shifts x 32 samples in one
    grf_sample_batched call (captured HIP graph replayed each step)."""
    cfg, Gs, outs = _batch_setup()
    kw = dict(tol=args.tol if args.tol else cfg["tol"], precision=args.precision, sweep_block=args.sweep_block,
              shift_block=args.shift_block)
    net = None
    if args.precond == "learned":
        net = train_network()[0]
        kw["learned"] = net
        if args.learned_variants == "op":
            kw["pcg_class_modes"] = ["op"] * 5 + ["guess"]
    elif args.precond == "nn":
        kw["precond"] = "nn"
    r = run_batched(cfg, Gs, outs, args.steps, args.warmup, **kw)
    line = {
        "metric": METRIC, "value": r["value"], "unit": "DOF-shift-solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": f"64 uneven graphs (trees + lattices, 100..20000 edges) h=1/128 beta=0.75 "
                               f"S={r['samples']} PCG tol {kw['tol']:g} batched-{args.precision}-{args.precond}"
                               + ("-op" if "pcg_class_modes" in kw else ""),
                   "n_dof": r["n_dof"], "shifts": r["shifts"], "samples": r["samples"], "graphs": r["graphs"],
                   "parallelism": "1 GPU"},
        "roofline": None, "cpu_baseline": None, "first_call_s": r["first_call_s"], "pcg": r["pcg"],
    }
    print(json.dumps(line), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--beta", type=float, default=0.6)
    ap.add_argument("--samples", type=int, default=256)
    ap.add_argument("--sweep-block", type=int, default=0)
    ap.add_argument("--shift-block", type=int, default=0)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="mixed: FP32 edge sweeps, FP64 noise/Schur/PCG/accumulation")
    ap.add_argument("--tol", type=float, default=0.0,
                    help="PCG tolerance of the batched64 workload (0: the configuration's, 1e-12)")
    ap.add_argument("--precond", choices=["jacobi", "learned", "nn"], default="jacobi",
                    help="vertex PCG preconditioner of the batched64 workload (learned: trained first, on the GPU)")
    ap.add_argument("--learned-variants", choices=["auto", "op"], default="auto",
                    help="batched64 with the learned preconditioner: PCG variant per size class as the autotuner "
                         "picks it, or the learned operator forced in every class")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the mixed / batched / learned forms")
    ap.add_argument("--workload", choices=["lattice64", "batched64", "rgg100k", "lattice256"], default="lattice64",
                    help="lattice64: one 64x64 lattice (default); batched64: 64 uneven graphs in one batched call; "
                         "rgg100k: the learned preconditioner's held-out random geometric graph; lattice256: the "
                         "256x256 lattice in FP64 and mixed precision")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built "
              "(samples shard across GPUs with no communication)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2605_02670_amd import grf
    from workloads import config_c2

    grf.load()
    torch.cuda.set_device(0)
    if args.workload == "batched64":
        return bench_batched(args)
    if args.workload == "rgg100k":
        return bench_rgg(args)
    if args.workload == "lattice256":
        return bench_lattice256(args)
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg = config_c2(beta=args.beta, n_samples=args.samples)
    g = cfg["graph"]
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    S = cfg["n_samples"]
    km, kp, k = G.shift_count(cfg["beta"], cfg["quad_step"])
    L = km + kp + 1
    out = torch.empty((S, G.n_dof), dtype=torch.float64, device="cuda")
    kw = dict(tol=cfg["tol"], sweep_block=args.sweep_block, shift_block=args.shift_block, precision=args.precision)

    def step(timing=False):
        _, st = G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"], out=out, timing=timing, **kw)
        return st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step(timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps

    value = G.n_dof * L * S / dt
    # dominant kernel over the timed steps (HIP events on the library's launch stream)
    ktot = {k_: sum(s["kernel_ms"][k_] for s in stats) for k_ in stats[0]["kernel_ms"]}
    kl = {k_: sum(s["kernel_launches"][k_] for s in stats) for k_ in stats[0]["kernel_launches"]}
    dom = max(ktot, key=ktot.get)
    mode = ("mixed" if args.precision == "mixed" else "blocked") if stats[0]["sweep_block"] == 0 else "streamed"
    roof = None
    if dom in EDGE_FLOPS[mode] and kl[dom] > 0:
        avg_ms = ktot[dom] / kl[dom]
        launches_per_step = kl[dom] / args.steps
        flops = EDGE_FLOPS[mode][dom] * G.n_interior * L * S / launches_per_step
        achieved = flops / (avg_ms * 1e-3) / 1e12
        peak = FP32_MFMA_PEAK_TFLOPS if mode == "mixed" else FP64_PEAK_TFLOPS
        roof = {"bound": "alu" if mode == "streamed" else "mfma", "kernel": HIP_KERNEL[mode][dom],
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": _traffic(dom, mode),
                "avg_launch_ms": avg_ms, "flops_per_launch": flops}

    # correctness at full size: <diag M_L, u> = q_k(kappa^2) <1, W> per sample (any size, exact identity)
    from oracle import quadrature as oquad

    w = G.noise(8, cfg["seed"]).cpu().numpy()
    u = out[:8].cpu().numpy()
    from oracle import mesh as omesh

    m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    ML = omesh.lumped_mass(m)
    q = oquad.q_k(cfg["kappa"] ** 2, cfg["beta"], cfg["quad_step"])
    lhs, rhs = (u * ML).sum(1), q * w.sum(1)
    cons_err = float(np.max(np.abs(lhs - rhs)) / np.max(np.abs(rhs)))
    check = {"conservation_rel_err": cons_err}
    if args.precision == "mixed":
        # error of the mixed result against the FP64 path (itself within 1e-10 of the oracle), 8 samples,
        # relative in the lumped-mass norm
        ref, _ = G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], 8, cfg["seed"], tol=cfg["tol"],
                          sweep_block=args.sweep_block, shift_block=args.shift_block)
        d = (out[:8] - ref).cpu().numpy()
        r = ref.cpu().numpy()
        check["rel_err_vs_fp64"] = float(np.max(np.sqrt((d * d * ML).sum(1) / (r * r * ML).sum(1))))

    cpu = None if args.no_cpu_baseline else cpu_baseline(cfg, L, S)
    n_dof, n_interior = G.n_dof, G.n_interior
    forms = None
    if not args.no_forms and args.precision == "fp64":
        forms = {"plain": {"value": value, "ms_per_step": dt * 1e3}}
        # mixed precision on the same lattice
        kwm = dict(kw, precision="mixed")
        outm = torch.empty_like(out)
        for _ in range(args.warmup):
            G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"], out=outm, **kwm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"], out=outm, **kwm)
        torch.cuda.synchronize()
        dtm = (time.perf_counter() - t0) / args.steps
        d = (outm - out).cpu().numpy()
        r_ = out.cpu().numpy()
        errm = float(np.max(np.sqrt((d * d * ML).sum(1) / (r_ * r_ * ML).sum(1))))
        forms["mixed"] = {"value": G.n_dof * L * S / dtm, "ms_per_step": dtm * 1e3, "rel_err_vs_fp64": errm}
        # the paper's Neumann-Neumann preconditioner on the same lattice (FP64)
        kwn = dict(kw, precond="nn")
        for _ in range(args.warmup):
            G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"], out=outm, **kwn)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stn = [G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"], out=outm, **kwn)[1]
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        dtn = (time.perf_counter() - t0) / args.steps
        d = (outm - out).cpu().numpy()
        forms["nn"] = {"value": G.n_dof * L * S / dtn, "ms_per_step": dtn * 1e3,
                       "rel_err_vs_jacobi": float(np.max(np.sqrt((d * d * ML).sum(1) / (r_ * r_ * ML).sum(1)))),
                       "pcg": {"max_iterations": max(s_["max_iterations"] for s_ in stn),
                               "mean_iterations": stn[0]["total_iterations"] / max(1, stn[0]["n_systems"])}}
        del outm
        # the lattice handle's workspace would otherwise shrink the batch's shift blocks
        n_dof, n_interior = G.n_dof, G.n_interior
        G.close()
        del out
        torch.cuda.empty_cache()
        # the 64-graph batch, every form at the metric's accuracy: PCG tolerance
        # METRIC_TOL, error against the FP64 batch at tol 1e-12 reported
        from workloads import config_c3

        bsteps = max(1, min(args.steps, 2))
        pg, pg_outs = run_per_graph(config_c3(), bsteps, tol=METRIC_TOL)
        bcfg, Gs, bouts = _batch_setup()
        run_batched(bcfg, Gs, bouts, 1, 1, tol=bcfg["tol"])
        ref = [o.cpu() for o in bouts]  # host copies: HBM stays free for the forms' shift blocks
        pg["rel_err_vs_fp64_tol1e-12"] = _batch_rel_err(Gs, bcfg, pg_outs, ref)
        del pg_outs
        torch.cuda.empty_cache()
        forms["batch_plain_per_graph"] = dict(pg, workload=BATCH_WORKLOAD + "; plain method: one grf_sample per "
                                                                            "graph, FP64, Jacobi")
        for name, kwb, what in (("batch_plain", {}, "FP64, Jacobi"),
                                ("batch_mixed", {"precision": "mixed"}, "FP32 edge sweeps, Jacobi"),
                                ("batch_nn", {"precond": "nn"}, "FP64, Neumann-Neumann preconditioner")):
            r_ = run_batched(bcfg, Gs, bouts, bsteps, 1, tol=METRIC_TOL, **kwb)
            r_["rel_err_vs_fp64_tol1e-12"] = _batch_rel_err(Gs, bcfg, bouts, ref)
            forms[name] = dict(r_, workload=BATCH_WORKLOAD + "; one batched call, " + what)
        net, t_train, l0, l1 = train_network()
        torch.cuda.empty_cache()
        bl = run_batched(bcfg, Gs, bouts, bsteps, 1, tol=METRIC_TOL, learned=net, precision="mixed")
        bl["rel_err_vs_fp64_tol1e-12"] = _batch_rel_err(Gs, bcfg, bouts, ref)
        bl["training"] = {"seconds": t_train, "steps": TRAIN_STEPS, "phases": TRAIN_PHASES, "loss_first400": l0,
                          "loss_last400": l1,
                          "graphs": "8 trees/lattices, 100..2000 edges"}
        forms["batch_learned_mixed"] = dict(bl, workload=BATCH_WORKLOAD + "; one batched call, FP32 edge sweeps, "
                                                                          "learned preconditioner, PCG variant per "
                                                                          "size class as the autotuner picks it")
        blo = run_batched(bcfg, Gs, bouts, bsteps, 1, tol=METRIC_TOL, learned=net, precision="mixed",
                          pcg_class_modes=["op"] * 5 + ["guess"])
        blo["rel_err_vs_fp64_tol1e-12"] = _batch_rel_err(Gs, bcfg, bouts, ref)
        forms["batch_learned_mixed_op"] = dict(blo, workload=BATCH_WORKLOAD + "; one batched call, FP32 edge "
                                                                              "sweeps, learned operator and initial "
                                                                              "guess forced in every size class")
        base = forms["batch_plain_per_graph"]["value"]
        forms["batch_speedup_vs_plain_per_graph"] = {k: forms[k]["value"] / base for k in
                                                     ("batch_plain", "batch_mixed", "batch_nn",
                                                      "batch_learned_mixed", "batch_learned_mixed_op")}
    line = {
        "metric": METRIC, "value": value, "unit": "DOF-shift-solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": f"lattice64x64 U[0.5,1.5] h=1/256 kappa=10 beta={cfg['beta']} k=0.3 "
                               f"S={S} {'plain-fp64' if args.precision == 'fp64' else 'mixed-fp32sweeps'}-jacobi",
                   "n_dof": n_dof, "n_interior": n_interior, "shifts": L, "samples": S,
                   "shift_block": stats[0]["shift_block"], "sweep_block": stats[0]["sweep_block"],
                   "parallelism": "1 GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernel_ms_per_step": {k_: v / args.steps for k_, v in ktot.items() if v > 0},
        "pcg": {"max_iterations": max(s["max_iterations"] for s in stats),
                "mean_iterations": stats[0]["total_iterations"] / max(1, stats[0]["n_systems"])},
        "check": check,
        "forms": forms,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
