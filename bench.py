"""Throughput benchmark: sample-shift DOF-solves per second on one MI355X.

Headline (default): the metric's comparison, the learned + batched (+ mixed)
form against the plain method, on 64 uneven graphs (32 preferential-attachment
trees and 32 near-square lattices, 100..20000 edges, lengths U[0.1, 2],
h = 1/128, kappa_g ~ U[2, 20], beta = 0.75, the paper's step: 176 shifts,
32 samples, 27,969,427 DOFs).  One step is one grf_sample_batched call: noise,
every shift's condensed solve, accumulation and the output layout for all 64
graphs, with the PCG at tolerance 1e-8 and the learned preconditioner's size
class variants as the autotuner picks them (the network is trained on the GPU
first, on small graphs of the same kinds).  value = sum_g N_g * 176 * 32 /
seconds per step; the plain method (one FP64 Jacobi grf_sample per graph) is
timed beside it and every form's error against the FP64 result at tolerance
1e-12 is reported (the metric counts results within 1e-6).

The JSON line also carries:
  roofline      the dominant kernel of the headline step (largest summed time in
                a separate run with per-kernel HIP events), its algorithmic work
                per launch over its average launch time against its peak;
  hbm           the step's HBM fraction from the algorithmic bytes of the edge
                work, and from rocprofv3 counter bytes when they are recorded for
                these sources;
  cpu_baseline  the FP64 condensed oracle timed on a bounded sample of the same
                workload, on all host cores (one process per shift) and on one;
  forms         the other forms: the batch forms, the 64x64 lattice (beta 0.6:
                FP64, mixed, Neumann-Neumann, with its own roofline; beta 0.85),
                the 256x256 lattice (FP64, mixed) and the learned
                preconditioner's held-out random geometric graph (Jacobi, learned,
                Neumann-Neumann, learned + mixed).
--workload picks one workload alone (lattice64, batched64, lattice256, rgg100k).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sample-shift DOF-solves/sec at 1e-6 rel err: learned+batched vs plain, 1 GPU"
UNIT = "DOF-shift-solves/s"
# PCG tolerance of the timed forms: their samples stay within 1e-6 of the FP64
# result at tolerance 1e-12 (reported with each form)
METRIC_TOL = 1e-8
# Adam phases (steps, learning rate) of the learned preconditioner's training, 16 shifts x 4 samples per step
TRAIN_PHASES = ((3000, 5e-3), (3000, 2e-3), (1000, 5e-4))
TRAIN_STEPS = sum(n for n, _ in TRAIN_PHASES)
BATCH_WORKLOAD = ("64 uneven graphs (32 preferential-attachment trees + 32 lattices, 100..20000 edges) "
                  "lengths U[0.1,2] h=1/128 kappa_g~U[2,20] beta=0.75 paper step (176 shifts) S=32, PCG tol 1e-8")

# MI355X peaks (dense): HBM3E, FP64 (matrix cores and vector units alike), FP32 matrix cores
PEAK = {"hbm": 8000.0, "fp64": 78.6, "fp32_mfma": 157.3}

# Algorithmic FP64/FP32 flops per (interior DOF, real shift, sample) of the edge
# work, 10 in all (the plain Thomas solve and recovery of one DOF-shift-solve):
# the solve of T w = W (forward elimination 2, back substitution 3) split evenly
# over the two directions of pass A (5 for the blocked launch that runs both), and
# pass B's two end-column updates (4) plus the accumulation into u (1).
EDGE_FLOPS = {"ends_fwd": 2.5, "ends_bwd": 2.5, "acc_fwd": 5.0}
# Algorithmic HBM bytes of the streaming steps, per unit:
#   noise    8 per (DOF, sample) written
#   coeff    32 per (edge, shift): |b|, rho_{m-1} and the Schur block (s_d, s_o) written
#   table    the Thomas rows of every (interior DOF, shift): 8 (FP64) or 4 (FP32 tables)
#   condense 16 per (edge, shift, sample) of end values read + 8 per (vertex, shift, sample) written
#   scatter  24 per (vertex, shift, sample)
#   layout   16 per (DOF, sample) (the output transpose)
# Vertex PCG per size class (FP64 vector ALU): 2 flops per edge end and 11 per
# vertex for each iteration of each system (the Jacobi-scaled product, two dot
# products and three vector updates).
PCG_FLOPS_PER_END, PCG_FLOPS_PER_VERTEX = 2.0, 11.0


def _hip_kernels(mode: str) -> dict:
    if mode == "mixed":
        return {"ends_fwd": "k_sweep_blocked32<NT>", "ends_bwd": "k_sweep_ends<BL, false>",
                "acc_fwd": "k_corr_blocked32<NT>", "table": "k_blocktab<float, PACK>"}
    return {"ends_fwd": "k_sweep_blocked<NT>", "ends_bwd": "k_sweep_ends<BL, false>",
            "acc_fwd": "k_corr_blocked<NT>", "table": "k_blocktab<double, PACK>"}


PCG_KERNELS = ["k_pcg_chip<64, 1>", "k_pcg_chip<64, 4>", "k_pcg_chip<128, 8>", "k_pcg_chip<512, 8>",
               "k_pcg_chip<1024, 10>", "k_pcg_chip<1024, 20>", "k_pcg_mrhs<4>"]

# rocprofv3 counter bytes (FETCH_SIZE x 2 + WRITE_SIZE x 1 KiB, the factors a plain 1 GiB
# copy reads on these counters) per step, recorded for these sources only
COUNTER_SOURCES = ["paper_2605_02670_amd/csrc/" + f for f in
                   ("blocked.hip", "pcg.hip", "sample.hip", "noise.hip", "layout.hip", "graph.hip", "common.h")]
COUNTER_SHA = "28ad82b3c908de622f011a67d3af6a6d78fc1d08a464219e398dfc8d93c3b100"  # sha256 over COUNTER_SOURCES when the counters below were taken
# workload -> {"step_bytes": B, "kernels": {kernel id: bytes per launch}}, from the two counter passes
# of profiles/grf_sample_batched64_S32_hbm_counters.md and grf_sample_lattice64_S256_hbm_counters.md
COUNTERS = {
    "batched64": {"step_bytes": 542124682750, "kernels": {"ends_fwd": 90680296214, "table": 65918028787}},
    "lattice64_beta0.6": {"step_bytes": 87645906277, "kernels": {"ends_fwd": 35494569415, "table": 12285991058}},
}




def _sources_sha() -> str:
    h = hashlib.sha256()
    for f in COUNTER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counters(workload: str):
    if COUNTER_SHA is None or workload not in COUNTERS or _sources_sha() != COUNTER_SHA:
        return None
    return COUNTERS[workload]


def _sync():
    import torch

    torch.cuda.synchronize()


def _rel_err(outs, refs, mls) -> float:
    """max over graphs and samples of ||u - ref||_{M_L} / ||ref||_{M_L} (M_L from the library)."""
    import torch

    worst = 0.0
    for a, b, ml in zip(outs, refs, mls):
        b = b.to(a.device)
        m = torch.from_numpy(ml).to(a.device)
        d = a - b
        worst = max(worst, float(torch.sqrt((d * d * m).sum(1) / (b * b * m).sum(1)).max()))
    return worst


def _timed(fn, steps: int, warmup: int):
    """warmup untimed calls, then `steps` calls bracketed by device synchronisation;
    returns (seconds per step, median of per-call times over min(steps, 10) calls synchronised
    one by one, the last call's result)."""
    r = None
    for _ in range(warmup):
        r = fn()
    _sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = fn()
    _sync()
    dt = (time.perf_counter() - t0) / max(1, steps)
    per = []
    for _ in range(min(steps, 10)):
        t1 = time.perf_counter()
        fn()
        _sync()
        per.append(time.perf_counter() - t1)
    return dt, statistics.median(per) if per else dt, r


# ---- roofline of the dominant kernel ---------------------------------------------------

def roofline(st: dict, n_dof: int, n_interior: int, n_vertices: int, n_edges: int, L: int, S: int,
             mode: str) -> dict:
    """The kernel with the largest summed time in a timed call (stats with per-kernel HIP
    events), with its algorithmic work per launch over its average launch time."""
    flops_peak = PEAK["fp32_mfma"] if mode == "mixed" else PEAK["fp64"]
    names = _hip_kernels(mode)
    cands = []
    ms, nl = st["kernel_ms"], st["kernel_launches"]
    for k in ("ends_fwd", "ends_bwd", "acc_fwd"):
        if nl[k]:
            # the blocked pass A runs both directions in one launch (no separate backward launches)
            fl = EDGE_FLOPS[k] * (2 if k == "ends_fwd" and not nl["ends_bwd"] else 1)
            w = fl * n_interior * L * S
            cands.append((ms[k], k, names[k], "mfma", w / nl[k], ms[k] / nl[k], "TFLOP/s", flops_peak,
                          f"{fl} flops per (interior DOF, shift, sample)"))
    hb = {"noise": (8.0 * n_dof * S, "8 B per (DOF, sample)", "k_noise"),
          "coeff": (32.0 * n_edges * L, "32 B per (edge, shift)", "k_edge_coeff"),
          "table": ((4.0 if mode == "mixed" else 8.0) * n_interior * L,
                    f"{4 if mode == 'mixed' else 8} B per (interior DOF, shift) (the Thomas rows)", names["table"]),
          "condense": ((16.0 * n_edges + 8.0 * n_vertices) * L * S,
                       "16 B per (edge, shift, sample) + 8 B per (vertex, shift, sample)", "k_condense"),
          "scatter": (24.0 * n_vertices * L * S, "24 B per (vertex, shift, sample)", "k_vertex_scatter"),
          "layout": (16.0 * n_dof * S, "16 B per (DOF, sample)", "k_from_interleaved")}
    for k, (b, rule, kn) in hb.items():
        if nl[k]:
            cands.append((ms[k], k, kn, "hbm", b / nl[k], ms[k] / nl[k], "GB/s", PEAK["hbm"], rule))
    for c in range(7):
        n = st["pcg_class_launches"][c]
        if n:
            f = PCG_FLOPS_PER_END * st["pcg_class_end_its"][c] + PCG_FLOPS_PER_VERTEX * st["pcg_class_vertex_its"][c]
            cands.append((st["pcg_class_ms"][c], f"pcg_class{c}", PCG_KERNELS[c], "alu", f / n,
                          st["pcg_class_ms"][c] / n, "TFLOP/s", PEAK["fp64"],
                          "2 flops per edge end + 11 per vertex, per iteration and system"))
    tot, kid, kname, bound, work, avg_ms, unit, peak, rule = max(cands)
    scale = 1e9 if unit == "GB/s" else 1e12
    achieved = work / (avg_ms * 1e-3) / scale
    return {"bound": bound, "kernel": kname, "kernel_id": kid, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": None, "avg_launch_ms": avg_ms,
            "launches_per_step": (nl[kid] if kid in nl else st["pcg_class_launches"][int(kid[-1])]),
            "work_per_launch": work, "work_rule": rule,
            "share_of_step": tot / max(1e-9, sum(ms.values()))}


def with_traffic(roof: dict, workload: str) -> dict:
    """roofline["traffic"]: the dominant kernel's counter bytes per launch, when counters were taken
    on these sources for this workload and kernel (else None)."""
    c = _counters(workload)
    roof["traffic"] = None if c is None else c["kernels"].get(roof["kernel_id"])
    return roof


def step_hbm(n_dof: int, n_interior: int, L: int, S: int, n_passes: int, mode: str, step_ms: float,
             workload: str) -> dict:
    """The step's HBM bandwidth fraction, from the edge work's algorithmic bytes: per shift pass,
    W read twice and the accumulator read and written (32 B per DOF and sample in FP64, 16 in
    mixed precision), plus the Thomas rows of every (interior DOF, shift) (8 or 4 B)."""
    per = 16.0 if mode == "mixed" else 32.0
    rows = 4.0 if mode == "mixed" else 8.0
    alg = per * n_dof * S * n_passes + rows * n_interior * L
    out = {"algorithmic_bytes": alg, "algorithmic_frac": alg / (step_ms * 1e-3) / (PEAK["hbm"] * 1e9),
           "rule": f"{per:g} B per (DOF, sample) per shift pass + {rows:g} B per (interior DOF, shift)",
           "counter_bytes": None, "counter_frac": None}
    c = _counters(workload)
    if c is not None:
        out["counter_bytes"] = c["step_bytes"]
        out["counter_frac"] = c["step_bytes"] / (step_ms * 1e-3) / (PEAK["hbm"] * 1e9)
    return out


# ---- CPU baseline: the condensed oracle on the host -------------------------------------

def _cpu_info() -> dict:
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def _one_thread():
    from threadpoolctl import threadpool_limits

    threadpool_limits(limits=1)


def _oracle_task(args):
    """One (graph, shift) of the job on the host: factor, then solve n_rhs loads."""
    import numpy as np

    from oracle import condensed as ocond
    from oracle import mesh as omesh

    nv, edges, lengths, h, rule, kappa, cI, cL, n_rhs = args
    m = omesh.build_mesh(nv, edges, lengths, h, rule)
    W = np.random.default_rng(0).standard_normal((n_rhs, m.n_dof))
    t0 = time.perf_counter()
    ocond.Shifted(m, kappa, cI, cL).solve(W)
    return time.perf_counter() - t0


def cpu_baseline(graphs, kappas, h, rule, beta, L: int, S: int) -> dict:
    """The FP64 oracle (oracle/condensed.py: LAPACK tridiagonal factorisation per shift, the
    vertex system by SuperLU, the Philox noise of oracle/noise.py) on a bounded sample of the
    job: four of its graphs (smallest to largest), three shifts each, 1 and 4 loads.  One core:
    per-DOF costs of noise, factorisation and each load, extrapolated to the whole job
    (sum_g N_g (S t_noise + L (t_factor + S t_rhs))).  All cores: the same (graph, shift)
    tasks, 4 loads each, run by one process per core; value = one-core value x the measured
    parallel speedup (sum of task times / wall time)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import condensed as ocond
    from oracle import mesh as omesh
    from oracle import noise as onoise
    from oracle import quadrature as oquad

    order = np.argsort([g.edges.shape[0] for g in graphs])
    pick = [int(order[i]) for i in np.linspace(0, len(order) - 1, 4).round().astype(int)]
    k = oquad.paper_step(beta, h)
    _, cI, cL = oquad.shifts(beta, k)
    sidx = [0, len(cI) // 2, len(cI) - 1]
    n_samp = 4
    t_noise = t_fac = t_rhs = 0.0
    n_pick = 0
    tasks = []
    with threadpool_limits(limits=1):
        for gi in pick:
            g = graphs[gi]
            m = omesh.build_mesh(g.n_vertices, g.edges, g.lengths, h, rule)
            ML = omesh.lumped_mass(m)
            n_pick += m.n_dof
            t0 = time.perf_counter()
            W = onoise.white_noise(ML, 0, n_samp)
            t_noise += (time.perf_counter() - t0) / n_samp
            for i in sidx:
                t0 = time.perf_counter()
                sh = ocond.Shifted(m, float(kappas[gi]), float(cI[i]), float(cL[i]))
                t1 = time.perf_counter()
                sh.solve(W[:1])
                t2 = time.perf_counter()
                sh.solve(W)
                t3 = time.perf_counter()
                r = max(0.0, ((t3 - t2) - (t2 - t1)) / (n_samp - 1))
                t_rhs += r / len(sidx)
                t_fac += ((t1 - t0) + max(0.0, (t2 - t1) - r)) / len(sidx)
                tasks.append((g.n_vertices, g.edges, g.lengths, h, rule, float(kappas[gi]), float(cI[i]),
                              float(cL[i]), n_samp))
    n_tot = sum(omesh.build_mesh(g.n_vertices, g.edges, g.lengths, h, rule).n_dof for g in graphs)
    per_dof = (S * t_noise + L * (t_fac + S * t_rhs)) / n_pick
    t_job = per_dof * n_tot
    one = n_tot * L * S / t_job
    info = _cpu_info()
    P = max(1, min(16, info["affinity"]))
    speedup = 1.0
    if P > 1:
        with cf.ProcessPoolExecutor(max_workers=P, mp_context=mp.get_context("spawn"), initializer=_one_thread) as ex:
            list(ex.map(_oracle_task, [tasks[0]] * P))  # start the workers
            work = tasks * max(1, (2 * P + len(tasks) - 1) // len(tasks))
            t0 = time.perf_counter()
            times = list(ex.map(_oracle_task, work))
            wall = time.perf_counter() - t0
        speedup = sum(times) / wall
    return {"value": one * speedup, "unit": UNIT, "cores": P, "kind": "oracle",
            "single_core_value": one, "parallel_speedup": speedup, **info,
            "sample": (f"condensed FP64 oracle on 4 of the 64 graphs ({n_pick} of {n_tot} DOFs) x 3 shifts x 1 and "
                       f"{n_samp} loads, one core: noise {t_noise / n_pick * 1e9:.1f} ns, factorisation "
                       f"{t_fac / n_pick * 1e9:.1f} ns, solve {t_rhs / n_pick * 1e9:.1f} ns per DOF; whole job "
                       f"(S={S}, L={L}) extrapolated as sum_g N_g (S t_noise + L (t_factor + S t_rhs)); "
                       f"all cores: {P} processes, one (graph, shift) task each")}


# ---- workloads -----------------------------------------------------------------------------

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
    return net, {"seconds": t, "steps": TRAIN_STEPS, "phases": TRAIN_PHASES,
                 "loss_first400": float(losses[:400].mean()), "loss_last400": float(losses[-400:].mean()),
                 "graphs": "8 trees/lattices, 100..2000 edges"}


def bench_batched(args, with_forms: bool = True) -> dict:
    """The headline: grf_sample_batched over the 64 uneven graphs, learned + mixed,
    against the plain method and the other batch forms."""
    import torch

    from paper_2605_02670_amd import grf
    from workloads import config_c3

    cfg = config_c3()
    S, beta, seed = cfg["n_samples"], cfg["beta"], cfg["seed"]
    Gs = [grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"]) for g in cfg["graphs"]]
    mls = [G.lumped_mass() for G in Gs]
    n_dof = sum(G.n_dof for G in Gs)
    n_int = sum(G.n_interior for G in Gs)
    n_v = sum(g.n_vertices for g in cfg["graphs"])
    n_e = sum(g.edges.shape[0] for g in cfg["graphs"])
    outs = [torch.empty((S, G.n_dof), dtype=torch.float64, device="cuda") for G in Gs]
    forms = {}

    def batch(**kw):
        return grf.sample_batched(Gs, cfg["kappas"], beta, 0.0, S, seed, outs=outs, **kw)[1]

    # FP64 reference at tolerance 1e-12 (host copies: HBM stays free for the forms' shift blocks)
    st = batch(tol=1e-12)
    L = st["n_shifts"]
    ref = [o.cpu() for o in outs]

    def form(name, what, steps, warmup=1, **kw):
        t0 = time.perf_counter()
        batch(tol=METRIC_TOL, **kw)  # tunes and captures
        first = time.perf_counter() - t0
        dt, med, st_ = _timed(lambda: batch(tol=METRIC_TOL, **kw), steps, warmup)
        f = {"value": n_dof * L * S / dt, "ms_per_step": dt * 1e3, "median_ms": med * 1e3, "first_call_s": first,
             "rel_err_vs_fp64_tol1e-12": _rel_err(outs, ref, mls),
             "pcg": {"mean_iterations": st_["total_iterations"] / max(1, st_["n_systems"]),
                     "max_iterations": st_["max_iterations"],
                     "class_variants": grf.class_modes(st_["pcg_class_modes"])},
             "workload": BATCH_WORKLOAD + "; " + what}
        forms[name] = f
        print(f"# {name}: {dt * 1e3:.1f} ms per step", file=sys.stderr, flush=True)
        return f, st_

    steps_f = max(1, min(args.steps, 3))
    if with_forms:
        # the plain method: one FP64 Jacobi grf_sample per graph, each timed after a
        # warm-up call on a handle of its own, released before the next (a handle keeps
        # its workspace)
        total = 0.0
        pouts = []
        for g, kap in zip(cfg["graphs"], cfg["kappas"]):
            G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
            o = torch.empty((S, G.n_dof), dtype=torch.float64, device="cuda")
            G.sample(float(kap), beta, 0.0, S, seed, out=o, tol=METRIC_TOL)
            _sync()
            t0 = time.perf_counter()
            for _ in range(steps_f):
                G.sample(float(kap), beta, 0.0, S, seed, out=o, tol=METRIC_TOL)
            _sync()
            total += (time.perf_counter() - t0) / steps_f
            pouts.append(o)
            G.close()
        forms["plain_per_graph"] = {"value": n_dof * L * S / total, "ms_per_step": total * 1e3,
                                    "rel_err_vs_fp64_tol1e-12": _rel_err(pouts, ref, mls),
                                    "workload": BATCH_WORKLOAD + "; the plain method: one grf_sample per graph, "
                                                                 "FP64, Jacobi PCG"}
        del pouts
        torch.cuda.empty_cache()
        form("batch_fp64", "one batched call, FP64, Jacobi", steps_f)
        form("batch_mixed", "one batched call, FP32 edge sweeps, Jacobi", steps_f, precision="mixed")
        form("batch_nn", "one batched call, FP64, Neumann-Neumann preconditioner", steps_f, precond="nn")
    net, training = train_network()
    torch.cuda.empty_cache()
    kw_head = dict(learned=net, precision="mixed")
    # the headline: W warm-up steps, then K timed steps
    head, st_h = form("batch_learned_mixed", "one batched call, FP32 edge sweeps, learned preconditioner, PCG "
                      "variant per size class as the autotuner picks it", args.steps, args.warmup, **kw_head)
    head["training"] = training
    # per-kernel HIP events in a separate call of the same form (launches uncaptured)
    stk = batch(tol=METRIC_TOL, timing=True, **kw_head)
    if with_forms:
        form("batch_learned_mixed_op", "one batched call, FP32 edge sweeps, learned operator and initial guess "
             "forced in every size class", steps_f, pcg_class_modes=["op"] * 5 + ["guess"], **kw_head)
        base = forms["plain_per_graph"]["value"]
        forms["speedup_vs_plain_per_graph"] = {k: forms[k]["value"] / base for k in forms
                                               if k.startswith("batch_")}
    roof = with_traffic(roofline(stk, n_dof, n_int, n_v, n_e, L, S, "mixed"), "batched64")
    res = {"value": head["value"], "ms_per_step": head["ms_per_step"], "median_ms": head["median_ms"],
           "n_dof": n_dof, "shifts": L, "samples": S, "graphs": len(Gs), "shift_block": st_h["shift_block"],
           "roofline": roof, "kernel_ms_per_step": {k: v for k, v in stk["kernel_ms"].items() if v > 0},
           "pcg_class_ms_per_step": stk["pcg_class_ms"],
           "hbm": step_hbm(n_dof, n_int, L, S, stk["kernel_launches"]["condense"], "mixed", head["ms_per_step"],
                           "batched64"),
           "forms": forms, "cfg": cfg}
    for G in Gs:
        G.close()
    del outs
    torch.cuda.empty_cache()
    return res


def bench_lattice64(args, beta: float, with_forms: bool = True) -> dict:
    """The 64x64 lattice (2,066,964 DOFs), 256 samples: FP64 (timed, with its roofline),
    and on beta = 0.6 mixed precision, the Neumann-Neumann preconditioner and the
    consistent-mass arm."""
    import torch

    from paper_2605_02670_amd import grf
    from workloads import config_c2

    cfg = config_c2(beta=beta, n_samples=args.samples)
    g = cfg["graph"]
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    S = cfg["n_samples"]
    ml = G.lumped_mass()
    out = torch.empty((S, G.n_dof), dtype=torch.float64, device="cuda")
    args_ = (cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"])

    def run(o, **kw):
        return G.sample(*args_, out=o, tol=cfg["tol"], **kw)[1]

    steps = args.steps if not with_forms else max(1, min(args.steps, 10))
    dt, med, st = _timed(lambda: run(out), steps, max(1, min(args.warmup, 3)))
    L = st["n_shifts"]
    stk = run(out, timing=True)
    res = {"value": G.n_dof * L * S / dt, "ms_per_step": dt * 1e3, "median_ms": med * 1e3, "n_dof": G.n_dof,
           "shifts": L, "samples": S, "shift_block": st["shift_block"],
           "pcg": {"mean_iterations": st["total_iterations"] / max(1, st["n_systems"]),
                   "max_iterations": st["max_iterations"]},
           "kernel_ms_per_step": {k: v for k, v in stk["kernel_ms"].items() if v > 0},
           "roofline": with_traffic(roofline(stk, G.n_dof, G.n_interior, g.n_vertices, g.edges.shape[0], L, S, "fp64"),
                                    f"lattice64_beta{beta}"),
           "hbm": step_hbm(G.n_dof, G.n_interior, L, S, stk["kernel_launches"]["condense"], "fp64", dt * 1e3,
                           f"lattice64_beta{beta}"),
           "workload": f"lattice64x64 U[0.5,1.5] h=1/256 kappa=10 beta={beta} k=0.3 S={S} FP64 Jacobi tol 1e-12"}
    if with_forms:
        o2 = torch.empty_like(out)
        for name, kw in (("mixed", {"precision": "mixed"}), ("nn", {"precond": "nn"})):
            dtf, medf, stf = _timed(lambda: run(o2, **kw), max(1, min(args.steps, 5)), 1)
            d = o2 - out
            m = torch.from_numpy(ml).cuda()
            err = float(torch.sqrt((d * d * m).sum(1) / (out * out * m).sum(1)).max())
            res[name] = {"value": G.n_dof * L * S / dtf, "ms_per_step": dtf * 1e3, "median_ms": medf * 1e3,
                         "rel_err_vs_fp64": err,
                         "pcg": {"mean_iterations": stf["total_iterations"] / max(1, stf["n_systems"])}}
        # the paper's consistent arm: consistent mass in the systems and consistent-mass
        # noise (element factors), the same graph and shifts; a different method, so its
        # result is not compared with the lumped one
        Gc = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"], mass="consistent",
                       noise="consistent")

        def run_c():
            return Gc.sample(*args_, out=o2, tol=cfg["tol"])[1]

        o2 = torch.empty_like(out)
        dtc, medc, stc = _timed(run_c, max(1, min(args.steps, 5)), 1)
        stck = Gc.sample(*args_, out=o2, tol=cfg["tol"], timing=True)[1]
        res["consistent_arm"] = {"value": Gc.n_dof * L * S / dtc, "ms_per_step": dtc * 1e3, "median_ms": medc * 1e3,
                                 "vs_lumped_fp64": dt / dtc, "sweep_block": stc["sweep_block"],
                                 "noise_ms": stck["kernel_ms"]["noise"],
                                 "pcg": {"mean_iterations": stc["total_iterations"] / max(1, stc["n_systems"])},
                                 "workload": "the same lattice and shifts, consistent mass in the shifted systems "
                                             "and consistent-mass noise, FP64 streamed sweeps"}
        del o2
        Gc.close()
    del out
    G.close()
    torch.cuda.empty_cache()
    return res


def bench_lattice256(args) -> dict:
    """The 256x256 lattice (65,536 vertices, 130,560 edges, h = 1/512, 66.8M DOFs), kappa = 20,
    beta = 0.55, step 0.2 with |l| <= 46 (93 shifts, e^{2y} in [1e-8, 1e8]), 64 samples: FP64
    and mixed precision, the mixed sample's error against the FP64 one (8 samples)."""
    import torch

    from paper_2605_02670_amd import grf
    from workloads import config_c4

    cfg = config_c4()
    g = cfg["graph"]
    S = cfg["n_samples"]
    res, keep = {}, {}
    ml = None
    for name, prec in (("fp64", "fp64"), ("mixed", "mixed")):
        G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
        if ml is None:
            ml = G.lumped_mass()
        out = torch.empty((S, G.n_dof), dtype=torch.float64, device="cuda")
        kw = dict(tol=cfg["tol"], precision=prec, k_minus=cfg["k_minus"], k_plus=cfg["k_plus"])
        dt, med, st = _timed(lambda: G.sample(cfg["kappa"], cfg["beta"], cfg["quad_step"], S, cfg["seed"], out=out,
                                              **kw)[1], max(1, min(args.steps, 3)), 1)
        res[name] = {"value": G.n_dof * st["n_shifts"] * S / dt, "ms_per_step": dt * 1e3, "median_ms": med * 1e3,
                     "shift_block": st["shift_block"],
                     "pcg": {"mean_iterations": st["total_iterations"] / max(1, st["n_systems"])}}
        keep[name] = out[:8].clone()
        res["n_dof"] = G.n_dof
        del out
        G.close()
        torch.cuda.empty_cache()
        print(f"# lattice256 {name}: {dt * 1e3:.1f} ms per call", file=sys.stderr, flush=True)
    m = torch.from_numpy(ml).cuda()
    d = keep["mixed"] - keep["fp64"]
    res["mixed"]["rel_err_vs_fp64_8_samples"] = float(torch.sqrt((d * d * m).sum(1) /
                                                                 (keep["fp64"] ** 2 * m).sum(1)).max())
    res["mixed"]["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"]
    res["workload"] = (f"lattice256x256 U[0.5,1.5] h=1/512 kappa=20 beta=0.55 k=0.2 |l|<=46 (93 shifts) S={S}, "
                       "Jacobi tol 1e-12")
    return res


def bench_rgg(args) -> dict:
    """The learned preconditioner's held-out random geometric graph (98,129 vertices, 199,826
    edges, h = 1/256, 38.4M DOFs), kappa = 2, beta = 0.75 (229 shifts), 64 samples, PCG tol
    1e-8: Jacobi, learned (trained first on 16 smaller graphs of the kind), Neumann-Neumann,
    learned + mixed; errors against the FP64 Jacobi result at tolerance 1e-12 (8 samples)."""
    import torch

    from paper_2605_02670_amd import grf
    from workloads import config_c5_eval, config_c5_train
    from workloads.learned_init import init_params

    tr = config_c5_train()
    Gt = [grf.Graph(d["graph"].n_vertices, d["graph"].edges, d["graph"].lengths, 1.0 / 256, "round") for d in tr]
    net = grf.Learned(init_params(0))
    t0 = time.perf_counter()
    for k, (n, lr) in enumerate(TRAIN_PHASES):
        net.train(Gt, [d["kappa"] for d in tr], 0.75, 0.0, n_samples=4, seed=11 + 7 * k, n_steps=n,
                  shifts_per_step=16, lr=lr)
    t_train = time.perf_counter() - t0
    for G in Gt:
        G.close()
    torch.cuda.empty_cache()
    cfg = config_c5_eval()
    g = cfg["graph"]
    G = grf.Graph(g.n_vertices, g.edges, g.lengths, cfg["h"], cfg["rule"])
    S = cfg["n_samples"]
    m = torch.from_numpy(G.lumped_mass()).cuda()
    out = torch.empty((S, G.n_dof), dtype=torch.float64, device="cuda")
    G.sample(cfg["kappa"], cfg["beta"], 0.0, S, cfg["seed"], out=out, tol=1e-12)
    ref = out[:8].clone()
    res = {}
    for name, kw in (("jacobi", {}), ("learned", {"learned": net}), ("nn", {"precond": "nn"}),
                     ("learned_mixed", {"learned": net, "precision": "mixed"})):
        def call():
            return G.sample(cfg["kappa"], cfg["beta"], 0.0, S, cfg["seed"], out=out, tol=METRIC_TOL, **kw)[1]

        dt, med, st = _timed(call, 1, 1)
        d = out[:8] - ref
        res[name] = {"value": G.n_dof * st["n_shifts"] * S / dt, "ms_per_step": dt * 1e3,
                     "rel_err_vs_fp64_tol1e-12": float(torch.sqrt((d * d * m).sum(1) / (ref * ref * m).sum(1)).max()),
                     "pcg": {"mean_iterations": st["total_iterations"] / max(1, st["n_systems"]),
                             "max_iterations": st["max_iterations"]}}
        print(f"# rgg100k {name}: {dt * 1e3:.0f} ms", file=sys.stderr, flush=True)
    for k in ("learned", "nn", "learned_mixed"):
        res[k]["speedup_vs_jacobi"] = res["jacobi"]["ms_per_step"] / res[k]["ms_per_step"]
    res["training"] = {"seconds": t_train, "steps": TRAIN_STEPS, "graphs": "16 random geometric graphs, 2k..20k points"}
    res["n_dof"] = G.n_dof
    res["workload"] = (f"held-out random geometric graph {g.n_vertices} vertices {g.edges.shape[0]} edges h=1/256 "
                       f"kappa=2 beta=0.75 (229 shifts) S={S}, PCG tol {METRIC_TOL:g}")
    del out
    G.close()
    torch.cuda.empty_cache()
    return res


def _line(value, steps, warmup, ms, dtype, workload, extra) -> dict:
    d = {"metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": steps, "warmup": warmup,
         "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
         "data": "synthetic", "config": {"workload": workload, "parallelism": "1 GPU"}}
    d.update(extra)
    return d


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--samples", type=int, default=256, help="samples of the 64x64 lattice")
    ap.add_argument("--beta", type=float, default=0.6, help="beta of --workload lattice64")
    ap.add_argument("--workload", choices=["default", "lattice64", "batched64", "lattice256", "rgg100k"],
                    default="default",
                    help="default: the batched headline with every form; otherwise that workload alone")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="the headline only (no other forms or workloads)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built "
              "(samples shard across GPUs with no communication)", file=sys.stderr)
        return 2

    import torch

    from paper_2605_02670_amd import grf

    grf.load()
    torch.cuda.set_device(0)
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        _sync()
        del src, dst
    wl = args.workload
    if wl == "lattice64":
        r = bench_lattice64(args, args.beta, with_forms=not args.no_forms)
        print(json.dumps(_line(r["value"], args.steps, args.warmup, r["ms_per_step"], "f64", r["workload"],
                               {"roofline": r["roofline"], "cpu_baseline": None, "detail": r})), flush=True)
        return 0
    if wl == "lattice256":
        r = bench_lattice256(args)
        print(json.dumps(_line(r["mixed"]["value"], 1, 1, r["mixed"]["ms_per_step"], "f32+f64", r["workload"],
                               {"roofline": None, "cpu_baseline": None, "detail": r})), flush=True)
        return 0
    if wl == "rgg100k":
        r = bench_rgg(args)
        print(json.dumps(_line(r["learned"]["value"], 1, 1, r["learned"]["ms_per_step"], "f64", r["workload"],
                               {"roofline": None, "cpu_baseline": None, "detail": r})), flush=True)
        return 0
    forms_on = wl == "default" and not args.no_forms
    b = bench_batched(args, with_forms=forms_on)
    cfg = b.pop("cfg")
    forms = b.pop("forms")
    if forms_on:
        forms["lattice64_beta0.6"] = bench_lattice64(args, 0.6, with_forms=True)
        forms["lattice64_beta0.85"] = bench_lattice64(args, 0.85, with_forms=False)
        forms["lattice256"] = bench_lattice256(args)
        forms["rgg100k"] = bench_rgg(args)
    cpu = None if args.no_cpu_baseline else cpu_baseline(cfg["graphs"], cfg["kappas"], cfg["h"], cfg["rule"],
                                                         cfg["beta"], b["shifts"], b["samples"])
    vs_plain = (b["value"] / forms["plain_per_graph"]["value"]) if "plain_per_graph" in forms else None
    line = _line(b["value"], args.steps, args.warmup, b["ms_per_step"], "f32+f64",
                 BATCH_WORKLOAD + "; learned preconditioner + batched + FP32 edge sweeps",
                 {"roofline": b.pop("roofline"), "cpu_baseline": cpu, "vs_plain_fp64_per_graph": vs_plain})
    line["config"].update({"n_dof": b["n_dof"], "shifts": b["shifts"], "samples": b["samples"],
                           "graphs": b["graphs"], "shift_block": b["shift_block"]})
    line["median_ms_per_step"] = b["median_ms"]
    line["hbm"] = b["hbm"]
    line["kernel_ms_per_step"] = b["kernel_ms_per_step"]
    line["pcg_class_ms_per_step"] = b["pcg_class_ms_per_step"]
    line["forms"] = forms
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
