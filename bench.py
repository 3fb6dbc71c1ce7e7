"""Benchmark: event-NLL(+gradient) evaluations per second on one MI355X.

Workload (one step = one pass of the hot path): the three-body Dalitz model
with eight resonances, 1M synthetic events (s12, s13) in HBM, sixteen free
coefficient parameters; a step is prologue -> per-event evaluation with the
adjoint gradient -> deterministic level-2 reduction -> normalization from the
cached grid matrix -> NLL and gradient in device memory.  `value` is
events x steps / second.

Also reported (same process): the dominant kernel's duration from HIP events
on its stream and its roofline, the plain finite-difference gradient path,
the other model configurations, single-fit wall times with and without the
adjoint, and the CPU oracle on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
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

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector, FMA counted as 2
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the config-1 event kernel from the FETCH_SIZE and
# WRITE_SIZE counter runs (profiles/dalitz_events_grad_1M.md), by (summation
# chunk, events per thread), and its executed FP64 FLOPs per event from
# SQ_INSTS_VALU_FLOPS_FP64, valid for the kernel sources with this hash;
# reported as null once they change or for a choice without a counter run.
TRAFFIC_BYTES = {(2048, 1): 1.620e7}
COUNTED_FP64_FLOPS_PER_EVENT = {(2048, 1): 404.9}
TRAFFIC_SOURCES = ["paper_1710_08826_amd/csrc/dalitz_device.hpp", "paper_1710_08826_amd/csrc/dalitz3.hip",
                   "paper_1710_08826_amd/csrc/fastmath.hpp", "paper_1710_08826_amd/csrc/device_common.hpp",
                   "paper_1710_08826_amd/csrc/model.hpp"]
TRAFFIC_HASH = "ea741244afb06c3e"


def counters_current() -> bool:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16] == TRAFFIC_HASH


def measured_traffic(chunk: int, ept: int = 1):
    return TRAFFIC_BYTES.get((chunk, ept)) if counters_current() else None


def counted_flops(chunk: int, ept: int = 1):
    return COUNTED_FP64_FLOPS_PER_EVENT.get((chunk, ept)) if counters_current() else None

# FP64 FLOPs of the correctly rounded gfx950 sequences of the ROCm device
# library (FMA = 2, other FP64 arithmetic = 1, compares 0), counted from the
# ISA of this toolchain: the price of each elementary function in the
# algorithmic FLOP count (the kernels use cheaper Newton-refined forms).
W_SQRT, W_RSQRT, W_DIV, W_LOG, W_EXP = 19, 9, 17, 85, 30
W_SINCOS = 59  # the small-argument path (|x| below the large-reduction threshold)


def log_sum_flops(chunk: int) -> float:
    """FLOPs per event of -sum ln P as the passes evaluate it: one multiply
    into the thread's running product per event, and one logarithm per
    thread (chunk / 256 events each), shared by its events."""
    return 1 + W_LOG * 256 / chunk


def dalitz_amp_flops(desc: dict) -> int:
    """FP64 FLOPs per point of the Dalitz amplitudes and their coherent sum:
    per-pair kinematics shared by the pair's resonances, one complex
    reciprocal per resonance."""
    pairs = {}
    for r in desc["resonances"]:
        pairs.setdefault(r["pair"], set()).add(int(r["L"]))
    K = len(desc["resonances"])
    f = 2                                          # s23
    for Ls in pairs.values():
        f += 11 + W_RSQRT + W_SQRT                 # 1/sqrt s, 1/s, lambda_q, lambda_p, q^2, q/sqrt s
        if 1 in Ls or 2 in Ls:
            f += 7                                 # p^2, z_q, z_p, Z1
        if 1 in Ls:
            f += 6 + W_DIV + W_RSQRT               # G1 = (q/sqrt s) q^2/(1+z_q), H1 = Z1/sqrt(..)
        if 2 in Ls:
            f += 17 + W_DIV + W_RSQRT              # polynomials, G2, Z2, H2
    f += K * (16 + W_DIV)                          # T = (a + i b)/(a^2 + b^2), A, coherent sum
    return f


def dalitz_flops_per_event(desc: dict, grad: int, chunk: int) -> float:
    """Algorithmic FP64 FLOPs per event of the Dalitz NLL (grad: 0 none,
    1 coefficients, 2 coefficients + masses and widths), counted from the
    formula as evaluated: the amplitudes (dalitz_amp_flops), |S|^2 and the
    log sum (log_sum_flops), the gradient terms."""
    K = len(desc["resonances"])
    f = dalitz_amp_flops(desc) + 3 + log_sum_flops(chunk)  # |S|^2, -sum ln P~
    if grad >= 1:
        f += 4 + W_DIV + 6 * K                     # -1/P~, 2 Re(conj(S) A) per coefficient
    if grad >= 2:
        f += 31 * K                                # mass and width derivatives
    return f


def td4_flops_per_event(desc: dict, grad: bool, chunk: int) -> float:
    """Algorithmic FP64 FLOPs per (event, fit) of the time-dependent
    four-body NLL, counted from the formula as evaluated: per-pair kinematics
    shared by the pair's resonances, one complex reciprocal per resonance,
    products with flat (non-resonant) entries free, the three time terms
    through the rational Faddeeva approximation (40 coefficients, Horner),
    the log sum (log_sum_flops)."""
    N = 40
    f = 0
    pairs = (desc["r12"], desc["r34"])
    for entries in pairs:
        res = [e for e in entries if e["m0"] != 0.0]
        f += 7 + W_DIV + W_SQRT                    # s, 1/m, lambda, q^2, q, G0
        if any(int(e["L"]) == 1 for e in res):
            f += 6 + W_RSQRT                       # z, F1 = (1+z)^-1/2, G1
        f += len(res) * (9 + W_DIV)                # a, b, 1/(a^2+b^2), amplitude
    types = [int(a[2]) for a in desc["amps"]]
    f += 2 * (2 + W_SQRT) + 2                      # sin12 sin34 / 2
    if any(t >= 4 for t in types):
        f += W_SINCOS                              # e^{i phi}
    if 3 in types:
        f += 1                                     # c12 c34
    flat12 = [e["m0"] == 0.0 for e in desc["r12"]]
    flat34 = [e["m0"] == 0.0 for e in desc["r34"]]
    members = 0                                    # (basis function, sum) memberships
    for a in desc["amps"]:
        i12, i34, t = a[:3]
        f += 0 if (flat12[i12] or flat34[i34]) else 6
        f += 0 if t == 0 else (2 if t <= 3 else 6)
        members += 2 if len(a) < 4 or a[3] == "both" else 1
    f += 8 * members                               # A and Abar
    f += 2 + W_EXP                                 # exp(-t^2 / 2 sigma^2)
    horner_r = (N - 1) * 2
    h_real = 3 + (1 + W_DIV) + 2 + horner_r + 4 + (4 + W_EXP) + 3
    horner_c = (N - 1) * 7
    w_c = 1 + (5 + W_DIV) + 7 + horner_c + 8 + 7
    h_cplx = 5 + w_c + 9 + W_SINCOS + W_EXP + 7
    f += 2 * h_real + h_cplx
    f += 27 + log_sum_flops(chunk)                 # rate, -sum ln R
    if grad:
        f += 2 * 3 + 8                             # dh/da of the three time terms
        f += 1 + W_DIV + 2 + 24 + 8 * members + 20  # -1/R, the two complex weights, lc B_k and lb B_k, x and y
    return f


def time_terms_flops() -> int:
    """The three resolution-convolved time terms per event (rational Faddeeva
    approximation, 40 coefficients) and exp(-t^2 / 2 sigma^2)."""
    N = 40
    h_real = 3 + (1 + W_DIV) + 2 + (N - 1) * 2 + 4 + (4 + W_EXP) + 3
    w_c = 1 + (5 + W_DIV) + 7 + (N - 1) * 7 + 8 + 7
    h_cplx = 5 + w_c + 9 + W_SINCOS + W_EXP + 7
    return 2 + W_EXP + 2 * h_real + h_cplx


def tddp3_flops_per_event(desc: dict, grad: bool, chunk: int) -> float:
    """Algorithmic FP64 FLOPs per event of the time-dependent Dalitz NLL: the
    three-body amplitudes at (s12, s13) and at (s13, s12) (per-pair kinematics
    shared by the pair's resonances, one complex reciprocal per resonance),
    both coherent sums, the time terms, the rate and the log sum."""
    K = len(desc["resonances"])
    amp = dalitz_amp_flops(dict(desc, kind="dalitz3"))  # one amplitude set + sum
    f = 2 * amp + time_terms_flops() + 27 + log_sum_flops(chunk)
    if grad:
        f += 2 * 3 + 8                              # dh/da of the three time terms
        f += 1 + W_DIV + 2 + 24 + 16 * K + 20       # -1/R, the two complex weights, c and cbar slots, x and y
    return f


def mix1d_flops_per_event(grad: bool, chunk: int) -> float:
    """Config-0 mixture (Gaussian + exponential): 2 exp, the log sum, ~14
    others; the gradient adds one division and ~22 FLOPs."""
    f = 2 * W_EXP + log_sum_flops(chunk) + 14
    if grad:
        f += W_DIV + 22
    return f


def gpu_info():
    import torch
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "cus": p.multi_processor_count, "arch": getattr(p, "gcnArchName", "")}


# Wall-time trials: each trial times exactly `steps` steps; trials repeat until
# at least MIN_TRIALS of them and MIN_TIMED_S seconds of timed work, and the
# median trial is reported.
MIN_TRIALS = 5
MIN_TIMED_S = 0.1
MAX_TRIALS = 2000
# Launches of the separate loop that times the per-event kernel itself (every
# launch carries a HIP event pair; none of them is inside a wall-timed trial).
KERNEL_TIMING_LAUNCHES = 50


GRAPH_STEPS = 8  # NLL steps per captured graph (a replay costs about 4.7 us of launch latency)


def capture_steps(model, thetas, ev, out, with_grad):
    """Captured step graphs: for each size 8, 4, 2, 1 one hipGraph holding that
    many asynchronous NLL(+grad) calls (prologue if any, events pass, level-2
    step) with theta alternating between the trial points, captured on a side
    stream after the model's caches are built; None when capture fails."""
    import torch
    graphs = {}
    s = torch.cuda.Stream()
    try:
        for size in (GRAPH_STEPS, 4, 2, 1):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
                for i in range(size):
                    model.nll_async(thetas[i % len(thetas)], ev, out, with_grad)
            graphs[size] = g
    except Exception as e:  # noqa: BLE001 - reported in the bench line
        print(f"[bench] graph capture failed ({e}); timing direct launches", file=sys.stderr, flush=True)
        return None
    return graphs


def replay_steps(graphs, k):
    """Exactly k steps from the captured graphs: k // 8 replays of the 8-step
    graph, then the remainder by its binary digits."""
    for _ in range(k // GRAPH_STEPS):
        graphs[GRAPH_STEPS].replay()
    r = k % GRAPH_STEPS
    for size in (4, 2, 1):
        if r >= size:
            graphs[size].replay()
            r -= size


def time_async(model, theta_dev, ev, out, steps, warmup, with_grad=True, alt=None, graph=True):
    """NLL(+grad) steps with device theta alternating between two points, so no
    cache short-circuits the work.  Returns (median wall seconds of a trial of
    exactly `steps` steps, average per-event kernel duration in ms, info).
    Dalitz models: the kernel duration is the average span of the per-event
    launches of a second, identical loop of trials, measured by the launches
    themselves on the device wall clock (fn_model_timing span mode, captured
    into the replayed graphs; its bookkeeping adds about 2 us to a step, so
    the wall-timed trials run without it); other models: a separate loop of
    launches each timed by its own dispatch (HIP events)."""
    import torch
    thetas = [theta_dev] if alt is None else [theta_dev, alt]
    span = model.desc.get("kind") == "dalitz3"
    for i in range(max(warmup, 2)):
        model.nll_async(thetas[i % len(thetas)], ev, out, with_grad)
    torch.cuda.synchronize()

    def trials_of(graphs):
        def run(k):
            if graphs:
                replay_steps(graphs, k)
            else:
                for i in range(k):
                    model.nll_async(thetas[i % len(thetas)], ev, out, with_grad)
        run(max(warmup, 2))
        torch.cuda.synchronize()
        if span:
            model.kernel_time()  # drop the warm-up launches
        trials = []
        while len(trials) < MAX_TRIALS and (len(trials) < MIN_TRIALS or sum(trials) < MIN_TIMED_S):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run(steps)
            torch.cuda.synchronize()
            trials.append(time.perf_counter() - t0)
        return trials

    graphs = capture_steps(model, thetas, ev, out, with_grad) if graph else None
    trials = trials_of(graphs)
    info = {"trials": len(trials), "timed_s": sum(trials), "graph": graphs is not None,
            "trial_ms_min": 1e3 * min(trials), "trial_ms_max": 1e3 * max(trials)}
    if span:
        model.set_timing(True, span=True)
        model.nll_async(thetas[0], ev, out, with_grad)  # sizes the stamp buffer before capture
        torch.cuda.synchronize()
        sgraphs = capture_steps(model, thetas, ev, out, with_grad) if graph else None
        strials = trials_of(sgraphs)
        kms, launches = model.kernel_time()
        model.set_timing(False)
        info.update({"kernel_timing": "in-kernel spans of every launch of a second loop of trials",
                     "kernel_launches_timed": launches, "span_loop_ms_per_step": 1e3 * float(np.median(strials)) / steps})
    else:
        # the kernel's own duration, outside the wall-timed trials
        model.kernel_time()
        model.set_timing(True, every=1)
        for i in range(KERNEL_TIMING_LAUNCHES):
            model.nll_async(thetas[i % len(thetas)], ev, out, with_grad)
        torch.cuda.synchronize()
        model.set_timing(False)
        kms, launches = model.kernel_time()
        info.update({"kernel_timing": f"{KERNEL_TIMING_LAUNCHES} separately timed launches (dispatch events)",
                     "kernel_launches_timed": launches})
    return float(np.median(trials)), kms / max(launches, 1), info


def cpu_info():
    """nproc, the threads torch uses and the CPU model string of this host."""
    import torch
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "threads": torch.get_num_threads(),
            "cpu_model": model}


def _median_rate(fn, units, trials=5, min_s=0.3):
    """Median over trials of units/second; a trial repeats fn until min_s."""
    rates = []
    for _ in range(trials):
        calls = 0
        t0 = time.perf_counter()
        while True:
            fn()
            calls += 1
            if time.perf_counter() - t0 >= min_s:
                break
        rates.append(units * calls / (time.perf_counter() - t0))
    return float(np.median(rates))


def cpu_baseline(events: np.ndarray, desc: dict, theta):
    """The CPU oracle on a bounded sample of the config-1 workload, the same
    work as the GPU step: the event term -sum ln P~ and its autograd gradient
    (the GPU step takes I = c^H M c from the cached grid matrix, a 16 x 16
    quadratic form).  Median of 5 trials with all host threads and with one.
    Also the oracle call as it stands (grid normalization recomputed every
    call) for reference."""
    import torch
    from oracle import dalitz3 as OD
    from oracle.common import as_t
    model = OD.Dalitz(desc)
    s12, s13 = as_t(events[0]), as_t(events[1])
    n = events.shape[1]

    def event_term():
        th = as_t(theta, requires_grad=True)
        (-torch.log(model.density_unnorm(th, s12, s13)).sum()).backward()

    info = cpu_info()
    nthreads = torch.get_num_threads()
    rate = _median_rate(event_term, n)
    torch.set_num_threads(1)
    sub = max(1, n // 8)
    s12_1, s13_1 = s12[:sub].clone(), s13[:sub].clone()

    def event_term_1():
        th = as_t(theta, requires_grad=True)
        (-torch.log(model.density_unnorm(th, s12_1, s13_1)).sum()).backward()

    rate_1 = _median_rate(event_term_1, sub)
    torch.set_num_threads(nthreads)
    cells = model.grid_cells()
    t0 = time.perf_counter()
    OD.nll_grad(theta, events, desc, cells)
    full = n / (time.perf_counter() - t0)
    return {"value": rate, "unit": "events/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n} events of the config-1 Dalitz workload: the oracle's event term -sum ln P~ with its "
                      f"autograd gradient (16 parameters), median of 5 trials of >= 0.3 s; normalization excluded on "
                      f"both sides (the GPU step reads the cached grid matrix)",
            "one_core_events_per_s": rate_1, "one_core_sample_events": sub,
            "oracle_call_with_grid_events_per_s": full, **info}


def variation_serving_leg(n_req: int = 192, slots: int = 64, lam_frac: float = 0.7, n: int = 1_000_000,
                          max_iter: int = 2000):
    """Systematic-variation fits of the twenty-amplitude four-body model served
    continuously (fn_vbatch_serve): 1M toys of the model drawn on the device
    at the generation point, the 5M-point normalization sample, 64 slots, 192
    requests (ten kinds of +-shifted lineshape constants and time resolution,
    start points near the generation point, all coefficients but Abar's
    reference and x, y free, each request capped at max_iter minimizer
    iterations).  Closed loop (all requests at t = 0), then Poisson arrivals
    at lam_frac of the closed-loop rate."""
    import torch
    import synth
    from paper_1710_08826_amd import Model, VariationBatch
    desc = synth.td4_split_desc()
    th = synth.td4_split_truth()
    m = Model(desc)
    m.generate_norm_sample(5_000_000, seed=synth.BASE_SEED + 5)
    ev, _ = m.generate(th, n, seed=synth.BASE_SEED + 40)
    m.autotune(th, ev, reps=5)
    P = m.n_params
    fx = m.fixed()
    n12, n34 = len(desc["r12"]), len(desc["r34"])
    shifted = (3, 2 * n12 + 2, 2 * n12 + 3, 2 * n12 + 5, 2 * (n12 + n34))
    free = np.ones(P, np.int32)
    n_abar = sum(1 for a in desc["amps"] if a[3] != "A")
    free[P - 2 - 2 * n_abar: P - 2 * n_abar] = 0
    rng = np.random.default_rng(17100882)

    def make(arrivals):
        reqs = []
        for i, t in enumerate(arrivals):
            v = fx.copy()
            v[shifted[i % 5]] *= 1.0 + 0.002 * (1 if (i // 5) % 2 else -1)
            th0 = th * (1.0 + 2e-3 * np.sin(np.arange(P) + i))
            th0[free == 0] = th[free == 0]
            reqs.append((i, float(t), v, th0))
        return reqs

    b = VariationBatch(m, slots)
    out = {"events": n, "mc_points": 5_000_000, "params": P, "slots": slots, "requests": n_req,
           "max_iter": max_iter, "chunk": m.chunk, "data": "model toys drawn on the device"}
    b.serve(make([0.0] * 8), ev, free=free, max_iter=max_iter)  # warm-up: graph capture, kernels
    for label, arrivals in (("closed_loop", np.zeros(n_req)), ("poisson", None)):
        if arrivals is None:
            lam = lam_frac * out["closed_loop"]["fits_per_s"]
            arrivals = np.cumsum(rng.exponential(1.0 / lam, n_req))
        reqs = make(arrivals)
        t0 = time.perf_counter()
        r = b.serve(reqs, ev, free=free, max_iter=max_iter)
        wall = time.perf_counter() - t0
        lat = r["t_done"] - arrivals
        out[label] = {"wall_s": wall, "fits_per_s": n_req / wall, "converged": int((r["status"] == 2).sum()),
                      "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                      "mean_iterations": float(r["iters"].mean()), "mean_evaluations": float(r["n_evals"].mean())}
        if label == "poisson":
            out[label]["rate_per_s"] = float(lam)
    b.close()
    return out


def cpu_baselines_other():
    """The oracle on bounded samples of configs 0, 3 and 4 (events/s of NLL +
    autograd gradient, median of 5 trials, all host threads), each with the
    work its GPU step does: config 0 analytic normalization; config 3 the
    event term at 4M events plus the full 1024 x 1024 grid every call
    (per-call time from the two measured rates); config 4 the event term
    (the GPU single fit reads the cached sample matrix)."""
    import torch
    import synth
    from oracle import dalitz3 as OD, mix1d as OM, td4 as OT
    from oracle.common import as_t
    out = {}
    x0 = synth.mix1d_events(100_000)
    d0 = synth.mix1d_desc()
    th0 = synth.mix1d_truth()
    out["config0_events_per_s"] = _median_rate(lambda: OM.nll_grad(th0, x0, d0), x0.size, min_s=0.2)
    d3 = synth.dalitz_desc(free_lineshapes=True)
    th3 = synth.dalitz_truth(free_lineshapes=True)
    ev3 = synth.dalitz_events(20_000, seed=synth.BASE_SEED + 3)
    m3 = OD.Dalitz(d3)
    a12, a13 = as_t(ev3[0]), as_t(ev3[1])

    def ev_term3():
        th = as_t(th3, requires_grad=True)
        (-torch.log(m3.density_unnorm(th, a12, a13)).sum()).backward()

    ev_rate3 = _median_rate(ev_term3, ev3.shape[1], min_s=0.2)
    c12, c13, da = m3.grid_cells()
    sub = 100_000
    g12, g13 = as_t(c12[:sub]), as_t(c13[:sub])

    def grid_term3():
        th = as_t(th3, requires_grad=True)
        (da * m3.density_unnorm(th, g12, g13).sum()).backward()

    cell_rate3 = _median_rate(grid_term3, sub, min_s=0.2)
    call3 = 4_000_000 / ev_rate3 + c12.size / cell_rate3
    out["config3_events_per_s"] = 4_000_000 / call3
    out["config3_grid_cells_per_s"] = cell_rate3
    d4 = synth.td4_desc()
    th4 = synth.td4_truth()
    ev4 = synth.td4_events(5_000, seed=synth.BASE_SEED + 4)
    m4 = OT.TD4(d4)
    e4 = as_t(ev4)

    def ev_term4():
        th = as_t(th4, requires_grad=True)
        (-torch.log(m4.rate(th, e4)).sum()).backward()

    out["config4_events_per_s"] = _median_rate(ev_term4, ev4.shape[1], min_s=0.2)
    out["sample"] = ("config 0: 100k events, analytic normalization; config 3: 20k events and 100k grid cells "
                     "timed, per-call time of 4M events + 497,806 cells derived; config 4: 5k events, event term")
    return out


def pmc_probe(steps: int, chunk: int, workload: str = "config1"):
    """Workload for hardware-counter runs: a plain 256 MiB copy (its counter
    reading calibrates bytes per counter unit), then `steps` NLL+gradient
    evaluations of one workload: config1 (Dalitz, 1M events, at the given
    summation chunk), config3 (free lineshapes, 4M events), tddp3 (sixteen
    resonances, 1M events), td4 (twenty amplitudes, 10M events), td4batch (64
    variation fits of td4), config0mall (1-D mixture, 2^26 events)."""
    import torch
    import synth
    from paper_1710_08826_amd import Model, VariationBatch
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")  # 256 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    seed = synth.BASE_SEED
    batch = None
    if workload == "config1":
        ev = torch.from_numpy(synth.dalitz_events(1_000_000, seed=seed)).cuda()
        m = Model(synth.dalitz_desc(chunk=chunk))
        th = synth.dalitz_truth()
    elif workload == "config3":
        ev = torch.from_numpy(synth.dalitz_events(4_000_000, seed=seed + 3)).cuda()
        m = Model(synth.dalitz_desc(free_lineshapes=True))
        th = synth.dalitz_truth(free_lineshapes=True)
    elif workload == "tddp3":
        res = synth.TDDP_RESONANCES16
        ev = torch.from_numpy(synth.tddp3_events(1_000_000, seed=seed + 7, resonances=res)).cuda()
        m = Model(synth.tddp3_desc(resonances=res))
        th = synth.tddp3_truth(resonances=res)
    elif workload in ("td4", "td4batch"):
        ev = torch.from_numpy(synth.td4_events(10_000_000, seed=seed + 4)).cuda()
        m = Model(synth.td4_split_desc(chunk=8192))
        m.generate_norm_sample(5_000_000, seed=seed + 5)
        th = synth.td4_split_truth()
        if workload == "td4batch":
            batch = VariationBatch(m, 64)
            fx = m.fixed()
            for f in range(64):
                v = fx.copy()
                v[-1] *= 1.0 + 0.002 * (f - 32)
                batch.set_fixed(f, v)
            ths = np.stack([th * (1.0 + 1e-3 * np.sin(np.arange(th.size) + f)) for f in range(64)])
    elif workload == "config0mall":
        ev = torch.from_numpy(synth.mix1d_events(1 << 26, seed=seed + 1)[None, :]).cuda()
        m = Model(dict(synth.mix1d_desc(), chunk=1024))
        th = synth.mix1d_truth()
    else:
        raise ValueError(workload)
    tdev = torch.from_numpy(np.asarray(th, dtype=np.float64)).cuda()
    out = torch.empty(1 + m.n_params, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        if batch is not None:
            batch.nll(ths, ev, grad=True)
        else:
            m.nll_async(tdev, ev, out, True)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": workload, "copy_bytes": 2 * 32 * 1024 * 1024 * 8, "steps": steps,
                      "chunk": m.chunk, "nll": float(out[0]) if batch is None else None}), flush=True)


def serving_leg(n_fits: int = 4096, fd_fits: int = 32, lam_frac: float = 0.7):
    """Config 2: toy fits of the config-0 model with per-fit sizes drawn
    log-uniform in [1e3, 2e6], events generated on the device at admission.
    Returns fits/s and latency percentiles for (a) all requests at t = 0 and
    (b) Poisson arrivals at lam_frac x the batched throughput, on the
    continuous-batching server; (c) one fit at a time (host BFGS, adjoint
    gradient) on every request at the same Poisson arrivals, and (d) one fit
    at a time with finite-difference gradients on a subsample."""
    import torch
    import synth
    from paper_1710_08826_amd import Model, Server, generate_mix1d
    truth = synth.mix1d_truth()
    start = truth * np.array([1.1, 0.9, 1.15, 0.95])
    sizes = synth.lognormal_sizes(n_fits)
    model = Model(synth.mix1d_desc())
    base = [dict(id=i, n_events=int(sizes[i]), seed=synth.BASE_SEED, fit=i, theta_gen=truth, theta0=start,
                 arrival_s=0.0) for i in range(n_fits)]
    budget = int(min(200 << 30, 2 * int(sizes.sum()) * 8 + (1 << 30)))

    def serve(reqs, slots):
        srv = Server(model, max_slots=slots, max_events_per_fit=2_000_000, budget_bytes=budget)
        srv.submit(reqs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        srv.run(poll_every=2)
        wall = time.perf_counter() - t0
        res = srv.results()
        srv.close()
        lat = np.array([r.latency for r in res])
        ok = sum(1 for r in res if r.status == 2)
        return {"fits": len(res), "converged": ok, "wall_s": wall, "fits_per_s": len(res) / wall,
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "events": int(sum(r["n_events"] for r in reqs))}

    out = {}
    serve(base[:64], 64)  # warm-up: graph capture, allocations
    out["closed_loop"] = serve(base, n_fits)
    rate = lam_frac * out["closed_loop"]["fits_per_s"]
    u, _ = synth.uniforms(n_fits, synth.key_from_seed(synth.BASE_SEED, 0xABC), 5)
    arrivals = np.cumsum(-np.log1p(-u) / rate)
    pois = [dict(r, arrival_s=float(arrivals[i])) for i, r in enumerate(base)]
    out["poisson"] = serve(pois, n_fits)
    out["poisson"]["rate_per_s"] = rate

    def sequential(reqs, mode):
        """One fit at a time in arrival order (host BFGS on the single-fit
        path, events generated on the device per request); a request waits
        until it has arrived and until the previous fit is done."""
        lat = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q in reqs:
            wait = q["arrival_s"] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            ev = generate_mix1d(q["n_events"], q["seed"], q["fit"], truth)
            model.fit(start, ev, grad_mode=mode, raise_on_fail=False)
            lat.append(time.perf_counter() - t0 - q["arrival_s"])
        wall = time.perf_counter() - t0
        lat = np.array(lat)
        return {"fits": len(reqs), "wall_s": wall, "fits_per_s": len(reqs) / wall,
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "events": int(sum(r["n_events"] for r in reqs))}

    # every request, one at a time, at the batched run's Poisson arrivals
    out["one_at_a_time_poisson"] = sequential(pois, "adjoint")
    out["one_at_a_time_poisson"]["rate_per_s"] = rate
    subfd = base[:: max(1, n_fits // fd_fits)][:fd_fits]
    out["one_at_a_time_fd"] = sequential(subfd, "fd")
    # the same request subsample on the batched server, for a like-for-like ratio
    out["batched_same_subsample_fd"] = serve(subfd, len(subfd))
    out["speedup_batched_vs_plain_fd"] = out["closed_loop"]["fits_per_s"] / out["one_at_a_time_fd"]["fits_per_s"]
    out["speedup_batched_vs_one_at_a_time_adjoint"] = (out["closed_loop"]["fits_per_s"]
                                                      / out["one_at_a_time_poisson"]["fits_per_s"])
    return out


def config0_above_mall(n: int = 1 << 26, steps: int = 20):
    """Config-0 events pass at 2^26 events (512 MB, above the 256 MB
    Infinity Cache), events generated on the device: NLL + gradient steps and
    the events kernel's duration, HBM GB/s and FP64 rate."""
    import torch
    import synth
    from paper_1710_08826_amd import Model, generate_mix1d
    truth = synth.mix1d_truth()
    x = generate_mix1d(n, synth.BASE_SEED, 26, truth)
    m = Model(synth.mix1d_desc())
    t = torch.from_numpy(truth).cuda()
    tb = torch.from_numpy(truth * 1.001).cuda()
    o = torch.empty(1 + m.n_params, dtype=torch.float64, device="cuda")
    w, k, info = time_async(m, t, x, o, steps, 3, True, alt=tb)
    fl = mix1d_flops_per_event(True, m.chunk)
    r = {"config0_mall_events": n, "config0_mall_chunk": m.chunk, "config0_mall_events_per_s": n * steps / w,
         "config0_mall_ms_per_step": 1e3 * w / steps, "config0_mall_event_kernel_us": 1e3 * k,
         "config0_mall_hbm_gbs": 8.0 * n / (k * 1e-3) / 1e9,
         "config0_mall_tflops": fl * n / (k * 1e-3) / 1e12, "config0_mall_flops_per_event": fl,
         "config0_mall_timing": info}
    del x
    return r


def config3_leg(steps: int = 20):
    """Config 3: masses and widths free (32 parameters), 4M events, the full
    grid normalization every call; then whole fits of 4M device-generated
    events with the adjoint gradient and with central finite differences
    (h = 1e-6 max(|theta|, 1)), from the same shifted start."""
    import torch
    import synth
    from paper_1710_08826_amd import Model
    desc3 = synth.dalitz_desc(free_lineshapes=True)
    th3 = synth.dalitz_truth(free_lineshapes=True)
    ev3 = torch.from_numpy(synth.dalitz_events(4_000_000, seed=synth.BASE_SEED + 3)).cuda()
    m3 = Model(desc3)
    t3 = torch.from_numpy(th3).cuda()
    t3b = torch.from_numpy(th3 * (1.0 + 1e-4 * np.cos(np.arange(th3.size)))).cuda()
    o3 = torch.empty(1 + m3.n_params, dtype=torch.float64, device="cuda")
    w3, k3, info = time_async(m3, t3, ev3, o3, steps, 3, True, alt=t3b)
    r = {"config3_events_per_s": 4_000_000 / w3 * steps, "config3_ms_per_step": 1e3 * w3 / steps,
         "config3_event_kernel_us": k3 * 1e3,
         "config3_event_kernel_tflops": dalitz_flops_per_event(desc3, 2, m3.chunk) * 4e6 / (k3 * 1e-3) / 1e12,
         "config3_timing": info}
    r.update(config3_fits(m3, th3))
    return r


def config3_fits(m3, th3, n: int = 4_000_000):
    """Minimizer wall time with and without the adjoint gradient on the
    config-3 model: n events generated on the device at the truth, start at
    coefficients x 1.03, masses x 1.002 and widths x 1.05 (c_0 fixed as the
    reference amplitude), 30 free parameters."""
    import torch
    import synth
    ev, _ = m3.generate(th3, n, seed=synth.BASE_SEED + 33)
    P = th3.size
    K = P // 4
    free = np.ones(P, np.int32)
    free[0:2] = 0
    start = th3.copy()
    start[2:2 * K] *= 1.03
    start[2 * K::2] *= 1.002
    start[2 * K + 1::2] *= 1.05
    out = {"config3_fit_events": n, "config3_fit_free_params": int(free.sum())}
    for mode in ("adjoint", "fd"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fr = m3.fit(start, ev, free=free, grad_mode=mode, raise_on_fail=False)
        wall = time.perf_counter() - t0
        pull = np.abs(fr.theta - th3)[free == 1] / np.maximum(fr.errors[free == 1], 1e-300)
        out[f"config3_fit_{mode}_wall_s"] = wall
        out[f"config3_fit_{mode}_iterations"] = fr.n_iter
        out[f"config3_fit_{mode}_nll_calls"] = fr.n_calls
        out[f"config3_fit_{mode}_status"] = fr.status
        out[f"config3_fit_{mode}_nll"] = fr.nll
        out[f"config3_fit_{mode}_max_pull"] = float(pull.max())
    out["config3_fit_speedup_adjoint_vs_fd"] = out["config3_fit_fd_wall_s"] / out["config3_fit_adjoint_wall_s"]
    return out


def tddp3_leg(steps: int = 50, k16: bool = True):
    """Time-dependent Dalitz-plot fit (the paper's pi+ pi- pi0 mixing
    workload class): 1M events, sixteen resonances (66 parameters; eight
    resonances and 34 parameters with k16 False), NLL + adjoint gradient, and
    the plain finite-difference gradient (2P + 1 NLL-only calls)."""
    import torch
    import synth
    from paper_1710_08826_amd import Model
    n = 1_000_000
    res = synth.TDDP_RESONANCES16 if k16 else synth.TDDP_RESONANCES
    desc = synth.tddp3_desc(resonances=res)
    th = synth.tddp3_truth(resonances=res)
    ev = torch.from_numpy(synth.tddp3_events(n, seed=synth.BASE_SEED + 7, resonances=res)).cuda()
    m = Model(desc)
    P = m.n_params
    _, tune_us = m.autotune(th, ev, reps=10)
    tdev = torch.from_numpy(th).cuda()
    tb = torch.from_numpy(th * (1.0 + 1e-3 * np.cos(np.arange(P)))).cuda()
    out = torch.empty(1 + P, dtype=torch.float64, device="cuda")
    w, k, info = time_async(m, tdev, ev, out, steps, 3, True, alt=tb)
    w0, k0, _ = time_async(m, tdev, ev, out, steps, 3, False, alt=tb)
    fl = tddp3_flops_per_event(desc, True, m.chunk)
    fd_step = (2 * P + 1) * w0 / steps
    return {"resonances": len(res), "events": n, "params": P, "grid": desc["grid"], "chunk": m.chunk,
            "autotune_us": {str(c): v for c, v in tune_us.items()},
            "events_per_s": n * steps / w, "ms_per_step": 1e3 * w / steps,
            "event_kernel_us": k * 1e3, "nll_only_event_kernel_us": k0 * 1e3,
            "flops_per_event": fl, "event_kernel_tflops": fl * n / (k * 1e-3) / 1e12,
            "plain_fd_grad_events_per_s": n / fd_step, "adjoint_vs_plain_fd": fd_step / (w / steps),
            "timing": info, **tddp3_whole_fit(m, th, n)}


def tddp3_whole_fit(m, th, n):
    """A whole fit (context for the paper's example wall times, which are for
    whole fits of a recorded sample): n events generated on the device at the
    truth, then the host quasi-Newton fit with the adjoint gradient from a
    shifted start, c_1..c_7 and x, y free (c_0 and cbar fixed, as in the
    parity tests), parabolic errors included."""
    import torch
    import synth
    ev, _ = m.generate(th, n, seed=synth.BASE_SEED + 8)
    P = th.size
    K = (P - 2) // 4
    free = np.zeros(P, np.int32)
    free[2:2 * K] = 1
    free[-2:] = 1
    start = th.copy()
    start[2:2 * K] *= 1.03
    start[-2:] *= 1.5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fr = m.fit(start, ev, free=free, raise_on_fail=False)
    wall = time.perf_counter() - t0
    pull = np.abs(fr.theta - th)[free == 1] / np.maximum(fr.errors[free == 1], 1e-300)
    return {"fit_events": n, "fit_free_params": int(free.sum()), "fit_wall_s": wall,
            "fit_iterations": fr.n_iter, "fit_nll_calls": fr.n_calls, "fit_status": fr.status,
            "fit_max_pull": float(pull.max())}


def td4_events_device():
    """The four-body event sample of the config-4 legs: 10M events, drawn on the host."""
    import torch
    import synth
    t0 = time.perf_counter()
    ev = torch.from_numpy(synth.td4_events(10_000_000, seed=synth.BASE_SEED + 4)).cuda()
    return ev, time.perf_counter() - t0


def td4_leg(steps: int = 10, split: bool = True, ev=None):
    """Config 4: the time-dependent four-body model, 10M events, 5M-point
    phase-space normalization sample; single-fit NLL + adjoint gradient, the
    plain finite-difference gradient, and 64 systematic-variation fits sharing
    the events (one events pass for all fits per step).  split: twenty
    distinct basis functions, ten in A and ten in Abar; otherwise ten shared
    basis functions with two coefficient sets."""
    import torch
    import synth
    from paper_1710_08826_amd import Model, VariationBatch
    n, n_mc, F = 10_000_000, 5_000_000, 64
    gen_s = None
    if ev is None:
        ev, gen_s = td4_events_device()
    desc = synth.td4_split_desc() if split else synth.td4_desc()
    th = synth.td4_split_truth() if split else synth.td4_truth()
    m = Model(desc)
    # the normalization sample generated on the device (the same points as
    # synth.td4_phase_space(n_mc, seed=BASE_SEED + 5))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.generate_norm_sample(n_mc, seed=synth.BASE_SEED + 5)
    mc_gen_s = time.perf_counter() - t0
    P = m.n_params
    tdev = torch.from_numpy(th).cuda()
    tb = torch.from_numpy(th * (1.0 + 1e-3 * np.cos(np.arange(P)))).cuda()
    out = torch.empty(1 + P, dtype=torch.float64, device="cuda")
    _, tune_us = m.autotune(th, ev, reps=5)
    fl_g, fl_0 = td4_flops_per_event(desc, True, m.chunk), td4_flops_per_event(desc, False, m.chunk)
    w, k, info = time_async(m, tdev, ev, out, steps, 2, True, alt=tb)
    w0, k0, _ = time_async(m, tdev, ev, out, steps, 2, False, alt=tb)
    r = {"model": ("20 distinct basis functions, 10 in A and 10 in Abar" if split else
                   "10 basis functions shared by A and Abar"),
         "events": n, "mc_points": n_mc, "params": P, "chunk": m.chunk,
         "autotune_us": {str(c): v for c, v in tune_us.items()},
         "cpu_generation_s": gen_s, "device_mc_sample_s": mc_gen_s,
         "single_events_per_s": n * steps / w, "single_ms_per_step": 1e3 * w / steps,
         "single_event_kernel_ms": k, "single_event_kernel_tflops": fl_g * n / (k * 1e-3) / 1e12,
         "nll_only_event_kernel_ms": k0, "nll_only_event_kernel_tflops": fl_0 * n / (k0 * 1e-3) / 1e12,
         "flops_per_event_fit": fl_g, "flops_per_event_fit_nll_only": fl_0, "timing": info}
    # plain finite differences: 2P + 1 NLL-only evaluations per gradient, one call at a time
    reps = 2
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        m.nll(th, ev)
        for p in range(P):
            h = 1e-6 * max(abs(th[p]), 1.0)
            tp = th.copy(); tp[p] += h
            tm = th.copy(); tm[p] -= h
            m.nll(tp, ev)
            m.nll(tm, ev)
    fd = (time.perf_counter() - t0) / reps
    r["plain_fd_grad_events_per_s"] = n / fd
    r["adjoint_vs_plain_fd"] = r["single_events_per_s"] / r["plain_fd_grad_events_per_s"]
    # 64 systematic variations: +-shifts of lineshape constants and the time resolution
    b = VariationBatch(m, F)
    fx = m.fixed()
    # phi(1020) width, rho(770) mass and width, f0(980) width, time resolution
    n12, n34 = len(desc["r12"]), len(desc["r34"])
    shifted = (3, 2 * n12 + 2, 2 * n12 + 3, 2 * n12 + 5, 2 * (n12 + n34))
    for f in range(F):
        v = fx.copy()
        j = shifted[f % 5]
        v[j] *= 1.0 + 0.002 * ((f // 5) - 6)
        b.set_fixed(f, v)
    ths = np.stack([th * (1.0 + 1e-3 * np.sin(np.arange(P) + f)) for f in range(F)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.nll(ths, ev, grad=True)  # builds the 64 normalization matrices
    r["batch_first_call_s"] = time.perf_counter() - t0
    b.nll(ths, ev, grad=True)  # one more untimed call
    reps = 8
    t0 = time.perf_counter()
    for _ in range(reps):
        b.nll(ths, ev, grad=True)
    wb = (time.perf_counter() - t0) / reps
    r["batch_fits"] = F
    r["batch_event_fits_per_s"] = n * F / wb
    r["batch_ms_per_step"] = 1e3 * wb
    r["batch_tflops"] = fl_g * n * F / wb / 1e12
    r["batch_vs_single_calls"] = (F * r["single_ms_per_step"]) / r["batch_ms_per_step"]
    # batched minimizer steps (evaluation + device BFGS update), a few iterations
    free = np.ones(P, np.int32)
    n_abar = sum(1 for a in desc["amps"] if len(a) < 4 or a[3] != "A")
    ref = P - 2 - 2 * n_abar
    free[ref: ref + 2] = 0  # Abar's first coefficient is the reference amplitude
    t0 = time.perf_counter()
    res = b.fit(ths, ev, free=free, max_iter=4)
    wf = time.perf_counter() - t0
    r["batch_fit_steps"] = int(res.n_evals.max())
    r["batch_fit_ms_per_step"] = 1e3 * wf / max(1, int(res.n_evals.max()))
    b.close()
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--quick", action="store_true", help="skip the side measurements and the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time direct launches instead of captured steps")
    ap.add_argument("--leg", choices=["td4", "serve", "vserve", "tddp3", "config3", "config0-mall", "cpu"],
                    help="run only the four-body leg or the serving leg and print its figures (for profiling)")
    ap.add_argument("--pmc-probe", nargs="?", const="config1",
                    choices=["config1", "config3", "tddp3", "td4", "td4batch", "config0mall"],
                    help="for counter runs: one 256 MiB device copy (calibration) then --steps "
                         "NLL+gradient steps of one workload, nothing printed but a summary line")
    ap.add_argument("--chunk", type=int, default=2048, help="summation chunk of the --pmc-probe steps")
    ap.add_argument("--chunk-c1", type=int, default=0,
                    help="config-1 summation chunk instead of the autotuner's choice (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(sharding events or fits across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.pmc_probe:
        pmc_probe(args.steps, args.chunk, args.pmc_probe)
        return
    if args.leg == "td4":
        ev4, gen_s = td4_events_device()
        c4 = td4_leg(ev=ev4)
        c4["cpu_generation_s"] = gen_s
        print(json.dumps({"config4": c4, "config4_shared_basis": td4_leg(split=False, ev=ev4)}), flush=True)
        return
    if args.leg == "serve":
        print(json.dumps({"config2_serving": serving_leg()}), flush=True)
        return
    if args.leg == "vserve":
        print(json.dumps({"config4_variation_serving": variation_serving_leg()}), flush=True)
        return
    if args.leg == "tddp3":
        print(json.dumps({"tddp3": tddp3_leg(), "tddp3_8res": tddp3_leg(k16=False)}), flush=True)
        return
    if args.leg == "config3":
        print(json.dumps(config3_leg()), flush=True)
        return
    if args.leg == "config0-mall":
        print(json.dumps(config0_above_mall()), flush=True)
        return
    if args.leg == "cpu":
        import synth
        print(json.dumps({"cpu_baseline": cpu_baseline(synth.dalitz_events(100_000, seed=synth.BASE_SEED),
                                                       synth.dalitz_desc(), synth.dalitz_truth()),
                          "cpu_baselines": cpu_baselines_other()}), flush=True)
        return

    import torch
    import synth
    from paper_1710_08826_amd import Model

    dev = "cuda"
    n1 = 1_000_000
    desc1 = synth.dalitz_desc()
    th1 = synth.dalitz_truth()
    th1b = th1 * (1.0 + 1e-3 * np.cos(np.arange(th1.size)))
    ev1_np = synth.dalitz_events(n1, seed=synth.BASE_SEED)
    ev1 = torch.from_numpy(ev1_np).to(dev)
    m1 = Model(desc1)
    P1 = m1.n_params
    tdev = torch.from_numpy(th1).to(dev)
    tdev_b = torch.from_numpy(th1b).to(dev)
    out = torch.empty(1 + P1, dtype=torch.float64, device=dev)
    # summation chunk from the library's autotuner on this sample (or given, for profiling runs)
    if args.chunk_c1:
        m1 = Model(dict(desc1, chunk=args.chunk_c1))
        tune_us = {}
    else:
        m1.autotune(th1, ev1, reps=20)
        # "chunk" for one event per thread and loop iteration, "chunk x2" for two
        tune_us = {(str(c) if e == 1 else f"{c} x2"): t for (c, e), t in m1.tune_table.items()}
    print(f"[bench] config1 dalitz: {n1} events, P={P1}, chunk {m1.chunk}, events per thread "
          f"{m1.events_per_thread}, warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    wall, kern_ms, info1 = time_async(m1, tdev, ev1, out, args.steps, args.warmup, True, alt=tdev_b,
                                      graph=not args.no_graph)
    ms_step = 1e3 * wall / args.steps
    value = n1 * args.steps / wall
    flops_ev = dalitz_flops_per_event(desc1, 1, m1.chunk)
    achieved = flops_ev * n1 / (kern_ms * 1e-3) / 1e12
    extra = {"config1_autotune_us": tune_us, "config1_timing": info1}
    print(f"[bench] {value:.4g} events/s, step {ms_step:.4f} ms, kernel {kern_ms * 1e3:.2f} us",
          file=sys.stderr, flush=True)

    if not args.quick:
        # NLL-only evaluations and the plain finite-difference gradient path:
        # one FD gradient = 2P+1 NLL-only evaluations, one call at a time
        w0, k0, _ = time_async(m1, tdev, ev1, out, args.steps, 5, False, alt=tdev_b)
        nll_only_rate = n1 * args.steps / w0
        nfd = max(10, args.steps // (2 * P1 + 1))
        theta_host = th1.copy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nfd):
            m1.nll(theta_host, ev1)
            for p in range(P1):
                h = 1e-6 * max(abs(theta_host[p]), 1.0)
                tp = theta_host.copy(); tp[p] += h
                tm = theta_host.copy(); tm[p] -= h
                m1.nll(tp, ev1)
                m1.nll(tm, ev1)
        fd_dt = (time.perf_counter() - t0) / nfd
        extra["config1_nll_only_events_per_s"] = nll_only_rate
        extra["config1_plain_fd_grad_events_per_s"] = n1 / fd_dt
        extra["config1_adjoint_vs_plain_fd"] = value / (n1 / fd_dt)
        extra["config1_nll_only_kernel_us"] = k0 * 1e3
        print(f"[bench] plain FD gradient {n1 / fd_dt:.4g} events/s", file=sys.stderr, flush=True)
        # device toy generation of 1M config-1 events (accept-reject on the model density)
        _, wgen = m1.generate(th1, 1000, seed=7)
        m1.generate(th1, n1, seed=7, envelope=wgen)
        t0 = time.perf_counter()
        for r in range(3):
            m1.generate(th1, n1, seed=8 + r, envelope=wgen)
        extra["config1_generate_events_per_s"] = 3 * n1 / (time.perf_counter() - t0)
        print(f"[bench] device generation {extra['config1_generate_events_per_s']:.4g} events/s",
              file=sys.stderr, flush=True)

        extra.update(config3_leg(max(10, args.steps // 10)))
        print(f"[bench] config3 {extra['config3_events_per_s']:.4g} events/s", file=sys.stderr, flush=True)

        # config 0: 1-D mixture, 100k events
        d0 = synth.mix1d_desc()
        x0 = torch.from_numpy(synth.mix1d_events(100_000)[None, :]).to(dev)
        m0 = Model(d0)
        t0d = torch.from_numpy(np.array(synth.CONFIG0_TRUTH)).to(dev)
        o0 = torch.empty(5, dtype=torch.float64, device=dev)
        t0d_b = torch.from_numpy(np.array(synth.CONFIG0_TRUTH) * 1.001).to(dev)
        w00, k00, _ = time_async(m0, t0d, x0, o0, args.steps, 10, True, alt=t0d_b)
        extra["config0_events_per_s"] = 100_000 * args.steps / w00
        extra["config0_ms_per_step"] = 1e3 * w00 / args.steps
        extra["config0_event_kernel_us"] = k00 * 1e3
        extra.update(config0_above_mall())
        # single fits: adjoint vs finite-difference gradient (config 0, 100k events)
        start = np.array(synth.CONFIG0_TRUTH) * 1.1
        for mode in ("adjoint", "fd"):
            m0.fit(start, x0, grad_mode=mode)
            t0 = time.perf_counter()
            reps = 5
            for _ in range(reps):
                r = m0.fit(start, x0, grad_mode=mode)
            dt = (time.perf_counter() - t0) / reps
            extra[f"config0_fit_{mode}_ms"] = dt * 1e3
            extra[f"config0_fit_{mode}_calls"] = r.n_calls
        extra["config0_fit_speedup_adjoint_vs_fd"] = extra["config0_fit_fd_ms"] / extra["config0_fit_adjoint_ms"]
        print(f"[bench] config0 fits: adjoint {extra['config0_fit_adjoint_ms']:.2f} ms, "
              f"fd {extra['config0_fit_fd_ms']:.2f} ms", file=sys.stderr, flush=True)

    if not args.quick:
        print("[bench] time-dependent Dalitz (pi+ pi- pi0-like, 16 and 8 resonances, 1M events) ...",
              file=sys.stderr, flush=True)
        extra["tddp3"] = tddp3_leg()
        extra["tddp3_8res"] = tddp3_leg(k16=False)
        for key in ("tddp3", "tddp3_8res"):
            t3 = extra[key]
            print(f"[bench] {key} ({t3['resonances']} resonances): {t3['events_per_s']:.4g} events/s "
                  f"({t3['event_kernel_tflops']:.2f} TFLOP/s), adjoint vs FD {t3['adjoint_vs_plain_fd']:.1f}x, "
                  f"whole fit {t3['fit_wall_s']:.3f} s", file=sys.stderr, flush=True)

    if not args.quick:
        print("[bench] config4 td4 (10M events, 5M-point sample, 64 variation fits) ...", file=sys.stderr,
              flush=True)
        ev4, gen_s = td4_events_device()
        extra["config4"] = td4_leg(ev=ev4)
        extra["config4"]["cpu_generation_s"] = gen_s
        extra["config4_shared_basis"] = td4_leg(split=False, ev=ev4)
        del ev4
        for key in ("config4", "config4_shared_basis"):
            c4 = extra[key]
            print(f"[bench] {key} ({c4['model']}): single {c4['single_events_per_s']:.4g} events/s "
                  f"({c4['single_event_kernel_tflops']:.2f} TFLOP/s), 64 fits {c4['batch_event_fits_per_s']:.4g} "
                  f"event-fits/s, adjoint vs FD {c4['adjoint_vs_plain_fd']:.1f}x", file=sys.stderr, flush=True)

    if not args.quick:
        print("[bench] config4 variation serving (192 requests, 64 slots) ...", file=sys.stderr, flush=True)
        vs = variation_serving_leg()
        extra["config4_variation_serving"] = vs
        print(f"[bench] config4 variations: {vs['closed_loop']['fits_per_s']:.4g} fits/s closed loop, Poisson "
              f"p50 {vs['poisson']['p50_latency_s']:.3f} s p99 {vs['poisson']['p99_latency_s']:.3f} s",
              file=sys.stderr, flush=True)

    if not args.quick:
        print("[bench] config2 serving (4096 toy fits) ...", file=sys.stderr, flush=True)
        sv = serving_leg()
        extra["config2_serving"] = sv
        print(f"[bench] config2: {sv['closed_loop']['fits_per_s']:.4g} fits/s closed loop, "
              f"Poisson p50 {sv['poisson']['p50_latency_s'] * 1e3:.2f} ms p99 "
              f"{sv['poisson']['p99_latency_s'] * 1e3:.2f} ms; one-at-a-time adjoint "
              f"{sv['one_at_a_time_poisson']['fits_per_s']:.4g} fits/s (p50 "
              f"{sv['one_at_a_time_poisson']['p50_latency_s'] * 1e3:.1f} ms), plain FD "
              f"{sv['one_at_a_time_fd']['fits_per_s']:.4g} fits/s", file=sys.stderr, flush=True)

    cpu = None
    if not args.quick and not args.no_cpu:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(ev1_np[:, :100_000], desc1, th1)
        extra["cpu_baselines"] = cpu_baselines_other()

    line = {
        "metric": "event-NLL(+grad) evals/sec vs plain; toy fits/sec with p50/p99 latency",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "dalitz3 8-resonance amplitude fit, NLL + adjoint gradient",
                   "events": n1, "params": P1, "grid": [1024, 1024], "normalization": "cached grid matrix",
                   "chunk": m1.chunk, "events_per_thread": m1.events_per_thread, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic(m1.chunk, m1.events_per_thread),
                     "kernel": "fn_dal_ev1 (Dalitz events pass, coefficient gradient)",
                     "kernel_us": kern_ms * 1e3, "flops_per_event": flops_ev,
                     "counted_fp64_flops_per_event": counted_flops(m1.chunk, m1.events_per_thread),
                     "counted_fp64_tflops": (counted_flops(m1.chunk, m1.events_per_thread) * n1
                                             / (kern_ms * 1e-3) / 1e12
                                             if counted_flops(m1.chunk, m1.events_per_thread) else None),
                     "hbm_gbs": 16 * n1 / (kern_ms * 1e-3) / 1e9},
        "cpu_baseline": cpu,
        "extra": extra,
        "gpu": gpu_info(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
