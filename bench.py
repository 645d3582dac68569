"""Benchmark: Chebyshev density-matrix columns per second on one MI355X.

Workload (the configuration the metric is quoted on): K = 4096 basis
functions (1024 atoms in a sphere, four s-Gaussians each), FP64 recursion
over all K columns (64 blocks of 64, advanced together), order N = 1000,
beta = 200 /hartree, N_e = 2048, spin factor 2.

One step = the whole path for one (F, S): operator setup and Lanczos bounds
(dm_set_fock), coefficients, start block and the N-term recursion with the
fused P accumulation and moment reductions for every column
(dm_chebyshev_block), then the chemical-potential bisection and band energy
from that step's moments (dm_solve_mu, dm_trace).  The step computes P at the
mu solved by the previous step (steady state of a self-consistent loop; the
first warm-up step solves it from a pass at mu = 0) and checks the electron
count of its own moments.

Besides the headline line's own roofline (the FP64 recursion kernel), the
JSON carries more measured points: hbm_point (the FP32 recursion of the
K = 32768 cluster against a 32-column block, HBM-bound), hbm_point_refined
(the same pass with FP32 storage and FP64 sums) and factored_point
(the paper's factored application of S^-1 F on the benchmark cluster: a
sparse product with F and a preconditioned CG solve with S per step, with
the roofline of its S products).

Prints one JSON line.  --gpus N with N > 1 is not supported (one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "K4096_sphere1024_fp64"
METRIC = "density-matrix columns/sec and SpMM GB/s (% HBM roofline) at max|dP|<=1e-6"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE averages per recursion launch of this
# workload (KiB), and the scale factors from a plain 1 GiB copy (FETCH_SIZE
# counts half of the bytes a copy reads on this part, WRITE_SIZE all of them).
# Valid only for the recursion-step code they were taken with: the text of
# gemm.hip before the persistent-batch section (GEMM_STEP_END).
GEMM_STEP_END = b"// ------------------------------------------------------------ persistent batch"
COUNTERS = {"kernel_source_sha256_16": "5d81961b90d81fd3", "fetch_kib": 997402.8,
            "write_kib": 262023.8, "fetch_scale": 2.0, "write_scale": 1.0}


HBM_WORKLOAD = "K32768_sphere8192_fp32"
HBM_COLUMNS = 32
HBM_ORDER = 200
# tile shapes of the HBM point, pinned (the library's defaults for this pass):
# 128 x 32, three slabs in flight, 8 k per lane, the column panel in LDS;
# the refined twin with the panel read by every wave (no LDS)
HBM_CFG, HBM_KERNEL = 30, "cheb_step_kernel<float,2,2,4,1,8,4,true>"
HBM_CFG_REFINED, HBM_KERNEL_REFINED = 22, "cheb_step_kernel<W32,2,2,4,1,8,4,false>"
# the K = 32768 workload's whole configuration (every column): pass width and
# tile shape, and the steps timed
FULL_WIDTH, FULL_CFG, FULL_STEPS = 16384, 27, 4
# the same counters for the recursion launch of the HBM point (FP32, 32 columns)
COUNTERS_HBM = {"kernel_source_sha256_16": "5d81961b90d81fd3", "cfg": 30, "fetch_kib": 2124152.9, "write_kib": 12215.8,
                "fetch_scale": 2.0, "write_scale": 1.0}


# the factored form (S^-1 F applied by a product with F and a CG solve with S
# per step): all K columns of the benchmark cluster in one block, a bounded
# number of recursion steps (each one solve); the rate scales to order N
FACT_ORDER = 8
# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of the S product (rg_spmm_kernel<1,2>)
# of the factored point, averaged over the launches that did work (launches
# queued after every column converged return at once and are left out);
# valid for the device code (the text before the host-side marker) hashed here
COUNTERS_FACT = {"kernel_source_sha256_16": "418518f5b6973c24", "fetch_kib": 3195347.1, "write_kib": 505611.7,
                 "fetch_scale": 2.0, "write_scale": 1.0}


# the device-code part of factored.hip ends at this line (host code follows)
FACT_DEVICE_END = b"// --------------------------------------------------------------- host side"
# the part of each source that a counter or profile is valid for ends here
SOURCE_MARKERS = {"factored.hip": FACT_DEVICE_END, "gemm.hip": GEMM_STEP_END}


def kernel_source_hash(name="gemm.hip", upto=None):
    """sha256[:16] of a kernel source file, or of its text before `upto`."""
    import hashlib

    path = os.path.join(ROOT, "paper_2108_13478_amd", "csrc", name)
    with open(path, "rb") as f:
        data = f.read()
    if upto is not None:
        data = data[:data.index(upto)]
    return hashlib.sha256(data).hexdigest()[:16]


def cpu_baseline(cluster, order, beta, n_e, budget_s=30.0):
    """The oracle (generalized eigh + C p_N(e) C^T for every column) on the host."""
    import numpy as np

    import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    reps = 0
    while True:
        sp = O.spectrum(cluster)
        w = sp.e[-1] - sp.e[0]
        emin, emax = sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w
        mu = O.solve_mu_poly(sp, n_e, order, beta, emin, emax, tol=1e-6)
        P = O.density_matrix_poly(sp, np.arange(cluster.K), order, mu, beta, emin, emax)
        del P
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s / 3 or reps >= 3:
            break
    out = {"value": reps * cluster.K / el, "unit": "columns/s", "cores": threads, "kind": "oracle",
           "sample": f"{reps} full density matrix(es), K={cluster.K}: eigh(F,S) + mu bisection + "
                     f"C diag(p_N) C^T for all columns, numpy/scipy FP64, {el:.1f} s"}
    # like-for-like CPU rate: the same column recursion in numpy (dense
    # H_N = (S^-1 F - Ebar)/dE, FP64, one block of 64 columns), a bounded
    # number of steps, scaled to the order of the workload
    import scipy.linalg

    nb, steps = 64, 40
    F, S = cluster.F_dense(), cluster.S_dense()
    ebar, de = 0.5 * (emax + emin), 0.5 * (emax - emin)
    t0 = time.perf_counter()
    HN = (scipy.linalg.solve(S, F, assume_a="pos") - ebar * np.eye(cluster.K)) / de
    t_setup = time.perf_counter() - t0
    E = np.zeros((cluster.K, nb))
    E[np.arange(nb), np.arange(nb)] = 1.0
    t0 = time.perf_counter()
    U0 = scipy.linalg.solve(S, E, assume_a="pos")
    U1 = HN @ U0
    for _ in range(steps - 1):
        U0, U1 = U1, 2.0 * (HN @ U1) - U0
    t_rec = time.perf_counter() - t0
    rate = nb * steps / t_rec / order
    out["recursion"] = {"value": rate, "unit": "columns/s", "cores": threads, "kind": "numpy recursion",
                        "sample": f"{nb} columns x {steps} steps of the dense FP64 column recursion "
                                  f"(H_N built by a dense solve, {t_setup:.1f} s, not counted) in "
                                  f"{t_rec:.2f} s, scaled to N={order}"}
    return out


def hbm_point(stream, refined=False):
    """The memory-bound point of the recursion: the FP32 operator of the
    K = 32768 workload streamed against a 32-column block (arithmetic
    intensity 16 flop/B, below the FP32 ridge of 19.7), timed live with HIP
    events on the library's stream.  refined: the same pass in the refined
    precision (FP32 storage, FP64 MFMA sums: 16 flop per FP32 byte against
    the FP64 ridge of 9.8, so bound by the f64 matrix cores)."""
    import numpy as np
    import torch

    import paper_2108_13478_amd as dmlib
    from synth import WORKLOADS, workload

    w = WORKLOADS[HBM_WORKLOAD]
    print(f"[bench] building inputs {HBM_WORKLOAD}", file=sys.stderr, flush=True)
    c = workload(HBM_WORKLOAD)
    K = c.K
    prec = dmlib.DM_FP32_ACC64 if refined else dmlib.DM_FP32
    ctx = dmlib.Context(device=0, stream=stream.cuda_stream, precision=prec)
    ctx.set_cluster(c)
    ctx.dm_set_pass_shape(HBM_COLUMNS, HBM_CFG_REFINED if refined else HBM_CFG)
    cols = torch.arange(HBM_COLUMNS, dtype=torch.int64, device="cuda:0")
    ctx.dm_chebyshev_block(cols, 20, 0.0, w["beta"], None)  # warm-up pass
    ctx.dm_reset_moments()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.dm_chebyshev_block(cols, HBM_ORDER, 0.0, w["beta"], None)
    e1.record(stream)
    torch.cuda.synchronize()
    launch_ms = e0.elapsed_time(e1) / HBM_ORDER
    full = None
    if not refined:
        # the same operator's whole configuration: every column, advanced in
        # passes of 16384 columns on the 128 x 128 tile (the autotuned choice
        # at this size); per-step time from two passes that differ by
        # FULL_STEPS steps, so start and end of a pass cancel
        allc = torch.arange(K, dtype=torch.int64, device="cuda:0")
        ctx.dm_set_pass_shape(FULL_WIDTH, FULL_CFG)
        ms = []
        for n in (2, 2 + FULL_STEPS):
            f0 = torch.cuda.Event(enable_timing=True)
            f1 = torch.cuda.Event(enable_timing=True)
            f0.record(stream)
            ctx.dm_chebyshev_block(allc, n, 0.0, w["beta"], None)
            f1.record(stream)
            torch.cuda.synchronize()
            ms.append(f0.elapsed_time(f1))
        step_ms = (ms[1] - ms[0]) / FULL_STEPS
        full = {"columns": K, "pass_width": FULL_WIDTH, "tile": "128x128 (8 k per lane, three slabs)",
                "step_ms": step_ms, "tflops": 2.0 * K ** 3 / (step_ms * 1e-3) / 1e12,
                "order": w["order"], "columns_per_s_at_order": K / ((w["order"] + 1) * step_ms * 1e-3)}
    ctx.close()
    # per launch: the FP32 operator once, U_l, U_{l-1} read and U_{l+1} written
    # (FP32), Z read (FP64), P read and written (FP64)
    alg_bytes = 4.0 * K * K + K * HBM_COLUMNS * (3 * 4 + 8 + 16)
    flops = 2.0 * K * K * HBM_COLUMNS
    gbs = alg_bytes / (launch_ms * 1e-3) / 1e9
    if refined:
        tf = flops / (launch_ms * 1e-3) / 1e12
        return {"workload": HBM_WORKLOAD, "K": K, "columns": HBM_COLUMNS, "steps_timed": HBM_ORDER,
                "precision": "fp32 storage, fp64 sums", "bound": "mfma", "kernel": HBM_KERNEL_REFINED,
                "launch_ms": launch_ms, "algorithmic_bytes": alg_bytes, "achieved": tf, "unit": "TFLOP/s",
                "peak": PEAK_FP64_TFLOPS, "frac": tf / PEAK_FP64_TFLOPS, "algorithmic_GBps": gbs,
                "hbm_frac": gbs / PEAK_HBM_GBS, "traffic": None}
    traffic = None
    if (kernel_source_hash("gemm.hip", GEMM_STEP_END) == COUNTERS_HBM["kernel_source_sha256_16"]
            and COUNTERS_HBM["cfg"] == HBM_CFG):
        traffic = 1024.0 * (COUNTERS_HBM["fetch_kib"] * COUNTERS_HBM["fetch_scale"]
                            + COUNTERS_HBM["write_kib"] * COUNTERS_HBM["write_scale"])
    return {"workload": HBM_WORKLOAD, "K": K, "columns": HBM_COLUMNS, "steps_timed": HBM_ORDER,
            "precision": "fp32", "bound": "hbm", "kernel": HBM_KERNEL,
            "launch_ms": launch_ms, "algorithmic_bytes": alg_bytes, "achieved": gbs, "unit": "GB/s",
            "peak": PEAK_HBM_GBS, "frac": gbs / PEAK_HBM_GBS, "traffic": traffic,
            "counter_GBps": None if traffic is None else traffic / (launch_ms * 1e-3) / 1e9,
            "tflops": flops / (launch_ms * 1e-3) / 1e12, "all_columns": full}


def factored_point(stream, mu):
    """The factored form on the benchmark cluster: every application of
    H = S^-1 F is a sparse product with F and an FSAI-preconditioned CG solve
    with S (the paper's route).  Times a pass over all K columns with
    FACT_ORDER recursion steps (FACT_ORDER + 1 solves) with HIP events on the
    library's stream, and the S products inside the CG iterations (the
    dominant kernel) with the library's own per-launch HIP events.  P of the
    pass is compared with the explicit-operator path at the same order."""
    import numpy as np
    import torch

    import paper_2108_13478_amd as dmlib
    from synth import WORKLOADS, workload

    w = WORKLOADS[WORKLOAD]
    beta, order = w["beta"], w["order"]
    print("[bench] factored form", file=sys.stderr, flush=True)
    c = workload(WORKLOAD)
    K = c.K
    dev = torch.device("cuda:0")
    ctx = dmlib.Context(device=0, stream=stream.cuda_stream, precision=dmlib.DM_FP64)
    ctx.dm_set_operator_form(dmlib.DM_FORM_FACTORED)
    t0 = time.perf_counter()
    ctx.set_cluster(c)
    setup_s = time.perf_counter() - t0
    lo, hi = ctx.dm_get_bounds()
    cols = torch.arange(K, dtype=torch.int64, device=dev)
    Pf = torch.empty((K, K), dtype=torch.float64, device=dev)
    ctx.dm_chebyshev_block(cols, 2, mu, beta, None)  # warm-up pass
    ctx.dm_cg_stats()
    ctx.dm_cg_timing(1)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.dm_chebyshev_block(cols, FACT_ORDER, mu, beta, Pf)
    e1.record(stream)
    torch.cuda.synchronize()
    pass_ms = e0.elapsed_time(e1)
    n_launch, spmm_ms = ctx.dm_cg_timing(0)
    solves, iters, max_iters = ctx.dm_cg_stats()
    ctx.close()
    # the explicit-operator path on the same interval, order and columns
    ctxd = dmlib.Context(device=0, stream=stream.cuda_stream, precision=dmlib.DM_FP64)
    ctxd.set_cluster(c)
    ctxd.dm_set_bounds(lo, hi)
    Pd = torch.empty((K, K), dtype=torch.float64, device=dev)
    ctxd.dm_chebyshev_block(cols, FACT_ORDER, mu, beta, Pd)
    torch.cuda.synchronize()
    ctxd.close()
    diff = float((Pf - Pd).abs().max())
    del Pf, Pd
    col_steps = K * (FACT_ORDER + 1) / (pass_ms * 1e-3)
    nnz_S = len(c.S_val)
    launch_ms = spmm_ms / max(n_launch, 1)
    # useful flops of one S product over the block (2 per stored entry and
    # column), and its algorithmic bytes: S in CSR once, the block Z read
    # once, the fused direction update (Pd, Q read and written)
    flops = 2.0 * nnz_S * K
    alg_bytes = 12.0 * nnz_S + 8.0 * (K + 1) + 5.0 * 8.0 * K * K
    achieved = flops / (launch_ms * 1e-3) / 1e12
    gbs = alg_bytes / (launch_ms * 1e-3) / 1e9
    traffic = None
    if COUNTERS_FACT and kernel_source_hash("factored.hip", FACT_DEVICE_END) == COUNTERS_FACT["kernel_source_sha256_16"]:
        traffic = 1024.0 * (COUNTERS_FACT["fetch_kib"] * COUNTERS_FACT["fetch_scale"]
                            + COUNTERS_FACT["write_kib"] * COUNTERS_FACT["write_scale"])
    return {"workload": WORKLOAD, "K": K, "columns": K, "steps_timed": FACT_ORDER, "solves_timed": solves,
            "precision": "fp64", "setup_s": setup_s, "pass_ms": pass_ms,
            "column_steps_per_s": col_steps, "columns_per_s_at_order": col_steps / (order + 1),
            "order": order, "cg_iterations_per_solve": iters / max(solves, 1),
            "cg_max_iterations": max_iters, "cg_tol": 1e-11, "max_abs_dP_vs_explicit_operator": diff,
            "roofline": {"bound": "alu", "kernel": "rg_spmm_kernel<1,2> (S product of the CG iteration)",
                         "launches_timed": n_launch, "launch_ms": launch_ms, "achieved": achieved,
                         "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                         "algorithmic_bytes": alg_bytes, "spmm_GBps": gbs, "spmm_hbm_frac": gbs / PEAK_HBM_GBS,
                         "traffic": traffic,
                         "counter_GBps": None if traffic is None else traffic / (launch_ms * 1e-3) / 1e9}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-factored-point", action="store_true",
                    help="skip the factored-form (sparse F, CG solve with S) measurement")
    ap.add_argument("--factored-only", action="store_true",
                    help="only the factored-form measurement (at mu = 0), for profiling")
    ap.add_argument("--no-hbm-point", action="store_true",
                    help="skip the memory-bound FP32 K=32768 / 32-column measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1, "
                                   "the multi-GPU column sharding is not part of this build"}))
        sys.exit(2)
    if args.copy_calibration:
        import torch

        n = 1 << 27  # 2^27 doubles = 1 GiB read + 1 GiB written per copy
        x = torch.ones(n, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 8 * n, "copy_calibration_bytes_written": 8 * n,
                          "copies": 3}), flush=True)
        return

    import numpy as np
    import torch

    import paper_2108_13478_amd as dmlib
    from synth import WORKLOADS, workload

    if args.factored_only:
        stream = torch.cuda.Stream()
        torch.cuda.set_stream(stream)
        print(json.dumps({"factored_point": factored_point(stream, 0.0)}), flush=True)
        return

    w = WORKLOADS[WORKLOAD]
    order, beta, n_e = w["order"], w["beta"], w["n_electrons"]
    print(f"[bench] building inputs {WORKLOAD}", file=sys.stderr, flush=True)
    c = workload(WORKLOAD)
    K = c.K
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    F = (t(c.F_rowptr), t(c.F_col), t(c.F_val))
    S = (t(c.S_rowptr), t(c.S_col), t(c.S_val))
    cols = torch.arange(K, dtype=torch.int64, device=dev)
    P = torch.empty((K, K), dtype=torch.float64, device=dev)  # row j = column j of P
    stream = torch.cuda.Stream()  # a real stream: the library and the events share it
    torch.cuda.set_stream(stream)
    ctx = dmlib.Context(device=0, stream=stream.cuda_stream, precision=dmlib.DM_FP64)
    rec_ms = []
    state = {"mu": 0.0, "tr_err": None}

    def step(timed):
        ctx.dm_set_fock(K, *F, *S, 4)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.dm_chebyshev_block(cols, order, state["mu"], beta, P)
        e1.record(stream)
        tr, eb = ctx.dm_trace(state["mu"], beta)
        state["tr_err"] = abs(2.0 * tr - n_e)
        state["eband"] = eb
        state["mu"] = ctx.dm_solve_mu(n_e, beta, tol=1e-6)
        if timed:
            rec_ms.append(e0.elapsed_time(e1))

    for i in range(args.warmup):
        print(f"[bench] warmup {i}", file=sys.stderr, flush=True)
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        print(f"[bench] step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = 1e3 * el / args.steps

    # dominant kernel: the recursion step, 2 K^2 flops per column per launch
    launch_ms = float(np.mean(rec_ms)) / order
    flops = 2.0 * K * K * K
    achieved = flops / (launch_ms * 1e-3) / 1e12
    traffic = None
    if kernel_source_hash("gemm.hip", GEMM_STEP_END) == COUNTERS["kernel_source_sha256_16"]:
        traffic = 1024.0 * (COUNTERS["fetch_kib"] * COUNTERS["fetch_scale"]
                            + COUNTERS["write_kib"] * COUNTERS["write_scale"])
    # algorithmic bytes per launch: operator K^2, reads of U_l, U_{l-1}, Z, P and
    # writes of U_{l+1}, P (K x columns each), FP64
    alg_bytes = 8.0 * (K * K + 6.0 * K * K)
    out = {
        "metric": METRIC,
        "value": K * args.steps / el,
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "K": K, "order": order, "beta": beta, "n_electrons": n_e,
                   "columns_per_step": K, "column_block": 64, "precision": "fp64",
                   "nnz_per_row_F_S": [round(x, 1) for x in c.nnz_per_row]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": "cheb_step_kernel<double,4,4,2,2,4,4,false>", "launch_ms": launch_ms,
                     "algorithmic_bytes": alg_bytes,
                     "algorithmic_GBps": alg_bytes / (launch_ms * 1e-3) / 1e9,
                     "counter_GBps": None if traffic is None else traffic / (launch_ms * 1e-3) / 1e9,
                     "hbm_peak_GBps": PEAK_HBM_GBS},
        "electron_count_error": state["tr_err"],
        "mu": state["mu"],
        "band_energy": state["eband"],
    }
    ctx.close()
    if not args.no_hbm_point:
        out["hbm_point"] = hbm_point(stream)
        out["hbm_point_refined"] = hbm_point(stream, refined=True)
    if not args.no_factored_point:
        out["factored_point"] = factored_point(stream, state["mu"])
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(c, order, beta, n_e)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
