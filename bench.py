#!/usr/bin/env python3
"""Benchmark of the refinement hot path on one MI355X.

One step = one complete zf_refine call on one synthetic overlap matrix: setup
(split, Z0), every low-precision sweep, the refinement phase with its residual
evaluations, and the copy-out of Z.  Inputs are resident in HBM before the timed
region starts.  The headline refinement (--refine, default crt_first) takes its
first residual from FP64 products emulated through residues on the int8 matrix
cores and every later one, the stopping norm and the final residual included, in
FP64; the other modes are timed beside it (refine_modes).

Reported (one JSON line):
  value        refined-Z TFLOP/s of the mixed path (BF16x3 sweeps + the
               refinement phase) on the N = 4096 overlap: the method's irreducible
               flops / time, where one residual evaluation counts 3 N^3 (S Z and
               the symmetric Z^T (S Z)) and one update of order m counts
               (m + 1) N^3 (m - 1 symmetric delta products and Z Q);
               tflops_paper_count gives the dense count (4 N^3 + 2 m N^3)
  ms_per_step  its time-to-solution; fp64.* holds the plain FP64 path
  roofline     the dominant kernel (most time in the timed region), timed with
               HIP events on the library's stream, and every BF16 kernel together
  cpu_baseline the CPU FP64 oracle on the same matrix (one evaluation and one
               update, all threads and one thread), extrapolated to the solve:
               T_oracle / T_gpu
  configs      the other workloads (N = 256 FP64, the N = 5049 cluster, the
               N = 3000 MD warm start, the 512-matrix batch), each with its
               oracle-checked residual (--headline-only skips them)
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("refined-Z TFLOP/s + time-to-‖ZᵀSZ−I‖≤1e-6, mixed vs FP64 path, "
          "1 MI355X")
PEAK_TFLOPS = {"bf16": 2500.0, "fp64": 78.6, "fp32": 157.3, "int8": 5000.0}
# Sources of the GEMM kernels; an HBM-traffic record in profiles/ is used only while
# they hash to the value it was measured with.
GEMM_SOURCES = ["paper_2404_19163_amd/csrc/gemm.hip", "paper_2404_19163_amd/csrc/gemm_tiles.inc",
                "paper_2404_19163_amd/csrc/zf_tiles.h", "paper_2404_19163_amd/csrc/zf_internal.h"]
TRAFFIC_PROFILE = "profiles/gemm_gauss4096.md"


def measured_traffic(kernel: str, n: int):
    """(HBM bytes per launch, algorithmic bytes per launch) of `kernel` at order n from
    the rocprofv3 FETCH_SIZE / WRITE_SIZE record in profiles/, or (None, None) when
    there is none or the kernel sources changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, TRAFFIC_PROFILE)).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        h = hashlib.sha256()
        for f in GEMM_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
    except (OSError, AttributeError, ValueError):
        return None, None
    if not isinstance(rec, dict) or rec.get("kernel") != kernel or rec.get("n") != n or rec.get("sources_sha256") != h.hexdigest():
        return None, None
    return rec["traffic_bytes_per_dispatch"], rec.get("alg_bytes_per_dispatch")
KCLASS_DTYPE = {"gemm_x3": "bf16", "gemm_x3_sym": "bf16", "gemm_f64": "fp64", "gemm_f64_sym": "fp64",
                "gemm_hh": "bf16", "gemm_hh_sym": "bf16", "gemm_f32": "fp32", "gemm_f32_sym": "fp32",
                "gemm_x3f16": "bf16", "gemm_x3f16_sym": "bf16", "gemm_hhf16": "bf16",
                "gemm_hhf16_sym": "bf16", "gemm_oz": "int8", "gemm_oz_sym": "int8",
                "gemm_crt": "int8", "gemm_crt_sym": "int8"}

WORKLOADS = {
    "gauss4096": dict(n=4096, sigma=1.0,
                      desc="Gaussian-kernel overlap, N=4096 atoms at 0.1/A^3 (random sequential "
                           "addition, d_min 0.8 A), S_ij=exp(-r^2/2), sigma 1.0 A"),
    "gauss256": dict(n=256, sigma=1.2,
                     desc="Gaussian-kernel overlap, N=256, sigma 1.2 A"),
    "gauss3000": dict(n=3000, sigma=1.0,
                      desc="Gaussian-kernel overlap, N=3000, sigma 1.0 A (one frame of md3000)"),
    "cluster5049": dict(n=5049, sigma=None,
                        desc="561-atom fcc cuboctahedron, 1s+3p+5d Gaussians, alpha 0.08 bohr^-2, "
                             "N=5049"),
}


REFINE_DESC = {
    "crt_first": "refinement phase (Algorithm 3): first residual from FP64 products emulated "
                 "through residues on the int8 matrix cores, the stopping norm and the final "
                 "residual in FP64, BF16x3 corrections",
    "f64_delta": "refinement phase (Algorithm 3): FP64 residuals, BF16x3 corrections",
    "crt": "refinement phase (Algorithm 3): every residual from FP64 products emulated through "
           "residues, BF16x3 corrections",
    "emu": "refinement phase (Algorithm 3): every residual from FP64 products emulated with "
           "integer slices, BF16x3 corrections",
    "f64_full": "refinement phase (Algorithm 3): FP64 residuals and FP64 corrections",
}


def alg_flops(n: int, order: int, evals: int, updates: int) -> float:
    """The method's irreducible flops: a residual evaluation is S Z (2 N^3) plus the
    symmetric Z^T (S Z) (N^3); an update of order m is m - 1 symmetric delta products
    plus Z Q (2 N^3).  Order 2: 6 N^3 per sweep."""
    n3 = float(n) ** 3
    return n3 * (3.0 * evals + (order + 1.0) * updates)


def paper_flops(n: int, order: int, evals: int, updates: int) -> float:
    """The paper's count of the same work with every product dense (Sec. III.B: the
    four N x N products of a sweep): 4 N^3 per evaluation, 2 m N^3 per update."""
    return float(n) ** 3 * (4.0 * evals + 2.0 * order * updates)


def kernel_alg_flops(cls: str, n: int) -> float:
    """Algorithmic flops of one launch at order n (no padding, no duplicated work)."""
    n = float(n)
    return {"gemm_x3": 6 * n ** 3, "gemm_x3_sym": 3 * n * n * (n + 1),
            "gemm_f64": 2 * n ** 3, "gemm_f64_sym": n * n * (n + 1),
            "gemm_hh": 2 * n ** 3, "gemm_hh_sym": n * n * (n + 1),
            "gemm_f32": 2 * n ** 3, "gemm_f32_sym": n * n * (n + 1),
            "gemm_x3f16": 6 * n ** 3, "gemm_x3f16_sym": 3 * n * n * (n + 1),
            "gemm_hhf16": 2 * n ** 3, "gemm_hhf16_sym": n * n * (n + 1),
            # emulated FP64 products: the FP64 flops they stand for
            "gemm_crt": 2 * n ** 3, "gemm_crt_sym": n * n * (n + 1),
            "gemm_oz": 2 * n ** 3, "gemm_oz_sym": n * n * (n + 1)}.get(cls, 0.0)


def timed_solves(fn, steps: int, warmup: int):
    """Median-free mean wall time per call of fn() over `steps` calls after `warmup`
    untimed ones, bracketed by device synchronizations; returns (seconds, last result)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(steps):
        last = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, last


def lowdin_error(S_np, Z_list):
    """Relative Frobenius distance of each Z to the Loewdin factor S^(-1/2) (dense
    eigendecomposition, the closed form every polynomial-in-S guess converges to)."""
    from oracle import zf_oracle as O
    L = O.lowdin(S_np)
    nl = float(np.linalg.norm(L))
    return [float(np.linalg.norm(Z - L) / nl) for Z in Z_list]


def cpu_oracle_baseline(S_np, order: int, evals: int, updates: int, gpu_s: float,
                        workload: str):
    """The CPU FP64 oracle on the same matrix: one residual evaluation and one update of
    its recursion with every BLAS thread the process may use, and one evaluation on a
    single thread.  The solve's oracle time is extrapolated from these to the FP64
    path's evaluation and update counts; T_oracle / T_gpu is a time ratio of the same
    solve."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import zf_oracle as O
    n = S_np.shape[0]
    eye = np.eye(n)
    Z = O.scaled_identity_guess(S_np)

    def one_eval(Z):
        delta = eye - O.gram(S_np, Z)
        return delta, O.frobenius(delta)

    t0 = time.perf_counter()
    delta, _ = one_eval(Z)
    t_eval = time.perf_counter() - t0
    t0 = time.perf_counter()
    Z = Z + Z @ O.correction(delta, order)
    t_upd = time.perf_counter() - t0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        one_eval(Z)
        t_eval1 = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    est = t_eval * evals + t_upd * updates
    flops = alg_flops(n, order, 1, 1)
    try:
        blas = np.show_config(mode="dicts")["Build Dependencies"]["blas"]["name"]
    except Exception:  # noqa: BLE001 (older numpy: no dict mode)
        blas = "unknown"
    return {"value": round(flops / (t_eval + t_upd) / 1e12, 5), "unit": "TFLOP/s",
            "cores": len(os.sched_getaffinity(0)), "threads": threads, "kind": "oracle",
            "blas": blas,
            "sample": f"{workload}: one residual evaluation ({t_eval:.2f} s) and one update "
                      f"({t_upd:.2f} s) of the FP64 oracle recursion, irreducible-flop basis",
            "eval_s": round(t_eval, 3), "update_s": round(t_upd, 3),
            "eval_s_1thread": round(t_eval1, 3),
            "solve_s_est": round(est, 2),
            "solve_s_est_1thread": round(est * t_eval1 / t_eval, 1),
            "solve_counts": {"evals": evals, "updates": updates},
            "time_ratio_vs_gpu": round(est / gpu_s, 1),
            "time_ratio_vs_gpu_1thread": round(est * t_eval1 / t_eval / gpu_s, 1)}


def run_single(args, name: str, S_np, with_profile: bool,
               legs=("fp64", "f64_delta", "emu", "crt")) -> dict:
    """Mixed (headline) and FP64 legs of zf_refine on one matrix, with per-kernel
    times, roofline fractions and oracle checks."""
    import torch

    from oracle import zf_oracle as O
    from paper_2404_19163_amd import zf

    n = S_np.shape[0]
    dev = torch.device("cuda:0")
    S = torch.from_numpy(S_np).to(dev)
    stream = torch.cuda.current_stream()

    def run(precision, out, refine=None):
        refine = refine or getattr(args, "refine", "crt_first")
        return zf.refine(S, None, order=args.order, precision=precision, out=out, stream=stream,
                         refine=refine)

    Zm = torch.empty_like(S)
    for _ in range(args.warmup):
        run("bf16x3", Zm)
    torch.cuda.synchronize()
    if with_profile:
        zf.profile_reset()
        zf.profile_enable(True)
    mixed_s, last = timed_solves(lambda: run("bf16x3", Zm), args.steps, 0)
    prof = {}
    if with_profile:
        zf.profile_enable(False)
        prof = zf.profile_read()
    print(f"[bench] {name} mixed: {mixed_s * 1e3:.3f} ms/step iters={last.iters} "
          f"evals={last.low_evals}+{last.high_evals} rms={last.final_rms:.3e}", file=sys.stderr,
          flush=True)
    # the same steps without the per-GEMM event pairs
    noev_s, _ = timed_solves(lambda: run("bf16x3", Zm), args.steps, 0) if with_profile else (mixed_s, None)
    evals = last.low_evals + last.high_evals
    updates = (last.low_evals - 1) + max(last.high_evals - 1, 0)
    out = {"ms": round(mixed_s * 1e3, 4), "ms_without_events": round(noev_s * 1e3, 4),
           "iters": last.iters, "low_evals": last.low_evals, "high_evals": last.high_evals,
           "final_rms": last.final_rms,
           "tflops": round(alg_flops(n, args.order, evals, updates) / mixed_s / 1e12, 3),
           "tflops_paper_count": round(paper_flops(n, args.order, evals, updates) / mixed_s / 1e12, 3)}
    res = {"n": n, "mixed": out, "prof": prof, "steps_timed": args.steps}

    if "fp64" in legs and args.fp64_steps > 0:
        Zd = torch.empty_like(S)
        fp64_s, r64 = timed_solves(lambda: run("fp64", Zd), args.fp64_steps, 1)
        updates64 = r64.high_evals - 1
        res["fp64"] = {"ms": round(fp64_s * 1e3, 3),
                       "tflops": round(alg_flops(n, args.order, r64.high_evals, updates64) / fp64_s / 1e12, 3),
                       "tflops_paper_count": round(paper_flops(n, args.order, r64.high_evals, updates64) / fp64_s / 1e12, 3),
                       "iters": r64.iters, "evals": r64.high_evals, "final_rms": r64.final_rms}
        res["Zd"] = Zd
        print(f"[bench] {name} fp64: {fp64_s * 1e3:.3f} ms/step iters={r64.iters} "
              f"rms={r64.final_rms:.3e}", file=sys.stderr, flush=True)
    # the other refinement modes of the mixed path, each timed without events
    head = getattr(args, "refine", "crt_first")
    other = {"f64_delta": "fp64 residual", "crt_first": "residue-emulated first residual",
             "crt": "residue-emulated residuals", "emu": "slice-emulated residuals"}
    for mode, what in other.items():
        if mode == head or args.fp64_steps <= 0 or (mode != "f64_delta" and n > 16384):
            continue
        if mode not in legs and not (mode in ("crt_first", "crt") and "crt" in legs):
            continue
        Zo = torch.empty_like(S)
        o_s, ro = timed_solves(lambda: run("bf16x3", Zo, mode), max(args.fp64_steps, 5), 1)
        res[mode] = {"ms": round(o_s * 1e3, 3), "evals": [ro.low_evals, ro.high_evals],
                     "final_rms": ro.final_rms, "fp64_rms": zf.residual(S, Zo),
                     "headline_speedup_over_this": round(o_s / noev_s, 3)}
        if mode == "emu":
            res[mode]["slices"] = int(os.environ.get("ZF_EMU_SLICES", "7"))
        if mode.startswith("crt"):
            res[mode]["moduli"] = int(os.environ.get("ZF_EMU_MODULI", "14"))
        print(f"[bench] {name} mixed, {what}: {o_s * 1e3:.3f} ms/step rms={ro.final_rms:.3e}",
              file=sys.stderr, flush=True)

    # residuals and distances checked by the CPU oracle
    Zm_np = Zm.cpu().numpy()
    checks = {"oracle_rms_mixed": O.residual_rms(S_np, Zm_np)}
    Zs = [Zm_np]
    if "Zd" in res:
        Zd_np = res.pop("Zd").cpu().numpy()
        checks["oracle_rms_fp64"] = O.residual_rms(S_np, Zd_np)
        checks["rel_diff_mixed_vs_fp64"] = float(np.linalg.norm(Zm_np - Zd_np) / np.linalg.norm(Zd_np))
        Zs.append(Zd_np)
    if not args.no_lowdin:
        t0 = time.perf_counter()
        errs = lowdin_error(S_np, Zs)
        checks["lowdin_rel_err_mixed"] = errs[0]
        if len(errs) > 1:
            checks["lowdin_rel_err_fp64"] = errs[1]
        checks["lowdin_eigh_s"] = round(time.perf_counter() - t0, 2)
    res["checks"] = checks
    return res


def kernel_table(prof: dict, n: int, total_s: float) -> dict:
    return {k: {"launches": v[0], "total_ms": round(v[1], 4),
                "avg_us": round(v[1] / max(v[0], 1) * 1e3, 2),
                "share": round(v[1] / max(total_s * 1e3, 1e-9), 4),
                "alg_tflops": round(kernel_alg_flops(k, n) / (v[1] / 1e3 / v[0]) / 1e12, 2),
                "exec_tflops": round(v[2] / (v[1] / 1e3) / 1e12, 2)}
            for k, v in prof.items() if v[0]}


def roofline(prof: dict, n: int, total_s: float) -> dict:
    """Dominant kernel (most time) against its dtype's peak, plus the time-weighted
    fraction of all BF16 kernels together (algorithmic and executed MFMA flops over
    their summed time) and the whole call's matrix-core fraction."""
    dom = max(prof, key=lambda k: prof[k][1])
    launches, tot_ms, _ = prof[dom]
    avg_s = tot_ms / 1e3 / max(launches, 1)
    ach = kernel_alg_flops(dom, n) / avg_s / 1e12
    peak = PEAK_TFLOPS[KCLASS_DTYPE[dom]]
    bf = {k: v for k, v in prof.items() if v[0] and KCLASS_DTYPE.get(k) == "bf16"}
    bf_s = sum(v[1] for v in bf.values()) / 1e3
    bf_alg = sum(kernel_alg_flops(k, n) * v[0] for k, v in bf.items())
    bf_exec = sum(v[2] for v in bf.values())
    mfma_s = sum(v[2] / (PEAK_TFLOPS[KCLASS_DTYPE[k]] * 1e12) for k, v in prof.items() if v[0])
    traffic, alg_bytes = measured_traffic(dom, n)
    return {"bound": "mfma", "kernel": dom, "achieved": round(ach, 2), "peak": peak,
            "unit": "TFLOP/s", "frac": round(ach / peak, 4), "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated)",
            "alg_bytes": alg_bytes,
            "bf16_kernels_frac": round(bf_alg / bf_s / 1e12 / PEAK_TFLOPS["bf16"], 4) if bf_s else None,
            "bf16_kernels_exec_frac": round(bf_exec / bf_s / 1e12 / PEAK_TFLOPS["bf16"], 4) if bf_s else None,
            "bf16_kernels_share_of_call": round(bf_s / total_s, 4),
            "whole_call_frac": round(mfma_s / total_s, 4)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gauss4096",
                    choices=sorted(WORKLOADS) + ["batched512", "md3000", "table1", "congruence"])
    ap.add_argument("--n", type=int, default=4096, help="order of the table1 workload")
    ap.add_argument("--frames", type=int, default=64, help="frames of the md3000 workload")
    ap.add_argument("--graph-sweeps", type=int, default=None,
                    help="macro-sweeps per graph launch of the batched workload (0: all)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--order", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lowdin", action="store_true",
                    help="skip the dense-eigendecomposition distance checks")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the N=4096 workload (skip the other configurations)")
    ap.add_argument("--mixed-only", action="store_true", help="skip the FP64 path (profiling runs)")
    ap.add_argument("--refine", default="crt_first",
                    choices=["f64_delta", "crt_first", "crt", "emu", "f64_full"],
                    help="refinement mode of the headline mixed path")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(args.copy_calibration << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_calibration, "launches": 3}))
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the refinement of one matrix runs on one device and "
              "the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    from paper_2404_19163_amd import inputs

    if args.workload == "batched512":
        print(json.dumps(bench_batched(args)), flush=True)
        return 0
    if args.workload == "md3000":
        print(json.dumps(bench_md(args)), flush=True)
        return 0
    if args.workload == "table1":
        return bench_table1(args)
    if args.workload == "congruence":
        return bench_congruence(args)
    if args.mixed_only:
        args.fp64_steps = 0
    wl = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    S_np = inputs.workload(args.workload, args.seed)
    n = S_np.shape[0]
    print(f"[bench] generated {args.workload} N={n} in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)

    r = run_single(args, args.workload, S_np, with_profile=True)
    mixed = r["mixed"]
    mixed_s = mixed["ms"] / 1e3
    total_s = mixed_s * r["steps_timed"]
    prof = r["prof"]
    fp64 = r.get("fp64")

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle runs the FP64 recursion: its counts are the FP64 path's (equal by
        # the parity tests), else the mixed path's
        ev = fp64["evals"] if fp64 else mixed["low_evals"] + mixed["high_evals"]
        cpu = cpu_oracle_baseline(S_np, args.order, ev, ev - 1, mixed_s, args.workload)
        if fp64:
            cpu["time_ratio_vs_gpu_fp64_path"] = round(cpu["solve_s_est"] / (fp64["ms"] / 1e3), 1)
        print(f"[bench] cpu oracle: eval {cpu['eval_s']} s, update {cpu['update_s']} s, "
              f"1-thread eval {cpu['eval_s_1thread']} s", file=sys.stderr, flush=True)

    configs = {}
    if not args.headline_only and args.workload == "gauss4096":
        configs = other_configs(args)

    line = {
        "metric": METRIC,
        "value": mixed["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3+fp64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": n, "seed": args.seed, "order": args.order,
                   "z0": "scaled identity", "stop": "ratio (Algorithm 2)",
                   "refine": REFINE_DESC[args.refine]},
        "flop_basis": "irreducible: 3 N^3 per residual evaluation (S Z and the symmetric "
                      "Z^T (S Z)), (m + 1) N^3 per update (6 N^3 per order-2 sweep); "
                      "tflops_paper_count uses 4 N^3 + 2 m N^3 (every product dense)",
        "time_to_solution_ms": mixed["ms"],
        "ms_per_step_without_events": mixed["ms_without_events"],
        "tflops_paper_count": mixed["tflops_paper_count"],
        "iters": mixed["iters"],
        "low_evals": mixed["low_evals"],
        "high_evals": mixed["high_evals"],
        "final_rms": mixed["final_rms"],
        "fp64": fp64,
        # both legs timed without per-GEMM events
        "speedup_vs_fp64": round(fp64["ms"] / mixed["ms_without_events"], 3) if fp64 else None,
        "refine_modes": {m: r[m] for m in ("f64_delta", "crt_first", "crt", "emu") if m in r},
        "checks": r["checks"],
        "kernels": kernel_table(prof, n, total_s),
        "roofline": roofline(prof, n, total_s),
        "cpu_baseline": cpu,
        "configs": configs,
    }
    print(json.dumps(line), flush=True)
    return 0


def other_configs(args) -> dict:
    """The remaining workloads in the same run, each reduced to its figures: N = 256
    FP64 (the plain method), the N = 5049 cluster (mixed and FP64), the MD warm start at
    N = 3000 and the 512-matrix batch.  Every result carries its oracle-checked RMS."""
    import torch

    from oracle import zf_oracle as O
    from paper_2404_19163_amd import inputs, zf

    out = {}
    # plain method, N = 256, FP64, both stop rules
    S_np = inputs.workload("gauss256", args.seed)
    S = torch.from_numpy(S_np).to("cuda:0")
    Z = torch.empty_like(S)
    ref = O.refine(S_np, O.scaled_identity_guess(S_np), order=2, rule="monotone")
    c1 = {"workload": WORKLOADS["gauss256"]["desc"] + ", FP64 path, 3rd-order series"}
    for rule in ("monotone", "ratio"):
        s, r = timed_solves(lambda: zf.refine(S, None, precision="fp64", stop=rule, out=Z), 100, 5)
        Zn = Z.cpu().numpy()
        c1[rule] = {"ms": round(s * 1e3, 4), "iters": r.iters, "evals": r.high_evals,
                    "final_rms": r.final_rms, "oracle_rms": O.residual_rms(S_np, Zn)}
        if rule == "monotone":
            c1[rule]["oracle_iters"] = ref.iters
            c1[rule]["rel_diff_vs_oracle"] = float(np.linalg.norm(Zn - ref.Z) / np.linalg.norm(ref.Z))
            c1[rule]["lowdin_rel_err"] = lowdin_error(S_np, [Zn])[0]
    out["gauss256_fp64"] = c1
    print(f"[bench] gauss256 fp64: {c1['monotone']['ms']} ms", file=sys.stderr, flush=True)

    # ill-conditioned cluster, N = 5049
    S_np = inputs.workload("cluster5049", args.seed)
    sub = argparse.Namespace(**vars(args))
    sub.steps, sub.warmup, sub.fp64_steps = 5, 2, 2
    r = run_single(sub, "cluster5049", S_np, with_profile=False, legs=("fp64", "f64_delta", "crt"))
    c3 = {"workload": WORKLOADS["cluster5049"]["desc"], "mixed": r["mixed"], "fp64": r.get("fp64"),
          "refine_modes": {m: r[m] for m in ("f64_delta", "crt_first", "crt") if m in r},
          "checks": r["checks"]}
    if r.get("fp64"):
        c3["speedup_vs_fp64"] = round(r["fp64"]["ms"] / r["mixed"]["ms"], 3)
    out["cluster5049"] = c3

    # MD warm start (N = 3000) and the batch
    sub = argparse.Namespace(**vars(args))
    out["md3000"] = bench_md(sub)
    sub = argparse.Namespace(**vars(args))
    sub.steps, sub.warmup = 3, 1
    out["batched512"] = bench_batched(sub)
    torch.cuda.synchronize()
    return out


def bench_table1(args) -> int:
    """The schemes of the paper's Table I on its synthetic family (Sec. V.A): S =
    sym(exp(-|i-j|/2) sin(i+1)) shifted to lowest eigenvalue 0.5, Z0 = S^(-1/2) + 0.005 U.
    Per scheme: time per solve, updates, residual evaluations, ||X - I||_2 and the RMS
    ||Z^T S Z - I||_F / sqrt(N) of the returned Z (both evaluated in FP64 outside the
    timed region)."""
    import numpy as np
    import torch

    from paper_2404_19163_amd import inputs, zf

    n = args.n
    t0 = time.perf_counter()
    S_np = inputs.paper_synthetic(n, 0.5)
    w, V = np.linalg.eigh(S_np)
    Z0_np = (V / np.sqrt(w)) @ V.T + 0.005 * inputs.uniform_noise(n, args.seed)
    print(f"[bench] synthetic S and Z0 (N={n}) in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    S = torch.from_numpy(S_np).to("cuda:0")
    Z0 = torch.from_numpy(Z0_np).to("cuda:0")
    out = torch.empty_like(S)
    eye = torch.eye(n, dtype=torch.float64, device="cuda:0")
    schemes = [("double", "fp64", "off"), ("single", "fp32", "off"),
               ("(h)(h) BF16", "bf16", "off"), ("(h)(h)+refi BF16", "bf16", "f32"),
               ("(h)(h)+(h)(l)+(l)(h) BF16", "bf16x3", "off"),
               ("(h)(h)+(h)(l)+(l)(h)+refi BF16", "bf16x3", "f64_full"),
               ("(h)(h)+(h)(l)+(l)(h)+refi(delta) BF16", "bf16x3", "f64_delta"),
               ("(h)(h) FP16", "fp16", "off"), ("(h)(h)+refi FP16", "fp16", "f32"),
               ("(h)(h)+(h)(l)+(l)(h) FP16", "fp16x3", "off"),
               ("(h)(h)+(h)(l)+(l)(h)+refi(delta) FP16", "fp16x3", "f64_delta")]
    rows = {}
    for name, prec, ref in schemes:
        for _ in range(args.warmup):
            zf.refine(S, Z0, precision=prec, refine=ref, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = None
        for _ in range(args.steps):
            r = zf.refine(S, Z0, precision=prec, refine=ref, out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        X = out.T @ (S @ out)
        e2 = float(torch.linalg.eigvalsh((X + X.T) / 2 - eye).abs().max())
        rms = float(torch.linalg.norm(X - eye)) / math.sqrt(n)
        rows[name] = {"ms": round(ms, 3), "updates": r.iters, "evals": [r.low_evals, r.high_evals],
                      "err2": e2, "rms": rms}
        print(f"[bench] {name}: {ms:.2f} ms, err2 {e2:.2e}", file=sys.stderr, flush=True)
    # context (Fig. runtime): S^(-1/2) by dense diagonalization on the GPU (torch.linalg.eigh,
    # the ROCm solver), timed the same way
    def diag():
        w_, V_ = torch.linalg.eigh(S)
        return (V_ * w_.rsqrt()) @ V_.T
    for _ in range(args.warmup):
        diag()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Zd = diag()
    torch.cuda.synchronize()
    X = Zd.T @ (S @ Zd)
    rows["diagonalization (eigh, FP64)"] = {
        "ms": round((time.perf_counter() - t0) / args.steps * 1e3, 3),
        "err2": float(torch.linalg.eigvalsh((X + X.T) / 2 - eye).abs().max())}
    line = {"metric": "Table I schemes on the paper's synthetic family: time per solve and "
                      "||Z^T S Z - I||_2", "n": n, "unit": "ms", "higher_is_better": False,
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "data": "synthetic",
            "config": {"workload": f"Sec. V.A synthetic S (gamma 0.5), N={n}, Z0 = S^-1/2 + 0.005 U",
                       "seed": args.seed},
            "schemes": rows}
    print(json.dumps(line), flush=True)
    return 0


def bench_congruence(args) -> int:
    """The consumer of Z (Sec. II.A, Eq. standard_form): H_perp = Z^T H Z for the N = 4096
    Gaussian-kernel overlap and its extended-Hueckel Hamiltonian, Z from the mixed
    refinement.  Per precision: time per transform, algorithmic TFLOP/s (4 N^3: two dense
    products), the largest deviation of H_perp's spectrum from that of the FP64 transform,
    and relative Frobenius error.  torch's FP64 Z^T (H Z) (the vendor BLAS) is timed as
    context."""
    import numpy as np
    import torch

    from paper_2404_19163_amd import inputs, zf

    S_np = inputs.workload("gauss4096", args.seed)
    H_np = inputs.huckel_hamiltonian(S_np, 100 + args.seed)
    n = S_np.shape[0]
    S = torch.from_numpy(S_np).to("cuda:0")
    H = torch.from_numpy(H_np).to("cuda:0")
    Z = zf.refine(S, None, precision="bf16x3").Z
    out = torch.empty_like(S)
    ref = zf.congruence(H, Z, precision="fp64")
    w_ref = torch.linalg.eigvalsh(ref)
    flops = 4.0 * n ** 3

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps * 1e3

    rows = {}
    for prec in ("fp64", "bf16x3", "fp16x3", "fp32", "bf16", "fp16"):
        ms = timed(lambda: zf.congruence(H, Z, precision=prec, out=out))
        w = torch.linalg.eigvalsh(out)
        rows[prec] = {"ms": round(ms, 3), "alg_tflops": round(flops / ms / 1e9, 1),
                      "eig_dev": float((w - w_ref).abs().max()),
                      "rel_fro": float(torch.linalg.norm(out - ref) / torch.linalg.norm(ref))}
        print(f"[bench] congruence {prec}: {ms:.3f} ms", file=sys.stderr, flush=True)
    ms = timed(lambda: Z.T @ (H @ Z))
    rows["torch fp64 (vendor BLAS)"] = {"ms": round(ms, 3), "alg_tflops": round(flops / ms / 1e9, 1)}
    line = {"metric": "congruence transform Z^T H Z: time per transform", "unit": "ms",
            "higher_is_better": False, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "data": "synthetic", "config": {"workload": "gauss4096 overlap + extended-Hueckel H, "
                                                        "N=4096, Z from the mixed refinement",
                                            "seed": args.seed},
            "max_abs_eig": float(w_ref.abs().max()), "precisions": rows}
    print(json.dumps(line), flush=True)
    return 0


def bench_md(args) -> dict:
    """MD-like warm start: frames of the N = 3000 Gaussian-kernel system with positions
    random-walking by N(0, 0.01 A) per coordinate; each frame refined from (a) the
    previous frame's Z, (b) the learned guess, (c) the scaled identity.  The network
    is trained on the first 16 frames (labels from their refined Z) and evaluated on
    the rest; reported per strategy: mean updates and ms per frame.  Every frame's
    refinement phase takes the bench's --refine (default: first residual from
    residues, final residual in FP64), as the single-matrix legs do."""
    import numpy as np
    import torch

    from paper_2404_19163_amd import guess, inputs, zf

    frames = args.frames
    n = 3000
    t0 = time.perf_counter()
    mats = list(inputs.md_trajectory(n, frames, args.seed))
    print(f"[bench] generated {frames} frames in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    S = [torch.from_numpy(m).to("cuda:0") for m in mats]
    ntrain = min(16, frames // 4)
    X, Y = guess.training_pairs(mats[:ntrain], precision="bf16x3")
    losses, _ = guess.train(X, Y, steps=300, lr=3e-3, seed=args.seed)
    stats = {"warm": [], "learned": [], "identity": []}
    Z = torch.empty_like(S[0])
    rf = args.refine
    prev = zf.refine(S[ntrain - 1], None, refine=rf).Z.clone()
    for f in range(ntrain, frames):
        for kind in ("warm", "learned", "identity"):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if kind == "warm":
                r = zf.refine(S[f], prev, out=Z, refine=rf)
            elif kind == "learned":
                r = zf.refine(S[f], None, out=Z, guess="learned", refine=rf)
            else:
                r = zf.refine(S[f], None, out=Z, refine=rf)
            torch.cuda.synchronize()
            stats[kind].append((time.perf_counter() - t1, r.iters, r.low_evals, r.high_evals,
                                r.final_rms, getattr(r, "z0_used", -1)))
            if kind == "warm":
                prev = Z.clone()
    summary = {}
    for kind, v in stats.items():
        a = np.array([x[:5] for x in v])
        summary[kind] = {"ms_per_frame": round(float(a[:, 0].mean()) * 1e3, 3),
                         "mean_updates": round(float(a[:, 1].mean()), 3),
                         "mean_low_evals": round(float(a[:, 2].mean()), 3),
                         "mean_fp64_evals": round(float(a[:, 3].mean()), 3),
                         "worst_rms": float(a[:, 4].max())}
    summary["learned"]["accepted"] = int(sum(1 for x in stats["learned"] if x[5] == 2))
    line = {
        "metric": METRIC + " (MD warm start)",
        "value": summary["warm"]["ms_per_frame"], "unit": "ms per frame (warm start)",
        "higher_is_better": False, "n_gpus": 1, "steps": frames - ntrain, "warmup": ntrain,
        "dtype": "bf16x3+fp64", "data": "synthetic",
        "config": {"workload": f"{frames} frames of the N=3000 Gaussian-kernel system (sigma 1.0 A), "
                               "positions random-walking by N(0, 0.01 A) per coordinate",
                   "network": f"trained on frames 0..{ntrain - 1} ({len(losses)} Adam steps, "
                              f"loss {losses[0]:.3g} -> {losses[-1]:.3g})",
                   "refine": REFINE_DESC[rf]},
        "strategies": summary,
    }
    return line


def bench_batched(args) -> dict:
    """512 Gaussian-kernel overlaps, N log-uniform in [64, 1024], condition number
    log-uniform in [10, 1e4], refined in one zf_refine_batched call per step.  Matrices
    start from the learned guess (per-matrix acceptance, scaled-identity fallback); the
    network is trained beforehand on 128 other matrices of the same distribution.  The
    scaled-identity start is timed beside it."""
    import numpy as np
    import torch

    from paper_2404_19163_amd import guess, inputs, zf

    count = 512
    t0 = time.perf_counter()
    mats = inputs.batched_overlaps(count, args.seed)
    train_mats = inputs.batched_overlaps(128, args.seed + 1000)
    print(f"[bench] generated {count} + 128 matrices in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    X, Y = guess.training_pairs(train_mats)
    losses, _ = guess.train(X, Y, steps=400, lr=3e-3, seed=0)
    print(f"[bench] trained the guess network in {time.perf_counter() - t0:.1f}s "
          f"(loss {losses[0]:.3g} -> {losses[-1]:.3g})", file=sys.stderr, flush=True)
    S = [torch.from_numpy(m).to("cuda:0") for m in mats]
    out = [torch.empty_like(s) for s in S]
    ns = [m.shape[0] for m in mats]
    if getattr(args, "graph_sweeps", None) is not None:
        zf.batched_set_graph_sweeps(args.graph_sweeps)

    def leg(kind):
        for _ in range(args.warmup):
            zf.refine_batched(S, out=out, guess=kind)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = None
        for _ in range(args.steps):
            last = zf.refine_batched(S, out=out, guess=kind)
        torch.cuda.synchronize()
        step_s = (time.perf_counter() - t0) / args.steps
        # the method's irreducible flops, plus the symmetric S^2 of each learned guess
        flops = sum(alg_flops(n, 2, r.low_evals + r.high_evals,
                              (r.low_evals - 1) + max(r.high_evals - 1, 0))
                    + (float(n) ** 3 if r.z0_used == zf.Z0_LEARNED else 0.0)
                    for n, r in zip(ns, last.results))
        print(f"[bench] {kind}: {step_s * 1e3:.2f} ms per batch", file=sys.stderr, flush=True)
        return step_s, flops, last

    step_s, flops, last = leg("learned")
    sweeps, launches = zf.batched_last_stats()
    worst = max(r.final_rms for r in last.results)
    from oracle import zf_oracle as O
    idx = sorted(set(np.linspace(0, count - 1, 8).astype(int).tolist()))
    oracle_rms = {int(ns[i]): O.residual_rms(mats[i], out[i].cpu().numpy()) for i in idx}
    id_s, id_flops, id_last = leg("identity")
    line = {
        "metric": METRIC + " (batched)",
        "value": round(flops / step_s / 1e12, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3+fp64", "data": "synthetic",
        "config": {"workload": f"{count} Gaussian-kernel overlaps, N log-uniform in [64, 1024], "
                               "condition number log-uniform in [10, 1e4], learned Z0 with "
                               "scaled-identity fallback, one grouped-GEMM graph",
                   "seed": args.seed, "tiles": zf.batched_get_tiles(),
                   "network": f"trained on 128 matrices of the same distribution (seed "
                              f"{args.seed + 1000}), 400 Adam steps, loss {losses[0]:.3g} -> "
                              f"{losses[-1]:.3g}"},
        "worst_final_rms": worst,
        "graph": {"macro_sweeps": sweeps, "graph_launches": launches,
                  "host_syncs": launches + 1},
        "mean_iters": float(np.mean([r.iters for r in last.results])),
        "mean_low_evals": float(np.mean([r.low_evals for r in last.results])),
        "learned_accepted": int(sum(r.z0_used == zf.Z0_LEARNED for r in last.results)),
        "oracle_rms_sample": oracle_rms,
        "scaled_identity": {"ms_per_step": round(id_s * 1e3, 3),
                            "tflops": round(id_flops / id_s / 1e12, 3),
                            "mean_iters": float(np.mean([r.iters for r in id_last.results])),
                            "mean_low_evals": float(np.mean([r.low_evals for r in id_last.results])),
                            "worst_final_rms": max(r.final_rms for r in id_last.results)},
    }
    return line


if __name__ == "__main__":
    sys.exit(main())
