#!/usr/bin/env python3
"""LM step solves per second on one MI355X for the block-angular scale workload.

Workload: J = [blkdiag(A_1..A_50000) | B], A_i 12x3, B 600,000 x 90, b 600,000,
entries N(0,1) with column scales 10^(3t) (cond(J) ~ 1e3), float32 values, D = diag of
the column norms, lambda = 1e-2.  One step = factor (per-block Householder QR with
Q_i^T applied to B and b, tall-skinny QR of the reduced rows) + solve (structured
back-substitution) + the float64-residual refinement sweeps needed to reach a
relative error <= 1e-10 against the float64 oracle.  Inputs are resident in HBM
before the timed region; the whole step runs in libqrkit.so's HIP kernels.

Prints one JSON line.  `python bench.py` runs on one GPU; --gpus above 1 is refused
(the library and this benchmark run on a single GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "LM step solves/sec, mixed+refined vs plain FP32 at rel err ≤1e-10 vs FP64"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6

# HBM bytes per launch of a phase's kernels, from two rocprofv3 PMC runs of this script
# (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, factors read off a 256 MiB device copy), and the
# matrix-core work of the same launches (SQ_INSTS_VALU_MFMA_MOPS_BF16 / _F32 x 512 flops, and
# SQ_VALU_MFMA_BUSY_CYCLES per SIMD); runs and figures in
# profiles/blockangular_scale_pmc_counters.md.  The dense-part phase is the leaf launch plus the
# merge-tree launch.  A figure holds only for the workload it was taken on and while the
# kernels' sources hash to the recorded digest.
_TSQR_SOURCES = ["paper_1802_03773_amd/csrc/tsqr_mfma.hpp", "paper_1802_03773_amd/csrc/tsqr_mfma.hip",
                 "paper_1802_03773_amd/csrc/tsqr_mfma_ncb6.hip", "paper_1802_03773_amd/csrc/qrk_device.hpp",
                 "paper_1802_03773_amd/csrc/tsqr_tree.hpp", "paper_1802_03773_amd/csrc/tsqr_tree.hip",
                 "paper_1802_03773_amd/csrc/qrk_layout.hpp",  # the reduced-row stride
                 "paper_1802_03773_amd/csrc/qrk_batch.hpp"]   # the batch layout the kernels read
_TSQR_DIGEST = "d6ab8199b786af42fb6027b0c8fd74a2ee83f9236ca8f51e6c29066056fe1bb5"
MEASURED_TRAFFIC = {
    ("dense_leaves", "bf16x3"): {"bytes": (114471.7 * 2.000 + 21504.0 + 22583.3 * 2.000 + 21845.7) * 1024.0,
                                 "lam": 1e-2, "sources": _TSQR_SOURCES, "sha256": _TSQR_DIGEST},
    ("dense_leaves", "plain"): {"bytes": (114305.9 * 2.000 + 21504.0 + 22576.1 * 2.000 + 21845.8) * 1024.0,
                                "lam": 1e-2, "sources": _TSQR_SOURCES, "sha256": _TSQR_DIGEST},
}
# matrix-core flops per launch (leaves + tree) and the SIMDs' matrix-core busy cycles per launch
MEASURED_MFMA = {
    ("dense_leaves", "bf16x3"): {"bf16_flops": 88473600.0 * 512, "f32_flops": (1228800.0 + 1391280.0) * 512,
                                 "busy_cycles_per_simd": (54067200.0 + 11130240.0) / 1024.0,
                                 "lam": 1e-2, "sources": _TSQR_SOURCES, "sha256": _TSQR_DIGEST},
    ("dense_leaves", "plain"): {"bf16_flops": 0.0, "f32_flops": (20889600.0 + 1391280.0) * 512,
                                "busy_cycles_per_simd": (167116800.0 + 11130240.0) / 1024.0,
                                "lam": 1e-2, "sources": _TSQR_SOURCES, "sha256": _TSQR_DIGEST},
}
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_FP32_MFMA_TFLOPS = 157.3
CLOCK_GHZ = 2.4


def _sources_match(rec):
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for src in rec["sources"]:
        path = os.path.join(root, src)
        if not os.path.exists(path):
            return False
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest() == rec["sha256"]


def measured_mfma(phase, lam, mode, avg_ms):
    """Matrix-core utilisation of `phase` at this run's duration, if a PMC figure matches."""
    rec = MEASURED_MFMA.get((phase, mode))
    if rec is None or rec["lam"] != lam or not _sources_match(rec):
        return None
    sec = avg_ms * 1e-3
    bf = rec["bf16_flops"] / sec / 1e12
    f32 = rec["f32_flops"] / sec / 1e12
    return {"bf16_tflops": bf, "bf16_peak": PEAK_BF16_MFMA_TFLOPS, "bf16_frac": bf / PEAK_BF16_MFMA_TFLOPS,
            "f32_tflops": f32, "f32_peak": PEAK_FP32_MFMA_TFLOPS, "f32_frac": f32 / PEAK_FP32_MFMA_TFLOPS,
            "busy_frac": rec["busy_cycles_per_simd"] / (sec * CLOCK_GHZ * 1e9),
            "flops_basis": "SQ_INSTS_VALU_MFMA_MOPS_* x 512 per launch (leaves + tree)"}


def measured_traffic(phase, lam, mode):
    """Bytes per launch for `phase` if a PMC figure matches this workload and these sources."""
    rec = MEASURED_TRAFFIC.get((phase, mode))
    if rec is None or rec["lam"] != lam:
        return None
    return rec["bytes"] if _sources_match(rec) else None


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--lam", type=float, default=1e-2)
    ap.add_argument("--seed", type=int, default=100)
    ap.add_argument("--sweeps", type=int, default=-1, help="-1: smallest count reaching 1e-10")
    ap.add_argument("--mode", default="auto", choices=["auto", "plain", "bf16x3"],
                    help="factor mode of the refined step; auto measures both and reports the faster")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (cpu_baseline) leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for PMC byte scaling)")
    ap.add_argument("--workload", default="scale",
                    choices=["scale", "ragged-batch", "banded-batch", "lm-scale", "lm-banded-batch", "lambda-retry",
                             "new-rhs", "configs", "camera"],
                    help="scale: one block-angular problem (the headline); ragged-batch: 512 block-angular "
                         "problems in one batch; banded-batch: 2,048 banded problems in one batch")
    ap.add_argument("--problems", type=int, default=0, help="batch workloads: problems (0 = the recipe's count)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="block-angular workloads: skip the library's autotuner (leaf height, leaf queue, "
                         "refinement workgroups) and run the default launch shape")
    ap.add_argument("--banded-method", default="auto", choices=["auto", "givens", "blockwy", "blockwy-bf16x3"],
                    help="banded-batch: factorisation (Givens rotations or the block-banded compact-WY steps); "
                         "auto times every method and reports the fastest")
    return ap.parse_args()


def _cpu_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        n = [int(i.get("num_threads", 1)) for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return max(n)
    except Exception:
        pass
    return len(os.sched_getaffinity(0))


def _blas_build() -> str:
    """NumPy version and the BLAS it was built against (numpy.show_config)."""
    import numpy as np
    try:
        cfg = np.show_config(mode="dicts")
        blas = cfg.get("Build Dependencies", {}).get("blas", {})
        return "numpy %s, %s %s" % (np.__version__, blas.get("name", "?"), blas.get("version", "?"))
    except Exception:
        return "numpy %s" % np.__version__


def algorithmic_work(inst):
    """Per-phase algorithmic bytes / flops of one step: what the method must move or compute
    (inputs read once, factor and solution written once; scratch and re-reads excluded)."""
    K, n, nB, M = inst.K, inst.n, inst.nB, inst.M
    L = nB + 1
    N = K * n + nB
    es = inst.A.dtype.itemsize
    rows = M + nB
    blk_in = M * n * es + M * nB * es + M * es + N * 8 + (K + 1) * 8
    blk_out = K * n * n * es + K * n * L * es + M * L * es
    leaf_flops = 2.0 * rows * L * L - (2.0 / 3.0) * L ** 3
    backsub_bytes = K * n * L * es + K * n * n * es + N * 8 + L * L * es
    sweep_bytes = (M * n * es + M * nB * es + M * es + N * 8 + (K + 1) * 8   # J, b, d, offsets (per sweep)
                   + 2 * N * 8 + K * n * n * es * 2 + K * n * L * es * 2      # p in/out, R_i, S twice
                   + 2 * K * n * 8)                                           # y out/in
    return dict(block_qr=("hbm", blk_in + blk_out, K),
                dense_leaves=("alu", leaf_flops, rows),
                backsub=("hbm", backsub_bytes, K),
                refine=("hbm", sweep_bytes, K))


def run_batch(args):
    """Batch workloads: every problem of the batch is one LM step solve (factor + solve + the
    fewest float64 sweeps reaching 1e-10 on the sampled problems), all problems in the same
    launches."""
    import numpy as np
    import torch

    from paper_1802_03773_amd import BandedSolver, BlockAngularBatch
    from workloads import generators as gen

    ragged = args.workload == "ragged-batch"
    P = args.problems or (512 if ragged else 2048)
    print(f"[bench] generating {args.workload} ({P} problems)", file=sys.stderr, flush=True)
    if ragged:
        insts = gen.ragged_batch(200, P=P, lam=args.lam)
        st = gen.stack_batch(insts)
        dev = {k: torch.from_numpy(np.ascontiguousarray(st[k])).cuda() for k in ("A", "B", "b", "d", "lam")}
        N_p = [i.N for i in insts]
        rows = int(st["row_off"][-1])
        # BF16x3 trailing updates are the faster factor on this batch (auto picks them)
        mode = "bf16x3" if args.mode == "auto" else args.mode
        solver = BlockAngularBatch(st["K"], st["nB"], st["row_off"], st["n"], dtype="float32", mode=mode)

        def factor():
            solver.factor(dev["A"], dev["B"], dev["b"], dev["d"], dev["lam"])
        desc = {"workload": "ragged block-angular batch: %d problems, K_p ~ U{500..8000} blocks of m_i x 3 "
                            "(m_i ~ U{4,6,..,40}), dense parts n_B ~ U{6,30,90}, float32, lambda = %g" % (P, args.lam),
                "problems": P, "blocks": int(st["K"].sum()), "rows": rows, "unknowns": int(sum(N_p)), "mode": mode}
    else:
        insts = gen.banded_batch(300, P=P, lam=args.lam)
        i0 = insts[0]
        dev = {"rs": torch.from_numpy(np.stack([i.row_start for i in insts])).cuda(),
               "vals": torch.from_numpy(np.stack([i.vals for i in insts])).cuda(),
               "b": torch.from_numpy(np.stack([i.b for i in insts])).cuda(),
               "d": torch.from_numpy(np.stack([i.d for i in insts])).cuda()}
        N_p = [i.N for i in insts]
        mode = "plain"
        solver = BandedSolver(i0.M, i0.N, i0.w, dtype="float32", P=P)
        methods = (["givens", "blockwy", "blockwy-bf16x3"] if args.banded_method == "auto"
                   else [args.banded_method])

        def factor():
            solver.factor(dev["rs"], dev["vals"], dev["b"], dev["d"], args.lam)
        desc = {"workload": "banded batch: %d problems of n = %d unknowns, %d rows, %d values per row, float32, "
                            "lambda = %g" % (P, i0.N, i0.M, i0.w, args.lam),
                "problems": P, "rows": P * i0.M, "unknowns": P * i0.N, "band_values": i0.w}
    p = torch.empty(sum(N_p), dtype=torch.float64, device="cuda")
    offs = np.concatenate([[0], np.cumsum(N_p)])

    def step(sweeps):
        factor()
        solver.solve(sweeps=sweeps, out=p)

    sample = sorted({0, P // 2, P - 1})
    errors, cpu_baseline = {}, None
    if not args.no_cpu:
        from oracle import banded as obanded
        from oracle import refine, structured
        print(f"[bench] oracle on problems {sample}", file=sys.stderr, flush=True)
        refs, t_cpu = {}, 0.0
        for q in sample:
            t0 = time.perf_counter()
            if ragged:
                p0, fac = structured.solve_blockangular(insts[q])
                t_cpu += time.perf_counter() - t0
                refs[q] = refine.refine(insts[q], fac, p0, sweeps=2).astype(np.float64)
            else:
                R, c, _ = obanded.factor_lapack(insts[q])
                import scipy.linalg
                scipy.linalg.solve_triangular(R, c, lower=False)
                t_cpu += time.perf_counter() - t0
                refs[q] = obanded.reference_solution(insts[q])[0]
        cpu_baseline = {"value": len(sample) / t_cpu, "unit": "steps/s", "cores": _cpu_threads(), "kind": "oracle",
                        "sample": "float64 oracle solves of problems %s of the batch (%s), %.2f s" % (
                            sample, "structured LAPACK per block and dense part" if ragged else
                            "LAPACK QR of the assembled band", t_cpu)}

    def measure_errors():
        errs = {}
        if refs_ok:
            for s_ in range(0, 4):
                step(s_)
                torch.cuda.synchronize()
                x = p.cpu().numpy()
                errs[s_] = max(float(np.linalg.norm(x[offs[q]:offs[q + 1]] - refs[q]) / np.linalg.norm(refs[q]))
                               for q in sample)
        st_ = solver.status()
        if st_[0] != 0:
            raise RuntimeError(f"device status {st_}")
        if args.sweeps >= 0:
            sw = args.sweeps
        elif errs:
            ok = [s_ for s_ in sorted(errs) if errs[s_] <= 1e-10]
            sw = ok[0] if ok else 3
        else:
            sw = 1
        return errs, sw

    def time_steps(sw):
        for _ in range(args.warmup):
            step(sw)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(args.steps):
            step(sw)
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / args.steps

    refs_ok = not args.no_cpu
    method_rows = None
    if ragged and not args.no_autotune:
        from paper_1802_03773_amd import qrkit
        factor()
        solver.autotune()
        desc["autotune"] = qrkit.tune_choice(solver)
        print(f"[bench] autotune: {desc['autotune']}", file=sys.stderr, flush=True)
    if not ragged:
        # every banded method: its errors, sweep count and step time; the fastest is reported
        method_rows = {}
        for meth in methods:
            solver.set_method(meth)
            errs_m, sw_m = measure_errors()
            ms_m = time_steps(sw_m)
            method_rows[meth] = {"ms_per_step": ms_m, "value": P * 1000.0 / ms_m, "refine_sweeps": sw_m,
                                 "max_rel_err_sampled": errs_m.get(sw_m), "by_sweeps": errs_m}
            print(f"[bench] banded {meth}: {ms_m:.3f} ms per batched step ({sw_m} sweeps)", file=sys.stderr,
                  flush=True)
        best = min(method_rows, key=lambda k: method_rows[k]["ms_per_step"])
        solver.set_method(best)
        desc["method"] = best
        mode = "bf16x3" if best.endswith("bf16x3") else "plain"
    errors, sweeps = measure_errors()
    for _ in range(args.warmup):
        step(sweeps)
    torch.cuda.synchronize()
    # the per-phase HIP events in one timed loop, the step rate in another without them
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    solver.profile_enable(args.steps + 1)
    e0.record()
    for _ in range(args.steps):
        step(sweeps)
    e1.record()
    torch.cuda.synchronize()
    ms_prof = e0.elapsed_time(e1) / args.steps
    phases = solver.profile_read()
    solver.profile_enable(0)
    e0.record()
    for _ in range(args.steps):
        step(sweeps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    phase_out = {k: {"avg_ms": v[0] / v[1], "launches": v[1]} for k, v in phases.items() if v[1]}
    dominant = max(phase_out, key=lambda k: phases[k][0])
    if ragged:
        # the single-problem per-phase work, summed over the batch's problems
        work = {}
        for i in insts:
            for k, (bound, amount, _units) in algorithmic_work(i).items():
                prev = work.get(k)
                work[k] = (bound, amount + (prev[1] if prev else 0.0))
        work = {k: ((b_, a_, PEAK_FP32_VECTOR_TFLOPS, "TFLOP/s", 1e12) if b_ == "alu" else
                    (b_, a_, PEAK_HBM_GBS, "GB/s", 1e9)) for k, (b_, a_) in work.items()}
    else:
        # banded factor: J, b, d in; R (N x w) and c out.  One refinement sweep: J, row starts,
        # b, d, p in; R read by both triangular solves; p out
        fbytes = sum(i.M * i.w * 4 + i.M * 4 + i.M * 4 + i.N * 8 + i.N * i.w * 4 + i.N * 4 for i in insts)
        rbytes = sum(i.M * i.w * 4 + i.M * 4 + i.M * 4 + i.N * 8 + i.N * 8 + 2 * i.N * i.w * 4 + i.N * 8
                     for i in insts)
        work = {"banded": ("hbm", fbytes, PEAK_HBM_GBS, "GB/s", 1e9),
                "refine": ("hbm", rbytes, PEAK_HBM_GBS, "GB/s", 1e9)}
    for k, (bound, amount, peak, unit, scale) in work.items():
        if k in phase_out:
            amount = amount * (sweeps if k == "refine" else 1)  # one refine record per solve
            ach = amount / (phase_out[k]["avg_ms"] * 1e-3) / scale
            phase_out[k].update(bound=bound, achieved=ach, peak=peak, unit=unit, frac=ach / peak)
    dom = phase_out[dominant]
    roofline = {"kernel": dominant, "bound": dom.get("bound"), "achieved": dom.get("achieved"),
                "peak": dom.get("peak"), "unit": dom.get("unit"), "frac": dom.get("frac"), "traffic": None}
    desc.update(refine_sweeps=sweeps, refine_dtype="f64")
    out = {"metric": METRIC, "value": P * 1000.0 / ms, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "ms_per_step_with_phase_events": ms_prof,
           "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if mode == "plain" else "bf16x3", "data": "synthetic",
           "config": desc, "accuracy": {"max_rel_err_sampled": errors.get(sweeps), "by_sweeps": errors,
                                        "sampled_problems": sample},
           "roofline": roofline, "phases": phase_out, "cpu_baseline": cpu_baseline}
    if method_rows is not None:
        out["methods"] = method_rows
    print(json.dumps(out))
    return 0


def run_lm(args):
    """Device-side Backtrack-LM iterations replayed from one captured HIP graph: every LM
    iteration of every problem is one LM step solve (model evaluation, structured factor,
    solve with float64 refinement, gain ratio and damping update, all on the device)."""
    import numpy as np
    import torch

    from oracle import lm as olm
    from paper_1802_03773_amd import BandedSolver, BlockAngularSolver, LMDriver
    from workloads import generators as gen

    banded = args.workload == "lm-banded-batch"
    c, sweeps = 0.1, 1
    check_iters = 5 if banded else 2
    P = (args.problems or 2048) if banded else 1
    print(f"[bench] generating {args.workload} ({P} problems)", file=sys.stderr, flush=True)
    if banded:
        probs = [gen.lm_banded(320 + k, N=2048, w=12, c=c)[:3] for k in range(P)]
        i0 = probs[0][0]
        solver = BandedSolver(i0.M, i0.N, i0.w, dtype="float32", P=P)
        # the block-banded compact-WY factor is the faster one on this batch (auto picks it)
        solver.set_method("blockwy-bf16x3" if args.banded_method == "auto" else args.banded_method)
        A0 = torch.from_numpy(np.concatenate([q[0].row_start for q in probs]).astype(np.int32)).cuda()
        B0 = torch.from_numpy(np.concatenate([q[0].vals for q in probs])).cuda()
        desc = {"workload": "LM on a banded batch: %d problems of n = %d unknowns, %d rows, %d values per row, "
                            "f(x) = J0 (x + %g x^3) - y, float32 factor, %d float64 sweep" % (P, i0.N, i0.M, i0.w, c, sweeps),
                "problems": P, "rows": P * i0.M, "unknowns": P * i0.N, "method": solver.method}
    else:
        probs = [gen.lm_blockangular(310, K=50_000, m=12, n=3, nB=90, c=c)[:3]]
        i0 = probs[0][0]
        # the BF16x3 trailing updates are the faster factor here (auto picks them)
        mode = "plain" if args.mode == "plain" else "bf16x3"
        solver = BlockAngularSolver(i0.row_off, i0.n, i0.nB, dtype="float32", mode=mode)
        A0 = torch.from_numpy(i0.A).cuda()
        B0 = torch.from_numpy(i0.B).cuda()
        desc = {"workload": "LM on one block-angular problem: 50,000 blocks of 12x3 + dense 600,000x90, "
                            "f(x) = J0 (x + %g x^3) - y, float32 factor (%s), %d float64 sweep" % (c, mode, sweeps),
                "problems": 1, "rows": i0.M, "unknowns": i0.N, "mode": mode}
    y = torch.from_numpy(np.concatenate([q[1] for q in probs]).astype(np.float32)).cuda()
    x0 = torch.from_numpy(np.concatenate([q[2] for q in probs])).cuda()
    lam0 = torch.full((P,), 1e-2, dtype=torch.float64, device="cuda")
    drv = LMDriver(solver, A0, B0, y, c, sweeps=sweeps, max_log=check_iters)

    # agreement with the LM oracle over the first iterations (sampled problems)
    drv.reset(x0, lam0)
    drv.run(check_iters)
    _, _, lg, _ = drv.get()
    lg = lg.cpu().numpy()
    sample = sorted({0, P // 2, P - 1})
    errors, cpu_baseline = None, None
    if not args.no_cpu:
        worst, flips, t_cpu = 0.0, 0, 0.0
        for q in sample:
            inst0, yq, x0q = probs[q]
            model = (olm.BandedModel(inst0, yq.astype(np.float64), c) if banded else
                     olm.BlockAngularModel(inst0, yq.astype(np.float64), c))
            t0 = time.perf_counter()
            _, _, lgo = (olm.bd_lm if banded else olm.ba_lm)(model, x0q, 1e-2, check_iters, store=np.float32)
            t_cpu += time.perf_counter() - t0
            F = lg[:, q, 0]
            worst = max(worst, float(np.max(np.abs(F - lgo[:, 0]) / np.abs(lgo[:, 0]))))
            flips += int(np.sum(lg[:, q, 3] != lgo[:, 3]))
        errors = {"max_rel_err_F_first_%d_iterations" % check_iters: worst,
                  "accept_decisions_differing": flips, "sampled_problems": sample}
        cpu_baseline = {"value": len(sample) * check_iters / t_cpu, "unit": "steps/s", "cores": _cpu_threads(),
                        "kind": "oracle", "sample": "%d Backtrack-LM iterations of problems %s with the float64 "
                        "oracle step (float32-rounded J), %.2f s" % (check_iters, sample, t_cpu)}

    # per-phase timing from eager iterations (profiling is off inside a graph)
    drv.reset(x0, lam0)
    drv.run(1)
    solver.profile_enable(64)
    drv.run(3)
    torch.cuda.synchronize()
    phases = solver.profile_read()
    solver.profile_enable(0)

    drv.reset(x0, lam0)
    drv.run(args.warmup, graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    drv.run(args.steps, graph=True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps

    phase_out = {k: {"avg_ms": v[0] / v[1], "launches": v[1]} for k, v in phases.items() if v[1]}
    if banded:
        ins = [q[0] for q in probs]
        fb = sum(i.M * i.w * 4 + i.M * 4 + i.M * 4 + i.N * 8 + i.N * i.w * 4 + i.N * 4 for i in ins)
        rb = sum(i.M * i.w * 4 + i.M * 4 + i.M * 4 + i.N * 8 + i.N * 8 + 2 * i.N * i.w * 4 + i.N * 8 for i in ins)
        work = {"banded": ("hbm", fb, PEAK_HBM_GBS, "GB/s", 1e9), "refine": ("hbm", rb, PEAK_HBM_GBS, "GB/s", 1e9)}
    else:
        wk = algorithmic_work(i0)
        work = {k: (b_, a_, PEAK_FP32_VECTOR_TFLOPS if b_ == "alu" else PEAK_HBM_GBS,
                    "TFLOP/s" if b_ == "alu" else "GB/s", 1e12 if b_ == "alu" else 1e9)
                for k, (b_, a_, _u) in wk.items()}
    for k, (bound, amount, peak, unit, scale) in work.items():
        if k in phase_out:
            amount = amount * (sweeps if k == "refine" else 1)
            ach = amount / (phase_out[k]["avg_ms"] * 1e-3) / scale
            phase_out[k].update(bound=bound, achieved=ach, peak=peak, unit=unit, frac=ach / peak)
    dominant = max(phase_out, key=lambda k: phase_out[k]["avg_ms"]) if phase_out else None
    dom = phase_out.get(dominant, {})
    roofline = {"kernel": dominant, "bound": dom.get("bound"), "achieved": dom.get("achieved"),
                "peak": dom.get("peak"), "unit": dom.get("unit"), "frac": dom.get("frac"), "traffic": None}
    desc.update(refine_sweeps=sweeps, refine_dtype="f64", graph=True)
    out = {"metric": METRIC, "value": P * 1000.0 / ms, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16x3" if desc.get("mode") == "bf16x3" else "f32", "data": "synthetic",
           "config": desc, "accuracy": errors, "roofline": roofline, "phases": phase_out, "cpu_baseline": cpu_baseline}
    print(json.dumps(out))
    return 0


def run_lambda(args):
    """Damping retries with Moré's two-stage factor (Section 5.2): J of the 50,000-block workload is
    factored once (lambda = 0, untimed); every timed step is one LM step solve at a new lambda:
    the structured QR of [R; sqrt(lambda) D] (qrk_factor_lambda) and the solve with one float64
    sweep against the original J."""
    import dataclasses

    import numpy as np
    import torch

    from paper_1802_03773_amd import BlockAngularSolver
    from workloads import generators as gen

    # BF16x3 trailing updates are the faster factor here too (auto picks them)
    mode = "bf16x3" if args.mode == "auto" else args.mode
    lams = [1e-2, 1e-3, 1e-1, 1e-4]
    print("[bench] generating workload", file=sys.stderr, flush=True)
    inst = gen.scale_blockangular(args.seed, lam=0.0)
    A, B, b, d = (torch.from_numpy(x).cuda() for x in (inst.A, inst.B, inst.b, inst.d))
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32", mode=mode)
    s.factor(A, B, b, d, 0.0)
    p = torch.empty(inst.N, dtype=torch.float64, device="cuda")

    def step(k):
        s.factor_lambda(lams[k % len(lams)])
        s.solve(sweeps=1, out=p)

    for k in range(max(args.warmup, 1)):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # the same step with the direct factor of [J; sqrt(lambda) D], for comparison
    t0 = time.perf_counter()
    for k in range(args.steps):
        s.factor(A, B, b, d, lams[k % len(lams)])
        s.solve(sweeps=1, out=p)
    torch.cuda.synchronize()
    ms_direct = (time.perf_counter() - t0) * 1e3 / args.steps
    s.factor(A, B, b, d, 0.0)

    accuracy, cpu_baseline = None, None
    if not args.no_cpu:
        from oracle import refine, structured
        lam = lams[0]
        s.factor_lambda(lam)
        pg = s.solve(sweeps=1).cpu().numpy()
        s.raise_on_status()
        inst_l = dataclasses.replace(inst, lam=lam)
        print("[bench] oracle (cpu_baseline leg)", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        f2 = structured.factor_two_stage(inst, lam)
        p0 = structured.solve_factor(f2)
        t_oracle = time.perf_counter() - t0
        p_ref = refine.refine(inst_l, structured.factor_blockangular(inst_l), p0, sweeps=2)
        accuracy = {"max_rel_err": float(np.linalg.norm(pg - p_ref) / np.linalg.norm(p_ref)), "lambda": lam}
        cpu_baseline = {"value": 1.0 / t_oracle, "unit": "steps/s", "cores": _cpu_threads(), "kind": "oracle",
                        "sample": "one two-stage float64 oracle step of the full workload (structured QR of J, "
                                  "then of [R; sqrt(lambda) D], back-substitution); %.2f s" % t_oracle}
    out = {"metric": METRIC, "value": 1000.0 / ms, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if mode == "plain" else "bf16x3", "data": "synthetic",
           "config": {"workload": "damping retries with the two-stage factor: 50,000 blocks of 12x3 + dense "
                                  "600,000x90, J factored once, each step [R; sqrt(lambda) D] + solve with one "
                                  "float64 sweep", "lambdas": lams, "refine_sweeps": 1, "refine_dtype": "f64"},
           "direct_ms_per_step": ms_direct, "accuracy": accuracy, "roofline": None,
           "cpu_baseline": cpu_baseline}
    print(json.dumps(out))
    return 0


def run_new_rhs(args):
    """New right-hand sides with the kept factor of the 50,000-block workload (Sections 5.1 and 5.2):
    J is factored once with the stored Q (untimed); every timed step solves for the next of four
    right-hand sides: Q^T b from the stored reflectors, the back-substitution and one float64
    sweep (qrk_solve_qt).  For comparison, the same right-hand sides by corrected semi-normal
    sweeps from p = 0 with J and R only (qrk_solve_rhs, four sweeps, the count that reaches 1e-10
    without Q), and the cost of storing Q in the factor call."""
    import dataclasses

    import numpy as np
    import torch

    from paper_1802_03773_amd import BlockAngularSolver
    from workloads import generators as gen

    mode = "bf16x3" if args.mode == "auto" else args.mode
    print("[bench] generating workload", file=sys.stderr, flush=True)
    inst = gen.scale_blockangular(args.seed, lam=1e-2)
    A, B, b, d = (torch.from_numpy(x).cuda() for x in (inst.A, inst.B, inst.b, inst.d))
    rng = np.random.default_rng(args.seed + 1)
    rhs = [torch.from_numpy(rng.standard_normal(inst.b.shape[0]).astype(np.float32)).cuda() for _ in range(4)]

    def timed(fn, steps):
        for k in range(max(args.warmup, 1)):
            fn(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            fn(k)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32", mode=mode)
    ms_factor = timed(lambda k: s.factor(A, B, b, d, inst.lam), args.steps)
    s.set_keep_q(True)
    ms_factor_keep = timed(lambda k: s.factor(A, B, b, d, inst.lam), args.steps)
    p = torch.empty(inst.N, dtype=torch.float64, device="cuda")
    c = torch.empty(inst.N, dtype=torch.float64, device="cuda")
    ms = timed(lambda k: s.solve_qt(rhs[k % 4], sweeps=1, out=p), args.steps)
    ms_qt0 = timed(lambda k: s.solve_qt(rhs[k % 4], sweeps=0, out=p), args.steps)
    ms_apply = timed(lambda k: s.apply_qt(rhs[k % 4], out=c), args.steps)
    ms_rhs4 = timed(lambda k: s.solve_rhs(rhs[k % 4], sweeps=4, out=p), args.steps)
    s.raise_on_status()

    accuracy, cpu_baseline = None, None
    if not args.no_cpu:
        from oracle import refine
        b2 = rhs[0].cpu().numpy()
        errs = {"solve_qt_0": s.solve_qt(rhs[0], sweeps=0).cpu().numpy(),
                "solve_qt_1": s.solve_qt(rhs[0], sweeps=1).cpu().numpy(),
                "solve_rhs_4": s.solve_rhs(rhs[0], sweeps=4).cpu().numpy()}
        print("[bench] oracle (cpu_baseline leg)", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        p_ref, _ = refine.reference_solution(dataclasses.replace(inst, b=b2), sweeps=2)
        t_oracle = time.perf_counter() - t0
        d_ = inst.d
        accuracy = {k: float(np.max(d_ * np.abs(v - p_ref)) / np.max(d_ * np.abs(p_ref))) for k, v in errs.items()}
        cpu_baseline = {"value": 1.0 / t_oracle, "unit": "solves/s", "cores": _cpu_threads(), "kind": "oracle",
                        "sample": "one float64 oracle solve of the full workload for a new right-hand side "
                                  "(structured QR with the right-hand side carried, two refinement sweeps); "
                                  "%.2f s" % t_oracle}
    out = {"metric": "new right-hand side solves/sec with the kept factor", "value": 1000.0 / ms,
           "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if mode == "plain" else "bf16x3", "data": "synthetic",
           "config": {"workload": "new right-hand sides with the stored Q: 50,000 blocks of 12x3 + dense "
                                  "600,000x90, lambda 1e-2, factored once; each step Q^T b, back-substitution "
                                  "and one float64 sweep", "refine_sweeps": 1, "refine_dtype": "f64"},
           "ms": {"solve_qt_1sweep": ms, "solve_qt_0sweeps": ms_qt0, "apply_qt": ms_apply,
                  "solve_rhs_4sweeps": ms_rhs4, "factor": ms_factor, "factor_keep_q": ms_factor_keep},
           "accuracy": accuracy, "roofline": None, "cpu_baseline": cpu_baseline}
    print(json.dumps(out))
    return 0


def run_camera(args):
    """Camera columns at bundle-adjustment size (the Jacobian of Section 6.2, each row on one point
    block and at most one camera): 22,106 points seen by 2..6 of 14 cameras of 9 parameters
    (176,844 rows, 126 coupled columns), lambda 1e-2, float32.  A step is the factor with B passed
    compressed (each row's 9 camera values and its camera index) plus the solve with one float64
    sweep; the same J with B stored dense is timed beside it."""
    import numpy as np
    import torch

    from paper_1802_03773_amd import BlockAngularCamSolver, BlockAngularSolver
    from workloads import generators as gen

    mode = "bf16x3" if args.mode == "auto" else args.mode
    print("[bench] generating workload", file=sys.stderr, flush=True)
    K = 22106
    inst = gen.make_blockangular_cam(args.seed + 7, K=K, obs=2 + (np.arange(K) * 13) % 5, ncam=14, cw=9, n=3,
                                     lam=1e-2, dtype=np.float32)
    A, Bv, cam, b, d = (torch.from_numpy(np.ascontiguousarray(x)).cuda()
                        for x in (inst.A, inst.Bv, inst.cam, inst.b, inst.d))
    Bdense = np.zeros((inst.M, inst.nB), dtype=np.float32)  # the same rows stored dense (a layout change)
    for c in range(inst.ncam):
        sel = inst.cam == c
        Bdense[sel, c * inst.cw:(c + 1) * inst.cw] = inst.Bv[sel]
    Bd = torch.from_numpy(Bdense).cuda()
    p = torch.empty(inst.N, dtype=torch.float64, device="cuda")

    def timed(fn, steps):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    sc = BlockAngularCamSolver(inst.row_off, inst.n, inst.ncam, inst.cw, dtype="float32", mode=mode)
    sd = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32", mode=mode)
    ms_dense = timed(lambda: (sd.factor(A, Bd, b, d, inst.lam), sd.solve(sweeps=1, out=p)), args.steps)
    p_dense = p.clone()
    step = lambda: (sc.factor(A, Bv, cam, b, d, inst.lam), sc.solve(sweeps=1, out=p))  # noqa: E731
    ms = timed(step, args.steps)
    sc.raise_on_status()
    same = bool(torch.equal(p, p_dense))
    # per-phase times of the timed step, and their rooflines
    sc.profile_enable(4 * args.steps)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ph = sc.profile_read()
    M, n, nB, cw = inst.M, inst.n, inst.nB, inst.cw
    L, N, es = nB + 1, inst.N, 4
    Bc = M * (cw * es + 4)  # compressed B: values and camera index per row
    work = {"block_qr": ("hbm", M * n * es + Bc + M * es + N * 8 + (K + 1) * 8
                         + K * n * n * es + K * n * L * es + M * L * es),
            "dense_leaves": ("alu", 2.0 * (M + nB) * L * L - (2.0 / 3.0) * L ** 3),
            "refine": ("hbm", M * n * es + Bc + M * es + N * 8 + (K + 1) * 8 + 2 * N * 8
                       + K * n * n * es * 2 + K * n * L * es * 2 + 2 * K * n * 8)}
    phases = {}
    for k, (bound, amount) in work.items():
        t_ms, cnt = ph[k]
        if k == "dense_leaves":
            t_ms += ph["dense_tree"][0]
        if cnt == 0:
            continue
        avg = t_ms / cnt
        if bound == "hbm":
            ach, peak, unit = amount / (avg * 1e-3) / 1e9, 8000.0, "GB/s"
        else:
            ach, peak, unit = amount / (avg * 1e-3) / 1e12, 157.3, "TFLOP/s"
        phases[k] = {"avg_ms": avg, "bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak}
    dom = max(phases, key=lambda k: phases[k]["avg_ms"])
    roofline = dict(phases[dom], kernel=dom, traffic=None)
    roofline.pop("avg_ms")
    accuracy, cpu_baseline = None, None
    if not args.no_cpu:
        from oracle import dense as odense
        from oracle import structured as ostruct
        print("[bench] oracle (cpu_baseline leg)", file=sys.stderr, flush=True)
        ba = odense.blockangular_from_cam(inst)
        t0 = time.perf_counter()
        p_ref, _ = ostruct.solve_blockangular(ba)
        t_oracle = time.perf_counter() - t0
        rel, scaled = _errs(p.cpu().numpy(), p_ref, inst.d)
        accuracy = {"rel_err": rel, "scaled_err": scaled}
        cpu_baseline = {"value": 1.0 / t_oracle, "unit": "steps/s", "cores": _cpu_threads(), "kind": "oracle",
                        "sample": "one structured float64 oracle solve of the full workload (B assembled dense, "
                                  "per-block LAPACK QR, LAPACK QR of the reduced rows); %.2f s" % t_oracle}
    out = {"metric": "LM step solves/sec, camera columns at bundle-adjustment size", "value": 1000.0 / ms,
           "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if mode == "plain" else "bf16x3", "data": "synthetic",
           "config": {"workload": "camera columns: 22,106 points seen by 2..6 of 14 cameras of 9 parameters, "
                                  "176,844 rows, B compressed, float32, lambda 1e-2, one float64 sweep",
                      "points": K, "rows": M, "cameras": inst.ncam, "camera_width": cw, "dense_cols": nB,
                      "refine_sweeps": 1, "refine_dtype": "f64"},
           "ms_per_step_dense_B": ms_dense, "bit_identical_to_dense_B": same,
           "B_bytes_compressed": Bc, "B_bytes_dense": M * nB * es,
           "phases": phases, "accuracy": accuracy, "roofline": roofline, "cpu_baseline": cpu_baseline}
    print(json.dumps(out))
    return 0


def _errs(p, p_ref, d):
    """(2-norm relative error, largest column-scaled componentwise error) of p against p_ref."""
    import numpy as np
    p, p_ref, d = (np.asarray(x, np.float64) for x in (p, p_ref, d))
    return (float(np.linalg.norm(p - p_ref) / np.linalg.norm(p_ref)),
            float(np.max(d * np.abs(p - p_ref)) / np.max(d * np.abs(p_ref))))


def run_configs(args):
    """One row per workload configuration of the step solve besides the headline: the tiny
    100-block problem (latency of one solve, float64 and float32), the 50,000-block problem at
    lambda 1e-4, 1e-2 and 1 (steps/s, both update modes), the column-scaled precision problems
    (k = 3, 4, 5: error against the float64 oracle by refinement sweeps, both modes; also with the
    scales rotated across B's columns, damped and undamped) and the
    10,000-block adjoint (time of factor + solve + adjoint, gradient against the oracle's), and
    a bundle-adjustment-sized problem with camera columns (compressed B against the same J with
    B stored dense)."""
    import numpy as np
    import torch

    from paper_1802_03773_amd import BlockAngularSolver
    from workloads import generators as gen

    def timed(fn, steps):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    def dev(inst):
        return tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (inst.A, inst.B, inst.b, inst.d))

    oracle = not args.no_cpu
    if oracle:
        from oracle import adjoint as oadj
        from oracle import dense as odense
        from oracle import refine
    rows = {}
    # tiny problem: one solve's latency
    tiny = {}
    for dt, sweeps in ((np.float64, 0), (np.float32, 1)):
        inst = gen.tiny_blockangular(args.seed, dtype=dt)
        A, B, b, d = dev(inst)
        s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype=np.dtype(dt).name)
        p = torch.empty(inst.N, dtype=torch.float64, device="cuda")
        ms = timed(lambda: (s.factor(A, B, b, d, inst.lam), s.solve(sweeps=sweeps, out=p)), max(args.steps, 50))
        row = {"us_per_solve": ms * 1e3, "refine_sweeps": sweeps}
        if oracle:
            p_ref, _ = refine.reference_solution(inst)
            row["rel_err"], row["scaled_err"] = _errs(p.cpu().numpy(), p_ref, inst.d)
        # the same step captured as one HIP graph and replayed (no launch cost per kernel)
        eager = p.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            s.factor(A, B, b, d, inst.lam)
            s.solve(sweeps=sweeps, out=p)
        row["us_per_solve_graph_replay"] = timed(g.replay, max(args.steps, 100)) * 1e3
        row["graph_replay_bit_identical"] = bool(torch.equal(p, eager))
        tiny[np.dtype(dt).name] = row
    rows["tiny_100_blocks"] = tiny
    print("[bench] tiny done", file=sys.stderr, flush=True)
    # the 50,000-block problem at three damping values
    lam_rows = {}
    for lam in (1e-4, 1e-2, 1.0):
        inst = gen.scale_blockangular(args.seed, lam=lam)
        A, B, b, d = dev(inst)
        p = torch.empty(inst.N, dtype=torch.float64, device="cuda")
        row = {}
        for mode in ("plain", "bf16x3"):
            s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32", mode=mode)
            ms = timed(lambda: (s.factor(A, B, b, d, lam), s.solve(sweeps=1, out=p)), args.steps)
            row[mode] = {"steps_per_s": 1000.0 / ms, "ms_per_step": ms}
            if oracle:
                if "p_ref" not in row:
                    row["p_ref"], _ = refine.reference_solution(inst, sweeps=2)
                row[mode]["rel_err"], row[mode]["scaled_err"] = _errs(p.cpu().numpy(), row["p_ref"], inst.d)
        row.pop("p_ref", None)
        lam_rows[repr(lam)] = row
        print(f"[bench] lambda {lam} done", file=sys.stderr, flush=True)
    rows["scale_by_lambda"] = lam_rows
    # column-scaled precision problems: error by refinement sweeps
    if oracle:
        prec = {}
        for k in (3.0, 4.0, 5.0):
            inst = gen.precision_blockangular(args.seed, k)
            A, B, b, d = dev(inst)
            p_ref, _ = refine.reference_solution(inst)
            cond = float(np.linalg.cond(np.vstack([odense.assemble_blockangular(inst),
                                                   np.sqrt(inst.lam) * np.diag(inst.d)])))
            row = {"cond": cond}
            for mode in ("plain", "bf16x3"):
                s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32", mode=mode)
                s.factor(A, B, b, d, inst.lam)
                row[mode] = {str(sw): _errs(s.solve(sweeps=sw).cpu().numpy(), p_ref, inst.d)[1] for sw in range(4)}
            prec[f"k={int(k)}"] = row
        rows["precision_scaled_err_by_sweeps"] = prec
        # the rotated stress variant (B's column scales rotated by a Haar-orthogonal H): errors
        # by refinement sweeps, damped and undamped
        rot = {}
        for k in (3, 4, 5):
            for lam in (1e-4, 0.0):
                inst = gen.precision_rotated(400 + k, k, lam=lam)
                A, B, b, d = dev(inst)
                p_ref, _ = refine.reference_solution(inst)
                Aaug = np.vstack([odense.assemble_blockangular(inst), np.sqrt(lam) * np.diag(inst.d)])
                row = {"cond": float(np.linalg.cond(Aaug)),
                       "cond_equilibrated": float(np.linalg.cond(Aaug / np.linalg.norm(Aaug, axis=0)))}
                for mode in ("plain", "bf16x3"):
                    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32", mode=mode)
                    s.factor(A, B, b, d, lam)
                    row[mode] = {str(sw): _errs(s.solve(sweeps=sw).cpu().numpy(), p_ref, inst.d)[1]
                                 for sw in range(9)}
                rot[f"k={k} lambda={lam}"] = row
        rows["precision_rotated_scaled_err_by_sweeps"] = rot
        print("[bench] precision done", file=sys.stderr, flush=True)
    # the adjoint
    inst, p_star = gen.adjoint_blockangular(500)
    A, B, b, d = dev(inst)
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32")
    ps = torch.from_numpy(p_star).cuda()
    out = {}

    def adj_step():
        s.factor(A, B, b, d, inst.lam)
        p = s.solve(sweeps=1)
        out["p"] = p
        out["g"] = s.solve_adjoint(p, p - ps)

    ms = timed(adj_step, args.steps)
    row = {"ms_factor_solve_adjoint": ms}
    if oracle:
        p_ref, f = refine.reference_solution(inst, sweeps=2)
        ref = oadj.adjoint_blockangular(inst, f, p_ref, p_ref - p_star)
        g = {k: v.cpu().numpy() for k, v in out["g"].items()}
        for k in ("dA", "dB", "db", "dd"):
            row[f"rel_err_{k}"] = float(np.linalg.norm(g[k] - ref[k]) / np.linalg.norm(ref[k]))
        row["rel_err_dlam"] = float(abs(g["dlam"][0] - ref["dlam"]) / abs(ref["dlam"]))
    rows["adjoint_10000_blocks"] = row
    # camera columns at bundle-adjustment size: 22,106 points seen by 2..6 of 14 cameras of 9
    # parameters, compressed B (qrk_create_blockangular_cam) against the same J with B dense
    from paper_1802_03773_amd import BlockAngularCamSolver
    K = 22106
    inst = gen.make_blockangular_cam(args.seed + 7, K=K, obs=2 + (np.arange(K) * 13) % 5, ncam=14, cw=9, n=3,
                                     lam=1e-2, dtype=np.float32)
    A, Bv, cam, b, d = (torch.from_numpy(np.ascontiguousarray(x)).cuda()
                        for x in (inst.A, inst.Bv, inst.cam, inst.b, inst.d))
    Bdense = np.zeros((inst.M, inst.nB), dtype=np.float32)  # the same rows stored dense (a layout change)
    for c in range(inst.ncam):
        sel = inst.cam == c
        Bdense[sel, c * inst.cw:(c + 1) * inst.cw] = inst.Bv[sel]
    Bd = torch.from_numpy(Bdense).cuda()
    p = torch.empty(inst.N, dtype=torch.float64, device="cuda")
    row = {"points": K, "rows": inst.M, "cameras": inst.ncam, "camera_width": inst.cw,
           "B_bytes_compressed": inst.M * (inst.cw + 1) * 4, "B_bytes_dense": inst.M * inst.nB * 4}
    sc = BlockAngularCamSolver(inst.row_off, inst.n, inst.ncam, inst.cw, dtype="float32", mode="bf16x3")
    sd = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32", mode="bf16x3")
    row["ms_per_step_camera"] = timed(lambda: (sc.factor(A, Bv, cam, b, d, inst.lam), sc.solve(sweeps=1, out=p)),
                                      args.steps)
    pc = p.clone()
    row["ms_per_step_dense_B"] = timed(lambda: (sd.factor(A, Bd, b, d, inst.lam), sd.solve(sweeps=1, out=p)),
                                       args.steps)
    row["bit_identical_to_dense_B"] = bool(torch.equal(p, pc))
    if oracle:
        from oracle import structured as ostruct
        p_ref, _ = ostruct.solve_blockangular(odense.blockangular_from_cam(inst))
        row["rel_err"], row["scaled_err"] = _errs(pc.cpu().numpy(), p_ref, inst.d)
    rows["camera_columns_bundle_adjustment_size"] = row
    print("[bench] camera columns done", file=sys.stderr, flush=True)
    head = rows["scale_by_lambda"]["0.01"]["bf16x3"]
    out_line = {"metric": METRIC, "value": head["steps_per_s"], "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3", "data": "synthetic",
                "config": {"workload": "per-configuration rows: the 100-block problem (float64, float32), the "
                                       "50,000-block problem at lambda 1e-4, 1e-2, 1 (no autotuning), the "
                                       "column-scaled precision problems k = 3, 4, 5, the 10,000-block adjoint, "
                                       "a bundle-adjustment-sized camera-column problem"},
                "rows": rows, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out_line))
    return 0


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the step runs on a "
              "single GPU (several GPUs would split the blocks and all-gather the dense-part triangles).",
              file=sys.stderr)
        return 2
    if args.workload in ("lm-scale", "lm-banded-batch"):
        return run_lm(args)
    if args.workload == "lambda-retry":
        return run_lambda(args)
    if args.workload == "new-rhs":
        return run_new_rhs(args)
    if args.workload == "configs":
        return run_configs(args)
    if args.workload == "camera":
        return run_camera(args)
    if args.workload != "scale":
        return run_batch(args)
    import numpy as np
    import torch

    from paper_1802_03773_amd import BlockAngularSolver
    from workloads import generators as gen

    print(f"[bench] generating workload (seed {args.seed})", file=sys.stderr, flush=True)
    inst = gen.scale_blockangular(args.seed, lam=args.lam)
    A = torch.from_numpy(inst.A).cuda()
    B = torch.from_numpy(inst.B).cuda()
    b = torch.from_numpy(inst.b).cuda()
    d = torch.from_numpy(inst.d).cuda()
    p = torch.empty(inst.N, dtype=torch.float64, device="cuda")

    cpu_baseline = None
    p_ref = None
    if not args.no_cpu:
        from oracle import refine, structured
        print("[bench] oracle (cpu_baseline leg)", file=sys.stderr, flush=True)

        def oracle_time():
            t0 = time.perf_counter()
            out = structured.solve_blockangular(inst)
            return time.perf_counter() - t0, out

        # the oracle as it stands, on the host's cores and on one core: the median of three runs
        # after one warm-up (whose solution seeds the refined reference)
        _, (p0, fac) = oracle_time()
        p_ref = refine.refine(inst, fac, p0, sweeps=2).astype(np.float64)
        t_all = sorted(oracle_time()[0] for _ in range(3))[1]
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                t_one = sorted(oracle_time()[0] for _ in range(3))[1]
        except ImportError:
            t_one = None
        cpu_baseline = {
            "value": 1.0 / t_all, "unit": "steps/s", "cores": _cpu_threads(), "kind": "oracle",
            "sample": "one structured float64 oracle solve of the full workload (per-block LAPACK QR, "
                      "Q_i^T applied to B and b, LAPACK QR of the 600,090 x 91 reduced rows, "
                      "back-substitution): median of 3 after one warm-up, %.2f s on %d threads%s" % (
                          t_all, _cpu_threads(), "" if t_one is None else ", %.2f s on 1 thread" % t_one),
            "one_core_value": None if t_one is None else 1.0 / t_one,
            "blas": _blas_build(),
        }

    def rel_err(x):
        x = x.cpu().numpy()
        return float(np.linalg.norm(x - p_ref) / np.linalg.norm(p_ref))

    def measure(mode):
        from paper_1802_03773_amd import qrkit
        solver = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32", mode=mode)

        def step(sweeps):
            solver.factor(A, B, b, d, args.lam)
            solver.solve(sweeps=sweeps, out=p)

        if not args.no_autotune:
            solver.factor(A, B, b, d, args.lam)
            solver.autotune()
        tune = qrkit.tune_choice(solver)
        print(f"[bench] {mode}: launch shape {tune}", file=sys.stderr, flush=True)

        errors = {}
        if p_ref is not None:
            for s_ in range(0, 4):
                step(s_)
                torch.cuda.synchronize()
                errors[s_] = rel_err(p)
        st = solver.status()
        if st[0] != 0:
            raise RuntimeError(f"device status {st} ({mode})")
        if args.sweeps >= 0:
            sweeps = args.sweeps
        elif errors:
            ok = [s_ for s_ in sorted(errors) if errors[s_] <= 1e-10]
            sweeps = ok[0] if ok else 3
        else:
            sweeps = 1

        def timed(sweeps_, steps, warmup, profile):
            for _ in range(warmup):
                step(sweeps_)
            torch.cuda.synchronize()
            if profile:
                solver.profile_enable(steps + 1)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                step(sweeps_)
            e1.record()
            torch.cuda.synchronize()
            ms_ = e0.elapsed_time(e1) / steps
            phases_ = solver.profile_read() if profile else None
            if profile:
                solver.profile_enable(0)
            return ms_, phases_

        print(f"[bench] {mode}: timing {args.steps} steps ({sweeps} sweeps)", file=sys.stderr, flush=True)
        # the per-phase HIP events (roofline) in one timed loop, the step rate in another without
        # them: each event pair adds a marker packet between the phases' kernels
        ms_prof, phases_ = timed(sweeps, args.steps, args.warmup, True)
        ms_, _ = timed(sweeps, args.steps, 1, False)
        ms_unref, _ = timed(0, args.steps, 1, False)
        return dict(mode=mode, sweeps=sweeps, errors=errors, ms=ms_, ms_profiled=ms_prof, phases=phases_,
                    ms_unrefined=ms_unref, tune=tune)

    modes = ["plain", "bf16x3"] if args.mode == "auto" else [args.mode]
    runs = {m: measure(m) for m in modes}
    ok_runs = [r for r in runs.values() if not r["errors"] or r["errors"].get(r["sweeps"], 1.0) <= 1e-10]
    best = min(ok_runs or list(runs.values()), key=lambda r: r["ms"])
    ms, phases, sweeps, errors = best["ms"], best["phases"], best["sweeps"], best["errors"]

    work = algorithmic_work(inst)
    phase_out = {}
    dominant = None
    for name, (tot_ms, cnt) in phases.items():
        if cnt == 0:
            continue
        avg_ms = tot_ms / cnt
        entry = {"avg_ms": avg_ms, "launches": cnt}
        if name in work:
            bound, amount, units = work[name]
            # one refine record covers all of a solve's sweeps
            per_launch = amount * (sweeps if name == "refine" else 1)
            if bound == "hbm":
                entry.update(bound="hbm", achieved=per_launch / (avg_ms * 1e-3) / 1e9, unit="GB/s",
                             peak=PEAK_HBM_GBS, algorithmic_bytes=per_launch, units=units)
            else:
                entry.update(bound="alu", achieved=per_launch / (avg_ms * 1e-3) / 1e12,
                             unit="TFLOP/s", peak=PEAK_FP32_VECTOR_TFLOPS, algorithmic_flops=per_launch,
                             units=units)
            entry["frac"] = entry["achieved"] / entry["peak"]
        phase_out[name] = entry
        if dominant is None or tot_ms > phases[dominant][0]:
            dominant = name
    dom = phase_out[dominant]
    roofline = {"kernel": dominant, "bound": dom.get("bound"), "achieved": dom.get("achieved"),
                "peak": dom.get("peak"), "unit": dom.get("unit"), "frac": dom.get("frac"),
                "traffic": measured_traffic(dominant, args.lam, best["mode"]),
                # `frac` prices the algorithmic flops against the fp32 vector peak: the Householder
                # panels run on the VALU, which bounds the phase; the matrix-core share is below
                "mfma": measured_mfma(dominant, args.lam, best["mode"], dom["avg_ms"])}

    if args.copy_calibration:
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")  # 256 MiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()

    plain = runs.get("plain")
    mode_rows = {m: {"value": 1000.0 / r["ms"], "ms_per_step": r["ms"], "ms_per_step_with_phase_events":
                     r["ms_profiled"], "refine_sweeps": r["sweeps"],
                     "rel_err_vs_oracle": r["errors"].get(r["sweeps"]), "by_sweeps": r["errors"],
                     "autotune": r["tune"]}
                 for m, r in runs.items()}

    out = {
        "metric": METRIC,
        "value": 1000.0 / ms,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if best["mode"] == "plain" else "bf16x3",
        "data": "synthetic",
        "config": {
            "workload": "block-angular LM step: 50,000 blocks of 12x3 + dense 600,000x90, float32, "
                        "column scales 10^(3t), D = column norms, lambda = %g" % args.lam,
            "K": inst.K, "block_rows": 12, "block_cols": 3, "dense_cols": inst.nB, "rows": inst.M,
            "unknowns": inst.N, "lambda": args.lam, "mode": best["mode"], "refine_sweeps": sweeps,
            "refine_dtype": "f64", "autotune": best["tune"],
        },
        "accuracy": {"rel_err_vs_oracle": errors.get(sweeps), "by_sweeps": errors},
        "plain_fp32": ({"value": 1000.0 / plain["ms_unrefined"], "ms_per_step": plain["ms_unrefined"],
                        "rel_err_vs_oracle": plain["errors"].get(0)} if plain else None),
        "modes": mode_rows,
        "roofline": roofline,
        "phases": phase_out,
        "cpu_baseline": cpu_baseline,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
