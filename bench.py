"""Benchmark: two-dot DMRG sigma = H psi on one MI355X.

A step is one sigma call over the whole two-dot problem (all operator
families, R-step and L-step GEMMs with the fused reduction), FP64, with the
operators and psi already resident in HBM.  Default workload: K=73, N=114
(57 alpha, 57 beta), Sz=0, D=2000, two dots at the middle of the chain
(sites 36, 37 counting from 1), seeded synthetic integrals and MPS.

Prints one JSON line (see the design doc for every field).
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H·ψ sigma TFLOP/s & ms/call (K=73, D=2000); Davidson time to 1e-6 Eh"
# MI355X dense matrix peaks (TFLOP/s) per sigma precision; split-BF16 runs
# three BF16 products per algorithmic product, so its peak in algorithmic
# flops is a third of the BF16 rate.
PEAKS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0}
PREC_ID = {"fp64": 0, "fp32": 1, "bf16x3": 2}

CONFIGS = {
    # name: (K, N_alpha, N_beta, D, bond, seed)
    "1": (8, 4, 4, 64, 3, 1),
    "2": (24, 12, 12, 1000, 11, 2),
    "3": (36, 18, 18, 3000, 17, 3),
    "5": (73, 57, 57, 2000, 35, 5),
}
BATCH = "4"   # 64 independent problems, fused launch sequence vs sequential calls


def batch_specs(n=64):
    """K even uniform in [16, 32], N = K (Sz = 0), D log-uniform in [256, 2000],
    mid-chain dots; (K, D) drawn with default_rng(4000); problem i uses integral seed
    4000 + i, MPS seed 6000 + i and psi seed 8000 + i."""
    rng = np.random.default_rng(4000)
    out = []
    for i in range(n):
        K = int(rng.choice(np.arange(16, 33, 2)))
        D = int(round(float(np.exp(rng.uniform(np.log(256), np.log(2000))))))
        out.append((K, K // 2, K // 2, D, K // 2 - 1, i))
    return out


def bench_batched(args):
    """64 independent sigma problems: one fused, autotuned, graph-replayed launch
    sequence (dmrg_sigma_batched) against 64 sequential dmrg_sigma calls."""
    import torch
    import synth
    from paper_2311_02854_amd import binding as B
    from paper_2311_02854_amd import gpu_context
    ctx = gpu_context(0)
    specs = batch_specs()
    t0 = time.time()
    ops, xs, ys, flops = [], [], [], 0.0
    for i, (K, Na, Nb, D, k, seed) in enumerate(specs):
        ints = synth.make_integrals(K, 4000 + seed)
        mps = synth.make_mps(K, Na, Nb, D, k, 6000 + seed)
        psi = synth.make_psi(mps, 8000 + seed)
        o = ctx.build_ops(ints, mps, x_budget=256 << 20)
        flops += o.stats()["flops_sigma"]
        ops.append(o)
        xs.append(torch.from_numpy(psi).cuda())
        ys.append(torch.empty_like(xs[-1]))
        if (i + 1) % 8 == 0:
            log(f"[bench] built {i + 1}/64 problems ({time.time() - t0:.0f} s)")
    ptr_x, ptr_y = [x.data_ptr() for x in xs], [y.data_ptr() for y in ys]

    def sequential():
        for o, a, b in zip(ops, ptr_x, ptr_y):
            o.sigma(a, b, 0)

    def fused():
        B.sigma_batched(ctx, ops, ptr_x, ptr_y, 0, 0)

    res = {}
    for name, fn in (("sequential", sequential), ("fused_graph", fused)):
        for _ in range(max(1, args.warmup)):
            fn()                       # the fused plan autotunes and captures on its first call
        torch.cuda.synchronize()
        log(f"[bench] {name}: warm")
        t1 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        res[name] = {"ms_per_step": dt * 1e3, "tflops": flops / dt / 1e12}
        log(f"[bench] {name}: {dt * 1e3:.1f} ms per 64 problems, {flops / dt / 1e12:.2f} TFLOP/s")
    out = {
        "metric": "aggregate sigma TFLOP/s, 64 independent problems (fused graph launch)",
        "value": res["fused_graph"]["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["fused_graph"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "64 independent two-dot DMRG sigma problems, K even U[16,32], N=K, Sz=0, "
                               "D log-uniform [256,2000], mid-chain, seeds 4000+i",
                   "tflop_per_step": flops / 1e12, "build_s": time.time() - t0},
        "sequential": res["sequential"],
        "speedup_vs_sequential": res["sequential"]["ms_per_step"] / res["fused_graph"]["ms_per_step"],
    }
    print(json.dumps(out), flush=True)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SRC = os.path.join(ROOT, "paper_2311_02854_amd", "csrc", "kernels.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "gemm_kernel_f64_sigma_K73_D2000_pmc.md")


def measured_traffic(config, precision):
    """HBM bytes per sigma call from the committed rocprofv3 PMC summary
    (FETCH_SIZE x fetch factor + WRITE_SIZE x write factor, KiB -> bytes), or
    None if there is none for this workload or the GEMM kernel source changed
    since the counters were taken."""
    import hashlib
    if config != "5" or precision != "fp64" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    vals = {}
    for line in open(TRAFFIC_PROFILE):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if vals.get("kernel_source_sha256") != src:
        return None
    try:
        return float(vals["hbm_bytes_per_call"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(ctx):
    """The oracle (O1) timed on the host on a bounded sample of the workload."""
    import synth
    from oracle import blocks
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    K, Na, Nb, D, k, seed = 12, 6, 6, 200, 5, 6
    ints = synth.make_integrals(K, 1000 + seed)
    mps = synth.make_mps(K, Na, Nb, D, k, 3000 + seed)
    psi = synth.make_psi(mps, 2000 + seed)
    flops = ctx.build_ops(ints, mps).stats()["flops_sigma"]
    t0 = time.time()
    ob = blocks.TwoDotBlocks(ints, mps)
    t_build = time.time() - t0
    ts = []
    for _ in range(3):
        t0 = time.time()
        ob.sigma(psi)
        ts.append(time.time() - t0)
    t = float(np.median(ts))
    return {"value": flops / t / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"oracle O1 sigma (dense super-block bipartition) on a K={K}, N={Na + Nb}, D={D} "
                       f"two-dot at sites ({k},{k + 1}) of the same synthetic family; median of 3 calls "
                       f"= {t * 1e3:.1f} ms/call; rate = the GPU plan's {flops / 1e9:.3f} GFLOP per call "
                       f"of that sample / oracle time; oracle operator build {t_build:.1f} s excluded")}


def davidson_leg(ops, psi, mlp_path):
    """Davidson time to 1e-6 Eh from the seeded start vector.

    Solvers: plain FP64 sigma with the textbook diagonal preconditioner
    (kappa = 0); FP64 with the shifted diagonal preconditioner (kappa = 1, the
    library default); split-BF16 sigma (FP64 polish) with the shifted diagonal
    one; the same with the learned preconditioner.  E_ref is the energy of the
    split-BF16 shifted run converged to ||r|| <= 1e-5 with FP64 sigma; its time to
    E_ref + 1e-6 comes from its trace, the other solvers stop there.  The FP32
    operator copies and the per-bond feature tables are built before the timed
    runs (they belong to the operator build)."""
    import torch
    w = np.load(mlp_path).astype(np.float32)
    y = torch.empty(len(psi), dtype=torch.float64, device="cuda")
    x = torch.from_numpy(psi).cuda()
    t = torch.empty_like(y)
    ops.sigma(x.data_ptr(), y.data_ptr(), 2)                           # FP32 operator copies
    ops.mlp_apply(w, x.data_ptr(), y.data_ptr(), 0.0, t.data_ptr())    # per-bond feature tables
    torch.cuda.synchronize()
    del t
    out = {"start": "seeded Gaussian psi (the bench input)", "mlp_weights": os.path.relpath(mlp_path, ROOT)}
    log("[bench] davidson bf16x3_shift (reference run) ...")
    x = torch.from_numpy(psi).cuda()
    eref, st = ops.davidson(x.data_ptr(), trace=4000, precision=2, precond_shift=1.0, tol_residual=1e-5,
                            max_iter=2000)
    tr = st["trace"]
    hit = np.nonzero((tr[:, 1] <= eref + 1e-6) & (tr[:, 3] == 0))[0]
    out["E_ref"] = eref
    out["bf16x3_shift"] = {"seconds_to_1e-6": float(tr[hit[0], 0]), "iterations_to_1e-6": int(hit[0] + 1),
                           "switch_iter": st["switch_iter"], "seconds_total": st["seconds"],
                           "iterations_total": st["iterations"], "residual": st["residual"],
                           "converged": st["converged"]}
    log(f"[bench] davidson bf16x3_shift: {out['bf16x3_shift']}")
    for name, kw in (("plain_fp64_diag", {"precond_shift": 0.0}), ("fp64_shift", {"precond_shift": 1.0}),
                     ("bf16x3_mlp_shift", {"precision": 2, "precond_shift": 1.0, "precond": 1, "mlp_weights": w})):
        log(f"[bench] davidson {name} ...")
        x = torch.from_numpy(psi).cuda()
        e, st = ops.davidson(x.data_ptr(), e_ref=eref, e_tol=1e-6, stop_at_ref=1, max_iter=2000,
                             tol_residual=1e-5, **kw)
        out[name] = {"seconds_to_1e-6": st["seconds_to_ref"], "iterations_to_1e-6": st["iters_to_ref"],
                     "fp64_sigma_calls": st["sigma_fp64"], "switch_iter": st["switch_iter"],
                     "mlp_fallbacks": st["mlp_fallbacks"], "E-E_ref": e - eref}
        log(f"[bench] davidson {name}: {out[name]}")
    t0 = out["plain_fp64_diag"]["seconds_to_1e-6"]
    for name in ("fp64_shift", "bf16x3_shift", "bf16x3_mlp_shift"):
        t1 = out[name]["seconds_to_1e-6"]
        out[f"speedup_{name}_vs_plain"] = (t0 / t1) if (t0 and t0 > 0 and t1 and t1 > 0) else None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="5", choices=sorted(list(CONFIGS) + [BATCH]))
    ap.add_argument("--precision", default="fp64", choices=sorted(PREC_ID),
                    help="arithmetic of the sigma contraction (psi and sigma stay binary64)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle cpu_baseline leg")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes (no autotuning)")
    ap.add_argument("--x-budget-gb", type=float, default=0.0,
                    help="R-step scratch per slot in GB (0: library default)")
    ap.add_argument("--davidson", action="store_true",
                    help="also time Davidson to 1e-6 Eh (plain FP64 + diagonal vs shifted, split-BF16, learned)")
    ap.add_argument("--mlp", default=os.path.join(ROOT, "paper_2311_02854_amd", "data", "precond_mlp.npy"),
                    help="learned preconditioner weights for --davidson")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy a 1 GiB device buffer 3 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU operator-parallel "
              f"path is a design in DESIGN.md, not built", file=sys.stderr)
        sys.exit(2)

    if args.config == BATCH:
        bench_batched(args)
        return

    import torch
    import synth
    from paper_2311_02854_amd import gpu_context

    K, Na, Nb, D, k, seed = CONFIGS[args.config]
    log(f"[bench] config {args.config}: K={K} N=({Na},{Nb}) D={D} bond={k}")
    t0 = time.time()
    ints = synth.make_integrals(K, 1000 + seed)
    mps = synth.make_mps(K, Na, Nb, D, k, 3000 + seed)
    psi = synth.make_psi(mps, 2000 + seed)
    log(f"[bench] synthetic inputs {time.time() - t0:.1f} s, n_psi={len(psi)}")
    ctx = gpu_context(0)
    t0 = time.time()
    ops = ctx.build_ops(ints, mps, x_budget=int(args.x_budget_gb * 1e9))
    t_build = time.time() - t0
    st = ops.stats()
    log(f"[bench] build_ops {t_build:.1f} s ({st['build_flops'] / 1e12:.1f} TFLOP renormalization), "
        f"sigma plan {st['flops_sigma'] / 1e12:.3f} TFLOP/call, ops {st['op_bytes'] / 1e9:.1f} GB")
    x = torch.from_numpy(psi).cuda()
    y = torch.empty_like(x)
    if args.copy_probe:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("[bench] copy probe: 3 x 1 GiB device-to-device copies done")
    prec = PREC_ID[args.precision]
    tune = None
    if not args.no_tune:
        t0 = time.time()
        ms0, ms1 = ops.autotune(prec)
        tune = {"ms_default_shapes": ms0, "ms_tuned": ms1, "tune_s": time.time() - t0}
        log(f"[bench] autotune: {ms0:.1f} ms/call with 64x64 tiles -> {ms1:.1f} ms/call ({time.time() - t0:.1f} s)")
    for i in range(args.warmup):
        ops.sigma(x.data_ptr(), y.data_ptr(), prec)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    ops.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ops.sigma(x.data_ptr(), y.data_ptr(), prec)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ops.stats()
    ops.profile(False)
    ms = dt / args.steps * 1e3
    flops = st["flops_sigma"]
    tflops = flops / (dt / args.steps) / 1e12
    kern_ms = prof["prof_gemm_ms"] / max(1, prof["prof_sigma_calls"])
    achieved = flops / (kern_ms * 1e-3) / 1e12 if kern_ms > 0 else None
    log(f"[bench] {args.steps} steps: {ms:.1f} ms/call, {tflops:.2f} TFLOP/s; GEMM kernels {kern_ms:.1f} ms/call")
    out = {
        "metric": METRIC, "value": tflops, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": (f"two-dot DMRG sigma, K={K}, N={Na + Nb} ({Na}a,{Nb}b), Sz=0, D={D}, "
                                f"dots at sites ({k + 1},{k + 2}) of 1..K, seeded integrals and MPS"),
                   "n_psi": int(st["n_psi"]), "psi_blocks": int(st["n_blocks"]), "terms": int(st["n_terms"]),
                   "gemms_per_call": int(st["n_rgemm"] + st["n_lgemm"]), "tflop_per_call": flops / 1e12,
                   "build_ops_s": t_build, "operator_GB": st["op_bytes"] / 1e9, "autotune": tune},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAKS[args.precision], "unit": "TFLOP/s",
                     "frac": (achieved / PEAKS[args.precision]) if achieved else None,
                     "traffic": measured_traffic(args.config, args.precision), "traffic_unit": "bytes per sigma call",
                     "kernel": f"gemm_kernel<{args.precision}>", "kernel_ms_per_call": kern_ms,
                     "launches_per_call": prof["prof_launches"] / max(1, prof["prof_sigma_calls"])},
    }
    if args.davidson:
        out["davidson"] = davidson_leg(ops, psi, args.mlp)
    if not args.no_cpu:
        log("[bench] cpu_baseline: oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
