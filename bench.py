"""Benchmark: two-dot DMRG sigma = H psi on one MI355X.

A step is one sigma call over the whole two-dot problem (all operator
families, R-step and L-step GEMMs with the fused reduction), FP64, with the
operators and psi already resident in HBM.  Default workload: K=73, N=114
(57 alpha, 57 beta), Sz=0, D=2000, two dots at the middle of the chain
(sites 36, 37 counting from 1), seeded synthetic integrals and MPS.

Prints one JSON line: the sigma rate (value, ms_per_step), the roofline of
the GEMM kernels (HIP-event timed, with the HBM traffic of the committed
counter summary), the measured DGEMM / copy / batched peaks, the Davidson
time to 1e-6 Eh against an independent FP64 reference, the 64-problem fused
launch against sequential calls, and the oracle's CPU rate on a sample.
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


def batched_leg(steps, warmup, ctx=None):
    """64 independent sigma problems (the batch_specs workload): one fused,
    autotuned, graph-replayed launch sequence (dmrg_sigma_batched) against 64
    sequential dmrg_sigma calls.  Returns the timings and the problems' flops."""
    import torch
    import synth
    from paper_2311_02854_amd import binding as B
    from paper_2311_02854_amd import gpu_context
    ctx = ctx or gpu_context(0)
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
    build_s = time.time() - t0
    ptr_x, ptr_y = [x.data_ptr() for x in xs], [y.data_ptr() for y in ys]

    def sequential():
        for o, a, b in zip(ops, ptr_x, ptr_y):
            o.sigma(a, b, 0)

    def fused():
        B.sigma_batched(ctx, ops, ptr_x, ptr_y, 0, 0)

    res = {}
    for name, fn in (("sequential", sequential), ("fused_graph", fused)):
        for _ in range(max(1, warmup)):
            fn()                       # the fused plan autotunes and captures on its first call
        torch.cuda.synchronize()
        log(f"[bench] {name}: warm")
        t1 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / steps
        res[name] = {"ms_per_step": dt * 1e3, "tflops": flops / dt / 1e12}
        log(f"[bench] {name}: {dt * 1e3:.1f} ms per 64 problems, {flops / dt / 1e12:.2f} TFLOP/s")
    for o in ops:
        o.destroy()
    return {"workload": "64 independent two-dot DMRG sigma problems, K even U[16,32], N=K, Sz=0, "
                        "D log-uniform [256,2000], mid-chain, seeds 4000+i",
            "tflop_per_step": flops / 1e12, "build_s": build_s, "steps": steps, "warmup": warmup,
            "sequential": res["sequential"], "fused_graph": res["fused_graph"],
            "speedup_vs_sequential": res["sequential"]["ms_per_step"] / res["fused_graph"]["ms_per_step"]}


def bench_batched(args):
    """The batched workload as the bench line itself (--config 4)."""
    r = batched_leg(args.steps, args.warmup)
    out = {
        "metric": "aggregate sigma TFLOP/s, 64 independent problems (fused graph launch)",
        "value": r["fused_graph"]["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["fused_graph"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": r["workload"], "tflop_per_step": r["tflop_per_step"], "build_s": r["build_s"]},
        "sequential": r["sequential"],
        "speedup_vs_sequential": r["speedup_vs_sequential"],
    }
    print(json.dumps(out), flush=True)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SRC = os.path.join(ROOT, "paper_2311_02854_amd", "csrc", "kernels.hip")
# committed rocprofv3 counter summaries, by (workload, precision)
TRAFFIC_PROFILE = {("5", prec): os.path.join(ROOT, "profiles", f"gemm_kernel_{tag}_sigma_K73_D2000_pmc.md")
                   for prec, tag in (("fp64", "f64"), ("fp32", "f32"), ("bf16x3", "bf16x3"))}
TRAFFIC_PROFILE.update({("3", prec): os.path.join(ROOT, "profiles", f"gemm_kernel_{tag}_sigma_K36_D3000_pmc.md")
                        for prec, tag in (("fp64", "f64"), ("fp32", "f32"), ("bf16x3", "bf16x3"))})


def measured_traffic(config, precision):
    """HBM bytes per sigma call from the committed rocprofv3 PMC summary of
    this workload and precision (FETCH_SIZE x fetch factor + WRITE_SIZE x
    write factor, KiB -> bytes), or None if there is none for them or the GEMM
    kernel source changed since the counters were taken."""
    import hashlib
    path = TRAFFIC_PROFILE.get((config, precision))
    if path is None or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
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


def cpu_baseline(flops_call, n_psi, K, Na, Nb, D, k, seed, nrows=2000):
    """The oracle timed on the host on a bounded sample of the benchmark size.

    O2 (oracle/detci) evaluates rows of sigma = P^T H P psi directly from
    Eq. (Hsq) in the determinant basis; it needs renormalized states that are
    short determinant sums, so the sample uses the determinant-state MPS of
    the same K, N, D, bond and sector dimensions (synth.make_det_mps).  The
    rate is the benchmark plan's flops per call scaled by the fraction of
    the rows computed, over the oracle's time.  The renormalized-operator
    oracle O1 cannot reach this size (dense super-blocks)."""
    import synth
    from oracle import detci
    from synth.mps import make_det_mps
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    cores = int(os.environ.get("OMP_NUM_THREADS", cores))
    ints = synth.make_integrals(K, 1000 + seed)
    mps = make_det_mps(K, Na, Nb, D, k, 5000 + seed)
    psi = synth.make_psi(mps, 2000 + seed)
    ds = detci.DetSpace(ints, mps)
    rows = np.random.default_rng(0).choice(ds.n_psi, nrows, replace=False)
    ds.sigma_rows(psi, rows[:2])          # warm (library load)
    t0 = time.time()
    ds.sigma_rows(psi, rows)
    t = time.time() - t0
    frac = nrows / ds.n_psi
    return {"value": flops_call * frac / t / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": (f"oracle O2 (determinant-basis rows of sigma from Eq. Hsq) on {nrows} random rows of the "
                       f"K={K}, N={Na + Nb}, D={D} two-dot at sites ({k + 1},{k + 2}) with the determinant-state "
                       f"MPS of the same sectors; {t:.1f} s = {t / nrows * 1e3:.0f} ms/row; rate = the benchmark "
                       f"plan's {flops_call / 1e12:.2f} TFLOP/call x {nrows}/{ds.n_psi} rows / oracle time; "
                       f"a whole sigma call would take {t / frac / 3600:.0f} h")}


def davidson_leg(ops, psi, mlp_path):
    """Davidson time to 1e-6 Eh from the seeded start vector.

    E_ref comes first, from its own FP64 run (shifted diagonal preconditioner)
    converged to ||r||_2 <= 1e-7: its error is of order ||r||^2 / gap, far below
    1e-6 Eh, so the threshold does not depend on the solvers compared.  The
    FP64 shifted solver's time to E_ref + 1e-6 is read from that run's trace.
    The other solvers stop at the first FP64 Ritz value <= E_ref + 1e-6:
    plain FP64 sigma with the textbook diagonal preconditioner (kappa = 0);
    split-BF16 sigma (FP64 polish) with the shifted diagonal one; the same
    with the learned preconditioner.  The FP32 operator copies and the per-bond
    feature tables are built before the timed runs (they belong to the operator
    build)."""
    import torch
    w = np.load(mlp_path).astype(np.float32)
    y = torch.empty(len(psi), dtype=torch.float64, device="cuda")
    x = torch.from_numpy(psi).cuda()
    t = torch.empty_like(y)
    ops.sigma(x.data_ptr(), y.data_ptr(), 2)                           # FP32 operator copies
    ops.mlp_apply(w, x.data_ptr(), y.data_ptr(), 0.0, t.data_ptr())    # per-bond feature tables
    torch.cuda.synchronize()
    del t, y
    out = {"start": "seeded Gaussian psi (the bench input)", "mlp_weights": os.path.relpath(mlp_path, ROOT)}
    tol_ref = 1e-7
    log(f"[bench] davidson reference: FP64, shifted diagonal, to ||r|| <= {tol_ref:g} ...")
    x = torch.from_numpy(psi).cuda()
    eref, st = ops.davidson(x.data_ptr(), trace=4000, precision=0, precond_shift=1.0, tol_residual=tol_ref,
                            max_iter=2000)
    tr = st["trace"]
    hit = np.nonzero(tr[:, 1] <= eref + 1e-6)[0]
    out["E_ref"] = eref
    out["E_ref_provenance"] = (f"FP64 sigma, shifted diagonal preconditioner, converged to ||r||_2 = "
                               f"{st['residual']:.2e} in {st['iterations']} iterations ({st['seconds']:.1f} s)")
    out["E_ref_residual"] = st["residual"]
    out["fp64_shift"] = {"seconds_to_1e-6": float(tr[hit[0], 0]), "iterations_to_1e-6": int(hit[0] + 1),
                         "note": "read from the reference run's trace"}
    log(f"[bench] davidson reference E={eref:.10f}: {out['E_ref_provenance']}")
    for name, kw in (("plain_fp64_diag", {"precond_shift": 0.0}),
                     ("bf16x3_shift", {"precision": 2, "precond_shift": 1.0}),
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
    m, b = out["bf16x3_mlp_shift"]["seconds_to_1e-6"], out["bf16x3_shift"]["seconds_to_1e-6"]
    out["mixed_learned_faster_than_plain"] = bool(m and t0 and 0 < m < t0)
    out["learned_faster_than_shifted_diag"] = bool(m and b and 0 < m < b)
    return out


def mixed_leg(ops, psi):
    """Reduced-precision sigma and energy errors against FP64 on this workload.

    sigma: relative 2-norm and max-element errors of the FP32 and split-BF16
    sigma of the bench input against the FP64 one.  Energy: Davidson from the
    same start in FP64 and with each reduced precision (switching to FP64
    sigma near its noise floor), all to ||r||_2 <= 1e-5; the difference of the
    returned FP64 Rayleigh quotients, and wall times."""
    import torch
    x = torch.from_numpy(psi).cuda()
    ys = {}
    for name, p in (("fp64", 0), ("fp32", 1), ("bf16x3", 2)):
        y = torch.empty_like(x)
        ops.sigma(x.data_ptr(), y.data_ptr(), p)
        torch.cuda.synchronize()
        ys[name] = y.cpu().numpy()
    out = {"sigma": {}, "davidson": {}}
    ref = ys["fp64"]
    for name in ("fp32", "bf16x3"):
        d = ys[name] - ref
        out["sigma"][name] = {"rel2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
                              "relmax": float(np.abs(d).max() / np.abs(ref).max())}
    for name, p in (("fp64", 0), ("bf16x3", 2), ("fp32", 1)):
        x = torch.from_numpy(psi).cuda()
        t0 = time.time()
        e, st = ops.davidson(x.data_ptr(), tol_residual=1e-5, max_iter=600, precision=p)
        out["davidson"][name] = {"E": e, "seconds": time.time() - t0, "iterations": st["iterations"],
                                 "fp64_sigma_calls": st["sigma_fp64"], "converged": st["converged"]}
        if name != "fp64":
            out["davidson"][name]["E-E_fp64"] = e - out["davidson"]["fp64"]["E"]
        log(f"[bench] mixed {name}: {out['davidson'][name]}")
    log(f"[bench] mixed sigma errors: {out['sigma']}")
    return out


def sweep_leg(ctx, ints, K, Na, Nb, D, seed):
    """Config 2: sigma and Davidson at every bond of one left-to-right pass of
    the two-dot sweep (operators rebuilt per bond, decimation to D after each
    bond), then E(w): two full sweeps at each of three smaller D, each started
    from the previous one's MPS, the last pass's lowest energy and largest
    discarded weight w, and the least-squares line E = E0 + a w.""" 
    import torch
    import synth
    from paper_2311_02854_amd.sweep import sweep
    mps0 = synth.make_mps(K, Na, Nb, D, 0, 3000 + seed)
    bonds = []

    def per_bond(rec):
        bonds.append(rec)
        log(f"[bench] sweep k={rec['k']} E={rec['energy']:.8f} it={rec['iterations']} "
            f"w={rec.get('discarded', 0):.2e} {rec['seconds']:.2f} s")

    t0 = time.time()
    hist, mps = sweep(ctx, ints, mps0, D, first_pass_only=True, tol_residual=1e-5, log=per_bond)
    t_pass = time.time() - t0
    # sigma timing per bond on the final pass's MPS would need the operators
    # again: time sigma at three bonds of the decimated MPS instead
    out = {"pass_seconds": t_pass, "bonds": len(hist),
           "energies": [h["energy"] for h in hist], "discarded": [h.get("discarded", 0.0) for h in hist],
           "davidson_iterations": [h["iterations"] for h in hist],
           "build_seconds": [h["build_s"] for h in hist], "n_psi": [h["n_psi"] for h in hist]}
    ew = []
    m = synth.make_mps(K, Na, Nb, D // 10, 0, 3000 + seed)
    for d in (D // 10, D // 5, D // 2):   # each D warm-started from the previous one's MPS
        h2, m = sweep(ctx, ints, m, d, nsweeps=2, tol_residual=1e-6)
        last = [h for h in h2 if h["pass"] == 3]
        w = max(h.get("discarded", 0.0) for h in last)
        e = min(h["energy"] for h in last)
        ew.append({"D": d, "E": e, "w": w})
        log(f"[bench] E(w): D={d} E={e:.8f} w={w:.3e}")
    A = np.array([[1.0, e["w"]] for e in ew])
    coef, *_ = np.linalg.lstsq(A, np.array([e["E"] for e in ew]), rcond=None)
    out["E_of_w"] = {"points": ew, "E0": float(coef[0]), "slope": float(coef[1])}
    return out


def measured_peaks():
    """This GPU's own peaks beside the datasheet ones: FP64 DGEMM (torch.matmul,
    8192^3, the library GEMM), device-to-device copy bandwidth (4 GiB), and the
    paper's uniform batched-GEMM model of Sec. 3 (M = N = K = d_max(D = 2000)
    = 308, 10 GB of operands, torch.bmm = the library's batched DGEMM)."""
    import torch
    out = {}
    a = torch.randn(8192, 8192, dtype=torch.float64, device="cuda")
    b = torch.randn_like(a)
    for _ in range(2):
        c = a @ b
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        c = a @ b
    torch.cuda.synchronize()
    out["dgemm_fp64_8192_tflops"] = 5 * 2 * 8192 ** 3 / (time.perf_counter() - t0) / 1e12
    del a, b, c
    x = torch.empty(1 << 29, dtype=torch.float64, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    out["copy_GBps"] = 5 * 2 * x.numel() * 8 / (time.perf_counter() - t0) / 1e9
    del x, y
    d = 308
    nb = int(10e9 / (2 * d * d * 8))
    A = torch.randn(nb, d, d, dtype=torch.float64, device="cuda")
    B = torch.randn(nb, d, d, dtype=torch.float64, device="cuda")
    C = torch.bmm(A, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        C = torch.bmm(A, B)
    torch.cuda.synchronize()
    out["uniform_batched_dmax308_tflops"] = 3 * 2 * nb * d ** 3 / (time.perf_counter() - t0) / 1e12
    out["uniform_batched_note"] = f"{nb} FP64 GEMMs of 308^3 (10 GB of operands), torch.bmm"
    del A, B, C
    torch.cuda.empty_cache()
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
    ap.add_argument("--tile", type=int, default=None,
                    help="launch every sigma GEMM with this mode (0-3 uniform tiles, 4 mixed 64/32 strips, 5 128x128 "
                         "on 1024-thread workgroups, 6 128x128 interiors of long-k tasks + the rest mixed) "
                         "instead of autotuning")
    ap.add_argument("--grid", type=int, default=0, help="grid mode with --tile (0 one workgroup per job, -1 dynamic)")
    ap.add_argument("--x-budget-gb", type=float, default=0.0,
                    help="R-step scratch per slot in GB (0: library default)")
    ap.add_argument("--no-davidson", action="store_true",
                    help="skip the Davidson time-to-1e-6 Eh leg (plain FP64 + diagonal vs shifted, split-BF16, learned)")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured DGEMM / copy / batched peaks")
    ap.add_argument("--no-sweep", action="store_true", help="skip the sweep leg of --config 2")
    ap.add_argument("--ksplit", type=int, default=0,
                    help="split-k threshold of the L-step in k tiles (0: the library default, 512)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-problem fused-launch leg of the default run")
    ap.add_argument("--build-only", action="store_true",
                    help="only build the operators (dmrg_build_ops) and print its wall time (for profiling)")
    ap.add_argument("--mixed", action="store_true",
                    help="also report FP32 / split-BF16 sigma and energy errors (on by default for --config 3)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg of --config 3")
    ap.add_argument("--mlp", default=os.path.join(ROOT, "paper_2311_02854_amd", "data", "precond_mlp.npy"),
                    help="learned preconditioner weights for --davidson")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy a 1 GiB device buffer 3 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU operator-parallel "
              f"path is designed but not built", file=sys.stderr)
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
    ops = ctx.build_ops(ints, mps, x_budget=int(args.x_budget_gb * 1e9), ksplit_tiles=args.ksplit)
    t_build = time.time() - t0
    st = ops.stats()
    log(f"[bench] build_ops {t_build:.1f} s ({st['build_flops'] / 1e12:.1f} TFLOP renormalization), "
        f"sigma plan {st['flops_sigma'] / 1e12:.3f} TFLOP/call, ops {st['op_bytes'] / 1e9:.1f} GB")
    if args.build_only:
        print(json.dumps({"build_ops_s": t_build, "build_tflop": st["build_flops"] / 1e12,
                          "build_tflops_per_s": st["build_flops"] / t_build / 1e12,
                          "operator_GB": st["op_bytes"] / 1e9}), flush=True)
        return
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
    if args.tile is not None:
        ops.launch_shape(prec, args.tile, args.grid)
        tune = {"fixed_tile": args.tile, "grid": args.grid}
    elif not args.no_tune:
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
    if not args.no_peaks:
        log("[bench] measured peaks ...")
        out["roofline"]["measured_peaks"] = measured_peaks()
        if args.precision == "fp64":
            out["roofline"]["frac_of_measured_dgemm"] = (
                achieved / out["roofline"]["measured_peaks"]["dgemm_fp64_8192_tflops"] if achieved else None)
        log(f"[bench] measured peaks: {out['roofline']['measured_peaks']}")
    if args.config == "2" and not args.no_sweep:
        out["sweep"] = sweep_leg(ctx, ints, K, Na, Nb, D, seed)
    if (args.config == "3" and not args.no_mixed) or args.mixed:
        out["mixed_precision"] = mixed_leg(ops, psi)
    if args.config == "5" and not args.no_davidson:
        out["davidson"] = davidson_leg(ops, psi, args.mlp)
    if args.config == "5" and not args.no_batched:
        # the fused many-problem launch (the batched workload), after the K73
        # operators are released
        ops.destroy()
        del x, y
        torch.cuda.empty_cache()
        log("[bench] batched: 64 problems, fused graph launch against sequential calls ...")
        out["batched"] = batched_leg(2, 1, ctx)
    if not args.no_cpu:
        log("[bench] cpu_baseline: oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(flops, int(st["n_psi"]), K, Na, Nb, D, k, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
