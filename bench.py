"""Benchmark of the Paraexp exp-action path on one MI355X.

One step = one complete solve of the 8192-point advection-diffusion workload on [0, 1]
(shifted samples, truncated SVD, Chebyshev fit, restarted block Krylov exp-action with
60 block steps per restart and the projected exponential, outputs at 32 times), inputs
already resident in device memory.  The Krylov space is by default the shift-and-invert
one (Sec. 2.1, the remark on rational Krylov acceleration); --krylov poly uses the
polynomial block Krylov space of eq. 2.4.  --windows P splits the interval into P
Paraexp windows (Sec. 2.2) solved as one batch and superposed (u = u0 + sum_j v_j).
Beside the timed configuration the same inputs are solved at the other precision, as
P = 4 windows and with the polynomial Krylov space, in the same process.
Prints one JSON line.  Only one GPU is used: --gpus above 1 exits with a message.
"""
import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
F64_MFMA_PEAK_TFS = 78.6  # MI355X published dense FP64 matrix rate
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _pmc_record(kernel, windows, krylov):
    tag = (f"_paraexp{windows}" if windows > 1 else "") + ("_sai" if krylov == "sai" else "")
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_c2_n8192{tag}.txt")
    try:
        return json.loads(open(path).read().split("\n---\n", 1)[1])
    except (OSError, IndexError, ValueError):
        return None


def measured_traffic(kernel, windows, krylov):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary of
    the same window split and Krylov space (FETCH_SIZE + WRITE_SIZE, scaled by a device
    copy of known size), or None when the summary is missing or was taken on a different
    kernel source."""
    import hashlib
    rec = _pmc_record(kernel, windows, krylov)
    src = os.path.join(ROOT, "paper_1509_04567_amd", "csrc", "kernels.hip")
    if rec is None:
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    return rec["traffic_bytes_per_launch"] if rec.get("kernels_hip_sha256") == sha else None


def measured_tiles(kernel, windows, krylov):
    """The block-kernel tiling the counter summary was taken on (as bench.py reports it)."""
    rec = _pmc_record(kernel, windows, krylov)
    return rec.get("tiles") if rec else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--batch", type=int, default=1,
                    help="independent windows solved together per step (seeds 2, 3, ...); 1 = the workload")
    ap.add_argument("--windows", type=int, default=1,
                    help="Paraexp windows per solve (Sec. 2.2): the window subproblems run as one batch "
                         "(s / P samples each) and u = u0 + sum_j v_j is superposed; 1 = one window")
    ap.add_argument("--krylov", choices=["sai", "poly"], default="sai",
                    help="Krylov space: shift-and-invert (rational) or polynomial block Krylov")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the other precision, the other window split and the other Krylov space "
                         "(same inputs, same process)")
    ap.add_argument("--roofline-kernel", default=None, choices=["block_update", "block_proj"],
                    help="kernel family of the roofline figure (default: the one with the most GPU time, "
                         "block_update, or block_proj for the polynomial space split into windows)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run one device copy of this many MiB first (reference for memory counters)")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for the baseline")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-instances figure (128 independent advection-diffusion instances)")
    ap.add_argument("--no-kernels", action="store_true",
                    help="skip the GEMM (MFMA) and stencil (HBM) kernel figures")
    ap.add_argument("--tiles", default="default",
                    help="tiling of the block kernels: 'tuned' (pe_autotune on this GPU before any timed "
                         "run), 'default' (the built-in choice) or a tile cache file of pe_autotune")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1509_04567_amd as pe

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    import oracle

    P = max(1, args.windows)
    if args.roofline_kernel is None:
        args.roofline_kernel = "block_proj" if (P > 1 and args.krylov == "poly") else "block_update"
    ctx = pe.Context(0)
    refs = {}
    if args.tiles != "default":
        rank_max = synth.config_c2(n=args.n).rank_max
        precs = [args.precision] if args.no_compare else ["fp64", "mixed"]
        tt = time.perf_counter()
        ntuned = ctx.autotune([(args.n, rank_max, pe.PE_FP64 if pr == "fp64" else pe.PE_MIXED) for pr in precs],
                              None if args.tiles == "tuned" else args.tiles)
        print(f"autotune: {ntuned} keys timed in {time.perf_counter() - tt:.2f} s", file=sys.stderr, flush=True)

    def run(precision, windows, steps, warmup, profile, krylov, family=None):
        """Time `steps` solves of the workload at one precision, window split and Krylov
        space; returns the figures of that run (accuracy against the oracle checked
        outside the timing)."""
        prec = pe.PE_FP64 if precision == "fp64" else pe.PE_MIXED
        kr = pe.PE_KRYLOV_SAI if krylov == "sai" else pe.PE_KRYLOV_POLY
        # the FP32-stored basis puts a floor of ~1e-9 under the residual estimate, so the
        # mixed path runs at tol 1e-8 (its accuracy target is 1e-7 against the FP64 oracle)
        tol = 1e-12 if precision == "fp64" else 1e-8
        probs = [synth.config_c2(n=args.n, seed=2 + i, tol=tol) for i in range(max(1, args.batch))]
        if windows > 1:
            # each instance as P Paraexp windows, all windows of all instances in one batch
            subs = []
            for i, pr in enumerate(probs):
                _, g_at = synth.c2_source(args.n, 2 + i)
                subs += synth.split_windows(pr, windows, g_at, s=max(2, pr.s // windows))
        else:
            subs = probs
        for sp in subs:
            sp.krylov = kr
        staged = ctx.prepare(subs, prec)

        def solve():
            outs, reps = ctx.solve_prepared(staged)
            if windows > 1:
                outs = [ctx.superpose(pr.u0, outs[i * windows:(i + 1) * windows]) for i, pr in enumerate(probs)]
            return outs, reps
        torch.cuda.synchronize()
        for i in range(warmup):
            tw = time.perf_counter()
            solve()
            print(f"[{krylov} {precision} P={windows}] warmup {i}: {time.perf_counter() - tw:.3f} s", file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        if profile:  # per-launch HIP-event timing of the dominant kernel family, on the solve's stream
            ctx.profile_enable(family or args.roofline_kernel)
        t0 = time.perf_counter()
        for i in range(steps):
            ts = time.perf_counter()
            outs, reps = solve()
            print(f"[{krylov} {precision} P={windows}] step {i}: {time.perf_counter() - ts:.3f} s "
                  f"cycles={reps[0]['cycles']} rejected={reps[0]['rejected']}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        prof = ctx.profile_read() if profile else None
        if profile:
            ctx.profile_enable(None)
        err = 0.0
        for i, pr in enumerate(probs):
            key = (args.n, 2 + i)
            if key not in refs:
                tc = time.perf_counter()
                refs[key] = (oracle.solve_window(pr, "spectral")[0], time.perf_counter() - tc)
            ref = refs[key][0]
            if windows > 1:  # the superposed u(t_k) = u0 + v(t_k)
                ref = pr.u0[:, None] + ref
            got = outs[i].detach().cpu().numpy().T
            err = max(err, float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
        return {"solves_per_s": len(probs) * steps / elapsed, "ms_per_step": 1e3 * elapsed / max(steps, 1),
                "rel_l2_vs_oracle": err, "report": reps[0], "prof": prof, "probs": probs}

    main_run = run(args.precision, P, args.steps, args.warmup, True, args.krylov)
    probs = main_run["probs"]
    prob = probs[0]
    prof = main_run["prof"]
    launches, k_ms, k_bytes, k_flops = prof["launches"], prof["ms"], prof["bytes"], prof["flops"]
    roof = None
    # the counter record of the single-window split covers three whole restart cycles,
    # whose launch mix is the solve's; with several windows the early cycles carry every
    # window at full width and later ones fewer, so that record is not the timed launches'
    traffic = (measured_traffic(args.roofline_kernel, P, args.krylov)
               if args.batch <= 1 and P == 1 and args.n == 8192 and args.precision == "fp64" else None)
    # the tiling the timed run used for its block widths (rank + 1, rank, 1)
    table = ctx.autotune_table()
    nlog2 = max(0, (args.n - 1).bit_length())
    mixed = 1 if args.precision == "mixed" else 0
    tiles = {"mode": args.tiles}
    for bw in sorted({main_run["report"]["rank"] + 1, max(1, main_run["report"]["rank"]), 1}):
        if (nlog2, bw, mixed) in table:
            tiles[f"width{bw}"] = {"rows_u": table[(nlog2, bw, mixed)][0], "rows_p": table[(nlog2, bw, mixed)][1]}
    if traffic is not None and tiles != measured_tiles(args.roofline_kernel, P, args.krylov):
        traffic = None  # the counters were taken on another tiling
    if launches > 0 and k_ms > 0:
        achieved = k_bytes / (k_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": args.roofline_kernel,
                "launches": launches, "avg_launch_us": 1e3 * k_ms / launches,
                "algorithmic_bytes_per_launch": k_bytes / launches,
                "flops_per_launch": k_flops / launches}
    rep = main_run["report"]
    err = main_run["rel_l2_vs_oracle"]

    # the same inputs at the other precision, the other window split and the other
    # Krylov space (same process)
    compare = {}
    if not args.no_compare:
        keys = ("solves_per_s", "ms_per_step", "rel_l2_vs_oracle", "report")
        other = "mixed" if args.precision == "fp64" else "fp64"
        other_kr = "poly" if args.krylov == "sai" else "sai"
        cmp_steps = max(1, min(args.steps, 2))
        tag = lambda prec, w, kr: f"{kr}_{prec}" + (f"_paraexp{w}" if w > 1 else "")
        o = run(other, P, cmp_steps, 1, False, args.krylov)
        compare[tag(other, P, args.krylov)] = {k: o[k] for k in keys}
        fp64_sps = main_run["solves_per_s"] if args.precision == "fp64" else o["solves_per_s"]
        mixed_sps = o["solves_per_s"] if args.precision == "fp64" else main_run["solves_per_s"]
        compare["speedup_mixed_over_fp64"] = mixed_sps / fp64_sps
        P2 = 4 if P == 1 else 1
        w = run(args.precision, P2, cmp_steps, 1, False, args.krylov)
        compare[tag(args.precision, P2, args.krylov)] = {k: w[k] for k in keys}
        pk = run(args.precision, P, 1, 1, False, other_kr)
        compare[tag(args.precision, P, other_kr)] = {k: pk[k] for k in keys}
        compare[f"speedup_{args.krylov}_over_{other_kr}"] = main_run["solves_per_s"] / pk["solves_per_s"]
    t_oracle = refs[(args.n, 2)][1]

    # the batched pipeline: the first 128 instances of the 512-instance advection-diffusion
    # workload (ragged n 512..16384, rank 1..8, l 40..100) solved as one batch; two
    # instances checked against the oracle
    batch = None
    if not args.no_batch:
        bprobs = synth.config_c4(tol=1e-9)[:128]
        for bp in bprobs:
            bp.krylov = pe.PE_KRYLOV_SAI

        def run_batch(c):
            staged_b = c.prepare(bprobs, pe.PE_FP64)  # the workload's tolerance 1e-9 is below the mixed floor
            c.solve_prepared(staged_b)  # warm-up: workspace growth and first-touch
            torch.cuda.synchronize()
            tb = time.perf_counter()
            bouts, breps = c.solve_prepared(staged_b)
            torch.cuda.synchronize()
            dtb = time.perf_counter() - tb
            berr = 0.0
            for i in (0, 64):
                ref = oracle.solve_window(bprobs[i], "spectral")[0]
                berr = max(berr, float(np.linalg.norm(bouts[i].detach().cpu().numpy().T - ref) / np.linalg.norm(ref)))
            return dtb, breps, berr

        dtb, breps, berr = run_batch(ctx)
        batch = {"workload": "advection_diffusion_instances_128_ragged_n512_16384", "precision": "fp64",
                 "instances": len(bprobs), "seconds": dtb, "instances_per_s": len(bprobs) / dtb,
                 "cycles_max": max(r["cycles"] for r in breps),
                 "cycles_mean": float(np.mean([r["cycles"] for r in breps])),
                 "not_converged": sum(1 for r in breps if r["flags"] & 1), "rel_l2_sampled_max": berr}
        # the same batch on block-kernel tiles tuned on this GPU (tuning is a one-off step
        # outside the timing, like a cache file from an earlier run)
        tctx = pe.Context(0)
        tt = time.perf_counter()
        keys = tctx.autotune([(bp.n, bp.rank_max, pe.PE_FP64) for bp in bprobs])
        tune_s = time.perf_counter() - tt
        dtt, treps, terr = run_batch(tctx)
        tctx.close()
        batch["tuned"] = {"seconds": dtt, "instances_per_s": len(bprobs) / dtt, "tune_seconds": tune_s,
                          "tuned_keys": keys, "speedup_over_default_tiles": dtb / dtt,
                          "not_converged": sum(1 for r in treps if r["flags"] & 1), "rel_l2_sampled_max": terr}

    # kernel figures beside the solve: the projected exponential's f64 MFMA products in the
    # same solve (one timed step), and the stencil S0 alone on a 2^20 x 32 block (the
    # long-grid, wide-block shape), each against its published peak
    kernels = {}
    if not args.no_kernels:
        g = run(args.precision, P, 1, 0, True, args.krylov, family="gemm")["prof"]
        if g["launches"] > 0 and g["ms"] > 0:
            tfs = g["flops"] / (g["ms"] * 1e-3) / 1e12
            kernels["gemm"] = {"bound": "mfma", "achieved": tfs, "peak": F64_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                               "frac": tfs / F64_MFMA_PEAK_TFS, "kernel": "k_gemm", "launches": g["launches"],
                               "avg_launch_us": 1e3 * g["ms"] / g["launches"],
                               "flops_per_launch": g["flops"] / g["launches"]}
        ns, cols = 1 << 20, 32
        X = torch.randn(cols, ns, dtype=torch.float64, device="cuda")
        coeffs = [1.0, -2.0, 1.0]
        ctx.stencil_apply(coeffs, X)  # warm
        ctx.profile_enable("stencil")
        for _ in range(20):
            ctx.stencil_apply(coeffs, X)
        sp = ctx.profile_read()
        ctx.profile_enable(None)
        del X
        if sp["launches"] > 0 and sp["ms"] > 0:
            gbs = sp["bytes"] / (sp["ms"] * 1e-3) / 1e9
            kernels["stencil"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": gbs / HBM_PEAK_GBS, "kernel": "k_stencil_cols", "n": ns, "columns": cols,
                                  "avg_launch_us": 1e3 * sp["ms"] / sp["launches"],
                                  "bytes_per_launch": sp["bytes"] / sp["launches"]}

    cpu = None
    if not args.no_cpu:
        reps_cpu, spent = 1, t_oracle
        while spent < args.cpu_budget and reps_cpu < 1000:
            tc = time.perf_counter()
            oracle.solve_window(prob, "spectral")
            spent += time.perf_counter() - tc
            reps_cpu += 1
        cores = len(os.sched_getaffinity(0))
        try:
            from threadpoolctl import threadpool_info
            th = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        except Exception:
            th = cores
        cpu = {"value": reps_cpu / spent, "unit": "solves/s", "cores": int(th), "kind": "oracle",
               "sample": f"{reps_cpu} full solves of the same n={args.n} window (spectral route: DFT + "
                         f"per-mode Pade-13 exponential of the source-augmented system), {spent:.1f} s"}

    line = {
        "metric": "Paraexp exp-action solves/s + HBM GB/s, mixed vs FP64 at 1e-7 rel L2",
        "value": main_run["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32basis",
        "data": "synthetic",
        "config": {"workload": f"c2_advection_diffusion_n{args.n}_krylov60_s256_nout32"
                               + ("_shift_invert" if args.krylov == "sai" else "_polynomial")
                               + (f"_paraexp{P}" if P > 1 else "")
                               + (f"_batch{len(probs)}" if len(probs) > 1 else ""), "n": args.n, "batch": len(probs),
                   "windows": P,
                   "krylov_steps": prob.krylov_steps, "samples": prob.s, "n_out": len(prob.t_out),
                   "krylov": "shift_invert" if args.krylov == "sai" else "polynomial",
                   "precision": args.precision},
        "rel_l2_vs_oracle": err,
        "report": rep,
        "tiles": tiles,
        "roofline": roof,
        "kernels": kernels,
        "batch": batch,
        "compare": compare,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
