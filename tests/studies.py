"""Accuracy studies of the HIP path against the FP64 oracle (test
infrastructure, like the rest of this folder; not collected by pytest):

    python tests/studies.py --precision   FP16 against FP32 storage of the
                                          measured modulus at 512^2
    python tests/studies.py --plain-128   the plain method at 128^2, device
                                          run against the oracle's run

Each prints one JSON line.  Inputs, schedules and timing helpers are the
benchmark's (bench.py at the repository root).
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from bench import (CACHE_BUDGET, HBM_PEAK_GBS, J, J_ER, J_EVAL, N, P, R,  # noqa: E402
                   make_inputs, mpr_params)


# ---------------------------------------------------------------------------
# Precision: FP16 against FP32 storage of the measured modulus
# ---------------------------------------------------------------------------
def precision_study(ctx, B, generations=20, sample=4):
    """512^2 clustered-sphere shot, P = 64 sphere starts.  For each storage:
    the error against the FP64 oracle (exact modulus) of one RAAR step, of 20
    ER iterations and of their Eq. error_calc fitness on `sample` members;
    steady-state RAAR-only and ER-only throughput (64 members, 2000
    iterations, no shrink-wrap); the throughput of MPR generations; and a full MPR run (`generations` x 100
    iterations) whose final best density and fitness are compared between the
    two storages, beside the divergence of two FP32 runs whose starts differ by
    FP32 rounding (how far any FP32 evaluation can drift on this trajectory)."""
    from oracle import mpr
    sh0, rho0, supp0 = make_inputs()
    M = mpr.to_fft_order(sh0["amp"].astype(np.float32).astype(np.float64))
    known = mpr.to_fft_order(sh0["mask"])
    S = supp0.astype(bool)
    x0 = rho0.astype(np.complex128)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    ref_raar = [mpr.raar(x0[p], S, M, known, 0.5, 0.9) for p in range(sample)]
    ref_er = [mpr.sequence(x0[p], S, M, known, 0.5, "HIO", 0.9, 0, 20) for p in range(sample)]
    ref_e = [mpr.get_error(x, S, M, known) for x in ref_er]
    out = {"workload": "512x512 clustered spheres (1e8 photons, 24x24 beamstop, 4-px gap), P=64 sphere starts",
           "sample_members": sample}
    finals = {}
    for name, fp16 in (("fp32", False), ("fp16", True)):
        shot = ctx.shot(sh0["amp"].astype(np.float32), sh0["mask"].astype(np.uint8), fp16=fp16)
        rec = {}
        pop = shot.population(rho0[:sample], supp0)
        pop.run(B.sched_ops([B.op(B.OP_RAAR, count=1, beta=0.9, chi=0.5)], ctx))
        rho, _, _ = pop.read()
        rec["raar_step_rel_l2_max"] = max(rel(rho[p], ref_raar[p]) for p in range(sample))
        pop.close()
        pop = shot.population(rho0[:sample], supp0)
        pop.run(B.sched_ops([B.op(B.OP_ER, count=20, chi=0.5), B.op(B.OP_GET_ERROR)], ctx))
        rho, _, err = pop.read()
        rec["er20_rel_l2_max"] = max(rel(rho[p], ref_er[p]) for p in range(sample))
        rec["er20_fitness_rel_max"] = max(abs(err[p] - ref_e[p]) / ref_e[p] for p in range(sample))
        pop.close()
        # steady-state microbenchmarks: RAAR-only and ER-only, 64 members, no
        # shrink-wrap, 2000 iterations (one launch chunk: the two work buffers
        # fit the memory-side cache)
        pop = shot.population(rho0[:64], supp0)
        b_m = 2.0 if fp16 else 4.0
        for alg, op, bpp in (("raar", B.OP_RAAR, 40.125), ("er", B.OP_ER, 32.125)):
            pop.run(B.sched_ops([B.op(op, count=20, beta=0.9, chi=0.5)], ctx))
            pop.sync()
            t0 = time.perf_counter()
            pop.run(B.sched_ops([B.op(op, count=2000, beta=0.9, chi=0.5)], ctx))
            pop.sync()
            dt = time.perf_counter() - t0
            mit = 64 * 2000 / dt
            rec[f"{alg}2000_member_iterations_per_s"] = mit
            rec[f"{alg}2000_pct_hbm_peak"] = mit * (bpp + b_m / 64) * N * N / (HBM_PEAK_GBS * 1e9)
        pop.close()
        # full MPR run from the same starts
        runs = [("main", rho0)]
        if not fp16:
            rng = np.random.default_rng(77)
            eps = np.finfo(np.float32).eps * np.abs(rho0).max()
            pert = (rho0 + eps * (rng.standard_normal(rho0.shape) + 1j * rng.standard_normal(rho0.shape))
                    ).astype(np.complex64)
            runs.append(("perturbed", pert))
        for tag, start in runs:
            pop = shot.population(start, supp0, memetic=True, seed=3004)
            G = generations
            scheds = [B.sched_mpr(ctx, **mpr_params(g, G, g == 1)) for g in range(1, G + 1)]
            t0 = time.perf_counter()
            for sc in scheds:
                pop.run(sc)
            pop.sync()
            dt = time.perf_counter() - t0
            rho, supp, err = pop.read()
            b = int(np.argmin(err))
            finals[(name, tag)] = (rho[b], float(err[b]))
            if tag == "main":
                rec["mpr_member_iterations_per_s"] = 2 * P * (R * (J + J_ER) + J_EVAL) * G / dt
                rec["mpr_best_fitness"] = float(err[b])
            pop.close()
        shot.close()
        out[name] = rec
    a32, e32 = finals[("fp32", "main")]
    a16, e16 = finals[("fp16", "main")]
    ap, ep = finals[("fp32", "perturbed")]
    out["mpr_generations"] = generations
    out["mpr_final_best_rel_l2_fp16_vs_fp32"] = rel(a16, a32)
    out["mpr_final_best_fitness_rel_fp16_vs_fp32"] = abs(e16 - e32) / e32
    out["mpr_final_best_rel_l2_fp32_perturbed_vs_fp32"] = rel(ap, a32)
    out["mpr_final_best_fitness_rel_fp32_perturbed_vs_fp32"] = abs(ep - e32) / e32
    return out


def plain_128_study(ctx, B):
    """128^2, five ellipses in a 40-px disk, 1e6 photons, 8x8 beamstop, P = 8
    random-phase starts (seed 2001), centred 48 x 48 start support; 10 blocks
    of HIO^j ER^(20-j) (j 16 -> 0, beta 0.9) with shrink-wrap (sigma 2 -> 1,
    tau 0.10) and a final GetError.  FP32 device run against the FP64 oracle
    run of the same schedule from the same start, beside the oracle's own
    divergence under an FP32-rounding perturbation of the start."""
    import torch
    from oracle import mpr
    from paper_2409_07413_amd import synth
    n, P, seed = 128, 8, 2001
    sh0 = synth.shot(n, "ellipses", 1001, 1e6, beamstop=8)
    amp = sh0["amp"].astype(np.float32)
    mask = sh0["mask"].astype(np.uint8)
    S0 = synth.centred_square(n, 48)
    sched = B.sched_plain(ctx, alg=B.ALG_HIO, G=10, j=16, j_er=4, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                          sigma_end=1.0, tau=0.10, tau_end=0.10)
    shot = ctx.shot(amp, mask)
    pop = shot.population(None, S0.astype(np.uint8), seed=seed, P=P)
    x0 = pop.read()[0].astype(np.complex128)
    stream = torch.cuda.Stream()
    reps = 20
    pops = [shot.population(None, S0.astype(np.uint8), seed=seed, P=P) for _ in range(reps)]
    pops[0].run(sched, stream)
    pops[0].sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in pops[1:]:
        q.run(sched, stream)
    torch.cuda.synchronize()
    gpu_s = (time.perf_counter() - t0) / (reps - 1)
    rho, supp, err = pops[0].read()
    for q in pops:
        q.close()
    pop.close()
    shot.close()
    sched.close()
    M = mpr.to_fft_order(amp.astype(np.float64))
    known = mpr.to_fft_order(sh0["mask"])
    prm = dict(alg="HIO", beta=0.9, chi=0.5, G=10, j=16, j_er=4, j_end=0, sigma=2.0, sigma_end=1.0,
               tau=0.10, tau_end=0.10)
    t0 = time.perf_counter()
    ref = mpr.run_plain(M, known, x0, S0, prm)
    cpu_s = time.perf_counter() - t0
    rng = np.random.default_rng(5)
    eps = np.finfo(np.float32).eps * np.abs(x0).max()
    pert = mpr.run_plain(M, known, x0 + eps * (rng.standard_normal(x0.shape) + 1j * rng.standard_normal(x0.shape)),
                         S0, prm)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    Eref = np.array(ref["E"])
    return {"n": n, "P": P, "iterations": 200,
            "gpu_ms_per_run": gpu_s * 1e3, "gpu_member_iterations_per_s": P * 200 / gpu_s,
            "oracle_s_per_run": cpu_s, "oracle_cores": 1,
            "best_gpu": int(np.argmin(err)), "best_oracle": int(np.argmin(Eref)),
            "fitness_gpu": [float(e) for e in err], "fitness_oracle": [float(e) for e in Eref],
            "density_rel_l2_gpu_vs_oracle": [rel(rho[p], ref["x"][p]) for p in range(P)],
            "density_rel_l2_oracle_perturbed_vs_oracle": [rel(pert["x"][p], ref["x"][p]) for p in range(P)],
            "support_mismatch_px_gpu_vs_oracle": [int((supp[p] != ref["S"][p]).sum()) for p in range(P)]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--precision", action="store_true", help="FP16 against FP32 modulus storage at 512^2")
    ap.add_argument("--plain-128", action="store_true", help="the plain method at 128^2 against the oracle")
    ap.add_argument("--variant", type=int, default=0,
                    help="kernel variant of the 128^2 study (1: the resident Sequence)")
    args = ap.parse_args()
    if not (args.precision or args.plain_128):
        ap.error("choose --precision or --plain-128")
    import torch  # noqa: F401
    from paper_2409_07413_amd import binding as B
    ctx = B.Context(0)
    ctx.set_cache_budget(CACHE_BUDGET)
    if args.precision:
        print(json.dumps({"precision": precision_study(ctx, B)}), flush=True)
    else:
        ctx.set_variant(128, args.variant)
        print(json.dumps({"plain_128": {"variant": args.variant, **plain_128_study(ctx, B)}}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
