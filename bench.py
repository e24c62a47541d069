"""Benchmark of the MPR hot path on one MI355X.

Workload (the headline configuration): 512 x 512 detector, clustered projected
spheres (150-px extent), 1e8 photons with Poisson noise, 24 x 24 beamstop plus
a 4-px horizontal gap; P = 64 parents (128 members with the children); the MPR
generation schedule of Alg. mpr / Alg. improve with RAAR (beta 0.9), R = 3
sequences of 20 iterations plus 40 ER evaluation iterations, i.e. 100
member-iterations per member per generation, shrink-wrap sigma 2 -> 0.5,
tau 0.10 -> 2/3 tau, crossover C_p 0.6, C_w 0.4, tiles 4..64.

One step = one full generation (crossover, statistics, self-improvement of all
128 members with shrink-wrap / support-area updates and fitness, selection).
Inputs are resident in HBM before timing starts.

Prints one JSON line: member-iterations/s, the roofline of the dominant kernel
(algorithmic bytes per launch / average launch time from HIP events on the
launch stream) and the FP64 oracle timed on the host cores on a bounded sample.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
N, P = 512, 64
R, J, J_ER, J_EVAL = 3, 16, 4, 40
G_SCHEDULE = 20
CACHE_BUDGET = 256 << 20  # the library default: the 256 MiB memory-side cache


def make_inputs():
    from paper_2409_07413_amd import synth
    sh = synth.shot(N, "spheres", 1004, 1e8, beamstop=24, gap=4)
    rho0 = synth.sphere_starts(sh["amp"], sh["mask"], P, 2004, sigma_init=180)
    supp0 = synth.centred_square(N, 180).astype(np.uint8)
    return sh, rho0.astype(np.complex64), supp0


def mpr_params(g, G, init):
    return dict(alg=2, G=G, R=R, j=J, j_er=J_ER, j_end=0, j_eval=J_EVAL, t_min=4, t_max=N // 8,
                gen_first=g, gen_count=1, init_error=1 if init else 0, beta=0.9, chi=0.5,
                sigma=2.0, sigma_end=0.5, tau=0.10, tau_end=0.10 * 2.0 / 3.0, c_p=0.6, c_w=0.4)


def algorithmic_bytes_per_px(kernel, members_sharing_m):
    """Bytes the method must move per pixel per launch of each iteration kernel.

    col_proj: read rowFFT(x) 8 + write rowFFT(P_M x) 8, plus the measured modulus
    (4 B) read once per launch for all members.  row_update (HIO/RAAR): read
    rowFFT(P_M x) 8 + rowFFT(x) 8 + support bits 1/8, write 8.  row_update (ER):
    read 8 + support 1/8, write 8.
    """
    if kernel == 1:
        return 16.0 + 4.0 / members_sharing_m
    if kernel == 3:
        return 24.125
    if kernel == 2:
        return 16.125
    return 16.125


def kernel_sources_digest():
    """Digest of the sources that define the iteration kernels, their launch
    configuration and their arguments."""
    import hashlib
    h = hashlib.sha256()
    for f in ("fft.hpp", "kernels_n.hip", "common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2409_07413_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def member_chunk(members, n=None, budget=CACHE_BUDGET):
    """The library's member-chunk rule for `members` members of an n x n shot
    (default: the benchmark's): one launch while their work buffers fit the
    budget, else launches of as many members as three quarters of it hold, the
    last one with the rest; returns (members per launch, mean members per
    launch)."""
    n = N if n is None else n
    per = 2 * n * n * 8
    chunk = members if members * per <= budget else min(members, max(1, budget // 4 * 3 // per))
    return chunk, members / -(-members // chunk)


def measured_traffic(kernel, chunk):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE measurement (copy-kernel calibrated, averaged over
    the kernel's launches in the measured generation), or None when the
    kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_512_pop64.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    if t.get("sources_digest") != kernel_sources_digest() or t.get("members_per_launch") != chunk:
        return None
    return t.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")


def trace_averages(chunk):
    """Average kernel durations (us) of the loop kernels from the committed
    rocprofv3 kernel trace of the benchmark (profiles/kernel_trace_512_pop64.json),
    or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "kernel_trace_512_pop64.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    if t.get("sources_digest") != kernel_sources_digest() or t.get("members_per_launch") != chunk:
        return None
    return {k: v.get("avg_us") for k, v in t.get("kernels", {}).items()}




def gpu_step_check(ctx, B, amp, mask, rho, supp):
    """The library's RAAR step (beta 0.9, chi 0.5) and ER step with the fitness
    after it, from given states of one shot: the device side of the oracle
    check (a fresh population per step; nothing else runs on it)."""
    shot = ctx.shot(amp, mask)
    pop = shot.population(rho, supp)
    pop.run(B.sched_ops([B.op(B.OP_RAAR, count=1, beta=0.9, chi=0.5)], ctx))
    raar, _, _ = pop.read()
    pop.close()
    pop = shot.population(rho, supp)
    pop.run(B.sched_ops([B.op(B.OP_ER, count=1, chi=0.5), B.op(B.OP_GET_ERROR)], ctx))
    er, _, err = pop.read()
    pop.close()
    shot.close()
    return {"amp": amp, "mask": mask, "rho": rho, "supp": supp, "raar": raar, "er": er, "err": err}


def _oracle_timed(a):
    """Worker: k RAAR then k ER oracle iterations on one member; seconds."""
    from oracle import mpr
    x, S, M, known, k = a
    t0 = time.perf_counter()
    mpr.sequence(x.astype(np.complex128), S, M, known, 0.5, "RAAR", 0.9, k, 0)
    mpr.sequence(x.astype(np.complex128), S, M, known, 0.5, "RAAR", 0.9, 0, k)
    return time.perf_counter() - t0


def _oracle_check(a):
    """Worker: one member's oracle RAAR step, ER step and fitness, against the
    device's; relative L2 errors and the fitness's relative error."""
    from oracle import mpr
    x, S, M, known, g_raar, g_er, g_err = a
    x = x.astype(np.complex128)
    ref_raar = mpr.raar(x, S, M, known, 0.5, 0.9)
    ref_er = mpr.er(x, S, M, known, 0.5)
    ref_e = mpr.get_error(ref_er, S, M, known)

    def rel(u, v):
        return float(np.linalg.norm(u - v) / np.linalg.norm(v))
    return rel(g_raar, ref_raar), rel(g_er, ref_er), abs(g_err - ref_e) / ref_e


def oracle_pool():
    """Worker processes for the oracle leg, started before this process
    initialises the GPU (they never touch it)."""
    import multiprocessing as mp
    workers = max(1, len(os.sched_getaffinity(0)))
    return mp.get_context("spawn").Pool(workers), workers


def cpu_baseline(states, checks, pool, workers, seconds_target=20.0):
    """The FP64 oracle on the host cores (reported, not the target), plus the
    device's error against it.

    Timing: k RAAR then k ER iterations on each of the benchmark's 64 parent
    states (after the timed generations), one process per member over one
    worker per core the process may run on; k is chosen so that the whole
    sample is about `seconds_target` of CPU work.  Also the
    single-core rate of one member.  Checks: for each (shot, states, device
    step results), the oracle's RAAR and ER steps and fitness from the same
    states (`gpu_step_check`)."""
    from oracle import mpr
    amp, mask, rho, supp = states
    M = mpr.to_fft_order(amp.astype(np.float64))
    known = mpr.to_fft_order(mask.astype(bool))
    affinity = len(os.sched_getaffinity(0))
    members = rho.shape[0]
    # single core: one member, one RAAR and one ER iteration (also calibrates k)
    t_one = _oracle_timed((rho[0], supp[0], M, known, 1))
    single = 2.0 / t_one
    k = int(max(1, min(20, round(seconds_target / (2 * members * (t_one / 2))))))
    t0 = time.perf_counter()
    pool.map(_oracle_timed, [(rho[p], supp[p], M, known, k) for p in range(members)])
    wall = time.perf_counter() - t0
    jobs, tags = [], []
    for c in checks:
        Mc = mpr.to_fft_order(c["amp"].astype(np.float64))
        kc = mpr.to_fft_order(c["mask"].astype(bool))
        for p in range(c["rho"].shape[0]):
            jobs.append((c["rho"][p], c["supp"][p], Mc, kc, c["raar"][p], c["er"][p], float(c["err"][p])))
            tags.append(c["tag"])
    res = pool.map(_oracle_check, jobs)
    check = {}
    for tag, (r1, r2, r3) in zip(tags, res):
        d = check.setdefault(tag, {"members": 0, "raar_step_rel_l2_max": 0.0, "er_step_rel_l2_max": 0.0,
                                   "fitness_rel_max": 0.0})
        d["members"] += 1
        d["raar_step_rel_l2_max"] = max(d["raar_step_rel_l2_max"], r1)
        d["er_step_rel_l2_max"] = max(d["er_step_rel_l2_max"], r2)
        d["fitness_rel_max"] = max(d["fitness_rel_max"], r3)
    base = {"value": members * 2 * k / wall, "unit": "member-iterations/s", "cores": workers, "kind": "oracle",
            "sample": f"{members} parent states of the benchmark population after the timed generations, "
                      f"{k} RAAR (beta 0.9, chi 0.5) then {k} ER iterations each at {rho.shape[1]}x{rho.shape[1]}, "
                      f"FP64 NumPy oracle, one process per member over {workers} host cores",
            "single_core_value": single, "cpu_count": os.cpu_count(), "affinity": affinity,
            "seconds": wall}
    return base, check


# ---------------------------------------------------------------------------
# Serving: streamed single shots of mixed sizes (Poisson arrivals)
# ---------------------------------------------------------------------------
SERVE_SIZES = (256, 384, 512, 768, 1024)
SERVE_P = 32
SERVE_G = 25          # 25 blocks of 20 iterations = 500 per member
SERVE_POOL = 3        # distinct synthetic shots per size, drawn at random per arrival


def serve_sched(B, ctx):
    """Per shot: 25 blocks of HIO (beta 0.9)^j then ER^(20-j), j 16 -> 0, each
    followed by shrink-wrap (sigma 2 -> 1, tau 0.10); GetError at the end."""
    return B.sched_plain(ctx, alg=B.ALG_HIO, G=SERVE_G, j=16, j_er=4, j_end=0, beta=0.9, chi=0.5,
                         sigma=2.0, sigma_end=1.0, tau=0.10, tau_end=0.10)


def serving_pool():
    """5 ellipses (semi-axes 4-15 px) in a 40-px disk, 1e6 photons, 8x8 beamstop;
    start support a centred 48 x 48 square; random-phase starts on the device."""
    from paper_2409_07413_amd import synth
    pool, supp = {}, {}
    for n in SERVE_SIZES:
        pool[n] = []
        for k in range(SERVE_POOL):
            sh = synth.shot(n, "ellipses", 1005 + 101 * k + n, 1e6, beamstop=8, gap=0)
            pool[n].append((sh["amp"].astype(np.float32), sh["mask"].astype(np.uint8)))
        supp[n] = synth.centred_square(n, 48).astype(np.uint8)
    return pool, supp


def serving_stream(rate, count, seed=4005):
    rng = np.random.default_rng([seed, int(round(rate * 1000)), count])
    gaps = rng.exponential(1.0 / rate, size=count)
    gaps[0] = 0.0
    return np.cumsum(gaps), rng.choice(SERVE_SIZES, size=count), rng.integers(0, SERVE_POOL, size=count)


def _latency_summary(lat, first_arrival, finishes, count, member_px):
    lat = np.asarray(lat)
    span = max(finishes) - first_arrival
    return {"shots": count, "shots_per_s": count / span, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3), "makespan_s": span,
            "member_iterations_per_s": SERVE_P * 20 * SERVE_G * count / span,
            "iteration_pixels_per_s": SERVE_P * 20 * SERVE_G * member_px / span}


def run_served(ctx, B, pool, supp, stream, max_shots, budget, warm=True, shortest=False):
    """Served form: continuous batching in the library's engine thread."""
    arrivals, sizes, picks = stream
    sched = serve_sched(B, ctx)
    sv = B.Server(ctx, sched, P=SERVE_P, hbm_budget=budget, max_shots=max_shots, shortest_first=shortest)
    if warm:  # one shot of every size through the engine first (pinned pool, kernels)
        ts = [sv.submit(pool[n][0][0], pool[n][0][1], supp[n], seed=1) for n in SERVE_SIZES]
        sv.drain(300.0)
        for t in ts:
            sv.poll(t, want_data=False)
    off = sv.stats()["now"] - time.perf_counter()
    t0 = time.perf_counter() + 0.02
    tickets = []
    for i, (a, n, k) in enumerate(zip(arrivals, sizes, picks)):
        target = t0 + a
        d = target - time.perf_counter()
        if d > 0:
            time.sleep(d)
        amp, mask = pool[int(n)][int(k)]
        tickets.append(sv.submit(amp, mask, supp[int(n)], seed=5000 + i, arrival=target + off))
    if not sv.drain(600.0):
        raise RuntimeError("served stream did not finish")
    last = {int(n): i for i, n in enumerate(sizes)}  # the last shot of every size keeps its data
    res = [sv.poll(t, want_data=(last.get(int(n)) == i)) for i, (t, n) in enumerate(zip(tickets, sizes))]
    st = sv.stats()
    sv.close()
    sched.close()
    samples = [(int(sizes[i]), int(picks[i]), res[i]["rho"], res[i]["supp"]) for i in sorted(last.values())]
    lat = [r["t_finish"] - r["t_arrival"] for r in res]
    out = _latency_summary(lat, min(r["t_arrival"] for r in res), [r["t_finish"] for r in res], len(res),
                           float(sum(int(n) ** 2 for n in sizes)))
    out.update({"max_resident": st["max_active"], "ticks": st["ticks"], "launches": st["launches"],
                "peak_shot_bytes": st["bytes_peak"], "max_shots": max_shots,
                "policy": "shortest-first" if shortest else "all"})
    out["_samples"] = samples
    return out


def run_plain_fifo(ctx, B, pool, supp, stream, warm=True):
    """Comparator: one shot at a time in arrival order (FIFO), the same kernels
    through spr_run, a fresh shot and population per request, no batching."""
    arrivals, sizes, picks = stream
    sched = serve_sched(B, ctx)

    def one(n, amp, mask, seed):
        sh = ctx.shot(amp, mask)
        pop = sh.population(None, supp[n], seed=seed, P=SERVE_P)
        pop.run(sched)
        err = pop.errors()
        pop.read_member(int(np.argmin(err)))
        pop.close()
        sh.close()

    if warm:
        for n in SERVE_SIZES:
            one(n, pool[n][0][0], pool[n][0][1], 1)
    t0 = time.perf_counter() + 0.02
    lat, fin = [], []
    for i, (a, n, k) in enumerate(zip(arrivals, sizes, picks)):
        target = t0 + a
        d = target - time.perf_counter()
        if d > 0:
            time.sleep(d)
        amp, mask = pool[int(n)][int(k)]
        one(int(n), amp, mask, 5000 + i)
        f = time.perf_counter()
        lat.append(f - target)
        fin.append(f - t0)
    sched.close()
    return _latency_summary(lat, 0.0, fin, len(lat), float(sum(int(n) ** 2 for n in sizes)))


def serving_leg(ctx, B, rates, count, max_shots, budget, forms=("served", "plain"), log=None, shortest=False,
                tune=True):
    """Both forms run on the same context, so with `tune` both use the kernel
    variant the run-time tuner picks per size (for the resident member count)."""
    pool, supp = serving_pool()
    if tune:
        for n in SERVE_SIZES:
            ctx.autotune(int(n), SERVE_P * max_shots)
    out = []
    for rate, cnt in zip(rates, count):
        stream = serving_stream(rate, cnt)
        rec = {"rate_per_s": rate}
        for form in forms:
            if form == "served":
                rec["served"] = run_served(ctx, B, pool, supp, stream, max_shots, budget, shortest=shortest)
            else:
                rec["plain"] = run_plain_fifo(ctx, B, pool, supp, stream)
            if log:
                log(f"serving rate {rate}/s, {cnt} shots, {form}: "
                    + json.dumps({k: round(v, 3) for k, v in rec[form].items() if isinstance(v, float)}))
        out.append(rec)
    return out


def served_checks(ctx, B, srv):
    """Device steps from the served results kept by the serving leg (the best
    member of the last shot of every size at the first rate) for the oracle
    check; removes the kept data from the records."""
    pool, _ = serving_pool()
    checks = []
    for rec in srv:
        samples = rec.get("served", {}).pop("_samples", None)
        if samples and not checks:
            for n, k, rho, supp in samples:
                amp, mask = pool[n][k]
                c = gpu_step_check(ctx, B, amp, mask, rho, supp.astype(np.uint8))
                c["tag"] = "served"
                checks.append(c)
    return checks


# ---------------------------------------------------------------------------
# Iteration kernels by detector size; captured versus eager schedules
# ---------------------------------------------------------------------------
SIZE_SWEEP = ((256, 128), (384, 64), (512, 64), (512, 128), (768, 28), (768, 64), (1024, 16), (1024, 64))


def size_sweep(ctx, B, iters=20):
    """Per size: RAAR^iters then ER^iters on `members` random members, one
    launch chunk (the member count is the chunk), every iteration kernel
    timed with HIP events; GB/s from the algorithmic bytes per launch."""
    import torch  # noqa: F401
    rng = np.random.default_rng(0)
    out = []
    for n, members in SIZE_SWEEP:
        amp = np.abs(rng.standard_normal((n, n))).astype(np.float32)
        from paper_2409_07413_amd import synth
        mask = synth.beamstop_gap_mask(n, 24, 4).astype(np.uint8)
        rho = (rng.standard_normal((members, n, n)) + 1j * rng.standard_normal((members, n, n))).astype(np.complex64)
        supp = synth.centred_square(n, n // 3).astype(np.uint8)
        ctx.set_cache_budget(members * 2 * n * n * 8)
        shot = ctx.shot(amp, mask)
        pop = shot.population(rho, supp)
        s = B.sched_ops([B.op(B.OP_RAAR, count=iters, beta=0.9), B.op(B.OP_ER, count=iters)], ctx)
        pop.run(s)
        pop.sync()
        pop.timing(True)
        for _ in range(3):
            pop.run(s)
        pop.sync()
        rec = {"n": n, "members_per_launch": members,
               "resident_bytes": members * 2 * n * n * 8}
        for k in range(4):
            nl, ms = pop.timing_read(k)
            if nl:
                us = ms / nl * 1e3
                rec[B.KERNEL_NAMES[k]] = {"avg_us": round(us, 2), "GBps": round(
                    algorithmic_bytes_per_px(k, members) * n * n * members / (us * 1e-6) / 1e9, 1)}
        out.append(rec)
        pop.close()
        shot.close()
        s.close()
    ctx.set_cache_budget(CACHE_BUDGET)
    return out


def steady_loop(ctx, B, n, members, iters, variant=0):
    """One warm-up pass and one timed pass of RAAR^iters then ER^iters on
    `members` random members of a synthetic N x N shot (24 x 24 beamstop,
    4-px gap), all members in one launch chunk: the launches a kernel profile
    of the projection loop is taken over."""
    import torch
    from paper_2409_07413_amd import synth
    rng = np.random.default_rng(0)
    amp = np.abs(rng.standard_normal((n, n))).astype(np.float32)
    mask = synth.beamstop_gap_mask(n, 24, 4).astype(np.uint8)
    rho = (rng.standard_normal((members, n, n)) + 1j * rng.standard_normal((members, n, n))).astype(np.complex64)
    supp = synth.centred_square(n, n // 3).astype(np.uint8)
    ctx.set_cache_budget(members * 2 * n * n * 8)
    ctx.set_variant(n, variant)
    shot = ctx.shot(amp, mask)
    pop = shot.population(rho, supp)
    s = B.sched_ops([B.op(B.OP_RAAR, count=iters, beta=0.9), B.op(B.OP_ER, count=iters)], ctx)
    stream = torch.cuda.Stream()
    pop.run(s, stream)
    pop.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    pop.run(s, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    pop.close()
    shot.close()
    s.close()
    ctx.set_variant(n, 0)
    ctx.set_cache_budget(CACHE_BUDGET)
    return {"n": n, "members": members, "iterations": 2 * iters, "variant": variant,
            "ms": ms, "member_iterations_per_s": members * 2 * iters / (ms * 1e-3)}


def graph_study(ctx, B, passes=10):
    """The plain schedule (10 blocks of HIO^j ER^(20-j), shrink-wrap each) run
    eagerly and replayed from a captured graph on twin populations."""
    import torch
    from paper_2409_07413_amd import synth
    out = []
    for n, P in ((128, 8), (256, 32), (512, 64)):
        sh0 = synth.shot(n, "ellipses", 1001, 1e6, beamstop=8)
        shot = ctx.shot(sh0["amp"].astype(np.float32), sh0["mask"].astype(np.uint8))
        supp = synth.centred_square(n, 48).astype(np.uint8)
        s = B.sched_plain(ctx, alg=B.ALG_HIO, G=10, j=16, j_er=4, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                          sigma_end=1.0, tau=0.1, tau_end=0.1)
        pa = shot.population(None, supp, seed=1, P=P)
        pb = shot.population(None, supp, seed=1, P=P)
        g = pb.graph(s)
        stream = torch.cuda.Stream()
        for _ in range(2):
            pa.run(s, stream)
            g.launch(stream)
        rec = {"n": n, "P": P}
        for tag, fn in (("eager", lambda: pa.run(s, stream)), ("graph", lambda: g.launch(stream))):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(passes):
                fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / passes
            rec[tag + "_ms_per_200_iterations"] = dt * 1e3
            rec[tag + "_member_iterations_per_s"] = P * 200 / dt
        ra, rb = pa.read(), pb.read()
        rec["bit_equal"] = bool(all(np.array_equal(u, v) for u, v in zip(ra, rb)))
        out.append(rec)
        g.close()
        pa.close()
        pb.close()
        shot.close()
        s.close()
    return out


# ---------------------------------------------------------------------------
# Batched uneven shots: autotuned kernels, one launch per size and step
# ---------------------------------------------------------------------------
def batch_study(ctx, B, shots=32, P_batch=32, G=50):
    """32 shots of sizes drawn from {256,...,1024}, P = 32 each, 1000 iterations
    (50 blocks of HIO^j ER^(20-j) with shrink-wrap) + GetError: (1) one
    population at a time (spr_run), (2) all shots in one batch (spr_run_batch:
    members of one size share every launch), (3) the batch replayed from a
    captured graph; kernels and member chunks tuned per size first."""
    import torch  # noqa: F401
    from paper_2409_07413_amd import synth
    rng = np.random.default_rng(1003)
    sizes = rng.choice(SERVE_SIZES, size=shots)
    photons = 10.0 ** rng.uniform(6.0, 8.0, size=shots)
    tuning = {int(n): ctx.autotune(int(n), P_batch * int((sizes == n).sum())) for n in sorted(set(sizes))}
    data = []
    for i, (n, ph) in enumerate(zip(sizes, photons)):
        sh = synth.shot(int(n), "ellipses", 1003 + 7 * i, float(ph), beamstop=8)
        data.append((int(n), sh["amp"].astype(np.float32), sh["mask"].astype(np.uint8)))
    supp = {n: synth.centred_square(n, 48).astype(np.uint8) for n in SERVE_SIZES}

    def make():
        out = []
        for i, (n, amp, mask) in enumerate(data):
            shot = ctx.shot(amp, mask)
            out.append((shot, shot.population(None, supp[n], seed=9000 + i, P=P_batch)))
        return out

    sched = B.sched_plain(ctx, alg=B.ALG_HIO, G=G, j=16, j_er=4, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                          sigma_end=1.0, tau=0.10, tau_end=0.10)
    member_its = shots * P_batch * 20 * G
    px_its = sum(n * n for n, _, _ in data) * P_batch * 20 * G
    res = {"shots": shots, "P": P_batch, "iterations": 20 * G, "sizes": [int(n) for n in sizes],
           "tuning": {str(k): {"variant": v["variant"], "chunk_members": v["chunk_members"]} for k, v in tuning.items()}}
    import torch
    # (1) one population at a time
    pops = make()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _, pop in pops:
        pop.run(sched)
    for _, pop in pops:
        pop.sync()
    res["one_at_a_time_s"] = time.perf_counter() - t0
    first = [pop.errors() for _, pop in pops]
    for shot, pop in pops:
        pop.close()
        shot.close()
    # (2) one batch, eager
    pops = make()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run_batch([p for _, p in pops], [sched] * shots)
    for _, pop in pops:
        pop.sync()
    res["batch_s"] = time.perf_counter() - t0
    res["batch_equals_one_at_a_time"] = bool(all(np.array_equal(a, pop.errors()) for a, (_, pop) in zip(first, pops)))
    for shot, pop in pops:
        pop.close()
        shot.close()
    # (3) the batch from a captured graph
    pops = make()
    g = ctx.graph_batch([p for _, p in pops], [sched] * shots)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.launch()
    for _, pop in pops:
        pop.sync()
    res["graph_s"] = time.perf_counter() - t0
    res["graph_equals_one_at_a_time"] = bool(all(np.array_equal(a, pop.errors()) for a, (_, pop) in zip(first, pops)))
    g.close()
    for shot, pop in pops:
        pop.close()
        shot.close()
    sched.close()
    for k in ("one_at_a_time", "batch", "graph"):
        t = res[k + "_s"]
        res[k] = {"member_iterations_per_s": member_its / t, "iteration_pixels_per_s": px_its / t,
                  "pct_hbm_peak_iterations": px_its * 40.0 / t / (HBM_PEAK_GBS * 1e9)}
    res["small"] = small_batch_study(ctx, B)
    return res


def small_batch_study(ctx, B, shots=24, P_batch=8, G=10, reps=5):
    """Small uneven shots, whose launches cannot fill the device: 24 shots with
    sides drawn from {48, 64, 96, 128, 192}, P = 8, 200 iterations (10 blocks
    of HIO^j ER^(20-j) with shrink-wrap) + GetError; one population at a time
    against one batch, whose size groups overlap on the device, and against
    the same batch with the groups one after another (a cache budget below
    the groups' sum and above each group's work buffers)."""
    import torch
    from paper_2409_07413_amd import synth
    rng = np.random.default_rng(1103)
    sides = (48, 64, 96, 128, 192)
    sizes = rng.choice(sides, size=shots)
    data = []
    for i, n in enumerate(sizes):
        sh = synth.shot(int(n), "ellipses", 1103 + 7 * i, 1e6, beamstop=4, count=3,
                        semi=(0.03 * n, 0.1 * n), disk_diameter=0.3 * n)
        data.append((int(n), sh["amp"].astype(np.float32), sh["mask"].astype(np.uint8)))
    supp = {n: synth.centred_square(n, n // 3).astype(np.uint8) for n in sides}
    sched = B.sched_plain(ctx, alg=B.ALG_HIO, G=G, j=16, j_er=4, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                          sigma_end=1.0, tau=0.10, tau_end=0.10)

    def make():
        out = []
        for i, (n, amp, mask) in enumerate(data):
            shot = ctx.shot(amp, mask)
            out.append((shot, shot.population(None, supp[n], seed=9100 + i, P=P_batch)))
        return out

    res = {"shots": shots, "P": P_batch, "iterations": 20 * G, "sizes": [int(n) for n in sizes]}
    times = {}
    errs = {}
    serial_budget = 30 << 20  # above each group's 2 x chunk x n^2 x 8 bytes, below their sum
    for form in ("one_at_a_time", "batch", "batch_groups_serial"):
        ctx.set_cache_budget(serial_budget if form == "batch_groups_serial" else CACHE_BUDGET)
        pops = make()
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if form != "one_at_a_time":
                ctx.run_batch([p for _, p in pops], [sched] * shots)
            else:
                for _, pop in pops:
                    pop.run(sched)
            for _, pop in pops:
                pop.sync()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        times[form] = best
        for shot, pop in pops:
            pop.close()
            shot.close()
        # one more fresh run for the comparison of results
        pops = make()
        if form != "one_at_a_time":
            ctx.run_batch([p for _, p in pops], [sched] * shots)
        else:
            for _, pop in pops:
                pop.run(sched)
        errs[form] = [pop.errors() for _, pop in pops]
        for shot, pop in pops:
            pop.close()
            shot.close()
    ctx.set_cache_budget(CACHE_BUDGET)
    sched.close()
    member_its = shots * P_batch * 20 * G
    for form, t in times.items():
        res[form] = {"seconds": t, "member_iterations_per_s": member_its / t}
    res["batch_equals_one_at_a_time"] = bool(all(
        np.array_equal(a, b) and np.array_equal(a, c)
        for a, b, c in zip(errs["one_at_a_time"], errs["batch"], errs["batch_groups_serial"])))
    return res


# ---------------------------------------------------------------------------
# The other single-shot configurations
# ---------------------------------------------------------------------------
def mpr_1024_study(ctx, B, generations=20):
    """1024^2, twelve clustered spheres (150-px extent), 1e8 photons, 24x24
    beamstop and 4-px gap, P = 64 sphere starts (Sigma_init 180, seed 2002,
    Philox 3002); the MPR schedule (RAAR beta 0.9, R = 3 x 20 + 40 ER, sigma
    2 -> 0.5, tau 0.10 -> 2/3 tau, C_p 0.6, C_w 0.4, tiles 4..128) for all
    generations: 2P x 100 x G member-iterations."""
    import torch
    from paper_2409_07413_amd import synth
    n, P = 1024, 64
    tune = ctx.autotune(n, 2 * P)
    sh0 = synth.shot(n, "spheres", 1002, 1e8, beamstop=24, gap=4)
    rho0 = synth.sphere_starts(sh0["amp"], sh0["mask"], P, 2002, sigma_init=180).astype(np.complex64)
    supp0 = synth.centred_square(n, 180).astype(np.uint8)
    shot = ctx.shot(sh0["amp"].astype(np.float32), sh0["mask"].astype(np.uint8))
    pop = shot.population(rho0, supp0, memetic=True, seed=3002)
    G = generations
    prm = lambda g: dict(alg=2, G=G, R=R, j=J, j_er=J_ER, j_end=0, j_eval=J_EVAL, t_min=4, t_max=n // 8,  # noqa: E731
                         gen_first=g, gen_count=1, init_error=1 if g == 1 else 0, beta=0.9, chi=0.5,
                         sigma=2.0, sigma_end=0.5, tau=0.10, tau_end=0.10 * 2.0 / 3.0, c_p=0.6, c_w=0.4)
    scheds = [B.sched_mpr(ctx, **prm(g)) for g in range(1, G + 1)]
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sc in scheds:
        pop.run(sc, stream)
    pop.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = pop.stats()
    pop.close()
    shot.close()
    its = 2 * P * (R * (J + J_ER) + J_EVAL) * G
    return {"n": n, "P": P, "members": 2 * P, "generations": G, "tuning": {"variant": tune["variant"],
            "chunk_members": tune["chunk_members"]}, "seconds": dt, "member_iterations_per_s": its / dt,
            "iteration_pixels_per_s": its * n * n / dt,
            "pct_hbm_peak_iterations": its * n * n * 40.0 / dt / (HBM_PEAK_GBS * 1e9),
            "best_fitness_last": stats[-1].err_best if stats else None}


def copy_calibration():
    """A plain copy kernel of known size: 256 MiB read + 256 MiB written per
    launch (torch copy_, a hipMemcpy device-to-device kernel).  Its FETCH_SIZE /
    WRITE_SIZE readings calibrate the HBM counters; its bandwidth is the
    practical ceiling of a read+write sweep."""
    import torch
    n = 256 * (1 << 20) // 8
    a = torch.randn(n, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "avg_ms": ms,
                      "GBps_read_plus_write": 2 * n * 8 / (ms * 1e-3) / 1e9}), flush=True)


# ---------------------------------------------------------------------------
# Summaries of rocprofv3 outputs (kernel traces and counter collections)
# ---------------------------------------------------------------------------
def _rocprof_rows(d, kind):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", f"*_{kind}.csv"), recursive=True)):
        rows += list(csv.DictReader(open(f)))
    if not rows:
        raise SystemExit(f"no *_{kind}.csv under {d}")
    return rows


def _loop_kernel_key(name):
    """Kernel key of a loop kernel's demangled name, or None."""
    base = name.replace("void ", "").replace("spr::(anonymous namespace)::", "").split("(")[0]
    if base.startswith("k_col_proj"):
        return "k_col_proj"
    if base == "k_row_update<1>":
        return "k_row_update_er"
    if base.startswith("k_row_update<"):
        return "k_row_update_ia"
    if base == "k_row_ingest":
        return "k_row_ingest"
    if "copyBuffer" in base:
        return "copy"
    return None


def profile_summary(d):
    """profiles/kernel_trace_512_pop64.json and profiles/traffic_512_pop64.json
    from the rocprofv3 outputs of the benchmark under d: d/trace (kernel trace),
    d/fetch and d/write (FETCH_SIZE, WRITE_SIZE) of `bench.py --steps 2 --warmup
    1 --no-cpu-baseline --no-serve`, and d/fetch_cal, d/write_cal of `bench.py
    --copy-calibration` (256 MiB read + written per copy)."""
    chunk, per_launch = member_chunk(2 * P)
    digest = kernel_sources_digest()
    dur = {}
    for r in _rocprof_rows(os.path.join(d, "trace"), "kernel_trace"):
        k = _loop_kernel_key(r["Kernel_Name"])
        if k and k != "copy":
            dur.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    trace = {"workload": "bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-serve (512x512, 128 members, "
                         f"{chunk} per launch)", "members_per_launch": chunk, "sources_digest": digest,
             "kernels": {k: {"calls": len(v), "avg_us": float(np.mean(v)), "median_us": float(np.median(v))}
                         for k, v in sorted(dur.items())}}

    def counter(sub, name):
        vals = {}
        for r in _rocprof_rows(os.path.join(d, sub), "counter_collection"):
            if r["Counter_Name"] != name:
                continue
            k = _loop_kernel_key(r["Kernel_Name"])
            if k:
                vals.setdefault(k, []).append(float(r["Counter_Value"]))
        return vals
    fcal, wcal = counter("fetch_cal", "FETCH_SIZE")["copy"], counter("write_cal", "WRITE_SIZE")["copy"]
    copy_bytes = 256 << 20
    fetch_factor = copy_bytes / (max(fcal) * 1024)
    write_factor = copy_bytes / (max(wcal) * 1024)
    fetch, write = counter("fetch", "FETCH_SIZE"), counter("write", "WRITE_SIZE")
    alg = {"k_col_proj": algorithmic_bytes_per_px(1, per_launch),
           "k_row_update_er": algorithmic_bytes_per_px(2, per_launch),
           "k_row_update_ia": algorithmic_bytes_per_px(3, per_launch),
           "k_row_ingest": algorithmic_bytes_per_px(0, per_launch)}
    kern = {}
    for k in sorted(fetch):
        if k == "copy" or k not in write:
            continue
        f, w = float(np.mean(fetch[k])), float(np.mean(write[k]))
        hbm = (f * fetch_factor + w * write_factor) * 1024
        a = alg[k] * N * N * per_launch
        kern[k] = {"dispatches": len(fetch[k]), "FETCH_SIZE_KiB_avg": f, "WRITE_SIZE_KiB_avg": w,
                   "hbm_bytes_per_launch": hbm, "algorithmic_bytes_per_launch": a, "ratio_to_algorithmic": hbm / a}
    traffic = {"workload": trace["workload"], "members_per_launch": chunk, "sources_digest": digest,
               "copy_calibration": {"bytes_read": copy_bytes, "bytes_written": copy_bytes,
                                    "FETCH_SIZE_KiB": max(fcal), "WRITE_SIZE_KiB": max(wcal),
                                    "fetch_factor": fetch_factor, "write_factor": write_factor},
               "kernels": kern}
    for name, obj in (("kernel_trace_512_pop64.json", trace), ("traffic_512_pop64.json", traffic)):
        with open(os.path.join(ROOT, "profiles", name), "w") as fh:
            json.dump(obj, fh, indent=1)
    print(json.dumps({"trace": trace, "traffic": traffic}, indent=1))


def counter_summary(d, sizes=("512", "1024")):
    """Markdown table of the loop kernels' hardware counters from the passes
    under d (d/p1_<n> ... d/p4_<n>, `bench.py --loop` runs): VALU busy, VALU
    instructions per wave, mean resident waves per CU, LDS bank-conflict
    share, memory-unit busy and stalled, average L2 read latency."""
    rows = []
    for n in sizes:
        acc = {}
        for pss in ("p1", "p2", "p3", "p4"):
            for r in _rocprof_rows(os.path.join(d, f"{pss}_{n}"), "counter_collection"):
                k = _loop_kernel_key(r["Kernel_Name"])
                if k in (None, "copy", "k_row_ingest"):
                    continue
                acc.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        for k, c in sorted(acc.items()):
            m = {name: float(np.mean(v)) for name, v in c.items()}
            cus, ses, xcds = 256, 32, 8
            gui = m["GRBM_GUI_ACTIVE"] / xcds  # cycles of one XCD (the counter sums the 8)
            rows.append({
                "n": n, "kernel": k,
                "VALU busy %": 100 * m["SQ_ACTIVE_INST_VALU"] / cus / gui,
                "VALU instr per wave": m["SQ_INSTS_VALU"] / m["SQ_WAVES"],
                "waves per CU (mean)": m.get("MeanOccupancyPerCU", float("nan")),
                "LDS bank conflict %": 100 * m["SQ_LDS_BANK_CONFLICT"] / cus / gui,
                "LDS instr per wave": m["SQ_INSTS_LDS"] / m["SQ_WAVES"],
                "TA busy %": 100 * m["TA_TA_BUSY_sum"] / cus / gui,
                "TCP data stall %": 100 * m["TCP_TCP_TA_DATA_STALL_CYCLES_sum"] / cus / gui,
                "L2 read latency (cycles)": m["TCP_TCC_READ_REQ_LATENCY_sum"] / m["TCP_TCC_READ_REQ_sum"],
                "L2 read requests per wave": m["TCP_TCC_READ_REQ_sum"] / m["SQ_WAVES"],
                "vector memory instr per wave": (m["SQ_INSTS_VMEM_RD"] + m["SQ_INSTS_VMEM_WR"]) / m["SQ_WAVES"],
                "wait for dependencies % of wave time": 100 * m["SQ_WAIT_INST_ANY"] / m["SQ_WAVE_CYCLES"],
            })
    keys = list(rows[0].keys())
    print("| " + " | ".join(keys) + " |")
    print("|" + "---|" * len(keys))
    for r in rows:
        print("| " + " | ".join(f"{v:.1f}" if isinstance(v, float) else str(v) for v in r.values()) + " |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain device copy of 256 MiB (reference for HBM counters) and exit")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--timing-every", type=int, default=8,
                    help="inside the timed region, HIP events around one launch in every N of each loop kernel")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg (one JSON line per rate on stderr, summary on stdout)")
    ap.add_argument("--serve-rates", type=str, default="50,5",
                    help="Poisson arrival rates (shots/s) of the serving leg")
    ap.add_argument("--serve-shots", type=str, default="60,20", help="shots per rate")
    ap.add_argument("--serve-max-shots", type=int, default=8, help="shots resident at once in the server")
    ap.add_argument("--serve-budget-gib", type=float, default=48.0, help="device memory of the server")
    ap.add_argument("--serve-forms", type=str, default="served,plain")
    ap.add_argument("--serve-policy", choices=("shortest", "all"), default="shortest",
                    help="ticks advance the shots of the least remaining work first, or every resident shot")
    ap.add_argument("--serve-no-tune", action="store_true",
                    help="serve with each size's default kernel variant instead of the tuned one")
    ap.add_argument("--size-sweep", action="store_true",
                    help="time the iteration kernels at every served detector size and exit")
    ap.add_argument("--graph-study", action="store_true",
                    help="compare captured-graph replays with eager schedule runs and exit")
    ap.add_argument("--mpr-1024", action="store_true", help="1024^2 MPR run (20 generations) and exit")
    ap.add_argument("--batch-study", action="store_true",
                    help="32 uneven shots: one at a time, one batch, one captured batch (after tuning) and exit")
    ap.add_argument("--loop", type=str, default=None, metavar="N,MEMBERS,ITERS[,VARIANT]",
                    help="steady-state projection loop only (RAAR^ITERS then ER^ITERS on MEMBERS random members "
                         "of one N x N shot, one launch chunk), for kernel profiles, and exit")
    ap.add_argument("--profile-summary", type=str, default=None, metavar="DIR",
                    help="write profiles/kernel_trace_512_pop64.json and profiles/traffic_512_pop64.json from "
                         "rocprofv3 outputs under DIR (trace, fetch, write, fetch_cal, write_cal) and exit")
    ap.add_argument("--counter-summary", type=str, default=None, metavar="DIR",
                    help="print a table of the loop kernels' counters from rocprofv3 passes under DIR and exit")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(args.profile_summary)
        return
    if args.counter_summary:
        counter_summary(args.counter_summary)
        return
    if args.loop:
        import torch  # noqa: F401
        from paper_2409_07413_amd import binding as B
        v = [int(t) for t in args.loop.split(",")]
        ctx = B.Context(0)
        print(json.dumps({"loop": steady_loop(ctx, B, *v)}), flush=True)
        ctx.close()
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.mpr_1024:
        import torch  # noqa: F401
        from paper_2409_07413_amd import binding as B
        ctx = B.Context(0)
        ctx.set_cache_budget(CACHE_BUDGET)
        print(json.dumps({"mpr_1024": mpr_1024_study(ctx, B)}), flush=True)
        ctx.close()
        return
    if args.batch_study:
        import torch  # noqa: F401
        from paper_2409_07413_amd import binding as B
        ctx = B.Context(0)
        ctx.set_cache_budget(CACHE_BUDGET)
        print(json.dumps({"batch_study": batch_study(ctx, B)}), flush=True)
        ctx.close()
        return
    if args.size_sweep or args.graph_study:
        import torch  # noqa: F401
        from paper_2409_07413_amd import binding as B
        ctx = B.Context(0)
        ctx.set_cache_budget(CACHE_BUDGET)
        if args.size_sweep:
            print(json.dumps({"size_sweep": size_sweep(ctx, B)}), flush=True)
        else:
            print(json.dumps({"graph_study": graph_study(ctx, B)}), flush=True)
        ctx.close()
        return
    rates = [float(r) for r in args.serve_rates.split(",")]
    counts = [int(c) for c in args.serve_shots.split(",")]
    if len(counts) == 1:
        counts = counts * len(rates)
    forms = tuple(args.serve_forms.split(","))

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.serve_only:
        import torch  # noqa: F401
        from paper_2409_07413_amd import binding as B
        ctx = B.Context(0)
        res = serving_leg(ctx, B, rates, counts, args.serve_max_shots, int(args.serve_budget_gib * (1 << 30)),
                          forms, log, shortest=args.serve_policy == "shortest", tune=not args.serve_no_tune)
        for rec in res:  # the kept result densities feed only the full run's oracle check
            rec.get("served", {}).pop("_samples", None)
        print(json.dumps({"serving": res, "config": {
            "workload": "serving stream: Poisson arrivals, sizes uniform over 256..1024 (5 sizes), "
                        "5 ellipses in a 40-px disk, 1e6 photons, 8x8 beamstop, P=32, 500 iterations",
            "max_shots": args.serve_max_shots, "budget_gib": args.serve_budget_gib,
            "policy": args.serve_policy}}), flush=True)
        ctx.close()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus above 1 is not "
                                   "supported (the population loop shards by member, see the design notes)"}))
        sys.exit(2)

    sh, rho0, supp0 = make_inputs()
    # the oracle leg's worker processes start before anything touches the GPU
    pool = None if args.no_cpu_baseline else oracle_pool()

    import torch
    from paper_2409_07413_amd import binding as B

    ctx = B.Context(0)
    shot = ctx.shot(sh["amp"].astype(np.float32), sh["mask"].astype(np.uint8))
    pop = shot.population(rho0, supp0, memetic=True, seed=3004)
    total = args.warmup + args.steps
    G = max(G_SCHEDULE, total + 1)
    ctx.set_cache_budget(CACHE_BUDGET)
    scheds = [B.sched_mpr(ctx, **mpr_params(g, G, g == 1)) for g in range(1, total + 2)]
    # a dedicated stream (default priority): its handle is non-null, so the
    # library's kernels and the timing events below share it
    stream = torch.cuda.Stream()

    for i in range(args.warmup):
        pop.run(scheds[i], stream)
    pop.sync()
    torch.cuda.synchronize()

    # timed region: K generations; HIP events around the launches of the two
    # projection-loop kernels (k_col_proj; k_row_update, ER and HIO/RAAR forms),
    # which run in every iteration, on the launch stream
    # (one launch in every args.timing_every of each, so that the events cost
    # little of the measured throughput)
    pop.timing_sample(args.timing_every)
    pop.timing(True, kernels=[B.KERNEL_COL_PROJ, B.KERNEL_ROW_UPDATE_ER, B.KERNEL_ROW_UPDATE_IA])
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.warmup, total):
        pop.run(scheds[i], stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pop.sync()
    gpu_ms = ev0.elapsed_time(ev1)
    n_er, ms_er = pop.timing_read(B.KERNEL_ROW_UPDATE_ER)
    n_ia, ms_ia = pop.timing_read(B.KERNEL_ROW_UPDATE_IA)
    n_cp, ms_cp = pop.timing_read(B.KERNEL_COL_PROJ)
    n_l, ms = n_er + n_ia, ms_er + ms_ia

    # one more generation with every iteration kernel timed (breakdown only)
    pop.timing_sample(1)
    pop.timing(True)
    pop.run(scheds[total], stream)
    pop.sync()
    kern = {}
    for k in range(4):
        nk, mk = pop.timing_read(k)
        if nk:
            kern[k] = (nk, mk)

    # the parents after the timed generations: the CPU baseline's sample, and
    # four of them for the device-against-oracle check
    amp32, mask8 = sh["amp"].astype(np.float32), sh["mask"].astype(np.uint8)
    st_rho, st_supp, _ = pop.read()
    st_supp = st_supp.astype(np.uint8)
    checks = []
    if not args.no_cpu_baseline:
        pick = [0, P // 3, 2 * P // 3, P - 1]
        c = gpu_step_check(ctx, B, amp32, mask8, st_rho[pick], st_supp[pick])
        c["tag"] = "benchmark"
        checks.append(c)

    member_its = 2 * P * (R * (J + J_ER) + J_EVAL) * args.steps
    value = member_its / wall
    # launches hold `chunk` members, the last the rest; byte counts use the mean
    chunk, per_launch = member_chunk(2 * P)
    bytes_total = (n_er * algorithmic_bytes_per_px(B.KERNEL_ROW_UPDATE_ER, per_launch)
                   + n_ia * algorithmic_bytes_per_px(B.KERNEL_ROW_UPDATE_IA, per_launch)) * N * N * per_launch
    bytes_per_launch = bytes_total / n_l
    achieved = bytes_per_launch / (ms / n_l * 1e-3) / 1e9
    t_er, t_ia = measured_traffic("k_row_update_er", chunk), measured_traffic("k_row_update_ia", chunk)
    traffic = (n_er * t_er + n_ia * t_ia) / n_l if t_er is not None and t_ia is not None else None
    roof_row = {"bound": "hbm", "kernel": "k_row_update", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic, "launches": n_l, "avg_launch_us": ms / n_l * 1e3,
                "timed_ms": ms, "algorithmic_bytes_per_launch": bytes_per_launch,
                "launch_mix": {"ER": n_er, "HIO/RAAR": n_ia}, "sample_every": args.timing_every}
    cp_bytes = algorithmic_bytes_per_px(B.KERNEL_COL_PROJ, per_launch) * N * N * per_launch
    cp_achieved = cp_bytes / (ms_cp / n_cp * 1e-3) / 1e9
    roof_col = {"bound": "hbm", "kernel": "k_col_proj", "achieved": cp_achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": cp_achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic("k_col_proj", chunk), "launches": n_cp,
                "avg_launch_us": ms_cp / n_cp * 1e3, "timed_ms": ms_cp, "algorithmic_bytes_per_launch": cp_bytes,
                "sample_every": args.timing_every}
    tr = trace_averages(chunk)
    if tr is not None:
        er_us, ia_us, cp_us = tr.get("k_row_update_er"), tr.get("k_row_update_ia"), tr.get("k_col_proj")
        if er_us and ia_us:
            us = (n_er * er_us + n_ia * ia_us) / n_l
            roof_row["trace_avg_launch_us"] = us
            roof_row["trace_frac"] = bytes_per_launch / (us * 1e-6) / 1e9 / HBM_PEAK_GBS
        if cp_us:
            roof_col["trace_avg_launch_us"] = cp_us
            roof_col["trace_frac"] = cp_bytes / (cp_us * 1e-6) / 1e9 / HBM_PEAK_GBS
    # the dominant kernel: the larger share of event-timed time in the timed region
    roofline = roof_row if ms >= ms_cp else roof_col
    # whole-step algorithmic bytes: iterations only (ingest/shrink-wrap/fitness/crossover excluded)
    ia_its = er_its = 0
    for i in range(args.warmup, total):
        for o in scheds[i].ops():
            if o.kind in (B.OP_HIO, B.OP_RAAR):
                ia_its += o.count
            elif o.kind == B.OP_ER:
                er_its += o.count
    step_bytes = 2 * P * N * N * (ia_its * (40.125 + 4.0 / per_launch) + er_its * (32.125 + 4.0 / per_launch))
    pct_hbm = step_bytes / wall / (HBM_PEAK_GBS * 1e9)
    out = {
        "metric": "member-iterations/s at 512^2 pop 64 (% HBM peak); p50/p99 shot latency",
        "value": value,
        "unit": "member-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "gpu_ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "iteration_pixels_per_s": value * N * N,
        "pct_hbm_peak_iterations": pct_hbm,
        "config": {"workload": "MPR generation, 512x512 clustered spheres (1e8 photons, 24x24 beamstop, "
                               "4-px gap), P=64 parents + 64 children, RAAR beta 0.9, "
                               "R=3 x 20 + 40 ER = 100 iterations per member per generation",
                   "n": N, "P": P, "members": 2 * P, "generations_timed": args.steps,
                   "schedule_G": G},
        "roofline": roofline,
        "rooflines": {"k_row_update": roof_row, "k_col_proj": roof_col},
        "members_per_launch": chunk,
        "kernels": {B.KERNEL_NAMES[k]: {"launches": v[0], "avg_us": v[1] / v[0] * 1e3,
                                        "GBps": algorithmic_bytes_per_px(k, per_launch) * N * N * per_launch
                                        / (v[1] / v[0] * 1e-3) / 1e9}
                    for k, v in kern.items()},
    }
    pop.close()
    shot.close()
    srv = None
    if not args.no_serve:
        srv = serving_leg(ctx, B, rates, counts, args.serve_max_shots, int(args.serve_budget_gib * (1 << 30)),
                          forms, log, shortest=args.serve_policy == "shortest", tune=not args.serve_no_tune)
        out["serving"] = {"workload": "Poisson arrivals, sizes uniform over {256,384,512,768,1024}, "
                                      "5 ellipses in a 40-px disk, 1e6 photons, 8x8 beamstop, P=32, "
                                      "500 iterations (25 x [HIO^j ER^(20-j), shrink-wrap]) + GetError; "
                                      "served = continuous batching, plain = FIFO one shot at a time",
                          "max_shots": args.serve_max_shots, "rates": srv}
        if "served" in srv[0]:
            out["shot_latency_p50_ms"] = srv[0]["served"]["p50_ms"]
            out["shot_latency_p99_ms"] = srv[0]["served"]["p99_ms"]
        if not args.no_cpu_baseline:
            checks += served_checks(ctx, B, srv)
        for rec in srv:
            rec.get("served", {}).pop("_samples", None)
    if not args.no_cpu_baseline:
        # the oracle runs in spawned worker processes (none of them touches the GPU)
        base, check = cpu_baseline((amp32, mask8, st_rho, st_supp), checks, *pool)
        pool[0].close()
        pool[0].join()
        out["cpu_baseline"] = base
        out["gpu_over_oracle"] = value / base["value"]
        out["oracle_check"] = dict(check, bars={"step_rel_l2": 1e-5, "fitness_rel": 1e-5}, what=(
            "one RAAR step and one ER step with the Eq. error_calc fitness, from device states, on the device "
            "and in the FP64 oracle: 4 parents of the benchmark population after the timed generations, and the "
            "best member of the last served shot of every size"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
