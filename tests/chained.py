"""Step-chained parity of device trajectories against the FP64 oracle.

An iterated projection map amplifies rounding-size differences: from a
random-phase start the FP64 oracle moves by about 1e-1 (HIO) and 1e-2 (RAAR)
after 20 iterations when its own input changes by 1e-7 of its maximum, so no
FP32 trajectory follows an FP64 one end to end.  What is checked instead is
every step: the device state after step k + 1 against one oracle step taken
from the device state after step k, promoted to FP64.

The device states come from runs of the same op list cut after each step.
Consecutive iteration ops form one chain on the device (the iterate is kept
as its row transform between steps); a chain cut after k steps computes the
same first k states as the whole chain, and only its last step writes the
real-space density instead of its row transform.  So the states read back
are the trajectory of the full schedule.

HIO (Fienup's rule, cited by the paper's section on the phase problem) keeps
y = P_M x where y is feasible (inside S and unchanged by the phase
constraint) and takes x - beta y elsewhere: a discontinuous choice.  A pixel
whose feasibility margin, computed by the oracle in FP64, lies within the
FP32 band of the test takes the decision the device's output shows; outside
the band the two decisions must agree.  Shrink-wrap and UpdateSupportSize
thresholds are compared the same way (exact outside a band of 1e-5 of the
maximum around the threshold).
"""

import numpy as np

from oracle import mpr

# (name, report) of every chained run of this process, for the test run's
# terminal summary
REPORTS = []

ITER_KINDS = (1, 2, 3)  # SPR_OP_ER, SPR_OP_HIO, SPR_OP_RAAR
BAND = 1e-5             # FP32 band of a threshold, relative to the largest value


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def feasibility_margin(y, chi):
    """Signed margin of the phase test |Im y| cos(theta) <= Re y sin(theta)
    (theta = chi pi); positive inside.  chi = 0.5 is Re y >= 0; no phase
    constraint gives +inf."""
    if mpr.phase_off(chi):
        return np.full(y.shape, np.inf)
    if chi == 0.5:
        return y.real.copy()
    th = chi * np.pi
    return y.real * np.sin(th) - np.abs(y.imag) * np.cos(th)


def hio_step_banded(x, g_next, S, M, known, chi, beta, band=BAND, bound=None):
    """One oracle HIO step from x with the band rule above (with `bound`, the
    upper-bounded modulus projector of Eq. pm_bounds).

    Returns (expected next state, pixels decided inside the band, decisions
    outside the band that disagree with the device)."""
    y = mpr.proj_modulus(x, M, known) if bound is None else mpr.proj_modulus_bounded(x, M, known, bound)
    feas_o = S & (mpr.proj_phase(y, chi) == y)
    A = y
    Bv = x - beta * y
    scale = float(np.abs(y).max())
    inband = S & (np.abs(feasibility_margin(y, chi)) <= band * scale)
    took_A = np.abs(g_next - A) <= np.abs(g_next - Bv)
    matters = np.abs(A - Bv) > 1e-6 * scale
    hard = int((matters & ~inband & (took_A != feas_o)).sum())
    feas = np.where(inband, took_A, feas_o)
    return np.where(feas, A, Bv), int((inband & matters).sum()), hard


def band_compare(got, a_sigma, thr, scale, band=BAND):
    """Support decisions S = {a > thr} outside the band; (mismatches, in band)."""
    inb = np.abs(a_sigma - thr) <= band * scale
    mism = (got != (a_sigma > thr)) & ~inb
    return int(mism.sum()), int(inb.sum())


def copy_op(B, o, **changes):
    q = B.Op()
    for name, _ in B.Op._fields_:
        setattr(q, name, getattr(o, name))
    for k, v in changes.items():
        setattr(q, k, v)
    return q


def steps(ops):
    """The trajectory's steps: (op index, iterations of that op done), one per
    iteration of an iteration op and one per other op (None)."""
    out = []
    for i, o in enumerate(ops):
        if o.kind in ITER_KINDS:
            out += [(i, k) for k in range(1, o.count + 1)]
        else:
            out.append((i, None))
    return out


def cut(B, ops, i, k):
    """ops[:i] and then k iterations of ops[i] (or ops[i] itself); i < 0 is
    the empty list (the start)."""
    if i < 0:
        return []
    sub = [copy_op(B, o) for o in ops[:i]]
    sub.append(copy_op(B, ops[i], count=k) if k is not None else copy_op(B, ops[i]))
    return sub


class Trajectory:
    """Device states of an op list after each of its steps, from fresh
    populations made by `make_pop` (same start every time)."""

    def __init__(self, ctx, B, make_pop, ops, memetic=False):
        self.ctx, self.B, self.make_pop, self.ops, self.memetic = ctx, B, make_pop, ops, memetic
        self.cache = {}

    def state(self, i, k):
        key = (i, k)
        if key in self.cache:
            return self.cache[key]
        pop = self.make_pop()
        st = {}
        if i >= 0:
            s = self.B.sched_ops(cut(self.B, self.ops, i, k), self.ctx)
            pop.run(s)
            pop.sync()
            s.close()
        st["par"] = pop.read()
        xover_done = any(o.kind == self.B.OP_CROSSOVER for o in self.ops[:i + 1])
        if self.memetic and xover_done:
            st["kid"] = pop.read(children=True)
            st["xover"] = pop.xover()
        if self.memetic:
            st["stats"] = pop.stats()
        pop.close()
        # only the previous state is needed again
        self.cache = {key: st}
        return st


def members(st, scope, B):
    """(tag, index, rho, supp, err) of the members an op with this scope acts on."""
    out = []
    if scope in (B.SCOPE_ALL, B.SCOPE_PARENTS):
        rho, supp, err = st["par"]
        out += [("par", p, rho[p], supp[p], err[p]) for p in range(rho.shape[0])]
    if scope in (B.SCOPE_ALL, B.SCOPE_CHILDREN) and "kid" in st:
        rho, supp, err = st["kid"]
        out += [("kid", p, rho[p], supp[p], err[p]) for p in range(rho.shape[0])]
    return out


def _same(a, b):
    return all(np.array_equal(u, v) for u, v in zip(a, b))


def check_trajectory(traj, M, known, seed=0, band=BAND, step_bar=1e-5, err_bar=1e-5, bound=None):
    """Walk the steps of traj.ops, checking each against the oracle applied to
    the device's previous state (M as the shot stores it; `bound` the upper
    bounds of the unknown pixels, if the shot has them).  Returns a report
    dict (maxima and counts)."""
    B = traj.B
    ops = traj.ops
    rep = {"steps": 0, "max_step_rel": 0.0, "hio_band_px": 0, "sw_band_px": 0, "area_band_px": 0,
           "max_err_rel": 0.0, "xover_flagged": 0, "xover_children": 0, "selections": 0}
    prev = traj.state(-1, None)
    for i, k in steps(ops):
        cur = traj.state(i, k)
        o = ops[i]
        where = f"op {i} (kind {o.kind}), step {k}"
        if o.kind in ITER_KINDS:
            before = {(t, p): (x, S) for t, p, x, S, _ in members(prev, o.scope, B)}
            for t, p, g, Sg, _ in members(cur, o.scope, B):
                x, S = before[(t, p)]
                x64 = x.astype(np.complex128)
                if o.kind == B.OP_ER:
                    ref = mpr.er(x64, S, M, known, o.chi, bound=bound)
                elif o.kind == B.OP_RAAR:
                    ref = mpr.raar(x64, S, M, known, o.chi, o.beta, bound=bound)
                else:
                    ref, nb, hard = hio_step_banded(x64, g.astype(np.complex128), S, M, known, o.chi, o.beta,
                                                    band, bound)
                    assert hard == 0, (where, t, p, "HIO decisions outside the FP32 band differ", hard)
                    rep["hio_band_px"] += nb
                r = rel(g, ref)
                assert r <= step_bar, (where, t, p, r)
                rep["max_step_rel"] = max(rep["max_step_rel"], r)
                np.testing.assert_array_equal(Sg, S)
        elif o.kind == B.OP_SHRINKWRAP:
            before = {(t, p): (x, S) for t, p, x, S, _ in members(prev, o.scope, B)}
            for t, p, g, Sg, _ in members(cur, o.scope, B):
                x, S = before[(t, p)]
                np.testing.assert_array_equal(g, x)
                a = mpr.smooth(np.abs(x.astype(np.complex128)), o.sigma)
                if not a.max() > 0:
                    np.testing.assert_array_equal(Sg, S)
                    continue
                mism, inb = band_compare(Sg, a, o.tau * a.max(), a.max(), band)
                assert mism == 0, (where, t, p, mism)
                rep["sw_band_px"] += inb
        elif o.kind == B.OP_SUPPORT_AREA:
            st = cur["stats"][-1] if o.which != B.AREA_ABS else None
            alpha = o.alpha if o.which == B.AREA_ABS else (
                st.alpha_best if o.which == B.AREA_BEST else st.alpha_eval)
            before = {(t, p): (x, S) for t, p, x, S, _ in members(prev, o.scope, B)}
            for t, p, g, Sg, _ in members(cur, o.scope, B):
                x, _ = before[(t, p)]
                np.testing.assert_array_equal(g, x)
                n2 = x.size
                kk = mpr.area_count(alpha, n2)
                assert int(Sg.sum()) == kk, (where, t, p, int(Sg.sum()), kk)
                if kk >= n2:
                    continue
                a = mpr.smooth(np.abs(x.astype(np.complex128)), o.sigma)
                vk = np.sort(a.ravel())[::-1][kk - 1]
                inb = np.abs(a - vk) <= band * a.max()
                ref = mpr.update_support_size(x.astype(np.complex128), o.sigma, alpha)
                assert int(((Sg != ref) & ~inb).sum()) == 0, (where, t, p)
                rep["area_band_px"] += int(inb.sum())
        elif o.kind == B.OP_GET_ERROR:
            before = {(t, p): (x, S) for t, p, x, S, _ in members(prev, o.scope, B)}
            for t, p, g, Sg, e in members(cur, o.scope, B):
                x, S = before[(t, p)]
                ref = mpr.get_error(x.astype(np.complex128), S, M, known)
                r = abs(e - ref) / ref
                assert r <= err_bar, (where, t, p, e, ref)
                rep["max_err_rel"] = max(rep["max_err_rel"], r)
        elif o.kind == B.OP_STATS:
            rho, S, E = prev["par"]
            ref = mpr.generation_stats(E, list(S), o.gen, o.gens)
            st = cur["stats"][-1]
            assert (st.best, st.alpha_best, st.alpha_all) == (ref["best"], ref["alpha_best"], ref["alpha_all"]), where
            assert st.alpha_eval == ref["alpha_eval"], where
            assert _same(cur["par"], prev["par"])
        elif o.kind == B.OP_CROSSOVER:
            rho, S, E = prev["par"]
            assert _same(cur["par"], prev["par"])
            kx, kS, _ = cur["kid"]
            info = cur["xover"]
            ox, oS, oinfo = mpr.crossover([x.astype(np.complex128) for x in rho], list(S), known, o.gen, seed,
                                          o.c_p, o.c_w, o.t_min, o.t_max)
            for p in range(rho.shape[0]):
                assert (info[p].a, info[p].b, info[p].c) == oinfo[p]["abc"], (where, p)
                got_map = (info[p].tx, info[p].ty, info[p].sx, info[p].sy, info[p].rot)
                assert got_map == mpr.map_params(rho.shape[1], seed, o.gen, p, o.t_min, o.t_max), (where, p)
                tied = False
                for q, al in enumerate(oinfo[p]["align"]):
                    vals = sorted([al["peak1"], al["peak2"], al["second1"], al["second2"]], reverse=True)
                    if vals[1] >= vals[0] * (1 - 1e-4):
                        tied = True
                        continue
                    got = ((info[p].dr[q], info[p].dc[q]), bool(info[p].twin[q]))
                    assert got == (al["shift"], al["twin"]), (where, p, q)
                rep["xover_children"] += 1
                if tied:
                    rep["xover_flagged"] += 1
                    continue
                r = rel(kx[p], ox[p])
                assert r <= step_bar, (where, p, r)
                rep["max_step_rel"] = max(rep["max_step_rel"], r)
                np.testing.assert_array_equal(kS[p], oS[p])
        elif o.kind == B.OP_SELECT:
            par, kid = prev["par"], prev["kid"]
            repl = mpr.select(list(par[2]), list(kid[2]))
            for p, r in enumerate(repl):
                win, lose = (kid, par) if r else (par, kid)
                for a, b in zip(cur["par"], win):
                    assert np.array_equal(a[p], b[p]), (where, p)
                for a, b in zip(cur["kid"], lose):
                    assert np.array_equal(a[p], b[p]), (where, p)
            assert cur["stats"][-1].replaced == sum(repl)
            rep["selections"] += len(repl)
        else:
            raise AssertionError(f"no chained check for op kind {o.kind}")
        rep["steps"] += 1
        prev = cur
    return rep
