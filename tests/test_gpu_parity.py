"""GPU parity of the HIP hot path against the FP64 oracle, through the C ABI.

Bars (FP32 GPU vs FP64 oracle): single operator applications <= 1e-5 relative
L2; 20-iteration runs <= 1e-3; integer decisions (RandomChoice, crossover-map
parameters, Reshift shifts/twins, selection) bit-exact, except near-ties that
the test detects from the oracle's own values and reports.  Support thresholds
are compared exactly outside a band of 1e-5 * max around the threshold.
"""

import numpy as np
import pytest

from oracle import mpr, philox
from paper_2409_07413_amd import synth

from gpu_cases import Case, NearSolutionCase, rel, self_sensitivity

pytestmark = pytest.mark.gpu

ALL_SIZES = (8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024)


@pytest.fixture(scope="module")
def ctx():
    from paper_2409_07413_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def B():
    from paper_2409_07413_amd import binding
    return binding


def run_ops(pop, B, ops):
    s = B.sched_ops(ops)
    pop.run(s)
    pop.sync()
    s.close()


# ---------------------------------------------------------------------------
# FFT
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", ALL_SIZES)
def test_fft2_parity(ctx, n):
    import torch
    batch = 3
    x = synth.random_complex((batch, n, n), n).astype(np.complex64)
    xt = torch.from_numpy(x).cuda()
    out = torch.empty_like(xt)
    ctx.fft2(xt, out, inverse=False)
    got = out.cpu().numpy()
    ref = np.stack([mpr.fft2(v.astype(np.complex128)) for v in x])
    assert rel(got, ref) <= 1e-5
    ctx.fft2(xt, out, inverse=True)
    got = out.cpu().numpy()
    ref = np.stack([mpr.ifft2(v.astype(np.complex128)) for v in x])
    assert rel(got, ref) <= 1e-5
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", (12, 128, 1024))
def test_fft2_in_place(ctx, n):
    # the entry point allows in == out: forward then inverse on one buffer
    import torch
    x = synth.random_complex((2, n, n), n + 1).astype(np.complex64)
    buf = torch.from_numpy(x).cuda()
    ctx.fft2(buf, buf, inverse=False)
    got = buf.cpu().numpy()
    assert rel(got, np.stack([mpr.fft2(v.astype(np.complex128)) for v in x])) <= 1e-5
    ctx.fft2(buf, buf, inverse=True)
    assert rel(buf.cpu().numpy(), x) <= 1e-5
    torch.cuda.synchronize()


def test_device_pointer_forms_equal_host_forms(ctx, B):
    # SPR_DEVICE_PTRS: shot, population, read and write from device memory
    # give the same bits as the host forms
    import torch
    n, P = 96, 3
    c = Case(n, P, seed=96 + 41, per_member_supp=True)
    ops = [B.op(B.OP_RAAR, count=2, beta=0.9, chi=0.5), B.op(B.OP_ER, count=1, chi=0.5), B.op(B.OP_GET_ERROR)]
    sh, pop = c.population(ctx)
    run_ops(pop, B, ops)
    rho_h, supp_h, err_h = pop.read()
    pop.close()
    sh.close()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    shd = ctx.shot(dev(c.amp32), dev(c.mask8))
    popd = shd.population(dev(c.rho32), dev(c.supp8))
    run_ops(popd, B, ops)
    rho_d = torch.empty((P, n, n), dtype=torch.complex64, device="cuda")
    supp_d = torch.empty((P, n, n), dtype=torch.uint8, device="cuda")
    err_d = torch.empty(P, dtype=torch.float64, device="cuda")
    popd.read_into(rho_d, supp_d, err_d)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(rho_d.cpu().numpy(), rho_h)
    np.testing.assert_array_equal(supp_d.cpu().numpy().astype(bool), supp_h.astype(bool))
    np.testing.assert_array_equal(err_d.cpu().numpy(), err_h)
    # write from device memory, then read back on the host
    popd.write(rho=torch.flip(rho_d, dims=(0,)).contiguous(), err=torch.flip(err_d, dims=(0,)).contiguous())
    rho_b, _, err_b = popd.read()
    np.testing.assert_array_equal(rho_b, rho_h[::-1])
    np.testing.assert_array_equal(err_b, err_h[::-1])
    popd.close()
    shd.close()


# ---------------------------------------------------------------------------
# Single operator applications
# ---------------------------------------------------------------------------
OP_SIZES = (12, 32, 128, 384, 512)


@pytest.mark.parametrize("n", OP_SIZES)
@pytest.mark.parametrize("chi", [0.5, 1.0, 0.3])
def test_single_iterations(ctx, B, n, chi):
    P = 3
    c = Case(n, P, seed=n + 1, per_member_supp=True)
    for kind, fn in ((B.OP_ER, lambda x, S: mpr.er(x, S, c.M, c.known, chi)),
                     (B.OP_HIO, lambda x, S: mpr.hio(x, S, c.M, c.known, chi, 0.9)),
                     (B.OP_RAAR, lambda x, S: mpr.raar(x, S, c.M, c.known, chi, 0.9))):
        sh, pop = c.population(ctx)
        run_ops(pop, B, [B.op(kind, count=1, beta=0.9, chi=chi)])
        rho, supp, _ = pop.read()
        for p in range(P):
            ref = fn(c.rho[p], c.S[p])
            assert rel(rho[p], ref) <= 1e-5, (kind, p)
        np.testing.assert_array_equal(supp, c.S)
        pop.close()
        sh.close()


def _size_variants():
    from paper_2409_07413_amd import build
    return [(n, v) for n in ALL_SIZES for v in ((0, 1) if n in build.VARIANT_SIZES else (0,))]


@pytest.mark.parametrize("n,variant", _size_variants())
def test_iterations_every_size_and_variant(ctx, B, n, variant):
    # every compiled loop kernel (both plans where a size has two): RAAR and ER
    # steps in one schedule (the iterate stays a row transform between them),
    # the fitness, and one HIO step, from per-member supports; three members,
    # so that small sizes put rows of several members in one wavefront.  HIO's
    # choice between y and x - beta y is discontinuous at the constraint
    # boundary, so it is checked over one step only (longer HIO runs are
    # compared between plans bit for bit below).
    P = 3
    c = Case(n, P, seed=n + 5 * variant + 11, per_member_supp=True)
    ctx.set_variant(n, variant)
    try:
        sh, pop = c.population(ctx)
        run_ops(pop, B, [B.op(B.OP_RAAR, count=2, beta=0.9, chi=0.5), B.op(B.OP_ER, count=2, chi=0.3),
                         B.op(B.OP_GET_ERROR)])
        rho, supp, err = pop.read()
        pop.close()
        sh.close()
        sh, pop = c.population(ctx)
        run_ops(pop, B, [B.op(B.OP_HIO, count=1, beta=0.8, chi=0.3)])
        rho_h, _, _ = pop.read()
        pop.close()
        sh.close()
    finally:
        ctx.set_variant(n, 0)
    for p in range(P):
        x = c.rho[p]
        for _ in range(2):
            x = mpr.raar(x, c.S[p], c.M, c.known, 0.5, 0.9)
        for _ in range(2):
            x = mpr.er(x, c.S[p], c.M, c.known, 0.3)
        assert rel(rho[p], x) <= 1e-4, (n, variant, p, rel(rho[p], x))
        e = mpr.get_error(x, c.S[p], c.M, c.known)
        assert abs(err[p] - e) <= 1e-4 * e
        assert rel(rho_h[p], mpr.hio(c.rho[p], c.S[p], c.M, c.known, 0.3, 0.8)) <= 1e-5
    np.testing.assert_array_equal(supp, c.S)


@pytest.mark.parametrize("n", (256, 384, 512, 768))
def test_plans_of_a_size_are_bit_identical(ctx, B, n):
    # at these sizes the two plans differ only in the column-tile width, which
    # changes no transform arithmetic: the same schedule, HIO steps included,
    # gives the same density bits; the fitness sums one FP64 partial per tile,
    # so its last bit follows the tile count (the two 1024 plans order their
    # radices differently, so they round differently; both meet the oracle bar
    # above)
    P = 3
    c = Case(n, P, seed=n + 400, per_member_supp=True)
    outs = []
    for variant in (0, 1):
        ctx.set_variant(n, variant)
        try:
            sh, pop = c.population(ctx)
            run_ops(pop, B, [B.op(B.OP_RAAR, count=2, beta=0.9, chi=0.5), B.op(B.OP_HIO, count=2, beta=0.8, chi=0.3),
                             B.op(B.OP_ER, count=2, chi=0.5), B.op(B.OP_GET_ERROR)])
            outs.append(pop.read())
            pop.close()
            sh.close()
        finally:
            ctx.set_variant(n, 0)
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_allclose(outs[0][2], outs[1][2], rtol=1e-14, atol=0)


@pytest.mark.parametrize("n", OP_SIZES)
def test_get_error(ctx, B, n):
    P = 4
    c = Case(n, P, seed=n + 2, per_member_supp=True)
    sh, pop = c.population(ctx)
    run_ops(pop, B, [B.op(B.OP_GET_ERROR)])
    _, _, err = pop.read()
    for p in range(P):
        ref = mpr.get_error(c.rho[p], c.S[p], c.M, c.known)
        assert abs(err[p] - ref) <= 1e-5 * ref
    pop.close()
    sh.close()


def _band_compare(got, a_sigma, thr, scale):
    band = np.abs(a_sigma - thr) <= 1e-5 * scale
    mism = (got != (a_sigma > thr)) & ~band
    return int(mism.sum()), int(band.sum())


@pytest.mark.parametrize("n", (12, 32, 96, 128, 512, 1024))
@pytest.mark.parametrize("sigma", (0.0, 1.0, 2.0, 3.5, 7.5))
def test_shrinkwrap(ctx, B, n, sigma):
    P = 3
    c = Case(n, P, seed=n + 3)
    sh, pop = c.population(ctx)
    run_ops(pop, B, [B.op(B.OP_SHRINKWRAP, sigma=sigma, tau=0.1)])
    _, supp, _ = pop.read()
    for p in range(P):
        a = mpr.smooth(np.abs(c.rho[p]), sigma)
        mism, inband = _band_compare(supp[p], a, 0.1 * a.max(), a.max())
        assert mism == 0, (p, mism, inband)
    pop.close()
    sh.close()


@pytest.mark.parametrize("n", (12, 32, 96, 128, 512, 1024))
@pytest.mark.parametrize("alpha", (1.0, 37.5, 300.4, 5000.0))
def test_support_area(ctx, B, n, alpha):
    P = 2
    c = Case(n, P, seed=n + 4)
    sh, pop = c.population(ctx)
    run_ops(pop, B, [B.op(B.OP_SUPPORT_AREA, sigma=2.0, which=B.AREA_ABS, alpha=alpha)])
    _, supp, _ = pop.read()
    k = mpr.area_count(alpha, n * n)
    for p in range(P):
        if k >= n * n:
            assert supp[p].all()
            continue
        assert supp[p].sum() == k
        a = mpr.smooth(np.abs(c.rho[p]), 2.0)
        vk = np.sort(a.ravel())[::-1][k - 1]
        band = np.abs(a - vk) <= 1e-5 * a.max()
        ref = mpr.update_support_size(c.rho[p], 2.0, alpha)
        assert int(((supp[p] != ref) & ~band).sum()) == 0
    pop.close()
    sh.close()


@pytest.mark.parametrize("n,alpha", [(32, 200.0), (128, 200.0), (128, 9000.0), (384, 70000.0)])
def test_support_area_exact_ties(ctx, B, n, alpha):
    # integer-valued densities: many exact ties, resolved by the lower index;
    # from 96 up the selection runs over many workgroups per member, and the
    # tie group of the k-th value spans several of them
    c = Case(n, 2, seed=5)
    rng = np.random.default_rng(3)
    vals = rng.integers(0, 4, size=(2, n, n)).astype(np.complex64)
    sh, pop = c.population(ctx)
    pop.write(rho=vals)
    run_ops(pop, B, [B.op(B.OP_SUPPORT_AREA, sigma=0.0, which=B.AREA_ABS, alpha=alpha)])
    _, supp, _ = pop.read()
    for p in range(2):
        np.testing.assert_array_equal(supp[p], mpr.update_support_size(vals[p].astype(complex), 0.0, alpha))
    pop.close()
    sh.close()


# ---------------------------------------------------------------------------
# 20-iteration runs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", (64, 128, 256, 512))
def test_twenty_iterations_er(ctx, B, n):
    # ER from random-phase starts: a well-conditioned map, bar 1e-3
    P = 2
    c = Case(n, P, seed=n + 5)
    sh, pop = c.population(ctx)
    run_ops(pop, B, [B.op(B.OP_ER, count=20, chi=0.5), B.op(B.OP_GET_ERROR)])
    rho, _, err = pop.read()
    for p in range(P):
        ref = mpr.sequence(c.rho[p], c.S[p], c.M, c.known, 0.5, "HIO", 0.9, 0, 20)
        assert rel(rho[p], ref) <= 1e-3
        e_ref = mpr.get_error(ref, c.S[p], c.M, c.known)
        assert abs(err[p] - e_ref) <= 1e-3 * e_ref
    pop.close()
    sh.close()


@pytest.mark.parametrize("n", (64, 128, 256, 512))
@pytest.mark.parametrize("alg", ("HIO", "RAAR"))
def test_twenty_iterations_near_solution(ctx, B, n, alg):
    # 16 HIO/RAAR + 4 ER from 5% around the true density (noiseless data),
    # end to end.  The 1e-3 bar holds where the map is well conditioned: where
    # the FP64 oracle itself moves by less than 1e-4 under a 1e-7 change of
    # its input.  Elsewhere (HIO's discontinuous feasibility choice) the
    # distance is reported, not gated: those trajectories are checked step by
    # step in tests/test_gpu_chained.py.
    P = 2
    c = NearSolutionCase(n, P, seed=n + 6)
    sh, pop = c.population(ctx)
    kind = B.OP_HIO if alg == "HIO" else B.OP_RAAR
    run_ops(pop, B, [B.op(kind, count=16, beta=0.9, chi=0.5), B.op(B.OP_ER, count=4, chi=0.5),
                     B.op(B.OP_GET_ERROR)])
    rho, _, err = pop.read()
    gated = 0
    for p in range(P):
        f = lambda x: mpr.sequence(x, c.S[p], c.M, c.known, 0.5, alg, 0.9, 16, 4)  # noqa: E731
        ref = f(c.rho[p])
        sens = self_sensitivity(f, c.rho[p])
        r = rel(rho[p], ref)
        e_ref = mpr.get_error(ref, c.S[p], c.M, c.known)
        if sens < 1e-4:
            assert r <= 1e-3
            assert abs(err[p] - e_ref) <= 1e-3 * e_ref
            gated += 1
        print(f"{alg} near solution {n}^2 member {p}: rel L2 {r:.2e}, oracle self-sensitivity {sens:.2e}"
              f" ({'gated at 1e-3' if sens < 1e-4 else 'reported only'})")
    if alg == "RAAR" and n <= 128:
        # measured: the oracle's own sensitivity stays below 1e-4 here
        assert gated == P
    pop.close()
    sh.close()


@pytest.mark.parametrize("n", (64, 512))
@pytest.mark.parametrize("alg", ("HIO", "RAAR"))
def test_twenty_iterations_random_start_report(ctx, B, n, alg):
    # From random-phase starts HIO/RAAR amplify rounding-size differences by
    # 1e4..1e6 within 20 iterations (the FP64 oracle does so to its own
    # inputs), so the end-to-end distance is reported beside the oracle's
    # self-sensitivity and is not a parity check; every step of these runs is
    # checked in tests/test_gpu_chained.py.
    P = 2
    c = Case(n, P, seed=n + 5)
    sh, pop = c.population(ctx)
    kind = B.OP_HIO if alg == "HIO" else B.OP_RAAR
    run_ops(pop, B, [B.op(kind, count=16, beta=0.9, chi=0.5), B.op(B.OP_ER, count=4, chi=0.5)])
    rho, _, _ = pop.read()
    for p in range(P):
        f = lambda x: mpr.sequence(x, c.S[p], c.M, c.known, 0.5, alg, 0.9, 16, 4)  # noqa: E731
        ref = f(c.rho[p])
        assert np.all(np.isfinite(rho[p]))
        print(f"{alg} random start {n}^2 member {p}: end-to-end rel L2 {rel(rho[p], ref):.2e}, "
              f"oracle self-sensitivity {self_sensitivity(f, c.rho[p]):.2e} (report, not a parity check)")
    pop.close()
    sh.close()


def test_twenty_iterations_with_shrinkwrap(ctx, B):
    # ER^15, shrink-wrap, ER^5.  The support decision is checked on the GPU's
    # own iterate (the oracle's FP64 smoothing of it; pixels outside the FP32
    # band of the threshold must agree exactly); the oracle then continues
    # from its own iterate with the support the GPU chose, and the final
    # densities must agree to the 20-iteration bar.
    n, P = 128, 3
    c = Case(n, P, seed=77)
    sh, pop = c.population(ctx)
    run_ops(pop, B, [B.op(B.OP_ER, count=15, chi=0.5)])
    x15g, _, _ = pop.read()
    run_ops(pop, B, [B.op(B.OP_SHRINKWRAP, sigma=2.0, tau=0.1), B.op(B.OP_ER, count=5, chi=0.5)])
    x20g, supp, _ = pop.read()
    for p in range(P):
        x15 = mpr.sequence(c.rho[p], c.S[p], c.M, c.known, 0.5, "HIO", 0.9, 0, 15)
        assert rel(x15g[p], x15) <= 1e-3
        ag = mpr.smooth(np.abs(x15g[p].astype(np.complex128)), 2.0)
        mism, _ = _band_compare(supp[p], ag, 0.1 * ag.max(), ag.max())
        assert mism == 0, (p, mism)
        a = mpr.smooth(np.abs(x15), 2.0)
        flips = int((supp[p] != (a > 0.1 * a.max())).sum())
        assert flips <= n * n // 500, (p, flips)
        x20 = mpr.sequence(x15, supp[p].astype(bool), c.M, c.known, 0.5, "HIO", 0.9, 0, 5)
        assert rel(x20g[p], x20) <= 1e-3
    pop.close()
    sh.close()


# ---------------------------------------------------------------------------
# Memetic operators
# ---------------------------------------------------------------------------
def test_choice_and_map_parameters_match_philox_stream(ctx, B):
    n, P = 16, 7
    c = Case(n, P, seed=8)
    sh, pop = c.population(ctx, memetic=True, seed=0xDEADBEEF12345)
    for g in (1, 2, 5, 40):
        run_ops(pop, B, [B.op(B.OP_CROSSOVER, gen=g, c_p=0.6, c_w=0.4, t_min=2, t_max=5)])
        info = pop.xover()
        for p in range(P):
            assert (info[p].a, info[p].b, info[p].c) == mpr.random_choice(p, P, 0xDEADBEEF12345, g)
            got = (info[p].tx, info[p].ty, info[p].sx, info[p].sy, info[p].rot)
            assert got == mpr.map_params(n, 0xDEADBEEF12345, g, p, 2, 5)
    pop.close()
    sh.close()


def _aligned_population(n, P, seed):
    """Parents that are shifted / twinned / phased copies of one object plus noise."""
    rng = np.random.default_rng(seed)
    c = Case(n, P, seed=seed)
    base = np.zeros((n, n), complex)
    base[:n // 4, :n // 5] = rng.uniform(0.5, 1.5, size=(n // 4, n // 5))
    xs, Ss = [], []
    for p in range(P):
        b = np.conj(np.roll(base[::-1, ::-1], 1, axis=(0, 1))) if p % 3 == 2 else base
        d = tuple(rng.integers(0, n, size=2))
        x = np.exp(1j * rng.uniform(0, 2 * np.pi)) * np.roll(b, d, axis=(0, 1))
        x = x + 0.05 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        xs.append(x.astype(np.complex64))
        Ss.append(np.roll(np.abs(b) > 0, d, axis=(0, 1)) | (rng.random((n, n)) < 0.05))
    c.rho32 = np.stack(xs)
    c.rho = c.rho32.astype(np.complex128)
    c.S = np.stack(Ss)
    c.supp8 = c.S.astype(np.uint8)
    return c


def _near_tie(info, tol=1e-4):
    vals = sorted([info["peak1"], info["peak2"], info["second1"], info["second2"]], reverse=True)
    return vals[1] >= vals[0] * (1 - tol)


XOVER_CASES = [(48, 5, True, 0), (64, 6, True, 0), (64, 5, False, 0), (128, 4, True, 0), (256, 4, True, 0),
               (384, 4, True, 0), (512, 4, True, 0), (768, 4, True, 0), (1024, 4, True, 0),
               (256, 4, True, 1), (384, 4, True, 1), (512, 4, True, 1), (768, 4, True, 1), (1024, 4, True, 1)]


@pytest.mark.parametrize("n,P,structured,variant", XOVER_CASES)
def test_crossover_parity(ctx, B, n, P, structured, variant):
    # every size-specialised crossover kernel (parent spectra, Reshift
    # correlations and argmax, alignment, the mix with the column IFFT) on
    # both plans of the tuned sizes
    c = _aligned_population(n, P, seed=n + P + 31 * variant) if structured else Case(n, P, seed=n + 9)
    seed = 3002
    if variant:
        ctx.set_variant(n, variant)
    try:
        sh, pop = c.population(ctx, memetic=True, seed=seed)
        t_max = mpr.default_t_max(n)
        run_ops(pop, B, [B.op(B.OP_CROSSOVER, gen=1, c_p=0.6, c_w=0.4, t_min=4, t_max=t_max)])
        kx, kS, _ = pop.read(children=True)
        info = pop.xover()
    finally:
        if variant:
            ctx.set_variant(n, 0)
    ox, oS, oinfo = mpr.crossover(list(c.rho), list(c.S), c.known, 1, seed, 0.6, 0.4, 4, t_max)
    flagged = 0
    for p in range(P):
        assert (info[p].a, info[p].b, info[p].c) == oinfo[p]["abc"]
        ties = [_near_tie(al) for al in oinfo[p]["align"]]
        exact = True
        for k, al in enumerate(oinfo[p]["align"]):
            if ties[k]:
                continue
            got = ((info[p].dr[k], info[p].dc[k]), bool(info[p].twin[k]))
            if got != (al["shift"], al["twin"]):
                exact = False
            assert got == (al["shift"], al["twin"]), (p, k)
        if any(ties):
            flagged += 1
            continue
        assert exact
        assert rel(kx[p], ox[p]) <= 1e-5, p
        np.testing.assert_array_equal(kS[p], oS[p])
    if structured:
        assert flagged == 0
    # parents are untouched by crossover
    rho, supp, _ = pop.read()
    np.testing.assert_array_equal(rho, c.rho32)
    pop.close()
    sh.close()


def test_select_bitexact_with_injected_errors(ctx, B):
    n, P = 16, 6
    c = Case(n, P, seed=10)
    sh, pop = c.population(ctx, memetic=True)
    e_par = np.array([0.5, 0.2, 0.3, 0.3, 0.1, 0.7])
    e_kid = np.array([0.4, 0.2, 0.31, 0.1, 0.1, 0.69999999999])
    kids = (c.rho32 * 2).astype(np.complex64)
    pop.write(rho=kids, supp=1 - c.supp8, err=e_kid, children=True)
    pop.write(err=e_par)
    run_ops(pop, B, [B.op(B.OP_SELECT, gen=1)])
    rho, supp, err = pop.read()
    repl = mpr.select(list(e_par), list(e_kid))
    for p in range(P):
        if repl[p]:
            assert err[p] == e_kid[p]
            np.testing.assert_array_equal(rho[p], kids[p])
            np.testing.assert_array_equal(supp[p], (1 - c.supp8[p]).astype(bool))
        else:
            assert err[p] == e_par[p]
            np.testing.assert_array_equal(rho[p], c.rho32[p])
    st = pop.stats()
    assert st[-1].replaced == sum(repl)
    final = [min(a, b) if r else a for a, b, r in zip(e_par, e_kid, repl)]
    assert st[-1].err_best == min(final) and st[-1].err_worst == max(final)
    pop.close()
    sh.close()


def test_generation_stats(ctx, B):
    n, P = 32, 5
    c = Case(n, P, seed=11, per_member_supp=True)
    rng = np.random.default_rng(4)
    S = rng.random((P, n, n)) < 0.2
    E = np.array([0.3, 0.2, 0.2, 0.5, 0.25])
    sh, pop = c.population(ctx, memetic=True)
    pop.write(supp=S.astype(np.uint8), err=E)
    run_ops(pop, B, [B.op(B.OP_STATS, gen=3, gens=10)])
    st = pop.stats()[-1]
    ref = mpr.generation_stats(E, list(S), 3, 10)
    assert (st.best, st.alpha_best, st.alpha_all) == (ref["best"], ref["alpha_best"], ref["alpha_all"])
    assert st.alpha_eval == ref["alpha_eval"]
    # the area ops then use these values
    run_ops(pop, B, [B.op(B.OP_SUPPORT_AREA, sigma=1.0, which=B.AREA_EVAL, scope=B.SCOPE_PARENTS)])
    _, supp, _ = pop.read()
    assert all(s.sum() == mpr.area_count(ref["alpha_eval"], n * n) for s in supp)
    pop.close()
    sh.close()


# ---------------------------------------------------------------------------
# Drivers
# ---------------------------------------------------------------------------
def test_plain_driver_small(ctx, B):
    n, P = 64, 4
    c = Case(n, P, seed=21)
    prm = dict(alg="HIO", beta=0.9, chi=0.5, G=2, j=6, j_er=4, j_end=0, sigma=2.0, sigma_end=1.0,
               tau=0.1, tau_end=0.1)
    sh, pop = c.population(ctx)
    s = B.sched_plain(alg=B.ALG_HIO, G=2, j=6, j_er=4, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                      sigma_end=1.0, tau=0.1, tau_end=0.1)
    pop.run(s)
    rho, supp, err = pop.read()
    out = mpr.run_plain(c.M, c.known, c.rho, c.S[0], prm)
    compared = 0
    for p in range(P):
        if (supp[p] != out["S"][p]).any():
            continue  # a threshold flip inside the FP32 band changes the trajectory
        assert rel(rho[p], out["x"][p]) <= 1e-3
        assert abs(err[p] - out["E"][p]) <= 1e-3 * out["E"][p]
        compared += 1
    pop.close()
    sh.close()
    # every step of this kind of schedule is also checked against the oracle
    # on the device's own states (tests/test_gpu_chained.py)
    print(f"plain driver 64^2: {compared} of {P} members compared end to end")
    assert compared >= P // 2


@pytest.mark.parametrize("n,P,seed", [(32, 6, 31), (64, 6, 33)])
def test_mpr_one_generation_small(ctx, B, n, P, seed):
    # one MPR generation end to end.  After Select the parent slots hold the
    # winners and the child slots the losers, so the GPU's own decisions are
    # checked exactly (winner error <= loser error), and against the oracle's
    # run wherever the pair of errors matches the oracle's pair (trajectories
    # can part at a support threshold inside the FP32 band) and is not a
    # near-tie
    c = Case(n, P, seed=seed)
    prm = dict(alg="RAAR", beta=0.9, chi=0.5, G=2, R=3, j=4, j_er=2, j_end=0, j_eval=4, sigma=2.0,
               sigma_end=0.5, tau=0.1, tau_end=0.1 * 2 / 3, c_p=0.6, c_w=0.4, t_min=4, t_max=4)
    seed_x = 99
    sh, pop = c.population(ctx, memetic=True, seed=seed_x)
    s = B.sched_mpr(alg=B.ALG_RAAR, G=2, R=3, j=4, j_er=2, j_end=0, j_eval=4, t_min=4, t_max=4,
                    gen_first=1, gen_count=1, init_error=1, beta=0.9, chi=0.5, sigma=2.0, sigma_end=0.5,
                    tau=0.1, tau_end=0.1 * 2 / 3, c_p=0.6, c_w=0.4)
    pop.run(s)
    _, _, err_win = pop.read()
    _, _, err_lose = pop.read(children=True)
    st = pop.stats()[-1]
    out = mpr.run_mpr(c.M, c.known, c.rho, c.S[0], prm, seed_x, generations=1)
    h = out["history"][0]
    assert st.alpha_best == h["stats"]["alpha_best"] and st.alpha_all == h["stats"]["alpha_all"]
    assert np.all(err_win <= err_lose)
    compared = 0
    for p in range(P):
        eo, en = h["E_par"][p], h["E_kid"][p]
        gpu = sorted((err_win[p], err_lose[p]))
        if not np.allclose(gpu, sorted((eo, en)), rtol=1e-3, atol=0):
            continue  # this pair's trajectory parted from the oracle's
        if abs(en - eo) < 1e-3 * eo:
            continue  # near-tie in selection
        kid_won_gpu = abs(err_win[p] - en) < abs(err_win[p] - eo)
        assert kid_won_gpu == (en < eo), (p, err_win[p], err_lose[p], eo, en)
        assert abs(err_win[p] - out["E"][p]) <= 1e-3 * out["E"][p]
        compared += 1
    pop.close()
    sh.close()
    print(f"n={n} P={P}: {compared} of {P} selections compared with the oracle")
    assert compared >= P // 2


# ---------------------------------------------------------------------------
# Launches of many members (one launch chunk of the whole population) against
# a launch of two of them: a member's arithmetic does not depend on the launch,
# so both give the same bits, and sampled members match the oracle.
# ---------------------------------------------------------------------------
MANY = [(256, 0, 64), (256, 1, 64), (384, 0, 40), (384, 1, 40), (512, 0, 40), (512, 1, 40),
        (768, 0, 24), (768, 1, 24), (1024, 0, 24), (1024, 1, 24)]


@pytest.mark.parametrize("n,variant,P", MANY)
def test_many_member_launch(ctx, B, n, variant, P):
    c = Case(n, P, seed=n + 71 * variant + P)
    ops = [B.op(B.OP_RAAR, count=2, beta=0.9, chi=0.5, which=B.ITER_TRACE),
           B.op(B.OP_ER, count=1, chi=0.5, which=B.ITER_TRACE), B.op(B.OP_GET_ERROR)]
    ctx.set_variant(n, variant)
    ctx.set_cache_budget(P * 2 * n * n * 8)  # one launch chunk of all members
    try:
        sh, pop = c.population(ctx)
        run_ops(pop, B, ops)
        rho, _, err = pop.read()
        tr = pop.trace()
        pop.close()
        few = sh.population(c.rho32[:2], c.supp8[:2])
        run_ops(few, B, ops)
        rho2, _, err2 = few.read()
        tr2 = few.trace()
        few.close()
        sh.close()
    finally:
        ctx.set_variant(n, 0)
        ctx.set_cache_budget(256 << 20)
    np.testing.assert_array_equal(rho[:2], rho2)
    np.testing.assert_array_equal(err[:2], err2)
    np.testing.assert_array_equal(tr[:, :2], tr2)
    for p in (0, P // 2, P - 1):
        ref = mpr.sequence(c.rho[p], c.S[p], c.M, c.known, 0.5, "RAAR", 0.9, 2, 1)
        assert rel(rho[p], ref) <= 1e-5, p
        e_ref = mpr.get_error(ref, c.S[p], c.M, c.known)
        assert abs(err[p] - e_ref) <= 1e-5 * e_ref


def test_member_chunks_do_not_change_results(ctx, B):
    # one launch (the 20 members' 80 MiB of work buffers fit the budget), the
    # budget rule's chunks once they do not (3/4 of 40 MiB: 7, 7, 6 members)
    # and an explicit chunk of 5: the same bits
    n, P = 512, 20
    c = Case(n, P, seed=5120)
    ops = [B.op(B.OP_RAAR, count=3, beta=0.9, chi=0.5), B.op(B.OP_ER, count=2, chi=0.5), B.op(B.OP_GET_ERROR)]
    outs = []
    try:
        for budget, chunk in ((256 << 20, 0), (40 << 20, 0), (256 << 20, 5)):
            ctx.set_cache_budget(budget)
            ctx.set_variant(n, 0, chunk)
            sh, pop = c.population(ctx)
            run_ops(pop, B, ops)
            rho, _, err = pop.read()
            outs.append((rho, err))
            pop.close()
            sh.close()
    finally:
        ctx.set_cache_budget(256 << 20)
        ctx.set_variant(n, 0)
    for rho, err in outs[1:]:
        np.testing.assert_array_equal(rho, outs[0][0])
        np.testing.assert_array_equal(err, outs[0][1])
    ref = mpr.sequence(c.rho[0], c.S[0], c.M, c.known, 0.5, "RAAR", 0.9, 3, 2)
    assert rel(outs[0][0][0], ref) <= 1e-5


# ---------------------------------------------------------------------------
# Full-size launch configuration of the benchmark: 512^2, P = 64 memetic
# (128 members), sampled members checked against the oracle one by one.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed,sample", [(512, 1004, (0, 37, 63)), (1024, 1002, (0, 63))])
def test_full_size_sampled(ctx, B, n, seed, sample):
    # 512^2 is the benchmark's shot, 1024^2 the large MPR shot; P = 64 memetic
    # (128 members), launched in the benchmark's member chunks
    P = 64
    c = Case(n, P, seed=seed, kind="spheres", photons=1e8, gap=4, side=180)
    ctx.set_cache_budget(256 << 20)
    sh, pop = c.population(ctx, memetic=True, seed=seed + 2000)
    run_ops(pop, B, [B.op(B.OP_RAAR, count=1, beta=0.9, chi=0.5), B.op(B.OP_ER, count=1, chi=0.5),
                     B.op(B.OP_GET_ERROR, scope=B.SCOPE_PARENTS)])
    rho, _, err = pop.read()
    for p in sample:
        ref = mpr.sequence(c.rho[p], c.S[p], c.M, c.known, 0.5, "RAAR", 0.9, 1, 1)
        assert rel(rho[p], ref) <= 1e-5
        e_ref = mpr.get_error(ref, c.S[p], c.M, c.known)
        assert abs(err[p] - e_ref) <= 1e-5 * e_ref
    pop.close()
    sh.close()


def test_invalid_inputs_are_rejected(ctx, B):
    n = 32
    c = Case(n, 3, seed=2)
    with pytest.raises(B.SprError) as e:
        ctx.shot(np.zeros((20, 20), np.float32), np.ones((20, 20), np.uint8))
    assert e.value.code == -2
    bad = c.amp32.copy()
    bad[3, 3] = np.nan
    with pytest.raises(B.SprError) as e:
        ctx.shot(bad, c.mask8)
    assert e.value.code == -7
    with pytest.raises(B.SprError) as e:
        ctx.shot(c.amp32, np.zeros_like(c.mask8))
    assert e.value.code == -1
    sh, pop = c.population(ctx, memetic=True)   # P = 3 < 4
    with pytest.raises(B.SprError):
        run_ops(pop, B, [B.op(B.OP_CROSSOVER, gen=1, c_p=0.5, c_w=0.4)])
    with pytest.raises(B.SprError) as e:
        sh.close()
    assert e.value.code == -6
    pop.close()
    sh.close()


def test_launch_timing_counts_and_sampling(ctx, B):
    # every launch timed, then one in every 4: counts follow the schedule
    c = Case(64, 3, seed=21)
    sh, pop = c.population(ctx)
    sched = B.sched_ops([B.op(B.OP_RAAR, count=6, beta=0.9, chi=0.5), B.op(B.OP_ER, count=6, chi=0.5)], ctx)
    pop.timing(True)
    pop.run(sched)
    n_col, ms_col = pop.timing_read(B.KERNEL_COL_PROJ)
    n_ia, _ = pop.timing_read(B.KERNEL_ROW_UPDATE_IA)
    n_er, _ = pop.timing_read(B.KERNEL_ROW_UPDATE_ER)
    assert (n_col, n_ia + n_er) == (12, 12) and ms_col > 0
    pop.timing_sample(4)
    pop.timing(True)
    pop.run(sched)
    assert pop.timing_read(B.KERNEL_COL_PROJ)[0] == 3
    with pytest.raises(B.SprError):
        pop.timing_sample(0)
    pop.close()
    sh.close()
