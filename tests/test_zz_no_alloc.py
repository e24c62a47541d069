"""The allocation-free form of the unitary 2D FFT entry point
(spr_fft2_noalloc, for callers that cannot allocate device memory) against
the ordinary one (spr_fft2) and the FP64 oracle, through the C ABI.

Both forms run the same row and column transform kernels; the allocation-free
one takes its twiddles (computed on the device in FP64, rounded once) and the
row-transform intermediate from the library's fixed device scratch array.
Bars: against spr_fft2 1e-6 relative L2 (the transforms agree to FP32
rounding), against the oracle 1e-5 (single operator).  The scratch array
keeps the last call's contents, so calls follow each other with changing
sizes, the second smaller than the first.
"""

import numpy as np
import pytest

from oracle import mpr
from paper_2409_07413_amd import synth

from gpu_cases import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2409_07413_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def _check(ctx, n, batch, seed, inverse):
    import torch
    x = synth.random_complex((batch, n, n), seed).astype(np.complex64)
    xt = torch.from_numpy(x).cuda()
    ref = torch.empty_like(xt)
    got = torch.full_like(xt, float("nan"))
    ctx.fft2(xt, ref, inverse=inverse)
    ctx.fft2_noalloc(xt, got, inverse=inverse)
    g, r = got.cpu().numpy(), ref.cpu().numpy()
    assert np.all(np.isfinite(g))
    assert rel(g, r) <= 1e-6, (n, batch, rel(g, r))
    fn = mpr.ifft2 if inverse else mpr.fft2
    for b in (0, batch - 1):
        assert rel(g[b], fn(x[b].astype(np.complex128))) <= 1e-5, (n, b)
    np.testing.assert_array_equal(xt.cpu().numpy(), x)  # the input is left as it was
    return float(rel(g, r))


def test_noalloc_fft2_twice_second_smaller(ctx):
    # two calls in a row on one device, the second with a smaller input, in
    # both directions; then again the larger one (the array keeps stale data)
    d1 = _check(ctx, 512, 6, 11, False)
    d2 = _check(ctx, 256, 2, 12, False)
    d3 = _check(ctx, 512, 6, 13, True)
    d4 = _check(ctx, 96, 3, 14, True)
    print(f"noalloc vs spr_fft2 rel L2: {d1:.1e} {d2:.1e} {d3:.1e} {d4:.1e}")


def test_noalloc_fft2_largest_batch_and_in_place(ctx):
    # the largest batch the scratch array holds at 1024^2 (7 images), in place
    import torch
    n, batch = 1024, 7
    x = synth.random_complex((batch, n, n), 21).astype(np.complex64)
    buf = torch.from_numpy(x).cuda()
    ref = torch.empty_like(buf)
    ctx.fft2(buf, ref)
    ctx.fft2_noalloc(buf, buf)
    assert rel(buf.cpu().numpy(), ref.cpu().numpy()) <= 1e-6
    ctx.fft2_noalloc(buf, buf, inverse=True)
    assert rel(buf.cpu().numpy(), x) <= 1e-5


def test_noalloc_fft2_rejects_more_than_the_scratch_holds(ctx):
    import torch
    from paper_2409_07413_amd import binding
    x = torch.zeros((8, 1024, 1024), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(binding.SprError) as e:
        ctx.fft2_noalloc(x, y)
    assert e.value.code == -1
    with pytest.raises(binding.SprError) as e:
        ctx.fft2_noalloc(x[:, :1000, :1000].contiguous(), y[:, :1000, :1000].contiguous())
    assert e.value.code == -2
