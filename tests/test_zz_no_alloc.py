"""The allocation-free propagation entry point (for callers that cannot
allocate) against the allocating one, through the C ABI: two calls in a row,
the second on a smaller input, with and without a caller stream, and the
size limit of its static scratch."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

D, LAM = 8e-6, 520e-9


@pytest.fixture(scope="module")
def ctx():
    import paper_2606_14173_amd as hpt
    c = hpt.Context(0)
    yield c
    c.close()


def _noalloc(ctx, src, dst, n, w, h, z, flags=1, stream=None):
    return ctx.lib.hpt_asm_propagate_noalloc(ctx.h, src.data_ptr(), dst.data_ptr(), n, w, h, D, LAM, z, flags,
                                             stream)


def _fields(n, h, w, seed):
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    re = torch.randn((n, h, w), generator=g)
    im = torch.randn((n, h, w), generator=g)
    return torch.complex(re, im).to(torch.complex64).to("cuda:0")


@pytest.mark.parametrize("use_stream", [False, True])
def test_noalloc_equals_allocating_propagation(ctx, use_stream):
    """Same kernels, same arguments: the output equals the allocating entry
    point's bit for bit, on a 1920 x 1080 field and then (the scratch keeping
    the first call's contents) on three 100 x 30 fields."""
    import torch
    import paper_2606_14173_amd as hpt
    s = torch.cuda.Stream() if use_stream else None
    for n, w, h, z, seed in ((1, 1920, 1080, 80e-3, 1), (3, 100, 30, -5e-3, 2)):
        src = _fields(n, h, w, seed)
        ref = torch.empty_like(src)
        out = torch.full_like(src, float("nan"))
        ctx.asm_propagate(src, ref, n, w, h, D, LAM, z)
        torch.cuda.synchronize()
        if s is not None:
            with torch.cuda.stream(s):
                st = _noalloc(ctx, src, out, n, w, h, z, stream=s.cuda_stream)
            s.synchronize()
        else:
            st = _noalloc(ctx, src, out, n, w, h, z)
        assert hpt.STATUS[st] == "HPT_OK", ctx.lib.hpt_last_error()
        assert torch.equal(out, ref), (n, w, h)
        rms = float(torch.sqrt(torch.mean(torch.abs(ref) ** 2)))
        assert rms > 0


def test_noalloc_rejects_what_does_not_fit(ctx):
    """Fields whose padded work buffers exceed the static scratch, and bad
    arguments, are refused before anything runs."""
    import torch
    import paper_2606_14173_amd as hpt
    buf = torch.zeros((1, 8, 8), dtype=torch.complex64, device="cuda:0")
    big = torch.zeros((1, 2048, 2048), dtype=torch.complex64, device="cuda:0")   # 2 * 2048 * 4096 > limit
    assert hpt.STATUS[_noalloc(ctx, big, big, 1, 2048, 2048, 1e-3)] == "HPT_EINVAL"
    for n, w, h, z, flags in ((0, 8, 8, 1e-3, 1), (1, 0, 8, 1e-3, 1), (1, 8, 8, float("nan"), 1), (1, 8, 8, 1e-3, 4)):
        assert hpt.STATUS[_noalloc(ctx, buf, buf, n, w, h, z, flags)] == "HPT_EINVAL"
