"""mrs_render_ex_noalloc (the render whose workspace is a fixed device array)
against mrs_render_ex, through the C ABI: bitwise the same images, on calls in a
row that reuse the array (the second smaller than the first), with no device
memory taken by the calls."""
import ctypes as C
import sys

import numpy as np
import pytest

from mrs_inputs import scenes as S

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _opts(sumsq=None, layers=None):
    from paper_2106_12802_amd import _lib
    o = _lib.RenderOpts()
    _lib.lib().mrs_render_opts_default(C.byref(o))
    o.out_sumsq_dev = None if sumsq is None else sumsq.data_ptr()
    o.out_layers_dev = None if layers is None else layers.data_ptr()
    return o


def _outputs(torch, W, H, extra):
    f = dict(dtype=torch.float32, device="cuda")
    out = {"rgb": torch.full((H, W, 3), -1.0, **f), "aux": torch.full((H, W, 7), -1.0, **f)}
    if extra:
        out["sumsq"] = torch.full((H, W, 3), -1.0, **f)
        out["layers"] = torch.full((H, W, 9), -1.0, **f)
    return out


def _call(fn, gs, W, H, spp, D, seed, out):
    from paper_2106_12802_amd import _lib
    _lib.use_current_stream()
    o = _opts(out.get("sumsq"), out.get("layers"))
    return fn(gs.handle, W, H, spp, D, C.c_uint64(seed), C.byref(o), out["rgb"].data_ptr(),
              out["aux"].data_ptr())


def _render_both(torch, gs, W, H, spp, D, seed, extra):
    from paper_2106_12802_amd import _lib
    L = _lib.lib()
    ref = _outputs(torch, W, H, extra)
    _lib.check(_call(L.mrs_render_ex, gs, W, H, spp, D, seed, ref))
    torch.cuda.synchronize()
    got = _outputs(torch, W, H, extra)
    free0 = torch.cuda.mem_get_info()[0]
    _lib.check(_call(L.mrs_render_ex_noalloc, gs, W, H, spp, D, seed, got))
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return ref, got, free0 - free1


def test_noalloc_matches_render_ex_on_calls_in_a_row(torch_cuda):
    import paper_2106_12802_amd as mrs
    torch = torch_cuda
    big = mrs.GpuScene(S.procedural(7))
    small = mrs.GpuScene(S.cornell(2))
    # warm-up: the first launch on a device loads the library's device code
    # (and with it the static array); later calls must take no device memory
    _render_both(torch, small, 8, 8, 1, 1, 1, False)
    # first call: the LRHS image of the bench scene, 3.7 M paths (14 super-chunks
    # of the 2^18 resident paths), depth 8, features
    ref, got, taken = _render_both(torch, big, 320, 180, 64, 8, 15, False)
    _log(f"noalloc 320x180@64: device memory taken by the call {taken} B")
    for k in ref:
        assert torch.equal(ref[k], got[k]), k
    assert taken == 0
    # second call, smaller, on another scene, with squares and render layers
    # (the array still holds the first call's pixel sums and counters)
    ref, got, taken = _render_both(torch, small, 64, 48, 16, 4, 1002, True)
    _log(f"noalloc 64x48@16 (+ squares, layers): device memory taken {taken} B")
    for k in ref:
        assert torch.equal(ref[k], got[k]), k
    assert taken == 0
    # FP64 sums (spp >= 1024), then FP32 sums again in the same array
    for W, H, spp, seed in [(24, 16, 1024, 2 ** 40 + 5), (40, 40, 8, 77)]:
        ref, got, taken = _render_both(torch, small, W, H, spp, 4, seed, False)
        for k in ref:
            assert torch.equal(ref[k], got[k]), (W, H, spp, k)
        assert taken == 0


def test_noalloc_refuses_windows_beyond_its_workspace(torch_cuda):
    """2^19 FP64 pixel sums fit; one pixel more does not (INVALID_ARGUMENT, nothing
    written); the same size with FP32 sums fits."""
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import _lib
    torch = torch_cuda
    gs = mrs.GpuScene(S.cornell(1))
    L = _lib.lib()
    W, H = 1024, 513  # 2^19 + 1024 pixels
    out = _outputs(torch, W, H, False)
    o = _opts()
    o.accum_fp64 = 1
    _lib.use_current_stream()
    rc = L.mrs_render_ex_noalloc(gs.handle, W, H, 1, 1, C.c_uint64(3), C.byref(o),
                                 out["rgb"].data_ptr(), out["aux"].data_ptr())
    assert rc == 1 and b"render it in windows" in L.mrs_last_error()
    torch.cuda.synchronize()
    assert torch.all(out["rgb"] == -1.0) and torch.all(out["aux"] == -1.0)
    o.accum_fp64 = 0  # 13 FP32 values per pixel: fits
    assert L.mrs_render_ex_noalloc(gs.handle, W, H, 1, 1, C.c_uint64(3), C.byref(o),
                                   out["rgb"].data_ptr(), out["aux"].data_ptr()) == 0
    torch.cuda.synchronize()
    ref, _ = mrs.render(gs, W, H, 1, 1, 3, accum_fp64=0)
    torch.cuda.synchronize()
    assert torch.equal(ref, out["rgb"])
