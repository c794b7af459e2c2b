"""cmp_rle_compress_noalloc (tickets and look-back flags in the library's
static scratch array) against cmp_rle_compress (the same kernels with the
caller's workspace): byte-identical streams, sizes and statuses, on two
calls in a row, the second with a smaller input, through the C ABI."""
import ctypes

import pytest
import torch

import paper_1902_08755_amd as cmp
import synth

pytestmark = pytest.mark.gpu


def _noalloc(batch, roi_dev, stream):
    """The same arguments as RleBatch.run, without the workspace."""
    batch.status.zero_()
    L = cmp.lib()
    st = L.cmp_rle_compress_noalloc(batch.arr, batch.n, cmp.RGBA8, batch.flags,
                                    roi_dev.data_ptr() if roi_dev is not None else None,
                                    batch.out_ptrs, batch.cap_arr, batch.sizes.data_ptr(),
                                    batch.status.data_ptr(), stream)
    assert st == 0, L.cmp_last_error().decode()


def _compare(images, roi_dev, swizzle):
    s = torch.cuda.current_stream().cuda_stream
    ref = cmp.RleBatch(images, roi_dev, swizzle=swizzle)
    got = cmp.RleBatch(images, roi_dev, swizzle=swizzle)
    for o in got.outs:
        o.fill_(0x5A)   # bytes the call must overwrite
    ref.run()
    _noalloc(got, roi_dev, s)
    torch.cuda.synchronize()
    assert torch.equal(ref.status, got.status) and int(ref.status.abs().sum()) == 0
    assert torch.equal(ref.sizes, got.sizes)
    for i, (a, b) in enumerate(zip(ref.outs, got.outs)):
        k = int(ref.sizes[i])
        assert torch.equal(a[:k], b[:k]), f"stream {i} differs"


def test_noalloc_compress_matches_workspace_path_twice():
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    # first call: 16 contributors of 640x480, ROIs found on the device
    print("noalloc: 16 x 640x480 ramps, device ROIs", flush=True)
    wl = synth.depth_ramps_full(seed=7, n=16, W=640, H=480, device=dev)
    roi = cmp.roi_detect(wl.images)
    _compare(wl.images, roi, swizzle=False)
    # second call, smaller: 5 contributors of 200x150, swizzled colour,
    # whole images (more of them empty than not is fine: blocks are fewer)
    print("noalloc: 5 x 200x150 ramps, swizzled, whole images", flush=True)
    wl2 = synth.depth_ramps_full(seed=8, n=5, W=200, H=150, device=dev)
    _compare(wl2.images, None, swizzle=True)
    # and the large input once more: nothing of the small call leaks into it
    print("noalloc: first input again", flush=True)
    _compare(wl.images, roi, swizzle=False)



def test_noalloc_at_its_maximum_size():
    """64 whole images of 3840x2160: 129,600 blocks of 4096 pixels, the most
    that fit the scratch's 131,072 look-back flags in whole images of that
    size. The no-allocation call gives the workspace path's streams, and they
    decode to the images."""
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    print("noalloc: 64 x 3840x2160 ramps, whole images", flush=True)
    wl = synth.depth_ramps_full(seed=9, n=64, W=3840, H=2160, device=dev)
    L = cmp.lib()
    scratch_bytes = 8192 + 256 + 8 * 131072   # CMP_RLE_SCRATCH_BYTES in cmp.h
    assert L.cmp_rle_workspace_size(cmp._images(wl.images, "u32"), 64) <= scratch_bytes
    _compare(wl.images, None, swizzle=False)
    streams, sizes, st = cmp.rle_compress(wl.images)
    outs = [cmp.Image(torch.zeros_like(im.color), torch.zeros_like(im.depth), im.roi)
            for im in wl.images]
    ro, dst = cmp.rle_decompress(streams, outs)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0 and int(dst.abs().sum()) == 0
    for im, o in zip(wl.images, outs):
        assert torch.equal(o.color[:, :3840], im.color[:, :3840])
        assert torch.equal(o.depth[:, :3840], im.depth[:, :3840])
    del wl, outs, streams
    torch.cuda.empty_cache()
