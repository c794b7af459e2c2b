"""The C-ABI library on the host: it loads, exports every function cmp.h
declares, and its host-side logic (argument validation, schedules, stream
sizes) behaves as documented. No call here reaches a GPU: every call either
computes on the host or is rejected before anything is enqueued."""
import ctypes
import os
import re

import pytest

import oracle
import paper_1902_08755_amd as cmp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "cmp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cmp_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_function():
    names = _declared()
    assert len(names) >= 20
    L = ctypes.CDLL(cmp.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_rle_occupancy_cap_arguments():
    # host-side only: negative caps are rejected, 0 restores the default
    L = cmp.lib()
    assert L.cmp_rle_set_groups_per_cu(-1, 0) == cmp.CMP_EINVAL
    assert L.cmp_rle_set_groups_per_cu(0, -2) == cmp.CMP_EINVAL
    assert L.cmp_rle_set_groups_per_cu(3, 3) == cmp.CMP_OK
    assert L.cmp_rle_set_groups_per_cu(0, 0) == cmp.CMP_OK


def test_version_and_status_strings():
    assert "gfx950" in cmp.version()
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert cmp.lib().cmp_status_string(s)


def test_schedule_regions():
    # binary swap over 16 owners: recursive halving along the longer side
    r = cmp.schedule_regions(("binary_swap", 16), (0, 0, 1920, 1080))
    assert len(r) == 16 and all(w == 480 and h == 270 for _, _, w, h in r)
    assert sorted((x, y) for x, y, _, _ in r) == sorted(
        (480 * i, 270 * j) for i in range(4) for j in range(4))
    # odd sizes: the first half is floor(len / 2); rows split on a tie
    assert cmp.schedule_regions(("binary_swap", 2), (3, 4, 5, 5)) == [(3, 4, 5, 2), (3, 6, 5, 3)]
    assert cmp.schedule_regions(("binary_swap", 2), (0, 0, 7, 3)) == [(0, 0, 3, 3), (3, 0, 4, 3)]
    # direct send strips: [floor(k H / P), floor((k+1) H / P))
    assert cmp.schedule_regions(("direct_send", 3), (0, 0, 10, 7)) == [
        (0, 0, 10, 2), (0, 2, 10, 2), (0, 4, 10, 3)]
    # more owners than rows: empty strips are left out; the union still tiles
    r = cmp.schedule_regions(("direct_send", 5), (0, 0, 4, 3))
    assert sum(w * h for _, _, w, h in r) == 12
    assert cmp.schedule_regions("seq", (1, 2, 3, 4)) == [(1, 2, 3, 4)]
    for bad in [("binary_swap", 3), ("binary_swap", 128), ("direct_send", 0), (7, 1)]:
        with pytest.raises(cmp.CmpError):
            cmp.schedule_regions(bad, (0, 0, 8, 8))


@pytest.mark.parametrize("P", [1, 2, 4, 8, 16, 32, 64])
def test_schedule_regions_partition_viewport(P):
    for vp in [(0, 0, 1920, 1080), (5, 7, 33, 17), (0, 0, 1, 1)]:
        for kind in ("binary_swap", "direct_send"):
            r = cmp.schedule_regions((kind, P), vp)
            covered = set()
            for x, y, w, h in r:
                cells = {(i, j) for i in range(x, x + w) for j in range(y, y + h)} if vp[2] * vp[3] < 2000 else None
                if cells is not None:
                    assert not (covered & cells)
                    covered |= cells
            assert sum(w * h for _, _, w, h in r) == vp[2] * vp[3]


def test_rle_max_size_matches_format():
    for w, h, npl in [(0, 0, 8), (1, 1, 8), (4096, 1, 4), (4097, 1, 8), (1920, 1080, 8), (13, 7, 4)]:
        assert cmp.rle_max_size(w, h, npl) == oracle.rle_max_size(w, h, npl)


def _img(roi, color=0x1000, depth=0x2000, pitch=None):
    return cmp.CImage(color, depth, roi[2] if pitch is None else pitch, cmp.Rect(*roi))


def _arr(imgs):
    a = (cmp.CImage * max(1, len(imgs)))()
    for i, im in enumerate(imgs):
        a[i] = im
    return a


SEQ = cmp.Schedule(0, 1)


def test_depth_argument_errors():
    L = cmp.lib()
    vp = cmp.Rect(0, 0, 8, 8)
    ok = _arr([_img((0, 0, 8, 8))])
    call = lambda imgs, n, **kw: L.cmp_composite_depth(
        imgs, n, kw.get("roi"), kw.get("vp", vp), kw.get("oc", 0x4000), kw.get("od", 0x5000),
        kw.get("op", 8), kw.get("sched", SEQ), cmp.Tile(*kw.get("tile", (0, 0))), None)
    assert call(ok, -1) == cmp.CMP_EINVAL
    assert call(None, 1) == cmp.CMP_EINVAL
    assert call(_arr([_img((0, 0, 8, 8), pitch=7)]), 1) == cmp.CMP_EINVAL
    assert call(_arr([_img((0, 0, -1, 8))]), 1) == cmp.CMP_EINVAL
    assert call(_arr([_img((0, 0, 8, 8), depth=None)]), 1) == cmp.CMP_EINVAL
    assert call(_arr([_img((0, 0, 8, 8), color=0x1002)]), 1) == cmp.CMP_EINVAL
    assert call(ok, 1, oc=None) == cmp.CMP_EINVAL
    assert call(ok, 1, op=7) == cmp.CMP_EINVAL
    assert call(ok, 1, vp=cmp.Rect(0, 0, -2, 3)) == cmp.CMP_EINVAL
    assert call(ok, 1, sched=cmp.Schedule(2, 3)) == cmp.CMP_EINVAL
    assert call(ok, 1, sched=cmp.Schedule(9, 1)) == cmp.CMP_EINVAL
    assert call(ok, 1, tile=(-4, 4)) == cmp.CMP_EINVAL
    assert call(ok, 1, roi=0x1004) == cmp.CMP_EINVAL   # misaligned device ROI table
    many = _arr([_img((0, 0, 8, 8))] * 49)
    assert call(many, 49, od=None) == cmp.CMP_EINVAL     # multi-pass needs out_depth
    assert L.cmp_last_error()
    # an empty viewport is a no-op that succeeds without touching the GPU
    assert call(ok, 1, vp=cmp.Rect(0, 0, 0, 5)) == cmp.CMP_OK


def test_over_argument_errors():
    L = cmp.lib()
    vp = cmp.Rect(0, 0, 8, 8)
    ok = _arr([_img((0, 0, 8, 8), color=0x10000, depth=None)] * 3)
    order = lambda *v: (ctypes.c_int32 * len(v))(*v)
    call = lambda imgs, n, fmt=cmp.RGBA32F, o=order(0, 1, 2), **kw: L.cmp_composite_over(
        imgs, n, fmt, o, kw.get("vp", vp), kw.get("out", 0x20000), kw.get("op", 8),
        kw.get("sched", SEQ), cmp.Tile(0, 0), None)
    assert call(ok, 3, o=order(0, 1, 1)) == cmp.CMP_EINVAL      # not a permutation
    assert call(ok, 3, o=order(0, 1, 3)) == cmp.CMP_EINVAL
    assert call(ok, 3, fmt=cmp.RGBA8) == cmp.CMP_EINVAL
    assert call(_arr([_img((0, 0, 8, 8), color=0x10008, depth=None)] * 3), 3) == cmp.CMP_EINVAL
    assert call(ok, 3, out=0x20008) == cmp.CMP_EINVAL           # output must be 16-aligned
    assert call(ok, 3, op=4) == cmp.CMP_EINVAL
    big = _arr([_img((0, 0, 8, 8), color=0x10000, depth=None)] * 65)
    assert call(big, 65, o=order(*range(65)), sched=cmp.Schedule(2, 2)) == cmp.CMP_EUNSUPPORTED
    gl = (ctypes.c_void_p * 3)(0x30000, 0x30000, 0x30000)
    gp = (ctypes.c_int64 * 3)(8, 8, 4)
    assert L.cmp_composite_over_backward(ok, 3, cmp.RGBA32F, order(0, 1, 2), vp, 0x40000, 8, gl,
                                         gp, None, 0, None) == cmp.CMP_EINVAL
    # more than 64 layers: the descriptors need a workspace; at most 256 layers
    assert L.cmp_over_backward_workspace_size(64) == 0
    need = L.cmp_over_backward_workspace_size(65)
    assert need >= 65 * 40 and L.cmp_over_backward_workspace_size(257) == 0
    gl65 = (ctypes.c_void_p * 65)(*([0x30000] * 65))
    gp65 = (ctypes.c_int64 * 65)(*([8] * 65))
    assert L.cmp_composite_over_backward(big, 65, cmp.RGBA32F, order(*range(65)), vp, 0x40000, 8,
                                         gl65, gp65, None, 0, None) == cmp.CMP_EINVAL
    assert L.cmp_composite_over_backward(big, 65, cmp.RGBA32F, order(*range(65)), vp, 0x40000, 8,
                                         gl65, gp65, 0x50000, need - 16, None) == cmp.CMP_ENOSPC
    huge = _arr([_img((0, 0, 8, 8), color=0x10000, depth=None)] * 257)
    gl257 = (ctypes.c_void_p * 257)(*([0x30000] * 257))
    gp257 = (ctypes.c_int64 * 257)(*([8] * 257))
    assert L.cmp_composite_over_backward(huge, 257, cmp.RGBA32F, order(*range(257)), vp, 0x40000,
                                         8, gl257, gp257, 0x50000, 1 << 20,
                                         None) == cmp.CMP_EUNSUPPORTED


def test_roi_and_rle_argument_errors():
    L = cmp.lib()
    imgs = _arr([_img((0, 0, 64, 64))] * 2)
    out = (ctypes.c_int32 * 8)()
    assert L.cmp_roi_detect(imgs, 65, 0, 0x1000, 0x2000, 1 << 20, None) == cmp.CMP_EINVAL
    assert L.cmp_roi_detect(imgs, 2, 0, None, 0x2000, 1 << 20, None) == cmp.CMP_EINVAL
    ws = L.cmp_roi_workspace_size(imgs, 2)
    assert ws > 256
    assert L.cmp_roi_detect(imgs, 2, 0, 0x1000, 0x2000, ws - 16, None) == cmp.CMP_ENOSPC
    mixed = _arr([_img((0, 0, 64, 64)), _img((0, 0, 64, 64), depth=None)])
    assert L.cmp_roi_detect(mixed, 2, 0, 0x1000, 0x2000, 1 << 20, None) == cmp.CMP_EINVAL
    # RLE: capacities below the bound, misaligned outputs, unsupported formats
    outs = (ctypes.c_void_p * 2)(0x100000, 0x200000)
    need = cmp.rle_max_size(64, 64, 8)
    caps = (ctypes.c_uint64 * 2)(need, need - 1)
    wsz = L.cmp_rle_workspace_size(imgs, 2)
    assert L.cmp_rle_compress(imgs, 2, cmp.RGBA8, 0, None, outs, caps, 0x3000, 0x3800, 0x4000, wsz,
                              None) == cmp.CMP_ENOSPC
    caps[1] = need
    assert L.cmp_rle_compress(imgs, 2, cmp.RGBA8, 0, None, outs, caps, 0x3000, 0x3800, 0x4000, wsz - 8,
                              None) == cmp.CMP_ENOSPC
    assert L.cmp_rle_compress(imgs, 2, cmp.RGBA32F, 0, None, outs, caps, 0x3000, 0x3800, 0x4000, wsz,
                              None) == cmp.CMP_EUNSUPPORTED
    # the status array is required
    assert L.cmp_rle_compress(imgs, 2, cmp.RGBA8, 0, None, outs, caps, 0x3000, None, 0x4000, wsz,
                              None) == cmp.CMP_EINVAL
    assert L.cmp_rle_set_wait_limit(5) == 0 and L.cmp_rle_set_wait_limit(-1) == 0
    bad = (ctypes.c_void_p * 2)(0x100008, 0x200000)
    assert L.cmp_rle_compress(imgs, 2, cmp.RGBA8, 0, None, bad, caps, 0x3000, 0x3800, 0x4000, wsz,
                              None) == cmp.CMP_EINVAL
    ins = (ctypes.c_void_p * 1)(0x100004)
    nb = (ctypes.c_uint64 * 1)(100)
    assert L.cmp_rle_decompress(ins, nb, 1, imgs, None, 0x5000, None) == cmp.CMP_EINVAL
    assert L.cmp_rle_decompress(ins, nb, 1, imgs, None, None, None) == cmp.CMP_EINVAL


def test_rle_compress_noalloc_rejects_inputs_beyond_its_scratch():
    # 131072 blocks of 4096 pixels is the static scratch's limit; 64 images
    # of 4096x4096 need 262144 (checked on the host, nothing is launched)
    L = cmp.lib()
    big = cmp.CImage()
    big.roi = cmp.Rect(0, 0, 4096, 4096)
    arr = (cmp.CImage * 64)(*([big] * 64))
    assert L.cmp_rle_workspace_size(arr, 64) == 8192 + 256 + 8 * 262144
    st = L.cmp_rle_compress_noalloc(arr, 64, cmp.RGBA8, 0, None, None, None, None, None, None)
    assert st == cmp.CMP_ENOSPC
    assert "static maximum" in L.cmp_last_error().decode()
    # n out of range and negative sizes are rejected first
    assert L.cmp_rle_compress_noalloc(arr, 65, cmp.RGBA8, 0, None, None, None, None, None,
                                      None) == cmp.CMP_EINVAL
    bad = cmp.CImage()
    bad.roi = cmp.Rect(0, 0, -1, 5)
    assert L.cmp_rle_compress_noalloc((cmp.CImage * 1)(bad), 1, cmp.RGBA8, 0, None, None, None,
                                      None, None, None) == cmp.CMP_EINVAL


def test_rle64_max_size_matches_oracle():
    L = cmp.lib()
    for w, h in [(0, 0), (1, 1), (3, 4), (300, 1), (4097, 1), (64, 64), (4096, 3), (1920, 1080),
                 (2049, 2)]:
        for ns in (1, 2):
            assert L.cmp_rle64_max_size(w, h, ns) == oracle.rle64_max_size(w, h, ns), (w, h, ns)
    assert L.cmp_rle64_max_size(4, 4, 3) == 0 and L.cmp_rle64_max_size(-1, 4, 1) == 0


def test_streams_create_rejects_bad_counts():
    # checked before any HIP call
    L = cmp.lib()
    arr = (ctypes.c_void_p * 17)()
    for count in (0, -1, 17):
        assert L.cmp_streams_create(count, arr) == cmp.CMP_EINVAL
    assert L.cmp_streams_create(2, None) == cmp.CMP_EINVAL
    assert L.cmp_streams_destroy(-1, arr) == cmp.CMP_EINVAL
    assert L.cmp_streams_destroy(1, None) == cmp.CMP_EINVAL
    assert L.cmp_streams_destroy(0, None) == 0


def test_cmp_log_writes_plans_to_stderr():
    # CMP_LOG=1: a schedule plan (host-only call) is written to stderr as one
    # "[cmp] ..." line; without it nothing is written
    import subprocess
    import sys
    code = ("import paper_1902_08755_amd as cmp; L = cmp.lib(); "
            "out = (cmp.Rect * 64)(); "
            "n = L.cmp_schedule_regions(cmp.Schedule(cmp.BINARY_SWAP, 16), cmp.Rect(0, 0, 1920, 1080), out, 64); "
            "assert n == 16, n")
    env = dict(os.environ, CMP_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = [l for l in r.stderr.splitlines() if l.startswith("[cmp] ")]
    assert len(lines) == 1 and "16 regions" in lines[0] and "1920x1080" in lines[0], r.stderr
    env.pop("CMP_LOG")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0 and "[cmp]" not in r.stderr, r.stderr


def test_autotune_without_cache_path_or_env_is_rejected():
    # no path and CMP_TUNE_CACHE unset: rejected on the host, nothing runs
    L = cmp.lib()
    saved = os.environ.pop("CMP_TUNE_CACHE", None)
    try:
        job = cmp.CJob()
        assert L.cmp_autotune(ctypes.byref(job), 1, None, 1, None) == cmp.CMP_EINVAL
        assert "CMP_TUNE_CACHE" in L.cmp_last_error().decode()
    finally:
        if saved is not None:
            os.environ["CMP_TUNE_CACHE"] = saved


def test_cmp_roctx_loads_ranges_only_when_asked():
    # CMP_ROCTX=1: the first entry point that enqueues work loads the roctx
    # library (CMP_LOG reports it) and opens a range; the call itself behaves
    # as without it (here: rejected on the host)
    import subprocess
    import sys
    code = ("import paper_1902_08755_amd as cmp; L = cmp.lib(); "
            "st = L.cmp_composite_depth(None, 2, None, cmp.Rect(0, 0, 8, 8), None, None, 8, "
            "cmp.Schedule(cmp.SEQ, 1), cmp.Tile(0, 0), None); "
            "assert st == cmp.CMP_EINVAL, st; "
            "st = L.cmp_composite_depth(None, 2, None, cmp.Rect(0, 0, 8, 8), None, None, 8, "
            "cmp.Schedule(cmp.SEQ, 1), cmp.Tile(0, 0), None); "
            "assert st == cmp.CMP_EINVAL, st")
    env = dict(os.environ, CMP_ROCTX="1", CMP_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = [l for l in r.stderr.splitlines() if l.startswith("[cmp] roctx")]
    assert lines == ["[cmp] roctx ranges on"], r.stderr
    env.pop("CMP_ROCTX")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0 and "roctx" not in r.stderr, r.stderr
