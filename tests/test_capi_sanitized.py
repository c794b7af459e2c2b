"""The host side of libcmp under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer. The library's sources are built once more with the
sanitizers on the host code only (device code as in the product build), and a
C driver (tests/sanitize_capi.c) runs every host-side path that needs no GPU:
schedules, sizes, the argument checks of every entry point, and the batch
planner over 300 synthetic jobs with valid, malformed and truncated tune
caches. Any out-of-bounds access, leak (outside the HIP runtime) or undefined
behaviour aborts the run."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1902_08755_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="no ROCm toolchain")
def test_capi_host_side_under_asan_lsan_ubsan(tmp_path):
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [HIPCC, "-x", "hip", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC",
               "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libcmp_asan.so")
    r = subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *SAN, "-o", lib, *objs],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "capi_sanitized")
    r = subprocess.run([CLANG, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize_capi.c"),
                        "-L", str(tmp_path), "-lcmp_asan", "-Wl,-rpath," + str(tmp_path), "-o", exe],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    supp = tmp_path / "lsan.supp"   # allocations the HIP runtime keeps until exit
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libamd_comgr\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               LSAN_OPTIONS=f"suppressions={supp}",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    env.pop("CMP_TUNE_CACHE", None)
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "sanitized capi run: ok" in r.stdout
