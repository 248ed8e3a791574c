"""The ABI's host-side validation under AddressSanitizer and
UndefinedBehaviorSanitizer, without a GPU: the two host translation units
(ddm_api.cpp, mlp_api.cpp) are rebuilt with host-only instrumentation and
linked with the library's kernel objects; a driver (sanitize/abi_validation.cpp)
calls every entry point with refused arguments and dead handles."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not installed")
def test_abi_validation_under_sanitizers(libddm_path, tmp_path):
    from paper_2012_05695_amd import build as b
    hip = b.HIPCC
    inst = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in ("ddm_api.cpp", "mlp_api.cpp"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.check_call([hip, "-x", "hip", "-c", os.path.join(b.CSRC, src), "-o", obj] + b.COMMON + inst)
        objs.append(obj)
    kernels = [os.path.join(b.BUILD, f) for f in sorted(os.listdir(b.BUILD))
               if f.endswith(".o") and f not in ("ddm_api.o", "mlp_api.o")]
    lib = str(tmp_path / "libddm_san.so")
    subprocess.check_call([hip, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", lib] + objs + kernels)
    exe = str(tmp_path / "abi_validation")
    san = "address,undefined"
    subprocess.check_call([CLANG, "-std=c++17", "-g", "-fsanitize=" + san, "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize",
                                                                              "abi_validation.cpp"),
                           lib, "-Wl,-rpath," + str(tmp_path), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "all refusals as expected" in r.stdout
