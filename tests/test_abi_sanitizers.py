"""The host side of the C ABI under AddressSanitizer and UndefinedBehavior-
Sanitizer (CPU only).  Every libqless source is compiled for the host alone
with both sanitizers, linked with abi_host_check.c (size queries over a grid
of arguments, the tuning table, batch plans, the argument checks of the entry
points -- nothing that reaches a kernel launch) and run; any sanitizer report
or failed expectation fails the test.  A host-only compile does not produce
the device binaries the objects refer to; since nothing is launched, zero-
filled stand-ins for those symbols satisfy the link (the runtime reads a
device binary only when one of its kernels is loaded)."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_20889_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
NM = shutil.which("nm") or shutil.which("llvm-nm") or os.path.join(ROCM, "llvm", "bin", "llvm-nm")


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert r.returncode == 0, "%s\n%s" % (" ".join(cmd), r.stdout[-4000:])
    return r.stdout


@pytest.mark.skipif(not all(os.path.exists(p) for p in (HIPCC, CLANG, CLANGXX, NM)), reason="ROCm toolchain missing")
def test_abi_host_code_under_sanitizers(tmp_path):
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    flags = ["--offload-arch=gfx950", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, *flags, "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    harness = str(tmp_path / "harness.o")
    _run([CLANG, "-O1", "-g", *san, "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROCM, "include"),
          "-D__HIP_PLATFORM_AMD__", "-c", os.path.join(ROOT, "tests", "abi_host_check.c"), "-o", harness])
    syms = sorted({line.split()[-1] for line in _run([NM, "-u", *objs]).splitlines()
                   if line.split() and line.split()[-1].startswith("__hip_fatbin_")})
    stub_c = tmp_path / "device_binary_stand_ins.c"
    stub_c.write_text("".join("char %s[64];\n" % s for s in syms))
    stub = str(tmp_path / "stand_ins.o")
    _run([CLANG, "-c", str(stub_c), "-o", stub])
    exe = str(tmp_path / "abi_check")
    lib = os.path.join(ROCM, "lib")
    _run([CLANGXX, *san, *objs, harness, stub, "-o", exe, "-L" + lib, "-lamdhip64", "-lrocblas",
          "-Wl,-rpath," + lib])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=300)
    assert "AddressSanitizer" not in r.stdout and "runtime error" not in r.stdout, r.stdout[-4000:]
    assert r.returncode == 0, r.stdout[-4000:]
