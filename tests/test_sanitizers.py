"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the CPU.

* The FP64 oracle (plain C) built with gcc's ASan and UBSan and driven
  through its whole-run, single-transition, density, tile, MH, HMC and
  unadjusted-jump entry points.
* The library's host side (the C ABI sources: descriptor validation,
  parameter packing, layout arithmetic) built with clang's host sanitizers
  (-Xarch_host, the device code unchanged) and driven through
  restore_state_bytes, restore_batch_state_bytes and the learned part's
  argument checks with valid and invalid descriptors.  No device work.

Each run happens in a child process with the sanitizer runtime preloaded and
halts at the first report; a positive control (a read one past the end of a
heap block) shows that a report does fail the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_07148_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "sanitize_driver.py")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
       "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_asan_runtime():
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()


def _clang_asan_runtime():
    out = subprocess.run([os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang"),
                          "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        import glob
        hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        path = hits[0] if hits else ""
    return path


def _run(preload, *args):
    env = dict(os.environ, LD_PRELOAD=preload, **ENV)
    return subprocess.run([sys.executable, *args], capture_output=True, text=True, env=env, timeout=600)


def _clean(r):
    bad = ("ERROR: AddressSanitizer" in r.stderr) or ("runtime error:" in r.stderr)
    return r.returncode == 0 and not bad and "driver done" in r.stdout


def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = tmp_path / "liboracle_asan.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", str(lib),
                    os.path.join(ROOT, "oracle", "restore_oracle.c"), "-lm", "-lpthread"], check=True)
    r = _run(_gcc_asan_runtime(), DRIVER, "oracle", str(lib))
    assert _clean(r), r.stderr[-3000:]


def test_host_validation_under_asan_and_ubsan(tmp_path):
    build = os.path.join(ROOT, "_build")
    kernels = ["step_kernels.hip", "step_kernels_hmc.hip", "step_kernels_rwu.hip", "splat_kernels.hip",
               "reduce_kernels.hip", "batch_kernels.hip", "learn_kernels.hip"]
    if not all(os.path.exists(os.path.join(build, k + ".o")) for k in kernels):
        from paper_2409_07148_amd import build as libbuild
        libbuild.build()
    runtime = _clang_asan_runtime()
    if not runtime:
        pytest.skip("no clang AddressSanitizer runtime in this image")
    objs, procs = [], []
    for src in ("restore_api.cpp", "batch_api.cpp", "learn_api.cpp"):
        obj = tmp_path / (src + ".o")
        objs.append(str(obj))
        procs.append(subprocess.Popen(
            [HIPCC, "-O1", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-x", "hip",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", str(obj)],
            stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        assert p.wait() == 0, p.stdout.read().decode()[-2000:]
    lib = tmp_path / "librestore_host_asan.so"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-o", str(lib), *objs,
                    *[os.path.join(build, k + ".o") for k in kernels]], check=True, capture_output=True)
    r = _run(runtime, DRIVER, "host", str(lib))
    assert _clean(r), r.stderr[-3000:]
    assert "invalid ones refused" in r.stdout


def test_a_planted_overflow_is_reported(tmp_path):
    src = tmp_path / "overflow.c"
    src.write_text("#include <stdlib.h>\nint read_past(int n) { int *a = malloc(n * sizeof(int));\n"
                   "  for (int i = 0; i < n; ++i) a[i] = i;\n  int v = a[n];\n  free(a);\n  return v; }\n")
    lib = tmp_path / "liboverflow.so"
    subprocess.run(["gcc", "-O0", "-g", "-fPIC", "-shared", "-fsanitize=address", "-o", str(lib), str(src)],
                   check=True)
    code = (f"import ctypes\nlib = ctypes.CDLL({str(lib)!r})\nlib.read_past(8)\nprint('driver done')\n")
    r = _run(_gcc_asan_runtime(), "-c", code)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr
