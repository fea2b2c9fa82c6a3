"""CPU runs under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed):

* the FP64 oracle built with -fsanitize=address,undefined, running every oracle pin;
* the renderer library with its host code sanitized (device code as always), running the
  host-side checks of the C ABI and the admission model (argument validation, defaults, the
  byte account), which exercise the library without a device.

Each run is a subprocess that preloads the matching sanitizer runtime (the Python binary is
not instrumented); a sanitizer report fails it."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _env(preload, extra):
    env = dict(os.environ, LD_PRELOAD=preload, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.update(extra)
    return env


def _pytest(files, env):
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *[os.path.join(ROOT, "tests", f) for f in files]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    from oracle import build as oracle_build
    lib = oracle_build.build(out=str(tmp_path / "liblgsr_ref_san.so"), sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    out = _pytest(["test_oracle_pins.py", "test_oracle_tie_pins.py", "test_oracle_objective_pins.py",
                   "test_oracle_scan_pins.py"], _env(f"{asan}:{ubsan}", {"LGSR_REF_LIB": lib}))
    print(out.strip().splitlines()[-1])


def test_library_host_code_under_sanitizers(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("no clang AddressSanitizer runtime")
    from paper_2607_04127_amd import build as lib_build
    lib = lib_build.build(out=str(tmp_path / "liblgsr_san.so"), host_sanitize=True)
    out = _pytest(["test_abi.py", "test_service_admission.py"], _env(rt[-1], {"LGSR_LIB": lib}))
    print(out.strip().splitlines()[-1])
