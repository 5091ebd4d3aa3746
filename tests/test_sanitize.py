"""AddressSanitizer / UndefinedBehaviorSanitizer builds (CPU, no GPU needed).

* The oracle's C part (test infrastructure) with gcc -fsanitize=address,undefined, driven
  by tests/sanitize/oracle_driver.c over 1-D, 2-D and 3-D grids with ragged sizes, a zero
  column, warm starts, both PCG forms and the error returns.
* The HIP library's host code with clang's sanitizers (the device code is built as usual,
  the sanitizers apply to the host pass only), driven by tests/sanitize/abi_driver.c:
  argument validation of the C ABI, the no-device error path of qo_create, null handles,
  the allocation-free Gram's argument errors, status strings.
Any sanitizer report fails the test (no recovery)."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def _cpu_env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


def test_oracle_c_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "orc_san")
    _run([gcc, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-fopenmp", os.path.join(ROOT, "oracle", "qo_oracle.c"),
          os.path.join(SAN, "oracle_driver.c"), "-lm", "-o", exe])
    r = _run([exe], env=_cpu_env())
    assert "all checks passed" in r.stdout


@pytest.mark.slow
def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2605_25149_amd import build as hb

    try:
        hipcc = hb.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    clang = "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang not found")
    inc = os.path.join(ROOT, "include")
    san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host",
           "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

    def one(src):
        obj = str(tmp_path / src.replace(".hip", ".o"))
        _run([hipcc, "-O1", "-g", "-std=c++17", f"--offload-arch={hb.ARCH}", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san, "-I", inc,
              "-c", os.path.join(hb.CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 2)) as ex:
        objs = list(ex.map(one, hb.SOURCES))
    drv = str(tmp_path / "abi_driver.o")
    _run([clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-I", inc, "-c", os.path.join(SAN, "abi_driver.c"),
          "-o", drv])
    exe = str(tmp_path / "abi_san")
    _run([clang + "++", "-fsanitize=address,undefined", drv, *objs, "-L/opt/rocm/lib",
          "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    env = _cpu_env()
    env["HIP_VISIBLE_DEVICES"] = ""  # host code only: no device is used even where one is present
    env["ROCR_VISIBLE_DEVICES"] = ""
    r = _run([exe], env=env)
    assert "all checks passed" in r.stdout
