"""Sanitizer runs on the CPU: the oracle's C code and the library's host code
under AddressSanitizer (with leak detection for the host code) and
UndefinedBehaviorSanitizer, any report fatal.

* The oracle (``oracle/pms_oracle.c``) built with gcc ``-fsanitize=address,
  undefined``, loaded into a fresh interpreter with the sanitizer runtime
  preloaded, runs every pin of ``tests/_pins.py`` and the real-sequence pins.
* The library's host code (validation, work planning, launch layout, code
  sorting, the autotune cache and the C ABI's error paths) built from its
  own source without device code (``hipcc --cuda-host-only``, sanitizers on
  the host pass) runs ``tests/host/host_checks.cpp``.

The same commands by hand::

    gcc -O1 -g -std=c11 -fPIC -shared -pthread -fsanitize=address,undefined \\
        -fno-sanitize-recover=all oracle/pms_oracle.c -o /tmp/liboracle_san.so
    hipcc -x hip --cuda-host-only -O1 -g -std=c++17 -Iinclude \\
        -Ipaper_1403_1313_amd/csrc -Xarch_host -fsanitize=address \\
        -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all \\
        tests/host/host_checks.cpp -o /tmp/host_checks -L/opt/rocm/lib \\
        -Wl,-rpath,/opt/rocm/lib -lrocprofiler-sdk-roctx && /tmp/host_checks /tmp
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _gcc_runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_asan_ubsan(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-pthread",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "pms_oracle.c"),
                    "-o", str(lib)], check=True)
    code = (
        "import sys\n"
        f"sys.path[:0] = [{ROOT!r}, {os.path.join(ROOT, 'tests')!r}]\n"
        "import oracle, _pins\n"
        f"orc = oracle.OracleLib({str(lib)!r})\n"
        "for pin in _pins.ALL_PINS + [_pins.pin_ex_definition_tiny, _pins.pin_ex_identities,\n"
        "                             _pins.pin_ex_closed_forms]:\n"
        "    pin(orc)\n"
        "print('oracle pins passed')\n")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "oracle pins passed" in res.stdout


def test_host_code_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    exe = tmp_path / "host_checks"
    cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17",
           "-fno-omit-frame-pointer", f"-I{os.path.join(ROOT, 'include')}",
           f"-I{os.path.join(ROOT, 'paper_1403_1313_amd', 'csrc')}",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "host", "host_checks.cpp"), "-o", str(exe),
           f"-L{ROCM}/lib", f"-Wl,-rpath,{ROCM}/lib", "-lrocprofiler-sdk-roctx"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stdout[-2000:] + build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    res = subprocess.run([str(exe), str(tmp_path)], env=env, capture_output=True, text=True,
                         timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "host checks passed" in res.stdout
