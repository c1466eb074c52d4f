"""Sanitizer builds of the host code, on the CPU:

* the serving layer (csrc/frt_server.cpp) on a CPU stand-in of the library
  (tests/cpu_server): its scenarios (arrival order and slots, the memory
  budget, failures injected into one request's creation, upload or step,
  a device failure of a batch, queue modes and bins, concurrent clients,
  destroying a server with requests in flight, batched vs one-at-a-time
  latency on the stand-in's virtual clock, the temperature of a finished
  request) built plain, under
  ThreadSanitizer (clang's runtime, which understands the condition
  variables' clock waits) and under AddressSanitizer + UBSan;
* the FP64 oracle under AddressSanitizer + UBSan, running its own pins;
* the library's host engine and serving layer under AddressSanitizer +
  UBSan (host code only; the kernels are those of the last build), running
  the host-side ABI checks.
A sanitizer report fails the test (UBSan is built not to recover)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SERVER_SRC = [os.path.join(ROOT, "tests", "cpu_server", "fake_backend.cpp"),
              os.path.join(ROOT, "tests", "cpu_server", "scenarios.cpp"),
              os.path.join(ROOT, "paper_2409_04521_amd", "csrc", "frt_server.cpp")]
INC = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2409_04521_amd", "csrc"),
       "-I", os.path.join(ROOT, "tests", "cpu_server")]
CLANG = "/opt/rocm/llvm/bin/clang++"
REPORTS = ("WARNING: ThreadSanitizer", "ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _run(cmd, env=None, timeout=600):
    e = dict(os.environ)
    e.update(env or {})
    p = subprocess.run(cmd, env=e, capture_output=True, text=True, timeout=timeout)
    out = p.stdout + p.stderr
    return p.returncode, out


def _compiler(name):
    path = shutil.which(name) if not os.path.isabs(name) else (name if os.path.exists(name) else None)
    if not path:
        pytest.skip(f"{name} not available")
    return path


@pytest.mark.parametrize("variant", ["plain", "tsan", "asan_ubsan"])
def test_server_scenarios(tmp_path, variant):
    exe = str(tmp_path / f"scenarios_{variant}")
    if variant == "tsan":
        cxx, flags = _compiler(CLANG), ["-fsanitize=thread"]
    elif variant == "asan_ubsan":
        cxx, flags = _compiler("g++"), ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                                         "-fno-omit-frame-pointer"]
    else:
        cxx, flags = _compiler("g++"), ["-Wall", "-Wextra", "-Werror"]
    rc, out = _run([cxx, "-std=c++17", "-O1", "-g", "-pthread", *flags, *INC, *SERVER_SRC, "-o", exe], timeout=300)
    assert rc == 0, out
    env = {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1", "ASAN_OPTIONS": "detect_leaks=1"}
    rc, out = _run([exe], env=env, timeout=300)
    print(out)
    assert rc == 0, out
    assert "all scenarios passed" in out
    for rep in REPORTS:
        assert rep not in out, rep


def test_oracle_under_asan_ubsan(tmp_path):
    from oracle import oracle as O

    _compiler("gcc")
    lib = O.build(force=True, out=str(tmp_path / "liboracle_san.so"), sanitize=True)
    rt = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(rt):
        pytest.skip("gcc's AddressSanitizer runtime not found")
    # the oracle's pins, without the three longest runs (a minute under the sanitizers)
    sel = ("not stromgren_front_converges and not equilibrium_opacity_stromgren and not c1_time_averaged")
    rc, out = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                    "-k", sel, os.path.join(ROOT, "tests", "test_oracle_avgchem.py"),
                    os.path.join(ROOT, "tests", "test_oracle_genopacity.py"),
                    os.path.join(ROOT, "tests", "test_oracle_geometry.py"),
                    os.path.join(ROOT, "tests", "test_oracle_merge.py"),
                    os.path.join(ROOT, "tests", "test_oracle_step.py"),
                    os.path.join(ROOT, "tests", "test_oracle_transport.py"),
                    os.path.join(ROOT, "tests", "test_oracle_temperature.py"),
                    os.path.join(ROOT, "tests", "test_oracle_gentemp.py"),
                    os.path.join(ROOT, "tests", "test_oracle_density.py")],
                   env={"FRT_ORACLE_LIB": lib, "LD_PRELOAD": rt, "ASAN_OPTIONS": "detect_leaks=0"})
    print(out[-2000:])
    assert rc == 0, out[-4000:]
    for rep in REPORTS:
        assert rep not in out, rep


def test_host_engine_under_asan_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2409_04521_amd import build as B

    if not os.path.exists(os.path.join(ROOT, "paper_2409_04521_amd", "csrc", "frt_kernels.o")):
        pytest.skip("no kernel objects: build the library first")
    try:
        rt = B.sanitizer_runtime()
    except (FileNotFoundError, subprocess.CalledProcessError):
        pytest.skip("no AddressSanitizer runtime for hipcc's host compiler")
    lib = B.build_host_sanitized(str(tmp_path / "libfrt_san.so"))
    rc, out = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                    os.path.join(ROOT, "tests", "test_abi_host.py")],
                   env={"FRT_LIB": lib, "LD_PRELOAD": rt, "ASAN_OPTIONS": "detect_leaks=0"})
    print(out[-2000:])
    assert rc == 0, out[-4000:]
    for rep in REPORTS:
        assert rep not in out, rep
