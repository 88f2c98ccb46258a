"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

* The oracle core (oracle/oracle.cpp) is rebuilt with g++ -fsanitize=address,
  undefined and the oracle pins run against that build (ORACLE_LIB), in a
  child process with the sanitizer runtimes preloaded.
* The library's host code (planning, argument checks, loss sizes, autotune
  keys and cache file) is rebuilt with the sanitizers on the host pass only
  and driven by tests/sanitize/abi_host_driver.cpp, which needs no GPU.
Any sanitizer report aborts the child and fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CSRC = os.path.join(ROOT, "paper_2506_06988_amd", "csrc")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["g++", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fopenmp", "-shared", "-fPIC", "-std=c++17", "-o", lib,
                           os.path.join(ROOT, "oracle", "oracle.cpp")])
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}", **SAN_ENV)
    # Python itself is not built for leak checking: leaks are left to the driver below
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    check = ("import oracle; L = oracle.lib(); "
             f"assert L._name == {lib!r}, L._name; print('oracle build:', L._name)")
    r = subprocess.run([sys.executable, "-c", check], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_host_library_code_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not installed")
    from paper_2506_06988_amd import build as hb
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    # the device pass keeps the library's own flags; debug info and frame
    # pointers go to the host pass only
    flags = hb.FLAGS + ["-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer"] + san
    objs, procs = [], []
    srcs = [os.path.join(CSRC, s) for s in hb.SOURCES]
    srcs.append(os.path.join(ROOT, "tests", "sanitize", "abi_host_driver.cpp"))
    for src in srcs:
        obj = str(tmp_path / (os.path.splitext(os.path.basename(src))[0] + ".o"))
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        procs.append(subprocess.Popen([HIPCC, *flags, *lang, "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    for p, src in zip(procs, srcs):
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, f"{src}:\n{err[-3000:]}"
    exe = str(tmp_path / "abi_host_driver")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", *san, "-o", exe, *objs])
    work = tmp_path / "cache"
    work.mkdir()
    r = subprocess.run([exe, str(work)], env=dict(os.environ, **SAN_ENV), capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "checks passed" in r.stdout
    shutil.rmtree(work, ignore_errors=True)
