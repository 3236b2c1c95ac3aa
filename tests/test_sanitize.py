"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code,
run on the CPU (no GPU needed):

  * the oracle (oracle/fmm_oracle.c) driven once through every entry at
    small sizes (tests/sanitize/oracle_main.c);
  * the host part of the C ABI (csrc/api.cpp: validation, error reporting,
    handle bookkeeping) and the autotuner (csrc/tuner.cpp), with the
    device-side functions replaced by stand-ins that report a device error
    (tests/sanitize/host_stubs.cpp, driven by tests/sanitize/host_main.c).

Any out-of-bounds access, use after free, leak or undefined operation
aborts the program; the test checks its exit status.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1"]


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr)
    return r


@pytest.fixture(scope="module")
def tmp(tmp_path_factory):
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("gcc/g++ not available")
    return str(tmp_path_factory.mktemp("sanitize"))


def test_oracle_under_asan_ubsan(tmp):
    exe = os.path.join(tmp, "oracle_san")
    _run(["gcc", "-std=c99", "-ffp-contract=off", *SAN, "-o", exe,
          os.path.join(ROOT, "tests", "sanitize", "oracle_main.c"), os.path.join(ROOT, "oracle", "fmm_oracle.c"),
          "-lm"], tmp)
    r = _run([exe], tmp)
    assert "ok" in r.stdout


def test_host_library_under_asan_ubsan(tmp):
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if not os.path.exists(os.path.join(rocm, "lib", "libamdhip64.so")):
        pytest.skip("HIP runtime library not found")
    csrc = os.path.join(ROOT, "paper_1311_1006_amd", "csrc")
    objs = []
    for src in (os.path.join(csrc, "api.cpp"), os.path.join(csrc, "tuner.cpp"),
                os.path.join(ROOT, "tests", "sanitize", "host_stubs.cpp")):
        obj = os.path.join(tmp, os.path.basename(src) + ".o")
        _run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(rocm, "include"), *SAN,
              "-c", src, "-o", obj], tmp)
        objs.append(obj)
    main = os.path.join(tmp, "host_main.o")
    _run(["gcc", "-std=c99", *SAN, "-c", os.path.join(ROOT, "tests", "sanitize", "host_main.c"), "-o", main], tmp)
    exe = os.path.join(tmp, "host_san")
    _run(["g++", *SAN, "-o", exe, main, *objs, "-L" + os.path.join(rocm, "lib"), "-lamdhip64",
          "-Wl,-rpath," + os.path.join(rocm, "lib"), "-lm"], tmp)
    env = dict(os.environ, HIP_VISIBLE_DEVICES="")   # host paths only, also on a machine with a GPU
    r = subprocess.run([exe], cwd=tmp, capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
