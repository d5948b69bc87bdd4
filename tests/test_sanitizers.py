"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle driven through random tables of every kind, call sequences,
push / pop, the fast mode and fixpoints; and the library's host runtime
(argument validation paths that return before any device work)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_driver"
    subprocess.run(["gcc", "-std=c11", *SAN, "-o", str(exe), os.path.join(ROOT, "tests", "native", "oracle_driver.c"),
                    os.path.join(ROOT, "oracle", "ct_oracle.c")], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "oracle driver: ok" in r.stdout


def test_runtime_host_paths_under_sanitizers(tmp_path):
    """The runtime's host sources built with the sanitizers (g++, host code
    only; the device code is the normal gfx950 build) and driven through the
    C ABI's validation paths."""
    from paper_2507_18413_amd import build as B
    libdir = B.torch_hip_runtime()
    if libdir is None or not shutil.which("g++"):
        pytest.skip("no HIP runtime library to link against")
    csrc = os.path.join(ROOT, "paper_2507_18413_amd", "csrc")
    objs = []
    for src in (s for s in B.SOURCES if s.endswith(".hip")):
        obj = tmp_path / (os.path.basename(src) + ".o")
        cmd = B.compile_cmd(src, str(obj))
        subprocess.run(cmd, check=True, capture_output=True)
        objs.append(str(obj))
    exe = tmp_path / "runtime_driver"
    subprocess.run(["g++", "-std=c++17", "-pthread", *SAN, "-D__HIP_PLATFORM_AMD__=1", "-I", "/opt/rocm/include",
                    "-I", os.path.join(ROOT, "include"), "-I", csrc, "-o", str(exe),
                    os.path.join(ROOT, "tests", "native", "runtime_driver.cpp"),
                    os.path.join(csrc, "ct_runtime.cpp"), os.path.join(csrc, "ct_server.cpp"),
                    os.path.join(csrc, "ct_split.cpp"), *objs, "-L", libdir, "-l:libamdhip64.so",
                    f"-Wl,-rpath,{libdir}"], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0", HIP_VISIBLE_DEVICES=""))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime driver: ok" in r.stdout
