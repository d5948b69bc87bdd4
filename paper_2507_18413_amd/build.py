"""Build the HIP library libct.so for gfx950 in-tree (hipcc, no JIT cache).

Device code is compiled by hipcc for gfx950.  The shared library is linked
against the HIP runtime that PyTorch loads (torch/lib/libamdhip64.so) when
PyTorch is installed: streams and device pointers handed over by torch are
then objects of the same runtime instance, and a process holds one HIP
runtime only.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libct.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = [os.path.join(CSRC, "ct_kernels.hip"), os.path.join(CSRC, "ct_engine.hip"),
           os.path.join(CSRC, "ct_split.hip"), os.path.join(CSRC, "ct_noalloc.hip"),
           os.path.join(CSRC, "ct_runtime.cpp"),
           os.path.join(CSRC, "ct_server.cpp"), os.path.join(CSRC, "ct_split.cpp")]
ARCH = os.environ.get("CT_OFFLOAD_ARCH", "gfx950")
HIPCC = "/opt/rocm/bin/hipcc"


def torch_hip_runtime():
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec is None or not spec.origin:
            return None
        libdir = os.path.join(os.path.dirname(spec.origin), "lib")
        if glob.glob(os.path.join(libdir, "libamdhip64.so*")):
            return libdir
    except Exception:
        pass
    return None


def compile_cmd(src, obj):
    if src.endswith(".cpp"):
        # host-only runtime: HIP runtime API, no device code
        return ["g++", "-O2", "-std=c++17", "-fPIC", "-pthread", "-c", "-Wall", "-D__HIP_PLATFORM_AMD__=1",
                "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", CSRC, src, "-o", obj]
    return [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c",
            "-Wall", "-Wno-unused-function",
            # packed fp32 instructions stay off in every device pass
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, src, "-o", obj]


def link_cmd(objs, out):
    libdir = torch_hip_runtime()
    if libdir:
        return ["g++", "-shared", "-pthread", "-o", out, *objs, "-L", libdir, "-l:libamdhip64.so",
                f"-Wl,-rpath,{libdir}", "-Wl,--no-undefined"]
    return [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", out, *objs]


PYFAST_SRC = os.path.join(CSRC, "ct_pyfast.c")


def pyfast_path() -> str:
    import sysconfig
    return os.path.join(HERE, "_ctfast" + sysconfig.get_config_var("EXT_SUFFIX"))


def build_pyfast(verbose: bool = False) -> str:
    """The CPython binding of the per-call entry points (host C, gcc)."""
    import sysconfig
    out = pyfast_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-shared", "-fPIC", "-Wall", "-I", sysconfig.get_paths()["include"], PYFAST_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        cmd = compile_cmd(src, obj)
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = link_cmd(objs, tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    build_pyfast(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
