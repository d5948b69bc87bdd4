"""The C-ABI library loads and exports every function include/ct.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import subprocess

import pytest

from paper_2507_18413_amd import ct

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def libpath():
    if not os.path.exists(ct.LIB_PATH):
        from paper_2507_18413_amd import build
        build.build()
    return ct.LIB_PATH


def test_header_declares_the_boundary():
    names = ct.exported_names()
    for need in ["ct_create", "ct_destroy", "ct_layout", "ct_get_supports", "ct_propagate",
                 "ct_propagate_slot", "ct_push", "ct_pop", "ct_push_slot", "ct_pop_slot",
                 "ct_get_state", "ct_slots_alloc", "ct_slot_stats", "ct_propagate_batch",
                 "ct_last_error"]:
        assert need in names


def test_library_exports_every_declared_symbol(libpath):
    L = ctypes.CDLL(libpath)
    for name in ct.exported_names():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    for name in ct.exported_names():
        assert name in exported, name


def test_binding_signatures_cover_header(libpath):
    L = ct.lib()
    for name in ct.exported_names():
        assert getattr(L, name).argtypes is not None or name == "ct_last_error", name


def test_host_side_errors_without_device(libpath):
    # argument validation happens before any HIP call
    L = ct.lib()
    h = ctypes.c_void_p()
    lo = (ctypes.c_int32 * 1)(0)
    ds = (ctypes.c_int32 * 1)(0)
    assert L.ct_create(None, 0, 1, lo, ds, None, None, ctypes.byref(h)) == ct.E_INVALID
    assert L.ct_create(None, 0, 0, lo, ds, None, None, ctypes.byref(h)) == ct.E_INVALID
    assert L.ct_create(None, -1, 1, lo, ds, None, None, ctypes.byref(h)) == ct.E_INVALID
    assert "arity" in ct.last_error() or "n_tuples" in ct.last_error()
    assert L.ct_propagate_batch(None, -1, None, None) == ct.E_INVALID


def test_cpython_binding_marshals_to_the_library(libpath):
    """The CPython binding of the per-call entry points is built beside the
    library, calls the library's own functions (a null handle gets the
    library's CT_E_INVALID, no device call) and hands back what is not a
    uint64 array to the ctypes marshalling (None)."""
    import numpy as np
    L = ct.lib()
    F = ct._F
    assert F is not None, "the CPython binding is not built"
    din, dout = np.zeros(5, np.uint64), np.zeros(5, np.uint64)
    assert F.propagate(0, 0, din, dout, 5) == ct.E_INVALID
    assert "null" in ct.last_error()
    assert F.push(0, 0) == ct.E_INVALID and F.pop(0, 0) == ct.E_INVALID
    assert F.propagate(0, 0, np.zeros(5, np.float64), dout, 5) is None
    assert F.propagate(0, 0, np.zeros(4, np.uint64), dout, 5) is None
    assert F.propagate(0, 0, din, np.zeros(5, np.uint64)[::-1], 5) is None  # not contiguous
    assert F.propagate(0, 0, [0] * 5, dout, 5) is None
    assert F.propagate(0, 0, din, np.zeros(5, np.uint64).view(np.int64), 5) is None
    assert L is ct.lib()


def test_no_oracle_in_product_path():
    """The package neither imports nor links the oracle."""
    import re
    pkg = os.path.join(ROOT, "paper_2507_18413_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            path = os.path.join(dirpath, f)
            if f.endswith(".py"):
                text = open(path).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, re.M), path
                assert "libct_oracle" not in text and "cto_" not in text, path
            elif f.endswith((".cpp", ".hip", ".h")):
                text = open(path).read()
                assert "cto_" not in text and "ct_oracle" not in text, path


def test_kernel_signatures_have_no_address_space_qualifier():
    """A __global__ parameter typed with the device-only address space would
    mangle the kernel's name differently in the host and device passes, and
    its launch would name a kernel that does not exist on the device."""
    import re
    src = open(os.path.join(ROOT, "paper_2507_18413_amd", "csrc", "ct_kernels.hip")).read()
    for m in re.finditer(r"__global__[^{]*\(([^)]*)\)\s*\{", src):
        assert "CT_G" not in m.group(1), m.group(0)[:120]


def test_host_and_device_kernel_names_match(tmp_path):
    """Every kernel the host stubs launch is defined in the gfx950 code."""
    import re
    src = os.path.join(ROOT, "paper_2507_18413_amd", "csrc", "ct_kernels.hip")
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-std=c++17", "-c", "--save-temps",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.dirname(src), src, "-o", str(tmp_path / "k.o")]
    subprocess.run(cmd, check=True, capture_output=True, cwd=tmp_path)
    dev = open(next(tmp_path.glob("*amdgcn*gfx950.s"))).read()
    host = open(next(tmp_path.glob("*host-x86_64*.s"))).read()
    dev_k = set(re.findall(r"^(_ZN3ctk\w*kernel\w*):", dev, re.M))
    host_k = {k for k in re.findall(r"(_ZN3ctk\w*kernel\w*)", host) if "__device_stub__" not in k}
    assert dev_k and host_k
    assert host_k <= dev_k, host_k - dev_k


def test_kernels_keep_their_registers(tmp_path):
    """No kernel of the library spills to scratch memory at -O3 for gfx950
    (a spill turns every register access of the hot loops into a memory
    round trip)."""
    import re
    csrc = os.path.join(ROOT, "paper_2507_18413_amd", "csrc")
    for name in ("ct_kernels.hip", "ct_engine.hip", "ct_split.hip"):
        cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-c",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I", os.path.join(ROOT, "include"), "-I", csrc, os.path.join(csrc, name),
               "-o", str(tmp_path / (name + ".o")), "-Rpass-analysis=kernel-resource-usage"]
        out = subprocess.run(cmd, check=True, capture_output=True, text=True).stderr
        kernels = re.findall(r"Function Name: (\S+)", out)
        scratch = [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", out)]
        assert kernels and len(kernels) == len(scratch), name
        spilling = [k for k, sz in zip(kernels, scratch) if sz]
        assert not spilling, (name, spilling)
