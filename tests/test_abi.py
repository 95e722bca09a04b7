"""The C-ABI library loads and exports what include/wf.h and include/wf_nn.h
declare (CPU only: no compute call is made)."""

import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wf.h")
NN_HEADER = os.path.join(ROOT, "include", "wf_nn.h")
LIB = os.path.join(ROOT, "paper_1704_00865_amd", "libwf.so")


def _declared(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("wf_ctx_create", "wf_ctx_destroy", "wf_solve", "wf_strerror"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() + _declared(NN_HEADER) if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwf.so not built")
def test_binding_declares_every_export():
    import paper_1704_00865_amd as wf
    import paper_1704_00865_amd.nn as nn
    assert sorted(wf.EXPORTS) == _declared()
    assert sorted(nn.EXPORTS) == _declared(NN_HEADER)
    wf.load()
    nn._lib()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwf.so not built")
def test_host_only_calls():
    import paper_1704_00865_amd as wf
    lib = wf.load()
    assert lib.wf_supported(2048, 2048, 0) == 1
    assert lib.wf_supported(4096, 4096, 0) == 1
    assert lib.wf_supported(4096, 4096, 1) == 0
    assert lib.wf_supported(100, 128, 0) == 0
    assert lib.wf_supported(32, 64, 0) == 0
    s = wf._Schedule()
    lib.wf_schedule_default(ctypes.byref(s))
    assert s.kind == 1 and s.lambda0 == 1.0e4 and s.shrink_exp == 0.7
    assert list(s.beta) == [0.9, 0.9, 1.0] and s.chain == 0
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert wf.strerror(code)
    import paper_1704_00865_amd.nn as nn
    offs = nn.layer_offsets()
    assert len(offs) == 15
    assert nn.param_count() == offs[-1][3] + offs[-1][1]
    assert offs[0][:2] == (32, 32) and offs[-1][:2] == (32, 32)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_ctypes_layout_matches_c_structs(tmp_path):
    import paper_1704_00865_amd as wf
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "wf_nn.h"\n'
                   "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(wf_schedule),"
                   " sizeof(wf_report), sizeof(wf_inputs), sizeof(wf_shape),"
                   " offsetof(wf_schedule, chain), offsetof(wf_report, kernel_ms),"
                   " sizeof(wf_nn_shape));return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", str(src), "-o", str(exe)])
    import paper_1704_00865_amd.nn as nn
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert got == [ctypes.sizeof(wf._Schedule), ctypes.sizeof(wf._Report),
                   ctypes.sizeof(wf._Inputs), ctypes.sizeof(wf._Shape),
                   wf._Schedule.chain.offset, wf._Report.kernel_ms.offset,
                   ctypes.sizeof(nn._NNShape)]


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwf.so not built")
def test_host_side_argument_checks():
    """Entry points reject bad arguments before any device call."""
    import paper_1704_00865_amd as wf
    import paper_1704_00865_amd.nn as nn
    lib = nn._lib()
    h = ctypes.c_void_p()
    for shape, code in (((100, 128, 1, 0), -6), ((32, 64, 1, 0), -6), ((64, 64, 0, 0), -1),
                        ((64, 64, 1, 7), -1), ((4096, 64, 1, 0), -6)):
        st = lib.wf_nn_create(ctypes.byref(nn._NNShape(*shape)), ctypes.byref(h))
        assert st == code, (shape, st)
        assert not h.value
    assert lib.wf_nn_create(None, ctypes.byref(h)) == -1
    # unsupported solver shapes and precisions
    s = wf._Shape(100, 128, 0)
    assert lib.wf_ctx_create(ctypes.byref(s), ctypes.byref(h)) == -6
    s = wf._Shape(64, 64, 5)
    assert lib.wf_ctx_create(ctypes.byref(s), ctypes.byref(h)) == -1
    # null handles
    assert lib.wf_solve(None, None, None, None, None, None, None, None) == -1
    assert lib.wf_solve_batch(None, 0, None, None, None, None, None, None) == -1
    assert lib.wf_nn_predict(None, 1, None, None, None, None, None) == -1
    assert lib.wf_nn_conv3x3(9, 1, 8, 8, 32, 32, None, None, None, None, None, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwf.so not built")
def test_noalloc_rejects_what_its_scratch_cannot_hold():
    """wf_solve_noalloc checks shape, schedule and workspace size on the host
    before any device call (the pointers below are never dereferenced)."""
    import paper_1704_00865_amd as wf
    lib = wf.load()
    assert lib.wf_noalloc_scratch_bytes() == 32 << 20
    fake = ctypes.c_void_p(0x1000)
    inp = wf._Inputs(fake, fake, fake, None, None, None)
    out = ctypes.c_void_p(0x2000)

    def call(ny, nx, prec, **kw):
        s = wf.Schedule(lambdas=[1.0], rtol=0.0, max_sweeps=kw.get("max_sweeps", 100),
                        monitor_every=kw.get("monitor_every", 16))
        c, keep = s._c()
        shape = wf._Shape(ny, nx, prec)
        return lib.wf_solve_noalloc(ctypes.byref(shape), ctypes.byref(inp), ctypes.byref(c),
                                    None, out, None, None, None)
    # only calls that are rejected before any device work: the pointers are
    # fake
    assert call(2048, 2048, 0) == -7          # 4 M pixels do not fit in 32 MiB
    assert call(1024, 1024, 0) == -7
    assert call(1024, 1024, 1) == -7
    assert call(768, 768, 1) == -7
    assert call(256, 256, 0, max_sweeps=70000) == -7
    assert call(100, 256, 0) == -6
    assert lib.wf_solve_noalloc(None, ctypes.byref(inp), None, None, out, None, None, None) == -1
