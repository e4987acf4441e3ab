"""C-ABI surface checks that need no GPU: the library loads, exports every
function include/rsf.h declares, and its host-only logic answers."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsf.h")
LIB = os.path.join(ROOT, "paper_2404_02813_amd", "librsf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for n in ("rsf_create", "rsf_evolve", "rsf_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librsf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librsf.so not built")
def test_binding_names_match_header():
    from paper_2404_02813_amd import rsf
    assert set(rsf.EXPORTS) == set(declared_functions())
    for n in rsf.EXPORTS:
        assert callable(getattr(rsf, n))


@pytest.mark.skipif(not os.path.exists(LIB), reason="librsf.so not built")
def test_host_only_entry_points():
    from paper_2404_02813_amd import rsf
    L = rsf.lib()
    # six float fields dominate the workspace
    nb = rsf.rsf_workspace_bytes(64, 64, 64, 20)
    assert 6 * 64 ** 3 * 4 <= nb < 6 * 64 ** 3 * 4 + (1 << 20)
    nh = rsf.rsf_workspace_bytes(64, 64, 64, 20, "f16")
    assert 14 * 64 ** 3 <= nh < 14 * 64 ** 3 + (1 << 20)
    assert rsf.rsf_workspace_bytes(0, 4, 4, 1) == 0
    assert rsf.rsf_workspace_bytes(8, 8, 8, 1, 7) == 0
    assert L.rsf_last_error(None) == b"null context"
    # a NULL context is rejected before anything touches a device
    st = L.rsf_evolve(None, None, 0, None, 8, 8, 8, 3.0, 1, 1, 0.001, 1, 0.1, 1, 1, None)
    assert st == rsf.RSF_ERR_INVALID_ARG
    L.rsf_destroy(None)   # no-op


@pytest.mark.skipif(not os.path.exists(LIB), reason="librsf.so not built")
def test_fault_spec_parsing_and_arming():
    """rsf_set_fault accepts alloc_fail:N[:K] and the disarming forms, keeps
    its state on a malformed spec, and restarts the count when armed."""
    from paper_2404_02813_amd import rsf
    L = rsf.lib()
    try:
        assert L.rsf_set_fault(None) == rsf.RSF_OK
        assert rsf.rsf_fault_allocations() == -1
        for spec in (b"alloc_fail:1", b"alloc_fail:3:2", b"alloc_fail:9223372036854775807:1"):
            assert L.rsf_set_fault(spec) == rsf.RSF_OK, spec
            assert rsf.rsf_fault_allocations() == 0
        for bad in (b"alloc_fail:", b"alloc_fail:0", b"alloc_fail:-1", b"alloc_fail:2:0",
                    b"alloc_fail:2:", b"alloc_fail:2x", b"alloc_fail:1:2:3", b"fail:1",
                    b"alloc_fail:99999999999999999999"):
            assert L.rsf_set_fault(bad) == rsf.RSF_ERR_INVALID_ARG, bad
            assert rsf.rsf_fault_allocations() == 0      # still armed as before
        for off in (b"", b"off"):
            assert L.rsf_set_fault(b"alloc_fail:1") == rsf.RSF_OK
            assert L.rsf_set_fault(off) == rsf.RSF_OK
            assert rsf.rsf_fault_allocations() == -1
        with pytest.raises(rsf.RsfError):
            rsf.rsf_set_fault("alloc_fail:x")
    finally:
        L.rsf_set_fault(None)


@pytest.mark.skipif(not os.path.exists(LIB), reason="librsf.so not built")
@pytest.mark.parametrize("value,armed,refused", [("alloc_fail:4:2", True, False),
                                                  ("alloc_fail:zero", False, True),
                                                  ("", False, False)])
def test_fault_environment_variable(value, armed, refused):
    """RSF_FAULT arms the fault when the library loads; a malformed value arms
    nothing, says so on stderr and makes rsf_create refuse before it looks
    for a device."""
    import subprocess
    import sys
    prog = ("import ctypes,sys\n"
            f"L = ctypes.CDLL({LIB!r})\n"
            "L.rsf_fault_allocations.restype = ctypes.c_int64\n"
            "c = ctypes.c_void_p()\n"
            "print(L.rsf_fault_allocations(), L.rsf_create(ctypes.byref(c), 10**6))\n")
    env = dict(os.environ, RSF_FAULT=value)
    r = subprocess.run([sys.executable, "-c", prog], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    count, st = map(int, r.stdout.split())
    assert count == (0 if armed else -1)
    assert st == -1      # RSF_ERR_INVALID_ARG: malformed spec, or no device 10^6
    assert ("malformed RSF_FAULT" in r.stderr) == refused
