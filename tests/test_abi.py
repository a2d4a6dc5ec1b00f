"""The C-ABI library loads on the CPU host and exports every declared symbol.

No compute call is made here (no GPU in this environment)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "vofmt.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return set(re.findall(r"\b(vofmt_[a-z_]+)\s*\(", hdr))


def test_header_declarations_bound_in_python():
    from paper_2407_07463_amd import vofmt

    assert declared_symbols() == set(vofmt._SIGNATURES)


def test_library_exports_every_declared_symbol():
    from paper_2407_07463_amd import vofmt

    if not os.path.exists(vofmt.LIB_PATH):
        pytest.skip("libvofmt.so not built")
    assert vofmt.exported_symbols() == declared_symbols()
    L = vofmt.load()
    assert L.vofmt_version().decode().startswith("vofmt")


def test_create_fails_cleanly_without_device():
    """vofmt_create validates the device index on the host and returns E_ARG."""
    import ctypes

    from paper_2407_07463_amd import vofmt

    if not os.path.exists(vofmt.LIB_PATH):
        pytest.skip("libvofmt.so not built")
    L = vofmt.load()
    h = ctypes.c_void_p()
    assert L.vofmt_create(ctypes.byref(h), 10_000) == vofmt.E_ARG
    assert not h.value
    assert L.vofmt_last_error(None).decode() == "null context"
