"""The C ABI library loads on the CPU and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mixlu.h")
LIB = os.path.join(ROOT, "paper_0808_2794_amd", "libmixlu.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mixlu_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for name in ("mixlu_create", "mixlu_dxgesv", "mixlu_getrf", "mixlu_getrs", "mixlu_refine",
                 "mixlu_dgesv", "mixlu_workspace_size", "mixlu_outer_update"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmixlu.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    from paper_0808_2794_amd import mixlu

    assert set(mixlu.EXPORTS) == set(declared_symbols())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmixlu.so not built")
def test_host_only_entry_points():
    """Calls that touch no GPU: status strings and default options."""
    from paper_0808_2794_amd import mixlu

    lib = mixlu.load()
    assert lib.mixlu_status_string(0) == b"MIXLU_OK"
    assert b"timeout" in lib.mixlu_status_string(5).lower() or b"wait" in lib.mixlu_status_string(5)
    o = mixlu.default_opts()
    assert o.itermax == 30 and o.fallback == 1 and o.equilibrate == -1 and abs(o.stall - 0.9) < 1e-15
    o = mixlu.default_opts(itermax=5)
    assert o.itermax == 5
    with pytest.raises(TypeError):
        mixlu.default_opts(bogus=1)
    # a NULL context is rejected as argument 1 without touching the device
    assert lib.mixlu_destroy(None) == -1
