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


def test_host_only_new_entry_points():
    """NULL contexts are refused as argument 1 before any device work; the
    new option and report fields sit where the header puts them; the
    capturing status has a string."""
    import ctypes

    from paper_0808_2794_amd import mixlu

    lib = mixlu.load()
    assert b"CAPTURING" in lib.mixlu_status_string(6)
    t = mixlu.mixlu_batched_tiles(16, 128, 2, 0)
    assert lib.mixlu_batched_set_tiles(None, mixlu.FP32, ctypes.byref(t)) == -1
    assert lib.mixlu_batched_get_tiles(None, mixlu.FP32, ctypes.byref(t)) == -1
    k = ctypes.c_double()
    assert lib.mixlu_condest(None, None, ctypes.byref(k)) == -1
    assert lib.mixlu_report_read(None, None, 0, None) == -1
    info = ctypes.c_int()
    assert lib.mixlu_sgesv(None, 1, 1, None, 1, None, 1, None, 1, None, 0, ctypes.byref(info)) == -1
    # layout: the condest option follows refine; the estimate follows converged
    assert mixlu.mixlu_opts.condest.offset == mixlu.mixlu_opts.refine.offset + 4
    assert mixlu.mixlu_report.cond_est.offset == mixlu.mixlu_report.converged.offset + 4
    assert mixlu.mixlu_report.outer.offset == mixlu.mixlu_report.cond_est.offset + 4
    assert lib.mixlu_sparse_fgmres(None, 1, 0, 0, None, None, None, None, None, 1, 1, None, 0,
                                   None, None) == -1
    assert ctypes.sizeof(mixlu.mixlu_report) == 64
    o = mixlu.default_opts()
    assert o.condest == 0 and o.refine == mixlu.REFINE_CLASSIC


def test_host_only_async_and_history():
    """The stream-ordered factorizations and the residual history refuse a
    NULL context before any device work; the restart option sits after
    condest, 0 by default (30 steps); the pending-outcome code is the
    header's."""
    import ctypes

    from paper_0808_2794_amd import mixlu

    lib = mixlu.load()
    F = mixlu.mixlu_factor()
    for name in ("mixlu_getrf_async", "mixlu_potrf_async"):
        assert getattr(lib, name)(None, mixlu.FP32, 4, None, 4, None, 0, None, ctypes.byref(F),
                                  None) == -1
    cnt = ctypes.c_int()
    assert lib.mixlu_refine_history(None, None, 0, ctypes.byref(cnt)) == -1
    assert mixlu.mixlu_opts.restart.offset == mixlu.mixlu_opts.condest.offset + 4
    assert mixlu.default_opts().restart == 0
    hdr = open(HEADER).read()
    assert "#define MIXLU_FACTOR_PENDING 1" in hdr and mixlu.FACTOR_PENDING == 1


def test_sweep_datta_bound():
    """The bound the experiment prints: ceil(ln eps_d / (ln eps_s + ln kappa)),
    finite only while kappa eps_s < 1 (worked by hand for FP32: kappa = 10
    gives ceil(36.74 / 14.33) = 3, kappa = 1e7 gives ceil(36.74 / 0.52) = 71)."""
    from paper_0808_2794_amd import sweep

    assert sweep.datta("fp32", 1e1) == 3
    assert sweep.datta("fp32", 1e7) == 71
    assert sweep.datta("fp32", 1e8) is None
    assert sweep.datta("fp16", 1e1) == 7
    assert sweep.datta("bf16", 1e2) == 40
    assert sweep.datta("fp16", 2.0 ** 11) is None
