"""Python binding of libmixlu: argument marshalling only.

Every function named ``mixlu_*`` calls the C entry point of the same name in
``libmixlu.so`` (declared in ``include/mixlu.h``) with raw device pointers
taken from torch tensors; all arithmetic happens in the HIP kernels behind
that C ABI.  ``Solver`` bundles a context with a workspace for repeated
calls.  Loading fails loudly when the library is missing: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmixlu.so")

FP64, FP32, BF16, FP16, FP8 = 0, 1, 2, 3, 4
PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp16": FP16, "fp8": FP8}
PREC_NAME = {v: k for k, v in PREC.items()}
OP_GESV, OP_POSV, OP_DGESV, OP_DPOSV, OP_SGESV = 0, 1, 2, 3, 4
REFINE_CLASSIC, REFINE_FGMRES = 0, 1
ROW_MAJOR, COL_MAJOR = 0, 1

OK = 0
ERR_HIP, ERR_WORKSPACE, ERR_NOT_IMPLEMENTED, ERR_UNSUPPORTED_ARCH, ERR_DEVICE_TIMEOUT = 1, 2, 3, 4, 5


class mixlu_opts(ctypes.Structure):
    _fields_ = [("itermax", ctypes.c_int), ("equilibrate", ctypes.c_int),
                ("fallback", ctypes.c_int), ("nb", ctypes.c_int), ("layout", ctypes.c_int),
                ("stall", ctypes.c_double), ("refine", ctypes.c_int),
                ("condest", ctypes.c_int), ("restart", ctypes.c_int),
                ("reserved", ctypes.c_int * 3)]


class mixlu_report(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int), ("info", ctypes.c_int), ("prec", ctypes.c_int),
                ("fallback_iter", ctypes.c_int), ("anorm", ctypes.c_double),
                ("rnorm", ctypes.c_double), ("xnorm", ctypes.c_double),
                ("berr", ctypes.c_double), ("converged", ctypes.c_int),
                ("cond_est", ctypes.c_float), ("outer", ctypes.c_int),
                ("reserved", ctypes.c_int * 1)]

    def as_dict(self) -> dict:
        return {"iter": self.iter, "info": self.info, "prec": PREC_NAME.get(self.prec, self.prec),
                "fallback_iter": self.fallback_iter, "anorm": self.anorm, "rnorm": self.rnorm,
                "xnorm": self.xnorm, "berr": self.berr, "converged": bool(self.converged),
                "cond_est": float(self.cond_est), "outer": self.outer}


class mixlu_factor(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("npad", ctypes.c_int), ("nb", ctypes.c_int),
                ("prec", ctypes.c_int), ("kind", ctypes.c_int), ("layout", ctypes.c_int),
                ("equilibrated", ctypes.c_int), ("lowp_status", ctypes.c_int),
                ("nrhs_max", ctypes.c_int), ("work", ctypes.c_void_p),
                ("lwork", ctypes.c_size_t), ("off", ctypes.c_size_t * 16)]


class mixlu_batched_tiles(ctypes.Structure):
    _fields_ = [("panel", ctypes.c_int), ("chunk", ctypes.c_int), ("groups", ctypes.c_int),
                ("tuned", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {"panel": self.panel, "chunk": self.chunk, "groups": self.groups,
                "tuned": bool(self.tuned)}


# candidate order of mixlu_batched_tune's timings
TILE_CANDIDATES = [(p, c, g) for p in (16, 8) for c in (128, 64, 32) for g in (2, 1)]


class mixlu_kstat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_longlong),
                ("ms", ctypes.c_double), ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


EXPORTS = ("mixlu_status_string", "mixlu_default_opts", "mixlu_create", "mixlu_destroy",
           "mixlu_set_stream", "mixlu_workspace_size", "mixlu_getrf", "mixlu_potrf",
           "mixlu_getrs", "mixlu_refine", "mixlu_dxgesv", "mixlu_dxposv", "mixlu_dgesv",
           "mixlu_dposv", "mixlu_outer_update", "mixlu_batched_workspace_size",
           "mixlu_dxgesv_batched", "mixlu_dxgesv_batched_noalloc", "mixlu_profile_enable",
           "mixlu_profile_read", "mixlu_sgesv", "mixlu_report_read", "mixlu_batched_tune", "mixlu_batched_get_tiles",
           "mixlu_batched_set_tiles", "mixlu_condest", "mixlu_sparse_workspace_size",
           "mixlu_sparse_fgmres", "mixlu_gemm_update", "mixlu_refine_history",
           "mixlu_getrf_async", "mixlu_potrf_async")

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmixlu.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libmixlu.so not built ({path}); run paper_0808_2794_amd.build")
    lib = ctypes.CDLL(path)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = {
        "mixlu_status_string": ([I], ctypes.c_char_p),
        "mixlu_default_opts": ([P], None),
        "mixlu_create": ([P, P], I),
        "mixlu_destroy": ([P], I),
        "mixlu_set_stream": ([P, P], I),
        "mixlu_workspace_size": ([P, I, I, I, I, P, P], I),
        "mixlu_getrf": ([P, I, I, P, I, P, S, P, P, P], I),
        "mixlu_potrf": ([P, I, I, P, I, P, S, P, P, P], I),
        "mixlu_getrf_async": ([P, I, I, P, I, P, S, P, P, P], I),
        "mixlu_potrf_async": ([P, I, I, P, I, P, S, P, P, P], I),
        "mixlu_getrs": ([P, P, I, I, P, I, P, I], I),
        "mixlu_refine": ([P, P, I, I, P, I, P, I, P, I, P, P], I),
        "mixlu_dxgesv": ([P, I, I, I, P, I, P, I, P, I, P, S, P, P], I),
        "mixlu_dxposv": ([P, I, I, I, P, I, P, I, P, I, P, S, P, P], I),
        "mixlu_dgesv": ([P, I, I, P, I, P, I, P, I, P, S, P], I),
        "mixlu_dposv": ([P, I, I, P, I, P, I, P, I, P, S, P], I),
        "mixlu_outer_update": ([P, I, I, P, I, P, I, P, I, D, D], I),
        "mixlu_batched_workspace_size": ([P, I, I, I, P, P], I),
        "mixlu_dxgesv_batched": ([P, I, I, P, P, P, P, P, I, P, S, P, P], I),
        "mixlu_dxgesv_batched_noalloc": ([P, I, I, P, P, P, P, P, I, P, P], I),
        "mixlu_refine_history": ([P, P, I, P], I),
        "mixlu_profile_enable": ([P, I], I),
        "mixlu_profile_read": ([P, P, I, P], I),
        "mixlu_sgesv": ([P, I, I, P, I, P, I, P, I, P, S, P], I),
        "mixlu_report_read": ([P, P, I, P], I),
        "mixlu_batched_tune": ([P, I, I, P, P, P, P, P, I, P, S, P, P, P, P, I], I),
        "mixlu_batched_get_tiles": ([P, I, P], I),
        "mixlu_batched_set_tiles": ([P, I, P], I),
        "mixlu_condest": ([P, P, P], I),
        "mixlu_sparse_workspace_size": ([P, I, I, I, I, I, P], I),
        "mixlu_sparse_fgmres": ([P, I, I, I, P, P, P, P, P, I, I, P, S, P, P], I),
        "mixlu_gemm_update": ([P, I, I, I, I, P, I, P, I, P, I, P, S, P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class MixluError(RuntimeError):
    pass


def check(rc: int, what: str = "") -> None:
    if rc != OK:
        msg = load().mixlu_status_string(rc).decode()
        raise MixluError(f"{what}: {msg} (code {rc})")


def default_opts(**kw) -> mixlu_opts:
    o = mixlu_opts()
    load().mixlu_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


# ----------------------------------------------------------- raw wrappers
def _p(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream_ptr(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def mixlu_create(stream=None):
    h = ctypes.c_void_p()
    check(load().mixlu_create(ctypes.byref(h), _stream_ptr(stream)), "mixlu_create")
    return h


def mixlu_destroy(ctx) -> None:
    check(load().mixlu_destroy(ctx), "mixlu_destroy")


def mixlu_set_stream(ctx, stream=None) -> None:
    check(load().mixlu_set_stream(ctx, _stream_ptr(stream)), "mixlu_set_stream")


def mixlu_workspace_size(ctx, op: int, prec: int, n: int, nrhs: int, opts=None) -> int:
    b = ctypes.c_size_t()
    check(load().mixlu_workspace_size(ctx, op, prec, n, nrhs,
                                      None if opts is None else ctypes.byref(opts),
                                      ctypes.byref(b)), "mixlu_workspace_size")
    return b.value


def _is_cm(t) -> bool:
    """True when a 2-D tensor with several rows and columns is stored
    column-major (unit row stride)."""
    return t.dim() == 2 and t.shape[0] > 1 and t.shape[1] > 1 and t.stride(0) == 1


def _ld(t, cm: bool = False):
    """Leading dimension of a 2-D tensor stored row-major (cm False) or
    column-major (cm True); raises if the storage is neither."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    r, c = t.shape
    if cm:
        if r > 1 and t.stride(0) != 1:
            raise ValueError("expected a column-major 2-D tensor")
        return max(1, r, t.stride(1) if c > 1 else r)
    if c > 1 and t.stride(1) != 1:
        raise ValueError("expected a row-major 2-D tensor")
    return max(1, c, t.stride(0) if r > 1 else c)


def _cm(opts) -> bool:
    return opts is not None and opts.layout == COL_MAJOR


def mixlu_dxgesv(ctx, prec: int, A, B, X, work, opts=None) -> mixlu_report:
    rep = mixlu_report()
    n, nrhs = B.shape
    cm = _cm(opts)
    check(load().mixlu_dxgesv(ctx, prec, n, nrhs, _p(A), _ld(A, cm), _p(B), _ld(B, cm), _p(X),
                              _ld(X, cm), _p(work), work.numel() * work.element_size(),
                              None if opts is None else ctypes.byref(opts), ctypes.byref(rep)),
          "mixlu_dxgesv")
    return rep


def mixlu_dxposv(ctx, prec: int, A, B, X, work, opts=None) -> mixlu_report:
    rep = mixlu_report()
    n, nrhs = B.shape
    cm = _cm(opts)
    check(load().mixlu_dxposv(ctx, prec, n, nrhs, _p(A), _ld(A, cm), _p(B), _ld(B, cm), _p(X),
                              _ld(X, cm), _p(work), work.numel() * work.element_size(),
                              None if opts is None else ctypes.byref(opts), ctypes.byref(rep)),
          "mixlu_dxposv")
    return rep


def _d_solve(name, ctx, A, B, X, work) -> int:
    info = ctypes.c_int()
    n, nrhs = B.shape
    check(getattr(load(), name)(ctx, n, nrhs, _p(A), _ld(A), _p(B), _ld(B), _p(X),
                                _ld(X), _p(work), work.numel() * work.element_size(),
                                ctypes.byref(info)), name)
    return info.value


def mixlu_dgesv(ctx, A, B, X, work) -> int:
    return _d_solve("mixlu_dgesv", ctx, A, B, X, work)


def mixlu_dposv(ctx, A, B, X, work) -> int:
    return _d_solve("mixlu_dposv", ctx, A, B, X, work)


def mixlu_sgesv(ctx, A, B, X, work) -> int:
    return _d_solve("mixlu_sgesv", ctx, A, B, X, work)


def mixlu_report_read(ctx, d_reps, count: int) -> list:
    """Copy count device reports (a device buffer, e.g. the batched d_reps)
    to the host and decode them."""
    out = (mixlu_report * max(count, 1))()
    check(load().mixlu_report_read(ctx, _p(d_reps), count, out), "mixlu_report_read")
    return [out[i].as_dict() for i in range(count)]


def _factor(name, ctx, prec: int, A, work, opts=None):
    F = mixlu_factor()
    info = ctypes.c_int()
    n = A.shape[0]
    check(getattr(load(), name)(ctx, prec, n, _p(A), _ld(A, _cm(opts)), _p(work),
                                work.numel() * work.element_size(),
                                None if opts is None else ctypes.byref(opts), ctypes.byref(F),
                                ctypes.byref(info)), name)
    return F, info.value


def mixlu_getrf(ctx, prec: int, A, work, opts=None):
    return _factor("mixlu_getrf", ctx, prec, A, work, opts)


def mixlu_potrf(ctx, prec: int, A, work, opts=None):
    return _factor("mixlu_potrf", ctx, prec, A, work, opts)


FACTOR_PENDING = 1


def _factor_async(name, ctx, prec: int, A, work, d_info, opts=None) -> mixlu_factor:
    F = mixlu_factor()
    n = A.shape[0]
    check(getattr(load(), name)(ctx, prec, n, _p(A), _ld(A, _cm(opts)), _p(work),
                                work.numel() * work.element_size(),
                                None if opts is None else ctypes.byref(opts), ctypes.byref(F),
                                _p(d_info)), name)
    return F


def mixlu_getrf_async(ctx, prec: int, A, work, d_info, opts=None) -> mixlu_factor:
    """Stream-ordered factorization; the outcome lands in d_info (device int32)."""
    return _factor_async("mixlu_getrf_async", ctx, prec, A, work, d_info, opts)


def mixlu_potrf_async(ctx, prec: int, A, work, d_info, opts=None) -> mixlu_factor:
    return _factor_async("mixlu_potrf_async", ctx, prec, A, work, d_info, opts)


def mixlu_getrs(ctx, F: mixlu_factor, B, X, trans: int = 0) -> None:
    n, nrhs = B.shape
    cm = F.layout == COL_MAJOR
    check(load().mixlu_getrs(ctx, ctypes.byref(F), trans, nrhs, _p(B), _ld(B, cm), _p(X),
                             _ld(X, cm)), "mixlu_getrs")


def mixlu_condest(ctx, F: mixlu_factor) -> float:
    """kappa_1(A) estimated with the factors in F (Hager / Higham)."""
    k = ctypes.c_double()
    check(load().mixlu_condest(ctx, ctypes.byref(F), ctypes.byref(k)), "mixlu_condest")
    return k.value


def mixlu_sparse_workspace_size(ctx, inner_prec: int, n: int, nnz: int, m_out: int,
                                m_in: int) -> int:
    out = ctypes.c_size_t()
    check(load().mixlu_sparse_workspace_size(ctx, inner_prec, n, nnz, m_out, m_in,
                                             ctypes.byref(out)), "mixlu_sparse_workspace_size")
    return out.value


def mixlu_sparse_fgmres(ctx, inner_prec: int, rowptr, colind, vals, b, x, m_out: int, m_in: int,
                        work, opts=None) -> mixlu_report:
    """Algorithm 2 on device CRS arrays (int32 rowptr / colind, FP64 vals);
    x (device, FP64) receives the solution."""
    rep = mixlu_report()
    n = b.numel()
    check(load().mixlu_sparse_fgmres(ctx, inner_prec, n, vals.numel(), _p(rowptr), _p(colind),
                                     _p(vals), _p(b), _p(x), m_out, m_in, _p(work),
                                     work.numel() * work.element_size(),
                                     None if opts is None else ctypes.byref(opts),
                                     ctypes.byref(rep)), "mixlu_sparse_fgmres")
    return rep


def mixlu_refine(ctx, F: mixlu_factor, A, B, X, opts=None, trans: int = 0) -> mixlu_report:
    rep = mixlu_report()
    cm = F.layout == COL_MAJOR
    nrhs = B.shape[1]
    check(load().mixlu_refine(ctx, ctypes.byref(F), trans, nrhs, _p(A), _ld(A, cm), _p(B),
                              _ld(B, cm),
                              _p(X), _ld(X, cm), None if opts is None else ctypes.byref(opts),
                              ctypes.byref(rep)), "mixlu_refine")
    return rep


def gemm_update_workspace_bytes(m: int, n: int, k: int) -> int:
    """Workspace mixlu_gemm_update needs for the rounded operands."""
    return 2 * (m + n) * k + (m + n) * k // 32 + 1024


def mixlu_gemm_update(ctx, prec: int, A, B, C, work=None, overflow: bool = False):
    """C -= A B (FP32 device tensors, row-major) with the operands rounded as
    the factorization's trailing update rounds L21 and U12; returns the count
    of out-of-range operands when ``overflow`` is set (synchronizes)."""
    m, k = A.shape
    n = B.shape[1]
    cnt = ctypes.c_int()
    nbytes = 0 if work is None else work.numel() * work.element_size()
    check(load().mixlu_gemm_update(ctx, prec, m, n, k, _p(A), _ld(A), _p(B), _ld(B), _p(C),
                                   _ld(C), _p(work), nbytes,
                                   ctypes.byref(cnt) if overflow else None),
          "mixlu_gemm_update")
    return cnt.value if overflow else None


def mixlu_outer_update(ctx, G, X, GA, alpha: float = -1.0, beta: float = 0.0) -> None:
    n, nrhs = G.shape
    check(load().mixlu_outer_update(ctx, n, nrhs, _p(G), _ld(G), _p(X), _ld(X), _p(GA),
                                    _ld(GA), alpha, beta), "mixlu_outer_update")


def mixlu_batched_workspace_size(ctx, prec: int, batch: int, nrhs: int, opts=None) -> int:
    b = ctypes.c_size_t()
    check(load().mixlu_batched_workspace_size(ctx, prec, batch, nrhs,
                                              None if opts is None else ctypes.byref(opts),
                                              ctypes.byref(b)), "mixlu_batched_workspace_size")
    return b.value


def mixlu_dxgesv_batched(ctx, prec: int, d_n, d_A, d_lda, d_B, d_X, nrhs: int, work, d_reps,
                         opts=None) -> None:
    """All array arguments are device tensors: d_n int32 [batch], d_A / d_B /
    d_X int64 device addresses [batch], d_lda int32 [batch] or None, d_reps
    uint8 [batch * sizeof(mixlu_report)]."""
    batch = d_n.numel()
    check(load().mixlu_dxgesv_batched(ctx, prec, batch, _p(d_n), _p(d_A), _p(d_lda), _p(d_B),
                                      _p(d_X), nrhs, _p(work), work.numel() * work.element_size(),
                                      None if opts is None else ctypes.byref(opts), _p(d_reps)),
          "mixlu_dxgesv_batched")


def mixlu_refine_history(ctx) -> list:
    """True-residual norms evaluated by the last refinement on ctx, in order."""
    cnt = ctypes.c_int()
    check(load().mixlu_refine_history(ctx, None, 0, ctypes.byref(cnt)), "mixlu_refine_history")
    buf = (ctypes.c_double * max(cnt.value, 1))()
    check(load().mixlu_refine_history(ctx, buf, cnt.value, ctypes.byref(cnt)),
          "mixlu_refine_history")
    return list(buf[:cnt.value])


def mixlu_dxgesv_batched_noalloc(ctx, prec: int, d_n, d_A, d_lda, d_B, d_X, nrhs: int, d_reps,
                                 opts=None) -> None:
    """mixlu_dxgesv_batched without a workspace (the library's device
    array serves as one); arguments as there."""
    batch = d_n.numel()
    check(load().mixlu_dxgesv_batched_noalloc(ctx, prec, batch, _p(d_n), _p(d_A), _p(d_lda),
                                              _p(d_B), _p(d_X), nrhs,
                                              None if opts is None else ctypes.byref(opts),
                                              _p(d_reps)),
          "mixlu_dxgesv_batched_noalloc")


def mixlu_batched_tune(ctx, prec: int, d_n, d_A, d_lda, d_B, d_X, nrhs: int, work, d_reps,
                       opts=None):
    """Time every candidate tile set on this batch; the context keeps the
    fastest.  Returns (chosen tiles as a dict, {candidate: ms})."""
    batch = d_n.numel()
    best = mixlu_batched_tiles()
    ms = (ctypes.c_float * len(TILE_CANDIDATES))()
    check(load().mixlu_batched_tune(ctx, prec, batch, _p(d_n), _p(d_A), _p(d_lda), _p(d_B),
                                    _p(d_X), nrhs, _p(work), work.numel() * work.element_size(),
                                    None if opts is None else ctypes.byref(opts), _p(d_reps),
                                    ctypes.byref(best), ms, len(TILE_CANDIDATES)),
          "mixlu_batched_tune")
    return best.as_dict(), {c: float(ms[i]) for i, c in enumerate(TILE_CANDIDATES)}


def mixlu_batched_get_tiles(ctx, prec: int) -> dict:
    t = mixlu_batched_tiles()
    check(load().mixlu_batched_get_tiles(ctx, prec, ctypes.byref(t)), "mixlu_batched_get_tiles")
    return t.as_dict()


def mixlu_batched_set_tiles(ctx, prec: int, panel: int, chunk: int, groups: int,
                            tuned: bool = False) -> None:
    t = mixlu_batched_tiles(panel, chunk, groups, int(tuned))
    check(load().mixlu_batched_set_tiles(ctx, prec, ctypes.byref(t)), "mixlu_batched_set_tiles")


def reports_from_bytes(buf) -> list:
    """Decode a host copy (bytes) of a device array of mixlu_report."""
    sz = ctypes.sizeof(mixlu_report)
    return [mixlu_report.from_buffer_copy(buf[i * sz:(i + 1) * sz]).as_dict()
            for i in range(len(buf) // sz)]


def mixlu_profile_enable(ctx, on: bool = True) -> None:
    check(load().mixlu_profile_enable(ctx, int(on)), "mixlu_profile_enable")


def mixlu_profile_read(ctx) -> dict:
    """Per-kernel-class totals: {name: {launches, ms, flops, bytes}}."""
    arr = (mixlu_kstat * 16)()
    cnt = ctypes.c_int()
    check(load().mixlu_profile_read(ctx, arr, 16, ctypes.byref(cnt)), "mixlu_profile_read")
    return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].ms,
                                   "flops": arr[i].flops, "bytes": arr[i].bytes}
            for i in range(min(cnt.value, 16))}


# ------------------------------------------------------------ convenience
@dataclass
class Result:
    x: object
    report: dict


class Solver:
    """A context plus a reusable workspace on the current device/stream."""

    def __init__(self, stream=None):
        import torch

        # torch allocates the buffers; its HIP runtime, initialized first,
        # is the one the library's calls then use
        torch.cuda.init()
        self.ctx = mixlu_create(stream)
        self._work = None

    def close(self):
        if self.ctx is not None:
            mixlu_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, op: int, prec: int, n: int, nrhs: int, opts=None):
        import torch

        need = mixlu_workspace_size(self.ctx, op, prec, n, nrhs, opts)
        if self._work is None or self._work.numel() < need:
            self._work = None
            torch.cuda.empty_cache()
            self._work = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        return self._work

    @staticmethod
    def _prep(A, B):
        """Keep A's storage order (row-major, or column-major as LAPACK) and
        bring B into the same one; X is allocated in it too."""
        import torch

        if A.dtype != torch.float64 or B.dtype != torch.float64:
            raise TypeError("A and B must be float64")
        vec = B.dim() == 1
        B2 = B.reshape(-1, 1) if vec else B
        if _is_cm(A):
            if not (_is_cm(B2) or B2.shape[1] == 1):
                B2 = B2.t().contiguous().t()
            X = torch.empty(B2.shape[1], B2.shape[0], dtype=B2.dtype, device=B2.device).t()
            return A, B2, X, vec, COL_MAJOR
        A = A.contiguous()
        B2 = B2.contiguous()
        return A, B2, torch.empty_like(B2), vec, ROW_MAJOR

    def dxgesv(self, A, B, prec="fp32", opts=None, **kw) -> Result:
        p = PREC[prec] if isinstance(prec, str) else prec
        A, B2, X, vec, layout = self._prep(A, B)
        o = opts if opts is not None else default_opts(**kw)
        o.layout = layout
        work = self.workspace(OP_GESV, p, A.shape[0], B2.shape[1], o)
        rep = mixlu_dxgesv(self.ctx, p, A, B2, X, work, o)
        return Result(X.reshape(-1) if vec else X, rep.as_dict())

    def dxposv(self, A, B, prec="fp32", opts=None, **kw) -> Result:
        """Symmetric positive definite A: Cholesky in prec + FP64 refinement."""
        p = PREC[prec] if isinstance(prec, str) else prec
        A, B2, X, vec, layout = self._prep(A, B)
        o = opts if opts is not None else default_opts(**kw)
        o.layout = layout
        work = self.workspace(OP_POSV, p, A.shape[0], B2.shape[1], o)
        rep = mixlu_dxposv(self.ctx, p, A, B2, X, work, o)
        return Result(X.reshape(-1) if vec else X, rep.as_dict())

    def batched_buffers(self, As, Bs, prec="fp32", opts=None):
        """Device arrays for mixlu_dxgesv_batched over the lists As (n_i x n_i)
        and Bs (n_i x nrhs): returns a dict of tensors, reusable for repeated
        (or graph-captured) calls on the same buffers."""
        import torch

        p = PREC[prec] if isinstance(prec, str) else prec
        dev = As[0].device
        As = [a.contiguous() for a in As]
        Bs = [(b.reshape(-1, 1) if b.dim() == 1 else b).contiguous() for b in Bs]
        nrhs = Bs[0].shape[1]
        Xs = [torch.empty_like(b) for b in Bs]
        batch = len(As)
        buf = {
            "A": As, "B": Bs, "X": Xs, "nrhs": nrhs, "prec": p,
            "n": torch.tensor([a.shape[0] for a in As], dtype=torch.int32, device=dev),
            "pA": torch.tensor([a.data_ptr() for a in As], dtype=torch.int64, device=dev),
            "pB": torch.tensor([b.data_ptr() for b in Bs], dtype=torch.int64, device=dev),
            "pX": torch.tensor([x.data_ptr() for x in Xs], dtype=torch.int64, device=dev),
            "reps": torch.zeros(batch * ctypes.sizeof(mixlu_report), dtype=torch.uint8, device=dev),
            "opts": opts if opts is not None else default_opts(),
        }
        need = mixlu_batched_workspace_size(self.ctx, p, batch, nrhs, buf["opts"])
        buf["work"] = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        return buf

    def run_batched(self, buf) -> None:
        """Enqueue the batched solve on the context's stream (no sync)."""
        mixlu_dxgesv_batched(self.ctx, buf["prec"], buf["n"], buf["pA"], None, buf["pB"],
                             buf["pX"], buf["nrhs"], buf["work"], buf["reps"], buf["opts"])

    def sparse_fgmres(self, rowptr, colind, vals, b, inner="fp32", m_out=20, m_in=30,
                      opts=None) -> Result:
        """FGMRES(m_out)-GMRES(m_in) (Algorithm 2) for the CRS matrix on the
        device; inner "fp32" is GMRES_SP, "fp64" GMRES_DP."""
        import torch

        p = PREC[inner]
        n, nnz = b.numel(), vals.numel()
        need = mixlu_sparse_workspace_size(self.ctx, p, n, nnz, m_out, m_in)
        work = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        rep = mixlu_sparse_fgmres(self.ctx, p, rowptr, colind, vals, b, x, m_out, m_in, work, opts)
        return Result(x, rep.as_dict())

    def tune_batched(self, buf):
        """Autotune the tile set for this batch's precision on this batch (the
        context keeps it for later launches); returns (tiles, timings)."""
        return mixlu_batched_tune(self.ctx, buf["prec"], buf["n"], buf["pA"], None, buf["pB"],
                                  buf["pX"], buf["nrhs"], buf["work"], buf["reps"], buf["opts"])

    def dxgesv_batched(self, As, Bs, prec="fp32", opts=None):
        """Solve every A_i x_i = b_i in one persistent launch; returns the list
        of X_i and the list of reports."""
        import torch

        buf = self.batched_buffers(As, Bs, prec, opts)
        self.run_batched(buf)
        torch.cuda.synchronize()
        return buf["X"], reports_from_bytes(bytes(buf["reps"].cpu().numpy()))

    def _d(self, op, fn, A, B) -> Result:
        A, B2, X, vec, layout = self._prep(A, B)
        if layout != ROW_MAJOR:
            raise ValueError("the FP64 comparators take row-major A")
        work = self.workspace(op, FP64, A.shape[0], B2.shape[1])
        info = fn(self.ctx, A, B2, X, work)
        return Result(X.reshape(-1) if vec else X, {"info": info})

    def dgesv(self, A, B) -> Result:
        return self._d(OP_DGESV, mixlu_dgesv, A, B)

    def dposv(self, A, B) -> Result:
        return self._d(OP_DPOSV, mixlu_dposv, A, B)

    def sgesv(self, A, B) -> Result:
        """FP32 LU and FP32 solves only (no refinement): the single-precision
        accuracy baseline."""
        A, B2, X, vec, layout = self._prep(A, B)
        if layout != ROW_MAJOR:
            raise ValueError("sgesv takes row-major A")
        work = self.workspace(OP_SGESV, FP32, A.shape[0], B2.shape[1])
        info = mixlu_sgesv(self.ctx, A, B2, X, work)
        return Result(X.reshape(-1) if vec else X, {"info": info})
