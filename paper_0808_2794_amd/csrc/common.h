// Internal definitions shared by the HIP sources of libmixlu (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "../../include/mixlu.h"

namespace mixlu {

// ------------------------------------------------------------ constants
constexpr int kPanelTPB = 512;     // threads of one panel workgroup
constexpr int kPanelRows = 1;      // panel rows held per thread
constexpr int kPanelRowsPerWG = kPanelTPB * kPanelRows;
constexpr int kPanelMaxWG = 64;    // at most 64 panel workgroups (m <= 32768)
constexpr int kPanelBF = 64;       // panel width, FP32 factors
constexpr int kPanelBD = 32;       // panel width, FP64 factors
constexpr int kXbufWords = 2 * (kPanelMaxWG * (4 + 64) + 64);  // panel exchange words
constexpr int kXcdStride = 8;      // workgroups are dealt round-robin to 8 XCDs
constexpr int kTrsvBS = 64;        // rows per block of the chained solves
constexpr int kTrsvPrefetch = 4;   // tile rows requested ahead in the chained solves
constexpr int kTrsvNRT = 8;        // right-hand sides per chained-solve launch
constexpr int kSparseMaxRestart = 512;  // largest m_out / m_in of the sparse solver
constexpr int kColChunks = 64;   // row chunks of the column-statistics pass
constexpr unsigned kSpinLimit = 1u << 23;  // polls before a device wait gives up
constexpr int kKrylov = 30;         // default flexible GMRES restart length
constexpr int kKrylovMax = 128;     // longest restart (the Krylov area's capacity)
constexpr int kMaxOuterBlock = 1024;  // widest outer block (pivots per wide row interchange)
constexpr int kMovesInts = 4 + 4 * kMaxOuterBlock;  // one composed row-move list
// one panel's composed interchanges: count, then (destination row, source
// row) pairs, at most 2 per pivot
constexpr int kPanelMovesInts = 4 + 4 * kPanelBF;
// the lists of one outer block's panels (the narrowest panel is kPanelBD)
constexpr int kPanelListInts = kMaxOuterBlock / kPanelBD * kPanelMovesInts;
constexpr int kBatchedNmax = 512;   // largest order of a batched system
constexpr int kBatchedSlots = 512;  // workgroups (and workspace slots) of a batched launch

// status words kept in the workspace (int32 each)
enum StatusWord {
    ST_BREAKDOWN = 0,  // min over zero/non-finite pivot columns + 1 (INT_MAX: none)
    ST_TIMEOUT = 1,    // nonzero: a bounded cross-workgroup wait gave up
    ST_OVERFLOW = 2,   // count of non-finite values after conversion
    ST_CHOL = 3,       // min over non-positive Cholesky pivots + 1 (INT_MAX: none)
    ST_COUNT = 8
};

// ------------------------------------------------------------- helpers
inline int round_up(int x, int m) { return (x + m - 1) / m * m; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Exchange words: 32-bit tag in the high half, 32-bit payload in the low half.
__device__ inline void xstore(unsigned long long *p, unsigned tag, unsigned payload) {
    __hip_atomic_store(p, ((unsigned long long)tag << 32) | payload, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
// Store for readers on the same XCD only: a workgroup-scope store goes
// through the compute unit's L1 into the XCD's L2, which every compute unit
// of that XCD shares, and the readers' agent-scope loads (xload) find it
// there.  Cheaper than an agent-scope store, which must become visible to
// all XCDs; used only when every participating workgroup sits on one XCD
// (the wait that reads it is bounded, so a broken placement ends in the
// timeout status, not a hang).
__device__ inline void xstore_near(unsigned long long *p, unsigned tag, unsigned payload) {
    __hip_atomic_store(p, ((unsigned long long)tag << 32) | payload, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline unsigned long long xload(const unsigned long long *p) {
    return __hip_atomic_load(const_cast<unsigned long long *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline bool flag_set(const int *p) {
    return __hip_atomic_load(const_cast<int *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}
// Poll *p until its tag equals `tag`; returns the payload.  Gives up after
// kSpinLimit polls or when *timeout is raised by another workgroup, raising
// *timeout and setting `bad`.
__device__ inline unsigned spin_tag(const unsigned long long *p, unsigned tag, int *timeout,
                                    bool &bad) {
    unsigned long long w = xload(p);
    unsigned spins = 0;
    while ((unsigned)(w >> 32) != tag) {
        ++spins;
        if (spins > kSpinLimit || ((spins & 1023u) == 0 && flag_set(timeout))) {
            __hip_atomic_store(timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bad = true;
            return 0u;
        }
        w = xload(p);
    }
    return (unsigned)w;
}

// Compensated accumulation of FP64 products (Ogita, Rump and Oishi's Dot2):
// the pair (s, c) holds a running sum and the accumulated rounding errors of
// its products (exact, from one FMA each) and additions (exact, from
// TwoSum), so s + c is as accurate as a sum formed in twice the working
// precision.  Residuals use it: their stopping test compares quantities
// near the unit roundoff, where an ordinary FP64 sum carries rounding of
// the same size.  Contraction is off so no product fuses into a sum.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
#pragma clang fp contract(off)
    s = a + b;
    const double z = s - a;
    e = (a - (s - z)) + (b - z);
}
__device__ __forceinline__ void dot2_add(double &s, double &c, double a, double x) {
#pragma clang fp contract(off)
    const double p = a * x;
    const double pe = __builtin_fma(a, x, -p);
    double t, e;
    two_sum(s, p, t, e);
    s = t;
    c += e + pe;
}
__device__ __forceinline__ void dot2_merge(double &s, double &c, double s2, double c2) {
#pragma clang fp contract(off)
    double t, e;
    two_sum(s, s2, t, e);
    s = t;
    c += e + c2;
}
// b - (s + c), rounded once
__device__ __forceinline__ double dot2_residual(double b, double s, double c) {
#pragma clang fp contract(off)
    double t, e;
    two_sum(b, -s, t, e);
    return t + (e - c);
}

// Uniform value of lane `lane` (a compile-time or wave-uniform index).
template <typename T> __device__ __forceinline__ T readlane_t(T v, int lane) {
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
    } else {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    }
}
// Compile-time loop: f(integral_constant<int, I>) for I = 0 .. N-1.
template <int I, int N, class F> __device__ __forceinline__ void sfor(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        sfor<I + 1, N>(f);
    }
}

// A register row as B / V vectors of V = 16 / sizeof(T) values: LDS copies
// are then plain 16-byte moves with no repacking.
template <typename T> struct Vq {
    static constexpr int V = 16 / sizeof(T);
    typedef T type __attribute__((ext_vector_type(V)));
};
// ---------------------------------------------------------------------
// Wave-wide reductions on DPP (no LDS traffic).  After the four in-row
// steps every lane of a 16-lane row holds the row's result; row_bcast:15
// and row_bcast:31 fold the rows so that lane 63 holds the wave's result,
// which is then read into a scalar register.
// ---------------------------------------------------------------------
template <int CTRL, int RM>
__device__ __forceinline__ unsigned dpp32(unsigned x) {
    return (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, RM, 0xF, false);
}
template <int CTRL, int RM>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long x) {
    const unsigned lo = dpp32<CTRL, RM>((unsigned)x);
    const unsigned hi = dpp32<CTRL, RM>((unsigned)(x >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
// Wave-wide maximum of a float or double with the result in every lane
// (read back as a uniform value).  For FP32 each step is one DPP-fused
// v_max; FP64 moves both halves and takes v_max_f64.
template <int CTRL, int RM> __device__ __forceinline__ float dppf(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), CTRL,
                                                      RM, 0xF, false));
}
template <int CTRL, int RM> __device__ __forceinline__ double dppd(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    return __longlong_as_double((long long)dpp64<CTRL, RM>(u));
}
// Candidate values are |x| >= 0 or -1 (no candidate).  For FP32 they order
// like their bit patterns read as signed integers, so the step is an integer
// max, which takes a DPP operand directly (a float max would have to
// canonicalize NaNs first).
template <int CTRL, int RM> __device__ __forceinline__ int dpp_maxi(int x) {
    // rows outside RM keep x: max(x, x) = x
    return max(x, __builtin_amdgcn_update_dpp(x, x, CTRL, RM, 0xF, false));
}
template <typename T, int CTRL, int RM> __device__ __forceinline__ T dmax(T x) {
    if constexpr (sizeof(T) == 4) return __int_as_float(dpp_maxi<CTRL, RM>(__float_as_int(x)));
    else return fmax(x, dppd<CTRL, RM>(x));
}
// max over all 64 lanes
template <typename T> __device__ __forceinline__ T wave_max(T x) {
    x = dmax<T, 0xB1, 0xF>(x);   // quad_perm [1,0,3,2]
    x = dmax<T, 0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
    x = dmax<T, 0x141, 0xF>(x);  // row_half_mirror
    x = dmax<T, 0x140, 0xF>(x);  // row_mirror
    x = dmax<T, 0x142, 0xA>(x);  // row_bcast:15 into rows 1, 3
    x = dmax<T, 0x143, 0xC>(x);  // row_bcast:31 into rows 2, 3
    return readlane_t(x, 63);
}
// max over lanes 0..7 (the other lanes must hold -1)
template <typename T> __device__ __forceinline__ T max8(T x) {
    x = dmax<T, 0xB1, 0xF>(x);
    x = dmax<T, 0x4E, 0xF>(x);
    x = dmax<T, 0x141, 0xF>(x);
    return readlane_t(x, 0);
}
// Index of the first lane whose predicate holds (64 if none).
__device__ __forceinline__ int first_lane(bool pred) {
    const unsigned long long m = __ballot(pred);
    return m ? __ffsll((long long)m) - 1 : 64;
}

// Pivot choice inside one wave: the largest |value| among the valid lanes,
// the smallest lane (= smallest row) on ties.  Invalid lanes hold -1.
template <typename T> struct WaveArgmax {
    T val;    // winning |value| (-1 if no valid lane)
    int lane; // winning lane (64 if none)
};
template <typename T> __device__ __forceinline__ WaveArgmax<T> wave_argmax(T v) {
    WaveArgmax<T> r;
    r.val = wave_max(v);
    r.lane = first_lane(r.val >= (T)0 && v == r.val);
    return r;
}

template <typename T> struct Words;
template <> struct Words<float> {
    static constexpr int n = 1;
    __device__ static unsigned get(float v, int) { return __float_as_uint(v); }
    __device__ static float make(const unsigned *w) { return __uint_as_float(w[0]); }
};
template <> struct Words<double> {
    static constexpr int n = 2;
    __device__ static unsigned get(double v, int i) {
        unsigned long long b = (unsigned long long)__double_as_longlong(v);
        return i ? (unsigned)(b >> 32) : (unsigned)b;
    }
    __device__ static double make(const unsigned *w) {
        return __longlong_as_double((long long)(((unsigned long long)w[1] << 32) | w[0]));
    }
};

// ------------------------------------------------------ workspace layout
// Offsets (bytes) of the regions of one solver workspace; see plan_layout.
struct Layout {
    int n, npad, nb, nrhs, prec, kind;
    bool fallback;
    size_t W;        // working factor: npad x npad, float (or double when prec = FP64)
    size_t W64;      // FP64 fallback factor (npad x npad double) or 0
    size_t Ap, Bp;   // packed low-precision GEMM operands
    size_t ipiv, perm;            // int[npad] each
    size_t R, C;     // double[npad] scales
    size_t vec_r;    // double[npad * nrhs] residual
    size_t vec_y;    // double[npad * nrhs] solve vector (float or double view)
    size_t vec_z;    // double[npad * nrhs] second solve vector (blocked solves)
    size_t krylov;   // flexible GMRES: V (kKrylovMax + 1 vectors), Z (kKrylovMax), h, y (doubles)
    size_t xbuf;     // panel exchange words
    size_t ybuf;     // chained-solve exchange words + tickets
    size_t moves;    // int[2 * (2 * nb + 64) + 4] row-move lists
    size_t tmp;      // scratch: row/column statistics (double[(kColChunks + 2) * npad])
    size_t status;   // int[ST_COUNT]
    size_t norms;    // double[4 + 3 * nrhs]: anorm, ..., rnorm[nrhs], xnorm[nrhs], prev[nrhs]
    size_t dinv;     // inverse diagonal blocks of W's factors (2 npad x 64, W's element type)
    size_t dinv64;   // the same for W64 (FP64), or 0
    size_t total;
};

size_t plan_layout(Layout &L, int op, int prec, int n, int nrhs, const mixlu_opts &o);

// -------------------------------------------------------- kernel launchers
// Every launcher enqueues on `s` and returns hipGetLastError().
hipError_t launch_fill_u32(unsigned *p, unsigned v, size_t count, hipStream_t s);
hipError_t launch_factor_info(const int *status, int chol, int fp64, int *info, hipStream_t s);

// a1/a2: norms, equilibration, conversion (k_convert.hip).  The n x n input
// is always read as the row-major matrix M (a column-major A is M = A^T).
// rowmax/rowsum/colpart are scratch arrays in the workspace.
hipError_t launch_row_stats(const double *A, int lda, int n, double *rowmax, double *rowsum,
                            hipStream_t s);
hipError_t launch_finish_rows(int n, int npad, const double *rowmax, const double *rowsum,
                              double *R, int equil, double *norms, hipStream_t s);
hipError_t launch_col_stats(const double *A, int lda, int n, int npad, const double *R,
                            double *colpart, double *C, int equil, double *norms, hipStream_t s);
template <typename Tw>
hipError_t launch_convert(const double *A, int lda, int n, int npad, const double *R,
                          const double *C, Tw *W, int ldw, int *status, hipStream_t s);
// Without equilibration: conversion, ||M||_inf and ||M||_1 in one pass over
// A (tmp: (2 kColChunks + 2) npad doubles), R = C = 1.
template <typename Tw>
hipError_t launch_convert_stats(const double *A, int lda, int n, int npad, Tw *W, int ldw,
                                double *tmp, double *R, double *C, double *norms, int *status,
                                hipStream_t s);

// a3: factorization kernels (k_lu.hip)
// GEPP of the B columns at (k0, k0) over m rows; with perm or sc1 > sc0 its
// interchanges are also applied to the columns [sc0, sc1) outside the panel
// (sc0 <= k0, sc1 >= k0 + B) and to perm; with pmoves they are also written
// there as a composed move list (kPanelMovesInts ints)
template <typename T>
hipError_t launch_panel(T *W, int ldw, int k0, int m, int *ipiv, unsigned long long *xb,
                        int *status, hipStream_t s, int *perm = nullptr, int sc0 = 0,
                        int sc1 = 0, int *pmoves = nullptr);
// pivots ipiv[k0 .. k0+cnt-1] applied to the columns [c0, c1) minus
// [skip0, skip1) of W, and to perm when given, in one launch
template <typename T>
hipError_t launch_row_swaps(const int *ipiv, int k0, int cnt, int npad, int *perm, T *W, int ldw,
                            int c0, int c1, int skip0, int skip1, int *moves, hipStream_t s);
// blocks of more pivots than this (with a moves buffer of 2 + 4 cnt ints)
// compose once in a separate launch
constexpr int kSwapsFused = 64;
// The two halves of a wide interchange, for one composition applied to
// several column ranges (possibly on different streams): the pivots
// ipiv[k0 .. k0+cnt-1] composed into moves (and perm, when given) once, then
// the rows of [c0, c1) minus [skip0, skip1) moved by that list.
hipError_t launch_swaps_compose(const int *ipiv, int k0, int cnt, int npad, int *perm, int *moves,
                                hipStream_t s);
// The same composition from the np panels' move lists (plist, stride ints
// apart, as the panel writes them) of the block whose first row is k0: the
// lists are applied in order, each in one parallel round.
hipError_t launch_swaps_merge(const int *plist, int np, int stride, int k0, int npad,
                              int *moves, hipStream_t s);
template <typename T>
hipError_t launch_swaps_apply(T *W, int ldw, const int *moves, int cnt, int c0, int c1, int skip0,
                              int skip1, hipStream_t s);
template <typename T>
hipError_t launch_trsm_diag(const T *Ldiag, int ldl, T *X, int ldx, int ncols, hipStream_t s);
// C -= op(A) op(B) with K split over nsplit workgroup slices: partial
// products in P ((nsplit - 1) M ldc elements), then summed into C
template <typename T>
hipError_t launch_gemm_splitk(int M, int N, int K, const T *A, int lda, const T *B, int ldb,
                              T *C, int ldc, int transb, int transa, T *P, int nsplit,
                              hipStream_t s);
template <typename T>
hipError_t launch_gemm(int M, int N, int K, const T *A, int lda, const T *B, int ldb, T *C,
                       int ldc, hipStream_t s, int transb = 0, int lower = 0, int transa = 0,
                       int spare_xcd0 = 0);
hipError_t launch_pack(int prec, const float *W, int ldw, int rows, int cols, int transpose,
                       void *dst, int *status, hipStream_t s);
hipError_t launch_gemm_lowp(int prec, int M, int N, int K, const void *Ap, const void *Bp,
                            float *C, int ldc, hipStream_t s, int lower = 0, int spare_xcd0 = 0);

// FP8 (E4M3 codes with one E8M0 scale per 32 K values) operands and update
hipError_t launch_pack_fp8(const float *W, int ldw, int rows, int K, int transpose, void *codes,
                           void *scales, int *status, hipStream_t s);
hipError_t launch_gemm_fp8(int M, int N, int K, const void *Ac, const void *As, const void *Bc,
                           const void *Bs, float *C, int ldc, hipStream_t s, int lower = 0,
                           int spare_xcd0 = 0);

// a3.5: Cholesky variant (k_chol.hip)
hipError_t launch_sym_scale(const double *A, int lda, int n, int npad, double *R, double *C,
                            int equil, hipStream_t s);
template <typename T>
hipError_t launch_chol_panel(T *W, int ldw, int k, int below, T *diag, int *status, hipStream_t s);
template <typename T>
hipError_t launch_chol_to_lu(T *W, int ldw, int npad, const T *diag, hipStream_t s);

// a10: batched solves (k_batched.hip)
size_t batched_slot_bytes();
// Tile choices of the batched launch (the autotuner's search space): panel
// width of the per-system LU (8 or 16), trailing-update chunk (32, 64 or
// 128 columns) and persistent workgroups per CU (1 or 2).
struct BatchedTiles {
    int panel, chunk, groups;
};
bool batched_tiles_valid(const BatchedTiles &t);
hipError_t launch_batched(int prec, int batch, int nrhs, int equil, int itermax, double stall,
                          int fallback, const int *n, const double *const *A, const int *lda,
                          const double *const *B, double *const *X, mixlu_report *rep,
                          int *order, int *counter, void *slots, int nslots,
                          const BatchedTiles &t, int num_cu, hipStream_t s);

// sparse inner-outer solver (k_sparse.hip)
template <typename TV>
hipError_t launch_csr_spmv(int n, const int *rowptr, const int *colind, const TV *vals, const TV *x,
                           TV *y, hipStream_t s);
hipError_t launch_csr_resid(int n, const int *rowptr, const int *colind, const double *vals,
                            const double *x, const double *b, double *r, double *norms,
                            hipStream_t s);
hipError_t launch_csr_norm_inf(int n, const int *rowptr, const double *vals, double *norms,
                               hipStream_t s);
template <typename TS, typename TD>
hipError_t launch_convert_vec(size_t n, const TS *x, TD *y, hipStream_t s);
template <typename T>
hipError_t launch_vdots(int n, int k, const T *V, size_t ldv, const T *w, T *h, T *part,
                        hipStream_t s);
constexpr int kVdotsChunks = 256;  // most partial sums per dot product
template <typename T>
hipError_t launch_vcombine(int n, int k, const T *V, size_t ldv, const T *h, T *w, hipStream_t s);
template <typename T>
hipError_t launch_vscale(int n, const T *x, const T *den, T *y, hipStream_t s);
template <typename TZ, typename TX>
hipError_t launch_vaxpy_basis(int n, int k, const TZ *Z, size_t ldz, const double *y, TX *x,
                              hipStream_t s, const int *kdev = nullptr);
// inner GMRES least squares on the device: G holds H ((m + 1) x m), cs, sn,
// g and beta; st[0] = running, st[1] = steps taken
constexpr size_t gmres_state_doubles(int m) { return (size_t)(m + 1) * m + 3 * (size_t)m + 2; }
template <typename T>
hipError_t launch_gmres_init(const T *hn, double *G, int m, int *st, hipStream_t s);
template <typename T>
hipError_t launch_gmres_col(const T *h, double *G, int m, int j, double eps_rel, int *st,
                            hipStream_t s);
hipError_t launch_gmres_backsub(const double *G, int m, const int *st, double *y, hipStream_t s);

// kappa_1 estimate (k_condest.hip)
hipError_t launch_cond_start(double *x, int n, int alt, hipStream_t s);
hipError_t launch_cond_sign(const double *y, int n, double *xi, double *out, hipStream_t s);
hipError_t launch_cond_test(const double *z, double *x, int n, double *out, hipStream_t s);

// a4-a8: solves and refinement (k_solve.hip)
template <typename Tw>
hipError_t launch_rhs_gather(int n, int npad, int nrhs, const double *B, int ldb, int b_col_major,
                             const int *perm, const double *R, Tw *Y, int ldy, hipStream_t s);
// Inverses of the 64 x 64 diagonal blocks of L and U in W (dinv: 2 npad x 64)
template <typename T>
hipError_t launch_tri_inv(const T *W, int ldw, int npad, T *dinv, hipStream_t s);
template <typename Tw>
hipError_t launch_trsv(int upper, int trans, const Tw *W, int ldw, const Tw *dinv, int npad,
                       Tw *Y, int ldy, int nrhs, unsigned long long *ybuf, int *status,
                       hipStream_t s);
template <typename Tw>
hipError_t launch_x_update(int n, int npad, int nrhs, int assign, const Tw *Y, int ldy,
                           const int *perm, const double *C, double *X, int ldx, int x_col_major,
                           double *xnorm, hipStream_t s);
hipError_t launch_residual(int n, int nrhs, const double *A, int lda, const double *X, int ldx,
                           const double *B, int ldb, int bx_col_major, double *Rv, int ldr,
                           double *rnorm, double *xnorm, hipStream_t s);
// Blocked triangular solve for several right-hand sides (same matrices as
// launch_trsv): one launch per 64-row block, each solving the diagonal block
// (one wave per right-hand side) and updating the remaining rows of Y; the
// solution is written to Yout (Y is consumed).
template <typename Tw>
hipError_t launch_trsm_blocked(int upper, int trans, const Tw *W, int ldw, int npad, Tw *Y,
                               Tw *Yout, int ldy, int nrhs, hipStream_t s);
// R = B - op(A) X for several right-hand sides on FP64 MFMA, with the
// column norms of R and X (rnorm, xnorm zeroed by the caller)
hipError_t launch_residual_mm(int n, int nrhs, const double *A, int lda, int transa,
                              const double *X, int ldx, const double *B, int ldb, int cm,
                              double *Rv, int ldr, double *rnorm, double *xnorm, double *P,
                              int nsplit, hipStream_t s);
// FP64 vector kernels of the flexible GMRES refinement (V[j * ldv + i])
hipError_t launch_dots(int n, int k, const double *V, size_t ldv, const double *w, double *h,
                       hipStream_t s);
hipError_t launch_combine(int n, int k, const double *V, size_t ldv, const double *h, double sign,
                          double *w, hipStream_t s);
hipError_t launch_scale_copy(int n, double alpha, const double *x, double *y, hipStream_t s);
// part: scratch of 16 * n * 8 doubles
hipError_t launch_residual_t(int n, int nrhs, const double *A, int lda, const double *X, int ldx,
                             const double *B, int ldb, int bx_col_major, double *Rv, int ldr,
                             double *rnorm, double *xnorm, double *part, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, size_t count, hipStream_t s);
hipError_t launch_iota(int *p, int count, hipStream_t s);
hipError_t launch_outer(int n, int nrhs, const double *G, int ldg, const double *X, int ldx,
                        double *GA, int ldga, double alpha, double beta, hipStream_t s);

}  // namespace mixlu
