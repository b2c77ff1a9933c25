// Batched mixed-precision solves: many independent systems of order <= 512,
// each solved completely (Algorithm 1 with its FP64 fallback) by one
// workgroup of a persistent launch.  Workgroups take systems from an atomic
// queue ordered largest first, so the launch needs no host synchronization
// and allocates nothing (it can be captured in a HIP graph).
//
// Per system, inside one 512-thread workgroup (thread i owns row i):
//   scales   row sums (||A||_inf), power-of-two row and column scales for
//            BF16/FP16 factors, W = fl(R A C) into the workgroup's slot
//   getrf    right-looking LU with partial pivoting, panels of 16 columns
//            held one row per thread, pivot search by wave argmax; row
//            interchanges outside the panel as one composed move list;
//            U12 by forward substitution and the rank-16 trailing update in
//            column chunks staged through LDS (BF16/FP16 operands rounded
//            before the FP32 multiply-add, as on the MFMA path)
//   getrs    P, then blocked forward/backward substitution (32 x 32 diagonal
//            blocks in one wave, row updates by all threads)
//
// The factor is stored column-major in the workgroup's slot (element (i, j)
// at j n + i): with one row per thread, every sweep over a column (panel
// loads, trailing update, triangular-solve updates) is then a contiguous
// access across the lanes of a wave.
//   refine   r = b - A x in FP64 with the original A, stopping test,
//            stall rule, x += z; FP64 LU of the same system on failure.
#include <climits>

#include "common.h"

namespace mixlu {

constexpr int kBT = 512;      // threads per workgroup = largest order
constexpr int kBW = kBT / 64; // waves
constexpr int kBB = 16;       // panel width
constexpr int kBC = 128;      // trailing-update chunk (columns)
constexpr int kBDiag = 32;    // diagonal block of the triangular solves
constexpr int kSUP = kBB + 4; // pitch of a staged U12 column (16-byte aligned)

struct BShared {
    double x[kBatchedNmax];   // solution column (FP64)
    double r[kBatchedNmax];   // right-hand side / residual (FP64)
    double R[kBatchedNmax], C[kBatchedNmax];
    double y[kBatchedNmax];   // solve vector (float or double storage)
    double L11[kBB * (kBB + 4)]; // unit lower block of the current panel (T storage)
    double sU[kBC * kSUP];    // staged U12 chunk, column-major (float or double storage)
    double prow[kBB], drow[kBB];
    double valw[kBW];
    double red[kBW][2];
    int pivw[kBW];
    int piv[kBatchedNmax];
    int perm[kBatchedNmax];   // row of A (before pivoting) now at each position
    int src[kBatchedNmax];
    int mv_dst[2 * kBB], mv_src[2 * kBB];
    int nmoves;
    int bad;                  // first failing pivot column + 1 (INT_MAX: none)
    int overflow;
    int sys;
};

// Value of a trailing-update operand after rounding to the operand format
// (identity for FP32/FP64 factors).
template <int LP, typename T> __device__ __forceinline__ T lowp_round(T v) {
    if constexpr (LP == MIXLU_FP16) return (T)(_Float16)v;
    else if constexpr (LP == MIXLU_BF16) return (T)(__bf16)v;
    else return v;
}

// ---------------------------------------------------------------- scales
// ||A||_inf -> return value (all threads); R, C in LDS (power-of-two
// equilibration when equil, else 1); W = fl(R A C) with ld = n.
template <typename T>
__device__ __noinline__ double sys_convert(const double *__restrict__ A, int lda, int n, int equil,
                              T *__restrict__ W, BShared &sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double anorm = 0.0;
    // row max and row sum: one wave per row, lanes along the row
    for (int i = wave; i < n; i += kBW) {
        double mx = 0.0, sm = 0.0;
        for (int j = lane; j < n; j += 64) {
            const double v = fabs(A[(size_t)i * lda + j]);
            mx = (v > mx || v != v) ? v : mx;
            sm += v;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(mx, off);
            mx = (o > mx || o != o) ? o : mx;
            sm += __shfl_xor(sm, off);
        }
        if (lane == 0) {
            double s = 1.0;
            if (equil && mx > 0.0 && mx <= 1.79769313486231570815e308) s = ldexp(1.0, -ilogb(mx));
            sh.R[i] = s;
            sh.x[i] = sm;  // row sums, reduced below
        }
    }
    __syncthreads();
    {
        double m = 0.0;
        for (int i = tid; i < n; i += kBT) {
            const double v = sh.x[i];
            m = (v > m || v != v) ? v : m;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(m, off);
            m = (o > m || o != o) ? o : m;
        }
        if (lane == 0) sh.red[wave][0] = m;
    }
    // column scales from the R-scaled column max: one thread per column
    for (int j = tid; j < n; j += kBT) {
        double s = 1.0;
        if (equil) {
            double mx = 0.0;
            for (int i = 0; i < n; ++i) {
                const double v = fabs(A[(size_t)i * lda + j]) * sh.R[i];
                mx = (v > mx || v != v) ? v : mx;
            }
            if (mx > 0.0 && mx <= 1.79769313486231570815e308) s = ldexp(1.0, -ilogb(mx));
        }
        sh.C[j] = s;
    }
    __syncthreads();
    for (int q = 0; q < kBW; ++q) {
        const double v = sh.red[q][0];
        anorm = (v > anorm || v != v) ? v : anorm;
    }
    // conversion into the column-major W through a 32 x 64 LDS tile: rows of
    // A are read along the lanes, columns of W written along the lanes
    T *tile = reinterpret_cast<T *>(sh.sU);
    constexpr int TR = 32, TC = 64, TP = TC + 1;
    static_assert(TR * TP * sizeof(T) <= sizeof(BShared::sU), "conversion tile");
    int bad = 0;
    for (int I = 0; I < n; I += TR) {
        for (int J = 0; J < n; J += TC) {
            for (int e = tid; e < TR * TC; e += kBT) {
                const int r = e / TC, c = e - r * TC;
                const int i = I + r, j = J + c;
                if (i < n && j < n) {
                    const T w = (T)(sh.R[i] * A[(size_t)i * lda + j] * sh.C[j]);
                    if (!(fabs((double)w) <= 1.79769313486231570815e308)) ++bad;
                    tile[r * TP + c] = w;
                }
            }
            __syncthreads();
            for (int e = tid; e < TR * TC; e += kBT) {
                const int c = e / TR, r = e - c * TR;
                const int i = I + r, j = J + c;
                if (i < n && j < n) W[(size_t)j * n + i] = tile[r * TP + c];
            }
            __syncthreads();
        }
    }
    if (bad) atomicAdd(&sh.overflow, bad);
    __syncthreads();
    return anorm;
}

// ------------------------------------------------------------------ getrf
// In-place LU with partial pivoting of the n x n column-major W (ld = n) by
// the whole workgroup; pivots in sh.piv; the first zero / non-finite pivot
// column is recorded in sh.bad.  Panels are BB columns wide; the trailing
// update runs in chunks of `chunk` (<= kBC) columns.
template <typename T, int LP, int BB>
__device__ __noinline__ void sys_getrf(T *__restrict__ W, int n, int chunk, BShared &sh) {
    static_assert(BB <= kBB && 2 * BB <= 64, "panel width");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row = tid;
    T *prow = reinterpret_cast<T *>(sh.prow);
    T *drow = reinterpret_cast<T *>(sh.drow);
    T *sU = reinterpret_cast<T *>(sh.sU);
    T *L11 = reinterpret_cast<T *>(sh.L11);
    T *valw = reinterpret_cast<T *>(sh.valw);
    constexpr int LP11 = kBB + 4;  // 16-byte aligned rows
    for (int r = tid; r < n; r += kBT) sh.perm[r] = r;
    for (int k = 0; k < n; k += BB) {
        const int w = n - k < BB ? n - k : BB;
        T a[BB];
        const bool mine = row >= k && row < n;
#pragma unroll
        for (int c = 0; c < BB; ++c) a[c] = (mine && c < w) ? W[(size_t)(k + c) * n + row] : (T)0;
        sfor<0, BB>([&](auto J) {
            constexpr int j = decltype(J)::value;
            if (j < w) {
                const int kj = k + j;
                const T av = fabs(a[j]);
                const T v = (row >= kj && row < n && av == av) ? av : (T)-1;
                const WaveArgmax<T> wa = wave_argmax(v);
                if (lane == 0) {
                    valw[wave] = wa.val;
                    sh.pivw[wave] = wa.lane < 64 ? wave * 64 + wa.lane : -1;
                }
                __syncthreads();
                T best = (T)-1;
                int p = -1;
#pragma unroll
                for (int q = 0; q < kBW; ++q) {
                    const T vq = valw[q];
                    if (vq > best) {
                        best = vq;
                        p = sh.pivw[q];
                    }
                }
                if (!(best > (T)0) || !(best < (T)INFINITY)) {
                    if (tid == 0) sh.bad = min(sh.bad, kj + 1);
                    p = kj;
                }
                if (row == p) {
#pragma unroll
                    for (int c = 0; c < BB; ++c) prow[c] = a[c];
                }
                if (row == kj) {
#pragma unroll
                    for (int c = 0; c < BB; ++c) drow[c] = a[c];
                }
                if (tid == 0) sh.piv[kj] = p;
                __syncthreads();
                if (row == kj) {
#pragma unroll
                    for (int c = 0; c < BB; ++c) a[c] = prow[c];
                } else if (row == p) {
#pragma unroll
                    for (int c = 0; c < BB; ++c) a[c] = drow[c];
                }
                if (row > kj && row < n) {
                    const T pv = prow[j];
                    const T l = a[j] / pv;
                    a[j] = l;
#pragma unroll
                    for (int c = j + 1; c < BB; ++c) a[c] -= l * prow[c];
                }
            }
        });
        if (mine) {
#pragma unroll
            for (int c = 0; c < BB; ++c)
                if (c < w) W[(size_t)(k + c) * n + row] = a[c];
        }
        // row-move composition
        for (int r = tid; r < n; r += kBT) sh.src[r] = r;
        if (tid == 0) sh.nmoves = 0;
        __syncthreads();
        // unit lower diagonal block for U12, read back from the stored panel
        for (int e = tid; e < w * BB; e += kBT) {
            const int c = e / w, r = e - c * w;
            L11[r * LP11 + c] = c < w ? W[(size_t)(k + c) * n + k + r] : (T)0;
        }
        if (tid == 0) {
            for (int j = 0; j < w; ++j) {
                const int kj = k + j, p = sh.piv[kj];
                const int t = sh.src[kj];
                sh.src[kj] = sh.src[p];
                sh.src[p] = t;
            }
        }
        __syncthreads();
        int pnew = -1;
        if (row < n && sh.src[row] != row) {
            const int m = atomicAdd(&sh.nmoves, 1);
            sh.mv_dst[m] = row;
            sh.mv_src[m] = sh.src[row];
            pnew = sh.perm[sh.src[row]];
        }
        __syncthreads();
        if (pnew >= 0) sh.perm[row] = pnew;
        const int nm = sh.nmoves;  // <= 2 BB <= 64: one lane per move
        // rows move in the columns left and right of the panel: one wave per
        // column, lane m carries move m (all loads of a column before its
        // stores, so cycles of moves are safe)
        if (lane < nm) {
            const int dst = sh.mv_dst[lane], srow = sh.mv_src[lane];
            constexpr int U = 2;  // columns in flight per wave
            for (int col0 = wave; col0 < n; col0 += U * kBW) {
                T v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int col = col0 + u * kBW;
                    const bool on = col < n && (col < k || col >= k + w);
                    v[u] = on ? W[(size_t)col * n + srow] : (T)0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int col = col0 + u * kBW;
                    if (col < n && (col < k || col >= k + w)) W[(size_t)col * n + dst] = v[u];
                }
            }
        }
        __syncthreads();
        // U12 = L11^{-1} A12 for every column right of the panel, one thread
        // per column (n <= kBT), by forward substitution in registers with
        // L11 read from LDS by broadcast
        {
            const int col = k + w + tid;
            if (col < n) {
                T *wc = W + (size_t)col * n + k;
                T x[BB];
#pragma unroll
                for (int r = 0; r < BB; ++r) x[r] = r < w ? wc[r] : (T)0;
#pragma unroll
                for (int r = 1; r < BB; ++r) {
                    if (r < w) {
#pragma unroll
                        for (int q = 0; q < r; ++q) x[r] -= L11[r * LP11 + q] * x[q];
                    }
                    // keep the L11 loads of later rows from being hoisted
                    // here (they would hold ~BB^2/2 registers)
                    __asm__ volatile("" ::: "memory");
                }
#pragma unroll
                for (int r = 0; r < BB; ++r) {
                    if (r < w) wc[r] = x[r];
                    if constexpr (LP == MIXLU_FP16)
                        if (fabs(x[r]) > (T)65504) atomicAdd(&sh.overflow, 1);
                }
            }
        }
        __syncthreads();
        // A22 -= L21 U12 by chunks of columns: the rounded L21 row of this
        // thread in registers (reloaded from the stored panel), the rounded
        // U12 chunk staged in sU
#pragma unroll
        for (int c = 0; c < BB; ++c)
            a[c] = (row >= k + w && row < n && c < w) ? lowp_round<LP>(W[(size_t)(k + c) * n + row])
                                                      : (T)0;
        for (int c0 = k + w; c0 < n; c0 += chunk) {
            const int nc = n - c0 < chunk ? n - c0 : chunk;
            if (tid < nc) {
                const T *wc = W + (size_t)(c0 + tid) * n + k;
                T *xs = sU + tid * kSUP;
#pragma unroll
                for (int r = 0; r < BB; ++r) xs[r] = r < w ? lowp_round<LP>(wc[r]) : (T)0;
            }
            __syncthreads();
            if (row >= k + w && row < n) {
                T *wr = W + (size_t)c0 * n + row;
#pragma unroll(sizeof(T) == 8 ? 1 : 2)
                for (int t = 0; t < nc; ++t) {
                    T acc = wr[(size_t)t * n];
#pragma unroll
                    for (int q = 0; q < BB; ++q) acc -= a[q] * sU[t * kSUP + q];
                    wr[(size_t)t * n] = acc;
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ getrs
// z = C U^{-1} L^{-1} P (R rhs) with rhs = sh.r (FP64); z into sh.y as double.
template <typename T>
__device__ __noinline__ void sys_getrs(const T *__restrict__ W, int n, BShared &sh) {
    const int tid = threadIdx.x, lane = tid & 63;
    T *y = reinterpret_cast<T *>(sh.y);
    for (int i = tid; i < n; i += kBT) {
        const int p = sh.perm[i];
        y[i] = (T)(sh.R[p] * sh.r[p]);
    }
    __syncthreads();
    // diagonal blocks are staged through LDS (the sU area is free here)
    T *sd = reinterpret_cast<T *>(sh.sU);
    constexpr int DP = kBDiag + 1;
    auto stage = [&](int b0) {
        for (int e = tid; e < kBDiag * kBDiag; e += kBT) {
            const int c = e / kBDiag, r = e - c * kBDiag;
            sd[r * DP + c] = (b0 + r < n && b0 + c < n) ? W[(size_t)(b0 + c) * n + b0 + r] : (T)0;
        }
        __syncthreads();
    };
    // forward: unit lower
    for (int b0 = 0; b0 < n; b0 += kBDiag) {
        stage(b0);
        if (tid < kBDiag) {
            const int i = b0 + lane;
            T yl = i < n ? y[i] : (T)0;
#pragma unroll 4
            for (int q = 0; q < kBDiag; ++q) {
                const T yq = readlane_t(yl, q);
                if (lane > q) yl -= sd[lane * DP + q] * yq;
            }
            if (i < n) y[i] = yl;
        }
        __syncthreads();
        const int e = n - b0 < kBDiag ? n - b0 : kBDiag;
        for (int i = b0 + kBDiag + tid; i < n; i += kBT) {
            T s = y[i];
            const T *wc = W + (size_t)b0 * n + i;
#pragma unroll 8
            for (int q = 0; q < e; ++q) s -= wc[(size_t)q * n] * y[b0 + q];
            y[i] = s;
        }
        __syncthreads();
    }
    // backward: U
    for (int b0 = ((n - 1) / kBDiag) * kBDiag; b0 >= 0; b0 -= kBDiag) {
        stage(b0);
        if (tid < kBDiag) {
            const int i = b0 + lane;
            T yl = i < n ? y[i] : (T)0;
            // each lane divides its row of the block and its right-hand side
            // by its own pivot first, so the chain below has a unit diagonal:
            // one broadcast and one multiply-add per step
            if (i < n) {
                const T d = sd[lane * DP + lane];
                yl /= d;
                for (int c = lane + 1; c < kBDiag; ++c) sd[lane * DP + c] /= d;
            }
#pragma unroll 4
            for (int q = kBDiag - 1; q >= 0; --q) {
                if (b0 + q < n) {
                    const T yq = readlane_t(yl, q);
                    if (lane < q) yl -= sd[lane * DP + q] * yq;
                }
            }
            if (i < n) y[i] = yl;
        }
        __syncthreads();
        const int e = n - b0 < kBDiag ? n - b0 : kBDiag;
        for (int i = tid; i < b0; i += kBT) {
            T s = y[i];
            const T *wc = W + (size_t)b0 * n + i;
#pragma unroll 8
            for (int q = 0; q < e; ++q) s -= wc[(size_t)q * n] * y[b0 + q];
            y[i] = s;
        }
        __syncthreads();
    }
    // promote and scale in place (each thread its own entries)
    for (int i = tid; i < n; i += kBT) {
        sh.r[i] = sh.C[i] * (double)y[i];
    }
    __syncthreads();
}

// ---------------------------------------------------------------- residual
// sh.r = b - A x (FP64, original A); returns (||r||_inf, ||x||_inf) in
// rn/xn on every thread.
__device__ __noinline__ void sys_residual(const double *__restrict__ A, int lda, int n,
                             const double *__restrict__ b, int ldb, BShared &sh, double &rn,
                             double &xn) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double rmax = 0.0, xmax = 0.0;
    // each wave takes RW rows at a time, lanes along the rows, so RW
    // independent row sums are in flight
    constexpr int RW = 4;
    for (int i0 = wave * RW; i0 < n; i0 += kBW * RW) {
        // compensated row sums (s, e): see dot2_add
        double acc[RW], err[RW];
#pragma unroll
        for (int u = 0; u < RW; ++u) acc[u] = err[u] = 0.0;
        for (int j = lane; j < n; j += 64) {
            const double xj = sh.x[j];
#pragma unroll
            for (int u = 0; u < RW; ++u)
                if (i0 + u < n) dot2_add(acc[u], err[u], A[(size_t)(i0 + u) * lda + j], xj);
        }
#pragma unroll
        for (int u = 0; u < RW; ++u) {
            double v = acc[u], e = err[u];
            for (int off = 32; off > 0; off >>= 1) dot2_merge(v, e, __shfl_xor(v, off), __shfl_xor(e, off));
            if (lane == 0 && i0 + u < n) {
                const double r = dot2_residual(b[(size_t)(i0 + u) * ldb], v, e);
                sh.r[i0 + u] = r;
                const double ar = fabs(r);
                rmax = (ar > rmax || ar != ar) ? ar : rmax;
            }
        }
    }
    for (int i = tid; i < n; i += kBT) {
        const double ax = fabs(sh.x[i]);
        xmax = (ax > xmax || ax != ax) ? ax : xmax;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(rmax, off);
        rmax = (o > rmax || o != o) ? o : rmax;
        const double p = __shfl_xor(xmax, off);
        xmax = (p > xmax || p != p) ? p : xmax;
    }
    if (lane == 0) {
        sh.red[wave][0] = rmax;
        sh.red[wave][1] = xmax;
    }
    __syncthreads();
    rn = 0.0;
    xn = 0.0;
#pragma unroll
    for (int q = 0; q < kBW; ++q) {
        const double a = sh.red[q][0], c = sh.red[q][1];
        rn = (a > rn || a != a) ? a : rn;
        xn = (c > xn || c != c) ? c : xn;
    }
    __syncthreads();
}

struct RefineOut {
    int iters;  // >= 0 converged after that many corrections; < 0 failure code
    double rn, xn;
};

// Algorithm 1 steps 4-7 for one right-hand-side column from x = sh.x, with
// the factor W (T storage).  Every thread takes the same decisions.
template <typename T>
__device__ __noinline__ RefineOut sys_refine(const double *__restrict__ A, int lda, int n,
                                const double *__restrict__ b, int ldb, const T *__restrict__ W,
                                double anorm, int itermax, double stall, BShared &sh) {
    const double thr = sqrt((double)n) * 1.1102230246251565404e-16 * anorm;
    double prev = 0.0, ratio_prev = 0.0;
    RefineOut out{0, 0.0, 0.0};
    for (int k = 0;; ++k) {
        double rn, xn;
        sys_residual(A, lda, n, b, ldb, sh, rn, xn);
        out.rn = rn;
        out.xn = xn;
        const bool finite = rn == rn && xn == xn && rn <= 1.79769313486231570815e308 &&
                            xn <= 1.79769313486231570815e308;
        if (finite && rn <= thr * xn) {
            out.iters = k;
            return out;
        }
        if (!finite) {
            out.iters = -4;
            return out;
        }
        if (k >= 1 && prev > 0.0) {
            const double rho = rn / prev;
            if ((k >= 2 && rho >= stall && ratio_prev >= stall) || (k >= 3 && rho >= 1.0)) {
                out.iters = -4;
                return out;
            }
            ratio_prev = rho;
        }
        prev = rn;
        if (k == itermax) {
            out.iters = -(itermax + 1);
            return out;
        }
        sys_getrs<T>(W, n, sh);  // z into sh.r
        for (int i = threadIdx.x; i < n; i += kBT) sh.x[i] += sh.r[i];
        __syncthreads();
    }
}

struct BatchArgs {
    int batch, nrhs, equil, itermax;
    double stall;
    const int *n;
    const double *const *A;
    const int *lda;
    const double *const *B;
    double *const *X;
    mixlu_report *rep;
    const int *order;
    int *counter;
    unsigned char *slots;
    size_t slot_bytes;
    int fallback;
    int chunk;
};

// Solve one system with the factor in precision T (LP: trailing operand
// rounding); falls back to FP64 inside the same slot.
template <typename T, int LP, int BB>
__device__ void sys_solve(const BatchArgs &g, int s, unsigned char *slot, BShared &sh) {
    const int tid = threadIdx.x;
    const int n = g.n[s];
    const double *A = g.A[s];
    const int lda = g.lda ? g.lda[s] : n;
    const double *B = g.B[s];
    double *X = g.X[s];
    mixlu_report rep{};
    rep.prec = sizeof(T) == 8 ? MIXLU_FP64 : (LP ? LP : MIXLU_FP32);
    if (n <= 0 || n > kBatchedNmax || lda < n) {
        if (tid == 0) {
            rep.info = n == 0 ? 0 : -1;
            rep.converged = n == 0 ? 1 : 0;
            g.rep[s] = rep;
        }
        return;
    }
    T *W = reinterpret_cast<T *>(slot);
    if (tid == 0) {
        sh.bad = INT_MAX;
        sh.overflow = 0;
    }
    __syncthreads();
    const double anorm = sys_convert<T>(A, lda, n, g.equil, W, sh);
    rep.anorm = anorm;
    if (sh.overflow == 0) sys_getrf<T, LP, BB>(W, n, g.chunk, sh);
    int reason = 0;
    if (sh.overflow) reason = -2;
    else if (sh.bad != INT_MAX) reason = sizeof(T) == 8 ? -1 : -3;
    double rn_all = 0.0, xn_all = 0.0;
    int iters_max = 0;
    if (reason == 0) {
        for (int c = 0; c < g.nrhs && reason == 0; ++c) {
            for (int i = tid; i < n; i += kBT) sh.r[i] = B[(size_t)i * g.nrhs + c];
            __syncthreads();
            sys_getrs<T>(W, n, sh);
            for (int i = tid; i < n; i += kBT) sh.x[i] = sh.r[i];
            __syncthreads();
            const RefineOut o = sys_refine<T>(A, lda, n, B + c, g.nrhs, W, anorm, g.itermax,
                                              g.stall, sh);
            if (o.iters < 0) {
                reason = o.iters;
            } else {
                iters_max = o.iters > iters_max ? o.iters : iters_max;
                rn_all = fmax(rn_all, o.rn);
                xn_all = fmax(xn_all, o.xn);
                for (int i = tid; i < n; i += kBT) X[(size_t)i * g.nrhs + c] = sh.x[i];
            }
            __syncthreads();
        }
    }
    if (reason == 0) {
        rep.iter = iters_max;
        rep.converged = 1;
        rep.rnorm = rn_all;
        rep.xnorm = xn_all;
        rep.berr = xn_all > 0 ? rn_all / (anorm * xn_all) : 0.0;
        if (tid == 0) g.rep[s] = rep;
        return;
    }
    // failure: the report says why; with a low-precision factor and the
    // fallback on, k_batched_fallback finishes the system in FP64
    rep.iter = reason;
    if (reason == -1) rep.info = sh.bad;
    if (tid == 0) g.rep[s] = rep;
}

// True when system s failed in the low precision and awaits the FP64 path.
__device__ __forceinline__ bool needs_fallback(const mixlu_report &r) {
    return r.converged == 0 && r.iter < 0 && r.prec != MIXLU_FP64;
}

// FP64 factorization and FP64 refinement of system s (Section 4: the
// double-precision solve used when refinement with the low-precision factor
// fails), in the workgroup's slot; completes the system's report.
__device__ void sys_fallback(const BatchArgs &g, int s, unsigned char *slot, BShared &sh) {
    const int tid = threadIdx.x;
    const int n = g.n[s];
    const double *A = g.A[s];
    const int lda = g.lda ? g.lda[s] : n;
    const double *B = g.B[s];
    double *X = g.X[s];
    mixlu_report rep = g.rep[s];
    const double anorm = rep.anorm;
    double *W64 = reinterpret_cast<double *>(slot);
    if (tid == 0) {
        sh.bad = INT_MAX;
        sh.overflow = 0;
    }
    __syncthreads();
    sys_convert<double>(A, lda, n, 0, W64, sh);
    sys_getrf<double, 0, kBB / 2>(W64, n, g.chunk, sh);
    rep.prec = MIXLU_FP64;
    if (sh.bad != INT_MAX) {
        rep.info = sh.bad;
        if (tid == 0) g.rep[s] = rep;
        return;
    }
    double rn_all = 0.0, xn_all = 0.0;
    int fit = 0, conv = 1;
    for (int c = 0; c < g.nrhs; ++c) {
        for (int i = tid; i < n; i += kBT) sh.r[i] = B[(size_t)i * g.nrhs + c];
        __syncthreads();
        sys_getrs<double>(W64, n, sh);
        for (int i = tid; i < n; i += kBT) sh.x[i] = sh.r[i];
        __syncthreads();
        const RefineOut o = sys_refine<double>(A, lda, n, B + c, g.nrhs, W64, anorm, g.itermax,
                                               g.stall, sh);
        if (o.iters < 0) conv = 0;
        fit = o.iters > fit ? o.iters : fit;
        rn_all = fmax(rn_all, o.rn);
        xn_all = fmax(xn_all, o.xn);
        for (int i = tid; i < n; i += kBT) X[(size_t)i * g.nrhs + c] = sh.x[i];
        __syncthreads();
    }
    rep.fallback_iter = fit;
    rep.converged = conv;
    rep.rnorm = rn_all;
    rep.xnorm = xn_all;
    rep.berr = xn_all > 0 ? rn_all / (anorm * xn_all) : 0.0;
    if (tid == 0) g.rep[s] = rep;
}

template <typename T, int LP, int BB>
__device__ __forceinline__ void batched_loop(const BatchArgs &g, BShared &sh) {
    unsigned char *slot = g.slots + (size_t)blockIdx.x * g.slot_bytes;
    for (;;) {
        if (threadIdx.x == 0) {
            const int q = atomicAdd(g.counter, 1);
            sh.sys = q < g.batch ? g.order[q] : -1;
        }
        __syncthreads();
        const int s = sh.sys;
        __syncthreads();
        if (s < 0) return;  // every workgroup leaves once the queue is empty
        sys_solve<T, LP, BB>(g, s, slot, sh);
        __syncthreads();
    }
}

// FP32-storage factors: two workgroups per CU, so at most 128 VGPRs (4
// waves per SIMD), which these code paths meet without spilling.
template <int LP, int BB>
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(4))) void k_batched(
    BatchArgs g) {
    __shared__ BShared sh;
    batched_loop<float, LP, BB>(g, sh);
}

// FP64 factors (the FP64 comparator), under the same register budget.
template <int BB>
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(4))) void k_batched_fp64(
    BatchArgs g) {
    __shared__ BShared sh;
    batched_loop<double, 0, BB>(g, sh);
}

// Second pass over the same queue (its own counter): the systems whose
// low-precision solve failed get the FP64 path; the others are skipped.  A
// launch of its own, so the registers of the FP64 code do not limit the
// occupancy of the low-precision pass.
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(4))) void k_batched_fallback(
    BatchArgs g) {
    __shared__ BShared sh;
    unsigned char *slot = g.slots + (size_t)blockIdx.x * g.slot_bytes;
    for (;;) {
        if (threadIdx.x == 0) {
            int sys = -1;
            for (;;) {
                const int q = atomicAdd(g.counter + 1, 1);
                if (q >= g.batch) break;
                const int cand = g.order[q];
                if (needs_fallback(g.rep[cand])) {
                    sys = cand;
                    break;
                }
            }
            sh.sys = sys;
        }
        __syncthreads();
        const int s = sh.sys;
        __syncthreads();
        if (s < 0) return;
        sys_fallback(g, s, slot, sh);
        __syncthreads();
    }
}

// order[] = system indices by decreasing n (counting sort in one workgroup);
// out-of-range n sort last.  Also resets the queue counter.
__global__ __launch_bounds__(1024) void k_batch_order(int batch, const int *__restrict__ n,
                                                      int *__restrict__ order,
                                                      int *__restrict__ counter) {
    constexpr int NB = kBatchedNmax + 2;
    __shared__ int cnt[NB];
    __shared__ int start[NB];
    for (int i = threadIdx.x; i < NB; i += 1024) cnt[i] = 0;
    __syncthreads();
    auto bin = [&](int v) { return (v < 0 || v > kBatchedNmax) ? kBatchedNmax + 1 : kBatchedNmax - v; };
    for (int i = threadIdx.x; i < batch; i += 1024) atomicAdd(&cnt[bin(n[i])], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int b = 0; b < NB; ++b) {
            start[b] = acc;
            acc += cnt[b];
        }
        counter[0] = 0;
        counter[1] = 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < batch; i += 1024) {
        const int pos = atomicAdd(&start[bin(n[i])], 1);
        order[pos] = i;
    }
}

size_t batched_slot_bytes() { return align_up((size_t)kBatchedNmax * kBatchedNmax * 8, 256); }

bool batched_tiles_valid(const BatchedTiles &t) {
    return (t.panel == 8 || t.panel == 16) && (t.chunk == 32 || t.chunk == 64 || t.chunk == 128) &&
           (t.groups == 1 || t.groups == 2);
}

template <int LP>
hipError_t launch_lowp(int panel, int grid, const BatchArgs &g, hipStream_t s) {
    if (panel == 8) k_batched<LP, 8><<<grid, kBT, 0, s>>>(g);
    else k_batched<LP, 16><<<grid, kBT, 0, s>>>(g);
    return hipGetLastError();
}

hipError_t launch_batched(int prec, int batch, int nrhs, int equil, int itermax, double stall,
                          int fallback, const int *n, const double *const *A, const int *lda,
                          const double *const *B, double *const *X, mixlu_report *rep,
                          int *order, int *counter, void *slots, int nslots,
                          const BatchedTiles &t, int num_cu, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    if (!batched_tiles_valid(t)) return hipErrorInvalidValue;
    k_batch_order<<<dim3(1), dim3(1024), 0, s>>>(batch, n, order, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    BatchArgs g{batch, nrhs, equil, itermax, stall, n, A, lda, B, X, rep, order, counter,
                static_cast<unsigned char *>(slots), batched_slot_bytes(), fallback, t.chunk};
    // persistent workgroups: `groups` per CU, at most one per slot and system
    int grid = t.groups * (num_cu > 0 ? num_cu : 256);
    if (grid > nslots) grid = nslots;
    if (grid > batch) grid = batch;
    switch (prec) {
        case MIXLU_FP32: e = launch_lowp<0>(t.panel, grid, g, s); break;
        case MIXLU_FP16: e = launch_lowp<MIXLU_FP16>(t.panel, grid, g, s); break;
        case MIXLU_BF16: e = launch_lowp<MIXLU_BF16>(t.panel, grid, g, s); break;
        case MIXLU_FP64:
            if (t.panel == 8) k_batched_fp64<8><<<grid, kBT, 0, s>>>(g);
            else k_batched_fp64<16><<<grid, kBT, 0, s>>>(g);
            e = hipGetLastError();
            break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || prec == MIXLU_FP64 || !fallback) return e;
    k_batched_fallback<<<grid, kBT, 0, s>>>(g);
    return hipGetLastError();
}

}  // namespace mixlu
