// Norms, power-of-two equilibration and conversion of A to the working
// format: the steps before Algorithm 1 step 1 ("the coefficient matrix A is
// converted to single precision for the LU factorization", Section 2.1), plus
// ||A||_inf for the stopping test of Section 3 (the DLANGE kernel of Table 7).
//
// All kernels are HBM-streaming: A is read row-major with coalesced 8-byte
// loads, one wave per row for the row statistics and one thread per column
// (over a chunk of rows) for the column statistics.
#include <cfloat>
#include <climits>

#include "common.h"

namespace mixlu {

__global__ void k_fill_u32(unsigned *p, unsigned v, size_t count) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

// Outcome of a factorization from its status words, for callers that do
// not synchronize: 0; k + 1 for an exact zero pivot in column k of an FP64
// factor; -2 (overflow or non-finite value on conversion) or -3 (zero,
// non-finite or non-positive pivot) for a low-precision factor; -100 when a
// bounded cross-workgroup wait gave up.
__global__ void k_factor_info(const int *__restrict__ status, int chol, int fp64,
                              int *__restrict__ info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int brk = chol ? status[ST_CHOL] : status[ST_BREAKDOWN];
    int v = 0;
    if (status[ST_TIMEOUT]) v = -100;
    else if (fp64) v = brk == INT_MAX ? 0 : brk;
    else if (status[ST_OVERFLOW]) v = -2;
    else if (brk != INT_MAX) v = -3;
    *info = v;
}

hipError_t launch_factor_info(const int *status, int chol, int fp64, int *info, hipStream_t s) {
    k_factor_info<<<dim3(1), dim3(64), 0, s>>>(status, chol, fp64, info);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, unsigned v, size_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_fill_u32<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(p, v, count);
    return hipGetLastError();
}

__global__ void k_fill_f64(double *p, double v, size_t count) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

hipError_t launch_fill_f64(double *p, double v, size_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_fill_f64<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(p, v, count);
    return hipGetLastError();
}

__global__ void k_iota(int *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = i;
}

hipError_t launch_iota(int *p, int count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    k_iota<<<dim3((count + 255) / 256), dim3(256), 0, s>>>(p, count);
    return hipGetLastError();
}

// rowmax[i] = max_j |a_ij|, rowsum[i] = sum_j |a_ij|; one wave per row.
__global__ __launch_bounds__(256) void k_row_stats(const double *__restrict__ A, int lda, int n,
                                                   double *__restrict__ rowmax,
                                                   double *__restrict__ rowsum) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const double *a = A + (size_t)row * lda;
    double mx = 0.0, sm = 0.0;
    for (int j = lane; j < n; j += 64) {
        double v = fabs(a[j]);
        mx = fmax(mx, v);
        sm += v;
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off));
        sm += __shfl_xor(sm, off);
    }
    if (lane == 0) {
        rowmax[row] = mx;
        rowsum[row] = sm;
    }
}

hipError_t launch_row_stats(const double *A, int lda, int n, double *rowmax, double *rowsum,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_row_stats<<<dim3((n + 3) / 4), dim3(256), 0, s>>>(A, lda, n, rowmax, rowsum);
    return hipGetLastError();
}

// Power of two p with p * v in [1, 2) (1 when v is 0 or not finite).
__device__ inline double pow2_scale(double v) {
    if (!(v > 0.0) || !isfinite(v)) return 1.0;
    int e;
    frexp(v, &e);  // v = f * 2^e, f in [0.5, 1)
    return ldexp(1.0, 1 - e);
}

// R_i (power-of-two row scales, 1 when equilibration is off or i >= n) and
// norms[0] = ||M||_inf = max_i rowsum_i.  One workgroup.
__global__ __launch_bounds__(1024) void k_finish_rows(int n, int npad,
                                                      const double *__restrict__ rowmax,
                                                      const double *__restrict__ rowsum,
                                                      double *__restrict__ R, int equil,
                                                      double *__restrict__ norms) {
    __shared__ double red[16];
    double best = 0.0;
    bool nan_seen = false;
    for (int i = threadIdx.x; i < npad; i += blockDim.x) {
        double r = 1.0;
        if (i < n) {
            double rs = rowsum[i];
            if (rs != rs) nan_seen = true;
            best = fmax(best, rs);
            if (equil) r = pow2_scale(rowmax[i]);
        }
        R[i] = r;
    }
    for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __shared__ int s_nan;
    if (threadIdx.x == 0) s_nan = 0;
    __syncthreads();
    if (nan_seen) s_nan = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) b = fmax(b, red[w]);
        norms[0] = s_nan ? __longlong_as_double(0x7ff8000000000000LL) : b;
    }
}

hipError_t launch_finish_rows(int n, int npad, const double *rowmax, const double *rowsum,
                              double *R, int equil, double *norms, hipStream_t s) {
    k_finish_rows<<<dim3(1), dim3(1024), 0, s>>>(n, npad, rowmax, rowsum, R, equil, norms);
    return hipGetLastError();
}

// Partial column statistics over a chunk of rows: colpart[0][chunk][j] =
// max_i R_i |a_ij| and colpart[1][chunk][j] = sum_i |a_ij| for the chunk.
__global__ __launch_bounds__(256) void k_col_part(const double *__restrict__ A, int lda, int n,
                                                  int npad, const double *__restrict__ R,
                                                  double *__restrict__ colpart) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int chunk = blockIdx.y;
    const int rows_per = (n + kColChunks - 1) / kColChunks;
    const int i0 = chunk * rows_per;
    const int i1 = min(n, i0 + rows_per);
    if (j >= npad) return;
    double mx = 0.0, sm = 0.0;
    if (j < n) {
        for (int i = i0; i < i1; ++i) {
            double v = fabs(A[(size_t)i * lda + j]);
            mx = fmax(mx, R[i] * v);
            sm += v;
        }
    }
    colpart[(size_t)chunk * npad + j] = mx;
    colpart[(size_t)(kColChunks + chunk) * npad + j] = sm;
}

constexpr int kMaxRpc = 512;  // rows per chunk of k_convert_stats (npad <= 64 * 512)

// Maximum of non-negative doubles (and NaN) by their bit patterns: for
// non-negative values the IEEE order is the order of the bits read as
// unsigned integers, and every NaN pattern lies above +inf, so a NaN
// anywhere wins.  *p starts at 0.
__device__ inline void atomic_max_bits(double *p, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(p),
              (unsigned long long)__double_as_longlong(v != v ? v : fabs(v)));
}

// C_j from the chunk maxima, and norms[1] = ||M||_1 = max_j sum_i |a_ij|
// (norms[1] zeroed by the caller): one thread per column.
__global__ __launch_bounds__(256) void k_col_finish(int n, int npad,
                                                    const double *__restrict__ colpart,
                                                    double *__restrict__ C, int equil,
                                                    double *__restrict__ norms) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    double sm = 0.0;
    if (j < npad) {
        double mx = 0.0;
        for (int c = 0; c < kColChunks; ++c) {
            mx = fmax(mx, colpart[(size_t)c * npad + j]);
            sm += colpart[(size_t)(kColChunks + c) * npad + j];
        }
        C[j] = (equil && j < n) ? pow2_scale(mx) : 1.0;
    }
    if (j >= n) sm = 0.0;
    // wave maximum (NaN wins), then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(sm, off);
        sm = (o > sm || o != o) ? o : sm;
    }
    if ((threadIdx.x & 63) == 0) atomic_max_bits(&norms[1], sm);
}

hipError_t launch_col_stats(const double *A, int lda, int n, int npad, const double *R,
                            double *colpart, double *C, int equil, double *norms,
                            hipStream_t s) {
    k_col_part<<<dim3((npad + 255) / 256, kColChunks), dim3(256), 0, s>>>(A, lda, n, npad, R,
                                                                          colpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_fill_f64(norms + 1, 0.0, 1, s);
    if (e != hipSuccess) return e;
    k_col_finish<<<dim3((npad + 255) / 256), dim3(256), 0, s>>>(n, npad, colpart, C, equil, norms);
    return hipGetLastError();
}

// Without equilibration (R = C = 1): the conversion and both norms in one
// pass over A.  Workgroup (jb, c) converts rows [c rpc, (c + 1) rpc) (rpc <=
// kMaxRpc) of the 1024 columns [1024 jb, 1024 jb + 1024), four adjacent
// columns per thread; it leaves the column sums of its rows in colsum[c][j]
// and, per row, the sum over its 1024 columns in rowpart[jb][i] (each wave's
// share combined in LDS at the end).
template <typename Tw>
__global__ __launch_bounds__(256) void k_convert_stats(const double *__restrict__ A, int lda,
                                                       int n, int npad, int rpc,
                                                       Tw *__restrict__ W, int ldw,
                                                       double *__restrict__ colsum,
                                                       double *__restrict__ rowpart,
                                                       int *__restrict__ status) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j0 = blockIdx.x * 1024 + 4 * threadIdx.x;
    const int c = blockIdx.y;
    const int i0 = c * rpc, i1 = min(npad, i0 + rpc);
    __shared__ double s_rows[4][kMaxRpc];
    double cs[4] = {0.0, 0.0, 0.0, 0.0};
    int bad = 0;
    const bool vec = (j0 + 4 <= n) && (lda % 2 == 0) &&
                     ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
    for (int i = i0; i < i1; ++i) {
        double v[4];
        if (i < n && vec) {
            const double2 p = *reinterpret_cast<const double2 *>(A + (size_t)i * lda + j0);
            const double2 q = *reinterpret_cast<const double2 *>(A + (size_t)i * lda + j0 + 2);
            v[0] = p.x;
            v[1] = p.y;
            v[2] = q.x;
            v[3] = q.y;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (i < n && j0 + e < n) ? A[(size_t)i * lda + j0 + e] : 0.0;
        }
        double rs = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = j0 + e;
            if (j >= npad) continue;
            Tw w;
            if (i < n && j < n) {
                w = (Tw)v[e];
                if (!isfinite(w)) ++bad;
                const double av = fabs(v[e]);
                cs[e] += av;
                rs += av;
            } else {
                w = (Tw)(i == j ? 1.0 : 0.0);
            }
            W[(size_t)i * ldw + j] = w;
        }
        for (int off = 32; off > 0; off >>= 1) rs += __shfl_xor(rs, off);
        if (lane == 0) s_rows[wave][i - i0] = rs;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (j0 + e < npad) colsum[(size_t)c * npad + j0 + e] = cs[e];
    if (bad) atomicAdd(&status[ST_OVERFLOW], bad);
    __syncthreads();
    for (int r = threadIdx.x; r < i1 - i0; r += 256)
        rowpart[(size_t)blockIdx.x * npad + i0 + r] =
            (s_rows[0][r] + s_rows[1][r]) + (s_rows[2][r] + s_rows[3][r]);
}

// R = C = 1, norms[0] = max_i sum over the nq row parts, norms[1] = max_j
// sum over the chunk column sums (both zeroed by the caller).
__global__ __launch_bounds__(256) void k_stats_finish(int n, int npad, int nq, int nc,
                                                      const double *__restrict__ rowpart,
                                                      const double *__restrict__ colsum,
                                                      double *__restrict__ R,
                                                      double *__restrict__ C,
                                                      double *__restrict__ norms) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double rs = 0.0, cs = 0.0;
    if (i < npad) {
        R[i] = 1.0;
        C[i] = 1.0;
        if (i < n) {
            for (int q = 0; q < nq; ++q) rs += rowpart[(size_t)q * npad + i];
            for (int c = 0; c < nc; ++c) cs += colsum[(size_t)c * npad + i];
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(rs, off);
        rs = (o > rs || o != o) ? o : rs;
        const double p = __shfl_xor(cs, off);
        cs = (p > cs || p != p) ? p : cs;
    }
    if ((threadIdx.x & 63) == 0) {
        atomic_max_bits(&norms[0], rs);
        atomic_max_bits(&norms[1], cs);
    }
}

template <typename Tw>
hipError_t launch_convert_stats(const double *A, int lda, int n, int npad, Tw *W, int ldw,
                                double *tmp, double *R, double *C, double *norms, int *status,
                                hipStream_t s) {
    if (npad == 0) return hipSuccess;
    const int rpc = (npad + kColChunks - 1) / kColChunks;
    const int nc = (npad + rpc - 1) / rpc;
    const int njb = (npad + 1023) / 1024;
    const int nq = njb;
    if (rpc > kMaxRpc) return hipErrorInvalidValue;
    // tmp: colsum[nc][npad] then rowpart[nq][npad]
    if (nc + nq > 2 * kColChunks + 2) return hipErrorInvalidValue;
    double *colsum = tmp, *rowpart = tmp + (size_t)nc * npad;
    hipError_t e = launch_fill_f64(norms, 0.0, 2, s);
    if (e != hipSuccess) return e;
    k_convert_stats<Tw><<<dim3(njb, nc), dim3(256), 0, s>>>(A, lda, n, npad, rpc, W, ldw, colsum,
                                                            rowpart, status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_stats_finish<<<dim3((npad + 255) / 256), dim3(256), 0, s>>>(n, npad, nq, nc, rowpart, colsum,
                                                                 R, C, norms);
    return hipGetLastError();
}
template hipError_t launch_convert_stats<float>(const double *, int, int, int, float *, int,
                                                double *, double *, double *, double *, int *,
                                                hipStream_t);
template hipError_t launch_convert_stats<double>(const double *, int, int, int, double *, int,
                                                 double *, double *, double *, double *, int *,
                                                 hipStream_t);

// W = fl(R M C) for i, j < n; identity in the padding (i or j >= n).
// Non-finite results are counted in status[ST_OVERFLOW].
template <typename Tw>
__global__ __launch_bounds__(256) void k_convert(const double *__restrict__ A, int lda, int n,
                                                 int npad, const double *__restrict__ R,
                                                 const double *__restrict__ C, Tw *__restrict__ W,
                                                 int ldw, int *__restrict__ status) {
    const int i = blockIdx.x;
    const double ri = (i < n) ? R[i] : 1.0;
    int bad = 0;
    for (int j = threadIdx.x; j < npad; j += 256) {
        Tw w;
        if (i < n && j < n) {
            w = (Tw)(ri * A[(size_t)i * lda + j] * C[j]);
            if (!isfinite(w)) ++bad;
        } else {
            w = (Tw)(i == j ? 1.0 : 0.0);
        }
        W[(size_t)i * ldw + j] = w;
    }
    if (bad) atomicAdd(&status[ST_OVERFLOW], bad);
}

template <typename Tw>
hipError_t launch_convert(const double *A, int lda, int n, int npad, const double *R,
                          const double *C, Tw *W, int ldw, int *status, hipStream_t s) {
    if (npad == 0) return hipSuccess;
    k_convert<Tw><<<dim3(npad), dim3(256), 0, s>>>(A, lda, n, npad, R, C, W, ldw, status);
    return hipGetLastError();
}

template hipError_t launch_convert<float>(const double *, int, int, int, const double *,
                                          const double *, float *, int, int *, hipStream_t);
template hipError_t launch_convert<double>(const double *, int, int, int, const double *,
                                           const double *, double *, int, int *, hipStream_t);

}  // namespace mixlu
