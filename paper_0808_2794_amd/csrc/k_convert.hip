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

// C_j from the chunk maxima, and norms[1] = ||M||_1 = max_j sum_i |a_ij|.
__global__ __launch_bounds__(1024) void k_col_finish(int n, int npad,
                                                     const double *__restrict__ colpart,
                                                     double *__restrict__ C, int equil,
                                                     double *__restrict__ norms) {
    __shared__ double red[16];
    double best = 0.0;
    bool nan_seen = false;
    for (int j = threadIdx.x; j < npad; j += blockDim.x) {
        double mx = 0.0, sm = 0.0;
        for (int c = 0; c < kColChunks; ++c) {
            mx = fmax(mx, colpart[(size_t)c * npad + j]);
            sm += colpart[(size_t)(kColChunks + c) * npad + j];
        }
        if (j < n) {
            if (sm != sm) nan_seen = true;
            best = fmax(best, sm);
        }
        C[j] = (equil && j < n) ? pow2_scale(mx) : 1.0;
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
        norms[1] = s_nan ? __longlong_as_double(0x7ff8000000000000LL) : b;
    }
}

hipError_t launch_col_stats(const double *A, int lda, int n, int npad, const double *R,
                            double *colpart, double *C, int equil, double *norms,
                            hipStream_t s) {
    k_col_part<<<dim3((npad + 255) / 256, kColChunks), dim3(256), 0, s>>>(A, lda, n, npad, R,
                                                                          colpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_col_finish<<<dim3(1), dim3(1024), 0, s>>>(n, npad, colpart, C, equil, norms);
    return hipGetLastError();
}

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
