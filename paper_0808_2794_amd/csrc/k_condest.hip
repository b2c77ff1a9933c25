// Condition-number estimate for the choice between the low-precision path
// and the FP64 solver (Section 4: refinement with a factor of precision
// eps_s converges only while kappa(A) eps_s stays below about one).  The
// estimate of ||A^{-1}||_1 is Hager's method as refined by Higham (the
// scheme of LAPACK's xGECON): solves with A and A^T by the stored factors,
// and the reductions below between them.  Each kernel is one workgroup
// sweeping the n-vector (n is at most a few tens of thousands).
#include <climits>

#include "common.h"

namespace mixlu {

namespace {
constexpr int kCT = 1024;  // threads

__device__ __forceinline__ double block_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < kCT / 64; ++q) s += red[q];
    __syncthreads();
    return s;
}
}  // namespace

// x_i = 1/n (start vector), or Higham's alternating vector
// x_i = (-1)^i (1 + i/(n-1)) when alt.
__global__ __launch_bounds__(kCT) void k_cond_start(double *__restrict__ x, int n, int alt) {
    for (int i = threadIdx.x; i < n; i += kCT) {
        if (!alt) x[i] = 1.0 / n;
        else x[i] = (i & 1 ? -1.0 : 1.0) * (1.0 + (n > 1 ? (double)i / (n - 1) : 0.0));
    }
}

// out[0] = ||y||_1; xi = sign(y) (sign(0) = +1).
__global__ __launch_bounds__(kCT) void k_cond_sign(const double *__restrict__ y, int n,
                                                   double *__restrict__ xi,
                                                   double *__restrict__ out) {
    __shared__ double red[kCT / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kCT) {
        const double v = y[i];
        s += fabs(v);
        xi[i] = v >= 0.0 ? 1.0 : -1.0;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[0] = s;
}

// out[1] = ||z||_inf, out[2] = z^T x, out[3] = first index j of the largest
// |z_j|; then x = e_j.
__global__ __launch_bounds__(kCT) void k_cond_test(const double *__restrict__ z,
                                                   double *__restrict__ x, int n,
                                                   double *__restrict__ out) {
    __shared__ double red[kCT / 64];
    __shared__ double bv[kCT / 64];
    __shared__ int bi[kCT / 64];
    __shared__ int jsel;
    double dot = 0.0, best = -1.0;
    int bj = INT_MAX;
    for (int i = threadIdx.x; i < n; i += kCT) {
        const double v = z[i];
        dot += v * x[i];
        const double a = fabs(v);
        if (a > best) {  // i increases per thread: keeps the first index
            best = a;
            bj = i;
        }
    }
    dot = block_sum(dot, red);
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oj = __shfl_xor(bj, off);
        if (ob > best || (ob == best && oj < bj)) {
            best = ob;
            bj = oj;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        bv[wave] = best;
        bi[wave] = bj;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = -1.0;
        int j = INT_MAX;
        for (int q = 0; q < kCT / 64; ++q)
            if (bv[q] > b || (bv[q] == b && bi[q] < j)) {
                b = bv[q];
                j = bi[q];
            }
        if (j == INT_MAX) j = 0;
        out[1] = b;
        out[2] = dot;
        out[3] = (double)j;
        jsel = j;
    }
    __syncthreads();
    const int j = jsel;
    for (int i = threadIdx.x; i < n; i += kCT) x[i] = i == j ? 1.0 : 0.0;
}

hipError_t launch_cond_start(double *x, int n, int alt, hipStream_t s) {
    k_cond_start<<<1, kCT, 0, s>>>(x, n, alt);
    return hipGetLastError();
}
hipError_t launch_cond_sign(const double *y, int n, double *xi, double *out, hipStream_t s) {
    k_cond_sign<<<1, kCT, 0, s>>>(y, n, xi, out);
    return hipGetLastError();
}
hipError_t launch_cond_test(const double *z, double *x, int n, double *out, hipStream_t s) {
    k_cond_test<<<1, kCT, 0, s>>>(z, x, n, out);
    return hipGetLastError();
}

}  // namespace mixlu
