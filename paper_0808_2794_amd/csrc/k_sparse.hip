// Kernels of the sparse inner-outer solver (Section 3.2, Algorithm 2:
// FGMRES(m_out) in double precision around GMRES(m_in) in single
// precision) on matrices in CRS storage.
//
//   k_csr_spmv      y = A x with the values in the inner precision (FP32
//                   copy for GMRES_SP) or in FP64; one thread per row (the
//                   stencil rows hold a few nonzeros)
//   k_csr_resid     r = b - A x in FP64, with ||r||_inf and ||x||_inf
//   k_csr_norm_inf  ||A||_inf
//   k_to_float      the FP32 copy of the values (and of vectors)
//   k_vdots(_fin)   h[j] = V_j . w for j < k (chunks over many workgroups,
//                   then the partial sums in a fixed order)
//   k_vcombine      w -= sum_j h[j] V_j  (one pass of Gram-Schmidt)
//   k_vscale        y = x / ||w||_2 (the squared norm from device memory)
//   k_vaxpy_basis   x += sum_j y[j] Z_j (the FGMRES update, FP64)
//   k_gmres_*       the small least-squares part of an inner GMRES cycle
//                   on the device (Givens rotations, stopping test, back
//                   substitution), so the cycle runs without the host
#include "common.h"

namespace mixlu {

template <typename TV>
__global__ __launch_bounds__(256) void k_csr_spmv(int n, const int *__restrict__ rowptr,
                                                  const int *__restrict__ colind,
                                                  const TV *__restrict__ vals,
                                                  const TV *__restrict__ x, TV *__restrict__ y) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    TV s = (TV)0;
    for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) s += vals[p] * x[colind[p]];
    y[i] = s;
}

__device__ __forceinline__ void amax_nonneg(double *p, double v) {
    // non-negative doubles order like their bit patterns as integers
    atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

__global__ __launch_bounds__(256) void k_csr_resid(int n, const int *__restrict__ rowptr,
                                                   const int *__restrict__ colind,
                                                   const double *__restrict__ vals,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ b,
                                                   double *__restrict__ r,
                                                   double *__restrict__ norms) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double ar = 0.0, ax = 0.0;
    if (i < n) {
        double s = 0.0;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) s += vals[p] * x[colind[p]];
        const double v = b[i] - s;
        r[i] = v;
        ar = fabs(v);
        ax = fabs(x[i]);
        if (ar != ar) ar = __longlong_as_double(0x7ff0000000000000LL);  // NaN -> +inf
        if (ax != ax) ax = __longlong_as_double(0x7ff0000000000000LL);
    }
    for (int off = 32; off > 0; off >>= 1) {
        ar = fmax(ar, __shfl_xor(ar, off));
        ax = fmax(ax, __shfl_xor(ax, off));
    }
    if ((threadIdx.x & 63) == 0) {
        amax_nonneg(&norms[0], ar);
        amax_nonneg(&norms[1], ax);
    }
}

// norms[0] = max over rows of sum |a_ij| (||A||_inf), by atomic maximum
__global__ __launch_bounds__(256) void k_csr_norm_inf(int n, const int *__restrict__ rowptr,
                                                      const double *__restrict__ vals,
                                                      double *__restrict__ norms) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double sum = 0.0;
    if (i < n)
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) sum += fabs(vals[p]);
    if (sum != sum) sum = __longlong_as_double(0x7ff0000000000000LL);
    for (int off = 32; off > 0; off >>= 1) sum = fmax(sum, __shfl_xor(sum, off));
    if ((threadIdx.x & 63) == 0) amax_nonneg(&norms[0], sum);
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_convert_vec(size_t n, const TS *__restrict__ x,
                                                     TD *__restrict__ y) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        y[i] = (TD)x[i];
}

// Dot products h[j] = V_j . w in two stages: workgroup (j, g) sums chunk g
// of the n entries into part[j * G + g]; k_vdots_fin adds the G partial
// sums of each j in a fixed order (so the result does not depend on
// scheduling).
template <typename T>
__global__ __launch_bounds__(256) void k_vdots(int n, int k, const T *__restrict__ V, size_t ldv,
                                               const T *__restrict__ w, T *__restrict__ part) {
    const int j = blockIdx.x, g = blockIdx.y, G = gridDim.y;
    if (j >= k) return;
    const int chunk = (n + G - 1) / G;
    const int i0 = g * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
    const T *v = V + (size_t)j * ldv;
    T s = (T)0;
    for (int i = i0 + threadIdx.x; i < i1; i += 256) s += v[i] * w[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    __shared__ T red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[(size_t)j * G + g] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T>
__global__ __launch_bounds__(64) void k_vdots_fin(int k, int G, const T *__restrict__ part,
                                                  T *__restrict__ h) {
    const int j = blockIdx.x;
    if (j >= k) return;
    T s = (T)0;
    for (int g = threadIdx.x; g < G; g += 64) s += part[(size_t)j * G + g];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (threadIdx.x == 0) h[j] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_vcombine(int n, int k, const T *__restrict__ V,
                                                  size_t ldv, const T *__restrict__ h,
                                                  T *__restrict__ w) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    T s = w[i];
    for (int j = 0; j < k; ++j) s -= h[j] * V[(size_t)j * ldv + i];
    w[i] = s;
}

// y = x / sqrt(*sq) (sq on the device: the squared norm just computed)
template <typename T>
__global__ __launch_bounds__(256) void k_vscale(int n, const T *__restrict__ x,
                                                const T *__restrict__ sq, T *__restrict__ y) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = x[i] / sqrt(sq[0]);
}

// x += sum_{j < k} y[j] Z_j, y in device memory; kdev (optional): the
// number of terms is min(k, kdev[1]) (the steps an inner cycle took)
template <typename TZ, typename TX>
__global__ __launch_bounds__(256) void k_vaxpy_basis(int n, int k, const TZ *__restrict__ Z,
                                                     size_t ldz, const double *__restrict__ y,
                                                     TX *__restrict__ x,
                                                     const int *__restrict__ kdev) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int kk = kdev && kdev[1] < k ? kdev[1] : k;
    double s = 0.0;
    for (int j = 0; j < kk; ++j) s += y[j] * (double)Z[(size_t)j * ldz + i];
    x[i] = (TX)((double)x[i] + s);
}

// Inner GMRES(m) least-squares state in G (doubles): H ((m + 1) x m,
// row-major), cs[m], sn[m], g[m + 1], beta; st[0] = 1 while the cycle
// runs, st[1] = steps taken.  One thread does the O(m) work of a step.
__device__ __forceinline__ double *gm_H(double *G) { return G; }
__device__ __forceinline__ size_t gm_cs(int m) { return (size_t)(m + 1) * m; }
template <typename T>
__global__ void k_gmres_init(const T *__restrict__ hn, double *__restrict__ G, int m,
                             int *__restrict__ st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double beta = sqrt((double)hn[0]);
    const size_t cs = gm_cs(m), sn = cs + m, g = sn + m, b = g + m + 1;
    for (size_t i = 0; i < b; ++i) G[i] = 0.0;
    G[g] = beta;
    G[b] = beta;
    st[0] = beta > 0.0 ? 1 : 0;
    st[1] = 0;
}
// step j: column j of H from the two Gram-Schmidt passes h[0..j] and
// h[j+1..2j+1] and the squared norm h[2j+2] of the new vector; the earlier
// rotations, a new one, g; the cycle ends when the new vector vanishes or
// the rotated residual |g[j+1]| falls to eps_rel beta
template <typename T>
__global__ void k_gmres_col(const T *__restrict__ h, double *__restrict__ G, int m, int j,
                            double eps_rel, int *__restrict__ st) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || st[0] == 0) return;
    const int k = j + 1;
    double *H = gm_H(G);
    double *cs = G + gm_cs(m), *sn = cs + m, *g = sn + m;
    const double beta = g[m + 1];
    for (int i = 0; i < k; ++i) H[(size_t)i * m + j] = (double)h[i] + (double)h[k + i];
    const double wn = sqrt((double)h[2 * k]);
    H[(size_t)k * m + j] = wn;
    for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], b2 = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * b2;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b2;
    }
    const double a = H[(size_t)j * m + j], b2 = H[(size_t)k * m + j];
    double c = 1.0, sv = 0.0;
    if (b2 != 0.0) {
        const double r = hypot(a, b2);
        c = a / r;
        sv = b2 / r;
    }
    cs[j] = c;
    sn[j] = sv;
    H[(size_t)j * m + j] = c * a + sv * b2;
    H[(size_t)k * m + j] = 0.0;
    g[k] = -sv * g[j];
    g[j] = c * g[j];
    st[1] = k;
    if (!(wn > 0.0) || fabs(g[k]) <= eps_rel * beta || k == m) st[0] = 0;
}
// y solving the st[1] x st[1] upper triangle of the rotated H against g
__global__ void k_gmres_backsub(const double *__restrict__ G, int m, const int *__restrict__ st,
                                double *__restrict__ y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double *H = G;
    const double *g = G + gm_cs(m) + 2 * (size_t)m;
    const int k = st[1];
    for (int i = k - 1; i >= 0; --i) {
        double sacc = g[i];
        for (int q = i + 1; q < k; ++q) sacc -= H[(size_t)i * m + q] * y[q];
        y[i] = sacc / H[(size_t)i * m + i];
    }
}

// ------------------------------------------------------------ launchers
static unsigned blocks_of(size_t n) { return (unsigned)((n + 255) / 256); }

template <typename TV>
hipError_t launch_csr_spmv(int n, const int *rowptr, const int *colind, const TV *vals, const TV *x,
                           TV *y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_csr_spmv<TV><<<blocks_of(n), 256, 0, s>>>(n, rowptr, colind, vals, x, y);
    return hipGetLastError();
}
hipError_t launch_csr_resid(int n, const int *rowptr, const int *colind, const double *vals,
                            const double *x, const double *b, double *r, double *norms,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_csr_resid<<<blocks_of(n), 256, 0, s>>>(n, rowptr, colind, vals, x, b, r, norms);
    return hipGetLastError();
}
hipError_t launch_csr_norm_inf(int n, const int *rowptr, const double *vals, double *norms,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_csr_norm_inf<<<blocks_of(n), 256, 0, s>>>(n, rowptr, vals, norms);
    return hipGetLastError();
}
template <typename TS, typename TD>
hipError_t launch_convert_vec(size_t n, const TS *x, TD *y, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned g = blocks_of(n) < 4096 ? blocks_of(n) : 4096;
    k_convert_vec<TS, TD><<<g, 256, 0, s>>>(n, x, y);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_vdots(int n, int k, const T *V, size_t ldv, const T *w, T *h, T *part,
                        hipStream_t s) {
    if (k <= 0) return hipSuccess;
    // about 4096 entries per workgroup, at most kVdotsChunks chunks
    int G = (n + 4095) / 4096;
    if (G < 1) G = 1;
    if (G > kVdotsChunks) G = kVdotsChunks;
    k_vdots<T><<<dim3(k, G), 256, 0, s>>>(n, k, V, ldv, w, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_vdots_fin<T><<<k, 64, 0, s>>>(k, G, part, h);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_vcombine(int n, int k, const T *V, size_t ldv, const T *h, T *w, hipStream_t s) {
    if (n <= 0 || k <= 0) return hipSuccess;
    k_vcombine<T><<<blocks_of(n), 256, 0, s>>>(n, k, V, ldv, h, w);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_vscale(int n, const T *x, const T *den, T *y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_vscale<T><<<blocks_of(n), 256, 0, s>>>(n, x, den, y);
    return hipGetLastError();
}
template <typename TZ, typename TX>
hipError_t launch_vaxpy_basis(int n, int k, const TZ *Z, size_t ldz, const double *y, TX *x,
                              hipStream_t s, const int *kdev) {
    if (n <= 0 || k <= 0) return hipSuccess;
    k_vaxpy_basis<TZ, TX><<<blocks_of(n), 256, 0, s>>>(n, k, Z, ldz, y, x, kdev);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_gmres_init(const T *hn, double *G, int m, int *st, hipStream_t s) {
    k_gmres_init<T><<<1, 64, 0, s>>>(hn, G, m, st);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_gmres_col(const T *h, double *G, int m, int j, double eps_rel, int *st,
                            hipStream_t s) {
    k_gmres_col<T><<<1, 64, 0, s>>>(h, G, m, j, eps_rel, st);
    return hipGetLastError();
}
hipError_t launch_gmres_backsub(const double *G, int m, const int *st, double *y, hipStream_t s) {
    k_gmres_backsub<<<1, 64, 0, s>>>(G, m, st, y);
    return hipGetLastError();
}
template hipError_t launch_gmres_init<float>(const float *, double *, int, int *, hipStream_t);
template hipError_t launch_gmres_init<double>(const double *, double *, int, int *, hipStream_t);
template hipError_t launch_gmres_col<float>(const float *, double *, int, int, double, int *,
                                            hipStream_t);
template hipError_t launch_gmres_col<double>(const double *, double *, int, int, double, int *,
                                             hipStream_t);

template hipError_t launch_csr_spmv<float>(int, const int *, const int *, const float *,
                                           const float *, float *, hipStream_t);
template hipError_t launch_csr_spmv<double>(int, const int *, const int *, const double *,
                                            const double *, double *, hipStream_t);
template hipError_t launch_convert_vec<double, float>(size_t, const double *, float *, hipStream_t);
template hipError_t launch_convert_vec<float, double>(size_t, const float *, double *, hipStream_t);
template hipError_t launch_convert_vec<double, double>(size_t, const double *, double *,
                                                       hipStream_t);
template hipError_t launch_vdots<float>(int, int, const float *, size_t, const float *, float *,
                                        float *, hipStream_t);
template hipError_t launch_vdots<double>(int, int, const double *, size_t, const double *,
                                         double *, double *, hipStream_t);
template hipError_t launch_vcombine<float>(int, int, const float *, size_t, const float *,
                                           float *, hipStream_t);
template hipError_t launch_vcombine<double>(int, int, const double *, size_t, const double *,
                                            double *, hipStream_t);
template hipError_t launch_vscale<float>(int, const float *, const float *, float *, hipStream_t);
template hipError_t launch_vscale<double>(int, const double *, const double *, double *,
                                          hipStream_t);
template hipError_t launch_vaxpy_basis<float, double>(int, int, const float *, size_t,
                                                      const double *, double *, hipStream_t,
                                                      const int *);
template hipError_t launch_vaxpy_basis<double, double>(int, int, const double *, size_t,
                                                       const double *, double *, hipStream_t,
                                                       const int *);

}  // namespace mixlu
