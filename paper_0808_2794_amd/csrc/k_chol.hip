// Cholesky variant of step 1 of Algorithm 1 for symmetric positive definite A
// (the SPOTRF / SPOTRS pair that replaces SGETRF / SGETRS in Section 3.1.1).
//
//   k_sym_scale   symmetric power-of-two scaling s_i from the diagonal, so
//                 that W = S A S stays symmetric with diagonal in [1, 4)
//   k_chol_panel  one 64-column step of the right-looking factorization:
//                 the 64 x 64 diagonal block L11 is factored by one wave
//                 with the rows in registers, then every row below solves
//                 x L11^T = a (L21 = A21 L11^{-T}) with L11 in LDS
//   k_chol_to_lu  rewrites L L^T as the unit-lower / upper pair L' U' with
//                 L' = L D^{-1}, U' = D L^T (D = diag(L)), so that the LU
//                 solve and refinement kernels serve both factorizations
//
// The symmetric trailing update A22 -= L21 L21^T runs on the GEMM kernels of
// k_lu.hip restricted to the lower triangle.
#include <climits>

#include "common.h"

namespace mixlu {

// s_i = 2^-floor(log2(a_ii) / 2): s_i^2 a_ii lies in [1, 4).  A diagonal
// entry that is not positive and finite keeps s_i = 1 (the factorization
// then breaks down and reports it).  Padding rows get 1.
__global__ __launch_bounds__(256) void k_sym_scale(const double *__restrict__ A, int lda, int n,
                                                   int npad, double *__restrict__ R,
                                                   double *__restrict__ C, int equil) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    double s = 1.0;
    if (equil && i < n) {
        const double d = A[(size_t)i * lda + i];
        if (d > 0.0 && d <= 1.79769313486231570815e308) {
            const int e = ilogb(d);
            s = ldexp(1.0, -(e >> 1));  // arithmetic shift: floor(e / 2)
        }
    }
    R[i] = s;
    C[i] = s;
}

hipError_t launch_sym_scale(const double *A, int lda, int n, int npad, double *R, double *C,
                            int equil, hipStream_t s) {
    if (npad <= 0) return hipSuccess;
    k_sym_scale<<<dim3((npad + 255) / 256), dim3(256), 0, s>>>(A, lda, n, npad, R, C, equil);
    return hipGetLastError();
}

// One 64-column step at diagonal position k of the npad x npad row-major W
// (lower triangle holds the partially updated matrix).  Every workgroup
// factors the diagonal block in its first wave (so no workgroup waits on
// another); workgroup 0 stores L11 and its diagonal.  Workgroup b then
// solves rows k + 64 + 256 b + tid (< k + 64 + below) for L21.
template <typename T>
__global__ __launch_bounds__(256) void k_chol_panel(T *__restrict__ W, int ld, int k, int below,
                                                    T *__restrict__ diag,
                                                    int *__restrict__ status) {
    constexpr int NB = 64, P = NB + 16 / (int)sizeof(T);  // LDS pitch keeps rows 16-byte aligned
    typedef typename Vq<T>::type vec_t;
    constexpr int V = Vq<T>::V, NQ = NB / V;
    __shared__ __attribute__((aligned(16))) T sL[NB * P];
    __shared__ T sRinv[NB];
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid < 64) {
        T a[NB];
        {
            const vec_t *src = reinterpret_cast<const vec_t *>(W + (size_t)(k + lane) * ld + k);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const vec_t v = src[q];
#pragma unroll
                for (int e = 0; e < V; ++e) a[q * V + e] = v[e];
            }
        }
        int bad = INT_MAX;
        sfor<0, NB>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const T ajj = readlane_t(a[j], j);
            if (!(ajj > (T)0) || !(ajj < (T)INFINITY)) bad = bad < j ? bad : j;
            const T d = sqrt(ajj);
            const T rinv = (T)1 / d;
            const T l = lane > j ? a[j] * rinv : (T)0;
            a[j] = lane == j ? d : (lane > j ? l : a[j]);
            sfor<j + 1, NB>([&](auto Cc) {
                constexpr int c = decltype(Cc)::value;
                a[c] -= l * readlane_t(l, c);
            });
        });
        // row `lane` of L11 (entries right of the diagonal are not used)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            vec_t v;
#pragma unroll
            for (int e = 0; e < V; ++e) v[e] = a[q * V + e];
            *reinterpret_cast<vec_t *>(&sL[lane * P + q * V]) = v;
        }
        T dl = a[0];
#pragma unroll
        for (int c = 1; c < NB; ++c) dl = lane == c ? a[c] : dl;
        sRinv[lane] = (T)1 / dl;
        if (blockIdx.x == 0) {
            T *dst = W + (size_t)(k + lane) * ld + k;
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c <= lane) dst[c] = a[c];
            diag[k + lane] = dl;
            if (lane == 0 && bad != INT_MAX) atomicMin(&status[ST_CHOL], k + bad + 1);
        }
    }
    __syncthreads();
    const int r = k + NB + blockIdx.x * 256 + tid;
    if (r >= k + NB + below) return;
    T x[NB];
    vec_t *row = reinterpret_cast<vec_t *>(W + (size_t)r * ld + k);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const vec_t v = row[q];
#pragma unroll
        for (int e = 0; e < V; ++e) x[q * V + e] = v[e];
    }
    // x_c = (a_c - sum_{t<c} x_t L11[c][t]) / L11[c][c]
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        T acc = x[c];
#pragma unroll
        for (int t = 0; t < c; ++t) acc -= x[t] * sL[c * P + t];
        x[c] = acc * sRinv[c];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        vec_t v;
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = x[q * V + e];
        row[q] = v;
    }
}

template <typename T>
hipError_t launch_chol_panel(T *W, int ldw, int k, int below, T *diag, int *status,
                             hipStream_t s) {
    if (below < 0) return hipErrorInvalidValue;
    const int grid = below > 0 ? (below + 255) / 256 : 1;
    k_chol_panel<T><<<dim3(grid), dim3(256), 0, s>>>(W, ldw, k, below, diag, status);
    return hipGetLastError();
}
template hipError_t launch_chol_panel<float>(float *, int, int, int, float *, int *, hipStream_t);
template hipError_t launch_chol_panel<double>(double *, int, int, int, double *, int *,
                                              hipStream_t);

// L L^T -> L' U': for each lower 64 x 64 tile (I, J), I >= J, write
// L'[i][j] = L[i][j] / d_j below the diagonal and U'[j][i] = d_j L[i][j] in
// the mirrored tile (J, I); U'[i][i] = d_i^2.  d comes from the separate
// diagonal vector because the diagonal tiles are overwritten.
template <typename T>
__global__ __launch_bounds__(256) void k_chol_to_lu(T *__restrict__ W, int ld,
                                                    const T *__restrict__ diag) {
    const int I = blockIdx.y, J = blockIdx.x;
    if (J > I) return;
    __shared__ T t[64][65];
    __shared__ T sd[64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const size_t r0 = (size_t)I * 64, c0 = (size_t)J * 64;
    if (threadIdx.x < 64) sd[tx] = diag[c0 + tx];
    for (int i = ty; i < 64; i += 4) t[i][tx] = W[(r0 + i) * ld + c0 + tx];
    __syncthreads();
    if (I > J) {
        for (int i = ty; i < 64; i += 4) W[(r0 + i) * ld + c0 + tx] = t[i][tx] / sd[tx];
        // U'[c0 + i][r0 + tx] = d_{c0+i} L[r0 + tx][c0 + i]
        for (int i = ty; i < 64; i += 4) W[(c0 + i) * ld + r0 + tx] = sd[i] * t[tx][i];
    } else {
        for (int i = ty; i < 64; i += 4) {
            T v;
            if (i > tx) v = t[i][tx] / sd[tx];      // L' below the diagonal
            else v = sd[i] * t[tx][i];              // U'[i][tx] = d_i L[tx][i], tx >= i
            W[(r0 + i) * ld + c0 + tx] = v;
        }
    }
}

template <typename T>
hipError_t launch_chol_to_lu(T *W, int ldw, int npad, const T *diag, hipStream_t s) {
    if (npad <= 0 || npad % 64) return hipErrorInvalidValue;
    const int nt = npad / 64;
    k_chol_to_lu<T><<<dim3(nt, nt), dim3(256), 0, s>>>(W, ldw, diag);
    return hipGetLastError();
}
template hipError_t launch_chol_to_lu<float>(float *, int, int, const float *, hipStream_t);
template hipError_t launch_chol_to_lu<double>(double *, int, int, const double *, hipStream_t);

}  // namespace mixlu
