// Triangular solves and FP64 refinement kernels: Algorithm 1 steps 2-3 and
// 5-6 (Ly = Pr, Uz = y in the factor's precision, the SGETRS of
// Section 3.1.1), step 4 (r = b - A x in FP64 with the original A, the
// DGEMM/DGEMV) and step 7 (x = x + z in FP64, the DAXPY), plus the norms of
// the stopping test of Section 3 and the outer product of the adjoint.
//
// The triangular solves are single launches over 64-row blocks: a block
// takes a ticket (so blocks start in order), accumulates the off-diagonal
// products as the solution blocks above it are published, solves its
// diagonal block in one wave, and publishes its 64 values as tagged words.
#include <climits>

#include "common.h"

namespace mixlu {

template <typename T> __device__ inline T bcast_lane(T v, int k);
template <> __device__ inline float bcast_lane<float>(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
template <> __device__ inline double bcast_lane<double>(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ inline void atomic_max_nonneg(double *p, double v) {
    // non-negative doubles (and +NaN) order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

// Y[i][c] = round(S[src] * B[src][c]) with src = perm[i] (perm = NULL: the
// identity) for rows that map into A, 0 for padding rows: the permuted,
// scaled right-hand side P(R b) of the solve with A, or C b for A^T.
template <typename Tw>
__global__ __launch_bounds__(256) void k_rhs_gather(int n, int npad, int nrhs,
                                                    const double *__restrict__ B, int ldb,
                                                    int b_col_major, const int *__restrict__ perm,
                                                    const double *__restrict__ R,
                                                    Tw *__restrict__ Y, int ldy) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= npad) return;
    const int src = perm ? perm[i] : i;
    for (int c = 0; c < nrhs; ++c) {
        Tw v = (Tw)0;
        if (src < n) {
            const double b = b_col_major ? B[src + (size_t)c * ldb] : B[(size_t)src * ldb + c];
            v = (Tw)(R[src] * b);
        }
        Y[(size_t)i * ldy + c] = v;
    }
}

template <typename Tw>
hipError_t launch_rhs_gather(int n, int npad, int nrhs, const double *B, int ldb, int b_col_major,
                             const int *perm, const double *R, Tw *Y, int ldy, hipStream_t s) {
    if (npad == 0 || nrhs == 0) return hipSuccess;
    k_rhs_gather<Tw><<<dim3((npad + 255) / 256), dim3(256), 0, s>>>(n, npad, nrhs, B, ldb,
                                                                    b_col_major, perm, R, Y, ldy);
    return hipGetLastError();
}
template hipError_t launch_rhs_gather<float>(int, int, int, const double *, int, int, const int *,
                                             const double *, float *, int, hipStream_t);
template hipError_t launch_rhs_gather<double>(int, int, int, const double *, int, int,
                                              const int *, const double *, double *, int,
                                              hipStream_t);

// Inverses of the 64 x 64 diagonal blocks of the factors stored in W
// (npad x npad, ld = ldw): block b of the unit lower L (blockIdx.y = 0) into
// dinv[b * 64 * 64 ..], of the upper U (blockIdx.y = 1) into
// dinv[(npad + b * 64) * 64 ..], row-major 64 x 64.  One wave per block;
// lane c forms column c of the inverse by substitution against the block
// staged in LDS (rows read with broadcast loads).
template <typename T>
__global__ __launch_bounds__(64) void k_tri_inv(const T *__restrict__ W, int ldw, int npad,
                                                T *__restrict__ dinv) {
    constexpr int BS = kTrsvBS;
    __shared__ __attribute__((aligned(16))) T sM[BS][BS];
    const int b = blockIdx.x, upper = blockIdx.y, lane = threadIdx.x;
    for (int r = 0; r < BS; ++r) sM[r][lane] = W[(size_t)(b * BS + r) * ldw + b * BS + lane];
    __syncthreads();
    T x[BS];
    if (!upper) {  // L x = e_c: x_i = [i = c] - sum_{k < i} l_ik x_k
#pragma unroll
        for (int i = 0; i < BS; ++i) {
            T v = (i == lane) ? (T)1 : (T)0;
#pragma unroll
            for (int k = 0; k < i; ++k) v -= sM[i][k] * x[k];
            x[i] = v;
        }
    } else {  // U x = e_c: x_i = ([i = c] - sum_{k > i} u_ik x_k) / u_ii
#pragma unroll
        for (int i = BS - 1; i >= 0; --i) {
            T v = (i == lane) ? (T)1 : (T)0;
#pragma unroll
            for (int k = i + 1; k < BS; ++k) v -= sM[i][k] * x[k];
            x[i] = v / sM[i][i];
        }
    }
    T *out = dinv + ((size_t)upper * npad + (size_t)b * BS) * BS;
#pragma unroll
    for (int r = 0; r < BS; ++r) out[r * BS + lane] = x[r];
}

template <typename T>
hipError_t launch_tri_inv(const T *W, int ldw, int npad, T *dinv, hipStream_t s) {
    if (npad == 0) return hipSuccess;
    if (npad % kTrsvBS) return hipErrorInvalidValue;
    k_tri_inv<T><<<dim3(npad / kTrsvBS, 2), dim3(64), 0, s>>>(W, ldw, npad, dinv);
    return hipGetLastError();
}
template hipError_t launch_tri_inv<float>(const float *, int, int, float *, hipStream_t);
template hipError_t launch_tri_inv<double>(const double *, int, int, double *, hipStream_t);

// Chained block triangular solve, in place in Y (npad x nrhs, ldy), nrhs <=
// NRT.  TRANS = false: upper = 0 solves with the unit lower L (below the
// diagonal of W), forward; upper = 1 with U (on and above the diagonal),
// backward.  TRANS = true solves with the transposed factors: upper = 0
// with U^T (lower, non-unit), forward; upper = 1 with L^T (upper, unit),
// backward.  Workgroup o (in ticket order) takes the blocks at chain
// positions 2o and 2o + 1, one per half (256 threads each): both halves
// accumulate the products of their block rows with the solved blocks as
// they are published (tile rows requested a few steps ahead), then the first
// block is finished by applying the inverse of its diagonal block (from
// k_tri_inv: dinv, 2 npad x 64) as a 64 x 64 product, and the second takes
// the first's solution from LDS instead of waiting for its publication, so
// one cross-workgroup hand-off serves two blocks.  yx holds the published
// solution words ((row * NRT + c) * PWV + word), zeroed before the launch
// together with the ticket counter at yx[npad * NRT * PWV].
template <typename T, int NRT, bool TRANS>
__global__ __launch_bounds__(512) void k_trsv(int upper, const T *__restrict__ W, int ldw,
                                              const T *__restrict__ dinv, int nblk,
                                              T *__restrict__ Y, int ldy, int nrhs,
                                              unsigned long long *__restrict__ yx,
                                              int *__restrict__ status) {
    constexpr int BS = kTrsvBS, PWV = Words<T>::n;
    constexpr int NWMAX = BS * NRT * PWV;          // words of one solution block
    constexpr int WPT = (NWMAX + 511) / 512;       // words per thread
    __shared__ unsigned swords[2][NWMAX];
    __shared__ T sy[2][BS][NRT];                   // each half's right-hand side
    __shared__ T sfirst[BS][NRT];                  // the first block's solution
    __shared__ int s_b, s_bad;
    const int tid = threadIdx.x, h = tid >> 8, t = tid & 255;
    const int npairs = (nblk + 1) / 2;
    int *ticket = reinterpret_cast<int *>(yx + (size_t)nblk * BS * NRT * PWV);
    if (tid == 0) {
        s_b = atomicAdd(ticket, 1);
        s_bad = 0;
    }
    __syncthreads();
    const int order = s_b;
    if (order >= npairs) return;
    const int i0 = 2 * order, i1 = i0 + 1;  // chain positions of the pair
    const bool has1 = i1 < nblk;
    const bool mine = h == 0 || has1;       // this half has a block (uniform per wave)
    const int cpos = h == 0 ? i0 : (has1 ? i1 : i0);
    const int b = upper ? nblk - 1 - cpos : cpos;
    const int r = t >> 2, q = t & 3;  // row of the block, quarter of the k range
    const int wblk = BS * nrhs * PWV;  // words of one solution block

    T acc[NRT];
#pragma unroll
    for (int c = 0; c < NRT; ++c) acc[c] = (T)0;
    // element (b*BS + r, jb*BS + q*16 + e) of the triangular matrix
    auto tile_ptr = [&](int jb) -> const T * {
        return TRANS ? W + (size_t)(jb * BS + q * 16) * ldw + (size_t)b * BS + r
                     : W + (size_t)(b * BS + r) * ldw + (size_t)jb * BS + q * 16;
    };
    const size_t estride = TRANS ? (size_t)ldw : (size_t)1;
    // row r, columns q*16 .. q*16+15 of the inverse diagonal block, requested
    // now (it does not depend on anything): inv(L) or inv(U), transposed for
    // the transposed solves (inv(U^T) = inv(U)^T)
    T dg[16];
    {
        const bool inv_u = (upper != 0) != TRANS;  // U (not transposed) or U^T
        const T *dblk = dinv + ((size_t)(inv_u ? nblk : 0) * BS + (size_t)b * BS) * BS;
#pragma unroll
        for (int e = 0; e < 16; ++e)
            dg[e] = TRANS ? dblk[(q * 16 + e) * BS + r] : dblk[r * BS + q * 16 + e];
    }
    // the second block's tile against the first (on the pair's own critical
    // path), requested now as well
    T lx[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) lx[e] = (T)0;
    if (h == 1 && has1) {
        const T *lrow = tile_ptr(upper ? nblk - 1 - i0 : i0);
#pragma unroll
        for (int e = 0; e < 16; ++e) lx[e] = TRANS ? lrow[e * estride] : lrow[e];
    }

    const int nsteps = i0;  // blocks before the pair, in chain order
    // tile rows of the next PF steps are requested ahead (they depend on
    // nothing), so a step costs the wait for its solution block, not a
    // memory latency of its own
    constexpr int PF = sizeof(T) == 4 ? kTrsvPrefetch : 2;
    T lv[PF][16];
    auto request = [&](int st, T(&dst)[16]) {
        if (mine && st < nsteps) {
            const T *lrow = tile_ptr(upper ? nblk - 1 - st : st);
#pragma unroll
            for (int e = 0; e < 16; ++e) dst[e] = TRANS ? lrow[e * estride] : lrow[e];
        }
    };
    sfor<0, PF>([&](auto dc) { request(decltype(dc)::value, lv[decltype(dc)::value]); });
    int par = 0;
    bool stop = false;  // uniform: a bounded wait gave up
    for (int st0 = 0; st0 < nsteps; st0 += PF) {
        sfor<0, PF>([&](auto dc) {
            constexpr int d = decltype(dc)::value;
            const int st = st0 + d;
            if (st >= nsteps || stop) return;  // uniform
            const int j = upper ? nblk - 1 - st : st;
            // the solution words of block j, requested before the next tile
            unsigned long long wv[WPT];
#pragma unroll
            for (int p = 0; p < WPT; ++p) {
                const int tt = tid + p * 512;
                wv[p] = 0ull;
                if (tt < wblk) {
                    const int i = tt / (nrhs * PWV), rr = tt - i * (nrhs * PWV);
                    wv[p] = xload(yx + ((size_t)(j * BS + i) * NRT) * PWV + rr);
                }
            }
            T cur[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) cur[e] = lv[d][e];
            request(st + PF, lv[d]);
            bool bad = false;
#pragma unroll
            for (int p = 0; p < WPT; ++p) {
                const int tt = tid + p * 512;
                if (tt < wblk) {
                    unsigned v = (unsigned)wv[p];
                    if ((unsigned)(wv[p] >> 32) != 1u && !bad) {
                        const int i = tt / (nrhs * PWV), rr = tt - i * (nrhs * PWV);
                        v = spin_tag(yx + ((size_t)(j * BS + i) * NRT) * PWV + rr, 1u,
                                     &status[ST_TIMEOUT], bad);
                    }
                    swords[par][tt] = v;
                }
            }
            if (bad) s_bad = 1;
            __syncthreads();
            if (s_bad) {
                stop = true;
                return;
            }
            if (mine) {
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int i = q * 16 + e;
#pragma unroll
                    for (int c = 0; c < NRT; ++c)
                        if (c < nrhs) acc[c] += cur[e] * Words<T>::make(&swords[par][(i * nrhs + c) * PWV]);
                }
            }
            par ^= 1;
        });
        if (stop) return;
    }
    // y = inv(M_bb) (rhs_b - sum_j M_bj y_j) for this half's block: 16
    // products per thread, then the four quarters of each row; q == 0
    // writes Y, publishes the words and (first block) keeps y in LDS
    auto finish = [&](int hh) {
        T yv[NRT];
#pragma unroll
        for (int c = 0; c < NRT; ++c) {
            T v = (T)0;
#pragma unroll
            for (int e = 0; e < 16; ++e) v += dg[e] * sy[hh][q * 16 + e][c];
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            yv[c] = v;
        }
        if (q == 0) {
            const int row = b * BS + r;
#pragma unroll
            for (int c = 0; c < NRT; ++c) {
                if (c < nrhs) {
                    Y[(size_t)row * ldy + c] = yv[c];
                    if (hh == 0) sfirst[r][c] = yv[c];
#pragma unroll
                    for (int wv = 0; wv < PWV; ++wv)
                        xstore(yx + ((size_t)row * NRT + c) * PWV + wv, 1u, Words<T>::get(yv[c], wv));
                }
            }
        }
    };
    // the first block: combine the four k-quarters of each row
    if (h == 0) {
#pragma unroll
        for (int c = 0; c < NRT; ++c) {
            acc[c] += __shfl_xor(acc[c], 1);
            acc[c] += __shfl_xor(acc[c], 2);
        }
        if (q == 0) {
#pragma unroll
            for (int c = 0; c < NRT; ++c)
                if (c < nrhs) sy[0][r][c] = Y[(size_t)(b * BS + r) * ldy + c] - acc[c];
        }
    }
    __syncthreads();
    if (h == 0) finish(0);
    __syncthreads();
    // the second block: its product with the first block's solution, from LDS
    if (h == 1 && has1) {
#pragma unroll
        for (int c = 0; c < NRT; ++c) {
            if (c < nrhs) {
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[c] += lx[e] * sfirst[q * 16 + e][c];
            }
            acc[c] += __shfl_xor(acc[c], 1);
            acc[c] += __shfl_xor(acc[c], 2);
        }
        if (q == 0) {
#pragma unroll
            for (int c = 0; c < NRT; ++c)
                if (c < nrhs) sy[1][r][c] = Y[(size_t)(b * BS + r) * ldy + c] - acc[c];
        }
    }
    __syncthreads();
    if (h == 1 && has1) finish(1);
}

template <typename Tw, bool TRANS>
hipError_t launch_trsv_t(int upper, const Tw *W, int ldw, const Tw *dinv, int npad, Tw *Y,
                         int ldy, int nrhs, unsigned long long *ybuf, int *status,
                         hipStream_t s) {
    if (npad == 0 || nrhs == 0) return hipSuccess;
    if (nrhs > kTrsvNRT || npad % kTrsvBS) return hipErrorInvalidValue;
    const int nblk = npad / kTrsvBS;
    constexpr int PWV = sizeof(Tw) / 4;
    hipError_t e = launch_fill_u32(reinterpret_cast<unsigned *>(ybuf), 0u,
                                   ((size_t)npad * kTrsvNRT * PWV + 1) * 2, s);
    if (e != hipSuccess) return e;
    // each instantiation lays its words (and ticket) out inside the zeroed region
    const int npairs = (nblk + 1) / 2;  // two blocks per workgroup
    if (nrhs == 1)
        k_trsv<Tw, 1, TRANS><<<dim3(npairs), dim3(512), 0, s>>>(upper, W, ldw, dinv, nblk, Y, ldy,
                                                                nrhs, ybuf, status);
    else
        k_trsv<Tw, kTrsvNRT, TRANS><<<dim3(npairs), dim3(512), 0, s>>>(upper, W, ldw, dinv, nblk, Y,
                                                                       ldy, nrhs, ybuf, status);
    return hipGetLastError();
}

template <typename Tw>
hipError_t launch_trsv(int upper, int trans, const Tw *W, int ldw, const Tw *dinv, int npad,
                       Tw *Y, int ldy, int nrhs, unsigned long long *ybuf, int *status,
                       hipStream_t s) {
    return trans ? launch_trsv_t<Tw, true>(upper, W, ldw, dinv, npad, Y, ldy, nrhs, ybuf, status, s)
                 : launch_trsv_t<Tw, false>(upper, W, ldw, dinv, npad, Y, ldy, nrhs, ybuf, status,
                                            s);
}
template hipError_t launch_trsv<float>(int, int, const float *, int, const float *, int, float *,
                                       int, int, unsigned long long *, int *, hipStream_t);
template hipError_t launch_trsv<double>(int, int, const double *, int, const double *, int,
                                        double *, int, int, unsigned long long *, int *,
                                        hipStream_t);

// One step of the blocked solve for several right-hand sides: workgroup
// (x, y) takes the 16 columns 16y .. 16y+15, four per wave.  Every workgroup
// solves the 64 x 64 diagonal block at j0 for its columns (the block's rows
// in registers, values shared with readlane); workgroup x = 0 stores the
// solved rows in Yout (never in Y, whose block rows the other workgroups of
// the launch may still be reading), and workgroup x = 1 + t updates the
// 64-row tile t of the rows still to be solved, in place in Y:
// Y[rows] -= M[rows, j0:j0+64] Yj.  The tile is read once per workgroup with
// coalesced loads, issued before the diagonal solve, and staged in LDS.
// MODE 0: unit lower L, forward; 1: U, backward; 2: U^T (lower, non-unit),
// forward; 3: L^T (unit upper), backward.  The triangular matrix is
// M[r][c] = W[r][c] (modes 0, 1) or W[c][r] (modes 2, 3).  Rows to update:
// j0+64 .. npad-1 (forward) or 0 .. j0-1 (backward).
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_trsm_step(const T *__restrict__ W, int ldw, int j0,
                                                   int npad, T *__restrict__ Y,
                                                   T *__restrict__ Yout, int ldy, int nrhs) {
    constexpr int BS = kTrsvBS, CPW = 4, CPG = 4 * CPW;  // columns per wave / workgroup
    constexpr int TPT = BS * BS / 256;                    // tile elements per thread
    constexpr bool TR = MODE >= 2;
    constexpr bool FWD = MODE == 0 || MODE == 2;
    constexpr bool UNIT = MODE == 0 || MODE == 3;
    __shared__ T sd[BS][BS + 1];
    __shared__ T sw[BS][BS + 1];
    __shared__ T sy[BS][CPG + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c0 = blockIdx.y * CPG + wave * CPW;  // this wave's first column
    const int t = blockIdx.x - 1;
    const int r0 = FWD ? j0 + BS + t * BS : t * BS;
    const int rows_end = FWD ? npad : j0;
    const bool tile = blockIdx.x > 0 && r0 < rows_end;
    const int row = r0 + lane;
    // element e = tid + 256 i of a 64 x 64 block: (e / 64, e % 64) is
    // (row, column) of W, so consecutive threads read consecutive words
    T tv[TPT];
    if (tile) {
#pragma unroll
        for (int i = 0; i < TPT; ++i) {
            const int e = tid + 256 * i, a = e / BS, b = e % BS;
            tv[i] = TR ? W[(size_t)(j0 + a) * ldw + r0 + b] : W[(size_t)(r0 + a) * ldw + j0 + b];
        }
    }
    T ypre[CPW], y[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const bool ok = c0 + c < nrhs;
        y[c] = ok ? Y[(size_t)(j0 + lane) * ldy + c0 + c] : (T)0;
        ypre[c] = (ok && tile) ? Y[(size_t)row * ldy + c0 + c] : (T)0;
    }
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
        const int e = tid + 256 * i, a = e / BS, b = e % BS;
        const T v = W[(size_t)(j0 + a) * ldw + j0 + b];
        if (TR) sd[b][a] = v;
        else sd[a][b] = v;
    }
    __syncthreads();
    {
        T mrow[BS];
#pragma unroll
        for (int k = 0; k < BS; ++k) mrow[k] = sd[lane][k];
        // non-unit triangles: scale this lane's row and values by the
        // reciprocal of its diagonal entry before the chain (the system
        // D^-1 M y = D^-1 r has a unit diagonal), so every dependent step is
        // one broadcast and one FMA per column
        if constexpr (!UNIT) {
            const T dinv = (T)1 / sd[lane][lane];
#pragma unroll
            for (int k = 0; k < BS; ++k) mrow[k] *= dinv;
#pragma unroll
            for (int c = 0; c < CPW; ++c) y[c] *= dinv;
        }
#pragma unroll
        for (int kk = 0; kk < BS; ++kk) {
            const int k = FWD ? kk : BS - 1 - kk;
            const bool below = FWD ? lane > k : lane < k;
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
                const T yk = readlane_t(y[c], k);
                if (below) y[c] -= mrow[k] * yk;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        sy[lane][wave * CPW + c] = y[c];
        if (blockIdx.x == 0 && c0 + c < nrhs) Yout[(size_t)(j0 + lane) * ldy + c0 + c] = y[c];
    }
    if (!tile) return;  // uniform over the workgroup
    // M[row][k] = sw[row - r0][k]
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
        const int e = tid + 256 * i, a = e / BS, b = e % BS;
        if (TR) sw[b][a] = tv[i];
        else sw[a][b] = tv[i];
    }
    __syncthreads();
    T acc[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) acc[c] = (T)0;
#pragma unroll 16
    for (int k = 0; k < BS; ++k) {
        const T m = sw[lane][k];
#pragma unroll
        for (int c = 0; c < CPW; ++c) acc[c] += m * sy[k][wave * CPW + c];
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c)
        if (c0 + c < nrhs) Y[(size_t)row * ldy + c0 + c] = ypre[c] - acc[c];
}

template <typename Tw>
hipError_t launch_trsm_blocked(int upper, int trans, const Tw *W, int ldw, int npad, Tw *Y,
                               Tw *Yout, int ldy, int nrhs, hipStream_t s) {
    constexpr int BS = kTrsvBS;
    if (npad == 0 || nrhs == 0) return hipSuccess;
    if (npad % BS) return hipErrorInvalidValue;
    const int nblk = npad / BS;
    const int mode = trans ? (upper ? 3 : 2) : (upper ? 1 : 0);
    for (int t = 0; t < nblk; ++t) {
        const int b = upper ? nblk - 1 - t : t;
        const int tiles = upper ? b : nblk - 1 - b;
        const dim3 grid(1 + tiles, (nrhs + 15) / 16);
        const int j0 = b * BS;
        switch (mode) {
            case 0: k_trsm_step<Tw, 0><<<grid, 256, 0, s>>>(W, ldw, j0, npad, Y, Yout, ldy, nrhs); break;
            case 1: k_trsm_step<Tw, 1><<<grid, 256, 0, s>>>(W, ldw, j0, npad, Y, Yout, ldy, nrhs); break;
            case 2: k_trsm_step<Tw, 2><<<grid, 256, 0, s>>>(W, ldw, j0, npad, Y, Yout, ldy, nrhs); break;
            default: k_trsm_step<Tw, 3><<<grid, 256, 0, s>>>(W, ldw, j0, npad, Y, Yout, ldy, nrhs); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
template hipError_t launch_trsm_blocked<float>(int, int, const float *, int, int, float *,
                                               float *, int, int, hipStream_t);
template hipError_t launch_trsm_blocked<double>(int, int, const double *, int, int, double *,
                                                double *, int, int, hipStream_t);

// Row i of the solve vector z goes to row d = perm[i] of X (perm = NULL: the
// identity; the transposed solve scatters through P^T): X[d] = S[d] z[i]
// (assign) or X[d] += S[d] z[i], z promoted to FP64, for d < n;
// xnorm[c] = max |X[:, c]| over the rows written.
template <typename Tw>
__global__ __launch_bounds__(256) void k_x_update(int n, int npad, int nrhs, int assign,
                                                  const Tw *__restrict__ Y, int ldy,
                                                  const int *__restrict__ perm,
                                                  const double *__restrict__ C,
                                                  double *__restrict__ X, int ldx, int x_col_major,
                                                  double *__restrict__ xnorm) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int d = i < npad ? (perm ? perm[i] : i) : n;
    for (int c = 0; c < nrhs; ++c) {
        double v = 0.0;
        if (d < n) {
            double *px = x_col_major ? X + d + (size_t)c * ldx : X + (size_t)d * ldx + c;
            v = C[d] * (double)Y[(size_t)i * ldy + c];
            if (!assign) v += *px;
            *px = v;
        }
        double a = fabs(v);
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(a, off);
            a = (o > a || o != o) ? o : a;  // NaN wins, so it reaches the norm
        }
        if ((threadIdx.x & 63) == 0) atomic_max_nonneg(&xnorm[c], a);
    }
}

template <typename Tw>
hipError_t launch_x_update(int n, int npad, int nrhs, int assign, const Tw *Y, int ldy,
                           const int *perm, const double *C, double *X, int ldx, int x_col_major,
                           double *xnorm, hipStream_t s) {
    if (n == 0 || nrhs == 0) return hipSuccess;
    const int rows = perm ? npad : n;
    k_x_update<Tw><<<dim3((rows + 255) / 256), dim3(256), 0, s>>>(n, rows, nrhs, assign, Y, ldy,
                                                                 perm, C, X, ldx, x_col_major,
                                                                 xnorm);
    return hipGetLastError();
}
template hipError_t launch_x_update<float>(int, int, int, int, const float *, int, const int *,
                                           const double *, double *, int, int, double *,
                                           hipStream_t);
template hipError_t launch_x_update<double>(int, int, int, int, const double *, int, const int *,
                                            const double *, double *, int, int, double *,
                                            hipStream_t);

// r = b - A x in FP64 (A row-major n x n), 16 rows per workgroup (4 per
// wave), up to NR right-hand sides; rnorm[c] = max_i |r_ic| and, from the
// first wave (which reads all of x), xnorm[c] = max_j |x_jc|: the stopping
// test then uses the norms of exactly the x this residual belongs to.
// VEC: rows are read as 16-byte pairs (needs even n and lda and 16-byte
// aligned A), two pairs in flight per lane and row.
__device__ inline double nanmax(double m, double a) { return (a > m || a != a) ? a : m; }

template <int NR, bool VEC>
__global__ __launch_bounds__(256) void k_residual(int n, int nrhs, const double *__restrict__ A,
                                                  int lda, const double *__restrict__ X, int ldx,
                                                  const double *__restrict__ B, int ldb, int bx_cm,
                                                  double *__restrict__ Rv, int ldr,
                                                  double *__restrict__ rnorm,
                                                  double *__restrict__ xnorm) {
    constexpr int RPW = 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = (blockIdx.x * 4 + wave) * RPW;
    double xm[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) xm[c] = 0.0;
    // compensated row sums (s, e): see dot2_add
    double acc[RPW][NR], err[RPW][NR];
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr)
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[rr][c] = err[rr][c] = 0.0;
    auto xat = [&](int j, int c) -> double {
        return (c < nrhs) ? (bx_cm ? X[j + (size_t)c * ldx] : X[(size_t)j * ldx + c]) : 0.0;
    };
    if constexpr (VEC) {
        for (int j0 = 2 * lane; j0 < n; j0 += 256) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int j = j0 + 128 * h;
                if (j < n) {
                    double x0[NR], x1[NR];
#pragma unroll
                    for (int c = 0; c < NR; ++c) {
                        x0[c] = xat(j, c);
                        x1[c] = xat(j + 1, c);
                        xm[c] = nanmax(nanmax(xm[c], fabs(x0[c])), fabs(x1[c]));
                    }
#pragma unroll
                    for (int rr = 0; rr < RPW; ++rr) {
                        const int row = r0 + rr;
                        if (row < n) {
                            const double2 a = *reinterpret_cast<const double2 *>(A + (size_t)row * lda + j);
#pragma unroll
                            for (int c = 0; c < NR; ++c) {
                                dot2_add(acc[rr][c], err[rr][c], a.x, x0[c]);
                                dot2_add(acc[rr][c], err[rr][c], a.y, x1[c]);
                            }
                        }
                    }
                }
            }
        }
    } else {
        for (int j = lane; j < n; j += 64) {
            double xv[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                xv[c] = xat(j, c);
                xm[c] = nanmax(xm[c], fabs(xv[c]));
            }
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr) {
                const int row = r0 + rr;
                if (row < n) {
                    const double a = A[(size_t)row * lda + j];
#pragma unroll
                    for (int c = 0; c < NR; ++c) dot2_add(acc[rr][c], err[rr][c], a, xv[c]);
                }
            }
        }
    }
    double rmax[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) rmax[c] = 0.0;
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            double v = acc[rr][c], e = err[rr][c];
            for (int off = 32; off > 0; off >>= 1) dot2_merge(v, e, __shfl_xor(v, off), __shfl_xor(e, off));
            acc[rr][c] = v;
            err[rr][c] = e;
        }
        const int row = r0 + rr;
        if (lane == 0 && row < n) {
#pragma unroll
            for (int c = 0; c < NR; ++c)
                if (c < nrhs) {
                    const double b = bx_cm ? B[row + (size_t)c * ldb] : B[(size_t)row * ldb + c];
                    const double r = dot2_residual(b, acc[rr][c], err[rr][c]);
                    Rv[(size_t)row * ldr + c] = r;
                    const double ar = fabs(r);
                    rmax[c] = (ar > rmax[c] || ar != ar) ? ar : rmax[c];
                }
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < NR; ++c)
            if (c < nrhs) atomic_max_nonneg(&rnorm[c], rmax[c]);
    }
    if (blockIdx.x == 0 && wave == 0) {
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            double v = xm[c];
            for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off));
            if (lane == 0 && c < nrhs) xnorm[c] = v;
        }
    }
}

hipError_t launch_residual(int n, int nrhs, const double *A, int lda, const double *X, int ldx,
                           const double *B, int ldb, int bx_col_major, double *Rv, int ldr,
                           double *rnorm, double *xnorm, hipStream_t s) {
    if (n == 0 || nrhs == 0) return hipSuccess;
    const dim3 grid((n + 15) / 16);
    const bool vec = (n % 2 == 0) && (lda % 2 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
    for (int c0 = 0; c0 < nrhs; c0 += 8) {
        const int nr = nrhs - c0 < 8 ? nrhs - c0 : 8;
        const double *Xc = bx_col_major ? X + (size_t)c0 * ldx : X + c0;
        const double *Bc = bx_col_major ? B + (size_t)c0 * ldb : B + c0;
        if (nr == 1) {
            if (vec)
                k_residual<1, true><<<grid, dim3(256), 0, s>>>(n, 1, A, lda, Xc, ldx, Bc, ldb,
                                                               bx_col_major, Rv + c0, ldr, rnorm + c0, xnorm + c0);
            else
                k_residual<1, false><<<grid, dim3(256), 0, s>>>(n, 1, A, lda, Xc, ldx, Bc, ldb,
                                                                bx_col_major, Rv + c0, ldr, rnorm + c0, xnorm + c0);
        } else {
            if (vec)
                k_residual<8, true><<<grid, dim3(256), 0, s>>>(n, nr, A, lda, Xc, ldx, Bc, ldb,
                                                               bx_col_major, Rv + c0, ldr, rnorm + c0, xnorm + c0);
            else
                k_residual<8, false><<<grid, dim3(256), 0, s>>>(n, nr, A, lda, Xc, ldx, Bc, ldb,
                                                                bx_col_major, Rv + c0, ldr, rnorm + c0, xnorm + c0);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// r = b - A^T x in FP64 for row-major A: column sums in two passes.  Pass 1:
// workgroup (column group g of 256 columns, row chunk h) accumulates
// part[h][j][c] = sum over its rows i of A[i][j] x[i][c] for up to 8
// right-hand sides (one column per thread: coalesced row segments); the
// workgroups of column group 0 also fold max |x| into xnorm (zeroed by the
// caller).  Pass 2: r[j][c] = b[j][c] - sum_h part[h][j][c] and
// rnorm[c] = max_j |r[j][c]| (zeroed by the caller).
constexpr int kResTChunks = 16;
__global__ __launch_bounds__(256) void k_residual_t_part(int n, int nrhs, int rows_per_chunk,
                                                         const double *__restrict__ A, int lda,
                                                         const double *__restrict__ X, int ldx,
                                                         int x_cm, double *__restrict__ part,
                                                         double *__restrict__ xnorm) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int h = blockIdx.y;
    const int i0 = h * rows_per_chunk;
    const int i1 = min(n, i0 + rows_per_chunk);
    __shared__ double sx[64][8];
    // compensated column sums (s, e) for up to 4 right-hand sides: see dot2_add
    double acc[4], err[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = err[c] = 0.0;
    // thread t always stages right-hand side c = t & 7 (256 is a multiple of 8)
    double xm = 0.0;
    for (int ib = i0; ib < i1; ib += 64) {
        const int cnt = min(64, i1 - ib);
        __syncthreads();
        for (int t = threadIdx.x; t < 64 * 8; t += 256) {
            const int ii = t >> 3, c = t & 7;
            double v = 0.0;
            if (ii < cnt && c < nrhs)
                v = x_cm ? X[(size_t)(ib + ii) + (size_t)c * ldx] : X[(size_t)(ib + ii) * ldx + c];
            sx[ii][c] = v;
            xm = nanmax(xm, fabs(v));
        }
        __syncthreads();
        if (j < n) {
            for (int ii = 0; ii < cnt; ++ii) {
                const double a = A[(size_t)(ib + ii) * lda + j];
#pragma unroll
                for (int c = 0; c < 4; ++c) dot2_add(acc[c], err[c], a, sx[ii][c]);
            }
        }
    }
    if (j < n) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < nrhs) {
                part[((size_t)h * n + j) * 8 + 2 * c] = acc[c];
                part[((size_t)h * n + j) * 8 + 2 * c + 1] = err[c];
            }
    }
    if (blockIdx.x == 0 && (threadIdx.x & 7) < nrhs) atomic_max_nonneg(&xnorm[threadIdx.x & 7], xm);
}

__global__ __launch_bounds__(256) void k_residual_t_fin(int n, int nrhs, int chunks,
                                                        const double *__restrict__ part,
                                                        const double *__restrict__ B, int ldb,
                                                        int b_cm, double *__restrict__ Rv, int ldr,
                                                        double *__restrict__ rnorm) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    for (int c = 0; c < nrhs; ++c) {
        double ar = 0.0;
        if (j < n) {
            double s = 0.0, e = 0.0;
            for (int h = 0; h < chunks; ++h)
                dot2_merge(s, e, part[((size_t)h * n + j) * 8 + 2 * c],
                           part[((size_t)h * n + j) * 8 + 2 * c + 1]);
            const double b = b_cm ? B[j + (size_t)c * ldb] : B[(size_t)j * ldb + c];
            const double r = dot2_residual(b, s, e);
            Rv[(size_t)j * ldr + c] = r;
            ar = fabs(r);
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(ar, off);
            ar = (o > ar || o != o) ? o : ar;
        }
        if ((threadIdx.x & 63) == 0) atomic_max_nonneg(&rnorm[c], ar);
    }
}

hipError_t launch_residual_t(int n, int nrhs, const double *A, int lda, const double *X, int ldx,
                             const double *B, int ldb, int bx_col_major, double *Rv, int ldr,
                             double *rnorm, double *xnorm, double *part, hipStream_t s) {
    if (n == 0 || nrhs == 0) return hipSuccess;
    const int chunks = n < kResTChunks * 64 ? (n + 63) / 64 : kResTChunks;
    const int rpc = (n + chunks - 1) / chunks;
    const dim3 grid((n + 255) / 256, chunks);
    for (int c0 = 0; c0 < nrhs; c0 += 4) {
        const int nr = nrhs - c0 < 4 ? nrhs - c0 : 4;
        const double *Xc = bx_col_major ? X + (size_t)c0 * ldx : X + c0;
        const double *Bc = bx_col_major ? B + (size_t)c0 * ldb : B + c0;
        k_residual_t_part<<<grid, dim3(256), 0, s>>>(n, nr, rpc, A, lda, Xc, ldx, bx_col_major,
                                                     part, xnorm + c0);
        k_residual_t_fin<<<dim3((n + 255) / 256), dim3(256), 0, s>>>(
            n, nr, chunks, part, Bc, ldb, bx_col_major, Rv + c0, ldr, rnorm + c0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Several right-hand sides: R = B - op(A) X as a copy of B followed by an
// FP64 MFMA GEMM (k_gemm<double>), then the per-column norms of R and X.
__global__ __launch_bounds__(256) void k_copy_rhs(int n, int nrhs, const double *__restrict__ B,
                                                  int ldb, int cm, double *__restrict__ R,
                                                  int ldr) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)n * nrhs) return;
    const int i = (int)(e / nrhs), c = (int)(e % nrhs);
    R[(size_t)i * ldr + c] = cm ? B[i + (size_t)c * ldb] : B[(size_t)i * ldb + c];
}

// rnorm[c] = max_i |R[i][c]|, xnorm[c] = max_i |X[i][c]| (both zeroed by the
// caller): 256 rows per workgroup, one wave reduction per column.
__global__ __launch_bounds__(256) void k_col_norms(int n, int nrhs, const double *__restrict__ R,
                                                   int ldr, const double *__restrict__ X, int ldx,
                                                   int x_cm, double *__restrict__ rnorm,
                                                   double *__restrict__ xnorm) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    for (int c = 0; c < nrhs; ++c) {
        double r = 0.0, x = 0.0;
        if (i < n) {
            r = fabs(R[(size_t)i * ldr + c]);
            x = fabs(x_cm ? X[i + (size_t)c * ldx] : X[(size_t)i * ldx + c]);
        }
        for (int off = 32; off > 0; off >>= 1) {
            r = nanmax(r, __shfl_xor(r, off));
            x = nanmax(x, __shfl_xor(x, off));
        }
        if ((threadIdx.x & 63) == 0) {
            atomic_max_nonneg(&rnorm[c], r);
            atomic_max_nonneg(&xnorm[c], x);
        }
    }
}

hipError_t launch_residual_mm(int n, int nrhs, const double *A, int lda, int transa,
                              const double *X, int ldx, const double *B, int ldb, int cm,
                              double *Rv, int ldr, double *rnorm, double *xnorm, double *P,
                              int nsplit, hipStream_t s) {
    if (n == 0 || nrhs == 0) return hipSuccess;
    const size_t cnt = (size_t)n * nrhs;
    k_copy_rhs<<<dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s>>>(n, nrhs, B, ldb, cm, Rv,
                                                                         ldr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // column-major X is the row-major nrhs x n matrix X^T: the "B transposed" form
    // K split over nsplit slices (partials in P): a few right-hand sides give
    // too few output tiles to keep the GPU busy over the long K = n
    e = launch_gemm_splitk<double>(n, nrhs, n, A, lda, X, ldx, Rv, ldr, cm, transa, P, nsplit, s);
    if (e != hipSuccess) return e;
    k_col_norms<<<dim3((n + 255) / 256), dim3(256), 0, s>>>(n, nrhs, Rv, ldr, X, ldx, cm, rnorm,
                                                            xnorm);
    return hipGetLastError();
}

// ----------------------------------------------------------------------
// FP64 vector kernels of the flexible GMRES refinement (Algorithm 2's outer
// loop).  Basis vectors are stored one after another: V[j * ldv + i].
// ----------------------------------------------------------------------
// h[j] = sum_i V[j][i] w[i] for j < k: workgroup j reduces one dot product.
__global__ __launch_bounds__(256) void k_dots(int n, int k, const double *__restrict__ V, size_t ldv,
                                              const double *__restrict__ w,
                                              double *__restrict__ h) {
    const int j = blockIdx.x;
    if (j >= k) return;
    const double *v = V + (size_t)j * ldv;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += v[i] * w[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) h[j] = (part[0] + part[1]) + (part[2] + part[3]);
}

// w[i] += sign * sum_{j<k} h[j] V[j][i]
__global__ __launch_bounds__(256) void k_combine(int n, int k, const double *__restrict__ V,
                                                 size_t ldv, const double *__restrict__ h,
                                                 double sign, double *__restrict__ w) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += h[j] * V[(size_t)j * ldv + i];
    w[i] += sign * s;
}

// y[i] = alpha * x[i]
__global__ __launch_bounds__(256) void k_scale_copy(int n, double alpha, const double *__restrict__ x,
                                                    double *__restrict__ y) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = alpha * x[i];
}

hipError_t launch_dots(int n, int k, const double *V, size_t ldv, const double *w, double *h,
                       hipStream_t s) {
    if (k <= 0) return hipSuccess;
    k_dots<<<dim3(k), dim3(256), 0, s>>>(n, k, V, ldv, w, h);
    return hipGetLastError();
}
hipError_t launch_combine(int n, int k, const double *V, size_t ldv, const double *h, double sign,
                          double *w, hipStream_t s) {
    if (k <= 0 || n <= 0) return hipSuccess;
    k_combine<<<dim3((n + 255) / 256), dim3(256), 0, s>>>(n, k, V, ldv, h, sign, w);
    return hipGetLastError();
}
hipError_t launch_scale_copy(int n, double alpha, const double *x, double *y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_scale_copy<<<dim3((n + 255) / 256), dim3(256), 0, s>>>(n, alpha, x, y);
    return hipGetLastError();
}

// GA = beta GA + alpha G X^T (all row-major FP64; G, X are n x nrhs).
__global__ __launch_bounds__(256) void k_outer(int n, int nrhs, const double *__restrict__ G,
                                               int ldg, const double *__restrict__ X, int ldx,
                                               double *__restrict__ GA, int ldga, double alpha,
                                               double beta) {
    __shared__ double sg[64][17], sx[64][17];
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    double acc[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = 0.0;
    for (int c0 = 0; c0 < nrhs; c0 += 16) {
        for (int e = threadIdx.x; e < 64 * 16; e += 256) {
            const int rr = e / 16, cc = e % 16;
            sg[rr][cc] = (i0 + rr < n && c0 + cc < nrhs) ? G[(size_t)(i0 + rr) * ldg + c0 + cc] : 0.0;
            sx[rr][cc] = (j0 + rr < n && c0 + cc < nrhs) ? X[(size_t)(j0 + rr) * ldx + c0 + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = ty * 16 + e;
            double sacc = 0.0;
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) sacc += sg[i][cc] * sx[tx][cc];
            acc[e] += sacc;
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = i0 + ty * 16 + e, j = j0 + tx;
        if (i < n && j < n) {
            double *p = GA + (size_t)i * ldga + j;
            *p = (beta == 0.0 ? 0.0 : beta * *p) + alpha * acc[e];
        }
    }
}

hipError_t launch_outer(int n, int nrhs, const double *G, int ldg, const double *X, int ldx,
                        double *GA, int ldga, double alpha, double beta, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_outer<<<dim3((n + 63) / 64, (n + 63) / 64), dim3(256), 0, s>>>(n, nrhs, G, ldg, X, ldx, GA,
                                                                    ldga, alpha, beta);
    return hipGetLastError();
}

}  // namespace mixlu
