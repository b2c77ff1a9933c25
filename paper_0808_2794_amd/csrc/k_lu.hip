// Blocked LU with partial pivoting on gfx950: Algorithm 1 step 1 (the
// SGETRF of Section 3.1.1), PA = LU with partial row pivoting (Section 2.1).
//
//   k_panel       GEPP on a tall panel of B columns; the panel rows are held
//                 in registers across up to 32 workgroups placed on one XCD;
//                 per column: argmax (first index on ties), the candidate
//                 rows published as tagged words and gathered by one wave,
//                 swap, scale; the rank-1 update overlaps the exchange.
//                 The panel's own interchanges on the other columns of its
//                 block (and on perm) run at the end of the same launch.
//   k_row_swaps   applies a block of pivots to the columns outside the panel
//   k_swaps_compose, k_rows_apply: the same for wide blocks, in two launches
//   k_trsm_diag   X = L^{-1} X with a unit lower diagonal block in LDS
//   k_gemm        C -= A B on MFMA (f32 16x16x4, f64 16x16x4)
//   k_pack_*      rounds L21 / U12 to FP16 or BF16 for the trailing update
//   k_gemm_lowp   C -= A B^T on MFMA f16/bf16 16x16x32 with FP32 accumulate
#include <climits>
#include <type_traits>

#include <hip/hip_fp8.h>

#include "common.h"

namespace mixlu {

// ======================================================================
// Panel factorization
// ======================================================================
// One thread holds one panel row (B values) in registers, as NG = B / 16
// blocks of 16.  Per column j (all rows' column j up to date):
//   1. wave argmax of |a_j| (first row on ties), then the workgroup's after
//      one barrier; the winner's signed value travels with it;
//   2. the winning wave stages its winner's row in LDS and brings it up to
//      date one element per lane (the pending rank-1 update of column j-1,
//      see 3), then publishes it with a header (signed pivot, row) as tagged
//      words; wave 1 of workgroup 0 does the same for row j (staged by its
//      owner before the barrier);
//   3. every row applies the pending rank-1 update of columns > j with the
//      previous pivot row, broadcast across lanes by DPP inside the
//      multiply-add, while the exchange is in flight;
//   4. the last wave gathers: it polls the P headers and row j, picks the
//      winner (largest |pivot|, then the smallest row: workgroups hold
//      increasing rows), computes 1 / pivot while that workgroup's row is
//      fetched, and leaves pivot, row j and the decision in LDS;
//   5. after a second barrier: the interchange, the multipliers of column j
//      and the update of column j + 1 only; the rest of that rank-1 update
//      is the next column's pending update.
// A single workgroup exchanges through LDS only.  The column loop runs over
// groups of 16 columns; at the end of a group the register blocks rotate by
// one, so the current block is always block 0 and the code of one group
// serves all of them.

// a += (lane K of every 16-lane row of nu) * l for K = 0..15, the broadcast
// folded into the multiply-add (DPP row_newbcast); the leading s_nop covers
// the hazard of a VALU write of nu just before a DPP read of it
template <typename T> struct BcastFma;
template <> struct BcastFma<float> {
    template <int K> __device__ static __forceinline__ void one(float &a, float nu, float l) {
        asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
            : "+v"(a)
            : "v"(nu), "v"(l), "i"(K));
    }
    __device__ static __forceinline__ void block(float (&a)[16], float nu, float l) {
#define MIXLU_FB(K) "v_fmac_f32_dpp %" #K ", %16, %17 row_newbcast:" #K " row_mask:0xf bank_mask:0xf\n\t"
        asm("s_nop 1\n\t" MIXLU_FB(0) MIXLU_FB(1) MIXLU_FB(2) MIXLU_FB(3) MIXLU_FB(4) MIXLU_FB(5)
                MIXLU_FB(6) MIXLU_FB(7) MIXLU_FB(8) MIXLU_FB(9) MIXLU_FB(10) MIXLU_FB(11)
                    MIXLU_FB(12) MIXLU_FB(13) MIXLU_FB(14) MIXLU_FB(15)
            : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]),
              "+v"(a[7]), "+v"(a[8]), "+v"(a[9]), "+v"(a[10]), "+v"(a[11]), "+v"(a[12]),
              "+v"(a[13]), "+v"(a[14]), "+v"(a[15])
            : "v"(nu), "v"(l));
#undef MIXLU_FB
    }
};
template <> struct BcastFma<double> {
    template <int K> __device__ static __forceinline__ void one(double &a, double nu, double l) {
        asm("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
            : "+v"(a)
            : "v"(nu), "v"(l), "i"(K));
    }
    __device__ static __forceinline__ void block(double (&a)[16], double nu, double l) {
#define MIXLU_FB(K) "v_fmac_f64_dpp %" #K ", %16, %17 row_newbcast:" #K " row_mask:0xf bank_mask:0xf\n\t"
        asm("s_nop 1\n\t" MIXLU_FB(0) MIXLU_FB(1) MIXLU_FB(2) MIXLU_FB(3) MIXLU_FB(4) MIXLU_FB(5)
                MIXLU_FB(6) MIXLU_FB(7) MIXLU_FB(8) MIXLU_FB(9) MIXLU_FB(10) MIXLU_FB(11)
                    MIXLU_FB(12) MIXLU_FB(13) MIXLU_FB(14) MIXLU_FB(15)
            : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]),
              "+v"(a[7]), "+v"(a[8]), "+v"(a[9]), "+v"(a[10]), "+v"(a[11]), "+v"(a[12]),
              "+v"(a[13]), "+v"(a[14]), "+v"(a[15])
            : "v"(nu), "v"(l));
#undef MIXLU_FB
    }
};

// LDS ordering between lanes of one wave
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Register row (NG blocks of 16, block b holding columns 16 ((g + b) % NG)
// ..) to and from a B-value row in LDS.
template <typename T, int NG>
__device__ __forceinline__ void blocks_to_lds(T *dst, const T (&a)[NG][16], int g) {
    using vq = typename Vq<T>::type;
    constexpr int V = Vq<T>::V;
#pragma unroll
    for (int b = 0; b < NG; ++b) {
        vq *d = reinterpret_cast<vq *>(dst + 16 * ((g + b) % NG));
#pragma unroll
        for (int q = 0; q < 16 / V; ++q) {
            vq v;
#pragma unroll
            for (int e = 0; e < V; ++e) v[e] = a[b][q * V + e];
            d[q] = v;
        }
    }
}
template <typename T, int NG>
__device__ __forceinline__ void blocks_from_lds(T (&a)[NG][16], const T *src, int g) {
    using vq = typename Vq<T>::type;
    constexpr int V = Vq<T>::V;
#pragma unroll
    for (int b = 0; b < NG; ++b) {
        const vq *s = reinterpret_cast<const vq *>(src + 16 * ((g + b) % NG));
#pragma unroll
        for (int q = 0; q < 16 / V; ++q) {
            const vq v = s[q];
#pragma unroll
            for (int e = 0; e < V; ++e) a[b][q * V + e] = v[e];
        }
    }
}

template <typename T, int B>
__global__ __launch_bounds__(kPanelTPB) void k_panel(T *__restrict__ W, int ldw, int k0, int m,
                                                     int *__restrict__ ipiv,
                                                     unsigned long long *__restrict__ xb,
                                                     int *__restrict__ status, int P, int stride,
                                                     int *__restrict__ perm, int sc0, int sc1,
                                                     int *__restrict__ pmv) {
    if (blockIdx.x % stride) return;
    const int w = blockIdx.x / stride;
    if (w >= P) return;
    constexpr int TPB = kPanelTPB, NW = TPB / 64;
    static_assert(NW >= 2 && NW <= 8, "two to eight waves");
    constexpr int GW = NW - 1;  // gathering wave
    constexpr int DW = 1;       // wave that publishes row j (workgroup 0)
    constexpr int NG = B / 16;
    constexpr int PWV = Words<T>::n;
    constexpr int RW = B * PWV;  // words of a row: one per lane
    static_assert(RW == 64 && B % 16 == 0, "one word of a row per lane");
    constexpr int HDR = 4, SLOT = HDR + RW;
    constexpr int DIAG = kPanelMaxWG * SLOT;
    constexpr int PAR = DIAG + RW;  // words per parity
    static_assert(2 * PAR <= kXbufWords, "exchange buffer");
    constexpr int HW = PWV + 1;     // header words: signed pivot, then row (~0u: no candidate)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pos = w * TPB + tid;
    const bool live = pos < m;

    __shared__ __attribute__((aligned(16))) T s_u[2][B];     // pivot row of the column
    __shared__ __attribute__((aligned(16))) T s_d[2][B];     // row j, moving to the pivot's place
    __shared__ __attribute__((aligned(16))) T s_cand[2][B];  // the candidate row, staged raw
    __shared__ __attribute__((aligned(16))) T s_draw[2][B];  // row j, staged raw
    __shared__ T s_dlp[2];
    __shared__ T s_wval[2][NW], s_wsv[2][NW];
    __shared__ int s_wpos[2][NW];
    __shared__ int s_p[2];
    __shared__ T s_pv[2], s_rcp[2];
    __shared__ int s_piv[B];

    T a[NG][16];
    {
        using vq = typename Vq<T>::type;
        constexpr int V = Vq<T>::V;
        const vq *src = reinterpret_cast<const vq *>(W + (size_t)(k0 + (live ? pos : 0)) * ldw + k0);
#pragma unroll
        for (int b = 0; b < NG; ++b)
#pragma unroll
            for (int q = 0; q < 16 / V; ++q) {
                const vq v = live ? src[b * (16 / V) + q] : vq{};
#pragma unroll
                for (int e = 0; e < V; ++e) a[b][q * V + e] = v[e];
            }
    }
    // The panel's interchanges on the columns [sc0, sc1) outside it and on
    // perm are applied at the end from LDS: the words of this workgroup's
    // slice of those columns (nd <= 64, one per lane) of every row that moves
    // are read while the pivots are chosen.  Slot i < B holds row i of the
    // panel, slot B + j the pivot row of column j when it lies below row B.
    // Nothing writes these columns during the launch, so every read sees the
    // rows as they were before the interchanges.  The waves that do not poll
    // take turns: a pivot row read into a register is written to LDS at that
    // wave's next turn, long after it has arrived.
    const bool swp = perm != nullptr || sc1 > sc0;
    const bool cmp = swp || pmv != nullptr;  // compose the swaps
    const int ncols = sc1 > sc0 ? sc1 - sc0 - B : 0;
    const int cpw = (ncols + P - 1) / P;
    const int lc0 = w * cpw;
    const int nd = max(0, min(cpw, ncols - lc0)) * PWV;
    const int nleft = k0 - sc0;
    __shared__ __attribute__((aligned(16))) unsigned s_rows[2 * B][64];
    __shared__ int s_pm[2 * B];
    const unsigned *Wd = reinterpret_cast<const unsigned *>(W);
    int lword = 0;  // this lane's word of a row of the slice
    if (lane < nd) {
        const int c = lc0 + lane / PWV;
        lword = (sc0 + c + (c >= nleft ? B : 0)) * PWV + lane % PWV;
    }
    const bool fetcher = swp && wave < GW;
    const bool pfetch = perm != nullptr && w == 0;
    constexpr int TR = (B + GW - 1) / GW;  // top rows per fetching wave
    unsigned rtop[TR];
    int ptop = 0;
    if (fetcher) {
#pragma unroll
        for (int i = 0; i < TR; ++i) {
            const int r = wave + GW * i;
            rtop[i] = (r < B && lane < nd) ? Wd[(size_t)(k0 + r) * ldw * PWV + lword] : 0u;
        }
    }
    if (pfetch && tid < B) ptop = perm[k0 + tid];
    if (fetcher) {
#pragma unroll
        for (int i = 0; i < TR; ++i) {
            const int r = wave + GW * i;
            if (r < B) s_rows[r][lane] = rtop[i];
        }
    }
    if (pfetch && tid < B) s_pm[tid] = ptop;
    unsigned rpiv = 0u;  // this wave's last pivot row word, bound for slot spend
    int ppiv = 0, spend = -1;
    // Wave 0 composes the swaps into moves (position <- slot) one column
    // behind, while it waits for the gather: position i < B is lane i of ca,
    // position cpos[t] >= B (t the first column whose pivot row it is) lane t
    // of cb; each holds the slot whose row ends there.
    int ca = lane, cb = B + lane, cpos = -1;
    int jprev = -1, pprev = 0;  // the last column and its pivot row
    auto compose = [&](int t, int qt) __attribute__((always_inline)) {
        if (qt == t) return;
        int sl = qt;
        if (qt >= B) {
            const unsigned long long hit = __ballot(cpos == qt);
            if (hit) {
                sl = B + __ffsll((long long)hit) - 1;
            } else {
                sl = B + t;
                if (lane == t) cpos = qt;
            }
        }
        // selects only (a branch on which register to write makes the
        // compiler put the pair in scratch)
        const bool low = sl < B;
        const int ls = low ? sl : sl - B;
        const int at = __builtin_amdgcn_readlane(ca, t);
        const int va = __builtin_amdgcn_readlane(ca, ls), vb = __builtin_amdgcn_readlane(cb, ls);
        const int aq = low ? va : vb;
        ca = lane == t ? aq : ca;
        ca = (low && lane == ls) ? at : ca;
        cb = (!low && lane == ls) ? at : cb;
    };

    T lp = (T)0;      // pending multiplier of the previous pivot row
    T nu[NG];         // that row negated, lane-replicated: nu[b] = -u[16 (g + b) + lane % 16]
#pragma unroll
    for (int b = 0; b < NG; ++b) nu[b] = (T)0;
    bool dead = false;
    const T tiny = sizeof(T) == 4 ? (T)1.17549435e-38f : (T)2.2250738585072014e-308;
    const bool near = stride == kXcdStride;
    auto put = [&](unsigned long long *p, unsigned tag, unsigned v) {
        if (near) xstore_near(p, tag, v);
        else xstore(p, tag, v);
    };

    for (int g = 0; g < NG; ++g) {
        sfor<0, 16>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            constexpr int par = k & 1;
            const int j = 16 * g + k;
            if (dead) return;
            const unsigned tag = (unsigned)(k0 + j + 1);
            const unsigned long long tagw = (unsigned long long)tag << 32;
            unsigned long long *X = xb + (size_t)par * PAR;
            // row j staged raw for its publisher (drains during the argmax)
            if (pos == j) {
                blocks_to_lds<T, NG>(s_draw[par], a, g);
                s_dlp[par] = lp;
            }
            // --- 1. argmax of column j
            const T aj = a[0][k];
            const T av = fabs(aj);
            const T cv = (live && pos >= j && av == av) ? av : (T)-1;
            const WaveArgmax<T> wa = wave_argmax(cv);
            const int wl = wa.lane < 64 ? wa.lane : 0;
            if (lane == 0) {
                s_wval[par][wave] = wa.val;
                s_wsv[par][wave] = readlane_t(aj, wl);
                s_wpos[par][wave] = w * TPB + wave * 64 + wl;
            }
            __syncthreads();
            T kv = (T)-1, ks = (T)0;
            int kp = 0;
            if (lane < NW) {
                kv = s_wval[par][lane];
                ks = s_wsv[par][lane];
                kp = s_wpos[par][lane];
            }
            const T gmax = max8(kv);
            const int qw = first_lane(lane < NW && gmax >= (T)0 && kv == gmax);
            const int pwg = qw < NW ? __builtin_amdgcn_readlane(kp, qw) : -1;
            const T psv = readlane_t(ks, qw < NW ? qw : 0);
            // --- 2. publish the candidate and row j, brought up to date
            if (qw < NW && wave == qw) {
                if (lane == wl) blocks_to_lds<T, NG>(s_cand[par], a, g);
                const T lw = readlane_t(lp, wl);
                wave_lds_sync();
                T v = (T)0;
                if (lane < B) {
                    v = s_cand[par][lane];
                    if (j > 0 && lane > j) v = fma(-s_u[par ^ 1][lane], lw, v);
                }
                if (P > 1) {
                    unsigned long long *slot = X + (size_t)w * SLOT;
                    if (lane < B) {
#pragma unroll
                        for (int h = 0; h < PWV; ++h)
                            put(slot + HDR + lane * PWV + h, tag, Words<T>::get(v, h));
                    }
                    if (lane < HW)
                        put(slot + lane, tag, lane < PWV ? Words<T>::get(psv, lane) : (unsigned)pwg);
                } else {
                    if (lane < B) s_u[par][lane] = v;
                    if (lane == 0) {
                        s_p[par] = pwg;
                        s_pv[par] = psv;
                        s_rcp[par] = (T)1 / psv;
                    }
                }
            }
            if (qw >= NW && wave == 0) {  // no candidate in this workgroup
                if (P > 1) {
                    if (lane < HW) put(X + (size_t)w * SLOT + lane, tag, lane < PWV ? 0u : ~0u);
                } else if (lane == 0) {
                    s_p[par] = -1;
                }
            }
            if (w == 0 && wave == DW && lane < B) {
                T v = s_draw[par][lane];
                if (j > 0 && lane > j) v = fma(-s_u[par ^ 1][lane], s_dlp[par], v);
                if (P > 1) {
#pragma unroll
                    for (int h = 0; h < PWV; ++h) put(X + DIAG + lane * PWV + h, tag, Words<T>::get(v, h));
                } else {
                    s_d[par][lane] = v;
                }
            }
            // --- 3. pending update of columns > j, every row, all lanes active
            if (j > 0) {
                sfor<k + 1, 16>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    BcastFma<T>::template one<c>(a[0][c], nu[0], lp);
                });
#pragma unroll
                for (int b = 1; b < NG; ++b)
                    if (b < NG - g) BcastFma<T>::block(a[b], nu[b], lp);
            }
            lp = (T)0;
            if (cmp && wave == 0 && jprev >= 0) compose(jprev, pprev);
            // --- 4. gather (last wave): headers and row j, then the winner's row
            if (P > 1 && wave == GW) {
                bool bad = false;
                unsigned long long hv[HW];
#pragma unroll
                for (int h = 0; h < HW; ++h) hv[h] = lane < P ? xload(X + lane * SLOT + h) : tagw;
                unsigned long long dv = xload(X + DIAG + lane);
                unsigned spins = 0;
                for (;;) {
                    bool stale = (unsigned)(dv >> 32) != tag;
#pragma unroll
                    for (int h = 0; h < HW; ++h) stale |= (unsigned)(hv[h] >> 32) != tag;
                    if (!__ballot(stale)) break;
                    ++spins;
                    if (spins > kSpinLimit ||
                        ((spins & 1023u) == 0 && flag_set(&status[ST_TIMEOUT]))) {
                        bad = true;
                        break;
                    }
#pragma unroll
                    for (int h = 0; h < HW; ++h)
                        if ((unsigned)(hv[h] >> 32) != tag) hv[h] = xload(X + lane * SLOT + h);
                    if ((unsigned)(dv >> 32) != tag) dv = xload(X + DIAG + lane);
                }
                T sval = (T)0;
                int row = -1;
                if (lane < P) {
                    if constexpr (sizeof(T) == 4) {
                        sval = __uint_as_float((unsigned)hv[0]);
                    } else {
                        sval = __longlong_as_double(
                            (long long)(((hv[1] & 0xffffffffull) << 32) | (hv[0] & 0xffffffffull)));
                    }
                    row = (int)(unsigned)hv[PWV];
                }
                const T val = (!bad && lane < P && row >= 0) ? fabs(sval) : (T)-1;
                const WaveArgmax<T> best = wave_argmax(val);
                int p = -1;
                T pv = (T)0;
                unsigned long long uv = tagw;
                if (best.lane < P) {
                    p = __builtin_amdgcn_readlane(row, best.lane);
                    pv = readlane_t(sval, best.lane);
                    uv = xload(X + best.lane * SLOT + HDR + lane);
                }
                const T rcp = (T)1 / pv;  // while the row is in flight
                if (best.lane < P) {
                    spins = 0;
                    while (!bad && __ballot((unsigned)(uv >> 32) != tag)) {
                        ++spins;
                        if (spins > kSpinLimit ||
                            ((spins & 1023u) == 0 && flag_set(&status[ST_TIMEOUT]))) {
                            bad = true;
                            break;
                        }
                        if ((unsigned)(uv >> 32) != tag) uv = xload(X + best.lane * SLOT + HDR + lane);
                    }
                }
                reinterpret_cast<unsigned *>(&s_u[par][0])[lane] = (unsigned)uv;
                reinterpret_cast<unsigned *>(&s_d[par][0])[lane] = (unsigned)dv;
                if (lane == 0) {
                    s_p[par] = bad ? INT_MIN : p;
                    s_pv[par] = pv;
                    s_rcp[par] = rcp;
                    if (bad)
                        __hip_atomic_store(&status[ST_TIMEOUT], 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            __syncthreads();
            // --- 5. interchange, multipliers, column j + 1
            int p = s_p[par];
            if (p == INT_MIN) {  // a bounded wait gave up (uniform)
                dead = true;
                return;
            }
            T piv = s_pv[par], rcp = s_rcp[par];
            const T *prow = s_u[par];
            const T *drow = s_d[par];
            if (p < j || p >= m) {  // no usable candidate (all NaN): keep row j
                p = j;
                prow = drow;
                piv = drow[j];
                rcp = (T)1 / piv;
            }
            jprev = j;
            pprev = p;
            if (fetcher && p >= B && wave == j % GW) {
                if (spend >= 0) {
                    s_rows[spend][lane] = rpiv;
                    if (pfetch && lane == 0) s_pm[spend] = ppiv;
                }
                rpiv = lane < nd ? Wd[(size_t)(k0 + p) * ldw * PWV + lword] : 0u;
                if (pfetch && lane == 0) ppiv = perm[k0 + p];
                spend = B + j;
            }
            const bool normal = fabs(piv) >= tiny && isfinite(piv);
            // no global stores inside the loop: the pivots are kept in LDS
            if (tid == 0) s_piv[j] = (!(piv != (T)0) || !isfinite(piv)) ? -(p + 1) : p;
            if (p != j) {
                if (pos == j) blocks_from_lds<T, NG>(a, prow, g);
                else if (pos == p) blocks_from_lds<T, NG>(a, drow, g);
            }
            if (j + 1 < B) {
#pragma unroll
                for (int b = 0; b < NG; ++b)
                    if (b < NG - g) nu[b] = -prow[16 * (g + b) + (lane & 15)];
                const T u1 = prow[j + 1];
                if (live && pos > j && piv != (T)0) {
                    T l;
                    if (normal) l = a[0][k] * rcp;
                    else l = a[0][k] / piv;
                    a[0][k] = l;
                    lp = l;
                    if constexpr (k + 1 < 16) a[0][k + 1] = fma(-u1, l, a[0][k + 1]);
                    else if constexpr (NG > 1) a[1][0] = fma(-u1, l, a[1][0]);
                }
            } else if (live && pos > j && piv != (T)0) {
                if (normal) a[0][k] = a[0][k] * rcp;
                else a[0][k] = a[0][k] / piv;
            }
        });
        if (dead) break;
        // rotate: the finished block goes last
        T t0[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) t0[e] = a[0][e];
#pragma unroll
        for (int b = 0; b + 1 < NG; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) a[b][e] = a[b + 1][e];
#pragma unroll
        for (int e = 0; e < 16; ++e) a[NG - 1][e] = t0[e];
        const T n0 = nu[0];
#pragma unroll
        for (int b = 0; b + 1 < NG; ++b) nu[b] = nu[b + 1];
        nu[NG - 1] = n0;
    }
    if (dead) return;  // uniform: every thread saw the same gather result
    if (spend >= 0) {
        s_rows[spend][lane] = rpiv;
        if (pfetch && lane == 0) s_pm[spend] = ppiv;
    }
    if (live) {
        using vq = typename Vq<T>::type;
        constexpr int V = Vq<T>::V;
        vq *dst = reinterpret_cast<vq *>(W + (size_t)(k0 + pos) * ldw + k0);
#pragma unroll
        for (int b = 0; b < NG; ++b)
#pragma unroll
            for (int q = 0; q < 16 / V; ++q) {
                vq v;
#pragma unroll
                for (int e = 0; e < V; ++e) v[e] = a[b][q * V + e];
                dst[b * (16 / V) + q] = v;
            }
    }
    __syncthreads();
    if (w == 0 && tid < B) {
        const int v = s_piv[tid];
        ipiv[k0 + tid] = k0 + (v < 0 ? -v - 1 : v);
        if (v < 0) atomicMin(&status[ST_BREAKDOWN], k0 + tid + 1);
    }
    if (!cmp) return;
    __shared__ int s_mv[4 * B];
    __shared__ int s_nmv;
    if (wave == 0) {
        if (jprev >= 0) compose(jprev, pprev);
        const bool ma = lane < B && ca != lane;
        const bool mb = cpos >= 0 && cb != B + lane;
        const unsigned long long ba = __ballot(ma), bb = __ballot(mb);
        const unsigned long long below = (1ull << lane) - 1ull;
        const int na = __popcll(ba), nm = na + __popcll(bb);
        // the rows the slots stand for, for the move list
        const int qa = __shfl(cpos, (ca - B) & 63), qb = __shfl(cpos, (cb - B) & 63);
        const bool lst = pmv != nullptr && w == 0;
        if (ma) {
            const int i = __popcll(ba & below);
            s_mv[2 * i] = k0 + lane;
            s_mv[2 * i + 1] = ca;
            if (lst) {
                pmv[1 + 2 * i] = k0 + lane;
                pmv[2 + 2 * i] = k0 + (ca < B ? ca : qa);
            }
        }
        if (mb) {
            const int i = na + __popcll(bb & below);
            s_mv[2 * i] = k0 + cpos;
            s_mv[2 * i + 1] = cb;
            if (lst) {
                pmv[1 + 2 * i] = k0 + cpos;
                pmv[2 + 2 * i] = k0 + (cb < B ? cb : qb);
            }
        }
        if (lane == 0) {
            s_nmv = nm;
            if (lst) pmv[0] = nm;
        }
    }
    if (!swp) return;
    __syncthreads();
    const int count = s_nmv;
    if (perm && w == 0 && tid < count) perm[s_mv[2 * tid]] = s_pm[s_mv[2 * tid + 1]];
    for (int e = tid; e < count * nd; e += TPB) {
        const int mq = e / nd, d = e % nd;
        const int c = lc0 + d / PWV;
        const int col = sc0 + c + (c >= nleft ? B : 0);
        reinterpret_cast<unsigned *>(W + (size_t)s_mv[2 * mq] * ldw + col)[d % PWV] =
            s_rows[s_mv[2 * mq + 1]][d];
    }
}

template <typename T> struct PanelWidth;
template <> struct PanelWidth<float> { static constexpr int v = kPanelBF; };
template <> struct PanelWidth<double> { static constexpr int v = kPanelBD; };

template <typename T>
hipError_t launch_panel(T *W, int ldw, int k0, int m, int *ipiv, unsigned long long *xb,
                        int *status, hipStream_t s, int *perm, int sc0, int sc1, int *pmoves) {
    constexpr int B = PanelWidth<T>::v;
    const int P = (m + kPanelRowsPerWG - 1) / kPanelRowsPerWG;
    if (P < 1 || P > kPanelMaxWG || m < B) return hipErrorInvalidValue;
    const bool swaps = perm != nullptr || sc1 > sc0;
    if (swaps && (sc0 > k0 || sc1 < k0 + B)) return hipErrorInvalidValue;
    // workers are dealt round-robin over the 8 XCDs: with stride 8 all of them
    // land on one XCD (32 CUs) and exchange through its L2
    const int stride = P == 1 ? 1 : (P <= 32 ? kXcdStride : kXcdStride / 2);
    // the interchanges ride in the panel launch when each workgroup's slice
    // is at most 64 words wide; otherwise they get a launch of their own
    const bool fuse = swaps && (sc1 - sc0 - B + P - 1) / P * (int)(sizeof(T) / 4) <= 64;
    k_panel<T, B><<<dim3(P * stride), dim3(kPanelTPB), 0, s>>>(
        W, ldw, k0, m, ipiv, xb, status, P, stride, fuse ? perm : nullptr, fuse ? sc0 : 0,
        fuse ? sc1 : 0, pmoves);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !swaps || fuse) return e;
    return launch_row_swaps<T>(ipiv, k0, B, k0 + m, perm, W, ldw, sc0, sc1, k0, k0 + B, nullptr,
                               s);
}
template hipError_t launch_panel<float>(float *, int, int, int, int *, unsigned long long *,
                                        int *, hipStream_t, int *, int, int, int *);
template hipError_t launch_panel<double>(double *, int, int, int, int *, unsigned long long *,
                                         int *, hipStream_t, int *, int, int, int *);

// ======================================================================
// Row interchanges outside the panel
// ======================================================================
// Row interchanges of pivots ipiv[k0 .. k0+cnt-1] applied in one launch:
// every workgroup composes the swaps into a move list in LDS (cur[i] = the
// row whose content ends at row k0 + i), then moves the rows of its CW
// columns of [c0, c1) minus [skip0, skip1) (staged in LDS, so the moves may
// form cycles).  Workgroup 0 also applies the moves to perm (when given).
constexpr int kSwapRegs = 8;  // moved values held in registers per thread (128 moves x 16 columns)
template <typename T, int CW>
__global__ __launch_bounds__(256) void k_row_swaps(const int *__restrict__ ipiv, int k0, int cnt,
                                                   int npad, int *__restrict__ perm,
                                                   T *__restrict__ W, int ldw, int c0, int nleft,
                                                   int gap, int ncols) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int m = npad - k0;
    int *cur = reinterpret_cast<int *>(smem);                 // m
    int *mv = cur + m;                                        // 2 * (2 * cnt)
    T *buf = reinterpret_cast<T *>(mv + 4 * cnt + 4);        // 2 * cnt * CW
    __shared__ int s_count;
    __shared__ int s_pv[512];  // the block's pivots, relative to k0 (cnt <= 512)
    for (int i = threadIdx.x; i < m; i += 256) cur[i] = i;
    for (int i = threadIdx.x; i < cnt; i += 256) {
        int q = ipiv[k0 + i] - k0;
        if (q < i || q >= m) q = i;  // never index outside [k0, npad)
        s_pv[i] = q;
    }
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        // the composition is sequential; its operands are all in LDS
        for (int s = 0; s < cnt; ++s) {
            const int q = s_pv[s];
            if (q != s) {
                const int t = cur[s];
                cur[s] = cur[q];
                cur[q] = t;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += 256) {
        const int src = cur[i];
        if (src != i) {
            const int q = atomicAdd(&s_count, 1);
            mv[2 * q] = k0 + i;
            mv[2 * q + 1] = k0 + src;
        }
    }
    __syncthreads();
    const int count = s_count;
    // the moved values of this workgroup's columns and (workgroup 0) of perm
    // are read in one round, all before any is written (so moves may form
    // cycles): one memory round trip instead of one per array
    const int lc0 = blockIdx.x * CW;
    const bool do_perm = perm && blockIdx.x == 0;
    if (count * CW <= kSwapRegs * 256) {
        T v[kSwapRegs];
        int keep[kSwapRegs / 2];
#pragma unroll
        for (int u = 0; u < kSwapRegs; ++u) {
            const int e = threadIdx.x + u * 256;
            const int q = e / CW, lc = lc0 + e % CW;
            v[u] = (T)0;
            if (e < count * CW && lc < ncols)
                v[u] = W[(size_t)mv[2 * q + 1] * ldw + c0 + lc + (lc >= nleft ? gap : 0)];
        }
#pragma unroll
        for (int u = 0; u < kSwapRegs / 2; ++u) {
            const int q = threadIdx.x + u * 256;
            keep[u] = (do_perm && q < count) ? perm[mv[2 * q + 1]] : 0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kSwapRegs; ++u) {
            const int e = threadIdx.x + u * 256;
            const int q = e / CW, lc = lc0 + e % CW;
            if (e < count * CW && lc < ncols)
                W[(size_t)mv[2 * q] * ldw + c0 + lc + (lc >= nleft ? gap : 0)] = v[u];
        }
#pragma unroll
        for (int u = 0; u < kSwapRegs / 2; ++u) {
            const int q = threadIdx.x + u * 256;
            if (do_perm && q < count) perm[mv[2 * q]] = keep[u];
        }
        return;
    }
    if (do_perm) {
        int keep[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = threadIdx.x + u * 256;
            keep[u] = q < count ? perm[mv[2 * q + 1]] : 0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = threadIdx.x + u * 256;
            if (q < count) perm[mv[2 * q]] = keep[u];
        }
    }
    for (int e = threadIdx.x; e < count * CW; e += 256) {
        const int q = e / CW, cc = e % CW;
        const int lc = lc0 + cc;
        if (lc < ncols) {
            const int col = c0 + lc + (lc >= nleft ? gap : 0);
            buf[e] = W[(size_t)mv[2 * q + 1] * ldw + col];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < count * CW; e += 256) {
        const int q = e / CW, cc = e % CW;
        const int lc = lc0 + cc;
        if (lc < ncols) {
            const int col = c0 + lc + (lc >= nleft ? gap : 0);
            W[(size_t)mv[2 * q] * ldw + col] = buf[e];
        }
    }
}

// Wide blocks of pivots (more than kSwapsFused): the composition is long and
// sequential, so it runs once, in k_swaps_compose (one workgroup), which
// writes moves = {count, pad, (dst, src)...} to global memory (after the
// swaps, row dst holds what row src held before); k_rows_apply then moves
// the rows of every column, CW columns per workgroup, through LDS.
__global__ __launch_bounds__(1024) void k_swaps_compose(const int *__restrict__ ipiv, int k0,
                                                        int cnt, int npad, int *__restrict__ perm,
                                                        int *__restrict__ moves) {
    extern __shared__ int cur[];
    __shared__ int s_count;
    __shared__ int s_pv[kMaxOuterBlock];
    __shared__ int s_dst[2 * kMaxOuterBlock], s_src[2 * kMaxOuterBlock];
    const int m = npad - k0;
    for (int i = threadIdx.x; i < m; i += blockDim.x) cur[i] = i;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        int q = ipiv[k0 + i] - k0;
        if (q < i || q >= m) q = i;  // never index outside [k0, npad)
        s_pv[i] = q;
    }
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int s = 0; s < cnt; ++s) {
            const int q = s_pv[s];
            if (q != s) {
                const int t = cur[s];
                cur[s] = cur[q];
                cur[q] = t;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const int src = cur[i];
        if (src != i) {
            const int q = atomicAdd(&s_count, 1);
            s_dst[q] = k0 + i;
            s_src[q] = k0 + src;
        }
    }
    __syncthreads();
    const int count = s_count;  // <= 2 cnt <= 2 blockDim.x
    int keep[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int t = threadIdx.x + h * blockDim.x;
        if (t < count) {
            moves[2 + 2 * t] = s_dst[t];
            moves[3 + 2 * t] = s_src[t];
            if (perm) keep[h] = perm[s_src[t]];
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int t = threadIdx.x + h * blockDim.x;
        if (perm && t < count) perm[s_dst[t]] = keep[h];
    }
    if (threadIdx.x == 0) moves[0] = count;
}

template <typename T, int CW>
__global__ __launch_bounds__(256) void k_rows_apply(T *__restrict__ W, int ldw,
                                                    const int *__restrict__ moves, int c0,
                                                    int nleft, int gap, int ncols, int mvmax) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    T *buf = reinterpret_cast<T *>(smem);                             // mvmax * CW values
    int *smv = reinterpret_cast<int *>(buf + (size_t)mvmax * CW);    // the move list
    const int count = min(moves[0], mvmax);
    for (int i = threadIdx.x; i < 2 * count; i += 256) smv[i] = moves[2 + i];
    __syncthreads();
    const int lc0 = blockIdx.x * CW;
    // U loads in flight per thread before their LDS writes (one at a time
    // would put a memory latency per element on the chain)
    constexpr int U = 8;
    for (int e0 = threadIdx.x; e0 < count * CW; e0 += 256 * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * 256;
            const int q = e / CW, lc = lc0 + e % CW;
            v[u] = (T)0;
            if (e < count * CW && lc < ncols)
                v[u] = W[(size_t)smv[2 * q + 1] * ldw + c0 + lc + (lc >= nleft ? gap : 0)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * 256;
            if (e < count * CW) buf[e] = v[u];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < count * CW; e += 256) {
        const int q = e / CW, lc = lc0 + e % CW;
        if (lc < ncols) W[(size_t)smv[2 * q] * ldw + c0 + lc + (lc >= nleft ? gap : 0)] = buf[e];
    }
}

template <typename T>
hipError_t launch_row_swaps(const int *ipiv, int k0, int cnt, int npad, int *perm, T *W, int ldw,
                            int c0, int c1, int skip0, int skip1, int *moves, hipStream_t s) {
    constexpr int CW = sizeof(T) == 4 ? 16 : 8;
    constexpr size_t kMaxLds = 152 * 1024;  // of the 160 KiB, leaving room for static LDS
    if (cnt > kMaxOuterBlock) return hipErrorInvalidValue;
    if (skip0 < c0) skip0 = c0;
    if (skip1 > c1) skip1 = c1;
    if (skip1 < skip0) skip1 = skip0;
    const int nleft = skip0 - c0;
    const int gap = skip1 - skip0;
    int ncols = (c1 - c0) - gap;
    const int m = npad - k0;
    if (cnt > kSwapsFused && moves) {
        // compose once, then apply in a second launch
        const size_t lds_c = (size_t)m * sizeof(int);
        const size_t lds_a = (size_t)2 * cnt * (CW * sizeof(T) + 2 * sizeof(int));
        if (lds_c > kMaxLds - 24 * 1024 || lds_a > kMaxLds) return hipErrorInvalidValue;
        static bool attr2_done = false;
        if (!attr2_done) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_swaps_compose),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)(kMaxLds - 24 * 1024));
            if (e == hipSuccess)
                e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rows_apply<T, CW>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
            if (e != hipSuccess) return e;
            attr2_done = true;
        }
        k_swaps_compose<<<dim3(1), dim3(1024), lds_c, s>>>(ipiv, k0, cnt, npad, perm, moves);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || ncols <= 0) return e;
        k_rows_apply<T, CW><<<dim3((ncols + CW - 1) / CW), dim3(256), lds_a, s>>>(
            W, ldw, moves, c0, nleft, gap, ncols, 2 * cnt);
        return hipGetLastError();
    }
    const size_t lds = align_up((size_t)(m + 4 * cnt + 4) * 4, 16) + (size_t)2 * cnt * CW * sizeof(T);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_row_swaps<T, CW>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    if (ncols < 0) ncols = 0;
    // at least one workgroup, so that perm is updated even with no columns
    const int grid = ncols > 0 ? (ncols + CW - 1) / CW : 1;
    k_row_swaps<T, CW><<<dim3(grid), dim3(256), lds, s>>>(ipiv, k0, cnt, npad, perm, W, ldw, c0,
                                                          nleft, gap, ncols);
    return hipGetLastError();
}
hipError_t launch_swaps_compose(const int *ipiv, int k0, int cnt, int npad, int *perm, int *moves,
                                hipStream_t s) {
    constexpr size_t kMaxLds = 152 * 1024;
    if (cnt > kMaxOuterBlock || cnt < 0 || k0 < 0 || k0 > npad) return hipErrorInvalidValue;
    const size_t lds_c = (size_t)(npad - k0) * sizeof(int);
    if (lds_c > kMaxLds - 24 * 1024) return hipErrorInvalidValue;
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_swaps_compose),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(kMaxLds - 24 * 1024));
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    k_swaps_compose<<<dim3(1), dim3(1024), lds_c, s>>>(ipiv, k0, cnt, npad, perm, moves);
    return hipGetLastError();
}

// The composition of a block's interchanges from its panels' move lists:
// cur[i] = the row whose content ends at row k0 + i, one parallel round per
// list (all sources read before any destination is written), then the moved
// rows gathered into one list as k_swaps_compose writes it.
__global__ __launch_bounds__(1024) void k_swaps_merge(const int *__restrict__ plist, int np,
                                                      int stride, int k0, int npad,
                                                      int *__restrict__ moves) {
    extern __shared__ int cur[];
    __shared__ int s_count;
    const int m = npad - k0;
    for (int i = threadIdx.x; i < m; i += blockDim.x) cur[i] = i;
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    for (int r = 0; r < np; ++r) {
        const int *L = plist + (size_t)r * stride;
        const int cnt = L[0];
        int d = -1, v = 0;
        if (threadIdx.x < cnt && threadIdx.x < 2 * kPanelBF) {
            const int dd = L[1 + 2 * threadIdx.x] - k0, ss = L[2 + 2 * threadIdx.x] - k0;
            if (dd >= 0 && dd < m && ss >= 0 && ss < m) {  // never index outside [k0, npad)
                d = dd;
                v = cur[ss];
            }
        }
        __syncthreads();
        if (d >= 0) cur[d] = v;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const int src = cur[i];
        if (src != i) {
            const int q = atomicAdd(&s_count, 1);
            if (q < 2 * kMaxOuterBlock) {
                moves[2 + 2 * q] = k0 + i;
                moves[3 + 2 * q] = k0 + src;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) moves[0] = min(s_count, 2 * kMaxOuterBlock);
}

hipError_t launch_swaps_merge(const int *plist, int np, int stride, int k0, int npad, int *moves,
                              hipStream_t s) {
    constexpr size_t kMaxLds = 152 * 1024;
    if (np < 0 || k0 < 0 || k0 > npad || stride < kPanelMovesInts) return hipErrorInvalidValue;
    const size_t lds_c = (size_t)(npad - k0) * sizeof(int);
    if (lds_c > kMaxLds - 24 * 1024) return hipErrorInvalidValue;
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_swaps_merge),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(kMaxLds - 24 * 1024));
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    k_swaps_merge<<<dim3(1), dim3(1024), lds_c, s>>>(plist, np, stride, k0, npad, moves);
    return hipGetLastError();
}

template <typename T, int CW>
hipError_t rows_apply(T *W, int ldw, const int *moves, int cnt, int c0, int nleft, int gap,
                      int ncols, hipStream_t s) {
    constexpr size_t kMaxLds = 152 * 1024;
    const size_t lds_a = (size_t)2 * cnt * (CW * sizeof(T) + 2 * sizeof(int));
    if (lds_a > kMaxLds) return hipErrorInvalidValue;
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rows_apply<T, CW>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    k_rows_apply<T, CW><<<dim3((ncols + CW - 1) / CW), dim3(256), lds_a, s>>>(
        W, ldw, moves, c0, nleft, gap, ncols, 2 * cnt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_swaps_apply(T *W, int ldw, const int *moves, int cnt, int c0, int c1, int skip0,
                              int skip1, hipStream_t s) {
    constexpr int CW = sizeof(T) == 4 ? 16 : 8;
    if (cnt > kMaxOuterBlock || cnt < 0) return hipErrorInvalidValue;
    if (skip0 < c0) skip0 = c0;
    if (skip1 > c1) skip1 = c1;
    if (skip1 < skip0) skip1 = skip0;
    const int nleft = skip0 - c0;
    const int gap = skip1 - skip0;
    const int ncols = (c1 - c0) - gap;
    if (ncols <= 0) return hipSuccess;
    // a narrow range (the next block's columns, on the critical path) in
    // slices of a quarter the width, so that it spreads over more compute units
    if (ncols <= 2048) return rows_apply<T, CW / 4>(W, ldw, moves, cnt, c0, nleft, gap, ncols, s);
    return rows_apply<T, CW>(W, ldw, moves, cnt, c0, nleft, gap, ncols, s);
}
template hipError_t launch_swaps_apply<float>(float *, int, const int *, int, int, int, int, int,
                                              hipStream_t);
template hipError_t launch_swaps_apply<double>(double *, int, const int *, int, int, int, int, int,
                                               hipStream_t);

template hipError_t launch_row_swaps<float>(const int *, int, int, int, int *, float *, int, int,
                                            int, int, int, int *, hipStream_t);
template hipError_t launch_row_swaps<double>(const int *, int, int, int, int *, double *, int, int,
                                             int, int, int, int *, hipStream_t);

// ======================================================================
// Triangular solve with a unit lower diagonal block (LDS-staged)
// ======================================================================
// X[0:DB, :] = L^{-1} X[0:DB, :] for the DB x DB unit lower L; one thread
// per column of X, the block of L in LDS (read by broadcast).
// X = L^{-1} X for the unit lower DB x DB diagonal block L (row-major, ld
// ldl) and ncols columns of X: one wave per column, lane r holding row r of
// L in registers; the solved value of row k reaches the other lanes by
// readlane, so the DB dependent steps touch no memory.
template <typename T, int DB>
__global__ __launch_bounds__(256) void k_trsm_diag(const T *__restrict__ L, int ldl,
                                                   T *__restrict__ X, int ldx, int ncols) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = blockIdx.x * 4 + wave;
    if (col >= ncols) return;
    const bool act = lane < DB;
    T lrow[DB];
#pragma unroll
    for (int k = 0; k < DB; ++k) lrow[k] = (act && k < lane) ? L[(size_t)lane * ldl + k] : (T)0;
    T x = act ? X[(size_t)lane * ldx + col] : (T)0;
#pragma unroll
    for (int k = 0; k < DB - 1; ++k) {
        const T xk = readlane_t(x, k);
        if (lane > k) x -= lrow[k] * xk;
    }
    if (act) X[(size_t)lane * ldx + col] = x;
}

// Same operation for many columns: one thread per column, L staged once per
// 64 columns in LDS (the per-wave register copy above would re-read L for
// every four columns).
template <typename T, int DB>
__global__ __launch_bounds__(64) void k_trsm_diag_wide(const T *__restrict__ L, int ldl,
                                                       T *__restrict__ X, int ldx, int ncols) {
    __shared__ T sL[DB][DB + 1];
    const int t = threadIdx.x;
    const int col = blockIdx.x * 64 + t;
    // the column is requested before L is staged, so the two loads overlap
    T x[DB];
#pragma unroll
    for (int i = 0; i < DB; ++i) x[i] = col < ncols ? X[(size_t)i * ldx + col] : (T)0;
    for (int i = 0; i < DB; ++i)
        for (int c = t; c < DB; c += 64) sL[i][c] = L[(size_t)i * ldl + c];
    __syncthreads();
    if (col >= ncols) return;
#pragma unroll
    for (int k = 0; k < DB; ++k) {
#pragma unroll
        for (int i = k + 1; i < DB; ++i) x[i] -= sL[i][k] * x[k];
    }
#pragma unroll
    for (int i = 0; i < DB; ++i) X[(size_t)i * ldx + col] = x[i];
}

template <typename T>
hipError_t launch_trsm_diag(const T *Ldiag, int ldl, T *X, int ldx, int ncols, hipStream_t s) {
    if (ncols <= 0) return hipSuccess;
    constexpr int DB = PanelWidth<T>::v;
    if (ncols <= 1024)
        k_trsm_diag<T, DB><<<dim3((ncols + 3) / 4), dim3(256), 0, s>>>(Ldiag, ldl, X, ldx, ncols);
    else
        k_trsm_diag_wide<T, DB><<<dim3((ncols + 63) / 64), dim3(64), 0, s>>>(Ldiag, ldl, X, ldx,
                                                                             ncols);
    return hipGetLastError();
}
template hipError_t launch_trsm_diag<float>(const float *, int, float *, int, int, hipStream_t);
template hipError_t launch_trsm_diag<double>(const double *, int, double *, int, int, hipStream_t);

// ======================================================================
// GEMM C -= A B (row-major) on MFMA, FP32 or FP64
// ======================================================================
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Output layout of the 16x16x4 MFMAs: element v of lane l holds
// D[row(l, v)][l % 16], row = 4*(l/16) + v for f32 and 4*v + l/16 for f64.
template <> struct Mfma<float> {
    typedef f32x4 acc_t;
    __device__ static int row(int lane, int v) { return (lane >> 4) * 4 + v; }
    __device__ static acc_t mac(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    typedef f64x4 acc_t;
    __device__ static int row(int lane, int v) { return v * 4 + (lane >> 4); }
    __device__ static acc_t mac(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// 64x64 output tile per workgroup, 4 waves of 32x32, K step 16.
// 16x16x4 operand layout: lane l supplies A[l%16][l/16] and B[l/16][l%16].
// Tile of a GEMM workgroup.  spare_xcd0 = 0: the 2-D grid position.
// spare_xcd0 = 1: a 1-D grid whose workgroups b with b % 8 == 0 (dealt to
// XCD 0 by the round-robin dispatch) do nothing, so that a panel kernel
// running concurrently on XCD 0 keeps its compute units; the other
// workgroups take the tiles in order.  Returns false for no tile.
__device__ __forceinline__ bool tile_of(int spare_xcd0, int tiles_x, int tiles_y, int &tx, int &ty) {
    if (!spare_xcd0) return true;
    const int b = blockIdx.x;
    if ((b & 7) == 0) return false;
    const int t = (b >> 3) * 7 + (b & 7) - 1;
    if (t >= tiles_x * tiles_y) return false;
    ty = t / tiles_x;
    tx = t - ty * tiles_x;
    return true;
}
inline dim3 gemm_grid(int spare_xcd0, int tiles_x, int tiles_y) {
    if (!spare_xcd0) return dim3(tiles_x, tiles_y);
    const long t = (long)tiles_x * tiles_y;
    return dim3((unsigned)((t + 6) / 7 * 8));
}

// TB: B is given transposed (Bm is N x K row-major, as L21 for the Cholesky
// update C -= L21 L21^T).  TA: A is given transposed (A is K x M row-major,
// as the off-diagonal blocks of the transposed triangular solves).
// lower != 0: only tiles that touch the lower triangle (col <= row) of C
// are computed.
// Split K (gridDim.z = S > 1): workgroup z takes the z-th slice of K (a
// multiple of BK); slice 0 updates C in place, slice z > 0 stores its
// -A_z B_z into P + (z - 1) pstride (leading dimension ldc), for a
// following reduction.
template <typename T, bool TB, bool TA = false>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const T *__restrict__ A, int lda,
                                              const T *__restrict__ Bm, int ldb, T *__restrict__ C,
                                              int ldc, int lower, int spare_xcd0,
                                              T *__restrict__ P = nullptr, size_t pstride = 0) {
    constexpr int BM = 64, BN = 64, BK = 16;
    const int nsplit = gridDim.z, z = blockIdx.z;
    int kb = 0, ke = K;
    if (nsplit > 1) {
        const int kc = (K + nsplit * BK - 1) / (nsplit * BK) * BK;
        kb = z * kc;
        ke = kb + kc < K ? kb + kc : K;
    }
    __shared__ T sA[BK][BM + 4];
    __shared__ T sB[BK][BN + 4];
    using acc_t = typename Mfma<T>::acc_t;
    int tx = blockIdx.x, ty = blockIdx.y;
    if (!tile_of(spare_xcd0, (N + BN - 1) / BN, (M + BM - 1) / BM, tx, ty)) return;
    const int m0 = ty * BM, n0 = tx * BN;
    if (lower && n0 > m0 + BM - 1) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    // slice 0 starts its accumulators from C, the others from zero; A is
    // negated on its way into LDS, so the epilogue only stores (C, or the
    // slice's -A_z B_z into P); the next K slab is read into registers while
    // the current one is multiplied
    acc_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 32 + i * 16 + Mfma<T>::row(lane, v);
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                acc[i][j][v] = (z == 0 && row < M && col < N) ? C[(size_t)row * ldc + col] : (T)0;
            }
    T ra[4], rb[4];
    auto load = [&](int k0) {
        if constexpr (TA) {
            const int kk = tid >> 4, r = (tid & 15) * 4;
            const int gk = k0 + kk;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gr = m0 + r + q;
                ra[q] = (gk < ke && gr < M) ? A[(size_t)gk * lda + gr] : (T)0;
            }
        } else {
            const int r = tid >> 2, kk = (tid & 3) * 4;
            const int gr = m0 + r;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gk = k0 + kk + q;
                ra[q] = (gr < M && gk < ke) ? A[(size_t)gr * lda + gk] : (T)0;
            }
        }
        if constexpr (TB) {
            const int c = tid >> 2, kk = (tid & 3) * 4;
            const int gc = n0 + c;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gk = k0 + kk + q;
                rb[q] = (gc < N && gk < ke) ? Bm[(size_t)gc * ldb + gk] : (T)0;
            }
        } else {
            const int kk = tid >> 4, c = (tid & 15) * 4;
            const int gk = k0 + kk;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gc = n0 + c + q;
                rb[q] = (gk < ke && gc < N) ? Bm[(size_t)gk * ldb + gc] : (T)0;
            }
        }
    };
    if (kb < ke) load(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
        if constexpr (TA) {
            const int kk = tid >> 4, r = (tid & 15) * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) sA[kk][r + q] = -ra[q];
        } else {
            const int r = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) sA[kk + q][r] = -ra[q];
        }
        if constexpr (TB) {
            const int c = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) sB[kk + q][c] = rb[q];
        } else {
            const int kk = tid >> 4, c = (tid & 15) * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) sB[kk][c + q] = rb[q];
        }
        __syncthreads();
        if (k0 + BK < ke) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + (lane >> 4);
            const T a0 = sA[kr][wm * 32 + (lane & 15)];
            const T a1 = sA[kr][wm * 32 + 16 + (lane & 15)];
            const T b0 = sB[kr][wn * 32 + (lane & 15)];
            const T b1 = sB[kr][wn * 32 + 16 + (lane & 15)];
            acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
            acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
            acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
            acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 32 + i * 16 + Mfma<T>::row(lane, v);
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row < M && col < N) {
                    if (z == 0) C[(size_t)row * ldc + col] = acc[i][j][v];
                    else P[(size_t)(z - 1) * pstride + (size_t)row * ldc + col] = acc[i][j][v];
                }
            }
}

// Large-tile GEMM C -= A B (row-major, no transposes) for the big trailing
// updates: 128 x 128 output tile per workgroup, 4 waves of 64 x 64 (4 x 4
// MFMA 16x16x4 blocks each), K step BK with the next K slab prefetched into
// registers while the current one is multiplied out of LDS, and stored into
// the second LDS buffer (one barrier per K slab).  LDS pitches
// make the MFMA operand reads conflict-free: A is kept [m][k] with pitch
// BK + 4, B [k][n] with pitch 128 + 16.  The accumulators start from C and
// A is negated on its way into LDS, so the epilogue only stores.
template <typename T, int BK>
__global__ __launch_bounds__(256) void k_gemm_big(int M, int N, int K, const T *__restrict__ A,
                                                  int lda, const T *__restrict__ Bm, int ldb,
                                                  T *__restrict__ C, int ldc, int lower,
                                                  int spare_xcd0) {
    constexpr int BM = 128, BN = 128, PA = BK + 4, PB = BN + 16;
    constexpr int V = 16 / sizeof(T);                 // elements per 16-byte load
    constexpr int NLA = BM * BK / V / 256;            // A vectors per thread per slab
    constexpr int NLB = BK * BN / V / 256;            // B vectors per thread per slab
    typedef T vec_t __attribute__((ext_vector_type(V)));
    // two LDS buffers: the next slab is stored into one while the other is
    // read, so each slab costs one barrier
    __shared__ __attribute__((aligned(16))) T sA2[2][BM * PA];
    __shared__ __attribute__((aligned(16))) T sB2[2][BK * PB];
    using acc_t = typename Mfma<T>::acc_t;
    int tx = blockIdx.x, ty = blockIdx.y;
    if (!tile_of(spare_xcd0, (N + BN - 1) / BN, (M + BM - 1) / BM, tx, ty)) return;
    const int m0 = ty * BM, n0 = tx * BN;
    if (lower && n0 > m0 + BM - 1) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    // the accumulators start from the C tile (requested before the first K
    // slab, so its latency overlaps the operand loads) and the MFMAs add
    // (-A) B: the epilogue is a plain store, no read-modify-write of C
    acc_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 64 + i * 16 + Mfma<T>::row(lane, v);
                const int col = n0 + wn * 64 + j * 16 + (lane & 15);
                acc[i][j][v] = (row < M && col < N) ? C[(size_t)row * ldc + col] : (T)0;
            }
    vec_t ra[NLA], rb[NLB];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NLA; ++q) {
            const int e = tid + q * 256;            // vector index in the BM x BK slab
            const int r = e / (BK / V), kv = (e % (BK / V)) * V;
            const int gr = m0 + r;
            if (gr < M && k0 + kv + V <= K) {
                ra[q] = *reinterpret_cast<const vec_t *>(A + (size_t)gr * lda + k0 + kv);
            } else {
#pragma unroll
                for (int t = 0; t < V; ++t)
                    ra[q][t] = (gr < M && k0 + kv + t < K) ? A[(size_t)gr * lda + k0 + kv + t] : (T)0;
            }
        }
#pragma unroll
        for (int q = 0; q < NLB; ++q) {
            const int e = tid + q * 256;            // vector index in the BK x BN slab
            const int kr = e / (BN / V), nv = (e % (BN / V)) * V;
            const int gk = k0 + kr, gc = n0 + nv;
            if (gk < K && gc + V <= N) {
                rb[q] = *reinterpret_cast<const vec_t *>(Bm + (size_t)gk * ldb + gc);
            } else {
#pragma unroll
                for (int t = 0; t < V; ++t)
                    rb[q][t] = (gk < K && gc + t < N) ? Bm[(size_t)gk * ldb + gc + t] : (T)0;
            }
        }
    };
    auto store = [&](int buf) {
        T *sA = sA2[buf];
        T *sB = sB2[buf];
#pragma unroll
        for (int q = 0; q < NLA; ++q) {
            const int e = tid + q * 256;
            const int r = e / (BK / V), kv = (e % (BK / V)) * V;
            *reinterpret_cast<vec_t *>(&sA[r * PA + kv]) = -ra[q];
        }
#pragma unroll
        for (int q = 0; q < NLB; ++q) {
            const int e = tid + q * 256;
            const int kr = e / (BN / V), nv = (e % (BN / V)) * V;
            *reinterpret_cast<vec_t *>(&sB[kr * PB + nv]) = rb[q];
        }
    };
    // A, B row-major with 16-byte aligned rows are required for the vector
    // loads; the launcher checks lda, ldb and the base pointers
    load(0);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < K; k0 += BK) {
        const bool more = k0 + BK < K;
        if (more) load(k0 + BK);
        const T *sA = sA2[cur];
        const T *sB = sB2[cur];
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + (lane >> 4);
            T a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sA[(wm * 64 + i * 16 + (lane & 15)) * PA + kr];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = sB[kr * PB + wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<T>::mac(a[i], b[j], acc[i][j]);
        }
        // the other buffer was last read before the previous barrier
        if (more) store(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 64 + i * 16 + Mfma<T>::row(lane, v);
                const int col = n0 + wn * 64 + j * 16 + (lane & 15);
                if (row < M && col < N) C[(size_t)row * ldc + col] = acc[i][j][v];
            }
}

template <typename T>
hipError_t launch_gemm(int M, int N, int K, const T *A, int lda, const T *B, int ldb, T *C,
                       int ldc, hipStream_t s, int transb, int lower, int transa, int spare_xcd0) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    constexpr int V = 16 / sizeof(T);
    const bool aligned = lda % V == 0 && ldb % V == 0 &&
                         (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
                         (reinterpret_cast<uintptr_t>(B) & 15) == 0;
    if constexpr (sizeof(T) == 4) {
        // (for FP64 the 64 x 64 kernel below measured faster)
        if (!transa && !transb && aligned && M >= 256 && N >= 256) {
            const dim3 g = gemm_grid(spare_xcd0, (N + 127) / 128, (M + 127) / 128);
            k_gemm_big<T, 32><<<g, dim3(256), 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, lower,
                                                      spare_xcd0);
            return hipGetLastError();
        }
    }
    const dim3 grid = gemm_grid(spare_xcd0, (N + 63) / 64, (M + 63) / 64);
    if (transa && transb)
        k_gemm<T, true, true><<<grid, dim3(256), 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, lower,
                                                         spare_xcd0);
    else if (transa)
        k_gemm<T, false, true><<<grid, dim3(256), 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, lower,
                                                          spare_xcd0);
    else if (transb)
        k_gemm<T, true><<<grid, dim3(256), 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, lower,
                                                   spare_xcd0);
    else
        k_gemm<T, false><<<grid, dim3(256), 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, lower,
                                                    spare_xcd0);
    return hipGetLastError();
}
template hipError_t launch_gemm<float>(int, int, int, const float *, int, const float *, int,
                                       float *, int, hipStream_t, int, int, int, int);
template hipError_t launch_gemm<double>(int, int, int, const double *, int, const double *, int,
                                        double *, int, hipStream_t, int, int, int, int);

// C[i][j] += sum_{z < nparts} P[z][i][j] (M x N, leading dimension ldc)
template <typename T>
__global__ __launch_bounds__(256) void k_splitk_reduce(int M, int N, T *__restrict__ C, int ldc,
                                                       const T *__restrict__ P, size_t pstride,
                                                       int nparts) {
    const size_t total = (size_t)M * N;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (size_t)gridDim.x * 256) {
        const int i = (int)(e / N), j = (int)(e % N);
        const size_t off = (size_t)i * ldc + j;
        T acc = C[off];
        for (int z = 0; z < nparts; ++z) acc += P[(size_t)z * pstride + off];
        C[off] = acc;
    }
}

template <typename T>
hipError_t launch_gemm_splitk(int M, int N, int K, const T *A, int lda, const T *B, int ldb,
                              T *C, int ldc, int transb, int transa, T *P, int nsplit,
                              hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    if (nsplit <= 1 || !P)
        return launch_gemm<T>(M, N, K, A, lda, B, ldb, C, ldc, s, transb, 0, transa, 0);
    const size_t pstride = (size_t)M * ldc;
    const dim3 grid((N + 63) / 64, (M + 63) / 64, nsplit);
    if (transa && transb)
        k_gemm<T, true, true><<<grid, dim3(256), 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, 0, 0, P,
                                                         pstride);
    else if (transa)
        k_gemm<T, false, true><<<grid, dim3(256), 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, 0, 0, P,
                                                          pstride);
    else if (transb)
        k_gemm<T, true><<<grid, dim3(256), 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, 0, 0, P,
                                                   pstride);
    else
        k_gemm<T, false><<<grid, dim3(256), 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, 0, 0, P,
                                                    pstride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t total = (size_t)M * N;
    const unsigned rgrid = (unsigned)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    k_splitk_reduce<T><<<rgrid, dim3(256), 0, s>>>(M, N, C, ldc, P, pstride, nsplit - 1);
    return hipGetLastError();
}
template hipError_t launch_gemm_splitk<double>(int, int, int, const double *, int, const double *,
                                               int, double *, int, int, int, double *, int,
                                               hipStream_t);

// ======================================================================
// Low-precision trailing update
// ======================================================================
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename H> struct LowP;
template <> struct LowP<_Float16> {
    typedef f16x8 vec_t;
    static constexpr float kMax = 65504.0f;
    __device__ static f32x4 mac(vec_t a, vec_t b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct LowP<__bf16> {
    typedef bf16x8 vec_t;
    static constexpr float kMax = 3.38953139e38f;
    __device__ static f32x4 mac(vec_t a, vec_t b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// dst[r][c] = round(W[r][c]) (ld of dst = cols); rows x cols.
template <typename H>
__global__ __launch_bounds__(256) void k_pack_rows(const float *__restrict__ W, int ldw, int rows,
                                                   int cols, H *__restrict__ dst,
                                                   int *__restrict__ status) {
    const int r = blockIdx.x;
    int bad = 0;
    for (int c = threadIdx.x; c < cols; c += 256) {
        const float v = W[(size_t)r * ldw + c];
        if (fabsf(v) > LowP<H>::kMax) ++bad;
        dst[(size_t)r * cols + c] = (H)v;
    }
    if (bad) atomicAdd(&status[ST_OVERFLOW], bad);
}

// dst[c][r] = round(W[r][c]) (ld of dst = rows): 64 x 64 tiles through LDS.
template <typename H>
__global__ __launch_bounds__(256) void k_pack_trans(const float *__restrict__ W, int ldw, int rows,
                                                    int cols, H *__restrict__ dst,
                                                    int *__restrict__ status) {
    __shared__ float tile[64][65];
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    int bad = 0;
    for (int i = ty; i < 64; i += 4) {
        const int r = r0 + i, c = c0 + tx;
        tile[i][tx] = (r < rows && c < cols) ? W[(size_t)r * ldw + c] : 0.0f;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int c = c0 + i, r = r0 + tx;
        if (c < cols && r < rows) {
            const float v = tile[tx][i];
            if (fabsf(v) > LowP<H>::kMax) ++bad;
            dst[(size_t)c * rows + r] = (H)v;
        }
    }
    if (bad) atomicAdd(&status[ST_OVERFLOW], bad);
}

hipError_t launch_pack(int prec, const float *W, int ldw, int rows, int cols, int transpose,
                       void *dst, int *status, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (prec == MIXLU_FP16) {
        if (transpose)
            k_pack_trans<_Float16><<<dim3((cols + 63) / 64, (rows + 63) / 64), dim3(256), 0, s>>>(
                W, ldw, rows, cols, (_Float16 *)dst, status);
        else
            k_pack_rows<_Float16><<<dim3(rows), dim3(256), 0, s>>>(W, ldw, rows, cols,
                                                                   (_Float16 *)dst, status);
    } else if (prec == MIXLU_BF16) {
        if (transpose)
            k_pack_trans<__bf16><<<dim3((cols + 63) / 64, (rows + 63) / 64), dim3(256), 0, s>>>(
                W, ldw, rows, cols, (__bf16 *)dst, status);
        else
            k_pack_rows<__bf16><<<dim3(rows), dim3(256), 0, s>>>(W, ldw, rows, cols,
                                                                 (__bf16 *)dst, status);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// C[M x N] -= Ap[M x K] * Bp[N x K]^T, Ap and Bp K-contiguous (Bp = Ap for the
// Cholesky update; lower != 0 skips tiles above the diagonal); 128 x 128 tile,
// 4 waves of 64 x 64 (4 x 4 MFMA 16x16x32 blocks), K step 64.
// 16x16x32 operand layout: lane l supplies A[l%16][8*(l/16) .. +8] and
// B[8*(l/16) .. +8][l%16]; result as for 16x16x4.
template <typename H>
__global__ __launch_bounds__(256) void k_gemm_lowp(int M, int N, int K, const H *__restrict__ Ap,
                                                   const H *__restrict__ Bp, float *__restrict__ C,
                                                   int ldc, int lower, int spare_xcd0) {
    constexpr int BM = 128, BN = 128, BK = 64, PITCH = BK + 8;
    using vec_t = typename LowP<H>::vec_t;
    __shared__ __attribute__((aligned(16))) H sA[BM * PITCH];
    __shared__ __attribute__((aligned(16))) H sB[BN * PITCH];
    int tx = blockIdx.x, ty = blockIdx.y;
    if (!tile_of(spare_xcd0, (N + BN - 1) / BN, (M + BM - 1) / BM, tx, ty)) return;
    const int m0 = ty * BM, n0 = tx * BN;
    if (lower && n0 > m0 + BM - 1) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    // the accumulators start from the C tile and A enters LDS negated (the
    // sign bit of each 16-bit value flipped), so the epilogue only stores;
    // the next K slab is loaded into registers while the current one is
    // multiplied
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 64 + i * 16 + (lane >> 4) * 4 + v;
                const int col = n0 + wn * 64 + j * 16 + (lane & 15);
                acc[i][j][v] = (row < M && col < N) ? C[(size_t)row * ldc + col] : 0.0f;
            }
    uint4 pa[4], pb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;
            const int row = e >> 3, seg = e & 7;
            pa[q] = make_uint4(0, 0, 0, 0);
            pb[q] = make_uint4(0, 0, 0, 0);
            if (m0 + row < M)
                pa[q] = *reinterpret_cast<const uint4 *>(Ap + (size_t)(m0 + row) * K + k0 + seg * 8);
            if (n0 + row < N)
                pb[q] = *reinterpret_cast<const uint4 *>(Bp + (size_t)(n0 + row) * K + k0 + seg * 8);
        }
    };
    load(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;
            const int row = e >> 3, seg = e & 7;
            constexpr unsigned kSign = 0x80008000u;
            *reinterpret_cast<uint4 *>(&sA[row * PITCH + seg * 8]) =
                make_uint4(pa[q].x ^ kSign, pa[q].y ^ kSign, pa[q].z ^ kSign, pa[q].w ^ kSign);
            *reinterpret_cast<uint4 *>(&sB[row * PITCH + seg * 8]) = pb[q];
        }
        __syncthreads();
        if (k0 + BK < K) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 32) {
            vec_t av[4], bv[4];
            const int ko = kk + (lane >> 4) * 8;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                av[i] = *reinterpret_cast<const vec_t *>(&sA[(wm * 64 + i * 16 + (lane & 15)) * PITCH + ko]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bv[j] = *reinterpret_cast<const vec_t *>(&sB[(wn * 64 + j * 16 + (lane & 15)) * PITCH + ko]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = LowP<H>::mac(av[i], bv[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 64 + i * 16 + (lane >> 4) * 4 + v;
                const int col = n0 + wn * 64 + j * 16 + (lane & 15);
                if (row < M && col < N) C[(size_t)row * ldc + col] = acc[i][j][v];
            }
}

hipError_t launch_gemm_lowp(int prec, int M, int N, int K, const void *Ap, const void *Bp,
                            float *C, int ldc, hipStream_t s, int lower, int spare_xcd0) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    if (K % 64) return hipErrorInvalidValue;
    const dim3 grid = gemm_grid(spare_xcd0, (N + 127) / 128, (M + 127) / 128);
    if (prec == MIXLU_FP16)
        k_gemm_lowp<_Float16><<<grid, dim3(256), 0, s>>>(M, N, K, (const _Float16 *)Ap,
                                                         (const _Float16 *)Bp, C, ldc, lower, spare_xcd0);
    else if (prec == MIXLU_BF16)
        k_gemm_lowp<__bf16><<<grid, dim3(256), 0, s>>>(M, N, K, (const __bf16 *)Ap,
                                                       (const __bf16 *)Bp, C, ldc, lower, spare_xcd0);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ======================================================================
// FP8 trailing update: OCP E4M3 operands with one E8M0 (power-of-two) scale
// per 32 consecutive K values of a row of L21 / a column of U12, multiplied
// on the gfx950 scaled MFMA (16x16x128, FP32 accumulate).
// ======================================================================
typedef int i32x8 __attribute__((ext_vector_type(8)));

// E4M3 (OCP, finite saturating) code of x, round to nearest even.
__device__ __forceinline__ unsigned char to_e4m3(float x) {
    return (unsigned char)__hip_cvt_float_to_fp8(x, __HIP_SATFINITE, __HIP_E4M3);
}

// Pack 32 values sharing one scale: the scale exponent e puts the block's
// largest magnitude below 2^8 (E4M3 reaches 448), the E8M0 byte is e + 127.
// Returns the scale byte; writes the 32 codes to out.  A non-finite value
// counts as an overflow.
__device__ __forceinline__ unsigned char pack_block32(const float (&v)[32], unsigned char *out,
                                                      int &bad) {
    float amax = 0.0f;
#pragma unroll
    for (int t = 0; t < 32; ++t) amax = fmaxf(amax, fabsf(v[t]));
    int e = -127;
    if (!(amax <= 3.40282347e38f)) {
        ++bad;
        e = 0;
    } else if (amax > 0.0f) {
        e = ilogbf(amax) - 7;
        e = e < -127 ? -127 : (e > 127 ? 127 : e);
    }
    const float inv = ldexpf(1.0f, -e);
#pragma unroll
    for (int t = 0; t < 32; ++t) out[t] = to_e4m3(v[t] * inv);
    return (unsigned char)(e + 127);
}

// rows x K row-major FP32 (ld ldw) -> codes[rows][K], scales[rows][K/32].
// transpose = 1: the operand is the K x cols matrix W (U12) and its columns
// are packed: codes[col][K], scales[col][K/32].  One thread per 32-value block.
__global__ __launch_bounds__(256) void k_pack_fp8(const float *__restrict__ W, int ldw, int rows,
                                                  int K, int transpose,
                                                  unsigned char *__restrict__ codes,
                                                  unsigned char *__restrict__ scales,
                                                  int *__restrict__ status) {
    const int kb = K / 32;
    const long blk = (long)blockIdx.x * 256 + threadIdx.x;
    if (blk >= (long)rows * kb) return;
    int r, b;
    if (transpose) {  // consecutive threads take consecutive columns (coalesced rows of W)
        b = (int)(blk / rows);
        r = (int)(blk % rows);
    } else {
        r = (int)(blk / kb);
        b = (int)(blk % kb);
    }
    float v[32];
#pragma unroll
    for (int t = 0; t < 32; ++t)
        v[t] = transpose ? W[(size_t)(b * 32 + t) * ldw + r] : W[(size_t)r * ldw + b * 32 + t];
    int bad = 0;
    unsigned char c[32];
    const unsigned char s = pack_block32(v, c, bad);
    uint4 *dst = reinterpret_cast<uint4 *>(codes + (size_t)r * K + b * 32);
    dst[0] = *reinterpret_cast<const uint4 *>(&c[0]);
    dst[1] = *reinterpret_cast<const uint4 *>(&c[16]);
    scales[(size_t)r * kb + b] = s;
    if (bad) atomicAdd(&status[ST_OVERFLOW], bad);
}

hipError_t launch_pack_fp8(const float *W, int ldw, int rows, int K, int transpose, void *codes,
                           void *scales, int *status, hipStream_t s) {
    if (rows <= 0 || K <= 0) return hipSuccess;
    if (K % 32) return hipErrorInvalidValue;
    const long nblk = (long)rows * (K / 32);
    k_pack_fp8<<<dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, s>>>(
        W, ldw, rows, K, transpose, static_cast<unsigned char *>(codes),
        static_cast<unsigned char *>(scales), status);
    return hipGetLastError();
}

// C[M x N] -= A B^T with A = codes/scales of M rows, B of N rows (both K
// codes per row, K % 128 == 0).  128 x 128 tile, 4 waves of 64 x 64 (4 x 4
// scaled MFMA blocks), K step 128.  Operand layout of the 16x16x128 scaled
// MFMA: lane (r = l % 16, g = l / 16) supplies K values 16g .. 16g+15 and
// 64+16g .. 64+16g+15 of its row and the scale of K block g (32 values).
__global__ __launch_bounds__(256) void k_gemm_fp8(int M, int N, int K,
                                                  const unsigned char *__restrict__ Ac,
                                                  const unsigned char *__restrict__ As,
                                                  const unsigned char *__restrict__ Bc,
                                                  const unsigned char *__restrict__ Bs,
                                                  float *__restrict__ C, int ldc, int lower,
                                                  int spare_xcd0) {
    constexpr int BM = 128, BN = 128, BK = 128, PITCH = BK + 16;
    __shared__ __attribute__((aligned(16))) unsigned char sA[BM * PITCH];
    __shared__ __attribute__((aligned(16))) unsigned char sB[BN * PITCH];
    __shared__ unsigned char ssA[BM * 4], ssB[BN * 4];
    int tx = blockIdx.x, ty = blockIdx.y;
    if (!tile_of(spare_xcd0, (N + BN - 1) / BN, (M + BM - 1) / BM, tx, ty)) return;
    const int m0 = ty * BM, n0 = tx * BN;
    if (lower && n0 > m0 + BM - 1) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int kb = K / 32;
    // accumulators from the C tile, A's codes negated (sign bit of each
    // E4M3 byte flipped): the epilogue only stores
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 64 + i * 16 + (lane >> 4) * 4 + v;
                const int col = n0 + wn * 64 + j * 16 + (lane & 15);
                acc[i][j][v] = (row < M && col < N) ? C[(size_t)row * ldc + col] : 0.0f;
            }
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;  // 16-byte vector index in a 128 x 128-byte slab
            const int row = e >> 3, seg = e & 7;
            uint4 va = make_uint4(0, 0, 0, 0), vb = make_uint4(0, 0, 0, 0);
            if (m0 + row < M) va = *reinterpret_cast<const uint4 *>(Ac + (size_t)(m0 + row) * K + k0 + seg * 16);
            if (n0 + row < N) vb = *reinterpret_cast<const uint4 *>(Bc + (size_t)(n0 + row) * K + k0 + seg * 16);
            constexpr unsigned kSign = 0x80808080u;
            *reinterpret_cast<uint4 *>(&sA[row * PITCH + seg * 16]) =
                make_uint4(va.x ^ kSign, va.y ^ kSign, va.z ^ kSign, va.w ^ kSign);
            *reinterpret_cast<uint4 *>(&sB[row * PITCH + seg * 16]) = vb;
        }
        for (int e = tid; e < BM * 4; e += 256) {
            const int row = e >> 2, g = e & 3;
            ssA[e] = m0 + row < M ? As[(size_t)(m0 + row) * kb + k0 / 32 + g] : (unsigned char)127;
            ssB[e] = n0 + row < N ? Bs[(size_t)(n0 + row) * kb + k0 / 32 + g] : (unsigned char)127;
        }
        __syncthreads();
        const int g = lane >> 4;
        i32x8 av[4], bv[4];
        int sa[4], sb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = wm * 64 + i * 16 + (lane & 15);
            const uint4 lo = *reinterpret_cast<const uint4 *>(&sA[row * PITCH + 16 * g]);
            const uint4 hi = *reinterpret_cast<const uint4 *>(&sA[row * PITCH + 64 + 16 * g]);
            av[i] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                          (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
            sa[i] = ssA[row * 4 + g];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = wn * 64 + j * 16 + (lane & 15);
            const uint4 lo = *reinterpret_cast<const uint4 *>(&sB[col * PITCH + 16 * g]);
            const uint4 hi = *reinterpret_cast<const uint4 *>(&sB[col * PITCH + 64 + 16 * g]);
            bv[j] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                          (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
            sb[j] = ssB[col * 4 + g];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                    av[i], bv[j], acc[i][j], 0, 0, 0, sa[i], 0, sb[j]);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 64 + i * 16 + (lane >> 4) * 4 + v;
                const int col = n0 + wn * 64 + j * 16 + (lane & 15);
                if (row < M && col < N) C[(size_t)row * ldc + col] = acc[i][j][v];
            }
}

hipError_t launch_gemm_fp8(int M, int N, int K, const void *Ac, const void *As, const void *Bc,
                           const void *Bs, float *C, int ldc, hipStream_t s, int lower,
                           int spare_xcd0) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    if (K % 128) return hipErrorInvalidValue;
    const dim3 grid = gemm_grid(spare_xcd0, (N + 127) / 128, (M + 127) / 128);
    k_gemm_fp8<<<grid, dim3(256), 0, s>>>(M, N, K, static_cast<const unsigned char *>(Ac),
                                          static_cast<const unsigned char *>(As),
                                          static_cast<const unsigned char *>(Bc),
                                          static_cast<const unsigned char *>(Bs), C, ldc, lower,
                                          spare_xcd0);
    return hipGetLastError();
}

}  // namespace mixlu
