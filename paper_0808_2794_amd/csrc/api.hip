// C ABI of libmixlu: argument checking, workspace layout and the host-side
// sequencing of Algorithm 1 (mixed-precision iterative refinement for direct
// solvers, Section 2.1) over the HIP kernels.  Every floating-point step
// runs on the GPU; the host only enqueues kernels and, once per refinement
// iteration, reads the per-column norms (a few bytes) to apply the stopping
// test of Section 3 and the failure policy (30 iterations mean failure,
// Section 4; fall back to FP64 when refinement cannot converge).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"

using namespace mixlu;

// Optional per-kernel-class timing: HIP events around the launches of the
// main kernel classes, harvested after the synchronizing calls.
struct ProfAcc {
    long long launches = 0;
    double ms = 0.0, flops = 0.0, bytes = 0.0;
};
struct ProfPending {
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
};
enum ProfClass { PC_PANEL, PC_TRAIL, PC_PACK, PC_TRSV, PC_RESID, PC_CPANEL, PC_BATCH, PC_SPMV, PC_COUNT };
static const char *const kProfNames[PC_COUNT] = {"panel_getf2", "trailing_update", "pack_operands",
                                                 "trsv", "residual", "panel_potf2",
                                                 "batched_solve", "sparse_spmv"};
struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<ProfPending> pending;
    ProfAcc acc[PC_COUNT];
};

struct mixlu_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;  // look-ahead: trailing updates overlapped with panels
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_next = nullptr;
    double *hbuf = nullptr;  // pinned host mirror of the norms / status
    size_t hbuf_bytes = 0;
    int num_cu = 256;
    mixlu::BatchedTiles btiles[5] = {{16, 128, 2}, {16, 128, 2}, {16, 128, 2}, {16, 128, 2},
                                     {16, 128, 1}};  // by mixlu_prec; FP64 last
    int btuned[5] = {0, 0, 0, 0, 0};
    Prof prof;
    std::vector<double> hist;  // true-residual norms of the last refinement, in order
};

namespace {

constexpr double kEpsD = 0x1p-53;

#define HIPCK(x)                                    \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return MIXLU_ERR_HIP; \
    } while (0)
#define RETCK(x)                        \
    do {                                \
        int r_ = (x);                   \
        if (r_ != MIXLU_OK) return r_;  \
    } while (0)

int auto_nb(int n) {
    const int n64 = round_up(n > 0 ? n : 1, 64);
    if (n64 <= 128) return 64;
    if (n64 <= 512) return 128;
    if (n64 <= 2048) return 256;
    return 512;
}

bool is_lowp(int prec) { return prec == MIXLU_BF16 || prec == MIXLU_FP16 || prec == MIXLU_FP8; }
bool prec_valid(int prec) {
    return prec == MIXLU_FP64 || prec == MIXLU_FP32 || prec == MIXLU_BF16 ||
           prec == MIXLU_FP16 || prec == MIXLU_FP8;
}

template <typename T> T *at(void *work, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(work) + off);
}

int ensure_hbuf(mixlu_ctx_s *ctx, size_t bytes) {
    if (ctx->hbuf_bytes >= bytes) return MIXLU_OK;
    if (ctx->hbuf) (void)hipHostFree(ctx->hbuf);
    ctx->hbuf = nullptr;
    ctx->hbuf_bytes = 0;
    HIPCK(hipHostMalloc(reinterpret_cast<void **>(&ctx->hbuf), bytes, hipHostMallocDefault));
    ctx->hbuf_bytes = bytes;
    return MIXLU_OK;
}

// Second stream (default priority) and the two events that order it with
// the context's stream, created on first use.
int ensure_side(mixlu_ctx_s *ctx) {
    if (ctx->side) return MIXLU_OK;
    HIPCK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    HIPCK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    HIPCK(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    HIPCK(hipEventCreateWithFlags(&ctx->ev_next, hipEventDisableTiming));
    return MIXLU_OK;
}

thread_local Prof *t_prof = nullptr;  // profiler of the context making the current call

hipEvent_t prof_event(Prof &p) {
    if (!p.pool.empty()) {
        hipEvent_t e = p.pool.back();
        p.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one launch with events when profiling is on.
struct ProfScope {
    bool active = false;
    hipStream_t s = nullptr;
    ProfPending p{};
    ProfScope(int cls, double flops, double bytes, hipStream_t st) {
        if (!t_prof || !t_prof->on) return;
        p = ProfPending{cls, prof_event(*t_prof), prof_event(*t_prof), flops, bytes};
        if (!p.a || !p.b) return;
        s = st;
        active = hipEventRecord(p.a, s) == hipSuccess;
    }
    ~ProfScope() {
        if (!active) return;
        if (hipEventRecord(p.b, s) == hipSuccess) t_prof->pending.push_back(p);
    }
};

// Fold finished event pairs into the totals (the stream has been synchronized).
void prof_harvest(Prof &p) {
    for (auto &q : p.pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
            ProfAcc &c = p.acc[q.cls];
            c.launches += 1;
            c.ms += ms;
            c.flops += q.flops;
            c.bytes += q.bytes;
        }
        p.pool.push_back(q.a);
        p.pool.push_back(q.b);
    }
    p.pending.clear();
}

struct ProfCall {  // binds the context's profiler to this thread for one API call
    mixlu_ctx_s *ctx;
    explicit ProfCall(mixlu_ctx_s *c) : ctx(c) { t_prof = c ? &c->prof : nullptr; }
    ~ProfCall() {
        if (ctx && ctx->prof.on && !ctx->prof.pending.empty() &&
            hipStreamSynchronize(ctx->stream) == hipSuccess)
            prof_harvest(ctx->prof);
        t_prof = nullptr;
    }
};

}  // namespace

size_t mixlu::plan_layout(Layout &L, int op, int prec, int n, int nrhs, const mixlu_opts &o) {
    L.n = n;
    L.nrhs = nrhs < 1 ? 1 : nrhs;
    L.prec = (op == MIXLU_OP_DGESV || op == MIXLU_OP_DPOSV) ? MIXLU_FP64
             : op == MIXLU_OP_SGESV                         ? MIXLU_FP32
                                                            : prec;
    L.kind = (op == MIXLU_OP_POSV || op == MIXLU_OP_DPOSV) ? 1 : 0;
    L.nb = o.nb > 0 ? o.nb : auto_nb(n);
    // the FP8 update multiplies K in steps of 128
    if (L.prec == MIXLU_FP8 && L.nb < 128) L.nb = 128;
    L.npad = round_up(n > 0 ? n : 1, L.nb);
    L.fallback = (L.prec != MIXLU_FP64) && o.fallback && op != MIXLU_OP_SGESV;
    const size_t np = (size_t)L.npad;
    const size_t wbytes = np * np * (L.prec == MIXLU_FP64 ? 8 : 4);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at_ = off;
        off = align_up(off + bytes, 256);
        return at_;
    };
    L.W = take(wbytes);
    L.W64 = L.fallback ? take(np * np * 8) : 0;
    // packed trailing-update operands, three sets (look-ahead: the next
    // blocks pack while an earlier block's update still reads its set)
    const size_t pk = is_lowp(L.prec) ? np * L.nb * 2 : 0;
    L.Ap = take(3 * pk);
    L.Bp = take(3 * pk);
    L.ipiv = take(np * 4);
    L.perm = take(np * 4);
    L.R = take(np * 8);
    L.C = take(np * 8);
    L.vec_r = take(np * L.nrhs * 8);
    L.vec_y = take(np * L.nrhs * 8);
    L.vec_z = L.nrhs > 1 ? take(np * L.nrhs * 8) : L.vec_y;
    L.xbuf = take((size_t)kXbufWords * 8);
    L.ybuf = take((np * kTrsvNRT * 2 + 64) * 8);
    L.moves = take((size_t)(2 * kMovesInts + kPanelListInts) * 4);  // + the panels' lists
    L.tmp = take((size_t)(2 * kColChunks + 2) * np * 8);
    L.status = take(ST_COUNT * 4);
    L.norms = take((size_t)(4 + 3 * L.nrhs) * 8);
    L.krylov = take(((size_t)(2 * kKrylovMax + 2) * np + 4 * kKrylovMax + 16) * 8);
    L.dinv = take(2 * np * kTrsvBS * (L.prec == MIXLU_FP64 ? 8 : 4));
    L.dinv64 = L.fallback ? take(2 * np * kTrsvBS * 8) : 0;
    L.total = off;
    return off;
}

namespace {

void fill_factor(mixlu_factor *F, const Layout &L, void *work, size_t lwork, int layout) {
    std::memset(F, 0, sizeof(*F));
    F->n = L.n;
    F->npad = L.npad;
    F->nb = L.nb;
    F->prec = L.prec;
    F->kind = L.kind;
    F->layout = layout;
    F->nrhs_max = L.nrhs;
    F->work = work;
    F->lwork = lwork;
    const size_t offs[16] = {L.W, L.W64, L.Ap, L.Bp, L.ipiv, L.perm, L.vec_z, L.R,
                             L.C, L.vec_r, L.vec_y, L.xbuf, L.ybuf, L.moves, L.tmp, L.status};
    std::memcpy(F->off, offs, sizeof(offs));
}

// Rebuild the layout from a factor description.
Layout layout_of(const mixlu_factor *F) {
    Layout L{};
    L.n = F->n;
    L.npad = F->npad;
    L.nb = F->nb;
    L.prec = F->prec;
    L.kind = F->kind;
    L.nrhs = F->nrhs_max;
    L.W = F->off[0];
    L.W64 = F->off[1];
    L.fallback = F->off[1] != 0;
    L.Ap = F->off[2];
    L.Bp = F->off[3];
    L.ipiv = F->off[4];
    L.perm = F->off[5];
    L.vec_z = F->off[6];
    L.R = F->off[7];
    L.C = F->off[8];
    L.vec_r = F->off[9];
    L.vec_y = F->off[10];
    L.xbuf = F->off[11];
    L.ybuf = F->off[12];
    L.moves = F->off[13];
    L.tmp = F->off[14];
    L.status = F->off[15];
    // norms and the Krylov area follow status (same rule as plan_layout)
    L.norms = align_up(L.status + ST_COUNT * 4, 256);
    L.krylov = align_up(L.norms + (size_t)(4 + 3 * L.nrhs) * 8, 256);
    // then the inverse diagonal blocks (same rule as plan_layout)
    const size_t np = (size_t)L.npad;
    L.dinv = align_up(L.krylov + ((2 * (size_t)kKrylovMax + 2) * np + 4 * kKrylovMax + 16) * 8, 256);
    L.dinv64 = L.fallback
                   ? align_up(L.dinv + 2 * np * kTrsvBS * (L.prec == MIXLU_FP64 ? 8 : 4), 256)
                   : 0;
    return L;
}

// Region of the inverse diagonal blocks that belongs to the factor at woff.
size_t dinv_of(const Layout &L, size_t woff) { return (L.W64 && woff == L.W64) ? L.dinv64 : L.dinv; }

// Blocked right-looking LU with partial pivoting of W (npad x npad, ld = npad)
// in place, with look-ahead over two streams.  Per outer block K of nb
// columns, the main stream factors the block's panels of B columns (GEPP with
// pivot search; their row interchanges, triangular solve and FP32/FP64
// update inside the block), then brings only the next block's columns up to
// date: its row interchanges, U12 = L11^{-1} A12 and A22 -= L21 U12 for
// those nb columns, and goes on to the next block's panels.  The side stream
// does the rest of block K: the interchanges on the columns left of the
// block and right of the next one, their U12, and their trailing update
// (in FP32/FP64, or with BF16/FP16/FP8 operands on MFMA), the block after
// next first, so that the main stream can take it at its next step.
// Events: ev_fork (main -> side: block K factored, its pivots composed and
// L21 packed), ev_next (side -> main: the block after next is up to date
// with block K), ev_join (side -> main at the end).
template <typename T>
int factor_lu(mixlu_ctx_s *ctx, void *work, const Layout &L, size_t woff, int trail_prec) {
    constexpr int B = sizeof(T) == 4 ? kPanelBF : kPanelBD;
    hipStream_t s = ctx->stream;
    const int np = L.npad, nb = L.nb;
    T *W = at<T>(work, woff);
    int *ipiv = at<int>(work, L.ipiv);
    int *perm = at<int>(work, L.perm);
    int *status = at<int>(work, L.status);
    auto *xbuf = at<unsigned long long>(work, L.xbuf);
    // row-move lists of the wide (outer) pivot blocks, one per parity: the
    // side stream may still apply block K's while block K+1 composes
    int *moves2[2] = {at<int>(work, L.moves), at<int>(work, L.moves) + kMovesInts};
    int *plist = at<int>(work, L.moves) + 2 * kMovesInts;  // this block's panels' move lists
    if (nb % B || nb % 64 || nb > kMaxOuterBlock) return MIXLU_ERR_NOT_IMPLEMENTED;
    RETCK(ensure_side(ctx));
    hipStream_t s2 = ctx->side;
    HIPCK(launch_iota(perm, np, s));
    HIPCK(launch_fill_u32(reinterpret_cast<unsigned *>(xbuf), 0u, (size_t)kXbufWords * 2, s));
    auto Wp = [&](int r, int c) { return W + (size_t)r * np + c; };
    const bool lowp = !(trail_prec == MIXLU_FP64 || trail_prec == MIXLU_FP32);
    if (lowp && sizeof(T) != 4) return MIXLU_ERR_NOT_IMPLEMENTED;
    const bool f8 = trail_prec == MIXLU_FP8;
    const int esz = f8 ? 1 : 2;                 // bytes per packed operand
    const size_t pk = (size_t)np * nb;          // elements of one packed operand set
    const bool wide = nb > kSwapsFused;         // interchanges composed once, applied per range
    bool side_used = false;   // the side stream holds work of this factorization
    bool next_ready = false;  // ev_next marks the next block's columns up to date
    int par = 0;              // move-list parity
    // packed-operand set of this block: three sets, because the side
    // stream's update of block K may still read L21(K) until the main stream
    // has waited for the side's next-block event of block K+1
    int pset = 0;
    // interchanges of block K on [c0, c1) minus [skip0, skip1), on stream st
    auto swaps = [&](int K0, int c0, int c1, int skip0, int skip1, hipStream_t st) -> int {
        if (wide)
            HIPCK(launch_swaps_apply<T>(W, np, moves2[par], nb, c0, c1, skip0, skip1, st));
        else
            HIPCK(launch_row_swaps<T>(ipiv, K0, nb, np, nullptr, W, np, c0, c1, skip0, skip1,
                                      nullptr, st));
        return MIXLU_OK;
    };
    // U12 = L11^{-1} A12 for the columns [c0, c0 + ncol) of block K's rows
    auto u12 = [&](int K0, int c0, int ncol, hipStream_t st) -> int {
        if (ncol <= 0) return MIXLU_OK;
        for (int ib = 0; ib < nb; ib += B) {
            HIPCK(launch_trsm_diag<T>(Wp(K0 + ib, K0 + ib), np, Wp(K0 + ib, c0), np, ncol, st));
            if (ib + B < nb)
                HIPCK(launch_gemm<T>(nb - ib - B, ncol, B, Wp(K0 + ib + B, K0 + ib), np,
                                     Wp(K0 + ib, c0), np, Wp(K0 + ib + B, c0), np, st));
        }
        return MIXLU_OK;
    };
    // A22[:, c0 : c0 + ncol] -= L21 U12[:, c0 : c0 + ncol] (rows kend..), with
    // U12's columns packed first on the low-precision path
    auto update = [&](int K0, int c0, int ncol, hipStream_t st, int spare) -> int {
        if (ncol <= 0) return MIXLU_OK;
        const int kend = K0 + nb, nr = np - kend, cr = c0 - kend;  // cr: column within U12
        if (!lowp) {
            ProfScope ps(PC_TRAIL, 2.0 * nr * ncol * nb,
                         (2.0 * nr * ncol + 1.0 * (nr + ncol) * nb) * sizeof(T), st);
            HIPCK(launch_gemm<T>(nr, ncol, nb, Wp(kend, K0), np, Wp(K0, c0), np, Wp(kend, c0), np,
                                 st, 0, 0, 0, spare));
            return MIXLU_OK;
        }
        if constexpr (sizeof(T) == 4) {
            auto *Ap = at<unsigned char>(work, L.Ap) + pset * pk * 2;
            auto *Bp = at<unsigned char>(work, L.Bp) + pset * pk * 2;
            auto *As = Ap + pk, *Bs = Bp + pk;  // FP8: codes, then one scale byte per 32 codes
            {
                ProfScope ps(PC_PACK, 0.0, 1.0 * ncol * nb * (4 + esz), st);
                if (f8)
                    HIPCK(launch_pack_fp8(Wp(K0, c0), np, ncol, nb, 1, Bp + (size_t)cr * nb,
                                          Bs + (size_t)cr * (nb / 32), status, st));
                else
                    HIPCK(launch_pack(trail_prec, Wp(K0, c0), np, nb, ncol, 1,
                                      Bp + (size_t)cr * nb * 2, status, st));
            }
            ProfScope ps(PC_TRAIL, 2.0 * nr * ncol * nb, 8.0 * nr * ncol + 1.0 * esz * (nr + ncol) * nb,
                         st);
            if (f8)
                HIPCK(launch_gemm_fp8(nr, ncol, nb, Ap, As, Bp + (size_t)cr * nb,
                                      Bs + (size_t)cr * (nb / 32), Wp(kend, c0), np, st, 0, spare));
            else
                HIPCK(launch_gemm_lowp(trail_prec, nr, ncol, nb, Ap, Bp + (size_t)cr * nb * 2,
                                       Wp(kend, c0), np, st, 0, spare));
        }
        return MIXLU_OK;
    };
    for (int K0 = 0; K0 < np; K0 += nb) {
        const int kend = K0 + nb;
        // panels of this block: only its columns, which are up to date
        for (int k = K0; k < kend; k += B) {
            {
                const double m = np - k;
                double fl = 0.0;
                for (int j = 0; j < B; ++j) fl += (m - j - 1) * (1.0 + 2.0 * (B - j - 1));
                ProfScope ps(PC_PANEL, fl, 2.0 * m * B * sizeof(T), s);
                HIPCK(launch_panel<T>(W, np, k, np - k, ipiv, xbuf, status, s, perm, K0, kend,
                                      wide ? plist + (k - K0) / B * kPanelMovesInts : nullptr));
            }
            if (k + B < kend) {
                HIPCK(launch_trsm_diag<T>(Wp(k, k), np, Wp(k, k + B), np, kend - k - B, s));
                HIPCK(launch_gemm<T>(np - k - B, kend - k - B, B, Wp(k + B, k), np, Wp(k, k + B),
                                     np, Wp(k + B, k + B), np, s));
            }
        }
        const int nr = np - kend;
        if (nr == 0) {
            // last block: its interchanges on the columns to the left, once
            // the side stream has finished
            if (side_used) HIPCK(hipStreamWaitEvent(s, ctx->ev_join, 0));
            side_used = false;
            if (wide) HIPCK(launch_swaps_merge(plist, nb / B, kPanelMovesInts, K0, np, moves2[par], s));
            RETCK(swaps(K0, 0, K0, K0, K0, s));
            break;
        }
        const int nx = nr < nb ? nr : nb;  // the next block's columns
        const int rest = nr - nx;
        if (wide) HIPCK(launch_swaps_merge(plist, nb / B, kPanelMovesInts, K0, np, moves2[par], s));
        if (lowp) {
            if constexpr (sizeof(T) == 4) {
                auto *Ap = at<unsigned char>(work, L.Ap) + pset * pk * 2;
                auto *As = Ap + pk;
                ProfScope ps(PC_PACK, 0.0, 1.0 * nr * nb * (4 + esz), s);
                if (f8) HIPCK(launch_pack_fp8(Wp(kend, K0), np, nr, nb, 0, Ap, As, status, s));
                else HIPCK(launch_pack(trail_prec, Wp(kend, K0), np, nr, nb, 0, Ap, status, s));
            }
        }
        // hand block K to the side stream
        HIPCK(hipEventRecord(ctx->ev_fork, s));
        HIPCK(hipStreamWaitEvent(s2, ctx->ev_fork, 0));
        side_used = true;
        // main: the next block's columns (the side stream brought them up to
        // date with the previous block)
        if (next_ready) HIPCK(hipStreamWaitEvent(s, ctx->ev_next, 0));
        RETCK(swaps(K0, kend, kend + nx, kend, kend, s));
        RETCK(u12(K0, kend, nx, s));
        RETCK(update(K0, kend, nx, s, 0));
        // side: the columns left of the block and right of the next one
        RETCK(swaps(K0, 0, np, K0, kend + nx, s2));
        RETCK(u12(K0, kend + nx, rest, s2));
        next_ready = false;
        if (rest > 0) {
            const int nx2 = rest < nb ? rest : nb;  // the block after next first
            RETCK(update(K0, kend + nx, nx2, s2, 1));
            HIPCK(hipEventRecord(ctx->ev_next, s2));
            next_ready = true;
            RETCK(update(K0, kend + nx + nx2, rest - nx2, s2, 1));
        }
        HIPCK(hipEventRecord(ctx->ev_join, s2));
        par ^= 1;
        pset = pset == 2 ? 0 : pset + 1;
    }
    if (side_used) HIPCK(hipStreamWaitEvent(s, ctx->ev_join, 0));
    return MIXLU_OK;
}

// Blocked right-looking Cholesky of the symmetric W (lower triangle used):
// per 64-column step the diagonal block and the rows below it (k_chol_panel),
// the update of the rest of the outer block in FP32/FP64, then per outer
// block the symmetric trailing update A22 -= L21 L21^T on the lower tiles
// (FP32/FP64, or BF16/FP16 operands on MFMA).  Finally L L^T is rewritten as
// L' U' (unit lower L' = L D^{-1}, U' = D L^T) and perm = identity, so the LU
// solves apply unchanged.
template <typename T>
int factor_chol(hipStream_t s, void *work, const Layout &L, size_t woff, int trail_prec) {
    constexpr int B = 64;
    const int np = L.npad, nb = L.nb;
    T *W = at<T>(work, woff);
    T *diag = at<T>(work, L.tmp);
    int *status = at<int>(work, L.status);
    if (nb % B || nb > kMaxOuterBlock) return MIXLU_ERR_NOT_IMPLEMENTED;
    HIPCK(launch_iota(at<int>(work, L.perm), np, s));
    HIPCK(launch_iota(at<int>(work, L.ipiv), np, s));
    auto Wp = [&](int r, int c) { return W + (size_t)r * np + c; };
    for (int K0 = 0; K0 < np; K0 += nb) {
        const int kend = K0 + nb;
        for (int k = K0; k < kend; k += B) {
            const int below = np - k - B;
            {
                ProfScope ps(PC_CPANEL, B * B * (B / 3.0) + (double)below * B * B,
                             ((double)B * B + 2.0 * below * B) * sizeof(T), s);
                HIPCK(launch_chol_panel<T>(W, np, k, below, diag, status, s));
            }
            if (k + B < kend)
                HIPCK(launch_gemm<T>(below, kend - k - B, B, Wp(k + B, k), np, Wp(k + B, k), np,
                                     Wp(k + B, k + B), np, s, 1, 1));
        }
        if (kend < np) {
            const int nr = np - kend;
            if (trail_prec == MIXLU_FP64 || trail_prec == MIXLU_FP32) {
                ProfScope ps(PC_TRAIL, 1.0 * nr * (nr + 1.0) * nb,
                             (1.0 * nr * (nr + 1.0) + 1.0 * nr * nb) * sizeof(T), s);
                HIPCK(launch_gemm<T>(nr, nr, nb, Wp(kend, K0), np, Wp(kend, K0), np,
                                     Wp(kend, kend), np, s, 1, 1));
            } else {
                if constexpr (sizeof(T) == 4) {
                    auto *Ap = at<unsigned char>(work, L.Ap);
                    auto *As = Ap + (size_t)np * nb;
                    const bool f8 = trail_prec == MIXLU_FP8;
                    {
                        ProfScope ps(PC_PACK, 0.0, 1.0 * nr * nb * (4 + (f8 ? 1 : 2)), s);
                        if (f8)
                            HIPCK(launch_pack_fp8(Wp(kend, K0), np, nr, nb, 0, Ap, As, status, s));
                        else
                            HIPCK(launch_pack(trail_prec, Wp(kend, K0), np, nr, nb, 0, Ap, status, s));
                    }
                    ProfScope ps(PC_TRAIL, 1.0 * nr * (nr + 1.0) * nb,
                                 4.0 * nr * (nr + 1.0) + (f8 ? 1.0 : 2.0) * nr * nb, s);
                    if (f8)
                        HIPCK(launch_gemm_fp8(nr, nr, nb, Ap, As, Ap, As, Wp(kend, kend), np, s, 1));
                    else
                        HIPCK(launch_gemm_lowp(trail_prec, nr, nr, nb, Ap, Ap, Wp(kend, kend), np, s, 1));
                } else {
                    return MIXLU_ERR_NOT_IMPLEMENTED;
                }
            }
        }
    }
    HIPCK(launch_chol_to_lu<T>(W, np, np, diag, s));
    return MIXLU_OK;
}

hipError_t init_status(hipStream_t s, int *status) {
    // ST_BREAKDOWN and ST_CHOL start at INT_MAX (no failure), the rest at 0
    hipError_t e = launch_fill_u32(reinterpret_cast<unsigned *>(status), 0u, ST_COUNT, s);
    if (e == hipSuccess)
        e = launch_fill_u32(reinterpret_cast<unsigned *>(status + ST_BREAKDOWN), (unsigned)INT_MAX,
                            1, s);
    if (e == hipSuccess)
        e = launch_fill_u32(reinterpret_cast<unsigned *>(status + ST_CHOL), (unsigned)INT_MAX, 1, s);
    return e;
}

// Failure column + 1 of the factorization (INT_MAX: none).
int breakdown_of(const Layout &L, const int st[ST_COUNT]) {
    return L.kind == 1 ? st[ST_CHOL] : st[ST_BREAKDOWN];
}

// Read status words and the two matrix norms (synchronizes).
int read_status(mixlu_ctx_s *ctx, const Layout &L, void *work, int st[ST_COUNT],
                double norms2[2]) {
    RETCK(ensure_hbuf(ctx, 4096));
    HIPCK(hipMemcpyAsync(ctx->hbuf, at<int>(work, L.status), ST_COUNT * 4, hipMemcpyDeviceToHost,
                         ctx->stream));
    HIPCK(hipMemcpyAsync(ctx->hbuf + 8, at<double>(work, L.norms), 2 * 8, hipMemcpyDeviceToHost,
                         ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    std::memcpy(st, ctx->hbuf, ST_COUNT * 4);
    norms2[0] = ctx->hbuf[8];
    norms2[1] = ctx->hbuf[9];
    return MIXLU_OK;
}

// Norms, power-of-two scales and conversion of the n x n FP64 input into the
// working factor at woff, with equilibration or for Cholesky (three passes
// over A: row statistics, column statistics with the row scales, conversion).
template <typename T>
int stats_and_convert(hipStream_t s, void *work, const Layout &L, size_t woff, const double *A,
                      int lda, int equil) {
    const int n = L.n, np = L.npad;
    double *tmp = at<double>(work, L.tmp);
    double *R = at<double>(work, L.R), *C = at<double>(work, L.C);
    double *norms = at<double>(work, L.norms);
    int *status = at<int>(work, L.status);
    HIPCK(launch_row_stats(A, lda, n, tmp, tmp + np, s));
    if (L.kind == 1) {
        // ||A||_inf from the row sums; symmetric scaling keeps W symmetric
        HIPCK(launch_finish_rows(n, np, tmp, tmp + np, R, 0, norms, s));
        HIPCK(launch_sym_scale(A, lda, n, np, R, C, equil, s));
    } else {
        HIPCK(launch_finish_rows(n, np, tmp, tmp + np, R, equil, norms, s));
        HIPCK(launch_col_stats(A, lda, n, np, R, tmp + 2 * (size_t)np, C, equil, norms, s));
    }
    HIPCK(launch_convert<T>(A, lda, n, np, R, C, at<T>(work, woff), np, status, s));
    return MIXLU_OK;
}

// Norms, scales, conversion and LU of the n x n FP64 input into the working
// factor at woff (FP32 or FP64 storage).
template <typename T>
int convert_and_factor(mixlu_ctx_s *ctx, void *work, const Layout &L, size_t woff,
                       const double *A, int lda, int equil, int trail_prec) {
    hipStream_t s = ctx->stream;
    const int n = L.n, np = L.npad;
    double *tmp = at<double>(work, L.tmp);
    double *R = at<double>(work, L.R), *C = at<double>(work, L.C);
    double *norms = at<double>(work, L.norms);
    int *status = at<int>(work, L.status);
    HIPCK(init_status(s, status));
    if (L.kind == 0 && !equil) {
        // no scaling: conversion and both norms in one pass over A
        HIPCK(launch_convert_stats<T>(A, lda, n, np, at<T>(work, woff), np, tmp, R, C, norms,
                                      status, s));
    } else {
        RETCK(stats_and_convert<T>(s, work, L, woff, A, lda, equil));
    }
    if (L.kind == 1) RETCK(factor_chol<T>(s, work, L, woff, trail_prec));
    else RETCK(factor_lu<T>(ctx, work, L, woff, trail_prec));
    // the solves apply the inverses of the factors' 64 x 64 diagonal blocks
    HIPCK(launch_tri_inv<T>(at<T>(work, woff), np, np, at<T>(work, dinv_of(L, woff)), s));
    return MIXLU_OK;
}

// Low-precision solve with the factors of W = R M C, P W = L U:
//   trans = 0: X (=|+=) C U^{-1} L^{-1} P (R rhs)          (M X = rhs)
//   trans = 1: X (=|+=) R P^T L^{-T} U^{-T} (C rhs)        (M^T X = rhs)
// rhs FP64; the factor's precision Tw inside.
template <typename Tw>
int lu_solve(hipStream_t s, void *work, const Layout &L, size_t woff, int nrhs,
             const double *rhs, int ldr, int rhs_cm, double *X, int ldx, int x_cm, int assign,
             int trans) {
    const int n = L.n, np = L.npad;
    const Tw *W = at<Tw>(work, woff);
    const Tw *Dinv = at<Tw>(work, dinv_of(L, woff));
    Tw *Y = at<Tw>(work, L.vec_y);
    int *status = at<int>(work, L.status);
    double *xnorm = at<double>(work, L.norms) + 4 + L.nrhs;
    auto *ybuf = at<unsigned long long>(work, L.ybuf);
    const int *perm = at<int>(work, L.perm);
    const double *R = at<double>(work, L.R), *C = at<double>(work, L.C);
    HIPCK(launch_rhs_gather<Tw>(n, np, nrhs, rhs, ldr, rhs_cm, trans ? nullptr : perm,
                                trans ? C : R, Y, nrhs, s));
    if (nrhs == 1) {
        // one right-hand side: the chained single-launch solve (latency bound)
        const double tb = 0.5 * np * (np + 64.0) * sizeof(Tw) + 2.0 * np * sizeof(Tw);
        {
            ProfScope ps(PC_TRSV, (double)np * np, tb, s);
            HIPCK(launch_trsv<Tw>(0, trans, W, np, Dinv, np, Y, 1, 1, ybuf, status, s));
        }
        {
            ProfScope ps(PC_TRSV, (double)np * np, tb, s);
            HIPCK(launch_trsv<Tw>(1, trans, W, np, Dinv, np, Y, 1, 1, ybuf, status, s));
        }
    } else {
        // several: diagonal blocks one column per thread plus GEMM updates
        const double tb = 0.5 * np * (np + 64.0) * sizeof(Tw) + 2.0 * np * nrhs * sizeof(Tw);
        Tw *Z = at<Tw>(work, L.vec_z);
        {
            ProfScope ps(PC_TRSV, (double)np * np * nrhs, tb, s);
            HIPCK(launch_trsm_blocked<Tw>(0, trans, W, np, np, Y, Z, nrhs, nrhs, s));
        }
        {
            ProfScope ps(PC_TRSV, (double)np * np * nrhs, tb, s);
            HIPCK(launch_trsm_blocked<Tw>(1, trans, W, np, np, Z, Y, nrhs, nrhs, s));
        }
    }
    HIPCK(launch_fill_f64(xnorm, 0.0, nrhs, s));
    HIPCK(launch_x_update<Tw>(n, np, nrhs, assign, Y, nrhs, trans ? perm : nullptr, trans ? R : C,
                              X, ldx, x_cm, xnorm, s));
    return MIXLU_OK;
}

struct LoopResult {
    int iters;      // corrections applied, or negative failure code
    int converged;
    double rnorm, xnorm, berr;
};

// Algorithm 1 steps 4-7 from the current X, with correction solves in the
// precision of the factor at woff (Tw storage).  Stops when every column
// meets ||r||_inf <= sqrt(n) eps_d ||A||_inf ||x||_inf.
template <typename Tw>
int refine_loop(mixlu_ctx_s *ctx, void *work, const Layout &L, size_t woff, const double *A,
                int lda, const double *B, int ldb, double *X, int ldx, int cm, int nrhs,
                double anorm, const mixlu_opts &o, LoopResult &res, int trans) {
    hipStream_t s = ctx->stream;
    const int n = L.n;
    double *Rv = at<double>(work, L.vec_r);
    double *norms = at<double>(work, L.norms);
    double *rnorm = norms + 4;
    double *xnorm = norms + 4 + L.nrhs;
    int *status = at<int>(work, L.status);
    RETCK(ensure_hbuf(ctx, (size_t)(2 * nrhs + 16) * 8));
    const double thr = std::sqrt((double)n) * kEpsD * anorm;
    std::vector<double> prev(nrhs, 0.0), ratio_prev(nrhs, 0.0);
    res = LoopResult{0, 0, 0.0, 0.0, 0.0};
    // several right-hand sides: the residual GEMM splits K; its partial
    // products go to the FP64 fallback region while that is unused (this is
    // not the fallback's own refinement), else to the Krylov vectors
    double *split_buf = nullptr;
    int nsplit = 1;
    if (nrhs > 1) {
        const bool w64_free = L.W64 && woff != L.W64;
        split_buf = at<double>(work, w64_free ? L.W64 : L.krylov);
        const size_t cap = w64_free ? (size_t)L.npad * L.npad : (size_t)(2 * kKrylovMax + 2) * L.npad;
        const size_t per = (size_t)n * nrhs;
        const size_t smax = 1 + cap / per;
        const int want = n / 512 < 16 ? (n / 512 > 1 ? n / 512 : 1) : 16;
        nsplit = (size_t)want < smax ? want : (int)smax;
    }
    for (int k = 0;; ++k) {
        HIPCK(launch_fill_f64(rnorm, 0.0, nrhs, s));
        HIPCK(launch_fill_f64(xnorm, 0.0, nrhs, s));
        {
            ProfScope ps(PC_RESID, 2.0 * n * n * nrhs,
                         8.0 * n * n + 8.0 * n * nrhs * 3.0, s);
            if (nrhs > 1)
                HIPCK(launch_residual_mm(n, nrhs, A, lda, trans, X, ldx, B, ldb, cm, Rv, nrhs,
                                         rnorm, xnorm, split_buf, nsplit, s));
            else if (trans)
                HIPCK(launch_residual_t(n, nrhs, A, lda, X, ldx, B, ldb, cm, Rv, nrhs, rnorm,
                                        xnorm, at<double>(work, L.tmp), s));
            else
                HIPCK(launch_residual(n, nrhs, A, lda, X, ldx, B, ldb, cm, Rv, nrhs, rnorm, xnorm,
                                      s));
        }
        // hbuf: ||r|| of the nrhs columns, their ||x||, then the status words
        HIPCK(hipMemcpyAsync(ctx->hbuf, rnorm, (size_t)nrhs * 8, hipMemcpyDeviceToHost, s));
        HIPCK(hipMemcpyAsync(ctx->hbuf + nrhs, xnorm, (size_t)nrhs * 8, hipMemcpyDeviceToHost, s));
        HIPCK(hipMemcpyAsync(ctx->hbuf + 2 * nrhs, status, ST_COUNT * 4, hipMemcpyDeviceToHost,
                             s));
        HIPCK(hipStreamSynchronize(s));
        int stl[ST_COUNT];
        std::memcpy(stl, ctx->hbuf + 2 * nrhs, ST_COUNT * 4);
        if (stl[ST_TIMEOUT]) return MIXLU_ERR_DEVICE_TIMEOUT;
        const double *rn = ctx->hbuf;
        const double *xn = ctx->hbuf + nrhs;
        {
            double rmax = 0.0;
            for (int c = 0; c < nrhs; ++c) rmax = (rn[c] > rmax || rn[c] != rn[c]) ? rn[c] : rmax;
            ctx->hist.push_back(rmax);
        }
        bool all_ok = true, nonfinite = false, stalled = false;
        res.rnorm = 0.0;
        res.xnorm = 0.0;
        res.berr = 0.0;
        for (int c = 0; c < nrhs; ++c) {
            const double r = rn[c], x = xn[c];
            if (!std::isfinite(r) || !std::isfinite(x)) nonfinite = true;
            if (!(r <= thr * x)) all_ok = false;
            res.rnorm = std::fmax(res.rnorm, r);
            res.xnorm = std::fmax(res.xnorm, x);
            const double den = anorm * x;
            res.berr = std::fmax(res.berr, den > 0 ? r / den : (r > 0 ? INFINITY : 0.0));
            if (k >= 1 && prev[c] > 0 && !(r <= thr * x)) {
                const double rho = r / prev[c];
                if ((k >= 2 && rho >= o.stall && ratio_prev[c] >= o.stall) || (k >= 3 && rho >= 1.0))
                    stalled = true;
                ratio_prev[c] = rho;
            }
            prev[c] = r;
        }
        if (nonfinite) res.berr = NAN;
        if (all_ok && !nonfinite) {
            res.iters = k;
            res.converged = 1;
            return MIXLU_OK;
        }
        if (nonfinite || stalled) {
            res.iters = -4;
            return MIXLU_OK;
        }
        if (k == o.itermax) {
            res.iters = -(o.itermax + 1);
            return MIXLU_OK;
        }
        RETCK(lu_solve<Tw>(s, work, L, woff, nrhs, Rv, nrhs, 0, X, ldx, cm, 0, trans));
    }
}

// Flexible GMRES refinement (the outer FGMRES of Algorithm 2, with one
// application of the low-precision LU solve M = (LU)^{-1} P as the
// preconditioner in place of the inner single-precision GMRES): FP64
// Arnoldi with classical Gram-Schmidt applied twice, Givens rotations on the
// host, restarts every o.restart steps (default kKrylov).  At each restart the true residual is
// formed in FP64 and the stopping test of Section 3 decides; within a cycle
// the rotated residual norm ends the cycle early once it is below the
// threshold.  One right-hand side, A not transposed.  res.iters counts
// preconditioner applications; failure codes as for refine_loop, with the
// cycle count playing the role of the iteration count (itermax cycles) and
// a stall being two cycles in a row that cut the true residual by < 1%.
template <typename Tw>
int fgmres_loop(mixlu_ctx_s *ctx, void *work, const Layout &L, size_t woff, const double *A,
                int lda, const double *B, double *X, double anorm, const mixlu_opts &o,
                LoopResult &res) {
    hipStream_t s = ctx->stream;
    const int n = L.n, np = L.npad;
    const int m = o.restart > 0 ? (o.restart < kKrylovMax ? o.restart : kKrylovMax) : kKrylov;
    double *Rv = at<double>(work, L.vec_r);
    double *norms = at<double>(work, L.norms);
    double *rnorm = norms + 4, *xnorm = norms + 4 + L.nrhs;
    int *status = at<int>(work, L.status);
    double *K = at<double>(work, L.krylov);
    double *V = K;                                // m + 1 basis vectors
    double *Z = K + (size_t)(m + 1) * np;        // m preconditioned vectors
    double *zero = K + (size_t)(2 * m + 1) * np; // zero right-hand side
    double *hd = K + (size_t)(2 * m + 2) * np;   // 4 * m + 16 scalars
    double *h1 = hd, *h2 = hd + (m + 2), *yd = hd + 2 * (m + 2);
    RETCK(ensure_hbuf(ctx, (size_t)(4 * m + 32) * 8));
    double *hb = ctx->hbuf;
    const double thr = std::sqrt((double)n) * kEpsD * anorm;
    HIPCK(launch_fill_f64(zero, 0.0, (size_t)np, s));
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    auto Hat = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
    res = LoopResult{0, 0, 0.0, 0.0, 0.0};
    double prev = 0.0, ratio_prev = 0.0;
    int its = 0;
    for (int cyc = 0;; ++cyc) {
        HIPCK(launch_fill_f64(rnorm, 0.0, 1, s));
        HIPCK(launch_fill_f64(xnorm, 0.0, 1, s));
        {
            ProfScope ps(PC_RESID, 2.0 * n * n, 8.0 * n * n + 24.0 * n, s);
            HIPCK(launch_residual(n, 1, A, lda, X, 1, B, 1, 0, Rv, 1, rnorm, xnorm, s));
        }
        HIPCK(launch_dots(n, 1, Rv, np, Rv, h1, s));
        HIPCK(hipMemcpyAsync(hb, rnorm, 8, hipMemcpyDeviceToHost, s));
        HIPCK(hipMemcpyAsync(hb + 1, xnorm, 8, hipMemcpyDeviceToHost, s));
        HIPCK(hipMemcpyAsync(hb + 2, h1, 8, hipMemcpyDeviceToHost, s));
        HIPCK(hipMemcpyAsync(hb + 4, status, ST_COUNT * 4, hipMemcpyDeviceToHost, s));
        HIPCK(hipStreamSynchronize(s));
        int stl[ST_COUNT];
        std::memcpy(stl, hb + 4, ST_COUNT * 4);
        if (stl[ST_TIMEOUT]) return MIXLU_ERR_DEVICE_TIMEOUT;
        const double r = hb[0], xn = hb[1], beta = std::sqrt(hb[2]);
        ctx->hist.push_back(r);
        res.rnorm = r;
        res.xnorm = xn;
        res.berr = anorm * xn > 0 ? r / (anorm * xn) : (r > 0 ? INFINITY : 0.0);
        const bool finite = std::isfinite(r) && std::isfinite(xn) && std::isfinite(beta);
        if (finite && r <= thr * xn) {
            res.iters = its;
            res.converged = 1;
            return MIXLU_OK;
        }
        if (!finite) {
            res.berr = NAN;
            res.iters = -4;
            return MIXLU_OK;
        }
        // a restart cycle that does not cut the true residual by 1% made no
        // progress; two such cycles in a row end the iteration (a slowly
        // converging solve keeps going until itermax cycles)
        if (cyc >= 1 && prev > 0) {
            const bool none = !(r < 0.99 * prev);
            if (none && ratio_prev >= 1.0) {
                res.iters = -4;
                return MIXLU_OK;
            }
            ratio_prev = none ? 1.0 : 0.0;
        }
        prev = r;
        if (cyc == o.itermax) {
            res.iters = -(o.itermax + 1);
            return MIXLU_OK;
        }
        // Arnoldi cycle from v_0 = r / beta
        HIPCK(launch_scale_copy(n, 1.0 / beta, Rv, V, s));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int kk = 0;
        for (int k = 0; k < m && k < n; ++k) {
            double *vk = V + (size_t)k * np, *zk = Z + (size_t)k * np, *w = V + (size_t)(k + 1) * np;
            RETCK(lu_solve<Tw>(s, work, L, woff, 1, vk, 1, 0, zk, 1, 0, 1, 0));
            {
                ProfScope ps(PC_RESID, 2.0 * n * n, 8.0 * n * n + 24.0 * n, s);
                HIPCK(launch_residual(n, 1, A, lda, zk, 1, zero, 1, 0, w, 1, rnorm, xnorm, s));
            }
            HIPCK(launch_scale_copy(n, -1.0, w, w, s));  // w = A z_k
            HIPCK(launch_dots(n, k + 1, V, np, w, h1, s));
            HIPCK(launch_combine(n, k + 1, V, np, h1, -1.0, w, s));
            HIPCK(launch_dots(n, k + 1, V, np, w, h2, s));
            HIPCK(launch_combine(n, k + 1, V, np, h2, -1.0, w, s));
            HIPCK(launch_dots(n, 1, w, np, w, h2 + (k + 1), s));
            HIPCK(hipMemcpyAsync(hb, h1, (size_t)(k + 1) * 8, hipMemcpyDeviceToHost, s));
            HIPCK(hipMemcpyAsync(hb + (m + 2), h2, (size_t)(k + 2) * 8, hipMemcpyDeviceToHost, s));
            HIPCK(hipStreamSynchronize(s));
            for (int j = 0; j <= k; ++j) Hat(j, k) = hb[j] + hb[m + 2 + j];
            const double hn = std::sqrt(hb[m + 2 + k + 1]);
            Hat(k + 1, k) = hn;
            ++its;
            kk = k + 1;
            if (hn > 0 && std::isfinite(hn)) HIPCK(launch_scale_copy(n, 1.0 / hn, w, w, s));
            // Givens: rotate column k, then zero H(k+1, k)
            for (int j = 0; j < k; ++j) {
                const double t = cs[j] * Hat(j, k) + sn[j] * Hat(j + 1, k);
                Hat(j + 1, k) = -sn[j] * Hat(j, k) + cs[j] * Hat(j + 1, k);
                Hat(j, k) = t;
            }
            const double a = Hat(k, k), bq = Hat(k + 1, k);
            const double d = std::hypot(a, bq);
            cs[k] = d > 0 ? a / d : 1.0;
            sn[k] = d > 0 ? bq / d : 0.0;
            Hat(k, k) = d;
            Hat(k + 1, k) = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            const double est = std::fabs(g[k + 1]);
            if (!(hn > 0) || !std::isfinite(est) || est <= 0.5 * thr * xn) break;
        }
        // y = H^{-1} g (upper triangular kk x kk), x += Z y
        for (int i = kk - 1; i >= 0; --i) {
            double t = g[i];
            for (int j = i + 1; j < kk; ++j) t -= Hat(i, j) * y[j];
            y[i] = Hat(i, i) != 0 ? t / Hat(i, i) : 0.0;
        }
        std::memcpy(hb, y.data(), (size_t)kk * 8);
        HIPCK(hipMemcpyAsync(yd, hb, (size_t)kk * 8, hipMemcpyHostToDevice, s));
        HIPCK(launch_combine(n, kk, Z, np, yd, 1.0, X, s));
        HIPCK(hipStreamSynchronize(s));  // hb is reused by the next residual read
    }
}

// Argument checks shared by the solve entry points; `pn` is the 1-based
// position of n in the caller's signature, followed by nrhs, A, lda, B, ldb,
// X, ldx.
int check_common(mixlu_ctx_s *ctx, int pn, int n, int nrhs, int lda, int ldb, int ldx,
                 const void *A, const void *B, const void *X, int cm = 0) {
    if (!ctx) return -1;
    if (n < 0) return -pn;
    if (nrhs < 0) return -(pn + 1);
    if (n > 0 && !A) return -(pn + 2);
    if (lda < (n > 1 ? n : 1)) return -(pn + 3);
    const int ldmin = cm ? (n > 1 ? n : 1) : (nrhs > 1 ? nrhs : 1);
    if (n > 0 && nrhs > 0 && !B) return -(pn + 4);
    if (ldb < ldmin) return -(pn + 5);
    if (n > 0 && nrhs > 0 && !X) return -(pn + 6);
    if (ldx < ldmin) return -(pn + 7);
    return MIXLU_OK;
}

// Effective operation on the stored matrix M: a column-major A is read as
// the row-major M = A^T, so op(A) X = B becomes M^T X = B for op = identity.
// A symmetric (Cholesky) factor needs no transposition.
int eff_trans(const Layout &L, int trans, int cm) { return L.kind == 1 ? 0 : (trans ^ cm); }

mixlu_opts opts_or_default(const mixlu_opts *o) {
    mixlu_opts d;
    mixlu_default_opts(&d);
    return o ? *o : d;
}

// Index of a precision's batched tile set in the context.
int tile_slot(int prec) { return prec == MIXLU_FP64 ? 4 : (prec >= 0 && prec < 4 ? prec : 0); }

int equil_for(int prec, const mixlu_opts &o) {
    if (o.equilibrate >= 0) return o.equilibrate ? 1 : 0;
    return is_lowp(prec) ? 1 : 0;
}

// FP64 factor of A in the W64 region (or W when the factor itself is FP64),
// x solve, and (optionally) FP64 refinement; trans/cm as for lu_solve.
int fp64_path(mixlu_ctx_s *ctx, void *work, const Layout &L, size_t woff, const double *A,
              int lda, const double *B, int ldb, double *X, int ldx, int nrhs,
              const mixlu_opts &o, bool refine, int *info, LoopResult *res, int trans, int cm) {
    hipStream_t s = ctx->stream;
    RETCK(convert_and_factor<double>(ctx, work, L, woff, A, lda, 0, MIXLU_FP64));
    int st[ST_COUNT];
    double nrm[2];
    RETCK(read_status(ctx, L, work, st, nrm));
    if (st[ST_TIMEOUT]) return MIXLU_ERR_DEVICE_TIMEOUT;
    *info = breakdown_of(L, st) == INT_MAX ? 0 : breakdown_of(L, st);
    if (*info) return MIXLU_OK;
    RETCK(lu_solve<double>(s, work, L, woff, nrhs, B, ldb, cm, X, ldx, cm, 1, trans));
    if (refine) RETCK(refine_loop<double>(ctx, work, L, woff, A, lda, B, ldb, X, ldx, cm, nrhs,
                                          trans ? nrm[1] : nrm[0], o, *res, trans));
    return MIXLU_OK;
}

// Conversion and factorization of A into the workspace for op GESV (LU) or
// POSV (Cholesky) and fill F; status words are read back (synchronizes).
// d_info != null: stream-ordered, no synchronization; the outcome goes to
// *d_info (device) and F->lowp_status is left pending.
int factor_into(mixlu_ctx_s *ctx, const Layout &L, int prec, const double *A, int lda,
                void *work, size_t lwork, const mixlu_opts &o, mixlu_factor *F, int *info,
                int *d_info = nullptr) {
    fill_factor(F, L, work, lwork, o.layout);
    if (info) *info = 0;
    const int equil = equil_for(prec, o);
    F->equilibrated = equil;
    if (prec == MIXLU_FP64)
        RETCK(convert_and_factor<double>(ctx, work, L, L.W, A, lda, equil, MIXLU_FP64));
    else
        RETCK(convert_and_factor<float>(ctx, work, L, L.W, A, lda, equil, prec));
    if (d_info) {
        HIPCK(launch_factor_info(at<int>(work, L.status), L.kind == 1, prec == MIXLU_FP64, d_info,
                                 ctx->stream));
        F->lowp_status = MIXLU_FACTOR_PENDING;
        return MIXLU_OK;
    }
    int st[ST_COUNT];
    double nrm[2];
    RETCK(read_status(ctx, L, work, st, nrm));
    if (st[ST_TIMEOUT]) return MIXLU_ERR_DEVICE_TIMEOUT;
    const int brk = breakdown_of(L, st);
    if (prec == MIXLU_FP64) {
        *info = brk == INT_MAX ? 0 : brk;
    } else {
        if (st[ST_OVERFLOW]) F->lowp_status = -2;
        else if (brk != INT_MAX) F->lowp_status = -3;
    }
    return MIXLU_OK;
}

int factor_entry(mixlu_ctx_s *ctx, int op, int prec, int n, const double *A, int lda, void *work,
                 size_t lwork, const mixlu_opts *o, mixlu_factor *F, int *info,
                 int *d_info = nullptr) {
    if (!prec_valid(prec)) return -2;
    if (n < 0) return -3;
    if (n > 0 && !A) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (!work) return -6;
    if (!F) return -9;
    if (!info && !d_info) return -10;
    const mixlu_opts op_ = opts_or_default(o);
    if (op_.layout != MIXLU_ROW_MAJOR && op_.layout != MIXLU_COL_MAJOR) return -8;
    Layout L{};
    plan_layout(L, op, prec, n, 1, op_);
    if (lwork < L.total) return MIXLU_ERR_WORKSPACE;
    if (L.npad > kPanelMaxWG * kPanelRowsPerWG) return MIXLU_ERR_NOT_IMPLEMENTED;
    {
        // the factor serves as many right-hand sides as the workspace holds
        int lo = 1, hi = 2;
        Layout T{};
        while (hi <= (1 << 16) && plan_layout(T, op, prec, n, hi, op_) <= lwork) {
            lo = hi;
            hi *= 2;
        }
        while (hi - lo > 1) {
            const int mid = lo + (hi - lo) / 2;
            if (plan_layout(T, op, prec, n, mid, op_) <= lwork) lo = mid;
            else hi = mid;
        }
        plan_layout(L, op, prec, n, lo, op_);
    }
    if (n == 0) {
        fill_factor(F, L, work, lwork, op_.layout);
        if (d_info) HIPCK(launch_fill_u32(reinterpret_cast<unsigned *>(d_info), 0u, 1, ctx->stream));
        else *info = 0;
        return MIXLU_OK;
    }
    return factor_into(ctx, L, prec, A, lda, work, lwork, op_, F, info, d_info);
}

// Unit roundoff of the low-precision factor (C1 of the readings: eps_s).
double eps_of(int prec) {
    switch (prec) {
        case MIXLU_FP32: return 0x1p-24;
        case MIXLU_FP16: return 0x1p-11;
        case MIXLU_BF16: return 0x1p-8;
        case MIXLU_FP8: return 0x1p-4;
        default: return 0x1p-53;
    }
}

// kappa_1 estimate with the factors in F (see mixlu_condest).
int condest_impl(mixlu_ctx_s *ctx, const mixlu_factor *F, double *kappa1) {
    const Layout L = layout_of(F);
    const int n = L.n;
    void *work = F->work;
    hipStream_t s = ctx->stream;
    int st[ST_COUNT];
    double nrm[2];
    RETCK(read_status(ctx, L, work, st, nrm));
    // ||A||_1 (= ||A||_inf for the symmetric A of a Cholesky factor, whose
    // column sums are not formed)
    const double a1 = L.kind == 1 ? nrm[0] : nrm[1];
    if (n == 0 || !(a1 > 0.0)) {
        *kappa1 = 0.0;
        return MIXLU_OK;
    }
    const int cm = F->layout == MIXLU_COL_MAJOR;
    double *K = at<double>(work, L.krylov);
    double *x = K, *y = K + L.npad, *z = K + 2 * (size_t)L.npad, *out = K + 3 * (size_t)L.npad;
    RETCK(ensure_hbuf(ctx, 4096));
    auto solve = [&](const double *b, double *xo, int trans) -> int {
        const int tr = eff_trans(L, trans, cm);
        if (F->prec == MIXLU_FP64)
            return lu_solve<double>(s, work, L, L.W, 1, b, 1, 0, xo, 1, 0, 1, tr);
        return lu_solve<float>(s, work, L, L.W, 1, b, 1, 0, xo, 1, 0, 1, tr);
    };
    auto fetch = [&]() -> int {
        HIPCK(hipMemcpyAsync(ctx->hbuf, out, 4 * 8, hipMemcpyDeviceToHost, s));
        HIPCK(hipStreamSynchronize(s));
        return MIXLU_OK;
    };
    HIPCK(launch_cond_start(x, n, 0, s));
    double est = 0.0;
    int jprev = -1;
    for (int sweep = 0; sweep < 5; ++sweep) {
        RETCK(solve(x, y, 0));                           // y = A^{-1} x
        HIPCK(launch_cond_sign(y, n, z, out, s));        // z <- sign(y), ||y||_1
        RETCK(solve(z, z, 1));                           // z = A^{-T} sign(y)
        HIPCK(launch_cond_test(z, x, n, out, s));        // tests, x <- e_j
        RETCK(fetch());
        const double ynorm = ctx->hbuf[0], zinf = ctx->hbuf[1], ztx = ctx->hbuf[2];
        const int j = (int)ctx->hbuf[3];
        if (!(ynorm == ynorm) || !(zinf == zinf)) {
            est = ynorm;
            break;
        }
        est = ynorm > est ? ynorm : est;
        if (zinf <= ztx || j == jprev) break;  // no better vertex
        jprev = j;
    }
    // Higham's alternating vector guards against the cases the sweeps miss
    HIPCK(launch_cond_start(x, n, 1, s));
    RETCK(solve(x, y, 0));
    HIPCK(launch_cond_sign(y, n, z, out, s));
    RETCK(fetch());
    const double alt = 2.0 * ctx->hbuf[0] / (3.0 * n);
    if (alt > est || !(alt == alt)) est = alt;
    *kappa1 = a1 * est;
    return MIXLU_OK;
}

// One-shot solve (op GESV or POSV): factor, x_0, refinement, fallback.
int dx_entry(mixlu_ctx_s *ctx, int op, int prec, int n, int nrhs, const double *A, int lda,
             const double *B, int ldb, double *X, int ldx, void *work, size_t lwork,
             const mixlu_opts *o, mixlu_report *rep) {
    ctx->hist.clear();
    if (!prec_valid(prec)) return -2;
    const mixlu_opts op_ = opts_or_default(o);
    if (op_.layout != MIXLU_ROW_MAJOR && op_.layout != MIXLU_COL_MAJOR) return -13;
    const int cm = op_.layout == MIXLU_COL_MAJOR;
    RETCK(check_common(ctx, 3, n, nrhs, lda, ldb, ldx, A, B, X, cm));
    if (!work) return -11;
    if (!rep) return -14;
    std::memset(rep, 0, sizeof(*rep));
    Layout L{};
    plan_layout(L, op, prec, n, nrhs, op_);
    if (lwork < L.total) return MIXLU_ERR_WORKSPACE;
    if (n == 0 || nrhs == 0) {
        rep->converged = 1;
        rep->prec = prec;
        return MIXLU_OK;
    }
    if (L.npad > kPanelMaxWG * kPanelRowsPerWG) return MIXLU_ERR_NOT_IMPLEMENTED;
    mixlu_factor F;
    int info = 0;
    RETCK(factor_into(ctx, L, prec, A, lda, work, lwork, op_, &F, &info));
    if (info) {
        rep->info = info;
        rep->prec = MIXLU_FP64;
        rep->iter = -1;
        return MIXLU_OK;
    }
    double kest = 0.0;
    if (F.lowp_status == 0 && op_.condest && prec != MIXLU_FP64) {
        RETCK(condest_impl(ctx, &F, &kest));
        if (!(kest * eps_of(prec) < 1.0)) F.lowp_status = -5;
    }
    if (F.lowp_status == 0) {
        const int tr = eff_trans(L, 0, cm);
        if (prec == MIXLU_FP64)
            RETCK(lu_solve<double>(ctx->stream, work, L, L.W, nrhs, B, ldb, cm, X, ldx, cm, 1, tr));
        else
            RETCK(lu_solve<float>(ctx->stream, work, L, L.W, nrhs, B, ldb, cm, X, ldx, cm, 1, tr));
    }
    RETCK(mixlu_refine(ctx, &F, 0, nrhs, A, lda, B, ldb, X, ldx, &op_, rep));
    rep->cond_est = (float)kest;
    return MIXLU_OK;
}

// FP64 factorization and solve without refinement (op DGESV or DPOSV).
int d_entry(mixlu_ctx_s *ctx, int op, int n, int nrhs, const double *A, int lda, const double *B,
            int ldb, double *X, int ldx, void *work, size_t lwork, int *info) {
    RETCK(check_common(ctx, 2, n, nrhs, lda, ldb, ldx, A, B, X));
    if (!work) return -9;
    if (!info) return -11;
    mixlu_opts op_;
    mixlu_default_opts(&op_);
    Layout L{};
    plan_layout(L, op, MIXLU_FP64, n, nrhs, op_);
    if (lwork < L.total) return MIXLU_ERR_WORKSPACE;
    *info = 0;
    if (n == 0 || nrhs == 0) return MIXLU_OK;
    if (L.npad > kPanelMaxWG * kPanelRowsPerWG) return MIXLU_ERR_NOT_IMPLEMENTED;
    LoopResult res{};
    return fp64_path(ctx, work, L, L.W, A, lda, B, ldb, X, ldx, nrhs, op_, false, info, &res, 0,
                     0);
}


// FP32 factorization and FP32 solves, no equilibration and no refinement.
int s_entry(mixlu_ctx_s *ctx, int n, int nrhs, const double *A, int lda, const double *B,
            int ldb, double *X, int ldx, void *work, size_t lwork, int *info) {
    RETCK(check_common(ctx, 2, n, nrhs, lda, ldb, ldx, A, B, X));
    if (!work) return -9;
    if (!info) return -11;
    mixlu_opts op_;
    mixlu_default_opts(&op_);
    Layout L{};
    plan_layout(L, MIXLU_OP_SGESV, MIXLU_FP32, n, nrhs, op_);
    if (lwork < L.total) return MIXLU_ERR_WORKSPACE;
    *info = 0;
    if (n == 0 || nrhs == 0) return MIXLU_OK;
    if (L.npad > kPanelMaxWG * kPanelRowsPerWG) return MIXLU_ERR_NOT_IMPLEMENTED;
    RETCK(convert_and_factor<float>(ctx, work, L, L.W, A, lda, 0, MIXLU_FP32));
    int st[ST_COUNT];
    double nrm[2];
    RETCK(read_status(ctx, L, work, st, nrm));
    if (st[ST_TIMEOUT]) return MIXLU_ERR_DEVICE_TIMEOUT;
    if (st[ST_OVERFLOW]) {
        *info = n + 1;
        return MIXLU_OK;
    }
    const int brk = breakdown_of(L, st);
    if (brk != INT_MAX) {
        *info = brk;
        return MIXLU_OK;
    }
    RETCK(lu_solve<float>(ctx->stream, work, L, L.W, nrhs, B, ldb, 0, X, ldx, 0, 1, 0));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MIXLU_OK;
}

// ---------------------------------------------------------------- sparse
// Workspace of the sparse inner-outer solver (offsets in bytes).
struct SparseLayout {
    size_t vals_s;  // nnz values in the inner precision
    size_t Vo, Zo;  // outer FP64 basis (m_out + 1 vectors) and preconditioned vectors (m_out)
    size_t r, w;    // FP64 residual and work vector
    size_t Vi, wi;  // inner basis (m_in + 1) and work vector, inner precision
    size_t h;       // device scalars: two Gram-Schmidt passes and a squared norm
    size_t y;       // least-squares solution staged for the basis update (doubles)
    size_t part;    // partial sums of the dot products
    size_t norms;   // ||r||_inf, ||x||_inf
    size_t gm;      // inner GMRES least-squares state (doubles), then its two status ints
    size_t total;
};

size_t plan_sparse(SparseLayout &S, int inner_prec, int n, int nnz, int m_out, int m_in) {
    const size_t ts = inner_prec == MIXLU_FP64 ? 8 : 4;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const int mh = (m_out > m_in ? m_out : m_in) + 2;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at_ = off;
        off = align_up(off + bytes, 256);
        return at_;
    };
    S.vals_s = take((size_t)(nnz > 0 ? nnz : 1) * ts);
    S.Vo = take((size_t)(m_out + 1) * nn * 8);
    S.Zo = take((size_t)m_out * nn * 8);
    S.r = take(nn * 8);
    S.w = take(nn * 8);
    S.Vi = take((size_t)(m_in + 1) * nn * ts);
    S.wi = take(nn * ts);
    S.h = take((size_t)3 * mh * 8);
    S.y = take((size_t)mh * 8);
    S.part = take((size_t)mh * kVdotsChunks * 8);
    S.norms = take(4 * 8);
    S.gm = take(gmres_state_doubles(m_in > 0 ? m_in : 1) * 8 + 16);
    S.total = off;
    return off;
}

// Host side of one flexible/standard GMRES step: apply the earlier Givens
// rotations to column j of H (rows 0..j+1), make the new one, update g.
void givens_column(std::vector<double> &H, int ld, int j, std::vector<double> &cs,
                   std::vector<double> &sn, std::vector<double> &g) {
    auto Hat = [&](int i) -> double & { return H[(size_t)i * ld + j]; };
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hat(i) + sn[i] * Hat(i + 1);
        Hat(i + 1) = -sn[i] * Hat(i) + cs[i] * Hat(i + 1);
        Hat(i) = t;
    }
    const double a = Hat(j), b = Hat(j + 1);
    double c = 1.0, s = 0.0;
    if (b != 0.0) {
        const double r = std::hypot(a, b);
        c = a / r;
        s = b / r;
    }
    cs[j] = c;
    sn[j] = s;
    Hat(j) = c * a + s * b;
    Hat(j + 1) = 0.0;
    g[j + 1] = -s * g[j];
    g[j] = c * g[j];
}

// y solving the k x k upper triangle of the rotated H against g.
void back_substitute(const std::vector<double> &H, int ld, int k, const std::vector<double> &g,
                     std::vector<double> &y) {
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int q = i + 1; q < k; ++q) s -= H[(size_t)i * ld + q] * y[q];
        y[i] = s / H[(size_t)i * ld + i];
    }
}

// One Arnoldi step on device vectors: w is orthogonalized against the k
// basis vectors V (Gram-Schmidt twice, classical), its squared norm formed;
// the host receives H[0..k-1][j] (both passes summed) and ||w||_2.
template <typename T>
int arnoldi_orth(mixlu_ctx_s *ctx, int n, int k, const T *V, T *w, T *hdev, T *part,
                 std::vector<double> &col, double &wnorm) {
    hipStream_t s = ctx->stream;
    const size_t nn = (size_t)n;
    T *h1 = hdev, *h2 = hdev + k, *hn = hdev + 2 * k;
    HIPCK(launch_vdots<T>(n, k, V, nn, w, h1, part, s));
    HIPCK(launch_vcombine<T>(n, k, V, nn, h1, w, s));
    HIPCK(launch_vdots<T>(n, k, V, nn, w, h2, part, s));
    HIPCK(launch_vcombine<T>(n, k, V, nn, h2, w, s));
    HIPCK(launch_vdots<T>(n, 1, w, nn, w, hn, part, s));
    T *hb = reinterpret_cast<T *>(ctx->hbuf);
    HIPCK(hipMemcpyAsync(hb, hdev, (size_t)(2 * k + 1) * sizeof(T), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    for (int i = 0; i < k; ++i) col[i] = (double)hb[i] + (double)hb[k + i];
    wnorm = std::sqrt((double)hb[2 * k]);
    return MIXLU_OK;
}

// One GMRES(m) cycle from z = 0 for A z = v in precision T (values vals_t),
// v given in FP64 (v64); z (FP64) = V y.  Everything stays on the device:
// the Arnoldi vectors, the Givens rotations and the stopping test (the
// rotated residual against eps_rel ||v||) in k_gmres_col, and the back
// substitution, so the cycle is enqueued without a host round trip; the
// steps after an early stop still run but touch only vectors the update
// leaves out (it uses the steps taken, from the device).
template <typename T>
int inner_gmres(mixlu_ctx_s *ctx, const SparseLayout &S, void *work, int n, int nnz,
                const int *rowptr, const int *colind, const T *vals_t, const double *v64,
                double *z64, int m) {
    hipStream_t s = ctx->stream;
    const size_t nn = (size_t)n;
    T *Vi = at<T>(work, S.Vi), *w = at<T>(work, S.wi);
    T *hdev = at<T>(work, S.h);
    T *part = at<T>(work, S.part);
    double *ydev = at<double>(work, S.y);
    double *G = at<double>(work, S.gm);
    int *st = reinterpret_cast<int *>(G + gmres_state_doubles(m));
    const double eps_rel = sizeof(T) == 4 ? 0x1p-24 : 0x1p-53;
    // V_0 = v / ||v||
    HIPCK((launch_convert_vec<double, T>(nn, v64, w, s)));
    HIPCK(launch_vdots<T>(n, 1, w, nn, w, hdev, part, s));
    HIPCK(launch_gmres_init<T>(hdev, G, m, st, s));
    HIPCK(launch_vscale<T>(n, w, hdev, Vi, s));
    for (int j = 0; j < m; ++j) {
        {
            ProfScope ps(PC_SPMV, 2.0 * nnz, (double)nnz * (sizeof(T) + 4) + 2.0 * nn * sizeof(T), s);
            HIPCK(launch_csr_spmv<T>(n, rowptr, colind, vals_t, Vi + (size_t)j * nn, w, s));
        }
        // Gram-Schmidt twice against V_0..V_j, then ||w||^2
        const int k = j + 1;
        T *h1 = hdev, *h2 = hdev + k, *hn = hdev + 2 * k;
        HIPCK(launch_vdots<T>(n, k, Vi, nn, w, h1, part, s));
        HIPCK(launch_vcombine<T>(n, k, Vi, nn, h1, w, s));
        HIPCK(launch_vdots<T>(n, k, Vi, nn, w, h2, part, s));
        HIPCK(launch_vcombine<T>(n, k, Vi, nn, h2, w, s));
        HIPCK(launch_vdots<T>(n, 1, w, nn, w, hn, part, s));
        HIPCK(launch_gmres_col<T>(hdev, G, m, j, eps_rel, st, s));
        if (j + 1 < m) HIPCK(launch_vscale<T>(n, w, hn, Vi + (size_t)(j + 1) * nn, s));
    }
    HIPCK(launch_gmres_backsub(G, m, st, ydev, s));
    HIPCK(launch_fill_f64(z64, 0.0, nn, s));
    HIPCK((launch_vaxpy_basis<T, double>(n, m, Vi, nn, ydev, z64, s, st)));
    return MIXLU_OK;
}

// Algorithm 2 (FGMRES(m_out) in FP64 around one GMRES(m_in) cycle in
// precision T per outer step) from x = 0; see mixlu_sparse_fgmres.
template <typename T>
int sparse_solve(mixlu_ctx_s *ctx, const SparseLayout &S, void *work, int n, int nnz,
                 const int *rowptr, const int *colind, const double *vals, const double *b,
                 double *x, int m_out, int m_in, const mixlu_opts &o, mixlu_report *rep) {
    hipStream_t s = ctx->stream;
    const size_t nn = (size_t)n;
    const T *vals_t;
    if constexpr (sizeof(T) == 4) {
        float *vs = at<float>(work, S.vals_s);
        HIPCK((launch_convert_vec<double, float>((size_t)nnz, vals, vs, s)));
        vals_t = vs;
    } else {
        vals_t = vals;
    }
    double *Vo = at<double>(work, S.Vo), *Zo = at<double>(work, S.Zo);
    double *r = at<double>(work, S.r), *w = at<double>(work, S.w);
    double *hdev = at<double>(work, S.h), *ydev = at<double>(work, S.y);
    double *norms = at<double>(work, S.norms);
    double anorm = 0.0;
    HIPCK(launch_fill_f64(norms, 0.0, 2, s));
    HIPCK(launch_csr_norm_inf(n, rowptr, vals, norms, s));
    HIPCK(hipMemcpyAsync(ctx->hbuf, norms, 8, hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    anorm = ctx->hbuf[0];
    const double thr = std::sqrt((double)n) * kEpsD * anorm;
    HIPCK(launch_fill_f64(x, 0.0, nn, s));
    std::vector<double> col(m_out + 1), H((size_t)(m_out + 1) * m_out), cs(m_out), sn(m_out),
        g(m_out + 1), y(m_out);
    double bnorm_inf = 0.0;
    int inner_calls = 0, outer = 0;
    double prev = 0.0, ratio_prev = 0.0;
    double rn = 0.0, xn = 0.0;
    int reason = 0;
    for (int it = 0;; ++it) {
        HIPCK(launch_fill_f64(norms, 0.0, 2, s));
        HIPCK(launch_csr_resid(n, rowptr, colind, vals, x, b, r, norms, s));
        HIPCK(launch_vdots<double>(n, 1, r, nn, r, hdev, at<double>(work, S.part), s));
        HIPCK(hipMemcpyAsync(ctx->hbuf, norms, 16, hipMemcpyDeviceToHost, s));
        HIPCK(hipMemcpyAsync(ctx->hbuf + 2, hdev, 8, hipMemcpyDeviceToHost, s));
        HIPCK(hipStreamSynchronize(s));
        rn = ctx->hbuf[0];
        xn = ctx->hbuf[1];
        const double beta = std::sqrt(ctx->hbuf[2]);
        if (it == 0) bnorm_inf = rn;  // x = 0: r = b
        const bool finite = std::isfinite(rn) && std::isfinite(xn) && std::isfinite(beta);
        if (finite && rn <= thr * xn) break;
        if (!finite) {
            reason = -4;
            break;
        }
        if (it >= 1 && prev > 0.0) {
            const double rho = rn / prev;
            if ((it >= 2 && rho >= o.stall && ratio_prev >= o.stall) || (it >= 3 && rho >= 1.0)) {
                reason = -4;
                break;
            }
            ratio_prev = rho;
        }
        prev = rn;
        if (it == o.itermax) {
            reason = -(o.itermax + 1);
            break;
        }
        const double scale = std::max(xn, anorm > 0.0 ? bnorm_inf / anorm : 0.0);
        const double thr2 = thr * scale;
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        HIPCK(launch_vscale<double>(n, r, hdev, Vo, s));
        int k = 0;
        for (int j = 0; j < m_out; ++j) {
            RETCK(inner_gmres<T>(ctx, S, work, n, nnz, rowptr, colind, vals_t,
                                 Vo + (size_t)j * nn, Zo + (size_t)j * nn, m_in));
            ++inner_calls;
            {
                ProfScope ps(PC_SPMV, 2.0 * nnz, (double)nnz * 12 + 2.0 * nn * 8, s);
                HIPCK(launch_csr_spmv<double>(n, rowptr, colind, vals, Zo + (size_t)j * nn, w, s));
            }
            double wn = 0.0;
            RETCK(arnoldi_orth<double>(ctx, n, j + 1, Vo, w, hdev, at<double>(work, S.part),
                                       col, wn));
            for (int i = 0; i <= j; ++i) H[(size_t)i * m_out + j] = col[i];
            H[(size_t)(j + 1) * m_out + j] = wn;
            givens_column(H, m_out, j, cs, sn, g);
            k = j + 1;
            if (!(wn > 0.0) || std::fabs(g[j + 1]) <= thr2) break;
            if (j + 1 < m_out)
                HIPCK(launch_vscale<double>(n, w, hdev + 2 * (j + 1), Vo + (size_t)(j + 1) * nn,
                                            s));
        }
        back_substitute(H, m_out, k, g, y);
        double *hy = ctx->hbuf + 2048;
        for (int i = 0; i < k; ++i) hy[i] = y[i];
        HIPCK(hipMemcpyAsync(ydev, hy, (size_t)k * 8, hipMemcpyHostToDevice, s));
        HIPCK((launch_vaxpy_basis<double, double>(n, k, Zo, nn, ydev, x, s)));
        HIPCK(hipStreamSynchronize(s));
        ++outer;
    }
    rep->iter = reason ? reason : inner_calls;
    rep->converged = reason ? 0 : 1;
    rep->outer = outer;
    rep->anorm = anorm;
    rep->rnorm = rn;
    rep->xnorm = xn;
    rep->berr = (xn > 0.0 && anorm > 0.0) ? rn / (anorm * xn) : 0.0;
    return MIXLU_OK;
}

}  // namespace

// ======================================================================
// exported entry points
// ======================================================================
extern "C" {

const char *mixlu_status_string(int status) {
    switch (status) {
        case MIXLU_OK: return "MIXLU_OK";
        case MIXLU_ERR_HIP: return "MIXLU_ERR_HIP: a HIP runtime call failed";
        case MIXLU_ERR_WORKSPACE: return "MIXLU_ERR_WORKSPACE: workspace too small";
        case MIXLU_ERR_NOT_IMPLEMENTED: return "MIXLU_ERR_NOT_IMPLEMENTED";
        case MIXLU_ERR_UNSUPPORTED_ARCH: return "MIXLU_ERR_UNSUPPORTED_ARCH: needs gfx950";
        case MIXLU_ERR_DEVICE_TIMEOUT: return "MIXLU_ERR_DEVICE_TIMEOUT: a device wait gave up";
        case MIXLU_ERR_CAPTURING: return "MIXLU_ERR_CAPTURING: synchronizing call during capture";
        default: return status < 0 ? "invalid argument" : "unknown status";
    }
}

void mixlu_default_opts(mixlu_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->itermax = 30;
    o->equilibrate = -1;
    o->fallback = 1;
    o->nb = 0;
    o->layout = MIXLU_ROW_MAJOR;
    o->stall = 0.9;
    o->refine = MIXLU_REFINE_CLASSIC;
    o->restart = 0;
}

// ---------------------------------------------------------------------
// Device-resident scratch of the allocation-free batched solve: the work
// queue, its two counters and kNoAllocSlots factor slots, in one file-scope
// array that every GPU holds once the library's code is loaded there.  Host
// code reaches it only through the address hipGetSymbolAddress returns on
// each device (the array's name is a host-side stand-in, not a device
// address).  Calls that overlap on one GPU share it and race.
// ---------------------------------------------------------------------
namespace {
constexpr int kNoAllocSlots = 32;        // persistent workgroups (and slots)
constexpr int kNoAllocMaxBatch = 65536;  // systems per call
constexpr size_t kNoAllocOrderBytes = (size_t)kNoAllocMaxBatch * 4;
constexpr size_t kNoAllocSlotBytes = (size_t)kBatchedNmax * kBatchedNmax * 8;
constexpr size_t kNoAllocBytes = kNoAllocOrderBytes + 256 + kNoAllocSlots * kNoAllocSlotBytes;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Address of this device's copy of `scratch` (device `dev` must be current
// on first use); null if the lookup failed.
static void *scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

int mixlu_create(mixlu_ctx_t *ctx, void *stream) {
    if (!ctx) return -1;
    *ctx = nullptr;
    int dev = 0;
    HIPCK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MIXLU_ERR_UNSUPPORTED_ARCH;
    auto *c = new mixlu_ctx_s;
    c->device = dev;
    c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->stream = static_cast<hipStream_t>(stream);
    // the allocation-free batched solve's scratch on this device (checked
    // again by that entry point, which reports a failed lookup)
    (void)scratch_on(dev);
    *ctx = c;
    return MIXLU_OK;
}

int mixlu_destroy(mixlu_ctx_t ctx) {
    if (!ctx) return -1;
    if (ctx->hbuf) (void)hipHostFree(ctx->hbuf);
    if (ctx->side) {
        (void)hipStreamSynchronize(ctx->side);
        (void)hipStreamDestroy(ctx->side);
        (void)hipEventDestroy(ctx->ev_fork);
        (void)hipEventDestroy(ctx->ev_join);
        (void)hipEventDestroy(ctx->ev_next);
    }
    for (auto &q : ctx->prof.pending) {
        (void)hipEventDestroy(q.a);
        (void)hipEventDestroy(q.b);
    }
    for (auto e : ctx->prof.pool) (void)hipEventDestroy(e);
    delete ctx;
    return MIXLU_OK;
}

int mixlu_set_stream(mixlu_ctx_t ctx, void *stream) {
    if (!ctx) return -1;
    ctx->stream = static_cast<hipStream_t>(stream);
    return MIXLU_OK;
}

int mixlu_workspace_size(mixlu_ctx_t ctx, int op, int prec, int n, int nrhs,
                         const mixlu_opts *o, size_t *bytes) {
    if (!ctx) return -1;
    if (op < MIXLU_OP_GESV || op > MIXLU_OP_SGESV) return -2;
    if (!prec_valid(prec)) return -3;
    if (n < 0) return -4;
    if (nrhs < 0) return -5;
    if (!bytes) return -7;
    const mixlu_opts op_ = opts_or_default(o);
    Layout L{};
    *bytes = plan_layout(L, op, prec, n, nrhs, op_);
    return MIXLU_OK;
}

int mixlu_getrf(mixlu_ctx_t ctx, int prec, int n, const double *A, int lda, void *work,
                size_t lwork, const mixlu_opts *o, mixlu_factor *F, int *info) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    return factor_entry(ctx, MIXLU_OP_GESV, prec, n, A, lda, work, lwork, o, F, info);
}

int mixlu_potrf(mixlu_ctx_t ctx, int prec, int n, const double *A, int lda, void *work,
                size_t lwork, const mixlu_opts *o, mixlu_factor *F, int *info) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    return factor_entry(ctx, MIXLU_OP_POSV, prec, n, A, lda, work, lwork, o, F, info);
}

int mixlu_getrf_async(mixlu_ctx_t ctx, int prec, int n, const double *A, int lda, void *work,
                      size_t lwork, const mixlu_opts *o, mixlu_factor *F, int *d_info) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    return factor_entry(ctx, MIXLU_OP_GESV, prec, n, A, lda, work, lwork, o, F, nullptr, d_info);
}

int mixlu_potrf_async(mixlu_ctx_t ctx, int prec, int n, const double *A, int lda, void *work,
                      size_t lwork, const mixlu_opts *o, mixlu_factor *F, int *d_info) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    return factor_entry(ctx, MIXLU_OP_POSV, prec, n, A, lda, work, lwork, o, F, nullptr, d_info);
}

int mixlu_getrs(mixlu_ctx_t ctx, const mixlu_factor *F, int trans, const int nrhs,
                const double *B, int ldb, double *X, int ldx) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    if (!F || !F->work) return -2;
    if (trans != 0 && trans != 1) return -3;
    const int cm = F->layout == MIXLU_COL_MAJOR;
    const int ldmin = cm ? (F->n > 1 ? F->n : 1) : (nrhs > 1 ? nrhs : 1);
    if (nrhs < 0 || nrhs > F->nrhs_max) return -4;
    if (nrhs > 0 && F->n > 0 && !B) return -5;
    if (ldb < ldmin) return -6;
    if (nrhs > 0 && F->n > 0 && !X) return -7;
    if (ldx < ldmin) return -8;
    if (F->n == 0 || nrhs == 0) return MIXLU_OK;
    const Layout L = layout_of(F);
    const int tr = eff_trans(L, trans, cm);
    if (F->prec == MIXLU_FP64)
        return lu_solve<double>(ctx->stream, F->work, L, L.W, nrhs, B, ldb, cm, X, ldx, cm, 1, tr);
    return lu_solve<float>(ctx->stream, F->work, L, L.W, nrhs, B, ldb, cm, X, ldx, cm, 1, tr);
}

int mixlu_refine(mixlu_ctx_t ctx, mixlu_factor *F, int trans, int nrhs, const double *A,
                 int lda, const double *B, int ldb, double *X, int ldx, const mixlu_opts *o,
                 mixlu_report *rep) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    ctx->hist.clear();
    if (!F || !F->work) return -2;
    if (trans != 0 && trans != 1) return -3;
    if (nrhs < 0 || nrhs > F->nrhs_max) return -4;
    if (F->n > 0 && !A) return -5;
    if (lda < (F->n > 1 ? F->n : 1)) return -6;
    if (!rep) return -12;
    const mixlu_opts op_ = opts_or_default(o);
    const int cm = F->layout == MIXLU_COL_MAJOR;
    const int ldmin = cm ? (F->n > 1 ? F->n : 1) : (nrhs > 1 ? nrhs : 1);
    if (!B && F->n > 0 && nrhs > 0) return -7;
    if (ldb < ldmin) return -8;
    if (!X && F->n > 0 && nrhs > 0) return -9;
    if (ldx < ldmin) return -10;
    std::memset(rep, 0, sizeof(*rep));
    rep->prec = F->prec;
    if (F->n == 0 || nrhs == 0) {
        rep->converged = 1;
        return MIXLU_OK;
    }
    const Layout L = layout_of(F);
    const int tr = eff_trans(L, trans, cm);
    int st[ST_COUNT];
    double nrm[2];
    RETCK(read_status(ctx, L, F->work, st, nrm));
    if (F->lowp_status == MIXLU_FACTOR_PENDING) {
        // outcome of an asynchronous factorization, known from here on
        if (st[ST_TIMEOUT]) return MIXLU_ERR_DEVICE_TIMEOUT;
        const int brk = breakdown_of(L, st);
        if (F->prec == MIXLU_FP64) F->lowp_status = brk != INT_MAX ? -1 : 0;
        else F->lowp_status = st[ST_OVERFLOW] ? -2 : (brk != INT_MAX ? -3 : 0);
        if (F->prec == MIXLU_FP64 && brk != INT_MAX) rep->info = brk;
    }
    // ||M^T||_inf = ||M||_1 when the solve is with the transposed matrix
    const double anorm = tr ? nrm[1] : nrm[0];
    rep->anorm = anorm;
    LoopResult res{};
    int reason = F->lowp_status;
    if (reason == 0) {
        // flexible GMRES for one right-hand side of A (not A^T); otherwise
        // the stationary refinement of Algorithm 1
        const bool krylov = op_.refine == MIXLU_REFINE_FGMRES && nrhs == 1 && !tr && ldb == 1 &&
                            ldx == 1;
        if (krylov && F->prec == MIXLU_FP64)
            RETCK(fgmres_loop<double>(ctx, F->work, L, L.W, A, lda, B, X, anorm, op_, res));
        else if (krylov)
            RETCK(fgmres_loop<float>(ctx, F->work, L, L.W, A, lda, B, X, anorm, op_, res));
        else if (F->prec == MIXLU_FP64)
            RETCK(refine_loop<double>(ctx, F->work, L, L.W, A, lda, B, ldb, X, ldx, cm, nrhs,
                                      anorm, op_, res, tr));
        else
            RETCK(refine_loop<float>(ctx, F->work, L, L.W, A, lda, B, ldb, X, ldx, cm, nrhs,
                                     anorm, op_, res, tr));
        reason = res.converged ? 0 : res.iters;
    }
    if (reason == 0) {
        rep->iter = res.iters;
        rep->converged = 1;
        rep->rnorm = res.rnorm;
        rep->xnorm = res.xnorm;
        rep->berr = res.berr;
        return MIXLU_OK;
    }
    rep->iter = reason;
    if (F->prec == MIXLU_FP64 || !L.fallback) {
        rep->rnorm = res.rnorm;
        rep->xnorm = res.xnorm;
        rep->berr = res.berr;
        return MIXLU_OK;
    }
    int info = 0;
    LoopResult fres{};
    RETCK(fp64_path(ctx, F->work, L, L.W64, A, lda, B, ldb, X, ldx, nrhs, op_, true, &info, &fres,
                    tr, cm));
    // The FP64 factorization rewrote the pivots, permutation, scales and
    // status words that the low-precision factor in W shares with it.  From
    // here on F describes the FP64 factor in W64 (unit scales, no further
    // fallback), so later solves, refinements and estimates with F use
    // consistent data instead of mixing the two factorizations.
    F->prec = MIXLU_FP64;
    F->equilibrated = 0;
    F->off[0] = L.W64;
    F->off[1] = 0;
    F->lowp_status = info ? -1 : 0;
    {
        // the inverse diagonal blocks where the rewritten description looks
        // for them (over the low-precision factor's, which are abandoned)
        const Layout L2 = layout_of(F);
        HIPCK(launch_tri_inv<double>(at<double>(F->work, L.W64), L.npad, L.npad,
                                     at<double>(F->work, L2.dinv), ctx->stream));
    }
    rep->info = info;
    rep->prec = MIXLU_FP64;
    rep->fallback_iter = fres.iters;
    rep->converged = fres.converged;
    rep->rnorm = fres.rnorm;
    rep->xnorm = fres.xnorm;
    rep->berr = fres.berr;
    return MIXLU_OK;
}

int mixlu_dxgesv(mixlu_ctx_t ctx, int prec, int n, int nrhs, const double *A, int lda,
                 const double *B, int ldb, double *X, int ldx, void *work, size_t lwork,
                 const mixlu_opts *o, mixlu_report *rep) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    return dx_entry(ctx, MIXLU_OP_GESV, prec, n, nrhs, A, lda, B, ldb, X, ldx, work, lwork, o,
                    rep);
}

int mixlu_dxposv(mixlu_ctx_t ctx, int prec, int n, int nrhs, const double *A, int lda,
                 const double *B, int ldb, double *X, int ldx, void *work, size_t lwork,
                 const mixlu_opts *o, mixlu_report *rep) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    return dx_entry(ctx, MIXLU_OP_POSV, prec, n, nrhs, A, lda, B, ldb, X, ldx, work, lwork, o,
                    rep);
}

int mixlu_dgesv(mixlu_ctx_t ctx, int n, int nrhs, const double *A, int lda, const double *B,
                int ldb, double *X, int ldx, void *work, size_t lwork, int *info) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    return d_entry(ctx, MIXLU_OP_DGESV, n, nrhs, A, lda, B, ldb, X, ldx, work, lwork, info);
}

int mixlu_condest(mixlu_ctx_t ctx, const mixlu_factor *F, double *kappa1) {
    if (!ctx) return -1;
    if (!F || !F->work) return -2;
    if (!kappa1) return -3;
    ProfCall pc_(ctx);
    return condest_impl(ctx, F, kappa1);
}

int mixlu_sgesv(mixlu_ctx_t ctx, int n, int nrhs, const double *A, int lda, const double *B,
                int ldb, double *X, int ldx, void *work, size_t lwork, int *info) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    return s_entry(ctx, n, nrhs, A, lda, B, ldb, X, ldx, work, lwork, info);
}

int mixlu_sparse_workspace_size(mixlu_ctx_t ctx, int inner_prec, int n, int nnz, int m_out,
                                int m_in, size_t *bytes) {
    if (!ctx) return -1;
    if (inner_prec != MIXLU_FP32 && inner_prec != MIXLU_FP64) return -2;
    if (n < 0) return -3;
    if (nnz < 0) return -4;
    if (m_out < 1 || m_out > kSparseMaxRestart) return -5;
    if (m_in < 1 || m_in > kSparseMaxRestart) return -6;
    if (!bytes) return -7;
    SparseLayout S{};
    *bytes = plan_sparse(S, inner_prec, n, nnz, m_out, m_in);
    return MIXLU_OK;
}

int mixlu_sparse_fgmres(mixlu_ctx_t ctx, int inner_prec, int n, int nnz, const int *rowptr,
                        const int *colind, const double *vals, const double *b, double *x,
                        int m_out, int m_in, void *work, size_t lwork, const mixlu_opts *o,
                        mixlu_report *rep) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    if (inner_prec != MIXLU_FP32 && inner_prec != MIXLU_FP64) return -2;
    if (n < 0) return -3;
    if (nnz < 0) return -4;
    if (n > 0 && !rowptr) return -5;
    if (nnz > 0 && !colind) return -6;
    if (nnz > 0 && !vals) return -7;
    if (n > 0 && !b) return -8;
    if (n > 0 && !x) return -9;
    if (m_out < 1 || m_out > kSparseMaxRestart) return -10;
    if (m_in < 1 || m_in > kSparseMaxRestart) return -11;
    if (n > 0 && !work) return -12;
    if (!rep) return -15;
    std::memset(rep, 0, sizeof(*rep));
    rep->prec = inner_prec;
    SparseLayout S{};
    if (lwork < plan_sparse(S, inner_prec, n, nnz, m_out, m_in)) return MIXLU_ERR_WORKSPACE;
    if (n == 0) {
        rep->converged = 1;
        return MIXLU_OK;
    }
    const mixlu_opts op_ = opts_or_default(o);
    RETCK(ensure_hbuf(ctx, (size_t)(2048 + 2 * kSparseMaxRestart + 16) * 8));
    if (inner_prec == MIXLU_FP32)
        return sparse_solve<float>(ctx, S, work, n, nnz, rowptr, colind, vals, b, x, m_out, m_in,
                                   op_, rep);
    return sparse_solve<double>(ctx, S, work, n, nnz, rowptr, colind, vals, b, x, m_out, m_in,
                                op_, rep);
}

int mixlu_report_read(mixlu_ctx_t ctx, const mixlu_report *d, int count, mixlu_report *h) {
    if (!ctx) return -1;
    if (count < 0) return -3;
    if (count > 0 && !d) return -2;
    if (count > 0 && !h) return -4;
    if (count == 0) return MIXLU_OK;
    HIPCK(hipMemcpyAsync(h, d, (size_t)count * sizeof(mixlu_report), hipMemcpyDeviceToHost,
                         ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MIXLU_OK;
}

int mixlu_dposv(mixlu_ctx_t ctx, int n, int nrhs, const double *A, int lda, const double *B,
                int ldb, double *X, int ldx, void *work, size_t lwork, int *info) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    return d_entry(ctx, MIXLU_OP_DPOSV, n, nrhs, A, lda, B, ldb, X, ldx, work, lwork, info);
}

int mixlu_batched_workspace_size(mixlu_ctx_t ctx, int prec, int batch, int nrhs,
                                 const mixlu_opts *o, size_t *bytes) {
    if (!ctx) return -1;
    if (!prec_valid(prec) || prec == MIXLU_FP8) return -2;
    if (batch < 0) return -3;
    if (nrhs < 1) return -4;
    if (!bytes) return -6;
    (void)o;
    const size_t slots = (size_t)(batch < kBatchedSlots ? batch : kBatchedSlots);
    *bytes = align_up((size_t)batch * 4, 256) + 256 + slots * batched_slot_bytes();
    return MIXLU_OK;
}

int mixlu_dxgesv_batched(mixlu_ctx_t ctx, int prec, int batch, const int *d_n,
                         const double *const *d_A, const int *d_lda, const double *const *d_B,
                         double *const *d_X, int nrhs, void *work, size_t lwork,
                         const mixlu_opts *o, mixlu_report *d_reps) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    if (!prec_valid(prec)) return -2;
    if (prec == MIXLU_FP8) return MIXLU_ERR_NOT_IMPLEMENTED;
    if (batch < 0) return -3;
    if (batch > 0 && !d_n) return -4;
    if (batch > 0 && !d_A) return -5;
    if (batch > 0 && !d_B) return -7;
    if (batch > 0 && !d_X) return -8;
    if (nrhs < 1) return -9;
    if (batch > 0 && !work) return -10;
    if (batch > 0 && !d_reps) return -13;
    const mixlu_opts op_ = opts_or_default(o);
    if (op_.layout != MIXLU_ROW_MAJOR) return MIXLU_ERR_NOT_IMPLEMENTED;
    size_t need = 0;
    RETCK(mixlu_batched_workspace_size(ctx, prec, batch, nrhs, &op_, &need));
    if (lwork < need) return MIXLU_ERR_WORKSPACE;
    if (batch == 0) return MIXLU_OK;
    auto *base = static_cast<unsigned char *>(work);
    int *order = reinterpret_cast<int *>(base);
    int *counter = reinterpret_cast<int *>(base + align_up((size_t)batch * 4, 256));
    void *slots = base + align_up((size_t)batch * 4, 256) + 256;
    const int nslots = batch < kBatchedSlots ? batch : kBatchedSlots;
    ProfScope ps(PC_BATCH, 0.0, 0.0, ctx->stream);
    HIPCK(launch_batched(prec, batch, nrhs, equil_for(prec, op_), op_.itermax, op_.stall,
                         prec != MIXLU_FP64 && op_.fallback, d_n, d_A, d_lda, d_B, d_X, d_reps,
                         order, counter, slots, nslots, ctx->btiles[tile_slot(prec)],
                         ctx->num_cu, ctx->stream));
    return MIXLU_OK;
}

int mixlu_dxgesv_batched_noalloc(mixlu_ctx_t ctx, int prec, int batch, const int *d_n,
                                 const double *const *d_A, const int *d_lda,
                                 const double *const *d_B, double *const *d_X, int nrhs,
                                 const mixlu_opts *o, mixlu_report *d_reps) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    if (!prec_valid(prec)) return -2;
    if (prec == MIXLU_FP8) return MIXLU_ERR_NOT_IMPLEMENTED;
    if (batch < 0) return -3;
    if (batch > 0 && !d_n) return -4;
    if (batch > 0 && !d_A) return -5;
    if (batch > 0 && !d_B) return -7;
    if (batch > 0 && !d_X) return -8;
    if (nrhs < 1) return -9;
    if (batch > 0 && !d_reps) return -11;
    if (batch > kNoAllocMaxBatch) return MIXLU_ERR_WORKSPACE;
    const mixlu_opts op_ = opts_or_default(o);
    if (op_.layout != MIXLU_ROW_MAJOR) return MIXLU_ERR_NOT_IMPLEMENTED;
    if (batch == 0) return MIXLU_OK;
    auto *base = static_cast<unsigned char *>(scratch_on(ctx->device));
    if (!base) return MIXLU_ERR_HIP;
    int *order = reinterpret_cast<int *>(base);
    int *counter = reinterpret_cast<int *>(base + kNoAllocOrderBytes);  // reset by the launch
    void *slots = base + kNoAllocOrderBytes + 256;
    const int nslots = batch < kNoAllocSlots ? batch : kNoAllocSlots;
    ProfScope ps(PC_BATCH, 0.0, 0.0, ctx->stream);
    HIPCK(launch_batched(prec, batch, nrhs, equil_for(prec, op_), op_.itermax, op_.stall,
                         prec != MIXLU_FP64 && op_.fallback, d_n, d_A, d_lda, d_B, d_X, d_reps,
                         order, counter, slots, nslots, ctx->btiles[tile_slot(prec)],
                         ctx->num_cu, ctx->stream));
    return MIXLU_OK;
}

int mixlu_batched_get_tiles(mixlu_ctx_t ctx, int prec, mixlu_batched_tiles *t) {
    if (!ctx) return -1;
    if (!prec_valid(prec) || prec == MIXLU_FP8) return -2;
    if (!t) return -3;
    const BatchedTiles &b = ctx->btiles[tile_slot(prec)];
    t->panel = b.panel;
    t->chunk = b.chunk;
    t->groups = b.groups;
    t->tuned = ctx->btuned[tile_slot(prec)];
    return MIXLU_OK;
}

int mixlu_batched_set_tiles(mixlu_ctx_t ctx, int prec, const mixlu_batched_tiles *t) {
    if (!ctx) return -1;
    if (!prec_valid(prec) || prec == MIXLU_FP8) return -2;
    if (!t) return -3;
    const BatchedTiles b{t->panel, t->chunk, t->groups};
    if (!batched_tiles_valid(b)) return -3;
    ctx->btiles[tile_slot(prec)] = b;
    ctx->btuned[tile_slot(prec)] = t->tuned ? 1 : 0;
    return MIXLU_OK;
}

int mixlu_batched_tune(mixlu_ctx_t ctx, int prec, int batch, const int *d_n,
                       const double *const *d_A, const int *d_lda, const double *const *d_B,
                       double *const *d_X, int nrhs, void *work, size_t lwork,
                       const mixlu_opts *o, mixlu_report *d_reps, mixlu_batched_tiles *best,
                       float *ms, int max_ms) {
    if (!ctx) return -1;
    if (!prec_valid(prec) || prec == MIXLU_FP8) return -2;
    if (max_ms < 0 || (max_ms > 0 && !ms)) return -16;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCK(hipStreamIsCapturing(ctx->stream, &cap));
    if (cap != hipStreamCaptureStatusNone) return MIXLU_ERR_CAPTURING;
    const int slot = tile_slot(prec);
    const BatchedTiles saved = ctx->btiles[slot];
    const int saved_tuned = ctx->btuned[slot];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MIXLU_ERR_HIP;
    }
    int rc = MIXLU_OK;
    float best_ms = 0.0f;
    BatchedTiles best_t = saved;
    int idx = 0;
    for (int panel : {16, 8}) {
        for (int chunk : {128, 64, 32}) {
            for (int groups : {2, 1}) {
                ctx->btiles[slot] = BatchedTiles{panel, chunk, groups};
                float t_min = 0.0f;
                for (int rep = 0; rep < 3 && rc == MIXLU_OK; ++rep) {
                    if (hipEventRecord(e0, ctx->stream) != hipSuccess) rc = MIXLU_ERR_HIP;
                    if (rc == MIXLU_OK)
                        rc = mixlu_dxgesv_batched(ctx, prec, batch, d_n, d_A, d_lda, d_B, d_X,
                                                  nrhs, work, lwork, o, d_reps);
                    if (rc == MIXLU_OK && (hipEventRecord(e1, ctx->stream) != hipSuccess ||
                                           hipEventSynchronize(e1) != hipSuccess))
                        rc = MIXLU_ERR_HIP;
                    float t = 0.0f;
                    if (rc == MIXLU_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess)
                        rc = MIXLU_ERR_HIP;
                    if (rep == 1 || (rep == 2 && t < t_min)) t_min = t;  // run 0 is untimed
                }
                if (rc != MIXLU_OK) break;
                if (idx < max_ms) ms[idx] = t_min;
                if (idx == 0 || t_min < best_ms) {
                    best_ms = t_min;
                    best_t = ctx->btiles[slot];
                }
                ++idx;
            }
            if (rc != MIXLU_OK) break;
        }
        if (rc != MIXLU_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != MIXLU_OK) {
        ctx->btiles[slot] = saved;
        ctx->btuned[slot] = saved_tuned;
        return rc;
    }
    ctx->btiles[slot] = best_t;
    ctx->btuned[slot] = 1;
    if (best) {
        best->panel = best_t.panel;
        best->chunk = best_t.chunk;
        best->groups = best_t.groups;
        best->tuned = 1;
    }
    return MIXLU_OK;
}

int mixlu_profile_enable(mixlu_ctx_t ctx, int on) {
    if (!ctx) return -1;
    if (on) {
        for (auto &c : ctx->prof.acc) c = ProfAcc{};
        ctx->prof.pending.clear();
    }
    ctx->prof.on = on != 0;
    return MIXLU_OK;
}

int mixlu_profile_read(mixlu_ctx_t ctx, mixlu_kstat *out, int max, int *count) {
    if (!ctx) return -1;
    if (max < 0 || (max > 0 && !out)) return -2;
    if (!count) return -4;
    HIPCK(hipStreamSynchronize(ctx->stream));
    prof_harvest(ctx->prof);
    const int nout = max < PC_COUNT ? max : PC_COUNT;
    for (int i = 0; i < nout; ++i) {
        out[i].name = kProfNames[i];
        out[i].launches = ctx->prof.acc[i].launches;
        out[i].ms = ctx->prof.acc[i].ms;
        out[i].flops = ctx->prof.acc[i].flops;
        out[i].bytes = ctx->prof.acc[i].bytes;
    }
    *count = PC_COUNT;
    return MIXLU_OK;
}

int mixlu_refine_history(mixlu_ctx_t ctx, double *h, int max, int *count) {
    if (!ctx) return -1;
    if (max < 0 || (max > 0 && !h)) return -3;
    if (!count) return -4;
    const int c = (int)ctx->hist.size();
    *count = c;
    for (int i = 0; i < c && i < max; ++i) h[i] = ctx->hist[i];
    return MIXLU_OK;
}

int mixlu_gemm_update(mixlu_ctx_t ctx, int prec, int m, int n, int k, const float *A, int lda,
                      const float *B, int ldb, float *C, int ldc, void *work, size_t lwork,
                      int *overflow) {
    if (!ctx) return -1;
    ProfCall pc_(ctx);
    if (prec != MIXLU_FP32 && !is_lowp(prec)) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0 || (is_lowp(prec) && k % (prec == MIXLU_FP8 ? 128 : 64))) return -5;
    if (m > 0 && k > 0 && !A) return -6;
    if (lda < (k > 1 ? k : 1)) return -7;
    if (k > 0 && n > 0 && !B) return -8;
    if (ldb < (n > 1 ? n : 1)) return -9;
    if (m > 0 && n > 0 && !C) return -10;
    if (ldc < (n > 1 ? n : 1)) return -11;
    const size_t mk = (size_t)m * k, nk = (size_t)n * k;
    const size_t need = 2 * (mk + nk) + (mk + nk) / 32 + 1024;
    if (is_lowp(prec) && !work) return -12;
    if (is_lowp(prec) && lwork < need) return MIXLU_ERR_WORKSPACE;
    hipStream_t s = ctx->stream;
    if (overflow) *overflow = 0;
    if (m == 0 || n == 0 || k == 0) return MIXLU_OK;
    if (prec == MIXLU_FP32) {
        ProfScope ps(PC_TRAIL, 2.0 * m * n * k, 8.0 * m * n + 4.0 * (mk + nk), s);
        HIPCK(launch_gemm<float>(m, n, k, A, lda, B, ldb, C, ldc, s));
        return MIXLU_OK;
    }
    auto *base = static_cast<unsigned char *>(work);
    int *status = reinterpret_cast<int *>(base);
    const bool f8 = prec == MIXLU_FP8;
    const size_t esz = f8 ? 1 : 2;
    unsigned char *Ap = base + 256;
    unsigned char *Bp = Ap + align_up(mk * esz, 256);
    unsigned char *As = Bp + align_up(nk * esz, 256);
    unsigned char *Bs = As + align_up(mk / 32, 256);
    HIPCK(launch_fill_u32(reinterpret_cast<unsigned *>(status), 0u, ST_COUNT, s));
    {
        ProfScope ps(PC_PACK, 0.0, (4.0 + esz) * (mk + nk), s);
        if (f8) {
            HIPCK(launch_pack_fp8(A, lda, m, k, 0, Ap, As, status, s));
            HIPCK(launch_pack_fp8(B, ldb, n, k, 1, Bp, Bs, status, s));
        } else {
            HIPCK(launch_pack(prec, A, lda, m, k, 0, Ap, status, s));
            HIPCK(launch_pack(prec, B, ldb, k, n, 1, Bp, status, s));
        }
    }
    {
        ProfScope ps(PC_TRAIL, 2.0 * m * n * k, 8.0 * m * n + 1.0 * esz * (mk + nk), s);
        if (f8)
            HIPCK(launch_gemm_fp8(m, n, k, Ap, As, Bp, Bs, C, ldc, s));
        else
            HIPCK(launch_gemm_lowp(prec, m, n, k, Ap, Bp, C, ldc, s));
    }
    if (overflow) {
        int h = 0;
        HIPCK(hipMemcpyAsync(&h, status + ST_OVERFLOW, 4, hipMemcpyDeviceToHost, s));
        HIPCK(hipStreamSynchronize(s));
        *overflow = h;
    }
    return MIXLU_OK;
}

int mixlu_outer_update(mixlu_ctx_t ctx, int n, int nrhs, const double *Gb, int ldg,
                       const double *X, int ldx, double *GA, int ldga, double alpha,
                       double GA_beta) {
    if (!ctx) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    if (n > 0 && nrhs > 0 && !Gb) return -4;
    if (ldg < (nrhs > 1 ? nrhs : 1)) return -5;
    if (n > 0 && nrhs > 0 && !X) return -6;
    if (ldx < (nrhs > 1 ? nrhs : 1)) return -7;
    if (n > 0 && !GA) return -8;
    if (ldga < (n > 1 ? n : 1)) return -9;
    HIPCK(launch_outer(n, nrhs, Gb, ldg, X, ldx, GA, ldga, alpha, GA_beta, ctx->stream));
    return MIXLU_OK;
}

}  // extern "C"
