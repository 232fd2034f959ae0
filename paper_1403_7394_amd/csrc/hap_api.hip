// C ABI of libhap (declared in include/hap.h): argument checks, the context and its
// workspace, and the host side of the iteration.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <new>
#include <algorithm>
#include <string>
#include <vector>

#include "hap_internal.h"

namespace hap {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

}  // namespace hap

using hap::DevState;
using hap::Launch;
using hap::LevelPtrs;

struct hap_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n = 0, lds = 0, ldw = 0;
    int64_t rows = 0;             // the sweeps update rows [0, rows) (hap_set_row_count; n by default)
    int L = 0;
    int schedule = HAP_SCHEDULE_SEQUENTIAL;
    int dtype = HAP_F32;
    size_t esz = 4;
    double lam = 0.0;
    const void *S = nullptr;
    // points mode (hap_set_points): the row pass recomputes s_ij from X
    const void *X = nullptr;
    int64_t ldx = 0;
    int d = 0;

    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;

    // workspace regions
    char *R = nullptr, *A = nullptr, *pref = nullptr, *Q = nullptr, *phi = nullptr, *tau = nullptr, *C = nullptr,
         *B = nullptr, *delta = nullptr;
    double kappa = 0.0;           // Eq. 2.7 weight (0: the update is off)
    int32_t *E = nullptr, *Efinal = nullptr, *mark = nullptr, *count = nullptr;
    char *Qpart = nullptr;        // column partials of up to nb_cap workgroups (in the workspace)
    // column partials of launches with more than nb_cap workgroups (for example one row per
    // workgroup at n > 2048): allocated by the library when such a launch is set
    char *Qbig = nullptr;
    size_t qbig_bytes = 0;
    DevState *ds = nullptr;
    double *dbl = nullptr;        // [0] median, [1..] net similarity per level + total
    void *select_scratch = nullptr;
    int nb_cap = 0;

    Launch lc{};
    bool no_fuse = false;         // HAP_LAUNCH_UNFUSED: per-level row passes under the MapReduce schedule
    // the paired row pass's exchange slots (library-owned, allocated with its first launch shape)
    uint64_t *pair_slots = nullptr;
    uint64_t pair_wait = 0;       // wall-clock ticks one of its waits may take
    // per-launch event timing (hap_profile)
    bool prof = false;
    int prof_period = 1;          // time the launches of every prof_period-th sweep
    long long prof_sweep = 0;     // sweeps issued since timing was switched on
    bool prof_now = false;        // the current sweep's launches are timed
    std::vector<hipEvent_t> ev;      // pairs: [2k] before, [2k+1] after launch k of the current chunk
    std::vector<int> ev_kind;        // 0 = row pass, 1 = column sums
    int ev_used = 0;
    double prof_ms[2] = {0.0, 0.0};
    long long prof_n[2] = {0, 0};
    // replayable graphs of sweep chunks (key: sweeps, stop-rule K)
    struct GraphEntry {
        int count, K;
        bool prof;
        hipGraphExec_t exec;
        int ev_pairs;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;
    bool use_graphs = true;       // HAP_LAUNCH_EAGER switches them off
    bool graphs_broken = false;   // capture is not available: launch eagerly
    int t_host = 0;               // completed iterations, mirrored on the host
    bool labels_ready = false;    // Efinal holds the labels of iteration t_host
    bool failed = false;
};

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kMaxPairs = 2048;   // pairs of the paired row pass's largest launch
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
    size_t R, A, pref, Q, phi, tau, C, B, delta, E, Efinal, mark, count, Qpart, ds, dbl, sel, total;
    int64_t ldw;
    int nb_cap;
};

Layout make_layout(int64_t n, int L, size_t esz) {
    Layout lo{};
    lo.ldw = (n + 63) / 64 * 64;
    lo.nb_cap = (int)(n < 2048 ? n : 2048);
    const size_t mat = (size_t)n * lo.ldw * esz;
    const size_t vec = (size_t)lo.ldw * esz;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    lo.R = take(mat * L);
    lo.A = take(mat * L);
    lo.pref = take(vec * L);
    lo.Q = take(vec * L);
    lo.phi = take(vec * L);
    lo.tau = take(vec * L);
    lo.C = take(vec * L);
    lo.B = take(vec * L);
    lo.delta = take(vec * L);
    lo.E = take((size_t)lo.ldw * 4 * L);
    lo.Efinal = take((size_t)lo.ldw * 4 * L);
    lo.mark = take((size_t)lo.ldw * 4);
    lo.count = take(64);
    lo.Qpart = take((size_t)2 * lo.nb_cap * vec);   // two buffers (the MapReduce schedule alternates)
    lo.ds = take(sizeof(DevState));
    lo.dbl = take(sizeof(double) * (size_t)(L + 4));
    lo.sel = take(hap::select_scratch_bytes());
    lo.total = off;
    return lo;
}

hap_status fail_hip(hipError_t e, const char *where, hap_ctx *ctx = nullptr) {
    std::string m = std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    hap::set_error(m);
    if (ctx) ctx->failed = true;
    return HAP_E_HIP;
}

hap_status fail_arg(const char *msg, hap_status code = HAP_E_ARG) {
    hap::set_error(msg);
    return code;
}

#define HIP_TRY(expr, ctx)                                   \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return fail_hip(_e, #expr, ctx); \
    } while (0)

template <typename T>
LevelPtrs<T> level_ptrs(const hap_ctx *c, int l) {
    LevelPtrs<T> p;
    const size_t mat = (size_t)c->n * c->ldw;
    p.R = (T *)c->R + mat * l;
    p.A = (T *)c->A + mat * l;
    p.pref = (T *)c->pref + (size_t)c->ldw * l;
    p.Q = (T *)c->Q + (size_t)c->ldw * l;
    p.phi = (T *)c->phi + (size_t)c->ldw * l;
    p.tau = (T *)c->tau + (size_t)c->ldw * l;
    p.C = (T *)c->C + (size_t)c->ldw * l;
    p.B = (T *)c->B + (size_t)c->ldw * l;
    p.E = c->E + (size_t)c->ldw * l;
    p.Efinal = c->Efinal + (size_t)c->ldw * l;
    p.delta = (T *)c->delta + (size_t)c->ldw * l;
    return p;
}

Launch default_launch(int64_t n, size_t esz) {
    const int vw = (int)(16 / esz);
    Launch lc{64, 1, 1, false, false};
    const int order[4] = {4, 2, 8, 1};
    bool found = false;
    for (int oi = 0; oi < 4 && !found; ++oi) {
        const int nch = order[oi];
        const int64_t need = (n + (int64_t)vw * nch - 1) / ((int64_t)vw * nch);
        int nt = 64;
        while (nt < need) nt <<= 1;
        if (hap::launch_supported(nt, nch, (int)esz)) {
            lc.threads = nt;
            lc.chunks = nch;
            found = true;
        }
    }
    if (!found && esz == 4 && n > 512 * 16 * 4 && n <= 512 * 32 * 4) {
        // FP32 rows of up to 65536 columns: the paired pass, two workgroups of 512 threads x 16
        // chunks per block of rows, 128 pairs (256 workgroups, one per CU)
        lc.threads = 512;
        lc.chunks = 32;
        lc.streaming = true;
        lc.rows_per_block = (int)((n + 127) / 128);
        lc.ordered = false;
        return lc;
    }
    if (!found && esz == 4 && n > 512 * 8 * 4 && n <= 512 * 16 * 4) {
        // FP32 rows of up to 32768 columns: the held-row pass (512 threads x 16 chunks keep the
        // row's s and rho in registers between the two phases)
        lc.threads = 512;
        lc.chunks = 16;
        lc.streaming = true;
        found = true;
    }
    if (!found) {
        // rows too long for registers: stream them with 1024 threads and 2..16 chunks
        lc.threads = 1024;
        lc.streaming = true;
        lc.chunks = (int)((n + 1024 * vw - 1) / (1024 * vw));
        if (lc.chunks > 16) {
            lc.threads = 0;
            return lc;
        }
    }
    // About 256 workgroups (one per CU) on large problems.  Small problems (FP32 up to 512
    // points, FP64 up to 2048) take one row per workgroup and sum the column partials in
    // row order, which is the order of a plain sequential column sum.
    int rb = (int)((n + 255) / 256);
    if (rb < 1) rb = 1;
    if (n <= (esz == 8 ? 2048 : 512)) rb = 1;
    lc.rows_per_block = rb;
    lc.ordered = (rb == 1);
    return lc;
}

bool launch_fits(const Launch &lc, int64_t n, int64_t rows, size_t esz) {
    const int64_t vw = (int64_t)(16 / esz);
    if (lc.streaming && lc.chunks == 32) {
        // the paired pass: FP32, each half of a row within one workgroup's 16 chunks, and the
        // whole grid resident at once
        if (esz != 4 || (lc.threads != 512 && lc.threads != 64)) return false;
        const int64_t h = (int64_t)lc.threads * 16 * 4;
        if (n <= h || n > 2 * h || lc.rows_per_block < 1) return false;
        const int64_t grid = hap::pair_grid(rows, lc.rows_per_block);
        return grid / 2 <= kMaxPairs && grid <= hap::pair_capacity(lc.threads);
    }
    if (lc.streaming) {
        const bool held = lc.threads == 512 && lc.chunks == 16 && esz == 4;
        if (lc.threads != 1024 && !held) return false;
        if (lc.chunks < 1 || lc.chunks > 16) return false;
    } else if (!hap::launch_supported(lc.threads, lc.chunks, (int)esz)) {
        return false;
    }
    if ((int64_t)lc.threads * lc.chunks * vw < n) return false;
    return lc.rows_per_block >= 1;
}

int64_t launch_blocks(const Launch &lc, int64_t rows) { return (rows + lc.rows_per_block - 1) / lc.rows_per_block; }

// The MapReduce schedule's fused all-level row pass applies: FP32, S read from memory (no points
// mode), no Eq. 2.7 update, a register-resident shape it was built for, 2..kMaxFused levels.
bool use_fused(const hap_ctx *c, const Launch &lc) {
    return c->schedule == HAP_SCHEDULE_MRHAP && !c->no_fuse && c->kappa == 0.0 && c->X == nullptr &&
           c->dtype == HAP_F32 && !lc.streaming && c->L >= 2 && c->rows == c->n &&
           hap::fused_supported(lc.threads, lc.chunks, c->L);
}

// Column-partial buffers a sweep needs: one per level for the fused pass, two for the
// per-level passes of the MapReduce schedule (they alternate), else one.
size_t partial_sets(const hap_ctx *c, const Launch &lc) {
    if (use_fused(c, lc)) return (size_t)c->L;
    return c->schedule == HAP_SCHEDULE_MRHAP ? 2 : 1;
}

// The workspace holds two partial buffers of nb_cap rows; larger needs use Qbig.
bool partials_in_workspace(const hap_ctx *c, const Launch &lc, int64_t rows) {
    return launch_blocks(lc, rows) <= c->nb_cap && partial_sets(c, lc) <= 2;
}


bool dtype_ok(int32_t dt) { return dt == HAP_F32 || dt == HAP_F64; }
size_t dtype_size(int32_t dt) { return dt == HAP_F64 ? 8 : 4; }

bool ld_ok(int64_t n, int64_t ld, int32_t dt) {
    const int64_t vw = (int64_t)(16 / dtype_size(dt));
    return ld >= n && ld % vw == 0;
}

// Event pair around the next launch when profiling (the pool grows on demand).
hipError_t prof_mark(hap_ctx *c, int kind, bool after) {
    if (!c->prof || !c->prof_now) return hipSuccess;
    if (!after) {
        const size_t need = (size_t)(c->ev_used + 1) * 2;
        while (c->ev.size() < need) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return err;
            c->ev.push_back(e);
        }
        if (c->ev_kind.size() < (size_t)c->ev_used + 1) c->ev_kind.resize(c->ev_used + 1);
        c->ev_kind[c->ev_used] = kind;
        return hipEventRecord(c->ev[2 * c->ev_used], c->stream);
    }
    hipError_t err = hipEventRecord(c->ev[2 * c->ev_used + 1], c->stream);
    c->ev_used += 1;
    return err;
}

// Accumulate the recorded pairs (the stream must have been synchronised).
hipError_t prof_collect(hap_ctx *c) {
    for (int k = 0; k < c->ev_used; ++k) {
        float ms = 0.f;
        hipError_t err = hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]);
        if (err != hipSuccess) return err;
        c->prof_ms[c->ev_kind[k]] += ms;
        c->prof_n[c->ev_kind[k]] += 1;
    }
    c->ev_used = 0;
    return hipSuccess;
}

template <typename T>
hap_status run_sweeps(hap_ctx *c, int count, int K) {
    const int L = c->L;
    const int nb = (int)launch_blocks(c->lc, c->rows);
    // the workspace's partial buffers, or the library's own when the launch has more workgroups
    // or the fused pass more levels
    const bool big = !partials_in_workspace(c, c->lc, c->rows);
    T *qbase = big ? (T *)c->Qbig : (T *)c->Qpart;
    const size_t qstride = (size_t)(big ? nb : c->nb_cap) * c->ldw;
    T *Qpart[2] = {qbase, qbase + qstride};
    const bool fused = use_fused(c, c->lc);
    hap::SweepExtra<T> ex;
    ex.X = (const T *)c->X;
    ex.ldx = c->ldx;
    ex.d = c->d;
    ex.rows = (int)c->rows;
    const bool kappa = c->kappa != 0.0;
    auto row = [&](int l, T *qp) -> hap_status {
        LevelPtrs<T> lv = level_ptrs<T>(c, l);
        LevelPtrs<T> down = level_ptrs<T>(c, l > 0 ? l - 1 : 0);
        // with the Eq. 2.7 update phi^{l-1} comes from level_phi (it needs the offsets of the
        // previous iteration, the row pass applies this iteration's)
        T *phi_down = (l > 0 && !kappa) ? down.phi : nullptr;
        hap::SweepExtra<T> e = ex;
        e.pair_slots = c->pair_slots;
        e.pair_wait = c->pair_wait;
        e.pair_level = l;
        if (kappa && l > 0) e.delta = lv.delta;
        const T *tau_l = nullptr;
        if (c->schedule == HAP_SCHEDULE_MRHAP) {
            e.mrhap = 1;
            if (l > 0) {
                e.tau_c = down.C;      // c^{l-1} of this iteration (its row pass ran just before)
                e.tau_q = down.Q;      // column sums of the previous iteration
                e.tau_store = lv.tau;
            }
        } else if (l > 0) {
            tau_l = lv.tau;
        }
        HIP_TRY(prof_mark(c, 0, false), c);
        HIP_TRY(hap::launch_sweep_level<T>((const T *)c->S, c->lds, lv, phi_down, tau_l, (int)c->n, c->ldw, c->lam,
                                           qp, c->lc, c->ds, c->stream, e),
                c);
        HIP_TRY(prof_mark(c, 0, true), c);
        return HAP_OK;
    };
    auto col = [&](int l, T *qp, bool with_tau) -> hap_status {
        LevelPtrs<T> lv = level_ptrs<T>(c, l);
        LevelPtrs<T> down = level_ptrs<T>(c, l > 0 ? l - 1 : 0);
        T *tau_next = (with_tau && l + 1 < L) ? level_ptrs<T>(c, l + 1).tau : nullptr;
        HIP_TRY(prof_mark(c, 1, false), c);
        HIP_TRY(hap::launch_colsum<T>(qp, c->ldw, nb, (int)c->n, lv, l > 0 ? &down : nullptr, tau_next, l == L - 1,
                                      l == L - 1, K, c->lc.ordered, c->ds, c->stream),
                c);
        HIP_TRY(prof_mark(c, 1, true), c);
        return HAP_OK;
    };
    for (int it = 0; it < count; ++it) {
        c->prof_now = c->prof && (c->prof_sweep++ % c->prof_period == 0);
        if (fused) {
            if constexpr (sizeof(T) == 4) {
                // every level's row pass in one launch, then the column sums in level order
                hap::FusedArgs<float> fa{};
                fa.S = (const float *)c->S;
                fa.lds = c->lds;
                fa.ldw = c->ldw;
                fa.n = (int)c->n;
                fa.rows = (int)c->rows;
                fa.rb = c->lc.rows_per_block;
                fa.row_stride = hap::row_stride_of(c->lc, c->rows);
                fa.L = L;
                fa.lam = (float)c->lam;
                fa.oml = (float)(1.0 - c->lam);
                fa.ds = c->ds;
                for (int l = 0; l < L; ++l) {
                    LevelPtrs<float> lv = level_ptrs<float>(c, l);
                    fa.R[l] = lv.R;
                    fa.A[l] = lv.A;
                    fa.pref[l] = lv.pref;
                    fa.C[l] = lv.C;
                    fa.phi[l] = lv.phi;
                    fa.B[l] = lv.B;
                    fa.Q[l] = lv.Q;
                    fa.tau[l] = lv.tau;
                    fa.E[l] = lv.E;
                    fa.Qpart[l] = (float *)qbase + (size_t)l * qstride;
                }
                HIP_TRY(prof_mark(c, 0, false), c);
                HIP_TRY(hap::launch_sweep_fused(fa, c->lc, c->stream), c);
                HIP_TRY(prof_mark(c, 0, true), c);
                for (int l = 0; l < L; ++l) {
                    const hap_status s = col(l, (T *)fa.Qpart[l], false);
                    if (s != HAP_OK) return s;
                }
                continue;
            }
        }
        if (c->schedule == HAP_SCHEDULE_MRHAP) {
            // Every row pass reads the previous iteration's column sums, so the column sums of
            // level l-1 run after the row pass of level l (two partial buffers alternate).
            hap_status s = row(0, Qpart[0]);
            for (int l = 1; l < L && s == HAP_OK; ++l) {
                s = row(l, Qpart[l & 1]);
                if (s == HAP_OK) s = col(l - 1, Qpart[(l - 1) & 1], false);
            }
            if (s == HAP_OK) s = col(L - 1, Qpart[(L - 1) & 1], false);
            if (s != HAP_OK) return s;
        } else {
            for (int l = 0; l < L; ++l) {
                hap_status s = row(l, Qpart[0]);
                if (s == HAP_OK) s = col(l, Qpart[0], true);
                if (s == HAP_OK && kappa && l + 1 < L) {
                    // Eq. 2.7: phi^l of iteration t-1, then the offsets delta^{l+1} of iteration t
                    LevelPtrs<T> lv = level_ptrs<T>(c, l);
                    LevelPtrs<T> up = level_ptrs<T>(c, l + 1);
                    HIP_TRY(hap::launch_level_phi<T>((const T *)c->S, c->lds, up, lv.phi, (int)c->n, c->ldw, c->lam,
                                                     c->ds, c->stream),
                            c);
                    HIP_TRY(hap::launch_level_delta<T>(lv, up.delta, (int)c->n, c->ldw, c->lam, c->kappa, c->ds,
                                                       c->stream),
                            c);
                }
                if (s != HAP_OK) return s;
            }
        }
    }
    return HAP_OK;
}

void drop_graphs(hap_ctx *c) {
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

// One chunk of sweeps.  The chunk's launches are captured once into a graph on a private
// stream and replayed on the context's stream, which removes the per-launch host overhead
// between the short kernels.  The kernels read the iteration counter from device memory, so
// every replay continues the run.  Per-launch timing (hap_profile) needs events around each
// launch that the host can read back, so timed chunks are launched one kernel at a time, as
// they are when capture is not available.
template <typename T>
hap_status launch_chunk(hap_ctx *c, int count, int K) {
    if (!c->use_graphs || c->graphs_broken || c->prof) return run_sweeps<T>(c, count, K);
    hap_ctx::GraphEntry *ge = nullptr;
    for (auto &g : c->graphs)
        if (g.count == count && g.K == K && g.prof == c->prof) ge = &g;
    if (!ge) {
        auto give_up = [&]() {
            (void)hipGetLastError();
            c->graphs_broken = true;
            c->failed = false;
            return run_sweeps<T>(c, count, K);
        };
        if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
            c->cap_stream = nullptr;
            return give_up();
        }
        const int ev0 = c->ev_used;
        if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return give_up();
        hipStream_t saved = c->stream;
        c->stream = c->cap_stream;
        const hap_status s = run_sweeps<T>(c, count, K);
        c->stream = saved;
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
        const int pairs = c->ev_used - ev0;
        c->ev_used = ev0;
        if (s != HAP_OK || e != hipSuccess || graph == nullptr) {
            if (graph) (void)hipGraphDestroy(graph);
            return give_up();
        }
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return give_up();
        c->graphs.push_back({count, K, c->prof, exec, pairs});
        ge = &c->graphs.back();
    }
    HIP_TRY(hipGraphLaunch(ge->exec, c->stream), c);
    c->ev_used += ge->ev_pairs;
    return HAP_OK;
}

template <typename T>
hap_status finalize_labels(hap_ctx *c) {
    // labels of iteration t: alpha^t materialised on the fly, nothing in the state written
    HIP_TRY(hipMemsetAsync(&c->ds->final_changed, 0, sizeof(int32_t), c->stream), c);
    for (int l = 0; l < c->L; ++l) {
        LevelPtrs<T> lv = level_ptrs<T>(c, l);
        HIP_TRY(hap::launch_finalize<T>((const T *)c->S, c->lds, lv, (int)c->n, c->ldw, c->lam, c->t_host, lv.Efinal,
                                        nullptr, 0, nullptr, nullptr, c->ds, c->stream, nullptr, (int)c->rows),
                c);
    }
    return HAP_OK;
}

// Column partials for a launch with more workgroups than the workspace holds: one row of ldw
// words per workgroup (two sets under the MapReduce schedule, whose passes alternate).  The
// library allocates them when such a launch is set and frees them in hap_destroy.
// The paired pass's exchange slots: room for the most pairs any launch can hold, all ones.
hap_status ensure_pair_slots(hap_ctx *c, const Launch &lc) {
    if (!(lc.streaming && lc.chunks == 32) || c->pair_slots) return HAP_OK;
    const size_t bytes = (size_t)hap::kPairSlotWords * kMaxPairs * sizeof(uint64_t);
    HIP_TRY(hipStreamSynchronize(c->stream), c);
    drop_graphs(c);
    if (hipMalloc((void **)&c->pair_slots, bytes) != hipSuccess) {
        (void)hipGetLastError();
        c->pair_slots = nullptr;
        return fail_arg("paired row pass: hipMalloc of its exchange slots failed", HAP_E_OOM);
    }
    HIP_TRY(hipMemsetAsync(c->pair_slots, 0xff, bytes, c->stream), c);
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device), c);
    c->pair_wait = (uint64_t)khz * 2000;   // two seconds
    // HAP_PAIR_WAIT_US shortens the bound (tests force the give-up path with it)
    if (const char *env = std::getenv("HAP_PAIR_WAIT_US")) {
        char *end = nullptr;
        const unsigned long long us = std::strtoull(env, &end, 10);
        if (end != env) c->pair_wait = (uint64_t)khz * us / 1000;
    }
    return HAP_OK;
}

hap_status ensure_partials(hap_ctx *c, const Launch &lc, int64_t rows) {
    const hap_status ss = ensure_pair_slots(c, lc);
    if (ss != HAP_OK) return ss;
    const int64_t nb = launch_blocks(lc, rows);
    if (partials_in_workspace(c, lc, rows)) return HAP_OK;
    const size_t sets = partial_sets(c, lc);
    const size_t need = sets * (size_t)nb * (size_t)c->ldw * c->esz;
    if (c->Qbig && c->qbig_bytes >= need) return HAP_OK;
    HIP_TRY(hipStreamSynchronize(c->stream), c);
    drop_graphs(c);   // captured sweeps hold the old buffer's address
    if (c->Qbig) {
        HIP_TRY(hipFree(c->Qbig), c);
        c->Qbig = nullptr;
        c->qbig_bytes = 0;
    }
    if (hipMalloc(&c->Qbig, need) != hipSuccess) {
        (void)hipGetLastError();
        c->Qbig = nullptr;
        return fail_arg("column partials of this launch: hipMalloc failed", HAP_E_OOM);
    }
    c->qbig_bytes = need;
    return HAP_OK;
}

}  // namespace

extern "C" {

const char *hap_version(void) { return "libhap 0.1.0 gfx950"; }

const char *hap_status_string(hap_status s) {
    switch (s) {
        case HAP_OK: return "ok";
        case HAP_E_ARG: return "invalid argument";
        case HAP_E_DTYPE: return "unsupported data type";
        case HAP_E_OOM: return "device allocation failed";
        case HAP_E_HIP: return "HIP runtime error";
        case HAP_E_STATE: return "context unusable after an earlier device error";
        case HAP_E_UNSUPPORTED: return "unsupported size or mode";
        default: return "unknown status";
    }
}

const char *hap_last_error(void) { return hap::g_last_error.c_str(); }

hap_status hap_build_similarity(const void *X, int64_t n, int64_t d, int64_t ldx, int32_t x_dtype, void *S,
                                int64_t lds, int32_t s_dtype, int32_t build_mode, double noise_rel, uint64_t seed,
                                void *stream) {
    if (!X || !S) return fail_arg("hap_build_similarity: null pointer");
    if (n < 1 || d < 1 || ldx < d || lds < n) return fail_arg("hap_build_similarity: bad sizes");
    if (n > (int64_t)1 << 20 || d > (int64_t)1 << 20) return fail_arg("hap_build_similarity: size too large", HAP_E_UNSUPPORTED);
    if (!dtype_ok(x_dtype) || !dtype_ok(s_dtype)) return fail_arg("hap_build_similarity: dtype", HAP_E_DTYPE);
    if (!(noise_rel >= 0.0) || !std::isfinite(noise_rel)) return fail_arg("hap_build_similarity: noise_rel");
    if (noise_rel > 0.0 && s_dtype != HAP_F64) return fail_arg("hap_build_similarity: noise needs FP64 output", HAP_E_DTYPE);
    if (build_mode < HAP_BUILD_DIRECT || build_mode > HAP_BUILD_DIRECT_L2)
        return fail_arg("hap_build_similarity: unknown build mode");
    if (build_mode == HAP_BUILD_GEMM && x_dtype != s_dtype)
        return fail_arg("hap_build_similarity: the GEMM build needs X and S of the same type", HAP_E_DTYPE);
    if ((build_mode == HAP_BUILD_BF16 || build_mode == HAP_BUILD_BF16X3) && (x_dtype != HAP_F32 || s_dtype != HAP_F32))
        return fail_arg("hap_build_similarity: BF16 builds take FP32 X and give FP32 S", HAP_E_DTYPE);
    if (noise_rel > 0.0 && (build_mode == HAP_BUILD_BF16 || build_mode == HAP_BUILD_BF16X3))
        return fail_arg("hap_build_similarity: noise needs FP64 output", HAP_E_DTYPE);
    hipError_t e = hap::launch_build(X, n, d, ldx, x_dtype, S, lds, s_dtype, build_mode, noise_rel, seed,
                                     (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "hap_build_similarity");
    return HAP_OK;
}

hap_status hap_median_offdiag(const void *S, int64_t n, int64_t lds, int32_t dtype, double *out_host, void *stream) {
    if (!S || !out_host) return fail_arg("hap_median_offdiag: null pointer");
    if (!dtype_ok(dtype)) return fail_arg("hap_median_offdiag: dtype", HAP_E_DTYPE);
    if (n < 2 || !ld_ok(n, lds, dtype)) return fail_arg("hap_median_offdiag: bad sizes");
    if (n > hap::kMaxSelectN)
        return fail_arg("hap_median_offdiag: n too large (at most 65536: the select counts n(n-1) keys in 32 bits)",
                        HAP_E_UNSUPPORTED);
    hipStream_t st = (hipStream_t)stream;
    void *scratch = nullptr;
    const size_t bytes = hap::select_scratch_bytes() + 256;
    hipError_t e = hipMallocAsync(&scratch, bytes, st);
    if (e != hipSuccess) return fail_hip(e, "hap_median_offdiag: hipMallocAsync");
    double *dev_out = (double *)((char *)scratch + hap::select_scratch_bytes());
    e = hap::launch_median_offdiag(S, n, lds, dtype, scratch, dev_out, st);
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, dev_out, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipError_t e2 = hipFreeAsync(scratch, st);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail_hip(e, "hap_median_offdiag");
    return HAP_OK;
}

hap_status hap_median_offdiag_noalloc(const void *S, int64_t n, int64_t lds, int32_t dtype, double *median_dev,
                                      void *stream) {
    if (!S || !median_dev) return fail_arg("hap_median_offdiag_noalloc: null pointer");
    if (!dtype_ok(dtype)) return fail_arg("hap_median_offdiag_noalloc: dtype", HAP_E_DTYPE);
    if (n < 2 || !ld_ok(n, lds, dtype)) return fail_arg("hap_median_offdiag_noalloc: bad sizes");
    if (n > hap::kMaxSelectN)
        return fail_arg("hap_median_offdiag_noalloc: n too large (at most 65536: the static scratch counts n(n-1) "
                        "keys in 32 bits)",
                        HAP_E_UNSUPPORTED);
    if (((uintptr_t)median_dev & 7u) != 0) return fail_arg("hap_median_offdiag_noalloc: median_dev not 8-byte aligned");
    void *scratch = nullptr;
    hipError_t e = hap::static_scratch(&scratch);
    if (e != hipSuccess) return fail_hip(e, "hap_median_offdiag_noalloc: hipGetSymbolAddress");
    e = hap::launch_median_offdiag(S, n, lds, dtype, scratch, median_dev, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "hap_median_offdiag_noalloc");
    return HAP_OK;
}

hap_status hap_bandwidth_probe(int32_t reads, int32_t writes, const float *const *in, float *const *out, int64_t rows,
                               int64_t cols, int64_t ld, int64_t rows_per_block, int32_t flags, void *stream) {
    const bool mix_ok = (reads == 0 && writes == 1) || (reads == 1 && writes == 0) || (reads == 1 && writes == 1) ||
                        (reads == 2 && writes == 2) || (reads == 3 && writes == 2);
    if (!mix_ok) return fail_arg("hap_bandwidth_probe: (reads, writes) must be (0,1), (1,0), (1,1), (2,2) or (3,2)");
    if ((reads > 0 && !in) || (writes > 0 && !out)) return fail_arg("hap_bandwidth_probe: null pointer");
    if (rows < 1 || cols < 1 || ld < cols || ld % 4 != 0 || cols % 4 != 0 || rows_per_block < 1)
        return fail_arg("hap_bandwidth_probe: bad sizes (cols and ld multiples of 4, ld >= cols)");
    if (flags & ~(HAP_PROBE_CACHED | HAP_PROBE_BLOCKS)) return fail_arg("hap_bandwidth_probe: unknown flags");
    if (cols > 8192) return fail_arg("hap_bandwidth_probe: at most 8192 columns", HAP_E_UNSUPPORTED);
    if (reads == 1 && writes == 0 && (!out || !out[0]))
        return fail_arg("hap_bandwidth_probe: the pure-read probe needs out[0] (one element, written only if the "
                        "data hold a marker pair)");
    hap::ProbeArgs a{};
    for (int r = 0; r < reads; ++r) {
        if (!in[r] || ((uintptr_t)in[r] & 15u)) return fail_arg("hap_bandwidth_probe: input null or not 16-byte aligned");
        a.in[r] = in[r];
    }
    for (int w = 0; w < writes; ++w) {
        if (!out[w] || ((uintptr_t)out[w] & 15u))
            return fail_arg("hap_bandwidth_probe: output null or not 16-byte aligned");
        a.out[w] = out[w];
    }
    if (writes == 0) a.out[0] = out[0];   // the pure-read mix's one-element sink
    a.rows = rows;
    a.cols = cols;
    a.ld = ld;
    a.rows_per_block = rows_per_block;
    hipError_t e = hap::launch_probe(reads, writes, (flags & HAP_PROBE_CACHED) != 0, (flags & HAP_PROBE_BLOCKS) != 0, a,
                                     (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "hap_bandwidth_probe");
    return HAP_OK;
}

hap_status hap_workspace_size(int64_t n, int32_t levels, int32_t dtype, size_t *bytes) {
    if (!bytes) return fail_arg("hap_workspace_size: null pointer");
    if (n < 2 || levels < 1 || levels > 64) return fail_arg("hap_workspace_size: bad sizes");
    if (!dtype_ok(dtype)) return fail_arg("hap_workspace_size: dtype", HAP_E_DTYPE);
    *bytes = make_layout(n, levels, dtype_size(dtype)).total;
    return HAP_OK;
}

hap_status hap_init(hap_ctx **out, const void *S, int64_t n, int64_t lds, int32_t dtype, const hap_params *p,
                    void *workspace, size_t workspace_bytes, void *stream) {
    if (!out || !S || !p) return fail_arg("hap_init: null pointer");
    *out = nullptr;
    if (p->struct_size < sizeof(hap_params)) return fail_arg("hap_init: hap_params.struct_size too small");
    if (!dtype_ok(dtype)) return fail_arg("hap_init: dtype", HAP_E_DTYPE);
    if (n < 2 || !ld_ok(n, lds, dtype)) return fail_arg("hap_init: need n >= 2, lds >= n, lds a multiple of 16 bytes");
    if (((uintptr_t)S & 15u) != 0) return fail_arg("hap_init: S must be 16-byte aligned");
    if (p->levels < 1 || p->levels > 64) return fail_arg("hap_init: levels must be in [1, 64]");
    if (!(p->damping >= 0.0 && p->damping < 1.0)) return fail_arg("hap_init: damping must be in [0, 1)");
    if (p->pref_mode == HAP_PREF_SCALAR) {
        if (!p->pref_scalar) return fail_arg("hap_init: pref_scalar is null");
        for (int l = 0; l < p->levels; ++l)
            if (!std::isfinite(p->pref_scalar[l])) return fail_arg("hap_init: non-finite preference");
    } else if (p->pref_mode == HAP_PREF_VECTOR) {
        if (!p->pref_vec) return fail_arg("hap_init: pref_vec is null");
    } else if (p->pref_mode != HAP_PREF_MEDIAN) {
        return fail_arg("hap_init: pref_mode");
    }
    if (p->schedule != HAP_SCHEDULE_SEQUENTIAL && p->schedule != HAP_SCHEDULE_MRHAP)
        return fail_arg("hap_init: schedule");
    if (!(p->kappa >= 0.0 && p->kappa <= 1.0)) return fail_arg("hap_init: kappa must be in [0, 1]");
    if (p->kappa != 0.0 && p->schedule != HAP_SCHEDULE_SEQUENTIAL)
        return fail_arg("hap_init: the level-wise similarity update (kappa > 0) needs the level-sequential schedule");
    const size_t esz = dtype_size(dtype);
    Layout lo = make_layout(n, p->levels, esz);
    Launch lc = default_launch(n, esz);
    if (lc.streaming && lc.chunks == 32 && !launch_fits(lc, n, n, esz)) {
        // the device holds fewer workgroups at once than the paired pass needs: stream the rows
        lc.threads = 1024;
        lc.chunks = (int)((n + 4095) / 4096);
        lc.rows_per_block = (int)((n + 255) / 256);
    }
    if (lc.threads == 0 || !launch_fits(lc, n, n, esz) || launch_blocks(lc, n) > lo.nb_cap)
        return fail_arg("hap_init: n too large (at most 65536 points in FP32, 32768 in FP64)", HAP_E_UNSUPPORTED);
    if (workspace) {
        if (workspace_bytes < lo.total) return fail_arg("hap_init: workspace too small");
        if (((uintptr_t)workspace & (kAlign - 1)) != 0) return fail_arg("hap_init: workspace must be 256-byte aligned");
    }

    hap_ctx *c = new (std::nothrow) hap_ctx();
    if (!c) return fail_arg("hap_init: host allocation failed", HAP_E_OOM);
    c->stream = (hipStream_t)stream;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        delete c;
        return fail_hip(e, "hap_init: hipGetDevice");
    }
    c->n = n;
    c->rows = n;
    c->lds = lds;
    c->ldw = lo.ldw;
    c->L = p->levels;
    c->schedule = p->schedule;
    c->kappa = p->kappa;
    c->dtype = dtype;
    c->esz = esz;
    c->lam = p->damping;
    c->S = S;
    c->lc = lc;
    c->nb_cap = lo.nb_cap;
    if (workspace) {
        c->ws = workspace;
        c->ws_bytes = workspace_bytes;
    } else {
        e = hipMalloc(&c->ws, lo.total);
        if (e != hipSuccess) {
            delete c;
            (void)hipGetLastError();
            return fail_arg("hap_init: hipMalloc of the workspace failed", HAP_E_OOM);
        }
        c->ws_bytes = lo.total;
        c->own_ws = true;
    }
    char *base = (char *)c->ws;
    c->R = base + lo.R;
    c->A = base + lo.A;
    c->pref = base + lo.pref;
    c->Q = base + lo.Q;
    c->phi = base + lo.phi;
    c->tau = base + lo.tau;
    c->C = base + lo.C;
    c->B = base + lo.B;
    c->delta = base + lo.delta;
    c->E = (int32_t *)(base + lo.E);
    c->Efinal = (int32_t *)(base + lo.Efinal);
    c->mark = (int32_t *)(base + lo.mark);
    c->count = (int32_t *)(base + lo.count);
    c->Qpart = base + lo.Qpart;
    c->ds = (DevState *)(base + lo.ds);
    c->dbl = (double *)(base + lo.dbl);
    c->select_scratch = base + lo.sel;

    hipStream_t st = c->stream;
    auto bail = [&](hipError_t err, const char *where) {
        hap_status s = fail_hip(err, where);
        if (c->own_ws) (void)hipFree(c->ws);
        delete c;
        return s;
    };
    // Algorithm 1 initial state: alpha = rho = 0, phi = c = 0, tau = +inf (tau^1 is never read;
    // tau^l for l > 1 is written before it is read), labels 0, counters 0.
    e = hipMemsetAsync(c->ws, 0, lo.Qpart, st);
    if (e == hipSuccess) e = hipMemsetAsync(c->ds, 0, sizeof(DevState), st);
    if (e == hipSuccess) {
        // padding columns of alpha hold -inf so they never win a row maximum
        if (dtype == HAP_F32)
            e = hap::launch_alpha_pad<float>((float *)c->A, (int64_t)c->L * n, (int)n, c->ldw, st);
        else
            e = hap::launch_alpha_pad<double>((double *)c->A, (int64_t)c->L * n, (int)n, c->ldw, st);
    }
    if (e != hipSuccess) return bail(e, "hap_init: clear workspace");

    const size_t vecb = (size_t)c->ldw * esz;
    if (p->pref_mode == HAP_PREF_MEDIAN) {
        e = hap::launch_median_offdiag(S, n, lds, dtype, c->select_scratch, c->dbl, st);
        if (e == hipSuccess) e = hap::launch_fill_pref(c->pref, c->ldw, (int)n, c->L, dtype, c->dbl, st);
    } else if (p->pref_mode == HAP_PREF_SCALAR) {
        for (int l = 0; l < c->L && e == hipSuccess; ++l) {
            e = hipMemcpyAsync(c->dbl + 1 + (l % 2), &p->pref_scalar[l], sizeof(double), hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hap::launch_fill_pref(c->pref + vecb * l, c->ldw, (int)n, 1, dtype, c->dbl + 1 + (l % 2), st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
        }
    } else {
        for (int l = 0; l < c->L && e == hipSuccess; ++l)
            e = hipMemcpyAsync(c->pref + vecb * l, (const char *)p->pref_vec + (size_t)n * esz * l, (size_t)n * esz,
                               hipMemcpyDeviceToDevice, st);
    }
    if (e != hipSuccess) return bail(e, "hap_init: preferences");
    e = hipGetLastError();
    if (e != hipSuccess) return bail(e, "hap_init: launch");
    *out = c;
    return HAP_OK;
}

hap_status hap_iterate(hap_ctx *c, int32_t max_iters, int32_t stable_iters, int32_t *iters_done, int32_t *converged) {
    if (!c) return fail_arg("hap_iterate: null context");
    if (c->failed) return fail_arg("hap_iterate: context failed earlier", HAP_E_STATE);
    if (max_iters < 0 || stable_iters < 0) return fail_arg("hap_iterate: negative count");
    DevState hs;
    // the partial buffers of the row pass the sweeps will use (points mode changes it)
    const hap_status ps = ensure_partials(c, c->lc, c->rows);
    if (ps != HAP_OK) return ps;
    // a previous early stop does not block continuing: clear the flag
    HIP_TRY(hipMemsetAsync(&c->ds->done, 0, sizeof(int32_t), c->stream), c);
    const int chunk = 16;
    int left = max_iters;
    bool stopped = false;
    while (left > 0) {
        const int now = left < chunk ? left : chunk;
        hap_status s = (c->dtype == HAP_F32) ? launch_chunk<float>(c, now, stable_iters)
                                             : launch_chunk<double>(c, now, stable_iters);
        if (s != HAP_OK) return s;
        left -= now;
        if (c->prof) {
            HIP_TRY(hipStreamSynchronize(c->stream), c);
            HIP_TRY(prof_collect(c), c);
        }
        if (stable_iters > 0) {
            HIP_TRY(hipMemcpyAsync(&hs, c->ds, sizeof(DevState), hipMemcpyDeviceToHost, c->stream), c);
            HIP_TRY(hipStreamSynchronize(c->stream), c);
            if (hs.done) {
                stopped = true;
                break;
            }
        }
    }
    HIP_TRY(hipMemcpyAsync(&hs, c->ds, sizeof(DevState), hipMemcpyDeviceToHost, c->stream), c);
    HIP_TRY(hipStreamSynchronize(c->stream), c);
    if (hs.pair_abort) {
        c->failed = true;
        return fail_arg("hap_iterate: the paired row pass gave up waiting for a partner workgroup (part of the "
                        "device was busy); the state is not valid",
                        HAP_E_HIP);
    }
    c->t_host = hs.t;
    int conv = 0, done_iter = hs.t;
    if (stopped || hs.done) {
        // labels of the stop iteration are the last ones the row pass recorded
        HIP_TRY(hipMemcpyAsync(c->Efinal, c->E, (size_t)c->ldw * 4 * c->L, hipMemcpyDeviceToDevice, c->stream), c);
        conv = 1;
        done_iter = hs.stop_iter;
    } else {
        hap_status s = (c->dtype == HAP_F32) ? finalize_labels<float>(c) : finalize_labels<double>(c);
        if (s != HAP_OK) return s;
        HIP_TRY(hipMemcpyAsync(&hs, c->ds, sizeof(DevState), hipMemcpyDeviceToHost, c->stream), c);
        HIP_TRY(hipStreamSynchronize(c->stream), c);
        if (stable_iters > 0 && c->t_host >= 2) {
            // stable count after comparing e^t with e^{t-1}; hs.stable is the count after iteration t-1
            const int st_after = hs.final_changed ? 0 : hs.stable + 1;
            conv = st_after >= stable_iters ? 1 : 0;
        }
    }
    c->labels_ready = true;
    if (iters_done) *iters_done = done_iter;
    if (converged) *converged = conv;
    return HAP_OK;
}

hap_status hap_exemplars(hap_ctx *c, int32_t level, int32_t *labels, int32_t *n_exemplars) {
    if (!c) return fail_arg("hap_exemplars: null context");
    if (level < 0 || level >= c->L) return fail_arg("hap_exemplars: level out of range");
    if (c->failed) return fail_arg("hap_exemplars: context failed earlier", HAP_E_STATE);
    if (!c->labels_ready) {
        hap_status s = (c->dtype == HAP_F32) ? finalize_labels<float>(c) : finalize_labels<double>(c);
        if (s != HAP_OK) return s;
        c->labels_ready = true;
    }
    const int32_t *src = c->Efinal + (size_t)c->ldw * level;
    if (labels) HIP_TRY(hipMemcpyAsync(labels, src, (size_t)c->n * 4, hipMemcpyDeviceToDevice, c->stream), c);
    if (n_exemplars) {
        HIP_TRY(hap::launch_count_distinct(src, (int)c->rows, (int)c->n, c->mark, c->count, c->stream), c);
        HIP_TRY(hipMemcpyAsync(n_exemplars, c->count, 4, hipMemcpyDeviceToHost, c->stream), c);
        HIP_TRY(hipStreamSynchronize(c->stream), c);
    }
    return HAP_OK;
}

hap_status hap_net_similarity(hap_ctx *c, int32_t level, const void *X, int64_t d, int64_t ldx, int32_t x_dtype,
                              double *out) {
    if (!c || !out) return fail_arg("hap_net_similarity: null pointer");
    if (level < -1 || level >= c->L) return fail_arg("hap_net_similarity: level out of range");
    if (X && (d < 1 || ldx < d || !dtype_ok(x_dtype))) return fail_arg("hap_net_similarity: bad X");
    if (c->failed) return fail_arg("hap_net_similarity: context failed earlier", HAP_E_STATE);
    if (!c->labels_ready) {
        hap_status s = (c->dtype == HAP_F32) ? finalize_labels<float>(c) : finalize_labels<double>(c);
        if (s != HAP_OK) return s;
        c->labels_ready = true;
    }
    double *dev = c->dbl + 1;
    HIP_TRY(hap::launch_net_similarity(c->S, c->lds, c->dtype, c->pref, c->ldw, c->Efinal, (int)c->n, c->L, X, d,
                                       ldx, x_dtype, dev, c->stream),
            c);
    const int slot = level < 0 ? c->L : level;
    HIP_TRY(hipMemcpyAsync(out, dev + slot, sizeof(double), hipMemcpyDeviceToHost, c->stream), c);
    HIP_TRY(hipStreamSynchronize(c->stream), c);
    return HAP_OK;
}

hap_status hap_preference(hap_ctx *c, double *out) {
    if (!c || !out) return fail_arg("hap_preference: null pointer");
    for (int l = 0; l < c->L; ++l) {
        const char *src = c->pref + (size_t)c->ldw * c->esz * l;
        if (c->dtype == HAP_F32) {
            float f;
            HIP_TRY(hipMemcpyAsync(&f, src, 4, hipMemcpyDeviceToHost, c->stream), c);
            HIP_TRY(hipStreamSynchronize(c->stream), c);
            out[l] = f;
        } else {
            HIP_TRY(hipMemcpyAsync(&out[l], src, 8, hipMemcpyDeviceToHost, c->stream), c);
            HIP_TRY(hipStreamSynchronize(c->stream), c);
        }
    }
    return HAP_OK;
}

hap_status hap_read_messages(hap_ctx *c, int32_t level, void *rho, void *alpha, int64_t ld, void *cvec, void *phi,
                             void *tau) {
    if (!c) return fail_arg("hap_read_messages: null context");
    if (level < 0 || level >= c->L) return fail_arg("hap_read_messages: level out of range");
    if ((rho || alpha) && ld < c->n) return fail_arg("hap_read_messages: ld < n");
    if (c->failed) return fail_arg("hap_read_messages: context failed earlier", HAP_E_STATE);
    const size_t esz = c->esz;
    hipStream_t st = c->stream;
    if (rho) {
        const char *src = c->R + (size_t)c->n * c->ldw * esz * level;
        HIP_TRY(hipMemcpy2DAsync(rho, (size_t)ld * esz, src, (size_t)c->ldw * esz, (size_t)c->n * esz, (size_t)c->n,
                                 hipMemcpyDeviceToDevice, st),
                c);
    }
    // alpha^{l,t} and c^l = max_j(alpha + rho) of the top level are not part of the method's state
    // (c is unused there); c of the top level is reported as 0.
    const bool top = level == c->L - 1;
    // Under the MapReduce schedule c^l and phi^l of iteration t are the values the row passes
    // of iteration t computed (from the state of iteration t-1) and stored; under the
    // level-sequential schedule they are recomputed from alpha^t and rho^t.
    const bool mr = c->schedule == HAP_SCHEDULE_MRHAP;
    void *c_fin = (cvec && !top && !mr) ? cvec : nullptr;
    if (alpha || c_fin) {
        if (c->dtype == HAP_F32) {
            LevelPtrs<float> lv = level_ptrs<float>(c, level);
            HIP_TRY(hap::launch_finalize<float>((const float *)c->S, c->lds, lv, (int)c->n, c->ldw, c->lam, c->t_host,
                                                nullptr, (float *)alpha, ld, (float *)c_fin, nullptr, c->ds, st),
                    c);
        } else {
            LevelPtrs<double> lv = level_ptrs<double>(c, level);
            HIP_TRY(hap::launch_finalize<double>((const double *)c->S, c->lds, lv, (int)c->n, c->ldw, c->lam, c->t_host,
                                                 nullptr, (double *)alpha, ld, (double *)c_fin, nullptr, c->ds, st),
                    c);
        }
    }
    if (cvec && mr && !top && c->t_host > 0) {
        const char *src = c->C + (size_t)c->ldw * esz * level;
        HIP_TRY(hipMemcpyAsync(cvec, src, (size_t)c->n * esz, hipMemcpyDeviceToDevice, st), c);
    }
    if (cvec && top) HIP_TRY(hipMemsetAsync(cvec, 0, (size_t)c->n * esz, st), c);
    if (cvec && c->t_host == 0) HIP_TRY(hipMemsetAsync(cvec, 0, (size_t)c->n * esz, st), c);
    if (phi) {
        // phi^l after iteration t is max_k(alpha^{l+1,t}_ik + s_ik) (level-sequential) or the
        // stored phi^l of iteration t (MapReduce); 0 at the top level and before iteration 1
        if (top || c->t_host == 0) {
            HIP_TRY(hipMemsetAsync(phi, 0, (size_t)c->n * esz, st), c);
        } else if (mr) {
            const char *src = c->phi + (size_t)c->ldw * esz * level;
            HIP_TRY(hipMemcpyAsync(phi, src, (size_t)c->n * esz, hipMemcpyDeviceToDevice, st), c);
        } else if (c->dtype == HAP_F32) {
            LevelPtrs<float> up = level_ptrs<float>(c, level + 1);
            HIP_TRY(hap::launch_finalize<float>((const float *)c->S, c->lds, up, (int)c->n, c->ldw, c->lam, c->t_host,
                                                nullptr, nullptr, 0, nullptr, (float *)phi, c->ds, st,
                                                c->kappa != 0.0 ? up.delta : nullptr),
                    c);
        } else {
            LevelPtrs<double> up = level_ptrs<double>(c, level + 1);
            HIP_TRY(hap::launch_finalize<double>((const double *)c->S, c->lds, up, (int)c->n, c->ldw, c->lam, c->t_host,
                                                 nullptr, nullptr, 0, nullptr, (double *)phi, c->ds, st,
                                                 c->kappa != 0.0 ? up.delta : nullptr),
                    c);
        }
    }
    if (tau) {
        if (level == 0 || c->t_host == 0) {
            // tau^1 = +inf (and every tau before iteration 1)
            const size_t cnt = (size_t)c->n;
            if (c->dtype == HAP_F32) {
                float *h = new float[cnt];
                for (size_t k = 0; k < cnt; ++k) h[k] = INFINITY;
                hipError_t e = hipMemcpyAsync(tau, h, cnt * 4, hipMemcpyHostToDevice, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                delete[] h;
                if (e != hipSuccess) return fail_hip(e, "hap_read_messages: tau", c);
            } else {
                double *h = new double[cnt];
                for (size_t k = 0; k < cnt; ++k) h[k] = INFINITY;
                hipError_t e = hipMemcpyAsync(tau, h, cnt * 8, hipMemcpyHostToDevice, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                delete[] h;
                if (e != hipSuccess) return fail_hip(e, "hap_read_messages: tau", c);
            }
        } else {
            const char *src = c->tau + (size_t)c->ldw * esz * level;
            HIP_TRY(hipMemcpyAsync(tau, src, (size_t)c->n * esz, hipMemcpyDeviceToDevice, st), c);
        }
    }
    HIP_TRY(hipStreamSynchronize(st), c);
    return HAP_OK;
}

hap_status hap_similarity_offsets(hap_ctx *c, int32_t level, void *delta) {
    if (!c || !delta) return fail_arg("hap_similarity_offsets: null pointer");
    if (level < 0 || level >= c->L) return fail_arg("hap_similarity_offsets: level out of range");
    if (c->failed) return fail_arg("hap_similarity_offsets: context failed earlier", HAP_E_STATE);
    const char *src = c->delta + (size_t)c->ldw * c->esz * level;
    HIP_TRY(hipMemcpyAsync(delta, src, (size_t)c->n * c->esz, hipMemcpyDeviceToDevice, c->stream), c);
    HIP_TRY(hipStreamSynchronize(c->stream), c);
    return HAP_OK;
}

hap_status hap_set_launch(hap_ctx *c, int32_t threads, int32_t chunks, int32_t rows_per_block, int32_t flags) {
    if (!c) return fail_arg("hap_set_launch: null context");
    Launch lc = c->lc;
    if (threads) lc.threads = threads;
    if (chunks) lc.chunks = chunks;
    if (rows_per_block) lc.rows_per_block = rows_per_block;
    if (flags >= 0) lc.streaming = (flags & HAP_LAUNCH_STREAM) != 0;
    if (flags >= 0) lc.blocks = (flags & HAP_LAUNCH_BLOCKS) != 0;
    lc.ordered = (lc.rows_per_block == 1);
    if (!launch_fits(lc, c->n, c->rows, c->esz))
        return fail_arg("hap_set_launch: shape does not fit this problem");
    const bool no_fuse = c->no_fuse;
    if (flags >= 0) c->no_fuse = (flags & HAP_LAUNCH_UNFUSED) != 0;
    const hap_status ps = ensure_partials(c, lc, c->rows);
    if (ps != HAP_OK) {
        c->no_fuse = no_fuse;
        return ps;
    }
    c->lc = lc;
    if (flags >= 0) c->use_graphs = (flags & HAP_LAUNCH_EAGER) == 0;
    drop_graphs(c);
    return HAP_OK;
}

hap_status hap_set_row_count(hap_ctx *c, int64_t rows) {
    if (!c) return fail_arg("hap_set_row_count: null context");
    if (rows < 1 || rows > c->n) return fail_arg("hap_set_row_count: rows must lie in [1, n]");
    if (rows < c->n && (c->schedule != HAP_SCHEDULE_SEQUENTIAL || c->kappa != 0.0))
        return fail_arg("hap_set_row_count: a row block needs the sequential schedule without kappa",
                        HAP_E_UNSUPPORTED);
    if (!launch_fits(c->lc, c->n, rows, c->esz))
        return fail_arg("hap_set_row_count: the launch shape does not fit this row count");
    const hap_status ps = ensure_partials(c, c->lc, rows);
    if (ps != HAP_OK) return ps;
    c->rows = rows;
    drop_graphs(c);
    return HAP_OK;
}

hap_status hap_get_row_count(hap_ctx *c, int64_t *rows) {
    if (!c || !rows) return fail_arg("hap_get_row_count: null argument");
    *rows = c->rows;
    return HAP_OK;
}

hap_status hap_set_points(hap_ctx *c, const void *X, int64_t n, int64_t d, int64_t ldx, int32_t x_dtype) {
    if (!c) return fail_arg("hap_set_points: null context");
    if (!X) {
        c->X = nullptr;
        c->ldx = 0;
        c->d = 0;
        drop_graphs(c);
        return HAP_OK;
    }
    if (c->failed) return fail_arg("hap_set_points: context failed earlier", HAP_E_STATE);
    if (n != c->n) return fail_arg("hap_set_points: the point count differs from the context's n");
    if (c->dtype != HAP_F32 || x_dtype != HAP_F32)
        return fail_arg("hap_set_points: points mode needs FP32 similarities and FP32 points", HAP_E_DTYPE);
    if (d != 2 && d != 3) return fail_arg("hap_set_points: points mode supports d = 2 or 3", HAP_E_UNSUPPORTED);
    if (ldx < d) return fail_arg("hap_set_points: ldx < d");
    // S must be the direct build of these points: recompute sampled entries and compare bits
    hap::PairSample ps{};
    uint64_t z = 0x9e3779b97f4a7c15ull ^ (uint64_t)n;
    auto next = [&]() {
        z += 0x9e3779b97f4a7c15ull;
        uint64_t x = z;
        x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
        x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
        return x ^ (x >> 31);
    };
    ps.count = 64;
    ps.i[0] = 0;
    ps.j[0] = (int32_t)(n - 1);
    ps.i[1] = (int32_t)(n - 1);
    ps.j[1] = 0;
    for (int k = 2; k < 64; ++k) {
        const int32_t i = (int32_t)(next() % (uint64_t)n);
        int32_t j = (int32_t)(next() % (uint64_t)n);
        if (j == i) j = (int32_t)((i + 1) % n);
        ps.i[k] = i;
        ps.j[k] = j;
    }
    HIP_TRY(hap::launch_points_check((const float *)c->S, c->lds, (const float *)X, ldx, (int)d, ps, c->count,
                                     c->stream),
            c);
    int32_t bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, c->count, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream), c);
    HIP_TRY(hipStreamSynchronize(c->stream), c);
    if (bad != 0)
        return fail_arg("hap_set_points: S is not the direct build of these points (sampled entries differ)");
    c->X = X;
    c->ldx = ldx;
    c->d = (int)d;
    drop_graphs(c);
    return HAP_OK;
}

hap_status hap_get_launch(hap_ctx *c, int32_t *threads, int32_t *chunks, int32_t *rows_per_block, int32_t *flags) {
    if (!c) return fail_arg("hap_get_launch: null context");
    if (flags)
        *flags = (c->lc.streaming ? HAP_LAUNCH_STREAM : 0) | (c->use_graphs ? 0 : HAP_LAUNCH_EAGER) |
                 (c->no_fuse ? HAP_LAUNCH_UNFUSED : 0) | (use_fused(c, c->lc) ? HAP_LAUNCH_FUSED : 0) |
                 (c->lc.blocks ? HAP_LAUNCH_BLOCKS : 0);
    if (threads) *threads = c->lc.threads;
    if (chunks) *chunks = c->lc.chunks;
    if (rows_per_block) *rows_per_block = c->lc.rows_per_block;
    return HAP_OK;
}

hap_status hap_profile(hap_ctx *c, int32_t enable) {
    if (!c) return fail_arg("hap_profile: null context");
    if (c->prof) {
        HIP_TRY(hipStreamSynchronize(c->stream), c);
        HIP_TRY(prof_collect(c), c);
    }
    if (enable < 0) return fail_arg("hap_profile: enable must be >= 0");
    if (enable) {
        c->prof_ms[0] = c->prof_ms[1] = 0.0;
        c->prof_n[0] = c->prof_n[1] = 0;
        c->prof_period = enable;
        c->prof_sweep = 0;
    }
    c->prof = enable != 0;
    return HAP_OK;
}

hap_status hap_profile_read(hap_ctx *c, double *row_ms, int64_t *row_n, double *col_ms, int64_t *col_n) {
    if (!c) return fail_arg("hap_profile_read: null context");
    if (c->ev_used) {
        HIP_TRY(hipStreamSynchronize(c->stream), c);
        HIP_TRY(prof_collect(c), c);
    }
    if (row_ms) *row_ms = c->prof_ms[0];
    if (row_n) *row_n = c->prof_n[0];
    if (col_ms) *col_ms = c->prof_ms[1];
    if (col_n) *col_n = c->prof_n[1];
    return HAP_OK;
}

hap_status hap_destroy(hap_ctx *c) {
    if (!c) return HAP_OK;
    hap_status s = HAP_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) s = fail_hip(e, "hap_destroy: synchronize");
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipEvent_t ev : c->ev) (void)hipEventDestroy(ev);
    if (c->own_ws) {
        e = hipFree(c->ws);
        if (e != hipSuccess && s == HAP_OK) s = fail_hip(e, "hap_destroy: hipFree");
    }
    if (c->pair_slots) {
        e = hipFree(c->pair_slots);
        if (e != hipSuccess && s == HAP_OK) s = fail_hip(e, "hap_destroy: hipFree");
    }
    if (c->Qbig) {
        e = hipFree(c->Qbig);
        if (e != hipSuccess && s == HAP_OK) s = fail_hip(e, "hap_destroy: hipFree");
    }
    delete c;
    return s;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form
// ---------------------------------------------------------------------------
struct hap_batch {
    int count = 0, levels = 0;
    int64_t d = 0;
    std::vector<int32_t> sizes;      // host copy of the instance sizes (re-planning)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    hap::BatchDesc *desc = nullptr;  // device
    hap::BatchItem *items = nullptr; // device, queue order
    int n_items = 0;
    int32_t *queue = nullptr;        // device
    float *wsf = nullptr;
    int32_t *wsi = nullptr;
    int threads = 512, workgroups = 512, row_groups = 4;
    int split_n = 0, max_members = 4;   // instances above split_n points are shared by a gang
    bool gangs = false;
};

namespace {

struct BatchPlan {
    std::vector<hap::BatchDesc> desc;
    std::vector<hap::BatchItem> items;
    size_t off_desc, off_items, off_queue, off_f, off_i, total;
    bool gangs = false;
};

// Gang of an instance: members K = min(max_members, ceil(n^2 / split_n^2)) for n > split_n
// (split_n = 0: never), rows per member ceil(n / K), then K recounted so no member is empty.
void gang_of(int n, int split_n, int max_members, int &K, int &rbm) {
    K = 1;
    rbm = n;
    if (split_n <= 0 || n <= split_n || n <= hap::kGangMinN) return;
    const int64_t want = ((int64_t)n * n + (int64_t)split_n * split_n - 1) / ((int64_t)split_n * split_n);
    K = (int)std::min<int64_t>(want, max_members);
    if (K < 2) {
        K = 1;
        return;
    }
    rbm = (n + K - 1) / K;
    K = (n + rbm - 1) / rbm;
}

bool plan_batch(int32_t count, const int32_t *n, int64_t d, int32_t levels, int split_n, int max_members, BatchPlan &pl,
                std::string &err) {
    if (count < 1 || !n || d < 1 || d > 32 || levels < 1 || levels > 64) {
        err = "hap_batch: need count >= 1, 1 <= d <= 32, 1 <= levels <= 64";
        return false;
    }
    pl.desc.resize(count);
    int64_t xo = 0, fo = 0, io = 0, oo = 0;
    for (int b = 0; b < count; ++b) {
        if (n[b] < 2 || n[b] > 2048) {
            err = "hap_batch: every problem needs 2 <= n <= 2048 points";
            return false;
        }
        const int ld = (n[b] + 63) / 64 * 64;
        hap::BatchDesc &D = pl.desc[b];
        D.n = n[b];
        D.ld = ld;
        D.x_off = xo;
        D.w_off = fo;
        D.i_off = io;
        D.out_off = oo;
        gang_of(n[b], split_n, max_members, D.K, D.rbm);
        pl.gangs = pl.gangs || D.K > 1;
        xo += n[b];
        fo += (hap::batch_floats(n[b], ld, levels) + 63) / 64 * 64;
        io += (hap::batch_ints(ld, levels) + 63) / 64 * 64;
        D.g_off = -1;
        D.s_off = -1;
        if (n[b] > hap::kGangMinN) {
            // room for the largest gang, whatever the current split
            D.g_off = fo;
            fo += (int64_t)2 * hap::kMaxGang * ld;
            D.s_off = io;
            io += hap::kGangInts;
        }
        oo += (int64_t)levels * n[b];
    }
    std::vector<int> order(count);
    for (int b = 0; b < count; ++b) order[b] = b;
    // largest problems first (ties by index, so the order is deterministic); a gang's members
    // are consecutive in the queue
    std::sort(order.begin(), order.end(), [&](int a, int b) { return n[a] != n[b] ? n[a] > n[b] : a < b; });
    pl.items.clear();
    for (int b : order)
        for (int m = 0; m < pl.desc[b].K; ++m) pl.items.push_back({b, m});
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    pl.off_desc = take(sizeof(hap::BatchDesc) * count);
    pl.off_items = take(sizeof(hap::BatchItem) * (size_t)count * hap::kMaxGang);
    pl.off_queue = take(64);
    pl.off_f = take((size_t)fo * 4);
    pl.off_i = take((size_t)io * 4);
    pl.total = off;
    return true;
}

hap_status upload_plan(hap_batch *b, const BatchPlan &pl, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(b->desc, pl.desc.data(), sizeof(hap::BatchDesc) * b->count, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->items, pl.items.data(), sizeof(hap::BatchItem) * pl.items.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail_hip(e, "hap_batch: upload of the plan");
    b->n_items = (int)pl.items.size();
    b->gangs = pl.gangs;
    return HAP_OK;
}

}  // namespace

extern "C" {

hap_status hap_batch_workspace_size(int32_t count, const int32_t *n, int64_t d, int32_t levels, size_t *bytes) {
    if (!bytes) return fail_arg("hap_batch_workspace_size: null pointer");
    BatchPlan pl;
    std::string err;
    if (!plan_batch(count, n, d, levels, 0, 1, pl, err)) return fail_arg(err.c_str());
    *bytes = pl.total;
    return HAP_OK;
}

hap_status hap_batch_create(hap_batch **out, int32_t count, const int32_t *n, int64_t d, int32_t levels,
                            void *workspace, size_t workspace_bytes, void *stream) {
    if (!out) return fail_arg("hap_batch_create: null pointer");
    *out = nullptr;
    BatchPlan pl;
    std::string err;
    if (!plan_batch(count, n, d, levels, 0, 1, pl, err)) return fail_arg(err.c_str());
    if (workspace && (workspace_bytes < pl.total || ((uintptr_t)workspace & (kAlign - 1)) != 0))
        return fail_arg("hap_batch_create: workspace too small or not 256-byte aligned");
    hap_batch *b = new (std::nothrow) hap_batch();
    if (!b) return fail_arg("hap_batch_create: host allocation failed", HAP_E_OOM);
    b->count = count;
    b->levels = levels;
    b->d = d;
    b->sizes.assign(n, n + count);
    if (workspace) {
        b->ws = workspace;
        b->ws_bytes = workspace_bytes;
    } else {
        if (hipMalloc(&b->ws, pl.total) != hipSuccess) {
            (void)hipGetLastError();
            delete b;
            return fail_arg("hap_batch_create: hipMalloc of the workspace failed", HAP_E_OOM);
        }
        b->ws_bytes = pl.total;
        b->own_ws = true;
    }
    char *base = (char *)b->ws;
    b->desc = (hap::BatchDesc *)(base + pl.off_desc);
    b->items = (hap::BatchItem *)(base + pl.off_items);
    b->queue = (int32_t *)(base + pl.off_queue);
    b->wsf = (float *)(base + pl.off_f);
    b->wsi = (int32_t *)(base + pl.off_i);
    const hap_status s = upload_plan(b, pl, (hipStream_t)stream);
    if (s != HAP_OK) {
        if (b->own_ws) (void)hipFree(b->ws);
        delete b;
        return s;
    }
    *out = b;
    return HAP_OK;
}

hap_status hap_batch_run(hap_batch *b, const void *X, double damping, int32_t max_iters, int32_t stable_iters,
                         int32_t *labels, double *net_similarity, int32_t *iters, void *stream) {
    if (!b || !X || !labels || !net_similarity || !iters) return fail_arg("hap_batch_run: null pointer");
    if (!(damping >= 0.0 && damping < 1.0)) return fail_arg("hap_batch_run: damping must be in [0, 1)");
    if (max_iters < 0 || stable_iters < 0) return fail_arg("hap_batch_run: negative count");
    hipError_t e = hap::launch_batch((const float *)X, b->d, b->desc, b->items, b->n_items, b->count, b->levels, damping,
                                     max_iters, stable_iters, b->wsf, b->wsi, b->queue, labels, net_similarity, iters,
                                     b->threads, b->workgroups, b->row_groups, b->gangs, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "hap_batch_run");
    return HAP_OK;
}

hap_status hap_batch_set_launch(hap_batch *b, int32_t threads, int32_t workgroups, int32_t row_groups) {
    if (!b) return fail_arg("hap_batch_set_launch: null pointer");
    if (workgroups < 0) return fail_arg("hap_batch_set_launch: workgroups must be >= 1");
    const int th = threads ? threads : b->threads;
    const int rg = row_groups ? row_groups : b->row_groups;
    const bool ok = (rg == 1 && (th == 256 || th == 512)) || (rg == 2 && th == 512) || (rg == 4 && (th == 512 || th == 1024));
    if (!ok)
        return fail_arg("hap_batch_set_launch: (threads, row_groups) must be (256, 1), (512, 1), (512, 2), (512, 4) "
                        "or (1024, 4)");
    b->threads = th;
    b->row_groups = rg;
    if (workgroups) b->workgroups = workgroups;
    return HAP_OK;
}

hap_status hap_batch_get_launch(hap_batch *b, int32_t *threads, int32_t *workgroups, int32_t *row_groups) {
    if (!b) return fail_arg("hap_batch_get_launch: null pointer");
    if (threads) *threads = b->threads;
    if (workgroups) *workgroups = b->workgroups;
    if (row_groups) *row_groups = b->row_groups;
    return HAP_OK;
}

hap_status hap_batch_set_split(hap_batch *b, int32_t split_n, int32_t max_members, void *stream) {
    if (!b) return fail_arg("hap_batch_set_split: null pointer");
    if (split_n < 0 || (split_n > 0 && split_n < hap::kGangMinN))
        return fail_arg("hap_batch_set_split: split_n must be 0 (off) or at least 256");
    if (max_members < 1 || max_members > hap::kMaxGang)
        return fail_arg("hap_batch_set_split: max_members must lie in [1, 16]");
    BatchPlan pl;
    std::string err;
    if (!plan_batch(b->count, b->sizes.data(), b->d, b->levels, split_n, max_members, pl, err))
        return fail_arg(err.c_str());
    const hap_status s = upload_plan(b, pl, (hipStream_t)stream);
    if (s != HAP_OK) return s;
    b->split_n = split_n;
    b->max_members = max_members;
    return HAP_OK;
}

hap_status hap_batch_get_split(hap_batch *b, int32_t *split_n, int32_t *max_members) {
    if (!b) return fail_arg("hap_batch_get_split: null pointer");
    if (split_n) *split_n = b->split_n;
    if (max_members) *max_members = b->max_members;
    return HAP_OK;
}

hap_status hap_batch_get_members(hap_batch *b, int32_t *members, int32_t *rows_per_member) {
    if (!b) return fail_arg("hap_batch_get_members: null pointer");
    for (int i = 0; i < b->count; ++i) {
        int K, rbm;
        gang_of(b->sizes[i], b->split_n, b->max_members, K, rbm);
        if (members) members[i] = K;
        if (rows_per_member) rows_per_member[i] = rbm;
    }
    return HAP_OK;
}

hap_status hap_batch_destroy(hap_batch *b) {
    if (!b) return HAP_OK;
    hap_status s = HAP_OK;
    if (b->own_ws && hipFree(b->ws) != hipSuccess) s = fail_hip(hipGetLastError(), "hap_batch_destroy");
    delete b;
    return s;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned warm start and its perceptron
// ---------------------------------------------------------------------------

namespace {

// Back to the Algorithm 1 initial state (the preferences stay), then, when Y is given, the
// warm initial availabilities of every level from the network outputs Y (n x L, row stride ldy).
template <typename T>
hap_status restart_state(hap_ctx *c, const float *Y, int64_t ldy, const T *diag = nullptr, int64_t ldd = 0) {
    const Layout lo = make_layout(c->n, c->L, c->esz);
    char *base = (char *)c->ws;
    hipStream_t st = c->stream;
    HIP_TRY(hipMemsetAsync(base + lo.R, 0, lo.pref - lo.R, st), c);
    HIP_TRY(hipMemsetAsync(base + lo.Q, 0, lo.Qpart - lo.Q, st), c);
    HIP_TRY(hipMemsetAsync(c->ds, 0, sizeof(DevState), st), c);
    if (c->pair_slots)
        HIP_TRY(hipMemsetAsync(c->pair_slots, 0xff, (size_t)hap::kPairSlotWords * kMaxPairs * sizeof(uint64_t), st),
                c);
    HIP_TRY(hap::launch_alpha_pad<T>((T *)c->A, (int64_t)c->L * c->n, (int)c->n, c->ldw, st), c);
    if (Y) {
        for (int l = 0; l < c->L; ++l) {
            LevelPtrs<T> lv = level_ptrs<T>(c, l);
            HIP_TRY(hap::launch_warm_alpha<T>(lv, (int)c->n, c->ldw, Y, ldy, l, (T *)c->Qpart, st), c);
        }
    } else if (diag) {
        for (int l = 0; l < c->L; ++l) {
            LevelPtrs<T> lv = level_ptrs<T>(c, l);
            HIP_TRY(hap::launch_warm_fill<T>(lv, (int)c->n, c->ldw, diag + l, ldd, st), c);
        }
    }
    HIP_TRY(hipStreamSynchronize(st), c);
    c->t_host = 0;
    c->labels_ready = false;
    return HAP_OK;
}

bool mlp_dims_ok(int32_t n_in, int32_t hidden, int32_t n_out) {
    return n_in >= 1 && hidden >= 1 && n_out >= 1 && n_in <= 4096 && hidden <= 4096 && n_out <= 4096;
}

}  // namespace

extern "C" {

hap_status hap_warm_features(hap_ctx *c, float *F, int64_t ldf) {
    if (!c || !F) return fail_arg("hap_warm_features: null pointer");
    if (c->failed) return fail_arg("hap_warm_features: context failed earlier", HAP_E_STATE);
    if (c->n < 2) return fail_arg("hap_warm_features: needs at least two points");
    if (ldf < HAP_WARM_FEATURES) return fail_arg("hap_warm_features: ldf < HAP_WARM_FEATURES");
    hipError_t e;
    if (c->dtype == HAP_F32)
        e = hap::launch_warm_features<float>((const float *)c->S, c->lds, (const float *)c->pref, (int)c->n, F, ldf,
                                             c->Qpart, c->stream);
    else
        e = hap::launch_warm_features<double>((const double *)c->S, c->lds, (const double *)c->pref, (int)c->n, F, ldf,
                                              c->Qpart, c->stream);
    if (e != hipSuccess) return fail_hip(e, "hap_warm_features", c);
    HIP_TRY(hipStreamSynchronize(c->stream), c);
    return HAP_OK;
}

hap_status hap_warm_targets(hap_ctx *c, float *T, int64_t ldt) {
    if (!c || !T) return fail_arg("hap_warm_targets: null pointer");
    if (c->failed) return fail_arg("hap_warm_targets: context failed earlier", HAP_E_STATE);
    if (ldt < c->L) return fail_arg("hap_warm_targets: ldt < levels");
    for (int l = 0; l < c->L; ++l) {
        hipError_t e;
        if (c->dtype == HAP_F32)
            e = hap::launch_warm_targets<float>(level_ptrs<float>(c, l), (int)c->n, c->ldw, c->lam, c->t_host, T + l,
                                                ldt, c->stream);
        else
            e = hap::launch_warm_targets<double>(level_ptrs<double>(c, l), (int)c->n, c->ldw, c->lam, c->t_host, T + l,
                                                 ldt, c->stream);
        if (e != hipSuccess) return fail_hip(e, "hap_warm_targets", c);
    }
    HIP_TRY(hipStreamSynchronize(c->stream), c);
    return HAP_OK;
}

hap_status hap_set_warm_start(hap_ctx *c, const float *Y, int64_t ldy) {
    if (!c) return fail_arg("hap_set_warm_start: null context");
    if (c->failed) return fail_arg("hap_set_warm_start: context failed earlier", HAP_E_STATE);
    if (Y && ldy < c->L) return fail_arg("hap_set_warm_start: ldy < levels");
    return c->dtype == HAP_F32 ? restart_state<float>(c, Y, ldy) : restart_state<double>(c, Y, ldy);
}

hap_status hap_set_warm_alpha(hap_ctx *c, const void *alpha_diag0, int64_t ld) {
    if (!c) return fail_arg("hap_set_warm_alpha: null context");
    if (c->failed) return fail_arg("hap_set_warm_alpha: context failed earlier", HAP_E_STATE);
    if (!alpha_diag0) return fail_arg("hap_set_warm_alpha: null alpha_diag0 (hap_set_warm_start(ctx, NULL, 0) restarts cold)");
    if (ld < c->L) return fail_arg("hap_set_warm_alpha: ld < levels");
    if (c->dtype == HAP_F32) return restart_state<float>(c, nullptr, 0, (const float *)alpha_diag0, ld);
    return restart_state<double>(c, nullptr, 0, (const double *)alpha_diag0, ld);
}

hap_status hap_iterate_warm(hap_ctx *c, const float *Y, int64_t ldy, int32_t max_iters, int32_t stable_iters,
                            int32_t *iters_done, int32_t *converged, int32_t *fell_back) {
    if (!c) return fail_arg("hap_iterate_warm: null context");
    if (stable_iters < 1) return fail_arg("hap_iterate_warm: the fallback needs a stop rule (stable_iters >= 1)");
    hap_status s = hap_set_warm_start(c, Y, ldy);
    if (s != HAP_OK) return s;
    int32_t it = 0, conv = 0, fell = 0;
    s = hap_iterate(c, max_iters, stable_iters, &it, &conv);
    if (s != HAP_OK) return s;
    if (!conv && Y) {
        s = hap_set_warm_start(c, nullptr, 0);
        if (s != HAP_OK) return s;
        s = hap_iterate(c, max_iters, stable_iters, &it, &conv);
        if (s != HAP_OK) return s;
        fell = 1;
    }
    if (iters_done) *iters_done = it;
    if (converged) *converged = conv;
    if (fell_back) *fell_back = fell;
    return HAP_OK;
}

hap_status hap_iterate_warm_judged(hap_ctx *c, const float *Y, int64_t ldy, int32_t max_iters, int32_t stable_iters,
                                   const void *X, int64_t d, int64_t ldx, int32_t x_dtype, int32_t *iters_done,
                                   int32_t *converged, int32_t *fell_back, double *ns_warm, double *ns_cold) {
    if (!c) return fail_arg("hap_iterate_warm_judged: null context");
    if (!Y) return fail_arg("hap_iterate_warm_judged: null warm start");
    if (stable_iters < 1) return fail_arg("hap_iterate_warm_judged: the judge needs a stop rule (stable_iters >= 1)");
    int32_t it_w = 0, cv_w = 0, it_c = 0, cv_c = 0;
    double sw = 0.0, sc = 0.0;
    hap_status s = hap_set_warm_start(c, Y, ldy);
    if (s == HAP_OK) s = hap_iterate(c, max_iters, stable_iters, &it_w, &cv_w);
    if (s == HAP_OK) s = hap_net_similarity(c, -1, X, d, ldx, x_dtype, &sw);
    if (s == HAP_OK) s = hap_set_warm_start(c, nullptr, 0);
    if (s == HAP_OK) s = hap_iterate(c, max_iters, stable_iters, &it_c, &cv_c);
    if (s == HAP_OK) s = hap_net_similarity(c, -1, X, d, ldx, x_dtype, &sc);
    if (s != HAP_OK) return s;
    // net similarity decides: a converged run whose clustering scores worse (such as one
    // where every point stays its own exemplar) loses against an unconverged better one
    const bool keep_warm = !(sc > sw);
    if (keep_warm) {
        int32_t it = 0, cv = 0;
        s = hap_set_warm_start(c, Y, ldy);
        if (s == HAP_OK) s = hap_iterate(c, max_iters, stable_iters, &it, &cv);
        if (s != HAP_OK) return s;
        if (it != it_w || cv != cv_w) return fail_arg("hap_iterate_warm_judged: the warm rerun differs", HAP_E_STATE);
    }
    if (iters_done) *iters_done = keep_warm ? it_w : it_c;
    if (converged) *converged = keep_warm ? cv_w : cv_c;
    if (fell_back) *fell_back = keep_warm ? 0 : 1;
    if (ns_warm) *ns_warm = sw;
    if (ns_cold) *ns_cold = sc;
    return HAP_OK;
}

int64_t hap_mlp_param_count(int32_t n_in, int32_t hidden, int32_t n_out) {
    if (!mlp_dims_ok(n_in, hidden, n_out)) return -1;
    return hap::mlp_layout(n_in, hidden, n_out, 0).count;
}

hap_status hap_mlp_workspace_size(int32_t n_in, int32_t hidden, int32_t n_out, int64_t rows, size_t *bytes) {
    if (!bytes) return fail_arg("hap_mlp_workspace_size: null pointer");
    if (!mlp_dims_ok(n_in, hidden, n_out) || rows < 0 || rows > INT32_MAX)
        return fail_arg("hap_mlp_workspace_size: bad sizes");
    *bytes = hap::mlp_layout(n_in, hidden, n_out, rows).bytes;
    return HAP_OK;
}

hap_status hap_mlp_forward(const float *params, int32_t n_in, int32_t hidden, int32_t n_out, int32_t precision,
                           const float *X, int64_t ldx, int64_t rows, float *Y, int64_t ldy, void *workspace,
                           size_t workspace_bytes, void *stream) {
    if (!params || !X || !Y || !workspace) return fail_arg("hap_mlp_forward: null pointer");
    if (!mlp_dims_ok(n_in, hidden, n_out) || rows < 0 || rows > INT32_MAX || ldx < n_in || ldy < n_out)
        return fail_arg("hap_mlp_forward: bad sizes");
    if (precision != HAP_F32 && precision != HAP_BF16)
        return fail_arg("hap_mlp_forward: precision must be HAP_F32 or HAP_BF16", HAP_E_DTYPE);
    const hap::MlpLayout lo = hap::mlp_layout(n_in, hidden, n_out, rows);
    if (workspace_bytes < lo.bytes) return fail_arg("hap_mlp_forward: workspace too small");
    hipError_t e = hap::mlp_forward(lo, n_in, hidden, n_out, precision == HAP_BF16, params, X, ldx, (int)rows, Y, ldy,
                                    (char *)workspace, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "hap_mlp_forward");
    return HAP_OK;
}

hap_status hap_mlp_loss_grad(const float *params, int32_t n_in, int32_t hidden, int32_t n_out, int32_t precision,
                             const float *X, int64_t ldx, const float *T, int64_t ldt, int64_t rows, float *grad,
                             double *loss, void *workspace, size_t workspace_bytes, void *stream) {
    if (!params || !X || !T || !grad || !loss || !workspace) return fail_arg("hap_mlp_loss_grad: null pointer");
    if (!mlp_dims_ok(n_in, hidden, n_out) || rows < 1 || rows > INT32_MAX || ldx < n_in || ldt < n_out)
        return fail_arg("hap_mlp_loss_grad: bad sizes");
    if (precision != HAP_F32 && precision != HAP_BF16)
        return fail_arg("hap_mlp_loss_grad: precision must be HAP_F32 or HAP_BF16", HAP_E_DTYPE);
    const hap::MlpLayout lo = hap::mlp_layout(n_in, hidden, n_out, rows);
    if (workspace_bytes < lo.bytes) return fail_arg("hap_mlp_loss_grad: workspace too small");
    hipError_t e = hap::mlp_loss_grad(lo, n_in, hidden, n_out, precision == HAP_BF16, params, X, ldx, T, ldt,
                                      (int)rows, grad, loss, (char *)workspace, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "hap_mlp_loss_grad");
    return HAP_OK;
}

hap_status hap_mlp_adam(float *params, const float *grad, float *opt_state, int64_t count, int64_t step, double lr,
                        double beta1, double beta2, double eps, void *stream) {
    if (!params || !grad || !opt_state) return fail_arg("hap_mlp_adam: null pointer");
    if (count < 0 || step < 1) return fail_arg("hap_mlp_adam: count < 0 or step < 1");
    if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0 && lr > 0.0))
        return fail_arg("hap_mlp_adam: bad hyper-parameters");
    hipError_t e = hap::mlp_adam(params, grad, opt_state, opt_state + count, count, step, lr, beta1, beta2, eps,
                                 (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "hap_mlp_adam");
    return HAP_OK;
}

hap_status hap_mlp_train(float *params, float *opt_state, int32_t n_in, int32_t hidden, int32_t n_out,
                         int32_t precision, int64_t step0, const float *X, int64_t ldx, const float *T, int64_t ldt,
                         int64_t rows, const int32_t *idx, int64_t batch, int64_t steps, double lr, double *loss_hist,
                         void *workspace, size_t workspace_bytes, void *stream) {
    if (!params || !opt_state || !X || !T || !idx || !workspace) return fail_arg("hap_mlp_train: null pointer");
    if (!mlp_dims_ok(n_in, hidden, n_out) || rows < 1 || rows > INT32_MAX || batch < 1 || batch > INT32_MAX ||
        steps < 0 || step0 < 0 || ldx < n_in || ldt < n_out)
        return fail_arg("hap_mlp_train: bad sizes");
    if (precision != HAP_F32 && precision != HAP_BF16)
        return fail_arg("hap_mlp_train: precision must be HAP_F32 or HAP_BF16", HAP_E_DTYPE);
    if (!(lr > 0.0)) return fail_arg("hap_mlp_train: lr must be positive");
    const hap::MlpLayout lo = hap::mlp_layout(n_in, hidden, n_out, batch);
    if (workspace_bytes < lo.bytes) return fail_arg("hap_mlp_train: workspace too small");
    char *ws = (char *)workspace;
    hipStream_t st = (hipStream_t)stream;
    float *Xb = (float *)(ws + lo.Xb), *Tb = (float *)(ws + lo.Tb), *G = (float *)(ws + lo.G);
    double *loss = (double *)(ws + lo.loss);
    for (int64_t s = 0; s < steps; ++s) {
        const int32_t *ix = idx + s * batch;
        hipError_t e = hap::mlp_gather(X, ldx, n_in, ix, (int)batch, (int)rows, Xb, st);
        if (e == hipSuccess) e = hap::mlp_gather(T, ldt, n_out, ix, (int)batch, (int)rows, Tb, st);
        if (e == hipSuccess)
            e = hap::mlp_loss_grad(lo, n_in, hidden, n_out, precision == HAP_BF16, params, Xb, n_in, Tb, n_out,
                                   (int)batch, G, loss_hist ? loss_hist + s : loss, ws, st);
        if (e == hipSuccess)
            e = hap::mlp_adam(params, G, opt_state, opt_state + lo.count, lo.count, step0 + s + 1, lr, 0.9, 0.999,
                              1e-8, st);
        if (e != hipSuccess) return fail_hip(e, "hap_mlp_train");
    }
    return HAP_OK;
}

}  // extern "C"
