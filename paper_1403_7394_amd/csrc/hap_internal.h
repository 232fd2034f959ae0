// Internal declarations shared by the libhap HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/hap.h"

namespace hap {

// Device-resident iteration state.  Kernels read the iteration counter from here
// (not from a launch argument) so that a captured sweep can be replayed.
struct DevState {
    int32_t t;              // completed iterations (sweeps)
    int32_t stable;         // consecutive iterations with unchanged labels (as of label iteration t-1)
    int32_t done;           // 1 once the stable count reached K: later sweeps do nothing
    int32_t stop_iter;      // iteration at which the run stopped
    int32_t changed;        // set by the row pass when any label changed in the current sweep
    int32_t final_changed;  // set by the finalize pass when e^t differs from e^{t-1}
    int32_t pair_abort;     // set when a paired row pass gave up waiting for a partner workgroup
    int32_t pad;
};

// 16-byte vectors: 4 floats or 2 doubles per lane access.
template <typename T> struct Vec;
template <> struct Vec<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int N = 4;
};
template <> struct Vec<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int N = 2;
};

template <typename T> __device__ __forceinline__ T neg_inf();
template <> __device__ __forceinline__ float neg_inf<float>() { return -__builtin_huge_valf(); }
template <> __device__ __forceinline__ double neg_inf<double>() { return -__builtin_huge_val(); }
template <typename T> __device__ __forceinline__ T pos_inf() { return -neg_inf<T>(); }

// Launch shape of the row pass.
struct Launch {
    int threads;        // threads per workgroup (one row at a time per workgroup)
    int chunks;         // 16-byte column chunks per thread
    int rows_per_block; // rows handled by one workgroup (column partials are per workgroup)
    bool ordered;       // column partials summed strictly in workgroup order
    bool streaming;     // large rows: 1024 threads, phase 2 re-reads S and R (chunks 2..16); or, FP32
                        // with 512 threads x 16 chunks, the held-row pass (phase 2 reads nothing)
    bool blocks = false; // workgroup g takes rows [g rb, (g + 1) rb) instead of g, g + G, g + 2G, ...
                         // (G workgroups), the default, under which the rows in flight at any
                         // moment are neighbours in memory
};
// Row stride of the row passes for this launch over `rows` rows (0: contiguous blocks).
inline int row_stride_of(const Launch &lc, int rows) {
    if (lc.blocks || lc.rows_per_block <= 1) return 0;
    return (rows + lc.rows_per_block - 1) / lc.rows_per_block;
}

// Pointers of one level inside the workspace.
template <typename T>
struct LevelPtrs {
    T *R, *A;          // n x ldw
    T *pref;           // [ldw]
    T *Q;              // [ldw] column sums of the last sweep
    T *phi;            // [ldw] phi^l (sent down by level l+1)
    T *tau;            // [ldw] tau^l (sent up by level l-1); unused at l = 0
    T *C;              // [ldw] cluster preference c^l
    T *B;              // [ldw] availability base c + phi + Q (Q at the top level) of the last sweep
    int32_t *E;        // [ldw] labels of the last label pass
    int32_t *Efinal;   // [ldw] labels reported by hap_exemplars
    T *delta;          // [ldw] Eq. 2.7 row offsets of s^l (0 at l = 0 and while the update is off)
};

// Host launchers (defined in the .hip files).
// Options of one row-pass launch.  X != nullptr selects the points mode of the
// register-resident row pass (FP32, d = 2 or 3): s_ij is recomputed from the coordinates
// instead of read from S.  tau_c/tau_q/tau_store/mrhap select the MapReduce schedule.
template <typename T>
struct SweepExtra {
    const T *X = nullptr;
    int64_t ldx = 0;
    int d = 0;
    const T *tau_c = nullptr, *tau_q = nullptr;
    T *tau_store = nullptr;
    int mrhap = 0;
    const T *delta = nullptr;   // Eq. 2.7 row offsets of this level's similarity
    int rows = 0;               // rows [0, rows) only (one block of a run split by rows); 0: all
    uint64_t *pair_slots = nullptr;   // the paired row pass's exchange slots (kPairSlotWords per pair)
    uint64_t pair_wait = 0;           // wall-clock ticks one of its waits may take
    int pair_level = 0;               // the level this launch updates (part of the exchange tags)
};
// The paired row pass (FP32 rows of 32768 < n <= 65536, two workgroups per block of rows):
// exchange slots in device memory, 20 words per pair, initialised to all ones (a tag no row
// carries).
struct PairArgs {
    uint64_t *slots;
    uint64_t wait_ticks;
    int level;
};
constexpr int kPairSlotWords = 20;
// Workgroups of the paired pass's launch that the device holds at once (the grid must fit).
int pair_capacity(int threads);
// Workgroups the paired pass launches for a block of rb rows per pair.
int64_t pair_grid(int64_t rows, int64_t rb);
template <typename T>
hipError_t launch_sweep_level(const T *S, int64_t lds, const LevelPtrs<T> &lv, T *phi_down,
                              const T *tau_l, int n, int64_t ldw, double lam, T *Qpart, const Launch &lc,
                              DevState *ds, hipStream_t st, const SweepExtra<T> &ex);
template <typename T>
hipError_t launch_colsum(const T *Qpart, int64_t ldw, int nb, int n, const LevelPtrs<T> &lv,
                         const LevelPtrs<T> *down, T *tau_next, bool top, bool last, int K, bool ordered,
                         DevState *ds, hipStream_t st);
template <typename T>
hipError_t launch_finalize(const T *S, int64_t lds, const LevelPtrs<T> &lv, int n, int64_t ldw, double lam, int t,
                           int32_t *labels_out, T *alpha_out, int64_t lda, T *c_out, T *phi_out, DevState *ds,
                           hipStream_t st, const T *delta = nullptr, int rows = 0);
// Optional level-wise similarity update (Eq. 2.7), level-sequential schedule.  Run after the
// column sums of level l in iteration t, before the row pass of level l+1:
//   launch_level_phi:   phi^l = max_k(alpha^{l+1,t-1}_ik + s^{l+1,t-1}_ik), alpha^{l+1,t-1}
//                       finished on the fly from the state of level l+1 (up), with up.delta still
//                       holding the offsets of iteration t-1; nothing in iteration 1 (phi^l = 0)
//   launch_level_delta: delta^{l+1}_i = delta^l_i + kappa * max_{j != i}(alpha^{l,t}_ij + rho^{l,t}_ij),
//                       alpha^{l,t} finished on the fly with B_j = (c^l_j + phi^l_j) + Q^l_j, which
//                       a first small launch writes to lv.B (the value the column sums of level
//                       l+1 store there again)
template <typename T>
hipError_t launch_level_phi(const T *S, int64_t lds, const LevelPtrs<T> &up, T *phi_out, int n, int64_t ldw,
                            double lam, const DevState *ds, hipStream_t st);
template <typename T>
hipError_t launch_level_delta(const LevelPtrs<T> &lv, T *delta_next, int n, int64_t ldw, double lam, double kappa,
                              const DevState *ds, hipStream_t st);
bool launch_supported(int threads, int chunks, int elem_size);

// The fused all-level row pass of the MapReduce schedule (FP32, S read from memory, the
// register-resident shapes with 4 chunks per thread, up to kMaxFused levels): one launch runs
// every level of each row, reading the row of S once.  Per level l: R, A, pref, C, E, B and
// the partial buffer Qpart (nb x ldw); Q[l] the column sums of the previous iteration (read as
// Q^{l-1} for tau^l); phi[l-1] and tau[l] written for l > 0.
constexpr int kMaxFused = 4;
template <typename T>
struct FusedArgs {
    const T *S;
    int64_t lds, ldw;
    int n, rows, rb, L;
    int row_stride;   // row order of a workgroup, as in the per-level row passes
    T lam, oml;
    DevState *ds;
    T *R[kMaxFused];
    T *A[kMaxFused];
    const T *pref[kMaxFused];
    T *C[kMaxFused];
    T *phi[kMaxFused];
    const T *B[kMaxFused];
    const T *Q[kMaxFused];
    T *tau[kMaxFused];
    int32_t *E[kMaxFused];
    T *Qpart[kMaxFused];
};
bool fused_supported(int threads, int chunks, int levels);
hipError_t launch_sweep_fused(const FusedArgs<float> &a, const Launch &lc, hipStream_t st);
template <typename T>
hipError_t launch_alpha_pad(T *A, int64_t rows, int n, int64_t ldw, hipStream_t st);

// Number of distinct values among labels[0, rows), every value in [0, n) (mark: int32 [n]).
hipError_t launch_count_distinct(const int32_t *labels, int rows, int n, int32_t *mark, int32_t *out, hipStream_t st);
hipError_t launch_net_similarity(const void *S, int64_t lds, int dtype, const void *pref_base,
                                 int64_t ldw, const int32_t *Efinal_base, int n, int levels,
                                 const void *X, int64_t d, int64_t ldx, int x_dtype, double *out,
                                 hipStream_t st);
// Bandwidth probe (hap_bandwidth_probe): reads/writes arrays of rows x cols floats (row
// stride ld) with the row pass's access pattern.  (reads, writes) in {(1,0), (1,1), (2,2), (3,2)}.
struct ProbeArgs {
    const float *in[3];
    float *out[2];
    int64_t rows, cols, ld;
    int64_t rows_per_block;
};
hipError_t launch_probe(int reads, int writes, bool cached, bool blocks, const ProbeArgs &a, hipStream_t st);

// Sampled off-diagonal pairs for the points-mode check (at most 64).
struct PairSample {
    int32_t i[64], j[64];
    int32_t count;
};
// bad[0] = number of sampled pairs whose s_ij recomputed from X (FP32, d coordinates, row
// stride ldx) by the direct build's arithmetic differs from S (FP32, row stride lds).
hipError_t launch_points_check(const float *S, int64_t lds, const float *X, int64_t ldx, int d, const PairSample &ps,
                               int32_t *bad, hipStream_t st);
hipError_t launch_fill_pref(void *pref_base, int64_t ldw, int n, int levels, int dtype,
                            const double *value_dev, hipStream_t st);

// Radix select of the two middle off-diagonal order statistics; writes their FP64 mean,
// rounded to the working type, to *median_dev (as double).
size_t select_scratch_bytes();
// Device address (on the current device) of the library's static select scratch, looked up with
// hipGetSymbolAddress on the first call per device; its size in bytes.
hipError_t static_scratch(void **out);
size_t static_scratch_bytes();
// Largest n the radix select takes: its histograms count up to n(n-1) keys in 32 bits.
constexpr int64_t kMaxSelectN = 65536;
hipError_t launch_median_offdiag(const void *S, int64_t n, int64_t lds, int dtype, void *scratch,
                                 double *median_dev, hipStream_t st);

hipError_t launch_build(const void *X, int64_t n, int64_t d, int64_t ldx, int x_dtype, void *S,
                        int64_t lds, int s_dtype, int mode, double noise_rel, uint64_t seed,
                        hipStream_t st);

// Batched form (batch.hip): one descriptor per instance.
struct BatchDesc {
    int64_t x_off;   // first row of the instance in the packed points
    int64_t w_off;   // first float of the instance's workspace
    int64_t i_off;   // first int of the instance's integer workspace
    int64_t out_off; // first label of the instance in the output (levels x n, level-major)
    int n;
    int ld;          // padded row length (multiple of 64) of S, R, A
    int K;           // workgroups sharing the instance (its gang); 1: one workgroup runs it alone
    int rbm;         // rows per member when K > 1: member m sweeps rows [m*rbm, min(n, (m+1)*rbm))
    int64_t g_off;   // first float of the gang's column partials P[2][K][ld] (instances that may be split)
    int64_t s_off;   // first int of the gang's sync words (instances that may be split; kGangInts ints)
};
// One unit of work handed out by the batch queue: member m of instance b.
struct BatchItem {
    int b, m;
};
// Instances above kGangMinN points may be split over up to kMaxGang workgroups; each such
// instance holds room for the largest gang.  Sync words: [0] barrier counter, [4 + 2m + p]
// label-changed flag of member m for iterations of parity p.
constexpr int kGangMinN = 256;
constexpr int kMaxGang = 16;
constexpr int kGangInts = 64;

// Per-instance workspace (floats): S, then per level R, A, then per level the vectors
// pref, Q, phi, tau, C, B.  Ints: per level E, then a DevState.
__host__ __device__ inline int64_t batch_floats(int n, int ld, int levels) {
    return (int64_t)n * ld * (1 + 2 * levels) + (int64_t)6 * levels * ld;
}
__host__ __device__ inline int64_t batch_ints(int ld, int levels) {
    return (int64_t)levels * ld + (int64_t)(sizeof(DevState) / sizeof(int32_t));
}

// queue[0]: next item handed out; queue[1]: set when a gang could not meet within the wait limit
hipError_t launch_batch(const float *X, int64_t d, const BatchDesc *desc, const BatchItem *items, int n_items,
                        int count, int levels, double lam, int max_iters, int stable_iters, float *wsf, int32_t *wsi,
                        int32_t *queue, int32_t *labels, double *ns, int32_t *iters, int threads, int workgroups,
                        int groups, bool gangs, hipStream_t st);

// Warm-start perceptron (mlp.hip).  Offsets of the flat parameter vector (floats) and of the
// workspace regions (bytes) for `rows` rows.
struct MlpLayout {
    int64_t oW1, ob1, oW2, ob2, oW3, ob3, count;
    size_t Xb, Tb, H1, H2, Y, dY, dH2, dH1, G, loss, bytes;
};
MlpLayout mlp_layout(int n_in, int hidden, int n_out, int64_t rows);
hipError_t mlp_forward(const MlpLayout &lo, int n_in, int hidden, int n_out, bool bf16, const float *P,
                       const float *X, int64_t ldx, int rows, float *Y, int64_t ldy, char *ws, hipStream_t st);
hipError_t mlp_loss_grad(const MlpLayout &lo, int n_in, int hidden, int n_out, bool bf16, const float *P,
                         const float *X, int64_t ldx, const float *T, int64_t ldt, int rows, float *G, double *loss,
                         char *ws, hipStream_t st);
hipError_t mlp_adam(float *P, const float *G, float *M, float *V, int64_t count, int64_t step, double lr, double b1,
                    double b2, double eps, hipStream_t st);
hipError_t mlp_gather(const float *X, int64_t ldx, int w, const int32_t *idx, int rows, int x_rows, float *out,
                      hipStream_t st);

// Warm start (warm.hip).  Features of every row of S (n x HAP_WARM_FEATURES floats) with
// scratch of warm_feature_scratch_bytes(n); training targets of the current state; warm
// initial availabilities from network outputs.
size_t warm_feature_scratch_bytes(int64_t n);
template <typename T>
hipError_t launch_warm_features(const T *S, int64_t lds, const T *pref, int n, float *F, int64_t ldf, void *scratch,
                                hipStream_t st);
template <typename T>
hipError_t launch_warm_targets(const LevelPtrs<T> &lv, int n, int64_t ldw, double lam, int t, float *out, int64_t ldo,
                               hipStream_t st);
template <typename T>
hipError_t launch_warm_alpha(const LevelPtrs<T> &lv, int n, int64_t ldw, const float *Y, int64_t ldy, int col,
                             T *bases_scratch, hipStream_t st);
// alpha^l from given diagonal values bases[j * stride] (alpha_ij = min(0, bases_j) off it).
template <typename T>
hipError_t launch_warm_fill(const LevelPtrs<T> &lv, int n, int64_t ldw, const T *bases, int64_t stride,
                            hipStream_t st);

void set_error(const std::string &msg);

}  // namespace hap
