// Batched HAP: many independent instances of up to 2048 points in ONE persistent launch.
//
// Workgroups pull work items from an atomic queue.  An item is either a whole instance, which
// one workgroup runs from start to end (the similarity build (FP64-accumulated, as
// HAP_BUILD_DIRECT), the median preference (radix select in LDS), the Algorithm 1 initial
// state, the sweeps over all rows, whose column partials are then complete column sums in row
// order, the labels of the final iteration (Eq. 2.8) and the FP64 net similarity), or one
// member of a gang: the K workgroups that share a large instance, member m owning a block of
// consecutive rows.  Members build their rows of S, compute the median themselves, sweep their
// rows and meet once per level at a barrier of the gang, where every member adds the members'
// column partials in member order (the order of the single-problem column sums with the same
// rows per workgroup) and forms the same column vectors.  The host orders the queue largest
// instance first with a gang's members consecutive, so only the gang being handed out can be
// incomplete while every earlier item runs to its end; the barrier's wait is bounded and gives
// up (raising an error flag and reporting the instance's iteration count as -1) rather than
// spin forever.
#include <algorithm>

#include "rowpass.h"

namespace hap {

struct BatchArgs {
    const float *X;
    int64_t d;
    const BatchDesc *desc;
    const BatchItem *items; // queue order
    int n_items;
    int count;
    int levels;
    float lam, oml;
    int max_iters, stable_iters;
    float *wsf;             // float workspace
    int32_t *wsi;           // int workspace
    int32_t *queue;         // [0]: next item handed out, [1]: a gang's wait gave up
    int32_t *labels;        // output labels
    double *ns;             // [count][levels + 1]
    int32_t *iters;         // [count]
    uint64_t wait_ticks;    // limit of one gang barrier wait, in wall-clock ticks
};

namespace {

typedef Vec<float>::type float4v;
constexpr int kBins = 2048;

__device__ __forceinline__ unsigned int fkey(float f) {
    const unsigned int u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float fval(unsigned int k) {
    return __uint_as_float((k & 0x80000000u) ? (k ^ 0x80000000u) : ~k);
}

template <int NT>
__device__ void build_instance(const float *__restrict__ X, int64_t d, int n, int ld, float *__restrict__ S,
                               double *xs /* LDS [64 * d] */, int r0, int r1) {
#pragma clang fp contract(off)
    // rows [r0, r1) of S; thread t computes column j = t + NT*c, the rows come through LDS in
    // blocks of 64
    for (int j0 = 0; j0 < n; j0 += NT) {
        const int j = j0 + threadIdx.x;
        for (int i0 = r0; i0 < r1; i0 += 64) {
            const int rows = min(64, r1 - i0);
            __syncthreads();
            for (int e = threadIdx.x; e < rows * d; e += NT) xs[e] = (double)X[(int64_t)(i0 + e / d) * d + e % d];
            __syncthreads();
            if (j < n) {
                const float *xj = X + (int64_t)j * d;
                for (int r = 0; r < rows; ++r) {
                    double acc = 0.0;
                    for (int k = 0; k < d; ++k) {
                        const double df = xs[r * d + k] - (double)xj[k];
                        const double sq = df * df;
                        acc = acc + sq;
                    }
                    const int i = i0 + r;
                    S[(int64_t)i * ld + j] = (i == j) ? 0.f : (float)(-acc);
                }
            }
        }
    }
    __syncthreads();
}

// Barrier of the K workgroups of a gang.  Every member arrives once per barrier, so barrier k
// of an instance completes when its counter reaches k*K.  Thread 0 publishes the workgroup's
// writes (agent-scope fence), arrives, and waits with a bounded spin: it gives up once another
// gang has given up or after `limit` wall-clock ticks, raising the batch's flag.  Returns
// whether the gang met (the same answer for every thread of the workgroup).
__device__ __forceinline__ bool gang_barrier(int32_t *ctr, int32_t target, int32_t *flag, uint64_t limit,
                                             int *sh_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            if ((uint64_t)wall_clock64() - t0 > limit) {
                __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        *sh_ok = ok;
    }
    __syncthreads();
    return *sh_ok != 0;
}

// Median of the off-diagonal entries: mean of the two middle order statistics (FP64),
// rounded to FP32.  Radix select on order-preserving keys with an LDS histogram.
template <int NT>
__device__ float median_instance(const float *__restrict__ S, int n, int ld, unsigned int *hist, int *sh) {
    const long long M = (long long)n * (n - 1);
    long long krem = M / 2 - 1;
    unsigned int prefix = 0, mask = 0;
    long long eqcount = 0;
    int hi = 32;
    while (hi > 0) {
        const int width = hi >= 11 ? 11 : hi;
        const int shift = hi - width;
        for (int b = threadIdx.x; b < kBins; b += NT) hist[b] = 0u;
        __syncthreads();
        for (long long e = threadIdx.x; e < (long long)n * n; e += NT) {
            const int i = (int)(e / n), j = (int)(e % n);
            if (i == j) continue;
            const unsigned int k = fkey(S[(int64_t)i * ld + j]);
            if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & ((1u << width) - 1u)], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            long long cum = 0;
            for (int b = 0; b < (1 << width); ++b) {
                const long long c = hist[b];
                if (krem < cum + c) {
                    sh[0] = b;
                    sh[1] = (int)(krem - cum);
                    sh[2] = (int)c;
                    break;
                }
                cum += c;
            }
        }
        __syncthreads();
        prefix |= ((unsigned int)sh[0]) << shift;
        mask |= ((1u << width) - 1u) << shift;
        krem = sh[1];
        eqcount = sh[2];
        __syncthreads();
        hi = shift;
    }
    const float lo = fval(prefix);
    float hi_v = lo;
    if (krem + 1 >= eqcount) {
        // smallest key above the selected one
        if (threadIdx.x == 0) hist[0] = 0xFFFFFFFFu;
        __syncthreads();
        unsigned int best = 0xFFFFFFFFu;
        for (long long e = threadIdx.x; e < (long long)n * n; e += NT) {
            const int i = (int)(e / n), j = (int)(e % n);
            if (i == j) continue;
            const unsigned int k = fkey(S[(int64_t)i * ld + j]);
            if (k > prefix && k < best) best = k;
        }
        atomicMin(&hist[0], best);
        __syncthreads();
        hi_v = fval(hist[0]);
        __syncthreads();
    }
    return (float)(((double)lo + (double)hi_v) / 2.0);
}


// The rows of one instance in G row groups of NTG threads (NT = G * NTG): at step k group
// g handles row row0 + k*G + g, so G rows are in flight per workgroup; every group takes
// the same number of steps and barriers.  Per row the work is that of sweep_rows (Eq.
// 2.1-2.6: finish alpha^{t-1}, reduce c/e and the top two of alpha + s, then rho^t).  The
// column sums stay in row order: groups 1..G-1 publish their rows' contributions through
// LDS and group 0 adds them, in row order, before it adds its own next row, so the sums
// (in group 0's registers) are the sequential column sums.
template <int NTG, int NCH, int G, bool FIRST>
__device__ __forceinline__ void sweep_rows_grouped(const SweepArgs<float> &a, const int t, const int row0,
                                                   const int row1, const float4v (&Bv)[NCH], float4v (&qv)[NCH],
                                                   float (*sh_m1)[G][NTG / 64], int (*sh_k1)[G][NTG / 64],
                                                   float (*sh_m2)[G][NTG / 64], float (*sh_cv)[G][NTG / 64],
                                                   int (*sh_ck)[G][NTG / 64], float4v (*contrib)[G][NCH][G > 1 ? NTG : 1],
                                                   int32_t *changed) {
#pragma clang fp contract(off)
    constexpr int VW = 4;
    constexpr int NWG = NTG / 64;
    const int tid = threadIdx.x;
    const int grp = tid / NTG, ltid = tid % NTG;
    const int lane = tid & 63, wid = ltid >> 6;
    const int n = a.n;
    const int64_t ldw = a.ldw;
    const float lam = a.lam, oml = a.oml;
    const float zero = 0.f, ninf = neg_inf<float>();
    const bool has_tau = a.tau != nullptr;
    const int base = ltid * VW;
    const int steps = (row1 - row0 + G - 1) / G;
    int chg = 0;   // a label of this group's rows changed (the group's thread 0)
    float4v xs[NCH], xr[NCH], xa[NCH];
    for (int k = 0; k < steps; ++k) {
        const int buf = k & 1;
        const int i = row0 + k * G + grp;
        const bool active = i < row1;
        float m1 = ninf, m2 = ninf, cv = ninf;
        int k1 = INT_MAX, ck = INT_MAX;
        int dcol = i - base;
        float p_i = 0.f, tau_i = 0.f;
        int e_old = 0;
        if (active) {
            const float *Srow = a.S + (int64_t)i * a.lds;
            const float *Rrow = a.R + (int64_t)i * ldw;
            float *Arow = a.A + (int64_t)i * ldw;
            // the row's scalars are loaded before its rows, so that waiting for them (memory
            // operations complete in issue order) never waits for the row loads or for stores
            p_i = a.pref[i];
            if (has_tau) tau_i = a.tau[i];
            if (!FIRST && ltid == 0) e_old = a.E[i];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int j0 = c * NTG * VW + base;
                if (j0 < n) {
                    xs[c] = __builtin_nontemporal_load((const float4v *)(Srow + j0));
                    xr[c] = __builtin_nontemporal_load((const float4v *)(Rrow + j0));
                    xa[c] = __builtin_nontemporal_load((const float4v *)(Arow + j0));
                } else {
                    xs[c] = (float4v)(0.f);
                    xr[c] = (float4v)(0.f);
                    xa[c] = (float4v)(ninf);
                }
            }
            // phase 1: finish alpha^{t-1}, reduce c/e over alpha + rho and the top two of alpha + s
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int j0 = c * NTG * VW + base;
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    const int j = c * NTG * VW + v;
                    const bool diag = dcol == j;
                    const float sj = diag ? p_i : xs[c][v];
                    xs[c][v] = sj;
                    const float rj = xr[c][v];
                    float al = xa[c][v];
                    if constexpr (!FIRST) {
                        const float Bj = Bv[c][v];
                        const float ah = diag ? Bj - rj : fminf(zero, Bj - fmaxf(zero, rj));
                        al = lam * al + oml * ah;
                        xa[c][v] = al;
                        const float cx = al + rj;
                        const bool gsel = cx > cv;
                        cv = gsel ? cx : cv;
                        ck = gsel ? j : ck;
                    }
                    const float y = al + sj;
                    const bool g1 = y > m1;
                    m2 = g1 ? m1 : fmaxf(m2, y);
                    k1 = g1 ? j : k1;
                    m1 = g1 ? y : m1;
                }
                if constexpr (!FIRST) {
                    if (j0 < n) __builtin_nontemporal_store(xa[c], (float4v *)(Arow + j0));
                }
            }
            k1 = (k1 == INT_MAX) ? INT_MAX : k1 + base;
            ck = (ck == INT_MAX) ? INT_MAX : ck + base;
            wave_reduce<float, !FIRST>(m1, k1, m2, cv, ck);
            if (lane == 0) {
                sh_m1[buf][grp][wid] = m1;
                sh_k1[buf][grp][wid] = k1;
                sh_m2[buf][grp][wid] = m2;
                if constexpr (!FIRST) {
                    sh_cv[buf][grp][wid] = cv;
                    sh_ck[buf][grp][wid] = ck;
                }
            }
        }
        // LDS exchange of the wave results and the contributions: wait for LDS traffic only,
        // so that this step's stores stay in flight across the barrier
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        // group 0: the previous step's rows of groups 1..G-1, in row order, before its own row
        if (grp == 0 && k > 0) {
            const int pb = buf ^ 1;
#pragma unroll
            for (int gg = 1; gg < G; ++gg) {
                if (row0 + (k - 1) * G + gg >= row1) break;
#pragma unroll
                for (int c = 0; c < NCH; ++c) qv[c] += contrib[pb][gg][c][ltid];
            }
        }
        if (active) {
            float *Rrow = a.R + (int64_t)i * ldw;
            m1 = sh_m1[buf][grp][0];
            k1 = sh_k1[buf][grp][0];
            m2 = sh_m2[buf][grp][0];
#pragma unroll
            for (int w = 1; w < NWG; ++w)
                top2_merge(m1, k1, m2, sh_m1[buf][grp][w], sh_k1[buf][grp][w], sh_m2[buf][grp][w]);
            if constexpr (!FIRST) {
                if (ltid == 0) {
                    cv = sh_cv[buf][grp][0];
                    ck = sh_ck[buf][grp][0];
                    for (int w = 1; w < NWG; ++w) argmax_merge(cv, ck, sh_cv[buf][grp][w], sh_ck[buf][grp][w]);
                    a.C[i] = cv;
                    if (a.phi_down) a.phi_down[i] = m1;
                    a.E[i] = ck;
                    chg |= (t >= 3 && e_old != ck) ? 1 : 0;
                }
            }
            // phase 2: rho^t and this row's column-sum contribution
            asm volatile("" : "+v"(dcol));
            const int k1r = k1 - base;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int j0 = c * NTG * VW + base;
                float4v out, q;
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    const int j = c * NTG * VW + v;
                    const float m = (j == k1r) ? m2 : m1;
                    const float rh = has_tau ? xs[c][v] + fminf(tau_i, -m) : xs[c][v] - m;
                    const float rn = lam * xr[c][v] + oml * rh;
                    out[v] = rn;
                    q[v] = (dcol == j) ? rn : fmaxf(zero, rn);
                }
                if (grp == 0)
                    qv[c] += q;
                else
                    contrib[buf][grp][c][ltid] = q;
                if (j0 < n) __builtin_nontemporal_store(out, (float4v *)(Rrow + j0));
            }
        }
    }
    if (chg) atomicOr(changed, 1);
    __syncthreads();
    // the last step's rows of groups 1..G-1
    if (grp == 0 && steps > 0) {
        const int pb = (steps - 1) & 1;
#pragma unroll
        for (int gg = 1; gg < G; ++gg) {
            if (row0 + (steps - 1) * G + gg >= row1) break;
#pragma unroll
            for (int c = 0; c < NCH; ++c) qv[c] += contrib[pb][gg][c][ltid];
        }
    }
}

template <int NT, int G, int CH>
__global__ __launch_bounds__(NT) void batch_kernel(BatchArgs g) {
#pragma clang fp contract(off)
    using V = Vec<float>::type;
    constexpr int VW = 4;
    constexpr int NW = NT / 64;
    constexpr int NTG = NT / G;          // threads per row group
    __shared__ float sh_cv[2][NW];
    __shared__ int sh_ck[2][NW];
    __shared__ float gm1[2][G][NTG / 64], gm2[2][G][NTG / 64], gcv[2][G][NTG / 64];
    __shared__ int gk1[2][G][NTG / 64], gck[2][G][NTG / 64];
    __shared__ float4v contrib[2][G][CH][G > 1 ? NTG : 1];
    __shared__ unsigned int hist[kBins];
    __shared__ double xs[64 * 32];
    __shared__ int sh[4];
    __shared__ int sh_ok;
    __shared__ double shd[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int ltid = tid % NTG;
    const int L = g.levels;
    for (;;) {
        if (tid == 0) sh[3] = atomicAdd(&g.queue[0], 1);
        __syncthreads();
        const int q = sh[3];
        __syncthreads();
        if (q >= g.n_items) break;
        const BatchItem item = g.items[q];
        const int b = item.b, m = item.m;
        const BatchDesc D = g.desc[b];
        const int n = D.n, ld = D.ld, K = D.K;
        // member m's rows (the whole instance when one workgroup runs it)
        const int r0 = (K > 1) ? m * D.rbm : 0;
        const int r1 = (K > 1) ? min(n, r0 + D.rbm) : n;
        float *S = g.wsf + D.w_off;
        float *RA = S + (int64_t)n * ld;                       // per level: R then A
        float *vec = RA + (int64_t)2 * L * n * ld;             // per level: pref, Q, phi, tau, C, B
        int32_t *E = g.wsi + D.i_off;
        DevState *ds = (DevState *)(E + (int64_t)L * ld);
        int32_t *sync = (K > 1) ? g.wsi + D.s_off : nullptr;   // [0] barrier counter, [4 + 2m + p] flags
        float *P = (K > 1) ? g.wsf + D.g_off : nullptr;        // column partials [2][K][ld]
        auto R = [&](int l) { return RA + (int64_t)(2 * l) * n * ld; };
        auto A = [&](int l) { return RA + (int64_t)(2 * l + 1) * n * ld; };
        auto vp = [&](int l, int k) { return vec + (int64_t)(6 * l + k) * ld; };
        int met = 0;   // gang barriers passed
        auto gang_sync = [&]() -> bool {
            if (K == 1) {
                __syncthreads();
                return true;
            }
            ++met;
            return gang_barrier(sync, met * K, &g.queue[1], g.wait_ticks, &sh_ok);
        };

        // 1. similarity rows, then the preference (every member computes the same median)
        build_instance<NT>(g.X + D.x_off * g.d, g.d, n, ld, S, xs, r0, r1);
        if (!gang_sync()) goto gave_up;
        {
            const float p = median_instance<NT>(S, n, ld, hist, sh);
            // 2. Algorithm 1 initial state (alpha = rho = 0, phi = c = 0; tau^1 is never read and
            //    tau^l is written before it is read); padding columns of alpha hold -inf.  Each
            //    member clears its own rows; member 0 the vectors and labels.
            for (int l = 0; l < L; ++l) {
                float *Rl = R(l), *Al = A(l);
                for (int64_t e = (int64_t)r0 * ld + tid; e < (int64_t)r1 * ld; e += NT) {
                    Rl[e] = 0.f;
                    Al[e] = ((int)(e % ld) < n) ? 0.f : neg_inf<float>();
                }
                if (m == 0) {
                    for (int j = tid; j < ld; j += NT) {
                        vp(l, 0)[j] = (j < n) ? p : 0.f;
                        for (int k = 1; k < 6; ++k) vp(l, k)[j] = 0.f;
                        E[(int64_t)l * ld + j] = 0;
                    }
                }
            }
            if (tid == 0) {
                ds->t = ds->stable = ds->done = ds->stop_iter = ds->changed = ds->final_changed = 0;
                if (K > 1) sync[4 + 2 * m] = sync[5 + 2 * m] = 0;
            }
            if (!gang_sync()) goto gave_up;
            // 3. sweeps
            int t = 0, stable = 0, stop_iter = -1, par = 0;
            for (int it = 0; it < g.max_iters; ++it) {
                t += 1;
                int32_t *chg_flag = (K > 1) ? &sync[4 + 2 * m + (t & 1)] : &ds->changed;
                for (int l = 0; l < L; ++l) {
                    SweepArgs<float> a;
                    a.S = S;
                    a.lds = ld;
                    a.R = R(l);
                    a.A = A(l);
                    a.ldw = ld;
                    a.pref = vp(l, 0);
                    a.C = vp(l, 4);
                    a.phi_down = l > 0 ? vp(l - 1, 2) : nullptr;
                    a.B = vp(l, 5);
                    a.tau = l > 0 ? vp(l, 3) : nullptr;
                    a.E = E + (int64_t)l * ld;
                    a.Qpart = nullptr;
                    a.X = nullptr;
                    a.ldx = 0;
                    a.tau_c = nullptr;
                    a.tau_q = nullptr;
                    a.tau_store = nullptr;
                    a.mrhap = 0;
                    a.delta = nullptr;
                    a.row_stride = 0;
                    a.n = n;
                    a.rb = n;
                    a.rows = n;
                    a.lam = g.lam;
                    a.oml = g.oml;
                    a.ds = ds;
                    V Bv[CH], qv[CH];
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        const int j0 = c * NTG * VW + ltid * VW;
                        Bv[c] = (t > 1 && j0 < n) ? *(const V *)(a.B + j0) : (V)(0.f);
                        qv[c] = (V)(0.f);
                    }
                    if (t == 1)
                        sweep_rows_grouped<NTG, CH, G, true>(a, t, r0, r1, Bv, qv, gm1, gk1, gm2, gcv, gck, contrib,
                                                             chg_flag);
                    else
                        sweep_rows_grouped<NTG, CH, G, false>(a, t, r0, r1, Bv, qv, gm1, gk1, gm2, gcv, gck, contrib,
                                                              chg_flag);
                    __syncthreads();   // c^l, phi^{l-1}, labels of this workgroup's rows are written
                    if (K > 1) {
                        // publish this member's column partials, then meet the gang
#pragma unroll
                        for (int c = 0; c < CH; ++c) {
                            const int j0 = c * NTG * VW + ltid * VW;
                            if (tid < NTG && j0 < n) *(V *)(P + ((int64_t)par * K + m) * ld + j0) = qv[c];
                        }
                        if (!gang_sync()) goto gave_up;
                    }
                    // column sums (row group 0: its own in row order, or the members' partials added
                    // in member order), tau^{l+1}, B^{l-1} and B^l at the top
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        const int j0 = c * NTG * VW + ltid * VW;
                        if (tid >= NTG || j0 >= n) continue;
                        V tot = qv[c];
                        if (K > 1) {
                            tot = *(const V *)(P + ((int64_t)par * K) * ld + j0);
                            for (int k = 1; k < K; ++k) tot += *(const V *)(P + ((int64_t)par * K + k) * ld + j0);
                        }
                        *(V *)(vp(l, 1) + j0) = tot;
                        if (l + 1 < L) *(V *)(vp(l + 1, 3) + j0) = *(const V *)(vp(l, 4) + j0) + tot;
                        if (l == L - 1) *(V *)(vp(l, 5) + j0) = tot;
                        if (l > 0)
                            *(V *)(vp(l - 1, 5) + j0) =
                                (*(const V *)(vp(l - 1, 4) + j0) + *(const V *)(vp(l - 1, 2) + j0)) +
                                *(const V *)(vp(l - 1, 1) + j0);
                    }
                    par ^= 1;
                    __syncthreads();
                }
                // With two levels no gang barrier separates the column sums of level 1 (which read
                // c^0 of every row) from the next iteration's level-0 pass (which rewrites c^0 of its
                // rows); with more levels one does.
                if (K > 1 && L == 2 && !gang_sync()) goto gave_up;
                // stop rule: the row passes of iteration t compared the labels of iteration t-1
                int changed_any;
                if (K > 1) {
                    changed_any = 0;
                    for (int k = 0; k < K; ++k)
                        changed_any |= __hip_atomic_load(&sync[4 + 2 * k + (t & 1)], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    changed_any = ds->changed;
                }
                if (t >= 2) {
                    const int lit = t - 1;
                    stable = (lit >= 2 && !changed_any) ? stable + 1 : 0;
                }
                __syncthreads();
                // this member's flag for the next iteration (every member has read it for iteration
                // t - 1 before the first barrier of iteration t)
                if (tid == 0) {
                    if (K > 1)
                        __hip_atomic_store(&sync[4 + 2 * m + ((t + 1) & 1)], 0, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    else
                        ds->changed = 0;
                }
                if (g.stable_iters > 0 && stable >= g.stable_iters) {
                    stop_iter = t - 1;
                    break;
                }
                __syncthreads();
            }
            __syncthreads();
            // 4. labels of this workgroup's rows: those recorded by the last row pass after an early
            //    stop, otherwise the labels of iteration t from alpha^t finished on the fly
            int32_t *out = g.labels + D.out_off;
            for (int l = 0; l < L; ++l) {
                if (stop_iter >= 0) {
                    for (int i = r0 + tid; i < r1; i += NT) out[(int64_t)l * n + i] = E[(int64_t)l * ld + i];
                    continue;
                }
                const float *Rl = R(l), *Al = A(l), *Bl = vp(l, 5);
                for (int i = r0; i < r1; ++i) {
                    float cv = neg_inf<float>();
                    int ck = INT_MAX;
                    for (int j = tid; j < n; j += NT) {
                        const float rj = Rl[(int64_t)i * ld + j];
                        float al = Al[(int64_t)i * ld + j];
                        if (t >= 1) {
                            const float ah = (j == i) ? Bl[j] - rj : fminf(0.f, Bl[j] - fmaxf(0.f, rj));
                            al = g.lam * al + g.oml * ah;
                        }
                        const float x = al + rj;
                        if (x > cv) {
                            cv = x;
                            ck = j;
                        }
                    }
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) {
                        const float ocv = __shfl_xor(cv, off, 64);
                        const int ock = __shfl_xor(ck, off, 64);
                        argmax_merge(cv, ck, ocv, ock);
                    }
                    if (lane == 0) {
                        sh_cv[0][wid] = cv;
                        sh_ck[0][wid] = ck;
                    }
                    __syncthreads();
                    if (tid == 0) {
                        cv = sh_cv[0][0];
                        ck = sh_ck[0][0];
                        for (int w = 1; w < NW; ++w) argmax_merge(cv, ck, sh_cv[0][w], sh_ck[0][w]);
                        out[(int64_t)l * n + i] = ck;
                    }
                    __syncthreads();
                }
            }
            if (!gang_sync()) goto gave_up;
            // 5. net similarity per level and total, FP64, fixed-order reduction (member 0)
            if (m == 0) {
                double total = 0.0;
                for (int l = 0; l < L; ++l) {
                    double acc = 0.0;
                    for (int i = tid; i < n; i += NT) {
                        const int e = out[(int64_t)l * n + i];
                        if (e < 0 || e >= n)
                            acc += __builtin_nan("");   // no valid exemplar (non-finite messages)
                        else
                            acc += (e == i) ? (double)p : (double)S[(int64_t)i * ld + e];
                    }
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
                    if (lane == 0) shd[wid] = acc;
                    __syncthreads();
                    if (tid == 0) {
                        double s2 = 0.0;
                        for (int w = 0; w < NW; ++w) s2 += shd[w];
                        g.ns[(int64_t)b * (L + 1) + l] = s2;
                        total += s2;
                    }
                    __syncthreads();
                }
                if (tid == 0) {
                    g.ns[(int64_t)b * (L + 1) + L] = total;
                    g.iters[b] = stop_iter >= 0 ? stop_iter : t;
                }
            }
            __syncthreads();
            continue;
        }
    gave_up:
        // the gang did not meet within the wait limit: the instance's results are not valid
        if (tid == 0) g.iters[b] = -1;
        __syncthreads();
    }
}

// Start of a run: the queue, the flag and every gang's barrier counter back to 0.
__global__ void batch_reset(int32_t *queue, const BatchDesc *desc, int count, int32_t *wsi) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) {
        queue[0] = 0;
        queue[1] = 0;
    }
    if (k < count && desc[k].K > 1) wsi[desc[k].s_off] = 0;
}



}  // namespace

namespace {

// Workgroups of one batch kernel instance that fit the device at once (all of them run from the
// start, so every gang's members are handed out to running workgroups).
template <int NT, int G, int CH>
int resident_workgroups() {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<NT, G, CH>, NT, 0) != hipSuccess) return 0;
    return per_cu * cus;
}

template <int NT, int G, int CH>
hipError_t launch_shape(const BatchArgs &g, int workgroups, bool gangs, hipStream_t st) {
    int grid = workgroups;
    if (gangs) {
        const int res = resident_workgroups<NT, G, CH>();
        if (res < kMaxGang) return hipErrorInvalidConfiguration;
        grid = std::min(grid, res);
    }
    hipLaunchKernelGGL((batch_kernel<NT, G, CH>), dim3(grid), dim3(NT), 0, st, g);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_batch(const float *X, int64_t d, const BatchDesc *desc, const BatchItem *items, int n_items,
                        int count, int levels, double lam, int max_iters, int stable_iters, float *wsf, int32_t *wsi,
                        int32_t *queue, int32_t *labels, double *ns, int32_t *iters, int threads, int workgroups,
                        int groups, bool gangs, hipStream_t st) {
    BatchArgs g;
    g.X = X;
    g.d = d;
    g.desc = desc;
    g.items = items;
    g.n_items = n_items;
    g.count = count;
    g.levels = levels;
    g.lam = (float)lam;
    g.oml = (float)(1.0 - lam);
    g.max_iters = max_iters;
    g.stable_iters = stable_iters;
    g.wsf = wsf;
    g.wsi = wsi;
    g.queue = queue;
    g.labels = labels;
    g.ns = ns;
    g.iters = iters;
    // a gang waits at most 60 s per barrier, longer for very long runs (a member may wait for
    // the other members to be handed out, which can take as long as one whole instance)
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return e;
    const double seconds = 60.0 * std::max(1.0, max_iters / 200.0);
    g.wait_ticks = (uint64_t)(seconds * 1000.0 * (double)(khz > 0 ? khz : 100000));
    hipLaunchKernelGGL(batch_reset, dim3((count + 255) / 256), dim3(256), 0, st, queue, desc, count, wsi);
    // threads x row groups: every row group covers 2048 columns
    if (threads == 256 && groups == 1) return launch_shape<256, 1, 2>(g, workgroups, gangs, st);
    if (threads == 512 && groups == 1) return launch_shape<512, 1, 1>(g, workgroups, gangs, st);
    if (threads == 512 && groups == 2) return launch_shape<512, 2, 2>(g, workgroups, gangs, st);
    if (threads == 512 && groups == 4) return launch_shape<512, 4, 4>(g, workgroups, gangs, st);
    if (threads == 1024 && groups == 4) return launch_shape<1024, 4, 2>(g, workgroups, gangs, st);
    return hipErrorInvalidValue;
}

}  // namespace hap
