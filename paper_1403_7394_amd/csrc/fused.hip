// The fused all-level row pass of the MapReduce schedule (Section 3).
//
// Under that schedule every level reads its inter-level messages from the previous
// iteration's state, except c^{l-1}_i, which comes from the same row of the level below in
// the same iteration (Eq. 2.4 with the c the row pass of level l-1 has just produced).  All
// of these are row-local or column vectors fixed for the whole sweep, so one launch can
// run every level of a row back to back: the row of S is read once per sweep instead of
// once per level, and each level still reads and writes its own rho and alpha rows.  Per
// level and sweep that is (4 + 1/L) N^2 words instead of 5 N^2.
//
// The arithmetic of each level is that of the per-level register-resident pass (sweep.hip):
// phase 1 finishes alpha^{t-1} and reduces c, e, M1, k1, M2; phase 2 forms rho^t and adds
// the column partials, which are kept in LDS per level (one slot per thread and column
// chunk), so with the same rows per workgroup the results are bit-identical to the per-level
// launches.  The rows' S, rho and alpha stay in registers (16-byte chunks, four per thread);
// the next (row, level) item's rows are loaded while an item is computed.
#include "rowpass.h"

namespace hap {

namespace {

template <int NT, int NCH, bool FIRST, bool TAIL>
__device__ __forceinline__ void fused_rows(const FusedArgs<float> &a, const int t, const int row0, const int row1,
                                           Vec<float>::type (*qs)[NCH][NT]) {
#pragma clang fp contract(off)
    using T = float;
    using V = Vec<float>::type;
    constexpr int VW = 4;
    constexpr int NW = NT / 64;
    constexpr int ML = kMaxFused;
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = a.n, L = a.L;
    const int64_t ldw = a.ldw;
    const T lam = a.lam, oml = a.oml;
    const T zero = T(0), ninf = neg_inf<T>();
    const int base = tid * VW;
    __shared__ T sh_m1[2][NW], sh_m2[2][NW], sh_cv[2][NW];
    __shared__ int sh_k1[2][NW], sh_ck[2][NW];
    __shared__ T st_p[ML][kWin], st_q[ML][kWin];
    __shared__ int st_e[ML][kWin];

    // per-column availability bases of every level (fixed for the sweep)
    V Bv[ML][NCH];
#pragma unroll
    for (int l = 0; l < ML; ++l)
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + base;
            Bv[l][c] = (!FIRST && l < L && (!TAIL || j0 < n)) ? *(const V *)(a.B[l] + j0) : (V)(zero);
        }

    // rows of the current and the next (row, level) item; S is loaded once per row
    V sx[NCH], sy[NCH], rx[NCH], ax[NCH], ry[NCH], ay[NCH];
    auto load_s = [&](int i, V (&s)[NCH]) {
        const float *Srow = a.S + (int64_t)i * a.lds;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + base;
            s[c] = (!TAIL || j0 < n) ? __builtin_nontemporal_load((const V *)(Srow + j0)) : (V)(zero);
        }
    };
    auto load_ra = [&](int i, int l) {
        const float *Rrow = a.R[l] + (int64_t)i * ldw;
        const float *Arow = a.A[l] + (int64_t)i * ldw;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + base;
            if (!TAIL || j0 < n) {
                ry[c] = __builtin_nontemporal_load((const V *)(Rrow + j0));
                ay[c] = __builtin_nontemporal_load((const V *)(Arow + j0));
            } else {
                ry[c] = (V)(zero);
                ay[c] = (V)(ninf);
            }
        }
    };
    int buf = 0, chg = 0;
    auto rowof = [&](int k) { return slot_row(k, row0, a.rb, a.row_stride); };
    if (row0 < row1) {
        load_s(rowof(row0), sy);
        load_ra(rowof(row0), 0);
    }
    for (int ii = row0; ii < row1; ++ii) {
        const int i = rowof(ii);
        const int r = (ii - row0) % kWin;
        if (r == 0) {
            __syncthreads();
            const int kk = ii + tid;
            const int k = rowof(kk);
            if (tid < kWin && kk < row1) {
                for (int l = 0; l < L; ++l) {
                    st_p[l][tid] = a.pref[l][k];
                    st_e[l][tid] = a.E[l][k];
                    st_q[l][tid] = l > 0 ? a.Q[l - 1][k] : zero;
                }
            }
            __syncthreads();
        }
        T c_below = zero;   // c^{l-1}_i of this iteration (the level below, this row)
#pragma unroll
        for (int l = 0; l < ML; ++l) {
            if (l >= L) break;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                if (l == 0) sx[c] = sy[c];
                rx[c] = ry[c];
                ax[c] = ay[c];
            }
            // the next item: the level above on this row, or level 0 of the next row
            if (l + 1 < L) {
                load_ra(i, l + 1);
            } else if (ii + 1 < row1) {
                const int nx = rowof(ii + 1);
                load_s(nx, sy);
                load_ra(nx, 0);
            }
            float *Rrow = a.R[l] + (int64_t)i * ldw;
            float *Arow = a.A[l] + (int64_t)i * ldw;
            const T p_i = st_p[l][r];
            int dcol = i - base;
            asm volatile("" : "+v"(dcol));
            T m1 = ninf, m2 = ninf, cv = ninf;
            int k1 = INT_MAX, ck = INT_MAX;
            // phase 1
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int j0 = c * NT * VW + base;
                V ac = ax[c];
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    const int j = c * NT * VW + v;
                    const bool diag = dcol == j;
                    const T sj = diag ? p_i : sx[c][v];
                    const T rj = rx[c][v];
                    T al = ac[v];
                    if constexpr (!FIRST) {
                        const T Bj = Bv[l][c][v];
                        // two selects (the same values as diag ? Bj - rj : min(0, Bj - max(0, rj)))
                        const T u = Bj - (diag ? rj : fmax(zero, rj));
                        const T ah = diag ? u : fmin(zero, u);
                        al = lam * al + oml * ah;
                        ac[v] = al;
                        const T cx = al + rj;
                        const bool g = cx > cv;
                        cv = g ? cx : cv;
                        ck = g ? j : ck;
                    }
                    const T y = al + sj;
                    const bool g1 = y > m1;
                    m2 = g1 ? m1 : fmax(m2, y);
                    k1 = g1 ? j : k1;
                    m1 = g1 ? y : m1;
                }
                if constexpr (!FIRST) {
                    if (!TAIL || j0 < n) __builtin_nontemporal_store(ac, (V *)(Arow + j0));
                }
            }
            k1 = (k1 == INT_MAX) ? INT_MAX : k1 + base;
            ck = (ck == INT_MAX) ? INT_MAX : ck + base;
            wave_reduce<T, !FIRST>(m1, k1, m2, cv, ck);
            if (lane == 0) {
                sh_m1[buf][wid] = m1;
                sh_k1[buf][wid] = k1;
                sh_m2[buf][wid] = m2;
                if constexpr (!FIRST) {
                    sh_cv[buf][wid] = cv;
                    sh_ck[buf][wid] = ck;
                }
            }
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            m1 = sh_m1[buf][0];
            k1 = sh_k1[buf][0];
            m2 = sh_m2[buf][0];
#pragma unroll
            for (int w = 1; w < NW; ++w) top2_merge(m1, k1, m2, sh_m1[buf][w], sh_k1[buf][w], sh_m2[buf][w]);
            // tau^l_i = c^{l-1}_i (this iteration, the level below on this row) + Q^{l-1}_i (previous
            // iteration); no clip at l = 0 or in iteration 1
            const bool has_tau = (l > 0) && (t >= 2);
            const T tau_i = c_below + st_q[l][r];
            if constexpr (!FIRST) {
                cv = sh_cv[buf][0];
                ck = sh_ck[buf][0];
#pragma unroll
                for (int w = 1; w < NW; ++w) argmax_merge(cv, ck, sh_cv[buf][w], sh_ck[buf][w]);
                if (tid == 0) {
                    a.C[l][i] = cv;
                    a.E[l][i] = ck;
                    chg |= (t >= 3 && st_e[l][r] != ck) ? 1 : 0;
                }
                c_below = cv;
            }
            if (tid == 0) {
                if (l > 0) a.phi[l - 1][i] = m1;
                if (l > 0) a.tau[l][i] = has_tau ? tau_i : pos_inf<T>();
            }
            buf ^= 1;
            // phase 2
            asm volatile("" : "+v"(dcol));
            const int k1r = k1 - base;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int j0 = c * NT * VW + base;
                V out;
                V q = qs[l][c][tid];
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    const int j = c * NT * VW + v;
                    const bool diag = dcol == j;
                    const T sj = diag ? p_i : sx[c][v];
                    const T m = (j == k1r) ? m2 : m1;
                    const T rh = has_tau ? sj + fmin(tau_i, -m) : sj - m;
                    const T rn = lam * rx[c][v] + oml * rh;
                    out[v] = rn;
                    q[v] += diag ? rn : fmax(zero, rn);
                }
                qs[l][c][tid] = q;
                if (!TAIL || j0 < n) __builtin_nontemporal_store(out, (V *)(Rrow + j0));
            }
        }
    }
    if (chg) atomicOr(&a.ds->changed, 1);
}

template <int NT, int NCH, bool TAIL>
__global__ __launch_bounds__(NT) void sweep_fused_kernel(FusedArgs<float> a) {
#pragma clang fp contract(off)
    using V = Vec<float>::type;
    constexpr int VW = 4;
    __shared__ V qs[kMaxFused][NCH][NT];
    const DevState *ds = a.ds;
    if (ds->done) return;
    const int t = ds->t + 1;
#pragma unroll
    for (int l = 0; l < kMaxFused; ++l)
#pragma unroll
        for (int c = 0; c < NCH; ++c) qs[l][c][threadIdx.x] = (V)(0.f);
    const int row0 = blockIdx.x * a.rb;
    const int row1 = slots_end(a.rows, a.rb, row0, a.row_stride);
    if (t == 1)
        fused_rows<NT, NCH, true, TAIL>(a, t, row0, row1, qs);
    else
        fused_rows<NT, NCH, false, TAIL>(a, t, row0, row1, qs);
    for (int l = 0; l < a.L; ++l) {
        float *qrow = a.Qpart[l] + (int64_t)blockIdx.x * a.ldw;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + threadIdx.x * VW;
            if (!TAIL || j0 < a.n) *(V *)(qrow + j0) = qs[l][c][threadIdx.x];
        }
    }
}

}  // namespace

bool fused_supported(int threads, int chunks, int levels) {
    return chunks == 4 && (threads == 64 || threads == 128 || threads == 256 || threads == 512) && levels >= 1 &&
           levels <= kMaxFused;
}

hipError_t launch_sweep_fused(const FusedArgs<float> &a, const Launch &lc, hipStream_t st) {
    if (lc.streaming || !fused_supported(lc.threads, lc.chunks, a.L)) return hipErrorInvalidValue;
    if ((int64_t)lc.threads * lc.chunks * 4 < a.n) return hipErrorInvalidValue;
    const int nb = (a.rows + a.rb - 1) / a.rb;
    const bool tail = (int64_t)lc.threads * lc.chunks * 4 != a.n;
#define HAP_LAUNCH_FUSED(NTC)                                                                           \
    do {                                                                                                \
        if (tail)                                                                                       \
            hipLaunchKernelGGL((sweep_fused_kernel<NTC, 4, true>), dim3(nb), dim3(NTC), 0, st, a);      \
        else                                                                                            \
            hipLaunchKernelGGL((sweep_fused_kernel<NTC, 4, false>), dim3(nb), dim3(NTC), 0, st, a);     \
    } while (0)
    switch (lc.threads) {
        case 64: HAP_LAUNCH_FUSED(64); break;
        case 128: HAP_LAUNCH_FUSED(128); break;
        case 256: HAP_LAUNCH_FUSED(256); break;
        default: HAP_LAUNCH_FUSED(512); break;
    }
#undef HAP_LAUNCH_FUSED
    return hipGetLastError();
}

}  // namespace hap
