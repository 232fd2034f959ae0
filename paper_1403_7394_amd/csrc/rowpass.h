// Device code of the fused per-level row pass, shared by the sweep launches and the
// batched persistent kernel.  See sweep.hip for the scheme (Eq. 2.1-2.6, Algorithm 1).
#pragma once

#include <climits>

#include "hap_internal.h"

namespace hap {

template <typename T>
struct SweepArgs {
    const T *__restrict__ S;
    int64_t lds;
    T *__restrict__ R;
    T *__restrict__ A;
    int64_t ldw;
    const T *__restrict__ pref;
    T *C;                 // [ldw] c^l, written by the row pass
    T *phi_down;          // phi^{l-1}, nullptr at l = 0
    const T *__restrict__ B;    // B^{l,t-1}_j = c_j + phi_j + Q_j (Q_j at the top level), formed by the column sums
    const T *__restrict__ tau;  // nullptr at l = 0 (tau^1 = +inf)
    int32_t *E;
    T *__restrict__ Qpart;
    int n;
    int rows;      // the pass covers rows [0, rows) (n, or one block of a run split by rows)
    int rb;
    T lam, oml;
    DevState *ds;
    const T *X;           // points mode: s_ij recomputed from X (row stride ldx) instead of read
    int64_t ldx;
    // MapReduce schedule (Section 3): tau_i = tau_c[i] + tau_q[i] (c^{l-1} of this iteration,
    // column sums Q^{l-1} of the previous one; no clip in the first iteration), stored in
    // tau_store; phi^{l-1} is also written in the first iteration.
    const T *tau_c, *tau_q;
    T *tau_store;
    int mrhap;
    // Eq. 2.7 (optional): row offsets of this level's similarity, s_ij + delta_i off the
    // diagonal (read by the D < 0 instances of the register-resident row pass and by the
    // streaming row pass); nullptr when the update is off
    const T *delta;
    // Row order of a workgroup: 0 = the block of rows [row0, row0 + rb); s > 0 = rows
    // first, first + s, first + 2s, ... (first = row0 / rb, s = the number of row groups), so
    // that the rows the workgroups work on at any moment are neighbours in memory
    int row_stride;
};

// Row of slot k of the workgroup whose slots are [row0, row1) (see SweepArgs::row_stride).
__device__ __forceinline__ int slot_row(int k, int row0, int rb, int stride) {
    return stride ? row0 / rb + (k - row0) * stride : k;
}
// End of the workgroup's slots: rb rows from row0, or fewer at the end of the rows.
__device__ __forceinline__ int slots_end(int rows, int rb, int row0, int stride) {
    if (stride == 0) return min(rows, row0 + rb);
    const int first = row0 / rb;
    if (first >= stride || first >= rows) return row0;
    return row0 + min(rb, (rows - first + stride - 1) / stride);
}

// The upward message this row pass clips with (Eq. 2.1 at l > 1), or false for no clip.
template <typename T>
__device__ __forceinline__ bool row_tau(const SweepArgs<T> &a, int i, int t, T &tau_i) {
    if (a.tau_c != nullptr) {
        if (t < 2) return false;
        tau_i = a.tau_c[i] + a.tau_q[i];
        return true;
    }
    if (a.tau != nullptr) {
        tau_i = a.tau[i];
        return true;
    }
    return false;
}

// Coordinates of the columns a thread owns (points mode, D coordinates per point).
template <typename T, int NCH, int D>
struct ColPoints {
    T x[NCH][Vec<T>::N][D > 0 ? D : 1];
};

// Merge two (max, argmax, second max) triples; the lower index wins a tie.
template <typename T>
__device__ __forceinline__ void top2_merge(T &m1, int &k1, T &m2, T om1, int ok1, T om2) {
    const bool take = om1 > m1 || (om1 == m1 && ok1 < k1);
    const T lo = take ? m1 : om1;     // the losing maximum competes for second place
    m2 = fmax(take ? om2 : m2, lo);
    m1 = take ? om1 : m1;
    k1 = take ? ok1 : k1;
}

template <typename T>
__device__ __forceinline__ void argmax_merge(T &v, int &k, T ov, int ok) {
    const bool take = ov > v || (ov == v && ok < k);
    v = take ? ov : v;
    k = take ? ok : k;
}

// One DPP lane move of a 32-bit value; lanes whose source row is masked off get `old`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i32(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROW_MASK, 0xf, false);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_val(float old, float v) {
    return __int_as_float(dpp_i32<CTRL, ROW_MASK>(__float_as_int(old), __float_as_int(v)));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_val(double old, double v) {
    const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
    const int lo = dpp_i32<CTRL, ROW_MASK>((int)(o & 0xffffffffll), (int)(x & 0xffffffffll));
    const int hi = dpp_i32<CTRL, ROW_MASK>((int)(o >> 32), (int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One step of the wave reduction: merge every lane's triple with the lane DPP control CTRL names
// (lanes of masked-off rows merge with the identity, which leaves them unchanged).
template <typename T, bool WITH_C, int CTRL, int ROW_MASK>
__device__ __forceinline__ void reduce_step(T &m1, int &k1, T &m2, T &cv, int &ck) {
    const T ninf = neg_inf<T>();
    const T om1 = dpp_val<CTRL, ROW_MASK>(ninf, m1);
    const int ok1 = dpp_i32<CTRL, ROW_MASK>(INT_MAX, k1);
    const T om2 = dpp_val<CTRL, ROW_MASK>(ninf, m2);
    top2_merge(m1, k1, m2, om1, ok1, om2);
    if constexpr (WITH_C) {
        const T ocv = dpp_val<CTRL, ROW_MASK>(ninf, cv);
        const int ock = dpp_i32<CTRL, ROW_MASK>(INT_MAX, ck);
        argmax_merge(cv, ck, ocv, ock);
    }
}

// Wave-wide (max, lowest argmax, second max) and (max, lowest argmax) with DPP lane moves:
// pairs, quads, 8-lane halves and 16-lane rows by quad permutes and mirrors, then the rows by
// two row broadcasts, which leave the whole wave's result in lane 63; it is read back into
// every lane.  The merges are exact and order-independent, so any tree gives the same bits.
template <typename T, bool WITH_C>
__device__ __forceinline__ void wave_reduce(T &m1, int &k1, T &m2, T &cv, int &ck) {
    reduce_step<T, WITH_C, 0xb1, 0xf>(m1, k1, m2, cv, ck);    // quad_perm [1,0,3,2]
    reduce_step<T, WITH_C, 0x4e, 0xf>(m1, k1, m2, cv, ck);    // quad_perm [2,3,0,1]
    reduce_step<T, WITH_C, 0x141, 0xf>(m1, k1, m2, cv, ck);   // row_half_mirror
    reduce_step<T, WITH_C, 0x140, 0xf>(m1, k1, m2, cv, ck);   // row_mirror
    reduce_step<T, WITH_C, 0x142, 0xa>(m1, k1, m2, cv, ck);   // row_bcast:15 into rows 1, 3
    reduce_step<T, WITH_C, 0x143, 0xc>(m1, k1, m2, cv, ck);   // row_bcast:31 into rows 2, 3
    if constexpr (sizeof(T) == 4) {
        m1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m1), 63));
        m2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m2), 63));
        if constexpr (WITH_C) cv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cv), 63));
    } else {
        auto rl = [](double v) {
            const long long x = __double_as_longlong(v);
            const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), 63);
            const int hi = __builtin_amdgcn_readlane((int)(x >> 32), 63);
            return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
        };
        m1 = rl(m1);
        m2 = rl(m2);
        if constexpr (WITH_C) cv = rl(cv);
    }
    k1 = __builtin_amdgcn_readlane(k1, 63);
    if constexpr (WITH_C) ck = __builtin_amdgcn_readlane(ck, 63);
}

// Rows whose per-row scalars are staged in LDS at a time.
constexpr int kWin = 64;

template <typename T, int NT, int NCH>
struct RowRegs {
    typename Vec<T>::type s[NCH], r[NCH], a[NCH];
};

// Columns j >= n: whole 16-byte vectors past n are not loaded (alpha reads as -inf so they
// never win a maximum); inside the last partial vector the padding columns of A hold -inf
// from initialisation and stay -inf or NaN, which '>' and fmax ignore.  Padding columns of
// R, A and the column partials are never read back as results.
//
// (D < 0, the optional level-wise similarity update of Eq. 2.7, adds the row offset where the
// row is used; D > 0, the points mode, has its own row pass below.)
template <typename T, int NT, int NCH, bool TAIL, int D>
__device__ __forceinline__ void load_row(const SweepArgs<T> &a, int i, RowRegs<T, NT, NCH> &x) {
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    const T *Srow = a.S + (int64_t)i * a.lds;
    const T *Rrow = a.R + (int64_t)i * a.ldw;
    const T *Arow = a.A + (int64_t)i * a.ldw;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int j0 = c * NT * VW + threadIdx.x * VW;
        if (!TAIL || j0 < a.n) {
            // every word is read once per pass: non-temporal loads (as the stores), which
            // measured 8-11% faster than cached loads of rho and alpha
            x.s[c] = __builtin_nontemporal_load((const V *)(Srow + j0));
            x.r[c] = __builtin_nontemporal_load((const V *)(Rrow + j0));
            x.a[c] = __builtin_nontemporal_load((const V *)(Arow + j0));
        } else {
            x.s[c] = (V)(T(0));
            x.r[c] = (V)(T(0));
            x.a[c] = (V)(neg_inf<T>());
        }
    }
}

// The rows of one workgroup.  FIRST: iteration 1, alpha is the initial value (nothing to
// finish, c and phi keep their initial 0).  TAIL: n is not exactly threads*chunks*VW, so
// accesses past n are guarded (an exact fit needs no guard at all).
template <typename T, int NT, int NCH, bool FIRST, bool TAIL, int D = 0>
__device__ __forceinline__ void sweep_rows(const SweepArgs<T> &a, const int t, const int row0, const int row1,
                                           const typename Vec<T>::type (&Bv)[NCH], typename Vec<T>::type (&qv)[NCH],
                                           T (*sh_m1)[NT / 64], int (*sh_k1)[NT / 64], T (*sh_m2)[NT / 64],
                                           T (*sh_cv)[NT / 64], int (*sh_ck)[NT / 64]) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = a.n;
    const int64_t ldw = a.ldw;
    const T lam = a.lam, oml = a.oml;
    const T zero = T(0), ninf = neg_inf<T>();

    // The next row's S, rho and alpha are loaded into a second register set while a row is
    // computed.  The per-row scalars (preference, tau, the Eq. 2.7 offset, the previous label)
    // of up to kWin rows are staged in LDS at the start of each window, so that no global load
    // issued after the prefetch has to be waited for inside a row (vector memory operations
    // complete in issue order).
    RowRegs<T, NT, NCH> x, y;
    int buf = 0;
    int chg = 0;   // a label of this workgroup's rows changed (thread 0; one atomic per workgroup)
    __shared__ T st_p[kWin], st_tau[kWin], st_d[kWin];
    __shared__ int st_e[kWin], st_has[kWin];
    auto rowof = [&](int k) { return slot_row(k, row0, a.rb, a.row_stride); };
    if (row0 < row1) load_row<T, NT, NCH, TAIL, D>(a, rowof(row0), y);
    for (int ii = row0; ii < row1; ++ii, buf ^= 1) {
        const int i = rowof(ii);
        const int r = (ii - row0) % kWin;
        if (r == 0) {
            __syncthreads();
            const int kk = ii + tid;
            const int k = rowof(kk);
            if (tid < kWin && kk < row1) {
                st_p[tid] = a.pref[k];
                T tv = zero;
                st_has[tid] = row_tau(a, k, t, tv) ? 1 : 0;
                st_tau[tid] = tv;
                st_d[tid] = (D < 0) ? a.delta[k] : zero;
                st_e[tid] = a.E[k];
            }
            __syncthreads();
        }
        x = y;
        if (ii + 1 < row1) load_row<T, NT, NCH, TAIL, D>(a, rowof(ii + 1), y);
        T *Rrow = a.R + (int64_t)i * ldw;
        T *Arow = a.A + (int64_t)i * ldw;
        const T p_i = st_p[r];
        const T d_i = st_d[r];   // Eq. 2.7 row offset (D < 0)
        // Column indices are handled relative to this thread's base tid*VW: element (c, v) is
        // column base + c*NT*VW + v, so compares and selects use compile-time offsets.
        const int base = tid * VW;
        int dcol = i - base;  // the diagonal sits at offset dcol
        T m1 = ninf, m2 = ninf, cv = ninf;
        int k1 = INT_MAX, ck = INT_MAX;   // offsets until the reduction
        // phase 1: finish alpha^{t-1}, reduce c/e over alpha + rho and the top two of alpha + s
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + base;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = c * NT * VW + v;
                const bool diag = dcol == j;
                const T sj = diag ? p_i : ((D < 0) ? x.s[c][v] + d_i : x.s[c][v]);
                x.s[c][v] = sj;
                const T rj = x.r[c][v];
                T al = x.a[c][v];
                if constexpr (!FIRST) {
                    const T Bj = Bv[c][v];
                    const T ah = diag ? Bj - rj : fmin(zero, Bj - fmax(zero, rj));
                    al = lam * al + oml * ah;
                    x.a[c][v] = al;
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
                if (!TAIL || j0 < n) __builtin_nontemporal_store(x.a[c], (V *)(Arow + j0));
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
        // LDS exchange of the wave results: wait for this wave's LDS writes only (not for the
        // prefetch and the stores in flight, which __syncthreads would also wait for), then the
        // barrier; the empty asm statements keep the LDS accesses on their side of it
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        m1 = sh_m1[buf][0];
        k1 = sh_k1[buf][0];
        m2 = sh_m2[buf][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) top2_merge(m1, k1, m2, sh_m1[buf][w], sh_k1[buf][w], sh_m2[buf][w]);
        if constexpr (!FIRST) {
            if (tid == 0) {
                cv = sh_cv[buf][0];
                ck = sh_ck[buf][0];
                for (int w = 1; w < NW; ++w) argmax_merge(cv, ck, sh_cv[buf][w], sh_ck[buf][w]);
                a.C[i] = cv;
                if (a.phi_down) a.phi_down[i] = m1;
                const int old = st_e[r];
                a.E[i] = ck;
                chg |= (t >= 3 && old != ck) ? 1 : 0;
            }
        } else {
            if (a.mrhap && tid == 0 && a.phi_down) a.phi_down[i] = m1;
        }
        // phase 2: rho^t, column partials.  dcol is made opaque so the diagonal masks are
        // recomputed here instead of being kept alive across the barrier.
        asm volatile("" : "+v"(dcol));
        const int k1r = k1 - base;
        const T tau_i = st_tau[r];
        const bool has_tau = st_has[r] != 0;
        if (a.tau_store && tid == 0) a.tau_store[i] = has_tau ? tau_i : pos_inf<T>();
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + base;
            V out;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = c * NT * VW + v;
                const T m = (j == k1r) ? m2 : m1;
                const T rh = has_tau ? x.s[c][v] + fmin(tau_i, -m) : x.s[c][v] - m;
                const T rn = lam * x.r[c][v] + oml * rh;
                out[v] = rn;
                qv[c][v] += (dcol == j) ? rn : fmax(zero, rn);
            }
            if (!TAIL || j0 < n) __builtin_nontemporal_store(out, (V *)(Rrow + j0));
        }
    }
    if (chg) atomicOr(&a.ds->changed, 1);
}

// Points mode: s_ij is recomputed from the coordinates (the thread's column coordinates stay
// in registers), and the next row's rho and alpha are loaded into registers while a row is
// computed.  The per-row scalars (preference, coordinates of point i, tau_i, the previous
// label) of up to kWin rows are staged in LDS at the start of each window, so no global load
// issued after the prefetch has to be waited for inside a row.
template <typename T, int NT, int NCH, int D>
struct PointsLds {
    T p[kWin];
    T tau[kWin];
    T x[kWin][D > 0 ? D : 1];
    int e[kWin];
};

template <typename T, int NT, int NCH, bool FIRST, bool TAIL, int D>
__device__ __forceinline__ void sweep_rows_points(const SweepArgs<T> &a, const int t, const int row0, const int row1,
                                                  const typename Vec<T>::type (&Bv)[NCH],
                                                  typename Vec<T>::type (&qv)[NCH], T (*sh_m1)[NT / 64],
                                                  int (*sh_k1)[NT / 64], T (*sh_m2)[NT / 64], T (*sh_cv)[NT / 64],
                                                  int (*sh_ck)[NT / 64], const ColPoints<T, NCH, D> &cp,
                                                  PointsLds<T, NT, NCH, D> &L) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = a.n;
    const int64_t ldw = a.ldw;
    const T lam = a.lam, oml = a.oml;
    const T zero = T(0), ninf = neg_inf<T>();
    const bool mr = a.tau_c != nullptr;
    const bool has_tau = mr ? (t >= 2) : (a.tau != nullptr);

    RowRegs<T, NT, NCH> x;
    int buf = 0;
    int chg = 0;
    // the column coordinates were loaded before this function: take them here, so that the
    // wait for them is not placed inside the row loop (where it would also wait for the
    // prefetch of the next row)
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < VW; ++v)
#pragma unroll
            for (int d = 0; d < D; ++d) asm volatile("" ::"v"(cp.x[c][v][d]));
    // rho and alpha of the next row are loaded into registers while this row is computed
    V yr[NCH], ya[NCH];
    auto fetch = [&](int row) {
        const T *Rr = a.R + (int64_t)row * ldw;
        const T *Ar = a.A + (int64_t)row * ldw;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + tid * VW;
            if (!TAIL || j0 < n) {
                yr[c] = __builtin_nontemporal_load((const V *)(Rr + j0));
                ya[c] = __builtin_nontemporal_load((const V *)(Ar + j0));
            } else {
                yr[c] = (V)(zero);
                ya[c] = (V)(ninf);
            }
        }
    };
    auto rowof = [&](int k) { return slot_row(k, row0, a.rb, a.row_stride); };
    if (row0 < row1) fetch(rowof(row0));
    for (int ii = row0; ii < row1; ++ii, buf ^= 1) {
        const int i = rowof(ii);
        const int r = (ii - row0) % kWin;
        if (r == 0) {
            // stage the scalars of this workgroup's next kWin rows
            __syncthreads();
            const int kk = ii + tid;
            const int k = rowof(kk);
            if (tid < kWin && kk < row1) {
                L.p[tid] = a.pref[k];
                L.tau[tid] = has_tau ? (mr ? a.tau_c[k] + a.tau_q[k] : a.tau[k]) : zero;
#pragma unroll
                for (int d = 0; d < D; ++d) L.x[tid][d] = a.X[(int64_t)k * a.ldx + d];
                L.e[tid] = a.E[k];
            }
            __syncthreads();
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            x.r[c] = yr[c];
            x.a[c] = ya[c];
        }
        if (ii + 1 < row1) fetch(rowof(ii + 1));
        // s_ij from the coordinates, with the direct build's arithmetic
        double xi[D];
#pragma unroll
        for (int d = 0; d < D; ++d) xi[d] = (double)L.x[r][d];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + tid * VW;
            if (!TAIL || j0 < n) {
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    double acc = 0.0;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        T xj = cp.x[c][v][d];
                        asm volatile("" : "+v"(xj));
                        const double df = xi[d] - (double)xj;
                        const double sq = df * df;
                        acc = acc + sq;
                    }
                    x.s[c][v] = (T)(-acc);
                }
            } else {
                x.s[c] = (V)(zero);
            }
        }
        T *Rrow = a.R + (int64_t)i * ldw;
        T *Arow = a.A + (int64_t)i * ldw;
        const T p_i = L.p[r];
        const int base = tid * VW;
        int dcol = i - base;
        T m1 = ninf, m2 = ninf, cv = ninf;
        int k1 = INT_MAX, ck = INT_MAX;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + base;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = c * NT * VW + v;
                const bool diag = dcol == j;
                const T sj = diag ? p_i : x.s[c][v];
                x.s[c][v] = sj;
                const T rj = x.r[c][v];
                T al = x.a[c][v];
                if constexpr (!FIRST) {
                    const T Bj = Bv[c][v];
                    const T ah = diag ? Bj - rj : fmin(zero, Bj - fmax(zero, rj));
                    al = lam * al + oml * ah;
                    x.a[c][v] = al;
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
                if (!TAIL || j0 < n) __builtin_nontemporal_store(x.a[c], (V *)(Arow + j0));
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
        // LDS exchange of the wave results: wait for this wave's LDS writes only (lgkmcnt 0; not
        // for the global stores and the prefetch in flight, which a workgroup fence would
        // wait for), then the barrier.  The empty asm statements keep the compiler from moving
        // the LDS accesses across it.
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        m1 = sh_m1[buf][0];
        k1 = sh_k1[buf][0];
        m2 = sh_m2[buf][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) top2_merge(m1, k1, m2, sh_m1[buf][w], sh_k1[buf][w], sh_m2[buf][w]);
        if constexpr (!FIRST) {
            if (tid == 0) {
                cv = sh_cv[buf][0];
                ck = sh_ck[buf][0];
                for (int w = 1; w < NW; ++w) argmax_merge(cv, ck, sh_cv[buf][w], sh_ck[buf][w]);
                a.C[i] = cv;
                if (a.phi_down) a.phi_down[i] = m1;
                a.E[i] = ck;
                chg |= (t >= 3 && L.e[r] != ck) ? 1 : 0;
            }
        } else {
            if (a.mrhap && tid == 0 && a.phi_down) a.phi_down[i] = m1;
        }
        asm volatile("" : "+v"(dcol));
        const int k1r = k1 - base;
        const T tau_i = L.tau[r];
        if (a.tau_store && tid == 0) a.tau_store[i] = has_tau ? tau_i : pos_inf<T>();
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + base;
            V out;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = c * NT * VW + v;
                const T m = (j == k1r) ? m2 : m1;
                const T rh = has_tau ? x.s[c][v] + fmin(tau_i, -m) : x.s[c][v] - m;
                const T rn = lam * x.r[c][v] + oml * rh;
                out[v] = rn;
                qv[c][v] += (dcol == j) ? rn : fmax(zero, rn);
            }
            if (!TAIL || j0 < n) __builtin_nontemporal_store(out, (V *)(Rrow + j0));
        }
    }
    if (chg) atomicOr(&a.ds->changed, 1);
}

}  // namespace hap
