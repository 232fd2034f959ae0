// HAP sweep kernels for gfx950: the fused per-level row pass, the column-sum
// epilogue and the non-destructive finalize pass.
//
// One iteration of Algorithm 1 visits the levels in order; at level l it
// updates rho (Eq. 2.1), then alpha from the new rho (Eq. 2.2-2.3), then emits
// tau^{l+1} (Eq. 2.4), phi^{l-1} (Eq. 2.5) and c^l (Eq. 2.6).  alpha needs the
// column sums of the new rho, a reduction over every row, so the pass that
// produces rho^{l,t} cannot also produce alpha^{l,t}.  The row pass of
// iteration t therefore first finishes alpha^{l,t-1} (deferred by one
// iteration), row by row, and then computes rho^{l,t} from it:
//
//   phase 1, row i:  alpha^{t-1}_ij = lam*A_ij + (1-lam)*avail(R_ij, B_j)  -> A
//                    c_i = max_j(alpha + R), e_i = argmax (Eq. 2.6, 2.8)
//                    M1 = max_j(alpha + s), k1 = argmax, M2 = max_{j != k1}
//                    phi^{l-1}_i = M1 (Eq. 2.5)
//   phase 2, row i:  rho^t_ij = lam*R_ij + (1-lam)*(s_ij + min(tau_i, -(j==k1 ? M2 : M1)))  -> R
//                    column partials of rho_jj / max(0, rho_ij)
//
// with R = rho^{t-1}, A = alpha^{t-2} and B_j = c_j + phi_j + Q_j (Q: column sums
// of rho^{t-1}; avail is Eq. 2.3 on the diagonal, where B_j - rho_jj is the sum
// over k != j, and Eq. 2.2 elsewhere, where B_j - max(0, rho_ij) is the sum over
// k not in {i, j} plus rho_jj).  Every value read is the one Algorithm 1
// reads at that point, so the trajectory is the level-sequential one, while
// each level moves 5 N^2 words per sweep (read S, R, A; write R, A).
//
// Each workgroup owns a set of rows (by default, of G workgroups, workgroup g takes rows g,
// g + G, g + 2G, ...; a contiguous block on request) and keeps its column partials in
// registers (every thread owns the same columns for every row); the partials are summed in a
// fixed order by the epilogue, so results are deterministic.
#include "rowpass.h"

namespace hap {

template <typename T, int NT, int NCH, bool TAIL, int D>
__global__ __launch_bounds__(NT) void sweep_kernel(SweepArgs<T> a) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    constexpr int NW = NT / 64;
    __shared__ T sh_m1[2][NW], sh_m2[2][NW], sh_cv[2][NW];
    __shared__ int sh_k1[2][NW], sh_ck[2][NW];

    const DevState *ds = a.ds;
    if (ds->done) return;
    const int t = ds->t + 1;
    const bool first = (t == 1);
    const int tid = threadIdx.x;
    const int n = a.n;
    const int64_t ldw = a.ldw;

    // Per-column constants of this pass (the same for every row) and column partials.
    V Bv[NCH], qv[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int j0 = c * NT * VW + tid * VW;
        Bv[c] = (!first && (!TAIL || j0 < n)) ? *(const V *)(a.B + j0) : (V)(T(0));
        qv[c] = (V)(T(0));
    }
    // points mode: the coordinates of this thread's columns, kept for every row
    ColPoints<T, NCH, D> cp;
    if constexpr (D > 0) {
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = c * NT * VW + tid * VW + v;
#pragma unroll
                for (int k = 0; k < D; ++k) cp.x[c][v][k] = (j < n) ? a.X[(int64_t)j * a.ldx + k] : T(0);
            }
    }
    const int row0 = blockIdx.x * a.rb;
    const int row1 = slots_end(a.rows, a.rb, row0, a.row_stride);
    if constexpr (D > 0) {
        __shared__ __attribute__((aligned(16))) PointsLds<T, NT, NCH, D> lds;
        if (first)
            sweep_rows_points<T, NT, NCH, true, TAIL, D>(a, t, row0, row1, Bv, qv, sh_m1, sh_k1, sh_m2, sh_cv, sh_ck,
                                                         cp, lds);
        else
            sweep_rows_points<T, NT, NCH, false, TAIL, D>(a, t, row0, row1, Bv, qv, sh_m1, sh_k1, sh_m2, sh_cv,
                                                          sh_ck, cp, lds);
    } else {
        if (first)
            sweep_rows<T, NT, NCH, true, TAIL, D>(a, t, row0, row1, Bv, qv, sh_m1, sh_k1, sh_m2, sh_cv, sh_ck);
        else
            sweep_rows<T, NT, NCH, false, TAIL, D>(a, t, row0, row1, Bv, qv, sh_m1, sh_k1, sh_m2, sh_cv, sh_ck);
    }

    T *qrow = a.Qpart + (int64_t)blockIdx.x * ldw;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int j0 = c * NT * VW + tid * VW;
        if (!TAIL || j0 < n) *(V *)(qrow + j0) = qv[c];
    }
}

// Buffer-resource accesses (raw buffer instructions): a per-row resource, the lane's byte
// offset in a VGPR and the chunk offset as a scalar, so a chunk costs no address registers.
// Loads past the resource's range return 0 and stores past it are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename V, int AUX>
__device__ __forceinline__ V buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
}
// Stores take the chunk offset in the VGPR offset and a constant zero scalar offset: a store of
// more than 64 bits reads its data registers after issue, and the compiler keeps a VALU write
// of those registers one wait state away from the store only when the scalar offset is not a
// register.  With an SGPR offset a write scheduled right behind the store has corrupted the
// stored values of some lanes.
template <typename V, int AUX>
__device__ __forceinline__ void buf_store(V v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    typedef unsigned int U4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, v), r, voff + soff, 0, AUX);
}
constexpr int kNT = 2;  // cache-policy operand: non-temporal

// Row pass for rows too long to keep in registers (large N, 1024 threads).  Same arithmetic
// as sweep_rows.  The chunks of a row are visited by a runtime loop: phase 1 streams S, R,
// A and B; phase 2 reads the row's S and R again (normal loads, so the second read is
// served by the caches the first read filled).  Column partials live in thread-private LDS
// slots (up to kLdsChunks chunks); further chunks keep theirs in this workgroup's own row
// of Qpart, read and written by the owning thread only.
constexpr int kLdsChunks = 8;

template <typename T, int NT, bool FIRST, bool TAIL>
__device__ __forceinline__ void stream_rows(const SweepArgs<T> &a, const int t, const int row0, const int row1,
                                            const int nch, typename Vec<T>::type (*qs)[NT],
                                            const __amdgpu_buffer_rsrc_t rQ, T (*sh_m1)[NT / 64],
                                            int (*sh_k1)[NT / 64], T (*sh_m2)[NT / 64], T (*sh_cv)[NT / 64],
                                            int (*sh_ck)[NT / 64]) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    constexpr int NW = NT / 64;
    constexpr int CB = NT * VW * (int)sizeof(T);  // bytes per chunk
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = a.n;
    const int64_t ldw = a.ldw;
    const T lam = a.lam, oml = a.oml;
    const T zero = T(0), ninf = neg_inf<T>();
    const int base = tid * VW;
    const int voff = tid * 16;
    const __amdgpu_buffer_rsrc_t rB = row_rsrc(a.B, ldw * (int64_t)sizeof(T));
    int buf = 0;
    int chg = 0;   // a label of this workgroup's rows changed (thread 0; one atomic per workgroup)
    // Software pipelining: every chunk's loads are issued one chunk ahead (and the first
    // chunk of each phase before the preceding reduction or the previous row's last chunk),
    // so the memory latency overlaps the arithmetic of the chunk before.
    auto row_s = [&](int row) { return row_rsrc(a.S + (int64_t)row * a.lds, a.lds * (int64_t)sizeof(T)); };
    auto row_w = [&](T *M, int row) { return row_rsrc(M + (int64_t)row * ldw, ldw * (int64_t)sizeof(T)); };
    V sv = (V)(zero), rv = (V)(zero), av = (V)(zero), bv = (V)(zero);   // phase-1 operands of the next chunk
    auto load1 = [&](__amdgpu_buffer_rsrc_t rS, __amdgpu_buffer_rsrc_t rR, __amdgpu_buffer_rsrc_t rA, int c) {
        sv = buf_load<V, 0>(rS, voff, c * CB);
        rv = buf_load<V, 0>(rR, voff, c * CB);
        av = buf_load<V, kNT>(rA, voff, c * CB);   // alpha is not read again in phase 2
        if constexpr (!FIRST) bv = buf_load<V, 0>(rB, voff, c * CB);
    };
    auto rowof = [&](int k) { return slot_row(k, row0, a.rb, a.row_stride); };
    if (row0 < row1) load1(row_s(rowof(row0)), row_w(a.R, rowof(row0)), row_w(a.A, rowof(row0)), 0);
    for (int ii = row0; ii < row1; ++ii, buf ^= 1) {
        const int i = rowof(ii);
        const __amdgpu_buffer_rsrc_t rS = row_s(i);
        const __amdgpu_buffer_rsrc_t rR = row_w(a.R, i);
        const __amdgpu_buffer_rsrc_t rA = row_w(a.A, i);
        const T p_i = a.pref[i];
        const int dcol = i - base;
        const bool has_d = a.delta != nullptr;
        const T d_i = has_d ? a.delta[i] : zero;
        T m1 = ninf, m2 = ninf, cv = ninf;
        int k1 = INT_MAX, ck = INT_MAX;   // offsets from base until the reduction
        V s2, r2;                         // phase-2 operands of the next chunk
        // phase 1
        for (int c = 0; c < nch; ++c) {
            const int off0 = c * NT * VW;   // this chunk's column offset from base
            V sc = sv, rc = rv, ac = av;
            const V bc = bv;
            if (c + 1 < nch) {
                load1(rS, rR, rA, c + 1);
            } else {
                s2 = buf_load<V, 0>(rS, voff, 0);
                r2 = buf_load<V, 0>(rR, voff, 0);
            }
            if (has_d) sc = sc + d_i;
            if constexpr (TAIL) {
                // columns past n: alpha reads as -inf so they never win a maximum
                if (off0 + base >= n) ac = (V)(ninf);
            }
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = off0 + v;
                const bool diag = dcol == j;
                const T sj = diag ? p_i : sc[v];
                const T rj = rc[v];
                T al = ac[v];
                if constexpr (!FIRST) {
                    const T ah = diag ? bc[v] - rj : fmin(zero, bc[v] - fmax(zero, rj));
                    al = lam * al + oml * ah;
                    ac[v] = al;
                    const T cx = al + rj;
                    const bool gg = cx > cv;
                    cv = gg ? cx : cv;
                    ck = gg ? j : ck;
                }
                const T y = al + sj;
                const bool g1 = y > m1;
                m2 = g1 ? m1 : fmax(m2, y);
                k1 = g1 ? j : k1;
                m1 = g1 ? y : m1;
            }
            if constexpr (!FIRST) buf_store<V, kNT>(ac, rA, voff, c * CB);
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
        __syncthreads();
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
                const int old = a.E[i];
                a.E[i] = ck;
                chg |= (t >= 3 && old != ck) ? 1 : 0;
            }
        } else {
            if (a.mrhap && tid == 0 && a.phi_down) a.phi_down[i] = m1;
        }
        // phase 2
        const int k1r = k1 - base;
        T tau_i = zero;
        const bool has_tau = row_tau(a, i, t, tau_i);
        if (a.tau_store && tid == 0) a.tau_store[i] = has_tau ? tau_i : pos_inf<T>();
        V qn = (V)(zero);   // column partial of the next chunk when it lives in Qpart
        for (int c = 0; c < nch; ++c) {
            const int off0 = c * NT * VW;
            V sc = s2;
            const V rc = r2;
            const V qc = qn;
            if (c + 1 < nch) {
                s2 = buf_load<V, 0>(rS, voff, (c + 1) * CB);
                r2 = buf_load<V, 0>(rR, voff, (c + 1) * CB);
                if (c + 1 >= kLdsChunks) qn = buf_load<V, 0>(rQ, voff, (c + 1) * CB);
            } else if (ii + 1 < row1) {
                const int nx = rowof(ii + 1);
                load1(row_s(nx), row_w(a.R, nx), row_w(a.A, nx), 0);
            }
            if (has_d) sc = sc + d_i;
            V out;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = off0 + v;
                const T sj = (dcol == j) ? p_i : sc[v];
                const T m = (j == k1r) ? m2 : m1;
                const T rh = has_tau ? sj + fmin(tau_i, -m) : sj - m;
                out[v] = lam * rc[v] + oml * rh;
            }
            buf_store<V, kNT>(out, rR, voff, c * CB);
            V q = (c < kLdsChunks) ? qs[c][tid] : qc;
#pragma unroll
            for (int v = 0; v < VW; ++v) q[v] += (dcol == off0 + v) ? out[v] : fmax(zero, out[v]);
            if (c < kLdsChunks)
                qs[c][tid] = q;
            else
                buf_store<V, 0>(q, rQ, voff, c * CB);
        }
    }
    if (chg) atomicOr(&a.ds->changed, 1);
}

// FP64: the same pass without the software pipelining, whose second set of operands would
// not fit the 128 registers of a 1024-thread workgroup.
template <typename T, int NT, bool FIRST, bool TAIL>
__device__ __forceinline__ void stream_rows_unpipelined(const SweepArgs<T> &a, const int t, const int row0, const int row1,
                                            const int nch, typename Vec<T>::type (*qs)[NT],
                                            const __amdgpu_buffer_rsrc_t rQ, T (*sh_m1)[NT / 64],
                                            int (*sh_k1)[NT / 64], T (*sh_m2)[NT / 64], T (*sh_cv)[NT / 64],
                                            int (*sh_ck)[NT / 64]) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    constexpr int NW = NT / 64;
    constexpr int CB = NT * VW * (int)sizeof(T);  // bytes per chunk
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = a.n;
    const int64_t ldw = a.ldw;
    const T lam = a.lam, oml = a.oml;
    const T zero = T(0), ninf = neg_inf<T>();
    const int base = tid * VW;
    const int voff = tid * 16;
    const __amdgpu_buffer_rsrc_t rB = row_rsrc(a.B, ldw * (int64_t)sizeof(T));
    int buf = 0;
    int chg = 0;   // a label of this workgroup's rows changed (thread 0; one atomic per workgroup)
    auto rowof = [&](int k) { return slot_row(k, row0, a.rb, a.row_stride); };
    for (int ii = row0; ii < row1; ++ii, buf ^= 1) {
        const int i = rowof(ii);
        const __amdgpu_buffer_rsrc_t rS = row_rsrc(a.S + (int64_t)i * a.lds, a.lds * (int64_t)sizeof(T));
        const __amdgpu_buffer_rsrc_t rR = row_rsrc(a.R + (int64_t)i * ldw, ldw * (int64_t)sizeof(T));
        const __amdgpu_buffer_rsrc_t rA = row_rsrc(a.A + (int64_t)i * ldw, ldw * (int64_t)sizeof(T));
        const T p_i = a.pref[i];
        const int dcol = i - base;
        const bool has_d = a.delta != nullptr;
        const T d_i = has_d ? a.delta[i] : zero;
        T m1 = ninf, m2 = ninf, cv = ninf;
        int k1 = INT_MAX, ck = INT_MAX;   // offsets from base until the reduction
        // phase 1
        for (int c = 0; c < nch; ++c) {
            const int off0 = c * NT * VW;   // this chunk's column offset from base
            V sv = buf_load<V, 0>(rS, voff, c * CB);
            if (has_d) sv = sv + d_i;
            const V rv = buf_load<V, 0>(rR, voff, c * CB);
            V av = buf_load<V, kNT>(rA, voff, c * CB);
            V bv = (V)(zero);
            if constexpr (!FIRST) bv = buf_load<V, 0>(rB, voff, c * CB);
            if constexpr (TAIL) {
                // columns past n: alpha reads as -inf so they never win a maximum
                if (off0 + base >= n) av = (V)(ninf);
            }
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = off0 + v;
                const bool diag = dcol == j;
                const T sj = diag ? p_i : sv[v];
                const T rj = rv[v];
                T al = av[v];
                if constexpr (!FIRST) {
                    const T ah = diag ? bv[v] - rj : fmin(zero, bv[v] - fmax(zero, rj));
                    al = lam * al + oml * ah;
                    av[v] = al;
                    const T cx = al + rj;
                    const bool gg = cx > cv;
                    cv = gg ? cx : cv;
                    ck = gg ? j : ck;
                }
                const T y = al + sj;
                const bool g1 = y > m1;
                m2 = g1 ? m1 : fmax(m2, y);
                k1 = g1 ? j : k1;
                m1 = g1 ? y : m1;
            }
            if constexpr (!FIRST) buf_store<V, kNT>(av, rA, voff, c * CB);
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
        __syncthreads();
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
                const int old = a.E[i];
                a.E[i] = ck;
                chg |= (t >= 3 && old != ck) ? 1 : 0;
            }
        } else {
            if (a.mrhap && tid == 0 && a.phi_down) a.phi_down[i] = m1;
        }
        // phase 2
        const int k1r = k1 - base;
        T tau_i = zero;
        const bool has_tau = row_tau(a, i, t, tau_i);
        if (a.tau_store && tid == 0) a.tau_store[i] = has_tau ? tau_i : pos_inf<T>();
        for (int c = 0; c < nch; ++c) {
            const int off0 = c * NT * VW;
            V sv = buf_load<V, 0>(rS, voff, c * CB);
            if (has_d) sv = sv + d_i;
            const V rv = buf_load<V, 0>(rR, voff, c * CB);
            V out;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = off0 + v;
                const T sj = (dcol == j) ? p_i : sv[v];
                const T m = (j == k1r) ? m2 : m1;
                const T rh = has_tau ? sj + fmin(tau_i, -m) : sj - m;
                out[v] = lam * rv[v] + oml * rh;
            }
            buf_store<V, kNT>(out, rR, voff, c * CB);
            V q = (c < kLdsChunks) ? qs[c][tid] : buf_load<V, 0>(rQ, voff, c * CB);
#pragma unroll
            for (int v = 0; v < VW; ++v) q[v] += (dcol == off0 + v) ? out[v] : fmax(zero, out[v]);
            if (c < kLdsChunks)
                qs[c][tid] = q;
            else
                buf_store<V, 0>(q, rQ, voff, c * CB);
        }
    }
    if (chg) atomicOr(&a.ds->changed, 1);
}

// Row pass for rows of up to NT*NCH*4 FP32 columns that do not fit the register-resident pass
// (16384 < n <= 32768 at 512 threads and 16 chunks): the row's S and rho are held in registers
// from phase 1 to phase 2 (128 registers), so phase 2 reads nothing from memory; alpha is
// finished and stored in phase 1, the column bases B are read per chunk, and the column
// partials live in LDS.  Phase 1's loads run one chunk ahead of the arithmetic, and the next
// row's first chunk is loaded during phase 2's last.  The per-row scalars are staged in LDS per
// window of kWin rows, so that no global load issued after those loads is waited for in a row.
//
// PAIR: the paired pass for rows twice as long (32768 < n <= 65536 at 512 threads): two
// workgroups share a set of rows, one holding columns [0, H) and the other [H, n) of every
// row (H = NT*NCH*4), each exactly as above on its half.  Between the phases of a row each
// workgroup publishes its half's (M1, k1, M2) and (c, e) and merges the partner's: thread 0
// writes five 64-bit words, each a value with a tag naming the sweep and the row in its upper
// half, with relaxed device-scope atomic stores, and polls the partner's five words until all
// carry the tag of the row, level and sweep (per-word tags need no fences: each word is read whole), with a
// wall-clock bound.  Two slots per side, by row parity, are enough: a workgroup can publish
// row i + 2 only after it has read the partner's row i + 1, which the partner publishes after it
// has read row i.  A wait that gives up sets a flag (sticky, checked by the host, which fails
// the run) that ends every other wait at once, so the launch always drains.
struct HeldPair {
    uint64_t *mine, *theirs;   // this side's and the partner's slots: [2 row parities][5 words]
    int32_t *abort;
    uint64_t limit;            // wall-clock ticks one wait may take
    int side;
    int level;
};

__device__ __forceinline__ void pair_exchange(const HeldPair &hp, int row, int t, float &m1, int &k1, float &m2,
                                              float &cv, int &ck) {
    // the tag names the sweep, the level and the row: consecutive launches (the next level, or
    // the next sweep's first) always differ in it, so a slot a pair left in its last launch
    // never passes for the current one
    const uint32_t tag = ((uint32_t)(t & 0x3ff) << 22) | ((uint32_t)(hp.level & 0x1f) << 17) | (uint32_t)row;
    uint64_t *mine = hp.mine + (row & 1) * 5;
    const uint64_t *theirs = hp.theirs + (row & 1) * 5;
    const uint32_t out[5] = {__float_as_uint(m1), (uint32_t)k1, __float_as_uint(m2), __float_as_uint(cv),
                             (uint32_t)ck};
#pragma unroll
    for (int k = 0; k < 5; ++k)
        __hip_atomic_store(mine + k, ((uint64_t)tag << 32) | out[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t w[5];
    bool ok = false;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        bool all = true;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            w[k] = __hip_atomic_load(theirs + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            all = all && (uint32_t)(w[k] >> 32) == tag;
        }
        if (all) {
            ok = true;
            break;
        }
        if (__hip_atomic_load(hp.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        if ((uint64_t)wall_clock64() - t0 > hp.limit) {
            __hip_atomic_store(hp.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    if (!ok) return;   // the run is failed; this half's values stand
    const float om1 = __uint_as_float((uint32_t)w[0]), om2 = __uint_as_float((uint32_t)w[2]);
    const float ocv = __uint_as_float((uint32_t)w[3]);
    const int ok1 = (int)(uint32_t)w[1], ock = (int)(uint32_t)w[4];
    // both sides merge the lower half first (the merges are exact, so this only fixes the form)
    if (hp.side == 0) {
        top2_merge(m1, k1, m2, om1, ok1, om2);
        argmax_merge(cv, ck, ocv, ock);
    } else {
        float a1 = om1, a2 = om2, c1 = ocv;
        int ak = ok1, cc = ock;
        top2_merge(a1, ak, a2, m1, k1, m2);
        argmax_merge(c1, cc, cv, ck);
        m1 = a1, k1 = ak, m2 = a2, cv = c1, ck = cc;
    }
}

template <int NT, int NCH, bool FIRST, bool TAIL, bool PAIR>
__device__ __forceinline__ void held_rows(const SweepArgs<float> &a, const int t, const int row0, const int row1,
                                          const int coff, const int ncols, Vec<float>::type (*qs)[NT],
                                          float (*sh_m1)[NT / 64], int (*sh_k1)[NT / 64], float (*sh_m2)[NT / 64],
                                          float (*sh_cv)[NT / 64], int (*sh_ck)[NT / 64], const HeldPair &hp) {
#pragma clang fp contract(off)
    using T = float;
    using V = Vec<float>::type;
    constexpr int VW = 4;
    constexpr int NW = NT / 64;
    // the wave index is wave-uniform: as a scalar it keeps the LDS slots' addresses out of vector registers
    const int tid = threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t ldw = a.ldw;
    const T lam = a.lam, oml = a.oml;
    const T zero = T(0), ninf = neg_inf<T>();
    const int base = tid * VW;
    // this workgroup's columns [coff, coff + ncols): the whole row, or one half of it (PAIR)
    const bool owner = !PAIR || hp.side == 0;   // writes the row's scalars
    __shared__ T st_p[kWin], st_tau[kWin], st_d[kWin];
    __shared__ int st_e[kWin], st_has[kWin];
    __shared__ T shx_m1[2], shx_m2[2];
    __shared__ int shx_k1[2];
    V hs[NCH], hr[NCH];            // this row's s (with the diagonal and the Eq. 2.7 offset) and rho^{t-1}
    V sv = (V)(zero), rv = (V)(zero), av = (V)(zero), bv = (V)(zero);   // the next chunk's operands
    // buffer-resource accesses: a resource per row, the lane's byte offset in one register and the
    // chunk's offset as a scalar, so the chunks cost no address registers (loads past the row's
    // resource return 0, which the ragged tail overrides)
    constexpr int CB = NT * VW * (int)sizeof(T);
    const int voff = tid * 16;
    const int64_t lds_h = a.lds - coff, ldw_h = ldw - coff;   // the resources start at column coff
    const __amdgpu_buffer_rsrc_t rB = row_rsrc(a.B + coff, ldw_h * (int64_t)sizeof(T));
    auto load1 = [&](int row, int c) {
        const __amdgpu_buffer_rsrc_t rS =
            row_rsrc(a.S + (int64_t)row * a.lds + coff, lds_h * (int64_t)sizeof(T));
        const __amdgpu_buffer_rsrc_t rR = row_rsrc(a.R + (int64_t)row * ldw + coff, ldw_h * (int64_t)sizeof(T));
        const __amdgpu_buffer_rsrc_t rA = row_rsrc(a.A + (int64_t)row * ldw + coff, ldw_h * (int64_t)sizeof(T));
        // rho and alpha non-temporal as in the other passes, except in the paired pass, where
        // cached loads measured 3% faster
        sv = buf_load<V, kNT>(rS, voff, c * CB);
        rv = buf_load<V, PAIR ? 0 : kNT>(rR, voff, c * CB);
        av = buf_load<V, PAIR ? 0 : kNT>(rA, voff, c * CB);
        if constexpr (!FIRST) bv = buf_load<V, 0>(rB, voff, c * CB);
        if constexpr (TAIL) {
            if (c * NT * VW + base >= ncols) av = (V)(ninf);   // columns past n never win a maximum
        }
    };
    int buf = 0;
    int chg = 0;
    auto rowof = [&](int k) { return slot_row(k, row0, a.rb, a.row_stride); };
    if (row0 < row1) load1(rowof(row0), 0);
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
                st_d[tid] = a.delta != nullptr ? a.delta[k] : zero;
                st_e[tid] = a.E[k];
            }
            __syncthreads();
        }
        const T p_i = st_p[r];
        const T d_i = st_d[r];
        const bool has_d = a.delta != nullptr;
        const __amdgpu_buffer_rsrc_t rA = row_rsrc(a.A + (int64_t)i * ldw + coff, ldw_h * (int64_t)sizeof(T));
        const __amdgpu_buffer_rsrc_t rR = row_rsrc(a.R + (int64_t)i * ldw + coff, ldw_h * (int64_t)sizeof(T));
        int dcol = i - coff - base;
        T m1 = ninf, m2 = ninf, cv = ninf;
        int k1 = INT_MAX, ck = INT_MAX;
        // phase 1: finish alpha^{t-1} (stored), reduce c/e over alpha + rho and the top two of alpha + s
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + base;
            V sc = sv, ac = av;
            hr[c] = rv;
            const V bc = bv;
            if (c + 1 < NCH) load1(i, c + 1);
            // dcol is made opaque per chunk, so the diagonal masks are formed where they are used
            // rather than all at once and held in scalar registers
            asm volatile("" : "+v"(dcol));
            if (has_d) sc = sc + d_i;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = c * NT * VW + v;
                const bool diag = dcol == j;
                const T sj = diag ? p_i : sc[v];
                sc[v] = sj;
                const T rj = hr[c][v];
                T al = ac[v];
                if constexpr (!FIRST) {
                    // two selects rather than one over two expressions, which the compiler
                    // turns into a branch
                    const T u = bc[v] - (diag ? rj : fmax(zero, rj));
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
            hs[c] = sc;
            if constexpr (!FIRST) buf_store<V, kNT>(ac, rA, voff, c * CB);
            // keep each chunk's memory accesses with its arithmetic (the compiler would otherwise
            // hoist later chunks' accesses and run out of registers)
            asm volatile("" ::: "memory");
        }
        k1 = (k1 == INT_MAX) ? INT_MAX : k1 + coff + base;
        ck = (ck == INT_MAX) ? INT_MAX : ck + coff + base;
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
        // LDS exchange of the wave results (waits for LDS writes only, not for the stores in flight)
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        m1 = sh_m1[buf][0];
        k1 = sh_k1[buf][0];
        m2 = sh_m2[buf][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) top2_merge(m1, k1, m2, sh_m1[buf][w], sh_k1[buf][w], sh_m2[buf][w]);
        if (tid == 0) {
            if constexpr (!FIRST) {
                cv = sh_cv[buf][0];
                ck = sh_ck[buf][0];
                for (int w = 1; w < NW; ++w) argmax_merge(cv, ck, sh_cv[buf][w], sh_ck[buf][w]);
            }
            if constexpr (PAIR) {
                // the whole row's values from the two halves, passed to every thread through LDS
                pair_exchange(hp, i, t, m1, k1, m2, cv, ck);
                shx_m1[buf] = m1;
                shx_k1[buf] = k1;
                shx_m2[buf] = m2;
            }
        }
        if constexpr (PAIR) {
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            m1 = shx_m1[buf];
            k1 = shx_k1[buf];
            m2 = shx_m2[buf];
        }
        if (owner && tid == 0) {
            if constexpr (!FIRST) {
                a.C[i] = cv;
                if (a.phi_down) a.phi_down[i] = m1;
                a.E[i] = ck;
                chg |= (t >= 3 && st_e[r] != ck) ? 1 : 0;
            } else {
                if (a.mrhap && a.phi_down) a.phi_down[i] = m1;
            }
        }
        // phase 2: rho^t from the held row, column partials in LDS
        asm volatile("" : "+v"(dcol));
        const int k1r = k1 - coff - base;
        const T tau_i = st_tau[r];
        const bool has_tau = st_has[r] != 0;
        if (a.tau_store && owner && tid == 0) a.tau_store[i] = has_tau ? tau_i : pos_inf<T>();
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + base;
            if (c + 1 == NCH && ii + 1 < row1) load1(rowof(ii + 1), 0);
            asm volatile("" : "+v"(dcol));
            V out;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = c * NT * VW + v;
                const T m = (j == k1r) ? m2 : m1;
                const T rh = has_tau ? hs[c][v] + fmin(tau_i, -m) : hs[c][v] - m;
                out[v] = lam * hr[c][v] + oml * rh;
            }
            buf_store<V, kNT>(out, rR, voff, c * CB);
            V q = qs[c][tid];
#pragma unroll
            for (int v = 0; v < VW; ++v) q[v] += (dcol == c * NT * VW + v) ? out[v] : fmax(zero, out[v]);
            qs[c][tid] = q;
            asm volatile("" ::: "memory");
        }
    }
    if (chg) atomicOr(&a.ds->changed, 1);
}

template <int NT, int NCH, bool TAIL>
__global__ __launch_bounds__(NT) void sweep_held_kernel(SweepArgs<float> a) {
#pragma clang fp contract(off)
    using V = Vec<float>::type;
    constexpr int VW = 4;
    constexpr int NW = NT / 64;
    __shared__ float sh_m1[2][NW], sh_m2[2][NW], sh_cv[2][NW];
    __shared__ int sh_k1[2][NW], sh_ck[2][NW];
    __shared__ V qs[NCH][NT];
    const DevState *ds = a.ds;
    if (ds->done) return;
    const int t = ds->t + 1;
#pragma unroll
    for (int c = 0; c < NCH; ++c) qs[c][threadIdx.x] = (V)(0.f);
    const int row0 = blockIdx.x * a.rb;
    const int row1 = slots_end(a.rows, a.rb, row0, a.row_stride);
    const HeldPair none{};
    if (t == 1)
        held_rows<NT, NCH, true, TAIL, false>(a, t, row0, row1, 0, a.n, qs, sh_m1, sh_k1, sh_m2, sh_cv, sh_ck, none);
    else
        held_rows<NT, NCH, false, TAIL, false>(a, t, row0, row1, 0, a.n, qs, sh_m1, sh_k1, sh_m2, sh_cv, sh_ck, none);
    float *qrow = a.Qpart + (int64_t)blockIdx.x * a.ldw;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int j0 = c * NT * VW + threadIdx.x * VW;
        if (!TAIL || j0 < a.n) *(V *)(qrow + j0) = qs[c][threadIdx.x];
    }
}

// The paired pass: workgroups b and b + 8 of every 16 form a pair (on the same XCD when the
// workgroups are dealt round-robin to the eight XCDs); the pair's rows are the block of its
// index, side 0 holds columns [0, H) and side 1 columns [H, n).  Every workgroup of the launch
// must be resident at once (the host sizes the grid to the device's capacity).
template <int NT, int NCH, bool TAIL>
__global__ __launch_bounds__(NT) void sweep_pair_kernel(SweepArgs<float> a, PairArgs p) {
#pragma clang fp contract(off)
    using V = Vec<float>::type;
    constexpr int VW = 4;
    constexpr int NW = NT / 64;
    constexpr int H = NT * NCH * VW;
    __shared__ float sh_m1[2][NW], sh_m2[2][NW], sh_cv[2][NW];
    __shared__ int sh_k1[2][NW], sh_ck[2][NW];
    __shared__ V qs[NCH][NT];
    const DevState *ds = a.ds;
    if (ds->done) return;
    const int t = ds->t + 1;
    const int b = blockIdx.x;
    const int side = (b >> 3) & 1, pair = (b >> 4) * 8 + (b & 7);
    const int coff = side * H;
    const int ncols = min(H, a.n - coff);
#pragma unroll
    for (int c = 0; c < NCH; ++c) qs[c][threadIdx.x] = (V)(0.f);
    const int row0 = pair * a.rb;
    const int row1 = slots_end(a.rows, a.rb, row0, a.row_stride);
    HeldPair hp;
    hp.mine = p.slots + ((size_t)pair * 2 + side) * 10;
    hp.theirs = p.slots + ((size_t)pair * 2 + (side ^ 1)) * 10;
    hp.abort = &a.ds->pair_abort;
    hp.limit = p.wait_ticks;
    hp.side = side;
    hp.level = p.level;
    if (t == 1)
        held_rows<NT, NCH, true, TAIL, true>(a, t, row0, row1, coff, ncols, qs, sh_m1, sh_k1, sh_m2, sh_cv, sh_ck, hp);
    else
        held_rows<NT, NCH, false, TAIL, true>(a, t, row0, row1, coff, ncols, qs, sh_m1, sh_k1, sh_m2, sh_cv, sh_ck, hp);
    if (row0 >= a.rows) return;
    float *qrow = a.Qpart + (int64_t)pair * a.ldw + coff;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int j0 = c * NT * VW + threadIdx.x * VW;
        if (!TAIL || j0 < ncols) *(V *)(qrow + j0) = qs[c][threadIdx.x];
    }
}

template <typename T, int NT, bool TAIL>
__global__ __launch_bounds__(NT) void sweep_stream_kernel(SweepArgs<T> a, int nch) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    constexpr int NW = NT / 64;
    constexpr int CB = NT * VW * (int)sizeof(T);
    __shared__ T sh_m1[2][NW], sh_m2[2][NW], sh_cv[2][NW];
    __shared__ int sh_k1[2][NW], sh_ck[2][NW];
    __shared__ V qs[kLdsChunks][NT];
    const DevState *ds = a.ds;
    if (ds->done) return;
    const int t = ds->t + 1;
    const __amdgpu_buffer_rsrc_t rQ = row_rsrc(a.Qpart + (int64_t)blockIdx.x * a.ldw, a.ldw * (int64_t)sizeof(T));
    for (int c = 0; c < nch; ++c) {
        if (c < kLdsChunks)
            qs[c][threadIdx.x] = (V)(T(0));
        else
            buf_store<V, 0>((V)(T(0)), rQ, threadIdx.x * 16, c * CB);
    }
    const int row0 = blockIdx.x * a.rb;
    const int row1 = slots_end(a.rows, a.rb, row0, a.row_stride);
    if constexpr (sizeof(T) == 4) {
        if (t == 1)
            stream_rows<T, NT, true, TAIL>(a, t, row0, row1, nch, qs, rQ, sh_m1, sh_k1, sh_m2, sh_cv, sh_ck);
        else
            stream_rows<T, NT, false, TAIL>(a, t, row0, row1, nch, qs, rQ, sh_m1, sh_k1, sh_m2, sh_cv, sh_ck);
    } else {
        if (t == 1)
            stream_rows_unpipelined<T, NT, true, TAIL>(a, t, row0, row1, nch, qs, rQ, sh_m1, sh_k1, sh_m2, sh_cv,
                                                       sh_ck);
        else
            stream_rows_unpipelined<T, NT, false, TAIL>(a, t, row0, row1, nch, qs, rQ, sh_m1, sh_k1, sh_m2, sh_cv,
                                                        sh_ck);
    }
    for (int c = 0; c < nch && c < kLdsChunks; ++c) buf_store<V, 0>(qs[c][threadIdx.x], rQ, threadIdx.x * 16, c * CB);
}

// Padding columns [n, ldw) of every A row of every level start at -inf.
template <typename T>
__global__ void alpha_pad_kernel(T *A, int64_t rows, int n, int64_t ldw) {
    const int pad = (int)(ldw - n);
    const int64_t total = rows * pad;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = k / pad;
        A[r * ldw + n + (k % pad)] = neg_inf<T>();
    }
}

// Column sums Q_j = sum over workgroups of the partials, in a fixed order (NG = 1:
// strictly in workgroup order, which with one row per workgroup is plain row order);
// then tau^{l+1}_j = c^l_j + Q^l_j (Eq. 2.4, c^l from before this iteration's update),
// and the availability base of the next pass: B^{l-1}_j = c^{l-1}_j + phi^{l-1}_j + Q^{l-1}_j
// (phi^{l-1} was just sent down by this level's row pass), or B^l_j = Q^l_j at the top
// level.  The launch for the top level also advances the iteration counter and applies
// the stop rule (workgroup 0, thread 0).
template <typename T>
struct ColArgs {
    const T *__restrict__ Qpart;
    int64_t ldw;
    int nb, n;
    T *Q;                // Q^l (written)
    const T *C;          // c^l
    T *tau_next;         // tau^{l+1} or nullptr at the top level
    T *B_top;            // B^l = Q^l at the top level, else nullptr
    T *B_down;           // B^{l-1}, nullptr at l = 0
    const T *C_down, *phi_down, *Q_down;
    int last, K;
    DevState *ds;
};

template <typename T, int NG>
__global__ __launch_bounds__(16 * NG) void colsum_kernel(ColArgs<T> a) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    __shared__ V sh[NG][16];
    // After an early stop the row passes do nothing and the shared partial buffer is stale, so
    // the levels below the top keep their sums.  The top level's partials are the last ones
    // written, so its launch (which also applies the stop rule, and is the only one that can
    // set the flag) recomputes the same values.
    if (!a.last && a.ds->done) return;
    // 16 column vectors per workgroup; group g sums partial rows g, g+NG, g+2NG, ... in order
    const int col = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int j0 = (blockIdx.x * 16 + col) * VW;
    const int n = a.n, nb = a.nb;
    // the vectors the sums are combined with were written before this launch: load them first,
    // so that their latency overlaps that of the partials
    V cv = (V)(T(0)), bd = (V)(T(0));
    if (g == 0 && j0 < n) {
        if (a.tau_next != nullptr) cv = *(const V *)(a.C + j0);
        if (a.B_down != nullptr)
            bd = (*(const V *)(a.C_down + j0) + *(const V *)(a.phi_down + j0)) + *(const V *)(a.Q_down + j0);
    }
    V acc = (V)(T(0));
    if (j0 < n) {
        if (NG == 1) {
            // strictly sequential adds; the loads are issued 16 ahead
#pragma unroll 16
            for (int b = 0; b < nb; ++b) acc += *(const V *)(a.Qpart + (int64_t)b * a.ldw + j0);
        } else {
#pragma unroll 4
            for (int b = g; b < nb; b += NG) acc += *(const V *)(a.Qpart + (int64_t)b * a.ldw + j0);
        }
    }
    if (NG > 1) {
        sh[g][col] = acc;
        __syncthreads();
    }
    if (g == 0 && j0 < n) {
        V tot = acc;
#pragma unroll
        for (int k = 1; k < NG; ++k) tot += sh[k][col];
        *(V *)(a.Q + j0) = tot;
        if (a.tau_next != nullptr) *(V *)(a.tau_next + j0) = cv + tot;
        if (a.B_top != nullptr) *(V *)(a.B_top + j0) = tot;
        if (a.B_down != nullptr) *(V *)(a.B_down + j0) = bd;
    }
    if (a.last && blockIdx.x == 0 && threadIdx.x == 0) {
        DevState *ds = a.ds;
        if (!ds->done) {
            const int tcur = ds->t + 1;
            if (tcur >= 2) {
                const int it = tcur - 1;  // label iteration compared during this sweep
                if (it >= 2 && !ds->changed)
                    ds->stable += 1;
                else
                    ds->stable = 0;
                if (a.K > 0 && ds->stable >= a.K) {
                    ds->done = 1;
                    ds->stop_iter = it;
                }
            }
            ds->changed = 0;
            ds->t = tcur;
        }
    }
}

// alpha^{l,t} materialised on the fly from A = alpha^{t-1}, R = rho^t (nothing in the
// iteration state is written).  Optional outputs: labels e^{l,t} (Eq. 2.8), alpha^{l,t},
// c^l = max_j(alpha + rho) (Eq. 2.6) and phi^{l-1} = max_j(alpha + s) (Eq. 2.5).
template <typename T>
struct FinArgs {
    const T *__restrict__ S;
    int64_t lds;
    const T *__restrict__ R;
    const T *__restrict__ A;
    int64_t ldw;
    const T *__restrict__ pref;
    const T *__restrict__ B;
    const int32_t *__restrict__ E;
    int32_t *labels;
    T *alpha_out;
    int64_t lda;
    T *c_out;
    T *phi_out;
    const T *delta;      // Eq. 2.7 row offsets of this level's s, or nullptr
    int n, t;
    int rows;            // rows [0, rows) are the updated ones (one block of a run split by rows)
    T lam, oml;
    DevState *ds;
};

template <typename T>
__global__ __launch_bounds__(256) void finalize_kernel(FinArgs<T> a) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    constexpr int NT = 256, NW = NT / 64;
    __shared__ T sh_m[NW], sh_cv[NW];
    __shared__ int sh_ck[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = a.n;
    const int i = blockIdx.x;
    const bool mat = a.t >= 1;
    const T zero = T(0);
    const T *Srow = a.S + (int64_t)i * a.lds;
    const T *Rrow = a.R + (int64_t)i * a.ldw;
    const T *Arow = a.A + (int64_t)i * a.ldw;
    const T p_i = a.pref[i];
    const bool has_d = a.delta != nullptr;
    const T d_i = has_d ? a.delta[i] : zero;
    T mx = neg_inf<T>(), cv = neg_inf<T>();
    int ck = INT_MAX;
    for (int j0 = tid * VW; j0 < n; j0 += NT * VW) {
        V sv = *(const V *)(Srow + j0);
        if (has_d) sv = sv + d_i;
        const V rv = *(const V *)(Rrow + j0);
        V av = *(const V *)(Arow + j0);
        const V bv = *(const V *)(a.B + j0);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            const int j = j0 + v;
            if (j >= n) continue;
            T al = av[v];
            if (mat) {
                const T ah = (j == i) ? bv[v] - rv[v] : fmin(zero, bv[v] - fmax(zero, rv[v]));
                al = a.lam * al + a.oml * ah;
            }
            av[v] = al;
            const T x = al + rv[v];
            if (x > cv) {
                cv = x;
                ck = j;
            }
            const T y = al + ((j == i) ? p_i : sv[v]);
            mx = fmax(mx, y);
        }
        if (a.alpha_out) {
            T *dst = a.alpha_out + (int64_t)i * a.lda + j0;
#pragma unroll
            for (int v = 0; v < VW; ++v)
                if (j0 + v < n) dst[v] = av[v];
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const T om = __shfl_xor(mx, off, 64);
        const T ocv = __shfl_xor(cv, off, 64);
        const int ock = __shfl_xor(ck, off, 64);
        mx = fmax(mx, om);
        argmax_merge(cv, ck, ocv, ock);
    }
    if (lane == 0) {
        sh_m[wid] = mx;
        sh_cv[wid] = cv;
        sh_ck[wid] = ck;
    }
    __syncthreads();
    if (tid == 0) {
        mx = sh_m[0];
        cv = sh_cv[0];
        ck = sh_ck[0];
        for (int w = 1; w < NW; ++w) {
            mx = fmax(mx, sh_m[w]);
            argmax_merge(cv, ck, sh_cv[w], sh_ck[w]);
        }
        if (a.labels) a.labels[i] = ck;
        if (a.c_out) a.c_out[i] = cv;
        if (a.phi_out) a.phi_out[i] = mx;
        // only the updated rows take part in the stop rule (the others keep their initial labels)
        if (a.E && a.t >= 2 && i < a.rows && a.E[i] != ck) atomicOr(&a.ds->final_changed, 1);
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

int64_t pair_grid(int64_t rows, int64_t rb) {
    const int64_t pairs = (rows + rb - 1) / rb;
    return (pairs + 7) / 8 * 16;   // pairs in groups of eight: workgroups b and b + 8 of each 16
}

int pair_capacity(int threads) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
    if (threads == 512)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sweep_pair_kernel<512, 16, true>, 512, 0);
    else if (threads == 64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sweep_pair_kernel<64, 16, true>, 64, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

bool launch_supported(int threads, int chunks, int elem_size) {
    (void)elem_size;
    switch (chunks) {
        case 1: return threads == 512 || threads == 1024 || threads == 64 || threads == 128 || threads == 256;
        case 2: return threads == 64 || threads == 128 || threads == 256 || threads == 512 || threads == 1024;
        case 4: return threads == 64 || threads == 128 || threads == 256 || threads == 512;
        case 8: return threads == 64 || threads == 128 || threads == 256;
        default: return false;
    }
}

// Shapes compiled: chunks 1 and 2 up to 1024 threads, 4 up to 512, 8 up to 256 (so a
// thread's row slice stays in registers).
#define HAP_DISPATCH_NT_NCH(NTV, NCHV, MACRO)                                                  \
    do {                                                                                       \
        const int _nt = (NTV), _nch = (NCHV);                                                  \
        if (_nch == 1 && _nt == 64) MACRO(64, 1);                                              \
        else if (_nch == 1 && _nt == 128) MACRO(128, 1);                                       \
        else if (_nch == 1 && _nt == 256) MACRO(256, 1);                                       \
        else if (_nch == 1 && _nt == 512) MACRO(512, 1);                                       \
        else if (_nch == 1 && _nt == 1024) MACRO(1024, 1);                                     \
        else if (_nch == 2 && _nt == 64) MACRO(64, 2);                                         \
        else if (_nch == 2 && _nt == 128) MACRO(128, 2);                                       \
        else if (_nch == 2 && _nt == 256) MACRO(256, 2);                                       \
        else if (_nch == 2 && _nt == 512) MACRO(512, 2);                                       \
        else if (_nch == 2 && _nt == 1024) MACRO(1024, 2);                                     \
        else if (_nch == 4 && _nt == 64) MACRO(64, 4);                                         \
        else if (_nch == 4 && _nt == 128) MACRO(128, 4);                                       \
        else if (_nch == 4 && _nt == 256) MACRO(256, 4);                                       \
        else if (_nch == 4 && _nt == 512) MACRO(512, 4);                                       \
        else if (_nch == 8 && _nt == 64) MACRO(64, 8);                                         \
        else if (_nch == 8 && _nt == 128) MACRO(128, 8);                                       \
        else if (_nch == 8 && _nt == 256) MACRO(256, 8);                                       \
        else return hipErrorInvalidValue;                                                      \
    } while (0)

template <typename T, int D>
hipError_t launch_resident(const SweepArgs<T> &a, const Launch &lc, int nb, bool tail, hipStream_t st) {
#define HAP_LAUNCH_SWEEP(NTC, NCHC)                                                                     \
    do {                                                                                                \
        if (tail)                                                                                       \
            hipLaunchKernelGGL((sweep_kernel<T, NTC, NCHC, true, D>), dim3(nb), dim3(NTC), 0, st, a);   \
        else                                                                                            \
            hipLaunchKernelGGL((sweep_kernel<T, NTC, NCHC, false, D>), dim3(nb), dim3(NTC), 0, st, a);  \
    } while (0)
    HAP_DISPATCH_NT_NCH(lc.threads, lc.chunks, HAP_LAUNCH_SWEEP);
#undef HAP_LAUNCH_SWEEP
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep_level(const T *S, int64_t lds, const LevelPtrs<T> &lv, T *phi_down,
                              const T *tau_l, int n, int64_t ldw, double lam, T *Qpart, const Launch &lc,
                              DevState *ds, hipStream_t st, const SweepExtra<T> &ex) {
    const T *X = ex.X;
    const int64_t ldx = ex.ldx;
    const int d = ex.d;
    SweepArgs<T> a;
    a.S = S;
    a.lds = lds;
    a.R = lv.R;
    a.A = lv.A;
    a.ldw = ldw;
    a.pref = lv.pref;
    a.C = lv.C;
    a.phi_down = phi_down;
    a.B = lv.B;
    a.tau = tau_l;
    a.E = lv.E;
    a.Qpart = Qpart;
    a.n = n;
    a.rb = lc.rows_per_block;
    a.rows = ex.rows > 0 ? ex.rows : n;
    a.lam = (T)lam;
    a.oml = (T)(1.0 - lam);
    a.ds = ds;
    a.X = X;
    a.ldx = ldx;
    a.tau_c = ex.tau_c;
    a.tau_q = ex.tau_q;
    a.tau_store = ex.tau_store;
    a.mrhap = ex.mrhap;
    a.delta = ex.delta;
    a.row_stride = row_stride_of(lc, a.rows);
    const int nb = (a.rows + lc.rows_per_block - 1) / lc.rows_per_block;
    const bool tail = (int64_t)lc.threads * lc.chunks * Vec<T>::N != n;
    if (lc.streaming && lc.chunks == 32) {
        // the paired pass: FP32, two workgroups of 512 (or, for tests, 64) threads x 16 chunks
        if constexpr (sizeof(T) == 4) {
            if ((lc.threads != 512 && lc.threads != 64) || ex.pair_slots == nullptr) return hipErrorInvalidValue;
            const int h = lc.threads * 16 * 4;
            if (n <= h || n > 2 * h) return hipErrorInvalidValue;
            const int64_t grid = pair_grid(a.rows, lc.rows_per_block);
            if (grid > pair_capacity(lc.threads)) return hipErrorInvalidValue;
            PairArgs pa{ex.pair_slots, ex.pair_wait, ex.pair_level};
            if (lc.threads == 512) {
                if (tail)
                    hipLaunchKernelGGL((sweep_pair_kernel<512, 16, true>), dim3(grid), dim3(512), 0, st, a, pa);
                else
                    hipLaunchKernelGGL((sweep_pair_kernel<512, 16, false>), dim3(grid), dim3(512), 0, st, a, pa);
            } else {
                if (tail)
                    hipLaunchKernelGGL((sweep_pair_kernel<64, 16, true>), dim3(grid), dim3(64), 0, st, a, pa);
                else
                    hipLaunchKernelGGL((sweep_pair_kernel<64, 16, false>), dim3(grid), dim3(64), 0, st, a, pa);
            }
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (lc.streaming && lc.threads == 512) {
        // the held-row pass: FP32, 512 threads x 16 chunks (n <= 32768)
        if constexpr (sizeof(T) == 4) {
            if (lc.chunks != 16 || n > 512 * 16 * 4) return hipErrorInvalidValue;
            if (tail)
                hipLaunchKernelGGL((sweep_held_kernel<512, 16, true>), dim3(nb), dim3(512), 0, st, a);
            else
                hipLaunchKernelGGL((sweep_held_kernel<512, 16, false>), dim3(nb), dim3(512), 0, st, a);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (lc.streaming) {
        if (lc.threads != 1024 || lc.chunks < 1 || lc.chunks > 16) return hipErrorInvalidValue;
        if (tail)
            hipLaunchKernelGGL((sweep_stream_kernel<T, 1024, true>), dim3(nb), dim3(1024), 0, st, a, lc.chunks);
        else
            hipLaunchKernelGGL((sweep_stream_kernel<T, 1024, false>), dim3(nb), dim3(1024), 0, st, a, lc.chunks);
        return hipGetLastError();
    }
    if (ex.delta != nullptr) return launch_resident<T, -1>(a, lc, nb, tail, st);   // reads S (no points mode)
    if (X == nullptr) return launch_resident<T, 0>(a, lc, nb, tail, st);
    if constexpr (sizeof(T) == 4) {
        if (d == 2) return launch_resident<T, 2>(a, lc, nb, tail, st);
        if (d == 3) return launch_resident<T, 3>(a, lc, nb, tail, st);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_colsum(const T *Qpart, int64_t ldw, int nb, int n, const LevelPtrs<T> &lv,
                         const LevelPtrs<T> *down, T *tau_next, bool top, bool last, int K, bool ordered,
                         DevState *ds, hipStream_t st) {
    constexpr int VW = Vec<T>::N;
    ColArgs<T> a;
    a.Qpart = Qpart;
    a.ldw = ldw;
    a.nb = nb;
    a.n = n;
    a.Q = lv.Q;
    a.C = lv.C;
    a.tau_next = tau_next;
    a.B_top = top ? lv.B : nullptr;
    a.B_down = down ? down->B : nullptr;
    a.C_down = down ? down->C : nullptr;
    a.phi_down = down ? down->phi : nullptr;
    a.Q_down = down ? down->Q : nullptr;
    a.last = last ? 1 : 0;
    a.K = K;
    a.ds = ds;
    const int blocks = (n + 16 * VW - 1) / (16 * VW);
    if (ordered)
        hipLaunchKernelGGL((colsum_kernel<T, 1>), dim3(blocks), dim3(16), 0, st, a);
    else
        hipLaunchKernelGGL((colsum_kernel<T, 64>), dim3(blocks), dim3(16 * 64), 0, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(const T *S, int64_t lds, const LevelPtrs<T> &lv, int n, int64_t ldw, double lam, int t,
                           int32_t *labels_out, T *alpha_out, int64_t lda, T *c_out, T *phi_out, DevState *ds,
                           hipStream_t st, const T *delta, int rows) {
    FinArgs<T> a;
    a.S = S;
    a.lds = lds;
    a.R = lv.R;
    a.A = lv.A;
    a.ldw = ldw;
    a.pref = lv.pref;
    a.B = lv.B;
    a.E = labels_out ? lv.E : nullptr;
    a.labels = labels_out;
    a.alpha_out = alpha_out;
    a.lda = lda;
    a.c_out = c_out;
    a.phi_out = phi_out;
    a.delta = delta;
    a.n = n;
    a.t = t;
    a.rows = rows > 0 ? rows : n;
    a.lam = (T)lam;
    a.oml = (T)(1.0 - lam);
    a.ds = ds;
    hipLaunchKernelGGL((finalize_kernel<T>), dim3(n), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_alpha_pad(T *A, int64_t rows, int n, int64_t ldw, hipStream_t st) {
    if (ldw == n) return hipSuccess;
    const int64_t total = rows * (ldw - n);
    const int grid = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    hipLaunchKernelGGL((alpha_pad_kernel<T>), dim3(grid), dim3(256), 0, st, A, rows, n, ldw);
    return hipGetLastError();
}

#define HAP_INSTANTIATE(T)                                                                                        \
    template hipError_t launch_alpha_pad<T>(T *, int64_t, int, int64_t, hipStream_t);                             \
    template hipError_t launch_sweep_level<T>(const T *, int64_t, const LevelPtrs<T> &, T *, const T *, int,      \
                                              int64_t, double, T *, const Launch &, DevState *, hipStream_t,      \
                                              const SweepExtra<T> &);                                             \
    template hipError_t launch_colsum<T>(const T *, int64_t, int, int, const LevelPtrs<T> &, const LevelPtrs<T> *, \
                                         T *, bool, bool, int, bool, DevState *, hipStream_t);                    \
    template hipError_t launch_finalize<T>(const T *, int64_t, const LevelPtrs<T> &, int, int64_t, double, int,   \
                                           int32_t *, T *, int64_t, T *, T *, DevState *, hipStream_t, const T *, int);
HAP_INSTANTIATE(float)
HAP_INSTANTIATE(double)
#undef HAP_INSTANTIATE

}  // namespace hap
