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
// Each workgroup owns a block of consecutive rows and keeps its column partials
// in registers (every thread owns the same columns for every row); the partials
// are summed in a fixed order by the epilogue, so results are deterministic.
#include "hap_internal.h"

#include <climits>

namespace hap {

template <typename T>
struct SweepArgs {
    const T *__restrict__ S;
    int64_t lds;
    T *__restrict__ R;
    T *__restrict__ A;
    int64_t ldw;
    const T *__restrict__ pref;
    T *C;                 // [2][ldw]
    const T *__restrict__ phi;
    T *phi_down;          // phi^{l-1}, nullptr at l = 0
    const T *__restrict__ Q;
    const T *__restrict__ tau;  // nullptr at l = 0 (tau^1 = +inf)
    int32_t *E;
    T *__restrict__ Qpart;
    int n;
    int rb;
    int top;              // level == L-1: B = Q (no c, no phi)
    T lam, oml;
    DevState *ds;
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

template <typename T, bool WITH_C>
__device__ __forceinline__ void wave_reduce(T &m1, int &k1, T &m2, T &cv, int &ck) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const T om1 = __shfl_xor(m1, off, 64);
        const int ok1 = __shfl_xor(k1, off, 64);
        const T om2 = __shfl_xor(m2, off, 64);
        top2_merge(m1, k1, m2, om1, ok1, om2);
        if constexpr (WITH_C) {
            const T ocv = __shfl_xor(cv, off, 64);
            const int ock = __shfl_xor(ck, off, 64);
            argmax_merge(cv, ck, ocv, ock);
        }
    }
}

template <typename T, int NT, int NCH>
struct RowRegs {
    typename Vec<T>::type s[NCH], r[NCH], a[NCH];
};

// Columns j >= n: whole 16-byte vectors past n are not loaded (alpha reads as -inf so they
// never win a maximum); inside the last partial vector the padding columns of A hold -inf
// from initialisation and stay -inf or NaN, which '>' and fmax ignore.  Padding columns of
// R, A and the column partials are never read back as results.
template <typename T, int NT, int NCH>
__device__ __forceinline__ void load_row(const SweepArgs<T> &a, int i, RowRegs<T, NT, NCH> &x) {
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    const T *Srow = a.S + (int64_t)i * a.lds;
    const T *Rrow = a.R + (int64_t)i * a.ldw;
    const T *Arow = a.A + (int64_t)i * a.ldw;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int j0 = c * NT * VW + threadIdx.x * VW;
        if (j0 < a.n) {
            // S streams through once per level: non-temporal, so it does not displace R/A lines
            x.s[c] = __builtin_nontemporal_load((const V *)(Srow + j0));
            x.r[c] = *(const V *)(Rrow + j0);
            x.a[c] = *(const V *)(Arow + j0);
        } else {
            x.s[c] = (V)(T(0));
            x.r[c] = (V)(T(0));
            x.a[c] = (V)(neg_inf<T>());
        }
    }
}

// The rows of one workgroup.  FIRST: iteration 1, alpha is the initial value (nothing to
// finish, c and phi keep their initial 0).  PF: the next row's S, R, A are loaded before the
// current row is reduced, so memory traffic overlaps the reductions and the barrier.
template <typename T, int NT, int NCH, bool FIRST, bool PF>
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
    const int cur = t & 1;
    const bool has_tau = a.tau != nullptr;

    RowRegs<T, NT, NCH> x;
    if (PF) load_row<T, NT, NCH>(a, row0, x);
    int buf = 0;
    for (int i = row0; i < row1; ++i, buf ^= 1) {
        RowRegs<T, NT, NCH> nx;
        if (PF) {
            if (i + 1 < row1) load_row<T, NT, NCH>(a, i + 1, nx);
        } else {
            load_row<T, NT, NCH>(a, i, x);
        }
        T *Rrow = a.R + (int64_t)i * ldw;
        T *Arow = a.A + (int64_t)i * ldw;
        const T p_i = a.pref[i];
        int dcol = i - tid * VW;  // the diagonal sits at chunk c, lane v iff dcol == c*NT*VW + v
        T m1 = ninf, m2 = ninf, cv = ninf;
        int k1 = INT_MAX, ck = INT_MAX;
        // phase 1: finish alpha^{t-1}, reduce c/e over alpha + rho and the top two of alpha + s
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + tid * VW;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = j0 + v;
                const bool diag = dcol == c * NT * VW + v;
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
                if (j0 < n) __builtin_nontemporal_store(x.a[c], (V *)(Arow + j0));
            }
        }
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
                a.C[cur * ldw + i] = cv;
                if (a.phi_down) a.phi_down[i] = m1;
                const int old = a.E[i];
                a.E[i] = ck;
                if (t >= 3 && old != ck) atomicOr(&a.ds->changed, 1);
            }
        }
        // phase 2: rho^t, column partials.  dcol is made opaque so the diagonal masks are
        // recomputed here instead of being kept alive across the barrier.
        asm volatile("" : "+v"(dcol));
        const T tau_i = has_tau ? a.tau[i] : zero;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = c * NT * VW + tid * VW;
            V out;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int j = j0 + v;
                const T m = (j == k1) ? m2 : m1;
                const T rh = has_tau ? x.s[c][v] + fmin(tau_i, -m) : x.s[c][v] - m;
                const T rn = lam * x.r[c][v] + oml * rh;
                out[v] = rn;
                const bool diag = dcol == c * NT * VW + v;
                qv[c][v] += diag ? rn : fmax(zero, rn);
            }
            if (j0 < n) __builtin_nontemporal_store(out, (V *)(Rrow + j0));
        }
        if (PF) x = nx;
    }
}

template <typename T, int NT, int NCH, bool PF>
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
    const int prev = (t & 1) ^ 1;
    const int tid = threadIdx.x;
    const int n = a.n;
    const int64_t ldw = a.ldw;

    // Per-column constants of this pass (the same for every row) and column partials.
    V Bv[NCH], qv[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int j0 = c * NT * VW + tid * VW;
        V bv = (V)(T(0));
        if (!first && j0 < n) {
            const V q = *(const V *)(a.Q + j0);
            if (a.top) {
                bv = q;
            } else {
                const V cc = *(const V *)(a.C + prev * ldw + j0);
                const V pv = *(const V *)(a.phi + j0);
                bv = (cc + pv) + q;
            }
        }
        Bv[c] = bv;
        qv[c] = (V)(T(0));
    }
    const int row0 = blockIdx.x * a.rb;
    const int row1 = min(n, row0 + a.rb);
    if (first)
        sweep_rows<T, NT, NCH, true, PF>(a, t, row0, row1, Bv, qv, sh_m1, sh_k1, sh_m2, sh_cv, sh_ck);
    else
        sweep_rows<T, NT, NCH, false, PF>(a, t, row0, row1, Bv, qv, sh_m1, sh_k1, sh_m2, sh_cv, sh_ck);

    T *qrow = a.Qpart + (int64_t)blockIdx.x * ldw;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int j0 = c * NT * VW + tid * VW;
        if (j0 < n) *(V *)(qrow + j0) = qv[c];
    }
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
// then
// tau^{l+1}_j = c^l_j + Q_j (Eq. 2.4, c^l from before this iteration's update).
// The launch for the top level also advances the iteration counter and applies
// the stop rule (in workgroup 0, thread 0).
template <typename T, int NG>
__global__ __launch_bounds__(16 * NG) void colsum_kernel(const T *__restrict__ Qpart, int64_t ldw, int nb, int n,
                                                         T *__restrict__ Q, const T *__restrict__ C,
                                                         T *__restrict__ tau_next, int last, int K, DevState *ds) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    __shared__ V sh[NG][16];
    // 16 column vectors per workgroup; group g sums partial rows g, g+NG, g+2NG, ... in order
    const int col = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int j0 = (blockIdx.x * 16 + col) * VW;
    V acc = (V)(T(0));
    if (j0 < n) {
        if (NG == 1) {
            // strictly sequential adds; the loads are issued 16 ahead
#pragma unroll 16
            for (int b = 0; b < nb; ++b) acc += *(const V *)(Qpart + (int64_t)b * ldw + j0);
        } else {
#pragma unroll 4
            for (int b = g; b < nb; b += NG) acc += *(const V *)(Qpart + (int64_t)b * ldw + j0);
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
        *(V *)(Q + j0) = tot;
        if (tau_next != nullptr) {
            const int cur = (ds->t + 1) & 1;
            *(V *)(tau_next + j0) = *(const V *)(C + cur * ldw + j0) + tot;
        }
    }
    if (last && blockIdx.x == 0 && threadIdx.x == 0 && !ds->done) {
        const int tcur = ds->t + 1;
        if (tcur >= 2) {
            const int it = tcur - 1;  // label iteration compared during this sweep
            if (it >= 2 && !ds->changed)
                ds->stable += 1;
            else
                ds->stable = 0;
            if (K > 0 && ds->stable >= K) {
                ds->done = 1;
                ds->stop_iter = it;
            }
        }
        ds->changed = 0;
        ds->t = tcur;
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
    const T *__restrict__ C;
    const T *__restrict__ phi;
    const T *__restrict__ Q;
    const int32_t *__restrict__ E;
    int32_t *labels;
    T *alpha_out;
    int64_t lda;
    T *c_out;
    T *phi_out;
    int n, t, top;
    T lam, oml;
    DevState *ds;
};

template <typename T, int NT, int NCH>
__global__ __launch_bounds__(NT) void finalize_kernel(FinArgs<T> a) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    constexpr int NW = NT / 64;
    __shared__ T sh_m[NW], sh_cv[NW];
    __shared__ int sh_ck[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = a.n;
    const int i = blockIdx.x;
    const int cur = a.t & 1;
    const bool mat = a.t >= 1;
    const T zero = T(0);
    const T *Srow = a.S + (int64_t)i * a.lds;
    const T *Rrow = a.R + (int64_t)i * a.ldw;
    const T *Arow = a.A + (int64_t)i * a.ldw;
    const T p_i = a.pref[i];
    T mx = neg_inf<T>(), cv = neg_inf<T>();
    int ck = INT_MAX;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int j0 = c * NT * VW + tid * VW;
        if (j0 >= n) continue;
        const V sv = *(const V *)(Srow + j0);
        const V rv = *(const V *)(Rrow + j0);
        V av = *(const V *)(Arow + j0);
        V bv = *(const V *)(a.Q + j0);
        if (!a.top) bv = (*(const V *)(a.C + cur * a.ldw + j0) + *(const V *)(a.phi + j0)) + bv;
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
        if (a.E && a.t >= 2 && a.E[i] != ck) atomicOr(&a.ds->final_changed, 1);
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

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

template <typename T>
hipError_t launch_sweep_level(const T *S, int64_t lds, const LevelPtrs<T> &lv, T *phi_down,
                              const T *tau_l, int n, int64_t ldw, int level, int levels, double lam,
                              T *Qpart, const Launch &lc, DevState *ds, hipStream_t st) {
    SweepArgs<T> a;
    a.S = S;
    a.lds = lds;
    a.R = lv.R;
    a.A = lv.A;
    a.ldw = ldw;
    a.pref = lv.pref;
    a.C = lv.C;
    a.phi = lv.phi;
    a.phi_down = phi_down;
    a.Q = lv.Q;
    a.tau = tau_l;
    a.E = lv.E;
    a.Qpart = Qpart;
    a.n = n;
    a.rb = lc.rows_per_block;
    a.top = (level == levels - 1);
    a.lam = (T)lam;
    a.oml = (T)(1.0 - lam);
    a.ds = ds;
    const int nb = (n + lc.rows_per_block - 1) / lc.rows_per_block;
#define HAP_LAUNCH_SWEEP(NTC, NCHC)                                                        \
    do {                                                                                   \
        if (lc.prefetch)                                                                   \
            hipLaunchKernelGGL((sweep_kernel<T, NTC, NCHC, true>), dim3(nb), dim3(NTC), 0, st, a); \
        else                                                                               \
            hipLaunchKernelGGL((sweep_kernel<T, NTC, NCHC, false>), dim3(nb), dim3(NTC), 0, st, a); \
    } while (0)
    HAP_DISPATCH_NT_NCH(lc.threads, lc.chunks, HAP_LAUNCH_SWEEP);
#undef HAP_LAUNCH_SWEEP
    return hipGetLastError();
}

template <typename T>
hipError_t launch_colsum(const T *Qpart, int64_t ldw, int nb, int n, const LevelPtrs<T> &lv,
                         T *tau_next, bool last, int K, bool ordered, DevState *ds, hipStream_t st) {
    constexpr int VW = Vec<T>::N;
    const int blocks = (n + 16 * VW - 1) / (16 * VW);
    if (ordered)
        hipLaunchKernelGGL((colsum_kernel<T, 1>), dim3(blocks), dim3(16), 0, st, Qpart, ldw, nb, n, lv.Q, lv.C,
                           tau_next, last ? 1 : 0, K, ds);
    else
        hipLaunchKernelGGL((colsum_kernel<T, 64>), dim3(blocks), dim3(16 * 64), 0, st, Qpart, ldw, nb, n, lv.Q,
                           lv.C, tau_next, last ? 1 : 0, K, ds);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(const T *S, int64_t lds, const LevelPtrs<T> &lv, int n, int64_t ldw,
                           int level, int levels, double lam, int t, const Launch &lc,
                           int32_t *labels_out, T *alpha_out, int64_t lda, T *c_out, T *phi_out,
                           DevState *ds, hipStream_t st) {
    FinArgs<T> a;
    a.S = S;
    a.lds = lds;
    a.R = lv.R;
    a.A = lv.A;
    a.ldw = ldw;
    a.pref = lv.pref;
    a.C = lv.C;
    a.phi = lv.phi;
    a.Q = lv.Q;
    a.E = labels_out ? lv.E : nullptr;
    a.labels = labels_out;
    a.alpha_out = alpha_out;
    a.lda = lda;
    a.c_out = c_out;
    a.phi_out = phi_out;
    a.n = n;
    a.t = t;
    a.top = (level == levels - 1);
    a.lam = (T)lam;
    a.oml = (T)(1.0 - lam);
    a.ds = ds;
#define HAP_LAUNCH_FIN(NTC, NCHC) \
    hipLaunchKernelGGL((finalize_kernel<T, NTC, NCHC>), dim3(n), dim3(NTC), 0, st, a)
    HAP_DISPATCH_NT_NCH(lc.threads, lc.chunks, HAP_LAUNCH_FIN);
#undef HAP_LAUNCH_FIN
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
template hipError_t launch_alpha_pad<float>(float *, int64_t, int, int64_t, hipStream_t);
template hipError_t launch_alpha_pad<double>(double *, int64_t, int, int64_t, hipStream_t);

template hipError_t launch_sweep_level<float>(const float *, int64_t, const LevelPtrs<float> &, float *,
                                              const float *, int, int64_t, int, int, double, float *,
                                              const Launch &, DevState *, hipStream_t);
template hipError_t launch_sweep_level<double>(const double *, int64_t, const LevelPtrs<double> &, double *,
                                               const double *, int, int64_t, int, int, double, double *,
                                               const Launch &, DevState *, hipStream_t);
template hipError_t launch_colsum<float>(const float *, int64_t, int, int, const LevelPtrs<float> &, float *,
                                         bool, int, bool, DevState *, hipStream_t);
template hipError_t launch_colsum<double>(const double *, int64_t, int, int, const LevelPtrs<double> &,
                                          double *, bool, int, bool, DevState *, hipStream_t);
template hipError_t launch_finalize<float>(const float *, int64_t, const LevelPtrs<float> &, int, int64_t, int,
                                           int, double, int, const Launch &, int32_t *, float *, int64_t,
                                           float *, float *, DevState *, hipStream_t);
template hipError_t launch_finalize<double>(const double *, int64_t, const LevelPtrs<double> &, int, int64_t,
                                            int, int, double, int, const Launch &, int32_t *, double *,
                                            int64_t, double *, double *, DevState *, hipStream_t);

}  // namespace hap
