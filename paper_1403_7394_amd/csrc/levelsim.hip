// Optional level-wise similarity update (Eq. 2.7, the optional step of Algorithm 1).
//
// The maximum in Eq. 2.7 runs over j != i and leaves one number per row, so the update is a
// row offset of the next level's off-diagonal similarity:
//     s^{l+1}_ij = s_ij + delta^{l+1}_i (j != i),   s^{l+1}_jj = p^{l+1}_j,
//     delta^{l+1}_i = delta^l_i + kappa * max_{j != i}(alpha^l_ij + rho^l_ij),   delta^1 = 0,
// evaluated as the last step of level l in every iteration, from that iteration's alpha^l and
// rho^l.  The row passes add delta_i to the s values they read; no N^2 matrix is stored.
//
// The row pass of iteration t finishes alpha^{t-1} and produces rho^t, so alpha^{l,t} (needed
// here) exists only after the column sums of rho^{l,t}, and its base
// B^{l,t}_j = (c^{l,t-1}_j + phi^{l,t-1}_j) + Q^{l,t}_j needs phi^{l,t-1} = max_k(alpha^{l+1,t-1}_ik
// + s^{l+1,t-1}_ik), which the row pass of level l+1 in iteration t would only produce after it
// has used delta^{l+1,t}.  Two row-parallel passes between the column sums of level l and the
// row pass of level l+1 resolve this (nothing is written to R or A):
//   level_phi_kernel    reads S, R^{l+1}, A^{l+1}, B^{l+1}: phi^l with the offsets of t-1
//   level_base_kernel   forms the availability base B^{l,t} = (c^l + phi^l) + Q^l once (the
//                       column sums of level l+1 write the same vector again later)
//   level_delta_kernel  reads R^l, A^l and B^l: delta^{l+1} of t
// The row pass of level l+1 then leaves phi^l alone.  Both passes are memory-bound streams
// (3 and 2 N^2 reads); one workgroup per row, rows independent, rows streamed non-temporally
// with two chunks per loop trip (7.1 TB/s for the phi pass at 8192 points).
#include "hap_internal.h"

namespace hap {

namespace {

template <typename T>
struct LevelArgs {
    const T *__restrict__ S;
    int64_t lds;
    const T *__restrict__ R;
    const T *__restrict__ A;
    int64_t ldw;
    const T *__restrict__ pref;
    const T *__restrict__ B;       // phi pass: B^{l+1} of iteration t-1; delta pass: B^l of t
    const T *__restrict__ C;       // base pass: c^l, phi^l, Q^l
    const T *__restrict__ phi;
    const T *__restrict__ Q;
    T *B_out;                      // base pass: B^l
    const T *__restrict__ delta_in;   // phi pass: delta^{l+1}; delta pass: delta^l
    T *out;                        // phi pass: phi^l; delta pass: delta^{l+1}
    int n;
    T lam, oml, kappa;
    const DevState *ds;
};

constexpr int kThreads = 256;

// Block-wide maximum of one value per thread (every thread gets the result).
template <typename T>
__device__ __forceinline__ T block_max(T v, T *sh) {
    constexpr int NW = kThreads / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    T m = sh[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) m = fmax(m, sh[w]);
    return m;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void level_phi_kernel(LevelArgs<T> a) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    __shared__ T sh[kThreads / 64];
    const DevState *ds = a.ds;
    if (ds->done) return;
    if (ds->t + 1 == 1) return;   // iteration 1 reads phi^l = 0, its initial value
    const int i = blockIdx.x, n = a.n;
    const T zero = T(0);
    const T *Srow = a.S + (int64_t)i * a.lds;
    const T *Rrow = a.R + (int64_t)i * a.ldw;
    const T *Arow = a.A + (int64_t)i * a.ldw;
    const T p_i = a.pref[i];
    const T d_i = a.delta_in[i];
    T mx = neg_inf<T>();
#pragma unroll 2
    for (int j0 = threadIdx.x * VW; j0 < n; j0 += kThreads * VW) {
        const V sv = __builtin_nontemporal_load((const V *)(Srow + j0));
        const V rv = __builtin_nontemporal_load((const V *)(Rrow + j0));
        const V av = __builtin_nontemporal_load((const V *)(Arow + j0));
        const V bv = *(const V *)(a.B + j0);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            const int j = j0 + v;
            if (j >= n) continue;
            const T ah = (j == i) ? bv[v] - rv[v] : fmin(zero, bv[v] - fmax(zero, rv[v]));
            const T al = a.lam * av[v] + a.oml * ah;
            const T sj = (j == i) ? p_i : sv[v] + d_i;
            mx = fmax(mx, al + sj);
        }
    }
    mx = block_max(mx, sh);
    if (threadIdx.x == 0) a.out[i] = mx;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void level_delta_kernel(LevelArgs<T> a) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    __shared__ T sh[kThreads / 64];
    const DevState *ds = a.ds;
    if (ds->done) return;
    const int i = blockIdx.x, n = a.n;
    const T zero = T(0);
    const T *Rrow = a.R + (int64_t)i * a.ldw;
    const T *Arow = a.A + (int64_t)i * a.ldw;
    T mx = neg_inf<T>();
#pragma unroll 2
    for (int j0 = threadIdx.x * VW; j0 < n; j0 += kThreads * VW) {
        const V rv = __builtin_nontemporal_load((const V *)(Rrow + j0));
        const V av = __builtin_nontemporal_load((const V *)(Arow + j0));
        const V bv = *(const V *)(a.B + j0);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            const int j = j0 + v;
            if (j >= n || j == i) continue;
            const T ah = fmin(zero, bv[v] - fmax(zero, rv[v]));
            const T al = a.lam * av[v] + a.oml * ah;
            mx = fmax(mx, al + rv[v]);
        }
    }
    mx = block_max(mx, sh);
    if (threadIdx.x == 0) a.out[i] = a.delta_in[i] + a.kappa * mx;
}

// B^l_j = (c^l_j + phi^l_j) + Q^l_j, in the order the column-sum kernel uses.
template <typename T>
__global__ __launch_bounds__(kThreads) void level_base_kernel(LevelArgs<T> a) {
#pragma clang fp contract(off)
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    if (a.ds->done) return;
    const int j0 = (blockIdx.x * kThreads + threadIdx.x) * VW;
    if (j0 < a.n)
        *(V *)(a.B_out + j0) = (*(const V *)(a.C + j0) + *(const V *)(a.phi + j0)) + *(const V *)(a.Q + j0);
}

}  // namespace

template <typename T>
hipError_t launch_level_phi(const T *S, int64_t lds, const LevelPtrs<T> &up, T *phi_out, int n, int64_t ldw,
                            double lam, const DevState *ds, hipStream_t st) {
    LevelArgs<T> a{};
    a.S = S;
    a.lds = lds;
    a.R = up.R;
    a.A = up.A;
    a.ldw = ldw;
    a.pref = up.pref;
    a.B = up.B;
    a.delta_in = up.delta;
    a.out = phi_out;
    a.n = n;
    a.lam = (T)lam;
    a.oml = (T)(1.0 - lam);
    a.ds = ds;
    hipLaunchKernelGGL((level_phi_kernel<T>), dim3(n), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_level_delta(const LevelPtrs<T> &lv, T *delta_next, int n, int64_t ldw, double lam, double kappa,
                              const DevState *ds, hipStream_t st) {
    LevelArgs<T> a{};
    a.C = lv.C;
    a.phi = lv.phi;
    a.Q = lv.Q;
    a.B_out = lv.B;
    a.n = n;
    a.ds = ds;
    constexpr int per_block = kThreads * Vec<T>::N;
    hipLaunchKernelGGL((level_base_kernel<T>), dim3((n + per_block - 1) / per_block), dim3(kThreads), 0, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    a.R = lv.R;
    a.A = lv.A;
    a.ldw = ldw;
    a.B = lv.B;
    a.delta_in = lv.delta;
    a.out = delta_next;
    a.n = n;
    a.lam = (T)lam;
    a.oml = (T)(1.0 - lam);
    a.kappa = (T)kappa;
    a.ds = ds;
    hipLaunchKernelGGL((level_delta_kernel<T>), dim3(n), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

#define HAP_INSTANTIATE(T)                                                                                      \
    template hipError_t launch_level_phi<T>(const T *, int64_t, const LevelPtrs<T> &, T *, int, int64_t, double, \
                                            const DevState *, hipStream_t);                                     \
    template hipError_t launch_level_delta<T>(const LevelPtrs<T> &, T *, int, int64_t, double, double,          \
                                              const DevState *, hipStream_t);
HAP_INSTANTIATE(float)
HAP_INSTANTIATE(double)
#undef HAP_INSTANTIATE

}  // namespace hap
