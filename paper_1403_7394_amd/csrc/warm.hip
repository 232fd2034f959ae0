// Learned warm start: per-point features of S, training targets of a finished run, and the
// warm initial availabilities (Eq. 2.2-2.3 evaluated at rho = 0 with a predicted base).
//
// Features of point i (HAP_WARM_FEATURES = 32 floats; a = |p_i|, p the level-1 preference):
//   [0,16)  the 16 largest off-diagonal s_ij of row i, descending (ties: lower j first), / a;
//           rows with fewer than 16 off-diagonal entries repeat the smallest one
//   16      p_i / a
//   17      #{j != i : s_ij > p_i} / (n - 1)
//   18      mean of the off-diagonal s_ij, / a
//   19      log(1 + #{j != i : s_ij > p_i}) / 10
//   20 + m log(1 + D_m(i)) / 10, D_m(i) = sum_{j != i} max(0, s_ij - 2^-m p_i) / a, m = 0..5
//   26 + m (D_m(i) - M_m(i)) / max(D_m(i), M_m(i)) (0 when both are 0), M_m(i) the largest
//           D_m over the 16 neighbours of the first block (all other points when n - 1 < 16)
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "hap_internal.h"

namespace hap {

namespace {

constexpr int kTop = 16;
constexpr int kScales = 6;

// One wave per row, four rows per workgroup.  Each lane keeps the top 16 (value, column) of
// its columns j = lane, lane + 64, ... (visited in increasing j, so a later equal value goes
// behind an earlier one); the wave then extracts the row's top 16 in 16 rounds of a
// (value descending, column ascending) maximum.
template <typename T>
__global__ __launch_bounds__(256) void warm_features_kernel(const T *__restrict__ S, int64_t lds,
                                                            const T *__restrict__ pref, int n, float *__restrict__ F,
                                                            int64_t ldf, int32_t *__restrict__ nbr,
                                                            double *__restrict__ Dout) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;   // the whole wave leaves; no workgroup barrier below
    const T *row = S + (int64_t)i * lds;
    const T p = pref[i];
    const double pd = (double)p, a = fabs(pd);
    const T ninf = neg_inf<T>();
    T tv[kTop];
    int ti[kTop];
#pragma unroll
    for (int k = 0; k < kTop; ++k) {
        tv[k] = ninf;
        ti[k] = INT_MAX;
    }
    int cnt = 0;
    double sum = 0.0;
    double D[kScales];
#pragma unroll
    for (int m = 0; m < kScales; ++m) D[m] = 0.0;
    for (int j = lane; j < n; j += 64) {
        if (j == i) continue;
        const T v = row[j];
        if (v > tv[kTop - 1]) {
#pragma unroll
            for (int k = kTop - 1; k > 0; --k) {
                const bool up = v > tv[k - 1];
                const bool here = !up && v > tv[k];
                tv[k] = up ? tv[k - 1] : (here ? v : tv[k]);
                ti[k] = up ? ti[k - 1] : (here ? j : ti[k]);
            }
            if (v > tv[0]) {
                tv[0] = v;
                ti[0] = j;
            }
        }
        cnt += v > p ? 1 : 0;
        const double vd = (double)v;
        sum += vd;
#pragma unroll
        for (int m = 0; m < kScales; ++m) {
            const double thr = pd * (1.0 / (double)(1 << m));
            D[m] += fmax(0.0, vd - thr);
        }
    }
    // row totals (fixed butterfly order)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        cnt += __shfl_xor(cnt, off, 64);
        sum += __shfl_xor(sum, off, 64);
#pragma unroll
        for (int m = 0; m < kScales; ++m) D[m] += __shfl_xor(D[m], off, 64);
    }
    float *Fi = F + (int64_t)i * ldf;
    int32_t *Ni = nbr + (int64_t)i * kTop;
    // top 16 of the row
    const int avail = n - 1;
    T last_v = ninf;
    int last_j = 0;
    for (int r = 0; r < kTop; ++r) {
        T bv = tv[0];
        int bj = ti[0];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const T ov = __shfl_xor(bv, off, 64);
            const int oj = __shfl_xor(bj, off, 64);
            const bool take = ov > bv || (ov == bv && oj < bj);
            bv = take ? ov : bv;
            bj = take ? oj : bj;
        }
        if (r < avail) {
            if (ti[0] == bj) {   // the owner of the extracted entry advances its list
#pragma unroll
                for (int k = 0; k < kTop - 1; ++k) {
                    tv[k] = tv[k + 1];
                    ti[k] = ti[k + 1];
                }
                tv[kTop - 1] = ninf;
                ti[kTop - 1] = INT_MAX;
            }
            last_v = bv;
            last_j = bj;
        }
        if (lane == 0) {
            Fi[r] = (float)((double)last_v / a);
            Ni[r] = last_j;
        }
    }
    if (lane == 0) {
        Fi[16] = (float)(pd / a);
        Fi[17] = (float)((double)cnt / (double)avail);
        Fi[18] = (float)((sum / (double)avail) / a);
        Fi[19] = (float)(log1p((double)cnt) / 10.0);
        double *Di = Dout + (int64_t)i * kScales;
#pragma unroll
        for (int m = 0; m < kScales; ++m) {
            const double dm = D[m] / a;
            Di[m] = dm;
            Fi[20 + m] = (float)(log1p(dm) / 10.0);
        }
    }
}

// Neighbourhood comparison of the soft counts: one thread per point.
__global__ __launch_bounds__(256) void warm_local_kernel(int n, const int32_t *__restrict__ nbr,
                                                         const double *__restrict__ D, float *__restrict__ F,
                                                         int64_t ldf) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int cnt = n - 1 < kTop ? n - 1 : kTop;
    double M[kScales];
#pragma unroll
    for (int m = 0; m < kScales; ++m) M[m] = 0.0;
    for (int r = 0; r < cnt; ++r) {
        const int j = nbr[(int64_t)i * kTop + r];
#pragma unroll
        for (int m = 0; m < kScales; ++m) M[m] = fmax(M[m], D[(int64_t)j * kScales + m]);
    }
#pragma unroll
    for (int m = 0; m < kScales; ++m) {
        const double d = D[(int64_t)i * kScales + m];
        const double top = fmax(d, M[m]);
        F[(int64_t)i * ldf + 26 + m] = top > 0.0 ? (float)((d - M[m]) / top) : 0.0f;
    }
}

// Targets g((alpha^t_jj + rho^t_jj) / |p_j|), g(v) = sign(v) |v| / (sqrt(1 + |v|) + 1), where
// alpha^t finishes the damped availability update of the last sweep (as its next row pass
// would) when t >= 1.
template <typename T>
__global__ __launch_bounds__(256) void warm_targets_kernel(const T *__restrict__ R, const T *__restrict__ A,
                                                           const T *__restrict__ B, const T *__restrict__ pref, int n,
                                                           int64_t ldw, T lam, T oml, int t, float *__restrict__ out,
                                                           int64_t ldo) {
#pragma clang fp contract(off)
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const T r = R[(int64_t)j * ldw + j];
    T al = A[(int64_t)j * ldw + j];
    if (t >= 1) al = lam * al + oml * (B[j] - r);
    const double v = ((double)al + (double)r) / fabs((double)pref[j]);
    const double av = fabs(v);
    const double g = av / (sqrt(1.0 + av) + 1.0);
    out[(int64_t)j * ldo] = (float)(v < 0.0 ? -g : g);
}

// Bases B_j = sign(y) |y| (|y| + 2) |p_j| of the network outputs of one level.
template <typename T>
__global__ __launch_bounds__(256) void warm_bases_kernel(const float *__restrict__ Y, int64_t ldy,
                                                         const T *__restrict__ pref, int n, T *__restrict__ bases) {
#pragma clang fp contract(off)
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double y = (double)Y[(int64_t)j * ldy];
    const double ay = fabs(y);
    const double g = ay * (ay + 2.0);
    const double b = (y < 0.0 ? -g : g) * fabs((double)pref[j]);
    bases[j] = (T)b;
}

// alpha_ij = min(0, B_j) (i != j), alpha_jj = B_j with B_j = bases[j * stride]; padding
// columns -inf.
template <typename T>
__global__ __launch_bounds__(256) void warm_fill_kernel(T *__restrict__ A, int n, int64_t ldw,
                                                        const T *__restrict__ bases, int64_t stride) {
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    const int64_t per_row = ldw / VW;
    const int64_t total = (int64_t)n * per_row;
    const T zero = T(0), ninf = neg_inf<T>();
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / per_row;
        const int j0 = (int)((e % per_row) * VW);
        V out;
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            const int j = j0 + v;
            T x = ninf;
            if (j < n) {
                const T b = bases[(int64_t)j * stride];
                x = (j == i) ? b : fmin(zero, b);
            }
            out[v] = x;
        }
        *(V *)(A + i * ldw + j0) = out;
    }
}

}  // namespace

size_t warm_feature_scratch_bytes(int64_t n) { return (size_t)n * (kTop * sizeof(int32_t) + kScales * sizeof(double)); }

template <typename T>
hipError_t launch_warm_features(const T *S, int64_t lds, const T *pref, int n, float *F, int64_t ldf, void *scratch,
                                hipStream_t st) {
    if (n < 2) return hipErrorInvalidValue;
    double *D = (double *)scratch;
    int32_t *nbr = (int32_t *)((char *)scratch + (size_t)n * kScales * sizeof(double));
    hipLaunchKernelGGL((warm_features_kernel<T>), dim3((n + 3) / 4), dim3(256), 0, st, S, lds, pref, n, F, ldf, nbr, D);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(warm_local_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, nbr, D, F, ldf);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_warm_targets(const LevelPtrs<T> &lv, int n, int64_t ldw, double lam, int t, float *out, int64_t ldo,
                               hipStream_t st) {
    hipLaunchKernelGGL((warm_targets_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, st, lv.R, lv.A, lv.B, lv.pref, n,
                       ldw, (T)lam, (T)(1.0 - lam), t, out, ldo);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_warm_alpha(const LevelPtrs<T> &lv, int n, int64_t ldw, const float *Y, int64_t ldy, int col,
                             T *bases_scratch, hipStream_t st) {
    hipLaunchKernelGGL((warm_bases_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, st, Y + col, ldy, lv.pref, n,
                       bases_scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_warm_fill<T>(lv, n, ldw, bases_scratch, 1, st);
}

template <typename T>
hipError_t launch_warm_fill(const LevelPtrs<T> &lv, int n, int64_t ldw, const T *bases, int64_t stride,
                            hipStream_t st) {
    const int64_t total = (int64_t)n * (ldw / Vec<T>::N);
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL((warm_fill_kernel<T>), dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), 0, st, lv.A,
                       n, ldw, bases, stride);
    return hipGetLastError();
}

#define HAP_WARM_INSTANTIATE(T)                                                                                   \
    template hipError_t launch_warm_features<T>(const T *, int64_t, const T *, int, float *, int64_t, void *,      \
                                                hipStream_t);                                                      \
    template hipError_t launch_warm_targets<T>(const LevelPtrs<T> &, int, int64_t, double, int, float *, int64_t,  \
                                               hipStream_t);                                                       \
    template hipError_t launch_warm_alpha<T>(const LevelPtrs<T> &, int, int64_t, const float *, int64_t, int, T *, \
                                             hipStream_t);                                                         \
    template hipError_t launch_warm_fill<T>(const LevelPtrs<T> &, int, int64_t, const T *, int64_t, hipStream_t);
HAP_WARM_INSTANTIATE(float)
HAP_WARM_INSTANTIATE(double)

}  // namespace hap
