// Similarity build S = -||x_i - x_j||^2 (Section 2) for gfx950.
//
// HAP_BUILD_DIRECT: sum over coordinates of (x_ik - x_jk)^2, accumulated in FP64
// in coordinate order with separate multiply and add roundings (no contraction),
// negated and rounded once to the output type.  Each 256-thread workgroup owns a
// 64 x 64 output tile; the two 64-point slices of X are staged through LDS in
// chunks of 16 coordinates; every thread owns 4 rows x 4 consecutive columns so a
// wavefront stores 4 rows of 64 contiguous elements.
//
// Optional tie-break noise (FP64 output): s_ij <- s_ij + (rel * |s_ij|) * u_ij for
// i != j, with u_ij = (splitmix64(seed ^ (i*n + j)) >> 11) * 2^-53 and splitmix64(x)
// the first output of a SplitMix64 generator (Steele, Lea and Flood, 2014) started
// at state x.
#include "hap_internal.h"

namespace hap {

namespace {

__device__ __forceinline__ unsigned long long splitmix64_first(unsigned long long x) {
    unsigned long long z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr int kTile = 64;
constexpr int kDk = 16;

template <typename TX, typename TS>
__global__ __launch_bounds__(256) void build_direct_kernel(const TX *__restrict__ X, int n, int d, int64_t ldx,
                                                           TS *__restrict__ S, int64_t lds, double noise_rel,
                                                           unsigned long long seed) {
#pragma clang fp contract(off)
    __shared__ double xi[kTile][kDk + 1];
    __shared__ double xj[kTile][kDk + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.y * kTile, j0 = blockIdx.x * kTile;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;

    for (int k0 = 0; k0 < d; k0 += kDk) {
        for (int e = threadIdx.x; e < kTile * kDk; e += 256) {
            const int r = e / kDk, k = e % kDk;
            const int gi = i0 + r, gj = j0 + r, gk = k0 + k;
            xi[r][k] = (gi < n && gk < d) ? (double)X[(int64_t)gi * ldx + gk] : 0.0;
            xj[r][k] = (gj < n && gk < d) ? (double)X[(int64_t)gj * ldx + gk] : 0.0;
        }
        __syncthreads();
        const int kend = (d - k0) < kDk ? (d - k0) : kDk;
        for (int k = 0; k < kend; ++k) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const double u = xi[ty + 16 * a][k];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double df = u - xj[tx * 4 + b][k];
                    const double sq = df * df;
                    acc[a][b] = acc[a][b] + sq;
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + ty + 16 * a;
        if (i >= n) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = j0 + tx * 4 + b;
            if (j >= n) continue;
            double s = -acc[a][b];
            if (i == j) {
                s = 0.0;
            } else if (noise_rel > 0.0) {
                const unsigned long long ctr = (unsigned long long)i * (unsigned long long)n + (unsigned long long)j;
                const unsigned long long z = splitmix64_first(seed ^ ctr);
                const double u = (double)(z >> 11) * 0x1.0p-53;
                double t = noise_rel * fabs(s);
                t = t * u;
                s = s + t;
            }
            S[(int64_t)i * lds + j] = (TS)s;
        }
    }
}

}  // namespace

hipError_t launch_build(const void *X, int64_t n, int64_t d, int64_t ldx, int x_dtype, void *S, int64_t lds,
                        int s_dtype, int mode, double noise_rel, uint64_t seed, hipStream_t st) {
    if (mode != HAP_BUILD_DIRECT) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + kTile - 1) / kTile), (unsigned)((n + kTile - 1) / kTile));
#define HAP_BD(TX, TS)                                                                                      \
    hipLaunchKernelGGL((build_direct_kernel<TX, TS>), grid, dim3(256), 0, st, (const TX *)X, (int)n, (int)d, \
                       ldx, (TS *)S, lds, noise_rel, (unsigned long long)seed)
    if (x_dtype == HAP_F32 && s_dtype == HAP_F32) HAP_BD(float, float);
    else if (x_dtype == HAP_F32 && s_dtype == HAP_F64) HAP_BD(float, double);
    else if (x_dtype == HAP_F64 && s_dtype == HAP_F32) HAP_BD(double, float);
    else HAP_BD(double, double);
#undef HAP_BD
    return hipGetLastError();
}

}  // namespace hap
