// Similarity build S = -||x_i - x_j||^2 (Section 2) for gfx950: a direct FP64-accumulated
// form on the vector ALUs and Gram-matrix forms on the matrix cores (MFMA).
//
// HAP_BUILD_DIRECT: sum over coordinates of (x_ik - x_jk)^2, accumulated in FP64
// in coordinate order with separate multiply and add roundings (no contraction),
// negated and rounded once to the output type.  HAP_BUILD_DIRECT_L2 takes the FP64
// square root of the sum before negating (the negative Euclidean distance).  Each 256-thread workgroup owns a
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

template <typename TX, typename TS, bool L2>
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
            double s = L2 ? -sqrt(acc[a][b]) : -acc[a][b];
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

// ---------------------------------------------------------------------------
// Gram-matrix builds on MFMA: S_ij = min(0, -((n_i + n_j) - 2 g_ij)), g = X X^T, S_ii = 0.
// n_i is the squared norm of the operand the matrix cores see (x itself for FP32/FP64,
// bf16(x) for BF16, hi + lo for BF16x3), summed in FP64, so that the diagonal cancels.
// The clamp keeps S <= 0 where cancellation leaves a tiny positive value.
//
// Both operands are rows of X: the A fragment of a lane is row (l%16) of the row block, the
// B fragment row (l%16) of the column block, with the same k slots, so the k order inside a
// fragment does not matter.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// float -> bf16, round to nearest even (finite inputs)
__device__ __forceinline__ __bf16 to_bf16(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    const unsigned short h = (unsigned short)(u >> 16);
    return __builtin_bit_cast(__bf16, h);
}
__device__ __forceinline__ float from_bf16(__bf16 h) {
    return __uint_as_float(((unsigned int)__builtin_bit_cast(unsigned short, h)) << 16);
}

enum { kModeF32 = 0, kModeBF16 = 1, kModeBF16x3 = 2 };

template <int MODE>
__global__ __launch_bounds__(256) void norms_kernel(const float *__restrict__ X, int n, int d, int64_t ldx,
                                                    float *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        const float x = X[(int64_t)i * ldx + k];
        if (MODE == kModeF32) {
            acc += (double)x * (double)x;
        } else if (MODE == kModeBF16) {
            const double h = (double)from_bf16(to_bf16(x));
            acc += h * h;
        } else {
            const float hf = from_bf16(to_bf16(x));
            const double h = (double)hf, lo = (double)from_bf16(to_bf16(x - hf));
            acc += h * h + 2.0 * h * lo;   // what hi.hi + hi.lo + lo.hi gives on the diagonal
        }
    }
    out[i] = (float)acc;
}

__global__ __launch_bounds__(256) void norms_kernel_f64(const double *__restrict__ X, int n, int d, int64_t ldx,
                                                        double *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        const double x = X[(int64_t)i * ldx + k];
        acc += x * x;
    }
    out[i] = acc;
}

// Each workgroup owns a 128 x 128 tile of S; its four waves own 64 x 64 quarters as 4 x 4 MFMA
// blocks.  The two 128-point slabs of X are staged through LDS in chunks of kKc coordinates
// with 16-byte loads issued all at once (so a chunk costs one memory latency, not one per
// k step), zero-filled past n and d; fragments are then read from LDS.  The same LDS holds
// the output tile for the epilogue.
constexpr int kTs = 128 + 4;          // padded LDS row of the output tile (64 rows at a time)
// Coordinates per staged chunk: 32 (36 KB of LDS, four workgroups per CU) for the FP32 and
// BF16 forms; BF16x3 needs more registers for its split operands, so it keeps fewer
// workgroups per CU and stages 64 coordinates at a time (fewer barriers).
template <int MODE> constexpr int build_kc() { return MODE == kModeBF16x3 ? 64 : 32; }
template <int MODE> constexpr int build_smem_floats() {
    // staged slabs, or the output rows of one epilogue pass (128 rows for BF16x3, else 64)
    return (2 * 128 * (build_kc<MODE>() + 4) > (MODE == kModeBF16x3 ? 128 : 64) * kTs)
               ? 2 * 128 * (build_kc<MODE>() + 4)
               : (MODE == kModeBF16x3 ? 128 : 64) * kTs;
}
template <int MODE> constexpr int build_min_waves() { return MODE == kModeBF16x3 ? 1 : 4; }

// FP32 and BF16 forms: a register budget of four waves per SIMD (128); with 36 KB of LDS per
// workgroup several workgroups share a CU, so one workgroup's epilogue stores overlap
// another's staging loads.
template <int MODE>
__global__ __launch_bounds__(256, (build_min_waves<MODE>())) void build_mfma_f32_kernel(const float *__restrict__ X, int n, int d, int64_t ldx,
                                                             const float *__restrict__ norms, float *__restrict__ S,
                                                             int64_t lds) {
#pragma clang fp contract(off)
    constexpr int kKc = build_kc<MODE>();
    constexpr int kXs = kKc + 4;          // padded LDS row of a staged slab
    __shared__ float smem[build_smem_floats<MODE>()];
    float(*xs)[128][kXs] = reinterpret_cast<float(*)[128][kXs]>(smem);   // [0]: rows i, [1]: rows j
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lg = lane >> 4;
    const int bi = blockIdx.y * 128, bj = blockIdx.x * 128;
    const int wi = (wave >> 1) * 64, wj = (wave & 1) * 64;
    const bool vec_x = ((ldx & 3) == 0) && ((((uintptr_t)X) & 15) == 0);
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f32x4)(0.f);

    for (int k0 = 0; k0 < d; k0 += kKc) {
        // stage both slabs: 2 x 128 rows x kKc coordinates, 16 bytes per access
        for (int e = tid; e < 2 * 128 * (kKc / 4); e += 256) {
            const int m = e / (128 * (kKc / 4));
            const int rem = e % (128 * (kKc / 4));
            const int r = rem / (kKc / 4), c4 = rem % (kKc / 4);
            const int g = (m == 0 ? bi : bj) + r;
            const int k = k0 + 4 * c4;
            f32x4 v = (f32x4)(0.f);
            if (g < n) {
                const float *src = X + (int64_t)g * ldx + k;
                if (vec_x && k + 3 < d) {
                    v = *(const f32x4 *)src;
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = (k + q < d) ? src[q] : 0.f;
                }
            }
            *(f32x4 *)&xs[m][r][4 * c4] = v;   // rows of kXs floats keep 16-byte alignment
        }
        __syncthreads();
        const int kc = (d - k0) < kKc ? (d - k0) : kKc;
        if (MODE == kModeF32) {
            for (int kk = 0; kk < kc; kk += 4) {
                float fa[4], fb[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    fa[q] = xs[0][wi + 16 * q + lr][kk + lg];
                    fb[q] = xs[1][wj + 16 * q + lr][kk + lg];
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[b], acc[a][b], 0, 0, 0);
            }
        } else if (MODE == kModeBF16) {
            // B fragments for the whole k step, A fragments one block row at a time (fewer
            // live registers)
            for (int kk = 0; kk < kc; kk += 32) {
                bf16x8 hb[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float *pb = &xs[1][wj + 16 * q + lr][kk + 8 * lg];
#pragma unroll
                    for (int e = 0; e < 8; ++e) hb[q][e] = to_bf16(pb[e]);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    bf16x8 ha;
                    const float *pa = &xs[0][wi + 16 * a + lr][kk + 8 * lg];
#pragma unroll
                    for (int e = 0; e < 8; ++e) ha[e] = to_bf16(pa[e]);
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha, hb[b], acc[a][b], 0, 0, 0);
                }
            }
        } else {
            for (int kk = 0; kk < kc; kk += 32) {
                bf16x8 ha[4], hb[4], la[4], lb[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float *pa = &xs[0][wi + 16 * q + lr][kk + 8 * lg];
                    const float *pb = &xs[1][wj + 16 * q + lr][kk + 8 * lg];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float xa = pa[e], xb = pb[e];
                        const __bf16 ya = to_bf16(xa), yb = to_bf16(xb);
                        ha[q][e] = ya;
                        hb[q][e] = yb;
                        if (MODE == kModeBF16x3) {
                            la[q][e] = to_bf16(xa - from_bf16(ya));
                            lb[q][e] = to_bf16(xb - from_bf16(yb));
                        }
                    }
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        if (MODE == kModeBF16x3) {
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(la[a], hb[b], acc[a][b], 0, 0, 0);
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[a], lb[b], acc[a][b], 0, 0, 0);
                        }
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[a], hb[b], acc[a][b], 0, 0, 0);
                    }
            }
        }
        __syncthreads();
    }
    // Epilogue, kRows rows of the tile at a time (FP32/BF16: two halves, waves 0-1 own rows
    // 0-63 and waves 2-3 rows 64-127; BF16x3: the whole tile): form S in the MFMA layout
    // (lane l, register r of a block holds row 4*(l/16) + r, column l%16) into the LDS tile,
    // then write it row by row with 16-byte non-temporal stores (each row segment is 512
    // contiguous bytes).
    constexpr int kRows = (MODE == kModeBF16x3) ? 128 : 64;
    float(*tile)[kTs] = reinterpret_cast<float(*)[kTs]>(smem);
    const int col4 = (tid & 31) * 4;
    const int jg = bj + col4;
    const bool vec_ok = ((lds & 3) == 0) && ((((uintptr_t)S) & 15) == 0);
#pragma unroll
    for (int pass = 0; pass < 128 / kRows; ++pass) {
        if (kRows == 128 || (wave >> 1) == pass) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int il = (kRows == 128 ? wi : 0) + 16 * a + 4 * lg + r;   // row inside the pass
                    const int i = bi + kRows * pass + il;
                    const float ni = norms[min(i, n - 1)];
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int jl = wj + 16 * b + lr;
                        const int j = bj + jl;
                        const float v = -((ni + norms[min(j, n - 1)]) - 2.f * acc[a][b][r]);
                        tile[il][jl] = (i == j) ? 0.f : fminf(0.f, v);
                    }
                }
            }
        }
        __syncthreads();
        for (int rr = tid >> 5; rr < kRows; rr += 8) {
            const int i = bi + kRows * pass + rr;
            if (i >= n) break;
            float *dst = S + (int64_t)i * lds + jg;
            if (vec_ok && jg + 3 < n) {
                f32x4 v;
                v[0] = tile[rr][col4];
                v[1] = tile[rr][col4 + 1];
                v[2] = tile[rr][col4 + 2];
                v[3] = tile[rr][col4 + 3];
                __builtin_nontemporal_store(v, (f32x4 *)dst);   // measured 2-7% faster than a cached store
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (jg + e < n) dst[e] = tile[rr][col4 + e];
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void build_mfma_f64_kernel(const double *__restrict__ X, int n, int d, int64_t ldx,
                                                             const double *__restrict__ norms, double *__restrict__ S,
                                                             int64_t lds, double noise_rel, unsigned long long seed) {
#pragma clang fp contract(off)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lg = lane >> 4;
    const int i0 = blockIdx.y * 128 + (wave >> 1) * 64;
    const int j0 = blockIdx.x * 128 + (wave & 1) * 64;
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f64x4)(0.0);
    const double *ra[4], *rb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        ra[q] = X + (int64_t)min(i0 + 16 * q + lr, n - 1) * ldx;
        rb[q] = X + (int64_t)min(j0 + 16 * q + lr, n - 1) * ldx;
    }
    for (int k0 = 0; k0 < d; k0 += 4) {
        const int k = k0 + lg;
        double fa[4], fb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            fa[q] = k < d ? ra[q][k] : 0.0;
            fb[q] = k < d ? rb[q][k] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    // the FP64 16x16x4 output interleaves rows by register: lane l, register r holds row
    // (l/16) + 4r, column l%16 of a block
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + 16 * a + lg + 4 * r;
            if (i >= n) continue;
            const double ni = norms[i];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = j0 + 16 * b + lr;
                if (j >= n) continue;
                double v = fmin(0.0, -((ni + norms[j]) - 2.0 * acc[a][b][r]));
                if (i == j) {
                    v = 0.0;
                } else if (noise_rel > 0.0) {
                    const unsigned long long ctr = (unsigned long long)i * (unsigned long long)n + (unsigned long long)j;
                    const double u = (double)(splitmix64_first(seed ^ ctr) >> 11) * 0x1.0p-53;
                    v = v + (noise_rel * fabs(v)) * u;
                }
                S[(int64_t)i * lds + j] = v;
            }
        }
    }
}

}  // namespace

hipError_t launch_build(const void *X, int64_t n, int64_t d, int64_t ldx, int x_dtype, void *S, int64_t lds,
                        int s_dtype, int mode, double noise_rel, uint64_t seed, hipStream_t st) {
    if (mode == HAP_BUILD_DIRECT || mode == HAP_BUILD_DIRECT_L2) {
        const dim3 grid((unsigned)((n + kTile - 1) / kTile), (unsigned)((n + kTile - 1) / kTile));
#define HAP_BD(TX, TS)                                                                                          \
    do {                                                                                                        \
        if (mode == HAP_BUILD_DIRECT_L2)                                                                        \
            hipLaunchKernelGGL((build_direct_kernel<TX, TS, true>), grid, dim3(256), 0, st, (const TX *)X,     \
                               (int)n, (int)d, ldx, (TS *)S, lds, noise_rel, (unsigned long long)seed);        \
        else                                                                                                    \
            hipLaunchKernelGGL((build_direct_kernel<TX, TS, false>), grid, dim3(256), 0, st, (const TX *)X,    \
                               (int)n, (int)d, ldx, (TS *)S, lds, noise_rel, (unsigned long long)seed);        \
    } while (0)
        if (x_dtype == HAP_F32 && s_dtype == HAP_F32) HAP_BD(float, float);
        else if (x_dtype == HAP_F32 && s_dtype == HAP_F64) HAP_BD(float, double);
        else if (x_dtype == HAP_F64 && s_dtype == HAP_F32) HAP_BD(double, float);
        else HAP_BD(double, double);
#undef HAP_BD
        return hipGetLastError();
    }
    // Gram-matrix builds: the squared norms go to a stream-ordered scratch allocation
    const dim3 grid((unsigned)((n + 127) / 128), (unsigned)((n + 127) / 128));
    const unsigned nb = (unsigned)((n + 255) / 256);
    void *norms = nullptr;
    hipError_t e = hipMallocAsync(&norms, (size_t)n * 8, st);
    if (e != hipSuccess) return e;
    if (mode == HAP_BUILD_GEMM && s_dtype == HAP_F64) {
        hipLaunchKernelGGL(norms_kernel_f64, dim3(nb), dim3(256), 0, st, (const double *)X, (int)n, (int)d, ldx,
                           (double *)norms);
        hipLaunchKernelGGL(build_mfma_f64_kernel, grid, dim3(256), 0, st, (const double *)X, (int)n, (int)d, ldx,
                           (const double *)norms, (double *)S, lds, noise_rel, (unsigned long long)seed);
    } else {
#define HAP_BM(MODE)                                                                                            \
    do {                                                                                                        \
        hipLaunchKernelGGL((norms_kernel<MODE>), dim3(nb), dim3(256), 0, st, (const float *)X, (int)n, (int)d,  \
                           ldx, (float *)norms);                                                                 \
        hipLaunchKernelGGL((build_mfma_f32_kernel<MODE>), grid, dim3(256), 0, st, (const float *)X, (int)n,     \
                           (int)d, ldx, (const float *)norms, (float *)S, lds);                                  \
    } while (0)
        if (mode == HAP_BUILD_GEMM) HAP_BM(kModeF32);
        else if (mode == HAP_BUILD_BF16) HAP_BM(kModeBF16);
        else HAP_BM(kModeBF16x3);
#undef HAP_BM
    }
    e = hipGetLastError();
    const hipError_t e2 = hipFreeAsync(norms, st);
    return e != hipSuccess ? e : e2;
}

}  // namespace hap
