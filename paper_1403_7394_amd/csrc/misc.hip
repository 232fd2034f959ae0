// Small kernels around the sweep: preference fill, distinct-exemplar count and the
// FP64 net similarity.
#include "hap_internal.h"

namespace hap {

namespace {

template <typename T>
__global__ void fill_pref_kernel(T *pref, int64_t ldw, int n, int levels, const double *value) {
    const T v = (T)(*value);
    const int64_t total = (int64_t)levels * ldw;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(k % ldw);
        if (j < n) pref[k] = v;
    }
}

__global__ void zero_i32(int32_t *p, int n) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) p[k] = 0;
}

__global__ void mark_labels(const int32_t *labels, int n, int32_t *mark) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int e = labels[k];
        if (e >= 0 && e < n) mark[e] = 1;
    }
}

__global__ __launch_bounds__(1024) void sum_marks(const int32_t *mark, int n, int32_t *out) {
    __shared__ int part[1024];
    int acc = 0;
    for (int k = threadIdx.x; k < n; k += 1024) acc += mark[k];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

// NS^l = sum_i s^l_{i,e_i}, s^l_ii = p^l_i, in FP64; out[l] per level and out[levels] the total.
// One workgroup; every thread accumulates a fixed subset of points, then a fixed-order tree,
// so the result does not depend on scheduling.
template <typename T, typename TX>
__global__ __launch_bounds__(1024) void net_similarity_kernel(const T *__restrict__ S, int64_t lds,
                                                              const T *__restrict__ pref, int64_t ldw,
                                                              const int32_t *__restrict__ E, int n, int levels,
                                                              const TX *__restrict__ X, int64_t d, int64_t ldx,
                                                              double *out) {
    __shared__ double part[1024];
    double total = 0.0;
    for (int l = 0; l < levels; ++l) {
        const int32_t *e = E + (int64_t)l * ldw;
        const T *p = pref + (int64_t)l * ldw;
        double acc = 0.0;
        for (int i = threadIdx.x; i < n; i += 1024) {
            const int k = e[i];
            double v;
            if (k < 0 || k >= n) {
                v = __builtin_nan("");   // no valid exemplar (non-finite messages)
            } else if (k == i) {
                v = (double)p[i];
            } else if (X != nullptr) {
                double s2 = 0.0;
                for (int64_t q = 0; q < d; ++q) {
                    const double df = (double)X[(int64_t)i * ldx + q] - (double)X[(int64_t)k * ldx + q];
                    s2 += df * df;
                }
                v = -s2;
            } else {
                v = (double)S[(int64_t)i * lds + k];
            }
            acc += v;
        }
        part[threadIdx.x] = acc;
        __syncthreads();
        for (int off = 512; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            out[l] = part[0];
            total += part[0];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[levels] = total;
}

}  // namespace

hipError_t launch_fill_pref(void *pref_base, int64_t ldw, int n, int levels, int dtype, const double *value_dev,
                            hipStream_t st) {
    const int64_t total = (int64_t)levels * ldw;
    const int grid = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    if (dtype == HAP_F32)
        hipLaunchKernelGGL((fill_pref_kernel<float>), dim3(grid), dim3(256), 0, st, (float *)pref_base, ldw, n,
                           levels, value_dev);
    else
        hipLaunchKernelGGL((fill_pref_kernel<double>), dim3(grid), dim3(256), 0, st, (double *)pref_base, ldw, n,
                           levels, value_dev);
    return hipGetLastError();
}

hipError_t launch_count_distinct(const int32_t *labels, int n, int32_t *mark, int32_t *out, hipStream_t st) {
    const int grid = (n + 255) / 256;
    hipLaunchKernelGGL(zero_i32, dim3(grid), dim3(256), 0, st, mark, n);
    hipLaunchKernelGGL(mark_labels, dim3(grid), dim3(256), 0, st, labels, n, mark);
    hipLaunchKernelGGL(sum_marks, dim3(1), dim3(1024), 0, st, mark, n, out);
    return hipGetLastError();
}

hipError_t launch_net_similarity(const void *S, int64_t lds, int dtype, const void *pref_base, int64_t ldw,
                                 const int32_t *Efinal_base, int n, int levels, const void *X, int64_t d,
                                 int64_t ldx, int x_dtype, double *out, hipStream_t st) {
#define HAP_NS(T, TX)                                                                                   \
    hipLaunchKernelGGL((net_similarity_kernel<T, TX>), dim3(1), dim3(1024), 0, st, (const T *)S, lds,  \
                       (const T *)pref_base, ldw, Efinal_base, n, levels, (const TX *)X, d, ldx, out)
    if (dtype == HAP_F32) {
        if (x_dtype == HAP_F64) HAP_NS(float, double); else HAP_NS(float, float);
    } else {
        if (x_dtype == HAP_F64) HAP_NS(double, double); else HAP_NS(double, float);
    }
#undef HAP_NS
    return hipGetLastError();
}

}  // namespace hap
