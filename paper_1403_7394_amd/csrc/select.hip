// Exact median of the off-diagonal entries of S by radix select (gfx950).
//
// Section 2 of the paper sets the preferences from the data (for example the
// mean of the extreme similarities, or random values); the data-driven constant
// used here is the median of the N(N-1) off-diagonal similarities, the mean of
// the order statistics v[M/2-1] and v[M/2] (M = N(N-1) is even).
//
// Floats are mapped to unsigned keys whose integer order is the numeric order
// (flip every bit of a negative value, set the sign bit of a non-negative one).
// The k-th smallest key is found digit by digit from the top, 11 bits per pass:
// each pass builds a histogram of the digit over the keys that match the digits
// fixed so far (per-workgroup LDS histograms, flushed with integer atomics,
// which give the same counts in any order), and a one-workgroup pick kernel
// locates the digit holding rank k.  v[M/2] is then either equal to v[M/2-1]
// (if the equal keys extend past rank k) or the smallest key above it, found by
// one min-reduction pass.  Everything stays on the device; no host round trip.
#include <mutex>

#include "hap_internal.h"

namespace hap {

namespace {

constexpr int kDigitBits = 11;
constexpr int kBins = 1 << kDigitBits;

struct SelectState {
    unsigned long long prefix;    // key bits fixed so far
    unsigned long long mask;      // which bits are fixed
    long long krem;               // rank of the wanted key among the keys matching prefix
    long long eqcount;            // number of keys equal to the selected key (after the last pass)
    unsigned long long minabove;  // smallest key greater than the selected key
    long long pad[3];
    unsigned int hist[kBins];
};

template <typename T> struct KeyOf;
template <> struct KeyOf<float> {
    typedef unsigned int K;
    static constexpr int bits = 32;
    __device__ static K key(float f) {
        const K u = __float_as_uint(f);
        return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    }
    __device__ static float value(unsigned long long k) {
        const K u = (K)k;
        return __uint_as_float((u & 0x80000000u) ? (u ^ 0x80000000u) : ~u);
    }
};
template <> struct KeyOf<double> {
    typedef unsigned long long K;
    static constexpr int bits = 64;
    __device__ static K key(double f) {
        const K u = (K)__double_as_longlong(f);
        return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
    }
    __device__ static double value(unsigned long long k) {
        const K u = k;
        return __longlong_as_double((long long)((u & 0x8000000000000000ull) ? (u ^ 0x8000000000000000ull) : ~u));
    }
};

__global__ void select_init(SelectState *st, long long k) {
    for (int b = threadIdx.x; b < kBins; b += blockDim.x) st->hist[b] = 0u;
    if (threadIdx.x == 0) {
        st->prefix = 0ull;
        st->mask = 0ull;
        st->krem = k;
        st->eqcount = 0;
        st->minabove = ~0ull;
    }
}

// Histogram of digit (key >> shift) & (2^width - 1) over off-diagonal keys matching the prefix.
template <typename T>
__global__ __launch_bounds__(256) void select_hist(const T *__restrict__ S, int n, int64_t lds, int shift,
                                                   int width, SelectState *st) {
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    __shared__ unsigned int h[kBins];
    for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    const unsigned long long prefix = st->prefix, mask = st->mask;
    const unsigned long long dmask = (1ull << width) - 1ull;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const T *row = S + (int64_t)i * lds;
        for (int j0 = threadIdx.x * VW; j0 < n; j0 += blockDim.x * VW) {
            const V v = *(const V *)(row + j0);
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const int j = j0 + e;
                if (j >= n || j == i) continue;
                const unsigned long long k = KeyOf<T>::key(v[e]);
                if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & dmask], 1u);
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += blockDim.x) {
        const unsigned int c = h[b];
        if (c) atomicAdd(&st->hist[b], c);
    }
}

// One workgroup of 1024 threads: find the digit holding rank krem, fix it, clear the histogram.
__global__ __launch_bounds__(1024) void select_pick(SelectState *st, int shift, int width) {
    __shared__ long long part[1024];
    const int tid = threadIdx.x;
    const long long c0 = st->hist[2 * tid], c1 = st->hist[2 * tid + 1];
    part[tid] = c0 + c1;
    __syncthreads();
    // inclusive scan (Hillis-Steele) of the pair sums
    for (int off = 1; off < 1024; off <<= 1) {
        const long long v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    const long long before = part[tid] - (c0 + c1);
    const long long krem = st->krem;
    int digit = -1;
    long long cum = 0, cnt = 0;
    if (krem >= before && krem < before + c0) {
        digit = 2 * tid;
        cum = before;
        cnt = c0;
    } else if (krem >= before + c0 && krem < before + c0 + c1) {
        digit = 2 * tid + 1;
        cum = before + c0;
        cnt = c1;
    }
    __syncthreads();
    if (digit >= 0) {
        st->prefix |= ((unsigned long long)digit) << shift;
        st->mask |= (((1ull << width) - 1ull)) << shift;
        st->krem = krem - cum;
        st->eqcount = cnt;
    }
    st->hist[2 * tid] = 0u;
    st->hist[2 * tid + 1] = 0u;
}

// Smallest key above the selected one, needed only when the equal keys end at rank k.
template <typename T>
__global__ __launch_bounds__(256) void select_min_above(const T *__restrict__ S, int n, int64_t lds,
                                                        SelectState *st) {
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::N;
    if (st->krem + 1 < st->eqcount) return;
    __shared__ unsigned long long sm[256];
    const unsigned long long sel = st->prefix;
    unsigned long long best = ~0ull;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const T *row = S + (int64_t)i * lds;
        for (int j0 = threadIdx.x * VW; j0 < n; j0 += blockDim.x * VW) {
            const V v = *(const V *)(row + j0);
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const int j = j0 + e;
                if (j >= n || j == i) continue;
                const unsigned long long k = KeyOf<T>::key(v[e]);
                if (k > sel && k < best) best = k;
            }
        }
    }
    sm[threadIdx.x] = best;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sm[threadIdx.x] = min(sm[threadIdx.x], sm[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && sm[0] != ~0ull) atomicMin(&st->minabove, sm[0]);
}

template <typename T>
__global__ void select_finish(const SelectState *st, double *out) {
    const T lo = KeyOf<T>::value(st->prefix);
    const T hi = (st->krem + 1 < st->eqcount) ? lo : KeyOf<T>::value(st->minabove);
    const double mid = ((double)lo + (double)hi) / 2.0;
    *out = (double)(T)mid;
}

template <typename T>
hipError_t median_impl(const T *S, int64_t n, int64_t lds, void *scratch, double *out, hipStream_t st) {
    SelectState *ss = (SelectState *)scratch;
    const long long M = (long long)n * (long long)(n - 1);
    const long long k = M / 2 - 1;
    hipLaunchKernelGGL(select_init, dim3(1), dim3(1024), 0, st, ss, k);
    const int grid = (int)(n < 2048 ? n : 2048);
    int hi = KeyOf<T>::bits;
    while (hi > 0) {
        const int width = hi >= kDigitBits ? kDigitBits : hi;
        const int shift = hi - width;
        hipLaunchKernelGGL((select_hist<T>), dim3(grid), dim3(256), 0, st, S, (int)n, lds, shift, width, ss);
        hipLaunchKernelGGL(select_pick, dim3(1), dim3(1024), 0, st, ss, shift, width);
        hi = shift;
    }
    hipLaunchKernelGGL((select_min_above<T>), dim3(grid), dim3(256), 0, st, S, (int)n, lds, ss);
    hipLaunchKernelGGL((select_finish<T>), dim3(1), dim3(1), 0, st, ss, out);
    return hipGetLastError();
}

}  // namespace

size_t select_scratch_bytes() { return (sizeof(SelectState) + 255) & ~size_t(255); }

// Scratch of the allocation-free median (hap_median_offdiag_noalloc): one select state in a
// file-scope device array, one copy per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it only stands for the symbol); it uses
// the device address hipGetSymbolAddress returns, looked up once per device.
constexpr size_t kStaticScratchBytes = 8448;
static_assert(sizeof(SelectState) <= kStaticScratchBytes, "select state does not fit the static scratch");
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

size_t static_scratch_bytes() { return kStaticScratchBytes; }

hipError_t launch_median_offdiag(const void *S, int64_t n, int64_t lds, int dtype, void *scratch,
                                 double *median_dev, hipStream_t st) {
    if (dtype == HAP_F32) return median_impl<float>((const float *)S, n, lds, scratch, median_dev, st);
    if (dtype == HAP_F64) return median_impl<double>((const double *)S, n, lds, scratch, median_dev, st);
    return hipErrorInvalidValue;
}

}  // namespace hap
