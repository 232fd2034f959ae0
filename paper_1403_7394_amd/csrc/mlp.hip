// The warm start's perceptron: n_in -> hidden -> hidden -> n_out with ReLU after both hidden
// layers, mean-squared-error loss, backpropagation and Adam.  Every product is one GEMM
// kernel on the matrix cores (FP32 operands on the 16x16x4 FP32 MFMA, or BF16 operands on the
// 16x16x32 BF16 MFMA, FP32 accumulation in both); bias, ReLU and the ReLU mask of the backward
// pass are fused into its epilogue.  Parameters are one flat FP32 vector (the master copy):
// W1 (n_in x hidden, row-major), b1, W2 (hidden x hidden), b2, W3 (hidden x n_out), b3.
#include <hip/hip_runtime.h>

#include <cmath>

#include "hap_internal.h"

namespace hap {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// float -> bf16, round to nearest even (finite inputs)
__device__ __forceinline__ __bf16 rne_bf16(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
}

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_MASK = 3 };

// C(m, n) = epilogue(sum_k A(m, k) B(k, n)) with A(m, k) = A[m*sam + k*sak] and
// B(k, n) = B[k*sbk + n*sbn], so transposed operands are plain stride choices.
struct GemmArgs {
    const float *A;
    int64_t sam, sak;
    const float *B;
    int64_t sbk, sbn;
    float *C;
    int64_t ldc;
    const float *bias;   // [N] (EPI_BIAS, EPI_BIAS_RELU)
    const float *mask;   // C(m, n) is kept where mask[m*ldm + n] > 0 (EPI_MASK)
    int64_t ldm;
    int M, N, K;
    int epi;
};

constexpr int TM = 64, TN = 64, TK = 32, LDT = TK + 4;

// 64 x 64 output tile per workgroup; four waves of 32 x 32, each 2 x 2 MFMA blocks of 16 x 16
// (lane l, register r of a block holds row 4*(l/16) + r, column l%16).  Tiles of A and of B^T
// are staged in LDS as FP32 with zero fill past M, N and K; the fragment of lane l is row
// l%16 of the A tile and row l%16 of the B^T tile at the same k slots.
template <bool BF16>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(GemmArgs g) {
    __shared__ float As[TM][LDT];
    __shared__ float Bs[TN][LDT];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int wm = (wid >> 1) * 32, wn = (wid & 1) * 32;
    const int r16 = lane & 15, kg = lane >> 4;
    const bool a_kfast = g.sak == 1, b_nfast = g.sbn == 1;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += TK) {
        for (int e = tid; e < TM * TK; e += 256) {
            const int m = a_kfast ? e / TK : e % TM;
            const int k = a_kfast ? e % TK : e / TM;
            const int gm = m0 + m, gk = k0 + k;
            As[m][k] = (gm < g.M && gk < g.K) ? g.A[(int64_t)gm * g.sam + (int64_t)gk * g.sak] : 0.f;
        }
        for (int e = tid; e < TN * TK; e += 256) {
            const int nn = b_nfast ? e % TN : e / TK;
            const int k = b_nfast ? e / TN : e % TK;
            const int gn = n0 + nn, gk = k0 + k;
            Bs[nn][k] = (gn < g.N && gk < g.K) ? g.B[(int64_t)gk * g.sbk + (int64_t)gn * g.sbn] : 0.f;
        }
        __syncthreads();
        if constexpr (BF16) {
            bf16x8 fa[2], fb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const float *pa = &As[wm + 16 * i + r16][8 * kg];
                const float *pb = &Bs[wn + 16 * i + r16][8 * kg];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    fa[i][e] = rne_bf16(pa[e]);
                    fb[i][e] = rne_bf16(pb[e]);
                }
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        } else {
#pragma unroll
            for (int kk = 0; kk < TK; kk += 4) {
                float fa[2], fb[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    fa[i] = As[wm + 16 * i + r16][kk + kg];
                    fb[i] = Bs[wn + 16 * i + r16][kk + kg];
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * kg + r;
                const int n = n0 + wn + 16 * j + r16;
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][r];
                if (g.epi == EPI_BIAS || g.epi == EPI_BIAS_RELU) v = v + g.bias[n];
                if (g.epi == EPI_BIAS_RELU) v = v > 0.f ? v : 0.f;
                if (g.epi == EPI_MASK) v = g.mask[(int64_t)m * g.ldm + n] > 0.f ? v : 0.f;
                g.C[(int64_t)m * g.ldc + n] = v;
            }
}

// dY = 2 (Y - T) / (rows * n_out) and loss = sum (Y - T)^2 / (rows * n_out); one workgroup,
// FP64 accumulation in a fixed order.
__global__ __launch_bounds__(1024) void mse_kernel(const float *__restrict__ Y, int64_t ldy, const float *__restrict__ T,
                                                   int64_t ldt, int rows, int nout, float *__restrict__ dY,
                                                   double *__restrict__ loss) {
    __shared__ double part[16];
    const int tid = threadIdx.x;
    const int64_t cnt = (int64_t)rows * nout;
    const float scale = (float)(2.0 / (double)cnt);
    double acc = 0.0;
    for (int64_t e = tid; e < cnt; e += 1024) {
        const int64_t r = e / nout, o = e % nout;
        const float d = Y[r * ldy + o] - T[r * ldt + o];
        dY[e] = scale * d;
        acc += (double)d * (double)d;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((tid & 63) == 0) part[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < 16; ++w) s += part[w];
        *loss = s / (double)cnt;
    }
}

// out[n] = sum over rows of X[r*ldx + n]; one workgroup per column, fixed order.
__global__ __launch_bounds__(256) void colsum_rows_kernel(const float *__restrict__ X, int64_t ldx, int rows,
                                                          float *__restrict__ out) {
    __shared__ float part[4];
    const int n = blockIdx.x, tid = threadIdx.x;
    float acc = 0.f;
    for (int r = tid; r < rows; r += 256) acc += X[(int64_t)r * ldx + n];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((tid & 63) == 0) part[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) out[n] = (part[0] + part[1]) + (part[2] + part[3]);
}

// Adam (Kingma and Ba, 2015): m and v are the first and second moment estimates, bc1 and bc2
// the bias corrections 1 - beta^step.
__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ P, const float *__restrict__ G,
                                                   float *__restrict__ Mv, float *__restrict__ Vv, int64_t count,
                                                   float b1, float omb1, float b2, float omb2, float lr, float eps,
                                                   float bc1, float bc2) {
#pragma clang fp contract(off)
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
        const float g = G[i];
        const float m = b1 * Mv[i] + omb1 * g;
        const float v = b2 * Vv[i] + omb2 * (g * g);
        Mv[i] = m;
        Vv[i] = v;
        P[i] = P[i] - lr * (m / bc1) / (sqrtf(v / bc2) + eps);
    }
}

// Rows idx[0..rows) of X (width w, row stride ldx, x_rows rows) into a packed buffer; an
// index outside [0, x_rows) yields NaN instead of a read.
__global__ __launch_bounds__(256) void gather_rows_kernel(const float *__restrict__ X, int64_t ldx, int w,
                                                          const int32_t *__restrict__ idx, int rows, int x_rows,
                                                          float *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)rows * w) return;
    const int64_t r = e / w, c = e % w;
    const int32_t src = idx[r];
    out[e] = (src >= 0 && src < x_rows) ? X[(int64_t)src * ldx + c] : __builtin_nanf("");
}

hipError_t gemm(bool bf16, const GemmArgs &g, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    const dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM);
    if (bf16)
        hipLaunchKernelGGL(mlp_gemm_kernel<true>, grid, dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL(mlp_gemm_kernel<false>, grid, dim3(256), 0, st, g);
    return hipGetLastError();
}

GemmArgs make_gemm(const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk, int64_t sbn, float *C,
                   int64_t ldc, int M, int N, int K, int epi, const float *bias = nullptr,
                   const float *mask = nullptr, int64_t ldm = 0) {
    GemmArgs g;
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.sbk = sbk;
    g.sbn = sbn;
    g.C = C;
    g.ldc = ldc;
    g.bias = bias;
    g.mask = mask;
    g.ldm = ldm;
    g.M = M;
    g.N = N;
    g.K = K;
    g.epi = epi;
    return g;
}

#define MLP_TRY(expr)                        \
    do {                                     \
        hipError_t _e = (expr);              \
        if (_e != hipSuccess) return _e;     \
    } while (0)

}  // namespace

MlpLayout mlp_layout(int n_in, int hidden, int n_out, int64_t rows) {
    MlpLayout lo{};
    const int64_t H = hidden;
    lo.oW1 = 0;
    lo.ob1 = lo.oW1 + (int64_t)n_in * H;
    lo.oW2 = lo.ob1 + H;
    lo.ob2 = lo.oW2 + H * H;
    lo.oW3 = lo.ob2 + H;
    lo.ob3 = lo.oW3 + H * n_out;
    lo.count = lo.ob3 + n_out;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    lo.Xb = take((size_t)rows * n_in * 4);
    lo.Tb = take((size_t)rows * n_out * 4);
    lo.H1 = take((size_t)rows * H * 4);
    lo.H2 = take((size_t)rows * H * 4);
    lo.Y = take((size_t)rows * n_out * 4);
    lo.dY = take((size_t)rows * n_out * 4);
    lo.dH2 = take((size_t)rows * H * 4);
    lo.dH1 = take((size_t)rows * H * 4);
    lo.G = take((size_t)lo.count * 4);
    lo.loss = take(64);
    lo.bytes = off;
    return lo;
}

hipError_t mlp_forward(const MlpLayout &lo, int n_in, int hidden, int n_out, bool bf16, const float *P,
                       const float *X, int64_t ldx, int rows, float *Y, int64_t ldy, char *ws, hipStream_t st) {
    float *H1 = (float *)(ws + lo.H1), *H2 = (float *)(ws + lo.H2);
    const int H = hidden;
    MLP_TRY(gemm(bf16, make_gemm(X, ldx, 1, P + lo.oW1, H, 1, H1, H, rows, H, n_in, EPI_BIAS_RELU, P + lo.ob1), st));
    MLP_TRY(gemm(bf16, make_gemm(H1, H, 1, P + lo.oW2, H, 1, H2, H, rows, H, H, EPI_BIAS_RELU, P + lo.ob2), st));
    MLP_TRY(gemm(bf16, make_gemm(H2, H, 1, P + lo.oW3, n_out, 1, Y, ldy, rows, n_out, H, EPI_BIAS, P + lo.ob3), st));
    return hipSuccess;
}

hipError_t mlp_loss_grad(const MlpLayout &lo, int n_in, int hidden, int n_out, bool bf16, const float *P,
                         const float *X, int64_t ldx, const float *T, int64_t ldt, int rows, float *G, double *loss,
                         char *ws, hipStream_t st) {
    const int H = hidden;
    float *H1 = (float *)(ws + lo.H1), *H2 = (float *)(ws + lo.H2), *Y = (float *)(ws + lo.Y);
    float *dY = (float *)(ws + lo.dY), *dH2 = (float *)(ws + lo.dH2), *dH1 = (float *)(ws + lo.dH1);
    MLP_TRY(mlp_forward(lo, n_in, hidden, n_out, bf16, P, X, ldx, rows, Y, n_out, ws, st));
    hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, st, Y, (int64_t)n_out, T, ldt, rows, n_out, dY, loss);
    MLP_TRY(hipGetLastError());
    // layer 3: gW3 = H2^T dY, gb3 = column sums of dY, dH2 = (dY W3^T) masked by H2 > 0
    MLP_TRY(gemm(bf16, make_gemm(H2, 1, H, dY, n_out, 1, G + lo.oW3, n_out, H, n_out, rows, EPI_STORE), st));
    hipLaunchKernelGGL(colsum_rows_kernel, dim3(n_out), dim3(256), 0, st, dY, (int64_t)n_out, rows, G + lo.ob3);
    MLP_TRY(hipGetLastError());
    MLP_TRY(gemm(bf16, make_gemm(dY, n_out, 1, P + lo.oW3, 1, n_out, dH2, H, rows, H, n_out, EPI_MASK, nullptr, H2, H),
                 st));
    // layer 2
    MLP_TRY(gemm(bf16, make_gemm(H1, 1, H, dH2, H, 1, G + lo.oW2, H, H, H, rows, EPI_STORE), st));
    hipLaunchKernelGGL(colsum_rows_kernel, dim3(H), dim3(256), 0, st, dH2, (int64_t)H, rows, G + lo.ob2);
    MLP_TRY(hipGetLastError());
    MLP_TRY(gemm(bf16, make_gemm(dH2, H, 1, P + lo.oW2, 1, H, dH1, H, rows, H, H, EPI_MASK, nullptr, H1, H), st));
    // layer 1
    MLP_TRY(gemm(bf16, make_gemm(X, 1, ldx, dH1, H, 1, G + lo.oW1, H, n_in, H, rows, EPI_STORE), st));
    hipLaunchKernelGGL(colsum_rows_kernel, dim3(H), dim3(256), 0, st, dH1, (int64_t)H, rows, G + lo.ob1);
    return hipGetLastError();
}

hipError_t mlp_adam(float *P, const float *G, float *M, float *V, int64_t count, int64_t step, double lr, double b1,
                    double b2, double eps, hipStream_t st) {
    const double bc1 = 1.0 - std::pow(b1, (double)step), bc2 = 1.0 - std::pow(b2, (double)step);
    const int64_t blocks = (count + 255) / 256;
    const int grid = (int)(blocks < 4096 ? blocks : 4096);
    hipLaunchKernelGGL(adam_kernel, dim3(grid), dim3(256), 0, st, P, G, M, V, count, (float)b1, (float)(1.0 - b1),
                       (float)b2, (float)(1.0 - b2), (float)lr, (float)eps, (float)bc1, (float)bc2);
    return hipGetLastError();
}

hipError_t mlp_gather(const float *X, int64_t ldx, int w, const int32_t *idx, int rows, int x_rows, float *out,
                      hipStream_t st) {
    const int64_t total = (int64_t)rows * w;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, X, ldx, w, idx,
                       rows, x_rows, out);
    return hipGetLastError();
}

}  // namespace hap
