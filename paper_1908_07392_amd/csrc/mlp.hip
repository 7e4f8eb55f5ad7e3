/*
 * mlp.hip -- learned GMRES warm start for a time series of second-kind BIE
 * solves (Sec. 3.2 BIE, solved once per time step of the implicit scheme of
 * Sec. 3): Fourier features of the boundary densities and a small multilayer
 * perceptron trained on the densities the solver itself produces.
 * Declarations and contracts: include/mhlp.h.
 *
 * Features.  For each closed curve c the density is expanded in the curve
 * parameter theta in [0, 2 pi):  c_k = (1/2 pi) int mu(theta) e^{-i k theta},
 * evaluated with the panel rule in theta (weights omega_m = half panel span in
 * theta times the Gauss-Legendre weight), k = 0..K-1, stored as (Re, Im)
 * pairs: F = 2 K n_curves reals per density.  Synthesis is the real Fourier
 * series c_0 + sum_{k>=1} 2 Re(c_k e^{i k theta}).  Both are FP64.
 *
 * Network.  n_in -> width -> width -> n_out with GELU (tanh form) after the
 * two hidden layers.  Master weights and Adam state are FP32; every product
 * runs on the matrix cores with operands rounded to BF16 and FP32
 * accumulation (v_mfma_f32_16x16x32_bf16).
 *
 * Warm start.  Input: the backward differences 0..H-1 of the coefficients of
 * the last H densities (an invertible linear map of the history that keeps
 * small differences at full BF16 relative precision), each group scaled to
 * unit RMS over the training samples; output: the error of the order-p
 * polynomial extrapolation of the history (p = 0: the increment over the
 * last density), in units of its training RMS; initial guess
 * extrapolation(mu_{s-p..s}) + synthesis(output).
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "mhlp.h"

__attribute__((visibility("hidden"))) mhlp_status mhlp_set_error(mhlp_status s, const char *msg);

static mhlp_status mfail(mhlp_status s, const std::string &msg) { return mhlp_set_error(s, msg.c_str()); }

#define MHIP(x)                                                                                          \
    do {                                                                                                 \
        hipError_t e_ = (x);                                                                             \
        if (e_ != hipSuccess) return mfail(MHLP_HIP_ERROR, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

static inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

/* ------------------------------------------------------------------------ */
/* BF16 GEMM on the matrix cores                                              */
/*   C_z[m][n] = sum_{k in chunk z} A(m,k) B(k,n)                             */
/*   A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn] (FP32 in memory,    */
/*   rounded to nearest-even BF16 as they are staged).  A block of four waves */
/*   owns a 32x32 output tile (each wave a 16x16 quarter); per step of 32 k   */
/*   its threads stage the tile's A rows and B columns in LDS as BF16 (each   */
/*   element read from global memory once per block) and every wave issues    */
/*   one v_mfma_f32_16x16x32_bf16.  blockIdx.z splits K into chunks of Kc (a  */
/*   multiple of 32) whose partial tiles go to C + z*split_stride and are     */
/*   summed by the consumer.                                                  */
/* v_mfma_f32_16x16x32_bf16 operand layout (lane l of 64):                    */
/*   A: row l%16, k = 8(l/16)..8(l/16)+7;  B: column l%16, same k;            */
/*   D: column l%16, rows 4(l/16)..4(l/16)+3.                                 */
/* AV / BV: the operand is contiguous along k and 16-byte aligned, so the     */
/* four k values a thread stages come in one load.                            */
/* ------------------------------------------------------------------------ */
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef short short8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f32_to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u); /* round to nearest even (inputs finite) */
    return (short)(u >> 16);
}

template <bool VEC>
__device__ __forceinline__ short4_t load_k4(const float *__restrict__ P, int64_t row_off, int64_t sk, int k, int kend,
                                            bool valid)
{
    short4_t r;
    if (VEC) {
        /* kend - k is either >= 4 or <= 0: chunk bounds and K are multiples of 4 */
        float4_t v = {0.f, 0.f, 0.f, 0.f};
        if (valid && k < kend) v = *reinterpret_cast<const float4_t *>(P + row_off + k);
#pragma unroll
        for (int t = 0; t < 4; ++t) r[t] = f32_to_bf16(v[t]);
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) r[t] = f32_to_bf16((valid && k + t < kend) ? P[row_off + (int64_t)(k + t) * sk] : 0.f);
    }
    return r;
}

constexpr int GT = 32;       /* output tile edge and k step */
constexpr int GT_PAD = 8;    /* LDS row padding (BF16 elements): rows of 80 bytes */

template <bool AV, bool BV>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, int Kc, const float *__restrict__ A,
                                                        int64_t sam, int64_t sak, const float *__restrict__ B,
                                                        int64_t sbk, int64_t sbn, float *__restrict__ C, int64_t ldc,
                                                        int64_t split_stride)
{
    __shared__ __attribute__((aligned(16))) short la[GT][GT + GT_PAD]; /* [m][k] */
    __shared__ __attribute__((aligned(16))) short lb[GT][GT + GT_PAD]; /* [n][k] */
    const int tm = blockIdx.y * GT, tn = blockIdx.x * GT;
    const int kbeg = blockIdx.z * Kc, kend = min(K, kbeg + Kc);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = (wv >> 1) * 16, wn = (wv & 1) * 16; /* the wave's quarter of the tile */
    /* staging: thread t takes row (column) t / 8 of the tile and k = 4 (t % 8) .. + 3 */
    const int sr = t >> 3, sk4 = (t & 7) * 4;
    const bool va = tm + sr < M, vb = tn + sr < N;
    const int64_t aoff = (int64_t)(tm + sr) * sam, boff = (int64_t)(tn + sr) * sbn;
    const int r = lane & 15, kg = lane >> 4;
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += GT) {
        const short4_t a = load_k4<AV>(A, aoff, sak, k0 + sk4, kend, va);
        const short4_t b = load_k4<BV>(B, boff, sbk, k0 + sk4, kend, vb);
        __syncthreads(); /* the previous step's operands are read */
        *reinterpret_cast<short4_t *>(&la[sr][sk4]) = a;
        *reinterpret_cast<short4_t *>(&lb[sr][sk4]) = b;
        __syncthreads();
        const short8_t av = *reinterpret_cast<const short8_t *>(&la[wm + r][8 * kg]);
        const short8_t bv = *reinterpret_cast<const short8_t *>(&lb[wn + r][8 * kg]);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, av),
                                                      __builtin_bit_cast(bf16x8_t, bv), acc, 0, 0, 0);
    }
    C += blockIdx.z * split_stride;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = tm + wm + 4 * kg + q, col = tn + wn + r;
        if (row < M && col < N) C[(int64_t)row * ldc + col] = acc[q];
    }
}

/* K chunking: enough blocks to fill the chip (about 256 blocks of four
   waves), chunks of at least 64 and a multiple of GT; at most MAX_SPLITS */
constexpr int MAX_SPLITS = 32;

static int splitk_chunk(int M, int N, int K)
{
    const int64_t tiles = (int64_t)nb(M, GT) * nb(N, GT);
    int splits = (int)std::min<int64_t>(MAX_SPLITS, std::max<int64_t>(1, (256 + tiles - 1) / tiles));
    splits = std::max(1, std::min(splits, K / 64));
    int Kc = (int)nb(K, splits);
    Kc = (Kc + GT - 1) / GT * GT;
    return Kc;
}

static bool kvec(const float *P, int64_t srow, int64_t sk, int K)
{
    return sk == 1 && srow % 4 == 0 && K % 4 == 0 && ((uintptr_t)P & 15u) == 0;
}

/* returns the number of K chunks written (C + z*split_stride, z < chunks) */
static int gemm_bf16(hipStream_t st, int M, int N, int K, const float *A, int64_t sam, int64_t sak, const float *B,
                     int64_t sbk, int64_t sbn, float *C, int64_t ldc, int64_t split_stride, bool allow_split)
{
    const int Kc = allow_split ? splitk_chunk(M, N, K) : (K + GT - 1) / GT * GT;
    const int splits = (int)nb(K, Kc);
    dim3 grid(nb(N, GT), nb(M, GT), (unsigned)splits);
    const bool av = kvec(A, sam, sak, K), bv = kvec(B, sbn, sbk, K);
    if (av && bv)
        gemm_bf16_kernel<true, true><<<grid, 256, 0, st>>>(M, N, K, Kc, A, sam, sak, B, sbk, sbn, C, ldc, split_stride);
    else if (av)
        gemm_bf16_kernel<true, false><<<grid, 256, 0, st>>>(M, N, K, Kc, A, sam, sak, B, sbk, sbn, C, ldc,
                                                            split_stride);
    else if (bv)
        gemm_bf16_kernel<false, true><<<grid, 256, 0, st>>>(M, N, K, Kc, A, sam, sak, B, sbk, sbn, C, ldc,
                                                            split_stride);
    else
        gemm_bf16_kernel<false, false><<<grid, 256, 0, st>>>(M, N, K, Kc, A, sam, sak, B, sbk, sbn, C, ldc,
                                                             split_stride);
    return splits;
}

/* out[r][c] = sum_z P[z*stride + r*cols + c] */
__global__ void splitk_sum_kernel(const float *__restrict__ P, int splits, int64_t stride, float *__restrict__ out,
                                  int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += P[z * stride + i];
    out[i] = s;
}

/* ------------------------------------------------------------------------ */
/* elementwise pieces of the network                                          */
/* ------------------------------------------------------------------------ */
constexpr float GELU_C = 0.7978845608028654f; /* sqrt(2/pi) */
constexpr float GELU_A = 0.044715f;

/* Z = sum_z Zp[z] + b (per column); A = gelu(Z) when A is non-null
   (Zp may alias Z when splits == 1) */
__global__ void bias_act_kernel(const float *Zp, int splits, int64_t sstride, const float *__restrict__ b, float *Z,
                                float *__restrict__ Aout, int rows, int cols)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows * cols) return;
    float z = b[i % cols];
    for (int q = 0; q < splits; ++q) z += Zp[q * sstride + i];
    Z[i] = z;
    if (Aout) {
        const float t = tanhf(GELU_C * (z + GELU_A * z * z * z));
        Aout[i] = 0.5f * z * (1.f + t);
    }
}

/* dZ = (sum_z dAp[z]) * gelu'(Z) */
__global__ void gelu_back_kernel(const float *__restrict__ Z, const float *__restrict__ dAp, int splits,
                                 int64_t sstride, float *__restrict__ dZ, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float da = 0.f;
    for (int q = 0; q < splits; ++q) da += dAp[q * sstride + i];
    const float z = Z[i];
    const float t = tanhf(GELU_C * (z + GELU_A * z * z * z));
    const float du = GELU_C * (1.f + 3.f * GELU_A * z * z);
    dZ[i] = da * (0.5f * (1.f + t) + 0.5f * z * (1.f - t * t) * du);
}

/* dY = 2 (Y - T) / n and loss = mean (Y - T)^2 (loss zeroed by the caller) */
__global__ __launch_bounds__(256) void mse_kernel(const float *__restrict__ Y, const float *__restrict__ T,
                                                  float *__restrict__ dY, int64_t n, float *__restrict__ loss)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float d = Y[i] - T[i];
        dY[i] = 2.f * d / (float)n;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, red[0] / (float)n);
}

/* db[c] = sum_r dZ[r][c] */
__global__ void colsum_kernel(const float *__restrict__ dZ, float *__restrict__ db, int rows, int cols)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += dZ[(int64_t)r * cols + c];
    db[c] = s;
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

/* Uniform(-scale, scale) on [w_begin, w_end) from a counter-based generator:
   the SplitMix64 output function applied to seed + index * golden-ratio step */
__global__ void init_uniform_kernel(float *__restrict__ p, int64_t w_begin, int64_t w_end, float scale, uint64_t seed)
{
    const int64_t i = w_begin + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= w_end) return;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0); /* [0,1) */
    p[i] = (float)((2.0 * u - 1.0) * scale);
}

__global__ void zero_f32_kernel(float *__restrict__ p, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

static void zero_f32(hipStream_t st, float *p, int64_t n)
{
    if (n > 0) zero_f32_kernel<<<nb(n, 256), 256, 0, st>>>(p, n);
}

/* ------------------------------------------------------------------------ */
/* the network                                                               */
/* ------------------------------------------------------------------------ */
struct mhlp_mlp {
    int n[4] = {0, 0, 0, 0}; /* layer widths: n0 (in), n1 = n2 (hidden), n3 (out) */
    int64_t off_w[3] = {0, 0, 0}, off_b[3] = {0, 0, 0}, nparam = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr;
    int cap = 0; /* batch capacity of the activation buffers */
    float *Z[3] = {nullptr, nullptr, nullptr}, *Ac[2] = {nullptr, nullptr}, *d0 = nullptr, *d1 = nullptr;
    float *ws = nullptr; /* split-K partial tiles: MAX_SPLITS x cap x max(n1, n2, n3) */
    int64_t ws_len = 0;
    int64_t step = 0;
};

template <class T>
static mhlp_status malloc_dev(T **p, int64_t n)
{
    *p = nullptr;
    if (n <= 0) return MHLP_OK;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (size_t)n);
    if (e != hipSuccess) {
        *p = nullptr;
        return mfail(MHLP_NO_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return MHLP_OK;
}

template <class T>
static void free_dev(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

static void free_acts(mhlp_mlp *N)
{
    for (auto &z : N->Z) free_dev(z);
    for (auto &a : N->Ac) free_dev(a);
    free_dev(N->d0);
    free_dev(N->d1);
    free_dev(N->ws);
    N->ws_len = 0;
    N->cap = 0;
}

extern "C" mhlp_status mhlp_mlp_destroy(mhlp_mlp *N)
{
    if (!N) return MHLP_OK;
    (void)hipDeviceSynchronize();
    free_acts(N);
    free_dev(N->p);
    free_dev(N->g);
    free_dev(N->m);
    free_dev(N->v);
    free_dev(N->loss);
    delete N;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_mlp_create(int32_t n_in, int32_t width, int32_t n_out, uint64_t seed, void *stream,
                                       mhlp_mlp **out)
{
    if (!out) return mfail(MHLP_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_in < 1 || width < 1 || n_out < 1) return mfail(MHLP_INVALID_ARG, "layer sizes must be >= 1");
    if ((int64_t)n_in * width > (int64_t)1 << 30 || (int64_t)width * n_out > (int64_t)1 << 30)
        return mfail(MHLP_INVALID_ARG, "layer too large");
    hipStream_t st = (hipStream_t)stream;
    mhlp_mlp *N = new mhlp_mlp();
    N->n[0] = n_in;
    N->n[1] = width;
    N->n[2] = width;
    N->n[3] = n_out;
    int64_t o = 0;
    for (int l = 0; l < 3; ++l) {
        N->off_w[l] = o;
        o += (int64_t)N->n[l + 1] * N->n[l];
        N->off_b[l] = o;
        o += N->n[l + 1];
    }
    N->nparam = o;
    mhlp_status s;
    if ((s = malloc_dev(&N->p, o)) || (s = malloc_dev(&N->g, o)) || (s = malloc_dev(&N->m, o)) ||
        (s = malloc_dev(&N->v, o)) || (s = malloc_dev(&N->loss, 1))) {
        mhlp_mlp_destroy(N);
        return s;
    }
    zero_f32(st, N->p, o);
    zero_f32(st, N->g, o);
    zero_f32(st, N->m, o);
    zero_f32(st, N->v, o);
    for (int l = 0; l < 3; ++l) {
        const int64_t cnt = N->off_b[l] - N->off_w[l];
        init_uniform_kernel<<<nb(cnt, 256), 256, 0, st>>>(N->p, N->off_w[l], N->off_b[l],
                                                           1.0f / std::sqrt((float)N->n[l]),
                                                           seed + 0x632BE59BD9B4E019ull * (uint64_t)(l + 1));
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        mhlp_mlp_destroy(N);
        return mfail(MHLP_HIP_ERROR, std::string("mlp_create: ") + hipGetErrorString(e));
    }
    *out = N;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_mlp_info(const mhlp_mlp *N, int64_t *n_params, int32_t *sizes4)
{
    if (!N) return mfail(MHLP_INVALID_ARG, "mlp is NULL");
    if (n_params) *n_params = N->nparam;
    if (sizes4)
        for (int l = 0; l < 4; ++l) sizes4[l] = N->n[l];
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_mlp_params(mhlp_mlp *N, float *dst, const float *src, void *stream)
{
    if (!N) return mfail(MHLP_INVALID_ARG, "mlp is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (dst) MHIP(hipMemcpyAsync(dst, N->p, sizeof(float) * N->nparam, hipMemcpyDeviceToDevice, st));
    if (src) {
        MHIP(hipMemcpyAsync(N->p, src, sizeof(float) * N->nparam, hipMemcpyDeviceToDevice, st));
        zero_f32(st, N->m, N->nparam);
        zero_f32(st, N->v, N->nparam);
        N->step = 0;
    }
    MHIP(hipGetLastError());
    return MHLP_OK;
}

static mhlp_status ensure_acts(mhlp_mlp *N, int B, hipStream_t st)
{
    if (N->cap >= B) return MHLP_OK;
    MHIP(hipStreamSynchronize(st)); /* buffers may still be in use by queued work */
    free_acts(N);
    const int64_t maxw = std::max(std::max(N->n[1], N->n[2]), N->n[3]);
    mhlp_status s;
    if ((s = malloc_dev(&N->Z[0], (int64_t)B * N->n[1])) || (s = malloc_dev(&N->Z[1], (int64_t)B * N->n[2])) ||
        (s = malloc_dev(&N->Z[2], (int64_t)B * N->n[3])) || (s = malloc_dev(&N->Ac[0], (int64_t)B * N->n[1])) ||
        (s = malloc_dev(&N->Ac[1], (int64_t)B * N->n[2])) || (s = malloc_dev(&N->d0, (int64_t)B * maxw)) ||
        (s = malloc_dev(&N->d1, (int64_t)B * maxw)) || (s = malloc_dev(&N->ws, MAX_SPLITS * (int64_t)B * maxw))) {
        free_acts(N);
        return s;
    }
    N->ws_len = MAX_SPLITS * (int64_t)B * maxw;
    N->cap = B;
    return MHLP_OK;
}

/* forward pass of X [B][n0]; pre-activations Z[l] and activations Ac[l] kept */
static void forward(mhlp_mlp *N, const float *X, int B, hipStream_t st)
{
    const float *in = X;
    for (int l = 0; l < 3; ++l) {
        const int ni = N->n[l], no = N->n[l + 1];
        const int64_t sz = (int64_t)B * no;
        /* Z = in W^T:  A(b,k) = in[b*ni + k],  B(k,o) = W[o*ni + k] */
        const int sp = gemm_bf16(st, B, no, ni, in, ni, 1, N->p + N->off_w[l], 1, ni, N->ws, no, sz, true);
        bias_act_kernel<<<nb(sz, 256), 256, 0, st>>>(N->ws, sp, sz, N->p + N->off_b[l], N->Z[l],
                                                     l < 2 ? N->Ac[l] : nullptr, B, no);
        if (l < 2) in = N->Ac[l];
    }
}

extern "C" mhlp_status mhlp_mlp_forward(mhlp_mlp *N, const float *X, int32_t batch, float *Y, void *stream)
{
    if (!N || !X || !Y) return mfail(MHLP_INVALID_ARG, "NULL argument");
    if (batch < 1) return mfail(MHLP_INVALID_ARG, "batch must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    if (mhlp_status s = ensure_acts(N, batch, st)) return s;
    forward(N, X, batch, st);
    MHIP(hipMemcpyAsync(Y, N->Z[2], sizeof(float) * (size_t)batch * N->n[3], hipMemcpyDeviceToDevice, st));
    MHIP(hipGetLastError());
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_mlp_loss_grad(mhlp_mlp *N, const float *X, const float *T, int32_t batch, float *loss,
                                          float *grad, void *stream)
{
    if (!N || !X || !T) return mfail(MHLP_INVALID_ARG, "NULL argument");
    if (batch < 1) return mfail(MHLP_INVALID_ARG, "batch must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    if (mhlp_status s = ensure_acts(N, batch, st)) return s;
    const int B = batch;
    forward(N, X, B, st);
    zero_f32(st, N->loss, 1);
    const int64_t ny = (int64_t)B * N->n[3];
    mse_kernel<<<std::min<unsigned>(nb(ny, 256), 240u), 256, 0, st>>>(N->Z[2], T, N->d0, ny, N->loss);
    /* back-propagate: cur holds dL/dZ of layer l */
    float *cur = N->d0, *nxt = N->d1;
    for (int l = 2; l >= 0; --l) {
        const int ni = N->n[l], no = N->n[l + 1];
        const float *in = l > 0 ? N->Ac[l - 1] : X;
        /* dW = dZ^T in : A(o,b) = dZ[b*no + o], B(b,k) = in[b*ni + k] */
        const int64_t szw = (int64_t)no * ni;
        const bool wsplit = MAX_SPLITS * szw <= N->ws_len;
        const int spw = gemm_bf16(st, no, ni, B, cur, 1, no, in, ni, 1, wsplit ? N->ws : N->g + N->off_w[l], ni, szw,
                                  wsplit);
        if (wsplit) splitk_sum_kernel<<<nb(szw, 256), 256, 0, st>>>(N->ws, spw, szw, N->g + N->off_w[l], szw);
        colsum_kernel<<<nb(no, 256), 256, 0, st>>>(cur, N->g + N->off_b[l], B, no);
        if (l > 0) {
            /* dA = dZ W : A(b,o) = dZ[b*no + o], B(o,k) = W[o*ni + k] */
            const int64_t sza = (int64_t)B * ni;
            const int spa = gemm_bf16(st, B, ni, no, cur, no, 1, N->p + N->off_w[l], ni, 1, N->ws, ni, sza, true);
            gelu_back_kernel<<<nb(sza, 256), 256, 0, st>>>(N->Z[l - 1], N->ws, spa, sza, nxt, sza);
            std::swap(cur, nxt);
        }
    }
    if (loss) MHIP(hipMemcpyAsync(loss, N->loss, sizeof(float), hipMemcpyDeviceToDevice, st));
    if (grad) MHIP(hipMemcpyAsync(grad, N->g, sizeof(float) * N->nparam, hipMemcpyDeviceToDevice, st));
    MHIP(hipGetLastError());
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_mlp_adam_step(mhlp_mlp *N, float lr, float beta1, float beta2, float eps, void *stream)
{
    if (!N) return mfail(MHLP_INVALID_ARG, "mlp is NULL");
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return mfail(MHLP_INVALID_ARG, "bad Adam hyper-parameters");
    hipStream_t st = (hipStream_t)stream;
    N->step += 1;
    const float c1 = 1.f - (float)std::pow((double)beta1, (double)N->step);
    const float c2 = 1.f - (float)std::pow((double)beta2, (double)N->step);
    adam_kernel<<<nb(N->nparam, 256), 256, 0, st>>>(N->p, N->g, N->m, N->v, N->nparam, lr, beta1, beta2, eps, c1, c2);
    MHIP(hipGetLastError());
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_gemm_bf16(int32_t m, int32_t n, int32_t k, const float *A, int64_t sam, int64_t sak,
                                      const float *B, int64_t sbk, int64_t sbn, float *C, int64_t ldc, void *stream)
{
    if (!A || !B || !C) return mfail(MHLP_INVALID_ARG, "NULL argument");
    if (m < 1 || n < 1 || k < 1) return mfail(MHLP_INVALID_ARG, "sizes must be >= 1");
    if (ldc < n) return mfail(MHLP_INVALID_ARG, "ldc < n");
    gemm_bf16((hipStream_t)stream, m, n, k, A, sam, sak, B, sbk, sbn, C, ldc, 0, false);
    MHIP(hipGetLastError());
    return MHLP_OK;
}

/* ------------------------------------------------------------------------ */
/* Fourier analysis / synthesis of densities on each curve                   */
/* ------------------------------------------------------------------------ */
constexpr double INV_2PI = 0.15915494309189533577;

/* coef[d][(c K + k) 2 + p] for block (c K + k, d) */
__global__ __launch_bounds__(256) void fourier_analysis_kernel(const double *__restrict__ theta,
                                                               const double *__restrict__ omega,
                                                               const int64_t *__restrict__ cptr,
                                                               const double *__restrict__ mu, int64_t n, int K,
                                                               int64_t F, double *__restrict__ coef)
{
    __shared__ double red[2][256];
    const int ck = blockIdx.x, c = ck / K, k = ck % K;
    const double *md = mu + (int64_t)blockIdx.y * n;
    double re = 0.0, im = 0.0;
    for (int64_t i = cptr[c] + threadIdx.x; i < cptr[c + 1]; i += 256) {
        double s, co;
        sincos((double)k * theta[i], &s, &co);
        const double wm = omega[i] * md[i];
        re = fma(wm, co, re);
        im = fma(-wm, s, im);
    }
    red[0][threadIdx.x] = re;
    red[1][threadIdx.x] = im;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *cd = coef + (int64_t)blockIdx.y * F + 2 * (int64_t)ck;
        cd[0] = red[0][0] * INV_2PI;
        cd[1] = red[1][0] * INV_2PI;
    }
}

/* History maps of the warm start (all FP64, by value).
   H rows of history, newest last.  Network input group h (h = 0..H-1) is the
   h-th backward difference of the newest row, sum_i (-1)^i C(h,i) row[H-1-i];
   the base prediction is the order-p polynomial extrapolation
   sum_i b_i row[H-1-i], b_i = (-1)^i C(p+1, i+1) (p = 0: the newest row). */
constexpr int MAX_HIST = 8;
struct WarmMap {
    int H, p;
    double diff[MAX_HIST][MAX_HIST]; /* diff[h][i] = (-1)^i C(h, i), i <= h */
    double b[4];
    const double *rec; /* learned recurrence [F/2][H] complex (Re, Im) of each coefficient, or NULL:
                          the base is then the order-p extrapolation */
};

static WarmMap make_map(int H, int p)
{
    WarmMap w{};
    w.H = H;
    w.p = p;
    w.rec = nullptr;
    double C[MAX_HIST + 1][MAX_HIST + 1] = {};
    for (int n = 0; n <= MAX_HIST; ++n) {
        C[n][0] = 1.0;
        for (int k = 1; k <= n; ++k) C[n][k] = C[n - 1][k - 1] + (k <= n - 1 ? C[n - 1][k] : 0.0);
    }
    for (int h = 0; h < MAX_HIST; ++h)
        for (int i = 0; i <= h; ++i) w.diff[h][i] = (i % 2 ? -1.0 : 1.0) * C[h][i];
    for (int i = 0; i <= p; ++i) w.b[i] = (i % 2 ? -1.0 : 1.0) * C[p + 1][i + 1];
    return w;
}

/* out[d][m] = base_d(m) + scale * sum_k s_k (Re c_k cos k theta - Im c_k sin k theta),
   s_0 = 1, s_k = 2; coefficients of type T (FP64 or the network's FP32), scale
   read from device memory (NULL = 1); base_d(m) = sum_{i<=p} b_i
   base[d*dstride + (last - i)*n + m] (base NULL = 0). */
template <class T>
__global__ void fourier_synthesis_kernel(const double *__restrict__ theta, const int32_t *__restrict__ cid, int64_t n,
                                         int K, int64_t F, const T *__restrict__ coef,
                                         const double *__restrict__ scale, const double *__restrict__ base,
                                         int64_t dstride, int last, int p, double b0, double b1, double b2, double b3,
                                         double *__restrict__ out)
{
    const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int64_t d = blockIdx.y;
    const T *cd = coef + d * F + (int64_t)cid[m] * K * 2;
    const double th = theta[m];
    double acc = (double)cd[0];
    for (int k = 1; k < K; ++k) {
        double s, co;
        sincos((double)k * th, &s, &co);
        acc += 2.0 * ((double)cd[2 * k] * co - (double)cd[2 * k + 1] * s);
    }
    if (scale) acc *= scale[0];
    double bv = 0.0;
    if (base) {
        const double bb[4] = {b0, b1, b2, b3};
        const double *bd = base + d * dstride + m;
        for (int i = 0; i <= p; ++i) bv += bb[i] * bd[(int64_t)(last - i) * n];
    }
    out[d * n + m] = bv + acc;
}

/* ------------------------------------------------------------------------ */
/* the warm-start model                                                       */
/* ------------------------------------------------------------------------ */
struct mhlp_warm {
    int64_t n = 0;
    int n_curves = 0, K = 0, H = 0, order = 0;
    int64_t F = 0;
    WarmMap map{};
    double *theta = nullptr, *omega = nullptr;
    int32_t *cid = nullptr;
    int64_t *cptr = nullptr;
    mhlp_mlp *net = nullptr;
    double *scales = nullptr; /* device [H+1]: input group factors, output unit */
    bool recurrence = false;  /* base: learned per-coefficient recurrence (else polynomial extrapolation) */
    double *rec = nullptr;    /* device [F/2][H] complex recurrence coefficients */
    double *D = nullptr;      /* device [F] correction of one prediction */
    double *coef = nullptr;
    int64_t coef_rows = 0;
    float *X = nullptr, *T = nullptr, *Y = nullptr, *losses = nullptr;
    int64_t samp_cap = 0, loss_cap = 0;
    bool trained = false;
};

/* input groups and target of sample j, feature f (coefficient rows j..j+H) */
__device__ __forceinline__ void warm_features(const WarmMap &w, const double *__restrict__ coef, int64_t F, int64_t j,
                                              int64_t f, double *grp, double *tgt, bool with_target)
{
    const double *c = coef + j * F + f; /* c[r*F] = row j + r */
    for (int h = 0; h < w.H; ++h) {
        double v = 0.0;
        for (int i = 0; i <= h; ++i) v += w.diff[h][i] * c[(int64_t)(w.H - 1 - i) * F];
        grp[h] = v;
    }
    if (with_target) {
        double e = c[(int64_t)w.H * F];
        if (w.rec) {
            /* complex coefficient k = f / 2: e = c_next - sum_i a_i c_{next-1-i} (Re or Im part) */
            const int64_t k = f >> 1;
            const double *cc = coef + j * F + 2 * k; /* its (Re, Im) in row j */
            const double *a = w.rec + k * 2 * (int64_t)w.H;
            for (int i = 0; i < w.H; ++i) {
                const double cr = cc[(int64_t)(w.H - 1 - i) * F], ci = cc[(int64_t)(w.H - 1 - i) * F + 1];
                const double ar = a[2 * i], ai = a[2 * i + 1];
                e -= (f & 1) ? fma(ar, ci, ai * cr) : fma(ar, cr, -ai * ci);
            }
        } else {
            for (int i = 0; i <= w.p; ++i) e -= w.b[i] * c[(int64_t)(w.H - 1 - i) * F];
        }
        *tgt = e;
    }
}

/* Least-squares recurrence of each complex coefficient k over the training
   windows j < S: a = argmin sum_j |c_k(j + H) - sum_i a_i c_k(j + H - 1 - i)|^2
   + lam |a|^2 with lam = REC_LAMBDA tr(G) / H + the smallest normal number,
   G = sum_j conj(h_j) h_j^T, h_j = (c_k(j + H - 1 - i))_i; from the normal
   equations (G + lam I) a = sum_j conj(h_j) c_k(j + H) by a complex Cholesky
   factorisation, one thread per coefficient (sums in sample order). */
constexpr double REC_LAMBDA = 1e-14;
__global__ void warm_rec_fit_kernel(const double *__restrict__ coef, int64_t S, int H, int64_t F,
                                    double *__restrict__ rec)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= F / 2) return;
    double gr[MAX_HIST][MAX_HIST], gi[MAX_HIST][MAX_HIST], rr[MAX_HIST], ri[MAX_HIST];
    for (int i = 0; i < H; ++i) {
        rr[i] = ri[i] = 0.0;
        for (int l = 0; l < H; ++l) gr[i][l] = gi[i][l] = 0.0;
    }
    for (int64_t j = 0; j < S; ++j) {
        const double *c = coef + j * F + 2 * k;
        double hr[MAX_HIST], hi[MAX_HIST];
        for (int i = 0; i < H; ++i) {
            hr[i] = c[(int64_t)(H - 1 - i) * F];
            hi[i] = c[(int64_t)(H - 1 - i) * F + 1];
        }
        const double yr = c[(int64_t)H * F], yi = c[(int64_t)H * F + 1];
        for (int i = 0; i < H; ++i) {
            /* conj(h_i) h_l and conj(h_i) y */
            for (int l = 0; l < H; ++l) {
                gr[i][l] += fma(hr[i], hr[l], hi[i] * hi[l]);
                gi[i][l] += fma(hr[i], hi[l], -hi[i] * hr[l]);
            }
            rr[i] += fma(hr[i], yr, hi[i] * yi);
            ri[i] += fma(hr[i], yi, -hi[i] * yr);
        }
    }
    double tr = 0.0;
    for (int i = 0; i < H; ++i) tr += gr[i][i];
    const double lam = REC_LAMBDA * tr / H + 2.2250738585072014e-308;
    for (int i = 0; i < H; ++i) gr[i][i] += lam;
    /* G = L L^H: L lower triangular, real positive diagonal */
    for (int i = 0; i < H; ++i) {
        for (int l = 0; l <= i; ++l) {
            double sr = gr[i][l], si = gi[i][l];
            for (int m = 0; m < l; ++m) { /* - L_im conj(L_lm) */
                sr -= fma(gr[i][m], gr[l][m], gi[i][m] * gi[l][m]);
                si -= fma(gi[i][m], gr[l][m], -gr[i][m] * gi[l][m]);
            }
            if (l == i) {
                gr[i][i] = sqrt(fmax(sr, lam));
                gi[i][i] = 0.0;
            } else {
                gr[i][l] = sr / gr[l][l];
                gi[i][l] = si / gr[l][l];
            }
        }
    }
    /* L z = r, then L^H a = z */
    for (int i = 0; i < H; ++i) {
        double sr = rr[i], si = ri[i];
        for (int m = 0; m < i; ++m) {
            sr -= fma(gr[i][m], rr[m], -gi[i][m] * ri[m]);
            si -= fma(gr[i][m], ri[m], gi[i][m] * rr[m]);
        }
        rr[i] = sr / gr[i][i];
        ri[i] = si / gr[i][i];
    }
    for (int i = H - 1; i >= 0; --i) {
        double sr = rr[i], si = ri[i];
        for (int m = i + 1; m < H; ++m) { /* - conj(L_mi) a_m */
            sr -= fma(gr[m][i], rr[m], gi[m][i] * ri[m]);
            si -= fma(gr[m][i], ri[m], -gi[m][i] * rr[m]);
        }
        rr[i] = sr / gr[i][i];
        ri[i] = si / gr[i][i];
    }
    for (int i = 0; i < H; ++i) {
        rec[(k * H + i) * 2] = rr[i];
        rec[(k * H + i) * 2 + 1] = ri[i];
    }
}

/* D[f] = (recurrence prediction - order-p extrapolation of the window)[f]
   + scale * Y[f]: the correction the synthesis adds to the extrapolated
   densities (rows of coef: the window, newest last) */
__global__ void warm_combine_kernel(WarmMap w, const double *__restrict__ coef, int64_t F,
                                    const float *__restrict__ Y, const double *__restrict__ scale,
                                    double *__restrict__ D)
{
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int64_t k = f >> 1;
    const double *cc = coef + 2 * k;
    const double *a = w.rec + k * 2 * (int64_t)w.H;
    double v = 0.0;
    for (int i = 0; i < w.H; ++i) {
        const double cr = cc[(int64_t)(w.H - 1 - i) * F], ci = cc[(int64_t)(w.H - 1 - i) * F + 1];
        const double ar = a[2 * i], ai = a[2 * i + 1];
        v += (f & 1) ? fma(ar, ci, ai * cr) : fma(ar, cr, -ai * ci);
    }
    for (int i = 0; i <= w.p; ++i) v -= w.b[i] * coef[(int64_t)(w.H - 1 - i) * F + f];
    D[f] = fma(scale[0], (double)Y[f], v);
}

/* scales[h] = 1 / RMS of input group h, scales[H] = RMS of the target, over
   all samples j < S and features */
__global__ __launch_bounds__(256) void warm_scales_kernel(WarmMap w, const double *__restrict__ coef, int64_t S,
                                                          int64_t F, double *__restrict__ scales)
{
    __shared__ double red[MAX_HIST + 1][256];
    double acc[MAX_HIST + 1];
    for (int h = 0; h <= MAX_HIST; ++h) acc[h] = 0.0;
    for (int64_t i = threadIdx.x; i < S * F; i += 256) {
        double grp[MAX_HIST], tgt;
        warm_features(w, coef, F, i / F, i % F, grp, &tgt, true);
        for (int h = 0; h < w.H; ++h) acc[h] += grp[h] * grp[h];
        acc[w.H] += tgt * tgt;
    }
    for (int h = 0; h <= w.H; ++h) red[h][threadIdx.x] = acc[h];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int h = 0; h <= w.H; ++h) red[h][threadIdx.x] += red[h][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x <= w.H) {
        const int h = threadIdx.x;
        const double r = sqrt(red[h][0] / (double)(S * F));
        scales[h] = h < w.H ? (r > 0.0 ? 1.0 / r : 1.0) : (r > 0.0 ? r : 1.0);
    }
}

/* X[j][h*F + f] = group h * scales[h];  T[j][f] = target / scales[H] (T optional) */
__global__ void warm_samples_kernel(WarmMap w, const double *__restrict__ coef, int64_t n_samples, int64_t F,
                                    const double *__restrict__ scales, float *__restrict__ X, float *__restrict__ T)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_samples * F) return;
    const int64_t j = i / F, f = i % F;
    double grp[MAX_HIST], tgt = 0.0;
    warm_features(w, coef, F, j, f, grp, &tgt, T != nullptr);
    float *xj = X + j * (int64_t)w.H * F;
    for (int h = 0; h < w.H; ++h) xj[(int64_t)h * F + f] = (float)(grp[h] * scales[h]);
    if (T) T[j * F + f] = (float)(tgt / scales[w.H]);
}

extern "C" mhlp_status mhlp_warm_destroy(mhlp_warm *W)
{
    if (!W) return MHLP_OK;
    (void)hipDeviceSynchronize();
    if (W->net) mhlp_mlp_destroy(W->net);
    free_dev(W->theta);
    free_dev(W->omega);
    free_dev(W->cid);
    free_dev(W->cptr);
    free_dev(W->scales);
    free_dev(W->rec);
    free_dev(W->D);
    free_dev(W->coef);
    free_dev(W->X);
    free_dev(W->T);
    free_dev(W->Y);
    free_dev(W->losses);
    delete W;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_warm_create(const double *theta, const double *omega, const int64_t *curve_ptr,
                                        int32_t n_curves, int32_t n_modes, int32_t n_hist, int32_t base_order,
                                        int32_t width, uint64_t seed, void *stream, mhlp_warm **out)
{
    if (!out) return mfail(MHLP_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!theta || !omega || !curve_ptr) return mfail(MHLP_INVALID_ARG, "NULL argument");
    if (n_curves < 1 || n_modes < 1 || n_hist < 1 || width < 1)
        return mfail(MHLP_INVALID_ARG, "n_curves, n_modes, n_hist and width must be >= 1");
    if (n_hist > MAX_HIST) return mfail(MHLP_INVALID_ARG, "n_hist > 8");
    if (base_order < -1 || base_order > 3 || base_order >= n_hist)
        return mfail(MHLP_INVALID_ARG, "base_order must be -1 (learned recurrence) or in [0, min(3, n_hist - 1)]");
    if ((int64_t)n_curves * n_modes > 65535) return mfail(MHLP_INVALID_ARG, "n_curves * n_modes > 65535");
    if (curve_ptr[0] != 0) return mfail(MHLP_INVALID_ARG, "curve_ptr[0] must be 0");
    for (int c = 0; c < n_curves; ++c)
        if (curve_ptr[c + 1] <= curve_ptr[c]) return mfail(MHLP_INVALID_ARG, "curve_ptr must be strictly increasing");
    const int64_t n = curve_ptr[n_curves];
    const int64_t F = 2LL * n_modes * n_curves;
    if (F * n_hist > (int64_t)1 << 24) return mfail(MHLP_INVALID_ARG, "feature vector too long");
    hipStream_t st = (hipStream_t)stream;
    mhlp_warm *W = new mhlp_warm();
    W->n = n;
    W->n_curves = n_curves;
    W->K = n_modes;
    W->H = n_hist;
    W->recurrence = base_order < 0;
    /* the densities beyond the modes follow the polynomial extrapolation:
       with the recurrence base, the cubic one (or the highest the history allows) */
    W->order = base_order < 0 ? std::min(3, n_hist - 1) : base_order;
    W->map = make_map(n_hist, W->order);
    W->F = F;
    std::vector<int32_t> cid(n);
    for (int c = 0; c < n_curves; ++c)
        for (int64_t i = curve_ptr[c]; i < curve_ptr[c + 1]; ++i) cid[i] = c;
    mhlp_status s;
    if ((s = malloc_dev(&W->theta, n)) || (s = malloc_dev(&W->omega, n)) || (s = malloc_dev(&W->cid, n)) ||
        (s = malloc_dev(&W->cptr, n_curves + 1)) || (s = malloc_dev(&W->scales, n_hist + 1)) ||
        (s = malloc_dev(&W->Y, F)) || (s = malloc_dev(&W->D, F)) ||
        (W->recurrence && (s = malloc_dev(&W->rec, F * n_hist)))) {
        mhlp_warm_destroy(W);
        return s;
    }
    hipError_t e = hipMemcpyAsync(W->theta, theta, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(W->omega, omega, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(W->cid, cid.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(W->cptr, curve_ptr, sizeof(int64_t) * (n_curves + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        mhlp_warm_destroy(W);
        return mfail(MHLP_HIP_ERROR, std::string("warm_create: ") + hipGetErrorString(e));
    }
    if ((s = mhlp_mlp_create((int32_t)(F * n_hist), width, (int32_t)F, seed, stream, &W->net))) {
        mhlp_warm_destroy(W);
        return s;
    }
    *out = W;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_warm_info(const mhlp_warm *W, int64_t *n_nodes, int64_t *n_features, mhlp_mlp **net,
                                      double *scales)
{
    if (!W) return mfail(MHLP_INVALID_ARG, "warm model is NULL");
    if (n_nodes) *n_nodes = W->n;
    if (n_features) *n_features = W->F;
    if (net) *net = W->net;
    if (scales) MHIP(hipMemcpy(scales, W->scales, (W->H + 1) * sizeof(double), hipMemcpyDeviceToHost));
    return MHLP_OK;
}

static mhlp_status ensure_coef(mhlp_warm *W, int64_t rows, hipStream_t st)
{
    if (W->coef_rows >= rows) return MHLP_OK;
    MHIP(hipStreamSynchronize(st));
    free_dev(W->coef);
    W->coef_rows = 0;
    if (mhlp_status s = malloc_dev(&W->coef, rows * W->F)) return s;
    W->coef_rows = rows;
    return MHLP_OK;
}

static void analysis(const mhlp_warm *W, const double *mu, int d, double *coef, hipStream_t st)
{
    dim3 grid((unsigned)(W->n_curves * W->K), (unsigned)d);
    fourier_analysis_kernel<<<grid, 256, 0, st>>>(W->theta, W->omega, W->cptr, mu, W->n, W->K, W->F, coef);
}

extern "C" mhlp_status mhlp_warm_coefficients(const mhlp_warm *W, const double *mu, int32_t n_dens, double *coef,
                                              void *stream)
{
    if (!W || !mu || !coef) return mfail(MHLP_INVALID_ARG, "NULL argument");
    if (n_dens < 1 || n_dens > 65535) return mfail(MHLP_INVALID_ARG, "n_dens must be in [1, 65535]");
    analysis(W, mu, n_dens, coef, (hipStream_t)stream);
    MHIP(hipGetLastError());
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_warm_synthesize(const mhlp_warm *W, const double *coef, int32_t n_dens,
                                            const double *base, double *out, void *stream)
{
    if (!W || !coef || !out) return mfail(MHLP_INVALID_ARG, "NULL argument");
    if (n_dens < 1 || n_dens > 65535) return mfail(MHLP_INVALID_ARG, "n_dens must be in [1, 65535]");
    dim3 grid(nb(W->n, 256), (unsigned)n_dens);
    fourier_synthesis_kernel<double><<<grid, 256, 0, (hipStream_t)stream>>>(
        W->theta, W->cid, W->n, W->K, W->F, coef, nullptr, base, W->n, 0, 0, 1.0, 0.0, 0.0, 0.0, out);
    MHIP(hipGetLastError());
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_warm_train(mhlp_warm *W, const double *mus, int32_t n_steps, int32_t iters, float lr,
                                       float *losses, void *stream)
{
    if (!W || !mus) return mfail(MHLP_INVALID_ARG, "NULL argument");
    if (n_steps < W->H + 1 || n_steps > 65535)
        return mfail(MHLP_INVALID_ARG, "n_steps must be in [n_hist + 1, 65535]");
    if (iters < 0) return mfail(MHLP_INVALID_ARG, "iters must be >= 0");
    if (!(lr > 0.f)) return mfail(MHLP_INVALID_ARG, "lr must be > 0");
    hipStream_t st = (hipStream_t)stream;
    const int64_t S = n_steps - W->H;
    if (mhlp_status s = ensure_coef(W, n_steps, st)) return s;
    if (W->samp_cap < S) {
        MHIP(hipStreamSynchronize(st));
        free_dev(W->X);
        free_dev(W->T);
        W->samp_cap = 0;
        mhlp_status s;
        if ((s = malloc_dev(&W->X, S * W->H * W->F)) || (s = malloc_dev(&W->T, S * W->F))) return s;
        W->samp_cap = S;
    }
    const int64_t lc = std::max<int64_t>(iters, 1);
    if (W->loss_cap < lc) {
        MHIP(hipStreamSynchronize(st));
        free_dev(W->losses);
        W->loss_cap = 0;
        if (mhlp_status s = malloc_dev(&W->losses, lc)) return s;
        W->loss_cap = lc;
    }
    analysis(W, mus, n_steps, W->coef, st);
    if (W->recurrence) {
        warm_rec_fit_kernel<<<nb(W->F / 2, 64), 64, 0, st>>>(W->coef, S, W->H, W->F, W->rec);
        W->map.rec = W->rec;
    }
    warm_scales_kernel<<<1, 256, 0, st>>>(W->map, W->coef, S, W->F, W->scales);
    warm_samples_kernel<<<nb(S * W->F, 256), 256, 0, st>>>(W->map, W->coef, S, W->F, W->scales, W->X, W->T);
    MHIP(hipGetLastError());
    for (int it = 0; it < iters; ++it) {
        if (mhlp_status s = mhlp_mlp_loss_grad(W->net, W->X, W->T, (int32_t)S, W->losses + it, nullptr, stream))
            return s;
        if (mhlp_status s = mhlp_mlp_adam_step(W->net, lr, 0.9f, 0.999f, 1e-8f, stream)) return s;
    }
    if (losses && iters > 0)
        MHIP(hipMemcpyAsync(losses, W->losses, sizeof(float) * iters, hipMemcpyDeviceToHost, st));
    MHIP(hipStreamSynchronize(st));
    W->trained = true;
    return MHLP_OK;
}

extern "C" mhlp_status mhlp_warm_predict(mhlp_warm *W, const double *hist, double *x0, void *stream)
{
    if (!W || !hist || !x0) return mfail(MHLP_INVALID_ARG, "NULL argument");
    if (!W->trained) return mfail(MHLP_INVALID_ARG, "warm model has not been trained");
    hipStream_t st = (hipStream_t)stream;
    if (mhlp_status s = ensure_coef(W, W->H, st)) return s;
    analysis(W, hist, W->H, W->coef, st);
    warm_samples_kernel<<<nb(W->F, 256), 256, 0, st>>>(W->map, W->coef, 1, W->F, W->scales, W->X, nullptr);
    if (mhlp_status s = mhlp_mlp_forward(W->net, W->X, 1, W->Y, stream)) return s;
    dim3 grid(nb(W->n, 256), 1);
    const WarmMap &w = W->map;
    if (W->recurrence) {
        warm_combine_kernel<<<nb(W->F, 256), 256, 0, st>>>(w, W->coef, W->F, W->Y, W->scales + W->H, W->D);
        fourier_synthesis_kernel<double><<<grid, 256, 0, st>>>(W->theta, W->cid, W->n, W->K, W->F, W->D, nullptr,
                                                               hist, 0, W->H - 1, w.p, w.b[0], w.b[1], w.b[2], w.b[3],
                                                               x0);
    } else {
        fourier_synthesis_kernel<float><<<grid, 256, 0, st>>>(W->theta, W->cid, W->n, W->K, W->F, W->Y,
                                                              W->scales + W->H, hist, 0, W->H - 1, w.p, w.b[0],
                                                              w.b[1], w.b[2], w.b[3], x0);
    }
    MHIP(hipGetLastError());
    return MHLP_OK;
}
