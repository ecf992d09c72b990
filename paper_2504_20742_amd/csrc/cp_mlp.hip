// cp_mlp.hip -- BF16 MFMA multilayer perceptron (forward, backward, Adam) for the
// learned phase-change source surrogate, gfx950.
//
// Network: n_in -> n_h -> n_h -> n_out, GELU (tanh form) after both hidden layers,
// mean-squared-error loss.  Weights and activations are bfloat16, products are
// accumulated in FP32 on the matrix cores (v_mfma_f32_16x16x16_bf16 in the training
// GEMM, v_mfma_f32_16x16x32_bf16 in the fused inference), master weights and Adam
// moments are FP32.  Parameters are flat in the order
// W1 [n_in][n_h], b1, W2 [n_h][n_h], b2, W3 [n_h][n_out], b3.
//
// One strided GEMM kernel serves every product of the forward and backward pass:
// C[M][N] = sum_k A(m, k) B(k, n) with A(m, k) = A[m*sam + k*sak] and
// B(k, n) = B[k*sbk + n*sbn], so transposed operands need no copies.  A 64 x 64
// output tile per 256-thread workgroup: the 64 x 16 A slab and 16 x 64 B slab of
// each K step are staged in LDS, each of the four waves owns 16 rows and issues
// four 16x16x16 MFMAs per step.  Long reductions (weight gradients over the
// batch) split K over blockIdx.z into FP32 partial tiles reduced in order.
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/contrail.h"
#include "cp_fused_net.hpp"
#include "cp_internal.hpp"

namespace cp {

typedef short bf16x4 __attribute__((ext_vector_type(4)));

// round to nearest even (the hardware conversion on gfx950)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ float gelu_grad_f(float z)
{
    // d/dz [z s(2u)] = s + 2 z s (1 - s) u'(z),  u' = sqrt(2/pi) (1 + 3 * 0.044715 z^2)
    const float sg = gelu_sig(z);
    return sg + 2.0f * z * sg * (1.0f - sg) * kGeluC * (1.0f + 3.0f * 0.044715f * z * z);
}

enum { EPI_BIAS = 0, EPI_BIAS_GELU = 1, EPI_DGELU = 2, EPI_PARTIAL = 3 };

struct GemmArgs {
    const uint16_t *A, *B;
    long sam, sak, sbk, sbn;
    int M, N, K;
    const int *M_dev;          // if set, rows beyond min(*M_dev, M) are skipped
    int kchunk;                // K range per blockIdx.z
    const float *bias;         // [N] (EPI_BIAS, EPI_BIAS_GELU)
    float *Cf;                 // fp32 output [M][ldc] (bias: pre-activation; partial: [z][M][ldc])
    uint16_t *Hb;              // bf16 output [M][ldh]: GELU(C) or C * GELU'(Zs)
    const float *Zs;           // saved pre-activation for EPI_DGELU [M][ldz]
    long ldc, ldh, ldz;
};

template <int EPI> __global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g)
{
    __shared__ uint16_t As[64][16 + 4];
    __shared__ uint16_t Bs[16][64 + 4];
    const int M = g.M_dev ? min(*g.M_dev, g.M) : g.M;
    const int n0 = blockIdx.y * 64;
    const int k_begin = blockIdx.z * g.kchunk, k_end = min(g.K, k_begin + g.kchunk);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // grid-stride over 64-row tiles: the row count may only be known on the device
    for (int m0 = blockIdx.x * 64; m0 < M; m0 += gridDim.x * 64) {
    f32x4 acc[4];
    #pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = k_begin; k0 < k_end; k0 += 16) {
        #pragma unroll
        for (int r = 0; r < 4; ++r) {   // A slab 64 x 16 and B slab 16 x 64, 4 elements per thread each
            const int e = tid + 256 * r;
            const int am = e >> 4, ak = e & 15;
            const int gm = m0 + am, gk = k0 + ak;
            As[am][ak] = (gm < M && gk < k_end) ? g.A[gm * g.sam + gk * g.sak] : (uint16_t)0;
            const int bk = e >> 6, bn = e & 63;
            const int hk = k0 + bk, hn = n0 + bn;
            Bs[bk][bn] = (hk < k_end && hn < g.N) ? g.B[hk * g.sbk + hn * g.sbn] : (uint16_t)0;
        }
        __syncthreads();
        // A operand: row 16*wave + lane%16, k = 4*(lane/16) .. +3
        bf16x4 a;
        const int ar = 16 * wave + (lane & 15), ak = 4 * (lane >> 4);
        #pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = (short)As[ar][ak + i];
        #pragma unroll
        for (int c = 0; c < 4; ++c) {
            bf16x4 b;
            const int bn = 16 * c + (lane & 15);
            #pragma unroll
            for (int i = 0; i < 4; ++i) b[i] = (short)Bs[ak + i][bn];
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[c], 0, 0, 0);
        }
        __syncthreads();
    }
    // D layout: lane holds rows 4*(lane/16) + i, column lane % 16 of each 16x16 tile
    #pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int n = n0 + 16 * c + (lane & 15);
        #pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + 16 * wave + 4 * (lane >> 4) + i;
            if (m >= M || n >= g.N) continue;
            const float v = acc[c][i];
            if (EPI == EPI_PARTIAL) {
                g.Cf[((long)blockIdx.z * g.M + m) * g.ldc + n] = v;
            } else if (EPI == EPI_DGELU) {
                g.Hb[m * g.ldh + n] = f2bf(v * gelu_grad_f(g.Zs[m * g.ldz + n]));
            } else {
                const float z = v + (g.bias ? g.bias[n] : 0.f);
                if (g.Cf) g.Cf[m * g.ldc + n] = z;   // pre-activation kept for training only
                if (EPI == EPI_BIAS_GELU) g.Hb[m * g.ldh + n] = f2bf(gelu_f(z));
            }
        }
    }
    }
}

// sum of the split-K partial tiles, in split order (deterministic)
__global__ void __launch_bounds__(256) k_reduce_splits(const float *part, int splits, long mn, float *out)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= mn) return;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[z * mn + e];
    out[e] = s;
}

// column sums of a bf16 matrix [M][N] (bias gradients), one column per thread
// block, rows in a fixed order
__global__ void __launch_bounds__(256) k_colsum_bf16(const uint16_t *D, int M, int N, long ld, float *out)
{
    const int n = blockIdx.x;
    float s = 0.f;
    for (int m = threadIdx.x; m < M; m += blockDim.x) s += bf2f(D[m * ld + n]);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ float part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[n] = part[0] + part[1] + part[2] + part[3];
}

__global__ void __launch_bounds__(256) k_to_bf16(const float *x, long n, uint16_t *y)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] = f2bf(x[e]);
}

// MSE loss: dY = 2 (Y - T) / (M N) in bf16, block partial sums of (Y - T)^2
__global__ void __launch_bounds__(256) k_mse(const float *Y, const float *T, long n, float scale, uint16_t *dY,
                                             float *partial)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    float s = 0.f;
    if (e < n) {
        const float d = Y[e] - T[e];
        dY[e] = f2bf(2.0f * d * scale);
        s = d * d;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ float part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Adam on the FP32 master parameters; refreshes the bf16 copies
__global__ void __launch_bounds__(256) k_adam(float *p, float *m, float *v, const float *g, long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2, uint16_t *pb)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float pe = p[e] - lr * (me * c1) / (sqrtf(ve * c2) + eps);
    p[e] = pe;
    pb[e] = f2bf(pe);
}

// ---------------------------------------------------------------- fused inference
// Weights repacked in B-fragment order: fragment (kb, nb) of W[K][N] holds, for lane l
// and i = 0..7, W[32 kb + 8 (l / 16) + i][16 nb + l % 16] (zero beyond K, N), 512 bf16
// in a row, fragments ordered kb-major.  Each lane fetches its B operand with one
// 16-byte load and a wavefront reads 1 KB contiguous.
__global__ void __launch_bounds__(256) k_pack_frag(const uint16_t *W, int K, int N, int KB, int NB, uint16_t *dst)
{
    const long total = (long)KB * NB * 512;   // KB x NB fragments, zero beyond K, N
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long f = e >> 9;
        const int r = (int)(e & 511), lane = r >> 3, i = r & 7;
        const int kb = (int)(f / NB), nb = (int)(f % NB);
        const int k = 32 * kb + 8 * (lane >> 4) + i, n = 16 * nb + (lane & 15);
        dst[e] = (k < K && n < N) ? W[(long)k * N + n] : (uint16_t)0;
    }
}

// Biases of the fused kernel: b1 (256), b2 (256), b3 (n_out) zero-padded to 16.
__global__ void __launch_bounds__(256) k_pack_bias(const float *b1, const float *b2, const float *b3, int n_out,
                                                   float *dst)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 528) return;
    dst[e] = e < 256 ? b1[e] : e < 512 ? b2[e - 256] : (e - 512 < n_out ? b3[e - 512] : 0.f);
}

// All three layers for 64-row tiles in one launch (fused_net_tile): rows past the
// device-side count are skipped; the workgroups stride over the row tiles.
__global__ void __launch_bounds__(256, 2) k_mlp_fused(const uint16_t *X, int n_in, int n_out, const int *M_dev, int M_max,
                                                   FusedNet w, float *Y)
{
    __shared__ FusedXTile Xs;
    __shared__ FusedHTile Hs;
    const int M = M_dev ? min(*M_dev, M_max) : M_max;
    if (blockIdx.x * 64 >= M) return;   // no row for this workgroup
    for (int m0 = blockIdx.x * 64; m0 < M; m0 += gridDim.x * 64) {
        for (int e = threadIdx.x; e < 64 * kFusedKin; e += 256) {
            const int r = e / kFusedKin, k = e % kFusedKin, m = m0 + r;
            Xs[r][k] = (m < M && k < n_in) ? X[(long)m * n_in + k] : (uint16_t)0;
        }
        __syncthreads();
        fused_net_tile(w, Xs, Hs, M - m0, n_out, Y + (long)m0 * n_out);
    }
}

}  // namespace cp

using namespace cp;

struct cp_mlp {
    int n_in = 0, n_h = 0, n_out = 0;
    long np = 0;
    long off[7] = {};            // offsets of W1, b1, W2, b2, W3, b3, end
    hipStream_t stream = nullptr;
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;   // fp32 master, Adam, gradient
    uint16_t *pb = nullptr;      // bf16 parameters
    int adam_t = 0;
    // activation buffers for batches of up to cap rows
    long cap = 0;
    uint16_t *Xb = nullptr, *H1 = nullptr, *H2 = nullptr, *dY = nullptr, *dZ2 = nullptr, *dZ1 = nullptr;
    float *Z1 = nullptr, *Z2 = nullptr, *Yf = nullptr, *part = nullptr, *lossp = nullptr;
    long part_cap = 0;
    uint16_t *fw = nullptr;      // weights packed for the fused inference kernel
    float *fb = nullptr;
    bool fused_stale = true;     // set whenever the parameters change
    std::vector<void *> allocs;
    std::string err;
};

namespace {

int mfail(cp_mlp *n, int code, const std::string &s)
{
    if (n) n->err = s;
    return code;
}

template <class T> T *malloc_dev(cp_mlp *n, size_t k)
{
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(k, 1) * sizeof(T)) != hipSuccess) return nullptr;
    n->allocs.push_back(p);
    return (T *)p;
}

int ensure_cap(cp_mlp *n, long rows)
{
    if (rows <= n->cap) return CP_OK;
    for (void *q : {(void *)n->Xb, (void *)n->H1, (void *)n->H2, (void *)n->dY, (void *)n->dZ2, (void *)n->dZ1,
                    (void *)n->Z1, (void *)n->Z2, (void *)n->Yf, (void *)n->lossp}) {
        if (!q) continue;
        hipFree(q);
        n->allocs.erase(std::find(n->allocs.begin(), n->allocs.end(), q));
    }
    const long c = std::max<long>(rows, 4096);
    n->Xb = malloc_dev<uint16_t>(n, c * n->n_in);
    n->H1 = malloc_dev<uint16_t>(n, c * n->n_h);
    n->H2 = malloc_dev<uint16_t>(n, c * n->n_h);
    n->dY = malloc_dev<uint16_t>(n, c * n->n_out);
    n->dZ2 = malloc_dev<uint16_t>(n, c * n->n_h);
    n->dZ1 = malloc_dev<uint16_t>(n, c * n->n_h);
    n->Z1 = malloc_dev<float>(n, c * n->n_h);
    n->Z2 = malloc_dev<float>(n, c * n->n_h);
    n->Yf = malloc_dev<float>(n, c * n->n_out);
    n->lossp = malloc_dev<float>(n, (c * n->n_out + 255) / 256);
    if (!n->Xb || !n->H1 || !n->H2 || !n->dY || !n->dZ2 || !n->dZ1 || !n->Z1 || !n->Z2 || !n->Yf || !n->lossp)
        return mfail(n, CP_ENOMEM, "activation buffers");
    n->cap = c;
    return CP_OK;
}

template <int EPI>
hipError_t gemm(const GemmArgs &a, int splits, hipStream_t s)
{
    dim3 grid((unsigned)std::min(512, (a.M + 63) / 64), (a.N + 63) / 64, splits);
    hipLaunchKernelGGL((k_gemm_bf16<EPI>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

GemmArgs gargs(const uint16_t *A, long sam, long sak, const uint16_t *B, long sbk, long sbn, int M, int N, int K)
{
    GemmArgs a{};
    a.A = A;
    a.B = B;
    a.sam = sam;
    a.sak = sak;
    a.sbk = sbk;
    a.sbn = sbn;
    a.M = M;
    a.N = N;
    a.K = K;
    a.kchunk = ((K + 15) / 16) * 16;
    return a;
}

// Activation buffers of one forward pass (Z1, Z2 nullable: inference keeps no
// pre-activations).
struct FwdBufs {
    const uint16_t *X;
    uint16_t *H1, *H2;
    float *Z1, *Z2, *Y;
};

// Forward pass on `rows` rows of b.X; M_dev (nullable) caps the rows on the device.
int forward_rows(cp_mlp *n, int rows, const int *M_dev, const FwdBufs &b, hipStream_t s)
{
    const uint16_t *W1 = n->pb + n->off[0], *W2 = n->pb + n->off[2], *W3 = n->pb + n->off[4];
    const float *b1 = n->p + n->off[1], *b2 = n->p + n->off[3], *b3 = n->p + n->off[5];
    GemmArgs a = gargs(b.X, n->n_in, 1, W1, n->n_h, 1, rows, n->n_h, n->n_in);
    a.M_dev = M_dev;
    a.bias = b1;
    a.Cf = b.Z1;
    a.ldc = n->n_h;
    a.Hb = b.H1;
    a.ldh = n->n_h;
    if (gemm<EPI_BIAS_GELU>(a, 1, s) != hipSuccess) return mfail(n, CP_EHIP, "gemm 1");
    a = gargs(b.H1, n->n_h, 1, W2, n->n_h, 1, rows, n->n_h, n->n_h);
    a.M_dev = M_dev;
    a.bias = b2;
    a.Cf = b.Z2;
    a.ldc = n->n_h;
    a.Hb = b.H2;
    a.ldh = n->n_h;
    if (gemm<EPI_BIAS_GELU>(a, 1, s) != hipSuccess) return mfail(n, CP_EHIP, "gemm 2");
    a = gargs(b.H2, n->n_h, 1, W3, n->n_out, 1, rows, n->n_out, n->n_h);
    a.M_dev = M_dev;
    a.bias = b3;
    a.Cf = b.Y;
    a.ldc = n->n_out;
    if (gemm<EPI_BIAS>(a, 1, s) != hipSuccess) return mfail(n, CP_EHIP, "gemm 3");
    return CP_OK;
}

int forward_rows(cp_mlp *n, int rows, hipStream_t s)
{
    return forward_rows(n, rows, nullptr, FwdBufs{n->Xb, n->H1, n->H2, n->Z1, n->Z2, n->Yf}, s);
}

// weight gradient dW[K_in][N_out] = A^T dZ over `rows` rows, split over the batch
int weight_grad(cp_mlp *n, const uint16_t *Aact, int kin, const uint16_t *dZ, int nout, int rows, float *dW,
                hipStream_t s)
{
    const int splits = std::max(1, std::min(64, rows / 512));
    const int chunk = (((rows + splits - 1) / splits + 15) / 16) * 16;
    const long mn = (long)kin * nout;
    if (splits * mn > n->part_cap) {
        if (n->part) {
            hipFree(n->part);
            n->allocs.erase(std::find(n->allocs.begin(), n->allocs.end(), (void *)n->part));
        }
        n->part = malloc_dev<float>(n, splits * mn);
        if (!n->part) return mfail(n, CP_ENOMEM, "partials");
        n->part_cap = splits * mn;
    }
    // C(m = input feature, nn = output) = sum_r A[r][m] dZ[r][nn]
    GemmArgs a = gargs(Aact, 1, kin, dZ, nout, 1, kin, nout, rows);
    a.kchunk = chunk;
    a.Cf = n->part;
    a.ldc = nout;
    if (gemm<EPI_PARTIAL>(a, splits, s) != hipSuccess) return mfail(n, CP_EHIP, "weight grad");
    hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, n->part, splits, mn, dW);
    return hipGetLastError() == hipSuccess ? CP_OK : mfail(n, CP_EHIP, "reduce");
}

}  // namespace

namespace cp {
bool mlp_fusable(const cp_mlp *n) { return n->n_in <= kFusedKin && n->n_h == kFusedNH && n->n_out <= 16; }

// Weights and biases of a fusable network packed for k_mlp_fused (kernels only, no
// allocation, no memset).
int pack_fused(cp_mlp *n, uint16_t *w, float *b, hipStream_t s)
{
    constexpr int NB = kFusedNH / 16, KB = kFusedNH / 32;
    hipLaunchKernelGGL(k_pack_frag, dim3(32), dim3(256), 0, s, n->pb + n->off[0], n->n_in, n->n_h, kFusedKin / 32, NB,
                       w);
    hipLaunchKernelGGL(k_pack_frag, dim3(256), dim3(256), 0, s, n->pb + n->off[2], n->n_h, n->n_h, KB, NB, w + kFusedW1);
    hipLaunchKernelGGL(k_pack_frag, dim3(16), dim3(256), 0, s, n->pb + n->off[4], n->n_h, n->n_out, KB, 1,
                       w + kFusedW1 + kFusedW2);
    hipLaunchKernelGGL(k_pack_bias, dim3(3), dim3(256), 0, s, n->p + n->off[1], n->p + n->off[3], n->p + n->off[5],
                       n->n_out, b);
    if (hipGetLastError() != hipSuccess) return mfail(n, CP_EHIP, "weight packing");
    return CP_OK;
}

int mlp_snapshot(cp_mlp *n, uint16_t *w, float *b, hipStream_t s)
{
    if (!mlp_fusable(n)) return CP_EUNSUPPORTED;
    // the network's own stream may still be updating the weights
    if (s != n->stream && hipStreamSynchronize(n->stream) != hipSuccess) return mfail(n, CP_EHIP, "sync");
    return pack_fused(n, w, b, s);
}

// Workgroups of k_mlp_fused that the device holds at once (CUs x resident blocks per
// CU): the launch uses no more, since the workgroups stride over the row tiles and a
// second round of workgroups would run on a mostly idle device.  Queried once.
static int fused_resident_blocks()
{
    static const int n = [] {
        int dev = 0, cus = 256, per_cu = 2;
        if (hipGetDevice(&dev) == hipSuccess) {
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mlp_fused, 256, 0) != hipSuccess) per_cu = 2;
        }
        return std::max(1, cus) * std::max(1, per_cu);
    }();
    return n;
}

hipError_t mlp_fused_forward(const FusedNet &w, const uint16_t *X, int n_in, int n_out, const int *rows_dev,
                             int max_rows, float *Y, hipStream_t s)
{
    const int blocks = std::max(1, std::min((max_rows + 63) / 64, fused_resident_blocks()));
    hipLaunchKernelGGL(k_mlp_fused, dim3(blocks), dim3(256), 0, s, X, n_in, n_out, rows_dev, max_rows, w, Y);
    return hipGetLastError();
}
void mlp_dims(const cp_mlp *n, int *n_in, int *n_out)
{
    *n_in = n->n_in;
    *n_out = n->n_out;
}
}  // namespace cp

// ------------------------------------------------ inference without allocation
// cp_mlp_forward_static keeps everything a call needs beyond its inputs and outputs
// -- the packed weights, the biases and the bf16 copy of the input rows -- in this
// device array.  Each GPU holds its own copy for the life of the process; every call
// on a GPU shares it, so calls that overlap on one GPU race.  Host code reaches the
// array only through the address hipGetSymbolAddress returns on that device.
constexpr int kStaticRows = 65536;                                            // rows per call, at most
constexpr size_t kStaticBOff = (size_t)(kFusedW1 + kFusedW2 + kFusedW3) * 2;  // packed weights first
constexpr size_t kStaticXOff = kStaticBOff + 2304;                            // 528 biases, 256-aligned
constexpr size_t kStaticBytes = kStaticXOff + (size_t)kStaticRows * kFusedKin * 2;
static_assert(kStaticBOff % 256 == 0 && kStaticXOff % 256 == 0, "scratch sections stay 256-byte aligned");
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_dev[kMaxDevices] = {};   // device address of `scratch`, per device

// Device address of the scratch array on the current device, looked up once per device.
int static_scratch(cp_mlp *n, unsigned char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return mfail(n, CP_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return mfail(n, CP_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return mfail(n, CP_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = (unsigned char *)ptr;
    }
    *out = g_scratch_dev[dev];
    return CP_OK;
}
}  // namespace

extern "C" {

int cp_mlp_forward_static(cp_mlp *n, const float *X, int rows, float *Y)
{
    if (!n || !X || !Y) return CP_EINVAL;
    if (rows < 1 || rows > kStaticRows)
        return mfail(n, CP_EINVAL, "cp_mlp_forward_static: rows must be in [1, " + std::to_string(kStaticRows) + "]");
    if (!mlp_fusable(n))
        return mfail(n, CP_EUNSUPPORTED, "cp_mlp_forward_static: needs n_in <= 32, 256 hidden units, n_out <= 16");
    unsigned char *sp = nullptr;
    int r = static_scratch(n, &sp);
    if (r) return r;
    uint16_t *w = (uint16_t *)sp;
    float *b = (float *)(sp + kStaticBOff);
    uint16_t *xb = (uint16_t *)(sp + kStaticXOff);
    const long nx = (long)rows * n->n_in;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, n->stream, X, nx, xb);
    if ((r = pack_fused(n, w, b, n->stream))) return r;
    const FusedNet fw{w, w + kFusedW1, w + kFusedW1 + kFusedW2, b, b + 256, b + 512};
    if (mlp_fused_forward(fw, xb, n->n_in, n->n_out, nullptr, rows, Y, n->stream) != hipSuccess)
        return mfail(n, CP_EHIP, "fused forward");
    return CP_OK;
}

int cp_mlp_create(int n_in, int n_hidden, int n_out, void *hip_stream, cp_mlp **out)
{
    if (!out || n_in < 1 || n_hidden < 1 || n_out < 1) return CP_EINVAL;
    cp_mlp *n = new cp_mlp();
    n->n_in = n_in;
    n->n_h = n_hidden;
    n->n_out = n_out;
    n->stream = (hipStream_t)hip_stream;
    const long sz[6] = {(long)n_in * n_hidden, n_hidden, (long)n_hidden * n_hidden, n_hidden, (long)n_hidden * n_out,
                        n_out};
    for (int k = 0; k < 6; ++k) n->off[k + 1] = n->off[k] + sz[k];
    n->np = n->off[6];
    n->p = malloc_dev<float>(n, n->np);
    n->m = malloc_dev<float>(n, n->np);
    n->v = malloc_dev<float>(n, n->np);
    n->g = malloc_dev<float>(n, n->np);
    n->pb = malloc_dev<uint16_t>(n, n->np);
    if (!n->p || !n->m || !n->v || !n->g || !n->pb) {
        cp_mlp_destroy(n);
        return CP_ENOMEM;
    }
    if (hipMemset(n->p, 0, n->np * 4) != hipSuccess || hipMemset(n->m, 0, n->np * 4) != hipSuccess ||
        hipMemset(n->v, 0, n->np * 4) != hipSuccess || hipMemset(n->pb, 0, n->np * 2) != hipSuccess) {
        cp_mlp_destroy(n);
        return CP_EHIP;
    }
    *out = n;
    return CP_OK;
}

void cp_mlp_destroy(cp_mlp *n)
{
    if (!n) return;
    if (n->stream) hipStreamSynchronize(n->stream);
    else hipDeviceSynchronize();
    for (void *q : n->allocs)
        if (q) hipFree(q);
    delete n;
}

long cp_mlp_num_params(const cp_mlp *n) { return n ? n->np : 0; }

int cp_mlp_set_params(cp_mlp *n, const float *host)
{
    if (!n || !host) return CP_EINVAL;
    if (hipMemcpyAsync(n->p, host, n->np * 4, hipMemcpyHostToDevice, n->stream) != hipSuccess)
        return mfail(n, CP_EHIP, "param upload");
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n->np + 255) / 256)), dim3(256), 0, n->stream, n->p, n->np, n->pb);
    if (hipMemsetAsync(n->m, 0, n->np * 4, n->stream) != hipSuccess ||
        hipMemsetAsync(n->v, 0, n->np * 4, n->stream) != hipSuccess)
        return mfail(n, CP_EHIP, "adam reset");
    n->adam_t = 0;
    n->fused_stale = true;
    return hipStreamSynchronize(n->stream) == hipSuccess ? CP_OK : mfail(n, CP_EHIP, "sync");
}

int cp_mlp_get_params(cp_mlp *n, float *host)
{
    if (!n || !host) return CP_EINVAL;
    if (hipMemcpyAsync(host, n->p, n->np * 4, hipMemcpyDeviceToHost, n->stream) != hipSuccess ||
        hipStreamSynchronize(n->stream) != hipSuccess)
        return mfail(n, CP_EHIP, "param download");
    return CP_OK;
}

int cp_mlp_forward(cp_mlp *n, const float *X, int rows, float *Y)
{
    if (!n || !X || !Y || rows < 1) return CP_EINVAL;
    int r = ensure_cap(n, rows);
    if (r) return r;
    const long nx = (long)rows * n->n_in;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, n->stream, X, nx, n->Xb);
    if (mlp_fusable(n)) {   // inference shape: all layers in one kernel
        if (!n->fw) {
            n->fw = malloc_dev<uint16_t>(n, kFusedW1 + kFusedW2 + kFusedW3);
            n->fb = malloc_dev<float>(n, 528);
            if (!n->fw || !n->fb) return mfail(n, CP_ENOMEM, "packed weights");
        }
        if (n->fused_stale) {
            if ((r = mlp_snapshot(n, n->fw, n->fb, n->stream))) return r;
            n->fused_stale = false;
        }
        const FusedNet w{n->fw, n->fw + kFusedW1, n->fw + kFusedW1 + kFusedW2, n->fb, n->fb + 256, n->fb + 512};
        if (mlp_fused_forward(w, n->Xb, n->n_in, n->n_out, nullptr, rows, Y, n->stream) != hipSuccess)
            return mfail(n, CP_EHIP, "fused forward");
        return CP_OK;
    }
    if ((r = forward_rows(n, rows, n->stream))) return r;
    if (hipMemcpyAsync(Y, n->Yf, (long)rows * n->n_out * 4, hipMemcpyDeviceToDevice, n->stream) != hipSuccess)
        return mfail(n, CP_EHIP, "output copy");
    return CP_OK;
}

int cp_mlp_loss_grad(cp_mlp *n, const float *X, const float *T, int rows, double *loss_host, float *grad_host)
{
    if (!n || !X || !T || rows < 1) return CP_EINVAL;
    int r = ensure_cap(n, rows);
    if (r) return r;
    hipStream_t s = n->stream;
    const long nx = (long)rows * n->n_in, ny = (long)rows * n->n_out;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, s, X, nx, n->Xb);
    if ((r = forward_rows(n, rows, s))) return r;
    const int nb = (int)((ny + 255) / 256);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, n->Yf, T, ny, 1.0f / (float)ny, n->dY, n->lossp);
    const uint16_t *W2 = n->pb + n->off[2], *W3 = n->pb + n->off[4];
    float *g = n->g;
    // layer 3: dW3 = H2^T dY, db3 = colsum dY, dZ2 = (dY W3^T) * GELU'(Z2)
    if ((r = weight_grad(n, n->H2, n->n_h, n->dY, n->n_out, rows, g + n->off[4], s))) return r;
    hipLaunchKernelGGL(k_colsum_bf16, dim3(n->n_out), dim3(256), 0, s, n->dY, rows, n->n_out, (long)n->n_out,
                       g + n->off[5]);
    GemmArgs a = gargs(n->dY, n->n_out, 1, W3, 1, n->n_out, rows, n->n_h, n->n_out);
    a.Hb = n->dZ2;
    a.ldh = n->n_h;
    a.Zs = n->Z2;
    a.ldz = n->n_h;
    if (gemm<EPI_DGELU>(a, 1, s) != hipSuccess) return mfail(n, CP_EHIP, "dZ2");
    // layer 2
    if ((r = weight_grad(n, n->H1, n->n_h, n->dZ2, n->n_h, rows, g + n->off[2], s))) return r;
    hipLaunchKernelGGL(k_colsum_bf16, dim3(n->n_h), dim3(256), 0, s, n->dZ2, rows, n->n_h, (long)n->n_h,
                       g + n->off[3]);
    a = gargs(n->dZ2, n->n_h, 1, W2, 1, n->n_h, rows, n->n_h, n->n_h);
    a.Hb = n->dZ1;
    a.ldh = n->n_h;
    a.Zs = n->Z1;
    a.ldz = n->n_h;
    if (gemm<EPI_DGELU>(a, 1, s) != hipSuccess) return mfail(n, CP_EHIP, "dZ1");
    // layer 1
    if ((r = weight_grad(n, n->Xb, n->n_in, n->dZ1, n->n_h, rows, g + n->off[0], s))) return r;
    hipLaunchKernelGGL(k_colsum_bf16, dim3(n->n_h), dim3(256), 0, s, n->dZ1, rows, n->n_h, (long)n->n_h,
                       g + n->off[1]);
    if (hipGetLastError() != hipSuccess) return mfail(n, CP_EHIP, "backward launch");
    std::vector<float> lp(nb);
    if (hipMemcpyAsync(lp.data(), n->lossp, nb * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
        return mfail(n, CP_EHIP, "loss copy");
    if (grad_host && hipMemcpyAsync(grad_host, g, n->np * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
        return mfail(n, CP_EHIP, "grad copy");
    if (hipStreamSynchronize(s) != hipSuccess) return mfail(n, CP_EHIP, "sync");
    double L = 0.0;
    for (float x : lp) L += x;
    if (loss_host) *loss_host = L / (double)ny;
    return CP_OK;
}

int cp_mlp_adam(cp_mlp *n, double lr, double beta1, double beta2, double eps)
{
    if (!n || !(lr > 0)) return CP_EINVAL;
    n->adam_t += 1;
    const float c1 = (float)(1.0 / (1.0 - pow(beta1, n->adam_t)));
    const float c2 = (float)(1.0 / (1.0 - pow(beta2, n->adam_t)));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n->np + 255) / 256)), dim3(256), 0, n->stream, n->p, n->m, n->v, n->g,
                       n->np, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2, n->pb);
    n->fused_stale = true;
    return hipGetLastError() == hipSuccess ? CP_OK : mfail(n, CP_EHIP, "adam launch");
}

const char *cp_mlp_error_string(const cp_mlp *n) { return n ? n->err.c_str() : "null mlp"; }

}  // extern "C"
