// cp_fused_net.hpp -- the fused inference of the surrogate network on one 64-row
// tile (gfx950 BF16 MFMA), shared by the plain inference kernel and the kernel that
// gates the active cells and evaluates the network in one launch.
#pragma once
#include <stdint.h>

#include "cp_internal.hpp"

namespace cp {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float kGeluC = 0.7978845608028654f;   // sqrt(2/pi)
// GELU in tanh form, evaluated through 0.5 (1 + tanh u) = 1 / (1 + e^{-2u}) with the
// hardware exp2 and reciprocal: z / (1 + e^{-2u}), u = sqrt(2/pi) (z + 0.044715 z^3).
// The error is a few 1e-7 relative, far below the bf16 rounding of the activations;
// e^{-2u} = inf gives 0 and e^{-2u} = 0 gives z, so it saturates cleanly.
constexpr float kGeluE = -2.0f * kGeluC * 1.4426950408889634f;   // -2 sqrt(2/pi) log2(e)
__device__ __forceinline__ float gelu_sig(float z)   // 1 / (1 + e^{-2u})
{
    // -2 u log2(e) = z (kGeluE + kGeluE 0.044715 z^2)
    const float t = z * fmaf(kGeluE * 0.044715f, z * z, kGeluE);
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
}
__device__ __forceinline__ float gelu_f(float z) { return z * gelu_sig(z); }

// gfx950 v_mfma_f32_16x16x32_bf16 (lane layout checked on the device): A operand of
// lane l holds row l % 16, k = 8 (l / 16) + i; B operand k = 8 (l / 16) + i, column
// l % 16; the 4 results are rows 4 (l / 16) + i, column l % 16.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16x8 ld_bf16x8(const uint16_t *p) { return __builtin_bit_cast(bf16x8, *(const uint4 *)p); }

// All three layers for a 64-row tile (n_in <= 32, n_h = 256, n_out <= 16).  Every
// product is formed transposed, Z^T = W^T A^T: the packed weight fragment is the
// MFMA's first operand and 16 rows of activations its second, so a lane's four results
// are four consecutive units of one row.  The bias is the accumulator's initial value,
// and the four GELU outputs leave as one 8-byte LDS write into the row-major activation
// tile, which the next layer reads with one 16-byte load per lane.  The input tile and
// each hidden activation stay in LDS; every wave owns 64 units of a hidden layer for
// all 64 rows (4 x 4 MFMA tiles) and one 16-row block of the output layer.  The weight
// fragments of the next k block are requested before the current block's MFMAs.
constexpr int kFusedNH = 256, kFusedKin = 32, kFusedPad = 8;
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));

// GELU of four accumulator values, rounded to bf16 and packed in order
__device__ __forceinline__ uint2 gelu_pack4(f32x4 z)
{
    const bf16x2v lo = __builtin_convertvector((f32x2v){gelu_f(z[0]), gelu_f(z[1])}, bf16x2v);
    const bf16x2v hi = __builtin_convertvector((f32x2v){gelu_f(z[2]), gelu_f(z[3])}, bf16x2v);
    return make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
}

typedef uint16_t FusedXTile[64][kFusedKin + kFusedPad];
typedef uint16_t FusedHTile[64][kFusedNH + kFusedPad];

// The network on the 64 input rows in Xs (bf16, zero beyond the inputs; filled, and a
// barrier passed, by the caller) with all 256 threads of the workgroup; outputs of the
// tile's rows r < rows go to Yt[r * n_out + o].  Ends with a barrier, so the caller may
// refill Xs and Hs at once.
__device__ __forceinline__ void fused_net_tile(const FusedNet &w, FusedXTile &Xs, FusedHTile &Hs, int rows, int n_out,
                                               float *Yt)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = 8 * (lane >> 4);   // second operand: row of the tile, first k
    const int ld = 4 * (lane >> 4);                     // results: first of the lane's four units
    constexpr int NB = kFusedNH / 16, KB = kFusedNH / 32;
    // biases of the lane's results, hidden units 16 (4 wave + mb) + ld + i and outputs
    // ld + i: four consecutive floats, one 16-byte load (the packed biases are 16-byte
    // aligned, b3 zero-padded to 16)
    const f32x4 *b1v = reinterpret_cast<const f32x4 *>(w.b1 + 16 * 4 * wave + ld);
    const f32x4 *b2v = reinterpret_cast<const f32x4 *>(w.b2 + 16 * 4 * wave + ld);
    f32x4 acc[4][4];   // [unit block][row block]
    // hidden layer 1: K = 32, one k block
    {
        bf16x8 wa[4], xb[4];
        #pragma unroll
        for (int mb = 0; mb < 4; ++mb) wa[mb] = ld_bf16x8(&w.w1[((long)(4 * wave + mb) * 64 + lane) * 8]);
        #pragma unroll
        for (int nb = 0; nb < 4; ++nb) xb[nb] = ld_bf16x8(&Xs[16 * nb + lr][lk]);
        #pragma unroll
        for (int mb = 0; mb < 4; ++mb)
            #pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[mb], xb[nb], b1v[4 * mb], 0, 0, 0);
    }
    #pragma unroll
    for (int mb = 0; mb < 4; ++mb)
        #pragma unroll
        for (int nb = 0; nb < 4; ++nb)
            *reinterpret_cast<uint2 *>(&Hs[16 * nb + lr][16 * (4 * wave + mb) + ld]) = gelu_pack4(acc[mb][nb]);
    __syncthreads();
    // hidden layer 2: K = 256, eight k blocks
    #pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        const f32x4 b = b2v[4 * mb];
        #pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = b;
    }
    bf16x8 wn[4];
    #pragma unroll
    for (int mb = 0; mb < 4; ++mb) wn[mb] = ld_bf16x8(&w.w2[((long)(4 * wave + mb) * 64 + lane) * 8]);
    #pragma unroll 1
    for (int kb = 0; kb < KB; ++kb) {
        bf16x8 wa[4], hb[4];
        #pragma unroll
        for (int mb = 0; mb < 4; ++mb) wa[mb] = wn[mb];
        if (kb + 1 < KB) {
            #pragma unroll
            for (int mb = 0; mb < 4; ++mb)
                wn[mb] = ld_bf16x8(&w.w2[(((long)(kb + 1) * NB + 4 * wave + mb) * 64 + lane) * 8]);
        }
        #pragma unroll
        for (int nb = 0; nb < 4; ++nb) hb[nb] = ld_bf16x8(&Hs[16 * nb + lr][32 * kb + lk]);
        #pragma unroll
        for (int mb = 0; mb < 4; ++mb)
            #pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[mb], hb[nb], acc[mb][nb], 0, 0, 0);
    }
    __syncthreads();   // every wave has read the first activation
    #pragma unroll
    for (int mb = 0; mb < 4; ++mb)
        #pragma unroll
        for (int nb = 0; nb < 4; ++nb)
            *reinterpret_cast<uint2 *>(&Hs[16 * nb + lr][16 * (4 * wave + mb) + ld]) = gelu_pack4(acc[mb][nb]);
    __syncthreads();
    // output layer: the wave's 16 rows, one 16-unit block, eight k blocks
    f32x4 c = *reinterpret_cast<const f32x4 *>(w.b3 + ld);
    #pragma unroll 4
    for (int kb = 0; kb < KB; ++kb) {
        const bf16x8 wa = ld_bf16x8(&w.w3[((long)kb * 64 + lane) * 8]);
        const bf16x8 hb = ld_bf16x8(&Hs[16 * wave + lr][32 * kb + lk]);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, hb, c, 0, 0, 0);
    }
    const int r = 16 * wave + lr;   // the lane's row; outputs ld .. ld + 3
    if (r < rows) {
        #pragma unroll
        for (int i = 0; i < 4; ++i)
            if (ld + i < n_out) Yt[(long)r * n_out + ld + i] = c[i];
    }
    __syncthreads();   // the next tile overwrites Xs and Hs
}

}  // namespace cp
