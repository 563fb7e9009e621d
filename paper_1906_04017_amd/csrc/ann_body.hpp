// Device code of the shallow-ANN local solver shared by the ANN kernels and
// the batched kernel (see ann.hip for the matrix-core mapping).
#pragma once

#include "cell.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace dgsn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short i16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Orders this wave's LDS writes before its following LDS reads of other
// lanes' slots.  The LDS processes the accesses of one wave in issue order, so
// only the compiler has to be kept from moving accesses across: wavefront-
// scope fences around the wave barrier emit no instruction.  (An explicit
// s_waitcnt intrinsic would also do, but the compiler then treats it as a
// store to global memory and stops keeping kernel-argument tables read
// through pointers in scalar registers.)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


constexpr int kParamW1 = 0;                  // [4][64] bf16x8
constexpr int kParamW2 = 4 * 64 * 16;        // [2][64] bf16x8
constexpr int kParamB2 = kParamW2 + 2 * 64 * 16;  // [8] f32, uniform over the wave
constexpr int kParamBytes = kParamB2 + 8 * 4;
constexpr int kHiddenPad = 64;
// the hidden bias b1 enters layer 1 through two padding features held at 1:
// its bf16 high part and the bf16 rounding of the remainder (b1 to about
// 2^-17 relative), so the layer's accumulator starts from zero
constexpr int kFeatBiasHi = 24;
constexpr int kFeatBiasLo = 25;

struct AnnRegs {
    bf16x8 w1[4];
    bf16x8 w2[2];
    const float *b2;   // [8], read as scalars
};

__device__ __forceinline__ void ann_load(const unsigned char *__restrict__ prm, int lane,
                                         AnnRegs &R)
{
#pragma unroll
    for (int m = 0; m < 4; ++m)
        R.w1[m] = *reinterpret_cast<const bf16x8 *>(prm + kParamW1 + (m * 64 + lane) * 16);
#pragma unroll
    for (int c = 0; c < 2; ++c)
        R.w2[c] = *reinterpret_cast<const bf16x8 *>(prm + kParamW2 + (c * 64 + lane) * 16);
    R.b2 = reinterpret_cast<const float *>(prm + kParamB2);
}

// Evaluates the network for the 64 samples held by the 64 lanes of the wave
// (one sample per lane, 24 FP32 features).  lds_in: 64*32 bf16 of this wave,
// lds_out: 64*8 floats of this wave.  Must be reached by every lane of the
// wave (it synchronises the wave's LDS traffic only).
__device__ __forceinline__ void ann_wave(const AnnRegs &R, const float feat[24],
                                         __bf16 *lds_in, float *lds_out, float out[8])
{
    const int lane = threadIdx.x & 63;
    {
        bf16x8 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int f = 8 * q + e;
                v[q][e] = (__bf16)(f < 24 ? feat[f]
                                          : (f == kFeatBiasHi || f == kFeatBiasLo ? 1.0f : 0.0f));
            }
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<bf16x8 *>(lds_in + lane * 32 + 8 * q) = v[q];
    }
    wave_lds_sync();
    const int col = lane & 15, grp = lane >> 4;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const bf16x8 xb = *reinterpret_cast<const bf16x8 *>(lds_in + (16 * b + col) * 32 + 8 * grp);
        f32x4 h[4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
            h[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(R.w1[m], xb, (f32x4)0.0f, 0, 0, 0);
        // ReLU after the rounding to bf16, on the packed pairs: bf16 is sign
        // and magnitude, so as 16-bit integers every negative value (and -0)
        // is below zero and max(x, 0) is the ReLU, equal to rounding the
        // ReLU of the FP32 value
        bf16x8 hb[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            u32x4 t;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const f32x4 &hv = h[2 * c + (p >> 1)];
                const f32x2 pr = {hv[2 * (p & 1)], hv[2 * (p & 1) + 1]};
                t[p] = __builtin_bit_cast(unsigned, __builtin_convertvector(pr, bf16x2));
            }
            const i16x8 r = __builtin_elementwise_max(__builtin_bit_cast(i16x8, t), (i16x8)0);
            hb[c] = __builtin_bit_cast(bf16x8, r);
        }
        f32x4 y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(R.w2[0], hb[0], (f32x4)0.0f, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(R.w2[1], hb[1], y, 0, 0, 0);
        if (grp < 2) {
#pragma unroll
            for (int r = 0; r < 4; ++r) lds_out[(16 * b + col) * 8 + 4 * grp + r] = y[r];
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] = lds_out[lane * 8 + k] + R.b2[k];
}

}  // namespace dgsn
