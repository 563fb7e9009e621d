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


// Operand images of the network (built by build_params in ann.hip), for
// v_mfma_f32_32x32x16_bf16.  Lane l (half h = l / 32) holds:
//   W1 tile t (hidden 32t .. 32t+31), K-step kk (features 16kk .. 16kk+15):
//     W1[32t + l%32][16kk + 8h + e], e = 0..7, at [2t + kk][l];
//   W2 K-step kc (16 hidden units): W2[l%32][hid(kc, h, e)] at [kc][l], where
//     hid(kc, h, e) = 16kc + 8(e/4) + 4h + e%4 is the hidden unit that layer 1
//     leaves in element e of lane half h (rows 0..7 of the output are the 8
//     outputs, the other 24 are zero);
//   b2: 8 floats, uniform over the wave.
constexpr int kParamW1 = 0;                        // [4][64] bf16x8
constexpr int kParamW2 = 4 * 64 * 16;              // [4][64] bf16x8
constexpr int kParamB2 = kParamW2 + 4 * 64 * 16;   // [8] f32
constexpr int kParamBytes = kParamB2 + 8 * 4;
constexpr int kHiddenPad = 64;
// the hidden bias b1 enters layer 1 through two padding features held at 1:
// its bf16 high part and the bf16 rounding of the remainder (b1 to about
// 2^-17 relative), so the layer's accumulator starts from zero
constexpr int kFeatBiasHi = 24;
constexpr int kFeatBiasLo = 25;

typedef float f32x16 __attribute__((ext_vector_type(16)));

struct AnnRegs {
    bf16x8 w1[4];
    bf16x8 w2[4];
    const float *b2;   // [8], read as scalars
};

__device__ __forceinline__ void ann_load(const unsigned char *__restrict__ prm, int lane,
                                         AnnRegs &R)
{
#pragma unroll
    for (int m = 0; m < 4; ++m)
        R.w1[m] = *reinterpret_cast<const bf16x8 *>(prm + kParamW1 + (m * 64 + lane) * 16);
#pragma unroll
    for (int c = 0; c < 4; ++c)
        R.w2[c] = *reinterpret_cast<const bf16x8 *>(prm + kParamW2 + (c * 64 + lane) * 16);
    R.b2 = reinterpret_cast<const float *>(prm + kParamB2);
}

// Exchanges the upper half of a (lanes 32..63) with the lower half of b
// (lanes 0..31): a becomes [a.lo, b.lo] and b becomes [a.hi, b.hi].
__device__ __forceinline__ void swap_halves(unsigned &a, unsigned &b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}

// bf16 pairs of two floats (round to nearest even), and of what the rounding
// left: hi = bf16(v), lo = bf16(v - hi), so that hi + lo carries v to about
// 2^-17 relative
__device__ __forceinline__ unsigned bf16_pair(float a, float b)
{
    const f32x2 pr = {a, b};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(pr, bf16x2));
}
__device__ __forceinline__ void bf16_split_pair(float a, float b, unsigned &hi, unsigned &lo)
{
    hi = bf16_pair(a, b);
    const bf16x2 h = __builtin_bit_cast(bf16x2, hi);
    lo = bf16_pair(a - (float)h[0], b - (float)h[1]);
}

// Evaluates the network for the 64 samples held by the 64 lanes of the wave
// (one sample per lane, 24 FP32 features), with no LDS traffic.  The
// samples of lanes 0..31 form batch 0 and those of lanes 32..63 batch 1; a
// 32x32x16 matrix instruction takes 32 samples as its columns, so the
// transposes between "one sample per lane" and the operand layout (lane
// half h holding features 8h .. 8h+7 of a K-step) are exchanges between the
// two halves of the wave.  Layer 1 computes H^T = W1 X^T per batch (two
// tiles of 32 hidden units, two K-steps of 16 features); its output
// registers, after ReLU and the rounding to bf16, are the B operand of
// layer 2, Y^T = W2' relu(H^T) (four K-steps of 16 hidden units, W2' the
// column order hid(kc, h, e) above).  kSplit: the features and the hidden
// activations enter as bf16 hi + lo pairs, each part through its own matrix
// instruction against the (bf16) weights, which removes their 2^-9 rounding
// and leaves about 2^-17 (twice the matrix instructions).  Must be reached
// by every lane.
template <bool kSplit = false>
__device__ __forceinline__ void ann_wave(const AnnRegs &R, const float feat[24], float out[8])
{
    constexpr int NP = kSplit ? 2 : 1;   // parts of each activation
    // the lane's 32 padded features as bf16 pairs: chunk q holds 8q .. 8q+7
    unsigned c[NP][4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            float v[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int f = 8 * q + 2 * p + k;
                v[k] = f < 24 ? feat[f] : (f == kFeatBiasHi || f == kFeatBiasLo ? 1.0f : 0.0f);
            }
            if constexpr (kSplit) bf16_split_pair(v[0], v[1], c[0][q][p], c[NP - 1][q][p]);
            else c[0][q][p] = bf16_pair(v[0], v[1]);
        }
    // K-step kk of batch bt needs chunk 2kk + h of the batch's samples in
    // lane half h: after the exchange c[2kk + bt] is that operand
#pragma unroll
    for (int part = 0; part < NP; ++part)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            swap_halves(c[part][0][p], c[part][1][p]);
            swap_halves(c[part][2][p], c[part][3][p]);
        }
    unsigned y[2][4];
#pragma unroll
    for (int bt = 0; bt < 2; ++bt) {
        bf16x8 x0[NP], x1[NP];
#pragma unroll
        for (int part = 0; part < NP; ++part) {
            const unsigned *a0 = c[part][bt], *a1 = c[part][2 + bt];
            const u32x4 u0 = {a0[0], a0[1], a0[2], a0[3]};
            const u32x4 u1 = {a1[0], a1[1], a1[2], a1[3]};
            x0[part] = __builtin_bit_cast(bf16x8, u0);
            x1[part] = __builtin_bit_cast(bf16x8, u1);
        }
        f32x16 acc = (f32x16)0.0f;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            f32x16 h = (f32x16)0.0f;
#pragma unroll
            for (int part = 0; part < NP; ++part) {
                h = __builtin_amdgcn_mfma_f32_32x32x16_bf16(R.w1[2 * t], x0[part], h, 0, 0, 0);
                h = __builtin_amdgcn_mfma_f32_32x32x16_bf16(R.w1[2 * t + 1], x1[part], h, 0, 0,
                                                            0);
            }
#pragma unroll
            for (int pp = 0; pp < 2; ++pp) {
                bf16x8 hb[NP];
                if constexpr (kSplit) {
                    // ReLU in FP32, then the hi + lo parts
                    u32x4 th, tl;
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        unsigned a, b;
                        bf16_split_pair(fmaxf(h[8 * pp + 2 * p], 0.0f),
                                        fmaxf(h[8 * pp + 2 * p + 1], 0.0f), a, b);
                        th[p] = a;
                        tl[p] = b;
                    }
                    hb[0] = __builtin_bit_cast(bf16x8, th);
                    hb[NP - 1] = __builtin_bit_cast(bf16x8, tl);
                } else {
                    // ReLU after the rounding to bf16, on the packed pairs: bf16
                    // is sign and magnitude, so as 16-bit integers every
                    // negative value (and -0) is below zero and max(x, 0) is
                    // the ReLU, equal to rounding the ReLU of the FP32 value
                    u32x4 tq;
#pragma unroll
                    for (int p = 0; p < 4; ++p)
                        tq[p] = bf16_pair(h[8 * pp + 2 * p], h[8 * pp + 2 * p + 1]);
                    const i16x8 r =
                        __builtin_elementwise_max(__builtin_bit_cast(i16x8, tq), (i16x8)0);
                    hb[0] = __builtin_bit_cast(bf16x8, r);
                }
#pragma unroll
                for (int part = 0; part < NP; ++part)
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(R.w2[2 * t + pp], hb[part], acc,
                                                                  0, 0, 0);
            }
        }
        // rows 0..3 of lane half h are outputs 4h .. 4h+3 of the column's sample
#pragma unroll
        for (int r = 0; r < 4; ++r) y[bt][r] = __float_as_uint(acc[r]);
    }
    // each sample's outputs back to its lane: after the exchange y[0] holds
    // outputs 0..3 and y[1] outputs 4..7 of the lane's own sample
#pragma unroll
    for (int r = 0; r < 4; ++r) swap_halves(y[0][r], y[1][r]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out[r] = __uint_as_float(y[0][r]) + R.b2[r];
        out[4 + r] = __uint_as_float(y[1][r]) + R.b2[4 + r];
    }
}

}  // namespace dgsn
