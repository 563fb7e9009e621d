// Device code of the paper-form shallow network (Sec. 3, Eq. (ANN:Eq1)-
// (ANN:Eq4)): one hidden layer of tanh units and an ELU output layer, one
// network per octant or one per quadrature direction, evaluated on the vector
// ALUs.  With 8 hidden units the network is 272 multiply-adds per cell, far
// too narrow for the matrix cores.
//
// Every lane of a block serves the same octant, so per-octant weights are
// uniform over the block: they are read through the constant address space,
// which makes them scalar loads (scalar registers as FMA operands, no LDS, no
// vector memory traffic).  The lanes of a wave serve several directions, so
// per-direction weights are read from the octant's images, which the block
// first copies to LDS (1 KB per direction).  The input
// scaling of Eq. (ANN:Eq2), the problem's cell
// sizes (constant inputs), the signs of the direction cosines and the node and
// face-node relabelling between the physical and the canonical (reflected)
// frame are folded into the weights on the host, so the kernel feeds the
// canonical quantities it already holds.
#pragma once

#include "common.hpp"

namespace dgsn {

constexpr int kPannHidden = 8;   // hidden units evaluated (smaller nets are zero-padded)
constexpr int kPannIn = 26;      // inputs of the paper's network
// Canonical-frame features of the sweep: inflow x, y, z faces (12, canonical
// face-node order), kappa_x, kappa_y, source nodes (8, canonical order),
// sigma_t.  The cell sizes are constants of the problem.
constexpr int kPannFeat = 23;
// per-octant weight image of a problem (floats)
constexpr int kPannW1 = 0;                                  // [8][23]
constexpr int kPannB1 = kPannW1 + kPannHidden * kPannFeat;  // [8]
constexpr int kPannW2 = kPannB1 + kPannHidden;              // [8][8]
constexpr int kPannB2 = kPannW2 + 8 * kPannHidden;          // [8]
constexpr int kPannBeta = kPannB2 + 8;                      // beta / max(psi_inc)
constexpr int kPannStride = 272;
// per-direction networks: at most this many nets in an artifact, matched to
// the problem's directions by every cosine within this distance
constexpr int kPannMaxDirs = 4096;
constexpr double kPannDirTol = 1e-6;
// A sweep block holds its octant's per-direction images in LDS, padded from
// 272 to kPannLdsStride floats so that the 16-byte reads of ten directions
// at one weight index fall in disjoint banks; at most kPannLdsMaxDo
// directions per octant fit the 64 KB of dynamic LDS.
constexpr int kPannLdsStride = 276;
constexpr int kPannLdsMaxDo = 65536 / (4 * kPannLdsStride);

typedef float pann_f32x4 __attribute__((ext_vector_type(4)));

// The Do per-direction images of octant o (img: [8][Do][kPannStride]) into
// LDS, [Do][kPannLdsStride]; the caller synchronises the block afterwards.
__device__ __forceinline__ void load_pann_dir_table(const float *img, int o, int Do, float *lds)
{
    constexpr int n4 = kPannStride / 4;
    const pann_f32x4 *src = reinterpret_cast<const pann_f32x4 *>(img + (size_t)o * Do * kPannStride);
    for (int i = threadIdx.x; i < Do * n4; i += blockDim.x) {
        const int d = i / n4, q = i - d * n4;
        reinterpret_cast<pann_f32x4 *>(lds + d * kPannLdsStride)[q] = src[i];
    }
}
// per-octant image of the raw-input evaluation (dgsn_ann_infer_octant)
constexpr int kPannRawW1 = 0;                                  // [8][26], scaling folded in
constexpr int kPannRawB1 = kPannRawW1 + kPannHidden * kPannIn;  // [8]
constexpr int kPannRawW2 = kPannRawB1 + kPannHidden;            // [8][8]
constexpr int kPannRawB2 = kPannRawW2 + 8 * kPannHidden;        // [8]
constexpr int kPannRawBeta = kPannRawB2 + 8;
constexpr int kPannRawStride = 296;

// Read-only weight at base[i]: kUniform, through the constant address space
// (a scalar load for a wave-uniform address; the address space exists in the
// device pass only); else an ordinary per-lane load (from LDS in the sweeps).
template <bool kUniform>
__device__ __forceinline__ float pann_w(const float *base, int i)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (kUniform) return ((const __attribute__((address_space(4))) float *)base)[i];
#endif
    return base[i];
}

// tanh(z) = sign(z) (1 - 2 / (exp(2|z|) + 1)), with the hardware base-2
// exponential and reciprocal: absolute error a few 1e-8, exact limits +-1.
__device__ __forceinline__ float pann_tanh(float z)
{
    const float e = __builtin_amdgcn_exp2f(fabsf(z) * 2.8853900817779268f);   // 2 log2(e)
    const float t = fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
    return copysignf(t, z);
}

// Eq. (ANN:Eq4): z for z >= 0, beta (exp(z) - 1) below.
__device__ __forceinline__ float pann_elu(float z, float beta)
{
    return z >= 0.0f ? z : beta * (__builtin_amdgcn_exp2f(z * 1.4426950408889634f) - 1.0f);
}

// Hidden and output layers on features f[nf] with the image at w (layout
// W1 [8][nf], b1 [8], W2 [8][8], b2 [8], beta scale).
template <int NF, int W1, int B1, int W2, int B2, int BETA, bool kUniform = true>
__device__ __forceinline__ void pann_layers(const float *w, const float f[NF], float pmax,
                                            float out[8])
{
    float h[kPannHidden];
#pragma unroll
    for (int k = 0; k < kPannHidden; ++k) {
        float z = pann_w<kUniform>(w, B1 + k);
#pragma unroll
        for (int j = 0; j < NF; ++j) z = fmaf(pann_w<kUniform>(w, W1 + k * NF + j), f[j], z);
        h[k] = pann_tanh(z);
    }
    const float beta = pann_w<kUniform>(w, BETA) * pmax;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        float z = pann_w<kUniform>(w, B2 + t);
#pragma unroll
        for (int k = 0; k < kPannHidden; ++k)
            z = fmaf(pann_w<kUniform>(w, W2 + t * kPannHidden + k), h[k], z);
        out[t] = pann_elu(z, beta);
    }
}

// One canonical cell of the sweep: kap = |Omega_a| / dx_a, st = sigma_t,
// sc = canonical source nodes, vx/vy/vz = canonical inflow faces.  A face
// with kappa_a = 0 carries no inflow and is fed as 0.  w: the octant's image
// (kUniform) or the lane's direction's.
template <bool kUniform = true>
__device__ __forceinline__ void pann_cell(const float *w, const float kap[3], float st,
                                          const float sc[8], const float vx[4], const float vy[4],
                                          const float vz[4], float psi[8])
{
    float f[kPannFeat];
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
        f[fn] = kap[0] != 0.0f ? vx[fn] : 0.0f;
        f[4 + fn] = kap[1] != 0.0f ? vy[fn] : 0.0f;
        f[8 + fn] = kap[2] != 0.0f ? vz[fn] : 0.0f;
    }
    float pmax = f[0];
#pragma unroll
    for (int j = 1; j < 12; ++j) pmax = fmaxf(pmax, f[j]);
    f[12] = kap[0];
    f[13] = kap[1];
#pragma unroll
    for (int n = 0; n < 8; ++n) f[14 + n] = sc[n];
    f[22] = st;
    pann_layers<kPannFeat, kPannW1, kPannB1, kPannW2, kPannB2, kPannBeta, kUniform>(w, f, pmax,
                                                                                   psi);
}

}  // namespace dgsn
