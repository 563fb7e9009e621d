// Device code of the GE transport sweep shared by the per-problem kernels
// and the batched kernel: canonical cell systems (paper and mass-inverse
// forms), their solves, and the tile sweep body.
#pragma once

#include "ann_body.hpp"
#include "cell.hpp"
#include "pann_body.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace dgsn {

constexpr double kInv4Pi = 0.07957747154594767;   // 1 / (4 pi)

// dynamic LDS of the sweep kernels (the per-direction network images)
extern __shared__ __align__(16) float dgsn_dyn_lds[];

// Reflect an 8-node vector between physical and canonical node order
// (v[n] <-> v[n ^ mask]); mask is uniform over the block, so each stage is a
// scalar branch around register moves.
template <typename Real>
__device__ __forceinline__ void reflect8(Real v[8], int mask)
{
    if (mask & 1) {
#pragma unroll
        for (int n = 0; n < 8; n += 2) { const Real t = v[n]; v[n] = v[n + 1]; v[n + 1] = t; }
    }
    if (mask & 2) {
#pragma unroll
        for (int n = 0; n < 8; ++n)
            if (!(n & 2)) { const Real t = v[n]; v[n] = v[n + 2]; v[n + 2] = t; }
    }
    if (mask & 4) {
#pragma unroll
        for (int n = 0; n < 4; ++n) { const Real t = v[n]; v[n] = v[n + 4]; v[n + 4] = t; }
    }
}

// 8-node record at p read into canonical order: v[n] = p[n ^ mask].  Node
// pairs (n, n ^ 1) are contiguous, so the y and z reflections permute the four
// pair addresses and only the x reflection moves registers (within a pair).
template <typename Real>
__device__ __forceinline__ void load8_reflect(const Real *p, int mask, Real v[8])
{
    const int pm = (mask >> 1) & 3;
#pragma unroll
    for (int pr = 0; pr < 4; ++pr) {
        const Real a = p[2 * (pr ^ pm)], b = p[2 * (pr ^ pm) + 1];
        v[2 * pr] = (mask & 1) ? b : a;
        v[2 * pr + 1] = (mask & 1) ? a : b;
    }
}

// Canonical 8-node vector v stored in physical order: p[n ^ mask] = v[n].
template <typename Real>
__device__ __forceinline__ void store8_reflect(Real *p, int mask, const Real v[8])
{
    const int pm = (mask >> 1) & 3;
#pragma unroll
    for (int pr = 0; pr < 4; ++pr) {
        p[2 * (pr ^ pm)] = (mask & 1) ? v[2 * pr + 1] : v[2 * pr];
        p[2 * (pr ^ pm) + 1] = (mask & 1) ? v[2 * pr] : v[2 * pr + 1];
    }
}

template <typename Real>
__device__ __forceinline__ void load4(const Real *p, Real v[4])
{
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = p[e];
}

template <typename Real>
__device__ __forceinline__ void store4(Real *p, Real a, Real b, Real c, Real d)
{
    p[0] = a;
    p[1] = b;
    p[2] = c;
    p[3] = d;
}

// Face-front access.  The hyperplane kernels move fronts through the caches
// (the kernel boundary between two steps writes the L2s back).  The dataflow
// kernel hands fronts between workgroups of one launch that may run on
// different XCDs, each with its own L2, so it uses device-scope coherent
// buffer operations (cache policy sc1): loads do not hit stale L2 lines and
// stores write through.  Byte offsets are 32-bit (fronts under 2 GiB) and the
// hardware bounds-checks every access against the buffer size.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCpolDevice = 16;               // sc1
constexpr int kRawBufferWord3 = 0x00020000;   // untyped 32-bit buffer, gfx9 family

template <typename Real>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t front_rsrc(Real *base, uint32_t elems)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)(elems * sizeof(Real)),
                                             kRawBufferWord3);
}

template <typename Real, bool kCoh>
__device__ __forceinline__ void front_load(const Real *base, __amdgpu_buffer_rsrc_t r, uint32_t e,
                                           Real v[4])
{
    if constexpr (!kCoh) {
        load4(base + e, v);
    } else if constexpr (sizeof(Real) == 4) {
        const u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(r, e * 4u, 0, kCpolDevice);
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = __uint_as_float(u[k]);
    } else {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, e * 8u, 0, kCpolDevice);
        const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(r, e * 8u + 16u, 0, kCpolDevice);
        v[0] = __hiloint2double((int)a[1], (int)a[0]);
        v[1] = __hiloint2double((int)a[3], (int)a[2]);
        v[2] = __hiloint2double((int)b[1], (int)b[0]);
        v[3] = __hiloint2double((int)b[3], (int)b[2]);
    }
}

template <typename Real, bool kCoh>
__device__ __forceinline__ void front_store(Real *base, __amdgpu_buffer_rsrc_t r, uint32_t e,
                                            Real a, Real b, Real c, Real d)
{
    if constexpr (!kCoh) {
        store4(base + e, a, b, c, d);
    } else if constexpr (sizeof(Real) == 4) {
        const u32x4 u = {__float_as_uint(a), __float_as_uint(b), __float_as_uint(c),
                         __float_as_uint(d)};
        __builtin_amdgcn_raw_buffer_store_b128(u, r, e * 4u, 0, kCpolDevice);
    } else {
        const u32x4 u = {(unsigned)__double2loint(a), (unsigned)__double2hiint(a),
                         (unsigned)__double2loint(b), (unsigned)__double2hiint(b)};
        const u32x4 w = {(unsigned)__double2loint(c), (unsigned)__double2hiint(c),
                         (unsigned)__double2loint(d), (unsigned)__double2hiint(d)};
        __builtin_amdgcn_raw_buffer_store_b128(u, r, e * 8u, 0, kCpolDevice);
        __builtin_amdgcn_raw_buffer_store_b128(w, r, e * 8u + 16u, 0, kCpolDevice);
    }
}

// Mass-inverse cell matrix P_d + sigma_t I, with the structural zeros of P_d
// as literal zeros.
template <typename Real>
__device__ __forceinline__ void massinv_matrix(const Real k[3], Real st, Real a[8][8])
{
    const Real base = fma(Real(3), k[0] + k[1] + k[2], st);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
        for (int c = 0; c < 8; ++c) a[r][c] = Real(0);
        Real dg = base;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const bool hi = (r >> ax) & 1;
            if (hi) dg = fma(Real(-2), k[ax], dg);
            a[r][r ^ (1 << ax)] = hi ? Real(-3) * k[ax] : k[ax];
        }
        a[r][r] = dg;
    }
}

// Mass-inverse right-hand side S + sum_a kappa_a c_a.
template <typename Real>
__device__ __forceinline__ void massinv_rhs(const Real k[3], const Real sc[8], const Real vx[4],
                                            const Real vy[4], const Real vz[4], Real b[8])
{
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        const int ix = n & 1, iy = (n >> 1) & 1, iz = (n >> 2) & 1;
        Real v = sc[n];
        v = fma(ix ? Real(-2) * k[0] : Real(4) * k[0], vx[iy + 2 * iz], v);
        v = fma(iy ? Real(-2) * k[1] : Real(4) * k[1], vy[ix + 2 * iz], v);
        v = fma(iz ? Real(-2) * k[2] : Real(4) * k[2], vz[ix + 2 * iy], v);
        b[n] = v;
    }
}

// Paper-form cell solve of one lane: A' = S_d + sigma_t M3 and
// b' = M3 S + sum_a kappa_a Mf psi_a from the direction entry, sigma_t, the
// canonical source and the three inflow faces, dense pivoted elimination;
// returns psi (canonical node order) in b.
template <typename Real>
__device__ __forceinline__ void dense_cell_solve(const Real *__restrict__ dp, const Real k[3],
                                                 Real st, const Real sc[8], const Real vx[4],
                                                 const Real vy[4], const Real vz[4], Real b[8])
{
    Real a[8][8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) a[r][c] = fma(st, Real(m3_entry(r, c)), dp[r * 8 + c]);
    Real m[8], f[4];
    mass3_216(sc, m);
#pragma unroll
    for (int n = 0; n < 8; ++n) b[n] = m[n] * Real(1.0 / 216.0);
    face_mass(vx, k[0] * Real(1.0 / 36.0), f);
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) b[2 * fn] += f[fn];
    face_mass(vy, k[1] * Real(1.0 / 36.0), f);
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) b[(fn & 1) + 4 * (fn >> 1)] += f[fn];
    face_mass(vz, k[2] * Real(1.0 / 36.0), f);
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) b[fn] += f[fn];
    ge_solve8(a, b);
}

// Tile sweep.  Each lane owns one (octant, B x B x B tile of cells,
// direction, group) and solves the tile's cells in upwind lexicographic order,
// carrying the faces between its own cells in registers: only the faces on the
// tile boundary go through the fronts in HBM (24/B face values per solve
// instead of 24).  Tiles with I + J + K = s are independent; one launch per
// tile hyperplane s.  B = 1 is the plain cell hyperplane sweep.
// ANN features of one canonical cell (see ann.hip): returns the scale m;
// feat[4..23] are divided by m.
__device__ __forceinline__ float ann_features(const float kap[3], float hh, float st,
                                              const float sc[8], const float vx[4],
                                              const float vy[4], const float vz[4],
                                              float feat[24])
{
    float kmax = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        feat[a] = kap[a] * hh;
        kmax = fmaxf(kmax, feat[a]);
    }
    const float tau = st * hh;
    feat[3] = tau;
    float pmax = 0.0f, smax = 0.0f;
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
        feat[4 + fn] = feat[0] != 0.0f ? vx[fn] : 0.0f;
        feat[8 + fn] = feat[1] != 0.0f ? vy[fn] : 0.0f;
        feat[12 + fn] = feat[2] != 0.0f ? vz[fn] : 0.0f;
        pmax = fmaxf(pmax, fmaxf(fabsf(feat[4 + fn]), fmaxf(fabsf(feat[8 + fn]),
                                                          fabsf(feat[12 + fn]))));
    }
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        feat[16 + n] = hh * sc[n];
        smax = fmaxf(smax, fabsf(feat[16 + n]));
    }
    // the two quotients by v_rcp_f32 (1 ulp): m only sets the scale of the
    // features and of the outputs, so its last bits do not matter, and the
    // correctly rounded division costs about ten instructions each
    float m = pmax;
    const float den = tau + kmax;
    if (den > 0.0f) m = fmaxf(m, smax * recip(den));
    const float rm = m > 0.0f ? recip(m) : 0.0f;
#pragma unroll
    for (int k = 4; k < 24; ++k) feat[k] *= rm;
    return m;
}

// Lane of a 256-lane sweep block (see PlaneArgs): direction d and group g of
// segment slot z; ok is false for the lanes beyond the last whole segment of
// the wave and beyond nc * G segments of the block.  All quotients are exact
// (numerators below 256, divisors at most 256).
struct SegLane {
    int d, g, z;
    bool ok;
};
template <typename Real>
__device__ __forceinline__ SegLane seg_lane(const PlaneArgs<Real> &A, int tid)
{
    const int w = tid >> 6, lane = tid & 63;
    const int sl = (lane * (int)A.mag_do) >> 16;   // segment within the wave
    const int seg = w * (int)A.spw + sl;
    const int z = (seg * (int)A.mag_g) >> 16;
    SegLane l;
    l.ok = sl < (int)A.spw && z < (int)A.nc;
    l.d = l.ok ? lane - sl * (int)A.Do : 0;
    l.g = l.ok ? seg - z * (int)A.G : 0;
    l.z = l.ok ? z : 0;
    return l;
}

// Anisotropic scattering source of one lane's direction (Eq. (T7) terms of
// order n >= 1): sc += sum_k Y_k(Omega_d) msrc_k at the cell's nodes
// (reflected into the canonical octant like the isotropic source).  NM
// moments, stored contiguously per (group, cell) so that their loads leave
// together.
template <typename Real, int NM>
__device__ __forceinline__ void add_moment_source(const PlaneArgs<Real> &A, const Real *yl,
                                                  uint32_t gc, int mask, Real sc[8])
{
    const Real *base = A.msrc + (size_t)gc * (NM * 8);
    Real m[NM][8];
#pragma unroll
    for (int k = 0; k < NM; ++k) load8_reflect(base + k * 8, mask, m[k]);
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        const Real y = yl[k];
#pragma unroll
        for (int n = 0; n < 8; ++n) sc[n] = fma(y, m[k][n], sc[n]);
    }
}

// Staged form of the same source: the NM x 8 values of the cell were written
// to LDS (stage, canonical order not yet applied) by the lanes of the
// segment, which all sweep that cell.
template <typename Real, int NM>
__device__ __forceinline__ void add_moment_source_staged(const Real *stage, const Real *yl,
                                                         int mask, Real sc[8])
{
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        Real m[8];
        load8_reflect(stage + k * 8, mask, m);
        const Real y = yl[k];
#pragma unroll
        for (int n = 0; n < 8; ++n) sc[n] = fma(y, m[n], sc[n]);
    }
}

// Moment-source staging of anisotropic FP32 sweeps with 8 or more moments
// (P2, P3): the Do lanes of a segment load their cell's NM x 8 sources once
// between them (16-byte pieces, piece q by lane q mod Do) into the segment's
// LDS slot, and each lane then reads all of them from LDS, instead of every
// lane loading all of them through the vector cache (at P3, 30 16-byte loads
// per lane and cell, which keep the texture-address pipe busy; at P1 the 6
// loads cost less than the staging's wave sync).  A block holds at most
// 4 * floor(64 / Do) segments; with Do >= kStageMinDo that is kStageSegs slots.
constexpr int kStageMinDo = 6;
constexpr int kStageSegs = 4 * (64 / kStageMinDo);
template <typename Real, int kMom>
constexpr bool kStageMoments = kMom >= 8 && sizeof(Real) == 4;
template <typename Real, int kMom>
constexpr int kStageFloats = kStageMoments<Real, kMom> ? kStageSegs * kMom * 8 : 4;

// The harmonics of octant o's directions into LDS, [Do][kYlmStride], for the
// moment reduction of anisotropic sweeps (every thread of the block, then a
// block barrier).
template <typename Real>
__device__ __forceinline__ void load_ylm_table(const PlaneArgs<Real> &A, int o, Real *ytab)
{
    const int n = (int)A.Do * kYlmStride;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        ytab[i] = A.ylm[(size_t)o * A.Do * kYlmStride + i];
    __syncthreads();
}

// Tile ti of one schedule step (cells: the step's packed tiles, ncp of them).
__device__ __forceinline__ uint32_t step_tile(const uint32_t *cells, uint32_t ncp, int ti,
                                              bool lane_ok, bool &tvalid)
{
    tvalid = lane_ok && ti < (int)ncp;
    return tvalid ? cells[ti] : 0u;
}

// LDS of the tile body: the direction reduction (double buffered) and the
// adjoint contraction reduction.
template <typename Real>
struct TileLds {
    Real red[2 * 256 * 9];
    Real gred[256 * 2];
};

// Device body of the tile sweep for one lane.  d, g: direction-in-octant and
// group of the lane; tid: its index in the block (segments of Do lanes with
// equal (group, tile) are contiguous); tvalid: the lane has a tile, pt: its
// packed canonical tile coordinates (i | j << 10 | k << 20, in tiles);
// o: octant slot; inc: the boundary inflow of octant slot o per canonical
// axis; lane_ok: the lane carries work.  Form: kFormMassInv,
// kFormDense (Gaussian elimination) or kFormAnn (the network, FP32 problems,
// blocks of full waves) or kFormAnnPaper / kFormAnnPaperDir (the
// paper-form networks per octant / per direction, FP32).  kCoh: device-coherent front access (dataflow
// kernel).  kMom: anisotropic scattering with kMom = A.nmom - 1 moments (their
// sources enter the gather, the moments leave with the scalar flux; source
// iteration only, separate instantiations so that the isotropic kernels
// carry none of it; 0: isotropic); ytab: the block's octant's harmonics in
// LDS, [Do][kYlmStride] (load_ylm_table).  Must be reached by every lane of the wave; lanes of one
// (group, tile) segment are in one wave (seg_lane), and the body synchronises
// only within the wave.
template <typename Real, int Form, int B, bool kStorePsi, bool kAdjoint, bool kCoh = false,
          int kMom = 0>
__device__ __forceinline__ void tile_body(const PlaneArgs<Real> &A, const Real inc[3], int d,
                                          int g, int tid, bool tvalid, uint32_t pt, int o,
                                          bool lane_ok, TileLds<Real> &L,
                                          const Real *ytab = nullptr, Real *mstage = nullptr,
                                          const float *pann_lds = nullptr)
{
    constexpr bool kNet = Form == kFormAnn || Form == kFormAnnSplit;   // matrix-core network
    constexpr bool kPaper = Form == kFormAnnPaper || Form == kFormAnnPaperDir;
    static_assert((!kNet && !kPaper) || sizeof(Real) == 4, "the ANN solvers run in FP32");
    const int mask = kAdjoint ? (o ^ 7) : o;
    const uint32_t dg = d + A.Do * g;
    const Real *dp = A.dir + (o * A.Do + (lane_ok ? d : 0)) * kDirStride;
    const Real w = lane_ok ? dp[kDirW] : Real(0);
    const Real kap[3] = {dp[kDirK], dp[kDirK + 1], dp[kDirK + 2]};
    // the lane's harmonics, from the block's octant table in LDS (read per
    // cell: cheaper than holding kMom more registers)
    const Real *yl = kMom > 0 ? ytab + (lane_ok ? d : 0) * kYlmStride : nullptr;
    // moment-source staging (FP32, 8 or more moments, Do >= kStageMinDo):
    // the lane's segment slot, from the same exact quotient as the lane layout
    constexpr bool kStage = kStageMoments<Real, kMom>;
    const bool stage = kStage && A.Do >= (uint32_t)kStageMinDo;
    Real *mslot = nullptr;
    if constexpr (kStage) {
        const int sl = ((tid & 63) * (int)A.mag_do) >> 16;
        const int seg = (tid >> 6) * (int)A.spw + sl;
        mslot = mstage + (lane_ok && stage ? seg : 0) * (kMom * 8);
    }
    AnnRegs R;
    if (kNet) ann_load(static_cast<const unsigned char *>(A.ann_params), tid & 63, R);
    uint32_t I0 = 0, J0 = 0, K0 = 0;
    if (tvalid) {
        I0 = (pt & 1023u) * B;
        J0 = ((pt >> 10) & 1023u) * B;
        K0 = (pt >> 20) * B;
    }
    const uint32_t slot = (o * A.Do + d) * A.G + g;
    // the tile's first cell: its front slots and its physical cell index; the
    // other cells of the tile step from them by whole strides (il, jl, kl are
    // compile-time in the unrolled body), so no per-cell multiplies remain
    const uint32_t ex0 = o * A.fx_o + K0 * A.fx_k + J0 * A.fx_j + dg * 4;
    const uint32_t ey0 = o * A.fy_o + K0 * A.fy_k + I0 * A.fy_j + dg * 4;
    const uint32_t ez0 = o * A.fz_o + J0 * A.fz_k + I0 * A.fz_j + dg * 4;
    const uint32_t nxy = A.nx * A.ny;
    const uint32_t c0 = ((mask & 1) ? A.nx - 1 - I0 : I0) +
                        A.nx * ((mask & 2) ? A.ny - 1 - J0 : J0) +
                        nxy * ((mask & 4) ? A.nz - 1 - K0 : K0);
    const uint32_t sx = (mask & 1) ? 0u - 1u : 1u;          // physical steps of il, jl, kl
    const uint32_t sy = (mask & 2) ? 0u - A.nx : A.nx;      // (modulo 2^32)
    const uint32_t sz = (mask & 4) ? 0u - nxy : nxy;
    const __amdgpu_buffer_rsrc_t rx = front_rsrc(A.fx, 8 * A.fx_o);
    const __amdgpu_buffer_rsrc_t ry = front_rsrc(A.fy, 8 * A.fy_o);
    const __amdgpu_buffer_rsrc_t rz = front_rsrc(A.fz, 8 * A.fz_o);
    Real xf[4] = {0, 0, 0, 0}, yf[B][4] = {}, zf[B][B][4] = {};
    // FP32 mass-inverse and matrix-core network kernels load the next cell's
    // sigma_t and source while the current cell is solved: the loads are
    // unconditional (an invalid cell reads element 0), so they can leave a
    // cell ahead.  The dense, paper-form network and FP64 kernels would lose
    // a wave per SIMD to the 9 (18) registers, and anisotropic sweeps load
    // their moment sources per cell.
    constexpr bool kPrefetch = sizeof(Real) == 4 && (Form == kFormMassInv || kNet) &&
                               kMom == 0;
    const uint32_t gbase = g * A.ncell;
    auto cell_ok = [&](int il2, int jl2, int kl2) {
        return tvalid && I0 + il2 < A.nx && J0 + jl2 < A.ny && K0 + kl2 < A.nz;
    };
    Real pst = 0, psc[8];
    if constexpr (kPrefetch) {
        const uint32_t gc = cell_ok(0, 0, 0) ? gbase + c0 : 0u;
        pst = A.sigma_t[gc];
        load8_reflect(A.src + gc * 8, mask, psc);
    }
    // layers of the tile (kl) are a rolled loop for B > 2 (the layer body,
    // B^2 cells, is unrolled so that every register front index is static)
#pragma unroll(B <= 2 ? B : 1)
    for (int kl = 0; kl < B; ++kl)
#pragma unroll
        for (int jl = 0; jl < B; ++jl)
#pragma unroll
            for (int il = 0; il < B; ++il) {
                const int cidx = il + B * (jl + B * kl);
                const uint32_t ic = I0 + il, jc = J0 + jl, kc = K0 + kl;
                const bool ok = tvalid && ic < A.nx && jc < A.ny && kc < A.nz;
                Real psi[8];
                uint32_t c = 0;
                Real gs = 0, gq = 0;
                Real st = 0, sc[8], vx[4], vy[4], vz[4];
                uint32_t ex = 0, ey = 0, ez = 0;   // front slots (elements)
                if constexpr (kPrefetch) {
                    st = pst;
#pragma unroll
                    for (int n = 0; n < 8; ++n) sc[n] = psc[n];
                    // the next cell of the tile in upwind order
                    const int il2 = il + 1 < B ? il + 1 : 0;
                    const int jl2 = il + 1 < B ? jl : (jl + 1 < B ? jl + 1 : 0);
                    const int kl2 = (il + 1 < B || jl + 1 < B) ? kl : kl + 1;
                    if (kl2 < B) {
                        const uint32_t gc = cell_ok(il2, jl2, kl2)
                                                ? gbase + c0 + il2 * sx + jl2 * sy + kl2 * sz
                                                : 0u;
                        pst = A.sigma_t[gc];
                        load8_reflect(A.src + gc * 8, mask, psc);
                    }
                }
                if constexpr (kStage) {
                    // the segment's lanes share the cell (ok is uniform over
                    // the segment); every lane of the wave reaches the sync
                    if (stage) {
                        if (ok) {
                            const uint32_t gcs = gbase + c0 + il * sx + jl * sy + kl * sz;
                            const f32x4 *srcv =
                                reinterpret_cast<const f32x4 *>(A.msrc + (size_t)gcs * (kMom * 8));
                            f32x4 *dst = reinterpret_cast<f32x4 *>(mslot);
                            for (int q = d; q < 2 * kMom; q += (int)A.Do) dst[q] = srcv[q];
                        }
                        wave_lds_sync();
                    }
                }
                // gather: sigma_t, the reflected source and the three inflows
                if (ok) {
                    c = c0 + il * sx + jl * sy + kl * sz;
                    const uint32_t gc = gbase + c;
                    if constexpr (!kPrefetch) {
                        st = A.sigma_t[gc];
                        if constexpr (Form == kFormDense) {
                            // (the address form costs this kernel a wave per SIMD)
                            load4(A.src + gc * 8, sc);
                            load4(A.src + gc * 8 + 4, sc + 4);
                            reflect8(sc, mask);
                        } else {
                            load8_reflect(A.src + gc * 8, mask, sc);
                        }
                    }
                    if constexpr (kMom > 0) {
                        if (stage)
                            add_moment_source_staged<Real, kMom>(mslot, yl, mask, sc);
                        else
                            add_moment_source<Real, kMom>(A, yl, gc, mask, sc);
                    }
                    ex = ex0 + kl * A.fx_k + jl * A.fx_j;
                    ey = ey0 + kl * A.fy_k + il * A.fy_j;
                    ez = ez0 + jl * A.fz_k + il * A.fz_j;
                    if (il > 0) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) vx[e] = xf[e];
                    } else if (ic) {
                        front_load<Real, kCoh>(A.fx, rx, ex, vx);
                    } else {
                        vx[0] = vx[1] = vx[2] = vx[3] = inc[0];
                    }
                    if (jl > 0) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) vy[e] = yf[il][e];
                    } else if (jc) {
                        front_load<Real, kCoh>(A.fy, ry, ey, vy);
                    } else {
                        vy[0] = vy[1] = vy[2] = vy[3] = inc[1];
                    }
                    if (kl > 0) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) vz[e] = zf[jl][il][e];
                    } else if (kc) {
                        front_load<Real, kCoh>(A.fz, rz, ez, vz);
                    } else {
                        vz[0] = vz[1] = vz[2] = vz[3] = inc[2];
                    }
                }
                // local solve
                if constexpr (kNet) {
                    float feat[24], y[8];
                    float m = 0.0f;
                    if (ok) {
                        m = ann_features(kap, A.hh, st, sc, vx, vy, vz, feat);
                    } else {
                        // a lane without a cell takes whatever its feature
                        // registers hold (an empty asm defines them, no
                        // instruction): each sample is its own column of the
                        // matrix products, so these inputs reach only this
                        // lane's outputs, which the select below drops
#pragma unroll
                        for (int e = 0; e < 24; ++e) asm volatile("" : "=v"(feat[e]));
                    }
                    ann_wave<Form == kFormAnnSplit>(R, feat, y);
#pragma unroll
                    for (int n = 0; n < 8; ++n) psi[n] = ok ? m * y[n] : 0.0f;
                } else if constexpr (kPaper) {
                    if (ok) {
                        // the octant's network, or the lane's direction's
                        // (from the block's LDS copy, pann_lds)
                        constexpr bool kUni = Form == kFormAnnPaper;
                        const float *wimg =
                            kUni ? static_cast<const float *>(A.ann_params) + o * kPannStride
                                 : pann_lds + (lane_ok ? d : 0) * kPannLdsStride;
                        pann_cell<kUni>(wimg, kap, st, sc, vx, vy, vz, psi);
                    } else {
#pragma unroll
                        for (int n = 0; n < 8; ++n) psi[n] = 0;
                    }
                } else if constexpr (Form == kFormMassInv) {
                    // (P_d + sigma_t I) psi = S + sum_a kappa_a c_a.  The
                    // factorisation is redone per cell: keeping it for the
                    // next cells of the tile (same sigma_t) saves half the
                    // arithmetic but holds 50 more registers per lane, which
                    // costs a wave per SIMD and more time than it saves.
                    if (ok) {
                        Real a[8][8];
                        massinv_matrix(kap, st, a);
                        massinv_rhs(kap, sc, vx, vy, vz, psi);
                        if (__any(ge_solve8_cube(a, psi))) {
                            // some lane of the wave needs a row exchange: the
                            // wave redoes the cell with the dense pivoted
                            // elimination
                            massinv_matrix(kap, st, a);
                            massinv_rhs(kap, sc, vx, vy, vz, psi);
                            ge_solve8(a, psi);
                        }
                    } else {
#pragma unroll
                        for (int n = 0; n < 8; ++n) psi[n] = 0;
                    }
                } else {
                    if (ok) {
                        dense_cell_solve(dp, kap, st, sc, vx, vy, vz, psi);
                    } else {
#pragma unroll
                        for (int n = 0; n < 8; ++n) psi[n] = 0;
                    }
                }
                // scatter: register fronts, tile-boundary fronts, psi store or
                // adjoint contraction
                // the register fronts take psi on every lane (zero where the
                // lane has no cell): a cell of the tile that exists never
                // reads a front written by one that does not, since the
                // cells beyond the mesh in a tile lie downstream of it
                xf[0] = psi[1]; xf[1] = psi[3]; xf[2] = psi[5]; xf[3] = psi[7];
                yf[il][0] = psi[2]; yf[il][1] = psi[3]; yf[il][2] = psi[6]; yf[il][3] = psi[7];
                zf[jl][il][0] = psi[4]; zf[jl][il][1] = psi[5];
                zf[jl][il][2] = psi[6]; zf[jl][il][3] = psi[7];
                if (ok) {
                    // a tile's last cell hands its outflow downstream; on the
                    // domain boundary there is no downstream cell, and the
                    // outflow is stored only for the balance tally (keep_out;
                    // the run uses whole tiles then, so the boundary cell is a
                    // tile's last)
                    if (il == B - 1 && (ic + 1 < A.nx || A.keep_out))
                        front_store<Real, kCoh>(A.fx, rx, ex, psi[1], psi[3], psi[5], psi[7]);
                    if (jl == B - 1 && (jc + 1 < A.ny || A.keep_out))
                        front_store<Real, kCoh>(A.fy, ry, ey, psi[2], psi[3], psi[6], psi[7]);
                    if (kl == B - 1 && (kc + 1 < A.nz || A.keep_out))
                        front_store<Real, kCoh>(A.fz, rz, ez, psi[4], psi[5], psi[6], psi[7]);
                    if (kStorePsi || (kAdjoint && A.grad_oct)) {
                        Real *pp = A.psi + ((size_t)slot * A.ncell + c) * 8;
                        if (kStorePsi) {
                            store8_reflect(pp, mask, psi);
                        } else {
                            // mu^T M psi with the stored forward flux, M = V M3
                            Real pf[8], m[8];
                            load8_reflect(pp, mask, pf);
                            mass3_216(pf, m);
                            Real s = 0, sm = 0;
#pragma unroll
                            for (int n = 0; n < 8; ++n) {
                                s = fma(psi[n], m[n], s);
                                sm += psi[n];
                            }
                            gs = -w * A.vol * s * Real(1.0 / 216.0);
                            gq = w * A.vol * sm * Real(0.125);
                        }
                    }
                }
                // deterministic per-octant reduction over the directions
                Real *rb = L.red + (cidx & 1) * (256 * 9);
#pragma unroll
                for (int n = 0; n < 8; ++n) rb[tid * 9 + n] = w * psi[n];
                if (kAdjoint) {
                    L.gred[tid * 2 + 0] = gs;
                    L.gred[tid * 2 + 1] = gq;
                }
                wave_lds_sync();   // a segment's lanes are in one wave
                if (ok) {
                    const int base = tid - d;
                    const uint32_t out = ((o * A.G + g) * A.ncell + c) * 8;
                    for (int n = d; n < 8; n += (int)A.Do) {
                        Real s = 0;
                        if constexpr (kMom > 0) {
                            // the octant's flux moments of this node from the
                            // same weighted values (Eq. (T8) over the octant)
                            Real mk[kMom];
#pragma unroll
                            for (int k = 0; k < kMom; ++k) mk[k] = 0;
                            for (int e = 0; e < (int)A.Do; ++e) {
                                const Real v = rb[(base + e) * 9 + n];
                                s += v;
#pragma unroll
                                for (int k = 0; k < kMom; ++k)
                                    mk[k] = fma(ytab[e * kYlmStride + k], v, mk[k]);
                            }
                            Real *mo = A.mom_oct + ((size_t)out + (n ^ mask)) * kMom;
#pragma unroll
                            for (int k = 0; k < kMom; ++k) __builtin_nontemporal_store(mk[k], mo + k);
                        } else {
                            for (int e = 0; e < (int)A.Do; ++e) s += rb[(base + e) * 9 + n];
                        }
                        // written once, read once by the octant reduction: a
                        // non-temporal store leaves the cache to the fronts
                        // where one store covers a cell's nodes (6 or more
                        // direction lanes); with fewer, a lane stores several
                        // nodes and the cache has to merge them
                        if (A.Do >= 6)
                            __builtin_nontemporal_store(s, A.phi_oct + out + (n ^ mask));
                        else
                            A.phi_oct[out + (n ^ mask)] = s;
                    }
                    if (kAdjoint && A.grad_oct) {
                        for (int k2 = d; k2 < 2; k2 += (int)A.Do) {
                            Real s = 0;
                            for (int e = 0; e < (int)A.Do; ++e) s += L.gred[(base + e) * 2 + k2];
                            A.grad_oct[((o * A.G + g) * A.ncell + c) * 2 + k2] = s;
                        }
                    }
                }
                if (kAdjoint) wave_lds_sync();
            }
}

}  // namespace dgsn
