// Hyperplane sweep kernels of the DGFEM S_n transport sweep (Sec. 2, the
// sweep paragraph after Eq. (T12)) with the Gaussian-elimination local solver
// (Eq. (T12), the step the paper identifies as the most expensive).
//
// Work decomposition.  In canonical coordinates (every direction reflected
// into the positive octant) cell (i', j', k') depends only on its three
// lower neighbours, so all cells with i' + j' + k' = p are independent.  One
// launch processes hyperplane p of all 8 octants, for every direction of the
// octant and every group: one lane per (octant, cell, group, direction), the
// direction index fastest.  The 8x8 system of each lane lives in registers.
//
// Data in HBM (Real = float or double):
//   sigma_t [G][ncell], src [G][ncell][8]               physical node order
//   front_x [8][nz][ny][4][Do*G], front_y [8][nz][nx][4][Do*G],
//   front_z [8][ny][nx][4][Do*G]     canonical face values, overwritten in
//           place: a cell reads its inflow slot and writes its outflow into
//           the same slot, which the downstream cell reads one step later.
//   phi_oct [8][G][ncell][8]          per-octant partial scalar flux (no
//           atomics: the 8 partials are summed in a fixed order afterwards).
#include "sweep_body.hpp"

namespace dgsn {

namespace {

template <typename Real, int Form, int B, bool kStorePsi, bool kAdjoint, int kMom = 0>
__global__ __launch_bounds__(256, (kMinWavesPerSimd<Real, Form, B, kMom>)) void sweep_tile_ge(PlaneArgs<Real> A)
{
    // 256 lanes: (direction, group, tile slot) segments, grid = (tile blocks, octant)
    __shared__ TileLds<Real> L;
    const int tid = threadIdx.x;
    const SegLane l = seg_lane(A, tid);
    bool tvalid;
    const uint32_t pt = step_tile(A.cells, A.ncp, blockIdx.x * (int)A.nc + l.z, l.ok, tvalid);
    const Real inc[3] = {A.inc[blockIdx.y][0], A.inc[blockIdx.y][1], A.inc[blockIdx.y][2]};
    __shared__ Real ytab[kMom > 0 ? 64 * kYlmStride : 1];
    __shared__ __align__(16) Real mstage[kStageFloats<Real, kMom>];
    if constexpr (kMom > 0) load_ylm_table(A, (int)blockIdx.y, ytab);
    if constexpr (Form == kFormAnnPaperDir) {
        load_pann_dir_table(static_cast<const float *>(A.ann_params), (int)blockIdx.y, (int)A.Do,
                            dgsn_dyn_lds);
        __syncthreads();
    }
    tile_body<Real, Form, B, kStorePsi, kAdjoint, false, kMom>(A, inc, l.d, l.g, tid, tvalid, pt,
                                                               blockIdx.y, l.ok, L, ytab, mstage,
                                                               dgsn_dyn_lds);
}

// ANN tile sweep: the same lane layout (full waves for the matrix cores).
template <int B, int Form>
__global__ __launch_bounds__(256) void sweep_tile_ann(PlaneArgs<float> A)
{
    __shared__ TileLds<float> L;
    const int tid = threadIdx.x;
    const SegLane l = seg_lane(A, tid);
    bool tvalid;
    const uint32_t pt = step_tile(A.cells, A.ncp, blockIdx.x * (int)A.nc + l.z, l.ok, tvalid);
    const float inc[3] = {A.inc[blockIdx.y][0], A.inc[blockIdx.y][1], A.inc[blockIdx.y][2]};
    tile_body<float, Form, B, false, false>(A, inc, l.d, l.g, tid, tvalid, pt, blockIdx.y,
                                                l.ok, L);
}

// phi = sum_o phi_oct[o]; optionally the FP64 SI residual partials, the
// absorption and source partials of the balance tally, and the next source
// S = qn + qc + sigma_s/(4 pi) phi.
template <typename Real>
__global__ __launch_bounds__(256) void reduce_octants(ReduceArgs<Real> R)
{
    __shared__ double sh[5][256];
    double dmax = 0.0, fmax = 0.0, esum = 0.0, babs = 0.0, bsrc = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < R.nv; e += stride) {
        Real nw[8];
#pragma unroll
        for (int n = 0; n < 8; ++n) nw[n] = 0;
        // the octant partials are read once: non-temporal loads keep them
        // from displacing the sweep's fronts in the last-level cache
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const Real *p = R.phi_oct + ((long long)o * R.nv + e) * 8;
#pragma unroll
            for (int n = 0; n < 8; ++n) nw[n] += __builtin_nontemporal_load(p + n);
        }
        Real *ph = R.phi + e * 8;
        if (R.resid) {
            const Real *po = R.phi_prev ? R.phi_prev + e * 8 : ph;
            double an = 0.0, ao = 0.0;
#pragma unroll
            for (int n = 0; n < 8; ++n) {
                const double vn = (double)nw[n], vo = (double)__builtin_nontemporal_load(po + n);
                dmax = fmax_d(dmax, fabs(vn - vo));
                fmax = fmax_d(fmax, fabs(vn));
                an += vn;
                ao += vo;
            }
            an *= 0.125;
            ao *= 0.125;
            esum += (an != 0.0) ? fabs(an - ao) / fabs(an) : (ao != 0.0 ? 1.0 : 0.0);
        }
        if (R.balance) {
            // the sweep's source is read before the next one overwrites it
            double fs = 0.0, ss = 0.0;
#pragma unroll
            for (int n = 0; n < 8; ++n) {
                fs += (double)nw[n];
                ss += (double)R.src_sweep[e * 8 + n];
            }
            babs = fma((double)R.sigma_t[e], fs, babs);
            bsrc += ss;
        }
#pragma unroll
        for (int n = 0; n < 8; ++n) __builtin_nontemporal_store(nw[n], ph + n);
        if (R.src_next) {
            const Real ss = R.sigma_s ? R.sigma_s[e] * Real(kInv4Pi) : Real(0);
            const Real qc = R.q_cell ? R.q_cell[e] : Real(0);
#pragma unroll
            for (int n = 0; n < 8; ++n) {
                const Real qn = R.q_nodal ? R.q_nodal[e * 8 + n] : Real(0);
                R.src_next[e * 8 + n] = fma(ss, nw[n], qc + qn);
            }
        }
    }
    if (!R.resid && !R.balance) return;
    const int tid = threadIdx.x;
    sh[0][tid] = dmax;
    sh[1][tid] = fmax;
    sh[2][tid] = esum;
    sh[3][tid] = babs;
    sh[4][tid] = bsrc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
            sh[0][tid] = fmax_d(sh[0][tid], sh[0][tid + s]);
            sh[1][tid] = fmax_d(sh[1][tid], sh[1][tid + s]);
            sh[2][tid] += sh[2][tid + s];
            sh[3][tid] += sh[3][tid + s];
            sh[4][tid] += sh[4][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        double *pb = R.partials + (size_t)blockIdx.x * kRedStride;
        pb[kRedMaxD] = sh[0][0];
        pb[kRedMaxF] = sh[1][0];
        pb[kRedEps] = sh[2][0];
        pb[kRedAbs] = sh[3][0];
        pb[kRedSrc] = sh[4][0];
    }
}

// Boundary leakage of the balance tally.  After a sweep run with keep_out,
// the slot of every front row holds the outflow face of the row's last cell,
// on the domain boundary.  Each thread takes one face slot (octant,
// row, direction-group) of one of the three fronts and adds
// w_d kappa_a(d) (psi_0 + psi_1 + psi_2 + psi_3) in FP64; the outflow
// integral over the face is V kappa_a times the mean of the four values.
template <typename Real>
__global__ __launch_bounds__(256) void leakage(PlaneArgs<Real> A, double *partials)
{
    __shared__ double sh[256];
    const uint32_t DG = A.DG;
    const long long nx_slots = 8LL * A.nz * A.ny * DG;
    const long long ny_slots = 8LL * A.nz * A.nx * DG;
    const long long nz_slots = 8LL * A.ny * A.nx * DG;
    const long long total = nx_slots + ny_slots + nz_slots;
    double acc = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        // each front holds fewer than 2^31 elements, so a slot index fits 32 bits
        int axis;
        uint32_t r;
        const Real *f;
        uint32_t per_octant;
        if (t < nx_slots) {
            axis = 0; r = (uint32_t)t; f = A.fx; per_octant = A.nz * A.ny * DG;
        } else if (t < nx_slots + ny_slots) {
            axis = 1; r = (uint32_t)(t - nx_slots); f = A.fy; per_octant = A.nz * A.nx * DG;
        } else {
            axis = 2; r = (uint32_t)(t - nx_slots - ny_slots); f = A.fz;
            per_octant = A.ny * A.nx * DG;
        }
        // r = (octant * rows + row) * DG + dg, dg = d + Do * g
        const uint32_t o = r / per_octant;
        const uint32_t dg = r % DG;
        const uint32_t d = dg % A.Do;
        const Real *dp = A.dir + (o * A.Do + d) * kDirStride;
        const Real *v = f + (size_t)r * 4;
        const double s = (double)v[0] + (double)v[1] + (double)v[2] + (double)v[3];
        acc = fma((double)dp[kDirW] * (double)dp[kDirK + axis], s, acc);
    }
    const int tid = threadIdx.x;
    sh[tid] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    if (tid == 0) partials[(size_t)blockIdx.x * kRedStride + kRedLeak] = sh[0];
}

// result[k] over the block partials: maxima for the residual terms, sums for
// the others (summed in block order, so the result is reproducible);
// nterms = kRedLeak + 1 with the balance tally, kRedEps + 1 without.
__global__ __launch_bounds__(256) void finalize_partials(const double *partials, int nblocks,
                                                         int nterms, double *result)
{
    __shared__ double sh[kRedLeak + 1][256];
    const int tid = threadIdx.x;
    double v[kRedLeak + 1];
#pragma unroll
    for (int k = 0; k <= kRedLeak; ++k) v[k] = 0.0;
    for (int i = tid; i < nblocks; i += blockDim.x) {
        const double *pb = partials + (size_t)i * kRedStride;
        v[kRedMaxD] = fmax_d(v[kRedMaxD], pb[kRedMaxD]);
        v[kRedMaxF] = fmax_d(v[kRedMaxF], pb[kRedMaxF]);
        for (int k = kRedEps; k < nterms; ++k) v[k] += pb[k];
    }
#pragma unroll
    for (int k = 0; k <= kRedLeak; ++k) sh[k][tid] = v[k];
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (tid < st) {
            sh[kRedMaxD][tid] = fmax_d(sh[kRedMaxD][tid], sh[kRedMaxD][tid + st]);
            sh[kRedMaxF][tid] = fmax_d(sh[kRedMaxF][tid], sh[kRedMaxF][tid + st]);
#pragma unroll
            for (int k = kRedEps; k <= kRedLeak; ++k) sh[k][tid] += sh[k][tid + st];
        }
        __syncthreads();
    }
    if (tid < nterms) result[tid] = sh[tid][0];
}

// S = q + sigma_s/(4 pi) phi  (initial source of an SI run)
template <typename Real>
__global__ __launch_bounds__(256) void build_source(long long nv, const Real *q,
                                                    const Real *sigma_s, const Real *phi,
                                                    Real *src)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nv * 8; e += stride) {
        const long long gc = e >> 3;
        src[e] = fma(sigma_s[gc] * Real(kInv4Pi), phi[e], q[gc]);
    }
}

// Multigroup source (the group sum of the isotropic scattering source): one
// thread per (cell, node); the G fluxes of the node, and the cell's G x G
// matrix from its cell-major run [c][g'][g] (the 8 threads of a cell share
// it).  Summed over the source group in ascending order.
template <typename Real>
__global__ __launch_bounds__(256) void build_source_gg(long long ncell, int G,
                                                       const Real *__restrict__ q_cell,
                                                       const Real *__restrict__ q_nodal,
                                                       const Real *__restrict__ sigma_gg,
                                                       const Real *__restrict__ phi,
                                                       Real *__restrict__ src, int transpose)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < ncell * 8;
         e += stride) {
        const long long c = e >> 3;
        const int n = (int)(e & 7);
        for (int g = 0; g < G; ++g) {
            const long long gc = (long long)g * ncell + c;
            Real v = q_cell ? q_cell[gc] : Real(0);
            if (q_nodal) v += q_nodal[gc * 8 + n];
            const Real *sig = sigma_gg + c * G * G;
            for (int g2 = 0; g2 < G; ++g2) {
                const Real s = sig[transpose ? g * G + g2 : g2 * G + g];
                v = fma(s * Real(kInv4Pi), phi[((long long)g2 * ncell + c) * 8 + n], v);
            }
            src[gc * 8 + n] = v;
        }
    }
}

// Flux moments of anisotropic scattering: one thread per (group, cell, node,
// moment) in the sweep's layout; the octant partials are summed in octant
// order, and the source moment is sigma_{s,n} times the moment, n the order
// of moment k.  Moments and source moments are stored [G][ncell][nm-1][8],
// so a wave's stores stay within a few cells.
template <typename Real>
__global__ __launch_bounds__(256) void reduce_moments(long long nv, int nm,
                                                      const Real *__restrict__ mom_oct,
                                                      const Real *__restrict__ sigma_sn,
                                                      Real *__restrict__ mom,
                                                      Real *__restrict__ msrc)
{
    const int nk = nm - 1;
    const long long total = nv * nk * 8;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const long long gc = e / (nk * 8);
        const int r = (int)(e - gc * (nk * 8));
        const int n = r / nk;
        const int k = r - n * nk + 1;
        Real s = 0;
        for (int o = 0; o < 8; ++o) s += __builtin_nontemporal_load(mom_oct + (long long)o * total + e);
        const int order = k >= 9 ? 3 : (k >= 4 ? 2 : 1);
        const long long m = (gc * nk + (k - 1)) * 8 + n;
        mom[m] = s;
        if (msrc) msrc[m] = sigma_sn[(long long)(order - 1) * nv + gc] * s;
    }
}

// The public layout of the flux moments: dst[k][gc][n] = src[gc][k][n] (one
// thread per destination value).
template <typename Real>
__global__ __launch_bounds__(256) void moments_public(long long nv, int nk,
                                                      const Real *__restrict__ src,
                                                      Real *__restrict__ dst)
{
    const long long total = nv * nk * 8;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const long long kg = e >> 3;
        const int n = (int)(e & 7);
        const int k = (int)(kg / nv);
        const long long gc = kg - (long long)k * nv;
        dst[e] = src[(gc * nk + k) * 8 + n];
    }
}

// Debug poisoning of the face fronts: every element set to a quiet NaN.
template <typename Real>
__global__ __launch_bounds__(256) void fill_nan(long long n, Real *__restrict__ p)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        p[e] = __builtin_nan("");
}

// Validity of the materials: bit 0 when some sigma_t is negative or not
// finite, bit 1 likewise for sigma_s, bit 2 when some q is not finite, bit 3
// when some sigma_s exceeds its cell's sigma_t (a vector atomic OR into *bad
// per offending thread).
template <typename Real>
__global__ __launch_bounds__(256) void check_materials(long long n, const Real *__restrict__ st,
                                                       const Real *__restrict__ ss,
                                                       const Real *__restrict__ q,
                                                       unsigned *__restrict__ bad)
{
    unsigned b = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const Real t = st[e], s = ss[e], v = q[e];
        if (!(t >= Real(0)) || isinf(t)) b |= 1u;   // a NaN fails the comparison
        if (!(s >= Real(0)) || isinf(s)) b |= 2u;
        if (!isfinite(v)) b |= 4u;
        if (s > t) b |= 8u;
    }
    if (b) atomicOr(bad, b);
}

// Cell-major copy of per-cell matrices: dst[c][j] = src[j][c] for nmat
// values j per cell (one thread per destination value).
template <typename Real>
__global__ __launch_bounds__(256) void cell_major(long long ncell, int nmat,
                                                  const Real *__restrict__ src,
                                                  Real *__restrict__ dst)
{
    const long long total = ncell * nmat;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const long long c = e / nmat;
        const int j = (int)(e - c * nmat);
        dst[e] = src[(long long)j * ncell + c];
    }
}

// Source moments of group-to-group anisotropic scattering: one thread per
// (cell, moment, node) in the layout of one group's block of msrc and mom,
// looping over the destination group g and summing the source groups g' in
// ascending order: msrc[g][c][k-1][n] = sum_g' sigma_{s,n(k)}(g' -> g)[c] mom[g'][c][k-1][n]
// (transpose: sigma(g -> g')).  sigma_cm [ncell][L][G][G] holds orders 1..L
// cell-major, from g' into g at [c][n-1][g'][g], so that the G*G matrix a
// thread reads lies in one run.
template <typename Real>
__global__ __launch_bounds__(256) void build_msrc_gg(long long ncell, int G, int nm, int L,
                                                     const Real *__restrict__ sigma_cm,
                                                     const Real *__restrict__ mom,
                                                     Real *__restrict__ msrc, int transpose)
{
    const int nk = nm - 1;
    const long long per_group = ncell * nk * 8;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < per_group;
         e += stride) {
        const long long c = e / (nk * 8);
        const int r = (int)(e - c * (nk * 8));
        const int k = (r >> 3) + 1;   // the node is r & 7
        const int order = k >= 9 ? 3 : (k >= 4 ? 2 : 1);
        const Real *sig = sigma_cm + (c * L + (order - 1)) * G * G;
        const Real *mk = mom + e;
        // the source groups' moments of this (cell, moment, node) are read
        // once, 16 at a time into registers (clamped loads, in bounds), and
        // serve every destination group; past 16 groups the partial sums
        // continue in msrc
        for (int g0 = 0; g0 < G; g0 += 16) {
            Real mv[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) mv[j] = mk[(long long)min(g0 + j, G - 1) * per_group];
            for (int g = 0; g < G; ++g) {
                Real *out = msrc + (long long)g * per_group + e;
                Real v = g0 ? *out : Real(0);
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int g2 = g0 + j;
                    if (g2 < G) {
                        v = fma(sig[transpose ? g * G + g2 : g2 * G + g], mv[j], v);
                    }
                }
                *out = v;
            }
        }
    }
}

// adjoint load: gl = M3^{-1} g / V (so that M3 gl = g / V)
template <typename Real>
__global__ __launch_bounds__(256) void adjoint_load(long long nv, const Real *gphi, Real inv_vol,
                                                    Real *gl)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nv; e += stride) {
        Real v[8], o[8];
#pragma unroll
        for (int n = 0; n < 8; ++n) v[n] = gphi[e * 8 + n] * inv_vol;
        mass3_inv(v, o);
#pragma unroll
        for (int n = 0; n < 8; ++n) gl[e * 8 + n] = o[n];
    }
}

template <typename Real>
__global__ __launch_bounds__(256) void reduce_grad(long long nv, const Real *grad_oct,
                                                   Real *grad_st, Real *grad_q)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nv; e += stride) {
        Real s = 0, q = 0;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            s += grad_oct[((long long)o * nv + e) * 2 + 0];
            q += grad_oct[((long long)o * nv + e) * 2 + 1];
        }
        if (grad_st) grad_st[e] = s;
        if (grad_q) grad_q[e] = q;
    }
}

int grid_for(long long n, int cap = 4096)
{
    long long b = (n + 255) / 256;
    if (b < 1) b = 1;
    return (int)(b > cap ? cap : b);
}

}  // namespace

int block_size_for(int Do) { return Do * (256 / Do); }

int cells_per_block(int Do, int G) { return Do > 64 ? 0 : 4 * (64 / Do) / G; }



template <typename Real, int Form, int B>
void launch_tile_form(const PlaneArgs<Real> &A, bool store_psi, bool adjoint, dim3 grid,
                      dim3 block, hipStream_t s)
{
    // anisotropic sweeps: tile edges 1 and 2 (the run clamps larger tiles);
    // the psi store and the adjoint with the mass-inverse form only
    if constexpr (B <= 2) {
        if (A.nmom > 1) {
            if constexpr (Form == kFormMassInv) {
                if (adjoint || store_psi) {
                    if (A.nmom == 4 && adjoint)
                        hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, false, true, 3>), grid, block,
                                           0, s, A);
                    else if (A.nmom == 4)
                        hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, true, false, 3>), grid, block,
                                           0, s, A);
                    else if (A.nmom == 9 && adjoint)
                        hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, false, true, 8>), grid, block,
                                           0, s, A);
                    else if (A.nmom == 9)
                        hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, true, false, 8>), grid, block,
                                           0, s, A);
                    else if (adjoint)
                        hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, false, true, 15>), grid, block,
                                           0, s, A);
                    else
                        hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, true, false, 15>), grid, block,
                                           0, s, A);
                    return;
                }
            }
            if (A.nmom == 4)
                hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, false, false, 3>), grid, block, 0,
                                   s, A);
            else if (A.nmom == 9)
                hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, false, false, 8>), grid, block, 0,
                                   s, A);
            else
                hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, false, false, 15>), grid, block,
                                   0, s, A);
            return;
        }
    }
    if (adjoint)
        hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, false, true>), grid, block, 0, s, A);
    else if (store_psi)
        hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, true, false>), grid, block, 0, s, A);
    else
        hipLaunchKernelGGL((sweep_tile_ge<Real, Form, B, false, false>), grid, block, 0, s, A);
}

template <typename Real, int Form>
void launch_tile_b(const PlaneArgs<Real> &A, int b, bool store_psi, bool adjoint, dim3 grid,
                   dim3 block, hipStream_t s)
{
    switch (b) {
    case 3: launch_tile_form<Real, Form, 3>(A, store_psi, adjoint, grid, block, s); break;
    case 2: launch_tile_form<Real, Form, 2>(A, store_psi, adjoint, grid, block, s); break;
    default: launch_tile_form<Real, Form, 1>(A, store_psi, adjoint, grid, block, s); break;
    }
}

int launch_tile_ann(const PlaneArgs<float> &A, int b, bool split, hipStream_t s)
{
    const dim3 grid((A.ncp + A.nc - 1) / A.nc, 8);
    if (split) {
        switch (b) {
        case 3: hipLaunchKernelGGL((sweep_tile_ann<3, kFormAnnSplit>), grid, dim3(256), 0, s, A); break;
        case 2: hipLaunchKernelGGL((sweep_tile_ann<2, kFormAnnSplit>), grid, dim3(256), 0, s, A); break;
        default: hipLaunchKernelGGL((sweep_tile_ann<1, kFormAnnSplit>), grid, dim3(256), 0, s, A); break;
        }
    } else {
        switch (b) {
        case 3: hipLaunchKernelGGL((sweep_tile_ann<3, kFormAnn>), grid, dim3(256), 0, s, A); break;
        case 2: hipLaunchKernelGGL((sweep_tile_ann<2, kFormAnn>), grid, dim3(256), 0, s, A); break;
        default: hipLaunchKernelGGL((sweep_tile_ann<1, kFormAnn>), grid, dim3(256), 0, s, A); break;
        }
    }
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

// The paper-form networks (per octant or per direction): FP32 forward
// sweeps only.
template <int Form>
void launch_tile_pann(const PlaneArgs<float> &A, int b, dim3 grid, dim3 block, hipStream_t s)
{
    // the per-direction images of the block's octant in dynamic LDS
    const size_t lds = Form == kFormAnnPaperDir ? (size_t)A.Do * kPannLdsStride * 4 : 0;
    switch (b) {
    case 3:
        hipLaunchKernelGGL((sweep_tile_ge<float, Form, 3, false, false>), grid, block, lds, s, A);
        break;
    case 2:
        hipLaunchKernelGGL((sweep_tile_ge<float, Form, 2, false, false>), grid, block, lds, s, A);
        break;
    default:
        hipLaunchKernelGGL((sweep_tile_ge<float, Form, 1, false, false>), grid, block, lds, s, A);
        break;
    }
}

template <typename Real>
int launch_tile(const PlaneArgs<Real> &A, int form, int b, bool store_psi, bool adjoint,
                hipStream_t s)
{
    const dim3 block(256);
    const dim3 grid((A.ncp + A.nc - 1) / A.nc, 8);
    const bool paper = form == kFormAnnPaper || form == kFormAnnPaperDir;
    if (paper && (sizeof(Real) != 4 || store_psi || adjoint))
        return set_error(DGSN_EUNSUPPORTED, "the paper-form network runs FP32 forward sweeps");
    if (A.nmom > 1 && (paper || (form == kFormDense && (store_psi || adjoint))))
        return set_error(DGSN_EUNSUPPORTED, "anisotropic sweeps run the GE solvers (the psi "
                         "store and the adjoint with the mass-inverse form)");
    if (A.nmom > 1 && ((A.nmom != 4 && A.nmom != 9 && A.nmom != 16) || b > 2))
        return set_error(DGSN_EINVAL, "anisotropic sweeps take (L+1)^2 moments, L = 1..3, and "
                         "tile edges 1..2 (moments %u, tile %d)", A.nmom, b);
    if (form == kFormDense) {
        launch_tile_b<Real, kFormDense>(A, b, store_psi, adjoint, grid, block, s);
    } else if (form == kFormAnnPaper) {
        if constexpr (sizeof(Real) == 4) launch_tile_pann<kFormAnnPaper>(A, b, grid, block, s);
    } else if (form == kFormAnnPaperDir) {
        if constexpr (sizeof(Real) == 4) launch_tile_pann<kFormAnnPaperDir>(A, b, grid, block, s);
    } else {
        launch_tile_b<Real, kFormMassInv>(A, b, store_psi, adjoint, grid, block, s);
    }
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_reduce(const ReduceArgs<Real> &R, int blocks, hipStream_t s)
{
    if ((R.resid || R.balance) && (blocks < 1 || blocks > 2048))
        return set_error(DGSN_EINVAL, "reduction over %d blocks (1..2048)", blocks);
    hipLaunchKernelGGL(reduce_octants<Real>, dim3(blocks), dim3(256), 0, s, R);
    DGSN_HIP(hipGetLastError());
    if (R.resid || R.balance) {
        // with the balance tally the leakage partials of this reduction's
        // blocks have been written by launch_leakage (enqueued before)
        const int nterms = R.balance ? kRedLeak + 1 : kRedEps + 1;
        hipLaunchKernelGGL(finalize_partials, dim3(1), dim3(256), 0, s, R.partials, blocks,
                           nterms, R.result);
        DGSN_HIP(hipGetLastError());
    }
    return DGSN_OK;
}

template <typename Real>
int launch_leakage(const PlaneArgs<Real> &A, double *partials, int blocks, hipStream_t s)
{
    if (blocks < 1 || blocks > 2048)
        return set_error(DGSN_EINVAL, "leakage over %d blocks (1..2048)", blocks);
    hipLaunchKernelGGL(leakage<Real>, dim3(blocks), dim3(256), 0, s, A, partials);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_build_source_gg(long long ncell, int G, const Real *q_cell, const Real *q_nodal,
                           const Real *sigma_gg, const Real *phi, Real *src, bool transpose,
                           hipStream_t s)
{
    hipLaunchKernelGGL(build_source_gg<Real>, dim3(grid_for(ncell * 8)), dim3(256), 0, s, ncell,
                       G, q_cell, q_nodal, sigma_gg, phi, src, transpose ? 1 : 0);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_build_source(long long nv, const Real *q, const Real *ss, const Real *phi, Real *src,
                        hipStream_t s)
{
    hipLaunchKernelGGL(build_source<Real>, dim3(grid_for(nv * 8)), dim3(256), 0, s, nv, q, ss,
                       phi, src);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_adjoint_load(long long nv, const Real *gphi, double vol, Real *gl, hipStream_t s)
{
    hipLaunchKernelGGL(adjoint_load<Real>, dim3(grid_for(nv)), dim3(256), 0, s, nv, gphi,
                       Real(1.0 / vol), gl);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_reduce_grad(long long nv, const Real *grad_oct, Real *gst, Real *gq, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_grad<Real>, dim3(grid_for(nv)), dim3(256), 0, s, nv, grad_oct, gst,
                       gq);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_reduce_moments(long long nv, int nm, const Real *mom_oct, const Real *sigma_sn,
                          Real *mom, Real *msrc, hipStream_t s)
{
    if (nm < 2 || nm > kYlmStride) return set_error(DGSN_EINVAL, "bad moment count %d", nm);
    hipLaunchKernelGGL(reduce_moments<Real>, dim3(grid_for((long long)(nm - 1) * nv * 8)),
                       dim3(256), 0, s, nv, nm, mom_oct, sigma_sn, mom, msrc);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_fill_nan(long long n, Real *p, hipStream_t s)
{
    if (n <= 0) return DGSN_OK;
    const long long blocks = std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(fill_nan<Real>, dim3((unsigned)blocks), dim3(256), 0, s, n, p);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_check_materials(long long n, const Real *st, const Real *ss, const Real *q,
                           unsigned *bad, hipStream_t s)
{
    hipLaunchKernelGGL(check_materials<Real>, dim3(grid_for(n)), dim3(256), 0, s, n, st, ss, q,
                       bad);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_moments_public(long long nv, int nm, const Real *src, Real *dst, hipStream_t s)
{
    if (nm < 2 || nm > kYlmStride) return set_error(DGSN_EINVAL, "bad moment count %d", nm);
    hipLaunchKernelGGL(moments_public<Real>, dim3(grid_for((long long)(nm - 1) * nv * 8)),
                       dim3(256), 0, s, nv, nm - 1, src, dst);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_cell_major(long long ncell, int nmat, const Real *src, Real *dst, hipStream_t s)
{
    hipLaunchKernelGGL(cell_major<Real>, dim3(grid_for(ncell * nmat)), dim3(256), 0, s, ncell,
                       nmat, src, dst);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_build_msrc_gg(long long ncell, int G, int nm, const Real *sigma_cm, const Real *mom,
                         Real *msrc, bool transpose, hipStream_t s)
{
    int L = 1;
    while ((L + 1) * (L + 1) < nm) ++L;
    if (nm < 2 || nm > kYlmStride || (L + 1) * (L + 1) != nm)
        return set_error(DGSN_EINVAL, "bad moment count %d", nm);
    hipLaunchKernelGGL(build_msrc_gg<Real>, dim3(grid_for((long long)(nm - 1) * ncell * 8)),
                       dim3(256), 0, s, ncell, G, nm, L, sigma_cm, mom, msrc, transpose ? 1 : 0);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

int reduce_blocks_for(long long nv) { return grid_for(nv, 2048); }

#define DGSN_INST(Real)                                                                        \
    template int launch_tile<Real>(const PlaneArgs<Real> &, int, int, bool, bool, hipStream_t);         \
    template int launch_reduce<Real>(const ReduceArgs<Real> &, int, hipStream_t);              \
    template int launch_leakage<Real>(const PlaneArgs<Real> &, double *, int, hipStream_t);    \
    template int launch_build_source<Real>(long long, const Real *, const Real *, const Real *, \
                                           Real *, hipStream_t);                               \
    template int launch_build_source_gg<Real>(long long, int, const Real *, const Real *,       \
                                              const Real *, const Real *, Real *, bool,         \
                                              hipStream_t);                                     \
    template int launch_adjoint_load<Real>(long long, const Real *, double, Real *,            \
                                           hipStream_t);                                       \
    template int launch_reduce_grad<Real>(long long, const Real *, Real *, Real *, hipStream_t); \
    template int launch_reduce_moments<Real>(long long, int, const Real *, const Real *, Real *,  \
                                             Real *, hipStream_t);                             \
    template int launch_build_msrc_gg<Real>(long long, int, int, const Real *, const Real *,    \
                                            Real *, bool, hipStream_t);                        \
    template int launch_cell_major<Real>(long long, int, const Real *, Real *, hipStream_t);   \
    template int launch_moments_public<Real>(long long, int, const Real *, Real *, hipStream_t); \
    template int launch_fill_nan<Real>(long long, Real *, hipStream_t);                            \
    template int launch_check_materials<Real>(long long, const Real *, const Real *, const Real *, \
                                              unsigned *, hipStream_t);
DGSN_INST(float)
DGSN_INST(double)

}  // namespace dgsn
