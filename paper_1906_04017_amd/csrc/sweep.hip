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
#include "cell.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace dgsn {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;   // 1 / (4 pi)

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

// Mass-inverse cell system (P_d + sigma_t I, S + sum_a kappa_a c_a), with the
// structural zeros of P_d as literal zeros.
template <typename Real>
__device__ __forceinline__ void massinv_system(const Real k[3], Real st, const Real sc[8],
                                               const Real vx[4], const Real vy[4],
                                               const Real vz[4], Real a[8][8], Real b[8])
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

// Canonical cell solve of one lane: builds the system in the chosen form from
// the direction entry, sigma_t, the canonical source and the three inflow
// faces, and returns psi (canonical node order) in b.
template <typename Real, int Form>
__device__ __forceinline__ void cell_solve(const Real *__restrict__ dp, const Real k[3], Real st,
                                           const Real sc[8], const Real vx[4], const Real vy[4],
                                           const Real vz[4], Real b[8])
{
    Real a[8][8];
    if (Form == kFormDense) {
        // paper form: A' = S_d + sigma_t M3, b' = M3 S + sum_a kappa_a Mf psi_a
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
    } else {
        // mass-inverse form: (P_d + sigma_t I) psi = S + sum_a kappa_a c_a
        massinv_system(k, st, sc, vx, vy, vz, a, b);
        if (__any(ge_solve8_cube(a, b))) {
            // some lane of the wave needs a row exchange: redo the wave with
            // the dense elimination and its partial pivoting
            massinv_system(k, st, sc, vx, vy, vz, a, b);
            ge_solve8(a, b);
        }
    }
}

// Inputs of one cell solve, gathered ahead of the solve that uses them.
template <typename Real>
struct CellIn {
    bool ok;
    uint32_t c, ic, jc, kc;
    Real st;
    Real sc[8];
    Real vx[4], vy[4], vz[4];
};

template <typename Real>
__device__ __forceinline__ void gather_cell(const PlaneArgs<Real> &A, int ci, int o, int mask,
                                            uint32_t g, uint32_t dg, CellIn<Real> &in)
{
    in.ok = ci < (int)A.ncp;
    if (!in.ok) return;
    const uint32_t pc = A.cells[ci];
    in.ic = pc & 1023u;
    in.jc = (pc >> 10) & 1023u;
    in.kc = pc >> 20;
    const uint32_t i = (mask & 1) ? A.nx - 1 - in.ic : in.ic;
    const uint32_t j = (mask & 2) ? A.ny - 1 - in.jc : in.jc;
    const uint32_t k = (mask & 4) ? A.nz - 1 - in.kc : in.kc;
    in.c = i + A.nx * (j + A.ny * k);
    const uint32_t gc = g * A.ncell + in.c;
    in.st = A.sigma_t[gc];
    const Real *sp = A.src + gc * 8;
    load4(sp, in.sc);
    load4(sp + 4, in.sc + 4);
    reflect8(in.sc, mask);
    // inflow faces: boundary value or the upwind neighbour's outflow;
    // fronts are [octant][outer][inner][direction-group][4 face nodes]
    if (in.ic) load4(A.fx + (o * A.fx_o + in.kc * A.fx_k + in.jc * A.fx_j + dg * 4), in.vx);
    else in.vx[0] = in.vx[1] = in.vx[2] = in.vx[3] = A.inc[o][0];
    if (in.jc) load4(A.fy + (o * A.fy_o + in.kc * A.fy_k + in.ic * A.fy_j + dg * 4), in.vy);
    else in.vy[0] = in.vy[1] = in.vy[2] = in.vy[3] = A.inc[o][1];
    if (in.kc) load4(A.fz + (o * A.fz_o + in.jc * A.fz_k + in.ic * A.fz_j + dg * 4), in.vz);
    else in.vz[0] = in.vz[1] = in.vz[2] = in.vz[3] = A.inc[o][2];
}

template <typename Real, int Form, bool kStorePsi, bool kAdjoint>
__global__ __launch_bounds__(256) void sweep_plane_ge(PlaneArgs<Real> A)
{
    // block = (direction, group, cell) lanes, grid = (cell tiles, octant); each
    // block visits A.cpt tiles of blockDim.z cells, the inputs of the next
    // tile being loaded before the current one is solved.
    __shared__ Real red[2][256 * 9];      // [lane][node], padded: conflict-free
    __shared__ Real gred[256 * 2];
    const int d = threadIdx.x, g = threadIdx.y;
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int o = blockIdx.y;                         // octant slot (block-uniform)
    const int mask = kAdjoint ? (o ^ 7) : o;
    const uint32_t dg = d + A.Do * g;
    const Real *dp = A.dir + (o * A.Do + d) * kDirStride;
    const Real w = dp[kDirW];
    const Real kap[3] = {dp[kDirK], dp[kDirK + 1], dp[kDirK + 2]};
    const int tile0 = blockIdx.x * A.cpt;
    const int nc = blockDim.z;

    CellIn<Real> nxt;
    gather_cell(A, tile0 * nc + (int)threadIdx.z, o, mask, g, dg, nxt);
    for (int t = 0; t < (int)A.cpt; ++t) {
        const CellIn<Real> cur = nxt;
        if (t + 1 < (int)A.cpt)
            gather_cell(A, (tile0 + t + 1) * nc + (int)threadIdx.z, o, mask, g, dg, nxt);
        Real psi[8];
        Real gs = 0, gq = 0;
        if (cur.ok) {
            cell_solve<Real, Form>(dp, kap, cur.st, cur.sc, cur.vx, cur.vy, cur.vz, psi);
            // outflow faces into the fronts (same slots, consumed next step)
            store4(A.fx + (o * A.fx_o + cur.kc * A.fx_k + cur.jc * A.fx_j + dg * 4), psi[1], psi[3],
                   psi[5], psi[7]);
            store4(A.fy + (o * A.fy_o + cur.kc * A.fy_k + cur.ic * A.fy_j + dg * 4), psi[2], psi[3],
                   psi[6], psi[7]);
            store4(A.fz + (o * A.fz_o + cur.jc * A.fz_k + cur.ic * A.fz_j + dg * 4), psi[4], psi[5],
                   psi[6], psi[7]);
            const uint32_t slot = (o * A.Do + d) * A.G + g;
            if (kStorePsi || (kAdjoint && A.grad_oct)) {
                Real *pp = A.psi + ((size_t)slot * A.ncell + cur.c) * 8;
                if (kStorePsi) {
                    Real ph[8];
#pragma unroll
                    for (int n = 0; n < 8; ++n) ph[n] = psi[n];
                    reflect8(ph, mask);
                    store4(pp, ph[0], ph[1], ph[2], ph[3]);
                    store4(pp + 4, ph[4], ph[5], ph[6], ph[7]);
                } else {
                    // contraction with the stored forward flux of the same
                    // direction: mu^T M psi, M = V M3 (invariant under reflection)
                    Real pf[8], m[8];
                    load4(pp, pf);
                    load4(pp + 4, pf + 4);
                    reflect8(pf, mask);
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
        } else {
#pragma unroll
            for (int n = 0; n < 8; ++n) psi[n] = 0;
        }
        // deterministic per-octant reduction over the directions of the segment
        Real *rb = red[t & 1];
#pragma unroll
        for (int n = 0; n < 8; ++n) rb[tid * 9 + n] = w * psi[n];
        if (kAdjoint) {
            gred[tid * 2 + 0] = gs;
            gred[tid * 2 + 1] = gq;
        }
        __syncthreads();
        if (cur.ok) {
            const int base = tid - d;
            const uint32_t out = ((o * A.G + g) * A.ncell + cur.c) * 8;
            for (int n = d; n < 8; n += (int)A.Do) {
                Real s = 0;
                for (int e = 0; e < (int)A.Do; ++e) s += rb[(base + e) * 9 + n];
                A.phi_oct[out + (n ^ mask)] = s;
            }
            if (kAdjoint && A.grad_oct) {
                for (int k2 = d; k2 < 2; k2 += (int)A.Do) {
                    Real s = 0;
                    for (int e = 0; e < (int)A.Do; ++e) s += gred[(base + e) * 2 + k2];
                    A.grad_oct[((o * A.G + g) * A.ncell + cur.c) * 2 + k2] = s;
                }
            }
        }
        // red alternates between two buffers; gred is single: fence its reuse
        if (kAdjoint) __syncthreads();
    }
}

// Tile sweep.  Each lane owns one (octant, B x B x B tile of cells,
// direction, group) and solves the tile's cells in upwind lexicographic order,
// carrying the faces between its own cells in registers: only the faces on the
// tile boundary go through the fronts in HBM (24/B face values per solve
// instead of 24).  Tiles with I + J + K = s are independent; one launch per
// tile hyperplane s.  B = 1 is the plain cell hyperplane sweep.
template <typename Real, int Form, int B, bool kStorePsi, bool kAdjoint>
__global__ __launch_bounds__(256) void sweep_tile_ge(PlaneArgs<Real> A)
{
    __shared__ Real red[2][256 * 9];      // [lane][node], padded: conflict-free
    __shared__ Real gred[256 * 2];
    const int d = threadIdx.x, g = threadIdx.y;
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int ti = blockIdx.x * blockDim.z + threadIdx.z;
    const int o = blockIdx.y;                         // octant slot (block-uniform)
    const int mask = kAdjoint ? (o ^ 7) : o;
    const bool tvalid = ti < (int)A.ncp;
    const uint32_t dg = d + A.Do * g;
    const Real *dp = A.dir + (o * A.Do + d) * kDirStride;
    const Real w = dp[kDirW];
    const Real kap[3] = {dp[kDirK], dp[kDirK + 1], dp[kDirK + 2]};
    uint32_t I0 = 0, J0 = 0, K0 = 0;
    if (tvalid) {
        const uint32_t pt = A.cells[ti];
        I0 = (pt & 1023u) * B;
        J0 = ((pt >> 10) & 1023u) * B;
        K0 = (pt >> 20) * B;
    }
    const uint32_t slot = (o * A.Do + d) * A.G + g;
    Real xf[4], yf[B][4], zf[B][B][4];
#pragma unroll
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
                if (ok) {
                    const uint32_t i = (mask & 1) ? A.nx - 1 - ic : ic;
                    const uint32_t j = (mask & 2) ? A.ny - 1 - jc : jc;
                    const uint32_t k = (mask & 4) ? A.nz - 1 - kc : kc;
                    c = i + A.nx * (j + A.ny * k);
                    const uint32_t gc = g * A.ncell + c;
                    const Real st = A.sigma_t[gc];
                    Real sc[8];
                    const Real *sp = A.src + gc * 8;
                    load4(sp, sc);
                    load4(sp + 4, sc + 4);
                    reflect8(sc, mask);
                    Real *fxp = A.fx + (o * A.fx_o + kc * A.fx_k + jc * A.fx_j + dg * 4);
                    Real *fyp = A.fy + (o * A.fy_o + kc * A.fy_k + ic * A.fy_j + dg * 4);
                    Real *fzp = A.fz + (o * A.fz_o + jc * A.fz_k + ic * A.fz_j + dg * 4);
                    Real vx[4], vy[4], vz[4];
                    if (il > 0) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) vx[e] = xf[e];
                    } else if (ic) {
                        load4(fxp, vx);
                    } else {
                        vx[0] = vx[1] = vx[2] = vx[3] = A.inc[o][0];
                    }
                    if (jl > 0) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) vy[e] = yf[il][e];
                    } else if (jc) {
                        load4(fyp, vy);
                    } else {
                        vy[0] = vy[1] = vy[2] = vy[3] = A.inc[o][1];
                    }
                    if (kl > 0) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) vz[e] = zf[jl][il][e];
                    } else if (kc) {
                        load4(fzp, vz);
                    } else {
                        vz[0] = vz[1] = vz[2] = vz[3] = A.inc[o][2];
                    }
                    cell_solve<Real, Form>(dp, kap, st, sc, vx, vy, vz, psi);
                    xf[0] = psi[1]; xf[1] = psi[3]; xf[2] = psi[5]; xf[3] = psi[7];
                    yf[il][0] = psi[2]; yf[il][1] = psi[3]; yf[il][2] = psi[6]; yf[il][3] = psi[7];
                    zf[jl][il][0] = psi[4]; zf[jl][il][1] = psi[5];
                    zf[jl][il][2] = psi[6]; zf[jl][il][3] = psi[7];
                    // tile-boundary outflow into the fronts (consumed by the
                    // next tile hyperplane; same slot as the inflow read)
                    if (il == B - 1 && ic + 1 < A.nx) store4(fxp, psi[1], psi[3], psi[5], psi[7]);
                    if (jl == B - 1 && jc + 1 < A.ny) store4(fyp, psi[2], psi[3], psi[6], psi[7]);
                    if (kl == B - 1 && kc + 1 < A.nz) store4(fzp, psi[4], psi[5], psi[6], psi[7]);
                    if (kStorePsi || (kAdjoint && A.grad_oct)) {
                        Real *pp = A.psi + ((size_t)slot * A.ncell + c) * 8;
                        if (kStorePsi) {
                            Real ph[8];
#pragma unroll
                            for (int n = 0; n < 8; ++n) ph[n] = psi[n];
                            reflect8(ph, mask);
                            store4(pp, ph[0], ph[1], ph[2], ph[3]);
                            store4(pp + 4, ph[4], ph[5], ph[6], ph[7]);
                        } else {
                            // mu^T M psi with the stored forward flux, M = V M3
                            Real pf[8], m[8];
                            load4(pp, pf);
                            load4(pp + 4, pf + 4);
                            reflect8(pf, mask);
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
                } else {
#pragma unroll
                    for (int n = 0; n < 8; ++n) psi[n] = 0;
                }
                // deterministic per-octant reduction over the directions
                Real *rb = red[cidx & 1];
#pragma unroll
                for (int n = 0; n < 8; ++n) rb[tid * 9 + n] = w * psi[n];
                if (kAdjoint) {
                    gred[tid * 2 + 0] = gs;
                    gred[tid * 2 + 1] = gq;
                }
                __syncthreads();
                if (ok) {
                    const int base = tid - d;
                    const uint32_t out = ((o * A.G + g) * A.ncell + c) * 8;
                    for (int n = d; n < 8; n += (int)A.Do) {
                        Real s = 0;
                        for (int e = 0; e < (int)A.Do; ++e) s += rb[(base + e) * 9 + n];
                        A.phi_oct[out + (n ^ mask)] = s;
                    }
                    if (kAdjoint && A.grad_oct) {
                        for (int k2 = d; k2 < 2; k2 += (int)A.Do) {
                            Real s = 0;
                            for (int e = 0; e < (int)A.Do; ++e) s += gred[(base + e) * 2 + k2];
                            A.grad_oct[((o * A.G + g) * A.ncell + c) * 2 + k2] = s;
                        }
                    }
                }
                if (kAdjoint) __syncthreads();
            }
}

// phi = sum_o phi_oct[o]; optionally the FP64 SI residual partials and the
// next source S = qn + qc + sigma_s/(4 pi) phi.
template <typename Real>
__global__ __launch_bounds__(256) void reduce_octants(ReduceArgs<Real> R)
{
    __shared__ double sh[3][256];
    double dmax = 0.0, fmax = 0.0, esum = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < R.nv; e += stride) {
        Real nw[8];
#pragma unroll
        for (int n = 0; n < 8; ++n) nw[n] = 0;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const Real *p = R.phi_oct + ((long long)o * R.nv + e) * 8;
#pragma unroll
            for (int n = 0; n < 8; ++n) nw[n] += p[n];
        }
        Real *ph = R.phi + e * 8;
        if (R.resid) {
            double an = 0.0, ao = 0.0;
#pragma unroll
            for (int n = 0; n < 8; ++n) {
                const double vn = (double)nw[n], vo = (double)ph[n];
                dmax = fmax_d(dmax, fabs(vn - vo));
                fmax = fmax_d(fmax, fabs(vn));
                an += vn;
                ao += vo;
            }
            an *= 0.125;
            ao *= 0.125;
            esum += (an != 0.0) ? fabs(an - ao) / fabs(an) : (ao != 0.0 ? 1.0 : 0.0);
        }
#pragma unroll
        for (int n = 0; n < 8; ++n) ph[n] = nw[n];
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
    if (!R.resid) return;
    const int tid = threadIdx.x;
    sh[0][tid] = dmax;
    sh[1][tid] = fmax;
    sh[2][tid] = esum;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
            sh[0][tid] = fmax_d(sh[0][tid], sh[0][tid + s]);
            sh[1][tid] = fmax_d(sh[1][tid], sh[1][tid + s]);
            sh[2][tid] += sh[2][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        R.partials[blockIdx.x * 3 + 0] = sh[0][0];
        R.partials[blockIdx.x * 3 + 1] = sh[1][0];
        R.partials[blockIdx.x * 3 + 2] = sh[2][0];
    }
}

__global__ __launch_bounds__(256) void finalize_partials(const double *partials, int nblocks,
                                                         double *result)
{
    __shared__ double sh[3][256];
    const int tid = threadIdx.x;
    double a = 0.0, b = 0.0, s = 0.0;
    for (int i = tid; i < nblocks; i += blockDim.x) {
        a = fmax_d(a, partials[i * 3 + 0]);
        b = fmax_d(b, partials[i * 3 + 1]);
        s += partials[i * 3 + 2];
    }
    sh[0][tid] = a;
    sh[1][tid] = b;
    sh[2][tid] = s;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (tid < st) {
            sh[0][tid] = fmax_d(sh[0][tid], sh[0][tid + st]);
            sh[1][tid] = fmax_d(sh[1][tid], sh[1][tid + st]);
            sh[2][tid] += sh[2][tid + st];
        }
        __syncthreads();
    }
    if (tid == 0) {
        result[0] = sh[0][0];
        result[1] = sh[1][0];
        result[2] = sh[2][0];
    }
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

int cells_per_block(int Do, int G) { return 256 / (Do * G); }

// Tiles visited by one block: enough blocks to keep every CU busy (about
// 8 per CU over the 8 octants), the rest of the work is looped over so that
// each lane overlaps the loads of its next cell with the current solve.
int tiles_per_block(int tiles)
{
    const int target = 256;   // blocks per octant
    int cpt = tiles / target;
    if (cpt < 1) cpt = 1;
    if (cpt > 8) cpt = 8;
    return cpt;
}

template <typename Real, int Form>
void launch_plane_form(const PlaneArgs<Real> &A, bool store_psi, bool adjoint, dim3 grid,
                       dim3 block, hipStream_t s)
{
    if (adjoint)
        hipLaunchKernelGGL((sweep_plane_ge<Real, Form, false, true>), grid, block, 0, s, A);
    else if (store_psi)
        hipLaunchKernelGGL((sweep_plane_ge<Real, Form, true, false>), grid, block, 0, s, A);
    else
        hipLaunchKernelGGL((sweep_plane_ge<Real, Form, false, false>), grid, block, 0, s, A);
}

template <typename Real>
int launch_plane(const PlaneArgs<Real> &A, int form, bool store_psi, bool adjoint, hipStream_t s)
{
    const dim3 block(A.Do, A.G, cells_per_block(A.Do, A.G));
    const int tiles = (int)((A.ncp + block.z - 1) / block.z);
    PlaneArgs<Real> B = A;
    B.cpt = tiles_per_block(tiles);
    const dim3 grid((tiles + B.cpt - 1) / B.cpt, 8);
    if (form == kFormDense)
        launch_plane_form<Real, kFormDense>(B, store_psi, adjoint, grid, block, s);
    else
        launch_plane_form<Real, kFormMassInv>(B, store_psi, adjoint, grid, block, s);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real, int Form, int B>
void launch_tile_form(const PlaneArgs<Real> &A, bool store_psi, bool adjoint, dim3 grid,
                      dim3 block, hipStream_t s)
{
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
    if (b == 2) launch_tile_form<Real, Form, 2>(A, store_psi, adjoint, grid, block, s);
    else launch_tile_form<Real, Form, 1>(A, store_psi, adjoint, grid, block, s);
}

template <typename Real>
int launch_tile(const PlaneArgs<Real> &A, int form, int b, bool store_psi, bool adjoint,
                hipStream_t s)
{
    const dim3 block(A.Do, A.G, cells_per_block(A.Do, A.G));
    const dim3 grid((A.ncp + block.z - 1) / block.z, 8);
    if (form == kFormDense)
        launch_tile_b<Real, kFormDense>(A, b, store_psi, adjoint, grid, block, s);
    else
        launch_tile_b<Real, kFormMassInv>(A, b, store_psi, adjoint, grid, block, s);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template <typename Real>
int launch_reduce(const ReduceArgs<Real> &R, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_octants<Real>, dim3(blocks), dim3(256), 0, s, R);
    DGSN_HIP(hipGetLastError());
    if (R.resid) {
        hipLaunchKernelGGL(finalize_partials, dim3(1), dim3(256), 0, s, R.partials, blocks,
                           R.result);
        DGSN_HIP(hipGetLastError());
    }
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

int reduce_blocks_for(long long nv) { return grid_for(nv, 2048); }

#define DGSN_INST(Real)                                                                        \
    template int launch_plane<Real>(const PlaneArgs<Real> &, int, bool, bool, hipStream_t);      \
    template int launch_tile<Real>(const PlaneArgs<Real> &, int, int, bool, bool, hipStream_t);         \
    template int launch_reduce<Real>(const ReduceArgs<Real> &, int, hipStream_t);              \
    template int launch_build_source<Real>(long long, const Real *, const Real *, const Real *, \
                                           Real *, hipStream_t);                               \
    template int launch_adjoint_load<Real>(long long, const Real *, double, Real *,            \
                                           hipStream_t);                                       \
    template int launch_reduce_grad<Real>(long long, const Real *, Real *, Real *, hipStream_t);
DGSN_INST(float)
DGSN_INST(double)

}  // namespace dgsn
