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

template <typename Real>
__device__ __forceinline__ void load_dir(const Real *__restrict__ dp, Real sd[64], Real k36[3],
                                         Real &w)
{
#pragma unroll
    for (int e = 0; e < 64; ++e) sd[e] = dp[e];
    k36[0] = dp[64];
    k36[1] = dp[65];
    k36[2] = dp[66];
    w = dp[67];
}

template <typename Real, bool kStorePsi, bool kAdjoint>
__global__ __launch_bounds__(256) void sweep_plane_ge(PlaneArgs<Real> A)
{
    __shared__ Real red[8][256];
    __shared__ Real gred[2][256];
    const int tid = threadIdx.x;
    const long long lin = (long long)blockIdx.x * blockDim.x + tid;
    const long long seg = lin / A.Do;
    const int d = (int)(lin - seg * A.Do);
    const int g = (int)(seg % A.G);
    const long long t = seg / A.G;
    const int o = (int)(t / A.ncp);
    const int ci = (int)(t - (long long)o * A.ncp);
    const bool valid = o < 8;

    Real psi[8];
    Real w = 0;
    int mask = 0;
    long long c = 0;
    Real gs = 0, gq = 0;
    if (valid) {
        const uint32_t pc = A.cells[ci];
        const int ic = pc & 1023, jc = (pc >> 10) & 1023, kc = pc >> 20;
        mask = kAdjoint ? (o ^ 7) : o;
        const int i = (mask & 1) ? A.nx - 1 - ic : ic;
        const int j = (mask & 2) ? A.ny - 1 - jc : jc;
        const int k = (mask & 4) ? A.nz - 1 - kc : kc;
        c = (long long)i + (long long)A.nx * ((long long)j + (long long)A.ny * k);
        const int dg = d + A.Do * g;
        const long long gc = (long long)g * A.ncell + c;

        Real a[8][8], k36[3];
        {
            Real sd[64];
            load_dir(A.dir + (long long)(o * A.Do + d) * kDirStride, sd, k36, w);
            const Real st = A.sigma_t[gc];
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int s = 0; s < 8; ++s) a[r][s] = fma(st, Real(m3_entry(r, s)), sd[r * 8 + s]);
        }
        // right-hand side: M3 S (source reflected into canonical order)
        Real b[8];
        {
            Real sc[8], m[8];
            const Real *sp = A.src + gc * 8;
#pragma unroll
            for (int n = 0; n < 8; ++n) sc[n] = sp[n ^ mask];
            mass3_216(sc, m);
#pragma unroll
            for (int n = 0; n < 8; ++n) b[n] = m[n] * Real(1.0 / 216.0);
        }
        // inflow faces: boundary value or the upwind neighbour's outflow
        const long long DG = A.DG;
        const long long ix_x = (((long long)o * A.nz + kc) * A.ny + jc) * 4 * DG + dg;
        const long long ix_y = (((long long)o * A.nz + kc) * A.nx + ic) * 4 * DG + dg;
        const long long ix_z = (((long long)o * A.ny + jc) * A.nx + ic) * 4 * DG + dg;
        {
            Real v[4], f[4];
#pragma unroll
            for (int fn = 0; fn < 4; ++fn) v[fn] = ic ? A.fx[ix_x + fn * DG] : A.inc[o][0];
            face_mass(v, k36[0], f);
#pragma unroll
            for (int fn = 0; fn < 4; ++fn) b[2 * fn] += f[fn];
#pragma unroll
            for (int fn = 0; fn < 4; ++fn) v[fn] = jc ? A.fy[ix_y + fn * DG] : A.inc[o][1];
            face_mass(v, k36[1], f);
#pragma unroll
            for (int fn = 0; fn < 4; ++fn) b[(fn & 1) + 4 * (fn >> 1)] += f[fn];
#pragma unroll
            for (int fn = 0; fn < 4; ++fn) v[fn] = kc ? A.fz[ix_z + fn * DG] : A.inc[o][2];
            face_mass(v, k36[2], f);
#pragma unroll
            for (int fn = 0; fn < 4; ++fn) b[fn] += f[fn];
        }
        ge_solve8(a, b);
#pragma unroll
        for (int n = 0; n < 8; ++n) psi[n] = b[n];
        // outflow faces into the fronts (same slots, consumed next step)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) {
            A.fx[ix_x + fn * DG] = psi[1 + 2 * fn];
            A.fy[ix_y + fn * DG] = psi[(fn & 1) + 2 + 4 * (fn >> 1)];
            A.fz[ix_z + fn * DG] = psi[4 + fn];
        }
        const long long slot = (long long)(o * A.Do + d) * A.G + g;
        if (kStorePsi) {
            Real *pp = A.psi + (slot * A.ncell + c) * 8;
#pragma unroll
            for (int n = 0; n < 8; ++n) pp[n ^ mask] = psi[n];
        }
        if (kAdjoint && A.grad_oct) {
            // contraction with the stored forward flux of the same direction:
            // mu^T M psi with M = V M3 (M3 is invariant under the reflection)
            const Real *pp = A.psi + (slot * A.ncell + c) * 8;
            Real pf[8], m[8];
#pragma unroll
            for (int n = 0; n < 8; ++n) pf[n] = pp[n ^ mask];
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
    } else {
#pragma unroll
        for (int n = 0; n < 8; ++n) psi[n] = 0;
    }
    // deterministic per-octant reduction over the directions of the segment
#pragma unroll
    for (int n = 0; n < 8; ++n) red[n][tid] = w * psi[n];
    if (kAdjoint) {
        gred[0][tid] = gs;
        gred[1][tid] = gq;
    }
    __syncthreads();
    if (valid) {
        const int base = tid - d;
        for (int n = d; n < 8; n += A.Do) {
            Real s = 0;
            for (int e = 0; e < A.Do; ++e) s += red[n][base + e];
            A.phi_oct[(((long long)o * A.G + g) * A.ncell + c) * 8 + (n ^ mask)] = s;
        }
        if (kAdjoint && A.grad_oct) {
            for (int k2 = d; k2 < 2; k2 += A.Do) {
                Real s = 0;
                for (int e = 0; e < A.Do; ++e) s += gred[k2][base + e];
                A.grad_oct[(((long long)o * A.G + g) * A.ncell + c) * 2 + k2] = s;
            }
        }
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

template <typename Real>
int launch_plane(const PlaneArgs<Real> &A, bool store_psi, bool adjoint, hipStream_t s)
{
    const long long total = 8LL * A.ncp * A.G * A.Do;
    const int bs = block_size_for(A.Do);
    const long long grid = (total + bs - 1) / bs;
    if (grid > 0x7fffffffLL) return set_error(DGSN_EUNSUPPORTED, "hyperplane too large");
    if (adjoint)
        hipLaunchKernelGGL((sweep_plane_ge<Real, false, true>), dim3((unsigned)grid), dim3(bs), 0,
                           s, A);
    else if (store_psi)
        hipLaunchKernelGGL((sweep_plane_ge<Real, true, false>), dim3((unsigned)grid), dim3(bs), 0,
                           s, A);
    else
        hipLaunchKernelGGL((sweep_plane_ge<Real, false, false>), dim3((unsigned)grid), dim3(bs),
                           0, s, A);
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
    template int launch_plane<Real>(const PlaneArgs<Real> &, bool, bool, hipStream_t);         \
    template int launch_reduce<Real>(const ReduceArgs<Real> &, int, hipStream_t);              \
    template int launch_build_source<Real>(long long, const Real *, const Real *, const Real *, \
                                           Real *, hipStream_t);                               \
    template int launch_adjoint_load<Real>(long long, const Real *, double, Real *,            \
                                           hipStream_t);                                       \
    template int launch_reduce_grad<Real>(long long, const Real *, Real *, Real *, hipStream_t);
DGSN_INST(float)
DGSN_INST(double)

}  // namespace dgsn
