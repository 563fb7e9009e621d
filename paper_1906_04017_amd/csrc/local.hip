// Batched one-cell solves of the canonical cell system (Sec. 3: the one-cell
// problem is fixed by the streaming weights, the optical size, the three
// inflow faces and the eight source nodes).  Each lane assembles
//   h A' = sum_a (kappa_a h) T_a + (sigma_t h) M3,
//   h b' = sum_a (kappa_a h) (M1 (x) M1) psi_in,a + M3 (h S)
// from its 24 inputs and solves it by Gaussian elimination.
#include "cell.hpp"
#include "common.hpp"

namespace dgsn {
namespace {

__host__ __device__ constexpr double t1c(int k, int j) { return (k == 1 && j == 0) ? -0.5 : 0.5; }
__host__ __device__ constexpr double m1c(int k, int j) { return k == j ? 1.0 / 3.0 : 1.0 / 6.0; }

// entry (k, j) of T_a (T on axis a, M1 on the other two)
__host__ __device__ constexpr double ta_entry(int a, int k, int j)
{
    double v = 1.0;
    for (int b = 0; b < 3; ++b) {
        const int kb = (k >> b) & 1, jb = (j >> b) & 1;
        v *= (b == a) ? t1c(kb, jb) : m1c(kb, jb);
    }
    return v;
}

template <typename Real>
__global__ __launch_bounds__(256) void local_solve_kernel(const Real *__restrict__ x,
                                                          Real *__restrict__ psi, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride) {
        const Real *xi = x + s * 24;
        const Real kx = xi[0], ky = xi[1], kz = xi[2], tau = xi[3];
        Real a[8][8], b[8];
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                Real v = tau * Real(m3_entry(r, c));
                v = fma(kx, Real(ta_entry(0, r, c)), v);
                v = fma(ky, Real(ta_entry(1, r, c)), v);
                v = fma(kz, Real(ta_entry(2, r, c)), v);
                a[r][c] = v;
            }
        Real sc[8], m[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) sc[k] = xi[16 + k];
        mass3_216(sc, m);
#pragma unroll
        for (int k = 0; k < 8; ++k) b[k] = m[k] * Real(1.0 / 216.0);
        Real v[4], f[4];
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) v[fn] = xi[4 + fn];
        face_mass(v, kx * Real(1.0 / 36.0), f);
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) b[2 * fn] += f[fn];
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) v[fn] = xi[8 + fn];
        face_mass(v, ky * Real(1.0 / 36.0), f);
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) b[(fn & 1) + 4 * (fn >> 1)] += f[fn];
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) v[fn] = xi[12 + fn];
        face_mass(v, kz * Real(1.0 / 36.0), f);
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) b[fn] += f[fn];
        ge_solve8(a, b);
#pragma unroll
        for (int k = 0; k < 8; ++k) psi[s * 8 + k] = b[k];
    }
}

}  // namespace
}  // namespace dgsn

using namespace dgsn;

extern "C" int dgsn_local_solve(dgsn_ctx *ctx, const void *x, void *psi, long long n, int precision,
                                void *stream)
{
    clear_error();
    if (!ctx) return set_error(DGSN_EINVAL, "ctx is NULL");
    if (n < 0) return set_error(DGSN_EINVAL, "n must be >= 0");
    if (n == 0) return DGSN_OK;
    if (!x || !psi) return set_error(DGSN_EINVAL, "x and psi must be set");
    if (precision != DGSN_FP32 && precision != DGSN_FP64)
        return set_error(DGSN_EINVAL, "precision must be DGSN_FP32 or DGSN_FP64");
    DGSN_HIP(hipSetDevice(ctx->device));
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (precision == DGSN_FP64)
        hipLaunchKernelGGL(local_solve_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<const double *>(x), static_cast<double *>(psi), n);
    else
        hipLaunchKernelGGL(local_solve_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<const float *>(x), static_cast<float *>(psi), n);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}
