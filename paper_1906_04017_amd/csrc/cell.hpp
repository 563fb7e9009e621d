// Device-side cell algebra of the trilinear DGFEM cell system (Sec. 2,
// Eq. (T10)-(T12)), in the canonical orientation where every direction
// component is non-negative.
//
// Reflecting the cell so that Omega points into the positive octant maps local
// node n to n ^ mask (mask bit a set when Omega_a < 0); the cell system is
// invariant under this relabelling.  Divided by the cell volume V, the
// canonical system is
//   A' = sum_a kappa_a T_a + sigma_t M3,   kappa_a = |Omega_a| / dx_a,
//   b' = sum_a kappa_a (M1 (x) M1) psi_in,a (rows of the inflow face a) + M3 S,
// with the 1D factors M1 = [[1/3, 1/6], [1/6, 1/3]] (mass) and
// T = [[1/2, 1/2], [-1/2, 1/2]] (streaming plus outflow trace, upwind
// direction), T_x = M1 (x) M1 (x) T etc. (x fastest), M3 = M1 (x) M1 (x) M1.
// The per-direction streaming part S_d = sum_a kappa_a T_a is built once per
// direction on the host (the paper's observation that a direction only
// re-weights L and L-, Sec. 2).
//
// Mass-inverse form.  M3 is known in closed form and M1^{-1} = [[4,-2],[-2,4]],
// so the same cell system premultiplied by M3^{-1} reads
//   (P_d + sigma_t I) psi = S + sum_a kappa_a c_a,
//   P_d = sum_a kappa_a (I (x) .. Q .. (x) I),  Q = M1^{-1} T = [[3, 1], [-3, 1]],
//   c_a = 4 psi_in,a on the inflow-face rows of axis a, -2 psi_in,a on the
//         opposite rows (M1^{-1} e_0 = [4, -2]).
// P_d couples a node only with itself and its three edge neighbours, so 32
// of the 64 entries are structurally zero; Gaussian elimination then touches
// only the entries that become non-zero (the fill), about half the work of
// the dense elimination, with the same solution.
#pragma once

#include <hip/hip_runtime.h>

namespace dgsn {

template <typename Real>
__device__ __forceinline__ Real recip(Real x);

template <>
__device__ __forceinline__ float recip<float>(float x)
{
    return __builtin_amdgcn_rcpf(x);   // v_rcp_f32, 1 ulp
}

template <>
__device__ __forceinline__ double recip<double>(double x)
{
    return 1.0 / x;                    // correctly rounded division
}

// (M1 (x) M1) v for a 4-vector on a face (two tangential bits, first fastest),
// times s/36 folded in: out = s * (M1 (x) M1) v with s = kappa already / 36.
template <typename Real>
__device__ __forceinline__ void face_mass(const Real v[4], Real s36, Real out[4])
{
    Real u[4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) u[a + 2 * b] = fma(Real(2), v[a + 2 * b], v[(a ^ 1) + 2 * b]);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a)
            out[a + 2 * b] = s36 * fma(Real(2), u[a + 2 * b], u[a + 2 * (b ^ 1)]);
}

// 216 * M3 v (three stages of [[2,1],[1,2]]).
template <typename Real>
__device__ __forceinline__ void mass3_216(const Real v[8], Real out[8])
{
    Real t[8], u[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) t[n] = fma(Real(2), v[n], v[n ^ 1]);
#pragma unroll
    for (int n = 0; n < 8; ++n) u[n] = fma(Real(2), t[n], t[n ^ 2]);
#pragma unroll
    for (int n = 0; n < 8; ++n) out[n] = fma(Real(2), u[n], u[n ^ 4]);
}

// 1/216 * M3^{-1} ... inverse of M1 is [[4,-2],[-2,4]]: (216 M3)^{-1} v = (1/216) * ...
// M3^{-1} v = kron of M1^{-1}: three stages of (4 v_same - 2 v_other).
template <typename Real>
__device__ __forceinline__ void mass3_inv(const Real v[8], Real out[8])
{
    Real t[8], u[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) t[n] = fma(Real(4), v[n], Real(-2) * v[n ^ 1]);
#pragma unroll
    for (int n = 0; n < 8; ++n) u[n] = fma(Real(4), t[n], Real(-2) * t[n ^ 2]);
#pragma unroll
    for (int n = 0; n < 8; ++n) out[n] = fma(Real(4), u[n], Real(-2) * u[n ^ 4]);
}

// Entries of M3 = prod_a (1/3 if same 1D node else 1/6).
__host__ __device__ constexpr double m3_entry(int k, int j)
{
    return (((k ^ j) & 1) ? 1.0 / 6.0 : 1.0 / 3.0) * (((k ^ j) & 2) ? 1.0 / 6.0 : 1.0 / 3.0) *
           (((k ^ j) & 4) ? 1.0 / 6.0 : 1.0 / 3.0);
}

// Gaussian elimination of the 8x8 system held in registers, solution
// returned in b.  Partial pivoting (largest |a_ik|, lowest row on ties) is
// decided per lane but tested for the whole wavefront first: the row
// exchange code runs only if some lane of the wave needs an exchange in this
// column.  For the canonical cell matrices the diagonal is the column maximum,
// so the exchange branch is normally skipped by every wave.
template <typename Real>
__device__ __forceinline__ void ge_solve8(Real a[8][8], Real b[8])
{
    Real rinv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k < 7) {
            Real cm = fabs(a[k + 1][k]);
#pragma unroll
            for (int i = k + 2; i < 8; ++i) cm = fmax(cm, fabs(a[i][k]));
            const bool need = cm > fabs(a[k][k]);
            if (__any(need)) {
                int p = k;
                Real best = fabs(a[k][k]);
#pragma unroll
                for (int i = k + 1; i < 8; ++i) {
                    const bool gt = fabs(a[i][k]) > best;
                    best = gt ? fabs(a[i][k]) : best;
                    p = gt ? i : p;
                }
#pragma unroll
                for (int i = k + 1; i < 8; ++i) {
                    const bool sw = (p == i);
#pragma unroll
                    for (int j = k; j < 8; ++j) {
                        const Real t = a[k][j];
                        a[k][j] = sw ? a[i][j] : t;
                        a[i][j] = sw ? t : a[i][j];
                    }
                    const Real t = b[k];
                    b[k] = sw ? b[i] : t;
                    b[i] = sw ? t : b[i];
                }
            }
        }
        rinv[k] = recip(a[k][k]);
#pragma unroll
        for (int i = k + 1; i < 8; ++i) {
            const Real l = a[i][k] * rinv[k];
#pragma unroll
            for (int j = k + 1; j < 8; ++j) a[i][j] = fma(-l, a[k][j], a[i][j]);
            b[i] = fma(-l, b[k], b[i]);
        }
    }
#pragma unroll
    for (int i = 7; i >= 0; --i) {
        Real s = b[i];
#pragma unroll
        for (int j = i + 1; j < 8; ++j) s = fma(-a[i][j], b[j], s);
        b[i] = s * rinv[i];
    }
}

// Structural pattern of Gaussian elimination (natural order) on a matrix
// whose initial non-zeros are the diagonal and the single-bit neighbours:
// pattern(k, i, j) is true when entry (i, j) may be non-zero before column k
// is eliminated (k = 8: the final upper-triangular factor).
struct CubeFill {
    unsigned char row[9][8];   // bit j of row[k][i]
    constexpr CubeFill() : row()
    {
        unsigned char cur[8] = {};
        for (int i = 0; i < 8; ++i) cur[i] = (unsigned char)((1u << i) | (1u << (i ^ 1)) |
                                                             (1u << (i ^ 2)) | (1u << (i ^ 4)));
        for (int k = 0; k <= 8; ++k) {
            for (int i = 0; i < 8; ++i) row[k][i] = cur[i];
            if (k == 8) break;
            for (int i = k + 1; i < 8; ++i)
                if (cur[i] & (1u << k))
                    for (int j = k + 1; j < 8; ++j)
                        if (cur[k] & (1u << j)) cur[i] |= (unsigned char)(1u << j);
        }
    }
};
constexpr CubeFill kCubeFill{};

__host__ __device__ constexpr bool cube_nz(int k, int i, int j)
{
    return (kCubeFill.row[k][i] >> j) & 1;
}

// Elimination restricted to the structurally non-zero entries of the
// mass-inverse cell matrix, without row exchanges, split into the
// factorisation of the matrix and the solve of one right-hand side.  The
// factorisation leaves the multipliers l_ik below the diagonal of a, the
// eliminated upper triangle above it and the reciprocal pivots in rinv; it
// returns, per lane, whether partial pivoting would have exchanged rows in
// some column (a structurally possible sub-diagonal entry larger than the
// pivot), in which case the caller uses the dense, pivoted ge_solve8 instead,
// so the result is always that of partial pivoting.  For these matrices the
// diagonal dominates its column and that never happens.  The solve applies
// the multipliers to b in the order in which the elimination meets them, so
// factor + solve performs exactly the operations of the interleaved
// elimination: one factorisation serves every cell with the same matrix
// (same direction and sigma_t) with bitwise the same result.
template <typename Real>
__device__ __forceinline__ bool cube_factor(Real a[8][8], Real rinv[8])
{
    bool exchange = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        Real cm = Real(0);
#pragma unroll
        for (int i = k + 1; i < 8; ++i)
            if (cube_nz(k, i, k)) cm = fmax(cm, fabs(a[i][k]));
        exchange = exchange || (cm > fabs(a[k][k]));
        rinv[k] = recip(a[k][k]);
#pragma unroll
        for (int i = k + 1; i < 8; ++i) {
            if (!cube_nz(k, i, k)) continue;
            const Real l = a[i][k] * rinv[k];
#pragma unroll
            for (int j = k + 1; j < 8; ++j)
                if (cube_nz(k, k, j)) a[i][j] = fma(-l, a[k][j], a[i][j]);
            a[i][k] = l;
        }
    }
    return exchange;
}

template <typename Real>
__device__ __forceinline__ void cube_solve(const Real a[8][8], const Real rinv[8], Real b[8])
{
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int i = k + 1; i < 8; ++i)
            if (cube_nz(k, i, k)) b[i] = fma(-a[i][k], b[k], b[i]);
#pragma unroll
    for (int i = 7; i >= 0; --i) {
        Real s = b[i];
#pragma unroll
        for (int j = i + 1; j < 8; ++j)
            if (cube_nz(8, i, j)) s = fma(-a[i][j], b[j], s);
        b[i] = s * rinv[i];
    }
}

template <typename Real>
__device__ __forceinline__ bool ge_solve8_cube(Real a[8][8], Real b[8])
{
    Real rinv[8];
    const bool exchange = cube_factor(a, rinv);
    cube_solve(a, rinv, b);
    return exchange;
}

}  // namespace dgsn
