/*
 * FP64 CPU oracle for the trilinear-hexahedron DGFEM S_n transport sweep of
 * Tano & Ragusa, "Acceleration of Radiation Transport Solves Using Artificial
 * Neural Networks" (arXiv 1906.04017).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  It is a plain, slow,
 * obviously-correct reference used only by the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark.  It shares no code with the HIP
 * library (no headers, helpers, tables or constant generators) and must never
 * be linked into it.
 *
 * What it follows in the paper:
 *   - Sec. 2, Eq. (T1): steady mono-energetic transport, Omega.grad psi + sigma_t psi = Q.
 *   - Eq. (T2)-(T8): Q = q_ext + sigma_s/(4 pi) phi, phi = sum_d w_d psi_d (P0,
 *     in-group or with a group-to-group matrix), and the anisotropic in-group
 *     P_L expansion, Q_d = q_ext + sum_{n,m} sigma_{s,n} Y_{n,m}(Omega_d)
 *     phi_{n,m} with phi_{n,m} = sum_d w_d Y_{n,m}(Omega_d) psi_d (Eq. (T7),
 *     (T8); real orthonormal spherical harmonics, orc_real_ylm), also with a
 *     group-to-group matrix per Legendre order (the group sum of Eq. (T3)).
 *   - Eq. (T9): trilinear nodal trial space on each hexahedron, 8 vertex nodes,
 *     local node n = ix + 2 iy + 4 iz.
 *   - The weak form below Eq. (T9): streaming by Green's theorem, element mass
 *     M, gradient matrices, face mass matrices on the inflow / outflow parts of
 *     the cell boundary, full upwinding of the inflow trace (Sec. 2, the
 *     "first order interpolation" paragraph), boundary inflow Eq. (TBC).
 *   - Eq. (T12): the per-cell system A psi_d = b solved by Gaussian elimination
 *     (partial pivoting, lowest row index on ties; the paper does not state the
 *     pivoting rule).
 *   - Sec. 2, the sweep paragraph after Eq. (T12): cells are visited from the
 *     inflow boundaries downstream; here by plain nested loops in upwind order.
 *   - Source iteration (Sec. 2, after Eq. (T6)); stopping metric Eq. (Test:Eq3).
 *
 * Element matrices are integrated with a 2-point Gauss-Legendre tensor rule
 * (exact for these polynomial integrands).  Everything is double precision.
 *
 * The adjoint (discrete transpose of the source-iteration system) is not in the
 * paper; it is the exact transpose of the operator above, written out with
 * explicit transposed matrices and a reversed (downwind-to-upwind) sweep.
 *
 * Two shallow networks replace assembly + GE when asked (Sec. 3, Sec. 4):
 *   - a canonical-octant network on 24 homogeneity-normalised features (the
 *     library's matrix-core network), and
 *   - the paper's own form, Eq. (ANN:Eq1)-(ANN:Eq4): 26 physical-frame inputs
 *     scaled by Eq. (ANN:Eq2), tanh hidden layer, ELU output with
 *     beta = 0.1 max(psi_inc), one network per octant or one per quadrature
 *     direction (orc_pann_*).
 * Both forward passes are written out literally in FP64; they are pinned by
 * hand-built networks with closed-form outputs, selector networks that read
 * the inputs back, homogeneity, mirror equivariance, and for the
 * per-direction set constant networks whose sweep is a weighted index sum
 * (tests).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ESINGULAR -3
#define ORC_ENOTCONV -4

static const double ORC_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ */
/* Basis functions on the reference cube [0,1]^3                        */
/* ------------------------------------------------------------------ */

/* 1D Lagrange basis on [0,1]: l0(s) = 1 - s, l1(s) = s. */
static double lag(int i, double s) { return i ? s : 1.0 - s; }
static double dlag(int i) { return i ? 1.0 : -1.0; }

static int node_bit(int n, int axis) { return (n >> axis) & 1; }

/* b_n at reference point (xi[0], xi[1], xi[2]). */
static double basis(int n, const double xi[3])
{
    return lag(node_bit(n, 0), xi[0]) * lag(node_bit(n, 1), xi[1]) * lag(node_bit(n, 2), xi[2]);
}

/* d b_n / d x_axis in physical units, cell sizes h[3]. */
static double dbasis(int n, int axis, const double xi[3], const double h[3])
{
    double v = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (a == axis) v *= dlag(node_bit(n, a)) / h[a];
        else v *= lag(node_bit(n, a), xi[a]);
    }
    return v;
}

/*
 * Element matrices of one hexahedron with edge lengths h[3]
 * (weak form under Eq. (T9)):
 *   M[k][j]     = int_V b_k b_j dV                      (mass)
 *   G[a][k][j]  = int_V (d_a b_k) b_j dV                (gradient of the test function)
 *   Mf[f][k][j] = int_{face f} b_k b_j dA               (face mass)
 * Faces: f = 2*axis + side, side 0 is the low face (outward normal -e_axis),
 * side 1 the high face (+e_axis).  2-point Gauss-Legendre per direction.
 */
void orc_element_matrices(const double h[3], double M[64], double G[3][64], double Mf[6][64])
{
    const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
    const double gw = 0.5;
    const double vol = h[0] * h[1] * h[2];
    memset(M, 0, 64 * sizeof(double));
    memset(G, 0, 3 * 64 * sizeof(double));
    memset(Mf, 0, 6 * 64 * sizeof(double));
    for (int qx = 0; qx < 2; ++qx)
        for (int qy = 0; qy < 2; ++qy)
            for (int qz = 0; qz < 2; ++qz) {
                const double xi[3] = {gp[qx], gp[qy], gp[qz]};
                const double wq = gw * gw * gw * vol;
                for (int k = 0; k < 8; ++k)
                    for (int j = 0; j < 8; ++j) {
                        M[k * 8 + j] += wq * basis(k, xi) * basis(j, xi);
                        for (int a = 0; a < 3; ++a)
                            G[a][k * 8 + j] += wq * dbasis(k, a, xi, h) * basis(j, xi);
                    }
            }
    for (int axis = 0; axis < 3; ++axis) {
        const int t1 = (axis + 1) % 3, t2 = (axis + 2) % 3;
        const double area = h[t1] * h[t2];
        for (int side = 0; side < 2; ++side) {
            const int f = 2 * axis + side;
            for (int q1 = 0; q1 < 2; ++q1)
                for (int q2 = 0; q2 < 2; ++q2) {
                    double xi[3];
                    xi[axis] = (double)side;
                    xi[t1] = gp[q1];
                    xi[t2] = gp[q2];
                    const double wq = gw * gw * area;
                    for (int k = 0; k < 8; ++k)
                        for (int j = 0; j < 8; ++j)
                            Mf[f][k * 8 + j] += wq * basis(k, xi) * basis(j, xi);
                }
        }
    }
}

/* Outward normal component of face f along its axis: -1 (low) or +1 (high). */
static double face_sign(int f) { return (f & 1) ? 1.0 : -1.0; }

/* ------------------------------------------------------------------ */
/* Gaussian elimination with partial pivoting (Eq. (T12) solve)         */
/* ------------------------------------------------------------------ */

/*
 * Solves A x = b for an n-by-n row-major A (n <= 8).  A and b are copied.
 * Partial pivoting: the pivot of column k is the row i >= k with the largest
 * |a_ik|; on ties the lowest index wins (strict comparison).
 */
int orc_ge_solve(int n, const double *A_in, const double *b_in, double *x)
{
    double A[64], b[8];
    if (n < 1 || n > 8) return ORC_EINVAL;
    memcpy(A, A_in, (size_t)n * n * sizeof(double));
    memcpy(b, b_in, (size_t)n * sizeof(double));
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); p = i; }
        if (best == 0.0) return ORC_ESINGULAR;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t;
            }
            double t = b[k]; b[k] = b[p]; b[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            const double l = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
            b[i] -= l * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * x[j];
        x[i] = s / A[i * n + i];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Local system of one cell and one direction (Eq. (T10)-(T12))         */
/* ------------------------------------------------------------------ */

/*
 * Cell matrix for direction omega (integration-by-parts form):
 *   A = - sum_a omega_a G_a + sum_{f: omega.n_f > 0} (omega.n_f) Mf_f + sigma_t M
 * The outflow face terms stay on the left, the inflow ones go to the right
 * hand side (the A_psi / b_psi split stated under Eq. (T12)).
 */
void orc_cell_matrix(const double omega[3], double sigma_t, const double M[64],
                     const double G[3][64], const double Mf[6][64], double A[64])
{
    for (int e = 0; e < 64; ++e) {
        double v = sigma_t * M[e];
        for (int a = 0; a < 3; ++a) v -= omega[a] * G[a][e];
        A[e] = v;
    }
    for (int f = 0; f < 6; ++f) {
        const double on = omega[f / 2] * face_sign(f);
        if (on > 0.0)
            for (int e = 0; e < 64; ++e) A[e] += on * Mf[f][e];
    }
}

/*
 * Right-hand side:
 *   b = sum_{f: omega.n_f < 0} |omega.n_f| Mf_f psi_up_f + M S
 * psi_up[f][n] holds the upwind trace at the face-f nodes n of this cell
 * (entries at nodes off the face are ignored by Mf_f).
 */
void orc_cell_rhs(const double omega[3], const double M[64], const double Mf[6][64],
                  const double S[8], const double psi_up[6][8], double b[8])
{
    for (int k = 0; k < 8; ++k) {
        double v = 0.0;
        for (int j = 0; j < 8; ++j) v += M[k * 8 + j] * S[j];
        b[k] = v;
    }
    for (int f = 0; f < 6; ++f) {
        const double on = omega[f / 2] * face_sign(f);
        if (on < 0.0)
            for (int k = 0; k < 8; ++k)
                for (int j = 0; j < 8; ++j) b[k] += -on * Mf[f][k * 8 + j] * psi_up[f][j];
    }
}

/* ------------------------------------------------------------------ */
/* Mesh helpers                                                         */
/* ------------------------------------------------------------------ */

typedef struct {
    int n[3];      /* cells per axis */
    double h[3];   /* cell edge lengths */
} orc_mesh;

static long cell_index(const orc_mesh *m, const int c[3])
{
    return (long)c[0] + (long)m->n[0] * ((long)c[1] + (long)m->n[1] * (long)c[2]);
}

/* Neighbour across face f; returns 0 if the face lies on the domain boundary. */
static int neighbour(const orc_mesh *m, const int c[3], int f, int nb[3])
{
    const int axis = f / 2;
    nb[0] = c[0]; nb[1] = c[1]; nb[2] = c[2];
    nb[axis] += (f & 1) ? 1 : -1;
    return nb[axis] >= 0 && nb[axis] < m->n[axis];
}

/*
 * Upwind trace for face f of cell c in direction omega (only called for
 * inflow faces): the neighbour's nodal values at the coincident nodes (node
 * index with the face-axis bit flipped), or the domain inflow value psi_inc[f]
 * on the boundary (Eq. (TBC); vacuum is 0).
 */
static void upwind_trace(const orc_mesh *m, const int c[3], int f, const double *psi_dir,
                         const double psi_inc[6], double out[8])
{
    int nb[3];
    const int axis = f / 2;
    if (neighbour(m, c, f, nb)) {
        const double *pn = psi_dir + 8 * cell_index(m, nb);
        for (int n = 0; n < 8; ++n) out[n] = pn[n ^ (1 << axis)];
    } else {
        for (int n = 0; n < 8; ++n) out[n] = psi_inc[f];
    }
}

/* Visit order along one axis: upwind to downwind. */
static int axis_start(int nax, double om) { return om >= 0.0 ? 0 : nax - 1; }
static int axis_step(double om) { return om >= 0.0 ? 1 : -1; }

/*
 * One transport sweep for one direction and one group: solves the per-cell
 * systems of Eq. (T12) cell by cell in upwind order (nested k, j, i loops, each
 * running from the inflow side; a valid topological order of the upwind
 * dependency graph).  psi_dir receives [ncell][8] nodal angular fluxes.
 */
typedef struct orc_ann orc_ann;
static int ann_cell(const orc_ann *net, const double h[3], const double omega[3], double sigma_t,
                    const double S[8], const double psi_up[6][8], double psi[8]);

static int sweep_one(const orc_mesh *m, const double omega[3], const double *sigma_t,
                     const double *src, const double psi_inc[6], const double M[64],
                     const double G[3][64], const double Mf[6][64], const orc_ann *net,
                     double *psi_dir)
{
    int c[3];
    const int s0 = axis_start(m->n[0], omega[0]), d0 = axis_step(omega[0]);
    const int s1 = axis_start(m->n[1], omega[1]), d1 = axis_step(omega[1]);
    const int s2 = axis_start(m->n[2], omega[2]), d2 = axis_step(omega[2]);
    for (int kk = 0; kk < m->n[2]; ++kk) {
        c[2] = s2 + d2 * kk;
        for (int jj = 0; jj < m->n[1]; ++jj) {
            c[1] = s1 + d1 * jj;
            for (int ii = 0; ii < m->n[0]; ++ii) {
                c[0] = s0 + d0 * ii;
                const long ci = cell_index(m, c);
                double up[6][8], A[64], b[8];
                memset(up, 0, sizeof(up));
                for (int f = 0; f < 6; ++f)
                    if (omega[f / 2] * face_sign(f) < 0.0)
                        upwind_trace(m, c, f, psi_dir, psi_inc, up[f]);
                int rc;
                if (net) {
                    rc = ann_cell(net, m->h, omega, sigma_t[ci], src + 8 * ci,
                                  (const double(*)[8])up, psi_dir + 8 * ci);
                } else {
                    orc_cell_matrix(omega, sigma_t[ci], M, G, Mf, A);
                    orc_cell_rhs(omega, M, Mf, src + 8 * ci, (const double(*)[8])up, b);
                    rc = orc_ge_solve(8, A, b, psi_dir + 8 * ci);
                }
                if (rc) return rc;
            }
        }
    }
    return ORC_OK;
}

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/*
 * Full sweep over all directions and groups (one application of the inverse
 * streaming-collision operator):
 *   sigma_t [G][ncell], src [G][ncell][8] total nodal source per steradian,
 *   psi_inc[6] per domain face, phi [G][ncell][8] out = sum_d w_d psi_d
 *   (Eq. (T11)), accumulated in direction order for every (g, cell, node).
 *   psi_store, if not NULL, receives [D][G][ncell][8].
 * Work units (d, g) are independent; blocks of them run in parallel and are
 * summed into phi in unit order afterwards, so the result does not depend on
 * the thread count.
 */
static int sweep_all(int nx, int ny, int nz, double lx, double ly, double lz, int ng, int nd,
                     const double *omega, const double *weight, const double *sigma_t,
                     const double *src, const double psi_inc[6], double *phi, double *psi_store,
                     const orc_ann *net, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || ng < 1 || nd < 1) return ORC_EINVAL;
    orc_mesh m = {{nx, ny, nz}, {lx / nx, ly / ny, lz / nz}};
    const long ncell = (long)nx * ny * nz;
    double M[64], G[3][64], Mf[6][64];
    orc_element_matrices(m.h, M, G, Mf);
    const int nt = set_threads(nthreads);
    const long nunits = (long)nd * ng;
    double *buf = (double *)malloc((size_t)nt * ncell * 8 * sizeof(double));
    if (!buf) return ORC_ENOMEM;
    memset(phi, 0, (size_t)ng * ncell * 8 * sizeof(double));
    int err = ORC_OK;
    for (long u0 = 0; u0 < nunits && !err; u0 += nt) {
        const long nb = (nunits - u0 < nt) ? nunits - u0 : nt;
#pragma omp parallel for schedule(static, 1)
        for (long t = 0; t < nb; ++t) {
            const long u = u0 + t;
            const int d = (int)(u / ng), g = (int)(u % ng);
            int rc = sweep_one(&m, omega + 3 * d, sigma_t + g * ncell, src + 8 * g * ncell,
                               psi_inc, M, G, Mf, net, buf + t * ncell * 8);
            if (rc) {
#pragma omp critical
                err = rc;
            }
        }
        if (err) break;
#pragma omp parallel for schedule(static)
        for (long ci = 0; ci < ncell; ++ci)
            for (long t = 0; t < nb; ++t) {
                const long u = u0 + t;
                const int d = (int)(u / ng), g = (int)(u % ng);
                const double *p = buf + (t * ncell + ci) * 8;
                double *f = phi + ((long)g * ncell + ci) * 8;
                for (int n = 0; n < 8; ++n) f[n] += weight[d] * p[n];
            }
        if (psi_store)
            for (long t = 0; t < nb; ++t) {
                const long u = u0 + t;
                const int d = (int)(u / ng), g = (int)(u % ng);
                memcpy(psi_store + ((long)d * ng + g) * ncell * 8, buf + t * ncell * 8,
                       (size_t)ncell * 8 * sizeof(double));
            }
    }
    free(buf);
    return err;
}

int orc_sweep(int nx, int ny, int nz, double lx, double ly, double lz, int ng, int nd,
              const double *omega, const double *weight, const double *sigma_t,
              const double *src, const double psi_inc[6], double *phi, double *psi_store,
              int nthreads)
{
    return sweep_all(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, src, psi_inc, phi,
                     psi_store, NULL, nthreads);
}

/*
 * Convergence measures of one source iteration step, from the new and the
 * previous scalar flux (nv = G * ncell values of 8 nodes each):
 *   r     = max_{g,c,n} |phi_new - phi_old| / max_{g,c,n} |phi_new|  (0 if phi_new = 0),
 *           the max-norm relative change used as the stopping test;
 *   eps_s = Eq. (Test:Eq3), the mean over the nv (group, cell) pairs of the
 *           pointwise relative change of the cell-average flux
 *           |avg_new - avg_old| / |avg_new|, avg the mean of the cell's 8
 *           nodal values (the trilinear flux integrated over the cell and
 *           divided by its volume).  A cell whose new average is 0 counts 0
 *           if the old one is 0 as well and 1 otherwise (the relative change
 *           of Eq. (Test:Eq3) is undefined there; a change from a non-zero
 *           value to zero is a full change).
 */
void orc_si_metrics(long nv, const double *phi_new, const double *phi_old, double *r,
                    double *eps_s)
{
    double dmax = 0.0, fmax = 0.0, esum = 0.0;
    for (long i = 0; i < nv * 8; ++i) {
        const double dd = fabs(phi_new[i] - phi_old[i]);
        if (dd > dmax) dmax = dd;
        if (fabs(phi_new[i]) > fmax) fmax = fabs(phi_new[i]);
    }
    for (long gc = 0; gc < nv; ++gc) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < 8; ++k) { a += phi_new[gc * 8 + k]; b += phi_old[gc * 8 + k]; }
        a /= 8.0; b /= 8.0;
        esum += (a != 0.0) ? fabs(a - b) / fabs(a) : (b != 0.0 ? 1.0 : 0.0);
    }
    *r = fmax > 0.0 ? dmax / fmax : 0.0;
    *eps_s = esum / (double)nv;
}

/* Nodal total source S = q_ext + sigma_s / (4 pi) phi (isotropic, Eq. (T5) P0 term). */
static void build_source(long n, const double *q, const double *sigma_s, const double *phi,
                         double *S)
{
    for (long gc = 0; gc < n; ++gc)
        for (int k = 0; k < 8; ++k)
            S[gc * 8 + k] = q[gc] + sigma_s[gc] / (4.0 * ORC_PI) * phi[gc * 8 + k];
}

/*
 * Multigroup isotropic scattering (the group sum of Eq. (T3)-(T8) at P0):
 *   S[g][c][k] = q[g][c] + sum_{g'} sigma_gg[g'][g][c] / (4 pi) phi[g'][c][k],
 * sigma_gg[g'][g][c] being the scattering cross section from group g' into
 * group g, summed over g' in ascending order.
 */
static void build_source_gg(int ng, long ncell, const double *q, const double *sigma_gg,
                            const double *phi, double *S)
{
    for (int g = 0; g < ng; ++g)
        for (long c = 0; c < ncell; ++c)
            for (int k = 0; k < 8; ++k) {
                double v = q[g * ncell + c];
                for (int g2 = 0; g2 < ng; ++g2)
                    v += sigma_gg[((long)g2 * ng + g) * ncell + c] / (4.0 * ORC_PI) *
                         phi[((long)g2 * ncell + c) * 8 + k];
                S[((long)g * ncell + c) * 8 + k] = v;
            }
}

/*
 * Scattering source iteration.  phi [G][ncell][8] holds the initial guess on
 * entry and the last iterate on exit.  Iterate: S = q + sigma_s/(4 pi) phi^n,
 * sweep, phi^{n+1}.  Residual r = max|phi^{n+1} - phi^n| / max|phi^{n+1}| over
 * all entries; eps_s is Eq. (Test:Eq3) on cell averages.  Stops when r < tol.
 * Returns ORC_ENOTCONV when max_iter sweeps did not reach tol.
 */
static int source_iterate(int nx, int ny, int nz, double lx, double ly, double lz, int ng,
                          int nd, const double *omega, const double *weight,
                          const double *sigma_t, const double *sigma_s, const double *q,
                          const double psi_inc[6], double *phi, double tol, int max_iter,
                          int *iters, double *resid, double *eps_s, double *psi_store,
                          const orc_ann *net, int nthreads, const double *sigma_gg,
                          int stop_on_eps_s)
{
    const long ncell = (long)nx * ny * nz;
    const long nv = (long)ng * ncell;
    double *S = (double *)malloc((size_t)nv * 8 * sizeof(double));
    double *phin = (double *)malloc((size_t)nv * 8 * sizeof(double));
    if (!S || !phin) { free(S); free(phin); return ORC_ENOMEM; }
    int it = 0, rc = ORC_OK;
    double r = INFINITY, es = INFINITY;
    while (it < max_iter) {
        if (sigma_gg) build_source_gg(ng, ncell, q, sigma_gg, phi, S);
        else build_source(nv, q, sigma_s, phi, S);
        rc = sweep_all(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, S, psi_inc, phin,
                       psi_store, net, nthreads);
        if (rc) break;
        orc_si_metrics(nv, phin, phi, &r, &es);
        memcpy(phi, phin, (size_t)nv * 8 * sizeof(double));
        ++it;
        if ((stop_on_eps_s ? es : r) < tol) break;
    }
    free(S);
    free(phin);
    if (iters) *iters = it;
    if (resid) *resid = r;
    if (eps_s) *eps_s = es;
    if (rc) return rc;
    return ((stop_on_eps_s ? es : r) < tol) ? ORC_OK : ORC_ENOTCONV;
}

int orc_source_iterate(int nx, int ny, int nz, double lx, double ly, double lz, int ng, int nd,
                       const double *omega, const double *weight, const double *sigma_t,
                       const double *sigma_s, const double *q, const double psi_inc[6],
                       double *phi, double tol, int max_iter, int *iters, double *resid,
                       double *eps_s, double *psi_store, int nthreads)
{
    return source_iterate(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, sigma_s, q,
                          psi_inc, phi, tol, max_iter, iters, resid, eps_s, psi_store, NULL,
                          nthreads, NULL, 0);
}

/* The same iteration stopped on the paper's criterion: eps_S of Eq.
   (Test:Eq3) below tol (the Problem 4 runs of Sec. 4 use 1e-4). */
int orc_source_iterate_eps(int nx, int ny, int nz, double lx, double ly, double lz, int ng,
                           int nd, const double *omega, const double *weight,
                           const double *sigma_t, const double *sigma_s, const double *q,
                           const double psi_inc[6], double *phi, double tol, int max_iter,
                           int *iters, double *resid, double *eps_s, double *psi_store,
                           int nthreads)
{
    return source_iterate(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, sigma_s, q,
                          psi_inc, phi, tol, max_iter, iters, resid, eps_s, psi_store, NULL,
                          nthreads, NULL, 1);
}

/* Source iteration with multigroup scattering sigma_gg [G][G][ncell] (from g'
   into g at [g'][g]); the in-group sigma_s is not used. */
int orc_source_iterate_gg(int nx, int ny, int nz, double lx, double ly, double lz, int ng,
                          int nd, const double *omega, const double *weight,
                          const double *sigma_t, const double *sigma_gg, const double *q,
                          const double psi_inc[6], double *phi, double tol, int max_iter,
                          int *iters, double *resid, double *eps_s, double *psi_store,
                          int nthreads)
{
    if (!sigma_gg) return ORC_EINVAL;
    return source_iterate(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, NULL, q,
                          psi_inc, phi, tol, max_iter, iters, resid, eps_s, psi_store, NULL,
                          nthreads, sigma_gg, 0);
}

/* ------------------------------------------------------------------ */
/* Anisotropic P_L scattering (Eq. (T3)-(T8))                           */
/* ------------------------------------------------------------------ */

/*
 * Real orthonormal spherical harmonics up to order L (L <= 8) at the unit
 * direction omega, polar axis z: mu = omega_z, azimuth phi = atan2(omega_y,
 * omega_x).  Y[k], k = n^2 + n + m:
 *   m = 0:  N_n0 P_n(mu)
 *   m > 0:  sqrt(2) N_nm P_n^m(mu) cos(m phi)
 *   m < 0:  sqrt(2) N_n|m| P_n^|m|(mu) sin(|m| phi)
 * with N_nm = sqrt((2n+1)/(4 pi) (n-m)!/(n+m)!) and the associated Legendre
 * functions P_n^m = (1 - mu^2)^(m/2) d^m/dmu^m P_n without the (-1)^m phase,
 * from the standard recurrences in n at fixed m:
 *   P_m^m = (2m-1)!! (1-mu^2)^(m/2),  P_{m+1}^m = (2m+1) mu P_m^m,
 *   (n-m) P_n^m = (2n-1) mu P_{n-1}^m - (n+m-1) P_{n-2}^m.
 * They satisfy the addition theorem sum_m Y_nm(a) Y_nm(b) = (2n+1)/(4 pi)
 * P_n(a.b) behind Eq. (T4) (pinned in the tests).
 */
int orc_real_ylm(int L, const double omega[3], double *Y)
{
    if (L < 0 || L > 8) return ORC_EINVAL;
    const double mu = omega[2];
    const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    const double az = atan2(omega[1], omega[0]);
    for (int m = 0; m <= L; ++m) {
        /* P_m^m */
        double pmm = 1.0;
        for (int i = 1; i <= m; ++i) pmm *= (2.0 * i - 1.0) * st;
        double p_prev = 0.0, p_cur = pmm;
        for (int n = m; n <= L; ++n) {
            double p;
            if (n == m) p = pmm;
            else if (n == m + 1) p = (2.0 * m + 1.0) * mu * pmm;
            else p = ((2.0 * n - 1.0) * mu * p_cur - (n + m - 1.0) * p_prev) / (double)(n - m);
            if (n > m) { p_prev = p_cur; p_cur = p; }
            /* (n-m)!/(n+m)! */
            double ratio = 1.0;
            for (int i = n - m + 1; i <= n + m; ++i) ratio /= (double)i;
            const double N = sqrt((2.0 * n + 1.0) / (4.0 * ORC_PI) * ratio);
            if (m == 0) {
                Y[n * n + n] = N * p;
            } else {
                Y[n * n + n + m] = sqrt(2.0) * N * p * cos(m * az);
                Y[n * n + n - m] = sqrt(2.0) * N * p * sin(m * az);
            }
        }
    }
    return ORC_OK;
}

/* sigma_{s,o} from group g2 into group g of cell c: in-group [o][g][c] (g2 =
   g), or with a matrix per order [o][g2][g][c] */
static double sn_coef(const double *sigma_sn, int gg, int o, int g2, int g, int ng, long ncell,
                      long c)
{
    return gg ? sigma_sn[(((long)o * ng + g2) * ng + g) * ncell + c]
              : sigma_sn[((long)o * ng + g) * ncell + c];
}

/*
 * Source iteration with P_L scattering, L >= 1.
 *   sigma_sn: the Legendre moments sigma_{s,n} of Eq. (T3), order 0 first
 *     (the isotropic part), either in-group, [L+1][G][ncell], or (gg != 0)
 *     a group-to-group matrix per order, [L+1][G][G][ncell] with the
 *     moment from group g' into group g at [n][g'][g];
 *   phi [G][ncell][8]: scalar flux (= the moment phi_{0,0} / Y_00), initial
 *     guess on entry, last iterate on exit;
 *   mom [(L+1)^2 - 1][G][ncell][8]: the flux moments phi_{n,m} of Eq. (T8)
 *     for k = n^2 + n + m >= 1, initial guess on entry, last iterate on exit.
 * Iteration: Q_{d,g} = q_g + sum_{g'} (sigma_{s,0}(g'->g)/(4 pi) phi_{g'} +
 * sum_{k>=1} sigma_{s,n(k)}(g'->g) Y_k(Omega_d) mom_{k,g'}) over the source
 * groups g' (g' = g only, in-group) in ascending order, one sweep per
 * (direction, group) with that source, then phi = sum_d w_d psi_d and
 * mom_k = sum_d w_d Y_k(Omega_d) psi_d, accumulated in direction order.
 * Residual and eps_s on phi as in source_iterate.  psi_store, if not NULL,
 * receives the last sweep's [D][G][ncell][8].
 */
static int source_iterate_pl(int nx, int ny, int nz, double lx, double ly, double lz, int ng,
                             int nd, const double *omega, const double *weight,
                             const double *sigma_t, int L, const double *sigma_sn, int gg,
                             const double *q, const double psi_inc[6], double *phi, double *mom,
                             double tol, int max_iter, int *iters, double *resid, double *eps_s,
                             double *psi_store, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || ng < 1 || nd < 1 || L < 1 || L > 8) return ORC_EINVAL;
    orc_mesh m = {{nx, ny, nz}, {lx / nx, ly / ny, lz / nz}};
    const long ncell = (long)nx * ny * nz;
    const long nv = (long)ng * ncell;
    const int nm = (L + 1) * (L + 1);
    double M[64], G[3][64], Mf[6][64];
    orc_element_matrices(m.h, M, G, Mf);
    const int nt = set_threads(nthreads);
    double *Y = (double *)malloc((size_t)nd * nm * sizeof(double));
    double *buf = (double *)malloc((size_t)nt * ncell * 8 * sizeof(double));
    double *src = (double *)malloc((size_t)nt * ncell * 8 * sizeof(double));
    double *phin = (double *)malloc((size_t)nv * 8 * sizeof(double));
    double *momn = (double *)malloc((size_t)(nm - 1) * nv * 8 * sizeof(double));
    if (!Y || !buf || !src || !phin || !momn) {
        free(Y); free(buf); free(src); free(phin); free(momn);
        return ORC_ENOMEM;
    }
    for (int d = 0; d < nd; ++d) orc_real_ylm(L, omega + 3 * d, Y + (long)d * nm);
    int it = 0, err = ORC_OK;
    double r = INFINITY, es = INFINITY;
    const long nunits = (long)nd * ng;
    while (it < max_iter && !err) {
        memset(phin, 0, (size_t)nv * 8 * sizeof(double));
        memset(momn, 0, (size_t)(nm - 1) * nv * 8 * sizeof(double));
        for (long u0 = 0; u0 < nunits && !err; u0 += nt) {
            const long nb = (nunits - u0 < nt) ? nunits - u0 : nt;
#pragma omp parallel for schedule(static, 1)
            for (long t = 0; t < nb; ++t) {
                const long u = u0 + t;
                const int d = (int)(u / ng), g = (int)(u % ng);
                const double *yd = Y + (long)d * nm;
                double *S = src + t * ncell * 8;
                for (long c = 0; c < ncell; ++c) {
                    const long gc = (long)g * ncell + c;
                    for (int n = 0; n < 8; ++n) {
                        double v = q[gc];
                        for (int g2 = gg ? 0 : g; g2 <= (gg ? ng - 1 : g); ++g2) {
                            const long g2c = (long)g2 * ncell + c;
                            v += sn_coef(sigma_sn, gg, 0, g2, g, ng, ncell, c) / (4.0 * ORC_PI) *
                                 phi[g2c * 8 + n];
                            for (int o = 1; o <= L; ++o) {
                                const double sig = sn_coef(sigma_sn, gg, o, g2, g, ng, ncell, c);
                                for (int mm = -o; mm <= o; ++mm) {
                                    const int k = o * o + o + mm;
                                    v += sig * yd[k] * mom[((long)(k - 1) * nv + g2c) * 8 + n];
                                }
                            }
                        }
                        S[c * 8 + n] = v;
                    }
                }
                int rc = sweep_one(&m, omega + 3 * d, sigma_t + g * ncell, S, psi_inc, M, G, Mf,
                                   NULL, buf + t * ncell * 8);
                if (rc) {
#pragma omp critical
                    err = rc;
                }
            }
            if (err) break;
            if (psi_store)
                for (long t = 0; t < nb; ++t) {
                    const long u = u0 + t;
                    const int d = (int)(u / ng), g = (int)(u % ng);
                    memcpy(psi_store + ((long)d * ng + g) * ncell * 8, buf + t * ncell * 8,
                           (size_t)ncell * 8 * sizeof(double));
                }
            /* each (group, cell) accumulates its units in unit order */
#pragma omp parallel for schedule(static)
            for (long c = 0; c < ncell; ++c)
                for (long t = 0; t < nb; ++t) {
                    const long u = u0 + t;
                    const int d = (int)(u / ng), g = (int)(u % ng);
                    const double *yd = Y + (long)d * nm;
                    const long gc = (long)g * ncell + c;
                    const double *p = buf + (t * ncell + c) * 8;
                    for (int n = 0; n < 8; ++n) {
                        phin[gc * 8 + n] += weight[d] * p[n];
                        for (int k = 1; k < nm; ++k)
                            momn[((long)(k - 1) * nv + gc) * 8 + n] += weight[d] * yd[k] * p[n];
                    }
                }
        }
        if (err) break;
        orc_si_metrics(nv, phin, phi, &r, &es);
        memcpy(phi, phin, (size_t)nv * 8 * sizeof(double));
        memcpy(mom, momn, (size_t)(nm - 1) * nv * 8 * sizeof(double));
        ++it;
        if (r < tol) break;
    }
    free(Y); free(buf); free(src); free(phin); free(momn);
    if (iters) *iters = it;
    if (resid) *resid = r;
    if (eps_s) *eps_s = es;
    if (err) return err;
    return (r < tol) ? ORC_OK : ORC_ENOTCONV;
}

/* In-group P_L: sigma_sn [L+1][G][ncell]. */
int orc_source_iterate_pl(int nx, int ny, int nz, double lx, double ly, double lz, int ng,
                          int nd, const double *omega, const double *weight,
                          const double *sigma_t, int L, const double *sigma_sn, const double *q,
                          const double psi_inc[6], double *phi, double *mom, double tol,
                          int max_iter, int *iters, double *resid, double *eps_s,
                          double *psi_store, int nthreads)
{
    return source_iterate_pl(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, L, sigma_sn,
                             0, q, psi_inc, phi, mom, tol, max_iter, iters, resid, eps_s,
                             psi_store, nthreads);
}

/* Group-to-group P_L: sigma_sn [L+1][G][G][ncell], from g' into g at [n][g'][g]. */
int orc_source_iterate_pl_gg(int nx, int ny, int nz, double lx, double ly, double lz, int ng,
                             int nd, const double *omega, const double *weight,
                             const double *sigma_t, int L, const double *sigma_sn,
                             const double *q, const double psi_inc[6], double *phi, double *mom,
                             double tol, int max_iter, int *iters, double *resid, double *eps_s,
                             double *psi_store, int nthreads)
{
    return source_iterate_pl(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, L, sigma_sn,
                             1, q, psi_inc, phi, mom, tol, max_iter, iters, resid, eps_s,
                             psi_store, nthreads);
}

/* ------------------------------------------------------------------ */
/* Adjoint (exact discrete transpose)                                   */
/* ------------------------------------------------------------------ */

/*
 * Inflow coupling of cell c' through its face f (omega.n_f < 0) to its upwind
 * neighbour: b_c' += U psi_nb, U = |omega.n_f| Mf_f P_f, where
 * (P_f psi_nb)[n] = psi_nb[n ^ bit(axis f)] for the face nodes n.  Built as an
 * explicit 8x8 matrix so that its transpose can be applied literally.
 */
static void coupling_matrix(const double omega[3], int f, const double Mf[6][64], double U[64])
{
    const int axis = f / 2;
    const double on = fabs(omega[axis]);
    double P[64];
    memset(P, 0, sizeof(P));
    for (int n = 0; n < 8; ++n)
        if (node_bit(n, axis) == (f & 1)) P[n * 8 + (n ^ (1 << axis))] = 1.0;
    for (int k = 0; k < 8; ++k)
        for (int j = 0; j < 8; ++j) {
            double v = 0.0;
            for (int l = 0; l < 8; ++l) v += Mf[f][k * 8 + l] * P[l * 8 + j];
            U[k * 8 + j] = on * v;
        }
}

/*
 * Transposed sweep for one direction and group: solves A_c^T mu_c = rhs_c
 * with rhs_c = load_c + sum over downwind neighbours c' of U_{c'}^T mu_{c'},
 * visiting cells from downwind to upwind (the exact reverse of sweep_one).
 * Homogeneous boundary condition.
 */
static int adjoint_sweep_one(const orc_mesh *m, const double omega[3], const double *sigma_t,
                             const double *load, const double M[64], const double G[3][64],
                             const double Mf[6][64], double *mu_dir)
{
    int c[3];
    double U[6][64];
    for (int f = 0; f < 6; ++f)
        if (omega[f / 2] * face_sign(f) < 0.0) coupling_matrix(omega, f, Mf, U[f]);
    /* reversed visit order: each axis runs from its downwind end */
    const int d0 = -axis_step(omega[0]), e0 = omega[0] >= 0.0 ? m->n[0] - 1 : 0;
    const int d1 = -axis_step(omega[1]), e1 = omega[1] >= 0.0 ? m->n[1] - 1 : 0;
    const int d2 = -axis_step(omega[2]), e2 = omega[2] >= 0.0 ? m->n[2] - 1 : 0;
    for (int kk = 0; kk < m->n[2]; ++kk) {
        c[2] = e2 + d2 * kk;
        for (int jj = 0; jj < m->n[1]; ++jj) {
            c[1] = e1 + d1 * jj;
            for (int ii = 0; ii < m->n[0]; ++ii) {
                c[0] = e0 + d0 * ii;
                const long ci = cell_index(m, c);
                double A[64], At[64], rhs[8];
                orc_cell_matrix(omega, sigma_t[ci], M, G, Mf, A);
                for (int k = 0; k < 8; ++k)
                    for (int j = 0; j < 8; ++j) At[k * 8 + j] = A[j * 8 + k];
                for (int k = 0; k < 8; ++k) rhs[k] = load[8 * ci + k];
                /* downwind neighbours: cells c' across the outflow faces of c;
                   c is upwind of c' through the opposite face f' of c'. */
                for (int f = 0; f < 6; ++f) {
                    if (!(omega[f / 2] * face_sign(f) > 0.0)) continue;
                    int nb[3];
                    if (!neighbour(m, c, f, nb)) continue;
                    const int fp = f ^ 1; /* face of c' shared with c */
                    const double *mun = mu_dir + 8 * cell_index(m, nb);
                    for (int j = 0; j < 8; ++j) {
                        double v = 0.0;
                        for (int k = 0; k < 8; ++k) v += U[fp][k * 8 + j] * mun[k];
                        rhs[j] += v;
                    }
                }
                int rc = orc_ge_solve(8, At, rhs, mu_dir + 8 * ci);
                if (rc) return rc;
            }
        }
    }
    return ORC_OK;
}

/*
 * Adjoint of the source-iteration fixed point for a response J(phi):
 *   (L - K)^T lambda = W^T g,   lambda_d = w_d mu_d,
 *   L_d^T mu_d = g + sigma_s/(4 pi) M phi_dag,  phi_dag = sum_d w_d mu_d,
 * iterated (adjoint source iteration) until the max-norm relative change of
 * phi_dag is below tol, then contracted with the stored forward psi:
 *   dJ/dsigma_t[g][c] = - sum_d w_d mu_dc^T M psi_dc   (sigma_s held fixed)
 *   dJ/dq[g][c]       =   sum_d w_d mu_dc^T M 1
 *   dJ/dsigma_s[g][c] =   sum_d w_d mu_dc^T M phi_c / (4 pi)
 * g = dJ/dphi [G][ncell][8]; psi [D][G][ncell][8] and phi [G][ncell][8] are the
 * converged forward solution.  Direct partial derivatives of J are not added.
 */
/*
 * Adjoint scattering load: load = g + (1/4 pi) sum_{g'} sigma(g -> g') M phi_dag[g']
 * (the transpose of the forward group coupling; in-group only without a matrix).
 */
static void adjoint_load(int ng, long ncell, const double *sigma_s, const double *sigma_gg,
                         const double M[64], const double *gphi, const double *phid,
                         double *load)
{
    for (int g = 0; g < ng; ++g)
        for (long c = 0; c < ncell; ++c) {
            const long gc = (long)g * ncell + c;
            for (int k = 0; k < 8; ++k) {
                double acc = gphi[gc * 8 + k];
                for (int g2 = 0; g2 < ng; ++g2) {
                    const double sig = sigma_gg ? sigma_gg[((long)g * ng + g2) * ncell + c]
                                                : (g2 == g ? sigma_s[gc] : 0.0);
                    if (sig == 0.0) continue;
                    const long g2c = (long)g2 * ncell + c;
                    double v = 0.0;
                    for (int j = 0; j < 8; ++j) v += M[k * 8 + j] * phid[g2c * 8 + j];
                    acc += sig / (4.0 * ORC_PI) * v;
                }
                load[gc * 8 + k] = acc;
            }
        }
}

/*
 * The anisotropic part of the adjoint load for direction d of group g (the
 * transpose of the forward moment coupling):
 *   lu[c] = load[g][c] + sum_{g'} sum_{k>=1} sigma_{s,n(k)}(g->g')[c]
 *           Y_k(Omega_d) M phid_k[g'][c],
 * over g' = g only (in-group, sigma_sn [L][G][ncell]) or every group
 * (gg != 0, sigma_sn [L][G][G][ncell] with g -> g' at [n-1][g][g']), with
 * mmom[k-1][g'][c] = M phid_k[g'][c] precomputed.
 */
static void adjoint_load_pl(long ncell, int ng, int g, int L, const double *sigma_sn, int gg,
                            const double *yd, const double *load, const double *mmom, long nv,
                            double *lu)
{
    for (long c = 0; c < ncell; ++c) {
        const long gc = (long)g * ncell + c;
        for (int n = 0; n < 8; ++n) {
            double v = load[gc * 8 + n];
            for (int g2 = gg ? 0 : g; g2 <= (gg ? ng - 1 : g); ++g2) {
                const long g2c = (long)g2 * ncell + c;
                for (int o = 1; o <= L; ++o) {
                    const double sig = gg ? sigma_sn[(((long)(o - 1) * ng + g) * ng + g2) * ncell + c]
                                          : sigma_sn[(long)(o - 1) * nv + gc];
                    for (int mm = -o; mm <= o; ++mm) {
                        const int k = o * o + o + mm;
                        v += sig * yd[k] * mmom[((long)(k - 1) * nv + g2c) * 8 + n];
                    }
                }
            }
            lu[c * 8 + n] = v;
        }
    }
}

/* one adjoint sweep of every (direction, group): mu = (A^T)^-1 load_d */
static int adjoint_sweep_all(const orc_mesh *m, int ng, int nd, const double *omega,
                             const double *sigma_t, const double *load, const double M[64],
                             const double G[3][64], const double Mf[6][64], int L,
                             const double *sigma_sn, int gg, const double *Y, const double *mmom,
                             double *ubuf, double *mu)
{
    const long ncell = (long)m->n[0] * m->n[1] * m->n[2];
    const long nv = (long)ng * ncell;
    const int nm = (L + 1) * (L + 1);
    int rc = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (long u = 0; u < (long)nd * ng; ++u) {
        const int d = (int)(u / ng), g = (int)(u % ng);
        const double *ld = load + 8 * g * ncell;
        if (L > 0) {
#ifdef _OPENMP
            double *lu = ubuf + (long)omp_get_thread_num() * ncell * 8;
#else
            double *lu = ubuf;
#endif
            adjoint_load_pl(ncell, ng, g, L, sigma_sn, gg, Y + (long)d * nm, load, mmom, nv, lu);
            ld = lu;
        }
        int e = adjoint_sweep_one(m, omega + 3 * d, sigma_t + g * ncell, ld, M, G, Mf,
                                  mu + ((long)d * ng + g) * ncell * 8);
        if (e) {
#pragma omp critical
            rc = e;
        }
    }
    return rc;
}

/* mmom[k-1] = M phid_k with phid_k = sum_d w_d Y_k(Omega_d) mu_d */
static void adjoint_moments(int nd, long nv, int nm, const double *weight, const double *Y,
                            const double *mu, const double M[64], double *mmom)
{
#pragma omp parallel for schedule(static)
    for (long gc = 0; gc < nv; ++gc)
        for (int k = 1; k < nm; ++k) {
            double pk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int d = 0; d < nd; ++d)
                for (int n = 0; n < 8; ++n)
                    pk[n] += weight[d] * Y[(long)d * nm + k] * mu[((long)d * nv + gc) * 8 + n];
            for (int n = 0; n < 8; ++n) {
                double v = 0.0;
                for (int j = 0; j < 8; ++j) v += M[n * 8 + j] * pk[j];
                mmom[((long)(k - 1) * nv + gc) * 8 + n] = v;
            }
        }
}

static int adjoint_run(int nx, int ny, int nz, double lx, double ly, double lz, int ng, int nd,
                       const double *omega, const double *weight, const double *sigma_t,
                       const double *sigma_s, const double *sigma_gg, const double *psi,
                       const double *phi, const double *gphi, double tol, int max_iter,
                       double *grad_sigma_t, double *grad_q, double *grad_sigma_s,
                       double *phi_dag_out, int *iters, int nthreads, int L,
                       const double *sigma_sn, int pl_gg)
{
    orc_mesh m = {{nx, ny, nz}, {lx / nx, ly / ny, lz / nz}};
    const long ncell = (long)nx * ny * nz;
    const long nv = (long)ng * ncell;
    const int nm = (L + 1) * (L + 1);
    double M[64], G[3][64], Mf[6][64];
    orc_element_matrices(m.h, M, G, Mf);
    const int nt = set_threads(nthreads);
    double *phid = (double *)calloc((size_t)nv * 8, sizeof(double));
    double *phidn = (double *)malloc((size_t)nv * 8 * sizeof(double));
    double *load = (double *)malloc((size_t)nv * 8 * sizeof(double));
    double *mu = (double *)malloc((size_t)nd * nv * 8 * sizeof(double));
    double *Y = NULL, *mmom = NULL, *ubuf = NULL;
    if (L > 0) {
        Y = (double *)malloc((size_t)nd * nm * sizeof(double));
        mmom = (double *)calloc((size_t)(nm - 1) * nv * 8, sizeof(double));
        ubuf = (double *)malloc((size_t)nt * ncell * 8 * sizeof(double));
    }
    if (!phid || !phidn || !load || !mu || (L > 0 && (!Y || !mmom || !ubuf))) {
        free(phid); free(phidn); free(load); free(mu); free(Y); free(mmom); free(ubuf);
        return ORC_ENOMEM;
    }
    if (L > 0)
        for (int d = 0; d < nd; ++d) orc_real_ylm(L, omega + 3 * d, Y + (long)d * nm);
    int it = 0, rc = ORC_OK;
    double r = INFINITY;
    while (it < max_iter) {
        /* load = g + sigma_s^T/(4 pi) M phi_dag (+ the anisotropic moments) */
        adjoint_load(ng, ncell, sigma_s, sigma_gg, M, gphi, phid, load);
        rc = adjoint_sweep_all(&m, ng, nd, omega, sigma_t, load, M, G, Mf, L, sigma_sn, pl_gg, Y,
                               mmom, ubuf, mu);
        if (rc) break;
        if (L > 0) adjoint_moments(nd, nv, nm, weight, Y, mu, M, mmom);
        memset(phidn, 0, (size_t)nv * 8 * sizeof(double));
        for (int d = 0; d < nd; ++d)
            for (long i = 0; i < nv * 8; ++i) phidn[i] += weight[d] * mu[(long)d * nv * 8 + i];
        double dmax = 0.0, fmax = 0.0;
        for (long i = 0; i < nv * 8; ++i) {
            if (fabs(phidn[i] - phid[i]) > dmax) dmax = fabs(phidn[i] - phid[i]);
            if (fabs(phidn[i]) > fmax) fmax = fabs(phidn[i]);
        }
        memcpy(phid, phidn, (size_t)nv * 8 * sizeof(double));
        ++it;
        r = fmax > 0.0 ? dmax / fmax : 0.0;
        if (r < tol) break;
    }
    if (!rc) {
        /* the mu of the last sweep are consistent with the phi_dag used to build
           its load; one more sweep with the converged phi_dag refines them */
        adjoint_load(ng, ncell, sigma_s, sigma_gg, M, gphi, phid, load);
        rc = adjoint_sweep_all(&m, ng, nd, omega, sigma_t, load, M, G, Mf, L, sigma_sn, pl_gg, Y,
                               mmom, ubuf, mu);
    }
    if (!rc) {
        for (long gc = 0; gc < nv; ++gc) {
            double gs = 0.0, gq = 0.0, gss = 0.0;
            for (int d = 0; d < nd; ++d) {
                const double *md = mu + ((long)d * nv + gc) * 8;
                const double *pd = psi + ((long)d * nv + gc) * 8;
                for (int k = 0; k < 8; ++k)
                    for (int j = 0; j < 8; ++j) {
                        const double mk = weight[d] * md[k] * M[k * 8 + j];
                        gs -= mk * pd[j];
                        gq += mk;
                        gss += mk * phi[gc * 8 + j] / (4.0 * ORC_PI);
                    }
            }
            if (grad_sigma_t) grad_sigma_t[gc] = gs;
            if (grad_q) grad_q[gc] = gq;
            if (grad_sigma_s) grad_sigma_s[gc] = gss;
        }
        if (phi_dag_out) memcpy(phi_dag_out, phid, (size_t)nv * 8 * sizeof(double));
    }
    free(phid); free(phidn); free(load); free(mu); free(Y); free(mmom); free(ubuf);
    if (iters) *iters = it;
    if (rc) return rc;
    return (r < tol) ? ORC_OK : ORC_ENOTCONV;
}

int orc_adjoint(int nx, int ny, int nz, double lx, double ly, double lz, int ng, int nd,
                const double *omega, const double *weight, const double *sigma_t,
                const double *sigma_s, const double *psi, const double *phi,
                const double *gphi, double tol, int max_iter, double *grad_sigma_t,
                double *grad_q, double *grad_sigma_s, double *phi_dag_out, int *iters,
                int nthreads)
{
    return adjoint_run(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, sigma_s, NULL, psi,
                       phi, gphi, tol, max_iter, grad_sigma_t, grad_q, grad_sigma_s, phi_dag_out,
                       iters, nthreads, 0, NULL, 0);
}

/* Adjoint with multigroup scattering (the gradient with respect to the
   in-group sigma_s is not defined there and is not returned). */
int orc_adjoint_gg(int nx, int ny, int nz, double lx, double ly, double lz, int ng, int nd,
                   const double *omega, const double *weight, const double *sigma_t,
                   const double *sigma_gg, const double *psi, const double *phi,
                   const double *gphi, double tol, int max_iter, double *grad_sigma_t,
                   double *grad_q, double *phi_dag_out, int *iters, int nthreads)
{
    if (!sigma_gg) return ORC_EINVAL;
    return adjoint_run(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, NULL, sigma_gg,
                       psi, phi, gphi, tol, max_iter, grad_sigma_t, grad_q, NULL, phi_dag_out,
                       iters, nthreads, 0, NULL, 0);
}

/* Adjoint with in-group P_L scattering: sigma_sn [L+1][G][ncell], order 0
   first (the gradient with respect to the scattering moments is not
   returned). */
int orc_adjoint_pl(int nx, int ny, int nz, double lx, double ly, double lz, int ng, int nd,
                   const double *omega, const double *weight, const double *sigma_t, int L,
                   const double *sigma_sn, const double *psi, const double *phi,
                   const double *gphi, double tol, int max_iter, double *grad_sigma_t,
                   double *grad_q, double *phi_dag_out, int *iters, int nthreads)
{
    if (L < 1 || L > 8 || !sigma_sn) return ORC_EINVAL;
    const long nv = (long)ng * nx * ny * nz;
    return adjoint_run(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, sigma_sn, NULL,
                       psi, phi, gphi, tol, max_iter, grad_sigma_t, grad_q, NULL, phi_dag_out,
                       iters, nthreads, L, sigma_sn + nv, 0);
}

/* Adjoint with group-to-group P_L scattering: sigma_sn [L+1][G][G][ncell],
   from g' into g at [n][g'][g], order 0 first (the adjoint couples through
   the transpose of every order's matrix). */
int orc_adjoint_pl_gg(int nx, int ny, int nz, double lx, double ly, double lz, int ng, int nd,
                      const double *omega, const double *weight, const double *sigma_t, int L,
                      const double *sigma_sn, const double *psi, const double *phi,
                      const double *gphi, double tol, int max_iter, double *grad_sigma_t,
                      double *grad_q, double *phi_dag_out, int *iters, int nthreads)
{
    if (L < 1 || L > 8 || !sigma_sn) return ORC_EINVAL;
    const long ngg = (long)ng * ng * nx * ny * nz;
    return adjoint_run(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, NULL, sigma_sn,
                       psi, phi, gphi, tol, max_iter, grad_sigma_t, grad_q, NULL, phi_dag_out,
                       iters, nthreads, L, sigma_sn + ngg, 1);
}

/* ------------------------------------------------------------------ */
/* Per-cell particle balance                                            */
/* ------------------------------------------------------------------ */

/*
 * 1^T (A psi - b) for one cell system: by the partition of unity of the
 * basis, this is outflow - inflow + sigma_t int psi - int S, which vanishes
 * for the exact solution of the cell system.
 */
double orc_cell_balance(const double h[3], const double omega[3], double sigma_t,
                        const double S[8], const double psi_up[6][8], const double psi[8])
{
    double M[64], G[3][64], Mf[6][64], A[64], b[8];
    orc_element_matrices(h, M, G, Mf);
    orc_cell_matrix(omega, sigma_t, M, G, Mf, A);
    orc_cell_rhs(omega, M, Mf, S, psi_up, b);
    double s = 0.0;
    for (int k = 0; k < 8; ++k) {
        double v = -b[k];
        for (int j = 0; j < 8; ++j) v += A[k * 8 + j] * psi[j];
        s += v;
    }
    return s;
}

/*
 * Particle balance of a whole sweep, term by term, from the stored angular
 * flux psi [D][G][ncell][8] of that sweep (the same sigma_t, src and psi_inc).
 * For each direction d, group g and cell c, with the partition of unity of
 * the basis (sum_k b_k = 1), the integrals over a face f and over the cell
 * are 1^T Mf_f v and 1^T M v of the nodal vector v.  Summed with the weights
 * w_d:
 *   out[0]  outflow through every cell face with omega.n_f > 0:  (omega.n_f) int_f psi
 *   out[1]  inflow through every cell face with omega.n_f < 0:   |omega.n_f| int_f psi_up
 *           (psi_up the upwind neighbour's trace, psi_inc on the domain boundary)
 *   out[2]  out[0] restricted to faces on the domain boundary
 *   out[3]  out[1] restricted to faces on the domain boundary
 *   out[4]  absorption  sigma_t int_c psi
 *   out[5]  source      int_c S
 * For the exact cell solutions out[0] - out[1] + out[4] - out[5] = 0 (the
 * weak form tested with 1), and the interior faces cancel in out[0] - out[1]
 * (a downwind cell's inflow trace is its upwind neighbour's outflow), so
 * out[2] - out[3] = out[0] - out[1].
 */
int orc_sweep_balance(int nx, int ny, int nz, double lx, double ly, double lz, int ng, int nd,
                      const double *omega, const double *weight, const double *sigma_t,
                      const double *src, const double psi_inc[6], const double *psi,
                      double out[6])
{
    if (nx < 1 || ny < 1 || nz < 1 || ng < 1 || nd < 1) return ORC_EINVAL;
    orc_mesh m = {{nx, ny, nz}, {lx / nx, ly / ny, lz / nz}};
    const long ncell = (long)nx * ny * nz;
    double M[64], G[3][64], Mf[6][64];
    orc_element_matrices(m.h, M, G, Mf);
    for (int t = 0; t < 6; ++t) out[t] = 0.0;
    for (int d = 0; d < nd; ++d)
        for (int g = 0; g < ng; ++g) {
            const double *om = omega + 3 * d;
            const double *pd = psi + ((long)d * ng + g) * ncell * 8;
            int c[3];
            for (c[2] = 0; c[2] < nz; ++c[2])
                for (c[1] = 0; c[1] < ny; ++c[1])
                    for (c[0] = 0; c[0] < nx; ++c[0]) {
                        const long ci = cell_index(&m, c);
                        const double *pc = pd + 8 * ci;
                        const double *sc = src + ((long)g * ncell + ci) * 8;
                        double vol_psi = 0.0, vol_src = 0.0;
                        for (int k = 0; k < 8; ++k)
                            for (int j = 0; j < 8; ++j) {
                                vol_psi += M[k * 8 + j] * pc[j];
                                vol_src += M[k * 8 + j] * sc[j];
                            }
                        out[4] += weight[d] * sigma_t[(long)g * ncell + ci] * vol_psi;
                        out[5] += weight[d] * vol_src;
                        for (int f = 0; f < 6; ++f) {
                            const double on = om[f / 2] * face_sign(f);
                            if (on == 0.0) continue;
                            int nb[3];
                            const int boundary = !neighbour(&m, c, f, nb);
                            double v[8];
                            if (on > 0.0) memcpy(v, pc, sizeof(v));
                            else upwind_trace(&m, c, f, pd, psi_inc, v);
                            double face = 0.0;
                            for (int k = 0; k < 8; ++k)
                                for (int j = 0; j < 8; ++j) face += Mf[f][k * 8 + j] * v[j];
                            const double term = weight[d] * fabs(on) * face;
                            if (on > 0.0) {
                                out[0] += term;
                                if (boundary) out[2] += term;
                            } else {
                                out[1] += term;
                                if (boundary) out[3] += term;
                            }
                        }
                    }
        }
    return ORC_OK;
}

/* One-cell solve in physical orientation: assemble and GE. */
int orc_cell_solve(const double h[3], const double omega[3], double sigma_t, const double S[8],
                   const double psi_up[6][8], double psi[8])
{
    double M[64], G[3][64], Mf[6][64], A[64], b[8];
    orc_element_matrices(h, M, G, Mf);
    orc_cell_matrix(omega, sigma_t, M, G, Mf, A);
    orc_cell_rhs(omega, M, Mf, S, psi_up, b);
    return orc_ge_solve(8, A, b, psi);
}

/* Batched one-cell solves (training targets / local-solve parity). */
int orc_cell_solve_batch(long n, const double *h, const double *omega, const double *sigma_t,
                         const double *S, const double *psi_up, double *psi, int nthreads)
{
    set_threads(nthreads);
    int err = ORC_OK;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        int rc = orc_cell_solve(h + 3 * i, omega + 3 * i, sigma_t[i], S + 8 * i,
                                (const double(*)[8])(psi_up + 48 * i), psi + 8 * i);
        if (rc) {
#pragma omp critical
            err = rc;
        }
    }
    return err;
}

/* ------------------------------------------------------------------ */
/* Shallow-ANN local solver (Sec. 3, Eq. (ANN:Eq1))                     */
/* ------------------------------------------------------------------ */

/*
 * One hidden layer MLP, FP64 forward of the stored (float32) parameters:
 *   hidden = act(W1 x + b1), y = W2 hidden + b2       (Eq. (ANN:Eq1))
 * W1 is [nh][nin] row-major, W2 is [nout][nh].  act 0 = ReLU, 1 = tanh.
 */
struct orc_pann;
struct orc_ann {
    int nin, nh, nout, act;
    const double *W1, *b1, *W2, *b2;
    const struct orc_pann *paper;   /* not NULL: the paper-form networks below */
};

/*
 * Input vector of the reduced one-cell problem (Sec. 3: the cell is fully
 * determined by its inflow face values, direction, source nodes, sigma_t and
 * shape).  The cell is first reflected so that every direction component is
 * non-negative (canonical octant); canonical node n' is physical node
 * n' ^ mask, mask bit a set when omega_a < 0.  With h = (dx dy dz)^(1/3):
 *   x[0..2]   = |omega_a| h / dx_a          (streaming weights)
 *   x[3]      = sigma_t h                   (optical size)
 *   x[4..15]  = inflow face values / m: canonical x face (node order iy+2iz),
 *               y face (ix+2iz), z face (ix+2iy)
 *   x[16..23] = h S[n'] / m
 *   m = max(max|psi_in|, max|h S| / (x[3] + max_a x[a]))
 * The cell solution is linear in (psi_in, h S) at fixed (x[0..3]), so the net
 * predicts psi/m and the result is rescaled by m; m = 0 gives psi = 0.
 * Faces with omega_a = 0 carry no inflow and are fed as 0.
 */
int orc_ann_features(const double h[3], const double omega[3], double sigma_t, const double S[8],
                     const double psi_up[6][8], double x[24], double *scale)
{
    int mask = 0;
    for (int a = 0; a < 3; ++a)
        if (omega[a] < 0.0) mask |= 1 << a;
    const double hh = cbrt(h[0] * h[1] * h[2]);
    double kmax = 0.0;
    for (int a = 0; a < 3; ++a) {
        x[a] = fabs(omega[a]) * hh / h[a];
        if (x[a] > kmax) kmax = x[a];
    }
    x[3] = sigma_t * hh;
    double pmax = 0.0, smax = 0.0;
    for (int a = 0; a < 3; ++a) {
        const int f = 2 * a + ((mask >> a) & 1); /* physical inflow face */
        const int t1 = (a + 1) % 3 < (a + 2) % 3 ? (a + 1) % 3 : (a + 2) % 3;
        const int t2 = (a + 1) % 3 < (a + 2) % 3 ? (a + 2) % 3 : (a + 1) % 3;
        for (int fn = 0; fn < 4; ++fn) {
            const int np = ((fn & 1) << t1) | (((fn >> 1) & 1) << t2); /* canonical, bit a = 0 */
            const double v = omega[a] != 0.0 ? psi_up[f][np ^ mask] : 0.0;
            x[4 + 4 * a + fn] = v;
            if (fabs(v) > pmax) pmax = fabs(v);
        }
    }
    for (int np = 0; np < 8; ++np) {
        x[16 + np] = hh * S[np ^ mask];
        if (fabs(x[16 + np]) > smax) smax = fabs(x[16 + np]);
    }
    double m = pmax;
    const double den = x[3] + kmax;
    if (den > 0.0 && smax / den > m) m = smax / den;
    if (m > 0.0)
        for (int i = 4; i < 24; ++i) x[i] /= m;
    *scale = m;
    return mask;
}

void orc_ann_forward(int nin, int nh, int nout, int act, const double *W1, const double *b1,
                     const double *W2, const double *b2, const double *x, double *y)
{
    double hid[1024];
    for (int k = 0; k < nh; ++k) {
        double v = b1[k];
        for (int j = 0; j < nin; ++j) v += W1[k * nin + j] * x[j];
        hid[k] = act == 1 ? tanh(v) : (v > 0.0 ? v : 0.0);
    }
    for (int t = 0; t < nout; ++t) {
        double v = b2[t];
        for (int k = 0; k < nh; ++k) v += W2[t * nh + k] * hid[k];
        y[t] = v;
    }
}

/*
 * Paper-form network (Sec. 3 and the first paragraphs of Sec. 4), one per
 * octant, evaluated on the cell in its physical orientation.
 *   Input (26, in the order the paper lists them):
 *     I[0..3]   inflow values of the x face, I[4..7] of the y face, I[8..11]
 *               of the z face: the upwind traces at the cell's face nodes,
 *               face node index = lower tangential bit + 2 * higher one
 *               (a face with omega_a = 0 has no inflow and is fed as 0);
 *     I[12], I[13] = omega_x, omega_y (the two independent direction
 *               cosines; the octant fixes the sign of omega_z);
 *     I[14..21] = nodal source S[n] (external + scattering, per steradian);
 *     I[22]     = sigma_t;  I[23..25] = dx, dy, dz.
 *   Scaling, Eq. (ANN:Eq2): In_j = (I_j - alpha (Imin_j + Imax_j) / 2) /
 *               |Imax_j - Imin_j|, the norm read as the mean of the bounds.
 *   Hidden:     h = tanh(W1 In + b1)                       (Eq. (ANN:Eq1), (ANN:Eq3))
 *   Output:     z = W2 h + b2, psi_t = z_t if z_t >= 0, else beta (exp(z_t) - 1),
 *               beta = beta_scale * max_j I_j over the 12 inflow values (Eq. (ANN:Eq4)).
 * W1 [K][nh][26], b1 [K][nh], W2 [K][8][nh], b2 [K][8].  One network per
 * octant (ndir = 0, K = 8): the cell's net is its octant's, o = [omega_x < 0]
 * + 2 [omega_y < 0] + 4 [omega_z < 0].  One network per quadrature direction
 * (the reading of Sec. 4's training paragraph that trains an ANN for each
 * direction; ndir = K > 0): the net k whose stored direction dir_omega[k]
 * is the cell's direction (every component within 1e-6; the stored
 * directions are FP32).  Output psi[n] in physical node order.
 */
struct orc_pann {
    int nh;
    double alpha, beta_scale;
    const double *imin, *imax, *W1, *b1, *W2, *b2;
    int ndir;                  /* 0: per octant; else the number of per-direction nets */
    const double *dir_omega;   /* [ndir][3] */
};

int orc_pann_octant(const double omega[3])
{
    return (omega[0] < 0.0 ? 1 : 0) + (omega[1] < 0.0 ? 2 : 0) + (omega[2] < 0.0 ? 4 : 0);
}

void orc_pann_inputs(const double h[3], const double omega[3], double sigma_t, const double S[8],
                     const double psi_up[6][8], double I[26])
{
    for (int a = 0; a < 3; ++a) {
        const int side = omega[a] < 0.0 ? 1 : 0;   /* inflow through the low face if omega_a > 0 */
        const int f = 2 * a + side;
        const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
        for (int fn = 0; fn < 4; ++fn) {
            const int n = (side << a) | ((fn & 1) << t1) | (((fn >> 1) & 1) << t2);
            I[4 * a + fn] = omega[a] != 0.0 ? psi_up[f][n] : 0.0;
        }
    }
    I[12] = omega[0];
    I[13] = omega[1];
    for (int n = 0; n < 8; ++n) I[14 + n] = S[n];
    I[22] = sigma_t;
    for (int a = 0; a < 3; ++a) I[23 + a] = h[a];
}

/* Index of the net that serves direction omega (see above), -1 if none. */
static int pann_net_index(const struct orc_pann *p, const double omega[3])
{
    if (p->ndir == 0) return orc_pann_octant(omega);
    for (int k = 0; k < p->ndir; ++k) {
        const double *w = p->dir_omega + 3 * k;
        if (fabs(w[0] - omega[0]) <= 1e-6 && fabs(w[1] - omega[1]) <= 1e-6 &&
            fabs(w[2] - omega[2]) <= 1e-6)
            return k;
    }
    return -1;
}

/* Forward pass of net `index` (an octant, or a direction with ndir > 0). */
int orc_pann_forward(int nh, double alpha, double beta_scale, const double *imin,
                     const double *imax, const double *W1, const double *b1, const double *W2,
                     const double *b2, int ndir, const double *dir_omega, int index,
                     const double I[26], double psi[8])
{
    double In[26], hid[64];
    (void)dir_omega;
    if (nh < 1 || nh > 64 || ndir < 0 || index < 0 || index >= (ndir ? ndir : 8))
        return ORC_EINVAL;
    for (int j = 0; j < 26; ++j)
        In[j] = (I[j] - alpha * 0.5 * (imin[j] + imax[j])) / fabs(imax[j] - imin[j]);
    const double *w1 = W1 + (long)index * nh * 26, *c1 = b1 + (long)index * nh;
    const double *w2 = W2 + (long)index * 8 * nh, *c2 = b2 + (long)index * 8;
    for (int k = 0; k < nh; ++k) {
        double v = c1[k];
        for (int j = 0; j < 26; ++j) v += w1[k * 26 + j] * In[j];
        hid[k] = tanh(v);
    }
    double pmax = I[0];
    for (int j = 1; j < 12; ++j)
        if (I[j] > pmax) pmax = I[j];
    const double beta = beta_scale * pmax;
    for (int t = 0; t < 8; ++t) {
        double z = c2[t];
        for (int k = 0; k < nh; ++k) z += w2[t * nh + k] * hid[k];
        psi[t] = z >= 0.0 ? z : beta * (exp(z) - 1.0);
    }
    return ORC_OK;
}

static int pann_cell(const struct orc_pann *p, const double h[3], const double omega[3],
                     double sigma_t, const double S[8], const double psi_up[6][8], double psi[8])
{
    double I[26];
    const int k = pann_net_index(p, omega);
    if (k < 0) return ORC_EINVAL;   /* no network for this direction */
    orc_pann_inputs(h, omega, sigma_t, S, psi_up, I);
    return orc_pann_forward(p->nh, p->alpha, p->beta_scale, p->imin, p->imax, p->W1, p->b1, p->W2,
                            p->b2, p->ndir, p->dir_omega, k, I, psi);
}

static int ann_cell(const orc_ann *net, const double h[3], const double omega[3], double sigma_t,
                    const double S[8], const double psi_up[6][8], double psi[8])
{
    if (net->paper) return pann_cell(net->paper, h, omega, sigma_t, S, psi_up, psi);
    double x[24], y[8], m;
    const int mask = orc_ann_features(h, omega, sigma_t, S, psi_up, x, &m);
    if (m == 0.0) {
        for (int n = 0; n < 8; ++n) psi[n] = 0.0;
        return ORC_OK;
    }
    orc_ann_forward(net->nin, net->nh, net->nout, net->act, net->W1, net->b1, net->W2, net->b2, x,
                    y);
    for (int np = 0; np < 8; ++np) psi[np ^ mask] = m * y[np];
    return ORC_OK;
}

/* Batched ANN one-cell solves in physical orientation. */
int orc_ann_cell_batch(long n, const double *h, const double *omega, const double *sigma_t,
                       const double *S, const double *psi_up, int nh, int act, const double *W1,
                       const double *b1, const double *W2, const double *b2, double *psi)
{
    orc_ann net = {24, nh, 8, act, W1, b1, W2, b2, NULL};
    if (nh < 1 || nh > 1024) return ORC_EINVAL;
    for (long i = 0; i < n; ++i)
        ann_cell(&net, h + 3 * i, omega + 3 * i, sigma_t[i], S + 8 * i,
                 (const double(*)[8])(psi_up + 48 * i), psi + 8 * i);
    return ORC_OK;
}

/* Sweep / source iteration with the ANN replacing assembly + GE (Sec. 4 intro). */
int orc_ann_sweep(int nx, int ny, int nz, double lx, double ly, double lz, int ng, int nd,
                  const double *omega, const double *weight, const double *sigma_t,
                  const double *src, const double psi_inc[6], int nh, int act, const double *W1,
                  const double *b1, const double *W2, const double *b2, double *phi,
                  int nthreads)
{
    orc_ann net = {24, nh, 8, act, W1, b1, W2, b2, NULL};
    if (nh < 1 || nh > 1024) return ORC_EINVAL;
    return sweep_all(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, src, psi_inc, phi,
                     NULL, &net, nthreads);
}

int orc_ann_source_iterate(int nx, int ny, int nz, double lx, double ly, double lz, int ng,
                           int nd, const double *omega, const double *weight,
                           const double *sigma_t, const double *sigma_s, const double *q,
                           const double psi_inc[6], int nh, int act, const double *W1,
                           const double *b1, const double *W2, const double *b2, double *phi,
                           double tol, int max_iter, int *iters, double *resid, double *eps_s,
                           int nthreads)
{
    orc_ann net = {24, nh, 8, act, W1, b1, W2, b2, NULL};
    if (nh < 1 || nh > 1024) return ORC_EINVAL;
    return source_iterate(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, sigma_s, q,
                          psi_inc, phi, tol, max_iter, iters, resid, eps_s, NULL, &net, nthreads,
                          NULL, 0);
}

/* Batched paper-form network one-cell solves (physical orientation). */
int orc_pann_cell_batch(long n, const double *h, const double *omega, const double *sigma_t,
                        const double *S, const double *psi_up, int nh, double alpha,
                        double beta_scale, const double *imin, const double *imax,
                        const double *W1, const double *b1, const double *W2, const double *b2,
                        int ndir, const double *dir_omega, double *psi)
{
    const struct orc_pann p = {nh, alpha, beta_scale, imin, imax, W1, b1, W2, b2, ndir,
                               dir_omega};
    if (nh < 1 || nh > 64 || ndir < 0) return ORC_EINVAL;
    for (long i = 0; i < n; ++i) {
        const int rc = pann_cell(&p, h + 3 * i, omega + 3 * i, sigma_t[i], S + 8 * i,
                                 (const double(*)[8])(psi_up + 48 * i), psi + 8 * i);
        if (rc) return rc;
    }
    return ORC_OK;
}

/* Sweep / source iteration with the paper-form network in place of assembly + GE. */
int orc_pann_sweep(int nx, int ny, int nz, double lx, double ly, double lz, int ng, int nd,
                   const double *omega, const double *weight, const double *sigma_t,
                   const double *src, const double psi_inc[6], int nh, double alpha,
                   double beta_scale, const double *imin, const double *imax, const double *W1,
                   const double *b1, const double *W2, const double *b2, int ndir,
                   const double *dir_omega, double *phi, double *psi_store, int nthreads)
{
    const struct orc_pann p = {nh, alpha, beta_scale, imin, imax, W1, b1, W2, b2, ndir,
                               dir_omega};
    orc_ann net = {26, nh, 8, 1, NULL, NULL, NULL, NULL, &p};
    if (nh < 1 || nh > 64 || ndir < 0) return ORC_EINVAL;
    return sweep_all(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, src, psi_inc, phi,
                     psi_store, &net, nthreads);
}

int orc_pann_source_iterate(int nx, int ny, int nz, double lx, double ly, double lz, int ng,
                            int nd, const double *omega, const double *weight,
                            const double *sigma_t, const double *sigma_s, const double *q,
                            const double psi_inc[6], int nh, double alpha, double beta_scale,
                            const double *imin, const double *imax, const double *W1,
                            const double *b1, const double *W2, const double *b2, int ndir,
                            const double *dir_omega, double *phi, double tol, int max_iter,
                            int *iters, double *resid, double *eps_s, int nthreads)
{
    const struct orc_pann p = {nh, alpha, beta_scale, imin, imax, W1, b1, W2, b2, ndir,
                               dir_omega};
    orc_ann net = {26, nh, 8, 1, NULL, NULL, NULL, NULL, &p};
    if (nh < 1 || nh > 64 || ndir < 0) return ORC_EINVAL;
    return source_iterate(nx, ny, nz, lx, ly, lz, ng, nd, omega, weight, sigma_t, sigma_s, q,
                          psi_inc, phi, tol, max_iter, iters, resid, eps_s, NULL, &net, nthreads,
                          NULL, 0);
}
