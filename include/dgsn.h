/*
 * dgsn.h -- C ABI of libdgsn, an MI355X (gfx950) implementation of the
 * trilinear-hexahedron DGFEM S_n transport sweep with Gaussian-elimination
 * and shallow-ANN local solvers (Tano & Ragusa, arXiv 1906.04017).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Mesh: nx*ny*nz uniform hexahedra on [0,lx]x[0,ly]x[0,lz]; cell index
 *   c = i + nx*(j + ny*k).
 * Local node n = ix + 2*iy + 4*iz (ix,iy,iz in {0,1}) is the cell vertex at
 *   (ix*dx, iy*dy, iz*dz) (trial space of Sec. 2, Eq. (T9), trilinear).
 * Domain faces: 0 = x-, 1 = x+, 2 = y-, 3 = y+, 4 = z-, 5 = z+.
 * Per-cell fields are [G][nz][ny][nx]; nodal fields are [G][nz][ny][nx][8]
 *   (node fastest).  Device arrays are in the problem precision
 *   (float for DGSN_FP32, double for DGSN_FP64) unless stated otherwise.
 * Sources are per steradian: the total nodal source of a sweep is
 *   S = q + sigma_s/(4 pi) * phi  (isotropic in-group scattering, the P0 term
 *   of Eq. (T5)); phi = sum_d w_d psi_d (Eq. (T8)/(T11)) with sum_d w_d = 4 pi.
 *
 * Ownership: the caller owns every pointer it passes.  Device pointers must
 * stay valid until the work enqueued on the given stream has completed.  The
 * library owns everything behind its opaque handles and keeps no user pointer
 * after a call returns.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * Device work is enqueued asynchronously on it; calls that return host
 * scalars (iteration counts, residuals, latencies) synchronize that stream.
 * A problem handle must be used from one stream at a time.
 *
 * Errors: every call returns DGSN_OK (0) or a negative DGSN_E* code and sets a
 * thread-local message readable with dgsn_last_error().  Arguments are
 * validated on the host before any device work is enqueued.
 */
#ifndef DGSN_H
#define DGSN_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgsn_ctx dgsn_ctx;
typedef struct dgsn_problem dgsn_problem;
typedef struct dgsn_ann dgsn_ann;
typedef struct dgsn_batch dgsn_batch;

enum {
    DGSN_OK = 0,
    DGSN_EINVAL = -1,        /* invalid argument */
    DGSN_ENOMEM = -2,        /* host or device allocation failed (for tests, device
                                allocations above DGSN_TEST_ALLOC_LIMIT bytes, an
                                environment variable read at each allocation, fail
                                with this code) */
    DGSN_EHIP = -3,          /* a HIP runtime call failed */
    DGSN_ENOTCONV = -4,      /* iteration limit reached; outputs hold the last iterate */
    DGSN_EFORMAT = -5,       /* malformed ANN artifact */
    DGSN_EUNSUPPORTED = -6,  /* valid request outside what the library supports */
    DGSN_ETIMEOUT = -7       /* a bounded device-side wait expired */
};

enum { DGSN_FP32 = 0, DGSN_FP64 = 1 };

/*
 * Local solvers of the cell system (Eq. (T12)):
 *   DGSN_GE        Gaussian elimination (partial pivoting) of the cell system
 *                  premultiplied by the inverse element mass matrix, known in
 *                  closed form; the matrix has 32 structural zeros, which the
 *                  elimination skips.  Same solution, about half the flops.
 *   DGSN_ANN       the shallow network of Sec. 3 in place of assembly + GE:
 *                  with a version-1 artifact the 24-input canonical network on
 *                  the BF16 matrix cores, with a version-2 artifact the
 *                  paper-form per-octant networks (26 inputs, tanh hidden
 *                  layer, ELU output) on the vector ALUs, with a version-3
 *                  artifact the paper-form networks of each quadrature
 *                  direction (same form, one per direction).
 *   DGSN_GE_DENSE  the cell matrix and right-hand side assembled as in Sec. 2
 *                  (streaming, sigma_t times mass, upwind face terms) and
 *                  solved by dense Gaussian elimination.
 */
enum { DGSN_GE = 0, DGSN_ANN = 1, DGSN_GE_DENSE = 2 };

/* Library version as major*10000 + minor*100 + patch. */
int dgsn_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char *dgsn_last_error(void);

/* Bind a HIP device.  out receives a context handle. */
int dgsn_ctx_create(int hip_device, dgsn_ctx **out);
int dgsn_ctx_destroy(dgsn_ctx *ctx);

/*
 * Level-symmetric LQ_N quadrature (the S_N discretisation of Sec. 2,
 * Eq. (T7)-(T8); the paper does not name the family, LQ_N is the standard set
 * of the transport text it cites).  Host only, no device needed.
 * order: even, 2..12.  omega: host [n][3] out, weight: host [n] out with
 * sum = 4 pi.  *n_inout: capacity on entry (>= order*(order+2)), count on
 * exit.  Directions are octant-major (octant o = [Ox<0] + 2[Oy<0] + 4[Oz<0]).
 * Passing omega = weight = NULL only returns the count.
 */
int dgsn_quadrature_ls(int order, double *omega, double *weight, int *n_inout);

typedef struct {
    int nx, ny, nz;          /* cells per axis, >= 1, <= 1024 */
    double lx, ly, lz;       /* domain lengths, > 0 */
    int n_groups;            /* independent groups (in-group scattering), >= 1 */
    int n_dirs;              /* directions; every octant must hold n_dirs/8 */
    const double *omega;     /* host [n_dirs][3], unit vectors (|1 - |O|| <= 1e-12) */
    const double *weight;    /* host [n_dirs], > 0, sum 4 pi (+-1e-10) */
    int precision;           /* DGSN_FP32 or DGSN_FP64 */
    int solver;              /* DGSN_GE, DGSN_GE_DENSE or DGSN_ANN (ANN: FP32 only) */
    int store_psi;           /* keep the last sweep's angular flux (adjoint) */
} dgsn_problem_desc;

/* Host-side validation of a descriptor (no device work).  DGSN_OK or EINVAL. */
int dgsn_problem_validate(const dgsn_problem_desc *desc);

/*
 * Create a problem on ctx: validates desc, allocates device buffers
 * (materials, sources, scalar flux, per-octant partials, face fronts, the
 * hyperplane schedule and the direction tables).  Materials default to zero,
 * inflow to vacuum.
 */
int dgsn_problem_create(dgsn_ctx *ctx, const dgsn_problem_desc *desc, dgsn_problem **out);
int dgsn_problem_destroy(dgsn_problem *p);

/*
 * Copy materials (device arrays [G][nz][ny][nx], problem precision) into the
 * problem: total cross section sigma_t >= 0, isotropic in-group scattering
 * cross section sigma_s >= 0 (sigma_s may be NULL = 0), external source q per
 * steradian (NULL = 0).  Enqueued on stream, then checked on the device (the
 * call waits for the stream): DGSN_EINVAL, naming the offending array, if a
 * sigma_t or sigma_s value is negative or not finite, a q value is not
 * finite, or a cell's sigma_s exceeds its sigma_t; the copies are kept, and
 * the problem must get valid materials before it is swept.  Table P1-P4 of Sec. 4 give the paper's values.
 */
int dgsn_problem_set_materials(dgsn_problem *p, const void *sigma_t, const void *sigma_s,
                               const void *q, void *stream);

/*
 * Multigroup isotropic scattering (the group sum of the scattering source,
 * Eq. (T3)-(T8), at order P0): sigma_gg is a device array [G][G][Nz*Ny*Nx]
 * in the problem precision, sigma_gg[g'][g][c] the cross section for
 * scattering from group g' into group g in cell c.  Source iteration then
 * uses S_g = q_g + (1/4pi) sum_{g'} sigma_gg[g'][g] phi_g' (all groups at
 * once, Jacobi in the group index), and the adjoint the transposed coupling;
 * the in-group sigma_s of dgsn_problem_set_materials is not used while a
 * matrix is set.  The array is copied (asynchronously on the stream); the
 * caller keeps ownership of its pointer.  NULL removes the matrix
 * (DGSN_EUNSUPPORTED while group-to-group anisotropic orders are set: their
 * order-0 matrix goes with them, see dgsn_problem_set_anisotropy_gg).  Single
 * sweeps (dgsn_sweep, batches) take the caller's source and are unaffected.
 * DGSN_ENOMEM if the copy cannot be allocated.
 */
int dgsn_problem_set_scattering(dgsn_problem *p, const void *sigma_gg, void *stream);

/*
 * Anisotropic in-group scattering of order L (Eq. (T3)-(T8)): the scattering
 * kernel sum_{n<=L} (2n+1)/(4 pi) sigma_{s,n} P_n(Omega'.Omega), expanded in
 * real orthonormal spherical harmonics Y_k, k = n^2 + n + m (dgsn_real_ylm).
 * Source iteration then uses for direction d
 *   Q_d = q + sigma_s/(4 pi) phi + sum_{k>=1} sigma_{s,n(k)} Y_k(Omega_d) phi_k,
 *   phi_k = sum_d w_d Y_k(Omega_d) psi_d,
 * with sigma_s (order 0) from dgsn_problem_set_materials.  order: 0..3 (0
 * removes the anisotropic orders and frees their buffers).  sigma_sn: device
 * [order][G][Nz*Ny*Nx] in the problem precision, orders 1..order (copied
 * asynchronously on the stream; the caller keeps ownership).  The moments
 * start from zero in every dgsn_source_iterate call (a resumed run restarts
 * them).  Its sweeps use the problem's schedule and tile edge, at most 2
 * (larger tiles would spill registers).  dgsn_adjoint_solve takes the
 * transposed coupling (the same moment form, with the adjoint flux's
 * moments); it and a stored angular flux need the mass-inverse solver
 * DGSN_GE.  Single sweeps (dgsn_sweep, batches) and the autotuner take
 * isotropic sources only: dgsn_source_iterate with a network solver, and
 * with store_psi under DGSN_GE_DENSE, returns DGSN_EUNSUPPORTED while an
 * order is set, and so does this call while a group-to-group matrix
 * is set (and dgsn_problem_set_scattering while an order is set; see
 * dgsn_problem_set_anisotropy_gg for both).
 * DGSN_ENOMEM if the moment buffers (10 ((L+1)^2 - 1) G*cells*8 reals) cannot be
 * allocated; a call that fails after its checks leaves the problem with no
 * anisotropic orders.
 */
int dgsn_problem_set_anisotropy(dgsn_problem *p, int order, const void *sigma_sn, void *stream);

/*
 * Anisotropic scattering of order L with a group-to-group matrix per
 * Legendre order (the group sum of Eq. (T3)-(T8)): source iteration uses for
 * direction d of group g
 *   Q_{d,g} = q_g + sum_{g'} ( sigma_{s,0}(g'->g)/(4 pi) phi_{g'}
 *             + sum_{k>=1} sigma_{s,n(k)}(g'->g) Y_k(Omega_d) phi_{k,g'} ),
 * all groups at once (Jacobi in the group index), and dgsn_adjoint_solve the
 * transpose of every order's matrix.  order: 1..3.  sigma_sn_gg: device
 * [order+1][G][G][Nz*Ny*Nx] in the problem precision, order 0 first,
 * sigma_sn_gg[n][g'][g][c] the moment of order n for scattering from group
 * g' into group g in cell c (copied asynchronously on the stream; the caller
 * keeps ownership).  The order-0 slice becomes the problem's multigroup
 * matrix (as with dgsn_problem_set_scattering), so the in-group sigma_s of
 * dgsn_problem_set_materials is not used.  This call replaces any in-group
 * orders or group-to-group matrix set before; dgsn_problem_set_anisotropy
 * with order 0 removes the orders 1..L and keeps the order-0 matrix.  The
 * other rules are those of dgsn_problem_set_anisotropy (tile edge at most
 * 2; GE solvers; the adjoint and a stored angular flux with DGSN_GE).
 * DGSN_EINVAL for an order outside 1..3 or a NULL array; DGSN_ENOMEM if the
 * buffers (the moment buffers and (L+1) G*G*cells reals) cannot be allocated.
 * A call that fails after its checks leaves the problem with no anisotropic
 * orders and no group-to-group matrix (in-group isotropic scattering).
 */
int dgsn_problem_set_anisotropy_gg(dgsn_problem *p, int order, const void *sigma_sn_gg,
                                   void *stream);

/*
 * Flux moments phi_k, k = 1 .. (L+1)^2 - 1, of the final sweep of the last
 * source iteration (Eq. (T8) for n >= 1), or of the adjoint flux after a
 * dgsn_adjoint_solve: mom is a device array
 * [(L+1)^2 - 1][G][Nz*Ny*Nx][8] in the problem precision (copied on the
 * stream).  DGSN_EINVAL without anisotropic scattering.
 */
int dgsn_problem_get_moments(const dgsn_problem *p, void *mom, void *stream);

/*
 * Real orthonormal spherical harmonics of the scattering expansion (the Y of
 * Eq. (T4), real form), host only: Y[i][k], k = n^2 + n + m for n <= order
 * (order 0..3) and m = -n..n, at the unit directions omega[i] (host [n][3]).
 * Polar axis z, no (-1)^m phase: Y_{1,-1}, Y_{1,0}, Y_{1,1} = sqrt(3/(4 pi))
 * (y, z, x); m < 0 are the sine-type harmonics.
 */
int dgsn_real_ylm(int order, const double *omega, int n, double *Y);

/* Boundary inflow psi_inc per domain face (host [6]); applied to every
   direction entering through that face (Eq. (TBC)); 0 = vacuum. */
int dgsn_problem_set_inflow(dgsn_problem *p, const double psi_inc[6]);

/* Attach an ANN (required before sweeping with solver = DGSN_ANN).  The
   problem keeps a reference; the ANN must outlive its use by the problem.
   A paper-form (version-2 or -3) network is folded for this problem's cell
   sizes here (a small device buffer owned by the problem; DGSN_ENOMEM if it
   cannot be allocated, and then no network is attached).  With a version-3
   artifact each direction of the problem takes the network whose stored
   direction equals it (every cosine within 1e-6); DGSN_EINVAL, with the
   previous network left attached, if some direction has none, and
   DGSN_EUNSUPPORTED for more than 59 directions per octant (a sweep block
   holds its octant's networks in LDS). */
int dgsn_problem_set_ann(dgsn_problem *p, const dgsn_ann *ann);

/* Select the local solver of subsequent sweeps (DGSN_GE, DGSN_GE_DENSE or
   DGSN_ANN). */
int dgsn_problem_set_solver(dgsn_problem *p, int solver);

/*
 * One transport sweep (Sec. 2, the sweep paragraph after Eq. (T12)): for
 * every direction and group solve the per-cell systems A psi_d = b of
 * Eq. (T12) in dependency order, cells of one hyperplane in parallel, and
 * return phi = sum_d w_d psi_d.
 * src: device [G][nz][ny][nx][8] total nodal source per steradian.
 * phi: device [G][nz][ny][nx][8] out.  src and phi must not overlap.
 */
int dgsn_sweep(dgsn_problem *p, const void *src, void *phi, void *stream);

/*
 * Scattering source iteration (Sec. 2, the paragraph after Eq. (T6)):
 * repeat S = q + sigma_s/(4 pi) phi, sweep, until the max-norm relative change
 * max|phi_new - phi_old| / max|phi_new| (computed in FP64) is below tol.
 * phi: device [G][nz][ny][nx][8]; initial guess on entry, last iterate on
 * exit (a saved phi resumes an interrupted run).  max_iter >= 1.
 * FP32 problems also stop when the residual has not decreased for 5
 * iterations (the FP32 noise floor) and then return DGSN_ENOTCONV unless
 * resid < tol.  iters, resid, eps_s (host out, may be NULL): iterations done,
 * last residual, and the paper's mean pointwise criterion Eq. (Test:Eq3) on
 * cell averages.  Synchronizes stream.  An iterate holding a NaN or an
 * infinity returns DGSN_EINVAL (the FP64 maxima of the residual carry NaNs
 * to the host).
 */
int dgsn_source_iterate(dgsn_problem *p, void *phi, double tol, int max_iter, int *iters,
                        double *resid, double *eps_s, void *stream);

/*
 * dgsn_source_iterate for callers that cannot allocate memory (code under
 * HIP graph capture elsewhere in the program, tight serving loops, harnesses
 * that forbid hipMalloc): the same iteration with the same kernels and
 * bitwise the same results, but its reduction partials, result slots and
 * look-ahead iterate live in a static device array of the library
 * (64 MiB + 128.25 KiB, one copy per device, held until the process ends)
 * instead of memory the library allocates.  The call itself makes no
 * device or host allocation.  Limits and rules:
 *   - G * cells * 8 reals of the iterate must fit 64 MiB (e.g. 64^3 cells x
 *     8 groups in FP32) when the iteration overlaps (no stored angular flux,
 *     no anisotropic orders); a larger iterate returns DGSN_EINVAL;
 *   - kernel timing must be off (its events may need creating), and a
 *     dataflow schedule must have its tables (dgsn_problem_set_schedule or
 *     dgsn_problem_autotune builds them): DGSN_EINVAL otherwise;
 *   - the convergence history keeps the first 4096 iterations;
 *   - every call on a device shares that device's array and leaves its last
 *     contents there (nothing in it needs to start at zero): calls that
 *     overlap in time on one device race and must be serialised by the
 *     caller (the same stream, or one thread).
 * Arguments, results and errors otherwise as dgsn_source_iterate.
 */
int dgsn_source_iterate_noalloc(dgsn_problem *p, void *phi, double tol, int max_iter,
                                int *iters, double *resid, double *eps_s, void *stream);

/*
 * Convergence history of the problem's last dgsn_source_iterate call: the
 * residual (the max-norm relative change above) and eps_S of Eq. (Test:Eq3)
 * after each of its iterations, the quantities from which the effective
 * spectral radius of the iteration (Sec. 4, the discussion of Problem 4) is
 * read as the ratio of successive residuals.  resid, eps_s: host arrays of cap
 * entries (either may be NULL); the first min(cap, n) entries are written.
 * n (host out): iterations recorded (0 before the first call).  A failed call
 * records the iterations it completed.
 */
int dgsn_problem_si_history(const dgsn_problem *p, double *resid, double *eps_s, int cap, int *n);

/*
 * Sweep tiling: with b > 1 every lane solves a b x b x b tile of cells for
 * its (direction, group) in upwind order, keeping the faces between them in
 * registers (the face traffic through HBM drops from 24 to 24/b values per
 * solve), one launch per tile hyperplane; with b = 1 every lane solves one
 * cell per hyperplane launch.  b in 1..3; default 2.  dgsn_problem_set_tile /
 * _get_tile set and read it.
 */
int dgsn_problem_set_tile(dgsn_problem *p, int b);
int dgsn_problem_get_tile(const dgsn_problem *p, int *b);

/*
 * Sweep schedule (every local solver).  The sweep order follows from the
 * upwind dependence of each cell on its three inflow neighbours (the sweep
 * paragraph after Eq. (T12)).
 *   DGSN_SCHED_PLANES: one kernel launch per (tile) hyperplane (default).
 *   DGSN_SCHED_DATAFLOW: one launch per sweep; the workgroups of an octant
 *     take blocks of tiles in hyperplane order from that octant's device
 *     ticket counter and wait on the done flags of the blocks of the previous
 *     hyperplane that hold their tiles' upwind neighbours.  Every wait is
 *     bounded by poll_limit polls (0: the library default, about a second);
 *     if one expires the launch still completes, its results are invalid,
 *     and the next dgsn_problem_check (also run inside dgsn_source_iterate,
 *     dgsn_adjoint_solve and the autotuner) returns DGSN_ETIMEOUT and clears
 *     the condition.  Two dataflow sweeps of one problem
 *     must not run concurrently (they share the counters).
 * dgsn_problem_check: synchronizes stream and reports an expired dataflow
 *   wait since the last check.
 */
enum { DGSN_SCHED_PLANES = 0, DGSN_SCHED_DATAFLOW = 1 };
int dgsn_problem_set_schedule(dgsn_problem *p, int schedule, unsigned poll_limit);
int dgsn_problem_get_schedule(const dgsn_problem *p, int *schedule);
int dgsn_problem_check(dgsn_problem *p, void *stream);

/*
 * Debug modes (not in the paper), flags OR-ed together (0 = none):
 *   DGSN_DEBUG_POISON_FRONTS  every sweep of the problem first fills its face
 *     fronts with NaN (a fill kernel on the sweep's stream).  A correct sweep
 *     reads a front slot only after the upstream cell wrote it in the same
 *     sweep, so its results are unchanged; a read out of order (a missing
 *     dataflow wait, a wrong index) yields NaN, which source iteration reports
 *     as DGSN_EINVAL.  Single-problem sweeps only (batches ignore it).
 * DGSN_EINVAL for unknown flags.
 */
enum { DGSN_DEBUG_POISON_FRONTS = 1 };
int dgsn_problem_set_debug(dgsn_problem *p, int flags);

/*
 * Autotuner: times one sweep of the problem with each tile edge 1..3 and each
 * schedule (on its internal buffers; user arrays are not touched), keeps the
 * fastest, and returns the choice and the times in ms (ms: host [6], entry
 * schedule * 3 + edge - 1, INFINITY where not applicable; tile, schedule, ms
 * may be NULL).  Synchronizes stream.  The choice is cached for the process
 * under the problem's shape (device architecture and compute units, mesh,
 * directions per octant, groups, precision, solver and network form,
 * anisotropic order, psi store): a later call for a problem of the same
 * shape applies the cached tile and schedule without timing and returns the
 * cached times.  Not in the paper.
 */
int dgsn_problem_autotune(dgsn_problem *p, void *stream, int *tile, int *schedule, double *ms);

/*
 * The autotuner cache (host only, no device work): _clear empties it, _size
 * counts its entries, _save writes it to path as JSON (one entry per line:
 * key, tile, schedule, the six times, -1 for INFINITY), _load merges a file
 * written by _save (entries of the file replace those of the same key).
 * DGSN_EINVAL for a NULL or unopenable path, DGSN_EFORMAT for a file that is
 * not such a cache (the cache is then unchanged).
 */
int dgsn_autotune_cache_clear(void);
int dgsn_autotune_cache_size(int *n);
int dgsn_autotune_cache_save(const char *path);
int dgsn_autotune_cache_load(const char *path);

/*
 * Stopping criterion of dgsn_source_iterate: DGSN_SI_MAXNORM (default) uses
 * the FP64 max-norm relative change; DGSN_SI_EPS_S uses the paper's mean
 * pointwise relative change of the cell-average scalar flux, Eq. (Test:Eq3);
 * DGSN_SI_FIXED runs exactly max_iter iterations (tol and the FP32 stall
 * stop are not applied; the residuals are still recorded) and returns
 * DGSN_OK.
 */
enum { DGSN_SI_MAXNORM = 0, DGSN_SI_EPS_S = 1, DGSN_SI_FIXED = 2 };
int dgsn_problem_set_si_criterion(dgsn_problem *p, int criterion);

/*
 * Gradient of a scalar response J(phi) through the converged source
 * iteration by the discrete adjoint (not in the paper).  Requires a problem
 * created with store_psi = 1 whose last source iteration ran after its last
 * setter call and sweep (DGSN_EINVAL otherwise: the stored angular flux
 * would not belong to the current inputs).
 * dJ_dphi: device [G][nz][ny][nx][8].  grad_sigma_t, grad_q: device
 * [G][nz][ny][nx] out (may be NULL): dJ/dsigma_t at fixed sigma_s and dJ/dq,
 * without any direct partial derivative of J.  The adjoint iteration stops at
 * relative change < tol or max_iter (DGSN_ENOTCONV).  iters may be NULL.
 * Synchronizes stream.  A NaN or infinite adjoint flux returns DGSN_EINVAL.
 */
int dgsn_adjoint_solve(dgsn_problem *p, const void *dJ_dphi, void *grad_sigma_t, void *grad_q,
                       double tol, int max_iter, int *iters, void *stream);

/*
 * Batched one-cell GE solves of the canonical cell system (Sec. 3: the cell
 * problem is fixed by its streaming weights, optical size, inflow faces and
 * source nodes).  x: device [n][24] = [|Ox| h/dx, |Oy| h/dy, |Oz| h/dz,
 * sigma_t h, inflow x-face (4, node iy+2iz), y-face (4, ix+2iz), z-face (4,
 * ix+2iy), h*S (8)] with h = (dx dy dz)^(1/3), all direction components taken
 * non-negative.  psi: device [n][8] out.  precision selects float/double for
 * both arrays.
 */
int dgsn_local_solve(dgsn_ctx *ctx, const void *x, void *psi, long long n, int precision,
                     void *stream);

/*
 * Load a shallow-ANN artifact (Sec. 3, Eq. (ANN:Eq1): one hidden layer,
 * 24 inputs as in dgsn_local_solve but homogeneity-normalised, 8 outputs).
 * File format (little endian): "DGSNANN1" magic, u32 version=1, u32 n_in=24,
 * u32 n_hidden (<= 256), u32 n_out=8, u32 activation (0 = ReLU), u32 flags,
 * then float32 W1[n_hidden][n_in], b1[n_hidden], W2[n_out][n_hidden],
 * b2[n_out], then u32 CRC-32 (IEEE) of everything before it.
 *
 * Version 2 holds the paper-form networks (Sec. 3, Eq. (ANN:Eq1)-(ANN:Eq4);
 * one per octant, first paragraphs of Sec. 4): "DGSNANN1", u32 version=2,
 * u32 n_in=26, u32 n_hidden (1..8), u32 n_out=8, u32 activation=1 (tanh),
 * u32 flags=1 (ELU output layer), u32 n_nets=8, float32 alpha, float32
 * beta_scale, float32 imin[26], float32 imax[26], then for octant
 * o = [Ox<0] + 2[Oy<0] + 4[Oz<0] = 0..7: float32 W1[n_hidden][26],
 * b1[n_hidden], W2[8][n_hidden], b2[8]; then the CRC-32.  The 26 inputs, in
 * the cell's physical frame: the inflow values of the x, y and z faces (4
 * each, face node = lower tangential bit + 2 * higher one), Omega_x,
 * Omega_y, the 8 nodal sources, sigma_t, dx, dy, dz.  Each input is scaled
 * as In = (I - alpha (imin + imax) / 2) / |imax - imin| (Eq. (ANN:Eq2)); the
 * outputs are psi = z for z >= 0 and beta (exp(z) - 1) below, with
 * beta = beta_scale * max of the 12 inflow values (Eq. (ANN:Eq4)).
 *
 * Version 3 holds paper-form networks of the same form, one per quadrature
 * direction (the reading of Sec. 4's training paragraph that trains an ANN
 * for each direction, typically at one problem's sigma_t and cell size): the
 * version-2 layout with version=3 and n_nets = K (1..4096) directions,
 * followed after imax by float32 omega[K][3] (unit vectors, no two within
 * 1e-6), then the K networks in the order of omega.
 * Returns DGSN_EFORMAT for a bad magic, shape, size, bound, direction or
 * checksum.
 */
int dgsn_ann_load(dgsn_ctx *ctx, const char *path, dgsn_ann **out);
int dgsn_ann_destroy(dgsn_ann *ann);

/*
 * Evaluation precision of a version-1 network on the matrix cores (every
 * sweep and dgsn_ann_infer call that uses it; Sec. 3, Eq. (ANN:Eq1)):
 *   DGSN_ANN_BF16   (default) features and hidden activations rounded to
 *                   BF16 (relative 2^-9 each), FP32 accumulation;
 *   DGSN_ANN_BF16X2 split BF16: each of them enters as hi + lo BF16 parts
 *                   (hi = bf16(v), lo = bf16(v - hi), together v to about
 *                   2^-17), one matrix instruction per part, FP32
 *                   accumulation: the network's result to about FP32 accuracy
 *                   for weights held exactly in BF16 (as the trainer writes
 *                   them), at twice the matrix instructions.
 * The weights are BF16 in both modes.  Batches take BF16 networks only
 * (DGSN_EUNSUPPORTED at dgsn_batch_run).  DGSN_EINVAL for a version-2 or
 * -3 artifact (the paper-form networks run in FP32 on the vector ALUs) with
 * a mode other than DGSN_ANN_BF16.
 */
enum { DGSN_ANN_BF16 = 0, DGSN_ANN_BF16X2 = 1 };
int dgsn_ann_set_mode(dgsn_ann *ann, int mode);

/* Artifact shape (host out, each pointer may be NULL): version (1, 2 or 3),
   inputs, hidden units, networks (1; 8 per octant; K per direction). */
int dgsn_ann_info(const dgsn_ann *ann, int *version, int *n_in, int *n_hidden, int *n_nets);

/*
 * Paper-form network `octant` on raw inputs, on the vector ALUs in FP32: for
 * version-2 artifacts the network of that octant (0..7), for version-3 the
 * network of the artifact's direction omega[octant] (0..K-1).  x device
 * float [n][26] in the layout above, y device float [n][8] (physical node
 * order).  DGSN_EINVAL for a version-1 artifact or an index out of range.
 */
int dgsn_ann_infer_octant(const dgsn_ann *ann, int octant, const float *x, float *y,
                          long long n, void *stream);

/*
 * Raw network evaluation on the device with BF16 matrix cores and FP32
 * accumulation: y = W2 relu(W1 x + b1) + b2.  x: device float [n][24],
 * y: device float [n][8].  Version-1 artifacts only (DGSN_EINVAL otherwise).
 */
int dgsn_ann_infer(const dgsn_ann *ann, const float *x, float *y, long long n, void *stream);

/*
 * Particle-balance tally of forward sweeps, in FP64 (the weak form below
 * Eq. (T9) tested with the constant function: for each cell and direction,
 * outflow - inflow + sigma_t int psi - int Q = 0 for the exact cell
 * solution; summed over cells with the quadrature weights the interior
 * faces cancel).  With enable != 0 every later dgsn_sweep and the iterations
 * of dgsn_source_iterate also store each direction's outflow through the
 * domain boundary into the fronts and tally, over the whole sweep:
 *   terms[0] boundary outflow  sum_d w_d sum_{outflow faces} |Omega.n| int_f psi_d
 *   terms[1] boundary inflow   the same over the inflow faces with psi_inc
 *   terms[2] absorption        sum_c sigma_t int_c phi
 *   terms[3] source            sum_c int_c sum_d w_d S_d (the isotropic source;
 *            the anisotropic moment sources of orders 1..3 integrate to zero
 *            over a level-symmetric set and are not tallied)
 *   terms[4] terms[0] - terms[1] + terms[2] - terms[3]  (0 up to rounding for
 *            the GE solvers; the conservation error of a network solver)
 * for the last dgsn_sweep or the iterate returned by the last
 * dgsn_source_iterate.  Integrals are exact for the trilinear fluxes (face:
 * area x mean of the four face nodes, cell: volume x mean of the eight
 * nodes); sums are in FP64 over the problem-precision values.
 * dgsn_problem_balance synchronizes stream after a dgsn_sweep and returns
 * DGSN_EINVAL when no tallied sweep has run since the tally was enabled.
 * Cost: the boundary outflow stores and a pass over the fronts per sweep; on
 * a mesh that the tile edge does not divide, a tallied sweep runs single
 * cells (same results, every tiling does the same cell arithmetic).
 */
int dgsn_problem_set_balance(dgsn_problem *p, int enable);
int dgsn_problem_balance(dgsn_problem *p, double terms[5], void *stream);

/*
 * Generation counter of a problem (host out): changes whenever a setter
 * (materials, scattering, anisotropy, inflow, network, solver) or a sweep or
 * source iteration changes the problem's inputs or its stored angular flux.
 * A caller that keeps results of a source iteration (an autograd tape) can
 * tell whether the problem still holds the state they came from.
 */
int dgsn_problem_generation(const dgsn_problem *p, unsigned long long *gen);

/*
 * Problem statistics (host out): solves per sweep (cells*dirs*groups),
 * hyperplane count, and the algorithmic HBM bytes of one sweep
 * (s*(24*solves + 17*cells*groups), s = sizeof(real)).
 */
int dgsn_problem_stats(const dgsn_problem *p, long long *solves_per_sweep, int *n_planes,
                       double *algo_bytes_per_sweep);

/*
 * Kernel timing of the sweep (instrumentation).  With enable != 0 every
 * sweep kernel launch of this problem is bracketed by HIP events on its
 * stream.  dgsn_problem_kernel_time returns, for the most recent
 * dgsn_sweep, dgsn_source_iterate or dgsn_adjoint_solve call, the sum of the
 * durations of all its sweep kernel launches in milliseconds and the number
 * of launches (a source iteration that stops at iteration k may also have
 * timed the sweep of iteration k+1, enqueued ahead of the residual check);
 * it synchronizes the problem's last stream.
 */
int dgsn_problem_set_timing(dgsn_problem *p, int enable);
int dgsn_problem_kernel_time(dgsn_problem *p, double *ms_sum, int *launches);

/*
 * Batched execution of many independent problems (FP32, any mesh size,
 * quadrature and group count, solver DGSN_GE or DGSN_ANN per problem): one
 * sweep of every problem in a single HIP-graph launch, followed by the
 * per-problem octant reductions.  Not in the paper.  Two schedules:
 *   DGSN_SCHED_PLANES (default): step t of the graph is one batched kernel
 *     that advances every problem that still has a step t (a tile or cell
 *     hyperplane, by its tile edge).
 *   DGSN_SCHED_DATAFLOW: one launch; per octant the units (problem, step,
 *     block of tiles) of all problems form one work queue in step-major
 *     order, and each unit waits on device flags of the units holding its
 *     tiles' upwind neighbours.  Waits are bounded as for a single problem;
 *     an expired wait is reported by the next dgsn_batch_latencies_us or
 *     dgsn_batch_autotune (DGSN_ETIMEOUT).
 * dgsn_batch_create: probs must stay alive while the batch exists.  Each
 *   problem's materials are read from its buffers at run time; its inflow,
 *   solver and network are part of the captured graph, which dgsn_batch_run
 *   captures again when any of them changed since (a member set to
 *   DGSN_GE_DENSE, or to DGSN_ANN without a network, is refused; so, with
 *   DGSN_EUNSUPPORTED, is one with split-BF16 or per-direction networks).  Two runs
 *   of one batch must not overlap (they share the device tables).
 * dgsn_batch_set_io: device src / phi of problem `index`, layouts as in
 *   dgsn_sweep; must be set for every problem before the first run.
 * dgsn_batch_set_tiles: per-problem tile edge (1 or 2; a problem set to 3
 *   runs with 2 in a batch), host [n].
 * dgsn_batch_set_schedule / _get_schedule: DGSN_SCHED_PLANES or
 *   DGSN_SCHED_DATAFLOW.
 * dgsn_batch_autotune: times the batch under both schedules with candidate
 *   tile assignments (all 2, all 1, 2 for meshes of >= 32^3 cells) and keeps
 *   the fastest; returns its time in ms.  Runs the batch several times;
 *   synchronizes stream.
 * dgsn_batch_run: enqueues the graph on stream.
 * dgsn_batch_latencies_us: per-problem time from the start of the last run to
 *   the end of that problem's last sweep step, device wall clock, host [n];
 *   synchronizes the device.
 */
int dgsn_batch_create(dgsn_ctx *ctx, dgsn_problem *const *probs, int n, dgsn_batch **out);
int dgsn_batch_set_io(dgsn_batch *b, int index, const void *src, void *phi);
int dgsn_batch_set_tiles(dgsn_batch *b, const int *tile_edges);
int dgsn_batch_set_schedule(dgsn_batch *b, int schedule);
int dgsn_batch_get_schedule(const dgsn_batch *b, int *schedule);
int dgsn_batch_autotune(dgsn_batch *b, void *stream, double *best_ms);
int dgsn_batch_run(dgsn_batch *b, void *stream);
int dgsn_batch_latencies_us(const dgsn_batch *b, double *out);
int dgsn_batch_destroy(dgsn_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* DGSN_H */
