// Kernel argument blocks and launch wrappers shared by the runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct dgsn_problem;

namespace dgsn {

// Maximum that carries a NaN in either operand (a NaN compares false, so a
// plain a > b ? a : b would drop a NaN in a).  The residual reductions rely
// on it: a NaN flux must reach the host as a NaN residual.
__device__ __forceinline__ double fmax_d(double a, double b) { return (a > b || a != a) ? a : b; }

// One hyperplane step of a sweep (all octants, directions, groups).
template <typename Real>
struct PlaneArgs {
    const uint32_t *cells;     // packed canonical cells of the plane (i | j<<10 | k<<20)
    uint32_t ncp;              // number of cells in the plane
    uint32_t nx, ny, nz;
    uint32_t G, Do, DG;
    uint32_t ncell;
    uint32_t fx_o, fx_k, fx_j; // front strides (elements): octant, outer, inner cell index
    uint32_t fy_o, fy_k, fy_j;
    uint32_t fz_o, fz_k, fz_j;
    // lane layout of the 256-lane sweep blocks: each wave holds spw = 64 / Do
    // segments of Do direction lanes; segment s of a block is group s % G of
    // tile slot s / G, and a block covers nc = 4 spw / G tiles.  Segments never
    // cross a wave, so the direction reductions need no block barrier.
    uint32_t spw, nc;
    uint32_t mag_do, mag_g;    // ceil(2^16 / Do), ceil(2^16 / G): exact quotients below 256
    const Real *dir;           // [8][Do][kDirStride]
    const Real *sigma_t;       // [G][ncell]
    const Real *src;           // [G][ncell][8]
    Real *fx, *fy, *fz;        // face fronts
    Real *phi_oct;             // [8][G][ncell][8]
    Real *psi;                 // [8*Do][G][ncell][8] (store or adjoint contraction)
    Real *grad_oct;            // [8][G][ncell][2] adjoint contraction output (or null)
    Real vol;                  // cell volume
    Real hh;                   // cube root of the cell volume (ANN features)
    const void *ann_params;    // device ANN operand images (ANN solver)
    Real inc[8][3];            // inflow value per octant slot and canonical axis
    // anisotropic in-group scattering (source iteration only; nmom <= 1:
    // isotropic): nmom = (L+1)^2 moments, of which k >= 1 enter the source
    // as sum_k Y_k(Omega_d) msrc_k and leave the sweep as the per-octant
    // moments sum_{d in octant} w_d Y_k(Omega_d) psi_d
    uint32_t nmom;
    // 1: also store the outflow faces on the domain boundary into the fronts
    // (no downstream cell reads them; the balance tally's leakage does)
    uint32_t keep_out;
    const Real *ylm;           // [8][Do][kYlmStride]
    const Real *msrc;          // [G][ncell][nmom-1][8] sigma_{s,n(k)} phi_k
    Real *mom_oct;             // [8][G][ncell][8][nmom-1] (moment fastest)
};

// Dataflow schedule of a sweep: one launch processes every step.  Workgroup
// b serves octant b & 7; it takes the next unit of its octant (a block of
// tiles in one step) from that octant's ticket counter, in step-major order,
// waits until the units of the previous step that hold its tiles' upwind
// neighbours are done, solves its tiles and flags itself done.  A unit only
// waits on units of its octant with smaller tickets, held by workgroups that
// are already running, so the launch always drains; every wait is also
// bounded by spin_limit polls, after which the unit raises the error word and
// proceeds.  A fill kernel clears the tickets and flags before each launch.
struct FlowArgs {
    // per unit of one octant, in ticket order: x = step, y = block of tiles
    // within the step, z = first tile of the step in the tile list, w = tiles
    // in the step
    const uint4 *unit_map;
    // per unit: the units (of the same octant) it waits for, [x, y]; x > y
    // for none
    const uint2 *unit_dep;
    unsigned *sync;            // tickets (one 128-byte line per octant), error word, done[8][units_o]
    unsigned units_o;          // units per octant
    unsigned spin_limit;       // polls of one wait before it gives up
};
constexpr int kFlowTicket = 0;      // + 32 * octant
constexpr int kFlowError = 256;
constexpr int kFlowDone = 288;      // + octant * units_o + unit
constexpr unsigned kFlowSpinDefault = 1u << 20;
// workgroups per octant of one dataflow launch at most (8 * 2^20 * 256 lanes
// stay below the 2^32 work-items of a launch).  A longer queue runs as several
// launches in stream order: the tickets continue across them, and a unit's
// dependencies have smaller tickets, so they lie in an earlier launch or in
// its own.
constexpr unsigned kFlowMaxGroupsPerOctant = 1u << 20;

// FP64 partials of the octant reduction, per block and in the result slot
// of an iteration: the residual terms and the particle-balance terms.
constexpr int kRedMaxD = 0;    // max |phi_new - phi_old|
constexpr int kRedMaxF = 1;    // max |phi_new|
constexpr int kRedEps = 2;     // sum of the eps_S terms (cell averages)
constexpr int kRedAbs = 3;     // sum_{g,c} sigma_t * sum_n phi_n
constexpr int kRedSrc = 4;     // sum_{g,c} sum_n S_n
constexpr int kRedLeak = 5;    // sum over boundary outflow slots of w kappa_a sum_e psi_e
constexpr int kRedStride = 8;  // doubles per block partial and per result slot

template <typename Real>
struct ReduceArgs {
    const Real *phi_oct;       // [8][nv][8]
    Real *phi;                 // [nv][8] in: previous iterate (if resid, unless phi_prev), out: new
    const Real *phi_prev;      // [nv][8] previous iterate in a separate buffer (or null)
    long long nv;              // G * ncell
    int resid;                 // compute residual partials
    int balance;               // compute the absorption and source partials of the tally
    const Real *sigma_t;       // [nv] (balance)
    const Real *src_sweep;     // [nv][8] source of the sweep just reduced (balance; read
                               // before src_next, which may be the same buffer, is written)
    double *partials;          // [blocks][kRedStride]
    double *result;            // [kRedStride]
    Real *src_next;            // next source (or null)
    const Real *q_cell;        // [nv] per-cell source (or null)
    const Real *q_nodal;       // [nv][8] nodal source (or null)
    const Real *sigma_s;       // [nv] (or null)
};

int block_size_for(int Do);

// helpers of the batched path (runtime.hip)
PlaneArgs<float> batch_plane_args(dgsn_problem *p, const void *src);
int batch_reduce(dgsn_problem *p, void *phi, hipStream_t s);
int cells_per_block(int Do, int G);
int reduce_blocks_for(long long nv);

// local-system forms of the GE solver
constexpr int kFormMassInv = 0;   // mass-inverse form, structured elimination
constexpr int kFormDense = 1;     // the paper's assembled A_psi, dense elimination
constexpr int kFormAnn = 2;       // the shallow network in place of assembly + elimination
constexpr int kFormAnnPaper = 3;  // the paper-form per-octant network (vector ALUs)
constexpr int kFormAnnSplit = 4;  // the shallow network with split-BF16 activations
constexpr int kFormAnnPaperDir = 5;   // the paper-form networks, one per direction

// Occupancy request of a sweep kernel (waves per SIMD; 1 = no request).  The
// FP64 single-cell mass-inverse kernel would take 176 registers and run at 2
// waves per SIMD; held to 168 it runs at 3 with no spills.  The FP64 2x2x2
// mass-inverse kernel otherwise runs at 1 wave; held to 2 it spills about
// 160 bytes per lane and is still faster (6.5 ms against 7.2 ms per sweep at
// 64^3 S8 G8).  The FP64 3x3x3 tiles and the dense form keep the compiler's
// choice.
template <typename Real, int Form, int B, int kMom = 0>
constexpr int kMinWavesPerSimd =
    (sizeof(Real) == 8 && Form == kFormMassInv && kMom == 0) ? (B == 1 ? 3 : (B == 2 ? 2 : 1))
                                                           : 1;

int launch_tile_ann(const PlaneArgs<float> &A, int b, bool split, hipStream_t s);

template <typename Real>
int launch_tile(const PlaneArgs<Real> &A, int form, int b, bool store_psi, bool adjoint,
                hipStream_t s);
template <typename Real>
int launch_flow(const PlaneArgs<Real> &A, const FlowArgs &F, int form, int b, bool store_psi,
                bool adjoint, hipStream_t s);   // all launches of one sweep
int launch_flow_reset(const FlowArgs &F, hipStream_t s);   // before every launch_flow
template <typename Real>
int launch_reduce(const ReduceArgs<Real> &R, int blocks, hipStream_t s);
// Boundary leakage partials of the balance tally: for every face slot of the
// three fronts (which hold the domain-boundary outflow after a sweep run with
// A.keep_out), w_d kappa_a(d) sum_e psi_e, summed per block into
// partials[block][kRedLeak]; blocks must equal the octant reduction's.
template <typename Real>
int launch_leakage(const PlaneArgs<Real> &A, double *partials, int blocks, hipStream_t s);
template <typename Real>
int launch_build_source(long long nv, const Real *q, const Real *ss, const Real *phi, Real *src,
                        hipStream_t s);
template <typename Real>
int launch_adjoint_load(long long nv, const Real *gphi, double vol, Real *gl, hipStream_t s);
// multigroup source S_g = q_g + (1/4pi) sum_g' sigma(g' -> g) phi_g' (transpose:
// sigma(g -> g')); q_cell [G][ncell] and/or q_nodal [G][ncell][8] may be null
template <typename Real>
int launch_build_source_gg(long long ncell, int G, const Real *q_cell, const Real *q_nodal,
                           const Real *sigma_gg, const Real *phi, Real *src, bool transpose,
                           hipStream_t s);
// flux moments of anisotropic scattering: mom [G][ncell][nm-1][8] = the sum
// over octants of mom_oct [8][G][ncell][8][nm-1], and msrc (same layout)
// = sigma_{s,n(k)} mom (moments k = 1 .. nm-1, order n(k) = floor(sqrt k));
// msrc (and sigma_sn) null: the moments only
template <typename Real>
int launch_reduce_moments(long long nv, int nm, const Real *mom_oct, const Real *sigma_sn,
                          Real *mom, Real *msrc, hipStream_t s);
// group-to-group source moments msrc[g] = sum_g' sigma_{s,n(k)}(g' -> g) mom[g']
// (transpose: sigma(g -> g')), both [G][ncell][nm-1][8], sigma_cm
// [ncell][L][G][G] orders 1..L, cell-major
template <typename Real>
int launch_build_msrc_gg(long long ncell, int G, int nm, const Real *sigma_cm, const Real *mom,
                         Real *msrc, bool transpose, hipStream_t s);
// n elements at p set to NaN (debug poisoning of the fronts)
template <typename Real>
int launch_fill_nan(long long n, Real *p, hipStream_t s);
// *bad |= 1 (sigma_t), 2 (sigma_s) where a value is negative or not finite,
// 4 where q is not finite, 8 where sigma_s > sigma_t; n values each
template <typename Real>
int launch_check_materials(long long n, const Real *st, const Real *ss, const Real *q,
                           unsigned *bad, hipStream_t s);
// the public layout of the moments: dst [nm-1][G][ncell][8] from src [G][ncell][nm-1][8]
template <typename Real>
int launch_moments_public(long long nv, int nm, const Real *src, Real *dst, hipStream_t s);
// dst [ncell][nmat] = the cell-major copy of src [nmat][ncell]
template <typename Real>
int launch_cell_major(long long ncell, int nmat, const Real *src, Real *dst, hipStream_t s);
template <typename Real>
int launch_reduce_grad(long long nv, const Real *grad_oct, Real *gst, Real *gq, hipStream_t s);

}  // namespace dgsn
