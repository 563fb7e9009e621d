// Internal declarations of libdgsn (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dgsn.h"
#include "kernels.hpp"

struct dgsn_problem;

namespace dgsn {

// ---- error reporting -------------------------------------------------------
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define DGSN_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::dgsn::set_error(DGSN_EHIP, "%s failed: %s (%s:%d)", #call,          \
                                     hipGetErrorString(e_), __FILE__, __LINE__);         \
    } while (0)

#define DGSN_TRY(expr)              \
    do {                            \
        int rc_ = (expr);           \
        if (rc_ != DGSN_OK) return rc_; \
    } while (0)

// ---- constants -------------------------------------------------------------
constexpr int kMaxCellsPerAxis = 1024;   // packed (i, j, k) in 10 bits each
// per direction: S_d[64] (paper form), kappa_a / 36 [3], weight, kappa_a [3], pad
constexpr int kDirStride = 72;
constexpr int kDirK36 = 64;
constexpr int kDirW = 67;
constexpr int kDirK = 68;
constexpr int kMaxHidden = 256;
constexpr int kMaxTile = 3;       // largest tile edge of the sweep
// anisotropic scattering: per direction the real harmonics Y_k(Omega),
// k = 1 .. (L+1)^2 - 1 at index k - 1, orders L <= kMaxPlOrder
constexpr int kYlmStride = 16;
constexpr int kMaxPlOrder = 3;
// iterations of the convergence history held without a host allocation (the
// no-allocation source iteration records at most this many)
constexpr int kSiHistoryReserve = 4096;

// ---- host-side quadrature ---------------------------------------------------
int level_symmetric(int order, std::vector<double> &omega, std::vector<double> &weight);
// real orthonormal spherical harmonics Y_k, k = n^2 + n + m, n <= L <= 3, of
// the unit direction om (Cartesian forms; polar axis z, no (-1)^m phase)
void real_ylm(int L, const double om[3], double *Y);

const void *ann_device_params(const dgsn_ann *a);
// Per-octant weight images of a paper-form network for a problem with cell
// sizes h (canonical-frame features, layout in pann_body.hpp).
int pann_problem_image(const dgsn_ann *a, const double h[3], std::vector<float> &out);
// Per-slot images of a per-direction paper-form network ([8][Do] slots of the
// problem's octant-sorted directions omega [8][Do][3]; valid[s] = 0 marks a
// padding slot); DGSN_EINVAL if a direction has no net.
int pann_problem_image_dir(const dgsn_ann *a, const double h[3], const double *omega, int Do,
                           const int *valid, std::vector<float> &out);

// one unit of the dataflow schedule (host copy; see flow_units_host)
struct FlowUnitHost {
    unsigned step, block, t0, cnt, dlo, dhi;
};
int flow_units_host(const dgsn_problem *p, int tb, std::vector<FlowUnitHost> &out);
int autotune_problem(dgsn_problem *p, hipStream_t s, double ms_out[6]);

// ---- device allocation helper ------------------------------------------------
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int alloc(size_t n);
    void release();
    ~DevBuf() { release(); }
};

// pinned host memory (hipHostMalloc), for stream-ordered readbacks
struct HostBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int alloc(size_t n);
    void release();
    ~HostBuf() { release(); }
};

}  // namespace dgsn

struct dgsn_ctx {
    int device = 0;
    int num_cu = 0;
    // this device's copy of the library's static scratch array (see
    // dgsn_source_iterate_noalloc), from hipGetSymbolAddress at creation
    void *static_scratch = nullptr;
};

struct dgsn_ann {
    dgsn_ctx *ctx = nullptr;
    int version = 1;                     // 1: canonical 24-input net, 2: paper-form per
                                         // octant, 3: paper-form per quadrature direction
    int mode = DGSN_ANN_BF16;            // version 1: evaluation precision on the matrix cores
    int n_in = 24, n_hidden = 0, n_out = 8, act = 0, n_nets = 1;
    float alpha = 0.0f, beta_scale = 0.0f;   // version 2: Eq. (ANN:Eq2) and (ANN:Eq4)
    std::vector<float> imin, imax;       // versions 2, 3: input bounds [26]
    std::vector<float> omega;            // version 3: the direction of each net [n_nets][3]
    std::vector<float> W1, b1, W2, b2;   // host copies (fp32), n_nets networks back to back
    // device: version 1, bf16 packed operand images and fp32 biases (layout in
    // ann.hip); version 2, the per-octant raw-input images (pann_body.hpp)
    dgsn::DevBuf d_params;
};

struct dgsn_problem {
    dgsn_ctx *ctx = nullptr;
    int n[3] = {0, 0, 0};
    double len[3] = {0, 0, 0};
    double h[3] = {0, 0, 0};
    long long ncell = 0;
    int G = 0, D = 0, Do = 0;
    int precision = DGSN_FP32;
    int solver = DGSN_GE;
    int store_psi = 0;
    int si_criterion = DGSN_SI_MAXNORM;
    int n_planes = 0;
    size_t real_size = 4;
    double psi_inc[6] = {0, 0, 0, 0, 0, 0};
    const dgsn_ann *ann = nullptr;
    dgsn::DevBuf d_pann;    // paper-form network folded for this problem (pann_body.hpp)

    std::vector<int> dir_user;       // octant-sorted slot -> user direction index
    std::vector<double> dir_host;    // [8][Do][kDirStride] in FP64
    std::vector<double> omega_host;  // [8][Do][3] the slot directions
    int pl_order = 0;                // anisotropic scattering order L (0: none)
    int pl_gg = 0;                   // 1: the orders 1..L are group-to-group matrices
    std::vector<int> plane_off;      // [n_planes + 1]
    // tile hyperplane schedules for B x B x B tiles (B = 2, 3; index B):
    // packed tile coordinates, tile-hyperplane major (B = 1 is the cell
    // schedule above)
    int tile_b = 2;                  // tile edge used by the sweep (1, 2 or 3)
    // dataflow schedule (one launch per sweep, GE solvers): per tile edge B
    // (1 = cells) the first unit and the first tile of every step, on device
    int schedule = DGSN_SCHED_PLANES;
    std::vector<double> si_resid, si_eps;   // per iteration of the last source iteration
                                            // (capacity kSiHistoryReserve from creation)
    int flow_ready = 0;
    dgsn::DevBuf d_unit_map[4];      // uint4 per unit of one octant (built on first use)
    dgsn::DevBuf d_unit_dep[4];      // uint2 per unit: range of units it waits for
    unsigned flow_units[4] = {0, 0, 0, 0};   // units per octant
    dgsn::DevBuf d_flow_sync;        // tickets, error word, done flags [8][units per octant]
    unsigned flow_spin = 0;          // 0: default poll limit
    int n_tplanes[4] = {0, 0, 0, 0};
    std::vector<int> tplane_off[4];  // [n_tplanes[B] + 1]
    dgsn::DevBuf d_tiles[4];

    dgsn::DevBuf d_dir;              // [8][Do][kDirStride] real
    dgsn::DevBuf d_plane_cells;      // uint32 packed canonical (i, j, k), plane-major
    dgsn::DevBuf sigma_t, sigma_s, q;        // [G][ncell]
    dgsn::DevBuf sigma_gg;                   // [ncell][G][G] multigroup scattering, cell-major
                                             // (from g' into g at [c][g'][g]; or empty)
    dgsn::DevBuf sigma_sn;                   // [L][G][ncell] Legendre moments of orders 1..L
                                             // (with pl_gg cell-major [ncell][L][G][G], from
                                             // g' into g at [c][n-1][g'][g])
    dgsn::DevBuf d_ylm;                      // [8][Do][kYlmStride] harmonics of the slot directions
    dgsn::DevBuf mom_oct;                    // [8][G][ncell][8][nm-1] per-octant flux moments
    dgsn::DevBuf mom;                        // [G][ncell][nm-1][8] flux moments (the public
                                             // layout [nm-1][G][ncell][8] on request)
    dgsn::DevBuf msrc;                       // [G][ncell][nm-1][8] sigma_{s,n} x moments
    dgsn::DevBuf src;                         // [G][ncell][8]
    dgsn::DevBuf phi_oct;                     // [8][G][ncell][8]
    dgsn::DevBuf front_x, front_y, front_z;   // [8][..][..][4][Do*G]
    dgsn::DevBuf psi;                         // [D][G][ncell][8] (store_psi)
    dgsn::DevBuf adj_phi, adj_src, grad_oct;  // adjoint work buffers
    dgsn::DevBuf red_partials;                // FP64 reduction partials
    dgsn::DevBuf red_result;                  // FP64 [2][4]: one slot per iteration in flight
    dgsn::HostBuf h_result;                   // pinned [2][4] FP64 + [2] error words
    hipEvent_t ev_result[2] = {nullptr, nullptr};   // each slot's readback is complete
    dgsn::DevBuf phi_alt;                     // [G][ncell][8] second iterate buffer
    dgsn::DevBuf d_check;                     // one flag word of the materials check
    int red_blocks = 0;

    // Generation counters.  gen changes with every call that changes the
    // problem's inputs (materials, scattering, inflow, solver, network) or
    // its stored angular flux (sweeps and source iterations); cfg_gen with
    // the inputs a captured batch graph holds by value (inflow, solver,
    // network).  psi_valid: the stored angular flux is that of a completed
    // source iteration on the current inputs (what the adjoint needs).
    unsigned long long gen = 1, cfg_gen = 1;
    int psi_valid = 0;
    void touch(bool cfg)
    {
        ++gen;
        if (cfg) ++cfg_gen;
        psi_valid = 0;
    }

    // FP64 particle-balance tally of forward sweeps (off by default): the
    // sweep keeps the domain-boundary outflow in the fronts and the octant
    // reduction adds the absorption and source partials.  bal_state: 0 none,
    // 1 the terms of the last dgsn_sweep are in red_result slot 0, 2 bal_host
    // holds the raw partial sums of the last source iteration's returned
    // iterate.  bal_inflow and bal_wsum: the boundary inflow and the weight
    // sum of the tallied sweep, from the direction table as the sweep used it.
    // debug flags (DGSN_DEBUG_*): POISON_FRONTS fills the face fronts with
    // NaN before every sweep
    int debug = 0;

    int balance = 0;
    int bal_state = 0;
    double bal_host[dgsn::kRedStride] = {};
    double bal_inflow = 0.0, bal_wsum = 0.0;

    // optional per-launch kernel timing of the last sweep
    int timing = 0;
    std::vector<hipEvent_t> ev;               // [2 * n_planes]
    int ev_used = 0;
    hipStream_t last_stream = nullptr;
    ~dgsn_problem();
};
