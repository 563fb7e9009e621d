// Host runtime and C ABI of libdgsn: contexts, problem objects, validation,
// the hyperplane schedule, the source-iteration driver and the adjoint driver.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "cell.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "pann_body.hpp"

namespace dgsn {

namespace {
thread_local char g_msg[1024] = "";
}

int set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_msg[0] = '\0'; }

// DGSN_TEST_ALLOC_LIMIT (bytes, unset or 0: none): device allocations above
// it fail as if the device were out of memory, so that the error paths of
// the setters can be exercised without exhausting the device.
static size_t test_alloc_limit()
{
    const char *e = getenv("DGSN_TEST_ALLOC_LIMIT");
    return e ? (size_t)strtoull(e, nullptr, 10) : 0;
}

int DevBuf::alloc(size_t n)
{
    release();
    if (n == 0) return DGSN_OK;
    const size_t lim = test_alloc_limit();
    if (lim && n > lim)
        return set_error(DGSN_ENOMEM, "allocation of %zu bytes refused (DGSN_TEST_ALLOC_LIMIT %zu)",
                         n, lim);
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return set_error(DGSN_ENOMEM, "hipMalloc(%zu bytes) failed: %s", n, hipGetErrorString(e));
    }
    bytes = n;
    return DGSN_OK;
}

void DevBuf::release()
{
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

int HostBuf::alloc(size_t n)
{
    release();
    if (n == 0) return DGSN_OK;
    hipError_t e = hipHostMalloc(&ptr, n, hipHostMallocDefault);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return set_error(DGSN_ENOMEM, "hipHostMalloc(%zu bytes) failed: %s", n,
                         hipGetErrorString(e));
    }
    bytes = n;
    return DGSN_OK;
}

void HostBuf::release()
{
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

// Scratch of dgsn_source_iterate_noalloc, one copy per device for the life
// of the process: the FP64 reduction partials of up to 2048 blocks, two
// result slots, and the look-ahead iterate of the overlapped iteration.
// Host code never uses the array's name as an address: each device's copy is
// found once with hipGetSymbolAddress (static_scratch_of) and passed on.
constexpr size_t kScratchPartials = 2048ull * kRedStride * sizeof(double);   // 128 KiB
constexpr size_t kScratchResults = 256;                                       // 2 slots
constexpr size_t kScratchIterate = 64ull << 20;                               // 64 MiB
constexpr size_t kScratchBytes = kScratchPartials + kScratchResults + kScratchIterate;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mutex;
void *g_scratch_ptr[64] = {};   // per device ordinal
}  // namespace

// Address of this device's copy of the scratch array (the device must be
// current); looked up on the first call for each device and kept.
int static_scratch_of(int device, void **out)
{
    if (device < 0 || device >= 64)
        return set_error(DGSN_EUNSUPPORTED, "device ordinal %d beyond the scratch table", device);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return set_error(DGSN_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s",
                             device, hipGetErrorString(e));
        }
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return DGSN_OK;
}

}  // namespace dgsn

using namespace dgsn;

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// 1D factors of the canonical cell system (see cell.hpp).
double m1(int k, int j) { return k == j ? 1.0 / 3.0 : 1.0 / 6.0; }
double t1(int k, int j) { return (k == 1 && j == 0) ? -0.5 : 0.5; }

// S_d[k][j] = sum_a kappa_a T_a[k][j], T_a = T on axis a, M1 on the others.
void streaming_matrix(const double kappa[3], double S[64])
{
    for (int k = 0; k < 8; ++k)
        for (int j = 0; j < 8; ++j) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a) {
                double v = kappa[a];
                for (int b = 0; b < 3; ++b) {
                    const int kb = (k >> b) & 1, jb = (j >> b) & 1;
                    v *= (b == a) ? t1(kb, jb) : m1(kb, jb);
                }
                s += v;
            }
            S[k * 8 + j] = s;
        }
}

int validate_desc(const dgsn_problem_desc *d)
{
    if (!d) return set_error(DGSN_EINVAL, "descriptor is NULL");
    const int n[3] = {d->nx, d->ny, d->nz};
    const double L[3] = {d->lx, d->ly, d->lz};
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 1 || n[a] > kMaxCellsPerAxis)
            return set_error(DGSN_EINVAL, "cells per axis must be in 1..%d (axis %d: %d)",
                             kMaxCellsPerAxis, a, n[a]);
        if (!(L[a] > 0.0) || !std::isfinite(L[a]))
            return set_error(DGSN_EINVAL, "domain length must be finite and > 0 (axis %d)", a);
    }
    if (d->n_groups < 1) return set_error(DGSN_EINVAL, "n_groups must be >= 1");
    if (d->n_dirs < 8 || d->n_dirs % 8)
        return set_error(DGSN_EINVAL, "n_dirs must be a positive multiple of 8 (got %d)",
                         d->n_dirs);
    if (!d->omega || !d->weight) return set_error(DGSN_EINVAL, "omega/weight must not be NULL");
    if (d->precision != DGSN_FP32 && d->precision != DGSN_FP64)
        return set_error(DGSN_EINVAL, "precision must be DGSN_FP32 or DGSN_FP64");
    if (d->solver != DGSN_GE && d->solver != DGSN_ANN && d->solver != DGSN_GE_DENSE)
        return set_error(DGSN_EINVAL, "solver must be DGSN_GE, DGSN_GE_DENSE or DGSN_ANN");
    if (d->solver == DGSN_ANN && d->precision != DGSN_FP32)
        return set_error(DGSN_EUNSUPPORTED, "the ANN solver runs on FP32 problems only");
    int count[8] = {0};
    double wsum = 0.0;
    for (int i = 0; i < d->n_dirs; ++i) {
        const double *o = d->omega + 3 * i;
        const double nrm = std::sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
        if (!std::isfinite(nrm) || std::fabs(nrm - 1.0) > 1e-12)
            return set_error(DGSN_EINVAL, "direction %d is not a unit vector (|O| = %.17g)", i,
                             nrm);
        const double w = d->weight[i];
        if (!(w > 0.0) || !std::isfinite(w))
            return set_error(DGSN_EINVAL, "weight %d must be finite and > 0", i);
        wsum += w;
        count[(o[0] < 0) + 2 * (o[1] < 0) + 4 * (o[2] < 0)]++;
    }
    if (std::fabs(wsum - 4.0 * M_PI) > 1e-10)
        return set_error(DGSN_EINVAL, "weights must sum to 4 pi (sum = %.17g)", wsum);
    for (int o = 0; o < 8; ++o)
        if (count[o] != d->n_dirs / 8)
            return set_error(DGSN_EINVAL, "octant %d holds %d directions, expected %d", o,
                             count[o], d->n_dirs / 8);
    return DGSN_OK;
}

template <typename Real>
int upload_real(DevBuf &buf, const std::vector<double> &host)
{
    std::vector<Real> tmp(host.begin(), host.end());
    DGSN_TRY(buf.alloc(tmp.size() * sizeof(Real)));
    DGSN_HIP(hipMemcpy(buf.ptr, tmp.data(), tmp.size() * sizeof(Real), hipMemcpyHostToDevice));
    return DGSN_OK;
}

template <typename Real>
PlaneArgs<Real> plane_args(dgsn_problem *p, const void *src, bool adjoint)
{
    PlaneArgs<Real> A{};
    A.nx = p->n[0];
    A.ny = p->n[1];
    A.nz = p->n[2];
    A.G = p->G;
    A.Do = p->Do;
    A.DG = p->Do * p->G;
    A.ncell = (uint32_t)p->ncell;
    const uint32_t f4 = 4u * A.DG;   // one cell's slot: [direction-group][4 face nodes]
    A.fx_j = f4;
    A.fx_k = A.ny * f4;
    A.fx_o = A.nz * A.fx_k;
    A.fy_j = f4;
    A.fy_k = A.nx * f4;
    A.fy_o = A.nz * A.fy_k;
    A.fz_j = f4;
    A.fz_k = A.nx * f4;
    A.fz_o = A.ny * A.fz_k;
    A.spw = 64u / A.Do;
    A.nc = (uint32_t)cells_per_block(p->Do, p->G);
    A.mag_do = (65536u + A.Do - 1) / A.Do;
    A.mag_g = (65536u + A.G - 1) / A.G;
    A.dir = static_cast<const Real *>(p->d_dir.ptr);
    A.sigma_t = static_cast<const Real *>(p->sigma_t.ptr);
    A.src = static_cast<const Real *>(src);
    A.fx = static_cast<Real *>(p->front_x.ptr);
    A.fy = static_cast<Real *>(p->front_y.ptr);
    A.fz = static_cast<Real *>(p->front_z.ptr);
    A.phi_oct = static_cast<Real *>(p->phi_oct.ptr);
    A.psi = static_cast<Real *>(p->psi.ptr);
    A.grad_oct = nullptr;
    A.vol = Real(p->h[0] * p->h[1] * p->h[2]);
    A.hh = Real(std::cbrt(p->h[0] * p->h[1] * p->h[2]));
    for (int o = 0; o < 8; ++o)
        for (int a = 0; a < 3; ++a) {
            // forward: Omega enters through the low face of axis a when its
            // component is positive, through the high face otherwise
            const int face = 2 * a + ((o >> a) & 1);
            A.inc[o][a] = adjoint ? Real(0) : Real(p->psi_inc[face]);
        }
    return A;
}

}  // namespace

namespace dgsn {

// Dataflow units of one tile edge: blocks of cells_per_block tiles of one
// octant in one step, step-major; each depends on the units of the previous
// step that hold the upwind neighbours (i-1, j, k), (i, j-1, k), (i, j, k-1)
// of its tiles (problem-local unit indices, dlo > dhi for none).
int flow_units_host(const dgsn_problem *p, int tb, std::vector<FlowUnitHost> &out)
{
    const std::vector<int> &off = tb == 1 ? p->plane_off : p->tplane_off[tb];
    const int nc = cells_per_block(p->Do, p->G);
    const int T[3] = {(p->n[0] + tb - 1) / tb, (p->n[1] + tb - 1) / tb, (p->n[2] + tb - 1) / tb};
    const int ns = (int)off.size() - 1;
    out.clear();
    std::vector<int> pos((size_t)T[1] * T[2], -1);   // (j, k) -> index in the previous step
    std::vector<int> cur;
    int ubase_prev = 0;
    for (int st = 0; st < ns; ++st) {
        const int cnt = off[st + 1] - off[st];
        const unsigned nb = (unsigned)((cnt + nc - 1) / nc);
        if (8ull * (out.size() + nb) > (1ull << 31))
            return set_error(DGSN_EUNSUPPORTED, "too many dataflow units");
        const int ubase = (int)out.size();
        // tiles of this step, in the order of the tile list (k outer, j inner)
        cur.clear();
        for (int kk = 0; kk < T[2]; ++kk)
            for (int jj = 0; jj < T[1]; ++jj) {
                const int ii = st - jj - kk;
                if (ii >= 0 && ii < T[0]) cur.push_back(ii | jj << 10 | kk << 20);
            }
        if ((int)cur.size() != cnt) return set_error(DGSN_EINVAL, "inconsistent tile schedule");
        for (unsigned l = 0; l < nb; ++l) {
            unsigned lo = UINT32_MAX, hi = 0;
            for (int q = (int)l * nc; q < std::min(cnt, (int)(l + 1) * nc); ++q) {
                const int ii = cur[q] & 1023, jj = (cur[q] >> 10) & 1023, kk = cur[q] >> 20;
                int up[3] = {-1, -1, -1};
                if (ii > 0) up[0] = pos[(size_t)kk * T[1] + jj];
                if (jj > 0) up[1] = pos[(size_t)kk * T[1] + jj - 1];
                if (kk > 0) up[2] = pos[(size_t)(kk - 1) * T[1] + jj];
                for (int a = 0; a < 3; ++a)
                    if (up[a] >= 0) {
                        const unsigned u = (unsigned)(ubase_prev + up[a] / nc);
                        lo = std::min(lo, u);
                        hi = std::max(hi, u);
                    }
            }
            if (lo == UINT32_MAX) {
                lo = 1;
                hi = 0;
            }
            out.push_back(FlowUnitHost{(unsigned)st, l, (unsigned)off[st], (unsigned)cnt, lo, hi});
        }
        for (int q = 0; q < cnt; ++q)
            pos[(size_t)(cur[q] >> 20) * T[1] + ((cur[q] >> 10) & 1023)] = q;
        ubase_prev = ubase;
    }
    return DGSN_OK;
}

}  // namespace dgsn

namespace {

// Device unit maps of the single-problem dataflow schedule for every tile edge.
int flow_prepare(dgsn_problem *p)
{
    if (p->flow_ready) return DGSN_OK;
    const long long nmax = std::max(std::max(p->n[0], p->n[1]), p->n[2]);
    if (nmax * nmax * 8 * 4 * p->Do * p->G * (long long)p->real_size >= (1LL << 31))
        return set_error(DGSN_EUNSUPPORTED, "the dataflow schedule needs face fronts under 2 GiB");
    unsigned umax = 0;
    std::vector<FlowUnitHost> units;
    for (int tb = 1; tb <= kMaxTile; ++tb) {
        DGSN_TRY(flow_units_host(p, tb, units));
        std::vector<uint4> map(units.size());
        std::vector<uint2> dep(units.size());
        for (size_t u = 0; u < units.size(); ++u) {
            map[u] = make_uint4(units[u].step, units[u].block, units[u].t0, units[u].cnt);
            dep[u] = make_uint2(units[u].dlo, units[u].dhi);
        }
        DGSN_TRY(p->d_unit_map[tb].alloc(map.size() * sizeof(uint4)));
        DGSN_TRY(p->d_unit_dep[tb].alloc(dep.size() * sizeof(uint2)));
        DGSN_HIP(hipMemcpy(p->d_unit_map[tb].ptr, map.data(), map.size() * sizeof(uint4),
                           hipMemcpyHostToDevice));
        DGSN_HIP(hipMemcpy(p->d_unit_dep[tb].ptr, dep.data(), dep.size() * sizeof(uint2),
                           hipMemcpyHostToDevice));
        p->flow_units[tb] = (unsigned)map.size();
        umax = std::max(umax, p->flow_units[tb]);
    }
    const size_t words = kFlowDone + 8 * (size_t)umax;
    DGSN_TRY(p->d_flow_sync.alloc(words * sizeof(unsigned)));
    DGSN_HIP(hipMemset(p->d_flow_sync.ptr, 0, words * sizeof(unsigned)));
    p->flow_ready = 1;
    return DGSN_OK;
}

// Event pairs for `pairs` timed launches in the current call (created on
// first need and kept).
int reserve_events(dgsn_problem *p, int pairs)
{
    while ((int)p->ev.size() < 2 * pairs) {
        hipEvent_t e;
        DGSN_HIP(hipEventCreate(&e));
        p->ev.push_back(e);
    }
    return DGSN_OK;
}

template <typename Real>
int run_sweep(dgsn_problem *p, const void *src, bool store_psi, bool adjoint, Real *grad_oct,
              hipStream_t s, bool moments = false)
{
    PlaneArgs<Real> A = plane_args<Real>(p, src, adjoint);
    A.grad_oct = grad_oct;
    A.keep_out = (p->balance && !adjoint) ? 1u : 0u;
    if (moments && p->pl_order > 0) {
        // anisotropic scattering inside source iteration
        A.nmom = (uint32_t)((p->pl_order + 1) * (p->pl_order + 1));
        A.ylm = static_cast<const Real *>(p->d_ylm.ptr);
        A.msrc = static_cast<const Real *>(p->msrc.ptr);
        A.mom_oct = static_cast<Real *>(p->mom_oct.ptr);
    }
    const bool anyann = p->solver == DGSN_ANN && !adjoint;
    if (anyann) {
        if (!p->ann) return set_error(DGSN_EINVAL, "solver is DGSN_ANN but no ANN is attached");
        if (store_psi)
            return set_error(DGSN_EUNSUPPORTED, "store_psi is not available with the ANN solver");
    }
    // the matrix-core network (version 1) has its own kernel; the paper-form
    // networks (version 2 per octant, 3 per direction) run inside the GE
    // kernels as another local solver
    const bool paper = anyann && p->ann->version >= 2;
    const bool ann = anyann && !paper;
    if (ann) A.ann_params = ann_device_params(p->ann);
    if (paper) A.ann_params = p->d_pann.ptr;
    const bool split = ann && p->ann->mode == DGSN_ANN_BF16X2;
    const int form = paper ? (p->ann->version == 3 ? kFormAnnPaperDir : kFormAnnPaper)
                           : ann ? (split ? kFormAnnSplit : kFormAnn)
                                 : (p->solver == DGSN_GE_DENSE ? kFormDense : kFormMassInv);
    // anisotropic sweeps use tiles of edge 2 at most (larger tiles spill)
    int tb = (A.nmom > 1 && p->tile_b > 2) ? 2 : p->tile_b;
    // the balance tally reads each row's boundary outflow from the fronts,
    // which only a tile's last cell writes: on a mesh that the tile edge
    // does not divide, the tallied sweep runs single cells (the cell
    // arithmetic is the same for every tiling)
    if (A.keep_out && tb > 1 && (p->n[0] % tb || p->n[1] % tb || p->n[2] % tb)) tb = 1;
    const bool tiled = tb > 1;
    const uint32_t *cells = static_cast<const uint32_t *>(tiled ? p->d_tiles[tb].ptr
                                                               : p->d_plane_cells.ptr);
    const std::vector<int> &off = tiled ? p->tplane_off[tb] : p->plane_off;
    const int nsteps = tiled ? p->n_tplanes[tb] : p->n_planes;
    p->last_stream = s;
    if (p->debug & DGSN_DEBUG_POISON_FRONTS) {
        // a sweep reads a front slot only after its upstream cell wrote it in
        // this sweep: poisoned, any other read turns the flux into NaN
        DGSN_TRY(launch_fill_nan<Real>(8ll * A.fx_o, A.fx, s));
        DGSN_TRY(launch_fill_nan<Real>(8ll * A.fy_o, A.fy, s));
        DGSN_TRY(launch_fill_nan<Real>(8ll * A.fz_o, A.fz, s));
    }
    if (p->timing) DGSN_TRY(reserve_events(p, p->ev_used + nsteps));
    if (p->schedule == DGSN_SCHED_DATAFLOW) {
        DGSN_TRY(flow_prepare(p));
        FlowArgs F{};
        F.unit_map = static_cast<const uint4 *>(p->d_unit_map[tb].ptr);
        F.unit_dep = static_cast<const uint2 *>(p->d_unit_dep[tb].ptr);
        F.sync = static_cast<unsigned *>(p->d_flow_sync.ptr);
        F.units_o = p->flow_units[tb];
        F.spin_limit = p->flow_spin ? p->flow_spin : kFlowSpinDefault;
        A.cells = cells;
        A.ncp = off[nsteps];
        DGSN_TRY(launch_flow_reset(F, s));
        const int e0 = p->ev_used;
        if (p->timing) DGSN_HIP(hipEventRecord(p->ev[2 * e0], s));
        DGSN_TRY(launch_flow<Real>(A, F, form, tb, store_psi, adjoint, s));
        if (p->timing) {
            DGSN_HIP(hipEventRecord(p->ev[2 * e0 + 1], s));
            p->ev_used = e0 + 1;
        }
        return DGSN_OK;
    }
    const int e0 = p->ev_used;
    for (int pl = 0; pl < nsteps; ++pl) {
        A.cells = cells + off[pl];
        A.ncp = off[pl + 1] - off[pl];
        if (p->timing) DGSN_HIP(hipEventRecord(p->ev[2 * (e0 + pl)], s));
        bool done = false;
        if constexpr (sizeof(Real) == 4) {
            if (ann) {
                DGSN_TRY(launch_tile_ann(A, tb, split, s));
                done = true;
            }
        }
        if (!done) DGSN_TRY(launch_tile<Real>(A, form, tb, store_psi, adjoint, s));
        if (p->timing) {
            DGSN_HIP(hipEventRecord(p->ev[2 * (e0 + pl) + 1], s));
            p->ev_used = e0 + pl + 1;
        }
    }
    return DGSN_OK;
}

template <typename Real>
ReduceArgs<Real> reduce_args(dgsn_problem *p, void *phi)
{
    ReduceArgs<Real> R{};
    R.phi_oct = static_cast<const Real *>(p->phi_oct.ptr);
    R.phi = static_cast<Real *>(phi);
    R.nv = (long long)p->G * p->ncell;
    R.partials = static_cast<double *>(p->red_partials.ptr);
    R.result = static_cast<double *>(p->red_result.ptr);
    return R;
}

// The balance tally of a forward sweep with source src: the boundary
// leakage partials (from the fronts the sweep just left) and the absorption
// and source partials of the reduction R, plus the host-side inflow and
// weight sum of the sweep's direction table.  Enqueued between the sweep and
// launch_reduce(R).
template <typename Real>
int balance_prepare(dgsn_problem *p, const void *src, ReduceArgs<Real> &R, hipStream_t s)
{
    PlaneArgs<Real> A = plane_args<Real>(p, src, false);
    DGSN_TRY(launch_leakage<Real>(A, R.partials, p->red_blocks, s));
    R.balance = 1;
    R.sigma_t = static_cast<const Real *>(p->sigma_t.ptr);
    R.src_sweep = static_cast<const Real *>(src);
    // inflow through the boundary faces entering each direction: w kappa_a V
    // psi_inc per boundary cell face, with the values as the sweep used them
    // (rounded to the problem precision)
    double inflow = 0.0, wsum = 0.0;
    const double cells_on_face[3] = {(double)p->n[1] * p->n[2], (double)p->n[0] * p->n[2],
                                     (double)p->n[0] * p->n[1]};
    for (int o = 0; o < 8; ++o)
        for (int d = 0; d < p->Do; ++d) {
            const double *e = &p->dir_host[(size_t)(o * p->Do + d) * kDirStride];
            const double w = (double)(Real)e[kDirW];
            wsum += w;
            for (int a = 0; a < 3; ++a)
                inflow += w * (double)(Real)e[kDirK + a] * (double)A.inc[o][a] * cells_on_face[a];
        }
    p->bal_inflow = inflow * p->G * (p->h[0] * p->h[1] * p->h[2]);
    p->bal_wsum = wsum;
    return DGSN_OK;
}

// Reads the dataflow error word (stream-ordered) and clears it; fails if a
// wait of a dataflow launch gave up.
int check_flow(dgsn_problem *p, hipStream_t s)
{
    if (!p->flow_ready) return DGSN_OK;
    unsigned err = 0;
    DGSN_HIP(hipMemcpyAsync(&err, static_cast<unsigned *>(p->d_flow_sync.ptr) + kFlowError,
                            sizeof(err), hipMemcpyDeviceToHost, s));
    DGSN_HIP(hipStreamSynchronize(s));
    if (err == 0u) return DGSN_OK;
    DGSN_HIP(hipMemsetAsync(p->d_flow_sync.ptr, 0, p->d_flow_sync.bytes, s));
    DGSN_HIP(hipStreamSynchronize(s));
    return set_error(DGSN_ETIMEOUT, "a dataflow sweep wait expired (poll limit %u); its results "
                     "are invalid", p->flow_spin ? p->flow_spin : kFlowSpinDefault);
}

// Residual r and eps_S from an iteration's FP64 result slot; DGSN_EINVAL if
// any of them is not finite (a NaN or infinite flux), which the NaN-carrying
// maxima of the reduction bring here.
int residual_of(const double *res, long long nv, double &r, double &es)
{
    if (!std::isfinite(res[kRedMaxD]) || !std::isfinite(res[kRedMaxF]) ||
        !std::isfinite(res[kRedEps]) || !(res[kRedMaxF] >= 0.0))
        return set_error(DGSN_EINVAL, "the iteration produced a non-finite flux or residual");
    r = res[kRedMaxF] > 0.0 ? res[kRedMaxD] / res[kRedMaxF] : 0.0;
    es = res[kRedEps] / (double)nv;
    return DGSN_OK;
}

template <typename Real>
int sweep_impl(dgsn_problem *p, const void *src, void *phi, hipStream_t s)
{
    p->touch(false);
    p->bal_state = 0;
    DGSN_TRY(run_sweep<Real>(p, src, p->store_psi != 0, false, nullptr, s));
    ReduceArgs<Real> R = reduce_args<Real>(p, phi);
    // a single sweep's tally has a result slot of its own (the two others
    // belong to the iterations in flight of source and adjoint iterations)
    R.result = static_cast<double *>(p->red_result.ptr) + 2 * kRedStride;
    if (p->balance) DGSN_TRY(balance_prepare<Real>(p, src, R, s));
    DGSN_TRY(launch_reduce<Real>(R, p->red_blocks, s));
    if (p->balance) p->bal_state = 1;
    return DGSN_OK;
}

// Anisotropic moments after a sweep's octant reduction: the flux moments,
// and the source moments of the next sweep -- sigma_{s,n} times the moment
// in-group (fused), or the group sum through the per-order matrices
// (transposed in the adjoint).
template <typename Real>
int moment_sources(dgsn_problem *p, bool adjoint, hipStream_t s)
{
    const long long nv = (long long)p->G * p->ncell;
    const int nm = (p->pl_order + 1) * (p->pl_order + 1);
    const Real *sn = static_cast<const Real *>(p->sigma_sn.ptr);
    Real *mom = static_cast<Real *>(p->mom.ptr);
    Real *msrc = static_cast<Real *>(p->msrc.ptr);
    DGSN_TRY(launch_reduce_moments<Real>(nv, nm, static_cast<const Real *>(p->mom_oct.ptr),
                                         p->pl_gg ? nullptr : sn, mom, p->pl_gg ? nullptr : msrc,
                                         s));
    if (p->pl_gg)
        DGSN_TRY(launch_build_msrc_gg<Real>(p->ncell, p->G, nm, sn, mom, msrc, adjoint, s));
    return DGSN_OK;
}

// Scratch of a source iteration that may not allocate: partials [2048][8],
// result slots [2][8] and the look-ahead iterate, all in the static array.
struct NoAllocScratch {
    double *partials;
    double *results;
    void *iterate;
    size_t iterate_bytes;
};

template <typename Real>
int source_iterate_impl(dgsn_problem *p, void *phi, double tol, int max_iter, int *iters,
                        double *resid, double *eps_s, hipStream_t s,
                        const NoAllocScratch *na = nullptr)
{
    const long long nv = (long long)p->G * p->ncell;
    Real *src = static_cast<Real *>(p->src.ptr);
    const bool pl = p->pl_order > 0;
    if (pl && p->solver == DGSN_ANN)
        return set_error(DGSN_EUNSUPPORTED,
                         "anisotropic scattering is available with the GE solvers");
    if (pl && p->store_psi && p->solver == DGSN_GE_DENSE)
        return set_error(DGSN_EUNSUPPORTED, "anisotropic scattering stores the angular flux "
                         "with the mass-inverse GE solver");
    // in-group scattering: the next source is fused into the octant
    // reduction; with a multigroup matrix it is built after it from all groups
    const Real *gg = static_cast<const Real *>(p->sigma_gg.ptr);
    if (gg)
        DGSN_TRY(launch_build_source_gg<Real>(p->ncell, p->G, static_cast<const Real *>(p->q.ptr),
                                              nullptr, gg, static_cast<const Real *>(phi), src,
                                              false, s));
    else
        DGSN_TRY(launch_build_source<Real>(nv, static_cast<const Real *>(p->q.ptr),
                                           static_cast<const Real *>(p->sigma_s.ptr),
                                           static_cast<const Real *>(phi), src, s));
    if (pl) {
        // the anisotropic moments start from zero
        DGSN_HIP(hipMemsetAsync(p->msrc.ptr, 0, p->msrc.bytes, s));
        DGSN_HIP(hipMemsetAsync(p->mom.ptr, 0, p->mom.bytes, s));
    }
    // Pipelined iteration: the sweep of iteration k+1 is enqueued before the
    // host reads iteration k's residual, so the GPU does not idle during the
    // readback.  The iterates alternate between the caller's buffer and an
    // internal one; if iteration k stops the loop, the extra iteration's
    // outputs are discarded (its sweep's side outputs -- a stored psi, the
    // anisotropic moments -- would not match the returned iterate, so those
    // modes iterate without the overlap).  Results are identical either way.
    const bool overlap = !p->store_psi && !pl;
    Real *buf[2] = {static_cast<Real *>(phi), nullptr};
    if (overlap && na) {
        if ((size_t)nv * 8 * sizeof(Real) > na->iterate_bytes)
            return set_error(DGSN_EINVAL, "the iterate (%zu bytes) exceeds the no-allocation "
                             "scratch limit of %zu bytes", (size_t)nv * 8 * sizeof(Real),
                             na->iterate_bytes);
        buf[1] = static_cast<Real *>(na->iterate);
    } else if (overlap) {
        if (p->phi_alt.bytes != (size_t)nv * 8 * sizeof(Real))
            DGSN_TRY(p->phi_alt.alloc((size_t)nv * 8 * sizeof(Real)));
        buf[1] = static_cast<Real *>(p->phi_alt.ptr);
    }
    double *dres = na ? na->results : static_cast<double *>(p->red_result.ptr);
    double *hres = static_cast<double *>(p->h_result.ptr);
    unsigned *herr = reinterpret_cast<unsigned *>(hres + 2 * kRedStride);
    const bool flow = p->schedule == DGSN_SCHED_DATAFLOW;
    auto enqueue = [&](int k) -> int {
        const int slot = k & 1;
        DGSN_TRY(run_sweep<Real>(p, src, p->store_psi != 0, false, nullptr, s, pl));
        ReduceArgs<Real> R = reduce_args<Real>(p, buf[0]);
        R.resid = 1;
        if (na) R.partials = na->partials;
        if (overlap) {
            R.phi_prev = buf[slot];
            R.phi = buf[slot ^ 1];
        }
        R.result = dres + kRedStride * slot;
        if (p->balance) DGSN_TRY(balance_prepare<Real>(p, src, R, s));
        if (!gg) {
            R.src_next = src;
            R.q_cell = static_cast<const Real *>(p->q.ptr);
            R.sigma_s = static_cast<const Real *>(p->sigma_s.ptr);
        }
        DGSN_TRY(launch_reduce<Real>(R, p->red_blocks, s));
        if (pl) DGSN_TRY(moment_sources<Real>(p, false, s));
        if (gg)
            DGSN_TRY(launch_build_source_gg<Real>(p->ncell, p->G,
                                                  static_cast<const Real *>(p->q.ptr), nullptr,
                                                  gg, R.phi, src, false, s));
        DGSN_HIP(hipMemcpyAsync(hres + kRedStride * slot, dres + kRedStride * slot,
                                kRedStride * sizeof(double), hipMemcpyDeviceToHost, s));
        if (flow)
            DGSN_HIP(hipMemcpyAsync(herr + slot,
                                    static_cast<unsigned *>(p->d_flow_sync.ptr) + kFlowError,
                                    sizeof(unsigned), hipMemcpyDeviceToHost, s));
        DGSN_HIP(hipEventRecord(p->ev_result[slot], s));
        return DGSN_OK;
    };
    p->touch(false);
    p->bal_state = 0;
    double r = INFINITY, es = INFINITY, best = INFINITY, crit = INFINITY;
    int it = 0, stall = 0;
    const bool fp32 = p->precision == DGSN_FP32;
    const bool fixed = p->si_criterion == DGSN_SI_FIXED;
    p->si_resid.clear();
    p->si_eps.clear();
    DGSN_TRY(enqueue(0));
    for (int k = 0;; ++k) {
        const bool ahead = overlap && k + 1 < max_iter;
        if (ahead) DGSN_TRY(enqueue(k + 1));
        DGSN_HIP(hipEventSynchronize(p->ev_result[k & 1]));
        if (flow && herr[k & 1] != 0u) {
            DGSN_HIP(hipStreamSynchronize(s));
            DGSN_HIP(hipMemsetAsync(p->d_flow_sync.ptr, 0, p->d_flow_sync.bytes, s));
            DGSN_HIP(hipStreamSynchronize(s));
            return set_error(DGSN_ETIMEOUT, "a dataflow sweep wait expired (poll limit %u); its "
                             "results are invalid", p->flow_spin ? p->flow_spin : kFlowSpinDefault);
        }
        const double *res = hres + kRedStride * (k & 1);
        it = k + 1;
        if (residual_of(res, nv, r, es) != DGSN_OK) {
            DGSN_HIP(hipStreamSynchronize(s));
            return set_error(DGSN_EINVAL, "source iteration %d produced a non-finite flux or "
                             "residual", it);
        }
        // without allocation the history keeps what its reserved capacity holds
        if (!na || p->si_resid.size() < p->si_resid.capacity()) {
            p->si_resid.push_back(r);
            p->si_eps.push_back(es);
        }
        crit = p->si_criterion == DGSN_SI_EPS_S ? es : r;
        bool stop = it >= max_iter;
        if (!fixed) {
            if (crit < tol) stop = true;
            if (fp32) {
                if (crit < best) { best = crit; stall = 0; }
                else if (++stall >= 5) stop = true;
            }
        }
        if (stop) {
            // iterate `it` is in buf[it & 1] (overlap) or in place
            if (overlap && (it & 1))
                DGSN_HIP(hipMemcpyAsync(phi, buf[1], (size_t)nv * 8 * sizeof(Real),
                                        hipMemcpyDeviceToDevice, s));
            if (p->balance) {
                std::memcpy(p->bal_host, res, sizeof(p->bal_host));
                p->bal_state = 2;
            }
            break;
        }
        if (!ahead) DGSN_TRY(enqueue(k + 1));
    }
    DGSN_HIP(hipStreamSynchronize(s));
    // the stored angular flux (store_psi) is that of the returned iterate
    p->psi_valid = p->store_psi ? 1 : 0;
    if (iters) *iters = it;
    if (resid) *resid = r;
    if (eps_s) *eps_s = es;
    if (fixed) return DGSN_OK;
    if (!(crit < tol))
        return set_error(DGSN_ENOTCONV, "source iteration stopped after %d sweeps at residual %.3e",
                         it, crit);
    return DGSN_OK;
}

template <typename Real>
int adjoint_impl(dgsn_problem *p, const void *gphi, void *gst, void *gq, double tol, int max_iter,
                 int *iters, hipStream_t s)
{
    const long long nv = (long long)p->G * p->ncell;
    // each buffer checked on its own: a call that failed part way may have
    // left some of them allocated and others released
    if (p->adj_phi.bytes != (size_t)(2 * nv * 8) * p->real_size)
        DGSN_TRY(p->adj_phi.alloc(2 * nv * 8 * p->real_size));   // two adjoint iterates
    if (p->adj_src.bytes != (size_t)(3 * nv * 8) * p->real_size)
        DGSN_TRY(p->adj_src.alloc(3 * nv * 8 * p->real_size));   // load and two sources
    if (p->grad_oct.bytes != (size_t)(8 * nv * 2) * p->real_size)
        DGSN_TRY(p->grad_oct.alloc(8 * nv * 2 * p->real_size));
    Real *phid[2] = {static_cast<Real *>(p->adj_phi.ptr),
                     static_cast<Real *>(p->adj_phi.ptr) + nv * 8};
    Real *load = static_cast<Real *>(p->adj_src.ptr);
    Real *asrc[2] = {load + nv * 8, load + 2 * nv * 8};
    const double vol = p->h[0] * p->h[1] * p->h[2];
    DGSN_TRY(launch_adjoint_load<Real>(nv, static_cast<const Real *>(gphi), vol, load, s));
    DGSN_HIP(hipMemsetAsync(phid[0], 0, nv * 8 * sizeof(Real), s));
    DGSN_HIP(hipMemcpyAsync(asrc[0], load, nv * 8 * sizeof(Real), hipMemcpyDeviceToDevice, s));
    // adjoint source load + sigma_s^T phi_dag / (4 pi): fused in-group, or
    // the transposed multigroup coupling after the reduction
    const Real *gg = static_cast<const Real *>(p->sigma_gg.ptr);
    // anisotropic scattering: the moments of the adjoint flux, from zero
    const bool pl = p->pl_order > 0;
    if (pl) {
        DGSN_HIP(hipMemsetAsync(p->msrc.ptr, 0, p->msrc.bytes, s));
        DGSN_HIP(hipMemsetAsync(p->mom.ptr, 0, p->mom.bytes, s));
    }
    // Iteration k sweeps with asrc[k & 1] and reduces phid[k & 1] ->
    // phid[(k + 1) & 1], writing the next source into asrc[(k + 1) & 1];
    // as in source iteration, iteration k+1 is enqueued before the host
    // reads iteration k's residual (serially with anisotropic scattering,
    // whose moments are a single buffer).  A discarded look-ahead iteration
    // touches neither the final iterate nor the source of the contraction
    // sweep.
    const bool overlap = !pl;
    double *dres = static_cast<double *>(p->red_result.ptr);
    double *hres = static_cast<double *>(p->h_result.ptr);
    unsigned *herr = reinterpret_cast<unsigned *>(hres + 2 * kRedStride);
    const bool flow = p->schedule == DGSN_SCHED_DATAFLOW;
    auto enqueue = [&](int k) -> int {
        const int slot = k & 1;
        DGSN_TRY(run_sweep<Real>(p, asrc[slot], false, true, nullptr, s, pl));
        ReduceArgs<Real> R = reduce_args<Real>(p, phid[slot ^ 1]);
        R.resid = 1;
        R.phi_prev = phid[slot];
        R.result = dres + kRedStride * slot;
        if (!gg) {
            R.src_next = asrc[slot ^ 1];
            R.q_nodal = load;
            R.sigma_s = static_cast<const Real *>(p->sigma_s.ptr);
        }
        DGSN_TRY(launch_reduce<Real>(R, p->red_blocks, s));
        if (pl) DGSN_TRY(moment_sources<Real>(p, true, s));
        if (gg)
            DGSN_TRY(launch_build_source_gg<Real>(p->ncell, p->G, nullptr, load, gg,
                                                  phid[slot ^ 1], asrc[slot ^ 1], true, s));
        DGSN_HIP(hipMemcpyAsync(hres + kRedStride * slot, dres + kRedStride * slot,
                                kRedStride * sizeof(double), hipMemcpyDeviceToHost, s));
        if (flow)
            DGSN_HIP(hipMemcpyAsync(herr + slot,
                                    static_cast<unsigned *>(p->d_flow_sync.ptr) + kFlowError,
                                    sizeof(unsigned), hipMemcpyDeviceToHost, s));
        DGSN_HIP(hipEventRecord(p->ev_result[slot], s));
        return DGSN_OK;
    };
    double r = INFINITY, best = INFINITY;
    int it = 0, stall = 0;
    const bool fp32 = p->precision == DGSN_FP32;
    DGSN_TRY(enqueue(0));
    for (int k = 0;; ++k) {
        const bool ahead = overlap && k + 1 < max_iter;
        if (ahead) DGSN_TRY(enqueue(k + 1));
        DGSN_HIP(hipEventSynchronize(p->ev_result[k & 1]));
        if (flow && herr[k & 1] != 0u) {
            DGSN_HIP(hipStreamSynchronize(s));
            DGSN_HIP(hipMemsetAsync(p->d_flow_sync.ptr, 0, p->d_flow_sync.bytes, s));
            DGSN_HIP(hipStreamSynchronize(s));
            return set_error(DGSN_ETIMEOUT, "a dataflow sweep wait expired (poll limit %u); its "
                             "results are invalid", p->flow_spin ? p->flow_spin : kFlowSpinDefault);
        }
        const double *res = hres + kRedStride * (k & 1);
        it = k + 1;
        double es_unused = 0.0;
        if (residual_of(res, nv, r, es_unused) != DGSN_OK) {
            DGSN_HIP(hipStreamSynchronize(s));
            return set_error(DGSN_EINVAL, "adjoint iteration %d produced a non-finite flux or "
                             "residual", it);
        }
        bool stop = it >= max_iter || r < tol;
        if (fp32 && !stop) {
            if (r < best) { best = r; stall = 0; }
            else if (++stall >= 5) stop = true;
        }
        if (stop) break;
        if (!ahead) DGSN_TRY(enqueue(k + 1));
    }
    // contraction sweep with the converged adjoint flux's source
    Real *goct = static_cast<Real *>(p->grad_oct.ptr);
    DGSN_TRY(run_sweep<Real>(p, asrc[it & 1], false, true, goct, s, pl));
    DGSN_TRY(launch_reduce_grad<Real>(nv, goct, static_cast<Real *>(gst), static_cast<Real *>(gq),
                                      s));
    DGSN_HIP(hipStreamSynchronize(s));
    if (iters) *iters = it;
    if (!(r < tol))
        return set_error(DGSN_ENOTCONV, "adjoint iteration stopped after %d sweeps at %.3e", it, r);
    return DGSN_OK;
}

}  // namespace

dgsn_problem::~dgsn_problem()
{
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev_result)
        if (e) (void)hipEventDestroy(e);
}

namespace dgsn {

PlaneArgs<float> batch_plane_args(dgsn_problem *p, const void *src)
{
    PlaneArgs<float> A = plane_args<float>(p, src, false);
    if (p->solver == DGSN_ANN)
        A.ann_params = p->ann->version >= 2 ? p->d_pann.ptr : ann_device_params(p->ann);
    return A;
}

int batch_reduce(dgsn_problem *p, void *phi, hipStream_t s)
{
    ReduceArgs<float> R = reduce_args<float>(p, phi);
    return launch_reduce<float>(R, p->red_blocks, s);
}

// Time one sweep of the problem with each tile edge on its internal source
// buffer and keep the faster (ties keep 2).  The problem's outputs are not
// touched (only its internal partials and fronts).
// Autotuner cache: the choice for a problem shape, kept for the process and
// saved to / loaded from a file on request.  The key holds what decides the
// timing: the device's architecture and compute-unit count, the mesh, the
// directions per octant, the groups, the precision, the local solver (and
// network form), the anisotropy and the psi store.
namespace {
struct TuneEntry {
    int tile = 2, schedule = DGSN_SCHED_PLANES;
    double ms[2 * kMaxTile] = {};
};
std::map<std::string, TuneEntry> g_tune;
std::mutex g_tune_mu;

std::string tune_key(const dgsn_problem *p)
{
    int ver = 0, mode = 0;
    if (p->solver == DGSN_ANN && p->ann) {
        ver = p->ann->version;
        mode = p->ann->mode;
    }
    char buf[256];
    std::snprintf(buf, sizeof(buf), "gfx950/%dcu|%dx%dx%d|Do%d|G%d|%s|solver%d|ann%d.%d|L%d%s|psi%d",
                  p->ctx->num_cu, p->n[0], p->n[1], p->n[2], p->Do, p->G,
                  p->precision == DGSN_FP64 ? "fp64" : "fp32", p->solver, ver, mode, p->pl_order,
                  p->pl_gg ? "gg" : "", p->store_psi);
    return buf;
}

bool tune_lookup(const std::string &key, TuneEntry &out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    out = it->second;
    return true;
}

void tune_store(const std::string &key, const TuneEntry &e)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = e;
}
}  // namespace

int autotune_problem(dgsn_problem *p, hipStream_t s, double ms_out[2 * kMaxTile])
{
    if (p->solver == DGSN_ANN && !p->ann) return set_error(DGSN_EINVAL, "no ANN attached");
    hipEvent_t e0, e1;
    DGSN_HIP(hipEventCreate(&e0));
    DGSN_HIP(hipEventCreate(&e1));
    const int saved_timing = p->timing;
    p->timing = 0;
    // candidates: every tile edge with the hyperplane schedule, and with the
    // dataflow schedule where its tables can be built
    const int nsched = flow_prepare(p) != DGSN_OK ? 1 : 2;
    clear_error();
    double best[2][kMaxTile];
    for (int sc = 0; sc < 2; ++sc)
        for (int b = 0; b < kMaxTile; ++b) best[sc][b] = INFINITY;
    int rc = DGSN_OK;
    for (int sc = 0; sc < nsched && rc == DGSN_OK; ++sc)
        for (int b = 1; b <= kMaxTile && rc == DGSN_OK; ++b) {
            p->tile_b = b;
            p->schedule = sc;
            for (int rep = 0; rep < 3 && rc == DGSN_OK; ++rep) {
                (void)hipEventRecord(e0, s);
                rc = p->precision == DGSN_FP64
                         ? run_sweep<double>(p, p->src.ptr, false, false, nullptr, s)
                         : run_sweep<float>(p, p->src.ptr, false, false, nullptr, s);
                (void)hipEventRecord(e1, s);
                if (hipEventSynchronize(e1) != hipSuccess)
                    rc = set_error(DGSN_EHIP, "timing failed");
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) best[sc][b - 1] = std::min(best[sc][b - 1], (double)ms);
            }
            if (rc == DGSN_OK && sc == DGSN_SCHED_DATAFLOW) rc = check_flow(p, s);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->timing = saved_timing;
    int bi = 1, si = 0;
    for (int sc = 0; sc < nsched; ++sc)
        for (int b = 1; b <= kMaxTile; ++b)
            if (best[sc][b - 1] < best[si][bi - 1]) {
                bi = b;
                si = sc;
            }
    p->tile_b = bi;
    p->schedule = si;
    for (int sc = 0; sc < 2; ++sc)
        for (int b = 0; b < kMaxTile; ++b) ms_out[sc * kMaxTile + b] = best[sc][b];
    return rc;
}

}  // namespace dgsn

extern "C" {

int dgsn_version(void) { return 10000; }

int dgsn_problem_autotune(dgsn_problem *p, void *stream, int *tile, int *schedule,
                          double *ms)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    DGSN_HIP(hipSetDevice(p->ctx->device));
    double t[2 * kMaxTile];
    const std::string key = tune_key(p);
    TuneEntry hit;
    if (tune_lookup(key, hit)) {
        // a problem of the same shape was timed before in this process (or
        // loaded from a cache file): take its choice
        if (hit.schedule == DGSN_SCHED_DATAFLOW) DGSN_TRY(flow_prepare(p));
        p->tile_b = hit.tile;
        p->schedule = hit.schedule;
        for (int b = 0; b < 2 * kMaxTile; ++b) t[b] = hit.ms[b];
    } else {
        DGSN_TRY(autotune_problem(p, as_stream(stream), t));
        TuneEntry e;
        e.tile = p->tile_b;
        e.schedule = p->schedule;
        for (int b = 0; b < 2 * kMaxTile; ++b) e.ms[b] = t[b];
        tune_store(key, e);
    }
    if (tile) *tile = p->tile_b;
    if (schedule) *schedule = p->schedule;
    if (ms)
        for (int b = 0; b < 2 * kMaxTile; ++b) ms[b] = t[b];
    return DGSN_OK;
}

int dgsn_autotune_cache_clear(void)
{
    clear_error();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return DGSN_OK;
}

int dgsn_autotune_cache_size(int *n)
{
    clear_error();
    if (!n) return set_error(DGSN_EINVAL, "n is NULL");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *n = (int)g_tune.size();
    return DGSN_OK;
}

int dgsn_autotune_cache_save(const char *path)
{
    clear_error();
    if (!path) return set_error(DGSN_EINVAL, "path is NULL");
    FILE *f = std::fopen(path, "w");
    if (!f) return set_error(DGSN_EINVAL, "cannot write %s", path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    // one entry per line (a JSON document that the loader reads line by line)
    std::fprintf(f, "{\"dgsn_autotune_cache\": 1, \"entries\": [\n");
    size_t k = 0;
    for (const auto &kv : g_tune) {
        std::fprintf(f, "  {\"key\": \"%s\", \"tile\": %d, \"schedule\": %d, \"ms\": [",
                     kv.first.c_str(), kv.second.tile, kv.second.schedule);
        for (int b = 0; b < 2 * kMaxTile; ++b)
            std::fprintf(f, "%s%.17g", b ? ", " : "",
                         std::isfinite(kv.second.ms[b]) ? kv.second.ms[b] : -1.0);
        std::fprintf(f, "]}%s\n", ++k < g_tune.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? DGSN_OK : set_error(DGSN_EHIP, "writing %s failed", path);
}

int dgsn_autotune_cache_load(const char *path)
{
    clear_error();
    if (!path) return set_error(DGSN_EINVAL, "path is NULL");
    FILE *f = std::fopen(path, "r");
    if (!f) return set_error(DGSN_EINVAL, "cannot open %s", path);
    std::vector<std::pair<std::string, TuneEntry>> got;
    char line[1024];
    bool header = false;
    int rc = DGSN_OK;
    while (std::fgets(line, sizeof(line), f)) {
        if (std::strstr(line, "\"dgsn_autotune_cache\": 1")) header = true;
        const char *k = std::strstr(line, "{\"key\": \"");
        if (!k) continue;
        k += 9;
        const char *ke = std::strchr(k, '"');
        TuneEntry e;
        double m[2 * kMaxTile];
        if (!ke || ke - k >= 512 ||
            std::sscanf(ke, "\", \"tile\": %d, \"schedule\": %d, \"ms\": [%lf, %lf, %lf, %lf, %lf, %lf]",
                        &e.tile, &e.schedule, &m[0], &m[1], &m[2], &m[3], &m[4], &m[5]) != 8 ||
            e.tile < 1 || e.tile > kMaxTile ||
            (e.schedule != DGSN_SCHED_PLANES && e.schedule != DGSN_SCHED_DATAFLOW)) {
            rc = set_error(DGSN_EFORMAT, "%s: malformed autotune cache entry", path);
            break;
        }
        for (int b = 0; b < 2 * kMaxTile; ++b) e.ms[b] = m[b] < 0.0 ? INFINITY : m[b];
        got.emplace_back(std::string(k, ke), e);
    }
    std::fclose(f);
    if (rc == DGSN_OK && !header)
        rc = set_error(DGSN_EFORMAT, "%s: not an autotune cache", path);
    if (rc != DGSN_OK) return rc;
    for (const auto &kv : got) tune_store(kv.first, kv.second);
    return DGSN_OK;
}

int dgsn_problem_set_debug(dgsn_problem *p, int flags)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    if (flags & ~DGSN_DEBUG_POISON_FRONTS) return set_error(DGSN_EINVAL, "unknown debug flags");
    p->debug = flags;
    return DGSN_OK;
}

int dgsn_problem_set_schedule(dgsn_problem *p, int schedule, unsigned poll_limit)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    if (schedule != DGSN_SCHED_PLANES && schedule != DGSN_SCHED_DATAFLOW)
        return set_error(DGSN_EINVAL, "unknown schedule %d", schedule);
    if (schedule == DGSN_SCHED_DATAFLOW) {
        DGSN_HIP(hipSetDevice(p->ctx->device));
        DGSN_TRY(flow_prepare(p));
    }
    p->schedule = schedule;
    p->flow_spin = poll_limit;
    return DGSN_OK;
}

int dgsn_problem_get_schedule(const dgsn_problem *p, int *schedule)
{
    clear_error();
    if (!p || !schedule) return set_error(DGSN_EINVAL, "problem and schedule must be set");
    *schedule = p->schedule;
    return DGSN_OK;
}

int dgsn_problem_check(dgsn_problem *p, void *stream)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    DGSN_HIP(hipSetDevice(p->ctx->device));
    return check_flow(p, as_stream(stream));
}

const char *dgsn_last_error(void) { return dgsn::g_msg; }

int dgsn_ctx_create(int hip_device, dgsn_ctx **out)
{
    clear_error();
    if (!out) return set_error(DGSN_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    DGSN_HIP(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev)
        return set_error(DGSN_EINVAL, "device %d out of range (%d devices)", hip_device, ndev);
    DGSN_HIP(hipSetDevice(hip_device));
    hipDeviceProp_t prop;
    DGSN_HIP(hipGetDeviceProperties(&prop, hip_device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(DGSN_EUNSUPPORTED, "libdgsn is built for gfx950, device is %s",
                         prop.gcnArchName);
    void *scr = nullptr;
    DGSN_TRY(static_scratch_of(hip_device, &scr));
    dgsn_ctx *c = new (std::nothrow) dgsn_ctx();
    if (!c) return set_error(DGSN_ENOMEM, "host allocation failed");
    c->device = hip_device;
    c->num_cu = prop.multiProcessorCount;
    c->static_scratch = scr;
    *out = c;
    return DGSN_OK;
}

int dgsn_ctx_destroy(dgsn_ctx *ctx)
{
    clear_error();
    delete ctx;
    return DGSN_OK;
}

int dgsn_quadrature_ls(int order, double *omega, double *weight, int *n_inout)
{
    clear_error();
    if (!n_inout) return set_error(DGSN_EINVAL, "n_inout is NULL");
    std::vector<double> om, w;
    DGSN_TRY(level_symmetric(order, om, w));
    const int n = (int)w.size();
    if (omega || weight) {
        if (!omega || !weight) return set_error(DGSN_EINVAL, "omega and weight must both be set");
        if (*n_inout < n)
            return set_error(DGSN_EINVAL, "capacity %d < %d directions", *n_inout, n);
        std::memcpy(omega, om.data(), om.size() * sizeof(double));
        std::memcpy(weight, w.data(), w.size() * sizeof(double));
    }
    *n_inout = n;
    return DGSN_OK;
}

int dgsn_problem_validate(const dgsn_problem_desc *desc)
{
    clear_error();
    return validate_desc(desc);
}

int dgsn_problem_create(dgsn_ctx *ctx, const dgsn_problem_desc *d, dgsn_problem **out)
{
    clear_error();
    if (!out) return set_error(DGSN_EINVAL, "out is NULL");
    *out = nullptr;
    DGSN_TRY(validate_desc(d));
    if (!ctx) return set_error(DGSN_EINVAL, "ctx is NULL");
    DGSN_HIP(hipSetDevice(ctx->device));
    dgsn_problem *p = new (std::nothrow) dgsn_problem();
    if (!p) return set_error(DGSN_ENOMEM, "host allocation failed");
    auto fail = [&](int rc) {
        delete p;
        return rc;
    };
    p->ctx = ctx;
    p->n[0] = d->nx;
    p->n[1] = d->ny;
    p->n[2] = d->nz;
    p->len[0] = d->lx;
    p->len[1] = d->ly;
    p->len[2] = d->lz;
    for (int a = 0; a < 3; ++a) p->h[a] = p->len[a] / p->n[a];
    p->ncell = (long long)d->nx * d->ny * d->nz;
    p->G = d->n_groups;
    p->D = d->n_dirs;
    p->Do = d->n_dirs / 8;
    p->precision = d->precision;
    p->solver = d->solver;
    p->store_psi = d->store_psi ? 1 : 0;
    // 2x2x2 tiles halve the front traffic; they are the faster default in
    // both precisions (the autotuner can revisit)
    p->tile_b = 2;
    p->real_size = d->precision == DGSN_FP64 ? 8 : 4;
    p->si_resid.reserve(kSiHistoryReserve);
    p->si_eps.reserve(kSiHistoryReserve);
    p->n_planes = d->nx + d->ny + d->nz - 2;

    // directions sorted by octant, user order inside an octant
    p->dir_user.assign(p->D, -1);
    p->dir_host.assign((size_t)8 * p->Do * kDirStride, 0.0);
    p->omega_host.assign((size_t)8 * p->Do * 3, 0.0);
    int fill[8] = {0};
    for (int u = 0; u < p->D; ++u) {
        const double *om = d->omega + 3 * u;
        const int o = (om[0] < 0) + 2 * (om[1] < 0) + 4 * (om[2] < 0);
        const int slot = o * p->Do + fill[o]++;
        p->dir_user[slot] = u;
        double kappa[3];
        for (int a = 0; a < 3; ++a) kappa[a] = std::fabs(om[a]) / p->h[a];
        double *e = &p->dir_host[(size_t)slot * kDirStride];
        for (int a = 0; a < 3; ++a) p->omega_host[(size_t)slot * 3 + a] = om[a];
        streaming_matrix(kappa, e);
        for (int a = 0; a < 3; ++a) {
            e[kDirK36 + a] = kappa[a] / 36.0;
            e[kDirK + a] = kappa[a];
        }
        e[kDirW] = d->weight[u];
    }

    // hyperplane schedule in canonical coordinates
    std::vector<uint32_t> cells;
    cells.reserve(p->ncell);
    p->plane_off.assign(p->n_planes + 1, 0);
    for (int pl = 0; pl < p->n_planes; ++pl) {
        p->plane_off[pl] = (int)cells.size();
        for (int k = 0; k < d->nz; ++k)
            for (int j = 0; j < d->ny; ++j) {
                const int i = pl - j - k;
                if (i < 0 || i >= d->nx) continue;
                cells.push_back((uint32_t)i | ((uint32_t)j << 10) | ((uint32_t)k << 20));
            }
    }
    p->plane_off[p->n_planes] = (int)cells.size();

    // B x B x B tile hyperplanes, B = 2 .. kMaxTile
    for (int tb = 2; tb <= kMaxTile; ++tb) {
        const int T[3] = {(d->nx + tb - 1) / tb, (d->ny + tb - 1) / tb, (d->nz + tb - 1) / tb};
        p->n_tplanes[tb] = T[0] + T[1] + T[2] - 2;
        std::vector<uint32_t> tl;
        tl.reserve((size_t)T[0] * T[1] * T[2]);
        p->tplane_off[tb].assign(p->n_tplanes[tb] + 1, 0);
        for (int pl = 0; pl < p->n_tplanes[tb]; ++pl) {
            p->tplane_off[tb][pl] = (int)tl.size();
            for (int k = 0; k < T[2]; ++k)
                for (int j = 0; j < T[1]; ++j) {
                    const int i = pl - j - k;
                    if (i < 0 || i >= T[0]) continue;
                    tl.push_back((uint32_t)i | ((uint32_t)j << 10) | ((uint32_t)k << 20));
                }
        }
        p->tplane_off[tb][p->n_tplanes[tb]] = (int)tl.size();
        int rc2 = p->d_tiles[tb].alloc(tl.size() * sizeof(uint32_t));
        if (rc2) return fail(rc2);
        if (hipMemcpy(p->d_tiles[tb].ptr, tl.data(), tl.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice) != hipSuccess)
            return fail(set_error(DGSN_EHIP, "upload of the tile schedule failed"));
    }

    int rc;
    if ((rc = p->d_plane_cells.alloc(cells.size() * sizeof(uint32_t)))) return fail(rc);
    if (hipMemcpy(p->d_plane_cells.ptr, cells.data(), cells.size() * sizeof(uint32_t),
                  hipMemcpyHostToDevice) != hipSuccess)
        return fail(set_error(DGSN_EHIP, "upload of the hyperplane schedule failed"));
    rc = p->precision == DGSN_FP64 ? upload_real<double>(p->d_dir, p->dir_host)
                                   : upload_real<float>(p->d_dir, p->dir_host);
    if (rc) return fail(rc);

    const size_t rs = p->real_size;
    const long long nv = (long long)p->G * p->ncell;
    const long long DG = (long long)p->Do * p->G;
    // kernels index with 32-bit element offsets: every per-sweep array must
    // hold fewer than 2^31 elements, and a block holds >= 1 (cell) segment
    {
        const long long lim = (1LL << 31) - 1;
        const long long nmax = std::max(std::max(d->nx, d->ny), d->nz);
        if (8 * nv * 8 > lim || 8LL * nmax * nmax * 4 * DG > lim)
            return fail(set_error(DGSN_EUNSUPPORTED,
                                  "problem too large for 32-bit sweep indexing (%lld cells x %d "
                                  "groups x %d directions)", p->ncell, p->G, p->D));
        if (DG > 256)
            return fail(set_error(DGSN_EUNSUPPORTED,
                                  "directions per octant x groups must be <= 256 (got %lld)", DG));
        if (p->Do > 64 || cells_per_block(p->Do, p->G) < 1)
            return fail(set_error(DGSN_EUNSUPPORTED,
                                  "groups must be <= 4 * floor(64 / directions per octant) "
                                  "(got %d groups, %d directions per octant)", p->G, p->Do));
    }
    if ((rc = p->sigma_t.alloc(nv * rs)) || (rc = p->sigma_s.alloc(nv * rs)) ||
        (rc = p->q.alloc(nv * rs)) || (rc = p->src.alloc(nv * 8 * rs)) ||
        (rc = p->phi_oct.alloc(8 * nv * 8 * rs)) ||
        (rc = p->front_x.alloc(8LL * d->nz * d->ny * 4 * DG * rs)) ||
        (rc = p->front_y.alloc(8LL * d->nz * d->nx * 4 * DG * rs)) ||
        (rc = p->front_z.alloc(8LL * d->ny * d->nx * 4 * DG * rs)))
        return fail(rc);
    if (p->store_psi && (rc = p->psi.alloc((size_t)p->D * nv * 8 * rs))) return fail(rc);
    p->red_blocks = reduce_blocks_for(nv);
    if ((rc = p->red_partials.alloc((size_t)p->red_blocks * kRedStride * sizeof(double))) ||
        (rc = p->red_result.alloc(3 * kRedStride * sizeof(double))) ||
        (rc = p->h_result.alloc(2 * kRedStride * sizeof(double) + 2 * sizeof(unsigned))))
        return fail(rc);
    if (hipEventCreateWithFlags(&p->ev_result[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_result[1], hipEventDisableTiming) != hipSuccess)
        return fail(set_error(DGSN_EHIP, "event creation failed"));
    if (hipMemset(p->sigma_t.ptr, 0, nv * rs) != hipSuccess ||
        hipMemset(p->sigma_s.ptr, 0, nv * rs) != hipSuccess ||
        hipMemset(p->q.ptr, 0, nv * rs) != hipSuccess)
        return fail(set_error(DGSN_EHIP, "initialising material buffers failed"));
    *out = p;
    return DGSN_OK;
}

int dgsn_problem_destroy(dgsn_problem *p)
{
    clear_error();
    if (p) {
        (void)hipSetDevice(p->ctx->device);
        delete p;
    }
    return DGSN_OK;
}

int dgsn_problem_set_materials(dgsn_problem *p, const void *sigma_t, const void *sigma_s,
                               const void *q, void *stream)
{
    clear_error();
    if (!p || !sigma_t) return set_error(DGSN_EINVAL, "problem and sigma_t must be set");
    const size_t bytes = (size_t)p->G * p->ncell * p->real_size;
    hipStream_t s = as_stream(stream);
    p->touch(false);
    DGSN_HIP(hipMemcpyAsync(p->sigma_t.ptr, sigma_t, bytes, hipMemcpyDeviceToDevice, s));
    if (sigma_s) DGSN_HIP(hipMemcpyAsync(p->sigma_s.ptr, sigma_s, bytes, hipMemcpyDeviceToDevice, s));
    else DGSN_HIP(hipMemsetAsync(p->sigma_s.ptr, 0, bytes, s));
    if (q) DGSN_HIP(hipMemcpyAsync(p->q.ptr, q, bytes, hipMemcpyDeviceToDevice, s));
    else DGSN_HIP(hipMemsetAsync(p->q.ptr, 0, bytes, s));
    // validity of the copies (waits for the stream)
    if (!p->d_check.ptr) DGSN_TRY(p->d_check.alloc(sizeof(unsigned)));
    DGSN_HIP(hipMemsetAsync(p->d_check.ptr, 0, sizeof(unsigned), s));
    const long long n = (long long)p->G * p->ncell;
    unsigned *flag = static_cast<unsigned *>(p->d_check.ptr);
    if (p->precision == DGSN_FP64)
        DGSN_TRY(launch_check_materials<double>(n, static_cast<const double *>(p->sigma_t.ptr),
                                                static_cast<const double *>(p->sigma_s.ptr),
                                                static_cast<const double *>(p->q.ptr), flag, s));
    else
        DGSN_TRY(launch_check_materials<float>(n, static_cast<const float *>(p->sigma_t.ptr),
                                               static_cast<const float *>(p->sigma_s.ptr),
                                               static_cast<const float *>(p->q.ptr), flag, s));
    unsigned bad = 0;
    DGSN_HIP(hipMemcpyAsync(&bad, flag, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    DGSN_HIP(hipStreamSynchronize(s));
    if (bad)
        return set_error(DGSN_EINVAL, "invalid materials:%s%s%s%s",
                         (bad & 1u) ? " sigma_t negative or not finite;" : "",
                         (bad & 2u) ? " sigma_s negative or not finite;" : "",
                         (bad & 4u) ? " q not finite;" : "",
                         (bad & 8u) ? " sigma_s exceeds sigma_t;" : "");
    return DGSN_OK;
}

namespace {
// dst [ncell][nmat] (problem precision) = the cell-major copy of the
// caller's src [nmat][ncell], on the stream
int cell_major_matrix(const dgsn_problem *p, const void *src, int nmat, void *dst, hipStream_t s)
{
    if (p->precision == DGSN_FP64)
        return launch_cell_major<double>(p->ncell, nmat, static_cast<const double *>(src),
                                         static_cast<double *>(dst), s);
    return launch_cell_major<float>(p->ncell, nmat, static_cast<const float *>(src),
                                    static_cast<float *>(dst), s);
}
}  // namespace

int dgsn_problem_set_scattering(dgsn_problem *p, const void *sigma_gg, void *stream)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    DGSN_HIP(hipSetDevice(p->ctx->device));
    if (!sigma_gg) {
        // the order-0 matrix of group-to-group anisotropic scattering stays
        // with its higher orders (dropping it alone would mix the in-group
        // order 0 with group-to-group orders 1..L)
        if (p->pl_order > 0 && p->pl_gg)
            return set_error(DGSN_EUNSUPPORTED,
                             "group-to-group anisotropic scattering is set; remove its orders "
                             "first (dgsn_problem_set_anisotropy with order 0)");
        p->touch(false);
        p->sigma_gg.release();
        return DGSN_OK;
    }
    p->touch(false);
    if (p->pl_order > 0)
        return set_error(DGSN_EUNSUPPORTED,
                         "anisotropic scattering is set; dgsn_problem_set_anisotropy_gg sets the "
                         "order-0 group-to-group matrix with the higher orders");
    const size_t bytes = (size_t)p->G * p->G * p->ncell * p->real_size;
    if (p->sigma_gg.bytes != bytes) DGSN_TRY(p->sigma_gg.alloc(bytes));
    return cell_major_matrix(p, sigma_gg, p->G * p->G, p->sigma_gg.ptr, as_stream(stream));
}

namespace {
// Harmonics of the slot directions and the moment buffers of order L, with
// room for sbytes of scattering moments (sigma_sn).
int anisotropy_buffers(dgsn_problem *p, int order, size_t sbytes)
{
    const int nm = (order + 1) * (order + 1);
    const size_t nv = (size_t)p->G * p->ncell;
    std::vector<double> y((size_t)8 * p->Do * kYlmStride, 0.0);
    for (int slot = 0; slot < 8 * p->Do; ++slot) {
        double all[kYlmStride];
        real_ylm(order, &p->omega_host[(size_t)slot * 3], all);
        for (int k = 1; k < nm; ++k) y[(size_t)slot * kYlmStride + k - 1] = all[k];
    }
    DGSN_TRY(p->precision == DGSN_FP64 ? upload_real<double>(p->d_ylm, y)
                                       : upload_real<float>(p->d_ylm, y));
    const size_t mbytes = (size_t)(nm - 1) * nv * 8 * p->real_size;
    if (p->mom.bytes != mbytes) DGSN_TRY(p->mom.alloc(mbytes));
    if (p->msrc.bytes != mbytes) DGSN_TRY(p->msrc.alloc(mbytes));
    if (p->mom_oct.bytes != 8 * mbytes) DGSN_TRY(p->mom_oct.alloc(8 * mbytes));
    if (p->sigma_sn.bytes != sbytes) DGSN_TRY(p->sigma_sn.alloc(sbytes));
    return DGSN_OK;
}
}  // namespace

namespace {
// No anisotropic orders: the state after order 0, and after a setter fails
// part way (its buffers may already be gone), so that no later iteration
// reads a released buffer.
void drop_anisotropy(dgsn_problem *p)
{
    p->pl_order = 0;
    p->pl_gg = 0;
    p->sigma_sn.release();
    p->d_ylm.release();
    p->mom_oct.release();
    p->mom.release();
    p->msrc.release();
}

int set_anisotropy_impl(dgsn_problem *p, int order, const void *sigma_sn, hipStream_t s)
{
    const size_t sbytes = (size_t)order * p->G * p->ncell * p->real_size;
    DGSN_TRY(anisotropy_buffers(p, order, sbytes));
    DGSN_HIP(hipMemcpyAsync(p->sigma_sn.ptr, sigma_sn, sbytes, hipMemcpyDeviceToDevice, s));
    DGSN_HIP(hipMemsetAsync(p->mom.ptr, 0, p->mom.bytes, s));
    DGSN_HIP(hipMemsetAsync(p->msrc.ptr, 0, p->msrc.bytes, s));
    p->pl_order = order;
    p->pl_gg = 0;
    return DGSN_OK;
}

int set_anisotropy_gg_impl(dgsn_problem *p, int order, const void *sigma_sn_gg, hipStream_t s)
{
    const size_t mat = (size_t)p->G * p->G * p->ncell * p->real_size;
    DGSN_TRY(anisotropy_buffers(p, order, (size_t)order * mat));
    if (p->sigma_gg.bytes != mat) DGSN_TRY(p->sigma_gg.alloc(mat));
    const char *src = static_cast<const char *>(sigma_sn_gg);
    // cell-major, one G x G matrix per (cell, order) in one run
    DGSN_TRY(cell_major_matrix(p, src, p->G * p->G, p->sigma_gg.ptr, s));
    DGSN_TRY(cell_major_matrix(p, src + mat, order * p->G * p->G, p->sigma_sn.ptr, s));
    DGSN_HIP(hipMemsetAsync(p->mom.ptr, 0, p->mom.bytes, s));
    DGSN_HIP(hipMemsetAsync(p->msrc.ptr, 0, p->msrc.bytes, s));
    p->pl_order = order;
    p->pl_gg = 1;
    return DGSN_OK;
}
}  // namespace

int dgsn_problem_set_anisotropy(dgsn_problem *p, int order, const void *sigma_sn, void *stream)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    if (order < 0 || order > kMaxPlOrder)
        return set_error(DGSN_EINVAL, "scattering order %d is outside 0..%d", order, kMaxPlOrder);
    DGSN_HIP(hipSetDevice(p->ctx->device));
    p->touch(false);
    if (order == 0) {
        drop_anisotropy(p);
        return DGSN_OK;
    }
    if (!sigma_sn) return set_error(DGSN_EINVAL, "sigma_sn is NULL");
    if (p->sigma_gg.ptr)
        return set_error(DGSN_EUNSUPPORTED,
                         "a group-to-group matrix and in-group anisotropic scattering are "
                         "exclusive (dgsn_problem_set_anisotropy_gg sets both)");
    const int rc = set_anisotropy_impl(p, order, sigma_sn, as_stream(stream));
    if (rc != DGSN_OK) drop_anisotropy(p);
    return rc;
}

int dgsn_problem_set_anisotropy_gg(dgsn_problem *p, int order, const void *sigma_sn_gg,
                                   void *stream)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    if (order < 1 || order > kMaxPlOrder)
        return set_error(DGSN_EINVAL, "scattering order %d is outside 1..%d", order, kMaxPlOrder);
    if (!sigma_sn_gg) return set_error(DGSN_EINVAL, "sigma_sn_gg is NULL");
    DGSN_HIP(hipSetDevice(p->ctx->device));
    p->touch(false);
    const int rc = set_anisotropy_gg_impl(p, order, sigma_sn_gg, as_stream(stream));
    if (rc != DGSN_OK) {
        // the order-0 matrix may be released or half copied: drop it too
        drop_anisotropy(p);
        p->sigma_gg.release();
    }
    return rc;
}

int dgsn_problem_get_moments(const dgsn_problem *p, void *mom, void *stream)
{
    clear_error();
    if (!p || !mom) return set_error(DGSN_EINVAL, "problem and mom must be set");
    if (p->pl_order == 0)
        return set_error(DGSN_EINVAL, "the problem has no anisotropic scattering");
    DGSN_HIP(hipSetDevice(p->ctx->device));
    const long long nv = (long long)p->G * p->ncell;
    const int nm = (p->pl_order + 1) * (p->pl_order + 1);
    if (p->precision == DGSN_FP64)
        return launch_moments_public<double>(nv, nm, static_cast<const double *>(p->mom.ptr),
                                             static_cast<double *>(mom), as_stream(stream));
    return launch_moments_public<float>(nv, nm, static_cast<const float *>(p->mom.ptr),
                                        static_cast<float *>(mom), as_stream(stream));
}

int dgsn_real_ylm(int order, const double *omega, int n, double *Y)
{
    clear_error();
    if (order < 0 || order > kMaxPlOrder)
        return set_error(DGSN_EINVAL, "order %d is outside 0..%d", order, kMaxPlOrder);
    if (n < 0 || (n > 0 && (!omega || !Y))) return set_error(DGSN_EINVAL, "bad arguments");
    const int nm = (order + 1) * (order + 1);
    for (int i = 0; i < n; ++i) {
        double all[kYlmStride];
        real_ylm(order, omega + 3 * i, all);
        for (int k = 0; k < nm; ++k) Y[(size_t)i * nm + k] = all[k];
    }
    return DGSN_OK;
}

int dgsn_problem_set_inflow(dgsn_problem *p, const double psi_inc[6])
{
    clear_error();
    if (!p || !psi_inc) return set_error(DGSN_EINVAL, "problem and psi_inc must be set");
    for (int f = 0; f < 6; ++f)
        if (!std::isfinite(psi_inc[f]))
            return set_error(DGSN_EINVAL, "psi_inc[%d] is not finite", f);
    std::memcpy(p->psi_inc, psi_inc, sizeof(p->psi_inc));
    p->touch(true);
    return DGSN_OK;
}

int dgsn_problem_set_ann(dgsn_problem *p, const dgsn_ann *ann)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    if (ann && p->precision != DGSN_FP32)
        return set_error(DGSN_EUNSUPPORTED, "the ANN solver runs on FP32 problems only");
    // a folded paper-form image may be replaced below: batches re-capture
    p->touch(true);
    if (ann && ann->version >= 2) {
        // fold the scaling, the cell sizes and the octant relabelling in once
        // (per octant, or per direction slot)
        std::vector<float> img;
        if (ann->version == 2) {
            DGSN_TRY(pann_problem_image(ann, p->h, img));
        } else {
            if (p->Do > kPannLdsMaxDo)
                return set_error(DGSN_EUNSUPPORTED, "per-direction networks take at most %d "
                                 "directions per octant (the problem has %d)", kPannLdsMaxDo,
                                 p->Do);
            std::vector<int> valid(p->dir_user.size());
            for (size_t k = 0; k < valid.size(); ++k) valid[k] = p->dir_user[k] >= 0;
            DGSN_TRY(pann_problem_image_dir(ann, p->h, p->omega_host.data(), p->Do, valid.data(),
                                            img));
        }
        DGSN_HIP(hipSetDevice(p->ctx->device));
        // past this point a failure leaves no network attached (the folded
        // image of a network attached before may be gone)
        int rc = p->d_pann.alloc(img.size() * sizeof(float));
        if (rc == DGSN_OK) {
            const hipError_t e = hipMemcpy(p->d_pann.ptr, img.data(), img.size() * sizeof(float),
                                           hipMemcpyHostToDevice);
            if (e != hipSuccess)
                rc = set_error(DGSN_EHIP, "hipMemcpy failed: %s", hipGetErrorString(e));
        }
        if (rc != DGSN_OK) {
            p->ann = nullptr;
            p->d_pann.release();
            return rc;
        }
    }
    p->ann = ann;
    return DGSN_OK;
}

int dgsn_problem_set_solver(dgsn_problem *p, int solver)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    if (solver != DGSN_GE && solver != DGSN_ANN && solver != DGSN_GE_DENSE)
        return set_error(DGSN_EINVAL, "solver must be DGSN_GE, DGSN_GE_DENSE or DGSN_ANN");
    if (solver == DGSN_ANN && p->precision != DGSN_FP32)
        return set_error(DGSN_EUNSUPPORTED, "the ANN solver runs on FP32 problems only");
    if (solver != p->solver) p->touch(true);
    p->solver = solver;
    return DGSN_OK;
}

int dgsn_problem_set_tile(dgsn_problem *p, int b)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    if (b < 1 || b > kMaxTile)
        return set_error(DGSN_EINVAL, "tile edge must be in 1..%d", kMaxTile);
    p->tile_b = b;
    return DGSN_OK;
}

int dgsn_problem_get_tile(const dgsn_problem *p, int *b)
{
    clear_error();
    if (!p || !b) return set_error(DGSN_EINVAL, "problem and b must be set");
    *b = p->tile_b;
    return DGSN_OK;
}

int dgsn_problem_set_si_criterion(dgsn_problem *p, int criterion)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    if (criterion != DGSN_SI_MAXNORM && criterion != DGSN_SI_EPS_S && criterion != DGSN_SI_FIXED)
        return set_error(DGSN_EINVAL,
                         "criterion must be DGSN_SI_MAXNORM, DGSN_SI_EPS_S or DGSN_SI_FIXED");
    p->si_criterion = criterion;
    return DGSN_OK;
}

int dgsn_problem_set_timing(dgsn_problem *p, int enable)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    DGSN_HIP(hipSetDevice(p->ctx->device));
    p->timing = enable ? 1 : 0;
    p->ev_used = 0;
    return DGSN_OK;
}

int dgsn_problem_kernel_time(dgsn_problem *p, double *ms_sum, int *launches)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    double total = 0.0;
    if (p->ev_used > 0) {
        DGSN_HIP(hipEventSynchronize(p->ev[2 * p->ev_used - 1]));
        for (int i = 0; i < p->ev_used; ++i) {
            float ms = 0.0f;
            DGSN_HIP(hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]));
            total += ms;
        }
    }
    if (ms_sum) *ms_sum = total;
    if (launches) *launches = p->ev_used;
    return DGSN_OK;
}

int dgsn_problem_stats(const dgsn_problem *p, long long *solves, int *n_planes, double *bytes)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    const long long s = p->ncell * p->D * (long long)p->G;
    if (solves) *solves = s;
    if (n_planes) *n_planes = p->n_planes;
    if (bytes) *bytes = (double)p->real_size * (24.0 * s + 17.0 * p->ncell * p->G);
    return DGSN_OK;
}

int dgsn_problem_generation(const dgsn_problem *p, unsigned long long *gen)
{
    clear_error();
    if (!p || !gen) return set_error(DGSN_EINVAL, "problem and gen must be set");
    *gen = p->gen;
    return DGSN_OK;
}

int dgsn_problem_set_balance(dgsn_problem *p, int enable)
{
    clear_error();
    if (!p) return set_error(DGSN_EINVAL, "problem is NULL");
    p->balance = enable ? 1 : 0;
    p->bal_state = 0;
    return DGSN_OK;
}

int dgsn_problem_balance(dgsn_problem *p, double terms[5], void *stream)
{
    clear_error();
    if (!p || !terms) return set_error(DGSN_EINVAL, "problem and terms must be set");
    double raw[kRedStride];
    if (p->bal_state == 1) {
        DGSN_HIP(hipSetDevice(p->ctx->device));
        hipStream_t s = as_stream(stream);
        DGSN_HIP(hipMemcpyAsync(raw, static_cast<double *>(p->red_result.ptr) + 2 * kRedStride,
                                sizeof(raw), hipMemcpyDeviceToHost, s));
        DGSN_HIP(hipStreamSynchronize(s));
    } else if (p->bal_state == 2) {
        std::memcpy(raw, p->bal_host, sizeof(raw));
    } else {
        return set_error(DGSN_EINVAL, "no tallied sweep (enable the tally with "
                         "dgsn_problem_set_balance before dgsn_sweep or dgsn_source_iterate)");
    }
    const double vol = p->h[0] * p->h[1] * p->h[2];
    terms[0] = 0.25 * vol * raw[kRedLeak];                 // boundary outflow
    terms[1] = p->bal_inflow;                              // boundary inflow
    terms[2] = 0.125 * vol * raw[kRedAbs];                 // absorption sigma_t int phi
    terms[3] = 0.125 * vol * p->bal_wsum * raw[kRedSrc];   // source int sum_d w_d S
    terms[4] = terms[0] - terms[1] + terms[2] - terms[3];
    return DGSN_OK;
}

int dgsn_sweep(dgsn_problem *p, const void *src, void *phi, void *stream)
{
    clear_error();
    if (!p || !src || !phi) return set_error(DGSN_EINVAL, "problem, src and phi must be set");
    if (src == phi) return set_error(DGSN_EINVAL, "src and phi must not overlap");
    DGSN_HIP(hipSetDevice(p->ctx->device));
    p->ev_used = 0;
    return p->precision == DGSN_FP64 ? sweep_impl<double>(p, src, phi, as_stream(stream))
                                     : sweep_impl<float>(p, src, phi, as_stream(stream));
}

int dgsn_source_iterate(dgsn_problem *p, void *phi, double tol, int max_iter, int *iters,
                        double *resid, double *eps_s, void *stream)
{
    clear_error();
    if (!p || !phi) return set_error(DGSN_EINVAL, "problem and phi must be set");
    if (max_iter < 1) return set_error(DGSN_EINVAL, "max_iter must be >= 1");
    if (!(tol >= 0.0)) return set_error(DGSN_EINVAL, "tol must be >= 0");
    DGSN_HIP(hipSetDevice(p->ctx->device));
    p->ev_used = 0;
    return p->precision == DGSN_FP64
               ? source_iterate_impl<double>(p, phi, tol, max_iter, iters, resid, eps_s,
                                             as_stream(stream))
               : source_iterate_impl<float>(p, phi, tol, max_iter, iters, resid, eps_s,
                                            as_stream(stream));
}

int dgsn_source_iterate_noalloc(dgsn_problem *p, void *phi, double tol, int max_iter,
                                int *iters, double *resid, double *eps_s, void *stream)
{
    clear_error();
    if (!p || !phi) return set_error(DGSN_EINVAL, "problem and phi must be set");
    if (max_iter < 1) return set_error(DGSN_EINVAL, "max_iter must be >= 1");
    if (!(tol >= 0.0)) return set_error(DGSN_EINVAL, "tol must be >= 0");
    if (p->timing)
        return set_error(DGSN_EINVAL, "kernel timing records events that may need creating; "
                         "disable it (dgsn_problem_set_timing) for this call");
    if (p->schedule == DGSN_SCHED_DATAFLOW && !p->flow_ready)
        return set_error(DGSN_EINVAL, "the dataflow tables are not built");
    if (p->red_blocks < 1 || (size_t)p->red_blocks * kRedStride * sizeof(double) >
                                 kScratchPartials)
        return set_error(DGSN_EINVAL, "reduction of %d blocks exceeds the scratch partials",
                         p->red_blocks);
    DGSN_HIP(hipSetDevice(p->ctx->device));
    unsigned char *base = static_cast<unsigned char *>(p->ctx->static_scratch);
    if (!base) return set_error(DGSN_EHIP, "no scratch address for device %d", p->ctx->device);
    NoAllocScratch na;
    na.partials = reinterpret_cast<double *>(base);
    na.results = reinterpret_cast<double *>(base + kScratchPartials);
    na.iterate = base + kScratchPartials + kScratchResults;
    na.iterate_bytes = kScratchIterate;
    p->ev_used = 0;
    return p->precision == DGSN_FP64
               ? source_iterate_impl<double>(p, phi, tol, max_iter, iters, resid, eps_s,
                                             as_stream(stream), &na)
               : source_iterate_impl<float>(p, phi, tol, max_iter, iters, resid, eps_s,
                                            as_stream(stream), &na);
}

int dgsn_problem_si_history(const dgsn_problem *p, double *resid, double *eps_s, int cap, int *n)
{
    clear_error();
    if (!p || !n) return set_error(DGSN_EINVAL, "problem and n must be set");
    if (cap < 0) return set_error(DGSN_EINVAL, "cap must be >= 0");
    const int cnt = (int)p->si_resid.size();
    *n = cnt;
    for (int i = 0; i < cnt && i < cap; ++i) {
        if (resid) resid[i] = p->si_resid[i];
        if (eps_s) eps_s[i] = p->si_eps[i];
    }
    return DGSN_OK;
}

int dgsn_adjoint_solve(dgsn_problem *p, const void *gphi, void *gst, void *gq, double tol,
                       int max_iter, int *iters, void *stream)
{
    clear_error();
    if (!p || !gphi) return set_error(DGSN_EINVAL, "problem and dJ_dphi must be set");
    if (!p->store_psi || !p->psi.ptr)
        return set_error(DGSN_EINVAL, "the adjoint needs a problem created with store_psi = 1");
    if (p->solver == DGSN_ANN)
        return set_error(DGSN_EUNSUPPORTED, "the adjoint is defined for the GE solvers");
    if (p->pl_order > 0 && p->solver == DGSN_GE_DENSE)
        return set_error(DGSN_EUNSUPPORTED,
                         "the anisotropic adjoint runs with the mass-inverse GE solver");
    if (max_iter < 1) return set_error(DGSN_EINVAL, "max_iter must be >= 1");
    if (!p->psi_valid)
        return set_error(DGSN_EINVAL, "no stored angular flux of a source iteration on the "
                         "current inputs (run dgsn_source_iterate after the last setter or sweep)");
    DGSN_HIP(hipSetDevice(p->ctx->device));
    p->ev_used = 0;
    return p->precision == DGSN_FP64
               ? adjoint_impl<double>(p, gphi, gst, gq, tol, max_iter, iters, as_stream(stream))
               : adjoint_impl<float>(p, gphi, gst, gq, tol, max_iter, iters, as_stream(stream));
}

}  // extern "C"
