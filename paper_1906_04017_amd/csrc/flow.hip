// Dataflow schedule of the tile sweep (the sweep paragraph after Eq. (T12):
// a cell is solved once its upwind neighbours are known).
//
// The hyperplane schedule issues one launch per tile hyperplane and pays a
// kernel boundary (drain, cache write-back, dispatch) at each of them, and
// every block of a hyperplane waits for the slowest block of the previous
// one.  Here one launch covers the whole sweep and each unit -- a block of
// tiles of one octant in one step -- waits only for the units of the previous
// step that hold the upwind neighbours of its tiles (a short range, computed
// on the host), so consecutive steps overlap.  Workgroup b serves octant
// b & 7 and takes the octant's next unit from its ticket counter, in
// step-major order; eight counters on separate cache lines keep the
// same-address atomics apart.
//
// Progress: a unit waits only on units of its octant with smaller tickets;
// those were taken by workgroups that are already resident, so the oldest
// unfinished unit of every octant can always run and the launch drains.
// Every wait is also bounded (spin_limit polls); a unit whose wait expires
// raises the error word, which makes every other wait give up too, and the
// host reports the error.
//
// Reuse of the in-place fronts is safe: the three face slots a tile reads and
// overwrites are touched only along one upwind chain of tiles, each of which
// waits for the previous one.
//
// Visibility across the XCDs (each has its own L2): the fronts are accessed
// with device-coherent buffer operations in this kernel (see front_load), so
// a producer only waits until its front stores are acknowledged before it
// sets its done flag, and a consumer that has seen the flags reads the fronts
// without a cache invalidation.  The other arrays are read-only during the
// launch or read only by later kernels.
#include <algorithm>

#include "flow.hpp"
#include "sweep_body.hpp"

namespace dgsn {

namespace {

// Wave 0: take a ticket of octant o and wait for the unit's dependencies
// (one flag per lane, up to 64 at a time); sh = the unit's map entry and
// ticket.  The launches of a sweep have exactly 8 * units_o workgroups, so
// every ticket is in range (clamped defensively).
__device__ __forceinline__ void flow_take(const FlowArgs &F, unsigned o, int lane, uint4 *sh)
{
    unsigned t = 0;
    if (lane == 0) t = flow_add(F.sync + kFlowTicket + 32 * o, 1u);
    t = __shfl(t, 0);
    if (t >= F.units_o) t = F.units_o - 1;
    const uint2 dep = F.unit_dep[t];
    flow_wait_range(F.sync + kFlowDone + o * F.units_o, dep.x, dep.y, 1u, lane, F.spin_limit,
                    F.sync + kFlowError);
    if (lane == 0) {
        sh[0] = F.unit_map[t];
        sh[1] = make_uint4(t, 0u, 0u, 0u);
    }
}

// Every thread: publish this unit's fronts and flag it done.
__device__ __forceinline__ void flow_finish(const FlowArgs &F, int tid, unsigned o, unsigned t)
{
    __builtin_amdgcn_s_waitcnt(0);   // this wave's coherent front stores are acknowledged
    __syncthreads();
    if (tid == 0) flow_store(F.sync + kFlowDone + o * F.units_o + t, 1u);
}

// Clears the tickets and done counts (not the error word) before a launch.
__global__ __launch_bounds__(256) void flow_reset(unsigned *sync, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (i != kFlowError) sync[i] = 0u;
}

template <typename Real, int Form, int B, bool kStorePsi, bool kAdjoint, int kMom = 0>
__global__ __launch_bounds__(256, (kMinWavesPerSimd<Real, Form, B, kMom>)) void sweep_flow_ge(PlaneArgs<Real> A, FlowArgs F)
{
    // 256 lanes as in the hyperplane kernel; A.cells is the whole tile list
    // of the schedule
    __shared__ TileLds<Real> L;
    __shared__ uint4 sh[2];
    const int tid = threadIdx.x;
    const unsigned o = blockIdx.x & 7u;
    if (tid < 64) flow_take(F, o, tid, sh);
    if constexpr (Form == kFormAnnPaperDir)
        load_pann_dir_table(static_cast<const float *>(A.ann_params), (int)o, (int)A.Do,
                            dgsn_dyn_lds);
    __syncthreads();
    // the unit is uniform over the block: keep it in scalar registers
    const unsigned blk = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[0].y);
    const unsigned t0 = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[0].z);
    const unsigned cnt = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[0].w);
    const unsigned t = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[1].x);
    const SegLane l = seg_lane(A, tid);
    bool tvalid;
    const uint32_t pt = step_tile(A.cells + t0, cnt, (int)(blk * A.nc) + l.z, l.ok, tvalid);
    const Real inc[3] = {A.inc[o][0], A.inc[o][1], A.inc[o][2]};
    __shared__ Real ytab[kMom > 0 ? 64 * kYlmStride : 1];
    __shared__ __align__(16) Real mstage[kStageFloats<Real, kMom>];
    if constexpr (kMom > 0) load_ylm_table(A, (int)o, ytab);
    tile_body<Real, Form, B, kStorePsi, kAdjoint, true, kMom>(A, inc, l.d, l.g, tid, tvalid, pt,
                                                              (int)o, l.ok, L, ytab, mstage,
                                                              dgsn_dyn_lds);
    flow_finish(F, tid, o, t);
}

// The matrix-core network under the dataflow schedule: the same unit
// protocol.
template <int B, int Form>
__global__ __launch_bounds__(256) void sweep_flow_ann(PlaneArgs<float> A, FlowArgs F)
{
    __shared__ TileLds<float> L;
    __shared__ uint4 sh[2];
    const int tid = threadIdx.x;
    const unsigned o = blockIdx.x & 7u;
    if (tid < 64) flow_take(F, o, tid, sh);
    __syncthreads();
    const unsigned blk = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[0].y);
    const unsigned t0 = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[0].z);
    const unsigned cnt = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[0].w);
    const unsigned t = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[1].x);
    const SegLane l = seg_lane(A, tid);
    bool tvalid;
    const uint32_t pt = step_tile(A.cells + t0, cnt, (int)(blk * A.nc) + l.z, l.ok, tvalid);
    const float inc[3] = {A.inc[o][0], A.inc[o][1], A.inc[o][2]};
    tile_body<float, Form, B, false, false, true>(A, inc, l.d, l.g, tid, tvalid, pt, (int)o,
                                                      l.ok, L);
    flow_finish(F, tid, o, t);
}

template <typename Real, int Form, int B>
void launch_flow_form(const PlaneArgs<Real> &A, const FlowArgs &F, bool store_psi, bool adjoint,
                      dim3 grid, dim3 block, hipStream_t s)
{
    // anisotropic sweeps: tile edges 1 and 2 (the run clamps larger tiles);
    // the psi store and the adjoint with the mass-inverse form only
    if constexpr (B <= 2) {
        if (A.nmom > 1) {
            if constexpr (Form == kFormMassInv) {
                if (adjoint || store_psi) {
                    if (A.nmom == 4 && adjoint)
                        hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, false, true, 3>), grid, block,
                                           0, s, A, F);
                    else if (A.nmom == 4)
                        hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, true, false, 3>), grid, block,
                                           0, s, A, F);
                    else if (A.nmom == 9 && adjoint)
                        hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, false, true, 8>), grid, block,
                                           0, s, A, F);
                    else if (A.nmom == 9)
                        hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, true, false, 8>), grid, block,
                                           0, s, A, F);
                    else if (adjoint)
                        hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, false, true, 15>), grid, block,
                                           0, s, A, F);
                    else
                        hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, true, false, 15>), grid, block,
                                           0, s, A, F);
                    return;
                }
            }
            if (A.nmom == 4)
                hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, false, false, 3>), grid, block, 0,
                                   s, A, F);
            else if (A.nmom == 9)
                hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, false, false, 8>), grid, block, 0,
                                   s, A, F);
            else
                hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, false, false, 15>), grid, block,
                                   0, s, A, F);
            return;
        }
    }
    if (adjoint)
        hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, false, true>), grid, block, 0, s, A, F);
    else if (store_psi)
        hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, true, false>), grid, block, 0, s, A, F);
    else
        hipLaunchKernelGGL((sweep_flow_ge<Real, Form, B, false, false>), grid, block, 0, s, A, F);
}

template <typename Real, int Form>
void launch_flow_b(const PlaneArgs<Real> &A, const FlowArgs &F, int b, bool store_psi,
                   bool adjoint, dim3 grid, dim3 block, hipStream_t s)
{
    switch (b) {
    case 3: launch_flow_form<Real, Form, 3>(A, F, store_psi, adjoint, grid, block, s); break;
    case 2: launch_flow_form<Real, Form, 2>(A, F, store_psi, adjoint, grid, block, s); break;
    default: launch_flow_form<Real, Form, 1>(A, F, store_psi, adjoint, grid, block, s); break;
    }
}

// The matrix-core network: FP32 forward sweeps only.
template <int Form>
void launch_flow_ann(const PlaneArgs<float> &A, const FlowArgs &F, int b, dim3 grid, dim3 block,
                     hipStream_t s)
{
    switch (b) {
    case 3: hipLaunchKernelGGL((sweep_flow_ann<3, Form>), grid, block, 0, s, A, F); break;
    case 2: hipLaunchKernelGGL((sweep_flow_ann<2, Form>), grid, block, 0, s, A, F); break;
    default: hipLaunchKernelGGL((sweep_flow_ann<1, Form>), grid, block, 0, s, A, F); break;
    }
}

// The paper-form networks (per octant or per direction): FP32 forward
// sweeps only.
template <int Form>
void launch_flow_pann(const PlaneArgs<float> &A, const FlowArgs &F, int b, dim3 grid, dim3 block,
                      hipStream_t s)
{
    // the per-direction images of the block's octant in dynamic LDS
    const size_t lds = Form == kFormAnnPaperDir ? (size_t)A.Do * kPannLdsStride * 4 : 0;
    switch (b) {
    case 3:
        hipLaunchKernelGGL((sweep_flow_ge<float, Form, 3, false, false>), grid, block, lds, s, A,
                           F);
        break;
    case 2:
        hipLaunchKernelGGL((sweep_flow_ge<float, Form, 2, false, false>), grid, block, lds, s, A,
                           F);
        break;
    default:
        hipLaunchKernelGGL((sweep_flow_ge<float, Form, 1, false, false>), grid, block, lds, s, A,
                           F);
        break;
    }
}

}  // namespace

template <typename Real>
int launch_flow(const PlaneArgs<Real> &A, const FlowArgs &F, int form, int b, bool store_psi,
                bool adjoint, hipStream_t s)
{
    const dim3 block(256);
    const bool net = form == kFormAnn || form == kFormAnnSplit;
    const bool paper = form == kFormAnnPaper || form == kFormAnnPaperDir;
    if ((paper || net) && (sizeof(Real) != 4 || store_psi || adjoint))
        return set_error(DGSN_EUNSUPPORTED, "the network solvers run FP32 forward sweeps");
    if (A.nmom > 1 && (paper || net ||
                       (form == kFormDense && (store_psi || adjoint))))
        return set_error(DGSN_EUNSUPPORTED, "anisotropic sweeps run the GE solvers (the psi "
                         "store and the adjoint with the mass-inverse form)");
    if (A.nmom > 1 && ((A.nmom != 4 && A.nmom != 9 && A.nmom != 16) || b > 2))
        return set_error(DGSN_EINVAL, "anisotropic sweeps take (L+1)^2 moments, L = 1..3, and "
                         "tile edges 1..2 (moments %u, tile %d)", A.nmom, b);
    for (unsigned done = 0; done < F.units_o; done += kFlowMaxGroupsPerOctant) {
        const dim3 grid(8 * std::min(F.units_o - done, kFlowMaxGroupsPerOctant));
        if (form == kFormDense) {
            launch_flow_b<Real, kFormDense>(A, F, b, store_psi, adjoint, grid, block, s);
        } else if (form == kFormAnnPaper) {
            if constexpr (sizeof(Real) == 4)
                launch_flow_pann<kFormAnnPaper>(A, F, b, grid, block, s);
        } else if (form == kFormAnnPaperDir) {
            if constexpr (sizeof(Real) == 4)
                launch_flow_pann<kFormAnnPaperDir>(A, F, b, grid, block, s);
        } else if (form == kFormAnn) {
            if constexpr (sizeof(Real) == 4) launch_flow_ann<kFormAnn>(A, F, b, grid, block, s);
        } else if (form == kFormAnnSplit) {
            if constexpr (sizeof(Real) == 4)
                launch_flow_ann<kFormAnnSplit>(A, F, b, grid, block, s);
        } else {
            launch_flow_b<Real, kFormMassInv>(A, F, b, store_psi, adjoint, grid, block, s);
        }
        DGSN_HIP(hipGetLastError());
    }
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

int launch_flow_reset(const FlowArgs &F, hipStream_t s)
{
    const int words = kFlowDone + 8 * (int)F.units_o;
    hipLaunchKernelGGL(flow_reset, dim3((words + 255) / 256), dim3(256), 0, s, F.sync, words);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

template int launch_flow<float>(const PlaneArgs<float> &, const FlowArgs &, int, int, bool, bool,
                                hipStream_t);
template int launch_flow<double>(const PlaneArgs<double> &, const FlowArgs &, int, int, bool,
                                 bool, hipStream_t);

}  // namespace dgsn
