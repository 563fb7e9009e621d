// Batched execution of many independent problems of any size, quadrature,
// group count and local solver (GE or ANN) in one HIP-graph launch.
//
// Two schedules, both captured once into a HIP graph together with a clock
// stamp and the per-problem octant reductions:
//
// * Steps (DGSN_SCHED_PLANES): launch t of the graph performs step t (a tile
//   or cell hyperplane) of every problem that still has one.  One batched
//   kernel serves the launch: a block finds its problem in a prefix table of
//   block counts, decodes its lanes for that problem's (direction, group,
//   tile) shape and runs the GE or the ANN tile body.  The small hyperplanes
//   at the start and end of each sweep, which leave a single-problem launch
//   mostly idle, are filled with the work of the other problems.
// * Dataflow (DGSN_SCHED_DATAFLOW): one launch for the whole batch.  Per
//   octant, the units (problem, step, block of tiles) of all problems form
//   one work queue in step-major order; a workgroup takes the next unit of
//   its octant from the queue's ticket counter, waits on the done flags of
//   the units holding its tiles' upwind neighbours (within its problem) and
//   runs the same tile bodies.  Flags hold the number of the run that set
//   them, so a graph replay needs no flag reset: the stamp kernel advances
//   the run number and clears the eight tickets.
//
// The last units of each problem's last step record the device wall clock,
// which gives per-problem completion latencies.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ann_body.hpp"
#include "flow.hpp"
#include "sweep_body.hpp"

namespace dgsn {

struct BatchStepArgs {
    const PlaneArgs<float> *args;   // [nprob] arguments of this step
    const int *prefix;              // [nprob + 1] block offsets of this step
    const int *meta;                // [nprob][4]: solver, tile edge, last step, unused
    unsigned long long *t_end;      // [nprob] completion wall clock
    int nprob;
    int step;
};

// Dataflow batch: one unit per queue entry, octant-independent.
struct BatchFlowArgs {
    const PlaneArgs<float> *args;   // [nprob]; A.cells is the problem's whole tile list
    const int *meta;                // [nprob][4]: solver, tile edge, last step, unused
    const uint4 *u0;                // [units]: problem, step, block, first tile of the step
    const uint4 *u1;                // [units]: tiles in the step, dependency lo, hi, unused
    unsigned *sync;                 // tickets, error word, run number, done[8][units]
    unsigned long long *t_end;      // [nprob] completion wall clock
    unsigned units;                 // units per octant
    unsigned spin_limit;
};
constexpr int kBatchRun = kFlowError + 1;   // run number word of the batch sync buffer

namespace {

__global__ __launch_bounds__(256) void batch_stamp(unsigned long long *t_start,
                                                   unsigned long long *t_end, int nprob,
                                                   unsigned *sync)
{
    // one block: clears the completion stamps, starts a new dataflow run
    // (tickets cleared, run number advanced) and records the start
    for (int i = threadIdx.x; i < nprob; i += blockDim.x) t_end[i] = 0ull;
    if (sync && threadIdx.x < 8) sync[kFlowTicket + 32 * threadIdx.x] = 0u;
    if (sync && threadIdx.x == 0) sync[kBatchRun] += 1u;
    if (threadIdx.x == 0) t_start[0] = wall_clock64();
}

// Argument block of problem b, read through the constant address space: the
// table is not written while a kernel runs, so its fields are loaded with
// scalar loads into scalar registers even after the body's global stores and
// the dataflow atomics.  The inflow of octant slot o is returned separately
// (the copy is then indexed with constants only and lives in registers).
typedef const __attribute__((address_space(4))) PlaneArgs<float> ConstPlaneArgs;

__device__ __forceinline__ PlaneArgs<float> problem_args(const PlaneArgs<float> *table, int b,
                                                         int o, float inc[3])
{
    PlaneArgs<float> r;
#if defined(__HIP_DEVICE_COMPILE__)   // the address space exists in the device pass only
    ConstPlaneArgs *t = (ConstPlaneArgs *)table;
    for (int a = 0; a < 3; ++a) inc[a] = t[b].inc[o][a];
    r = t[b];
#endif
    return r;
}

// solver code of a problem in the batch tables: DGSN_GE, DGSN_ANN (the
// matrix-core network) or the paper-form network
constexpr int kBatchPaperAnn = 3;

template <bool kCoh>
__device__ __forceinline__ void batch_body(const PlaneArgs<float> &A, const float inc[3],
                                           int solver, int tileb, const SegLane &l, int tid,
                                           bool tv, uint32_t pt, int o, TileLds<float> &L)
{
    if (solver == kBatchPaperAnn) {
        if (tileb == 2)
            tile_body<float, kFormAnnPaper, 2, false, false, kCoh>(A, inc, l.d, l.g, tid, tv, pt,
                                                                   o, l.ok, L);
        else
            tile_body<float, kFormAnnPaper, 1, false, false, kCoh>(A, inc, l.d, l.g, tid, tv, pt,
                                                                   o, l.ok, L);
    } else if (solver == DGSN_ANN) {
        if (tileb == 2)
            tile_body<float, kFormAnn, 2, false, false, kCoh>(A, inc, l.d, l.g, tid, tv, pt, o,
                                                              l.ok, L);
        else
            tile_body<float, kFormAnn, 1, false, false, kCoh>(A, inc, l.d, l.g, tid, tv, pt, o,
                                                              l.ok, L);
    } else {
        if (tileb == 2)
            tile_body<float, kFormMassInv, 2, false, false, kCoh>(A, inc, l.d, l.g, tid, tv, pt,
                                                                  o, l.ok, L);
        else
            tile_body<float, kFormMassInv, 1, false, false, kCoh>(A, inc, l.d, l.g, tid, tv, pt,
                                                                  o, l.ok, L);
    }
}

// held to 3 waves per SIMD (168 registers): the tile bodies of all solvers
// together would take 171 and fall to 2
__global__ __launch_bounds__(256, 3) void batch_flow(BatchFlowArgs F)
{
    __shared__ TileLds<float> L;
    __shared__ uint4 sh[2];
    const int tid = threadIdx.x;
    const unsigned o = blockIdx.x & 7u;
    if (tid < 64) {
        // the launches of a run have exactly 8 * units workgroups (clamped
        // defensively)
        unsigned t = 0;
        if (tid == 0) t = flow_add(F.sync + kFlowTicket + 32 * o, 1u);
        t = __shfl(t, 0);
        if (t >= F.units) t = F.units - 1;
        const unsigned run = flow_load(F.sync + kBatchRun);
        const uint4 a = F.u0[t];
        const uint4 c = F.u1[t];
        flow_wait_range(F.sync + kFlowDone + o * F.units, c.y, c.z, run, tid, F.spin_limit,
                        F.sync + kFlowError);
        if (tid == 0) {
            sh[0] = a;
            sh[1] = make_uint4(c.x, t, run, 0u);
        }
    }
    __syncthreads();
    // the unit is uniform over the block: keep it in scalar registers
    const int b = __builtin_amdgcn_readfirstlane((int)sh[0].x);
    const int step = __builtin_amdgcn_readfirstlane((int)sh[0].y);
    const int blk = __builtin_amdgcn_readfirstlane((int)sh[0].z);
    const unsigned t0 = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[0].w);
    const unsigned cnt = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[1].x);
    const unsigned t = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[1].y);
    const unsigned run = (unsigned)__builtin_amdgcn_readfirstlane((int)sh[1].z);
    float inc[3];
    const PlaneArgs<float> A = problem_args(F.args, b, (int)o, inc);
    const SegLane l = seg_lane(A, tid);
    bool tv;
    const uint32_t pt = step_tile(A.cells + t0, cnt, blk * (int)A.nc + l.z, l.ok, tv);
    batch_body<true>(A, inc, F.meta[4 * b + 0], F.meta[4 * b + 1], l, tid, tv, pt, (int)o, L);
    __builtin_amdgcn_s_waitcnt(0);   // this wave's coherent front stores are acknowledged
    __syncthreads();
    if (tid == 0) {
        flow_store(F.sync + kFlowDone + o * F.units + t, run);
        if (step == F.meta[4 * b + 2]) atomicMax(&F.t_end[b], (unsigned long long)wall_clock64());
    }
}

__global__ __launch_bounds__(256) void batch_step(BatchStepArgs S)
{
    __shared__ TileLds<float> L;
    // problem of this block: prefix[b] <= blockIdx.x < prefix[b + 1]
    int lo = 0, hi = S.nprob;
    const int bid = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (S.prefix[mid] <= bid) lo = mid;
        else hi = mid;
    }
    const int b = lo;
    const int local = bid - S.prefix[b];
    const int o = local & 7;                  // octant slot
    const int bx = local >> 3;                // block within the step
    float inc[3];
    const PlaneArgs<float> A = problem_args(S.args, b, o, inc);
    const int tid = threadIdx.x;
    const SegLane l = seg_lane(A, tid);
    bool tv;
    const uint32_t pt = step_tile(A.cells, A.ncp, bx * (int)A.nc + l.z, l.ok, tv);
    batch_body<false>(A, inc, S.meta[4 * b + 0], S.meta[4 * b + 1], l, tid, tv, pt, o, L);
    if (S.step == S.meta[4 * b + 2]) {
        __syncthreads();
        if (threadIdx.x == 0) atomicMax(&S.t_end[b], (unsigned long long)wall_clock64());
    }
}

}  // namespace
}  // namespace dgsn

using namespace dgsn;

struct dgsn_batch {
    dgsn_ctx *ctx = nullptr;
    std::vector<dgsn_problem *> probs;
    std::vector<const void *> src;
    std::vector<void *> phi;
    std::vector<int> tileb;            // per problem tile edge (GE)
    int nsteps = 0;
    std::vector<int> blocks_per_step;  // total blocks of each step
    DevBuf d_args, d_prefix, d_meta, d_tend, d_tstart;
    int schedule = DGSN_SCHED_PLANES;
    // dataflow tables: per-problem arguments, unit queue, sync words
    DevBuf d_fargs, d_u0, d_u1, d_fsync;
    unsigned funits = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool dirty = true;
    // each problem's cfg_gen when the graph was captured: the graph holds its
    // inflow, solver and network pointer by value
    std::vector<unsigned long long> cfg_gen;
    double clock_khz = 0.0;
    ~dgsn_batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

// blocks of a step of a problem inside the batched kernel: every block covers
// cells_per_block tiles (or cells) of one octant
int blocks_of(const dgsn_problem *p, int ncp)
{
    const int nc = cells_per_block(p->Do, p->G);
    return (ncp + nc - 1) / nc;
}

int batch_solver(const dgsn_problem *p)
{
    if (p->solver != DGSN_ANN) return DGSN_GE;
    return p->ann->version == 2 ? kBatchPaperAnn : DGSN_ANN;
}

int build_tables(dgsn_batch *B)
{
    const int n = (int)B->probs.size();
    std::vector<int> steps(n);
    B->nsteps = 0;
    for (int b = 0; b < n; ++b) {
        const dgsn_problem *p = B->probs[b];
        steps[b] = B->tileb[b] == 1 ? p->n_planes : p->n_tplanes[B->tileb[b]];
        B->nsteps = std::max(B->nsteps, steps[b]);
    }
    std::vector<PlaneArgs<float>> args((size_t)B->nsteps * n);
    std::vector<int> prefix((size_t)B->nsteps * (n + 1));
    std::vector<int> meta((size_t)4 * n);
    B->blocks_per_step.assign(B->nsteps, 0);
    for (int b = 0; b < n; ++b) {
        dgsn_problem *p = B->probs[b];
        meta[4 * b + 0] = batch_solver(p);
        meta[4 * b + 1] = B->tileb[b];
        meta[4 * b + 2] = steps[b] - 1;
        meta[4 * b + 3] = 0;
    }
    for (int t = 0; t < B->nsteps; ++t) {
        int acc = 0;
        for (int b = 0; b < n; ++b) {
            dgsn_problem *p = B->probs[b];
            PlaneArgs<float> A = batch_plane_args(p, B->src[b]);
            const int tb = B->tileb[b];
            const std::vector<int> &off = tb > 1 ? p->tplane_off[tb] : p->plane_off;
            const uint32_t *cells =
                static_cast<const uint32_t *>(tb > 1 ? p->d_tiles[tb].ptr : p->d_plane_cells.ptr);
            int ncp = 0;
            if (t < steps[b]) {
                A.cells = cells + off[t];
                ncp = off[t + 1] - off[t];
            } else {
                A.cells = cells;
            }
            A.ncp = (uint32_t)ncp;
            args[(size_t)t * n + b] = A;
            prefix[(size_t)t * (n + 1) + b] = acc;
            acc += 8 * blocks_of(p, ncp);
        }
        prefix[(size_t)t * (n + 1) + n] = acc;
        B->blocks_per_step[t] = acc;
    }
    DGSN_TRY(B->d_args.alloc(args.size() * sizeof(PlaneArgs<float>)));
    DGSN_TRY(B->d_prefix.alloc(prefix.size() * sizeof(int)));
    DGSN_TRY(B->d_meta.alloc(meta.size() * sizeof(int)));
    DGSN_HIP(hipMemcpy(B->d_args.ptr, args.data(), args.size() * sizeof(PlaneArgs<float>),
                       hipMemcpyHostToDevice));
    DGSN_HIP(hipMemcpy(B->d_prefix.ptr, prefix.data(), prefix.size() * sizeof(int),
                       hipMemcpyHostToDevice));
    DGSN_HIP(hipMemcpy(B->d_meta.ptr, meta.data(), meta.size() * sizeof(int),
                       hipMemcpyHostToDevice));
    return DGSN_OK;
}

// Dataflow queue: the units of every problem (each with its own tile edge),
// merged step-major; dependency ranges are translated to queue indices.
int build_flow_tables(dgsn_batch *B)
{
    const int n = (int)B->probs.size();
    std::vector<std::vector<FlowUnitHost>> units(n);
    std::vector<std::vector<unsigned>> first(n);   // first local unit of each step (+ end)
    int maxsteps = 0;
    std::vector<PlaneArgs<float>> args(n);
    std::vector<int> meta((size_t)4 * n);
    for (int b = 0; b < n; ++b) {
        dgsn_problem *p = B->probs[b];
        const int tb = B->tileb[b];
        const long long nmax = std::max(std::max(p->n[0], p->n[1]), p->n[2]);
        if (nmax * nmax * 8 * 4 * p->Do * p->G * 4LL >= (1LL << 31))
            return set_error(DGSN_EUNSUPPORTED,
                             "the dataflow schedule needs face fronts under 2 GiB (problem %d)", b);
        DGSN_TRY(flow_units_host(p, tb, units[b]));
        const int ns = tb == 1 ? p->n_planes : p->n_tplanes[tb];
        first[b].assign(ns + 1, (unsigned)units[b].size());
        for (int u = (int)units[b].size() - 1; u >= 0; --u) first[b][units[b][u].step] = u;
        maxsteps = std::max(maxsteps, ns);
        PlaneArgs<float> A = batch_plane_args(p, B->src[b]);
        A.cells = static_cast<const uint32_t *>(tb > 1 ? p->d_tiles[tb].ptr : p->d_plane_cells.ptr);
        A.ncp = 0;
        args[b] = A;
        meta[4 * b + 0] = batch_solver(p);
        meta[4 * b + 1] = tb;
        meta[4 * b + 2] = ns - 1;
        meta[4 * b + 3] = 0;
    }
    // queue index of the first unit of (problem, step)
    std::vector<std::vector<unsigned>> qbase(n);
    size_t total = 0;
    for (int b = 0; b < n; ++b) qbase[b].assign(first[b].size(), 0u);
    for (int s = 0; s < maxsteps; ++s)
        for (int b = 0; b < n; ++b)
            if (s + 1 < (int)first[b].size()) {
                qbase[b][s] = (unsigned)total;
                total += first[b][s + 1] - first[b][s];
            }
    if (8ull * total >= (1ull << 31)) return set_error(DGSN_EUNSUPPORTED, "batch too large");
    std::vector<uint4> u0(total), u1(total);
    for (int b = 0; b < n; ++b)
        for (size_t u = 0; u < units[b].size(); ++u) {
            const FlowUnitHost &f = units[b][u];
            const unsigned q = qbase[b][f.step] + (unsigned)(u - first[b][f.step]);
            unsigned lo = 1, hi = 0;
            if (f.dlo <= f.dhi) {
                const unsigned s0 = first[b][f.step - 1];
                lo = qbase[b][f.step - 1] + (f.dlo - s0);
                hi = qbase[b][f.step - 1] + (f.dhi - s0);
            }
            u0[q] = make_uint4((unsigned)b, f.step, f.block, f.t0);
            u1[q] = make_uint4(f.cnt, lo, hi, 0u);
        }
    B->funits = (unsigned)total;
    DGSN_TRY(B->d_fargs.alloc(args.size() * sizeof(PlaneArgs<float>)));
    DGSN_TRY(B->d_meta.alloc(meta.size() * sizeof(int)));
    DGSN_TRY(B->d_u0.alloc(total * sizeof(uint4)));
    DGSN_TRY(B->d_u1.alloc(total * sizeof(uint4)));
    const size_t words = kFlowDone + 8 * total;
    DGSN_TRY(B->d_fsync.alloc(words * sizeof(unsigned)));
    DGSN_HIP(hipMemcpy(B->d_fargs.ptr, args.data(), args.size() * sizeof(PlaneArgs<float>),
                       hipMemcpyHostToDevice));
    DGSN_HIP(hipMemcpy(B->d_meta.ptr, meta.data(), meta.size() * sizeof(int),
                       hipMemcpyHostToDevice));
    DGSN_HIP(hipMemcpy(B->d_u0.ptr, u0.data(), total * sizeof(uint4), hipMemcpyHostToDevice));
    DGSN_HIP(hipMemcpy(B->d_u1.ptr, u1.data(), total * sizeof(uint4), hipMemcpyHostToDevice));
    DGSN_HIP(hipMemset(B->d_fsync.ptr, 0, words * sizeof(unsigned)));
    return DGSN_OK;
}

int enqueue_batch(dgsn_batch *B, hipStream_t s)
{
    const int n = (int)B->probs.size();
    const bool flow = B->schedule == DGSN_SCHED_DATAFLOW;
    hipLaunchKernelGGL(batch_stamp, dim3(1), dim3(256), 0, s,
                       static_cast<unsigned long long *>(B->d_tstart.ptr),
                       static_cast<unsigned long long *>(B->d_tend.ptr), n,
                       flow ? static_cast<unsigned *>(B->d_fsync.ptr) : nullptr);
    DGSN_HIP(hipGetLastError());
    if (flow) {
        BatchFlowArgs F;
        F.args = static_cast<const PlaneArgs<float> *>(B->d_fargs.ptr);
        F.meta = static_cast<const int *>(B->d_meta.ptr);
        F.u0 = static_cast<const uint4 *>(B->d_u0.ptr);
        F.u1 = static_cast<const uint4 *>(B->d_u1.ptr);
        F.sync = static_cast<unsigned *>(B->d_fsync.ptr);
        F.t_end = static_cast<unsigned long long *>(B->d_tend.ptr);
        F.units = B->funits;
        F.spin_limit = kFlowSpinDefault;
        for (unsigned done = 0; done < B->funits; done += kFlowMaxGroupsPerOctant) {
            const unsigned g = std::min(B->funits - done, kFlowMaxGroupsPerOctant);
            hipLaunchKernelGGL(batch_flow, dim3(8 * g), dim3(256), 0, s, F);
            DGSN_HIP(hipGetLastError());
        }
        for (int b = 0; b < n; ++b) DGSN_TRY(batch_reduce(B->probs[b], B->phi[b], s));
        return DGSN_OK;
    }
    for (int t = 0; t < B->nsteps; ++t) {
        if (B->blocks_per_step[t] == 0) continue;
        BatchStepArgs S;
        S.args = static_cast<const PlaneArgs<float> *>(B->d_args.ptr) + (size_t)t * n;
        S.prefix = static_cast<const int *>(B->d_prefix.ptr) + (size_t)t * (n + 1);
        S.meta = static_cast<const int *>(B->d_meta.ptr);
        S.t_end = static_cast<unsigned long long *>(B->d_tend.ptr);
        S.nprob = n;
        S.step = t;
        hipLaunchKernelGGL(batch_step, dim3(B->blocks_per_step[t]), dim3(256), 0, s, S);
        DGSN_HIP(hipGetLastError());
    }
    for (int b = 0; b < n; ++b) DGSN_TRY(batch_reduce(B->probs[b], B->phi[b], s));
    return DGSN_OK;
}

int capture(dgsn_batch *B)
{
    if (B->exec) {
        (void)hipGraphExecDestroy(B->exec);
        B->exec = nullptr;
    }
    if (B->graph) {
        (void)hipGraphDestroy(B->graph);
        B->graph = nullptr;
    }
    DGSN_TRY(B->schedule == DGSN_SCHED_DATAFLOW ? build_flow_tables(B) : build_tables(B));
    DGSN_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_batch(B, B->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(B->cap, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess)
        return set_error(DGSN_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    B->graph = g;
    DGSN_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    B->dirty = false;
    B->cfg_gen.resize(B->probs.size());
    for (size_t b = 0; b < B->probs.size(); ++b) B->cfg_gen[b] = B->probs[b]->cfg_gen;
    return DGSN_OK;
}

// The member problems as a batch can run them now (their solver and network
// may have changed since the batch was created), and whether the captured
// graph is stale.
int batch_validate(dgsn_batch *B)
{
    for (size_t b = 0; b < B->probs.size(); ++b) {
        const dgsn_problem *p = B->probs[b];
        if (!B->src[b]) return set_error(DGSN_EINVAL, "problem %zu has no src/phi (set_io)", b);
        if (p->solver == DGSN_GE_DENSE)
            return set_error(DGSN_EUNSUPPORTED, "batched execution uses the DGSN_GE or DGSN_ANN "
                             "solvers (problem %zu)", b);
        if (p->solver == DGSN_ANN && !p->ann)
            return set_error(DGSN_EINVAL, "problem %zu uses the ANN solver without an ANN", b);
        if (p->solver == DGSN_ANN && p->ann->mode != DGSN_ANN_BF16)
            return set_error(DGSN_EUNSUPPORTED, "batched execution evaluates the networks in "
                             "BF16 (problem %zu uses split BF16)", b);
        if (p->solver == DGSN_ANN && p->ann->version == 3)
            return set_error(DGSN_EUNSUPPORTED, "batched execution takes per-octant networks "
                             "(problem %zu has per-direction networks)", b);
        if (B->cfg_gen.size() != B->probs.size() || B->cfg_gen[b] != p->cfg_gen) B->dirty = true;
    }
    return DGSN_OK;
}

// Reports (and clears) an expired dataflow wait of the last runs; the device
// must be idle.
int batch_check(dgsn_batch *B)
{
    if (!B->d_fsync.ptr) return DGSN_OK;
    unsigned err = 0;
    DGSN_HIP(hipMemcpy(&err, static_cast<unsigned *>(B->d_fsync.ptr) + kFlowError, sizeof(err),
                       hipMemcpyDeviceToHost));
    if (err == 0u) return DGSN_OK;
    const unsigned zero = 0u;
    DGSN_HIP(hipMemcpy(static_cast<unsigned *>(B->d_fsync.ptr) + kFlowError, &zero, sizeof(zero),
                       hipMemcpyHostToDevice));
    return set_error(DGSN_ETIMEOUT, "a dataflow wait of the batch expired; its results are "
                     "invalid");
}

}  // namespace

extern "C" {

int dgsn_batch_set_schedule(dgsn_batch *B, int schedule)
{
    clear_error();
    if (!B) return set_error(DGSN_EINVAL, "batch is NULL");
    if (schedule != DGSN_SCHED_PLANES && schedule != DGSN_SCHED_DATAFLOW)
        return set_error(DGSN_EINVAL, "unknown schedule %d", schedule);
    if (schedule != B->schedule) B->dirty = true;
    B->schedule = schedule;
    return DGSN_OK;
}

int dgsn_batch_get_schedule(const dgsn_batch *B, int *schedule)
{
    clear_error();
    if (!B || !schedule) return set_error(DGSN_EINVAL, "batch and schedule must be set");
    *schedule = B->schedule;
    return DGSN_OK;
}

int dgsn_batch_create(dgsn_ctx *ctx, dgsn_problem *const *probs, int n, dgsn_batch **out)
{
    clear_error();
    if (!out) return set_error(DGSN_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx || !probs || n < 1) return set_error(DGSN_EINVAL, "ctx, probs and n >= 1 required");
    for (int b = 0; b < n; ++b) {
        if (!probs[b]) return set_error(DGSN_EINVAL, "problem %d is NULL", b);
        if (probs[b]->ctx != ctx) return set_error(DGSN_EINVAL, "problem %d is on another context", b);
        if (probs[b]->precision != DGSN_FP32)
            return set_error(DGSN_EUNSUPPORTED, "batched execution runs FP32 problems (problem %d)", b);
        if (probs[b]->solver == DGSN_GE_DENSE)
            return set_error(DGSN_EUNSUPPORTED, "batched execution uses the DGSN_GE or DGSN_ANN "
                                                "solvers (problem %d)", b);
        if (probs[b]->solver == DGSN_ANN && !probs[b]->ann)
            return set_error(DGSN_EINVAL, "problem %d uses the ANN solver without an ANN", b);
    }
    DGSN_HIP(hipSetDevice(ctx->device));
    dgsn_batch *B = new (std::nothrow) dgsn_batch();
    if (!B) return set_error(DGSN_ENOMEM, "host allocation failed");
    B->ctx = ctx;
    B->probs.assign(probs, probs + n);
    B->src.assign(n, nullptr);
    B->phi.assign(n, nullptr);
    B->tileb.resize(n);
    // the batched kernel instantiates tile edges 1 and 2 only (a 3^3 tile
    // path would raise the register count of every block of the launch)
    for (int b = 0; b < n; ++b) B->tileb[b] = std::min(probs[b]->tile_b, 2);
    int rate = 0;
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess ||
        rate <= 0) {
        delete B;
        return set_error(DGSN_EHIP, "cannot read the device wall-clock rate");
    }
    B->clock_khz = rate;
    int rc;
    if ((rc = B->d_tend.alloc(n * sizeof(unsigned long long))) ||
        (rc = B->d_tstart.alloc(sizeof(unsigned long long)))) {
        delete B;
        return rc;
    }
    if (hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess) {
        delete B;
        return set_error(DGSN_EHIP, "cannot create the capture stream");
    }
    *out = B;
    return DGSN_OK;
}

int dgsn_batch_set_io(dgsn_batch *B, int index, const void *src, void *phi)
{
    clear_error();
    if (!B) return set_error(DGSN_EINVAL, "batch is NULL");
    if (index < 0 || index >= (int)B->probs.size())
        return set_error(DGSN_EINVAL, "index %d out of range", index);
    if (!src || !phi || src == phi) return set_error(DGSN_EINVAL, "src and phi must be distinct");
    B->src[index] = src;
    B->phi[index] = phi;
    B->dirty = true;
    return DGSN_OK;
}

int dgsn_batch_set_tiles(dgsn_batch *B, const int *tile_edges)
{
    clear_error();
    if (!B || !tile_edges) return set_error(DGSN_EINVAL, "batch and tile_edges must be set");
    for (size_t b = 0; b < B->probs.size(); ++b)
        if (tile_edges[b] != 1 && tile_edges[b] != 2)
            return set_error(DGSN_EINVAL, "tile edge %d of problem %zu must be 1 or 2",
                             tile_edges[b], b);
    for (size_t b = 0; b < B->probs.size(); ++b) B->tileb[b] = tile_edges[b];
    B->dirty = true;
    return DGSN_OK;
}

int dgsn_batch_autotune(dgsn_batch *B, void *stream, double *best_ms)
{
    clear_error();
    if (!B) return set_error(DGSN_EINVAL, "batch is NULL");
    DGSN_TRY(batch_validate(B));
    DGSN_HIP(hipSetDevice(B->ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int n = (int)B->probs.size();
    // candidates: tile assignment (all 2, all 1, 2 for meshes of >= 32^3
    // cells) under each schedule
    std::vector<std::vector<int>> cand(3, std::vector<int>(n));
    for (int b = 0; b < n; ++b) {
        cand[0][b] = 2;
        cand[1][b] = 1;
        cand[2][b] = B->probs[b]->ncell >= 32LL * 32 * 32 ? 2 : 1;
    }
    hipEvent_t e0, e1;
    DGSN_HIP(hipEventCreate(&e0));
    DGSN_HIP(hipEventCreate(&e1));
    double best = INFINITY;
    int bi = 0, bs = DGSN_SCHED_PLANES, rc = DGSN_OK;
    for (int sc = 0; sc < 2 && rc == DGSN_OK; ++sc)
        for (int c = 0; c < 3 && rc == DGSN_OK; ++c) {
            B->tileb = cand[c];
            B->schedule = sc;
            B->dirty = true;
            if ((rc = capture(B))) break;
            double t = INFINITY;
            for (int rep = 0; rep < 3; ++rep) {
                (void)hipEventRecord(e0, s);
                if (hipGraphLaunch(B->exec, s) != hipSuccess) {
                    rc = set_error(DGSN_EHIP, "graph launch failed");
                    break;
                }
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) t = std::min(t, (double)ms);
            }
            if (rc == DGSN_OK) rc = batch_check(B);
            if (t < best) {
                best = t;
                bi = c;
                bs = sc;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    B->tileb = cand[bi];
    B->schedule = bs;
    B->dirty = true;
    if (best_ms) *best_ms = best;
    return DGSN_OK;
}

int dgsn_batch_run(dgsn_batch *B, void *stream)
{
    clear_error();
    if (!B) return set_error(DGSN_EINVAL, "batch is NULL");
    DGSN_TRY(batch_validate(B));
    DGSN_HIP(hipSetDevice(B->ctx->device));
    if (B->dirty) DGSN_TRY(capture(B));
    DGSN_HIP(hipGraphLaunch(B->exec, reinterpret_cast<hipStream_t>(stream)));
    return DGSN_OK;
}

int dgsn_batch_latencies_us(const dgsn_batch *B, double *out)
{
    clear_error();
    if (!B || !out) return set_error(DGSN_EINVAL, "batch and out must be set");
    const int n = (int)B->probs.size();
    std::vector<unsigned long long> te(n);
    unsigned long long ts = 0;
    DGSN_HIP(hipDeviceSynchronize());
    DGSN_TRY(batch_check(const_cast<dgsn_batch *>(B)));
    DGSN_HIP(hipMemcpy(te.data(), B->d_tend.ptr, n * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost));
    DGSN_HIP(hipMemcpy(&ts, B->d_tstart.ptr, sizeof(ts), hipMemcpyDeviceToHost));
    for (int b = 0; b < n; ++b)
        out[b] = te[b] >= ts ? (double)(te[b] - ts) / B->clock_khz * 1e3 : 0.0;
    return DGSN_OK;
}

int dgsn_batch_destroy(dgsn_batch *B)
{
    clear_error();
    if (B) {
        (void)hipSetDevice(B->ctx->device);
        delete B;
    }
    return DGSN_OK;
}

}  // extern "C"
