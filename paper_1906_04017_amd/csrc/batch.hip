// Batched execution of many independent problems of any size, quadrature,
// group count and local solver (GE or ANN) in one HIP-graph launch.
//
// All problems advance together: launch t of the graph performs step t of
// every problem that still has one (a tile hyperplane for GE problems, a cell
// hyperplane for ANN problems).  One batched kernel serves the launch: a block
// finds its problem in a prefix table of block counts, decodes its lanes for
// that problem's (direction, group, tile) shape and runs the GE tile body or
// the ANN body.  The small hyperplanes at the start and end of each sweep,
// which leave a single-problem launch mostly idle, are thereby filled with the
// work of the other problems.  The whole sequence (a clock stamp, the steps and
// the per-problem octant reductions) is captured once into a HIP graph.  The
// last block of each problem's last step records the device wall clock, which
// gives per-problem completion latencies.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ann_body.hpp"
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

namespace {

__global__ __launch_bounds__(256) void batch_stamp(unsigned long long *t_start,
                                                   unsigned long long *t_end, int nprob)
{
    // one block: clears the completion stamps and records the start
    for (int i = threadIdx.x; i < nprob; i += blockDim.x) t_end[i] = 0ull;
    if (threadIdx.x == 0) t_start[0] = wall_clock64();
}

__global__ __launch_bounds__(256) void batch_step(BatchStepArgs S)
{
    __shared__ TileLds<float> L;
    __shared__ AnnLds al;
    // problem of this block: prefix[b] <= blockIdx.x < prefix[b + 1]
    int lo = 0, hi = S.nprob;
    const int bid = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (S.prefix[mid] <= bid) lo = mid;
        else hi = mid;
    }
    const int b = lo;
    const PlaneArgs<float> &A = S.args[b];
    const int local = bid - S.prefix[b];
    const int o = local & 7;                  // octant slot
    const int bx = local >> 3;                // block within the step
    const int solver = S.meta[4 * b + 0];
    const int tileb = S.meta[4 * b + 1];
    // lanes: (direction, group, tile) of this problem, exact quotients for
    // tid < 256 by multiplication with ceil(2^16 / divisor)
    const int tid = threadIdx.x;
    const int nc = 256 / (int)(A.Do * A.G);
    const int q1 = (tid * (int)A.mag_do) >> 16;
    const int z = (tid * (int)A.mag_dog) >> 16;
    const int d = tid - q1 * (int)A.Do;
    const int g = q1 - z * (int)A.G;
    const bool lane_ok = z < nc;
    const int dl = lane_ok ? d : 0, gl = lane_ok ? g : 0;
    bool tv;
    const uint32_t pt = step_tile(A.cells, A.ncp, bx * nc + z, lane_ok, tv);
    if (solver == DGSN_ANN) {
        if (tileb == 2)
            tile_body<float, kFormAnn, 2, false, false>(A, dl, gl, tid, tv, pt, o, lane_ok, L, &al);
        else
            tile_body<float, kFormAnn, 1, false, false>(A, dl, gl, tid, tv, pt, o, lane_ok, L, &al);
    } else {
        if (tileb == 2)
            tile_body<float, kFormMassInv, 2, false, false>(A, dl, gl, tid, tv, pt, o, lane_ok, L,
                                                            nullptr);
        else
            tile_body<float, kFormMassInv, 1, false, false>(A, dl, gl, tid, tv, pt, o, lane_ok, L,
                                                            nullptr);
    }
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
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool dirty = true;
    double clock_khz = 0.0;
    ~dgsn_batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

// lane shape of a problem inside the batched kernel: every block covers
// floor(256 / (Do G)) tiles (or cells) of one octant
int blocks_of(const dgsn_problem *p, int ncp) { return (ncp + 256 / (p->Do * p->G) - 1) / (256 / (p->Do * p->G)); }

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
        meta[4 * b + 0] = p->solver == DGSN_ANN ? DGSN_ANN : DGSN_GE;
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

int enqueue_batch(dgsn_batch *B, hipStream_t s)
{
    const int n = (int)B->probs.size();
    hipLaunchKernelGGL(batch_stamp, dim3(1), dim3(256), 0, s,
                       static_cast<unsigned long long *>(B->d_tstart.ptr),
                       static_cast<unsigned long long *>(B->d_tend.ptr), n);
    DGSN_HIP(hipGetLastError());
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
    DGSN_TRY(build_tables(B));
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
    return DGSN_OK;
}

}  // namespace

extern "C" {

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
    for (size_t b = 0; b < B->probs.size(); ++b)
        if (!B->src[b]) return set_error(DGSN_EINVAL, "problem %zu has no src/phi (set_io)", b);
    DGSN_HIP(hipSetDevice(B->ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int n = (int)B->probs.size();
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
    int bi = 0, rc = DGSN_OK;
    for (int c = 0; c < 3 && rc == DGSN_OK; ++c) {
        B->tileb = cand[c];
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
        if (t < best) {
            best = t;
            bi = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    B->tileb = cand[bi];
    B->dirty = true;
    if (best_ms) *best_ms = best;
    return DGSN_OK;
}

int dgsn_batch_run(dgsn_batch *B, void *stream)
{
    clear_error();
    if (!B) return set_error(DGSN_EINVAL, "batch is NULL");
    for (size_t b = 0; b < B->probs.size(); ++b)
        if (!B->src[b]) return set_error(DGSN_EINVAL, "problem %zu has no src/phi (set_io)", b);
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
