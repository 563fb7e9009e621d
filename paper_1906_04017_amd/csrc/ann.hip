// Shallow-ANN local solver (Sec. 3): one hidden layer, Eq. (ANN:Eq1) with a
// ReLU hidden activation and a linear output layer, evaluated on the BF16
// matrix cores with FP32 accumulation, and its use inside the sweep in place
// of assembly + Gaussian elimination (Sec. 4, first paragraphs).
//
// Matrix-core mapping (v_mfma_f32_16x16x32_bf16, one wave = 64 samples in 4
// batches of 16).  The layers are evaluated transposed so that no data moves
// between them:
//   H^T[64 x 16] = W1[64 x 32] X^T[32 x 16]   (4 tiles of 16 hidden units)
//   Y^T[16 x 16] = W2p[16 x 64] relu(H^T)     (2 K-chunks of 32)
// The B operand of layer 1 is the sample's 24 features padded to 32: lane l
// holds 8 features (index 8 (l/16) + e) of sample l % 16.  Layer 1 returns in
// lane l the hidden units 16 m + 4 (l/16) + r of sample l % 16; after bias
// (accumulator initialised with b1), ReLU and BF16 rounding these 16 values
// are exactly the lane's B operand of layer 2 if the columns of W2 are
// permuted accordingly on the host (W2p).  The contraction order inside one
// MFMA is irrelevant because A and B use the same lane/element pairing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ann_body.hpp"

namespace dgsn {

namespace {

__global__ __launch_bounds__(256) void ann_infer_kernel(const unsigned char *__restrict__ prm,
                                                        const float *__restrict__ x,
                                                        float *__restrict__ y, long long n)
{
    __shared__ __bf16 lin[4 * 64 * 32];
    __shared__ float lout[4 * 64 * 8];
    AnnRegs R;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    ann_load(prm, lane, R);
    const long long nblk = (n + 255) / 256;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long s = blk * 256 + threadIdx.x;
        float f[24], o[8];
#pragma unroll
        for (int k = 0; k < 24; ++k) f[k] = s < n ? x[s * 24 + k] : 0.0f;
        ann_wave(R, f, lin + wv * (64 * 32), lout + wv * (64 * 8), o);
        if (s < n) {
#pragma unroll
            for (int k = 0; k < 8; ++k) y[s * 8 + k] = o[k];
        }
        __syncthreads();
    }
}

// Hyperplane step with the ANN local solver.  Same lane mapping, fronts and
// reduction as the GE kernel; blocks are 256 threads of which the first
// Do * floor(256 / Do) carry work (full waves are required by the matrix
// cores).  Features of one cell (canonical orientation, h = V^(1/3)):
//   [kappa_a h (3), sigma_t h, inflow x/y/z faces (12) / m, h S (8) / m],
//   m = max(max|psi_in|, max|h S| / (sigma_t h + max_a kappa_a h)),
// and psi = m * y (m = 0 gives psi = 0): the cell solution is linear in the
// inflow and source, so the network only sees unit-scale inputs.
// ---- artifact I/O ----------------------------------------------------------

uint32_t crc32_ieee(const unsigned char *p, size_t n)
{
    uint32_t c = 0xFFFFFFFFu;
    for (size_t i = 0; i < n; ++i) {
        c ^= p[i];
        for (int k = 0; k < 8; ++k) c = (c >> 1) ^ (0xEDB88320u & (0u - (c & 1u)));
    }
    return c ^ 0xFFFFFFFFu;
}

uint16_t bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));
    const uint32_t round = 0x7FFFu + ((u >> 16) & 1u);   // nearest, ties to even
    return (uint16_t)((u + round) >> 16);
}

int build_params(dgsn_ann *a)
{
    std::vector<unsigned char> buf(kParamBytes, 0);
    auto put_bf16 = [&](size_t off, float v) {
        const uint16_t b = bf16_bits(v);
        std::memcpy(&buf[off], &b, 2);
    };
    auto put_f32 = [&](size_t off, float v) { std::memcpy(&buf[off], &v, 4); };
    const int H = a->n_hidden, NI = a->n_in, NO = a->n_out;
    for (int lane = 0; lane < 64; ++lane) {
        const int col = lane & 15, grp = lane >> 4;
        for (int m = 0; m < 4; ++m) {
            const int hid = 16 * m + col;
            for (int e = 0; e < 8; ++e) {
                const int f = 8 * grp + e;
                const float v = (hid < H && f < NI) ? a->W1[hid * NI + f] : 0.0f;
                put_bf16(kParamW1 + (m * 64 + lane) * 16 + 2 * e, v);
            }
            for (int r = 0; r < 4; ++r) {
                const int hid2 = 16 * m + 4 * grp + r;
                put_f32(kParamB1 + (m * 64 + lane) * 16 + 4 * r, hid2 < H ? a->b1[hid2] : 0.0f);
            }
        }
        for (int c = 0; c < 2; ++c)
            for (int e = 0; e < 8; ++e) {
                const int out = col;
                const int hid = 16 * (2 * c + (e >> 2)) + 4 * grp + (e & 3);
                const float v = (out < NO && hid < H) ? a->W2[out * H + hid] : 0.0f;
                put_bf16(kParamW2 + (c * 64 + lane) * 16 + 2 * e, v);
            }
        for (int r = 0; r < 4; ++r) {
            const int out = 4 * grp + r;
            put_f32(kParamB2 + lane * 16 + 4 * r, out < NO ? a->b2[out] : 0.0f);
        }
    }
    DGSN_TRY(a->d_params.alloc(buf.size()));
    DGSN_HIP(hipMemcpy(a->d_params.ptr, buf.data(), buf.size(), hipMemcpyHostToDevice));
    return DGSN_OK;
}

}  // namespace

const void *ann_device_params(const dgsn_ann *a) { return a ? a->d_params.ptr : nullptr; }

}  // namespace dgsn

using namespace dgsn;

extern "C" {

int dgsn_ann_load(dgsn_ctx *ctx, const char *path, dgsn_ann **out)
{
    clear_error();
    if (!path || !out) return set_error(DGSN_EINVAL, "path and out must be set");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return set_error(DGSN_EINVAL, "cannot open ANN artifact %s", path);
    std::vector<unsigned char> data;
    unsigned char chunk[4096];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) {
        data.insert(data.end(), chunk, chunk + got);
        if (data.size() > (1u << 24)) break;
    }
    std::fclose(f);
    const size_t hdr = 8 + 6 * 4;
    if (data.size() < hdr + 4 || std::memcmp(data.data(), "DGSNANN1", 8) != 0)
        return set_error(DGSN_EFORMAT, "%s: not a DGSNANN1 artifact", path);
    uint32_t v[6];
    std::memcpy(v, data.data() + 8, sizeof(v));
    const uint32_t version = v[0], n_in = v[1], n_hidden = v[2], n_out = v[3], act = v[4];
    if (version != 1 || n_in != 24 || n_out != 8 || n_hidden < 1 || n_hidden > kMaxHidden)
        return set_error(DGSN_EFORMAT, "%s: unsupported shape (version %u, %u-%u-%u)", path,
                         version, n_in, n_hidden, n_out);
    const size_t nparam = (size_t)n_hidden * n_in + n_hidden + (size_t)n_out * n_hidden + n_out;
    if (data.size() != hdr + 4 * nparam + 4)
        return set_error(DGSN_EFORMAT, "%s: size %zu does not match the header", path,
                         data.size());
    uint32_t crc;
    std::memcpy(&crc, data.data() + data.size() - 4, 4);
    if (crc != crc32_ieee(data.data(), data.size() - 4))
        return set_error(DGSN_EFORMAT, "%s: checksum mismatch", path);
    if (act != 0)
        return set_error(DGSN_EUNSUPPORTED, "%s: only ReLU hidden layers run on the matrix cores",
                         path);
    if (n_hidden > kHiddenPad)
        return set_error(DGSN_EUNSUPPORTED, "%s: at most %d hidden units are supported", path,
                         kHiddenPad);
    {
        const float *pw = reinterpret_cast<const float *>(data.data() + hdr);
        for (size_t i = 0; i < nparam; ++i)
            if (!std::isfinite(pw[i]))
                return set_error(DGSN_EFORMAT, "%s: non-finite parameter %zu", path, i);
    }
    // the file is fully checked before a device is needed
    if (!ctx) return set_error(DGSN_EINVAL, "ctx is NULL");
    dgsn_ann *a = new (std::nothrow) dgsn_ann();
    if (!a) return set_error(DGSN_ENOMEM, "host allocation failed");
    a->ctx = ctx;
    a->n_in = (int)n_in;
    a->n_hidden = (int)n_hidden;
    a->n_out = (int)n_out;
    a->act = (int)act;
    const float *pf = reinterpret_cast<const float *>(data.data() + hdr);
    a->W1.assign(pf, pf + (size_t)n_hidden * n_in);
    pf += (size_t)n_hidden * n_in;
    a->b1.assign(pf, pf + n_hidden);
    pf += n_hidden;
    a->W2.assign(pf, pf + (size_t)n_out * n_hidden);
    pf += (size_t)n_out * n_hidden;
    a->b2.assign(pf, pf + n_out);
    if (hipSetDevice(ctx->device) != hipSuccess) {
        delete a;
        return set_error(DGSN_EHIP, "hipSetDevice failed");
    }
    int rc = build_params(a);
    if (rc) {
        delete a;
        return rc;
    }
    *out = a;
    return DGSN_OK;
}

int dgsn_ann_destroy(dgsn_ann *ann)
{
    clear_error();
    delete ann;
    return DGSN_OK;
}

int dgsn_ann_infer(const dgsn_ann *ann, const float *x, float *y, long long n, void *stream)
{
    clear_error();
    if (!ann) return set_error(DGSN_EINVAL, "ann is NULL");
    if (n < 0) return set_error(DGSN_EINVAL, "n must be >= 0");
    if (n == 0) return DGSN_OK;
    if (!x || !y) return set_error(DGSN_EINVAL, "x and y must be set");
    DGSN_HIP(hipSetDevice(ann->ctx->device));
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(ann_infer_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream),
                       static_cast<const unsigned char *>(ann->d_params.ptr), x, y, n);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

}  // extern "C"
