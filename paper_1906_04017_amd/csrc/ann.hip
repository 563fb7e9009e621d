// Shallow-ANN local solver (Sec. 3): one hidden layer, Eq. (ANN:Eq1) with a
// ReLU hidden activation and a linear output layer, evaluated on the BF16
// matrix cores with FP32 accumulation, and its use inside the sweep in place
// of assembly + Gaussian elimination (Sec. 4, first paragraphs).
//
// Matrix-core mapping (v_mfma_f32_32x32x16_bf16, one wave = 64 samples in
// 2 batches of 32, ann_body.hpp).  The layers are evaluated transposed so
// that no data moves between them:
//   H^T[64 x 32] = W1[64 x 32] X^T[32 x 32]   (2 tiles of 32 hidden units x 2 K-steps)
//   Y^T[32 x 32] = W2'[32 x 64] relu(H^T)     (4 K-steps of 16; rows 0..7 are the outputs)
// The B operand of layer 1 is the samples' 24 features padded to 32 (two of
// the padding features carry the hidden bias): lane half h of a K-step holds
// 8 features of each of the batch's 32 samples.  Each lane computes its own
// sample's features, so the operands are formed by exchanging the upper and
// lower 32 lanes (v_permlane32_swap) instead of a round trip through LDS, and
// so are the outputs at the end.  Layer 1 leaves in lane half h the hidden
// units hid(kc, h, e) of its column's sample; after ReLU and BF16 rounding
// these are exactly the lane's B operand of layer 2 once the columns of W2
// are permuted accordingly on the host (W2').  The contraction order inside
// one instruction is irrelevant because A and B use the same lane/element
// pairing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ann_body.hpp"
#include "pann_body.hpp"

namespace dgsn {

namespace {

template <bool kSplit>
__global__ __launch_bounds__(256) void ann_infer_kernel(const unsigned char *__restrict__ prm,
                                                        const float *__restrict__ x,
                                                        float *__restrict__ y, long long n)
{
    AnnRegs R;
    const int lane = threadIdx.x & 63;
    ann_load(prm, lane, R);
    const long long nblk = (n + 255) / 256;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long s = blk * 256 + threadIdx.x;
        float f[24], o[8];
#pragma unroll
        for (int k = 0; k < 24; ++k) f[k] = s < n ? x[s * 24 + k] : 0.0f;
        ann_wave<kSplit>(R, f, o);
        if (s < n) {
#pragma unroll
            for (int k = 0; k < 8; ++k) y[s * 8 + k] = o[k];
        }
    }
}

// Paper-form network on raw inputs: one thread per sample, the octant's
// image (scaling folded into the first layer) read with scalar loads.
__global__ __launch_bounds__(256) void pann_infer_kernel(const float *__restrict__ w,
                                                         const float *__restrict__ x,
                                                         float *__restrict__ y, long long n)
{
    for (long long s = blockIdx.x * 256ll + threadIdx.x; s < n; s += (long long)gridDim.x * 256) {
        float f[kPannIn], o[8];
#pragma unroll
        for (int k = 0; k < kPannIn; ++k) f[k] = x[s * kPannIn + k];
        float pmax = f[0];
#pragma unroll
        for (int j = 1; j < 12; ++j) pmax = fmaxf(pmax, f[j]);
        pann_layers<kPannIn, kPannRawW1, kPannRawB1, kPannRawW2, kPannRawB2, kPannRawBeta>(
            w, f, pmax, o);
#pragma unroll
        for (int k = 0; k < 8; ++k) y[s * 8 + k] = o[k];
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

// the float value of the bf16 rounding of f
float bf16_value(float f)
{
    const uint32_t u = (uint32_t)bf16_bits(f) << 16;
    float v;
    std::memcpy(&v, &u, 4);
    return v;
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
    // operand layouts of v_mfma_f32_32x32x16_bf16 (see ann_body.hpp)
    for (int lane = 0; lane < 64; ++lane) {
        const int row = lane & 31, half = lane >> 5;
        for (int t = 0; t < 2; ++t)
            for (int kk = 0; kk < 2; ++kk) {
                const int hid = 32 * t + row;
                for (int e = 0; e < 8; ++e) {
                    const int f = 16 * kk + 8 * half + e;
                    float v = (hid < H && f < NI) ? a->W1[hid * NI + f] : 0.0f;
                    if (hid < H && f == kFeatBiasHi) v = bf16_value(a->b1[hid]);
                    if (hid < H && f == kFeatBiasLo) v = a->b1[hid] - bf16_value(a->b1[hid]);
                    put_bf16(kParamW1 + ((2 * t + kk) * 64 + lane) * 16 + 2 * e, v);
                }
            }
        for (int kc = 0; kc < 4; ++kc)
            for (int e = 0; e < 8; ++e) {
                const int out = row;
                const int hid = 16 * kc + 8 * (e >> 2) + 4 * half + (e & 3);
                const float v = (out < NO && hid < H) ? a->W2[out * H + hid] : 0.0f;
                put_bf16(kParamW2 + (kc * 64 + lane) * 16 + 2 * e, v);
            }
    }
    for (int out = 0; out < 8; ++out) put_f32(kParamB2 + 4 * out, out < NO ? a->b2[out] : 0.0f);
    DGSN_TRY(a->d_params.alloc(buf.size()));
    DGSN_HIP(hipMemcpy(a->d_params.ptr, buf.data(), buf.size(), hipMemcpyHostToDevice));
    return DGSN_OK;
}

// Versions 2 and 3: the raw-input images of the networks.  Eq. (ANN:Eq2)
// In_j = (I_j - c_j) / r_j with c_j = alpha (Imin_j + Imax_j) / 2 and
// r_j = |Imax_j - Imin_j| is folded into the first layer:
// W1' = W1 / r, b1' = b1 - W1 c / r (hidden units beyond n_hidden are zero).
int build_pann_params(dgsn_ann *a)
{
    const int H = a->n_hidden;
    std::vector<float> img((size_t)a->n_nets * kPannRawStride, 0.0f);
    for (int o = 0; o < a->n_nets; ++o) {
        float *w = img.data() + (size_t)o * kPannRawStride;
        const float *W1 = a->W1.data() + (size_t)o * H * kPannIn;
        const float *b1 = a->b1.data() + (size_t)o * H;
        const float *W2 = a->W2.data() + (size_t)o * 8 * H;
        const float *b2 = a->b2.data() + (size_t)o * 8;
        for (int k = 0; k < H; ++k) {
            double bias = b1[k];
            for (int j = 0; j < kPannIn; ++j) {
                const double c = (double)a->alpha * 0.5 * ((double)a->imin[j] + a->imax[j]);
                const double r = std::fabs((double)a->imax[j] - a->imin[j]);
                w[kPannRawW1 + k * kPannIn + j] = (float)(W1[k * kPannIn + j] / r);
                bias -= W1[k * kPannIn + j] * c / r;
            }
            w[kPannRawB1 + k] = (float)bias;
            for (int t = 0; t < 8; ++t) w[kPannRawW2 + t * kPannHidden + k] = W2[t * H + k];
        }
        for (int t = 0; t < 8; ++t) w[kPannRawB2 + t] = b2[t];
        w[kPannRawBeta] = a->beta_scale;
    }
    DGSN_TRY(a->d_params.alloc(img.size() * sizeof(float)));
    DGSN_HIP(hipMemcpy(a->d_params.ptr, img.data(), img.size() * sizeof(float),
                       hipMemcpyHostToDevice));
    return DGSN_OK;
}

}  // namespace

const void *ann_device_params(const dgsn_ann *a) { return a ? a->d_params.ptr : nullptr; }

// Folding of net k for one problem (cell sizes h) and reflection mask o
// (bit a set: Omega_a < 0; canonical node n' is physical node n' ^ o):
//   canonical inflow face node fn of axis a is physical face node
//   fn ^ (mask bits of the two tangential axes, lower axis first);
//   kappa_a = |Omega_a| / h_a, so Omega_a = s_a h_a kappa_a (s_a = -1 on set bits);
//   canonical source node n' is physical node n' ^ o;
//   the cell sizes are constant inputs, added to the bias;
//   canonical output t' is the physical output t' ^ o.
static void fold_pann(const dgsn_ann *a, int k, int o, const double h[3], float *w)
{
    const int H = a->n_hidden;
    const float *W1 = a->W1.data() + (size_t)k * H * kPannIn;
    const float *b1 = a->b1.data() + (size_t)k * H;
    const float *W2 = a->W2.data() + (size_t)k * 8 * H;
    const float *b2 = a->b2.data() + (size_t)k * 8;
    const int mx = o & 1, my = (o >> 1) & 1, mz = (o >> 2) & 1;
    const int tang[3] = {my | (mz << 1), mx | (mz << 1), mx | (my << 1)};
    for (int u = 0; u < H; ++u) {
        // scaled first layer on the raw physical inputs
        double ws[kPannIn];
        double bias = b1[u];
        for (int j = 0; j < kPannIn; ++j) {
            const double c = (double)a->alpha * 0.5 * ((double)a->imin[j] + a->imax[j]);
            const double r = std::fabs((double)a->imax[j] - a->imin[j]);
            ws[j] = W1[u * kPannIn + j] / r;
            bias -= W1[u * kPannIn + j] * c / r;
        }
        float *r1 = w + kPannW1 + u * kPannFeat;
        for (int ax = 0; ax < 3; ++ax)
            for (int fn = 0; fn < 4; ++fn) r1[4 * ax + fn] = (float)ws[4 * ax + (fn ^ tang[ax])];
        r1[12] = (float)(ws[12] * (mx ? -h[0] : h[0]));
        r1[13] = (float)(ws[13] * (my ? -h[1] : h[1]));
        for (int n = 0; n < 8; ++n) r1[14 + n] = (float)ws[14 + (n ^ o)];
        r1[22] = (float)ws[22];
        for (int ax = 0; ax < 3; ++ax) bias += ws[23 + ax] * h[ax];
        w[kPannB1 + u] = (float)bias;
        for (int t = 0; t < 8; ++t) w[kPannW2 + t * kPannHidden + u] = W2[(t ^ o) * H + u];
    }
    for (int t = 0; t < 8; ++t) w[kPannB2 + t] = b2[t ^ o];
    w[kPannBeta] = a->beta_scale;
}

int pann_problem_image(const dgsn_ann *a, const double h[3], std::vector<float> &out)
{
    if (!a || a->version != 2) return set_error(DGSN_EINVAL, "not a per-octant paper-form network");
    out.assign((size_t)8 * kPannStride, 0.0f);
    for (int o = 0; o < 8; ++o) fold_pann(a, o, o, h, out.data() + (size_t)o * kPannStride);
    return DGSN_OK;
}

// Per-direction networks: slot (o, d) of the problem's octant-sorted
// direction table takes the net whose stored direction equals the slot's
// (every component within kPannDirTol: the artifact holds FP32 cosines).
// Padding slots (valid[o * Do + d] == 0) get zero images.
int pann_problem_image_dir(const dgsn_ann *a, const double h[3], const double *omega, int Do,
                           const int *valid, std::vector<float> &out)
{
    if (!a || a->version != 3)
        return set_error(DGSN_EINVAL, "not a per-direction paper-form network");
    out.assign((size_t)8 * Do * kPannStride, 0.0f);
    for (int o = 0; o < 8; ++o)
        for (int d = 0; d < Do; ++d) {
            const int s = o * Do + d;
            if (!valid[s]) continue;
            const double *om = omega + 3 * (size_t)s;
            int k = -1;
            for (int j = 0; j < a->n_nets && k < 0; ++j) {
                const float *w = a->omega.data() + 3 * (size_t)j;
                if (std::fabs(w[0] - om[0]) <= kPannDirTol && std::fabs(w[1] - om[1]) <= kPannDirTol &&
                    std::fabs(w[2] - om[2]) <= kPannDirTol)
                    k = j;
            }
            if (k < 0)
                return set_error(DGSN_EINVAL,
                                 "direction (%.7f, %.7f, %.7f) of the problem has no network in "
                                 "the per-direction artifact",
                                 om[0], om[1], om[2]);
            fold_pann(a, k, o, h, out.data() + (size_t)s * kPannStride);
        }
    return DGSN_OK;
}

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
    if (data.size() < 8 + 6 * 4 + 4 || std::memcmp(data.data(), "DGSNANN1", 8) != 0)
        return set_error(DGSN_EFORMAT, "%s: not a DGSNANN1 artifact", path);
    uint32_t v[6];
    std::memcpy(v, data.data() + 8, sizeof(v));
    const uint32_t version = v[0], n_in = v[1], n_hidden = v[2], n_out = v[3], act = v[4];
    const uint32_t flags = v[5];
    uint32_t n_nets = 1;
    size_t hdr = 8 + 6 * 4;
    if (version == 2 || version == 3) {
        // u32 n_nets, f32 alpha, f32 beta_scale, f32 imin[26], f32 imax[26]
        // (version 3: then f32 omega[n_nets][3])
        if (data.size() < hdr + 4 + 8 + 8 * 26 + 4)
            return set_error(DGSN_EFORMAT, "%s: truncated version-%u header", path, version);
        std::memcpy(&n_nets, data.data() + hdr, 4);
        hdr += 4 + 8 + 2 * 4 * 26;
        const bool nets_ok = version == 2 ? n_nets == 8 : (n_nets >= 1 && n_nets <= kPannMaxDirs);
        if (n_in != (uint32_t)kPannIn || n_out != 8 || !nets_ok || n_hidden < 1 ||
            n_hidden > (uint32_t)kPannHidden || act != 1 || flags != 1)
            return set_error(DGSN_EFORMAT,
                             "%s: unsupported version-%u shape (%u-%u-%u, %u nets, act %u, "
                             "flags %u; expected 26-(1..8)-8, %s, tanh, ELU output)",
                             path, version, n_in, n_hidden, n_out, n_nets, act, flags,
                             version == 2 ? "8 nets" : "1..4096 nets");
        if (version == 3) {
            if (data.size() < hdr + 12 * (size_t)n_nets + 4)
                return set_error(DGSN_EFORMAT, "%s: truncated direction table", path);
            hdr += 12 * (size_t)n_nets;
        }
    } else if (version != 1 || n_in != 24 || n_out != 8 || n_hidden < 1 ||
               n_hidden > kMaxHidden) {
        return set_error(DGSN_EFORMAT, "%s: unsupported shape (version %u, %u-%u-%u)", path,
                         version, n_in, n_hidden, n_out);
    }
    const size_t per_net =
        (size_t)n_hidden * n_in + n_hidden + (size_t)n_out * n_hidden + n_out;
    const size_t nparam = per_net * n_nets;
    if (data.size() != hdr + 4 * nparam + 4)
        return set_error(DGSN_EFORMAT, "%s: size %zu does not match the header", path,
                         data.size());
    uint32_t crc;
    std::memcpy(&crc, data.data() + data.size() - 4, 4);
    if (crc != crc32_ieee(data.data(), data.size() - 4))
        return set_error(DGSN_EFORMAT, "%s: checksum mismatch", path);
    if (version == 1 && act != 0)
        return set_error(DGSN_EUNSUPPORTED, "%s: only ReLU hidden layers run on the matrix cores",
                         path);
    if (version == 1 && n_hidden > kHiddenPad)
        return set_error(DGSN_EUNSUPPORTED, "%s: at most %d hidden units are supported", path,
                         kHiddenPad);
    float alpha = 0.0f, beta_scale = 0.0f;
    std::vector<float> imin, imax, omega;
    if (version >= 2) {
        const unsigned char *q = data.data() + 8 + 6 * 4 + 4;
        std::memcpy(&alpha, q, 4);
        std::memcpy(&beta_scale, q + 4, 4);
        imin.resize(kPannIn);
        imax.resize(kPannIn);
        std::memcpy(imin.data(), q + 8, 4 * kPannIn);
        std::memcpy(imax.data(), q + 8 + 4 * kPannIn, 4 * kPannIn);
        if (!std::isfinite(alpha) || !std::isfinite(beta_scale) || beta_scale < 0.0f)
            return set_error(DGSN_EFORMAT, "%s: bad alpha / beta scale", path);
        for (int j = 0; j < kPannIn; ++j)
            if (!std::isfinite(imin[j]) || !std::isfinite(imax[j]) || imin[j] == imax[j])
                return set_error(DGSN_EFORMAT, "%s: bad input bounds of input %d", path, j);
        if (version == 3) {
            omega.resize(3 * (size_t)n_nets);
            std::memcpy(omega.data(), q + 8 + 8 * kPannIn, 12 * (size_t)n_nets);
            for (uint32_t k = 0; k < n_nets; ++k) {
                const float *w = omega.data() + 3 * (size_t)k;
                const double len2 = (double)w[0] * w[0] + (double)w[1] * w[1] + (double)w[2] * w[2];
                if (!std::isfinite(len2) || std::fabs(len2 - 1.0) > 1e-5)
                    return set_error(DGSN_EFORMAT, "%s: direction %u is not a unit vector", path,
                                     k);
                for (uint32_t j = 0; j < k; ++j) {
                    const float *v = omega.data() + 3 * (size_t)j;
                    if (std::fabs(w[0] - v[0]) <= kPannDirTol && std::fabs(w[1] - v[1]) <= kPannDirTol &&
                        std::fabs(w[2] - v[2]) <= kPannDirTol)
                        return set_error(DGSN_EFORMAT, "%s: directions %u and %u coincide", path,
                                         j, k);
                }
            }
        }
    }
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
    a->version = (int)version;
    a->n_in = (int)n_in;
    a->n_hidden = (int)n_hidden;
    a->n_out = (int)n_out;
    a->act = (int)act;
    a->n_nets = (int)n_nets;
    a->alpha = alpha;
    a->beta_scale = beta_scale;
    a->imin = imin;
    a->imax = imax;
    a->omega = omega;
    const float *pf = reinterpret_cast<const float *>(data.data() + hdr);
    for (uint32_t k = 0; k < n_nets; ++k) {
        a->W1.insert(a->W1.end(), pf, pf + (size_t)n_hidden * n_in);
        pf += (size_t)n_hidden * n_in;
        a->b1.insert(a->b1.end(), pf, pf + n_hidden);
        pf += n_hidden;
        a->W2.insert(a->W2.end(), pf, pf + (size_t)n_out * n_hidden);
        pf += (size_t)n_out * n_hidden;
        a->b2.insert(a->b2.end(), pf, pf + n_out);
        pf += n_out;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        delete a;
        return set_error(DGSN_EHIP, "hipSetDevice failed");
    }
    int rc = version >= 2 ? build_pann_params(a) : build_params(a);
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

int dgsn_ann_info(const dgsn_ann *ann, int *version, int *n_in, int *n_hidden, int *n_nets)
{
    clear_error();
    if (!ann) return set_error(DGSN_EINVAL, "ann is NULL");
    if (version) *version = ann->version;
    if (n_in) *n_in = ann->n_in;
    if (n_hidden) *n_hidden = ann->n_hidden;
    if (n_nets) *n_nets = ann->n_nets;
    return DGSN_OK;
}

int dgsn_ann_infer_octant(const dgsn_ann *ann, int octant, const float *x, float *y, long long n,
                          void *stream)
{
    clear_error();
    if (!ann) return set_error(DGSN_EINVAL, "ann is NULL");
    if (ann->version < 2)
        return set_error(DGSN_EINVAL, "dgsn_ann_infer_octant needs a paper-form (version 2 or "
                                      "3) artifact; use dgsn_ann_infer");
    if (octant < 0 || octant >= ann->n_nets)
        return set_error(DGSN_EINVAL, "net index %d is outside 0..%d", octant, ann->n_nets - 1);
    if (n < 0) return set_error(DGSN_EINVAL, "n must be >= 0");
    if (n == 0) return DGSN_OK;
    if (!x || !y) return set_error(DGSN_EINVAL, "x and y must be set");
    DGSN_HIP(hipSetDevice(ann->ctx->device));
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(pann_infer_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream),
                       static_cast<const float *>(ann->d_params.ptr) +
                           (size_t)octant * kPannRawStride,
                       x, y, n);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

int dgsn_ann_set_mode(dgsn_ann *ann, int mode)
{
    clear_error();
    if (!ann) return set_error(DGSN_EINVAL, "ann is NULL");
    if (mode != DGSN_ANN_BF16 && mode != DGSN_ANN_BF16X2)
        return set_error(DGSN_EINVAL, "mode must be DGSN_ANN_BF16 or DGSN_ANN_BF16X2");
    if (ann->version != 1 && mode != DGSN_ANN_BF16)
        return set_error(DGSN_EINVAL, "the paper-form networks run in FP32 on the vector ALUs");
    ann->mode = mode;
    return DGSN_OK;
}

int dgsn_ann_infer(const dgsn_ann *ann, const float *x, float *y, long long n, void *stream)
{
    clear_error();
    if (!ann) return set_error(DGSN_EINVAL, "ann is NULL");
    if (ann->version != 1)
        return set_error(DGSN_EINVAL, "dgsn_ann_infer needs a version-1 artifact; use "
                                      "dgsn_ann_infer_octant for the paper-form networks");
    if (n < 0) return set_error(DGSN_EINVAL, "n must be >= 0");
    if (n == 0) return DGSN_OK;
    if (!x || !y) return set_error(DGSN_EINVAL, "x and y must be set");
    DGSN_HIP(hipSetDevice(ann->ctx->device));
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (ann->mode == DGSN_ANN_BF16X2)
        hipLaunchKernelGGL(ann_infer_kernel<true>, dim3((unsigned)blocks), dim3(256), 0,
                           reinterpret_cast<hipStream_t>(stream),
                           static_cast<const unsigned char *>(ann->d_params.ptr), x, y, n);
    else
        hipLaunchKernelGGL(ann_infer_kernel<false>, dim3((unsigned)blocks), dim3(256), 0,
                           reinterpret_cast<hipStream_t>(stream),
                           static_cast<const unsigned char *>(ann->d_params.ptr), x, y, n);
    DGSN_HIP(hipGetLastError());
    return DGSN_OK;
}

}  // extern "C"
