#include "distill.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "distill_kernels.h"

namespace lic {

#define D_TRY(expr)                                                                \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
            return LIC_E_HIP;                                                      \
        }                                                                          \
    } while (0)

namespace {

// parameter arrays: t1.w [M][F][5][5], t1.b [F], t2.w [F][F][5][5], t2.b [F],
// t3.w [F][3][8][8], t3.b [3]
void param_layout(int M, int F, long* off, long* total)
{
    const long len[6] = {(long)M * F * 25, F, (long)F * F * 25, F, (long)F * 3 * 64, 3};
    long o = 0;
    for (int i = 0; i < 6; ++i) {
        off[i] = o;
        o += len[i];
    }
    *total = o;
}

long round_up(long v, long m) { return (v + m - 1) / m * m; }

}  // namespace

void* DistillNet::alloc(size_t bytes)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) return nullptr;
    allocs.push_back(p);
    return p;
}

DistillNet::~DistillNet()
{
    if (hipSetDevice(cfg.hip_device) == hipSuccess && stream) (void)hipStreamSynchronize(stream);
    for (void* p : allocs) (void)hipFree(p);
    if (stream) (void)hipStreamDestroy(stream);
}

int DistillNet::build_layer(Layer& L, int tag, int ld, int ep, int dt, PackKind kind, int ci, int co, int k, int s,
                            int p, bool w_deconv, int kimg, long src_w, long src_b, std::vector<int32_t>& idx,
                            std::vector<int32_t>& bidx)
{
    const PackMap pm = pack_map(kind, ci, co, k, s, p, w_deconv, kimg);
    L.shape = ConvShape{tag, ld, ep, dt, pm.cin, pm.cop, (int)pm.ph.size()};
    // every tap within one pixel of the (stride-1) phase grid: halo tiles allowed
    L.shape.halo1 = ld != LD_RGB;
    for (const PhaseDesc& d : pm.ph)
        for (int t = 0; t < d.ntaps; ++t)
            if (d.dy[t] < -1 || d.dy[t] > 1 || d.dx[t] < -1 || d.dx[t] > 1) L.shape.halo1 = 0;
    L.co = co;
    L.k = k;
    L.s = s;
    L.p = p;
    L.w_off = (long)idx.size();
    for (int32_t j : pm.idx) idx.push_back(j < 0 ? -1 : (int32_t)(src_w + j));
    L.ph = pm.ph;
    for (size_t i = 0; i < L.ph.size(); ++i) L.ph[i].woff = (int64_t)(L.w_off + pm.off[i]);
    if (src_b >= 0) {
        L.b_off = (long)bidx.size();
        for (int32_t j : pm.bias_idx) bidx.push_back(j < 0 ? -1 : (int32_t)(src_b + j));
    }
    return LIC_OK;
}

int DistillNet::create(const lic_distill_config& c, const float* params, size_t n)
{
    cfg = c;
    M = c.M;
    F = c.F;
    if (M <= 0 || M % 64 != 0 || (M != 192 && M != 320) || F != 64) { err = "supported shapes: M 192 or 320, F 64"; return LIC_E_ARG; }
    if (c.precision != LIC_PREC_FP32 && c.precision != LIC_PREC_BF16) { err = "precision must be FP32 or BF16"; return LIC_E_ARG; }
    if (c.train && c.precision != LIC_PREC_FP32) { err = "training needs the FP32 forward"; return LIC_E_ARG; }
    if (c.max_batch < 1 || c.max_batch > 64 || c.max_hy < 1 || c.max_wy < 1 || c.max_hy > 4096 || c.max_wy > 4096) {
        err = "max_batch must be 1..64 and the latent grid positive";
        return LIC_E_ARG;
    }
    param_layout(M, F, off, &nparam);
    if (!params || n != (size_t)nparam) { err = "parameter count does not match (M, F)"; return LIC_E_ARG; }
    D_TRY(hipSetDevice(c.hip_device));
    D_TRY(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));

    const int fdt = c.precision == LIC_PREC_BF16 ? DT_BF16 : DT_F32;
    std::vector<int32_t> idx, bidx;
    build_layer(fwd[0], TAG_DT1, LD_I8, EP_RELU, fdt, PK_DECONV, M, F, 5, 2, 2, true, 0, off[0], off[1], idx, bidx);
    build_layer(fwd[1], TAG_DT2, LD_F32, EP_RELU, fdt, PK_DECONV, F, F, 5, 2, 2, true, 0, off[2], off[3], idx, bidx);
    build_layer(fwd[2], TAG_DT3, LD_F32, EP_RGB, fdt, PK_ROWS, F, 3, 8, 4, 2, true, 0, off[4], off[5], idx, bidx);
    n_fwd_w = (long)idx.size();
    // input gradients: strided convolutions with the same weight arrays read
    // as [C_out = C_in of the transposed convolution][C_in][k][k]
    build_layer(dg2, TAG_DB2, LD_F32, EP_MASK, DT_F32, PK_CONV, F, F, 5, 2, 2, false, 0, off[2], -1, idx, bidx);
    build_layer(dg3, TAG_DB3, LD_RGB, EP_MASK, DT_F32, PK_IMG, 3, F, 8, 4, 2, false, 192, off[4], -1, idx, bidx);
    const long n_w = (long)idx.size();
    for (Layer* L : {&fwd[0], &fwd[1], &fwd[2]})
        if (L->b_off >= 0) L->b_off += n_w;
    idx.insert(idx.end(), bidx.begin(), bidx.end());
    n_arena = (long)idx.size();

    d_master = (float*)alloc(nparam * sizeof(float));
    d_pidx = (int32_t*)alloc(n_arena * sizeof(int32_t));
    d_arena32 = (float*)alloc(n_arena * sizeof(float));
    if (fdt == DT_BF16) d_arena16 = alloc(n_fwd_w * 2);
    d_zero = (float*)alloc(1024 * sizeof(float));
    if (!d_master || !d_pidx || !d_arena32 || (fdt == DT_BF16 && !d_arena16) || !d_zero) { err = "device allocation failed"; return LIC_E_NOMEM; }
    D_TRY(hipMemcpy(d_master, params, nparam * sizeof(float), hipMemcpyHostToDevice));
    D_TRY(hipMemcpy(d_pidx, idx.data(), n_arena * sizeof(int32_t), hipMemcpyHostToDevice));
    D_TRY(hipMemset(d_zero, 0, 1024 * sizeof(float)));
    for (Layer* L : {&fwd[0], &fwd[1], &fwd[2], &dg2, &dg3}) {
        const std::vector<PhaseDesc>& ph = L->ph;
        L->d_ph = (PhaseDesc*)alloc(ph.size() * sizeof(PhaseDesc));
        if (!L->d_ph) { err = "device allocation failed"; return LIC_E_NOMEM; }
        D_TRY(hipMemcpy(L->d_ph, ph.data(), ph.size() * sizeof(PhaseDesc), hipMemcpyHostToDevice));
    }

    // activations for the largest call
    const long B = c.max_batch, hy = c.max_hy, wy = c.max_wy;
    const size_t act = fdt == DT_BF16 ? 2 : 4;
    d_h1 = alloc(B * 4 * hy * wy * F * act);
    d_h2 = alloc(B * 16 * hy * wy * F * act);
    d_mpart = (float*)alloc(2 * B * 3 * 16 * sizeof(float));
    d_loss = (float*)alloc(16 * sizeof(float));
    if (!d_h1 || !d_h2 || !d_mpart || !d_loss) { err = "device allocation failed"; return LIC_E_NOMEM; }
    if (c.train) {
        const long img = B * 3 * 256 * hy * wy;
        d_m = (float*)alloc(nparam * sizeof(float));
        d_v = (float*)alloc(nparam * sizeof(float));
        d_grad = (float*)alloc(nparam * sizeof(float));
        d_pre = (float*)alloc(img * sizeof(float));
        d_dout = (float*)alloc(img * sizeof(float));
        d_tgt = (float*)alloc(img * sizeof(float));
        d_sym = (int8_t*)alloc(B * hy * wy * M);
        d_dh2 = (float*)alloc(B * 16 * hy * wy * F * sizeof(float));
        d_dh1 = (float*)alloc(B * 4 * hy * wy * F * sizeof(float));
        d_cpart = (float*)alloc(256 * F * sizeof(float));
        part_cap = 3L * 1024 * 1024 * 4;   // 48 MiB of weight-gradient partial sums
        d_part = (float*)alloc(part_cap * sizeof(float));
        if (!d_m || !d_v || !d_grad || !d_pre || !d_dout || !d_tgt || !d_sym || !d_dh2 || !d_dh1 || !d_cpart || !d_part) {
            err = "device allocation failed";
            return LIC_E_NOMEM;
        }
        D_TRY(hipMemset(d_m, 0, nparam * sizeof(float)));
        D_TRY(hipMemset(d_v, 0, nparam * sizeof(float)));
        D_TRY(hipMemset(d_grad, 0, nparam * sizeof(float)));
    }
    const int rc = repack();
    if (rc != LIC_OK) return rc;
    D_TRY(hipStreamSynchronize(stream));
    return LIC_OK;
}

int DistillNet::repack()
{
    D_TRY(launch_gather_pack(d_master, d_pidx, n_arena, d_arena32, nullptr, stream));
    if (d_arena16) D_TRY(launch_gather_pack(d_master, d_pidx, n_fwd_w, nullptr, d_arena16, stream));
    return LIC_OK;
}

int DistillNet::check_dims(int n, int hy, int wy)
{
    if (n < 1 || n > cfg.max_batch || hy < 1 || wy < 1 || hy > cfg.max_hy || wy > cfg.max_wy) {
        err = "batch or latent grid outside the configured maximum";
        return LIC_E_BUDGET;
    }
    return LIC_OK;
}

size_t DistillNet::hidden_bytes(int n, int hy, int wy, size_t* h2_off) const
{
    const size_t act = cfg.precision == LIC_PREC_BF16 ? 2 : 4;
    const size_t px = (size_t)n * hy * wy * F * act;
    const size_t b1 = (4 * px + 255) / 256 * 256;
    if (h2_off) *h2_off = b1;
    return b1 + 16 * px;
}

int DistillNet::forward(const int8_t* sym, const float* mu, int n, int hy, int wy, float* pre, float* x_hat, int H,
                        int W, hipStream_t s, void* h1, void* h2)
{
    int rc = check_dims(n, hy, wy);
    if (rc != LIC_OK) return rc;
    if (!h1) h1 = d_h1;
    if (!h2) h2 = d_h2;
    if (x_hat && (H < 1 || W < 1 || H > 16 * hy || W > 16 * wy)) { err = "crop larger than the decoded grid"; return LIC_E_ARG; }
    auto base = [&](const Layer& L, const void* in, void* out, void* aux, int Hin, int Win, int s_out, int Hout,
                    int Wout) {
        ConvArgs a{};
        a.in = in;
        a.out = out;
        a.aux = aux;
        a.ph = L.d_ph;
        a.w = L.shape.dt == DT_BF16 ? d_arena16 : (const void*)d_arena32;
        a.zero = d_zero;
        a.bias = L.b_off >= 0 ? d_arena32 + L.b_off : d_zero;
        a.mu_in = mu ? mu : d_zero;
        a.n = n;
        a.Hin = Hin;
        a.Win = Win;
        a.Hg = Hin;
        a.Wg = Win;
        a.s_in = 1;
        a.Hout = Hout;
        a.Wout = Wout;
        a.s_out = s_out;
        a.Co = L.co;
        a.nphase = L.shape.nphase;
        a.kk = L.k;
        a.pad = L.p;
        return a;
    };
    ConvArgs a1 = base(fwd[0], sym, h1, nullptr, hy, wy, 2, 2 * hy, 2 * wy);
    ConvArgs a2 = base(fwd[1], h1, h2, nullptr, 2 * hy, 2 * wy, 2, 4 * hy, 4 * wy);
    ConvArgs a3 = base(fwd[2], h2, x_hat, pre, 4 * hy, 4 * wy, 4, 16 * hy, 16 * wy);
    a3.Hc = H;
    a3.Wc = W;
    if ((rc = launch_conv_policy(fwd[0].shape, a1, (long)hy * wy, s, &err)) != LIC_OK) return rc;
    if ((rc = launch_conv_policy(fwd[1].shape, a2, 4L * hy * wy, s, &err)) != LIC_OK) return rc;
    return launch_conv_policy(fwd[2].shape, a3, 16L * hy * wy, s, &err);
}

int DistillNet::backward(const int8_t* sym, const float* mu, const float* target, int n, int hy, int wy,
                         float* loss_dev)
{
    if (!cfg.train) { err = "created without training state"; return LIC_E_STATE; }
    int rc = forward(sym, mu, n, hy, wy, d_pre, nullptr, 0, 0, stream);
    if (rc != LIC_OK) return rc;
    const int Ho = 16 * hy, Wo = 16 * wy;
    const long plane = (long)Ho * Wo;
    const int chunks = 16;
    D_TRY(launch_mse(d_pre, target, n, plane, chunks, d_dout, d_mpart, d_mpart + (long)n * 3 * chunks,
                     loss_dev ? loss_dev : d_loss, d_grad + off[5], stream));

    // splits the weight-gradient contraction over about 2048 blocks
    auto wgrad = [&](const void* x, int xt, const float* g, int gt, int H, int W, int ci, int Hg, int Wg, int co, int k,
                     int s, int p, float* dw) -> int {
        WgradArgs w{};
        w.x = x;
        w.mu = mu ? mu : d_zero;
        w.g = g;
        w.part = d_part;
        w.dw = dw;
        w.n = n;
        w.H = H;
        w.W = W;
        w.ci = ci;
        w.Ho = Hg;
        w.Wo = Wg;
        w.co = co;
        w.k = k;
        w.s = s;
        w.p = p;
        const long ncol = (long)k * k * co;
        w.ncol_tiles = (int)((ncol + 63) / 64);
        const long tiles = (long)(ci / 64) * w.ncol_tiles;
        const long P = (long)n * H * W;
        const long max_chunks = std::max(1L, part_cap / (ci * ncol));
        const long want = std::min(max_chunks, std::max(1L, 2048 / tiles));
        w.chunk = (int)std::max(64L, round_up((P + want - 1) / want, 16));
        if ((P + w.chunk - 1) / w.chunk > max_chunks) w.chunk = (int)round_up((P + max_chunks - 1) / max_chunks, 16);
        const hipError_t e = launch_wgrad(w, xt, gt, stream);
        if (e != hipSuccess) { err = std::string("weight-gradient launch failed: ") + hipGetErrorString(e); return LIC_E_HIP; }
        return LIC_OK;
    };
    auto colsum = [&](const float* g, long P, float* out) -> int {
        const int chunk = (int)std::max(256L, (P + 255) / 256);
        const hipError_t e = launch_colsum(g, P, F, chunk, d_cpart, out, stream);
        if (e != hipSuccess) { err = std::string("bias-gradient launch failed: ") + hipGetErrorString(e); return LIC_E_HIP; }
        return LIC_OK;
    };
    auto dgrad = [&](const Layer& L, const void* in, int Hin, int Win, int Hout, int Wout, const void* mask,
                     float* out) -> int {
        ConvArgs a{};
        a.in = in;
        a.out = out;
        a.aux = const_cast<void*>(mask);
        a.ph = L.d_ph;
        a.w = d_arena32;
        a.zero = d_zero;
        a.bias = d_zero;
        a.mu_in = d_zero;
        a.n = n;
        a.Hin = Hin;
        a.Win = Win;
        a.Hg = Hout;
        a.Wg = Wout;
        a.s_in = L.s;
        a.Hout = Hout;
        a.Wout = Wout;
        a.s_out = 1;
        a.Co = F;
        a.nphase = 1;
        a.kk = L.k;
        a.pad = L.p;
        return launch_conv_policy(L.shape, a, (long)Hout * Wout, stream, &err);
    };

    // third layer: weights from h2 and the output gradient; then dH2
    if ((rc = wgrad(d_h2, XT_F32, d_dout, GT_NCHW3, 4 * hy, 4 * wy, F, Ho, Wo, 3, 8, 4, 2, d_grad + off[4])) != LIC_OK) return rc;
    if ((rc = dgrad(dg3, d_dout, Ho, Wo, 4 * hy, 4 * wy, d_h2, d_dh2)) != LIC_OK) return rc;
    // second layer
    if ((rc = colsum(d_dh2, (long)n * 16 * hy * wy, d_grad + off[3])) != LIC_OK) return rc;
    if ((rc = wgrad(d_h1, XT_F32, d_dh2, GT_NHWC, 2 * hy, 2 * wy, F, 4 * hy, 4 * wy, F, 5, 2, 2, d_grad + off[2])) != LIC_OK) return rc;
    if ((rc = dgrad(dg2, d_dh2, 4 * hy, 4 * wy, 2 * hy, 2 * wy, d_h1, d_dh1)) != LIC_OK) return rc;
    // first layer
    if ((rc = colsum(d_dh1, (long)n * 4 * hy * wy, d_grad + off[1])) != LIC_OK) return rc;
    return wgrad(sym, XT_I8, d_dh1, GT_NHWC, hy, wy, M, 2 * hy, 2 * wy, F, 5, 2, 2, d_grad + off[0]);
}

int DistillNet::update()
{
    ++t;
    AdamCoef k;
    k.lr = (float)cfg.lr;
    k.b1 = (float)cfg.beta1;
    k.omb1 = (float)(1.0 - cfg.beta1);
    k.b2 = (float)cfg.beta2;
    k.omb2 = (float)(1.0 - cfg.beta2);
    k.eps = (float)cfg.eps;
    k.decay = (float)(1.0 - cfg.lr * cfg.weight_decay);
    k.c1 = (float)(1.0 - pow(cfg.beta1, (double)t));
    k.c2 = (float)(1.0 - pow(cfg.beta2, (double)t));
    D_TRY(launch_adamw(d_master, d_m, d_v, d_grad, nparam, k, stream));
    return repack();
}

}  // namespace lic

// ------------------------------------------------------------------ C ABI
using lic::DistillNet;

struct lic_distill : public DistillNet {};

extern "C" {

void lic_distill_default_config(lic_distill_config* c)
{
    if (!c) return;
    memset(c, 0, sizeof(*c));
    c->struct_size = sizeof(*c);
    c->M = 192;
    c->F = 64;
    c->precision = LIC_PREC_FP32;
    c->max_batch = 32;
    c->max_hy = 16;
    c->max_wy = 16;
    c->train = 1;
    c->lr = 1e-3;
    c->beta1 = 0.9;
    c->beta2 = 0.999;
    c->eps = 1e-8;
    c->weight_decay = 0.01;
    c->hip_device = 0;
}

size_t lic_distill_param_count(int M, int F)
{
    if (M <= 0 || F <= 0) return 0;
    long off[6], total;
    lic::param_layout(M, F, off, &total);
    return (size_t)total;
}

int lic_distill_create(const lic_distill_config* cfg, const float* params, size_t n_params, lic_distill_t** out)
{
    if (!cfg || !out || cfg->struct_size != sizeof(lic_distill_config)) return LIC_E_ARG;
    *out = nullptr;
    lic_distill* d = new (std::nothrow) lic_distill();
    if (!d) return LIC_E_NOMEM;
    const int rc = d->create(*cfg, params, n_params);
    *out = d;   // kept on failure so that lic_distill_last_error can report; caller destroys
    return rc;
}

void lic_distill_destroy(lic_distill_t* d) { delete d; }

const char* lic_distill_last_error(const lic_distill_t* d) { return d ? d->err.c_str() : "null handle"; }

int lic_distill_forward(lic_distill_t* d, const int8_t* sym, const float* mu, int n, int hy, int wy, float* pre,
                        float* x_hat, int H, int W)
{
    if (!d || !sym || (!pre && !x_hat)) return LIC_E_ARG;
    if (hipSetDevice(d->cfg.hip_device) != hipSuccess) return LIC_E_HIP;
    const int rc = d->forward(sym, mu, n, hy, wy, pre, x_hat, H, W, d->stream);
    if (rc != LIC_OK) return rc;
    if (hipStreamSynchronize(d->stream) != hipSuccess) { d->err = "forward failed"; return LIC_E_HIP; }
    return LIC_OK;
}

int lic_distill_forward_noalloc(lic_distill_t* d, const int8_t* sym, const float* mu, int n, int hy, int wy,
                                float* pre, float* x_hat, int H, int W)
{
    if (!d || !sym || (!pre && !x_hat)) return LIC_E_ARG;
    int rc = d->check_dims(n, hy, wy);
    if (rc != LIC_OK) return rc;
    if (hipSetDevice(d->cfg.hip_device) != hipSuccess) return LIC_E_HIP;
    void* ws = nullptr;
    size_t cap = 0;
    const hipError_t e = lic::distill_scratch(&ws, &cap);
    if (e != hipSuccess) {
        d->err = std::string("workspace lookup failed: ") + hipGetErrorString(e);
        return LIC_E_HIP;
    }
    size_t h2_off = 0;
    const size_t need = d->hidden_bytes(n, hy, wy, &h2_off);
    if (need > cap) {
        d->err = "hidden activations need " + std::to_string(need) + " bytes; the fixed workspace holds " +
                 std::to_string(cap);
        return LIC_E_BUDGET;
    }
    rc = d->forward(sym, mu, n, hy, wy, pre, x_hat, H, W, d->stream, ws, static_cast<char*>(ws) + h2_off);
    if (rc != LIC_OK) return rc;
    if (hipStreamSynchronize(d->stream) != hipSuccess) { d->err = "forward failed"; return LIC_E_HIP; }
    return LIC_OK;
}

int lic_distill_grads(lic_distill_t* d, const int8_t* sym, const float* mu, const float* target, int n, int hy,
                      int wy, float* grads, float* loss)
{
    if (!d || !sym || !target) return LIC_E_ARG;
    if (hipSetDevice(d->cfg.hip_device) != hipSuccess) return LIC_E_HIP;
    const int rc = d->backward(sym, mu, target, n, hy, wy, d->d_loss);
    if (rc != LIC_OK) return rc;
    if (grads && hipMemcpyAsync(grads, d->d_grad, d->nparam * sizeof(float), hipMemcpyDeviceToHost, d->stream) != hipSuccess)
        return LIC_E_HIP;
    if (loss && hipMemcpyAsync(loss, d->d_loss, sizeof(float), hipMemcpyDeviceToHost, d->stream) != hipSuccess)
        return LIC_E_HIP;
    if (hipStreamSynchronize(d->stream) != hipSuccess) { d->err = "backward failed"; return LIC_E_HIP; }
    return LIC_OK;
}

int lic_distill_step(lic_distill_t* d, const int8_t* sym_all, const float* mu, const float* target_all, long count,
                     const int32_t* idx, int n, int hy, int wy, float* loss_dev)
{
    if (!d || !sym_all || !target_all || !idx || count < 1) return LIC_E_ARG;
    if (!d->cfg.train) { d->err = "created without training state"; return LIC_E_STATE; }
    int rc = d->check_dims(n, hy, wy);
    if (rc != LIC_OK) return rc;
    if (hipSetDevice(d->cfg.hip_device) != hipSuccess) return LIC_E_HIP;
    lic::SampleList sl{};
    for (int i = 0; i < n; ++i) {
        if (idx[i] < 0 || idx[i] >= count) { d->err = "sample index out of range"; return LIC_E_ARG; }
        sl.idx[i] = idx[i];
    }
    const long sym_bytes = (long)hy * wy * d->M;
    const long tgt_bytes = 3L * 256 * hy * wy * sizeof(float);
    if (lic::launch_gather_samples(sym_all, sym_bytes, sl, n, d->d_sym, d->stream) != hipSuccess ||
        lic::launch_gather_samples(target_all, tgt_bytes, sl, n, d->d_tgt, d->stream) != hipSuccess) {
        d->err = "batch gather failed";
        return LIC_E_HIP;
    }
    if ((rc = d->backward(d->d_sym, mu, d->d_tgt, n, hy, wy, loss_dev)) != LIC_OK) return rc;
    return d->update();
}

int lic_distill_sync(lic_distill_t* d)
{
    if (!d) return LIC_E_ARG;
    if (hipSetDevice(d->cfg.hip_device) != hipSuccess || hipStreamSynchronize(d->stream) != hipSuccess) {
        d->err = "stream failed";
        return LIC_E_HIP;
    }
    return LIC_OK;
}

int lic_distill_get(lic_distill_t* d, int what, float* out, size_t n)
{
    if (!d || !out || n != (size_t)d->nparam || what < 0 || what > 3) return LIC_E_ARG;
    const float* src = what == 0 ? d->d_master : what == 1 ? d->d_m : what == 2 ? d->d_v : d->d_grad;
    if (!src) { d->err = "created without training state"; return LIC_E_STATE; }
    if (hipSetDevice(d->cfg.hip_device) != hipSuccess ||
        hipMemcpyAsync(out, src, n * sizeof(float), hipMemcpyDeviceToHost, d->stream) != hipSuccess ||
        hipStreamSynchronize(d->stream) != hipSuccess)
        return LIC_E_HIP;
    return LIC_OK;
}

int lic_distill_set(lic_distill_t* d, int what, const float* in, size_t n)
{
    if (!d || !in || n != (size_t)d->nparam || what < 0 || what > 2) return LIC_E_ARG;
    float* dst = what == 0 ? d->d_master : what == 1 ? d->d_m : d->d_v;
    if (!dst) { d->err = "created without training state"; return LIC_E_STATE; }
    if (hipSetDevice(d->cfg.hip_device) != hipSuccess ||
        hipMemcpyAsync(dst, in, n * sizeof(float), hipMemcpyHostToDevice, d->stream) != hipSuccess)
        return LIC_E_HIP;
    if (what == 0 && d->repack() != LIC_OK) return LIC_E_HIP;
    return hipStreamSynchronize(d->stream) == hipSuccess ? LIC_OK : LIC_E_HIP;
}

int lic_distill_get_step(lic_distill_t* d, int64_t* t)
{
    if (!d || !t) return LIC_E_ARG;
    *t = d->t;
    return LIC_OK;
}

int lic_distill_set_step(lic_distill_t* d, int64_t t)
{
    if (!d || t < 0) return LIC_E_ARG;
    d->t = t;
    return LIC_OK;
}

}  // extern "C"
