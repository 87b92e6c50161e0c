// C ABI entry points (include/lic.h).
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <new>
#include <vector>

#include "codec.h"

using lic::Codec;

struct codec : public Codec {};

namespace {

thread_local std::string g_create_error;

int fail(Codec* c, int code, const std::string& msg)
{
    c->err = msg;
    return code;
}

bool supported_shape(int kind, int N, int M)
{
    const bool hyper_ok = (N == 128 && M == 192) || (N == 192 && M == 320);
    if (kind == LIC_KIND_CONTEXT) return N == 128 && M == 192;
    return kind == LIC_KIND_HYPERPRIOR ? hyper_ok : (kind == LIC_KIND_FACTORIZED && hyper_ok);
}

bool check_frame(Codec* c, int n, int H, int W, int* rc)
{
    if (n < 0 || H < 1 || W < 1) { *rc = fail(c, LIC_E_ARG, "bad frame count or size"); return false; }
    if (H > c->cfg.max_h || W > c->cfg.max_w) { *rc = fail(c, LIC_E_BUDGET, "frame larger than max_h x max_w"); return false; }
    return true;
}

// Groups frames [0, n) into tasks of up to max_batch consecutive frames.
void make_tasks(Codec* c, lic::CallState& cs, const float* x, float* x_hat, size_t fsz)
{
    const int B = c->cfg.max_batch;
    for (int f = 0; f < cs.n; f += B) {
        lic::Task* t = new lic::Task();
        t->first = f;
        t->nb = std::min(B, cs.n - f);
        for (int b = 0; b < t->nb; ++b) {
            t->xs[b] = x ? x + (size_t)(f + b) * fsz : nullptr;
            t->xhats[b] = x_hat ? x_hat + (size_t)(f + b) * fsz : nullptr;
        }
        cs.tasks.emplace_back(t);
    }
}

}  // namespace

extern "C" {

void codec_default_config(codec_config* cfg)
{
    if (!cfg) return;
    memset(cfg, 0, sizeof(*cfg));
    cfg->struct_size = sizeof(codec_config);
    cfg->kind = LIC_KIND_HYPERPRIOR;
    cfg->N = 128;
    cfg->M = 192;
    cfg->precision = LIC_PREC_FP32;
    cfg->hs_out = LIC_HS_EXP;
    cfg->gs_mode = 0;
    cfg->y_slices = 8;
    cfg->entropy_threads = 8;
    cfg->zero_copy = 1;
    cfg->max_in_flight = 6;
    cfg->max_h = 1088;
    cfg->max_w = 1920;
    cfg->max_batch = 1;
    cfg->hbm_budget_bytes = 0;
    cfg->hip_device = 0;
    cfg->use_graphs = 1;
    cfg->norm = LIC_NORM_GDN;
    cfg->rans_lanes = 0;
}

int codec_create(const codec_config* cfg, const void* blob, size_t blob_len, codec_t** out)
{
    if (out) *out = nullptr;
    if (!cfg || !blob || !out) { g_create_error = "null argument"; return LIC_E_ARG; }
    if (cfg->struct_size != sizeof(codec_config)) { g_create_error = "codec_config size mismatch"; return LIC_E_ARG; }
    if (!supported_shape(cfg->kind, cfg->N, cfg->M)) { g_create_error = "unsupported kind/N/M"; return LIC_E_ARG; }
    if (cfg->precision != LIC_PREC_FP32 && cfg->precision != LIC_PREC_BF16 && cfg->precision != LIC_PREC_FP8) {
        g_create_error = "unsupported precision";
        return LIC_E_ARG;
    }
    if (cfg->hs_out != LIC_HS_EXP && cfg->hs_out != LIC_HS_RELU) { g_create_error = "bad hs_out"; return LIC_E_ARG; }
    if (cfg->kind == LIC_KIND_CONTEXT && cfg->gs_mode != 0) {
        g_create_error = "context model: full g_s only";
        return LIC_E_ARG;
    }
    if (cfg->gs_mode < 0 || cfg->gs_mode > 2) { g_create_error = "gs_mode must be 0, 1 or 2"; return LIC_E_ARG; }
    if (cfg->norm != LIC_NORM_GDN && cfg->norm != LIC_NORM_1DN) { g_create_error = "bad norm"; return LIC_E_ARG; }
    if (cfg->rans_lanes != 0 && !lic::rans_lanes_valid(cfg->rans_lanes)) {
        g_create_error = "rans_lanes must be 0, 2, 4, 8, 16 or 32";
        return LIC_E_ARG;
    }
    if (cfg->y_slices < 1 || cfg->y_slices > lic::kMaxSlices) { g_create_error = "y_slices must be 1..64"; return LIC_E_ARG; }
    if (cfg->entropy_threads < 1 || cfg->entropy_threads > 256) { g_create_error = "bad entropy_threads"; return LIC_E_ARG; }
    if (cfg->max_in_flight < 1 || cfg->max_in_flight > 64) { g_create_error = "max_in_flight must be 1..64"; return LIC_E_ARG; }
    if (cfg->max_h < 1 || cfg->max_w < 1 || cfg->max_h > 8192 || cfg->max_w > 8192) { g_create_error = "bad max_h/max_w"; return LIC_E_ARG; }
    if (cfg->max_batch < 1 || cfg->max_batch > lic::kMaxBatch) { g_create_error = "max_batch must be 1..8"; return LIC_E_ARG; }
    codec* c = new (std::nothrow) codec();
    if (!c) { g_create_error = "out of memory"; return LIC_E_NOMEM; }
    c->cfg = *cfg;
    int rc = c->load(blob, blob_len);
    if (rc == LIC_OK) rc = c->start();
    if (rc != LIC_OK) {
        g_create_error = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return LIC_OK;
}

void codec_destroy(codec_t* c) { delete c; }

const char* codec_last_error(const codec_t* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int codec_encode(codec_t* c, const float* x, int n, int H, int W, int is_device, uint8_t* out, size_t cap,
                 size_t* lens)
{
    if (!c) return LIC_E_ARG;
    int rc;
    if (!check_frame(c, n, H, W, &rc)) return rc;
    if (n > 0 && (!x || !lens)) return fail(c, LIC_E_ARG, "null buffer");
    lic::CallState cs;
    cs.n = n;
    cs.route.S = c->S;
    cs.route.dims = lic::FrameDims(H, W);
    cs.route.is_device = is_device;
    cs.route.stages = {lic::ST_GPU_ENC, lic::ST_CPU_ENC};
    cs.out = out;
    cs.cap = out ? cap : 0;
    cs.lens = lens;
    make_tasks(c, cs, x, nullptr, (size_t)3 * H * W);
    rc = c->run_call(cs);
    if (rc != LIC_OK) return rc;
    if (cs.overflow) return fail(c, LIC_E_SMALLBUF, "output capacity too small");
    return LIC_OK;
}

namespace {

int parse_all(Codec* c, const uint8_t* bits, const size_t* lens, int n, lic::CallState& cs,
              std::vector<lic::StreamHeader>* hdrs, std::vector<const uint8_t*>* zp, std::vector<size_t>* zl,
              std::vector<std::vector<const uint8_t*>>* yp, std::vector<std::vector<size_t>>* yl)
{
    size_t off = 0;
    hdrs->resize(n);
    zp->resize(n);
    zl->resize(n);
    yp->resize(n);
    yl->resize(n);
    for (int i = 0; i < n; ++i) {
        lic::StreamHeader& h = (*hdrs)[i];
        std::string e;
        if (!lic::parse_stream(bits + off, lens[i], &h, &(*zp)[i], &(*zl)[i], &(*yp)[i], &(*yl)[i], &e))
            return fail(c, LIC_E_CORRUPT, e);
        if (h.kind != c->kind || h.N != c->N || h.M != c->M || h.hs_exp != c->hs_exp || h.model_id != c->model_id ||
            h.norm != c->norm || h.lanes != c->lanes)
            return fail(c, LIC_E_MODEL, "bitstream was produced by another model");
        if (h.S > lic::kMaxSlices) return fail(c, LIC_E_CORRUPT, "too many slices");
        if (h.H != (*hdrs)[0].H || h.W != (*hdrs)[0].W || h.S != (*hdrs)[0].S)
            return fail(c, LIC_E_ARG, "frames of one call must share size and slices");
        off += lens[i];
    }
    cs.route.S = (*hdrs)[0].S;
    return LIC_OK;
}

}  // namespace

int codec_decode(codec_t* c, const uint8_t* bits, const size_t* lens, int n, float* x_hat, size_t cap_elems,
                 int is_device, int* H, int* W)
{
    if (!c) return LIC_E_ARG;
    if (n < 0) return fail(c, LIC_E_ARG, "bad frame count");
    if (n == 0) return LIC_OK;
    if (!bits || !lens || !x_hat || !H || !W) return fail(c, LIC_E_ARG, "null buffer");
    lic::CallState cs;
    std::vector<lic::StreamHeader> hdrs;
    std::vector<const uint8_t*> zp;
    std::vector<size_t> zl;
    std::vector<std::vector<const uint8_t*>> yp;
    std::vector<std::vector<size_t>> yl;
    int rc = parse_all(c, bits, lens, n, cs, &hdrs, &zp, &zl, &yp, &yl);
    if (rc != LIC_OK) return rc;
    const int h = hdrs[0].H, w = hdrs[0].W;
    if (!check_frame(c, n, h, w, &rc)) return rc;
    *H = h;
    *W = w;
    const size_t fsz = (size_t)3 * h * w;
    if (cap_elems < fsz * n) return fail(c, LIC_E_SMALLBUF, "x_hat capacity too small");
    cs.n = n;
    cs.route.dims = lic::FrameDims(h, w);
    cs.route.is_device = is_device;
    if (c->kind == LIC_KIND_CONTEXT)
        cs.route.stages = {lic::ST_CPU_DEC_Z, lic::ST_GPU_HS, lic::ST_CPU_DEC_Y, lic::ST_GPU_CTX, lic::ST_CPU_DEC_Y2,
                           lic::ST_GPU_GS};
    else if (c->kind == LIC_KIND_HYPERPRIOR)
        cs.route.stages = {lic::ST_CPU_DEC_Z, lic::ST_GPU_HS, lic::ST_CPU_DEC_Y, lic::ST_GPU_GS};
    else
        cs.route.stages = {lic::ST_CPU_DEC_Y, lic::ST_GPU_GS};
    make_tasks(c, cs, nullptr, x_hat, fsz);
    for (auto& t : cs.tasks)
        for (int b = 0; b < t->nb; ++b) {
            const int f = t->first + b;
            t->zp[b] = zp[f];
            t->zlen[b] = zl[f];
            for (size_t s = 0; s < yp[f].size(); ++s) {
                t->yp[b][s] = yp[f][s];
                t->ylen[b][s] = yl[f][s];
            }
        }
    return c->run_call(cs);
}

int codec_encode_decode(codec_t* c, const float* x, int n, int H, int W, int is_device, uint8_t* bits, size_t cap,
                        size_t* lens, float* x_hat)
{
    if (!c) return LIC_E_ARG;
    int rc;
    if (!check_frame(c, n, H, W, &rc)) return rc;
    if (n > 0 && (!x || !lens || !x_hat)) return fail(c, LIC_E_ARG, "null buffer");
    lic::CallState cs;
    cs.n = n;
    cs.route.S = c->S;
    cs.route.dims = lic::FrameDims(H, W);
    cs.route.is_device = is_device;
    if (c->kind == LIC_KIND_CONTEXT)
        cs.route.stages = {lic::ST_GPU_ENC, lic::ST_CPU_ENC,     lic::ST_CPU_DEC_Z,  lic::ST_GPU_HS,
                           lic::ST_CPU_DEC_Y, lic::ST_GPU_CTX, lic::ST_CPU_DEC_Y2, lic::ST_GPU_GS};
    else if (c->kind == LIC_KIND_HYPERPRIOR)
        cs.route.stages = {lic::ST_GPU_ENC, lic::ST_CPU_ENC, lic::ST_CPU_DEC_Z, lic::ST_GPU_HS, lic::ST_CPU_DEC_Y, lic::ST_GPU_GS};
    else
        cs.route.stages = {lic::ST_GPU_ENC, lic::ST_CPU_ENC, lic::ST_CPU_DEC_Y, lic::ST_GPU_GS};
    cs.out = bits;
    cs.cap = bits ? cap : 0;
    cs.lens = lens;
    make_tasks(c, cs, x, x_hat, (size_t)3 * H * W);
    rc = c->run_call(cs);
    if (rc != LIC_OK) return rc;
    if (cs.overflow) return fail(c, LIC_E_SMALLBUF, "output capacity too small");
    return LIC_OK;
}

int codec_last_latencies(const codec_t* c, double* ms, int max)
{
    if (!c || !ms || max < 0) return LIC_E_ARG;
    const int n = std::min<int>(max, (int)c->last_lat_ms.size());
    for (int i = 0; i < n; ++i) ms[i] = c->last_lat_ms[i];
    return n;
}

int codec_get_stats(const codec_t* c, char* buf, size_t cap)
{
    if (!c || !buf) return LIC_E_ARG;
    std::vector<double> lat = c->last_lat_ms;
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) {
        if (lat.empty()) return 0.0;
        size_t i = (size_t)(p * (lat.size() - 1) + 0.5);
        return lat[std::min(i, lat.size() - 1)];
    };
    const double fps = c->last_wall_s > 0 ? c->last_frames / c->last_wall_s : 0.0;
    int n = snprintf(buf, cap,
                     "{\"frames\": %d, \"wall_s\": %.6f, \"fps\": %.3f, \"p50_ms\": %.4f, \"p99_ms\": %.4f, "
                     "\"gpu_busy_s\": [%.6f, %.6f, %.6f], \"cpu_busy_s\": %.6f, \"device_bytes\": %zu, "
                     "\"alloc_events\": %ld, \"entropy_threads\": %d, \"max_in_flight\": %d, \"zero_copy\": %d, "
                     "\"gs_mode\": %d, \"gs_judged\": %ld, \"gs_judge_last_db\": %.4f, \"gs_fallback\": %d}",
                     c->last_frames, c->last_wall_s, fps, pct(0.50), pct(0.99), c->gpu[0].busy_s, c->gpu[1].busy_s,
                     c->gpu[2].busy_s, c->cpu_busy_us.load() * 1e-6, c->dev_bytes, c->alloc_events.load(),
                     c->cfg.entropy_threads, c->cfg.max_in_flight, c->cfg.zero_copy, c->cfg.gs_mode,
                     c->gs_judged.load(), c->gs_judge_last_db, (int)c->gs_fallback.load());
    if (n < 0 || (size_t)n >= cap) return LIC_E_SMALLBUF;
    return n;
}

int codec_calibrate(codec_t* c, const float* x, int n, int H, int W, int is_device)
{
    if (!c || !x) return LIC_E_ARG;
    int rc;
    if (!check_frame(c, n, H, W, &rc)) return rc;
    if (n < 1) return fail(c, LIC_E_ARG, "no calibration frames");
    if (hipSetDevice(c->cfg.hip_device) != hipSuccess) return fail(c, LIC_E_HIP, "hipSetDevice");
    const float* xd = x;
    void* tmp = nullptr;
    const size_t bytes = (size_t)n * 3 * H * W * sizeof(float);
    if (!is_device) {
        if (hipMalloc(&tmp, bytes) != hipSuccess) return fail(c, LIC_E_NOMEM, "calibration input");
        if (hipMemcpy(tmp, x, bytes, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(tmp);
            return fail(c, LIC_E_HIP, "calibration input copy");
        }
        xd = static_cast<const float*>(tmp);
    }
    rc = c->calibrate_fp8(xd, n, H, W);
    if (tmp) (void)hipFree(tmp);
    if (rc != LIC_OK) return fail(c, rc, c->err);
    return LIC_OK;
}

int codec_fp8_scales(const codec_t* c, float* q, int max, unsigned long long* saturated)
{
    if (!c || (!q && max > 0)) return LIC_E_ARG;
    for (int i = 0; i < std::min(max, (int)LIC_NUM_LAYERS); ++i) {
        const lic::LayerGPU& L = c->layers[i];
        const bool e8 = L.present && (L.dt == lic::DT_FP8 ? !L.out_bf16 : L.out_e4m3);
        q[i] = e8 ? L.out_q : 0.0f;
    }
    if (saturated) {
        *saturated = 0;
        if (c->d_sat && (hipSetDevice(c->cfg.hip_device) != hipSuccess ||
                         hipMemcpy(saturated, c->d_sat, sizeof(*saturated), hipMemcpyDeviceToHost) != hipSuccess))
            return LIC_E_HIP;
    }
    return LIC_NUM_LAYERS;
}

int codec_load_distilled(codec_t* c, const float* params, size_t n_params, float judge_psnr_db, int judge_every)
{
    if (!c || !params) return LIC_E_ARG;
    if (hipSetDevice(c->cfg.hip_device) != hipSuccess) return fail(c, LIC_E_HIP, "hipSetDevice");
    const int rc = c->load_distilled(params, n_params, judge_psnr_db, judge_every);
    if (rc != LIC_OK) return fail(c, rc, c->err);
    return LIC_OK;
}

int codec_run_layer(codec_t* c, int layer, int n, int H, int W, const void* in, void* out, void* aux)
{
    return codec_run_layer_ex(c, layer, n, H, W, in, out, aux, nullptr, nullptr);
}

int codec_run_layer_ex(codec_t* c, int layer, int n, int H, int W, const void* in, void* out, void* aux,
                       const void* in2, void* out2)
{
    if (!c) return LIC_E_ARG;
    if (layer < 0 || layer >= LIC_NUM_LAYERS || !c->layers[layer].present) return fail(c, LIC_E_ARG, "no such layer");
    if (n < 1 || H < 1 || W < 1 || H > 65535 || W > 65535) return fail(c, LIC_E_ARG, "bad size");
    if (!in || (!out && layer != LIC_HA2 && layer != LIC_GA3)) return fail(c, LIC_E_ARG, "null buffer");
    if ((layer == LIC_GA3 || layer == LIC_HA2) && !aux) return fail(c, LIC_E_ARG, "quantising layers need aux");
    if ((layer == LIC_EP2A || layer == LIC_EP2N) && !out2)
        return fail(c, LIC_E_ARG, "the last entropy-parameter layer needs out2 (y_hat or the means)");
    lic::FrameDims d(H, W);
    if (hipSetDevice(c->cfg.hip_device) != hipSuccess) return fail(c, LIC_E_HIP, "hipSetDevice");
    std::string e;
    int rc = c->launch_layer(layer, n, d, in, out, aux, c->layer_stream, &e, nullptr, in2, out2);
    if (rc != LIC_OK) return fail(c, rc, e);
    hipError_t he = hipStreamSynchronize(c->layer_stream);
    if (he != hipSuccess) return fail(c, LIC_E_HIP, hipGetErrorString(he));
    return LIC_OK;
}

int codec_layer_bytes(codec_t* c, int layer, int n, int H, int W, size_t* in_bytes, size_t* out_bytes,
                      size_t* aux_bytes)
{
    if (!c || !in_bytes || !out_bytes || !aux_bytes) return LIC_E_ARG;
    if (layer < 0 || layer >= LIC_NUM_LAYERS || !c->layers[layer].present) return fail(c, LIC_E_ARG, "no such layer");
    if (n < 1 || H < 1 || W < 1 || H > 65535 || W > 65535) return fail(c, LIC_E_ARG, "bad size");
    c->layer_bytes(layer, n, lic::FrameDims(H, W), in_bytes, out_bytes, aux_bytes);
    return LIC_OK;
}

int codec_layer_kernel(codec_t* c, int layer, int H, int W, int* form, int* ksplit)
{
    if (!c || !form || !ksplit) return LIC_E_ARG;
    if (layer < 0 || layer >= LIC_NUM_LAYERS || !c->layers[layer].present) return fail(c, LIC_E_ARG, "no such layer");
    if (H < 1 || W < 1 || H > 65535 || W > 65535) return fail(c, LIC_E_ARG, "bad size");
    lic::FrameDims d(H, W);
    lic::KernelKey key{};
    std::string e;
    const int rc = c->launch_layer(layer, 1, d, nullptr, nullptr, nullptr, nullptr, &e, &key);
    if (rc != LIC_OK) return fail(c, rc, e);
    *form = key.dt;
    *ksplit = key.ksplit;
    return LIC_OK;
}

int codec_time_layers(codec_t* c, uint32_t mask)
{
    if (!c) return LIC_E_ARG;
    if (mask >> LIC_NUM_LAYERS) return fail(c, LIC_E_ARG, "no such layer");
    std::lock_guard<std::mutex> g(c->lt_m);
    c->timed_mask.store(mask);
    for (int l = 0; l < LIC_NUM_LAYERS; ++l) {
        c->layer_ms[l] = 0.0;
        c->layer_launches[l] = 0;
    }
    return LIC_OK;
}

int codec_layer_time(codec_t* c, int layer, double* total_ms, long* launches)
{
    if (!c || !total_ms || !launches || layer < 0 || layer >= LIC_NUM_LAYERS) return LIC_E_ARG;
    std::lock_guard<std::mutex> g(c->lt_m);
    *total_ms = c->layer_ms[layer];
    *launches = c->layer_launches[layer];
    return LIC_OK;
}

long codec_tables(const codec_t* c, int which, uint32_t* freq, size_t cap)
{
    if (!c || !freq) return LIC_E_ARG;
    const lic::TableSet& T = which == 0 ? c->fact : c->gauss;
    if (which != 0 && which != 1) return LIC_E_ARG;
    if (T.freq.size() > cap) return LIC_E_SMALLBUF;
    std::copy(T.freq.begin(), T.freq.end(), freq);
    return (long)T.freq.size();
}

long codec_medians(const codec_t* c, float* mu, size_t cap)
{
    if (!c || !mu) return LIC_E_ARG;
    if (c->medians.size() > cap) return LIC_E_SMALLBUF;
    std::copy(c->medians.begin(), c->medians.end(), mu);
    return (long)c->medians.size();
}

long lic_rans_encode(const uint8_t* sym, const uint8_t* tab, long n, const uint32_t* freq, int ntab, uint8_t* out,
                     size_t cap)
{
    if (n < 0 || ntab < 1 || ntab > 256 || (n > 0 && (!sym || !tab)) || !freq || !out) return LIC_E_ARG;
    for (long i = 0; i < n; ++i)
        if (sym[i] >= lic::kNumSym || tab[i] >= ntab) return LIC_E_ARG;
    lic::TableSet T;
    T.init(ntab, freq, false);
    for (int t = 0; t < ntab; ++t)
        if (T.start[(size_t)t * (lic::kNumSym + 1) + lic::kNumSym] != (1u << lic::kPrecBits)) return LIC_E_ARG;
    std::vector<int8_t> v(n);
    for (long i = 0; i < n; ++i) v[i] = (int8_t)((int)sym[i] + lic::kSymMin);
    long len = lic::rans_encode(v.data(), tab, n, T, out, cap);
    return len < 0 ? LIC_E_SMALLBUF : len;
}

int lic_rans_decode(const uint8_t* in, size_t len, const uint8_t* tab, long n, const uint32_t* freq, int ntab,
                    uint8_t* sym)
{
    if (n < 0 || ntab < 1 || ntab > 256 || !in || !freq || (n > 0 && (!tab || !sym))) return LIC_E_ARG;
    for (long i = 0; i < n; ++i)
        if (tab[i] >= ntab) return LIC_E_ARG;
    lic::TableSet T;
    T.init(ntab, freq, true);
    for (int t = 0; t < ntab; ++t)
        if (T.start[(size_t)t * (lic::kNumSym + 1) + lic::kNumSym] != (1u << lic::kPrecBits)) return LIC_E_ARG;
    std::vector<int8_t> v(n);
    if (lic::rans_decode(in, len, tab, n, T, v.data()) != 0) return LIC_E_CORRUPT;
    for (long i = 0; i < n; ++i) sym[i] = (uint8_t)((int)v[i] - lic::kSymMin);
    return LIC_OK;
}

long lic_rans_ileave_encode(int lanes, const uint8_t* sym, const uint8_t* tab, long n, const uint32_t* freq, int ntab,
                            uint8_t* out, size_t cap)
{
    if (!lic::rans_lanes_valid(lanes) || n < 0 || ntab < 1 || ntab > 256 || (n > 0 && (!sym || !tab)) || !freq ||
        !out)
        return LIC_E_ARG;
    for (long i = 0; i < n; ++i)
        if (sym[i] >= lic::kNumSym || tab[i] >= ntab) return LIC_E_ARG;
    lic::TableSet T;
    T.init(ntab, freq, false);
    for (int t = 0; t < ntab; ++t)
        if (T.start[(size_t)t * (lic::kNumSym + 1) + lic::kNumSym] != (1u << lic::kPrecBits)) return LIC_E_ARG;
    std::vector<int8_t> v(n);
    for (long i = 0; i < n; ++i) v[i] = (int8_t)((int)sym[i] + lic::kSymMin);
    long len = lic::rans_ileave_encode(lanes, v.data(), tab, n, T, out, cap);
    return len < 0 ? LIC_E_SMALLBUF : len;
}

int lic_rans_ileave_decode(int lanes, const uint8_t* in, size_t len, const uint8_t* tab, long n, const uint32_t* freq,
                           int ntab, uint8_t* sym)
{
    if (!lic::rans_lanes_valid(lanes) || n < 0 || ntab < 1 || ntab > 256 || !in || !freq || (n > 0 && (!tab || !sym)))
        return LIC_E_ARG;
    for (long i = 0; i < n; ++i)
        if (tab[i] >= ntab) return LIC_E_ARG;
    lic::TableSet T;
    T.init(ntab, freq, true);
    for (int t = 0; t < ntab; ++t)
        if (T.start[(size_t)t * (lic::kNumSym + 1) + lic::kNumSym] != (1u << lic::kPrecBits)) return LIC_E_ARG;
    std::vector<int8_t> v(n);
    if (lic::rans_ileave_decode(lanes, in, len, tab, n, T, v.data()) != 0) return LIC_E_CORRUPT;
    for (long i = 0; i < n; ++i) sym[i] = (uint8_t)((int)v[i] - lic::kSymMin);
    return LIC_OK;
}

uint32_t lic_fnv1a(const void* data, size_t len) { return lic::fnv1a(data, len); }

int codec_open_stream(codec_t* c, int H, int W, int* stream_id)
{
    if (!c || !stream_id) return LIC_E_ARG;
    return c->open_stream(H, W, stream_id);
}

int codec_close_stream(codec_t* c, int stream_id)
{
    if (!c) return LIC_E_ARG;
    return c->close_stream(stream_id);
}

int codec_submit_encode(codec_t* c, int stream_id, const float* x, int is_device, uint8_t* out, size_t cap,
                        uint64_t* ticket)
{
    if (!c || !x || !out || !ticket) return LIC_E_ARG;
    if (c->kind == LIC_KIND_CONTEXT) return fail(c, LIC_E_ARG, "serving runs the factorized and hyperprior codecs");
    lic::Request* r = new (std::nothrow) lic::Request();
    if (!r) return fail(c, LIC_E_NOMEM, "out of memory");
    r->dir = 0;
    r->stream_id = stream_id;
    r->is_device = is_device ? 1 : 0;
    r->x = x;
    r->out = out;
    r->cap = cap;
    return c->server_submit(r, ticket);   // r is owned by the server from here on
}

int codec_submit_decode(codec_t* c, int stream_id, const uint8_t* bits, size_t len, float* x_hat, size_t cap_elems,
                        int is_device, uint64_t* ticket)
{
    if (!c || !bits || !x_hat || !ticket) return LIC_E_ARG;
    if (c->kind == LIC_KIND_CONTEXT) return fail(c, LIC_E_ARG, "serving runs the factorized and hyperprior codecs");
    lic::Request* r = new (std::nothrow) lic::Request();
    if (!r) return fail(c, LIC_E_NOMEM, "out of memory");
    std::vector<const uint8_t*> yp;
    std::vector<size_t> yl;
    std::string e;
    if (!lic::parse_stream(bits, len, &r->hdr, &r->zp, &r->zlen, &yp, &yl, &e)) {
        delete r;
        return fail(c, LIC_E_CORRUPT, e);
    }
    const lic::StreamHeader& h = r->hdr;
    if (h.kind != c->kind || h.N != c->N || h.M != c->M || h.hs_exp != c->hs_exp || h.model_id != c->model_id ||
            h.norm != c->norm || h.lanes != c->lanes) {
        delete r;
        return fail(c, LIC_E_MODEL, "bitstream was produced by another model");
    }
    if (h.S > lic::kMaxSlices) {
        delete r;
        return fail(c, LIC_E_CORRUPT, "too many slices");
    }
    if (cap_elems < (size_t)3 * h.H * h.W) {
        delete r;
        return fail(c, LIC_E_SMALLBUF, "x_hat capacity too small");
    }
    for (int s = 0; s < h.S; ++s) {
        r->yp[s] = yp[s];
        r->ylen[s] = yl[s];
    }
    r->dir = 1;
    r->stream_id = stream_id;
    r->is_device = is_device ? 1 : 0;
    r->xhat = x_hat;
    return c->server_submit(r, ticket);
}

int codec_poll(codec_t* c, lic_result* done, int max, int timeout_us)
{
    if (!c || !done || max < 0) return LIC_E_ARG;
    return c->server_poll(done, max, timeout_us);
}

long lic_blob_tables(const void* blob, size_t len, int which, uint32_t* freq, size_t cap, float* mu, size_t mu_cap)
{
    if (!blob || !freq) return LIC_E_ARG;
    return lic::blob_tables(blob, len, which, freq, cap, mu, mu_cap);
}

}  // extern "C"
