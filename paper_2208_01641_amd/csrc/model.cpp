// Model loading: weight blob parsing, entropy tables, weight packing for the
// implicit-GEMM kernels, per-layer geometry and launch planning.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>

#include "codec.h"
#include "packing.h"

namespace lic {

#define HIP_TRY(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
            return LIC_E_HIP;                                                      \
        }                                                                          \
    } while (0)

void* Codec::dev_alloc(size_t bytes)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) return nullptr;
    dev_allocs.push_back(p);
    dev_bytes += bytes;
    alloc_events++;
    return p;
}

void* Codec::host_alloc(size_t bytes)
{
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes ? bytes : 16, hipHostMallocMapped) != hipSuccess) return nullptr;
    host_allocs.push_back(p);
    alloc_events++;
    return p;
}

namespace {

using ParamMap = std::map<std::string, std::pair<std::vector<int>, std::vector<double>>>;

bool parse_blob(const uint8_t* b, size_t len, int* kind, int* N, int* M, ParamMap* P, std::string* err)
{
    auto rd32 = [&](size_t pos) {
        uint32_t v;
        memcpy(&v, b + pos, 4);
        return v;
    };
    if (len < 24 || memcmp(b, "LICW", 4) != 0) { *err = "weight blob: bad magic"; return false; }
    if (rd32(4) != 1) { *err = "weight blob: unsupported version"; return false; }
    *kind = (int)rd32(8);
    *N = (int)rd32(12);
    *M = (int)rd32(16);
    const uint32_t count = rd32(20);
    size_t pos = 24;
    for (uint32_t e = 0; e < count; ++e) {
        if (pos + 2 > len) { *err = "weight blob: truncated"; return false; }
        uint16_t nl;
        memcpy(&nl, b + pos, 2);
        pos += 2;
        if (pos + nl + 2 > len) { *err = "weight blob: truncated"; return false; }
        std::string name((const char*)b + pos, nl);
        pos += nl;
        const int code = b[pos], ndim = b[pos + 1];
        pos += 2;
        if ((code != 0 && code != 1) || ndim > 4 || pos + 4u * ndim > len) { *err = "weight blob: bad entry"; return false; }
        std::vector<int> dims(ndim);
        size_t count_el = 1;
        for (int d = 0; d < ndim; ++d) {
            dims[d] = (int)rd32(pos);
            pos += 4;
            count_el *= (size_t)dims[d];
        }
        const size_t esz = code == 0 ? 4 : 8;
        if (pos + count_el * esz > len) { *err = "weight blob: truncated data"; return false; }
        std::vector<double> vals(count_el);
        for (size_t i = 0; i < count_el; ++i) {
            if (code == 0) {
                float f;
                memcpy(&f, b + pos + 4 * i, 4);
                vals[i] = f;
            } else {
                memcpy(&vals[i], b + pos + 8 * i, 8);
            }
        }
        pos += count_el * esz;
        (*P)[name] = {dims, std::move(vals)};
    }
    return true;
}

}  // namespace

// float32 -> bfloat16, round to nearest even (NaN stays NaN)
uint16_t bf16_rne(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// GDN gamma [co][co] (row-major, FP64 from the weight blob, used as FP32)
// as three bf16 parts g0 + g1 + g2, each rounded to nearest from what the
// previous parts leave (remainders are exact in FP32), laid out for the
// GDN epilogue: part k of gamma[r][(2p + i/4) 16 + 4 kg + i%4] at
// (((k co + r) (co/32) + p) 4 + kg) 8 + i.
std::vector<uint16_t> gdn_gamma_split(const std::vector<double>& gamma, int co)
{
    const int npair = co / 32;
    std::vector<uint16_t> out((size_t)3 * co * co);
    for (int r = 0; r < co; ++r)
        for (int p = 0; p < npair; ++p)
            for (int kg = 0; kg < 4; ++kg)
                for (int i = 0; i < 8; ++i) {
                    const int c = (2 * p + i / 4) * 16 + 4 * kg + i % 4;
                    float rem = (float)gamma[(size_t)r * co + c];
                    for (int k = 0; k < 3; ++k) {
                        const uint16_t h = bf16_rne(rem);
                        out[((((size_t)k * co + r) * npair + p) * 4 + kg) * 8 + i] = h;
                        const uint32_t u = (uint32_t)h << 16;
                        float hv;
                        memcpy(&hv, &u, 4);
                        rem -= hv;
                    }
                }
    return out;
}

// OCP e4m3 (1 sign, 4 exponent bits with bias 7, 3 mantissa bits; largest
// finite 448, subnormal step 2^-9, no infinities) of f, rounding to nearest
// even and saturating at +-448.
uint8_t e4m3_rne(float f)
{
    const uint8_t sign = std::signbit(f) ? 0x80 : 0x00;
    double a = std::fabs((double)f);
    if (!(a == a)) return 0x7f;                     // NaN
    if (a >= 448.0) return sign | 0x7e;
    // quantum of the binade (2^-9 below the smallest normal 2^-6)
    int ex = 0;
    (void)std::frexp(a, &ex);                       // a = m 2^ex, m in [0.5, 1)
    int e = a > 0.0 ? ex - 1 : -6;
    if (e < -6) e = -6;
    const double q = std::ldexp(1.0, e - 3);
    double m = a / q;                               // exact: q is a power of two
    double r = std::nearbyint(m);                   // ties to even (default rounding mode)
    double v = r * q;
    if (v >= 448.0) return sign | 0x7e;
    if (v == 0.0) return sign;
    (void)std::frexp(v, &ex);
    const int ve = ex - 1;
    if (ve < -6) return sign | (uint8_t)std::lround(v / std::ldexp(1.0, -9));     // subnormal
    const int mant = (int)std::lround(v / std::ldexp(1.0, ve - 3)) - 8;
    return sign | (uint8_t)((ve + 7) << 3) | (uint8_t)mant;
}

bool build_tables(const ParamMap& P, int kind, int N, int M, std::vector<float>* medians,
                  std::vector<uint32_t>* fact_freq, std::vector<uint32_t>* gauss_freq, std::string* err)
{
    auto it = P.find("eb.density");
    const int C = kind == 0 ? M : N;
    if (it == P.end() || it->second.second.size() != (size_t)C * kDensityParams) {
        *err = "weight blob: eb.density missing or of the wrong size";
        return false;
    }
    const std::vector<double>& dens = it->second.second;
    medians->resize(C);
    fact_freq->assign((size_t)C * kNumSym, 0);
    std::vector<double> pmf(kNumSym);
    for (int c = 0; c < C; ++c) {
        const double* prm = dens.data() + (size_t)c * kDensityParams;
        (*medians)[c] = (float)density_median(prm);
        pmf_factorized(prm, (double)(*medians)[c], pmf.data());
        quantize_pmf(pmf.data(), fact_freq->data() + (size_t)c * kNumSym);
    }
    gauss_freq->clear();
    if (kind >= 1) {
        double t[kScales];
        scale_table(t);
        gauss_freq->assign((size_t)kScales * kNumSym, 0);
        for (int k = 0; k < kScales; ++k) {
            pmf_gaussian(t[k], pmf.data());
            quantize_pmf(pmf.data(), gauss_freq->data() + (size_t)k * kNumSym);
        }
    }
    return true;
}

int Codec::load(const void* blob, size_t len)
{
    ParamMap P;
    int bk, bn, bm;
    if (!parse_blob(static_cast<const uint8_t*>(blob), len, &bk, &bn, &bm, &P, &err)) return LIC_E_ARG;
    if (bk != cfg.kind || bn != cfg.N || bm != cfg.M) {
        err = "weight blob kind/N/M does not match the configuration";
        return LIC_E_MODEL;
    }
    kind = cfg.kind;
    N = cfg.N;
    M = cfg.M;
    hs_exp = cfg.hs_out == LIC_HS_EXP ? 1 : 0;
    norm = cfg.norm;
    lanes = cfg.rans_lanes;
    S = cfg.y_slices;
    model_id = fnv1a(blob, len);

    // entropy model: per-channel medians, factorized and Gaussian tables
    std::vector<uint32_t> ff, gf;
    if (!build_tables(P, kind, N, M, &medians, &ff, &gf, &err)) return LIC_E_MODEL;
    fact.init(kind == 0 ? M : N, ff.data(), kind == 0);
    if (kind >= 1) {
        gauss.init(kScales, gf.data(), true);
        double t[kScales];
        scale_table(t);
        thr.resize(63);
        for (int k = 0; k < 63; ++k) thr[k] = hs_exp ? (float)log(t[k]) : (float)t[k];
    }
    return build_layers(P);
}

long blob_tables(const void* blob, size_t len, int which, uint32_t* freq, size_t cap, float* mu, size_t mu_cap)
{
    ParamMap P;
    int kind, N, M;
    std::string e;
    if (!parse_blob(static_cast<const uint8_t*>(blob), len, &kind, &N, &M, &P, &e)) return LIC_E_ARG;
    std::vector<float> med;
    std::vector<uint32_t> ff, gf;
    if (!build_tables(P, kind, N, M, &med, &ff, &gf, &e)) return LIC_E_MODEL;
    const std::vector<uint32_t>& src = which == 0 ? ff : gf;
    if (which != 0 && which != 1) return LIC_E_ARG;
    if (src.size() > cap || (mu && med.size() > mu_cap)) return LIC_E_SMALLBUF;
    std::copy(src.begin(), src.end(), freq);
    if (mu) std::copy(med.begin(), med.end(), mu);
    return (long)src.size();
}

namespace {

struct Spec {
    int id;
    const char* name;
    int ld, ep;
    bool deconv;
    int k;
    int cb = -1;       // context model: the checkerboard set the layer is evaluated on
};

}  // namespace

int Codec::upload_rscale(LayerGPU& L)
{
    std::vector<float> rs(L.wsc.size());
    for (size_t r = 0; r < rs.size(); ++r) rs[r] = L.wsc[r] * L.in_scale;
    HIP_TRY(hipMemcpy(L.d_rscale, rs.data(), rs.size() * sizeof(float), hipMemcpyHostToDevice));
    return LIC_OK;
}

// Activation scales of the e4m3 form: each layer that stores e4m3
// activations gets q = 448 / (2 amax), amax the largest |value| it produces
// on the calibration frames (one binary order of headroom), with the scales
// of the layers before it already in place; the layer that reads its output
// undoes q in its epilogue.  The layers run once with bf16 outputs to
// measure amax and once more in e4m3 to feed the next layer.
int Codec::calibrate_fp8(const float* x, int n, int H, int W)
{
    if (cfg.precision != LIC_PREC_FP8) return LIC_OK;
    const FrameDims d(H, W);
    size_t cap = 0;
    for (int id : {LIC_GA0, LIC_GA1, LIC_GA2, LIC_GA3, LIC_GS0, LIC_GS1, LIC_GS2}) {
        size_t bi, bo, ba;
        layer_bytes(id, n, d, &bi, &bo, &ba);
        cap = std::max(cap, std::max(bi, std::max(bo, ba)) * 4);     // room for any storage type
    }
    // buf[0]: measured (bf16) outputs; buf[1], buf[2]: e4m3 activations; buf[3]: symbols of y
    void* buf[4] = {nullptr, nullptr, nullptr, nullptr};
    for (void*& b : buf)
        if (hipMalloc(&b, cap) != hipSuccess) {
            for (void* q : buf) (void)hipFree(q);
            err = "calibration buffers: device allocation failed";
            return LIC_E_NOMEM;
        }
    std::vector<uint16_t> host(cap / 2);
    std::string e;
    int rc = LIC_OK;
    // amax of layer id's output (bf16 storage) on input `in`
    auto measure = [&](int id, const void* in, float* amax) -> int {
        LayerGPU& L = layers[id];
        const bool e8 = L.out_e4m3, b16 = L.out_bf16;
        if (L.dt == DT_BF16) L.out_e4m3 = false; else L.out_bf16 = true;
        size_t bi, bo, ba;
        layer_bytes(id, n, d, &bi, &bo, &ba);
        int r = launch_layer(id, n, d, in, buf[0], nullptr, layer_stream, &e);
        L.out_e4m3 = e8;
        L.out_bf16 = b16;
        if (r != LIC_OK) { err = e; return r; }
        if (hipMemcpyAsync(host.data(), buf[0], bo, hipMemcpyDeviceToHost, layer_stream) != hipSuccess ||
            hipStreamSynchronize(layer_stream) != hipSuccess) { err = "calibration copy failed"; return LIC_E_HIP; }
        float m = 0.0f;
        for (size_t i = 0; i < bo / 2; ++i) {
            const uint32_t u = (uint32_t)host[i] << 16;
            float v;
            memcpy(&v, &u, 4);
            m = std::max(m, std::fabs(v));
        }
        *amax = m;
        return LIC_OK;
    };
    // sets layer id's scale from its output on `in`, runs it in e4m3 into out
    auto step = [&](int id, const void* in, void* out, void* aux) -> int {
        float amax = 0.0f;
        int r = measure(id, in, &amax);
        if (r != LIC_OK) return r;
        LayerGPU& L = layers[id];
        if (L.dt == DT_FP8 ? !L.out_bf16 : L.out_e4m3) {
            L.out_q = amax > 0.0f && std::isfinite(amax) ? 448.0f / (2.0f * amax) : kActQ;
            LayerGPU& next = layers[id + 1];
            next.in_scale = 1.0f / L.out_q;
            if ((r = upload_rscale(next)) != LIC_OK) return r;
        }
        if ((r = launch_layer(id, n, d, in, out, aux, layer_stream, &e)) != LIC_OK) { err = e; return r; }
        return LIC_OK;
    };
    if ((rc = step(LIC_GA0, x, buf[1], nullptr)) == LIC_OK && (rc = step(LIC_GA1, buf[1], buf[2], nullptr)) == LIC_OK &&
        (rc = step(LIC_GA2, buf[2], buf[1], nullptr)) == LIC_OK &&
        (rc = launch_layer(LIC_GA3, n, d, buf[1], buf[2], buf[3], layer_stream, &e)) == LIC_OK) {
        // the context model's g_s starts from y_hat = sym + mean in bf16; y
        // itself (within half a step of it) stands in for the calibration
        if (kind == 2) {
            const hipError_t he = launch_f32_to_bf16(static_cast<const float*>(buf[2]), buf[3],
                                                     (long)n * d.Hy * d.Wy * M, layer_stream);
            if (he != hipSuccess) { err = "calibration: conversion failed"; rc = LIC_E_HIP; }
        }
        if (rc == LIC_OK && (rc = step(LIC_GS0, buf[3], buf[1], nullptr)) == LIC_OK)
            rc = step(LIC_GS1, buf[1], buf[2], nullptr);
    }
    if (rc != LIC_OK && err.empty()) err = e;
    if (hipStreamSynchronize(layer_stream) != hipSuccess && rc == LIC_OK) { err = "calibration failed"; rc = LIC_E_HIP; }
    for (void* b : buf) (void)hipFree(b);
    // captured serving graphs hold the old scales in their kernel arguments
    server_drop_graphs(ST_GPU_ENC);
    server_drop_graphs(ST_GPU_GS);
    return rc;
}

int Codec::build_layers(const ParamMap& P)
{
    HIP_TRY(hipSetDevice(cfg.hip_device));
    if (cfg.precision == LIC_PREC_FP8) {
        d_sat = (unsigned long long*)dev_alloc(sizeof(unsigned long long));
        if (!d_sat) { err = "device allocation failed"; return LIC_E_NOMEM; }
        HIP_TRY(hipMemset(d_sat, 0, sizeof(unsigned long long)));
    }
    const int C = kind == 0 ? M : N;
    d_medians = (float*)dev_alloc(sizeof(float) * 512);
    d_zero = (float*)dev_alloc(sizeof(float) * 512);
    d_thr = (float*)dev_alloc(sizeof(float) * 64);
    if (!d_medians || !d_zero || !d_thr) { err = "device allocation failed"; return LIC_E_NOMEM; }
    std::vector<float> tmp(512, 0.0f);
    HIP_TRY(hipMemcpy(d_zero, tmp.data(), 512 * sizeof(float), hipMemcpyHostToDevice));
    std::copy(medians.begin(), medians.end(), tmp.begin());
    HIP_TRY(hipMemcpy(d_medians, tmp.data(), 512 * sizeof(float), hipMemcpyHostToDevice));
    if (!thr.empty()) HIP_TRY(hipMemcpy(d_thr, thr.data(), 63 * sizeof(float), hipMemcpyHostToDevice));
    (void)C;

    std::vector<Spec> specs = {
        {LIC_GA0, "ga0", LD_RGB, EP_GDN, false, 5}, {LIC_GA1, "ga1", LD_F32, EP_GDN, false, 5},
        {LIC_GA2, "ga2", LD_F32, EP_GDN, false, 5}, {LIC_GA3, "ga3", LD_F32, EP_QUANT, false, 5},
        {LIC_GS0, "gs0", LD_I8, EP_IGDN, true, 5},  {LIC_GS1, "gs1", LD_F32, EP_IGDN, true, 5},
        {LIC_GS2, "gs2", LD_F32, EP_IGDN, true, 5}, {LIC_GS3, "gs3", LD_F32, EP_RGB, true, 5},
    };
    if (kind >= 1) {
        // the context model's h_a sees y (the means need its signs), its h_s
        // ends in psi (2M channels, no activation) and g_s starts from the
        // float y_hat = sym + mean
        std::vector<Spec> hyper = {
            {LIC_HA0, "ha0", kind == 1 ? LD_F32_ABS : LD_F32, EP_RELU, false, 3},
            {LIC_HA1, "ha1", LD_F32, EP_RELU, false, 5},
            {LIC_HA2, "ha2", LD_F32, EP_QUANT, false, 5},    {LIC_HS0, "hs0", LD_I8, EP_RELU, true, 5},
            {LIC_HS1, "hs1", LD_F32, EP_RELU, true, 5},
            {LIC_HS2, "hs2", LD_F32, kind == 1 ? EP_INDEX : EP_NONE, false, 3},
        };
        specs.insert(specs.end(), hyper.begin(), hyper.end());
    }
    if (kind == 2) {
        specs[4].ld = LD_F32;                            // gs0
        std::vector<Spec> ctx = {
            {LIC_CX, "cx", LD_F32, EP_NONE, false, 5, 1},
            {LIC_EP0A, "ep0", LD_F32, EP_RELU, false, 1, 0},   {LIC_EP1A, "ep1", LD_F32, EP_RELU, false, 1, 0},
            {LIC_EP2A, "ep2", LD_F32, EP_MSCALE, false, 1, 0}, {LIC_EP0N, "ep0", LD_F32, EP_RELU, false, 1, 1},
            {LIC_EP1N, "ep1", LD_F32, EP_RELU, false, 1, 1},   {LIC_EP2N, "ep2", LD_F32, EP_MSCALE, false, 1, 1},
        };
        specs.insert(specs.end(), ctx.begin(), ctx.end());
    }

    for (const Spec& sp : specs) {
        LayerGPU& L = layers[sp.id];
        auto wit = P.find(std::string(sp.name) + ".w");
        auto bit = P.find(std::string(sp.name) + ".b");
        if (wit == P.end() || bit == P.end() || wit->second.first.size() != 4) {
            err = std::string("weight blob: missing ") + sp.name;
            return LIC_E_MODEL;
        }
        const std::vector<int>& dims = wit->second.first;
        const std::vector<double>& w = wit->second.second;
        const std::vector<double>& b = bit->second.second;
        const int k = dims[2];
        if (k != sp.k || dims[3] != k) { err = std::string("weight blob: bad kernel size in ") + sp.name; return LIC_E_MODEL; }
        const int ci = sp.deconv ? dims[0] : dims[1];
        const int co = sp.deconv ? dims[1] : dims[0];
        if ((int)b.size() != co) { err = std::string("weight blob: bad bias in ") + sp.name; return LIC_E_MODEL; }
        L.present = true;
        L.ld = sp.ld;
        L.ep = sp.ep;
        L.k = k;
        L.deconv = sp.deconv;
        L.co = co;
        L.rows = sp.ep == EP_RGB;
        // bf16 operands for the analysis / synthesis transforms in the BF16
        // form; h_a and h_s always run in FP32 (fixed-order scale index)
        const bool is_gags = sp.id <= LIC_GA3 || (sp.id >= LIC_GS0 && sp.id <= LIC_GS3);
        L.dt = !is_gags ? DT_F32 : cfg.precision == LIC_PREC_BF16 ? DT_BF16 : cfg.precision == LIC_PREC_FP8 ? DT_FP8 : DT_F32;
        // the e4m3 form's image layer: bf16 operands (a K of 75 is one
        // chunk; pixel values keep 8 bits), e4m3 activations out; so does
        // g_s's first layer (its symbol loader's conversion to e4m3 does not
        // fit two waves per SIMD, the bf16 kernel does; the context model's
        // y_hat = sym + mean arrives as bf16 anyway)
        L.out_e4m3 = L.dt == DT_FP8 && (sp.ld == LD_RGB || sp.id == LIC_GS0);
        if (L.out_e4m3) L.dt = DT_BF16;
        // and its output layer too (bf16 halo tiles: the 3 output channels
        // make a K chunk of 128 (tap, channel) pairs a poor fit), fed by a
        // last GDN layer that stores bf16
        if (L.dt == DT_FP8 && sp.id == LIC_GS3) L.dt = DT_BF16;
        L.out_bf16 = L.dt == DT_FP8 && sp.id == LIC_GS2;
        // 75 (tap, channel) pairs in whole K chunks
        const int krgb = L.dt == DT_FP8 ? 128 : 96;
        L.cin = sp.ld == LD_RGB ? krgb : ci;
        L.cop = L.rows ? 16 : co;
        if (sp.ld == LD_RGB && ci != 3) { err = "ga0 must take 3 channels"; return LIC_E_MODEL; }
        if (!L.rows && co % 16 != 0) { err = std::string("channels must be multiples of 16: ") + sp.name; return LIC_E_MODEL; }
        if (L.rows && co != 3) { err = "gs3 must produce 3 channels"; return LIC_E_MODEL; }
        // packed GEMM operands as index maps into the PyTorch-layout weights
        PackMap pm;
        if (sp.cb >= 0) pm = pack_map_checkerboard(ci, co, k, sp.cb, sp.ep == EP_MSCALE);
        else if (sp.ld == LD_RGB) pm = pack_map(PK_IMG, 3, co, k, 2, k / 2, false, krgb);
        else if (!sp.deconv) pm = pack_map(PK_CONV, ci, co, k, 1, k / 2, false);
        else if (!L.rows) pm = pack_map(PK_DECONV, ci, co, k, 2, k / 2, true);
        else pm = pack_map(PK_ROWS, ci, co, k, 2, k / 2, true);
        if (pm.cin != L.cin || pm.cop != L.cop) { err = std::string("packing mismatch in ") + sp.name; return LIC_E_MODEL; }
        std::vector<PhaseDesc> ph = pm.ph;
        L.nphase = (int)ph.size();

        const size_t total = pm.idx.size();
        const size_t esz = L.dt == DT_BF16 ? 2 : L.dt == DT_FP8 ? 1 : 4;
        L.d_w = (uint8_t*)dev_alloc(total * esz);
        L.d_ph = (PhaseDesc*)dev_alloc(ph.size() * sizeof(PhaseDesc));
        L.d_bias = (float*)dev_alloc(L.cop * sizeof(float));
        if (!L.d_w || !L.d_ph || !L.d_bias) { err = "device allocation failed"; return LIC_E_NOMEM; }
        std::vector<float> wp(total);
        for (size_t j = 0; j < total; ++j) wp[j] = pm.idx[j] < 0 ? 0.0f : (float)w[pm.idx[j]];
        if (L.dt == DT_BF16) {
            std::vector<uint16_t> hb(total);
            for (size_t j = 0; j < total; ++j) hb[j] = bf16_rne(wp[j]);
            HIP_TRY(hipMemcpy(L.d_w, hb.data(), total * esz, hipMemcpyHostToDevice));
        } else if (L.dt == DT_FP8) {
            // per packed row: scale = max |w| / 448 over every tap and phase
            // of the row, w8 = e4m3(w / scale); the epilogue multiplies by
            // scale and by the input's own scale (1 / kActQ for e4m3
            // activations, 1 for the image and for y_hat)
            const size_t cin = (size_t)L.cin;
            std::vector<double> amax(L.cop, 0.0);
            for (size_t i = 0; i < ph.size(); ++i) {
                const size_t end = i + 1 < ph.size() ? pm.off[i + 1] : total;
                for (size_t j = pm.off[i]; j < end; ++j) {
                    const size_t row = ((j - pm.off[i]) / cin) % (size_t)L.cop;
                    amax[row] = std::max(amax[row], (double)std::fabs(wp[j]));
                }
            }
            std::vector<float> wsc(L.cop);
            for (int r = 0; r < L.cop; ++r) wsc[r] = amax[r] > 0.0 ? (float)(amax[r] / 448.0) : 1.0f;
            std::vector<uint8_t> h8(total);
            for (size_t i = 0; i < ph.size(); ++i) {
                const size_t end = i + 1 < ph.size() ? pm.off[i + 1] : total;
                for (size_t j = pm.off[i]; j < end; ++j) h8[j] = e4m3_rne(wp[j] / wsc[((j - pm.off[i]) / cin) % (size_t)L.cop]);
            }
            L.in_scale = (sp.ld == LD_F32) ? 1.0f / kActQ : 1.0f;
            L.wsc = wsc;
            L.d_rscale = (float*)dev_alloc(L.cop * sizeof(float));
            if (!L.d_rscale) { err = "device allocation failed"; return LIC_E_NOMEM; }
            const int rc = upload_rscale(L);
            if (rc != LIC_OK) return rc;
            HIP_TRY(hipMemcpy(L.d_w, h8.data(), total, hipMemcpyHostToDevice));
        } else {
            HIP_TRY(hipMemcpy(L.d_w, wp.data(), total * esz, hipMemcpyHostToDevice));
            if (sp.ep == EP_GDN || sp.ep == EP_IGDN) {
                // split-FP32 operands of the whole-frame kernels: each group of
                // 8 packed values as [part 0 x8][part 1 x8][part 2 x8], the
                // parts rounded to nearest from what the previous ones leave
                if (total % 8 != 0) { err = std::string("packing mismatch in ") + sp.name; return LIC_E_MODEL; }
                std::vector<uint16_t> hx(3 * total);
                for (size_t j = 0; j < total; ++j) {
                    float rem = wp[j];
                    for (int g = 0; g < 3; ++g) {
                        const uint16_t h = bf16_rne(rem);
                        hx[24 * (j / 8) + 8 * g + j % 8] = h;
                        const uint32_t u = (uint32_t)h << 16;
                        float hv;
                        memcpy(&hv, &u, 4);
                        rem -= hv;
                    }
                }
                L.d_wx = (uint16_t*)dev_alloc(hx.size() * sizeof(uint16_t));
                if (!L.d_wx) { err = "device allocation failed"; return LIC_E_NOMEM; }
                HIP_TRY(hipMemcpy(L.d_wx, hx.data(), hx.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
            }
        }
        for (size_t i = 0; i < ph.size(); ++i) ph[i].woff = (int64_t)pm.off[i];
        HIP_TRY(hipMemcpy(L.d_ph, ph.data(), ph.size() * sizeof(PhaseDesc), hipMemcpyHostToDevice));
        L.host_ph = ph;
        L.halo1 = sp.ld != LD_RGB;
        for (const PhaseDesc& d : ph)
            for (int t = 0; t < d.ntaps; ++t)
                if (d.dy[t] < -1 || d.dy[t] > 1 || d.dx[t] < -1 || d.dx[t] > 1) L.halo1 = false;
        std::vector<float> bias(L.cop, 0.0f);
        for (int r = 0; r < L.cop; ++r)
            if (pm.bias_idx[r] >= 0) bias[r] = (float)b[pm.bias_idx[r]];
        HIP_TRY(hipMemcpy(L.d_bias, bias.data(), L.cop * sizeof(float), hipMemcpyHostToDevice));

        if (sp.ep == EP_GDN || sp.ep == EP_IGDN) {
            auto git = P.find(std::string(sp.name) + ".gamma");
            auto beit = P.find(std::string(sp.name) + ".beta");
            if (git == P.end() || beit == P.end() || git->second.second.size() != (size_t)co * co ||
                beit->second.second.size() != (size_t)co) {
                err = std::string("weight blob: GDN parameters missing in ") + sp.name;
                return LIC_E_MODEL;
            }
            if (co % 32 != 0) { err = std::string("GDN layers need a multiple of 32 channels: ") + sp.name; return LIC_E_MODEL; }
            const std::vector<uint16_t> g = gdn_gamma_split(git->second.second, co);
            std::vector<float> be(beit->second.second.begin(), beit->second.second.end());
            L.d_gsplit = (uint16_t*)dev_alloc(g.size() * sizeof(uint16_t));
            L.d_beta = (float*)dev_alloc(be.size() * sizeof(float));
            if (!L.d_gsplit || !L.d_beta) { err = "device allocation failed"; return LIC_E_NOMEM; }
            HIP_TRY(hipMemcpy(L.d_gsplit, g.data(), g.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(L.d_beta, be.data(), be.size() * sizeof(float), hipMemcpyHostToDevice));
        }
        // offsets: quantisation of y (factorized: channel medians; hyperprior: 0)
        // and of z (medians); dequantisation in the loaders likewise
        if (sp.id == LIC_GA3) L.d_qmu = kind == 0 ? d_medians : d_zero;
        if (sp.id == LIC_HA2) L.d_qmu = d_medians;
        if (sp.id == LIC_HS0) L.d_mu_in = d_medians;
        if (sp.id == LIC_GS0) L.d_mu_in = kind == 0 ? d_medians : d_zero;
    }
    if (kind == 2) {
        // kernels are instantiated for these widths (the entropy-parameter
        // layers' K is a template parameter)
        if (N != 128 || M != 192 || layers[LIC_EP1A].cin != 640 || layers[LIC_EP2A].cin != 512 ||
            layers[LIC_EP0A].cin != 4 * M || layers[LIC_EP2A].co != 2 * M || layers[LIC_HS2].co != 2 * M ||
            layers[LIC_CX].co != 2 * M || layers[LIC_CX].cin != M) {
            err = "context model: kernels exist for N = 128, M = 192 (entropy-parameter widths 768, 640, 512, 384)";
            return LIC_E_MODEL;
        }
    }
    return LIC_OK;
}

Geo Codec::geo(int id, const FrameDims& d) const
{
    const int Hp = d.Hp, Wp = d.Wp, Hy = d.Hy, Wy = d.Wy, Hz = d.Hz, Wz = d.Wz;
    switch (id) {
    case LIC_GA0: return {d.H, d.W, Hp / 2, Wp / 2, 2, Hp / 2, Wp / 2, 1};
    case LIC_GA1: return {Hp / 2, Wp / 2, Hp / 4, Wp / 4, 2, Hp / 4, Wp / 4, 1};
    case LIC_GA2: return {Hp / 4, Wp / 4, Hp / 8, Wp / 8, 2, Hp / 8, Wp / 8, 1};
    case LIC_GA3: return {Hp / 8, Wp / 8, Hy, Wy, 2, Hy, Wy, 1};
    case LIC_HA0: return {Hy, Wy, Hy, Wy, 1, Hy, Wy, 1};
    case LIC_HA1: return {Hy, Wy, Hy / 2, Wy / 2, 2, Hy / 2, Wy / 2, 1};
    case LIC_HA2: return {Hy / 2, Wy / 2, Hz, Wz, 2, Hz, Wz, 1};
    case LIC_HS0: return {Hz, Wz, Hz, Wz, 1, 2 * Hz, 2 * Wz, 2};
    case LIC_HS1: return {2 * Hz, 2 * Wz, 2 * Hz, 2 * Wz, 1, Hy, Wy, 2};
    case LIC_HS2: return {Hy, Wy, Hy, Wy, 1, Hy, Wy, 1};
    case LIC_GS0: return {Hy, Wy, Hy, Wy, 1, 2 * Hy, 2 * Wy, 2};
    case LIC_GS1: return {Hp / 8, Wp / 8, Hp / 8, Wp / 8, 1, Hp / 4, Wp / 4, 2};
    case LIC_GS2: return {Hp / 4, Wp / 4, Hp / 4, Wp / 4, 1, Hp / 2, Wp / 2, 2};
    case LIC_GS3: return {Hp / 2, Wp / 2, Hp / 2, Wp / 2, 1, Hp, Wp, 2};
    case LIC_CX: case LIC_EP0A: case LIC_EP1A: case LIC_EP2A: case LIC_EP0N: case LIC_EP1N: case LIC_EP2N:
        return {Hy, Wy, Hy / 2, Wy / 2, 2, Hy, Wy, 2};        // two stride-2 sub-grids per set
    }
    return {0, 0, 0, 0, 0, 0, 0, 0};
}

// Element size of the activations a layer stores (the GDN layers' forms).
static size_t act_bytes(const LayerGPU& L)
{
    if (L.dt == DT_F32 || L.dt == DT_F32X) return 4;
    if (L.dt == DT_BF16) return L.out_e4m3 ? 1 : 2;
    return L.out_bf16 ? 2 : 1;
}

void Codec::layer_bytes(int id, int n, const FrameDims& d, size_t* in, size_t* out, size_t* aux) const
{
    const Geo g = geo(id, d);
    const size_t nn = (size_t)n;
    const size_t img = nn * 3 * d.H * d.W;
    const size_t px_in = nn * g.Hin * g.Win, px_out = nn * g.Hout * g.Wout;
    *aux = 0;
    if (id >= LIC_CX) {
        // context model (float32 tensors on the full latent grid): cx reads
        // y_hat, ep0 the concatenation [psi; ctx] (4M channels), ep1 / ep2 the
        // hidden layers; ep2 writes indices (and symbols) checkerboard-major
        const size_t pl = nn * d.Hy * d.Wy;
        const LayerGPU& L = layers[id];
        *in = pl * L.cin * 4;
        if (id == LIC_CX) *out = pl * 4 * M * 4;
        else if (L.ep == EP_MSCALE) { *out = pl * M; *aux = pl * M; }
        else *out = pl * L.co * 4;
        return;
    }
    // input: the image, int8 symbols, y / z / hyper activations (FP32), or
    // the previous layer's stored activations
    if (id == LIC_GA0) *in = img * 4;
    else if (id == LIC_GS0 && kind == 2) *in = px_in * layers[id].cin * (layers[id].dt == DT_F32 ? 4 : 2);
    else if (id == LIC_HS0 || id == LIC_GS0) *in = px_in * layers[id].cin;
    else if (id >= LIC_HA0 && id <= LIC_HS2) *in = px_in * layers[id].cin * 4;
    else *in = px_in * layers[id].cin * act_bytes(layers[id - 1]);
    switch (id) {
    case LIC_GA3: case LIC_HA2:                       // float values, int8 symbols
        *out = px_out * layers[id].co * 4;
        *aux = px_out * layers[id].co;
        break;
    case LIC_HS2:                                     // uint8 indices, float values
        if (kind == 2) {                              // psi into [psi; ctx]
            *out = px_out * 4 * M * 4;
            break;
        }
        *out = px_out * layers[id].co;
        *aux = px_out * layers[id].co * 4;
        break;
    case LIC_GS3:                                     // cropped image, padded pre-clamp image
        *out = img * 4;
        *aux = nn * 3 * d.Hp * d.Wp * 4;
        break;
    case LIC_HA0: case LIC_HA1: case LIC_HS0: case LIC_HS1:
        *out = px_out * layers[id].co * 4;
        break;
    default:                                          // GDN layers
        *out = px_out * layers[id].co * act_bytes(layers[id]);
    }
}

int Codec::launch_layer(int id, int n, const FrameDims& d, const void* in, void* out, void* aux, hipStream_t s,
                        std::string* errp, KernelKey* chosen, const void* in2, void* out2)
{
    if (id < 0 || id >= LIC_NUM_LAYERS || !layers[id].present) { *errp = "layer not present in this model"; return LIC_E_ARG; }
    const LayerGPU& L = layers[id];
    const Geo g = geo(id, d);
    ConvArgs a{};
    a.in = in;
    a.out = out;
    a.aux = aux;
    a.ph = L.d_ph;
    a.w = L.d_w;
    a.wx = L.d_wx;
    a.zero = d_zero;
    a.bias = L.d_bias;
    a.mu_in = L.d_mu_in;
    a.gsplit = L.d_gsplit;
    a.beta = L.d_beta;
    a.qmu = L.d_qmu;
    a.thr = d_thr;
    a.n = n;
    a.Hin = g.Hin;
    a.Win = g.Win;
    a.Hg = g.Hg;
    a.Wg = g.Wg;
    a.s_in = g.s_in;
    a.Hout = g.Hout;
    a.Wout = g.Wout;
    a.s_out = g.s_out;
    a.Co = L.co;
    a.nphase = L.nphase;
    a.hs_exp = hs_exp;
    a.norm1 = norm;
    a.Hc = d.H;
    a.Wc = d.W;
    a.kk = L.k;
    a.pad = L.k / 2;
    a.rscale = L.d_rscale;
    a.out_q = L.out_q;
    a.sat = d_sat;
    a.out_e4m3 = L.out_e4m3 ? 1 : 0;
    a.out_bf16 = L.out_bf16 ? 1 : 0;

    // context model: psi and the context fill the two halves of [psi; ctx];
    // the last entropy-parameter layer takes y (encoder) and writes y_hat or
    // the means
    if (kind == 2 && (id == LIC_HS2 || id == LIC_CX)) {
        a.co_ld = 4 * M;
        a.co_off = id == LIC_CX ? 2 * M : 0;
    }
    if (L.ep == EP_MSCALE) {
        if (!out2 && !chosen) { *errp = "the last entropy-parameter layer needs its y_hat / mean output"; return LIC_E_ARG; }
        a.cb_part = id == LIC_EP2A ? 0 : 1;
        a.ysrc = static_cast<const float*>(in2);
        a.yq = static_cast<float*>(out2);
    }
    const ConvShape shape{id, L.ld, L.ep, L.dt, L.cin, L.cop, L.nphase, L.halo1 && g.s_in == 1 ? 1 : 0};
    return launch_conv_policy(shape, a, (long)g.Hg * g.Wg, s, errp, chosen);
}

int launch_conv_policy(const ConvShape& L, ConvArgs& a, long policy_pixels, hipStream_t s, std::string* errp,
                       KernelKey* chosen)
{
    KernelKey key{L.tag, L.cin, 0, 0, 0, 1, L.ld, L.ep, L.dt};
    const long pixels = (long)a.n * a.Hg * a.Wg;
    if (L.ep == EP_GDN || L.ep == EP_IGDN) {
        key.mt = L.cop / 16;
        key.nt = key.mt <= 8 ? 2 : 1;
        key.waves = 4;
        a.ncog = 1;
        // fewer than one wave per SIMD (1024 on the chip) from the pixel
        // grid of one image: split K over the 4 waves of a block instead
        const long img_waves = (policy_pixels + 16 * key.nt - 1) / (16 * key.nt) * L.nphase;
        if (L.ld != LD_RGB && img_waves < 1024) {
            // one 16-pixel group per wave first, if that gives at least half
            // a wave per SIMD (and such a kernel exists); else split K
            const long waves1 = (policy_pixels + 15) / 16 * L.nphase;
            KernelKey k1 = key;
            k1.nt = 1;
            if (k1.dt == DT_F32 && a.wx) k1.dt = DT_F32X;
            if (key.nt == 2 && waves1 >= 512 && kernel_available(k1)) key.nt = 1;
            else key.ksplit = 4;
        }
    } else if (L.ep == EP_RGB) {
        // every row of the transposed convolution to 3 channels in one wave;
        // halo tiles staged per block when the taps allow
        key.mt = L.cop / 16;
        key.nt = 4;
        key.waves = 4;
        a.ncog = 1;
        if (L.halo1 && L.ld == LD_F32) {
            KernelKey kt = key;
            kt.ld = LD_TILE;
            if (kernel_available(kt)) key = kt;
        }
    } else {
        // 64-channel x 32-pixel wave tiles; when the grid of one image gives
        // fewer than 2 waves per SIMD, split K over 4 or 8 waves of a block;
        // grids of fewer than 128 such tiles (the 24 x 40 and 12 x 20 hyper
        // layers of a 720p frame) take 16 x 16 tiles (split 8) instead, for
        // 8 times the blocks (measured: h_a's second layer 44 -> 30 us, h_s's
        // first 22 -> 16 us; the 48 x 80 layers are slower that way).  The
        // choice depends on the per-image size only, so a frame gives the
        // same bits alone or in a batch (split-K changes the summation order).
        const long tiles_big = ((policy_pixels + 31) / 32) * L.nphase * (L.cop / 64);
        key.mt = 4; key.nt = 2;
        if (L.cop % 64 != 0 || tiles_big < 128) {
            key.mt = 1; key.nt = 1; key.waves = 8; key.ksplit = 8;
        } else if (tiles_big >= 2048) {
            key.waves = 4; key.ksplit = 1;
        } else if (tiles_big * 4 >= 2048) {
            key.waves = 4; key.ksplit = 4;
        } else {
            key.waves = 8; key.ksplit = 8;
        }
        a.ncog = L.cop / (16 * key.mt);
    }
    // whole-frame GDN layers of the FP32 form run on split-FP32 operands
    if (key.dt == DT_F32 && key.ksplit == 1 && a.wx && (L.ep == EP_GDN || L.ep == EP_IGDN)) {
        KernelKey kx = key;
        kx.dt = DT_F32X;
        if (kernel_available(kx)) {
            key = kx;
            a.w = a.wx;
        }
    }
    const long per_block = (long)(key.waves / key.ksplit) * key.nt * 16;
    // halo tiles: one block per key.waves grid rows x 16 key.nt pixels
    const long tiles = key.ld == LD_TILE
                           ? (long)a.n * ((a.Hg + key.waves - 1) / key.waves) * ((a.Wg + 16 * key.nt - 1) / (16 * key.nt))
                           : (pixels + per_block - 1) / per_block;
    const long nblocks = tiles * L.nphase * a.ncog;
    if (nblocks <= 0 && !chosen) return LIC_OK;
    if (nblocks > (1L << 30)) { *errp = "launch too large"; return LIC_E_BUDGET; }
    if (!kernel_available(key)) { *errp = "no kernel instantiated for this layer shape"; return LIC_E_ARG; }
    if (chosen) {
        *chosen = key;
        return LIC_OK;
    }
    hipError_t e = launch_conv(key, a, (int)nblocks, s);
    if (e != hipSuccess) {
        *errp = std::string("kernel launch failed: ") + hipGetErrorString(e);
        return LIC_E_HIP;
    }
    return LIC_OK;
}

}  // namespace lic
