// Pipeline runtime (Section III.A-B, D of the paper, rebuilt for one MI355X):
//
//  * every frame is a Task that moves through an ordered list of stages;
//  * each GPU stage has one control thread and its own HIP stream; it keeps
//    one frame queued on the stream while it waits for the previous one, so
//    the GPU never idles between frames;
//  * CPU stages (rANS encode, rANS decode of z, rANS decode of y) are split
//    into jobs (the z stream and S row slices of y) run by a worker pool;
//  * per-frame buffers come from a fixed pool of slots (pinned host memory
//    mapped into the device address space, plus device buffers) allocated at
//    create time; the hot path never allocates or frees device memory;
//  * results are delivered in frame order by an in-order sink that also
//    releases the slots.
//
// Encoder (both codecs): GPU (g_a, quantise y; hyperprior: h_a, quantise z,
// h_s, scale index) -> CPU (rANS).  Factorized decoder: CPU -> GPU (g_s).
// Hyperprior decoder: CPU1 (z) -> GPU1 (h_s, index) -> CPU2 (y) -> GPU2 (g_s).
#include <string.h>

#include <algorithm>
#include <chrono>

#include "codec.h"

namespace lic {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

#define HIP_OK(expr)                                                               \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            t->err = std::string(#expr) + ": " + hipGetErrorString(e_);            \
            return LIC_E_HIP;                                                      \
        }                                                                          \
    } while (0)

#define LAUNCH(layer, nimg, in, out, aux, stream)                                  \
    do {                                                                           \
        const bool timed_ = (timed_mask.load() >> (layer)) & 1u;                    \
        if (timed_) hipEventRecord(G.lev[G.cur][layer][0], stream);                \
        int r_ = launch_layer(layer, nimg, d, in, out, aux, stream, &t->err);      \
        if (r_ != LIC_OK) return r_;                                               \
        if (timed_) {                                                              \
            hipEventRecord(G.lev[G.cur][layer][1], stream);                        \
            G.lrec[G.cur][layer] = true;                                           \
        }                                                                          \
    } while (0)

static int stage_gpu_index(StageKind k)
{
    return k == ST_GPU_ENC ? 0 : k == ST_GPU_HS ? 1 : k == ST_GPU_GS ? 2 : -1;
}

// ----------------------------------------------------------------- start
int Codec::start()
{
    const FrameDims d(cfg.max_h, cfg.max_w);
    const size_t ny = (size_t)d.Hy * d.Wy * M;
    const size_t nz = kind == 1 ? (size_t)d.Hz * d.Wz * N : 0;
    const size_t img = (size_t)3 * cfg.max_h * cfg.max_w;
    // worst case rANS: 2 bytes per symbol (f = 1) + 4 state bytes per stream
    const size_t scratch = 2 * (ny + nz) + 16 * (kMaxSlices + 1);
    const size_t bits = header_size(kind, S) + scratch;

    auto fail = [&](const char* what) {
        err = std::string("allocation failed: ") + what;
        return LIC_E_NOMEM;
    };
    if (hipSetDevice(cfg.hip_device) != hipSuccess) { err = "hipSetDevice failed"; return LIC_E_HIP; }
    if (hipStreamCreateWithFlags(&layer_stream, hipStreamNonBlocking) != hipSuccess) { err = "stream"; return LIC_E_HIP; }

    slots.resize(cfg.max_in_flight);
    for (Slot& s : slots) {
        s.h_sym_y = (int8_t*)host_alloc(ny);
        s.d_sym_y = (int8_t*)dev_alloc(ny);
        if (!s.h_sym_y || !s.d_sym_y) return fail("slot y");
        if (kind == 1) {
            s.h_sym_z = (int8_t*)host_alloc(nz);
            s.d_sym_z = (int8_t*)dev_alloc(nz);
            s.h_idx = (uint8_t*)host_alloc(ny);
            s.d_idx = (uint8_t*)dev_alloc(ny);
            if (!s.h_sym_z || !s.d_sym_z || !s.h_idx || !s.d_idx) return fail("slot z/idx");
        }
        s.h_scratch = (uint8_t*)host_alloc(scratch);
        s.scratch_cap = scratch;
        s.h_bits = (uint8_t*)host_alloc(bits);
        s.bits_cap = bits;
        s.d_x = (float*)dev_alloc(img * sizeof(float));
        s.d_xhat = (float*)dev_alloc(img * sizeof(float));
        if (!s.h_scratch || !s.h_bits || !s.d_x || !s.d_xhat) return fail("slot staging");
        void* p = nullptr;
        if (hipHostGetDevicePointer(&p, s.h_sym_y, 0) != hipSuccess) return fail("mapped y");
        s.dm_sym_y = (int8_t*)p;
        if (kind == 1) {
            if (hipHostGetDevicePointer(&p, s.h_idx, 0) != hipSuccess) return fail("mapped idx");
            s.dm_idx = (uint8_t*)p;
            if (hipHostGetDevicePointer(&p, s.h_sym_z, 0) != hipSuccess) return fail("mapped z");
            s.dm_sym_z = (int8_t*)p;
        }
    }
    for (int i = 0; i < (int)slots.size(); ++i) free_slots.push(i);

    // per-stage device scratch, sized for max_h x max_w
    const size_t nA = (size_t)N * (d.Hp / 2) * (d.Wp / 2);
    const size_t nB = (size_t)N * (d.Hp / 4) * (d.Wp / 4);
    const size_t nY = (size_t)M * d.Hy * d.Wy;
    const size_t nH1 = (size_t)N * d.Hy * d.Wy;
    const size_t nH2 = (size_t)N * (d.Hy / 2) * (d.Wy / 2);
    for (int g = 0; g < 3; ++g) {
        GpuStage& G = gpu[g];
        G.kind = g == 0 ? ST_GPU_ENC : g == 1 ? ST_GPU_HS : ST_GPU_GS;
        if (hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking) != hipSuccess) { err = "stream"; return LIC_E_HIP; }
        StageScratch& sc = G.scratch;
        if (g == 0 || g == 2) {
            sc.a = (float*)dev_alloc(nA * sizeof(float));
            sc.b = (float*)dev_alloc(nB * sizeof(float));
            if (!sc.a || !sc.b) return fail("stage scratch");
        }
        if (g == 0) {
            sc.y = (float*)dev_alloc(nY * sizeof(float));
            if (!sc.y) return fail("stage scratch");
        }
        if (kind == 1 && g <= 1) {
            sc.h1 = (float*)dev_alloc(nH1 * sizeof(float));
            sc.h2 = (float*)dev_alloc(nH2 * sizeof(float));
            if (!sc.h1 || !sc.h2) return fail("stage scratch");
        }
    }
    if (cfg.hbm_budget_bytes && dev_bytes > cfg.hbm_budget_bytes) {
        err = "pools exceed the device memory budget";
        return LIC_E_BUDGET;
    }
    for (int g = 0; g < 3; ++g) gpu[g].thread = std::thread(&Codec::gpu_loop, this, g);
    for (int w = 0; w < cfg.entropy_threads; ++w) workers.emplace_back(&Codec::worker_loop, this);
    started = true;
    return LIC_OK;
}

void Codec::stop()
{
    if (!started) return;
    for (int g = 0; g < 3; ++g) gpu[g].queue.close();
    jobs.close();
    for (int g = 0; g < 3; ++g)
        if (gpu[g].thread.joinable()) gpu[g].thread.join();
    for (auto& w : workers)
        if (w.joinable()) w.join();
    workers.clear();
    started = false;
}

Codec::~Codec()
{
    stop();
    hipSetDevice(cfg.hip_device);
    hipDeviceSynchronize();
    for (int g = 0; g < 3; ++g)
        if (gpu[g].stream) hipStreamDestroy(gpu[g].stream);
    if (layer_stream) hipStreamDestroy(layer_stream);
    for (void* p : dev_allocs) hipFree(p);
    for (void* p : host_allocs) hipHostFree(p);
}

// ------------------------------------------------------------- dispatch
void Codec::advance(Task* t)
{
    CallState& cs = *call;
    if (t->status != 0) {
        finish_task(t);
        return;
    }
    t->stage++;
    if (t->stage >= (int)cs.stages.size()) {
        finish_task(t);
        return;
    }
    const StageKind k = cs.stages[t->stage];
    const int g = stage_gpu_index(k);
    if (g >= 0) {
        gpu[g].queue.push(t);
    } else {
        const int parts = cpu_parts(k);
        t->jobs_left.store(parts);
        for (int p = 0; p < parts; ++p) jobs.push(Job{t, p});
    }
}

void Codec::finish_task(Task* t)
{
    CallState& cs = *call;
    t->t_done = now_s();
    std::lock_guard<std::mutex> g(cs.m);
    cs.finished[t->frame] = 1;
    while (cs.next_sink < cs.n && cs.finished[cs.next_sink]) {
        Task* s = cs.tasks[cs.next_sink].get();
        if (s->status != 0 && cs.status == 0) {
            cs.status = s->status;
            cs.err = s->err;
        }
        if (cs.lens && s->status == 0) {
            cs.lens[s->frame] = s->bits_len;
            if (cs.out && !cs.overflow && cs.offset + s->bits_len <= cs.cap)
                memcpy(cs.out + cs.offset, slots[s->slot].h_bits, s->bits_len);
            else
                cs.overflow = true;
            cs.offset += s->bits_len;
        }
        free_slots.push(s->slot);
        cs.next_sink++;
        cs.done++;
    }
    cs.cv.notify_all();
}

// ------------------------------------------------------------- GPU side
void Codec::gpu_loop(int gi)
{
    GpuStage& G = gpu[gi];
    hipSetDevice(cfg.hip_device);
    hipEvent_t ev_start[2], ev_end[2];
    for (int i = 0; i < 2; ++i) {
        hipEventCreate(&ev_start[i]);
        hipEventCreate(&ev_end[i]);
        for (int l = 0; l < LIC_NUM_LAYERS; ++l) {
            hipEventCreate(&G.lev[i][l][0]);
            hipEventCreate(&G.lev[i][l][1]);
        }
    }
    Task* pending = nullptr;
    int pend_ev = 0, cur_ev = 0;
    auto complete = [&](Task* t, int e) {
        if (hipEventSynchronize(ev_end[e]) != hipSuccess && t->status == 0) {
            t->status = LIC_E_HIP;
            t->err = "GPU stage failed";
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev_start[e], ev_end[e]) == hipSuccess) G.busy_s += ms * 1e-3;
        for (int l = 0; l < LIC_NUM_LAYERS; ++l) {
            if (!G.lrec[e][l]) continue;
            float lms = 0.0f;
            if (hipEventElapsedTime(&lms, G.lev[e][l][0], G.lev[e][l][1]) == hipSuccess) {
                std::lock_guard<std::mutex> g(lt_m);
                layer_ms[l] += lms;
                layer_launches[l]++;
            }
            G.lrec[e][l] = false;
        }
        advance(t);
    };
    for (;;) {
        Task* t = nullptr;
        if (pending) {
            if (!G.queue.try_pop(&t)) {
                complete(pending, pend_ev);
                pending = nullptr;
                continue;
            }
        } else if (!G.queue.pop(&t)) {
            break;
        }
        hipEventRecord(ev_start[cur_ev], G.stream);
        G.cur = cur_ev;
        int rc = G.kind == ST_GPU_ENC ? gpu_encode(t, G) : G.kind == ST_GPU_HS ? gpu_hs(t, G) : gpu_gs(t, G);
        if (rc != LIC_OK) t->status = rc;
        hipEventRecord(ev_end[cur_ev], G.stream);
        if (pending) complete(pending, pend_ev);
        pending = t;
        pend_ev = cur_ev;
        cur_ev ^= 1;
    }
    if (pending) complete(pending, pend_ev);
    for (int i = 0; i < 2; ++i) {
        hipEventDestroy(ev_start[i]);
        hipEventDestroy(ev_end[i]);
        for (int l = 0; l < LIC_NUM_LAYERS; ++l) {
            hipEventDestroy(G.lev[i][l][0]);
            hipEventDestroy(G.lev[i][l][1]);
        }
    }
}

int Codec::gpu_encode(Task* t, GpuStage& G)
{
    const FrameDims& d = call->dims;
    Slot& s = slots[t->slot];
    StageScratch& sc = G.scratch;
    hipStream_t st = G.stream;
    const size_t ny = (size_t)d.Hy * d.Wy * M, nz = (size_t)d.Hz * d.Wz * N;
    const float* x = t->x;
    if (!call->is_device) {
        HIP_OK(hipMemcpyAsync(s.d_x, t->x, (size_t)3 * d.H * d.W * sizeof(float), hipMemcpyHostToDevice, st));
        x = s.d_x;
    }
    const bool zc = cfg.zero_copy != 0;
    LAUNCH(LIC_GA0, 1, x, sc.a, nullptr, st);
    LAUNCH(LIC_GA1, 1, sc.a, sc.b, nullptr, st);
    LAUNCH(LIC_GA2, 1, sc.b, sc.a, nullptr, st);
    LAUNCH(LIC_GA3, 1, sc.a, kind == 1 ? sc.y : nullptr, zc ? (void*)s.dm_sym_y : (void*)s.d_sym_y, st);
    if (kind == 1) {
        LAUNCH(LIC_HA0, 1, sc.y, sc.h1, nullptr, st);
        LAUNCH(LIC_HA1, 1, sc.h1, sc.h2, nullptr, st);
        LAUNCH(LIC_HA2, 1, sc.h2, nullptr, s.d_sym_z, st);
        // h_s runs on the quantised z exactly as the decoder will
        LAUNCH(LIC_HS0, 1, s.d_sym_z, sc.h2, nullptr, st);
        LAUNCH(LIC_HS1, 1, sc.h2, sc.h1, nullptr, st);
        LAUNCH(LIC_HS2, 1, sc.h1, zc ? (void*)s.dm_idx : (void*)s.d_idx, nullptr, st);
        HIP_OK(hipMemcpyAsync(s.h_sym_z, s.d_sym_z, nz, hipMemcpyDeviceToHost, st));
        if (!zc) HIP_OK(hipMemcpyAsync(s.h_idx, s.d_idx, ny, hipMemcpyDeviceToHost, st));
    }
    if (!zc) HIP_OK(hipMemcpyAsync(s.h_sym_y, s.d_sym_y, ny, hipMemcpyDeviceToHost, st));
    return LIC_OK;
}

int Codec::gpu_hs(Task* t, GpuStage& G)
{
    const FrameDims& d = call->dims;
    Slot& s = slots[t->slot];
    StageScratch& sc = G.scratch;
    hipStream_t st = G.stream;
    const size_t ny = (size_t)d.Hy * d.Wy * M, nz = (size_t)d.Hz * d.Wz * N;
    const bool zc = cfg.zero_copy != 0;
    HIP_OK(hipMemcpyAsync(s.d_sym_z, s.h_sym_z, nz, hipMemcpyHostToDevice, st));
    LAUNCH(LIC_HS0, 1, s.d_sym_z, sc.h2, nullptr, st);
    LAUNCH(LIC_HS1, 1, sc.h2, sc.h1, nullptr, st);
    LAUNCH(LIC_HS2, 1, sc.h1, zc ? (void*)s.dm_idx : (void*)s.d_idx, nullptr, st);
    if (!zc) HIP_OK(hipMemcpyAsync(s.h_idx, s.d_idx, ny, hipMemcpyDeviceToHost, st));
    return LIC_OK;
}

int Codec::gpu_gs(Task* t, GpuStage& G)
{
    const FrameDims& d = call->dims;
    Slot& s = slots[t->slot];
    StageScratch& sc = G.scratch;
    hipStream_t st = G.stream;
    const size_t ny = (size_t)d.Hy * d.Wy * M;
    HIP_OK(hipMemcpyAsync(s.d_sym_y, s.h_sym_y, ny, hipMemcpyHostToDevice, st));
    float* xo = call->is_device ? t->xhat : s.d_xhat;
    LAUNCH(LIC_GS0, 1, s.d_sym_y, sc.a, nullptr, st);
    LAUNCH(LIC_GS1, 1, sc.a, sc.b, nullptr, st);
    LAUNCH(LIC_GS2, 1, sc.b, sc.a, nullptr, st);
    LAUNCH(LIC_GS3, 1, sc.a, xo, nullptr, st);
    if (!call->is_device)
        HIP_OK(hipMemcpyAsync(t->xhat, s.d_xhat, (size_t)3 * d.H * d.W * sizeof(float), hipMemcpyDeviceToHost, st));
    return LIC_OK;
}

// ------------------------------------------------------------- CPU side
int Codec::cpu_parts(StageKind k) const
{
    switch (k) {
    case ST_CPU_ENC: return call->S + (kind == 1 ? 1 : 0);
    case ST_CPU_DEC_Z: return 1;
    case ST_CPU_DEC_Y: return call->S;
    default: return 0;
    }
}

void Codec::worker_loop()
{
    Job j;
    while (jobs.pop(&j)) {
        Task* t = j.task;
        const StageKind k = call->stages[t->stage];
        const double t0 = now_s();
        if (t->status == 0) {
            int rc = cpu_job(t, j.part);
            if (rc != LIC_OK && t->status == 0) t->status = rc;   // first failure wins (benign race)
        }
        cpu_busy_us += (long)((now_s() - t0) * 1e6);
        if (t->jobs_left.fetch_sub(1) == 1) {
            if (t->status == 0) {
                int rc = cpu_finalize(t, k);
                if (rc != LIC_OK) t->status = rc;
            }
            advance(t);
        }
    }
}

// Slice s of y covers latent rows [s*Hy/S, (s+1)*Hy/S).
static inline void slice_rows(int Hy, int S, int s, int* r0, int* r1)
{
    *r0 = (int)((long)s * Hy / S);
    *r1 = (int)((long)(s + 1) * Hy / S);
}

int Codec::cpu_job(Task* t, int part)
{
    const FrameDims& d = call->dims;
    Slot& s = slots[t->slot];
    const StageKind k = call->stages[t->stage];
    const size_t row = (size_t)d.Wy * M;
    const size_t ny = (size_t)d.Hy * row, nz = kind == 1 ? (size_t)d.Hz * d.Wz * N : 0;
    if (k == ST_CPU_ENC) {
        // scratch regions: z first, then each slice, each 2 bytes/symbol + 16
        if (kind == 1 && part == 0) {
            long len = rans_encode_channel(s.h_sym_z, (long)nz, N, fact, s.h_scratch, 2 * nz + 16);
            if (len < 0) { t->err = "rANS z overflow"; return LIC_E_STATE; }
            t->part_len[0] = (size_t)len;
            return LIC_OK;
        }
        const int si = part - (kind == 1 ? 1 : 0);
        int r0, r1;
        slice_rows(d.Hy, call->S, si, &r0, &r1);
        uint8_t* region = s.h_scratch + (kind == 1 ? 2 * nz + 16 : 0) + 2 * (size_t)r0 * row + 16 * (size_t)si;
        const size_t cap = 2 * (size_t)(r1 - r0) * row + 16;
        const size_t off = (size_t)r0 * row, cnt = (size_t)(r1 - r0) * row;
        long len = kind == 1 ? rans_encode(s.h_sym_y + off, s.h_idx + off, (long)cnt, gauss, region, cap)
                             : rans_encode_channel(s.h_sym_y + off, (long)cnt, M, fact, region, cap);
        if (len < 0) { t->err = "rANS y overflow"; return LIC_E_STATE; }
        t->part_len[part] = (size_t)len;
        return LIC_OK;
    }
    if (k == ST_CPU_DEC_Z) {
        if (rans_decode_channel(t->zp, t->zlen, (long)nz, N, fact, s.h_sym_z) != 0) {
            t->err = "corrupt z stream";
            return LIC_E_CORRUPT;
        }
        return LIC_OK;
    }
    if (k == ST_CPU_DEC_Y) {
        int r0, r1;
        slice_rows(d.Hy, call->S, part, &r0, &r1);
        const size_t off = (size_t)r0 * row, cnt = (size_t)(r1 - r0) * row;
        int rc = kind == 1 ? rans_decode(t->yp[part], t->ylen[part], s.h_idx + off, (long)cnt, gauss, s.h_sym_y + off)
                           : rans_decode_channel(t->yp[part], t->ylen[part], (long)cnt, M, fact, s.h_sym_y + off);
        if (rc != 0) { t->err = "corrupt y stream"; return LIC_E_CORRUPT; }
        (void)ny;
        return LIC_OK;
    }
    return LIC_E_STATE;
}

int Codec::cpu_finalize(Task* t, StageKind k)
{
    if (k != ST_CPU_ENC) return LIC_OK;
    const FrameDims& d = call->dims;
    const int S = call->S;
    Slot& s = slots[t->slot];
    const size_t row = (size_t)d.Wy * M;
    const size_t nz = kind == 1 ? (size_t)d.Hz * d.Wz * N : 0;
    StreamHeader h;
    h.kind = kind;
    h.hs_exp = hs_exp;
    h.S = S;
    h.H = d.H;
    h.W = d.W;
    h.N = N;
    h.M = M;
    h.model_id = model_id;
    uint32_t ylen[kMaxSlices];
    const int y0 = kind == 1 ? 1 : 0;
    size_t total = header_size(kind, S) + (kind == 1 ? t->part_len[0] : 0);
    for (int i = 0; i < S; ++i) {
        ylen[i] = (uint32_t)t->part_len[y0 + i];
        total += ylen[i];
    }
    if (total > s.bits_cap) { t->err = "bitstream exceeds slot"; return LIC_E_STATE; }
    write_header(s.h_bits, h, kind == 1 ? (uint32_t)t->part_len[0] : 0, ylen);
    uint8_t* p = s.h_bits + header_size(kind, S);
    if (kind == 1) {
        memcpy(p, s.h_scratch, t->part_len[0]);
        t->zp = p;
        t->zlen = t->part_len[0];
        p += t->part_len[0];
    }
    for (int i = 0; i < S; ++i) {
        int r0, r1;
        slice_rows(d.Hy, S, i, &r0, &r1);
        const uint8_t* region = s.h_scratch + (kind == 1 ? 2 * nz + 16 : 0) + 2 * (size_t)r0 * row + 16 * (size_t)i;
        memcpy(p, region, ylen[i]);
        t->yp[i] = p;
        t->ylen[i] = ylen[i];
        p += ylen[i];
    }
    t->bits_len = total;
    return LIC_OK;
}

// ------------------------------------------------------------- one call
int Codec::run_call(CallState& cs)
{
    call = &cs;
    cs.finished.assign(cs.n, 0);
    const double t0 = now_s();
    for (int i = 0; i < cs.n; ++i) {
        int slot;
        if (!free_slots.pop(&slot)) { call = nullptr; err = "codec stopped"; return LIC_E_STATE; }
        Task* t = cs.tasks[i].get();
        t->slot = slot;
        t->stage = -1;
        t->t_admit = now_s();
        advance(t);
    }
    {
        std::unique_lock<std::mutex> g(cs.m);
        cs.cv.wait(g, [&] { return cs.done == cs.n; });
    }
    last_wall_s = now_s() - t0;
    last_frames = cs.n;
    last_lat_ms.resize(cs.n);
    for (int i = 0; i < cs.n; ++i) last_lat_ms[i] = (cs.tasks[i]->t_done - cs.tasks[i]->t_admit) * 1e3;
    call = nullptr;
    if (cs.status != 0) {
        err = cs.err;
        return cs.status;
    }
    return LIC_OK;
}

}  // namespace lic
