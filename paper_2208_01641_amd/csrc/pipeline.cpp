// Pipeline runtime (Section III.A-B, D of the paper, rebuilt for one MI355X):
//
//  * frames travel in tasks (up to max_batch consecutive frames) through an
//    ordered list of stages - the per-frame state machine of the paper;
//  * each GPU stage has one control thread and its own HIP stream; it keeps
//    one task queued on the stream while it waits for the previous one, so
//    the GPU never idles between tasks;
//  * CPU stages (rANS encode, rANS decode of z, rANS decode of y) are split
//    into jobs (per frame: the z stream and S row slices of y) run by a
//    worker pool;
//  * per-task buffers come from a fixed pool of slots (pinned host memory
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

#include <math.h>

#include "codec.h"
#include "distill_kernels.h"

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
            t->fail(LIC_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
            return LIC_E_HIP;                                                      \
        }                                                                          \
    } while (0)

#define LAUNCH(layer, in, out, aux, stream)                                        \
    do {                                                                           \
        const bool timed_ = !G.capturing && ((timed_mask.load() >> (layer)) & 1u);  \
        if (timed_) (void)hipEventRecord(G.lev[G.cur][layer][0], stream);          \
        std::string e_;                                                            \
        int r_ = launch_layer(layer, t->nb, d, in, out, aux, stream, &e_);         \
        if (r_ != LIC_OK) {                                                        \
            t->fail(r_, e_);                                                       \
            return r_;                                                             \
        }                                                                          \
        if (timed_) {                                                              \
            (void)hipEventRecord(G.lev[G.cur][layer][1], stream);                  \
            G.lrec[G.cur][layer] = true;                                           \
        }                                                                          \
    } while (0)

// the same for the last entropy-parameter layer (second input and output)
#define LAUNCH2(layer, in, out, aux, in2, out2, stream)                            \
    do {                                                                           \
        const bool timed_ = !G.capturing && ((timed_mask.load() >> (layer)) & 1u);  \
        if (timed_) (void)hipEventRecord(G.lev[G.cur][layer][0], stream);          \
        std::string e_;                                                            \
        int r_ = launch_layer(layer, t->nb, d, in, out, aux, stream, &e_, nullptr, in2, out2); \
        if (r_ != LIC_OK) {                                                        \
            t->fail(r_, e_);                                                       \
            return r_;                                                             \
        }                                                                          \
        if (timed_) {                                                              \
            (void)hipEventRecord(G.lev[G.cur][layer][1], stream);                  \
            G.lrec[G.cur][layer] = true;                                           \
        }                                                                          \
    } while (0)

static int stage_gpu_index(StageKind k)
{
    return k == ST_GPU_ENC ? 0 : (k == ST_GPU_HS || k == ST_GPU_CTX) ? 1 : k == ST_GPU_GS ? 2 : -1;
}

// worst case rANS output: 2 bytes per symbol (f = 1) + 4 state bytes per
// stream; regions of the per-frame scratch: z first, then each y slice
static size_t scratch_bytes(size_t ny, size_t nz) { return 2 * (ny + nz) + kStreamSlack * (2 * kMaxSlices + 1); }

// ----------------------------------------------------------------- start
int Codec::start()
{
    const FrameDims d(cfg.max_h, cfg.max_w);
    const int B = cfg.max_batch;
    const size_t ny = (size_t)d.Hy * d.Wy * M;
    const size_t nz = kind >= 1 ? (size_t)d.Hz * d.Wz * N : 0;
    const size_t img = (size_t)3 * cfg.max_h * cfg.max_w;
    const size_t scratch = scratch_bytes(ny, nz);
    const size_t bits = header_size(kind, kMaxSlices) + scratch;

    auto fail = [&](const char* what) {
        err = std::string("allocation failed: ") + what;
        return LIC_E_NOMEM;
    };
    if (hipSetDevice(cfg.hip_device) != hipSuccess) { err = "hipSetDevice failed"; return LIC_E_HIP; }
    if (hipStreamCreateWithFlags(&layer_stream, hipStreamNonBlocking) != hipSuccess) { err = "stream"; return LIC_E_HIP; }

    slots.resize(cfg.max_in_flight);
    for (Slot& s : slots) {
        s.h_sym_y = (int8_t*)host_alloc(B * ny);
        s.d_sym_y = (int8_t*)dev_alloc(B * ny);
        if (!s.h_sym_y || !s.d_sym_y) return fail("slot y");
        if (kind >= 1) {
            s.h_sym_z = (int8_t*)host_alloc(B * nz);
            s.d_sym_z = (int8_t*)dev_alloc(B * nz);
            s.h_idx = (uint8_t*)host_alloc(B * ny);
            s.d_idx = (uint8_t*)dev_alloc(B * ny);
            if (!s.h_sym_z || !s.d_sym_z || !s.h_idx || !s.d_idx) return fail("slot z/idx");
        }
        if (kind == 2) {
            s.d_zc = (float*)dev_alloc(B * ny * 4 * sizeof(float));
            s.d_mu = (float*)dev_alloc(B * ny * sizeof(float));
            if (!s.d_zc || !s.d_mu) return fail("slot context");
        }
        s.h_scratch = (uint8_t*)host_alloc(B * scratch);
        s.scratch_per_frame = scratch;
        s.h_bits = (uint8_t*)host_alloc(B * bits);
        s.bits_per_frame = bits;
        s.d_x = (float*)dev_alloc(B * img * sizeof(float));
        s.d_xhat = (float*)dev_alloc(B * img * sizeof(float));
        if (!s.h_scratch || !s.h_bits || !s.d_x || !s.d_xhat) return fail("slot staging");
        void* p = nullptr;
        if (hipHostGetDevicePointer(&p, s.h_sym_y, 0) != hipSuccess) return fail("mapped y");
        s.dm_sym_y = (int8_t*)p;
        if (kind >= 1) {
            if (hipHostGetDevicePointer(&p, s.h_idx, 0) != hipSuccess) return fail("mapped idx");
            s.dm_idx = (uint8_t*)p;
        }
    }
    for (int i = 0; i < (int)slots.size(); ++i) free_slots.push(i);

    // per-stage device scratch, sized for max_batch frames of max_h x max_w
    const size_t nA = (size_t)B * N * (d.Hp / 2) * (d.Wp / 2);
    const size_t nB = (size_t)B * N * (d.Hp / 4) * (d.Wp / 4);
    const size_t nY = (size_t)B * M * d.Hy * d.Wy;
    const size_t nH1 = (size_t)B * N * d.Hy * d.Wy;
    const size_t nH2 = (size_t)B * N * (d.Hy / 2) * (d.Wy / 2);
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
        if (kind >= 1 && g <= 1) {
            sc.h1 = (float*)dev_alloc(nH1 * sizeof(float));
            sc.h2 = (float*)dev_alloc(nH2 * sizeof(float));
            if (!sc.h1 || !sc.h2) return fail("stage scratch");
        }
        if (kind == 2) {
            const size_t pl = (size_t)B * d.Hy * d.Wy;
            if (g <= 1) {
                sc.e1 = (float*)dev_alloc(pl * layers[LIC_EP0A].co * sizeof(float));
                sc.e2 = (float*)dev_alloc(pl * layers[LIC_EP1A].co * sizeof(float));
                if (!sc.e1 || !sc.e2) return fail("stage scratch");
            }
            sc.yh = (float*)dev_alloc(nY * sizeof(float));
            if (!sc.yh) return fail("stage scratch");
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


// ------------------------------------------------------------- dispatch
void Codec::advance(Task* t)
{
    const Route& rt = *t->route;
    if (t->status.load() != 0) {
        finish_task(t);
        return;
    }
    t->stage++;
    if (t->stage >= (int)rt.stages.size()) {
        finish_task(t);
        return;
    }
    const StageKind k = rt.stages[t->stage];
    const int g = stage_gpu_index(k);
    if (g >= 0) {
        gpu[g].queue.push(t);
    } else {
        const int parts = cpu_parts(t, k) * t->nb;
        t->jobs_left.store(parts);
        for (int p = 0; p < parts; ++p) jobs.push(Job{t, p});
    }
}

void Codec::finish_task(Task* t)
{
    t->t_done = now_s();
    if (!t->call) {
        server_finish(t);
        return;
    }
    CallState& cs = *t->call;
    std::lock_guard<std::mutex> g(cs.m);
    cs.finished[t->index] = 1;
    while (cs.next_sink < (int)cs.tasks.size() && cs.finished[cs.next_sink]) {
        Task* s = cs.tasks[cs.next_sink].get();
        if (s->status.load() != 0 && cs.status == 0) {
            cs.status = s->status.load();
            cs.err = s->err;
        }
        if (cs.lens && s->status.load() == 0) {
            const Slot& sl = slots[s->slot];
            for (int b = 0; b < s->nb; ++b) {
                cs.lens[s->first + b] = s->bits_len[b];
                if (cs.out && !cs.overflow && cs.offset + s->bits_len[b] <= cs.cap)
                    memcpy(cs.out + cs.offset, sl.h_bits + (size_t)b * sl.bits_per_frame, s->bits_len[b]);
                else
                    cs.overflow = true;
                cs.offset += s->bits_len[b];
            }
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
    (void)hipSetDevice(cfg.hip_device);
    hipEvent_t ev_start[2], ev_end[2];
    for (int i = 0; i < 2; ++i) {
        (void)hipEventCreate(&ev_start[i]);
        (void)hipEventCreate(&ev_end[i]);
        for (int l = 0; l < LIC_NUM_LAYERS; ++l) {
            (void)hipEventCreate(&G.lev[i][l][0]);
            (void)hipEventCreate(&G.lev[i][l][1]);
        }
    }
    Task* pending = nullptr;
    int pend_ev = 0, cur_ev = 0;
    auto complete = [&](Task* t, int e) {
        if (hipEventSynchronize(ev_end[e]) != hipSuccess) t->fail(LIC_E_HIP, "GPU stage failed");
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
        (void)hipEventRecord(ev_start[cur_ev], G.stream);
        G.cur = cur_ev;
        t->judge = false;
        if (G.kind == ST_GPU_GS && cfg.gs_mode == 2 && distill && !gs_fallback.load()) {
            // judge the task holding frame f with f % judge_every == 0
            const long f0 = gs_frames.fetch_add(t->nb);
            t->judge = f0 % judge_every == 0 || f0 % judge_every + t->nb > judge_every;
        }
        const StageKind sk = t->route->stages[t->stage];
        int (Codec::*body)(Task*, GpuStage&) = sk == ST_GPU_ENC ? &Codec::gpu_encode
                                               : sk == ST_GPU_HS ? &Codec::gpu_hs
                                               : sk == ST_GPU_CTX ? &Codec::gpu_ctx : &Codec::gpu_gs;
        if (!t->call && cfg.use_graphs) {
            // serving: request buffers in and out around a per-(stage, size,
            // batch, slot) graph that only touches pool buffers
            const FrameDims& d = t->route->dims;
            const size_t fsz = (size_t)3 * d.H * d.W;
            const hipMemcpyKind kin = t->route->is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
            const hipMemcpyKind kout = t->route->is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
            bool ok = true;
            if (G.kind == ST_GPU_ENC)
                for (int b = 0; b < t->nb && ok; ++b)
                    ok = hipMemcpyAsync(slots[t->slot].d_x + b * fsz, t->xs[b], fsz * sizeof(float), kin, G.stream) ==
                         hipSuccess;
            t->staged = true;
            if (!ok) t->fail(LIC_E_HIP, "input copy failed");
            // a judged task runs eagerly: the judge waits for its result
            else if ((t->judge ? (this->*body)(t, G) : gpu_stage_graph(t, G, body)) == LIC_OK && G.kind == ST_GPU_GS)
                for (int b = 0; b < t->nb && ok; ++b)
                    ok = hipMemcpyAsync(t->xhats[b], slots[t->slot].d_xhat + b * fsz, fsz * sizeof(float), kout,
                                        G.stream) == hipSuccess;
            if (!ok) t->fail(LIC_E_HIP, "output copy failed");
        } else {
            t->staged = false;
            (this->*body)(t, G);
        }
        (void)hipEventRecord(ev_end[cur_ev], G.stream);
        if (pending) complete(pending, pend_ev);
        pending = t;
        pend_ev = cur_ev;
        cur_ev ^= 1;
    }
    if (pending) complete(pending, pend_ev);
    for (int i = 0; i < 2; ++i) {
        (void)hipEventDestroy(ev_start[i]);
        (void)hipEventDestroy(ev_end[i]);
        for (int l = 0; l < LIC_NUM_LAYERS; ++l) {
            (void)hipEventDestroy(G.lev[i][l][0]);
            (void)hipEventDestroy(G.lev[i][l][1]);
        }
    }
}

// Frames of a task read in place when they are contiguous device memory,
// else gathered into the slot's staging buffer.
static bool frames_contiguous(const Task* t, size_t fsz, bool out)
{
    for (int b = 1; b < t->nb; ++b)
        if (out ? t->xhats[b] != t->xhats[0] + b * fsz : t->xs[b] != t->xs[0] + b * fsz) return false;
    return true;
}

int Codec::gpu_encode(Task* t, GpuStage& G)
{
    const FrameDims& d = t->route->dims;
    Slot& s = slots[t->slot];
    StageScratch& sc = G.scratch;
    hipStream_t st = G.stream;
    const size_t ny = (size_t)t->nb * d.Hy * d.Wy * M, nz = (size_t)t->nb * d.Hz * d.Wz * N;
    const size_t fsz = (size_t)3 * d.H * d.W;
    const bool dev = t->route->is_device != 0;
    const float* x = t->xs[0];
    if (t->staged) {
        x = s.d_x;
    } else if (!dev || !t->call || !frames_contiguous(t, fsz, false)) {
        for (int b = 0; b < t->nb; ++b)
            HIP_OK(hipMemcpyAsync(s.d_x + b * fsz, t->xs[b], fsz * sizeof(float),
                                  dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
        x = s.d_x;
    }
    const bool zc = cfg.zero_copy != 0;
    LAUNCH(LIC_GA0, x, sc.a, nullptr, st);
    LAUNCH(LIC_GA1, sc.a, sc.b, nullptr, st);
    LAUNCH(LIC_GA2, sc.b, sc.a, nullptr, st);
    if (kind == 2) {
        // context model: y's symbols come from the two checkerboard passes
        // (quantised around the means), which write them checkerboard-major
        // into device buffers
        LAUNCH(LIC_GA3, sc.a, sc.y, s.d_sym_y, st);
        LAUNCH(LIC_HA0, sc.y, sc.h1, nullptr, st);
        LAUNCH(LIC_HA1, sc.h1, sc.h2, nullptr, st);
        LAUNCH(LIC_HA2, sc.h2, nullptr, s.d_sym_z, st);
        LAUNCH(LIC_HS0, s.d_sym_z, sc.h2, nullptr, st);
        LAUNCH(LIC_HS1, sc.h2, sc.h1, nullptr, st);
        LAUNCH(LIC_HS2, sc.h1, s.d_zc, nullptr, st);
        HIP_OK(launch_cb_fill(s.d_zc, t->nb, d.Hy, d.Wy, 4 * M, 2 * M, 2 * M, 0, 0.0f, st));
        LAUNCH(LIC_EP0A, s.d_zc, sc.e1, nullptr, st);
        LAUNCH(LIC_EP1A, sc.e1, sc.e2, nullptr, st);
        LAUNCH2(LIC_EP2A, sc.e2, s.d_idx, s.d_sym_y, sc.y, sc.yh, st);
        LAUNCH(LIC_CX, sc.yh, s.d_zc, nullptr, st);
        LAUNCH(LIC_EP0N, s.d_zc, sc.e1, nullptr, st);
        LAUNCH(LIC_EP1N, sc.e1, sc.e2, nullptr, st);
        LAUNCH2(LIC_EP2N, sc.e2, s.d_idx, s.d_sym_y, sc.y, sc.yh, st);
        HIP_OK(hipMemcpyAsync(s.h_sym_z, s.d_sym_z, nz, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(s.h_idx, s.d_idx, ny, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(s.h_sym_y, s.d_sym_y, ny, hipMemcpyDeviceToHost, st));
        return LIC_OK;
    }
    LAUNCH(LIC_GA3, sc.a, kind == 1 ? sc.y : nullptr, zc ? (void*)s.dm_sym_y : (void*)s.d_sym_y, st);
    if (kind == 1) {
        LAUNCH(LIC_HA0, sc.y, sc.h1, nullptr, st);
        LAUNCH(LIC_HA1, sc.h1, sc.h2, nullptr, st);
        LAUNCH(LIC_HA2, sc.h2, nullptr, s.d_sym_z, st);
        // h_s runs on the quantised z exactly as the decoder will
        LAUNCH(LIC_HS0, s.d_sym_z, sc.h2, nullptr, st);
        LAUNCH(LIC_HS1, sc.h2, sc.h1, nullptr, st);
        LAUNCH(LIC_HS2, sc.h1, zc ? (void*)s.dm_idx : (void*)s.d_idx, nullptr, st);
        HIP_OK(hipMemcpyAsync(s.h_sym_z, s.d_sym_z, nz, hipMemcpyDeviceToHost, st));
        if (!zc) HIP_OK(hipMemcpyAsync(s.h_idx, s.d_idx, ny, hipMemcpyDeviceToHost, st));
    }
    if (!zc) HIP_OK(hipMemcpyAsync(s.h_sym_y, s.d_sym_y, ny, hipMemcpyDeviceToHost, st));
    return LIC_OK;
}

int Codec::gpu_hs(Task* t, GpuStage& G)
{
    const FrameDims& d = t->route->dims;
    Slot& s = slots[t->slot];
    StageScratch& sc = G.scratch;
    hipStream_t st = G.stream;
    const size_t ny = (size_t)t->nb * d.Hy * d.Wy * M, nz = (size_t)t->nb * d.Hz * d.Wz * N;
    const bool zc = cfg.zero_copy != 0;
    HIP_OK(hipMemcpyAsync(s.d_sym_z, s.h_sym_z, nz, hipMemcpyHostToDevice, st));
    LAUNCH(LIC_HS0, s.d_sym_z, sc.h2, nullptr, st);
    LAUNCH(LIC_HS1, sc.h2, sc.h1, nullptr, st);
    if (kind == 2) {
        // psi, then the anchors' means and indices (the pass that needs z only)
        LAUNCH(LIC_HS2, sc.h1, s.d_zc, nullptr, st);
        HIP_OK(launch_cb_fill(s.d_zc, t->nb, d.Hy, d.Wy, 4 * M, 2 * M, 2 * M, 0, 0.0f, st));
        LAUNCH(LIC_EP0A, s.d_zc, sc.e1, nullptr, st);
        LAUNCH(LIC_EP1A, sc.e1, sc.e2, nullptr, st);
        LAUNCH2(LIC_EP2A, sc.e2, s.d_idx, nullptr, nullptr, s.d_mu, st);
        const size_t half = (size_t)d.Hy * d.Wy * M / 2;
        for (int b = 0; b < t->nb; ++b)
            HIP_OK(hipMemcpyAsync(s.h_idx + 2 * b * half, s.d_idx + 2 * b * half, half, hipMemcpyDeviceToHost, st));
        return LIC_OK;
    }
    LAUNCH(LIC_HS2, sc.h1, zc ? (void*)s.dm_idx : (void*)s.d_idx, nullptr, st);
    if (!zc) HIP_OK(hipMemcpyAsync(s.h_idx, s.d_idx, ny, hipMemcpyDeviceToHost, st));
    return LIC_OK;
}

// Context model, decoder: with the anchors decoded, their y_hat gives the
// context of the other positions, whose means and indices follow.
int Codec::gpu_ctx(Task* t, GpuStage& G)
{
    const FrameDims& d = t->route->dims;
    Slot& s = slots[t->slot];
    StageScratch& sc = G.scratch;
    hipStream_t st = G.stream;
    const size_t half = (size_t)d.Hy * d.Wy * M / 2;
    for (int b = 0; b < t->nb; ++b)
        HIP_OK(hipMemcpyAsync(s.d_sym_y + 2 * b * half, s.h_sym_y + 2 * b * half, half, hipMemcpyHostToDevice, st));
    HIP_OK(launch_cb_dequant(s.d_sym_y, s.d_mu, sc.yh, nullptr, t->nb, d.Hy, d.Wy, M, 0, st));
    LAUNCH(LIC_CX, sc.yh, s.d_zc, nullptr, st);
    LAUNCH(LIC_EP0N, s.d_zc, sc.e1, nullptr, st);
    LAUNCH(LIC_EP1N, sc.e1, sc.e2, nullptr, st);
    LAUNCH2(LIC_EP2N, sc.e2, s.d_idx, nullptr, nullptr, s.d_mu, st);
    for (int b = 0; b < t->nb; ++b)
        HIP_OK(hipMemcpyAsync(s.h_idx + (2 * b + 1) * half, s.d_idx + (2 * b + 1) * half, half,
                              hipMemcpyDeviceToHost, st));
    return LIC_OK;
}

int Codec::gpu_gs(Task* t, GpuStage& G)
{
    const FrameDims& d = t->route->dims;
    Slot& s = slots[t->slot];
    StageScratch& sc = G.scratch;
    hipStream_t st = G.stream;
    const size_t ny = (size_t)t->nb * d.Hy * d.Wy * M;
    const size_t fsz = (size_t)3 * d.H * d.W;
    const bool dev = t->route->is_device != 0;
    const bool direct = !t->staged && dev && t->call && frames_contiguous(t, fsz, true);
    const void* gs_in = s.d_sym_y;
    if (kind == 2) {
        // the second pass's symbols join the anchors' (already on the
        // device); y_hat = sym + mean in g_s's input type
        const size_t half = ny / t->nb / 2;
        for (int b = 0; b < t->nb; ++b)
            HIP_OK(hipMemcpyAsync(s.d_sym_y + (2 * b + 1) * half, s.h_sym_y + (2 * b + 1) * half, half,
                                  hipMemcpyHostToDevice, st));
        const bool f32 = layers[LIC_GS0].dt == DT_F32;
        for (int part = 0; part < 2; ++part)
            HIP_OK(launch_cb_dequant(s.d_sym_y, s.d_mu, f32 ? sc.yh : nullptr, f32 ? nullptr : (void*)sc.yh, t->nb,
                                     d.Hy, d.Wy, M, part, st));
        gs_in = sc.yh;
    } else {
        HIP_OK(hipMemcpyAsync(s.d_sym_y, s.h_sym_y, ny, hipMemcpyHostToDevice, st));
    }
    float* xo = direct ? t->xhats[0] : s.d_xhat;
    if (cfg.gs_mode != 0 && !distill) {
        t->fail(LIC_E_STATE, "no distilled synthesis transform loaded");
        return LIC_E_STATE;
    }
    if (cfg.gs_mode != 0 && !gs_fallback.load()) {
        // the distilled net reads the same symbols and writes the same
        // clamped, cropped image as the full g_s
        std::string e;
        const int r = distill->forward(s.d_sym_y, layers[LIC_GS0].d_mu_in, t->nb, d.Hy, d.Wy, nullptr, xo, d.H, d.W, st);
        if (r != LIC_OK) {
            t->fail(r, distill->err);
            return r;
        }
        if (t->judge) {
            const int rj = gs_judge(t, G, xo);
            if (rj != LIC_OK) return rj;
        }
    } else {
        LAUNCH(LIC_GS0, gs_in, sc.a, nullptr, st);
        LAUNCH(LIC_GS1, sc.a, sc.b, nullptr, st);
        LAUNCH(LIC_GS2, sc.b, sc.a, nullptr, st);
        LAUNCH(LIC_GS3, sc.a, xo, nullptr, st);
    }
    if (!direct && !t->staged)
        for (int b = 0; b < t->nb; ++b)
            HIP_OK(hipMemcpyAsync(t->xhats[b], s.d_xhat + b * fsz, fsz * sizeof(float),
                                  dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    return LIC_OK;
}

// Sampled check of the distilled g_s: frame 0 of the task also goes through
// the full g_s; when the two reconstructions are further apart than the
// threshold (PSNR of one against the other), the codec falls back to the
// full g_s for good and this task's frames are decoded again with it.
int Codec::gs_judge(Task* t, GpuStage& G, float* xo)
{
    const FrameDims& d = t->route->dims;
    Slot& s = slots[t->slot];
    StageScratch& sc = G.scratch;
    hipStream_t st = G.stream;
    const long fsz = 3L * d.H * d.W;
    std::string e;
    int r = LIC_OK;
    if ((r = launch_layer(LIC_GS0, 1, d, s.d_sym_y, sc.a, nullptr, st, &e)) != LIC_OK ||
        (r = launch_layer(LIC_GS1, 1, d, sc.a, sc.b, nullptr, st, &e)) != LIC_OK ||
        (r = launch_layer(LIC_GS2, 1, d, sc.b, sc.a, nullptr, st, &e)) != LIC_OK ||
        (r = launch_layer(LIC_GS3, 1, d, sc.a, d_judge_img, nullptr, st, &e)) != LIC_OK) {
        t->fail(r, e);
        return r;
    }
    const int chunk = 65536;
    if (launch_sqdiff(xo, d_judge_img, fsz, chunk, d_judge_part, d_judge_part + (fsz + chunk - 1) / chunk, st) !=
            hipSuccess ||
        hipMemcpyAsync(h_judge, d_judge_part + (fsz + chunk - 1) / chunk, sizeof(float), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        t->fail(LIC_E_HIP, "judge failed");
        return LIC_E_HIP;
    }
    const double mse = (double)h_judge[0] / (double)fsz;
    const double db = mse > 0.0 ? 10.0 * log10(1.0 / mse) : 99.0;
    gs_judge_last_db = db;
    gs_judged++;
    if (db < judge_db) {
        gs_fallback.store(true);
        if ((r = launch_layer(LIC_GS0, t->nb, d, s.d_sym_y, sc.a, nullptr, st, &e)) != LIC_OK ||
            (r = launch_layer(LIC_GS1, t->nb, d, sc.a, sc.b, nullptr, st, &e)) != LIC_OK ||
            (r = launch_layer(LIC_GS2, t->nb, d, sc.b, sc.a, nullptr, st, &e)) != LIC_OK ||
            (r = launch_layer(LIC_GS3, t->nb, d, sc.a, xo, nullptr, st, &e)) != LIC_OK) {
            t->fail(r, e);
            return r;
        }
    }
    return LIC_OK;
}

int Codec::load_distilled(const float* params, size_t n, float judge_psnr_db, int every)
{
    if (kind != 1 && kind != 0) { err = "no model"; return LIC_E_STATE; }
    if (every < 1) { err = "judge interval must be positive"; return LIC_E_ARG; }
    lic_distill_config dc;
    lic_distill_default_config(&dc);
    dc.M = M;
    dc.F = 64;
    dc.precision = cfg.precision == LIC_PREC_FP32 ? LIC_PREC_FP32 : LIC_PREC_BF16;   // e4m3 codecs: bf16 net
    dc.max_batch = cfg.max_batch;
    dc.max_hy = FrameDims(cfg.max_h, cfg.max_w).Hy;
    dc.max_wy = FrameDims(cfg.max_h, cfg.max_w).Wy;
    dc.train = 0;
    dc.hip_device = cfg.hip_device;
    std::unique_ptr<DistillNet> net(new DistillNet());
    const int rc = net->create(dc, params, n);
    if (rc != LIC_OK) {
        err = net->err;
        return rc;
    }
    if (!d_judge_img) {
        const long fsz = 3L * cfg.max_h * cfg.max_w;
        d_judge_img = (float*)dev_alloc(fsz * sizeof(float));
        d_judge_part = (float*)dev_alloc(((fsz + 65535) / 65536 + 1) * sizeof(float));
        h_judge = (float*)host_alloc(sizeof(float));
        if (!d_judge_img || !d_judge_part || !h_judge) { err = "allocation failed"; return LIC_E_NOMEM; }
    }
    // graphs of the g_s stage captured with the previous net point at its
    // buffers: drop them before that net is freed
    server_drop_graphs(ST_GPU_GS);
    distill = std::move(net);
    gs_gen++;
    judge_db = judge_psnr_db;
    judge_every = every;
    gs_fallback.store(false);
    gs_frames.store(0);
    gs_judged.store(0);
    return LIC_OK;
}

// ------------------------------------------------------------- CPU side
int Codec::cpu_parts(const Task* t, StageKind k) const
{
    switch (k) {
    case ST_CPU_ENC: return y_streams(kind, t->route->S) + (kind >= 1 ? 1 : 0);
    case ST_CPU_DEC_Z: return 1;
    case ST_CPU_DEC_Y: case ST_CPU_DEC_Y2: return t->route->S;
    default: return 0;
    }
}

void Codec::worker_loop()
{
    Job j;
    while (jobs.pop(&j)) {
        Task* t = j.task;
        const StageKind k = t->route->stages[t->stage];
        const int ppf = cpu_parts(t, k);
        const double t0 = now_s();
        if (t->status.load() == 0) cpu_job(t, j.part / ppf, j.part % ppf);
        cpu_busy_us += (long)((now_s() - t0) * 1e6);
        if (t->jobs_left.fetch_sub(1) == 1) {
            if (t->status.load() == 0) cpu_finalize(t, k);
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

// y stream si of a frame: its symbols' offset and count in the frame's y
// symbols (row = Wy M symbols per latent row).  Stream si is row slice si;
// for the context model, slice si % S of set si / S (anchors, then the rest)
// in the checkerboard-major layout, Wy M / 2 symbols per row of a set.
static inline void y_span(int kind, size_t row, int Hy, int S, int si, size_t* off, size_t* cnt)
{
    const int set = kind == 2 ? si / S : 0, sl = kind == 2 ? si % S : si;
    int r0, r1;
    slice_rows(Hy, S, sl, &r0, &r1);
    const size_t srow = kind == 2 ? row / 2 : row;
    *off = (size_t)set * Hy * srow + (size_t)r0 * srow;
    *cnt = (size_t)(r1 - r0) * srow;
}

// Offset of y stream si in a frame's rANS scratch: the z stream's region
// comes first, then one region per stream, each 2 bytes per symbol plus
// kStreamSlack.
static inline size_t y_region(int kind, size_t nz, size_t row, int Hy, int S, int si)
{
    size_t off, cnt;
    y_span(kind, row, Hy, S, si, &off, &cnt);
    return (kind >= 1 ? 2 * nz + kStreamSlack : 0) + 2 * off + kStreamSlack * (size_t)si;
}

int Codec::cpu_job(Task* t, int b, int part)
{
    const FrameDims& d = t->route->dims;
    Slot& s = slots[t->slot];
    const StageKind k = t->route->stages[t->stage];
    const int S = t->route->S;
    const size_t row = (size_t)d.Wy * M;
    const size_t ny = (size_t)d.Hy * row, nz = kind >= 1 ? (size_t)d.Hz * d.Wz * N : 0;
    int8_t* sym_y = s.h_sym_y + (size_t)b * ny;        // frame b of the task (current size)
    int8_t* sym_z = kind >= 1 ? s.h_sym_z + (size_t)b * nz : nullptr;
    const uint8_t* idx = kind >= 1 ? s.h_idx + (size_t)b * ny : nullptr;
    uint8_t* scratch = s.h_scratch + (size_t)b * s.scratch_per_frame;
    const bool gaussian = kind >= 1;                   // y coded with the scale-indexed tables
    if (k == ST_CPU_ENC) {
        if (kind >= 1 && part == 0) {
            long len = lanes ? rans_ileave_encode_channel(lanes, sym_z, (long)nz, N, fact, scratch, 2 * nz + kStreamSlack)
                             : rans_encode_channel(sym_z, (long)nz, N, fact, scratch, 2 * nz + kStreamSlack);
            if (len < 0) { t->fail(LIC_E_STATE, "rANS z overflow"); return LIC_E_STATE; }
            t->part_len[b][0] = (size_t)len;
            return LIC_OK;
        }
        const int si = part - (kind >= 1 ? 1 : 0);
        size_t off, cnt;
        y_span(kind, row, d.Hy, S, si, &off, &cnt);
        uint8_t* region = scratch + y_region(kind, nz, row, d.Hy, S, si);
        const size_t cap = 2 * cnt + kStreamSlack;
        long len;
        if (lanes)
            len = gaussian ? rans_ileave_encode(lanes, sym_y + off, idx + off, (long)cnt, gauss, region, cap)
                           : rans_ileave_encode_channel(lanes, sym_y + off, (long)cnt, M, fact, region, cap);
        else
            len = gaussian ? rans_encode(sym_y + off, idx + off, (long)cnt, gauss, region, cap)
                           : rans_encode_channel(sym_y + off, (long)cnt, M, fact, region, cap);
        if (len < 0) { t->fail(LIC_E_STATE, "rANS y overflow"); return LIC_E_STATE; }
        t->part_len[b][part] = (size_t)len;
        return LIC_OK;
    }
    if (k == ST_CPU_DEC_Z) {
        const int rc = lanes ? rans_ileave_decode_channel(lanes, t->zp[b], t->zlen[b], (long)nz, N, fact, sym_z)
                             : rans_decode_channel(t->zp[b], t->zlen[b], (long)nz, N, fact, sym_z);
        if (rc != 0) {
            t->fail(LIC_E_CORRUPT, "corrupt z stream");
            return LIC_E_CORRUPT;
        }
        return LIC_OK;
    }
    if (k == ST_CPU_DEC_Y || k == ST_CPU_DEC_Y2) {
        const int si = (k == ST_CPU_DEC_Y2 ? S : 0) + part;
        size_t off, cnt;
        y_span(kind, row, d.Hy, S, si, &off, &cnt);
        int rc;
        if (lanes)
            rc = gaussian ? rans_ileave_decode(lanes, t->yp[b][si], t->ylen[b][si], idx + off, (long)cnt, gauss,
                                               sym_y + off)
                          : rans_ileave_decode_channel(lanes, t->yp[b][si], t->ylen[b][si], (long)cnt, M, fact,
                                                       sym_y + off);
        else
            rc = gaussian ? rans_decode(t->yp[b][si], t->ylen[b][si], idx + off, (long)cnt, gauss, sym_y + off)
                          : rans_decode_channel(t->yp[b][si], t->ylen[b][si], (long)cnt, M, fact, sym_y + off);
        if (rc != 0) {
            t->fail(LIC_E_CORRUPT, "corrupt y stream");
            return LIC_E_CORRUPT;
        }
        return LIC_OK;
    }
    t->fail(LIC_E_STATE, "bad stage");
    return LIC_E_STATE;
}

// Assembles each frame's bitstream (header, z, y slices) in the slot.
int Codec::cpu_finalize(Task* t, StageKind k)
{
    if (k != ST_CPU_ENC) return LIC_OK;
    const FrameDims& d = t->route->dims;
    const int S = t->route->S;
    Slot& s = slots[t->slot];
    const size_t row = (size_t)d.Wy * M;
    const size_t nz = kind >= 1 ? (size_t)d.Hz * d.Wz * N : 0;
    const int ns = y_streams(kind, S);
    StreamHeader h;
    h.kind = kind;
    h.hs_exp = hs_exp;
    h.norm = norm;
    h.lanes = lanes;
    h.S = S;
    h.H = d.H;
    h.W = d.W;
    h.N = N;
    h.M = M;
    h.model_id = model_id;
    const int y0 = kind >= 1 ? 1 : 0;
    for (int b = 0; b < t->nb; ++b) {
        uint32_t ylen[2 * kMaxSlices];
        size_t total = header_size(kind, S) + (kind >= 1 ? t->part_len[b][0] : 0);
        for (int i = 0; i < ns; ++i) {
            ylen[i] = (uint32_t)t->part_len[b][y0 + i];
            total += ylen[i];
        }
        if (total > s.bits_per_frame) {
            t->fail(LIC_E_STATE, "bitstream exceeds slot");
            return LIC_E_STATE;
        }
        uint8_t* bits = s.h_bits + (size_t)b * s.bits_per_frame;
        const uint8_t* scratch = s.h_scratch + (size_t)b * s.scratch_per_frame;
        write_header(bits, h, kind >= 1 ? (uint32_t)t->part_len[b][0] : 0, ylen);
        uint8_t* p = bits + header_size(kind, S);
        if (kind >= 1) {
            memcpy(p, scratch, t->part_len[b][0]);
            t->zp[b] = p;
            t->zlen[b] = t->part_len[b][0];
            p += t->part_len[b][0];
        }
        for (int i = 0; i < ns; ++i) {
            const uint8_t* region = scratch + y_region(kind, nz, row, d.Hy, S, i);
            memcpy(p, region, ylen[i]);
            t->yp[b][i] = p;
            t->ylen[b][i] = ylen[i];
            p += ylen[i];
        }
        t->bits_len[b] = total;
    }
    return LIC_OK;
}

// ------------------------------------------------------------- one call
// The caller has filled cs.tasks (frames grouped into tasks); this admits
// them one slot at a time and waits for the in-order sink to drain.
int Codec::run_call(CallState& cs)
{
    cs.finished.assign(cs.tasks.size(), 0);
    const double t0 = now_s();
    for (size_t i = 0; i < cs.tasks.size(); ++i) {
        int slot;
        if (!free_slots.pop(&slot)) {
            // should not happen: the pool is only closed at destroy; drain what was admitted
            std::unique_lock<std::mutex> g(cs.m);
            cs.cv.wait(g, [&] { return cs.done == (int)i; });
            err = "codec stopped";
            return LIC_E_STATE;
        }
        Task* t = cs.tasks[i].get();
        t->route = &cs.route;
        t->call = &cs;
        t->index = (int)i;
        t->slot = slot;
        t->stage = -1;
        t->t_admit = now_s();
        advance(t);
    }
    {
        std::unique_lock<std::mutex> g(cs.m);
        cs.cv.wait(g, [&] { return cs.done == (int)cs.tasks.size(); });
    }
    last_wall_s = now_s() - t0;
    last_frames = cs.n;
    last_lat_ms.assign(cs.n, 0.0);
    for (auto& up : cs.tasks)
        for (int b = 0; b < up->nb; ++b) last_lat_ms[up->first + b] = (up->t_done - up->t_admit) * 1e3;
    if (cs.status != 0) {
        err = cs.err;
        return cs.status;
    }
    return LIC_OK;
}

}  // namespace lic
