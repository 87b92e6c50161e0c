// Internal codec object: model (packed weights, tables), device pools and
// the pipeline runtime behind the C ABI.
#pragma once
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lic.h"
#include "conv_args.h"
#include "entropy.h"
#include "distill.h"
#include "kernels.h"

namespace lic {

// ------------------------------------------------------------------ model
struct LayerGPU {
    bool present = false;
    int ld = 0, ep = 0, dt = 0;
    int cin = 0, co = 0, cop = 0;
    int k = 5;
    bool deconv = false;
    bool rows = false;                 // 4 phases as GEMM rows (transposed conv to 3 channels)
    int nphase = 1;
    bool halo1 = false;                // every tap within one pixel of a stride-1 grid
    bool out_e4m3 = false;             // bf16 GEMM storing e4m3 activations (e4m3 form, image layer)
    bool out_bf16 = false;             // e4m3 GEMM storing bf16 activations (e4m3 form, GS2)
    float out_q = 8.0f;                // e4m3 activations out hold out_q x the value
    float in_scale = 1.0f;             // e4m3 form: 1 / out_q of the layer whose e4m3 output this reads
    std::vector<float> wsc;            // e4m3 form: per packed row, the weight scale
    std::vector<PhaseDesc> host_ph;
    PhaseDesc* d_ph = nullptr;
    uint8_t* d_w = nullptr;            // packed weights (float, bf16 or e4m3)
    uint16_t* d_wx = nullptr;          // FP32 GDN layers: the same as three bf16 parts (ConvArgs::wx)
    float* d_bias = nullptr;
    float* d_rscale = nullptr;         // e4m3 form: per packed row, weight scale x input scale
    uint16_t* d_gsplit = nullptr;      // gamma as bf16 parts (layout in ConvArgs::gsplit)
    float* d_beta = nullptr;
    const float* d_qmu = nullptr;      // EP_QUANT offsets
    const float* d_mu_in = nullptr;    // LD_I8 offsets
};

// e4m3 activations between layers hold q x the value: kActQ (|value| <= 56
// fits) until codec_calibrate sets each layer's q from calibration frames
constexpr float kActQ = 8.0f;
uint8_t e4m3_rne(float f);
std::vector<uint16_t> gdn_gamma_split(const std::vector<double>& gamma, int co);

struct Geo {
    int Hin, Win, Hg, Wg, s_in, Hout, Wout, s_out;
};

// Tensor sizes for an H x W frame (padded to multiples of 64).
struct FrameDims {
    int H, W, Hp, Wp, Hy, Wy, Hz, Wz;
    explicit FrameDims(int h = 0, int w = 0)
        : H(h), W(w), Hp(64 * ((h + 63) / 64)), Wp(64 * ((w + 63) / 64)),
          Hy(Hp / 16), Wy(Wp / 16), Hz(Hp / 64), Wz(Wp / 64) {}
};

// ------------------------------------------------------------- pipeline
struct Codec;

constexpr int kMaxSlices = 64;
constexpr int kMaxBatch = 8;

struct Route;
struct CallState;
struct Request;

// A task: up to max_batch consecutive frames of one call that travel
// together through the stage queues (the state machine of the pipeline).
// GPU stages launch every layer once for the whole batch; CPU stages split
// it into per-frame, per-stream jobs.
struct Task {
    const Route* route = nullptr;      // frame size, slices, stage list
    CallState* call = nullptr;         // synchronous call (in-order sink), or
    Request* req[kMaxBatch] = {};      // serving requests (completion queue)
    int index = 0;                     // position of the task in the call
    int first = 0;                     // index of the first frame in the call
    int nb = 1;                        // frames in this task
    int slot = -1;
    int stage = -1;                    // index into the route's stage list
    const float* xs[kMaxBatch] = {};   // input frame of each batch entry
    float* xhats[kMaxBatch] = {};      // output frame of each batch entry
    bool staged = false;               // request buffers copied in / out by the caller
    bool judge = false;                // g_s stage: also run the full g_s on frame 0 and compare
    std::atomic<int> jobs_left{0};
    std::atomic<int> status{0};
    std::mutex err_m;
    std::string err;
    double t_admit = 0.0, t_done = 0.0;
    size_t bits_len[kMaxBatch] = {};
    // encoder: stream lengths (z = part 0 for the hyperpriors, then the y
    // streams: S slices, 2 S for the context model)
    size_t part_len[kMaxBatch][2 * kMaxSlices + 1] = {};
    // decoder: payload spans of each parsed bitstream
    const uint8_t* zp[kMaxBatch] = {};
    size_t zlen[kMaxBatch] = {};
    const uint8_t* yp[kMaxBatch][2 * kMaxSlices] = {};
    size_t ylen[kMaxBatch][2 * kMaxSlices] = {};

    void fail(int code, const std::string& msg)
    {
        std::lock_guard<std::mutex> g(err_m);
        if (status.load() == 0) {
            err = msg;
            status.store(code);
        }
    }
};

// Pooled buffers of one task (max_batch frames).  Host buffers are pinned
// and mapped into the device address space, so the epilogues can store
// symbols and indices straight into them (zero-copy) or a DMA copy can.
struct Slot {
    int8_t* h_sym_y = nullptr;   int8_t* d_sym_y = nullptr;    // [B][Hy][Wy][M] (context model:
    int8_t* h_sym_z = nullptr;   int8_t* d_sym_z = nullptr;    // [B][Hz][Wz][N]  checkerboard-major
    uint8_t* h_idx = nullptr;    uint8_t* d_idx = nullptr;     // [B][Hy][Wy][M]  y symbols and indices)
    float* d_zc = nullptr;       // context model: [psi; ctx], [B][Hy][Wy][4M]
    float* d_mu = nullptr;       // context model (decoder): the means, checkerboard-major
    int8_t* dm_sym_y = nullptr;  uint8_t* dm_idx = nullptr;    // device views of the pinned buffers
    uint8_t* h_scratch = nullptr; size_t scratch_per_frame = 0; // per-stream rANS output regions
    uint8_t* h_bits = nullptr;    size_t bits_per_frame = 0;    // assembled bitstreams
    float* d_x = nullptr;                                       // input staging (host input)
    float* d_xhat = nullptr;                                    // output staging (host output)
};

// Device scratch of one GPU stage (reused frame after frame in stream order).
struct StageScratch {
    float* a = nullptr;   // N x Hp/2 x Wp/2
    float* b = nullptr;   // N x Hp/4 x Wp/4
    float* y = nullptr;   // M x Hy x Wy
    float* h1 = nullptr;  // N x Hy x Wy
    float* h2 = nullptr;  // N x Hy/2 x Wy/2 (and h_s middle: N x Hy/2 x Wy/2)
    float* e1 = nullptr;  // context model: entropy-parameter hidden layers (E1, E2 x Hy x Wy)
    float* e2 = nullptr;
    float* yh = nullptr;  // context model: y_hat M x Hy x Wy (float32, or bf16 for g_s)
};

// ST_GPU_CTX and ST_CPU_DEC_Y2: the context model's second pass (the context
// of the decoded anchors and the other positions' parameters, then their
// symbols); ST_CPU_DEC_Y then decodes the anchors only
enum StageKind { ST_GPU_ENC, ST_CPU_ENC, ST_CPU_DEC_Z, ST_GPU_HS, ST_CPU_DEC_Y, ST_GPU_GS, ST_GPU_CTX, ST_CPU_DEC_Y2 };

// What every task of a call (or of a serving bucket) shares.
struct Route {
    FrameDims dims;
    int S = 1;                     // y slices of every frame
    int is_device = 0;             // caller buffers are device memory
    std::vector<StageKind> stages;
};

struct Job {
    Task* task;
    int part;
};

template <class T>
class BlockingQueue {
public:
    void push(T v)
    {
        {
            std::lock_guard<std::mutex> g(m_);
            q_.push_back(std::move(v));
        }
        cv_.notify_one();
    }
    // false once closed and drained
    bool pop(T* out)
    {
        std::unique_lock<std::mutex> g(m_);
        cv_.wait(g, [&] { return closed_ || !q_.empty(); });
        if (q_.empty()) return false;
        *out = std::move(q_.front());
        q_.pop_front();
        return true;
    }
    bool try_pop(T* out)
    {
        std::lock_guard<std::mutex> g(m_);
        if (q_.empty()) return false;
        *out = std::move(q_.front());
        q_.pop_front();
        return true;
    }
    bool empty()
    {
        std::lock_guard<std::mutex> g(m_);
        return q_.empty();
    }
    void close()
    {
        {
            std::lock_guard<std::mutex> g(m_);
            closed_ = true;
        }
        cv_.notify_all();
    }

private:
    std::mutex m_;
    std::condition_variable cv_;
    std::deque<T> q_;
    bool closed_ = false;
};

struct CallState {
    int n = 0;                     // frames
    Route route;
    std::vector<std::unique_ptr<Task>> tasks;
    // in-order sink
    std::mutex m;
    std::condition_variable cv;
    int next_sink = 0;             // next task to deliver
    int done = 0;                  // delivered tasks
    std::vector<char> finished;
    uint8_t* out = nullptr;        // encoded output (packed back to back)
    size_t cap = 0;
    size_t* lens = nullptr;
    size_t offset = 0;
    bool overflow = false;
    int status = 0;
    std::string err;
};

struct GpuStage {
    StageKind kind;
    hipStream_t stream = nullptr;
    StageScratch scratch;
    BlockingQueue<Task*> queue;
    std::thread thread;
    double busy_s = 0.0;
    bool capturing = false;            // recording a HIP graph (no timing events)
    // events bracketing timed layers: [in-flight task][layer][start/end]
    int cur = 0;
    hipEvent_t lev[2][LIC_NUM_LAYERS][2] = {};
    bool lrec[2][LIC_NUM_LAYERS] = {};
};

// ---------------------------------------------------------------- serving
// One asynchronous request (a frame to encode or a bitstream to decode).
struct Request {
    uint64_t ticket = 0;
    int stream_id = 0;
    int dir = 0;                       // 0 encode, 1 decode
    int is_device = 0;
    const float* x = nullptr;          // encode input
    uint8_t* out = nullptr;            // encode output buffer
    size_t cap = 0;
    float* xhat = nullptr;             // decode output
    // parsed decode input
    StreamHeader hdr;
    const uint8_t* zp = nullptr;
    size_t zlen = 0;
    const uint8_t* yp[kMaxSlices] = {};
    size_t ylen[kMaxSlices] = {};
    double t_submit = 0.0;
};

struct ServeStream {
    int H = 0, W = 0;
    size_t cost = 0;                   // device bytes reserved against the budget
    bool open = false;
};

struct Server;

struct Codec {
    codec_config cfg{};
    std::string err;
    int kind = 1, N = 128, M = 192, hs_exp = 1, S = 8;
    int norm = 0;                      // 0 GDN / IGDN, 1 1DN (container flag bit 1)
    int lanes = 0;                     // rANS: 0 byte-wise one state, K interleaved states
    uint32_t model_id = 0;
    std::vector<float> medians;        // channel offsets of the factorized tables
    TableSet fact;                     // [C] factorized tables
    TableSet gauss;                    // [64] Gaussian tables
    std::vector<float> thr;            // 63 scale-index thresholds
    LayerGPU layers[LIC_NUM_LAYERS];
    float* d_medians = nullptr;
    float* d_zero = nullptr;
    float* d_thr = nullptr;
    std::vector<void*> dev_allocs, host_allocs;
    size_t dev_bytes = 0;
    std::atomic<long> alloc_events{0};

    // runtime
    hipStream_t layer_stream = nullptr;      // codec_run_layer
    GpuStage gpu[3];                         // encoder GPU, decoder GPU1 (h_s and the context
                                             // model's second pass), decoder GPU2 (g_s)
    std::vector<Slot> slots;
    BlockingQueue<int> free_slots;
    BlockingQueue<Job> jobs;
    std::vector<std::thread> workers;
    std::vector<double> last_lat_ms;
    double last_wall_s = 0.0;
    int last_frames = 0;
    std::atomic<long> cpu_busy_us{0};
    bool started = false;
    // kernel timing of selected layers inside the pipeline (HIP events)
    std::atomic<uint32_t> timed_mask{0};
    std::mutex lt_m;
    double layer_ms[LIC_NUM_LAYERS] = {};
    long layer_launches[LIC_NUM_LAYERS] = {};

    // serving (continuous batching over per-shape buckets)
    std::unique_ptr<Server> server;

    // distilled synthesis transform (gs_mode 1, 2) and its sampled judge
    std::unique_ptr<DistillNet> distill;
    float judge_db = 0.0f;                   // fall back when PSNR(full, distilled) < judge_db
    int judge_every = 30;                    // frames between judged frames
    std::atomic<bool> gs_fallback{false};
    int gs_gen = 0;                          // distilled nets loaded so far (graph cache key)
    std::atomic<long> gs_frames{0}, gs_judged{0};
    double gs_judge_last_db = 0.0;
    float* d_judge_img = nullptr;            // 3 x max_h x max_w
    float* d_judge_part = nullptr;
    float* h_judge = nullptr;                // pinned: the squared error of the last judge
    int load_distilled(const float* params, size_t n, float judge_psnr_db, int every);
    int gs_judge(Task* t, GpuStage& G, float* xo);
    int server_submit(Request* r, uint64_t* ticket);
    int server_poll(lic_result* out, int max, int timeout_us);
    void server_finish(Task* t);
    void server_stop();
    void server_loop();
    int open_stream(int H, int W, int* id);
    int close_stream(int id);
    int gpu_stage_graph(Task* t, GpuStage& G, int (Codec::*body)(Task*, GpuStage&));
    void server_drop_graphs(int stage_kind);

    Codec();
    ~Codec();
    // model
    int load(const void* blob, size_t len);
    int build_layers(const std::map<std::string, std::pair<std::vector<int>, std::vector<double>>>& P);
    Geo geo(int layer, const FrameDims& d) const;
    // Bytes of a layer's input, output and aux tensors for n frames of d
    // (codec_run_layer's buffers; 0 where the layer takes none).
    void layer_bytes(int layer, int n, const FrameDims& d, size_t* in, size_t* out, size_t* aux) const;
    // in2 / out2: the last entropy-parameter layer of the context model
    // (ConvArgs::ysrc, ConvArgs::yq)
    int launch_layer(int layer, int n, const FrameDims& d, const void* in, void* out, void* aux,
                     hipStream_t s, std::string* errp, KernelKey* chosen = nullptr, const void* in2 = nullptr,
                     void* out2 = nullptr);
    // e4m3 form: per-row scales of a layer's epilogue (weight scale x input scale)
    int upload_rscale(LayerGPU& L);
    // e4m3 form: activation scales from calibration frames (device, n x 3 x H x W)
    int calibrate_fp8(const float* x, int n, int H, int W);
    unsigned long long* d_sat = nullptr;     // e4m3 stores clamped at +-448 (counter)
    // pools and threads
    int start();
    void stop();
    // pipeline
    int run_call(CallState& cs);
    void gpu_loop(int g);
    void worker_loop();
    void advance(Task* t);
    void finish_task(Task* t);
    int gpu_encode(Task* t, GpuStage& g);
    int gpu_hs(Task* t, GpuStage& g);
    int gpu_ctx(Task* t, GpuStage& g);
    int gpu_gs(Task* t, GpuStage& g);
    int cpu_job(Task* t, int frame, int part);
    int cpu_parts(const Task* t, StageKind k) const;   // jobs per frame
    int cpu_finalize(Task* t, StageKind k);
    // allocation helpers (create time only)
    void* dev_alloc(size_t bytes);
    void* host_alloc(size_t bytes);
};

double now_s();
// Host-only: entropy tables a codec would build from a blob (no GPU needed).
long blob_tables(const void* blob, size_t len, int which, uint32_t* freq, size_t cap, float* mu, size_t mu_cap);

}  // namespace lic
