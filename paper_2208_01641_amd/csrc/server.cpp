// Serving: continuous batching of many concurrent streams of mixed frame
// sizes over the same pipeline stages, pools and worker threads.
//
// Requests queue in per-(direction, frame size, slices, memory kind)
// buckets.  A batcher thread waits for a free pool slot, takes up to
// max_batch requests from the bucket whose oldest request has waited
// longest, and sends them through the stages as one task, so requests that
// arrive while others are on the GPU or the entropy workers are admitted as
// soon as a slot frees up.  Each GPU stage of a serving task can run as a
// captured HIP graph keyed by (stage, frame size, batch, slot, synthesis
// variant): every pointer inside it is a slot or stage buffer, and the
// request buffers are copied in and out around the graph.  Streams are admitted against the
// device-memory budget.
#include <string.h>

#include <limits>
#include <map>
#include <tuple>

#include "codec.h"

namespace lic {

struct BucketKey {
    int dir, H, W, S, is_device;
    bool operator<(const BucketKey& o) const
    {
        return std::tie(dir, H, W, S, is_device) < std::tie(o.dir, o.H, o.W, o.S, o.is_device);
    }
};

struct Server {
    std::mutex m;
    std::condition_variable cv;
    std::map<BucketKey, std::deque<Request*>> buckets;
    std::map<BucketKey, std::unique_ptr<Route>> routes;
    std::vector<std::unique_ptr<Task>> tasks;          // one per pool slot
    std::vector<ServeStream> streams;
    size_t reserved = 0;
    uint64_t next_ticket = 1;
    long queued = 0;                                   // submitted, not yet admitted
    long pending = 0;                                  // submitted, not yet completed
    bool stop = false;
    std::thread thread;
    std::mutex done_m;
    std::condition_variable done_cv;
    std::deque<lic_result> done;
    std::mutex graph_m;
    // (stage, H, W, batch, slot, synthesis variant) -> executable graph
    std::map<std::tuple<int, int, int, int, int, int>, hipGraphExec_t> graphs;
};

// Device footprint of one in-flight frame of a stream: input and
// reconstruction images plus the two largest activations.
static size_t stream_cost(int N, int H, int W)
{
    const FrameDims d(H, W);
    return sizeof(float) * ((size_t)6 * H * W + (size_t)N * (d.Hp / 2) * (d.Wp / 2) + (size_t)N * (d.Hp / 4) * (d.Wp / 4));
}

int Codec::open_stream(int H, int W, int* id)
{
    if (H < 1 || W < 1 || H > cfg.max_h || W > cfg.max_w) { err = "stream larger than max_h x max_w"; return LIC_E_BUDGET; }
    if (!server) {
        server.reset(new Server());
        server->tasks.resize(slots.size());
        for (auto& t : server->tasks) t.reset(new Task());
        server->thread = std::thread(&Codec::server_loop, this);
    }
    Server& S = *server;
    std::lock_guard<std::mutex> g(S.m);
    const size_t cost = stream_cost(N, H, W);
    if (cfg.hbm_budget_bytes && dev_bytes + S.reserved + cost > cfg.hbm_budget_bytes) {
        err = "stream does not fit in the device memory budget";
        return LIC_E_BUDGET;
    }
    S.reserved += cost;
    ServeStream st;
    st.H = H;
    st.W = W;
    st.cost = cost;
    st.open = true;
    S.streams.push_back(st);
    *id = (int)S.streams.size() - 1;
    return LIC_OK;
}

int Codec::close_stream(int id)
{
    if (!server) { err = "no such stream"; return LIC_E_ARG; }
    Server& S = *server;
    std::lock_guard<std::mutex> g(S.m);
    if (id < 0 || id >= (int)S.streams.size() || !S.streams[id].open) { err = "no such stream"; return LIC_E_ARG; }
    S.streams[id].open = false;
    S.reserved -= S.streams[id].cost;
    return LIC_OK;
}

int Codec::server_submit(Request* r, uint64_t* ticket)
{
    if (!server) { err = "no open stream"; delete r; return LIC_E_STATE; }
    Server& S = *server;
    std::lock_guard<std::mutex> g(S.m);
    if (S.stop) { err = "codec is shutting down"; delete r; return LIC_E_STATE; }
    if (r->stream_id < 0 || r->stream_id >= (int)S.streams.size() || !S.streams[r->stream_id].open) {
        err = "no such stream";
        delete r;
        return LIC_E_ARG;
    }
    const ServeStream& st = S.streams[r->stream_id];
    const int Sl = r->dir == 0 ? this->S : r->hdr.S;
    if (r->dir == 1 && (r->hdr.H != st.H || r->hdr.W != st.W)) {
        err = "bitstream frame size differs from the stream's";
        delete r;
        return LIC_E_ARG;
    }
    BucketKey key{r->dir, st.H, st.W, Sl, r->is_device};
    auto& route = S.routes[key];
    if (!route) {
        route.reset(new Route());
        route->dims = FrameDims(st.H, st.W);
        route->S = Sl;
        route->is_device = r->is_device;
        if (r->dir == 0) route->stages = {ST_GPU_ENC, ST_CPU_ENC};
        else if (kind == 1) route->stages = {ST_CPU_DEC_Z, ST_GPU_HS, ST_CPU_DEC_Y, ST_GPU_GS};
        else route->stages = {ST_CPU_DEC_Y, ST_GPU_GS};
    }
    r->ticket = S.next_ticket++;
    *ticket = r->ticket;
    r->t_submit = now_s();
    S.buckets[key].push_back(r);
    S.queued++;
    S.pending++;
    S.cv.notify_one();
    return LIC_OK;
}

void Codec::server_loop()
{
    Server& S = *server;
    for (;;) {
        {
            std::unique_lock<std::mutex> g(S.m);
            S.cv.wait(g, [&] { return S.stop || S.queued > 0; });
            if (S.queued == 0) return;                   // stopping and drained
        }
        int slot;
        if (!free_slots.pop(&slot)) return;
        Task* t = S.tasks[slot].get();
        {
            std::lock_guard<std::mutex> g(S.m);
            auto best = S.buckets.end();
            double oldest = std::numeric_limits<double>::infinity();
            for (auto it = S.buckets.begin(); it != S.buckets.end(); ++it)
                if (!it->second.empty() && it->second.front()->t_submit < oldest) {
                    oldest = it->second.front()->t_submit;
                    best = it;
                }
            if (best == S.buckets.end()) {
                free_slots.push(slot);
                continue;
            }
            std::deque<Request*>& q = best->second;
            const int nb = std::min<int>(cfg.max_batch, (int)q.size());
            t->route = S.routes[best->first].get();
            t->call = nullptr;
            t->slot = slot;
            t->stage = -1;
            t->nb = nb;
            t->first = 0;
            t->staged = false;
            t->status.store(0);
            t->err.clear();
            for (int b = 0; b < nb; ++b) {
                Request* r = q.front();
                q.pop_front();
                t->req[b] = r;
                t->xs[b] = r->x;
                t->xhats[b] = r->xhat;
                t->zp[b] = r->zp;
                t->zlen[b] = r->zlen;
                for (int s = 0; s < r->hdr.S && s < kMaxSlices; ++s) {
                    t->yp[b][s] = r->yp[s];
                    t->ylen[b][s] = r->ylen[s];
                }
            }
            S.queued -= nb;
            t->t_admit = now_s();
        }
        advance(t);
    }
}

void Codec::server_finish(Task* t)
{
    Server& S = *server;
    // the batcher reuses this task as soon as its slot is free again, so
    // everything needed afterwards is read now and the slot is freed last
    const int nb = t->nb, slot = t->slot;
    const Slot& sl = slots[slot];
    std::vector<lic_result> res(nb);
    for (int b = 0; b < nb; ++b) {
        Request* r = t->req[b];
        lic_result& o = res[b];
        memset(&o, 0, sizeof(o));
        o.ticket = r->ticket;
        o.status = t->status.load();
        o.stream_id = r->stream_id;
        o.direction = r->dir;
        o.H = t->route->dims.H;
        o.W = t->route->dims.W;
        if (o.status == 0 && r->dir == 0) {
            o.bytes = t->bits_len[b];
            if (t->bits_len[b] <= r->cap) memcpy(r->out, sl.h_bits + (size_t)b * sl.bits_per_frame, t->bits_len[b]);
            else o.status = LIC_E_SMALLBUF;
        }
        o.latency_ms = (t->t_done - r->t_submit) * 1e3;
        delete r;
        t->req[b] = nullptr;
    }
    {
        std::lock_guard<std::mutex> g(S.done_m);
        for (auto& o : res) S.done.push_back(o);
    }
    {
        std::lock_guard<std::mutex> g(S.m);
        S.pending -= nb;
    }
    free_slots.push(slot);
    S.done_cv.notify_all();
}

int Codec::server_poll(lic_result* out, int max, int timeout_us)
{
    if (!server) return 0;
    Server& S = *server;
    std::unique_lock<std::mutex> g(S.done_m);
    if (S.done.empty() && timeout_us > 0)
        S.done_cv.wait_for(g, std::chrono::microseconds(timeout_us), [&] { return !S.done.empty(); });
    int n = 0;
    while (n < max && !S.done.empty()) {
        out[n++] = S.done.front();
        S.done.pop_front();
    }
    return n;
}

// Drains every queued and in-flight request, then stops the batcher.
void Codec::server_stop()
{
    if (!server) return;
    Server& S = *server;
    {
        std::lock_guard<std::mutex> g(S.m);
        S.stop = true;
    }
    S.cv.notify_all();
    {
        std::unique_lock<std::mutex> g(S.done_m);
        S.done_cv.wait(g, [&] {
            std::lock_guard<std::mutex> g2(S.m);
            return S.pending == 0;
        });
    }
    if (S.thread.joinable()) S.thread.join();
    for (auto& kv : S.graphs) (void)hipGraphExecDestroy(kv.second);
    S.graphs.clear();
}

// Defined here, where the serving state is a complete type.
Codec::Codec() = default;

Codec::~Codec()
{
    server_stop();
    stop();
    if (hipSetDevice(cfg.hip_device) == hipSuccess) (void)hipDeviceSynchronize();
    for (int g = 0; g < 3; ++g)
        if (gpu[g].stream) (void)hipStreamDestroy(gpu[g].stream);
    if (layer_stream) (void)hipStreamDestroy(layer_stream);
    for (void* p : dev_allocs) (void)hipFree(p);
    for (void* p : host_allocs) (void)hipHostFree(p);
}

// Destroys the cached graphs of one stage kind (the g_s stage when another
// distilled net is loaded: its graphs point at the old net's buffers).
void Codec::server_drop_graphs(int stage_kind)
{
    if (!server) return;
    Server& S = *server;
    std::lock_guard<std::mutex> g(S.graph_m);
    for (auto it = S.graphs.begin(); it != S.graphs.end();) {
        if (std::get<0>(it->first) == stage_kind) {
            (void)hipGraphExecDestroy(it->second);
            it = S.graphs.erase(it);
        } else {
            ++it;
        }
    }
}

// Runs one GPU stage of a serving task as a captured HIP graph.  The body
// only touches slot and stage buffers (the request buffers are copied in and
// out by the caller), so a graph is valid for every task with the same
// stage, frame size, batch and slot - and, for the g_s stage, the same
// synthesis transform: the full g_s (variant 0) or the distilled net loaded
// as the gs_gen-th one (variant gs_gen), which is part of the key so that a
// fallback to the full g_s never replays a graph of the distilled net.  The
// variant is read on the g_s stage's own thread, the only one that sets the
// fallback.
int Codec::gpu_stage_graph(Task* t, GpuStage& G, int (Codec::*body)(Task*, GpuStage&))
{
    Server& S = *server;
    const int variant = G.kind == ST_GPU_GS && cfg.gs_mode != 0 && distill && !gs_fallback.load() ? gs_gen : 0;
    const auto key = std::make_tuple((int)G.kind, t->route->dims.H, t->route->dims.W, t->nb, t->slot, variant);
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> g(S.graph_m);
        auto it = S.graphs.find(key);
        if (it != S.graphs.end()) exec = it->second;
    }
    if (!exec) {
        if (hipStreamBeginCapture(G.stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            t->fail(LIC_E_HIP, "hipStreamBeginCapture failed");
            return LIC_E_HIP;
        }
        G.capturing = true;
        const int rc = (this->*body)(t, G);
        G.capturing = false;
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(G.stream, &graph);
        if (rc != LIC_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            t->fail(rc != LIC_OK ? rc : LIC_E_HIP, "graph capture failed");
            return rc != LIC_OK ? rc : LIC_E_HIP;
        }
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            t->fail(LIC_E_HIP, "hipGraphInstantiate failed");
            return LIC_E_HIP;
        }
        std::lock_guard<std::mutex> g(S.graph_m);
        S.graphs[key] = exec;
    }
    if (hipGraphLaunch(exec, G.stream) != hipSuccess) {
        t->fail(LIC_E_HIP, "hipGraphLaunch failed");
        return LIC_E_HIP;
    }
    return LIC_OK;
}

}  // namespace lic
