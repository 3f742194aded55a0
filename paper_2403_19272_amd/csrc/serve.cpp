// Batched stepping and a continuous-batching step server.
//
// cloth_step_batch: several scenes step concurrently.  The caller's stream
// forks to a pool of streams (default priority), each scene's recorded step
// graph is launched on its own stream, and the caller's stream joins them, so
// the small kernels of uneven scenes overlap on the device.
//
// cloth_server_*: a host thread takes step requests as they arrive, keeps at
// most `slots` steps in flight (one stream per slot), never runs two steps of
// one scene at once (step n+1 needs step n's state), and starts queued
// requests as soon as a slot and their scene are free: continuous batching
// at the granularity of whole steps.  Scenes are admitted against an HBM
// budget by their footprint.  Per request it records the time from
// submission to completion (host clock) and the device time of the step
// (HIP events around its graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "contact.hpp"
#include "scene.hpp"

namespace cloth {
cloth_status prepare_step_graph(cloth_scene_s* sc, const float g[3]);   // api.cpp
cloth_status record_step_graph(cloth_scene_s* sc, const float g[3], hipGraph_t* out);   // api.cpp
cloth_status scene_stats(cloth_scene_s* sc, hipStream_t st, cloth_step_stats* out);  // api.cpp
}  // namespace cloth

using namespace cloth;

namespace {

#define HC(expr)                                                                                        \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return set_error(CLOTH_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct StreamPool {
    std::mutex mu;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;   // one join event per stream
    hipEvent_t fork = nullptr;
};

StreamPool& pool() {
    static StreamPool p;
    return p;
}

cloth_status ensure_pool(size_t n) {
    StreamPool& p = pool();
    if (!p.fork) HC(hipEventCreateWithFlags(&p.fork, hipEventDisableTiming));
    while (p.streams.size() < n) {
        hipStream_t s;
        HC(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        hipEvent_t e;
        HC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        p.streams.push_back(s);
        p.events.push_back(e);
    }
    return CLOTH_OK;
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

cloth_status cloth_step_batch(cloth_scene* scenes, int32_t n, const float gravity[3], void* stream,
                              cloth_step_stats* stats) {
    if (!scenes || n < 0 || !gravity) return set_error(CLOTH_E_INVALID, "null argument");
    if (n == 0) return CLOTH_OK;
    for (int i = 0; i < n; ++i) {
        if (!scenes[i] || !scenes[i]->s.basis_set) return set_error(CLOTH_E_INVALID, "scene without basis");
        for (int j = 0; j < i; ++j)
            if (scenes[j] == scenes[i]) return set_error(CLOTH_E_INVALID, "scene listed twice");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamPool& p = pool();
    std::lock_guard<std::mutex> lock(p.mu);
    const size_t width = std::min<size_t>((size_t)n, 16);
    cloth_status rc = ensure_pool(width);
    if (rc != CLOTH_OK) return rc;
    for (int i = 0; i < n; ++i) {
        rc = prepare_step_graph(scenes[i], gravity);
        if (rc != CLOTH_OK) return rc;
    }
    HC(hipEventRecord(p.fork, st));
    for (size_t k = 0; k < width; ++k) HC(hipStreamWaitEvent(p.streams[k], p.fork, 0));
    for (int i = 0; i < n; ++i) HC(hipGraphLaunch(scenes[i]->s.graph_exec, p.streams[i % width]));
    for (size_t k = 0; k < width; ++k) {
        HC(hipEventRecord(p.events[k], p.streams[k]));
        HC(hipStreamWaitEvent(st, p.events[k], 0));
    }
    if (stats)
        for (int i = 0; i < n; ++i) {
            rc = scene_stats(scenes[i], st, &stats[i]);
            if (rc != CLOTH_OK) return rc;
        }
    return CLOTH_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batch graph
//
// One graph for many scenes: each scene's recorded step is a child graph of
// one parent graph, with no edges between them, so one hipGraphLaunch steps
// every scene and the device runs their kernels side by side.

struct cloth_batch_s {
    std::vector<cloth_scene> scenes;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

cloth_status cloth_batch_create(cloth_scene* scenes, int32_t n, const float gravity[3], cloth_batch* out) {
    if (!scenes || n <= 0 || !gravity || !out) return set_error(CLOTH_E_INVALID, "null argument");
    for (int i = 0; i < n; ++i) {
        if (!scenes[i] || !scenes[i]->s.basis_set) return set_error(CLOTH_E_INVALID, "scene without basis");
        for (int j = 0; j < i; ++j)
            if (scenes[j] == scenes[i]) return set_error(CLOTH_E_INVALID, "scene listed twice");
    }
    auto b = std::make_unique<cloth_batch_s>();
    b->scenes.assign(scenes, scenes + n);
    HC(hipGraphCreate(&b->graph, 0));
    for (int i = 0; i < n; ++i) {
        hipGraph_t child = nullptr;
        cloth_status rc = record_step_graph(scenes[i], gravity, &child);
        if (rc != CLOTH_OK) {
            (void)hipGraphDestroy(b->graph);
            return rc;
        }
        hipGraphNode_t node;
        hipError_t e = hipGraphAddChildGraphNode(&node, b->graph, nullptr, 0, child);
        (void)hipGraphDestroy(child);   // the node holds its own copy
        if (e != hipSuccess) {
            (void)hipGraphDestroy(b->graph);
            return set_error(CLOTH_E_DEVICE, std::string("hipGraphAddChildGraphNode: ") + hipGetErrorString(e));
        }
    }
    hipError_t e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(b->graph);
        return set_error(CLOTH_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    *out = b.release();
    return CLOTH_OK;
}

cloth_status cloth_batch_step(cloth_batch b, int32_t steps, void* stream) {
    if (!b || steps < 0) return set_error(CLOTH_E_INVALID, "invalid argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int i = 0; i < steps; ++i) HC(hipGraphLaunch(b->exec, st));
    return CLOTH_OK;
}

cloth_status cloth_batch_destroy(cloth_batch b) {
    if (!b) return CLOTH_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
    return CLOTH_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ server

struct cloth_server_s {
    struct Req {
        int64_t ticket;
        cloth_scene scene;
        float g[3];
        double t_submit;
    };
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t start = nullptr, end = nullptr;
        int* status = nullptr;   // pinned host word: the step's status bits, copied after its graph
        bool busy = false;
        Req req{};
    };
    struct Done {
        bool done = false;
        cloth_status status = CLOTH_OK;
        double latency_ms = 0, service_ms = 0;
    };

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req> queue;
    std::map<cloth_scene, int> queued;        // requests in `queue` per scene
    std::vector<Slot> slots;
    std::unordered_map<int64_t, Done> results;
    std::map<cloth_scene, size_t> admitted;   // scene -> footprint
    std::map<cloth_scene, bool> busy;
    std::map<cloth_scene, double> last_used;  // admitted scenes: when their last step started
    std::deque<cloth_scene> waiting;          // scenes with requests, waiting for admission
    size_t budget = 0, used = 0;
    int64_t next_ticket = 1;
    int64_t in_flight = 0;
    int64_t evictions = 0;
    bool stop = false;
    cloth_status error = CLOTH_OK;
    std::string error_msg;
    std::thread worker;

    void run();
    bool admit_locked(cloth_scene sc);
    void admit_waiting();
};

// admits sc if its footprint fits the budget (caller holds mu)
bool cloth_server_s::admit_locked(cloth_scene sc) {
    if (admitted.count(sc)) return true;
    const size_t fp = sc->s.arena_bytes;
    if (budget && used + fp > budget) return false;
    admitted[sc] = fp;
    used += fp;
    busy[sc] = false;
    last_used[sc] = now_ms();
    return true;
}

// Admits waiting scenes in arrival order; when the next one does not fit,
// admitted scenes with no queued or running step are released, least
// recently used first, until it does (caller holds mu).
void cloth_server_s::admit_waiting() {
    while (!waiting.empty()) {
        cloth_scene sc = waiting.front();
        if (admit_locked(sc)) {
            waiting.pop_front();
            continue;
        }
        std::vector<std::pair<double, cloth_scene>> idle;
        for (auto& kv : admitted) {
            cloth_scene a = kv.first;
            if (busy[a]) continue;
            if (queued[a] > 0) continue;
            idle.push_back({last_used[a], a});
        }
        std::sort(idle.begin(), idle.end());
        const size_t need = sc->s.arena_bytes;
        size_t freed = 0;
        size_t k = 0;
        while (k < idle.size() && used - freed + need > budget) freed += admitted[idle[k++].second];
        if (used - freed + need > budget) return;   // wait for running steps to finish
        for (size_t i = 0; i < k; ++i) {
            cloth_scene a = idle[i].second;
            used -= admitted[a];
            admitted.erase(a);
            busy.erase(a);
            last_used.erase(a);
            ++evictions;
        }
        admit_locked(sc);
        waiting.pop_front();
    }
}

void cloth_server_s::run() {
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        // retire finished steps
        bool progressed = false;
        for (auto& sl : slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.end);
            if (q == hipErrorNotReady) continue;
            Done& d = results[sl.req.ticket];
            d.done = true;
            d.latency_ms = now_ms() - sl.req.t_submit;
            float ms = 0.f;
            if (q != hipSuccess || hipEventElapsedTime(&ms, sl.start, sl.end) != hipSuccess) {
                d.status = CLOTH_E_DEVICE;
            } else if (const int bits = *sl.status) {
                // the step was rolled back on the device (see cloth_step)
                d.status = (bits & STEP_DIVERGED) ? CLOTH_E_DIVERGED
                           : (bits & STEP_TANGLED) ? CLOTH_E_TANGLED
                                                   : CLOTH_E_CAPACITY;
            }
            d.service_ms = ms;
            busy[sl.req.scene] = false;
            sl.busy = false;
            --in_flight;
            progressed = true;
        }
        if (progressed) cv_done.notify_all();
        admit_waiting();
        // start queued requests whose scene is admitted and idle, oldest first
        for (auto& sl : slots) {
            if (sl.busy) continue;
            auto it = std::find_if(queue.begin(), queue.end(),
                                   [&](const Req& r) { return admitted.count(r.scene) && !busy[r.scene]; });
            if (it == queue.end()) break;
            Req r = *it;
            queue.erase(it);
            --queued[r.scene];
            cloth_status rc = prepare_step_graph(r.scene, r.g);
            hipError_t e = hipSuccess;
            if (rc == CLOTH_OK) {
                e = hipEventRecord(sl.start, sl.stream);
                if (e == hipSuccess) e = hipGraphLaunch(r.scene->s.graph_exec, sl.stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(sl.status, r.scene->c.cnt + CNT_LAST_STATUS, sizeof(int),
                                       hipMemcpyDeviceToHost, sl.stream);
                if (e == hipSuccess) e = hipEventRecord(sl.end, sl.stream);
            }
            if (rc != CLOTH_OK || e != hipSuccess) {
                Done& d = results[r.ticket];
                d.done = true;
                d.status = rc != CLOTH_OK ? rc : CLOTH_E_DEVICE;
                cv_done.notify_all();
                continue;
            }
            sl.busy = true;
            sl.req = r;
            busy[r.scene] = true;
            last_used[r.scene] = now_ms();
            ++in_flight;
        }
        if (stop && queue.empty() && in_flight == 0) break;
        if (in_flight == 0 && queue.empty()) {
            cv_work.wait(lk, [&] { return stop || !queue.empty(); });
        } else {
            // poll the device without holding the lock
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

extern "C" {

cloth_status cloth_server_create(int32_t n_slots, size_t hbm_budget, cloth_server* out) {
    if (!out || n_slots <= 0 || n_slots > 64) return set_error(CLOTH_E_INVALID, "slots must be in [1, 64]");
    auto* sv = new (std::nothrow) cloth_server_s();
    if (!sv) return set_error(CLOTH_E_OOM, "host allocation");
    sv->budget = hbm_budget;
    sv->slots.resize(n_slots);
    for (auto& sl : sv->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&sl.start) != hipSuccess || hipEventCreate(&sl.end) != hipSuccess ||
            hipHostMalloc((void**)&sl.status, sizeof(int), hipHostMallocDefault) != hipSuccess) {
            delete sv;
            return set_error(CLOTH_E_DEVICE, "stream/event creation");
        }
    }
    sv->worker = std::thread([sv] { sv->run(); });
    *out = sv;
    return CLOTH_OK;
}

cloth_status cloth_server_admit(cloth_server sv, cloth_scene sc, int32_t* admitted) {
    if (!sv || !sc || !admitted) return set_error(CLOTH_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    *admitted = sv->admit_locked(sc) ? 1 : 0;
    return CLOTH_OK;
}

cloth_status cloth_server_release(cloth_server sv, cloth_scene sc) {
    if (!sv || !sc) return set_error(CLOTH_E_INVALID, "null argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->admitted.find(sc);
    if (it == sv->admitted.end()) return set_error(CLOTH_E_INVALID, "scene not admitted");
    sv->cv_done.wait(lk, [&] {
        return !sv->busy[sc] && sv->queued[sc] == 0;
    });
    it = sv->admitted.find(sc);   // the worker may have released it meanwhile
    if (it == sv->admitted.end()) return CLOTH_OK;
    sv->used -= it->second;
    sv->admitted.erase(it);
    sv->busy.erase(sc);
    sv->last_used.erase(sc);
    return CLOTH_OK;
}

cloth_status cloth_server_submit(cloth_server sv, cloth_scene sc, const float gravity[3], int64_t* ticket) {
    if (!sv || !sc || !gravity || !ticket) return set_error(CLOTH_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->budget && sc->s.arena_bytes > sv->budget)
        return set_error(CLOTH_E_OOM, "the scene's footprint exceeds the server's budget");
    if (!sv->admitted.count(sc) &&
        std::find(sv->waiting.begin(), sv->waiting.end(), sc) == sv->waiting.end())
        sv->waiting.push_back(sc);   // admitted by the worker when its footprint fits
    cloth_server_s::Req r;
    r.ticket = sv->next_ticket++;
    r.scene = sc;
    std::memcpy(r.g, gravity, sizeof(r.g));
    r.t_submit = now_ms();
    sv->results[r.ticket] = cloth_server_s::Done{};
    sv->queue.push_back(r);
    ++sv->queued[sc];
    *ticket = r.ticket;
    sv->cv_work.notify_one();
    return CLOTH_OK;
}

cloth_status cloth_server_poll(cloth_server sv, int64_t ticket, int32_t* done, double* latency_ms,
                               double* service_ms) {
    if (!sv || !done) return set_error(CLOTH_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->results.find(ticket);
    if (it == sv->results.end()) return set_error(CLOTH_E_INVALID, "unknown ticket");
    *done = it->second.done ? 1 : 0;
    if (it->second.done) {
        if (latency_ms) *latency_ms = it->second.latency_ms;
        if (service_ms) *service_ms = it->second.service_ms;
        return it->second.status;
    }
    return CLOTH_OK;
}

cloth_status cloth_server_wait(cloth_server sv, int64_t ticket, double* latency_ms, double* service_ms) {
    if (!sv) return set_error(CLOTH_E_INVALID, "null argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->results.find(ticket);
    if (it == sv->results.end()) return set_error(CLOTH_E_INVALID, "unknown ticket");
    sv->cv_done.wait(lk, [&] { return sv->results[ticket].done; });
    const auto& d = sv->results[ticket];
    if (latency_ms) *latency_ms = d.latency_ms;
    if (service_ms) *service_ms = d.service_ms;
    return d.status;
}

cloth_status cloth_server_info(cloth_server sv, int32_t* n_admitted, int32_t* n_waiting, size_t* used_bytes,
                               int64_t* evictions) {
    if (!sv) return set_error(CLOTH_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (n_admitted) *n_admitted = (int32_t)sv->admitted.size();
    if (n_waiting) *n_waiting = (int32_t)sv->waiting.size();
    if (used_bytes) *used_bytes = sv->used;
    if (evictions) *evictions = sv->evictions;
    return CLOTH_OK;
}

cloth_status cloth_server_destroy(cloth_server sv) {
    if (!sv) return CLOTH_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv_work.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    for (auto& sl : sv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.start) (void)hipEventDestroy(sl.start);
        if (sl.end) (void)hipEventDestroy(sl.end);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.status) (void)hipHostFree(sl.status);
    }
    delete sv;
    return CLOTH_OK;
}

}  // extern "C"
