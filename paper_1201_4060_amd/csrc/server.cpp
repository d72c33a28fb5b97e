// Serving: resident fields, particle-query requests admitted by device memory
// and evaluated concurrently on several HIP streams (continuous batching).
//
// Client threads submit requests (field id, host positions, host outputs);
// one scheduler thread owns all GPU work of the server.  It admits waiting
// requests in arrival order whenever a slot (one HIP stream, default
// priority) and enough of the device arena are free, enqueues
//   copy positions in -> bin + gather -> copy u (and grad) out
// on the slot's stream, and retires requests whose completion event has
// fired, so requests that arrive while others run start as soon as resources
// free up and their work overlaps on the device.  The arena is allocated once
// at creation; requests never allocate device memory.  Every request runs the
// single-field evaluation with the configuration the context picks for its
// field and size, so its result does not depend on what else is running.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "common.hpp"

namespace bsi {
namespace {

using Clock = std::chrono::steady_clock;

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device buffer (host-side bookkeeping only).
class Arena {
   public:
    void init(char* base, size_t bytes) {
        base_ = base;
        free_.clear();
        if (bytes) free_[0] = bytes;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    char* ptr(size_t off) const { return base_ + off; }
    size_t peak() const { return peak_; }

   private:
    char* base_ = nullptr;
    std::map<size_t, size_t> free_;  // offset -> length
    size_t used_ = 0, peak_ = 0;
};

struct Request {
    uint64_t ticket = 0;
    bsi_field* field = nullptr;
    const double* pos = nullptr;
    int64_t P = 0;
    void* u = nullptr;
    void* grad = nullptr;
    int64_t t_submit = 0;
    bsi_eval_config cfg{};
    size_t bytes = 0;    // arena footprint
    size_t off = 0;      // arena offset
    int slot = -1;
};

struct Done {
    bsi_status status = BSI_OK;
    int64_t latency_ns = 0;
    int64_t device_ns = 0;
    std::string msg;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t start = nullptr, stop = nullptr;
    bool busy = false;
    Request req;
};

}  // namespace
}  // namespace bsi

using namespace bsi;

struct bsi_server {
    bsi_ctx* ctx = nullptr;
    bsi_server_config cfg{};
    void* arena_mem = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    std::unordered_map<int32_t, bsi_field*> fields;

    std::mutex mu;                    // guards everything below
    std::condition_variable cv_done;  // a request finished
    std::condition_variable cv_work;  // new request or shutdown
    std::deque<Request> waiting;
    // tickets submitted and not finished; finished and not yet collected (a
    // record is released when bsi_server_wait returns it or bsi_server_poll
    // reports it done)
    std::unordered_set<uint64_t> pending;
    std::unordered_map<uint64_t, Done> done;
    uint64_t next_ticket = 1;
    int64_t inflight = 0, queued_or_running = 0;
    bool stop = false;
    // statistics since the last reset: latencies of at most STATS_CAP
    // completed requests (a uniform sample of them beyond that)
    std::vector<int64_t> lat_ns, dev_ns;
    int64_t completed = 0, points = 0, rejected = 0, t_first = 0, t_last = 0, max_inflight = 0;
    uint64_t sample_state = 0x9e3779b97f4a7c15ull;

    std::thread worker;
};

namespace bsi {
namespace {

size_t request_bytes(const bsi_field* f, int64_t P, const bsi_eval_config& c, bool grad) {
    const size_t osz = f->desc.coef == BSI_F64 ? 8 : 4;
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t b = up(3 * size_t(P) * sizeof(double)) + up(size_t(P) * f->C * osz);
    if (grad) b += up(size_t(P) * f->C * 3 * osz);
    return b + up(eval_ws_bytes(f, P, c));
}

// Enqueue one admitted request on its slot's stream (scheduler thread).
bsi_status launch(bsi_server* sv, Slot& sl) {
    Request& r = sl.req;
    bsi_field* f = r.field;
    const size_t osz = f->desc.coef == BSI_F64 ? 8 : 4;
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    char* base = sv->arena.ptr(r.off);
    double* d_pos = reinterpret_cast<double*>(base);
    char* d_u = base + up(3 * size_t(r.P) * sizeof(double));
    char* d_g = d_u + up(size_t(r.P) * f->C * osz);
    char* d_ws = r.grad ? d_g + up(size_t(r.P) * f->C * 3 * osz) : d_g;
    const hipStream_t s = sl.stream;
    BSI_HIP(hipEventRecord(sl.start, s));
    BSI_HIP(hipMemcpyAsync(d_pos, r.pos, 3 * size_t(r.P) * sizeof(double), hipMemcpyHostToDevice, s));
    BSI_TRY(eval_run_ws(f, d_pos, r.P, d_u, r.grad ? d_g : nullptr, r.cfg, s, d_ws));
    BSI_HIP(hipMemcpyAsync(r.u, d_u, size_t(r.P) * f->C * osz, hipMemcpyDeviceToHost, s));
    if (r.grad) BSI_HIP(hipMemcpyAsync(r.grad, d_g, size_t(r.P) * f->C * 3 * osz, hipMemcpyDeviceToHost, s));
    BSI_HIP(hipEventRecord(sl.stop, s));
    return BSI_OK;
}

// Latency samples kept for the percentiles.
constexpr size_t STATS_CAP = size_t(1) << 20;

// SplitMix64 step (Steele, Lea and Flood 2014) for the latency sample.
uint64_t next_sample(uint64_t& state) {
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

void finish(bsi_server* sv, const Request& r, bsi_status st, const std::string& msg, int64_t dev_ns) {
    const int64_t t = now_ns();
    std::lock_guard<std::mutex> lk(sv->mu);
    Done d;
    d.status = st;
    d.latency_ns = t - r.t_submit;
    d.device_ns = dev_ns;
    d.msg = msg;
    sv->done[r.ticket] = d;
    sv->pending.erase(r.ticket);
    sv->queued_or_running--;
    if (st == BSI_OK) {
        // reservoir sample: request k (1-based) replaces a kept one with
        // probability STATS_CAP / k once the sample is full
        sv->completed++;
        if (sv->lat_ns.size() < STATS_CAP) {
            sv->lat_ns.push_back(d.latency_ns);
            sv->dev_ns.push_back(dev_ns);
        } else {
            const uint64_t j = next_sample(sv->sample_state) % uint64_t(sv->completed);
            if (j < STATS_CAP) {
                sv->lat_ns[j] = d.latency_ns;
                sv->dev_ns[j] = dev_ns;
            }
        }
        sv->points += r.P;
        sv->t_last = std::max(sv->t_last, t);
    } else {
        sv->rejected++;
    }
    sv->cv_done.notify_all();
}

void scheduler(bsi_server* sv) {
    (void)hipSetDevice(sv->ctx->device);
    for (;;) {
        bool progressed = false;
        // retire finished requests
        for (Slot& sl : sv->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.stop);
            if (q == hipErrorNotReady) continue;
            float ms = 0.f;
            bsi_status st = BSI_OK;
            std::string msg;
            if (q != hipSuccess) {
                st = BSI_E_DEVICE;
                msg = std::string("request failed on the device: ") + hipGetErrorString(q);
                (void)hipGetLastError();
            } else if (hipEventElapsedTime(&ms, sl.start, sl.stop) != hipSuccess) {
                (void)hipGetLastError();
            }
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->arena.release(sl.req.off, sl.req.bytes);
                sv->inflight--;
            }
            sl.busy = false;
            finish(sv, sl.req, st, msg, int64_t(double(ms) * 1e6));
            progressed = true;
        }
        // admit waiting requests in arrival order
        for (;;) {
            Slot* free_slot = nullptr;
            for (Slot& sl : sv->slots)
                if (!sl.busy) {
                    free_slot = &sl;
                    break;
                }
            if (!free_slot) break;
            Request r;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                if (sv->waiting.empty()) break;
                Request& head = sv->waiting.front();
                size_t off = 0;
                if (!sv->arena.alloc(head.bytes, &off)) break;  // wait for memory to free up
                head.off = off;
                r = head;
                sv->waiting.pop_front();
                sv->inflight++;
                sv->max_inflight = std::max(sv->max_inflight, sv->inflight);
            }
            free_slot->req = r;
            free_slot->busy = true;
            const bsi_status st = launch(sv, *free_slot);
            if (st != BSI_OK) {
                const std::string msg = bsi_last_error();
                (void)hipStreamSynchronize(free_slot->stream);
                (void)hipGetLastError();
                {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    sv->arena.release(r.off, r.bytes);
                    sv->inflight--;
                }
                free_slot->busy = false;
                finish(sv, r, st, msg, 0);
            }
            progressed = true;
        }
        std::unique_lock<std::mutex> lk(sv->mu);
        if (sv->stop && sv->waiting.empty() && sv->inflight == 0) return;
        if (!progressed) {
            if (sv->inflight == 0 && sv->waiting.empty())
                sv->cv_work.wait(lk, [&] { return sv->stop || !sv->waiting.empty(); });
            else if (sv->inflight > 0)
                sv->cv_work.wait_for(lk, std::chrono::microseconds(20));
            else  // waiting but nothing in flight and nothing admitted: cannot happen (budget checked at submit)
                sv->cv_work.wait_for(lk, std::chrono::microseconds(200));
        }
    }
}

double percentile(std::vector<int64_t> v, double q) {
    if (v.empty()) return 0.0;
    const size_t k = std::min(v.size() - 1, size_t(q * double(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return double(v[k]);
}

}  // namespace
}  // namespace bsi

extern "C" {

bsi_status bsi_server_create(bsi_ctx* ctx, const bsi_server_config* cfg, bsi_server** out) {
    clear_error();
    BSI_CHECK(ctx && cfg && out, BSI_E_INVAL, "NULL argument");
    *out = nullptr;
    BSI_CHECK(cfg->max_slots >= 1 && cfg->max_slots <= 64, BSI_E_INVAL, "max_slots must be in [1, 64]");
    BSI_CHECK(cfg->queue_capacity >= 1, BSI_E_INVAL, "queue_capacity must be >= 1");
    BSI_CHECK(cfg->hbm_budget >= (size_t(1) << 20), BSI_E_INVAL, "hbm_budget must be at least 1 MiB");
    BSI_CHECK(cfg->reserved[0] == 0 && cfg->reserved[1] == 0 && cfg->reserved[2] == 0 && cfg->reserved[3] == 0,
              BSI_E_INVAL, "reserved fields must be 0");
    BSI_HIP(hipSetDevice(ctx->device));
    auto* sv = new (std::nothrow) bsi_server();
    BSI_CHECK(sv != nullptr, BSI_E_NOMEM, "host allocation failed");
    sv->ctx = ctx;
    sv->cfg = *cfg;
    if (hipMalloc(&sv->arena_mem, cfg->hbm_budget) != hipSuccess) {
        (void)hipGetLastError();
        delete sv;
        set_error("server arena of " + std::to_string(cfg->hbm_budget) + " bytes does not fit");
        return BSI_E_NOMEM;
    }
    sv->arena.init(static_cast<char*>(sv->arena_mem), cfg->hbm_budget);
    sv->slots.resize(cfg->max_slots);
    for (Slot& sl : sv->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&sl.start) != hipSuccess || hipEventCreate(&sl.stop) != hipSuccess) {
            (void)hipGetLastError();
            for (Slot& t : sv->slots) {
                if (t.stream) (void)hipStreamDestroy(t.stream);
                if (t.start) (void)hipEventDestroy(t.start);
                if (t.stop) (void)hipEventDestroy(t.stop);
            }
            (void)hipFree(sv->arena_mem);
            delete sv;
            set_error("stream or event creation failed");
            return BSI_E_DEVICE;
        }
    }
    sv->worker = std::thread(scheduler, sv);
    *out = sv;
    return BSI_OK;
}

bsi_status bsi_server_add_field(bsi_server* sv, int32_t field_id, bsi_field* field) {
    clear_error();
    BSI_CHECK(sv && field, BSI_E_INVAL, "NULL argument");
    BSI_CHECK(field->ctx == sv->ctx, BSI_E_INVAL, "field belongs to another context");
    std::lock_guard<std::mutex> lk(sv->mu);
    BSI_CHECK(sv->fields.find(field_id) == sv->fields.end(), BSI_E_INVAL,
              "field id " + std::to_string(field_id) + " is already registered");
    sv->fields[field_id] = field;
    return BSI_OK;
}

bsi_status bsi_server_submit(bsi_server* sv, int32_t field_id, const double* pos_host, int64_t P, void* u_host,
                             void* grad_host, uint64_t* ticket) {
    clear_error();
    BSI_CHECK(sv && ticket, BSI_E_INVAL, "NULL argument");
    BSI_CHECK(P >= 1 && P < (int64_t(1) << 31), BSI_E_INVAL, "P must be in [1, 2^31)");
    BSI_CHECK(pos_host && u_host, BSI_E_INVAL, "pos and u must be given");
    const int64_t t = now_ns();
    Request r;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->fields.find(field_id);
        BSI_CHECK(it != sv->fields.end(), BSI_E_INVAL, "unknown field id " + std::to_string(field_id));
        r.field = it->second;
    }
    BSI_TRY(lookup_config(sv->ctx, r.field, P, &r.cfg));
    r.pos = pos_host;
    r.P = P;
    r.u = u_host;
    r.grad = grad_host;
    r.t_submit = t;
    r.bytes = request_bytes(r.field, P, r.cfg, grad_host != nullptr);
    BSI_CHECK(r.bytes <= sv->cfg.hbm_budget, BSI_E_NOMEM,
              "request needs " + std::to_string(r.bytes) + " device bytes, more than the server budget");
    std::lock_guard<std::mutex> lk(sv->mu);
    BSI_CHECK(!sv->stop, BSI_E_CANCELLED, "server is shutting down");
    BSI_CHECK(int64_t(sv->waiting.size()) < sv->cfg.queue_capacity, BSI_E_BUSY, "request queue is full");
    r.ticket = sv->next_ticket++;
    if (sv->t_first == 0) sv->t_first = t;
    sv->pending.insert(r.ticket);
    sv->waiting.push_back(r);
    sv->queued_or_running++;
    *ticket = r.ticket;
    sv->cv_work.notify_one();
    return BSI_OK;
}

bsi_status bsi_server_poll(bsi_server* sv, uint64_t ticket, int32_t* done, int64_t* latency_ns) {
    clear_error();
    BSI_CHECK(sv && done, BSI_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    BSI_CHECK(ticket >= 1 && ticket < sv->next_ticket, BSI_E_INVAL, "unknown ticket");
    auto it = sv->done.find(ticket);
    if (it == sv->done.end()) {
        BSI_CHECK(sv->pending.count(ticket) != 0, BSI_E_INVAL, "ticket already collected");
        *done = 0;
        return BSI_OK;
    }
    *done = 1;
    if (latency_ns) *latency_ns = it->second.latency_ns;
    const bsi_status st = it->second.status;
    if (st != BSI_OK) set_error(it->second.msg);
    sv->done.erase(it);
    return st;
}

bsi_status bsi_server_wait(bsi_server* sv, uint64_t ticket, int64_t* latency_ns) {
    clear_error();
    BSI_CHECK(sv != nullptr, BSI_E_INVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    BSI_CHECK(ticket >= 1 && ticket < sv->next_ticket, BSI_E_INVAL, "unknown ticket");
    BSI_CHECK(sv->done.count(ticket) != 0 || sv->pending.count(ticket) != 0, BSI_E_INVAL,
              "ticket already collected");
    sv->cv_done.wait(lk, [&] { return sv->done.count(ticket) != 0; });
    auto it = sv->done.find(ticket);
    if (latency_ns) *latency_ns = it->second.latency_ns;
    const bsi_status st = it->second.status;
    if (st != BSI_OK) set_error(it->second.msg);
    sv->done.erase(it);
    return st;
}

bsi_status bsi_server_drain(bsi_server* sv) {
    clear_error();
    BSI_CHECK(sv != nullptr, BSI_E_INVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->queued_or_running == 0; });
    return BSI_OK;
}

bsi_status bsi_server_stats(bsi_server* sv, bsi_server_report* out) {
    clear_error();
    BSI_CHECK(sv && out, BSI_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = bsi_server_report{};
    out->completed = sv->completed;
    out->failed = sv->rejected;
    out->p50_ns = percentile(sv->lat_ns, 0.50);
    out->p99_ns = percentile(sv->lat_ns, 0.99);
    out->device_p50_ns = percentile(sv->dev_ns, 0.50);
    out->device_p99_ns = percentile(sv->dev_ns, 0.99);
    out->points = sv->points;
    const double span = double(sv->t_last - sv->t_first) * 1e-9;
    out->points_per_s = (span > 0 && sv->points) ? double(sv->points) / span : 0.0;
    out->max_inflight = sv->max_inflight;
    out->peak_arena_bytes = sv->arena.peak();
    return BSI_OK;
}

bsi_status bsi_server_reset_stats(bsi_server* sv) {
    clear_error();
    BSI_CHECK(sv != nullptr, BSI_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->lat_ns.clear();
    sv->dev_ns.clear();
    sv->completed = sv->points = sv->rejected = sv->t_first = sv->t_last = sv->max_inflight = 0;
    return BSI_OK;
}

void bsi_server_destroy(bsi_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv_work.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();  // finishes every submitted request first
    (void)hipSetDevice(sv->ctx->device);
    for (Slot& sl : sv->slots) {
        (void)hipStreamSynchronize(sl.stream);
        (void)hipStreamDestroy(sl.stream);
        (void)hipEventDestroy(sl.start);
        (void)hipEventDestroy(sl.stop);
    }
    (void)hipFree(sv->arena_mem);
    delete sv;
}

}  // extern "C"
