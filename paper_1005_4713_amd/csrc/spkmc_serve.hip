// spkmc_serve.hip -- the request server of include/spkmc.h (host side).
//
// Continuous batching for spkMC lattices: requests queue in FIFO order, are
// admitted as slots and pool memory free up, stay resident, and advance
// together in macro-steps.  Every lattice keeps its own cycle counter, clock
// and random streams (the streams are keyed by the cycle number and the domain,
// section 3 of the method), so how requests are grouped into launches and
// macro-steps never changes a result.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "api_internal.hpp"

using namespace spkmc;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First fit over the lattice part of the pool, lowest address first; freed
// blocks merge with free neighbours.
class PoolAlloc {
  public:
    void reset(size_t off, size_t len) {
        free_.clear();
        if (len) free_[off] = len;
    }
    bool alloc(size_t n, size_t &off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            off = it->first;
            size_t rest = it->second - n;
            free_.erase(it);
            if (rest) free_[off + n] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }

  private:
    std::map<size_t, size_t> free_;
};

struct Request {
    uint64_t id = 0;
    spkmc_params p{};
    uint64_t ncycles = 0, enq = 0;
    uint32_t obs_every = 0, flags = 0;
    int state = SPKMC_REQ_QUEUED;
    size_t bytes = 0, off = 0;
    bool holds_pool = false;
    spkmc_ctx *ctx = nullptr;
    bool batched = false;  // advances in batch launches (else alone with spkmc_run)
    int slot = -1;         // pinned slot its final state header is copied to
    double t_arrival = 0, t_admit = -1, t_done = -1;
    spkmc_obs obs{};
};

struct MacroStep {
    hipEvent_t ev = nullptr;
    std::vector<uint64_t> finishing;  // requests whose last cycles are in this step
};

}  // namespace

struct spkmc_server {
    spkmc_server_config cfg{};
    char *pool = nullptr;
    size_t pool_bytes = 0, ws_bytes = 0;
    hipStream_t stream = nullptr;
    PoolAlloc alloc;
    std::unordered_map<uint64_t, Request> reqs;
    std::deque<uint64_t> queue;
    std::vector<uint64_t> live;  // admitted, cycles still to enqueue
    std::deque<MacroStep> inflight;
    std::vector<hipEvent_t> spare_events;
    DevState *pinned = nullptr;  // max_live * (inflight + 1) headers
    std::vector<int> free_slots;
    uint32_t cap[2] = {0, 0};  // resident workgroups of the batch kernel, h = 8 and 16, most passes
    uint64_t next_id = 1;
    uint64_t n_done = 0, n_failed = 0, n_finishing = 0;
    uint64_t macro_steps = 0, launches = 0, in_use = 0, peak = 0;
    std::chrono::steady_clock::time_point t0;
    std::string err;
};

static thread_local std::string g_serve_error = "no error";

static spkmc_status sfail(spkmc_server *s, spkmc_status st, const std::string &msg) {
    if (s)
        s->err = msg;
    else
        g_serve_error = msg;
    return st;
}

static double now_s(const spkmc_server *s) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

static bool config_ok(const spkmc_server_config *c) {
    return c && c->struct_size == sizeof(spkmc_server_config) && c->macro_cycles > 0 && c->max_live > 0 &&
           c->max_live <= 4096 && c->inflight >= 1 && c->inflight <= 8 && c->wg_domains >= 0 && c->reserved == 0;
}

// Retire the oldest outstanding macro-step: its finishing requests become DONE.
static void retire_front(spkmc_server *s) {
    MacroStep &m = s->inflight.front();
    const double t = now_s(s);
    for (uint64_t id : m.finishing) {
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) continue;
        Request &r = it->second;
        const DevState &st = s->pinned[r.slot];
        if (st.error) {
            r.state = SPKMC_REQ_FAILED;
            ++s->n_failed;
            char msg[128];
            snprintf(msg, sizeof msg, "request %llu: device-side wait gave up (code %u)", (unsigned long long)id,
                     st.error);
            s->err = msg;
        } else {
            // the context is gone already unless the lattice is kept
            obs_from_state(r.p, (uint64_t)r.p.L * r.p.L * r.p.L, st, &r.obs);
            r.state = SPKMC_REQ_DONE;
            ++s->n_done;
        }
        r.t_done = t;
        s->free_slots.push_back(r.slot);
        r.slot = -1;
        --s->n_finishing;
    }
    s->spare_events.push_back(m.ev);
    s->inflight.pop_front();
}

static void drop_memory(spkmc_server *s, Request &r) {
    if (r.ctx) {
        spkmc_destroy(r.ctx);
        r.ctx = nullptr;
    }
    if (r.holds_pool) {
        s->alloc.release(r.off, r.bytes);
        s->in_use -= r.bytes;
        r.holds_pool = false;
    }
}

// Admit queued requests in FIFO order while a slot and pool memory are free.
static spkmc_status admit(spkmc_server *s) {
    while (!s->queue.empty() && s->live.size() < s->cfg.max_live) {
        Request &r = s->reqs[s->queue.front()];
        size_t off = 0;
        if (!s->alloc.alloc(r.bytes, off)) break;  // head of line waits for memory
        s->queue.pop_front();
        r.off = off;
        r.holds_pool = true;
        s->in_use += r.bytes;
        s->peak = std::max(s->peak, s->in_use);
        spkmc_params p = r.p;
        p.engine = SPKMC_ENGINE_AUTO;
        p.wg_domains = 0;
        spkmc_status st = spkmc_init(&p, s->pool + off, r.bytes, (void *)s->stream, &r.ctx);
        r.t_admit = now_s(s);
        if (st != SPKMC_OK) {
            std::string why = r.ctx ? spkmc_last_error(r.ctx) : spkmc_last_error(nullptr);
            drop_memory(s, r);
            r.state = SPKMC_REQ_FAILED;
            ++s->n_failed;
            s->err = "request " + std::to_string(r.id) + ": " + why;
            if (st == SPKMC_E_DEVICE) return sfail(s, st, s->err);
            continue;
        }
        std::string why;
        const int h = r.ctx->g.h;
        r.batched = persistent_supported(r.ctx->g, r.ctx->p, false, why) &&
                    batch_wgs(r.ctx->g, batch_max_passes(h)) <= s->cap[h == 16];
        r.state = SPKMC_REQ_RUNNING;
        s->live.push_back(r.id);
    }
    return SPKMC_OK;
}

// First fit by decreasing workgroups into launches the device holds at once.
static std::vector<std::vector<Request *>> pack(std::vector<Request *> rs, uint32_t cap) {
    auto wgs = [](const Request *r) { return batch_wgs(r->ctx->g, batch_max_passes(r->ctx->g.h)); };
    std::sort(rs.begin(), rs.end(), [&](Request *a, Request *b) {
        uint32_t wa = wgs(a), wb = wgs(b);
        return wa != wb ? wa > wb : a->id < b->id;
    });
    std::vector<std::vector<Request *>> bins;
    std::vector<uint32_t> used;
    for (Request *r : rs) {
        uint32_t w = wgs(r);
        size_t b = 0;
        while (b < bins.size() && used[b] + w > cap) ++b;
        if (b == bins.size()) {
            bins.emplace_back();
            used.push_back(0);
        }
        bins[b].push_back(r);
        used[b] += w;
    }
    return bins;
}

// After a failed launch the state of every resident request is unknown.
static spkmc_status fail_live(spkmc_server *s, spkmc_status st, const std::string &msg) {
    for (uint64_t id : s->live) {
        Request &r = s->reqs[id];
        r.state = SPKMC_REQ_FAILED;
        r.t_done = now_s(s);
        drop_memory(s, r);
        ++s->n_failed;
    }
    s->live.clear();
    return sfail(s, st, msg);
}

// Enqueue one macro-step over every live request.
static spkmc_status enqueue_step(spkmc_server *s) {
    MacroStep m;
    const uint64_t mc = s->cfg.macro_cycles;
    std::vector<Request *> by_h[2];
    std::vector<Request *> all;
    for (uint64_t id : s->live) {
        Request &r = s->reqs[id];
        all.push_back(&r);
        if (r.ncycles - r.enq == 0) continue;
        if (r.batched)
            by_h[r.ctx->g.h == 16].push_back(&r);
        else {
            uint64_t n = std::min(mc, r.ncycles - r.enq);
            spkmc_status st = spkmc_run(r.ctx, n, r.obs_every);
            if (st != SPKMC_OK) return fail_live(s, st, "request " + std::to_string(id) + ": " + spkmc_last_error(r.ctx));
            ++s->launches;
        }
    }
    for (int hi = 0; hi < 2; ++hi) {
        if (by_h[hi].empty()) continue;
        for (auto &bin : pack(by_h[hi], s->cap[hi])) {
            std::vector<spkmc_ctx *> ctxs;
            std::vector<uint64_t> nc;
            uint32_t obs = bin[0]->obs_every;
            bool same_obs = true;
            for (Request *r : bin) same_obs &= r->obs_every == obs;
            if (same_obs) {
                for (Request *r : bin) {
                    ctxs.push_back(r->ctx);
                    nc.push_back(std::min(mc, r->ncycles - r->enq));
                }
                spkmc_status st = spkmc_run_batch(ctxs.data(), ctxs.size(), nc.data(), obs, s->cfg.wg_domains,
                                                  s->pool, s->ws_bytes, nullptr);
                if (st != SPKMC_OK) return fail_live(s, st, std::string("batch launch: ") + spkmc_last_error(nullptr));
                ++s->launches;
            } else {
                // the batch kernel takes one observation interval: one launch per interval
                std::map<uint32_t, std::vector<Request *>> by_obs;
                for (Request *r : bin) by_obs[r->obs_every].push_back(r);
                for (auto &kv : by_obs) {
                    ctxs.clear();
                    nc.clear();
                    for (Request *r : kv.second) {
                        ctxs.push_back(r->ctx);
                        nc.push_back(std::min(mc, r->ncycles - r->enq));
                    }
                    spkmc_status st = spkmc_run_batch(ctxs.data(), ctxs.size(), nc.data(), kv.first,
                                                      s->cfg.wg_domains, s->pool, s->ws_bytes, nullptr);
                    if (st != SPKMC_OK)
                        return fail_live(s, st, std::string("batch launch: ") + spkmc_last_error(nullptr));
                    ++s->launches;
                }
            }
        }
    }
    // requests whose last cycles are now enqueued: copy their state header out,
    // and give back the memory of those not kept (later work on the stream,
    // such as the next admission's initialisation, runs after this copy)
    std::vector<uint64_t> still;
    for (Request *r : all) {
        r->enq += std::min(mc, r->ncycles - r->enq);
        if (r->enq < r->ncycles) {
            still.push_back(r->id);
            continue;
        }
        if (s->free_slots.empty()) return sfail(s, SPKMC_E_STATE, "no pinned slot free (internal)");
        r->slot = s->free_slots.back();
        s->free_slots.pop_back();
        hipError_t e = hipMemcpyAsync(&s->pinned[r->slot], r->ctx->dev, sizeof(DevState), hipMemcpyDeviceToHost,
                                      s->stream);
        if (e != hipSuccess) return sfail(s, SPKMC_E_DEVICE, std::string("state copy: ") + hipGetErrorString(e));
        if (!(r->flags & SPKMC_SERVE_KEEP)) drop_memory(s, *r);
        m.finishing.push_back(r->id);
        ++s->n_finishing;
    }
    s->live.swap(still);
    if (s->spare_events.empty()) {
        hipEvent_t ev;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return sfail(s, SPKMC_E_DEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
        s->spare_events.push_back(ev);
    }
    m.ev = s->spare_events.back();
    s->spare_events.pop_back();
    hipError_t e = hipEventRecord(m.ev, s->stream);
    if (e != hipSuccess) {
        s->spare_events.push_back(m.ev);
        return sfail(s, SPKMC_E_DEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e));
    }
    s->inflight.push_back(std::move(m));
    ++s->macro_steps;
    return SPKMC_OK;
}

static void fill_stats(const spkmc_server *s, spkmc_server_stats *o) {
    o->queued = s->queue.size();
    o->live = s->live.size();
    o->finishing = s->n_finishing;
    o->done = s->n_done;
    o->failed = s->n_failed;
    o->macro_steps = s->macro_steps;
    o->launches = s->launches;
    o->pool_in_use = s->in_use;
    o->pool_peak = s->peak;
    o->inflight = s->inflight.size();
}

#pragma GCC visibility push(default)
extern "C" {

size_t spkmc_server_reserved_bytes(const spkmc_server_config *cfg) {
    if (!config_ok(cfg)) return 0;
    return align_up(spkmc_batch_workspace_bytes(cfg->max_live));
}

spkmc_status spkmc_server_create(const spkmc_server_config *cfg, void *dev_pool, size_t pool_bytes,
                                 void *hip_stream, spkmc_server **out) {
    if (!out) return sfail(nullptr, SPKMC_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!config_ok(cfg)) return sfail(nullptr, SPKMC_E_INVAL, "invalid server configuration");
    if (!dev_pool || ((uintptr_t)dev_pool % kAlign)) return sfail(nullptr, SPKMC_E_INVAL, "pool NULL or not 256-byte aligned");
    const size_t ws = spkmc_server_reserved_bytes(cfg);
    if (pool_bytes < ws) return sfail(nullptr, SPKMC_E_RANGE, "pool smaller than the server's reserved bytes");
    spkmc_server *s = new (std::nothrow) spkmc_server;
    if (!s) return sfail(nullptr, SPKMC_E_NOMEM, "out of host memory");
    s->cfg = *cfg;
    s->pool = static_cast<char *>(dev_pool);
    s->pool_bytes = pool_bytes;
    s->ws_bytes = ws;
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->alloc.reset(ws, (pool_bytes - ws) & ~(kAlign - 1));
    const size_t slots = (size_t)cfg->max_live * (cfg->inflight + 1);
    hipError_t e = hipHostMalloc((void **)&s->pinned, slots * sizeof(DevState), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete s;
        return sfail(nullptr, SPKMC_E_DEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    memset((void *)s->pinned, 0, slots * sizeof(DevState));
    for (size_t i = slots; i-- > 0;) s->free_slots.push_back((int)i);
    s->cap[0] = batch_capacity(8, batch_max_passes(8));
    s->cap[1] = batch_capacity(16, batch_max_passes(16));
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return SPKMC_OK;
}

spkmc_status spkmc_server_submit(spkmc_server *s, const spkmc_params *p, uint64_t ncycles, uint32_t obs_every,
                                 uint32_t flags, double t_arrival, uint64_t *id) {
    if (!s) return sfail(nullptr, SPKMC_E_INVAL, "server is NULL");
    if (!p || !id) return sfail(s, SPKMC_E_INVAL, "params or id is NULL");
    if (flags & ~(uint32_t)SPKMC_SERVE_KEEP) return sfail(s, SPKMC_E_INVAL, "unknown flags");
    const size_t need = spkmc_state_bytes(p);
    if (need == 0) return sfail(s, SPKMC_E_INVAL, std::string("invalid parameters: ") + spkmc_last_error(nullptr));
    const size_t bytes = align_up(need);
    if (bytes > s->pool_bytes - s->ws_bytes) return sfail(s, SPKMC_E_RANGE, "the lattice does not fit in the pool");
    Request r;
    r.id = s->next_id++;
    r.p = *p;
    r.ncycles = ncycles;
    r.obs_every = obs_every;
    r.flags = flags;
    r.bytes = bytes;
    r.t_arrival = t_arrival < 0 ? now_s(s) : t_arrival;
    s->reqs.emplace(r.id, r);
    s->queue.push_back(r.id);
    *id = r.id;
    return SPKMC_OK;
}

spkmc_status spkmc_server_step(spkmc_server *s, int wait, spkmc_server_stats *stats) {
    if (!s) return sfail(nullptr, SPKMC_E_INVAL, "server is NULL");
    bool retired = false;
    while (!s->inflight.empty()) {
        hipError_t e = hipEventQuery(s->inflight.front().ev);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) return sfail(s, SPKMC_E_DEVICE, std::string("hipEventQuery: ") + hipGetErrorString(e));
        retire_front(s);
        retired = true;
    }
    if (wait && !retired && !s->inflight.empty()) {
        hipError_t e = hipEventSynchronize(s->inflight.front().ev);
        if (e != hipSuccess) return sfail(s, SPKMC_E_DEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
        retire_front(s);
    }
    spkmc_status st = admit(s);
    if (st != SPKMC_OK) return st;
    while (s->inflight.size() < s->cfg.inflight && !s->live.empty()) {
        st = enqueue_step(s);
        if (st != SPKMC_OK) return st;
        // requests admitted after this step's finishers left join the next one
        st = admit(s);
        if (st != SPKMC_OK) return st;
    }
    if (stats) fill_stats(s, stats);
    return SPKMC_OK;
}

spkmc_status spkmc_server_poll(const spkmc_server *s, uint64_t id, spkmc_request_status *out) {
    if (!s) return sfail(nullptr, SPKMC_E_INVAL, "server is NULL");
    if (!out) return SPKMC_E_INVAL;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return SPKMC_E_INVAL;
    const Request &r = it->second;
    out->state = r.state;
    out->flags = r.flags;
    out->ncycles = r.ncycles;
    out->cycles_enqueued = r.enq;
    out->bytes = r.bytes;
    out->t_arrival = r.t_arrival;
    out->t_admit = r.t_admit;
    out->t_done = r.t_done;
    out->obs = r.obs;
    return SPKMC_OK;
}

spkmc_status spkmc_server_context(spkmc_server *s, uint64_t id, spkmc_ctx **ctx) {
    if (!s) return sfail(nullptr, SPKMC_E_INVAL, "server is NULL");
    if (!ctx) return sfail(s, SPKMC_E_INVAL, "ctx is NULL");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return sfail(s, SPKMC_E_INVAL, "unknown request id");
    Request &r = it->second;
    if (r.state != SPKMC_REQ_DONE || !r.ctx) return sfail(s, SPKMC_E_STATE, "request is not done or not kept");
    *ctx = r.ctx;
    return SPKMC_OK;
}

spkmc_status spkmc_server_release(spkmc_server *s, uint64_t id) {
    if (!s) return sfail(nullptr, SPKMC_E_INVAL, "server is NULL");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return sfail(s, SPKMC_E_INVAL, "unknown request id");
    Request &r = it->second;
    if (r.state != SPKMC_REQ_DONE && r.state != SPKMC_REQ_FAILED)
        return sfail(s, SPKMC_E_STATE, "request is still queued or running");
    drop_memory(s, r);
    if (r.state == SPKMC_REQ_DONE)
        --s->n_done;
    else
        --s->n_failed;
    s->reqs.erase(it);
    return SPKMC_OK;
}

double spkmc_server_clock(const spkmc_server *s) { return s ? now_s(s) : 0.0; }

const char *spkmc_server_last_error(const spkmc_server *s) {
    return s ? s->err.c_str() : g_serve_error.c_str();
}

void spkmc_server_destroy(spkmc_server *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    for (auto &kv : s->reqs)
        if (kv.second.ctx) spkmc_destroy(kv.second.ctx);
    for (auto &m : s->inflight) (void)hipEventDestroy(m.ev);
    for (hipEvent_t ev : s->spare_events) (void)hipEventDestroy(ev);
    if (s->pinned) (void)hipHostFree(s->pinned);
    delete s;
}

}  // extern "C"
#pragma GCC visibility pop
