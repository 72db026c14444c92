// hjr_server.cpp -- continuous batching of safe-set update requests.
//
// Each request names a subsystem instance and a new disturbance bound (the
// online update of paper Sec. II-C, accelerated by warm starts, Sec. III-B).
// A worker thread owns one Engine with `max_active` slots.  Between chunks
// it admits queued requests into free slots while the device-memory budget
// allows, so requests that arrive while others are iterating join the next
// chunk and share its kernel launches.  Every instance keeps its last
// converged value resident in HBM; the next request of that instance starts
// from it.  A request that does not converge leaves the resident value
// untouched (the last good safe set stays valid).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/hjr.h"
#include "hjr_engine.hpp"

using namespace hjr;
using Clock = std::chrono::steady_clock;

namespace {

size_t align256(size_t x)
{
    return (x + 255) & ~size_t(255);
}

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Instance {
    uint64_t id = 0;
    hjr_dyn dyn;
    hjr_grid grid;
    int64_t N = 0;
    void* l = nullptr;
    void* V_res = nullptr;
    bool has_value = false;
    bool busy = false;
    uint64_t last_use = 0;
};

struct Ticket {
    uint64_t id = 0;
    hjr_request req;
    std::vector<char> l_host;  // copy of req.l
    std::vector<char> f_host;  // copy of req.dfield (empty: the boxes req.d)
    Clock::time_point t_submit, t_admit;
    bool admitted = false;
    bool done = false;
    hjr_reply reply;
    // running state
    std::unique_ptr<Job> job;
    void* V_work = nullptr;
    void* Vhat = nullptr;
    void* table = nullptr;
    void* field = nullptr;     // device copy of f_host while running
    size_t work_bytes = 0;
};

// Whether every (lower, upper) pair of a host field is finite and ordered.
template <typename T>
bool field_ok(const T* f, int nch, int64_t N)
{
    for (int c = 0; c < nch; c++)
        for (int64_t i = 0; i < N; i++) {
            const double lo = (double)f[2 * c * N + i], hi = (double)f[(2 * c + 1) * N + i];
            if (!(lo <= hi) || !std::isfinite(lo) || !std::isfinite(hi)) return false;
        }
    return true;
}

}  // namespace

struct hjr_server {
    hjr_server_cfg cfg;
    size_t budget = 0;
    size_t used = 0;  // device bytes held (live + cached)
    hipStream_t stream = nullptr;
    std::unique_ptr<Engine> eng;
    std::thread worker;
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::unique_ptr<Ticket>> tickets;
    std::map<uint64_t, Instance> inst;
    std::map<uint64_t, int> pending;                     // queued + running tickets per instance
    std::map<uint64_t, std::vector<char>> l_host;        // host copy of each instance's constraint
    std::map<uint64_t, std::pair<hjr_grid, int32_t>> shape;  // grid and model of every instance seen
    std::map<size_t, std::vector<void*>> cache;  // free blocks by size
    uint64_t next_ticket = 1;
    uint64_t use_clock = 0;
    bool stop = false;
    hjr_status fatal = HJR_OK;

    size_t esz() const { return elem_size(cfg.dtype); }

    // ---- device memory with a per-size cache, bounded by the budget ----
    void* take(size_t bytes)
    {
        bytes = align256(bytes);
        auto it = cache.find(bytes);
        if (it != cache.end() && !it->second.empty()) {
            void* p = it->second.back();
            it->second.pop_back();
            return p;
        }
        // release cached blocks of other sizes until the new one fits
        while (used + bytes > budget) {
            bool freed = false;
            for (auto& kv : cache)
                if (!kv.second.empty()) {
                    (void)hipStreamSynchronize(stream);
                    (void)hipFree(kv.second.back());
                    kv.second.pop_back();
                    used -= kv.first;
                    freed = true;
                    break;
                }
            if (!freed) return nullptr;
        }
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        used += bytes;
        return p;
    }
    void give(void* p, size_t bytes)
    {
        if (p) cache[align256(bytes)].push_back(p);
    }
    size_t cached_bytes() const
    {
        size_t b = 0;
        for (auto& kv : cache) b += kv.first * kv.second.size();
        return b;
    }

    size_t instance_bytes(const hjr_grid& g) const { return 2 * align256(grid_size(g) * esz()); }
    size_t work_bytes(const hjr_grid& g) const
    {
        const int64_t n2 = g.ndim >= 3 ? g.n[2] : 1;
        return 2 * align256(grid_size(g) * esz()) + align256(n2 * esz());
    }

    // Can `need` more bytes be held, counting reusable cache and evictable
    // idle instances?  Evicting an instance drops only its warm start: its
    // constraint stays on the host and is uploaded again when it returns.
    // With `any` set (nothing running, so nothing will free up by itself)
    // instances that still have queued tickets may be evicted as well.
    bool make_room(size_t need, uint64_t keep_id, bool any)
    {
        while (used - cached_bytes() + need > budget) {
            Instance* victim = nullptr;
            for (auto& kv : inst) {
                Instance& I = kv.second;
                if (I.id == keep_id || I.busy) continue;
                if (!any && pending[I.id] > 0) continue;
                if (!victim || I.last_use < victim->last_use) victim = &I;
            }
            if (!victim) return false;
            give(victim->l, grid_size(victim->grid) * esz());
            if (victim->V_res) give(victim->V_res, grid_size(victim->grid) * esz());
            inst.erase(victim->id);
        }
        return true;
    }

    void finish(Ticket& t, Job& j)
    {
        Instance& I = inst[t.req.instance_id];
        const size_t vb = grid_size(I.grid) * esz();
        if (j.status == HJR_OK) {
            // the working buffer becomes the resident value
            give(I.V_res, vb);
            I.V_res = t.V_work;
            I.has_value = true;
        } else {
            give(t.V_work, vb);
        }
        give(t.Vhat, vb);
        const int64_t n2 = I.grid.ndim >= 3 ? I.grid.n[2] : 1;
        give(t.table, n2 * esz());
        if (t.field) give(t.field, t.f_host.size());
        t.f_host.clear();
        t.V_work = t.Vhat = t.table = t.field = nullptr;
        I.busy = false;
        pending[I.id]--;
        I.last_use = ++use_clock;
        t.reply.status = j.status;
        t.reply.iterations = j.level_iters[0];
        t.reply.residual = j.residual;
        t.reply.latency_ms = ms_between(t.t_submit, Clock::now());
        t.reply.queue_ms = ms_between(t.t_submit, t.t_admit);
        t.done = true;
    }

    // Admit queued requests into free engine slots (called with m held).
    void admit()
    {
        std::vector<uint64_t> blocked;  // instances whose earlier ticket waits
        for (auto it = queue.begin(); it != queue.end();) {
            if (eng->free_slots() == 0) break;
            Ticket& t = *tickets[*it];
            const uint64_t iid = t.req.instance_id;
            if (std::find(blocked.begin(), blocked.end(), iid) != blocked.end()) {
                ++it;
                continue;
            }
            auto ii = inst.find(iid);
            const bool known = ii != inst.end();
            if (known && ii->second.busy) {
                blocked.push_back(iid);
                ++it;
                continue;
            }
            const hjr_grid& g = t.req.grid;
            const size_t fbytes = t.f_host.empty() ? 0 : align256(t.f_host.size());
            const size_t need = work_bytes(g) + fbytes + (known ? 0 : instance_bytes(g));
            if (!make_room(need, iid, !eng->busy())) {
                blocked.push_back(iid);
                ++it;
                continue;
            }
            bool upload = !t.l_host.empty() || !known;
            if (!t.l_host.empty()) l_host[iid] = std::move(t.l_host);
            t.l_host.clear();
            if (!known) {
                Instance I;
                I.id = iid;
                I.dyn = t.req.dyn;
                I.grid = g;
                I.N = grid_size(g);
                I.l = take(I.N * esz());
                I.V_res = nullptr;
                inst[iid] = I;
                ii = inst.find(iid);
                if (!ii->second.l) {
                    fatal = HJR_ENOMEM;
                    return;
                }
                upload = true;
            }
            Instance& I = ii->second;
            if (upload) {
                const std::vector<char>& src = l_host[iid];
                if (hipMemcpyAsync(I.l, src.data(), src.size(), hipMemcpyHostToDevice, stream) !=
                        hipSuccess ||
                    hipStreamSynchronize(stream) != hipSuccess) {
                    fatal = HJR_EDEVICE;
                    return;
                }
            }
            const int64_t n2 = g.ndim >= 3 ? g.n[2] : 1;
            t.V_work = take(I.N * esz());
            t.Vhat = take(I.N * esz());
            t.table = take(n2 * esz());
            if (!t.V_work || !t.Vhat || !t.table) {
                fatal = HJR_ENOMEM;
                return;
            }
            if (!t.f_host.empty()) {
                t.field = take(t.f_host.size());
                if (!t.field) {
                    fatal = HJR_ENOMEM;
                    return;
                }
                if (hipMemcpyAsync(t.field, t.f_host.data(), t.f_host.size(), hipMemcpyHostToDevice,
                                   stream) != hipSuccess ||
                    hipStreamSynchronize(stream) != hipSuccess) {
                    fatal = HJR_EDEVICE;
                    return;
                }
            }
            auto job = std::make_unique<Job>();
            job->dyn = t.req.dyn;
            std::memset(job->d, 0, sizeof(job->d));
            for (int c = 0; c < dyn_channels(t.req.dyn.kind); c++) job->d[c] = t.req.d[c];
            job->tol = t.req.tol;
            job->band = t.req.band;
            job->nlev = 1;
            job->lev[0].grid = g;
            job->lev[0].l = I.l;
            job->lev[0].V = t.V_work;
            job->lev[0].mask = nullptr;
            job->lev[0].dfield = t.field;
            const bool warm = I.has_value && !t.req.cold;
            job->V0 = warm ? I.V_res : nullptr;
            job->Vhat = t.Vhat;
            job->table = t.table;
            Ticket* tp = &t;
            job->on_done = [this, tp](Job& j) {
                std::lock_guard<std::mutex> lk(m);
                finish(*tp, j);
                cv_done.notify_all();
            };
            t.reply.warm = warm ? 1 : 0;
            t.admitted = true;
            t.t_admit = Clock::now();
            I.busy = true;
            t.job = std::move(job);
            if (eng->add(t.job.get()) != HJR_OK) {
                fatal = HJR_EDEVICE;
                return;
            }
            it = queue.erase(it);
        }
    }

    void run()
    {
        (void)hipSetDevice(cfg.device);
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(m);
                if (fatal == HJR_OK) admit();
                if (fatal != HJR_OK) {
                    // fail every waiting ticket
                    for (uint64_t id : queue) {
                        Ticket& t = *tickets[id];
                        t.reply.status = fatal;
                        t.done = true;
                    }
                    queue.clear();
                    cv_done.notify_all();
                }
                if (!eng->busy()) {
                    lk.unlock();
                    (void)eng->drain();
                    lk.lock();
                    if (stop && queue.empty()) return;
                    if (!queue.empty() && fatal == HJR_OK && !eng->busy()) {
                        // idle and still nothing admissible: retry once with
                        // the slots and budget fully free, else give up on
                        // the head of the queue
                        admit();
                        if (!eng->busy() && !queue.empty() && fatal == HJR_OK) {
                            Ticket& t = *tickets[queue.front()];
                            t.reply.status = HJR_ENOMEM;
                            t.done = true;
                            pending[t.req.instance_id]--;
                            queue.pop_front();
                            cv_done.notify_all();
                        }
                        continue;
                    }
                    if (queue.empty() || fatal != HJR_OK) {
                        cv_work.wait(lk, [&] { return stop || (!queue.empty() && fatal == HJR_OK); });
                        if (stop && queue.empty()) return;
                    }
                    continue;
                }
            }
            hjr_status st = eng->step();
            if (st != HJR_OK) {
                std::lock_guard<std::mutex> lk(m);
                fatal = st;
            }
        }
    }
};

extern "C" {

hjr_status hjr_server_create(const hjr_server_cfg* cfg, hjr_server** out)
{
    if (!out) return HJR_EINVAL;
    *out = nullptr;
    hjr_server_cfg c;
    std::memset(&c, 0, sizeof(c));
    if (cfg) c = *cfg;
    if (c.hbm_budget_bytes == 0) c.hbm_budget_bytes = size_t(8) << 30;
    if (c.max_active <= 0) c.max_active = 256;
    if (c.order == 0) c.order = 2;
    if (c.chunk <= 0) c.chunk = 16;
    if (c.cfl == 0.0) c.cfl = 0.8;
    if (c.max_iter <= 0) c.max_iter = 100000;
    if ((c.dtype != HJR_F32 && c.dtype != HJR_F64) || (c.order != 1 && c.order != 2) ||
        !(c.cfl > 0.0 && c.cfl <= 1.0) || c.chunk > kMaxChunk)
        return HJR_EINVAL;
    std::unique_ptr<hjr_server> s;
    try {
        s.reset(new hjr_server());
    } catch (const std::bad_alloc&) {
        return HJR_ENOMEM;
    }
    s->cfg = c;
    s->budget = c.hbm_budget_bytes;
    if (hipSetDevice(c.device) != hipSuccess) return HJR_EINVAL;
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) return HJR_EDEVICE;
    EngineCfg ec;
    ec.dtype = c.dtype;
    ec.order = c.order;
    ec.cfl = c.cfl;
    ec.max_iter = c.max_iter;
    ec.K = c.chunk;
    ec.cap = c.max_active;
    ec.flags = c.flags;
    s->eng.reset(new Engine(ec));
    const size_t tb = Engine::table_bytes(c.max_active, c.chunk);
    if (tb >= s->budget) return HJR_ENOMEM;
    if (s->eng->init(s->stream, nullptr) != HJR_OK) return HJR_EDEVICE;
    s->used = align256(tb);
    s->worker = std::thread([p = s.get()] { p->run(); });
    *out = s.release();
    return HJR_OK;
}

hjr_status hjr_server_submit(hjr_server* s, const hjr_request* req, uint64_t* ticket)
{
    if (!s || !req || !ticket) return HJR_EINVAL;
    const hjr_grid& g = req->grid;
    if (!grid_valid(g) || !dyn_valid(req->dyn, g)) return HJR_EINVAL;
    const int nch = dyn_channels(req->dyn.kind);
    if (!req->dfield)
        for (int c = 0; c < nch; c++)
            if (!(req->d[c].lo <= req->d[c].hi)) return HJR_EINVAL;
    if (!(req->tol > 0.0)) return HJR_EINVAL;
    if (!(req->band >= 0.0)) return HJR_EINVAL;
    std::unique_ptr<Ticket> t(new Ticket());
    t->req = *req;
    std::memset(&t->reply, 0, sizeof(t->reply));
    t->t_submit = Clock::now();
    const size_t bytes = grid_size(g) * s->esz();
    const size_t fbytes = req->dfield ? 2 * (size_t)nch * bytes : 0;
    if (req->dfield) {
        const bool ok = s->cfg.dtype == HJR_F32
                            ? field_ok((const float*)req->dfield, nch, grid_size(g))
                            : field_ok((const double*)req->dfield, nch, grid_size(g));
        if (!ok) return HJR_EINVAL;
        t->f_host.resize(fbytes);
        std::memcpy(t->f_host.data(), req->dfield, fbytes);
    }
    t->req.dfield = nullptr;
    std::lock_guard<std::mutex> lk(s->m);
    if (s->fatal != HJR_OK) return s->fatal;
    // an instance keeps its grid and model; its first request brings l
    auto sh = s->shape.find(req->instance_id);
    if (sh != s->shape.end()) {
        const hjr_grid& h = sh->second.first;
        bool same = h.ndim == g.ndim && sh->second.second == req->dyn.kind;
        for (int i = 0; same && i < g.ndim; i++)
            same = h.n[i] == g.n[i] && h.lo[i] == g.lo[i] && h.hi[i] == g.hi[i];
        if (!same) return HJR_EINVAL;
    } else if (!req->l) {
        return HJR_EINVAL;
    }
    const size_t table = Engine::table_bytes(s->cfg.max_active, s->cfg.chunk);
    if (align256(table) + s->instance_bytes(g) + s->work_bytes(g) + align256(fbytes) > s->budget)
        return HJR_ENOMEM;
    if (req->l) {
        t->l_host.resize(bytes);
        std::memcpy(t->l_host.data(), req->l, bytes);
    }
    t->req.l = nullptr;
    t->id = s->next_ticket++;
    *ticket = t->id;
    s->pending[req->instance_id]++;
    s->shape[req->instance_id] = {g, req->dyn.kind};
    s->queue.push_back(t->id);
    s->tickets[t->id] = std::move(t);
    s->cv_work.notify_all();
    return HJR_OK;
}

static hjr_status poll_locked(hjr_server* s, uint64_t ticket, hjr_reply* reply)
{
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return HJR_ENOTFOUND;
    if (!it->second->done) return HJR_EBUSY;
    if (reply) *reply = it->second->reply;
    return HJR_OK;
}

hjr_status hjr_server_poll(hjr_server* s, uint64_t ticket, hjr_reply* reply)
{
    if (!s) return HJR_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    return poll_locked(s, ticket, reply);
}

hjr_status hjr_server_wait(hjr_server* s, uint64_t ticket, double timeout_ms, hjr_reply* reply)
{
    if (!s) return HJR_EINVAL;
    std::unique_lock<std::mutex> lk(s->m);
    auto ready = [&] {
        auto it = s->tickets.find(ticket);
        return it == s->tickets.end() || it->second->done;
    };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, ready);
    else
        s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready);
    return poll_locked(s, ticket, reply);
}

hjr_status hjr_server_read_value(hjr_server* s, uint64_t instance_id, void* dst, size_t bytes)
{
    if (!s || !dst) return HJR_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    auto ii = s->inst.find(instance_id);
    if (ii == s->inst.end() || !ii->second.has_value) return HJR_ENOTFOUND;
    const size_t need = grid_size(ii->second.grid) * s->esz();
    if (bytes < need) return HJR_EINVAL;
    if (hipMemcpyAsync(dst, ii->second.V_res, need, hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return HJR_EDEVICE;
    return HJR_OK;
}

hjr_status hjr_server_memory(hjr_server* s, size_t* used, size_t* budget)
{
    if (!s) return HJR_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    if (used) *used = s->used;
    if (budget) *budget = s->budget;
    return HJR_OK;
}

hjr_status hjr_server_destroy(hjr_server* s)
{
    if (!s) return HJR_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    hjr_status st = s->fatal;
    s->eng.reset();
    (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->inst) {
        if (kv.second.l) (void)hipFree(kv.second.l);
        if (kv.second.V_res) (void)hipFree(kv.second.V_res);
    }
    for (auto& kv : s->cache)
        for (void* p : kv.second) (void)hipFree(p);
    for (auto& kv : s->tickets) {
        Ticket& t = *kv.second;
        if (t.V_work) (void)hipFree(t.V_work);
        if (t.Vhat) (void)hipFree(t.Vhat);
        if (t.table) (void)hipFree(t.table);
        if (t.field) (void)hipFree(t.field);
    }
    (void)hipStreamDestroy(s->stream);
    delete s;
    return st;
}

}  // extern "C"
