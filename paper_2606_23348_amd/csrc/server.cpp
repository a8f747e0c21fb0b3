// server.cpp -- the served form of the batched Generals.io step: an
// environment server with continuous batching over a caller-provided device
// arena (see generals.h).
//
// Threads: client threads call open / submit / wait / close; one scheduler
// thread owns every launch.  It drains the request queue, puts the requests
// of all groups that are not on the GPU into one launch of k_serve (a table
// of requests, one workgroup per env), keeps up to n_launch_streams launches
// in flight on their own streams, polls their completion events and wakes
// the waiting clients.  Requests that arrive while launches run form the
// next launch as soon as a stream frees up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
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

#include "../../include/generals.h"
#include "internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

int64_t now_ns() { return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch()).count(); }

// Test-and-test-and-set lock for the server state.  Its critical sections
// last microseconds and are taken by the scheduler once per launch and by
// every client thread once per batch of submissions; with a sleeping mutex
// each contended hand-over costs the waiter a futex wake-up of tens of
// microseconds, which the scheduler paid on every launch.  A waiter spins
// (with the pause hint), then yields its core.
class SpinLock {
public:
    void lock()
    {
        for (int spins = 0;;) {
            if (!held_.exchange(true, std::memory_order_acquire)) return;
            while (held_.load(std::memory_order_relaxed)) {
                if (++spins < 2048) __builtin_ia32_pause();
                else std::this_thread::yield();
            }
        }
    }
    bool try_lock() { return !held_.load(std::memory_order_relaxed) && !held_.exchange(true, std::memory_order_acquire); }
    void unlock() { held_.store(false, std::memory_order_release); }

private:
    std::atomic<bool> held_{false};
};
using Lock = std::unique_lock<SpinLock>;
using Guard = std::lock_guard<SpinLock>;

// First-fit allocator over [0, size) of the arena, 256-byte granules.
class Arena {
  public:
    void init(uint64_t size) { free_.clear(); free_[0] = size; size_ = size; used_ = 0; }
    bool alloc(uint64_t n, uint64_t *off)
    {
        n = (n + 255) & ~uint64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        n = (n + 255) & ~uint64_t(255);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
        }
    }
    uint64_t used() const { return used_; }
    uint64_t size() const { return size_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_ = 0, used_ = 0;
};

// Latency histogram of fixed size: values in nanoseconds, exact below 64,
// then 32 buckets per power of two (a bucket spans 1/32 of its lower bound,
// so a quantile read at the bucket middle is within 1.6% of the sample).
class LatHist {
  public:
    static constexpr int kSub = 32, kTop = 46;         // up to 2^46 ns (about 19 hours)
    static constexpr int kBuckets = 64 + (kTop - 6) * kSub;
    void clear()
    {
        std::fill(n_, n_ + kBuckets, 0ull);
        count_ = 0;
        sum_ns_ = 0.0;
        max_ns_ = 0;
    }
    void add(int64_t ns)
    {
        const uint64_t v = ns < 0 ? 0 : (uint64_t)ns;
        n_[index(v)] += 1;
        count_ += 1;
        sum_ns_ += (double)v;
        max_ns_ = std::max(max_ns_, v);
    }
    uint64_t count() const { return count_; }
    double mean_us() const { return count_ ? sum_ns_ / (double)count_ / 1e3 : 0.0; }
    double max_us() const { return (double)max_ns_ / 1e3; }
    // q-quantile (0 < q <= 1): the middle of the bucket holding the
    // ceil(q * count)-th smallest sample, in microseconds
    double quantile_us(double q) const
    {
        if (count_ == 0) return 0.0;
        uint64_t rank = (uint64_t)std::ceil(q * (double)count_);
        if (rank < 1) rank = 1;
        uint64_t acc = 0;
        for (int i = 0; i < kBuckets; ++i) {
            acc += n_[i];
            if (acc >= rank) return mid(i) / 1e3;
        }
        return max_us();
    }

  private:
    static int index(uint64_t v)
    {
        if (v < 64) return (int)v;
        int e = 63 - __builtin_clzll(v);                // 2^e <= v < 2^(e+1), e >= 6
        if (e >= kTop) return kBuckets - 1;
        return 64 + (e - 6) * kSub + (int)((v >> (e - 5)) & (kSub - 1));
    }
    static double mid(int i)
    {
        if (i < 64) return (double)i;
        const int e = 6 + (i - 64) / kSub, m = (i - 64) % kSub;
        const double lo = std::ldexp((double)(kSub + m), e - 5), width = std::ldexp(1.0, e - 5);
        return lo + width / 2.0;
    }
    uint64_t n_[kBuckets] = {};
    uint64_t count_ = 0;
    double sum_ns_ = 0.0;
    uint64_t max_ns_ = 0;
};

struct Group {
    uint64_t id = 0;
    gen_pool *pool = nullptr;
    int32_t n_envs = 0;
    int32_t actor = 0;
    uint64_t actor_seed = 0;
    uint64_t off_state = 0, off_obs = 0, off_act = 0, off_rew = 0, off_done = 0;
    uint64_t sz_state = 0, sz_obs = 0, sz_act = 0, sz_done = 0;
    enum Phase { PENDING, ADMITTING, OPEN } phase = PENDING;   // waiting for memory, maps being made, steppable
    bool busy = false;          // a request of this group is in a launch, or it is not OPEN yet
    bool closing = false;
    bool failed = false;        // its admission failed (map generation); its tickets fail
    int waiters = 0;            // clients blocked on cv (close waits for them to leave)
    std::condition_variable_any cv; // completion of this group's tickets
    // requests finished (lock-free progress check), on a cache line of its
    // own: client threads poll it while the scheduler updates the fields above
    alignas(64) std::atomic<uint64_t> completed{0};
    alignas(64) gen::ServeReq req{};   // its request record (filled once its buffers are carved)
    uint32_t tidx = 0;                 // its record's index in the device table of group records
};

// A ticket lives in a ring slot (id & mask) until it is collected or
// 2^18 newer tickets have been issued; a pending ticket is never
// overwritten.  Its group pointer is valid while the ticket is pending:
// a group is closed only after its queued tickets were failed and its work
// in flight finished.
struct Ticket {
    uint64_t id = 0;            // 0: free slot
    Group *g = nullptr;
    int64_t t_submit = 0;
    int status = 0;             // 1 pending, 0 done, <0 failed
};
constexpr uint64_t kTicketRing = 1ull << 18;

struct QEntry {                 // a queued request
    uint64_t ticket;
    Group *g;                   // valid while the ticket is pending
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<std::pair<uint64_t, Group *>> reqs;    // (ticket, group) of the launch
    gen::ServeLaunch la{};                             // the launch's kernel argument
    uint64_t envs = 0;
};

}  // namespace

struct gen_server {
    uint8_t *arena = nullptr;
    uint64_t arena_bytes = 0;
    int device = 0;
    uint32_t max_batch_envs = 0;
    uint32_t max_reqs = 0;
    // batching window while another launch is in flight (gen_server_set_batching)
    int64_t min_batch_envs = 0;                        // 0: a quarter of the open envs
    int64_t max_wait_us = 100;
    int64_t open_envs = 0;                             // envs of the open groups
    Arena alloc;
    SpinLock mu;
    std::condition_variable_any cv_sched;
    std::atomic<bool> sched_idle{false};              // the scheduler sleeps on cv_sched
    std::unordered_map<uint64_t, std::unique_ptr<Group>> groups;
    std::vector<Ticket> ring = std::vector<Ticket>(kTicketRing);   // tickets by id & (kTicketRing - 1)
    std::deque<QEntry> queue;                          // pending requests, arrival order
    std::vector<Slot> slots;
    uint64_t d_groups_off = 0;                         // device table of group records (in the arena)
    std::vector<uint32_t> free_tidx;                   // its free entries
    uint64_t next_group = 1, next_ticket = 1;
    std::thread sched;
    std::atomic<bool> stop{false};
    std::atomic<int64_t> n_queued{0};                  // requests in `queue` (lock-free hint)
    std::atomic<uint64_t> n_submitted{0};              // submits and admissions so far (lock-free hint:
                                                       // either can make a waiting request launchable)
    std::string error;                                 // sticky scheduler error
    // stats
    std::deque<uint64_t> pending;                      // groups waiting for memory, in order of arrival
    uint64_t capacity = 0;                             // arena bytes left for groups (after the request tables)
    uint64_t st_requests = 0, st_frames = 0, st_launches = 0, st_queued = 0, st_launch_envs = 0;
    LatHist lat;
};

namespace {

int sfail(int code, const std::string &msg) { return gen::set_error(code, msg.c_str()); }

Ticket *ticket_of(gen_server &s, uint64_t tk)
{
    Ticket &t = s.ring[tk & (kTicketRing - 1)];
    return (tk != 0 && t.id == tk) ? &t : nullptr;
}

// A new pending ticket of group g (lock held); 0 if its ring slot still
// holds a pending ticket 2^18 tickets older.
uint64_t new_ticket(gen_server &s, Group *g)
{
    const uint64_t tk = s.next_ticket;
    Ticket &t = s.ring[tk & (kTicketRing - 1)];
    if (t.id != 0 && t.status == 1) return 0;
    s.next_ticket += 1;
    t.id = tk;
    t.g = g;
    t.t_submit = now_ns();
    t.status = 1;
    return tk;
}

// Fail every queued request of group g with `status` (lock held).
void fail_queued(gen_server &s, const Group *g, int status)
{
    for (const QEntry &q : s.queue) {
        Ticket *t = ticket_of(s, q.ticket);
        if (t != nullptr && t->status == 1 && q.g == g) t->status = status;
    }
}

void complete_slot(gen_server &s, Slot &sl, int status)
{
    const int64_t t = now_ns();
    for (auto &[tk, g] : sl.reqs) {
        Ticket *tp = ticket_of(s, tk);
        if (tp != nullptr) {
            tp->status = status;
            if (status == 0) s.lat.add(t - tp->t_submit);
        }
        g->busy = false;                 // a group in a launch is never closed before it finishes
        if (status == 0) {
            s.st_requests += 1;
            s.st_frames += (uint64_t)g->n_envs;
        }
        g->completed.fetch_add(1, std::memory_order_release);
        if (g->waiters > 0 || g->closing) g->cv.notify_all();   // a waiting client or close
    }
    sl.reqs.clear();
    sl.busy = false;
}

void fill_req(const gen_server &s, const Group &g, gen::ServeReq *r)
{
    const gen_pool &pl = *g.pool;
    std::memset(r, 0, sizeof *r);
    r->off_desc = g.off_state + pl.off_desc;
    r->off_sc = g.off_state + pl.off_scalars;
    r->off_owner = g.off_state + pl.off_owner;
    r->off_type = g.off_state + pl.off_type;
    r->off_army = g.off_state + pl.off_army;
    r->off_actions = g.off_act;
    r->off_rewards = g.off_rew;
    r->off_dones = g.off_done;
    r->off_obs = g.off_obs;
    r->seed = pl.seed;
    r->env_base = pl.env_base;
    r->actor_seed = g.actor_seed;
    r->prm = gen::prm_of(pl.common);
    r->n_envs = (uint32_t)pl.n;
    r->actor = g.actor ? 1u : 0u;
    // one shape and one set of settings for the whole group, envs in their
    // own order: the kernel derives every env's descriptor from the first
    const gen::PoolDesc &d0 = pl.desc[0];
    const uint32_t cells = pl.n > 1 ? pl.desc[1].cell_off : 0, ob16 = pl.n > 1 ? pl.desc[1].obs_off16 : 0;
    bool uni = true;
    for (int32_t i = 0; i < pl.n && uni; ++i) {
        const gen::PoolDesc &d = pl.desc[(size_t)i];
        uni = pl.order[(size_t)i] == (uint32_t)i && d.H == d0.H && d.W == d0.W && d.mode == d0.mode && d.P == d0.P &&
              d.cmin == d0.cmin && d.cmax == d0.cmax && d.dmin == d0.dmin && d.env == (uint32_t)i &&
              d.cell_off == (uint32_t)i * cells && d.obs_off16 == (uint32_t)i * ob16 &&
              d.act_off == (uint32_t)i * d0.P;
    }
    r->tmpl = d0;
    r->uniform = uni ? 1u : 0u;
    r->cells_per_env = cells;
    r->obs16_per_env = ob16;
    (void)s;
}

// The five buffers of a group carved out of the arena (lock held); false
// (nothing kept) if they do not fit now.
bool carve(gen_server &s, Group &g)
{
    uint64_t o[5];
    const uint64_t sz[5] = {g.sz_state, g.sz_obs, g.sz_act, g.sz_act, g.sz_done};
    int k = 0;
    for (; k < 5; ++k)
        if (!s.alloc.alloc(sz[k], &o[k])) break;
    if (k < 5) {
        for (int j = 0; j < k; ++j) s.alloc.release(o[j], sz[j]);
        return false;
    }
    g.off_state = o[0];
    g.off_obs = o[1];
    g.off_act = o[2];
    g.off_rew = o[3];
    g.off_done = o[4];
    fill_req(s, g, &g.req);
    return true;
}

void uncarve(gen_server &s, const Group &g)
{
    const uint64_t sz[5] = {g.sz_state, g.sz_obs, g.sz_act, g.sz_act, g.sz_done};
    const uint64_t o[5] = {g.off_state, g.off_obs, g.off_act, g.off_rew, g.off_done};
    for (int j = 0; j < 5; ++j) s.alloc.release(o[j], sz[j]);
}

uint64_t group_bytes(const Group &g)
{
    auto a = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
    return a(g.sz_state) + a(g.sz_obs) + 2 * a(g.sz_act) + a(g.sz_done);
}

// Generate a carved group's first maps on a stream of its own (blocking;
// called without the lock).
int make_maps(gen_server &s, Group &g)
{
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    int rc = GEN_OK;
    if (e == hipSuccess) {
        // the group's record in the device table, read by every launch of its requests
        e = hipMemcpyAsync(reinterpret_cast<gen::ServeReq *>(s.arena + s.d_groups_off) + g.tidx, &g.req,
                           sizeof(gen::ServeReq), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            rc = gen_pool_reset(g.pool, s.arena + g.off_state, g.sz_state, s.arena + g.off_obs,
                            g.actor ? reinterpret_cast<int32_t *>(s.arena + g.off_act) : nullptr, g.actor_seed, st);
        if (rc == GEN_OK) e = hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    if (e != hipSuccess) return gen::set_error(GEN_EHIP, hipGetErrorString(e));
    return rc;
}

// Groups waiting for memory are admitted in order of arrival as long as
// the first of them fits (a large group is not overtaken by smaller ones).
// Called without the lock, after memory was released.
void admit_pending(gen_server &s)
{
    std::vector<Group *> todo;
    {
        Guard lk(s.mu);
        while (!s.pending.empty()) {
            auto it = s.groups.find(s.pending.front());
            if (it == s.groups.end() || it->second->phase != Group::PENDING) {
                s.pending.pop_front();
                continue;
            }
            Group &g = *it->second;
            if (!carve(s, g)) break;
            g.phase = Group::ADMITTING;
            s.pending.pop_front();
            todo.push_back(&g);              // stays in the map: close waits while busy
        }
    }
    for (Group *g : todo) {
        const int rc = make_maps(s, *g);
        Guard lk(s.mu);
        g->phase = Group::OPEN;
        g->busy = false;
        if (rc == GEN_OK) {
            s.open_envs += g->n_envs;
        } else {
            g->failed = true;
            uncarve(s, *g);
            fail_queued(s, g, GEN_EHIP);
        }
        g->cv.notify_all();
    }
    if (!todo.empty()) {
        // requests already queued for these groups can launch now
        s.n_submitted.fetch_add(1, std::memory_order_release);
        s.cv_sched.notify_one();
    }
}

void scheduler(gen_server *sp)
{
    gen_server &s = *sp;
    (void)hipSetDevice(s.device);
    const size_t ns = s.slots.size();
    uint64_t last_submits = UINT64_MAX;   // submits seen by the last attempt that launched nothing
    int64_t retry_at = INT64_MAX;         // when that attempt's batching window closes
    while (true) {
        // Completions are polled without the lock (only this thread touches
        // the slots), and the lock is taken only when there is something to
        // do, so client threads are not starved while launches run.
        int n_busy = 0;
        bool done[4] = {false, false, false, false};
        hipError_t qs[4] = {hipSuccess, hipSuccess, hipSuccess, hipSuccess};
        bool any_done = false;
        for (size_t i = 0; i < ns; ++i) {
            Slot &sl = s.slots[i];
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) { ++n_busy; continue; }
            done[i] = true;
            qs[i] = q;
            any_done = true;
        }
        const bool queued = s.n_queued.load(std::memory_order_acquire) > 0;
        const uint64_t submits = s.n_submitted.load(std::memory_order_acquire);
        const bool stopping = s.stop.load();
        const bool try_launch =
            n_busy < (int)ns && queued && (submits != last_submits || now_ns() >= retry_at || stopping);
        if (!any_done && !try_launch) {
            if (stopping && n_busy == 0) {
                // shutting down: leave once nothing more can be launched
                Guard g(s.mu);
                for (auto it = s.queue.begin(); it != s.queue.end();) {
                    const Ticket *t = ticket_of(s, it->ticket);
                    if (t == nullptr || t->status != 1) {
                        it = s.queue.erase(it);
                        s.n_queued.fetch_sub(1, std::memory_order_release);
                    } else {
                        ++it;
                    }
                }
                if (s.queue.empty() || !s.error.empty()) break;
            }
            if (n_busy > 0 || queued) {
                // work pending: keep polling (a timed sleep overshoots by tens
                // of microseconds, which every request's latency would pay)
                std::this_thread::yield();
            } else {
                Lock lk(s.mu);
                s.sched_idle.store(true, std::memory_order_release);
                s.cv_sched.wait_for(lk, std::chrono::milliseconds(5),
                                    [&] { return s.n_queued.load() > 0 || s.stop.load(); });
                s.sched_idle.store(false, std::memory_order_release);
            }
            continue;
        }
        Lock lk(s.mu);
        for (size_t i = 0; i < ns; ++i) {
            if (!done[i]) continue;
            if (qs[i] == hipSuccess) {
                complete_slot(s, s.slots[i], 0);
            } else {
                s.error = std::string("launch failed: ") + hipGetErrorString(qs[i]);
                complete_slot(s, s.slots[i], GEN_EHIP);
            }
        }
        // form a launch from the queue: every request whose group is free
        Slot *free_slot = nullptr;
        for (auto &sl : s.slots)
            if (!sl.busy) { free_slot = &sl; break; }
        bool launch_now = free_slot && !s.queue.empty() && s.error.empty();
        retry_at = INT64_MAX;
        if (launch_now) {
            // Launch when no other open group can still join (every group is
            // either on the GPU or has a request waiting), when the ready
            // requests reach the batch size, or when the oldest has waited
            // max_wait_us.  Closed-loop clients then settle into cohorts that
            // alternate between the GPU and the queue.
            int64_t ready = 0, oldest = INT64_MAX, inflight = 0;
            for (const QEntry &q : s.queue) {
                const Ticket *t = ticket_of(s, q.ticket);
                if (t == nullptr || t->status != 1 || q.g->busy) continue;
                ready += q.g->n_envs;
                oldest = std::min(oldest, t->t_submit);
            }
            for (const auto &x : s.slots)
                if (x.busy) inflight += (int64_t)x.envs;
            const int64_t idle = s.open_envs - inflight - ready;
            const int64_t want = s.min_batch_envs > 0 ? s.min_batch_envs : std::max<int64_t>(1, s.open_envs / 4);
            const int64_t deadline = oldest == INT64_MAX ? INT64_MAX : oldest + s.max_wait_us * 1000;
            launch_now = ready > 0 && (idle <= 0 || ready >= want || now_ns() >= deadline || stopping);
            if (!launch_now && ready > 0) retry_at = deadline;
        }
        uint32_t n_req = 0;
        if (launch_now) {
            Slot &sl = *free_slot;
            uint32_t wg = 0, lds = 0;
            bool all_uni = true;
            for (auto it = s.queue.begin(); it != s.queue.end() && n_req < s.max_reqs;) {
                Ticket *tk = ticket_of(s, it->ticket);
                if (tk == nullptr || tk->status != 1) {
                    it = s.queue.erase(it);
                    s.n_queued.fetch_sub(1, std::memory_order_release);
                    continue;
                }
                Group &g = *it->g;
                if (g.closing) {
                    tk->status = GEN_ENOTFOUND;
                    it = s.queue.erase(it);
                    s.n_queued.fetch_sub(1, std::memory_order_release);
                    continue;
                }
                if (g.busy || (s.max_batch_envs && n_req > 0 && wg + (uint32_t)g.n_envs > s.max_batch_envs)) { ++it; continue; }
                g.busy = true;
                sl.la.idx[n_req] = (uint16_t)g.tidx;
                sl.la.first[n_req] = wg;
                sl.reqs.emplace_back(it->ticket, &g);
                wg += (uint32_t)g.n_envs;
                lds = std::max(lds, g.pool->lds_per_wave);
                all_uni = all_uni && g.req.uniform != 0;
                ++n_req;
                it = s.queue.erase(it);
                s.n_queued.fetch_sub(1, std::memory_order_release);
            }
            if (n_req > 0) {
                sl.busy = true;
                sl.envs = wg;
                s.st_launches += 1;
                s.st_launch_envs += wg;
                sl.la.n_req = n_req;
                lk.unlock();
                hipError_t e = gen::launch_serve(sl.la, wg, lds, all_uni, sl.stream);
                if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
                if (e != hipSuccess) {
                    lk.lock();
                    s.error = std::string("launch failed: ") + hipGetErrorString(e);
                    complete_slot(s, sl, GEN_EHIP);
                }
            }
        }
        last_submits = n_req > 0 ? UINT64_MAX : submits;
    }
}

}  // namespace

extern "C" {

int gen_server_create(void *d_arena, uint64_t arena_bytes, int32_t n_launch_streams, int32_t max_batch_envs,
                      gen_server **out)
{
    if (out == nullptr) return sfail(GEN_EINVAL, "out is NULL");
    *out = nullptr;
    if (d_arena == nullptr || (reinterpret_cast<uintptr_t>(d_arena) & 255)) return sfail(GEN_EINVAL, "arena must be 256-byte aligned");
    if (n_launch_streams < 1 || n_launch_streams > 4) return sfail(GEN_EINVAL, "n_launch_streams must be 1..4");
    if (max_batch_envs < 0) return sfail(GEN_EINVAL, "max_batch_envs must be >= 0");
    auto s = std::make_unique<gen_server>();
    s->arena = static_cast<uint8_t *>(d_arena);
    s->arena_bytes = arena_bytes;
    s->max_batch_envs = (uint32_t)max_batch_envs;
    s->max_reqs = gen::kServeMaxReqs;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, d_arena) != hipSuccess) return sfail(GEN_EINVAL, "arena is not device memory");
    s->device = attr.device;
    (void)hipSetDevice(s->device);
    s->alloc.init(arena_bytes);
    const uint64_t table_bytes = (uint64_t)gen::kServeMaxGroups * sizeof(gen::ServeReq);
    if (!s->alloc.alloc(table_bytes, &s->d_groups_off)) return sfail(GEN_EBUDGET, "arena too small for the group table");
    s->free_tidx.resize(gen::kServeMaxGroups);
    for (uint32_t i = 0; i < gen::kServeMaxGroups; ++i) s->free_tidx[i] = gen::kServeMaxGroups - 1 - i;
    s->slots.resize((size_t)n_launch_streams);
    for (auto &sl : s->slots) {
        sl.la.arena = s->arena;
        sl.la.groups = reinterpret_cast<const gen::ServeReq *>(s->arena + s->d_groups_off);
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
            return sfail(GEN_EHIP, "stream or event creation failed");
    }
    s->capacity = arena_bytes - s->alloc.used();
    s->sched = std::thread(scheduler, s.get());
    *out = s.release();
    return GEN_OK;
}

int gen_server_destroy(gen_server *s)
{
    if (s == nullptr) return GEN_OK;
    {
        Guard lk(s->mu);
        // groups still waiting for memory will not be admitted: their
        // requests fail, so the scheduler can drain the rest and stop
        for (uint64_t id : s->pending) {
            auto it = s->groups.find(id);
            if (it == s->groups.end()) continue;
            fail_queued(*s, it->second.get(), GEN_ENOTFOUND);
            it->second->cv.notify_all();
        }
        s->pending.clear();
        s->stop = true;
    }
    s->cv_sched.notify_all();
    if (s->sched.joinable()) s->sched.join();
    for (auto &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto &[id, g] : s->groups) gen_pool_destroy(g->pool);
    delete s;
    return GEN_OK;
}

int gen_server_open(gen_server *s, uint64_t seed, uint64_t env_base, int32_t n_envs, const gen_env_spec *h_specs,
                    const gen_params *common, int32_t actor, uint64_t actor_seed, uint64_t *group)
{
    if (s == nullptr || group == nullptr) return sfail(GEN_EINVAL, "server and group are required");
    gen_pool *pool = nullptr;
    int rc = gen_pool_create(seed, env_base, n_envs, h_specs, common, &pool);
    if (rc != GEN_OK) return sfail(rc, gen_last_error());
    auto g = std::make_unique<Group>();
    g->pool = pool;
    g->n_envs = n_envs;
    g->actor = actor;
    g->actor_seed = actor_seed;
    g->sz_state = pool->state_bytes;
    g->sz_obs = std::max<uint64_t>(pool->obs_bytes, 16);
    g->sz_act = pool->n_actions * 4;
    g->sz_done = (uint64_t)n_envs;
    g->busy = true;              // not steppable until its maps exist
    Group *gp = g.get();
    {
        Guard lk(s->mu);
        if (group_bytes(*gp) > s->capacity) {
            gen_pool_destroy(pool);
            return sfail(GEN_EINVAL, "group of " + std::to_string(n_envs) + " envs needs " +
                                         std::to_string(group_bytes(*gp)) + " bytes, more than the arena holds");
        }
        if (s->free_tidx.empty()) {
            gen_pool_destroy(pool);
            return sfail(GEN_EBUSY, std::to_string(gen::kServeMaxGroups) + " groups are open already");
        }
        gp->tidx = s->free_tidx.back();
        s->free_tidx.pop_back();
        gp->id = s->next_group++;
        *group = gp->id;
        const bool now = s->pending.empty() && carve(*s, *gp);
        gp->phase = now ? Group::ADMITTING : Group::PENDING;
        s->groups[gp->id] = std::move(g);
        if (!now) {
            // queued: admitted by a later close that frees enough memory
            s->pending.push_back(gp->id);
            s->st_queued += 1;
            return sfail(GEN_EBUDGET, "group " + std::to_string(gp->id) + " of " + std::to_string(n_envs) +
                                          " envs queued until memory frees up");
        }
    }
    rc = make_maps(*s, *gp);
    Guard lk(s->mu);
    if (rc != GEN_OK) {
        const std::string why = gen_last_error();
        uncarve(*s, *gp);
        gen_pool_destroy(gp->pool);
        s->free_tidx.push_back(gp->tidx);
        s->groups.erase(gp->id);        // its id was never returned with GEN_OK, so no one holds tickets
        return sfail(rc, why);
    }
    gp->phase = Group::OPEN;
    gp->busy = false;
    s->open_envs += gp->n_envs;
    return GEN_OK;
}

int gen_server_wait_admitted(gen_server *s, uint64_t group, int64_t timeout_us)
{
    if (s == nullptr) return sfail(GEN_EINVAL, "server is NULL");
    Lock lk(s->mu);
    auto it = s->groups.find(group);
    if (it == s->groups.end() || it->second->closing) return sfail(GEN_ENOTFOUND, "unknown group");
    Group &g = *it->second;
    const auto deadline = Clock::now() + std::chrono::microseconds(timeout_us < 0 ? 0 : timeout_us);
    g.waiters += 1;
    bool timed_out = false;
    while (g.phase != Group::OPEN && !g.closing) {
        if (timeout_us < 0) {
            g.cv.wait(lk);
        } else if (g.cv.wait_until(lk, deadline) == std::cv_status::timeout) {
            timed_out = g.phase != Group::OPEN && !g.closing;
            break;
        }
    }
    g.waiters -= 1;
    if (g.closing) {
        g.cv.notify_all();
        return sfail(GEN_ENOTFOUND, "group closed");
    }
    if (timed_out) return GEN_EBUSY;
    if (g.failed) return sfail(GEN_EHIP, "admission of the group failed");
    return GEN_OK;
}

int gen_server_buffers(gen_server *s, uint64_t group, gen_group_buffers *out)
{
    if (s == nullptr || out == nullptr) return sfail(GEN_EINVAL, "server and out are required");
    Guard lk(s->mu);
    auto it = s->groups.find(group);
    if (it == s->groups.end()) return sfail(GEN_ENOTFOUND, "unknown group");
    const Group &g = *it->second;
    if (g.failed) return sfail(GEN_EHIP, "admission of the group failed");
    if (g.phase != Group::OPEN) return sfail(GEN_EBUSY, "group not admitted yet");
    out->state_off = g.off_state;
    out->obs_off = g.off_obs;
    out->actions_off = g.off_act;
    out->rewards_off = g.off_rew;
    out->dones_off = g.off_done;
    out->obs_bytes = g.pool->obs_bytes;
    out->n_actions = g.pool->n_actions;
    out->n_envs = g.n_envs;
    out->reserved = 0;
    out->pool = g.pool;
    return GEN_OK;
}

int gen_server_submit(gen_server *s, uint64_t group, uint64_t *ticket)
{
    if (s == nullptr || ticket == nullptr) return sfail(GEN_EINVAL, "server and ticket are required");
    {
        Guard lk(s->mu);
        if (!s->error.empty()) return sfail(GEN_EHIP, s->error);
        auto it = s->groups.find(group);
        if (it == s->groups.end() || it->second->closing) return sfail(GEN_ENOTFOUND, "unknown group");
        if (it->second->failed) return sfail(GEN_EHIP, "admission of the group failed");
        const uint64_t tk = new_ticket(*s, it->second.get());
        if (tk == 0) return sfail(GEN_EBUSY, "too many requests pending");
        s->queue.push_back({tk, it->second.get()});
        s->n_queued.fetch_add(1, std::memory_order_release);
        s->n_submitted.fetch_add(1, std::memory_order_release);
        *ticket = tk;
    }
    if (s->sched_idle.load(std::memory_order_acquire)) s->cv_sched.notify_one();
    return GEN_OK;
}

int gen_server_wait(gen_server *s, uint64_t ticket, int64_t timeout_us)
{
    if (s == nullptr) return sfail(GEN_EINVAL, "server is NULL");
    Lock lk(s->mu);
    Ticket *t = ticket_of(*s, ticket);
    if (t == nullptr) return sfail(GEN_ENOTFOUND, "unknown ticket");
    if (t->status == 1) {
        Group &g = *t->g;                  // a pending ticket's group is open; close waits for waiters
        const auto deadline = Clock::now() + std::chrono::microseconds(timeout_us < 0 ? 0 : timeout_us);
        g.waiters += 1;
        bool timed_out = false;
        while (t->status == 1) {           // a pending ticket's slot is never reused
            if (timeout_us < 0) {
                g.cv.wait(lk);
            } else if (g.cv.wait_until(lk, deadline) == std::cv_status::timeout) {
                timed_out = t->status == 1;
                break;
            }
        }
        g.waiters -= 1;
        if (g.closing) g.cv.notify_all();
        if (timed_out) return GEN_EBUSY;
    }
    const int st = t->status;
    t->id = 0;                             // collected
    if (st != 0) return sfail(st, s->error.empty() ? "request failed" : s->error);
    return GEN_OK;
}

int gen_server_close(gen_server *s, uint64_t group)
{
    if (s == nullptr) return sfail(GEN_EINVAL, "server is NULL");
    {
        Lock lk(s->mu);
        auto it = s->groups.find(group);
        if (it == s->groups.end()) return sfail(GEN_ENOTFOUND, "unknown group");
        Group &g = *it->second;
        g.closing = true;
        fail_queued(*s, &g, GEN_ENOTFOUND);
        g.cv.notify_all();
        if (g.phase == Group::PENDING) {
            // never admitted: it holds no memory
            s->pending.erase(std::find(s->pending.begin(), s->pending.end(), group));
            while (g.waiters > 0) g.cv.wait(lk);
        } else {
            // in a launch or being admitted: wait for that to finish
            while (g.busy || g.waiters > 0) g.cv.wait(lk);
            if (!g.failed) {
                uncarve(*s, g);
                s->open_envs -= g.n_envs;
            }
        }
        gen_pool_destroy(g.pool);
        s->free_tidx.push_back(g.tidx);
        s->groups.erase(it);
    }
    admit_pending(*s);
    return GEN_OK;
}

int gen_server_set_batching(gen_server *s, int64_t min_batch_envs, int64_t max_wait_us)
{
    if (s == nullptr) return sfail(GEN_EINVAL, "server is NULL");
    if (min_batch_envs < 0 || max_wait_us < 0) return sfail(GEN_EINVAL, "min_batch_envs and max_wait_us must be >= 0");
    {
        Guard lk(s->mu);
        s->min_batch_envs = min_batch_envs;
        s->max_wait_us = max_wait_us;
    }
    s->cv_sched.notify_one();
    return GEN_OK;
}

int gen_server_report(gen_server *s, gen_server_stats *out, int32_t reset)
{
    if (s == nullptr || out == nullptr) return sfail(GEN_EINVAL, "server and out are required");
    Guard lk(s->mu);
    std::memset(out, 0, sizeof *out);
    out->requests = s->st_requests;
    out->frames = s->st_frames;
    out->launches = s->st_launches;
    for (const auto &[id, g] : s->groups) out->groups_open += (g->phase == Group::OPEN && !g->failed) ? 1u : 0u;
    out->groups_queued = s->st_queued;
    out->groups_pending = s->pending.size();
    out->arena_bytes = s->arena_bytes;
    out->bytes_in_use = s->alloc.used();
    out->envs_per_launch = s->st_launches ? (double)s->st_launch_envs / (double)s->st_launches : 0.0;
    out->lat_samples = s->lat.count();
    out->lat_p50_us = s->lat.quantile_us(0.50);
    out->lat_p99_us = s->lat.quantile_us(0.99);
    out->lat_mean_us = s->lat.mean_us();
    out->lat_max_us = s->lat.max_us();
    if (reset) {
        s->st_requests = s->st_frames = s->st_launches = s->st_launch_envs = s->st_queued = 0;
        s->lat.clear();
    }
    return GEN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- load generator
namespace {

constexpr int64_t kDriveWaitUs = 30000000;   // a request taking longer than this fails the run

struct ClientGroup {
    uint64_t id = 0;
    uint64_t ticket = 0;
    bool outstanding = false;
    int32_t steps = 0;
    int32_t spec_begin = 0, n_envs = 0;
    uint64_t env_base = 0;
    Group *g = nullptr;          // the server's group object (stable until closed)
    uint64_t mark = 0;           // its completion count when the request was submitted
};

Group *group_of(gen_server *s, uint64_t id)
{
    Guard lk(s->mu);
    auto it = s->groups.find(id);
    return it == s->groups.end() ? nullptr : it->second.get();
}

}  // namespace

extern "C" int gen_server_drive(gen_server *s, int32_t n_clients, int32_t groups_per_client, const int32_t *h_group_envs,
                                const gen_env_spec *h_specs, const gen_params *common, uint64_t seed,
                                uint64_t actor_seed, const double *h_gaps_us, int32_t gaps_per_client,
                                int64_t duration_us, int32_t steps_per_group, gen_server_stats *out)
{
    if (s == nullptr || out == nullptr || h_group_envs == nullptr || h_specs == nullptr || h_gaps_us == nullptr)
        return sfail(GEN_EINVAL, "missing argument");
    if (n_clients < 1 || groups_per_client < 1 || gaps_per_client < 1 || duration_us < 1)
        return sfail(GEN_EINVAL, "bad client configuration");
    const int32_t n_groups = n_clients * groups_per_client;
    std::vector<int32_t> spec_begin((size_t)n_groups + 1, 0);
    for (int32_t g = 0; g < n_groups; ++g) spec_begin[(size_t)g + 1] = spec_begin[(size_t)g] + h_group_envs[g];
    const uint64_t total_envs = (uint64_t)spec_begin[(size_t)n_groups];
    std::atomic<int> failure{0};
    std::atomic<uint64_t> reopen_base{total_envs};
    std::vector<std::vector<ClientGroup>> cg((size_t)n_clients);
    // open every group first (blocking map generation), then measure
    for (int32_t c = 0; c < n_clients && !failure; ++c) {
        for (int32_t k = 0; k < groups_per_client; ++k) {
            const int32_t g = c * groups_per_client + k;
            ClientGroup x;
            x.spec_begin = spec_begin[(size_t)g];
            x.n_envs = h_group_envs[g];
            x.env_base = (uint64_t)x.spec_begin;
            int rc = gen_server_open(s, seed, x.env_base, x.n_envs, h_specs + x.spec_begin, common, 1,
                                     actor_seed, &x.id);
            if (rc == GEN_EBUDGET) rc = gen_server_wait_admitted(s, x.id, kDriveWaitUs);   // queued for memory
            if (rc != GEN_OK) { failure = rc; break; }
            cg[(size_t)c].push_back(x);
        }
    }
    if (failure) return failure.load();
    for (auto &v : cg)
        for (auto &x : v) x.g = group_of(s, x.id);
    gen_server_stats tmp;
    gen_server_report(s, &tmp, 1);
    const auto t0 = Clock::now();
    const auto t_end = t0 + std::chrono::microseconds(duration_us);
    auto gap = [&](int32_t c, int32_t k) {
        return std::chrono::nanoseconds((int64_t)(h_gaps_us[(size_t)c * gaps_per_client + (k % gaps_per_client)] * 1000.0));
    };
    // The clients are logical: a few threads each run many of them as state
    // machines (timer fired -> previous request of the group finished ->
    // submit), polling completions lock-free, so the measurement is not
    // bounded by waking one OS thread per client.
    const int32_t n_threads = std::min<int32_t>(n_clients, 8);
    auto worker = [&](int32_t t) {
        struct Cl { int32_t c, gi, k; Clock::time_point next; };
        std::vector<Cl> cl;
        for (int32_t c = t; c < n_clients; c += n_threads) cl.push_back({c, 0, 1, t0 + gap(c, 0)});
        std::vector<Cl *> ready;
        ready.reserve(cl.size());
        while (!failure) {
            const auto now = Clock::now();
            if (now >= t_end) break;
            // 1. clients whose timer fired and whose group has no request on the GPU
            ready.clear();
            for (auto &x : cl) {
                if (x.next >= t_end || now < x.next) continue;
                ClientGroup &grp = cg[(size_t)x.c][(size_t)x.gi];
                if (grp.outstanding && grp.g->completed.load(std::memory_order_acquire) <= grp.mark) continue;
                ready.push_back(&x);
            }
            if (ready.empty()) {
                std::this_thread::yield();
                continue;
            }
            // 2. groups due for replacement are closed and reopened one by one
            for (Cl *x : ready) {
                ClientGroup &grp = cg[(size_t)x->c][(size_t)x->gi];
                if (steps_per_group <= 0 || grp.steps + (grp.outstanding ? 1 : 0) < steps_per_group) continue;
                if (grp.outstanding) {
                    const int rc = gen_server_wait(s, grp.ticket, kDriveWaitUs);
                    if (rc != GEN_OK) { failure = rc; break; }
                    grp.outstanding = false;
                    grp.steps += 1;
                }
                if (gen_server_close(s, grp.id) != GEN_OK) { failure = GEN_EHIP; break; }
                grp.env_base = reopen_base.fetch_add((uint64_t)grp.n_envs);
                int rc = gen_server_open(s, seed, grp.env_base, grp.n_envs, h_specs + grp.spec_begin, common,
                                         1, actor_seed, &grp.id);
                if (rc == GEN_EBUDGET) rc = gen_server_wait_admitted(s, grp.id, kDriveWaitUs);
                if (rc != GEN_OK) { failure = rc; break; }
                grp.g = group_of(s, grp.id);
                grp.steps = 0;
            }
            if (failure) break;
            // 3. collect the finished tickets and submit the next requests
            // under one lock acquisition for the whole batch
            {
                Guard lk(s->mu);
                if (!s->error.empty()) { failure = GEN_EHIP; break; }
                for (Cl *x : ready) {
                    ClientGroup &grp = cg[(size_t)x->c][(size_t)x->gi];
                    if (grp.outstanding) {
                        Ticket *t = ticket_of(*s, grp.ticket);
                        if (t == nullptr || t->status != 0) { failure = GEN_EHIP; break; }
                        t->id = 0;                  // collected
                        grp.outstanding = false;
                        grp.steps += 1;
                    }
                    if (grp.g->closing) { failure = GEN_ENOTFOUND; break; }
                    grp.mark = grp.g->completed.load(std::memory_order_acquire);
                    const uint64_t tk = new_ticket(*s, grp.g);
                    if (tk == 0) { failure = GEN_EBUSY; break; }
                    s->queue.push_back({tk, grp.g});
                    s->n_queued.fetch_add(1, std::memory_order_release);
                    s->n_submitted.fetch_add(1, std::memory_order_release);
                    grp.ticket = tk;
                    grp.outstanding = true;
                    x->gi = (x->gi + 1) % (int32_t)cg[(size_t)x->c].size();
                    x->next += gap(x->c, x->k++);
                }
            }
            if (s->sched_idle.load(std::memory_order_acquire)) s->cv_sched.notify_one();
        }
        for (auto &x : cl)
            for (auto &grp : cg[(size_t)x.c])
                if (grp.outstanding) { gen_server_wait(s, grp.ticket, kDriveWaitUs); grp.outstanding = false; }
    };
    std::vector<std::thread> th;
    th.reserve((size_t)n_threads);
    for (int32_t t = 0; t < n_threads; ++t) th.emplace_back(worker, t);
    for (auto &t : th) t.join();
    const double secs = std::chrono::duration<double>(Clock::now() - t0).count();
    gen_server_report(s, out, 1);
    out->wall_s = secs;
    for (auto &groups : cg)
        for (auto &x : groups) gen_server_close(s, x.id);
    if (failure) return failure.load();
    return GEN_OK;
}
