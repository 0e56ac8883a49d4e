// Serving loop: continuous batching of reconstruction and energy requests
// over many boxes, cutoffs and meshes on one GPU (see include/pwcoul.h).
//
// One scheduler thread owns every HIP call.  Each iteration it
//   1. reaps slots whose completion event has fired (results, latencies,
//      table references released, scratch budget returned),
//   2. admits queued requests in arrival order while a slot is free and the
//      HBM budget allows: the table is taken from the cache or planned,
//      priced (exact device bytes), evicted-for and built, then the request's
//      kernels are enqueued on the slot's stream followed by the copies of
//      the energies and of the error words into pinned host memory and an
//      event.
// A small reconstruction at the head of the queue (at most the table's
// direct-kernel size) takes along the later queued small reconstructions
// whose tables are resident, up to kDirectMaxJobs: one launch of the direct
// kernel serves them all, each job with its own table, precision, buffers
// and error word.  Otherwise a request that cannot be admitted for memory
// blocks the ones behind it, so the head is always served first and nothing
// starves.
#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <thread>

#include <sys/prctl.h>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "pwc_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// Table cache key: the three box sides, cutoff and every mesh field.
using Key = std::tuple<double, double, double, int, int, int, double, int, int, double>;

double side_y(const pwc_request &r) { return r.Ly > 0.0 ? r.Ly : r.L; }
double side_z(const pwc_request &r) { return r.Lz > 0.0 ? r.Lz : r.L; }

Key key_of(const pwc_request &r, const pwc_mesh &m) {
    return Key(r.L, side_y(r), side_z(r), r.n2max, m.kind, m.n_sub, m.ratio, m.q_sub, m.q_tail,
               m.alpha_c);
}

struct Cached {
    pwc_table *t = nullptr;
    size_t bytes = 0;
    int refs = 0;
    uint64_t last_use = 0;
};

struct Pending {
    uint64_t ticket;
    pwc_request r;
    pwc_mesh mesh;
    Clock::time_point t_submit;
};

struct Member {
    uint64_t ticket = 0;
    pwc_request r{};
    Cached *tab = nullptr;
    int built = 0;
    Clock::time_point t_submit;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    double *h_e = nullptr;     // pinned [2]
    // Error word per member, in mapped pinned host memory: cleared by the
    // host before the launch, set by the kernels, read by the host once the
    // slot's event has fired (no device copy either way).
    int *h_err = nullptr;      // [kDirectMaxJobs], host address
    int *d_err = nullptr;      // the same words, device address
    bool busy = false;
    bool direct = false;       // members share one direct-kernel launch
    std::vector<Member> members;
    size_t scratch = 0;
    Clock::time_point t_launch;
};

pwc_status from_hip(hipError_t e) {
    if (e == hipSuccess) return PWC_OK;
    if (e == hipErrorOutOfMemory) return PWC_ERR_NOMEM;
    return PWC_ERR_DEVICE;
}

}  // namespace

struct pwc_server {
    int device = 0;
    size_t budget = 0, used = 0;
    std::vector<Slot> slots;
    hipStream_t build_stream = nullptr;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> pending;
    std::unordered_map<uint64_t, pwc_result> finished;
    std::unordered_map<uint64_t, bool> known;   // submitted, not yet collected
    uint64_t next_ticket = 1;
    bool stopping = false;

    // scheduler-thread state
    std::map<Key, Cached> cache;
    uint64_t clock = 0;
    // plan of the queue head's table while it waits for memory
    pwc_table *planned = nullptr;
    pwc::TableSetup planned_su;
    Key planned_key{};
    std::atomic<size_t> resident_bytes{0};
    std::atomic<int> resident_tables{0};

    // statistics (guarded by mu)
    uint64_t submitted = 0, completed = 0, failed = 0, builds = 0, evictions = 0;
    uint64_t launches = 0, batched = 0;
    std::vector<double> latencies;
    double integrals = 0.0, pairs = 0.0;
    bool have_first = false;
    Clock::time_point t_first, t_last;

    std::thread worker;

    void run();
    bool reap();
    bool admit();
    void fail(const Pending &p, pwc_status st, double queue_ms, int built);
    void publish_residency();
    size_t scratch_bytes(const pwc::Table &t, const pwc_request &r) const;
    bool make_room(size_t need);
};

// Device scratch the request's kernels allocate on its table (stream-ordered
// allocations, priced from the path they take): none for the direct kernel
// or the fused node sums, the decoded stream for the node passes, the
// pair-sum partials for energies (kernel-table or node-sum grid).  Rounded
// up to 64 KiB.
size_t pwc_server::scratch_bytes(const pwc::Table &t, const pwc_request &r) const {
    size_t b = 0;
    if (r.kind == PWC_REQ_RECONSTRUCT)
        b = r.n <= t.direct_max ? 0 : pwc::reconstruct_scratch_bytes(t, r.n, static_cast<pwc_precision>(r.prec));
    else b = pwc::energies_scratch_bytes(t, r.n, static_cast<pwc_pair_algo>(r.algo));
    return (b + 65535) / 65536 * 65536;
}

// Evict unreferenced tables, least recently used first, until `need` more
// bytes fit in the budget.
bool pwc_server::make_room(size_t need) {
    while (used + need > budget) {
        auto victim = cache.end();
        for (auto it = cache.begin(); it != cache.end(); ++it)
            if (it->second.refs == 0 && (victim == cache.end() || it->second.last_use < victim->second.last_use))
                victim = it;
        if (victim == cache.end()) return false;
        used -= victim->second.bytes;
        pwc_table_destroy(victim->second.t);
        cache.erase(victim);
        publish_residency();
        std::lock_guard<std::mutex> lk(mu);
        ++evictions;
    }
    return true;
}

void pwc_server::publish_residency() {
    size_t b = 0;
    for (const auto &kv : cache) b += kv.second.bytes;
    resident_bytes.store(b);
    resident_tables.store(static_cast<int>(cache.size()));
}

void pwc_server::fail(const Pending &p, pwc_status st, double queue_ms, int built) {
    pwc_result res{};
    res.status = st;
    res.queue_ms = queue_ms;
    res.latency_ms = ms_between(p.t_submit, Clock::now());
    res.table_built = built;
    std::lock_guard<std::mutex> lk(mu);
    ++failed;
    finished[p.ticket] = res;
    cv_done.notify_all();
}

bool pwc_server::reap() {
    bool any = false;
    for (Slot &s : slots) {
        if (!s.busy) continue;
        const hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) continue;
        any = true;
        const auto now = Clock::now();
        for (size_t i = 0; i < s.members.size(); ++i) {
            Member &m = s.members[i];
            pwc_result res{};
            res.status = from_hip(q);
            if (res.status == PWC_OK && s.h_err[i]) res.status = PWC_ERR_RANGE;
            if (m.r.kind == PWC_REQ_ENERGIES) {
                res.e_h = s.h_e[0];
                res.e_x = s.h_e[1];
            }
            res.queue_ms = ms_between(m.t_submit, s.t_launch);
            res.latency_ms = ms_between(m.t_submit, now);
            res.table_built = m.built;
            m.tab->refs -= 1;
            std::lock_guard<std::mutex> lk(mu);
            finished[m.ticket] = res;
            if (res.status == PWC_OK) {
                ++completed;
                latencies.push_back(res.latency_ms);
                if (m.r.kind == PWC_REQ_RECONSTRUCT) integrals += static_cast<double>(m.r.n);
                else pairs += static_cast<double>(m.r.n) * static_cast<double>(m.r.n);
            } else {
                ++failed;
            }
            t_last = now;
        }
        used -= s.scratch;
        s.busy = false;
        s.members.clear();
        std::lock_guard<std::mutex> lk(mu);
        cv_done.notify_all();
    }
    return any;
}

bool pwc_server::admit() {
    bool any = false;
    for (;;) {
        Slot *slot = nullptr;
        for (Slot &s : slots)
            if (!s.busy) { slot = &s; break; }
        if (!slot) return any;
        Pending p;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (pending.empty()) return any;
            p = pending.front();
        }
        const Key key = key_of(p.r, p.mesh);
        size_t scratch = 0;
        auto it = cache.find(key);
        int built = 0;
        if (it == cache.end()) {
            pwc_status st = PWC_OK;
            if (!planned || planned_key != key) {
                if (planned) pwc_table_destroy(planned);
                planned = new (std::nothrow) pwc_table;
                planned_key = key;
                const double sides[3] = {p.r.L, side_y(p.r), side_z(p.r)};
                st = planned ? pwc::plan_table(sides, p.r.n2max, p.mesh, planned->t, planned_su)
                             : PWC_ERR_NOMEM;
            }
            if (st == PWC_OK) scratch = scratch_bytes(planned->t, p.r);
            if (st == PWC_OK && planned->t.bytes + scratch > budget) st = PWC_ERR_NOMEM;
            if (st == PWC_OK && p.r.kind == PWC_REQ_ENERGIES && p.r.algo == PWC_PAIR_KTABLE &&
                planned->t.kt_n == 0)
                st = PWC_ERR_ARG;
            if (st != PWC_OK) {
                if (planned) pwc_table_destroy(planned);
                planned = nullptr;
                { std::lock_guard<std::mutex> lk(mu); pending.pop_front(); }
                fail(p, st, 0.0, 0);
                any = true;
                continue;
            }
            if (!make_room(planned->t.bytes + scratch)) return any;   // wait for running requests
            pwc_table *h = planned;
            planned = nullptr;
            st = pwc::build_table(h->t, planned_su, build_stream);
            if (st != PWC_OK) {
                delete h;
                { std::lock_guard<std::mutex> lk(mu); pending.pop_front(); }
                fail(p, st, 0.0, 0);
                any = true;
                continue;
            }
            // The block may be a cached one up to 1/8 larger than planned:
            // count what the table holds, and evict for the difference.
            Cached c;
            c.t = h;
            c.bytes = std::max(h->t.bytes, h->t.block_bytes);
            it = cache.emplace(key, c).first;
            used += c.bytes;
            built = 1;
            it->second.refs += 1;
            if (used > budget) (void)make_room(0);
            it->second.refs -= 1;
            publish_residency();
            std::lock_guard<std::mutex> lk(mu);
            ++builds;
        } else {
            if (p.r.kind == PWC_REQ_ENERGIES && p.r.algo == PWC_PAIR_KTABLE && it->second.t->t.kt_n == 0) {
                { std::lock_guard<std::mutex> lk(mu); pending.pop_front(); }
                fail(p, PWC_ERR_ARG, 0.0, 0);
                any = true;
                continue;
            }
            scratch = scratch_bytes(it->second.t->t, p.r);
            if (it->second.bytes + scratch > budget) {   // can never fit beside its table
                { std::lock_guard<std::mutex> lk(mu); pending.pop_front(); }
                fail(p, PWC_ERR_NOMEM, 0.0, 0);
                any = true;
                continue;
            }
            it->second.refs += 1;                    // pin while making room
            const bool ok = make_room(scratch);
            it->second.refs -= 1;
            if (!ok) return any;
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            pending.pop_front();
        }
        Cached &c = it->second;
        c.refs += 1;
        c.last_use = ++clock;
        used += scratch;
        Slot &s = *slot;
        s.busy = true;
        s.scratch = scratch;
        s.t_launch = Clock::now();
        s.members.clear();
        Member head;
        head.ticket = p.ticket;
        head.r = p.r;
        head.tab = &c;
        head.built = built;
        head.t_submit = p.t_submit;
        s.members.push_back(head);
        const pwc::Table &t = c.t->t;
        s.direct = p.r.kind == PWC_REQ_RECONSTRUCT && p.r.n <= t.direct_max;
        hipError_t e = hipSuccess;
        // The table's construction (queued on the build stream) and the
        // caller's pending work on the request's buffers come first.
        auto wait_ready = [&](const pwc_request &r, const pwc::Table &tab) {
            if (e == hipSuccess) e = pwc::wait_ready(tab, s.stream);
            if (e == hipSuccess && r.ready_event)
                e = hipStreamWaitEvent(s.stream, static_cast<hipEvent_t>(r.ready_event), 0);
        };
        if (s.direct) {
            // Later queued small reconstructions on resident tables join the launch.
            {
                std::lock_guard<std::mutex> lk(mu);
                for (auto q = pending.begin(); q != pending.end() &&
                                               static_cast<int>(s.members.size()) < pwc::kDirectMaxJobs;) {
                    if (q->r.kind != PWC_REQ_RECONSTRUCT) { ++q; continue; }
                    auto ct = cache.find(key_of(q->r, q->mesh));
                    if (ct == cache.end() || q->r.n > ct->second.t->t.direct_max) { ++q; continue; }
                    Member m;
                    m.ticket = q->ticket;
                    m.r = q->r;
                    m.tab = &ct->second;
                    m.t_submit = q->t_submit;
                    ct->second.refs += 1;
                    ct->second.last_use = ++clock;
                    s.members.push_back(m);
                    q = pending.erase(q);
                }
            }
            pwc::DirectBatch b{};
            b.njobs = static_cast<int>(s.members.size());
            for (int i = 0; i < b.njobs; ++i) {
                const Member &m = s.members[i];
                b.job[i] = pwc::direct_job(m.tab->t->t, m.r.d_idx, m.r.n, m.r.d_out,
                                           static_cast<pwc_precision>(m.r.prec), s.d_err + i);
                wait_ready(m.r, m.tab->t->t);
            }
            std::memset(s.h_err, 0, sizeof(int) * b.njobs);
            if (e == hipSuccess) e = pwc::launch_direct(b, s.stream);
            for (const Member &m : s.members) pwc::note_use(m.tab->t->t, s.stream);
        } else {
            // The slot's own error word, not the table's: requests on one
            // table may run in several slots at once.
            wait_ready(p.r, t);
            s.h_err[0] = 0;
            if (e == hipSuccess && p.r.kind == PWC_REQ_RECONSTRUCT) {
                e = pwc::launch_reconstruct(t, p.r.d_idx, p.r.n, p.r.d_out,
                                            static_cast<pwc_precision>(p.r.prec), s.stream,
                                            nullptr, s.d_err);
            } else if (e == hipSuccess) {
                e = pwc::launch_energies(t, p.r.d_idx, p.r.d_f, p.r.n,
                                         static_cast<pwc_precision>(p.r.prec),
                                         static_cast<pwc_pair_algo>(p.r.algo), p.r.d_out, s.stream,
                                         s.d_err);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(s.h_e, p.r.d_out, 2 * sizeof(double), hipMemcpyDeviceToHost, s.stream);
            }
            pwc::note_use(t, s.stream);
        }
        if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
        if (e == hipSuccess) {
            std::lock_guard<std::mutex> lk(mu);
            ++launches;
            batched += s.members.size() - 1;
        } else {
            (void)hipStreamSynchronize(s.stream);
            s.busy = false;
            used -= scratch;
            for (const Member &m : s.members) {
                m.tab->refs -= 1;
                Pending fp;
                fp.ticket = m.ticket;
                fp.r = m.r;
                fp.t_submit = m.t_submit;
                fail(fp, from_hip(e), ms_between(m.t_submit, s.t_launch), m.built);
            }
            s.members.clear();
        }
        any = true;
    }
}

void pwc_server::run() {
    (void)hipSetDevice(device);
    // While requests run, the loop polls their events every 20 us; Linux's
    // default timer slack (50 us) would stretch each of those waits to about
    // 70 us, which is most of a small request's latency (p50 0.10 ms against
    // 0.07 ms with 1 us).
    (void)prctl(PR_SET_TIMERSLACK, 1000UL);
    for (;;) {
        const bool a = reap();
        const bool b = admit();
        bool idle_slots = true;
        for (const Slot &s : slots) idle_slots = idle_slots && !s.busy;
        std::unique_lock<std::mutex> lk(mu);
        if (stopping && pending.empty() && idle_slots) break;
        if (!a && !b) {
            if (idle_slots && pending.empty())
                cv_work.wait(lk, [&] { return stopping || !pending.empty(); });
            else
                cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

extern "C" {

pwc_status pwc_server_create(size_t hbm_budget_bytes, int max_inflight, pwc_server **out) {
    if (!out) return PWC_ERR_ARG;
    *out = nullptr;
    if (hbm_budget_bytes == 0 || max_inflight < 1 || max_inflight > 64) return PWC_ERR_ARG;
    pwc_server *s = new (std::nothrow) pwc_server;
    if (!s) return PWC_ERR_NOMEM;
    s->budget = hbm_budget_bytes;
    (void)hipGetDevice(&s->device);
    hipError_t e = hipStreamCreateWithFlags(&s->build_stream, hipStreamNonBlocking);
    s->slots.resize(max_inflight);
    for (Slot &sl : s->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&sl.h_e), 2 * sizeof(double));
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&sl.h_err), sizeof(int) * pwc::kDirectMaxJobs,
                              hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&sl.d_err), sl.h_err, 0);
    }
    if (e != hipSuccess) {
        for (Slot &sl : s->slots) {
            if (sl.h_e) (void)hipHostFree(sl.h_e);
            if (sl.h_err) (void)hipHostFree(sl.h_err);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        if (s->build_stream) (void)hipStreamDestroy(s->build_stream);
        delete s;
        return from_hip(e);
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return PWC_OK;
}

pwc_status pwc_server_submit(pwc_server *s, const pwc_request *r, uint64_t *ticket) {
    if (!s || !r || !ticket) return PWC_ERR_ARG;
    if (r->kind != PWC_REQ_RECONSTRUCT && r->kind != PWC_REQ_ENERGIES) return PWC_ERR_ARG;
    if (!(r->L > 0.0) || !std::isfinite(r->L) || r->n2max < 1 || r->n2max > PWC_MAX_N2MAX || r->n < 0) return PWC_ERR_ARG;
    if (!(r->Ly >= 0.0) || !(r->Lz >= 0.0) || !std::isfinite(r->Ly) || !std::isfinite(r->Lz))
        return PWC_ERR_ARG;
    if (!pwc::valid_precision(r->prec)) return PWC_ERR_ARG;
    if (r->kind == PWC_REQ_ENERGIES && r->prec == PWC_FP32) return PWC_ERR_ARG;   // reconstruction only
    if (!r->d_out || (r->n > 0 && !r->d_idx)) return PWC_ERR_ARG;
    if (r->kind == PWC_REQ_RECONSTRUCT && (reinterpret_cast<uintptr_t>(r->d_idx) & 15))
        return PWC_ERR_ARG;
    if (r->kind == PWC_REQ_ENERGIES) {
        if (r->algo < PWC_PAIR_AUTO || r->algo > PWC_PAIR_KTABLE || r->n > (1 << 17))
            return PWC_ERR_ARG;
    }
    pwc_mesh m{};
    if (r->has_mesh) {
        int q = 0;
        if (!pwc::mesh_valid(r->mesh, &q)) return PWC_ERR_ARG;
        m = r->mesh;
    } else if (pwc_mesh_default(r->n_nodes, &m) != PWC_OK) {
        return PWC_ERR_ARG;
    }
    Pending p;
    p.r = *r;
    p.mesh = m;
    p.t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return PWC_ERR_BUSY;
        p.ticket = s->next_ticket++;
        s->known[p.ticket] = true;
        s->pending.push_back(p);
        ++s->submitted;
        if (!s->have_first) {
            s->have_first = true;
            s->t_first = p.t_submit;
        }
    }
    s->cv_work.notify_one();
    *ticket = p.ticket;
    return PWC_OK;
}

pwc_status pwc_server_poll(pwc_server *s, uint64_t ticket, pwc_result *res) {
    if (!s || !res) return PWC_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->known.count(ticket)) return PWC_ERR_STATE;
    auto it = s->finished.find(ticket);
    if (it == s->finished.end()) return PWC_ERR_BUSY;
    *res = it->second;
    s->finished.erase(it);
    s->known.erase(ticket);
    s->cv_done.notify_all();
    return PWC_OK;
}

pwc_status pwc_server_wait(pwc_server *s, uint64_t ticket, pwc_result *res) {
    if (!s || !res) return PWC_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->known.count(ticket)) return PWC_ERR_STATE;
    // A second waiter on the same ticket wakes when the first collects it.
    s->cv_done.wait(lk, [&] { return s->finished.count(ticket) != 0 || !s->known.count(ticket); });
    if (!s->known.count(ticket)) return PWC_ERR_STATE;
    *res = s->finished[ticket];
    s->finished.erase(ticket);
    s->known.erase(ticket);
    s->cv_done.notify_all();
    return PWC_OK;
}

pwc_status pwc_server_get_stats(pwc_server *s, pwc_server_stats *st) {
    if (!s || !st) return PWC_ERR_ARG;
    std::memset(st, 0, sizeof(*st));
    std::vector<double> lat;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        st->submitted = s->submitted;
        st->completed = s->completed;
        st->failed = s->failed;
        st->table_builds = s->builds;
        st->evictions = s->evictions;
        st->launches = s->launches;
        st->batched = s->batched;
        lat = s->latencies;
        if (s->have_first && s->completed) st->wall_s = ms_between(s->t_first, s->t_last) * 1e-3;
        if (st->wall_s > 0) {
            st->integrals_per_s = s->integrals / st->wall_s;
            st->pairs_per_s = s->pairs / st->wall_s;
        }
    }
    st->resident_bytes = s->resident_bytes.load();
    st->resident_tables = s->resident_tables.load();
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {
            const size_t i = static_cast<size_t>(p * (lat.size() - 1) + 0.5);
            return lat[std::min(i, lat.size() - 1)];
        };
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
        st->max_ms = lat.back();
    }
    return PWC_OK;
}

pwc_status pwc_server_reset_stats(pwc_server *s) {
    if (!s) return PWC_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    s->submitted = s->completed = s->failed = s->builds = s->evictions = 0;
    s->launches = s->batched = 0;
    s->latencies.clear();
    s->integrals = s->pairs = 0.0;
    s->have_first = false;
    return PWC_OK;
}

pwc_status pwc_server_destroy(pwc_server *s) {
    if (!s) return PWC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto &kv : s->cache) pwc_table_destroy(kv.second.t);
    if (s->planned) pwc_table_destroy(s->planned);
    for (Slot &sl : s->slots) {
        (void)hipStreamSynchronize(sl.stream);
        (void)hipHostFree(sl.h_e);
        (void)hipHostFree(sl.h_err);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.stream);
    }
    (void)hipStreamDestroy(s->build_stream);
    delete s;
    return PWC_OK;
}

}  // extern "C"
