// server.hip -- the request server behind dwf_submit / dwf_poll: continuous
// batching of independent solves on one device.
//
// Requests on the same operator (context), inner precision and link format
// share a "lane": one solve engine of K slots, its own HIP stream and one
// worker thread.  A request enters a free slot at the next scheduling round of
// its lane and leaves it as soon as its own solve is done, while the other
// slots keep iterating in the same multi-right-hand-side kernels (each with
// its own quark mass).  Lanes of different operators run concurrently on
// their own streams.
//
// Admission: a lane's device memory (its engine plus a one-spinor staging
// buffer) is reserved from the HBM budget when the lane is created, with K
// as large as the budget allows (at most kMaxBatch).  A request whose lane
// does not exist and does not fit waits; idle lanes give their memory back
// while requests wait for memory.
//
// Scheduling: a lane whose lattice fills the GPU by itself ("large": at
// least kLargeV5h half 5D sites) runs only while it holds one of the
// kLargeLanes oldest requests among the large lanes with work; the others wait
// for their turn.  Large solves therefore run in arrival order at the full
// speed of the device instead of sharing it, while lanes of small lattices,
// whose iterations are bound by launch latency rather than bandwidth, run
// beside them at any time.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <deque>
#include <thread>

#include "dwf_ctx.h"

namespace dwf {
namespace {

using Clock = std::chrono::steady_clock;
constexpr int kMaxBatch = 8;
// graph replays (of 4 iterations) between scheduling rounds of a lane, so that
// a new request waits at most this long for its slot
constexpr int kReplayCap = 16;
// lanes of at least this many half 5D sites (16^3 x 32 x 8) fill the GPU alone
constexpr long kLargeV5h = 1L << 19;
// large requests in service at once, admitted in arrival order, and so large
// lanes that run at once (DWF_SERVE_LARGE_LANES overrides).  On the served
// stream of four fields (200 requests at 0.8 of the plain capacity, and 60 at
// once): 1 leaves the GPU part idle under the smaller "large" solves (fewer
// solves/s than a FIFO of plain solves, p99 9.1-9.2 s against 6.9 s); 2 beats
// the FIFO on p50, p99 and solves/s in every run (p99 5.7-6.1 s); 3 by less
// (p99 6.4 s); without the arrival order, lanes batched their newer requests
// ahead of older ones in other lanes and p99 varied from 6.4 to 8.8 s
int large_lanes() {
    static const int n = [] {
        const char* e = getenv("DWF_SERVE_LARGE_LANES");
        const int v = e ? atoi(e) : 2;
        return v > 0 ? v : 1;
    }();
    return n;
}
int large_requests() { return large_lanes(); }

struct Request {
    uint64_t ticket = 0;
    dwf_ctx* ctx = nullptr;
    double mq = 0;
    dwf_solve_params p{};
    std::vector<double> b, x;
    dwf_solve_stats st{};
    int status = DWF_PENDING;
    std::string err;
    Clock::time_point t_submit;
};
using ReqP = std::shared_ptr<Request>;

struct Server;

struct Lane {
    Server* srv = nullptr;
    std::string key;
    dwf_ctx* ctx = nullptr;
    dwf_solve_params p0{};
    int K = 0;
    size_t bytes = 0;  // reserved from the budget
    std::deque<ReqP> queue;
    std::vector<ReqP> slot;
    std::condition_variable cv;
    std::thread th;
    bool large = false;    // V5h >= kLargeV5h: runs in arrival order with the other large lanes
    bool cancel = false;   // fail everything and exit (context destroyed, shutdown)
    bool closing = false;  // idle and giving its memory back: takes no new requests
    bool exited = false;
};

struct Server {
    std::mutex mu;
    std::condition_variable cv_done;
    std::map<uint64_t, ReqP> reqs;
    std::map<std::string, std::unique_ptr<Lane>> lanes;
    std::vector<std::unique_ptr<Lane>> dead;  // exited, not yet joined
    std::condition_variable cv_exit;          // a lane thread has exited
    std::condition_variable cv_turn;          // the order of the large lanes may have changed
    std::deque<ReqP> waiting;  // their lane does not exist and does not fit yet
    uint64_t next_ticket = 1;
    size_t used = 0;
    size_t default_budget = 0;
    bool atexit_set = false;
    // statistics since the last reset
    int64_t completed = 0, admitted = 0, peak_batch = 0, waits = 0;
    std::vector<double> lat;
    double busy = 0;
    int in_service = 0;
    Clock::time_point busy_since;
};

Server& srv() {
    static Server* s = new Server;  // never destroyed: worker threads may outlive static destruction
    return *s;
}

size_t spinor_bytes_host(const dwf_ctx* c) { return (size_t)c->V4 * c->Ns * 24 * sizeof(double); }

std::string lane_key(const dwf_ctx* c, const dwf_solve_params& p) {
    char buf[64];
    snprintf(buf, sizeof(buf), "%p:%d:%d", (const void*)c, p.inner_prec, link_format(c, p));
    return buf;
}

// Finish a request (lock held).
void complete(Server& S, const ReqP& q, int status, const std::string& err) {
    q->status = status;
    q->err = err;
    S.cv_done.notify_all();
}

void service_end(Server& S) {
    S.completed++;
    if (--S.in_service == 0) S.busy += std::chrono::duration<double>(Clock::now() - S.busy_since).count();
}

void lane_main(Lane* L);

// Requests of large lanes (in service or queued) that arrived before ticket t
// (lock held).
int older_large(const Server& S, uint64_t t) {
    int older = 0;
    for (auto& kv : S.lanes) {
        const Lane* o = kv.second.get();
        if (!o->large || o->cancel || o->closing || o->exited) continue;
        for (auto& r : o->slot)
            if (r && r->ticket < t) ++older;
        for (auto& r : o->queue)
            if (r->ticket < t) ++older;
    }
    return older;
}

// Whether a large lane may admit request q: fewer than large_requests()
// requests of large lanes arrived before it (lock held).  Large requests thus
// enter service in arrival order, a few at a time: one such solve nearly
// fills the GPU, so running more of them at once only stretches each
// (batching them gains nothing), and letting a lane batch its newer requests
// would serve them ahead of older ones in other lanes.
bool large_admissible(const Server& S, const Request& q) { return older_large(S, q.ticket) < large_requests(); }

// A large lane's turn: its oldest request (in a slot or queued) is
// admissible, so that a lane whose requests all wait for older ones sleeps
// instead of spinning (lock held).
bool large_turn(const Server& S, const Lane* L) {
    const Request* oldest = nullptr;
    for (auto& q : L->slot)
        if (q && (!oldest || q->ticket < oldest->ticket)) oldest = q.get();
    if (!L->queue.empty() && (!oldest || L->queue.front()->ticket < oldest->ticket)) oldest = L->queue.front().get();
    return !oldest || large_admissible(S, *oldest);
}

// Join and drop the lanes whose thread has ended (lock held).  The lane of
// the calling thread goes to the graveyard and is joined later by another.
void reap(Server& S) {
    const auto me = std::this_thread::get_id();
    for (auto it = S.lanes.begin(); it != S.lanes.end();) {
        if (it->second->exited) {
            S.dead.push_back(std::move(it->second));
            it = S.lanes.erase(it);
        } else {
            ++it;
        }
    }
    for (auto it = S.dead.begin(); it != S.dead.end();) {
        if ((*it)->th.get_id() == me) {
            ++it;
            continue;
        }
        if ((*it)->th.joinable()) (*it)->th.join();
        it = S.dead.erase(it);
    }
}

size_t budget_of(Server& S, const dwf_ctx* c) {
    if (c->opts.hbm_budget_bytes) return c->opts.hbm_budget_bytes;
    if (!S.default_budget) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 0;
        S.default_budget = (size_t)(0.8 * (double)fr);
    }
    return S.default_budget;
}

void shutdown_all();

// Place a request in its lane, creating the lane if the budget allows and no
// earlier request waits for memory (unless this is that request: front).
// Lock held.  Returns false if it has to wait for memory.
bool route(Server& S, const ReqP& q, bool front) {
    const std::string key = lane_key(q->ctx, q->p);
    reap(S);
    auto it = S.lanes.find(key);
    if (it != S.lanes.end()) {
        Lane* L = it->second.get();
        // a closing lane takes nothing more: the request waits and gets a new
        // lane once this one has given its memory back
        if (L->cancel || L->closing || L->exited) return false;
        L->queue.push_back(q);
        L->cv.notify_all();
        return true;
    }
    if (!front && !S.waiting.empty()) return false;
    const size_t budget = budget_of(S, q->ctx);
    const size_t stage = spinor_bytes_host(q->ctx);
    const size_t per = engine_bytes(q->ctx, q->p.inner_prec, 1);
    if (S.used + stage + per > budget) return false;
    const int K = (int)std::min<size_t>(kMaxBatch, (budget - S.used - stage) / per);
    std::unique_ptr<Lane> L(new Lane);
    L->srv = &S;
    L->key = key;
    L->ctx = q->ctx;
    L->p0 = q->p;
    L->K = K;
    L->bytes = stage + engine_bytes(q->ctx, q->p.inner_prec, K);
    L->slot.assign(K, nullptr);
    L->large = q->ctx->V5h >= kLargeV5h;
    L->queue.push_back(q);
    S.used += L->bytes;
    Lane* raw = L.get();
    S.lanes[key] = std::move(L);
    if (!S.atexit_set) {
        S.atexit_set = true;
        std::atexit(shutdown_all);
    }
    raw->th = std::thread(lane_main, raw);
    return true;
}

// Route waiting requests in arrival order while they fit (lock held).
void dispatch_waiting(Server& S) {
    reap(S);
    while (!S.waiting.empty()) {
        if (!route(S, S.waiting.front(), true)) break;
        S.waiting.pop_front();
    }
    if (!S.waiting.empty())
        for (auto& kv : S.lanes) kv.second->cv.notify_all();  // idle lanes: give memory back
}

void lane_main(Lane* L) {
    Server& S = *L->srv;
    const size_t nb = spinor_bytes_host(L->ctx);
    hipStream_t st = nullptr;
    std::unique_ptr<EngineBase> eng;
    DevBuf stage;
    int rc = DWF_OK;
    std::string why;
    if (hipSetDevice(L->ctx->device) != hipSuccess ||
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        rc = fail(DWF_EDEVICE, "server: cannot create a stream");
    if (!rc) rc = make_engine(L->ctx, L->p0, L->K, st, &eng);
    if (!rc) rc = stage.alloc(nb);
    if (rc) why = dwf_last_error();
    if (eng) {
        eng->set_use_graph(true);
        eng->set_replay_cap(kReplayCap);
    }

    while (!rc) {
        std::vector<std::pair<int, ReqP>> adm;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            bool leave = false;
            while (!L->cancel && L->queue.empty() && eng->busy() == 0) {
                if (!S.waiting.empty()) {  // memory is wanted elsewhere: release this lane
                    leave = true;
                    L->closing = true;  // under the lock that found the queue empty
                    break;
                }
                L->cv.wait_for(lk, std::chrono::milliseconds(200));
            }
            if (leave || L->cancel) break;
            for (int r = 0; r < L->K && !L->queue.empty(); ++r) {
                if (L->slot[r]) continue;
                if (L->large && !large_admissible(S, *L->queue.front())) break;  // queue: arrival order
                adm.emplace_back(r, L->queue.front());
                L->queue.pop_front();
            }
            for (auto& a : adm) {
                L->slot[a.first] = a.second;
                S.admitted++;
                if (S.in_service++ == 0) S.busy_since = Clock::now();
            }
        }
        for (auto& a : adm) {
            if (hipMemcpyAsync(stage.p, a.second->b.data(), nb, hipMemcpyHostToDevice, st) != hipSuccess) {
                rc = fail(DWF_EDEVICE, "server: upload of b failed");
                break;
            }
            if ((rc = eng->admit(a.first, stage.as<double>(), nullptr, a.second->mq, a.second->p))) break;
        }
        if (rc) break;
        if (!adm.empty()) {
            if (hipStreamSynchronize(st) != hipSuccess) {
                rc = fail(DWF_EDEVICE, "server: upload of b failed");
                break;
            }
            for (auto& a : adm) std::vector<double>().swap(a.second->b);  // b is on the device now
        }
        {
            std::unique_lock<std::mutex> lk(S.mu);
            S.peak_batch = std::max<int64_t>(S.peak_batch, eng->busy());
            // a large lane waits for its turn (re-checked at least every 2 ms)
            while (L->large && !L->cancel && !large_turn(S, L))
                S.cv_turn.wait_for(lk, std::chrono::milliseconds(2));
            if (L->cancel) break;
        }
        if ((rc = eng->tick())) break;
        for (int r = 0; r < L->K && !rc; ++r) {
            if (!L->slot[r] || eng->phase(r) != PH_DONE) continue;
            ReqP q = L->slot[r];
            SlotResult res;
            q->x.resize(nb / sizeof(double));
            if ((rc = eng->retire(r, stage.as<double>(), &res))) break;
            if (hipMemcpyAsync(q->x.data(), stage.p, nb, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = fail(DWF_EDEVICE, "server: download of x failed");
                break;
            }
            dwf_solve_stats& o = q->st;
            memset(&o, 0, sizeof(o));
            o.status = res.status;
            o.iters = res.iters;
            o.restarts = res.restarts;
            o.reliable_updates = res.reliable_updates;
            o.fallback = res.fallback;
            o.true_residual = res.true_residual;
            o.schur_residual = res.schur_residual;
            o.seconds = res.seconds;
            o.gflops = res.seconds > 0 ? res.flops / res.seconds * 1e-9 : 0;
            o.hbm_gbytes = res.bytes * 1e-9;
            o.rhs_per_block = eng->rhs_per_block();
            eng->tile(&o.tile, &o.sites_per_block, &o.block_order);
            o.tile += 1;
            std::lock_guard<std::mutex> lk(S.mu);
            L->slot[r] = nullptr;
            S.lat.push_back(std::chrono::duration<double>(Clock::now() - q->t_submit).count());
            service_end(S);
            complete(S, q, res.status, res.status == DWF_OK ? "" : "solve did not reach the requested tolerance");
            S.cv_turn.notify_all();
        }
    }
    if (rc && why.empty()) why = dwf_last_error();
    if (st) (void)hipStreamSynchronize(st);
    eng.reset();
    stage.release();
    if (st) (void)hipStreamDestroy(st);
    std::lock_guard<std::mutex> lk(S.mu);
    const int code = rc ? rc : DWF_EINVAL;
    const std::string msg = rc ? "server: " + why : "server: the context was destroyed";
    for (auto& q : L->slot)
        if (q) {
            service_end(S);
            complete(S, q, code, msg);
        }
    for (auto& q : L->queue) complete(S, q, code, msg);
    L->queue.clear();
    S.used -= L->bytes;
    L->exited = true;
    S.cv_exit.notify_all();
    S.cv_turn.notify_all();
    // hand the memory to waiting requests; this lane is joined by the next
    // caller that reaps (never by itself)
    dispatch_waiting(S);
}

// Cancel the lanes that match and wait until their threads have exited.
template <class Pred>
void cancel_lanes(Server& S, std::unique_lock<std::mutex>& lk, Pred pred) {
    for (auto& kv : S.lanes)
        if (pred(kv.second.get())) {
            kv.second->cancel = true;
            kv.second->cv.notify_all();
            S.cv_turn.notify_all();
        }
    S.cv_exit.wait(lk, [&] {
        for (auto& kv : S.lanes)
            if (pred(kv.second.get()) && !kv.second->exited) return false;
        return true;
    });
    reap(S);
}

void shutdown_all() {
    Server& S = srv();
    std::unique_lock<std::mutex> lk(S.mu);
    S.waiting.clear();
    cancel_lanes(S, lk, [](Lane*) { return true; });
}

}  // namespace

void server_detach(dwf_ctx* c) {
    Server& S = srv();
    std::unique_lock<std::mutex> lk(S.mu);
    for (auto it = S.waiting.begin(); it != S.waiting.end();) {
        if ((*it)->ctx == c) {
            complete(S, *it, DWF_EINVAL, "server: the context was destroyed");
            it = S.waiting.erase(it);
        } else {
            ++it;
        }
    }
    cancel_lanes(S, lk, [c](Lane* L) { return L->ctx == c; });
}

}  // namespace dwf

using namespace dwf;

extern "C" {

int dwf_submit_mass(dwf_ctx* c, const double* b, double mq, const dwf_solve_params* params, uint64_t* ticket) {
    if (!c || !b || !ticket) return fail(DWF_EINVAL, "NULL context, b or ticket");
    if (!std::isfinite(mq)) return fail(DWF_EINVAL, "mq must be finite");
    dwf_solve_params p;
    if (params)
        p = *params;
    else
        dwf_default_params(&p);
    int rc = check_params(c, p);
    if (rc) return rc;
    p.use_guess = 0;
    DWF_HIP(hipSetDevice(c->device));
    if (!c->table_set(mq, &rc)) return rc;  // rejects a singular (1 + cL) or X for this mass
    ReqP q(new Request);
    q->ctx = c;
    q->mq = mq;
    q->p = p;
    q->b.assign(b, b + (size_t)c->V4 * c->Ns * 24);
    q->t_submit = Clock::now();
    Server& S = srv();
    std::lock_guard<std::mutex> lk(S.mu);
    reap(S);
    const size_t need = spinor_bytes_host(c) + engine_bytes(c, p.inner_prec, 1);
    if (need > budget_of(S, c)) return fail(DWF_ENOMEM, "server: one solve does not fit the HBM budget");
    q->ticket = S.next_ticket++;
    S.reqs[q->ticket] = q;
    *ticket = q->ticket;
    if (!route(S, q, false)) {
        S.waiting.push_back(q);
        S.waits++;
        dispatch_waiting(S);
    }
    return DWF_OK;
}

int dwf_submit(dwf_ctx* c, const double* b, const dwf_solve_params* params, uint64_t* ticket) {
    if (!c) return fail(DWF_EINVAL, "NULL context");
    return dwf_submit_mass(c, b, c->mq, params, ticket);
}

int dwf_poll(uint64_t ticket, double* x, dwf_solve_stats* st, int timeout_us) {
    Server& S = srv();
    ReqP q;
    {
        std::unique_lock<std::mutex> lk(S.mu);
        auto it = S.reqs.find(ticket);
        if (it == S.reqs.end()) return fail(DWF_ENOTFOUND, "unknown ticket");
        q = it->second;
        auto done = [&] { return q->status != DWF_PENDING; };
        if (timeout_us < 0)
            S.cv_done.wait(lk, done);
        else if (timeout_us > 0)
            S.cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done);
        if (!done()) return DWF_PENDING;
        S.reqs.erase(it);
    }
    if (q->status == DWF_OK || q->status == DWF_ENOCONV) {
        if (x) std::copy(q->x.begin(), q->x.end(), x);
        if (st) *st = q->st;
    } else if (st) {
        memset(st, 0, sizeof(*st));
        st->status = q->status;
    }
    if (q->status != DWF_OK) fail(q->status, q->err);
    return q->status;
}

int dwf_server_stats_get(dwf_server_stats* out, int reset) {
    if (!out) return fail(DWF_EINVAL, "NULL out");
    Server& S = srv();
    std::lock_guard<std::mutex> lk(S.mu);
    dwf_server_stats o{};
    o.completed = S.completed;
    o.admitted = S.admitted;
    o.peak_batch = S.peak_batch;
    o.waits_for_memory = S.waits;
    std::vector<double> l = S.lat;
    std::sort(l.begin(), l.end());
    auto pct = [&](double f) {
        if (l.empty()) return 0.0;
        size_t i = (size_t)std::ceil(f * (double)l.size()) - 1;
        return l[std::min(i, l.size() - 1)];
    };
    o.p50_latency = pct(0.50);
    o.p99_latency = pct(0.99);
    o.busy_seconds = S.busy + (S.in_service > 0 ? std::chrono::duration<double>(Clock::now() - S.busy_since).count()
                                                : 0.0);
    *out = o;
    if (reset) {
        S.completed = S.admitted = S.peak_batch = S.waits = 0;
        S.lat.clear();
        S.busy = 0;
        if (S.in_service > 0) S.busy_since = Clock::now();
    }
    return DWF_OK;
}

}  // extern "C"
