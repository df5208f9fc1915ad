// Serving: resident hierarchies answer a stream of solve requests.
//
// Every system added to a server keeps its hierarchy (set up once and reused
// for every solve, the preconditioner recycling of the paper's experiments)
// and a slot engine of K columns with a stream of its own, so the systems'
// work overlaps on the device.  A request brings k right-hand sides of one
// system.  It is admitted, first come first served per system, once k slots
// of that engine are free and its staging block (n * k doubles: the
// right-hand sides in, the solutions out) fits in the request arena, whose
// size is the memory budget left after the engines; until then it waits.
// Admitted columns join the running ones at the next batch boundary
// (continuous batching) and leave when they are final, freeing their slots
// for the next request while the other columns go on.
//
// One host thread drives the server with camg_server_poll: for each system
// whose last batch has finished it retires final columns, runs the true
// residual check (restarting, in mixed precision, a column whose true
// residual missed the tolerance, at most twice), copies finished requests
// out, admits waiting ones and enqueues the next batch of iterations.  The
// host never waits for the device inside poll.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "internal.hpp"

namespace camg {
namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device block: offsets aligned to 256 bytes,
// free neighbours merged.
class Arena {
  public:
    void init(int64_t size) {
        size_ = size;
        free_.clear();
        live_.clear();
        if (size > 0) free_[0] = size;
    }
    int64_t alloc(int64_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const int64_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest > 0) free_[off + bytes] = rest;
            live_[off] = bytes;
            used_ += bytes;
            return off;
        }
        return -1;
    }
    void release(int64_t off) {
        auto it = live_.find(off);
        if (it == live_.end()) return;
        int64_t start = off, len = it->second;
        used_ -= len;
        live_.erase(it);
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && nx->first == start + len) {
            len += nx->second;
            free_.erase(nx);
        }
        auto pv = free_.lower_bound(start);
        if (pv != free_.begin()) {
            --pv;
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }
    int64_t used() const { return used_; }
    int64_t size() const { return size_; }

  private:
    int64_t size_ = 0, used_ = 0;
    std::map<int64_t, int64_t> free_, live_;
};

struct SReq {
    int64_t tag = 0;
    int sys = 0, k = 0;
    const double *B = nullptr;
    int ldb = 0;
    double *X = nullptr;
    int ldx = 0;
    double rtol = 0.0;
    int max_iter = 0;
    int64_t off = -1;
    int8_t slot[kMaxSlots] = {};
    int pending = 0;
    int32_t status = 0, iters = 0;
    double relres = 0.0;
    double t_submit = 0.0, t_admit = 0.0;
};

struct SSys {
    Hier *h = nullptr;
    Engine *E = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    EngineSnap *dsnap = nullptr, *hsnap = nullptr;
    int K = 0, n = 0, ipb = 1;
    bool mixed = false;
    int owner[kMaxSlots];          // slot -> request id, -1 free
    int reps[kMaxSlots];           // residual replacements of the slot's column
    bool final_[kMaxSlots];        // column finished and checked
    bool fresh[kMaxSlots];         // started or restarted since the last snapshot
    unsigned long long checked = 0;  // slots whose true residual the in-flight snapshot carries
    std::deque<int64_t> queue;     // waiting requests
    std::vector<int64_t> copying;  // requests whose solutions are being copied out
    bool inflight = false;
    int64_t footprint = 0;
};

}  // namespace

struct Server {
    int64_t budget = 0, engines_bytes = 0;
    char *arena_base = nullptr;
    Arena arena;
    bool open = false;  // arena allocated: no more systems
    std::vector<std::unique_ptr<SSys>> sys;
    std::map<int64_t, SReq> reqs;
    int64_t next_id = 0;
    std::vector<camg_completion> done;
    ~Server();
};

namespace {

void open_arena(Server &S) {
    if (S.open) return;
    const int64_t left = S.budget - S.engines_bytes;
    if (left <= 0) fail(CAMG_E_NOMEM, "memory budget leaves no room for requests");
    HIPC(hipMalloc(&S.arena_base, (size_t)left));
    S.arena.init(left);
    S.open = true;
}

// Retire the batch that just finished on system `y`.
void retire(Server &S, SSys &y) {
    // requests whose copies were in that batch are complete
    for (int64_t id : y.copying) {
        SReq &r = S.reqs.at(id);
        camg_completion c{};
        c.tag = r.tag;
        c.status = r.status;
        c.iters = r.iters;
        c.true_relres = r.relres;
        c.queue_ms = r.t_admit - r.t_submit;
        c.latency_ms = now_ms() - r.t_submit;
        S.done.push_back(c);
        S.arena.release(r.off);
        S.reqs.erase(id);
    }
    y.copying.clear();
    const EngineSnap &sn = *y.hsnap;
    unsigned long long replace = 0, release = 0;
    for (int c = 0; c < y.K; ++c) {
        const int64_t id = y.owner[c];
        if (id < 0 || y.final_[c] || sn.done[c] != 1) continue;
        if (!((y.checked >> c) & 1ull)) continue;  // checked in the next snapshot
        SReq &r = S.reqs.at(id);
        const double rel = sn.bnorm[c] > 0.0 ? std::sqrt(std::max(sn.tres2[c], 0.0)) / sn.bnorm[c] : 0.0;
        const int32_t st = sn.status[c];
        if (y.mixed && st == CAMG_OK && r.rtol > 0.0 && rel >= r.rtol && y.reps[c] < 2 && sn.iter[c] < r.max_iter) {
            replace |= 1ull << c;
            y.reps[c] += 1;
            y.fresh[c] = true;
            continue;
        }
        y.final_[c] = true;
        r.iters = std::max(r.iters, sn.iter[c]);
        r.relres = std::max(r.relres, rel);
        camg_status cs = (camg_status)st;
        if (y.mixed && cs == CAMG_OK && r.rtol > 0.0 && rel >= r.rtol) cs = CAMG_E_ACCURACY;
        r.status = worse_status((camg_status)r.status, cs);
        if (--r.pending == 0) {
            // gather the request's columns into its staging block, copy out, free the slots
            SlotMap q;
            for (int j = 0; j < kMaxSlots; ++j) q.q[j] = j < r.k ? r.slot[j] : (int8_t)0;
            double *blk = reinterpret_cast<double *>(S.arena_base + r.off);
            engine_gather_x(*y.E, q, r.k, blk, y.s);
            if (r.ldx == r.k)
                HIPC(hipMemcpyAsync(r.X, blk, sizeof(double) * r.k * (size_t)y.n, hipMemcpyDefault, y.s));
            else
                HIPC(hipMemcpy2DAsync(r.X, sizeof(double) * r.ldx, blk, sizeof(double) * r.k,
                                      sizeof(double) * r.k, y.n, hipMemcpyDefault, y.s));
            for (int j = 0; j < r.k; ++j) {
                release |= 1ull << r.slot[j];
                y.owner[r.slot[j]] = -1;
            }
            y.copying.push_back(id);
        }
    }
    y.checked = 0;
    if (replace) engine_replace(*y.E, replace, y.s);
    engine_release_mask(*y.E, release, y.s);
}

// Admit waiting requests in arrival order while slots and arena room last.
void admit(Server &S, SSys &y) {
    while (!y.queue.empty()) {
        SReq &r = S.reqs.at(y.queue.front());
        int nfree = 0;
        for (int c = 0; c < y.K; ++c) nfree += y.owner[c] < 0 ? 1 : 0;
        if (nfree < r.k) return;
        const int64_t off = S.arena.alloc((int64_t)y.n * r.k * (int64_t)sizeof(double));
        if (off < 0) return;
        r.off = off;
        SlotMap q;
        for (int c = 0; c < kMaxSlots; ++c) q.q[c] = -1;
        for (int c = 0, j = 0; c < y.K && j < r.k; ++c)
            if (y.owner[c] < 0) {
                r.slot[j] = (int8_t)c;
                q.q[c] = (int8_t)j;
                y.owner[c] = (int)y.queue.front();
                y.reps[c] = 0;
                y.final_[c] = false;
                y.fresh[c] = true;
                ++j;
            }
        double *blk = reinterpret_cast<double *>(S.arena_base + off);
        if (r.ldb == r.k)
            HIPC(hipMemcpyAsync(blk, r.B, sizeof(double) * r.k * (size_t)y.n, hipMemcpyDefault, y.s));
        else
            HIPC(hipMemcpy2DAsync(blk, sizeof(double) * r.k, r.B, sizeof(double) * r.ldb, sizeof(double) * r.k,
                                  y.n, hipMemcpyDefault, y.s));
        engine_start_slots(*y.E, q, blk, r.k, r.rtol, r.max_iter, y.s);
        r.pending = r.k;
        r.t_admit = now_ms();
        y.queue.pop_front();
    }
}

// Enqueue the next batch of system `y` (iterations, the true residuals of
// the columns seen finished, the snapshot) and its event.
void launch(Server &S, SSys &y) {
    (void)S;
    const EngineSnap &sn = *y.hsnap;
    bool any = !y.copying.empty(), run = false;
    unsigned long long check = 0;
    for (int c = 0; c < y.K; ++c) {
        if (y.owner[c] < 0 || y.final_[c]) continue;
        any = true;
        // finished at the last snapshot: check its true residual (iterating
        // a finished column changes nothing)
        if (!y.fresh[c] && sn.done[c] == 1) check |= 1ull << c;
        else run = true;
    }
    if (!any) return;
    if (run) engine_launch(*y.E, y.ipb, y.s);
    engine_snapshot(*y.E, check != 0, y.dsnap, y.s);
    HIPC(hipMemcpyAsync(y.hsnap, y.dsnap, sizeof(EngineSnap), hipMemcpyDeviceToHost, y.s));
    HIPC(hipEventRecord(y.ev, y.s));
    for (int c = 0; c < y.K; ++c) y.fresh[c] = false;
    y.checked = check;
    y.inflight = true;
}

}  // namespace

Server::~Server() {
    for (auto &p : sys) {
        SSys &y = *p;
        if (y.s) (void)hipStreamSynchronize(y.s);
        if (y.E) engine_destroy(y.E);
        if (y.ev) (void)hipEventDestroy(y.ev);
        if (y.dsnap) (void)hipFree(y.dsnap);
        if (y.hsnap) (void)hipHostFree(y.hsnap);
        if (y.s) (void)hipStreamDestroy(y.s);
    }
    if (arena_base) (void)hipFree(arena_base);
}

Server *server_create(int64_t budget) {
    if (budget <= 0) fail(CAMG_E_ARG, "budget must be positive");
    auto *S = new Server();
    S->budget = budget;
    return S;
}

int server_add(Server &S, Hier &h, int slots, int ipb) {
    if (S.open) fail(CAMG_E_BUSY, "systems must be added before the first request");
    if (slots < 1 || slots > kMaxSlots || (slots & (slots - 1)))
        fail(CAMG_E_ARG, "slots must be a power of two in [1, 64]");
    const int64_t fp = engine_footprint(h, slots) + (int64_t)sizeof(EngineSnap);
    if (S.engines_bytes + fp > S.budget) fail(CAMG_E_NOMEM, "engine does not fit the memory budget");
    std::unique_ptr<SSys> y(new SSys());
    y->h = &h;
    y->K = slots;
    y->n = h.lev[0].A.nr;
    y->mixed = h.prm.precision == CAMG_MIXED_FP32;
    if (ipb <= 0) ipb = (int)std::clamp<int64_t>((int64_t)4000000 / std::max(y->n, 1), 1, 16);
    y->ipb = ipb;
    for (int c = 0; c < kMaxSlots; ++c) {
        y->owner[c] = -1;
        y->reps[c] = 0;
        y->final_[c] = false;
        y->fresh[c] = false;
    }
    HIPC(hipStreamCreateWithFlags(&y->s, hipStreamNonBlocking));
    HIPC(hipEventCreateWithFlags(&y->ev, hipEventDisableTiming));
    HIPC(hipMalloc((void **)&y->dsnap, sizeof(EngineSnap)));
    HIPC(hipHostMalloc((void **)&y->hsnap, sizeof(EngineSnap), hipHostMallocDefault));
    std::memset(y->hsnap, 0, sizeof(EngineSnap));
    y->E = engine_create(h, slots, 1, y->s);
    y->footprint = fp;
    S.engines_bytes += fp;
    S.sys.push_back(std::move(y));
    return (int)S.sys.size() - 1;
}

void server_submit(Server &S, int sys, int k, const double *B, int ldb, double *X, int ldx, double rtol,
                   int max_iter, int64_t tag) {
    if (sys < 0 || sys >= (int)S.sys.size()) fail(CAMG_E_ARG, "unknown system");
    SSys &y = *S.sys[sys];
    if (k < 1 || k > y.K || !B || !X || ldb < k || ldx < k || !std::isfinite(rtol) || max_iter < 1)
        fail(CAMG_E_ARG, "bad request");
    open_arena(S);
    if (((int64_t)y.n * k * (int64_t)sizeof(double) + 255) / 256 * 256 > S.arena.size())
        fail(CAMG_E_NOMEM, "request larger than the request arena");
    SReq r;
    r.tag = tag;
    r.sys = sys;
    r.k = k;
    r.B = B;
    r.ldb = ldb;
    r.X = X;
    r.ldx = ldx;
    r.rtol = rtol;
    r.max_iter = max_iter;
    r.t_submit = now_ms();
    const int64_t id = S.next_id++;
    S.reqs.emplace(id, r);
    y.queue.push_back(id);
}

int server_poll(Server &S) {
    for (auto &p : S.sys) {
        SSys &y = *p;
        if (y.inflight) {
            const hipError_t q = hipEventQuery(y.ev);
            if (q == hipErrorNotReady) continue;
            HIPC(q);
            y.inflight = false;
            retire(S, y);
        }
        if (S.open) admit(S, y);
        launch(S, y);
    }
    return (int)S.done.size();
}

int server_take(Server &S, camg_completion *out, int cap) {
    const int m = std::min<int>(cap, (int)S.done.size());
    for (int i = 0; i < m; ++i) out[i] = S.done[i];
    S.done.erase(S.done.begin(), S.done.begin() + m);
    return m;
}

void server_stats(const Server &S, int64_t *arena_used, int64_t *arena_size, int32_t *queued, int32_t *active) {
    int q = 0, a = 0;
    for (auto &p : S.sys) {
        q += (int)p->queue.size();
        for (int c = 0; c < p->K; ++c) a += p->owner[c] >= 0 ? 1 : 0;
    }
    if (arena_used) *arena_used = S.arena.used();
    if (arena_size) *arena_size = S.open ? S.arena.size() : S.budget - S.engines_bytes;
    if (queued) *queued = q;
    if (active) *active = a;
}

void server_destroy(Server *S) { delete S; }

}  // namespace camg
