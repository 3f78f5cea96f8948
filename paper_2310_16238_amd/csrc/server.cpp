// server.cpp -- the fit server: continuous batching of independent Cox fits
// (C ABI in include/coxmi.h, kernels in serve.hip).
//
// Threads:
//   caller      cox_server_submit: checks the arguments, queues the request
//               (copying the inputs unless they are borrowed) and returns a ticket
//   prep pool   puts each request in canonical order (Sec. 2.7) and writes its
//               device image (X column-major, row words, group indices) into a
//               pinned staging area
//   worker      owns the GPU: builds the work lists of the resident fits and keeps
//               batched Newton iterations of all of them queued (two ahead; the
//               kernels leave out fits that have finished), reports fits as they
//               finish (from host-mapped state), admits staged requests into free
//               slots of the device arena meanwhile (uploads on a copy stream), and
//               retires finished fits when it stops queueing on those lists.  With
//               fused_rounds > 0 one persistent launch runs many iterations instead
//               (serve.hip, round_kernel), asked to end after its current iteration
//               when new fits are ready to join
//
// Admission is first come, first served, by device footprint: a request is
// admitted when a slot is free and its block fits in the arena; the fits
// behind it wait.  Fits that finish free their block for the next ones.
#include "coxmi.h"

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

#include "canonical.h"
#include "internal.h"
#include "serve.h"

using namespace coxmi;
using namespace coxmi::serve;

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// First-fit allocator over [0, capacity).
class RangeAlloc {
public:
    void reset(size_t cap)
    {
        free_.clear();
        if (cap) free_[0] = cap;
        cap_ = cap;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = round_up(bytes, kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, next = it->first + bytes;
            free_.erase(it);
            if (rest) free_[next] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = round_up(bytes, kAlign);
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
    size_t capacity() const { return cap_; }
    size_t peak() const { return peak_; }

private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
};

// Where each piece of one fit lives inside its arena block (byte offsets).
struct FitLayout {
    int64_t n = 0, ld = 0, ldz = 0, tile = 0;
    int p = 0, G = 0, nxr = 0, nzr = 0, xrange = 0, zrange = 0, npairs = 0, ntile = 0, ntc = 0;
    bool device = false;                            // X is gathered from the caller's device memory
    size_t meta = 0, gidx = 0, gam = 0, beta0 = 0, src = 0, x = 0, upload = 0;
                                                    // [0, upload) is uploaded in one copy: meta, gidx, the
                                                    // l1 weights and start point (p each), then X (host
                                                    // request) or src (device)
    size_t xf = 0, rows = 0, bf = 0, z = 0, beta = 0, prev = 0;
    size_t vec = 0, free_col = 0, L = 0, part = 0, tilemax = 0, tpart = 0, cpart = 0, total = 0;
};

// Device rows of a request: when the fit is longer than one scan tile and every
// stratum fits in one, strata are kept inside scan tiles (padding rows fill the
// gaps); otherwise the fit is one scan tile.  pos[i] = device row of canonical
// row i; returns the padded row count and the scan tile length.
int64_t place_rows(const std::vector<uint32_t> &meta, std::vector<int64_t> &pos, int64_t *tile)
{
    const int64_t n = (int64_t)meta.size();
    pos.resize((size_t)n);
    int64_t longest = 0, start = 0;
    for (int64_t i = 1; i <= n; ++i)
        if (i == n || (meta[i] & kHeadBit)) {
            longest = std::max(longest, i - start);
            start = i;
        }
    if (n <= kScanTile || longest > kScanTile) {
        for (int64_t i = 0; i < n; ++i) pos[i] = i;
        *tile = (int64_t)round_up((size_t)n, kRowPad);
        return *tile;
    }
    int64_t cur = 0, i = 0;
    while (i < n) {
        int64_t e = i + 1;
        while (e < n && !(meta[e] & kHeadBit)) ++e;
        const int64_t m = e - i, room = kScanTile - (cur % kScanTile);
        if (m > room) cur += room;
        for (int64_t k = 0; k < m; ++k) pos[i + k] = cur + k;
        cur += m;
        i = e;
    }
    *tile = kScanTile;
    return (int64_t)round_up((size_t)cur, kScanTile);
}

FitLayout plan(int64_t n, int64_t ld, int64_t tile, int p, int64_t G, bool device)
{
    FitLayout L;
    L.device = device;
    L.n = n;
    L.p = p;
    L.G = (int)G;
    L.ld = ld;
    L.tile = tile;
    L.ntc = (int)(ld / tile);
    L.ldz = (int64_t)round_up((size_t)std::max<int64_t>(G, 1), kRowPad);
    const int nt = (p + kTile - 1) / kTile;
    L.npairs = nt * (nt + 1) / 2;
    // K ranges of about an eighth of the rows, 1024 to 4096 of them, a multiple of 256 (each of
    // the 4 waves of a contraction item then takes whole 64-row steps)
    auto range_for = [](int64_t rows) {
        const int64_t r = (int64_t)round_up((size_t)((rows + 7) / 8), 256);
        return (int)std::min<int64_t>(kMaxRange, std::max<int64_t>(kMinRange, r));
    };
    L.xrange = range_for(L.ld);
    L.zrange = range_for(L.ldz);
    L.nxr = (int)((L.ld + L.xrange - 1) / L.xrange);
    L.nzr = G > 0 ? (int)((L.ldz + L.zrange - 1) / L.zrange) : 0;
    L.ntile = (int)((L.ld + kEtaRows - 1) / kEtaRows);
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t at = o;
        o = round_up(o + bytes, kAlign);
        return at;
    };
    L.meta = take(sizeof(uint32_t) * (size_t)L.ld);
    L.gidx = take(sizeof(int32_t) * (size_t)L.ld);
    L.gam = take(sizeof(double) * p);
    L.beta0 = take(sizeof(double) * p);
    if (device) {
        L.src = take(sizeof(int32_t) * (size_t)L.ld);
        L.upload = o;
        L.x = take(sizeof(double) * (size_t)p * L.ld);
    } else {
        L.x = take(sizeof(double) * (size_t)p * L.ld);
        L.upload = o;
    }
    L.xf = take(sizeof(float) * (size_t)p * L.ld);
    L.rows = take(sizeof(double) * 5 * (size_t)L.ld);
    L.bf = take(sizeof(float) * (size_t)L.ld);
    L.z = take(sizeof(float) * (size_t)p * L.ldz);   // zeroed at admission, with beta and prev
    L.beta = take(sizeof(double) * p);
    L.prev = take(sizeof(double) * p);
    L.vec = take(sizeof(double) * 3 * p);
    L.free_col = take((size_t)p);
    L.L = take(sizeof(double) * (size_t)p * p);
    L.part = take(sizeof(float) * (size_t)(L.nxr + L.nzr) * L.npairs * kTile * kTile);
    L.tilemax = take(sizeof(double) * L.ntile);
    L.tpart = take(sizeof(double) * 2 * L.ntc);
    L.cpart = take(sizeof(double) * 3 * (size_t)L.ntc * p);
    L.total = o;
    return L;
}

struct Request {
    uint64_t ticket = 0;
    bool device = false;   // x (and, until the prep thread copies them, the keys) in device memory
    int64_t n = 0, p = 0, ldx = 0;
    const double *x = nullptr, *time = nullptr;
    const uint8_t *event = nullptr;
    const int32_t *stratum = nullptr;
    std::vector<double> own_x, own_t;
    std::vector<uint8_t> own_e;
    std::vector<int32_t> own_s;
    std::vector<double> gam;     // [p] l1 weights; empty: an unpenalised fit
    std::vector<double> beta0;   // [p] start point; empty: zeros
    double t_submit = 0.0;
    FitLayout lay;
    size_t stage_off = 0;
};

struct Result {
    std::vector<double> beta;
    cox_fit_info info{};
    cox_request_times times{};
};

struct Slot {
    bool used = false, active = false, frozen = false;
    bool reported = false;   // its result went to the caller while the launch still ran
    std::unique_ptr<Request> req;
    size_t arena_off = 0;
    double t_admit = 0.0;
};

}  // namespace

struct cox_server {
    cox_server_options opt{};
    int device = 0;
    hipStream_t compute = nullptr, copy = nullptr;
    hipEvent_t iter_ev = nullptr;
    std::chrono::steady_clock::time_point t0;

    char *arena = nullptr;
    RangeAlloc arena_alloc;
    FitDesc *d_desc = nullptr;
    FitState *d_state = nullptr;
    char *staging = nullptr;
    RangeAlloc stage_alloc;
    FitDesc *h_desc = nullptr;
    FitState *h_state = nullptr, *dh_state = nullptr;   // host-mapped (and its device address)
    double *h_beta = nullptr, *dh_beta = nullptr;
    // persistent rounds: control block, host-mapped hold word and launch results
    void *d_round_ctl = nullptr;
    uint64_t *h_round = nullptr, *dh_round = nullptr;   // [0] hold word; [2..9] the launch's results
    int round_grid_p = -1, round_grid = 0;                // most workgroups for fits of at most round_grid_p columns

    // work lists: pinned host copies and device arrays (capacity in bytes)
    struct List {
        char *h = nullptr, *d = nullptr;
        size_t cap = 0;
    } l_round,     // one block per round: every work list
        l_admit[2];   // admission blocks (descriptors, slots, items), alternating

    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_prep, cv_ready, cv_done, cv_stage;
    std::deque<std::unique_ptr<Request>> prep_q, ready_q;
    std::unordered_map<uint64_t, Result> results;
    std::unordered_map<uint64_t, char> pending;   // submitted, not finished
    uint64_t next_ticket = 1;
    int64_t outstanding = 0;
    bool stop = false;
    int fatal = 0;
    std::string err, fatal_msg;

    // statistics (worker thread; read under mu)
    int64_t submitted = 0, completed = 0, iterations = 0, resident_peak = 0, launches = 0;
    double resident_sum = 0.0, gpu_busy_s = 0.0;
    double phase_s[6] = {0, 0, 0, 0, 0, 0};

    std::vector<std::thread> preps;
    std::thread worker;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

int srv_fail(cox_server *s, int code, const std::string &msg)
{
    if (s) {
        std::lock_guard<std::mutex> g(s->mu);
        s->err = msg;
    }
    return code;
}

thread_local std::string g_create_error;

void finish_locked(cox_server *s, uint64_t ticket, Result &&r)
{
    s->pending.erase(ticket);
    s->results[ticket] = std::move(r);
    s->outstanding -= 1;
    s->completed += 1;
    s->cv_done.notify_all();
}

void fail_request_locked(cox_server *s, const Request &q, int code, double t)
{
    Result r;
    r.info.status = code;
    r.times.submit_s = q.t_submit;
    r.times.admit_s = t;
    r.times.done_s = t;
    finish_locked(s, q.ticket, std::move(r));
}

// ------------------------------------------------------------------ prep pool

void write_image(const Request &q, const std::vector<int64_t> &perm, const std::vector<uint32_t> &meta,
                 const std::vector<int64_t> &pos, char *dst)
{
    const FitLayout &L = q.lay;
    uint32_t *mw = reinterpret_cast<uint32_t *>(dst + L.meta);
    int32_t *gi = reinterpret_cast<int32_t *>(dst + L.gidx);
    // padding rows: one-row strata without events, X = 0
    for (int64_t i = 0; i < L.ld; ++i) {
        mw[i] = kHeadBit | kPadBit;
        gi[i] = -1;
    }
    if (L.device) {
        // the admit kernel gathers X: device row pos[i] is the caller's row perm[i]
        int32_t *sr = reinterpret_cast<int32_t *>(dst + L.src);
        for (int64_t i = 0; i < L.ld; ++i) sr[i] = -1;
        for (int64_t i = 0; i < q.n; ++i) sr[pos[i]] = (int32_t)perm[i];
    } else {
        double *x = reinterpret_cast<double *>(dst + L.x);
        for (int64_t j = 0; j < q.p; ++j) {
            double *col = x + j * L.ld;
            const double *src = q.x + j * q.ldx;
            std::memset(col, 0, sizeof(double) * L.ld);
            for (int64_t i = 0; i < q.n; ++i) col[pos[i]] = src[perm[i]];
        }
    }
    int32_t g = 0;
    for (int64_t i = 0; i < q.n; ++i) {
        mw[pos[i]] = meta[i];
        gi[pos[i]] = (meta[i] & kCountMask) ? g++ : -1;
    }
    double *gw = reinterpret_cast<double *>(dst + L.gam), *b0 = reinterpret_cast<double *>(dst + L.beta0);
    for (int64_t j = 0; j < q.p; ++j) {
        gw[j] = q.gam.empty() ? 0.0 : q.gam[(size_t)j];
        b0[j] = q.beta0.empty() ? 0.0 : q.beta0[(size_t)j];
    }
}

// Keys of a device-resident request (times, events, strata) are copied to the
// host for the canonical order; X stays where it is.  Returns an error message.
const char *fetch_keys(cox_server *s, Request &q, hipStream_t &st)
{
    if (!st) {
        if (hipSetDevice(s->device) != hipSuccess || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            st = nullptr;
            return "creating a stream for device-resident keys";
        }
    }
    const size_t n = (size_t)q.n;
    q.own_t.resize(n);
    q.own_e.resize(n);
    if (q.stratum) q.own_s.resize(n);
    if (hipMemcpyAsync(q.own_t.data(), q.time, sizeof(double) * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(q.own_e.data(), q.event, n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        (q.stratum &&
         hipMemcpyAsync(q.own_s.data(), q.stratum, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st) != hipSuccess) ||
        hipStreamSynchronize(st) != hipSuccess)
        return "copying device-resident keys";
    q.time = q.own_t.data();
    q.event = q.own_e.data();
    q.stratum = q.stratum ? q.own_s.data() : nullptr;
    return check_data(q.n, q.p, q.ldx, q.x, q.time, q.event);
}

void prep_loop(cox_server *s)
{
    std::vector<int64_t> perm, pos;
    std::vector<uint32_t> meta;
    hipStream_t key_stream = nullptr;
    struct StreamGuard {
        hipStream_t &st;
        ~StreamGuard()
        {
            if (st) (void)hipStreamDestroy(st);
        }
    } guard{key_stream};
    for (;;) {
        std::unique_ptr<Request> q;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_prep.wait(lk, [s] { return s->stop || !s->prep_q.empty(); });
            if (s->stop) return;
            q = std::move(s->prep_q.front());
            s->prep_q.pop_front();
        }
        if (q->device) {
            if (const char *bad = fetch_keys(s, *q, key_stream)) {
                (void)bad;
                std::lock_guard<std::mutex> g(s->mu);
                fail_request_locked(s, *q, COX_EINVAL, s->now());
                continue;
            }
        }
        canonical_order(q->n, q->time, q->event, q->stratum, perm, meta);
        int64_t G = 0;
        for (int64_t i = 0; i < q->n; ++i) G += (meta[i] & kCountMask) ? 1 : 0;
        int64_t tile = 0;
        const int64_t ld = place_rows(meta, pos, &tile);
        q->lay = plan(q->n, ld, tile, (int)q->p, G, q->device);
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (q->lay.total > s->arena_alloc.capacity() || q->lay.upload > s->stage_alloc.capacity()) {
                fail_request_locked(s, *q, COX_EUNSUPPORTED, s->now());
                continue;
            }
            s->cv_stage.wait(lk, [s, &q] { return s->stop || s->stage_alloc.alloc(q->lay.upload, &q->stage_off); });
            if (s->stop) return;
        }
        write_image(*q, perm, meta, pos, s->staging + q->stage_off);
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->ready_q.push_back(std::move(q));
        }
        s->cv_ready.notify_all();
    }
}

// ------------------------------------------------------------------ worker

bool ensure_list(cox_server::List &l, size_t bytes, std::string &err)
{
    if (bytes <= l.cap) return true;
    size_t cap = std::max<size_t>(bytes, 2 * l.cap);
    cap = round_up(cap, 4096);
    if (l.h) (void)hipHostFree(l.h);
    if (l.d) (void)hipFree(l.d);
    l.h = l.d = nullptr;
    l.cap = 0;
    if (hipHostMalloc(reinterpret_cast<void **>(&l.h), cap, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&l.d), cap) != hipSuccess) {
        err = "allocating a work list";
        return false;
    }
    l.cap = cap;
    return true;
}

FitDesc make_desc(cox_server *s, const Request &q, size_t off, int slot)
{
    const FitLayout &L = q.lay;
    char *B = s->arena + off;
    FitDesc F{};
    F.x = reinterpret_cast<double *>(B + L.x);
    if (L.device) {
        F.xs = q.x;
        F.ldxs = q.ldx;
        F.src = reinterpret_cast<const int32_t *>(B + L.src);
    }
    F.xf = reinterpret_cast<float *>(B + L.xf);
    F.meta = reinterpret_cast<const uint32_t *>(B + L.meta);
    F.gidx = reinterpret_cast<const int32_t *>(B + L.gidx);
    double *rows = reinterpret_cast<double *>(B + L.rows);
    F.eta = rows;
    F.w = rows + L.ld;
    F.zq = rows + 2 * L.ld;
    F.hz = rows + 3 * L.ld;
    F.b = rows + 4 * L.ld;
    F.bf = reinterpret_cast<float *>(B + L.bf);
    F.z = reinterpret_cast<float *>(B + L.z);
    F.beta = reinterpret_cast<double *>(B + L.beta);
    F.prev = reinterpret_cast<double *>(B + L.prev);
    double *vec = reinterpret_cast<double *>(B + L.vec);
    F.grad = vec;
    F.diag1 = vec + L.p;
    F.diag2 = vec + 2 * L.p;
    F.free_col = reinterpret_cast<uint8_t *>(B + L.free_col);
    F.L = reinterpret_cast<double *>(B + L.L);
    F.part = reinterpret_cast<float *>(B + L.part);
    F.tilemax = reinterpret_cast<double *>(B + L.tilemax);
    F.tpart = reinterpret_cast<double *>(B + L.tpart);
    F.cpart = reinterpret_cast<double *>(B + L.cpart);
    F.st = s->d_state + slot;
    F.hst = s->dh_state + slot;
    F.hbeta = s->dh_beta + (size_t)slot * kMaxP;
    F.n = L.n;
    F.tile = L.tile;
    F.ntc = L.ntc;
    F.ld = L.ld;
    F.ldz = L.ldz;
    F.p = L.p;
    F.G = L.G;
    F.nxr = L.nxr;
    F.nzr = L.nzr;
    F.xrange = L.xrange;
    F.zrange = L.zrange;
    F.npairs = L.npairs;
    F.ntile = L.ntile;
    F.gam = q.gam.empty() ? nullptr : reinterpret_cast<const double *>(B + L.gam);
    F.beta0 = q.beta0.empty() ? nullptr : reinterpret_cast<const double *>(B + L.beta0);
    F.tol = s->opt.tol;
    F.max_iter = s->opt.max_iter;
    F.freeze = 1;
    return F;
}

// Host-side guard before a descriptor reaches the device: every array lies in
// the fit's own arena block and the state is the slot's entry.
bool check_desc(const cox_server *s, const FitDesc &F, const FitLayout &L, size_t off, int slot)
{
    const char *lo = s->arena + off, *hi = s->arena + off + L.total;
    auto in = [lo, hi](const void *ptr, size_t bytes) {
        const char *c = static_cast<const char *>(ptr);
        return c && c >= lo && c + bytes <= hi;
    };
    const size_t p = (size_t)L.p, ld = (size_t)L.ld;
    return in(F.x, 8 * p * ld) && in(F.xf, 4 * p * ld) && in(F.meta, 4 * ld) && in(F.gidx, 4 * ld) &&
           in(F.eta, 8 * ld) && in(F.w, 8 * ld) && in(F.zq, 8 * ld) && in(F.hz, 8 * ld) && in(F.b, 8 * ld) && in(F.bf, 4 * ld) && in(F.z, 4 * p * (size_t)L.ldz) && in(F.beta, 8 * p) &&
           in(F.prev, 8 * p) && in(F.grad, 8 * p) && in(F.diag2, 8 * p) && in(F.free_col, p) &&
           in(F.L, 8 * p * p) && in(F.part, 4 * (size_t)(L.nxr + L.nzr) * L.npairs * kTile * kTile) &&
           F.xrange % 256 == 0 && F.zrange % 256 == 0 && F.xrange >= kMinRange && F.xrange <= kMaxRange &&
           F.zrange >= kMinRange && F.zrange <= kMaxRange && (int64_t)F.nxr * F.xrange >= L.ld &&
           (F.nzr == 0 || (int64_t)F.nzr * F.zrange >= L.ldz) &&
           in(F.tilemax, 8 * (size_t)L.ntile) && in(F.tpart, 16 * (size_t)L.ntc) &&
           in(F.cpart, 24 * (size_t)L.ntc * p) && (!F.gam || in(F.gam, 8 * p)) && (!F.beta0 || in(F.beta0, 8 * p)) &&
           (!L.device || (in(F.src, 4 * ld) && F.xs && F.ldxs >= L.n)) && F.tile > 0 && F.tile % kRowPad == 0 && F.ntc >= 1 &&
           F.tile * F.ntc == F.ld &&
           F.st == s->d_state + slot && F.hst == s->dh_state + slot && F.hbeta == s->dh_beta + (size_t)slot * kMaxP &&
           F.p == L.p && F.ld == L.ld &&
           F.n <= F.ld && F.ld % kRowPad == 0 && F.ldz % kRowPad == 0 && F.G <= F.ldz && F.p >= 1 &&
           F.p <= kMaxP && F.ntile * (int64_t)kEtaRows >= F.ld;
}

// Everything the worker does per round; returns false on a device error (message in `err`).
constexpr int kRoundsAhead = 2;   // rounds queued on the compute stream at once
// Below this many (fit, K range) contraction items a round gives each tile pair its own items.
constexpr size_t kSyrkPerFitItems = 512;

struct WorkerState {
    std::vector<int> uploading;   // slots whose upload was queued in the previous round
    std::vector<int> upload_stage_release;
    hipEvent_t copy_ev = nullptr;
    hipEvent_t round_ev[kRoundsAhead] = {};
    bool copy_pending = false;
    int admit_buf = 0;
};

#define WCHECK(expr, what)                      \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) {                 \
            err = std::string(what) + ": " + hipGetErrorString(e_); \
            return false;                       \
        }                                       \
    } while (0)

// Carves the round block into typed arrays at 16-byte aligned offsets.
struct Packer {
    size_t used = 0;
    template <class T>
    size_t take(size_t count)
    {
        const size_t at = used;
        used = round_up(used + sizeof(T) * count, 16);
        return at;
    }
};

bool admit_ready(cox_server *s, WorkerState &ws, std::string &err)
{
    // take staged requests in order while a slot is free and the arena has room
    std::vector<std::pair<int, std::unique_ptr<Request>>> taken;
    {
        std::lock_guard<std::mutex> g(s->mu);
        while (!s->ready_q.empty()) {
            Request &q = *s->ready_q.front();
            int slot = -1;
            for (int i = 0; i < (int)s->slots.size(); ++i)
                if (!s->slots[i].used) {
                    slot = i;
                    break;
                }
            size_t off = 0;
            if (slot < 0 || !s->arena_alloc.alloc(q.lay.total, &off)) break;
            Slot &S = s->slots[slot];
            S.used = true;
            S.active = false;
            S.frozen = false;
            S.reported = false;
            S.arena_off = off;
            // the host mirror still holds the previous occupant's final state; no kernel
            // writes it until this fit's first step
            std::memset(static_cast<void *>(&s->h_state[slot]), 0, sizeof(FitState));
            S.t_admit = s->now();
            taken.emplace_back(slot, std::move(s->ready_q.front()));
            s->ready_q.pop_front();
        }
    }
    if (taken.empty()) return true;
    for (auto &tk : taken) {
        const int slot = tk.first;
        Request &q = *tk.second;
        Slot &S = s->slots[slot];
        char *B = s->arena + S.arena_off;
        s->h_desc[slot] = make_desc(s, q, S.arena_off, slot);
        if (!check_desc(s, s->h_desc[slot], q.lay, S.arena_off, slot)) {
            err = "internal error: a fit descriptor points outside its block";
            return false;
        }
        WCHECK(hipMemcpyAsync(B, s->staging + q.stage_off, q.lay.upload, hipMemcpyHostToDevice, s->copy),
               "uploading a fit");
        S.req = std::move(tk.second);
        ws.uploading.push_back(slot);
    }
    // after the uploads, on the same stream (so beside this round's iteration): the admit
    // kernel installs the descriptors, clears z, beta and the states, and forms the FP32
    // copies (gathering X of device-resident requests).  Its block alternates between two
    // buffers: the one used two admissions ago is free, since the round after that
    // admission waited for it.
    size_t n_items = 0;
    for (auto &tk : taken) n_items += (size_t)s->slots[tk.first].req->lay.ntile;
    Packer pk;
    const size_t o_jd = pk.take<FitDesc>(taken.size()), o_js = pk.take<int>(taken.size());
    const size_t o_it = pk.take<int2>(n_items);
    cox_server::List &l = s->l_admit[ws.admit_buf];
    ws.admit_buf ^= 1;
    if (!ensure_list(l, pk.used, err)) return false;
    FitDesc *jd = reinterpret_cast<FitDesc *>(l.h + o_jd);
    int *js = reinterpret_cast<int *>(l.h + o_js);
    int2 *items = reinterpret_cast<int2 *>(l.h + o_it);
    size_t ka = 0;
    for (size_t k = 0; k < taken.size(); ++k) {
        const int sl = taken[k].first;
        jd[k] = s->h_desc[sl];
        js[k] = sl;
        for (int t = 0; t < s->slots[sl].req->lay.ntile; ++t) items[ka++] = make_int2((int)k, t);
    }
    WCHECK(hipMemcpyAsync(l.d, l.h, pk.used, hipMemcpyHostToDevice, s->copy), "admit list");
    WCHECK((hipError_t)launch_admit(s->d_desc, reinterpret_cast<const FitDesc *>(l.d + o_jd),
                                    reinterpret_cast<const int *>(l.d + o_js), reinterpret_cast<const int2 *>(l.d + o_it),
                                    (int)ka, s->copy),
           "admit kernel");
    WCHECK(hipEventRecord(ws.copy_ev, s->copy), "recording the upload");
    ws.copy_pending = true;
    return true;
}

// The result of the fit in slot sl from its host-mapped state and estimate.
Result make_result(const cox_server *s, int sl, double t_done)
{
    const Slot &S = s->slots[sl];
    const FitState &st = s->h_state[sl];
    Result r;
    r.beta.assign(s->h_beta + (size_t)sl * kMaxP, s->h_beta + (size_t)sl * kMaxP + S.req->p);
    r.info.status = st.status;
    r.info.iters = st.iters;
    r.info.coord_evals = st.evals;
    r.info.objective = st.obj;
    r.info.kkt_inf = st.kkt;
    r.info.last_step = st.last_step;
    r.info.n_pinned = st.n_pinned;
    r.times.submit_s = S.req->t_submit;
    r.times.admit_s = S.t_admit;
    r.times.done_s = t_done;
    return r;
}

// Work lists of one round (or persistent launch) over the fits in `act`, written to the
// round block and copied to the device on the compute stream.
struct RoundLists {
    size_t o_eta = 0, o_rows = 0, o_cols = 0, o_syrk = 0, o_info = 0, o_slots = 0;
    size_t ke = 0, kr = 0, kc = 0, ks = 0, ki = 0;
    int ks_nt[5] = {0, 0, 0, 0, 0};   // contraction items: per tile pair, then of fits with 1..4 tiles
    bool per_pair = false;
    int max_p = 1;
};

bool build_lists(cox_server *s, const std::vector<int> &act, RoundLists &R, std::string &err)
{
    size_t n_eta = 0, n_rows = 0, n_cols = 0, n_syrk = 0, n_syrk_pairs = 0, n_info = 0;
    for (int sl : act) {
        const FitLayout &L = s->slots[sl].req->lay;
        n_eta += L.ntile;
        n_rows += L.ntc;
        n_cols += (size_t)L.ntc * ((L.p + kColBlock - 1) / kColBlock);
        if (!s->slots[sl].frozen) {
            n_syrk += (size_t)(L.nxr + L.nzr);
            n_syrk_pairs += (size_t)L.npairs * (L.nxr + L.nzr);
            n_info += L.npairs;
        }
    }
    // a light round spreads each fit's tile pairs over workgroups (shorter critical path); a heavy
    // one gives a workgroup all pairs of a K range (each row of X read once per range)
    const bool per_pair = n_syrk < kSyrkPerFitItems;
    if (per_pair) n_syrk = n_syrk_pairs;
    Packer pk;
    R.o_eta = pk.take<int2>(n_eta);
    R.o_rows = pk.take<int2>(n_rows);
    R.o_cols = pk.take<int2>(n_cols);
    R.o_syrk = pk.take<int4>(n_syrk);
    R.o_info = pk.take<int2>(n_info);
    R.o_slots = pk.take<int>(act.size());
    if (!ensure_list(s->l_round, pk.used, err)) return false;
    char *H = s->l_round.h, *D = s->l_round.d;
    int2 *eta = reinterpret_cast<int2 *>(H + R.o_eta);
    int2 *rws = reinterpret_cast<int2 *>(H + R.o_rows);
    int2 *cols = reinterpret_cast<int2 *>(H + R.o_cols);
    int4 *syrk = reinterpret_cast<int4 *>(H + R.o_syrk);
    int2 *info = reinterpret_cast<int2 *>(H + R.o_info);
    int *sl_list = reinterpret_cast<int *>(H + R.o_slots);
    size_t ke = 0, kr = 0, kc = 0, ks = 0, ki = 0;
    int max_p = 1;
    for (size_t a = 0; a < act.size(); ++a) {
        const int sl = act[a];
        const FitLayout &L = s->slots[sl].req->lay;
        sl_list[a] = sl;
        max_p = std::max(max_p, L.p);
        for (int t = 0; t < L.ntile; ++t) eta[ke++] = make_int2(sl, t);
        for (int t = 0; t < L.ntc; ++t) {
            rws[kr++] = make_int2(sl, t);
            for (int j = 0; j < L.p; j += kColBlock) cols[kc++] = make_int2(sl, (t << 10) | j);
        }
        if (!s->slots[sl].frozen)
            for (int pr = 0; pr < L.npairs; ++pr) info[ki++] = make_int2(sl, pr);
    }
    // contraction items: (fit, tile pair, K range, product), or (fit, 0, K range, product) grouped
    // by the fit's tile count
    R.per_pair = per_pair;
    if (per_pair) {
        for (int sl : act) {
            const FitLayout &L = s->slots[sl].req->lay;
            if (s->slots[sl].frozen) continue;
            for (int pr = 0; pr < L.npairs; ++pr) {
                for (int r = 0; r < L.nxr; ++r) syrk[ks++] = make_int4(sl, pr, r, 0);
                for (int r = 0; r < L.nzr; ++r) syrk[ks++] = make_int4(sl, pr, r, 1);
            }
        }
        R.ks_nt[0] = (int)ks;
    } else {
        for (int nt = 1; nt <= 4; ++nt) {
            const size_t ks0 = ks;
            for (int sl : act) {
                const FitLayout &L = s->slots[sl].req->lay;
                if (s->slots[sl].frozen || (L.p + kTile - 1) / kTile != nt) continue;
                for (int r = 0; r < L.nxr; ++r) syrk[ks++] = make_int4(sl, 0, r, 0);
                for (int r = 0; r < L.nzr; ++r) syrk[ks++] = make_int4(sl, 0, r, 1);
            }
            R.ks_nt[nt] = (int)(ks - ks0);
        }
    }
    if (ke != n_eta || kr != n_rows || kc != n_cols || ks != n_syrk || ki != n_info) {
        err = "internal error: work list sizes";
        return false;
    }
    R.ke = ke;
    R.kr = kr;
    R.kc = kc;
    R.ks = ks;
    R.ki = ki;
    R.max_p = max_p;
    WCHECK(hipMemcpyAsync(D, H, pk.used, hipMemcpyHostToDevice, s->compute), "work lists");
    return true;
}

// The fits of the next round: those resident and those whose upload was queued in the
// previous round (the compute stream waits for that upload).
bool next_round_fits(cox_server *s, WorkerState &ws, std::vector<int> &act, std::vector<int> &joining,
                     std::string &err)
{
    if (ws.copy_pending) {
        WCHECK(hipStreamWaitEvent(s->compute, ws.copy_ev, 0), "ordering the upload");
        joining.swap(ws.uploading);
        ws.copy_pending = false;
    }
    for (int i = 0; i < (int)s->slots.size(); ++i)
        if (s->slots[i].used && (s->slots[i].active || std::find(joining.begin(), joining.end(), i) != joining.end()))
            act.push_back(i);
    for (int sl : joining) s->slots[sl].active = true;
    return true;
}

// After a round or a launch: release the staging of the fits that joined, retire the
// finished fits (reporting those not reported yet), note which factors are frozen.
void retire_fits(cox_server *s, const std::vector<int> &act, const std::vector<int> &joining, double t_launch,
                 double t_done, int64_t rounds, double resident_rounds)
{
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (int sl : joining) s->stage_alloc.release(s->slots[sl].req->stage_off, s->slots[sl].req->lay.upload);
    }
    if (!joining.empty()) s->cv_stage.notify_all();
    std::vector<int> done;
    for (int sl : act) {
        const FitState &st = s->h_state[sl];
        if (st.flags & kDone) done.push_back(sl);
        else s->slots[sl].frozen = (st.flags & kFrozen) != 0;
    }
    std::lock_guard<std::mutex> g(s->mu);
    s->iterations += rounds;
    s->resident_sum += resident_rounds;
    s->resident_peak = std::max<int64_t>(s->resident_peak, (int64_t)act.size());
    s->gpu_busy_s += t_done - t_launch;
    for (int sl : done) {
        Slot &S = s->slots[sl];
        s->arena_alloc.release(S.arena_off, S.req->lay.total);
        if (!S.reported) finish_locked(s, S.req->ticket, make_result(s, sl, t_done));
        S = Slot();
    }
    if (!done.empty()) s->cv_done.notify_all();   // drain waits for the slots too
}

// While launched rounds run: report the fits whose host-mapped state says they are done (the
// step writes the estimate before the final state), admit staged requests once (uploads and
// the admit kernel on the copy stream), and decide to hold -- run no further rounds on these
// lists -- when fits are ready to join or waiting requests could take finished fits' places.
struct Watch {
    std::vector<char> seen;
    bool admitted = false, held = false;
};

bool watch(cox_server *s, WorkerState &ws, const std::vector<int> &act, Watch &W, std::string &err)
{
    std::vector<int> newly;
    for (size_t a = 0; a < act.size(); ++a)
        if (!W.seen[a] && (__atomic_load_n(&s->h_state[act[a]].flags, __ATOMIC_ACQUIRE) & kDone)) {
            W.seen[a] = 1;
            newly.push_back(act[a]);
        }
    bool waiting = false;
    if (!newly.empty() || !W.held) {
        std::lock_guard<std::mutex> g(s->mu);
        const double t = s->now();
        for (int sl : newly) {
            finish_locked(s, s->slots[sl].req->ticket, make_result(s, sl, t));
            s->slots[sl].reported = true;
        }
        waiting = !s->ready_q.empty() || s->stop;
    }
    if (!W.held) {
        if (waiting && !W.admitted) {
            if (!admit_ready(s, ws, err)) return false;
            W.admitted = ws.copy_pending;
        }
        bool any_done = false;
        for (char c : W.seen) any_done |= c != 0;
        if (W.admitted || (waiting && any_done)) W.held = true;
    }
    return true;
}

// Rounds as separate launches on one set of work lists, kRoundsAhead of them queued at once
// (the kernels leave out fits that finished in an earlier round), until every fit is done or
// the watch holds; then the fits are retired and the next call builds new lists.
bool run_round(cox_server *s, WorkerState &ws, std::string &err)
{
    // fits uploaded in the previous round join this round
    std::vector<int> joining, act;
    if (!next_round_fits(s, ws, act, joining, err)) return false;
    if (act.empty()) return admit_ready(s, ws, err);   // nothing resident
    const double t_launch = s->now();
    RoundLists R;
    if (!build_lists(s, act, R, err)) return false;
    std::vector<int> evals0(act.size());
    for (size_t a = 0; a < act.size(); ++a) evals0[a] = s->h_state[act[a]].evals;
    const char *D = s->l_round.d;
    int queued = 0, completed = 0;
    auto enqueue = [&]() -> bool {
        WCHECK((hipError_t)launch_eta(s->d_desc, reinterpret_cast<const int2 *>(D + R.o_eta), (int)R.ke, s->compute),
               "eta");
        WCHECK((hipError_t)launch_rows(s->d_desc, reinterpret_cast<const int2 *>(D + R.o_rows), (int)R.kr, s->compute),
               "rows");
        WCHECK((hipError_t)launch_cols(s->d_desc, reinterpret_cast<const int2 *>(D + R.o_cols), (int)R.kc, s->compute),
               "cols");
        if (R.ks) {
            WCHECK((hipError_t)launch_syrk(s->d_desc, reinterpret_cast<const int4 *>(D + R.o_syrk), R.ks_nt,
                                           s->compute),
                   "syrk");
            WCHECK((hipError_t)launch_info(s->d_desc, reinterpret_cast<const int2 *>(D + R.o_info), (int)R.ki,
                                           s->compute),
                   "info");
        }
        // the step kernel writes each fit's state (and a final estimate) to host-mapped memory
        WCHECK((hipError_t)launch_step(s->d_desc, reinterpret_cast<const int *>(D + R.o_slots), (int)act.size(),
                                       R.max_p, s->compute),
               "step");
        WCHECK(hipEventRecord(ws.round_ev[queued % kRoundsAhead], s->compute), "recording a round");
        queued += 1;
        return true;
    };
    if (!enqueue()) return false;
    Watch W;
    W.seen.assign(act.size(), 0);
    while (completed < queued) {
        if (queued - completed < kRoundsAhead && !W.held) {
            bool all_done = true;
            for (char c : W.seen) all_done &= c != 0;
            if (!all_done && !enqueue()) return false;
        }
        const hipError_t q = hipEventQuery(ws.round_ev[completed % kRoundsAhead]);
        if (q != hipSuccess && q != hipErrorNotReady) {
            err = std::string("round: ") + hipGetErrorString(q);
            return false;
        }
        if (q == hipSuccess) completed += 1;
        if (!watch(s, ws, act, W, err)) return false;
        if (q != hipSuccess) std::this_thread::yield();
    }
    double resident_rounds = 0.0;
    for (size_t a = 0; a < act.size(); ++a) resident_rounds += (double)(s->h_state[act[a]].evals - evals0[a]);
    retire_fits(s, act, joining, t_launch, s->now(), completed, resident_rounds);
    return true;
}

// One persistent launch of up to fused_rounds rounds over the resident fits.  While it runs
// the worker reports fits whose host-mapped state says they are done (the kernel writes
// the estimate before the final state), admits staged requests once (uploads and the
// admit kernel on the copy stream), and sets the hold word -- the launch then ends after
// its current round -- when fits are ready to join or waiting requests could take the
// place of finished ones.  Slots and arena blocks are released only after the launch.
bool run_launch_fused(cox_server *s, WorkerState &ws, std::string &err)
{
    std::vector<int> joining, act;
    if (!next_round_fits(s, ws, act, joining, err)) return false;
    const double t_launch = s->now();
    if (act.empty()) return admit_ready(s, ws, err);
    RoundLists R;
    if (!build_lists(s, act, R, err)) return false;
    if (R.max_p != s->round_grid_p) {
        int g = 0;
        WCHECK((hipError_t)round_grid(R.max_p, &g), "sizing the round launch");
        if (g < 1) {
            err = "the round kernel does not fit on the device";
            return false;
        }
        s->round_grid_p = R.max_p;
        s->round_grid = g;
    }
    // workgroups: one per item of the largest phase (items are dealt over workgroups first),
    // a multiple of the 8 XCDs, at most what fits on the device at once
    const size_t need = std::max({R.ke, R.kr, R.kc, R.ks, R.ki, act.size()});
    const int grid = (int)std::min<size_t>((size_t)s->round_grid, std::max<size_t>(8, (need + 7) / 8 * 8));
    std::vector<int> evals0(act.size());
    for (size_t a = 0; a < act.size(); ++a) evals0[a] = s->h_state[act[a]].evals;
    uint32_t *hold = reinterpret_cast<uint32_t *>(s->h_round);
    __atomic_store_n(hold, 0u, __ATOMIC_SEQ_CST);
    for (int k = 2; k < 10; ++k) s->h_round[k] = 0u;
    WCHECK(hipMemsetAsync(s->d_round_ctl, 0, round_ctl_bytes(), s->compute), "clearing the round control block");
    const char *D = s->l_round.d;
    RoundWork w{};
    w.fits = s->d_desc;
    w.eta = reinterpret_cast<const int2 *>(D + R.o_eta);
    w.rows = reinterpret_cast<const int2 *>(D + R.o_rows);
    w.cols = reinterpret_cast<const int2 *>(D + R.o_cols);
    w.syrk = reinterpret_cast<const int4 *>(D + R.o_syrk);
    w.info = reinterpret_cast<const int2 *>(D + R.o_info);
    w.slots = reinterpret_cast<const int *>(D + R.o_slots);
    w.ne = (int)R.ke;
    w.nr = (int)R.kr;
    w.nc = (int)R.kc;
    w.ns = (int)R.ks;
    w.ni = (int)R.ki;
    w.nf = (int)act.size();
    w.syrk_per_pair = R.per_pair ? 1 : 0;
    w.max_rounds = s->opt.fused_rounds;
    w.max_p = R.max_p;
    w.hold = reinterpret_cast<const uint32_t *>(s->dh_round);
    w.ctl = s->d_round_ctl;
    w.hout = s->dh_round + 2;
    WCHECK((hipError_t)launch_rounds(w, grid, s->compute), "round kernel");
    WCHECK(hipEventRecord(s->iter_ev, s->compute), "recording the launch");
    Watch W;
    W.seen.assign(act.size(), 0);
    for (;;) {
        const hipError_t q = hipEventQuery(s->iter_ev);
        if (q != hipSuccess && q != hipErrorNotReady) {
            err = std::string("round kernel: ") + hipGetErrorString(q);
            return false;
        }
        const bool was_held = W.held;
        if (!watch(s, ws, act, W, err)) return false;
        if (W.held && !was_held) __atomic_store_n(hold, 1u, __ATOMIC_SEQ_CST);
        if (q == hipSuccess) break;
        std::this_thread::yield();
    }
    const double t_done = s->now();
    if (s->h_round[3] != 0u) {
        err = "round kernel: a grid-wide wait timed out; results are not valid";
        return false;
    }
    double resident_rounds = 0.0;
    for (size_t a = 0; a < act.size(); ++a) resident_rounds += (double)(s->h_state[act[a]].evals - evals0[a]);
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->launches += 1;
        for (int k = 0; k < 6; ++k) s->phase_s[k] += 1e-8 * (double)s->h_round[4 + k];   // 100 MHz clock
    }
    retire_fits(s, act, joining, t_launch, t_done, (int64_t)s->h_round[2], resident_rounds);
    return true;
}

void worker_loop(cox_server *s)
{
    (void)hipSetDevice(s->device);
    WorkerState ws;
    std::string err;
    bool ev_ok = hipEventCreateWithFlags(&ws.copy_ev, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < kRoundsAhead && ev_ok; ++k)
        ev_ok = hipEventCreateWithFlags(&ws.round_ev[k], hipEventDisableTiming) == hipSuccess;
    if (!ev_ok) {
        std::lock_guard<std::mutex> g(s->mu);
        s->fatal = COX_EDEVICE;
        s->fatal_msg = "creating an event";
    }
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->fatal) break;
            bool any_resident = false;
            for (const Slot &S : s->slots) any_resident |= S.used;
            if (!any_resident) {
                s->cv_ready.wait(lk, [s] { return s->stop || !s->ready_q.empty(); });
                if (s->stop) break;
            } else if (s->stop) {
                break;
            }
        }
        if (!(s->opt.fused_rounds > 0 ? run_launch_fused(s, ws, err) : run_round(s, ws, err))) {
            std::lock_guard<std::mutex> g(s->mu);
            s->fatal = COX_EDEVICE;
            s->fatal_msg = err;
            break;
        }
    }
    (void)hipStreamSynchronize(s->copy);
    (void)hipStreamSynchronize(s->compute);
    if (ws.copy_ev) (void)hipEventDestroy(ws.copy_ev);
    for (hipEvent_t e : ws.round_ev)
        if (e) (void)hipEventDestroy(e);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->fatal) {
        // fail everything still outstanding
        const double t = s->now();
        for (Slot &S : s->slots)
            if (S.used && S.req) {
                fail_request_locked(s, *S.req, s->fatal, t);
                S = Slot();
            }
        for (auto &q : s->ready_q) fail_request_locked(s, *q, s->fatal, t);
        s->ready_q.clear();
        for (auto &q : s->prep_q) fail_request_locked(s, *q, s->fatal, t);
        s->prep_q.clear();
        s->stop = true;
        s->cv_prep.notify_all();
        s->cv_stage.notify_all();
    }
    s->cv_done.notify_all();
}

void free_server(cox_server *s)
{
    if (s->arena) (void)hipFree(s->arena);
    if (s->d_desc) (void)hipFree(s->d_desc);
    if (s->d_state) (void)hipFree(s->d_state);
    if (s->staging) (void)hipHostFree(s->staging);
    if (s->h_desc) (void)hipHostFree(s->h_desc);
    if (s->h_state) (void)hipHostFree(s->h_state);
    if (s->h_beta) (void)hipHostFree(s->h_beta);
    if (s->d_round_ctl) (void)hipFree(s->d_round_ctl);
    if (s->h_round) (void)hipHostFree(s->h_round);
    for (cox_server::List *l : {&s->l_round, &s->l_admit[0], &s->l_admit[1]}) {
        if (l->h) (void)hipHostFree(l->h);
        if (l->d) (void)hipFree(l->d);
    }
    if (s->iter_ev) (void)hipEventDestroy(s->iter_ev);
    if (s->compute) (void)hipStreamDestroy(s->compute);
    if (s->copy) (void)hipStreamDestroy(s->copy);
}

}  // namespace

extern "C" void cox_server_default_options(cox_server_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->hbm_budget = (size_t)8 << 30;
    o->staging_bytes = (size_t)1 << 30;
    o->max_resident = 1024;
    o->prep_threads = 8;
    o->x_precision = COX_F32;
    o->tol = 1e-12;
    o->max_iter = 100;
    o->device = -1;
    o->fused_rounds = 0;
}

extern "C" int cox_server_create(cox_server **out, const cox_server_options *o)
{
    if (!out) return COX_EINVAL;
    *out = nullptr;
    cox_server_options opt;
    if (o) opt = *o;
    else cox_server_default_options(&opt);
    if (opt.x_precision != COX_F32) {
        g_create_error = "the server forms the information matrix in FP32 (x_precision = COX_F32)";
        return COX_EUNSUPPORTED;
    }
    if (opt.hbm_budget < ((size_t)1 << 20) || opt.staging_bytes < ((size_t)1 << 20) || opt.max_resident < 1 ||
        opt.prep_threads < 1 || !(opt.tol >= 0.0) || opt.max_iter < 1 || opt.fused_rounds < 0 ||
        opt.fused_rounds > 4096) {
        g_create_error = "invalid server options";
        return COX_EINVAL;
    }
    std::unique_ptr<cox_server> s(new cox_server());
    s->opt = opt;
    s->t0 = std::chrono::steady_clock::now();
    if (opt.device >= 0) {
        if (hipSetDevice(opt.device) != hipSuccess) {
            g_create_error = "hipSetDevice failed";
            return COX_EDEVICE;
        }
    }
    if (hipGetDevice(&s->device) != hipSuccess) {
        g_create_error = "no HIP device";
        return COX_EDEVICE;
    }
    const size_t ns = (size_t)opt.max_resident;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&s->iter_ev, hipEventDisableTiming)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&s->arena), opt.hbm_budget)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&s->d_desc), sizeof(FitDesc) * ns)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&s->d_state), sizeof(FitState) * ns)) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void **>(&s->staging), opt.staging_bytes, hipHostMallocDefault)) !=
            hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void **>(&s->h_desc), sizeof(FitDesc) * ns, hipHostMallocDefault)) !=
            hipSuccess ||
        // written by the step kernel, read by the worker after each iteration's event
        (e = hipHostMalloc(reinterpret_cast<void **>(&s->h_state), sizeof(FitState) * ns,
                           hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void **>(&s->h_beta), sizeof(double) * kMaxP * ns,
                           hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess ||
        (e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->dh_state), s->h_state, 0)) != hipSuccess ||
        (e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->dh_beta), s->h_beta, 0)) != hipSuccess ||
        (e = hipMalloc(&s->d_round_ctl, round_ctl_bytes())) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void **>(&s->h_round), 16 * sizeof(uint64_t),
                           hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess ||
        (e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->dh_round), s->h_round, 0)) != hipSuccess) {
        g_create_error = std::string("server allocation: ") + hipGetErrorString(e);
        free_server(s.get());
        return e == hipErrorOutOfMemory ? COX_ENOMEM : COX_EDEVICE;
    }
    s->arena_alloc.reset(opt.hbm_budget);
    s->stage_alloc.reset(opt.staging_bytes);
    s->slots.resize(ns);
    cox_server *raw = s.release();
    for (int i = 0; i < opt.prep_threads; ++i) raw->preps.emplace_back(prep_loop, raw);
    raw->worker = std::thread(worker_loop, raw);
    *out = raw;
    return COX_OK;
}

static int submit_impl(cox_server *s, const cox_data *d, int flags, const cox_fit_request *r, uint64_t *ticket)
{
    if (!s) return COX_EINVAL;
    if (!d || !ticket) return srv_fail(s, COX_EINVAL, "data and ticket are required");
    if (r) {
        if (!(r->gamma >= 0.0) || !std::isfinite(r->gamma)) return srv_fail(s, COX_EINVAL, "gamma must be finite and >= 0");
        if (r->beta0)
            for (int64_t j = 0; j < d->p; ++j)
                if (!std::isfinite(r->beta0[j])) return srv_fail(s, COX_EINVAL, "beta0 must be finite");
    }
    if (flags & ~(COX_SUBMIT_BORROW | COX_SUBMIT_DEVICE)) return srv_fail(s, COX_EINVAL, "unknown submit flags");
    const bool dev = (flags & COX_SUBMIT_DEVICE) != 0 || d->on_device;
    if (dev) {
        // shape and placement now; the keys are checked once the prep thread has them
        if (d->n < 1 || d->p < 1 || d->ldx < d->n || d->n > (int64_t)kCountMask)
            return srv_fail(s, COX_EINVAL, "need n >= 1, p >= 1, ldx >= n, n < 2^29");
        const void *ptrs[4] = {d->x, d->time, d->event, d->stratum};
        const size_t n = (size_t)d->n;
        const size_t bytes[4] = {sizeof(double) * ((size_t)d->ldx * (size_t)(d->p - 1) + n), sizeof(double) * n, n,
                                 sizeof(int32_t) * n};
        for (int k = 0; k < 4; ++k) {
            if (!ptrs[k]) {
                if (k == 3) continue;
                return srv_fail(s, COX_EINVAL, "x, time and event are required");
            }
            if (!device_range_ok(ptrs[k], bytes[k], s->device))
                return srv_fail(s, COX_EINVAL, "COX_SUBMIT_DEVICE needs device memory of the server's device, "
                                               "each array inside one allocation");
        }
    } else if (const char *bad = check_data(d->n, d->p, d->ldx, d->x, d->time, d->event)) {
        return srv_fail(s, COX_EINVAL, bad);
    }
    if (d->p > kMaxP) return srv_fail(s, COX_EUNSUPPORTED, "the server fits at most 128 columns");
    std::unique_ptr<Request> q(new Request());
    q->n = d->n;
    q->p = d->p;
    if (r && r->gamma > 0.0) {
        q->gam.assign((size_t)d->p, r->gamma);
        if (r->penalize)
            for (int64_t j = 0; j < d->p; ++j) q->gam[(size_t)j] = r->penalize[j] ? r->gamma : 0.0;
    }
    if (r && r->beta0) q->beta0.assign(r->beta0, r->beta0 + d->p);
    if (dev) {
        q->device = true;
        q->x = d->x;
        q->ldx = d->ldx;
        q->time = d->time;
        q->event = d->event;
        q->stratum = d->stratum;
    } else if (flags & COX_SUBMIT_BORROW) {
        q->x = d->x;
        q->ldx = d->ldx;
        q->time = d->time;
        q->event = d->event;
        q->stratum = d->stratum;
    } else {
        q->own_x.resize((size_t)d->n * d->p);
        for (int64_t j = 0; j < d->p; ++j)
            std::memcpy(q->own_x.data() + j * d->n, d->x + j * d->ldx, sizeof(double) * d->n);
        q->own_t.assign(d->time, d->time + d->n);
        q->own_e.assign(d->event, d->event + d->n);
        if (d->stratum) q->own_s.assign(d->stratum, d->stratum + d->n);
        q->x = q->own_x.data();
        q->ldx = d->n;
        q->time = q->own_t.data();
        q->event = q->own_e.data();
        q->stratum = d->stratum ? q->own_s.data() : nullptr;
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->fatal) {
            s->err = s->fatal_msg;
            return s->fatal;
        }
        if (s->stop) return COX_EINVAL;
        q->ticket = s->next_ticket++;
        q->t_submit = s->now();
        *ticket = q->ticket;
        s->pending[q->ticket] = 1;
        s->outstanding += 1;
        s->submitted += 1;
        s->prep_q.push_back(std::move(q));
    }
    s->cv_prep.notify_one();
    return COX_OK;
}

extern "C" int cox_server_submit(cox_server *s, const cox_data *d, int flags, uint64_t *ticket)
{
    return submit_impl(s, d, flags, nullptr, ticket);
}

extern "C" int cox_server_submit_fit(cox_server *s, const cox_data *d, int flags, const cox_fit_request *r,
                                     uint64_t *ticket)
{
    return submit_impl(s, d, flags, r, ticket);
}

extern "C" int cox_server_poll(cox_server *s, uint64_t ticket, double *beta_out, cox_fit_info *info,
                               cox_request_times *times)
{
    if (!s) return COX_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) {
        if (s->pending.count(ticket)) return 1;
        s->err = "unknown or already collected ticket";
        return COX_EINVAL;
    }
    if (beta_out) std::memcpy(beta_out, it->second.beta.data(), sizeof(double) * it->second.beta.size());
    if (info) *info = it->second.info;
    if (times) *times = it->second.times;
    s->results.erase(it);
    return COX_OK;
}

extern "C" int cox_server_wait(cox_server *s, uint64_t ticket, double timeout_s)
{
    if (!s) return COX_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->results.count(ticket) && !s->pending.count(ticket)) return COX_EINVAL;
    auto ready = [s, ticket] { return s->results.count(ticket) > 0 || s->fatal != 0; };
    if (timeout_s < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) return 1;
    return s->results.count(ticket) ? COX_OK : s->fatal;
}

extern "C" int cox_server_drain(cox_server *s, double timeout_s)
{
    if (!s) return COX_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto idle = [s] {
        if (s->outstanding != 0) return false;
        for (const Slot &S : s->slots)
            if (S.used) return false;
        return true;
    };
    auto ready = [s, &idle] { return s->fatal != 0 || idle(); };
    if (timeout_s < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) return 1;
    return idle() ? COX_OK : s->fatal;
}

extern "C" int cox_server_stats(cox_server *s, cox_server_counters *st)
{
    if (!s || !st) return COX_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->iterations = s->iterations;
    int64_t resident = 0;
    for (const Slot &S : s->slots) resident += S.used ? 1 : 0;
    st->resident_now = resident;
    st->resident_peak = s->resident_peak;
    st->mean_resident = s->iterations ? s->resident_sum / (double)s->iterations : 0.0;
    st->arena_bytes = s->arena_alloc.capacity();
    st->arena_peak = s->arena_alloc.peak();
    st->gpu_busy_s = s->gpu_busy_s;
    st->now_s = s->now();
    st->launches = s->launches;
    for (int k = 0; k < 6; ++k) st->phase_s[k] = s->phase_s[k];
    return COX_OK;
}

extern "C" const char *cox_server_last_error(cox_server *s)
{
    if (!s) return g_create_error.c_str();
    static thread_local std::string copy;
    std::lock_guard<std::mutex> g(s->mu);
    copy = s->err;
    return copy.c_str();
}

extern "C" void cox_server_destroy(cox_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_prep.notify_all();
    s->cv_ready.notify_all();
    s->cv_stage.notify_all();
    for (auto &t : s->preps) t.join();
    if (s->worker.joinable()) s->worker.join();
    free_server(s);
    delete s;
}
