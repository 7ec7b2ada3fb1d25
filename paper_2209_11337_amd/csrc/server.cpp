// server.cpp -- continuous batching of Greek requests on one device.
//
// A worker thread owns two launch slots (stream + workspace each).  While one
// launch runs, the worker packs the next runnable work into the other slot
// and enqueues it, so work of requests that arrived meanwhile overlaps on the
// device with work already running.  Requests are admitted in arrival order
// as long as their device footprint fits the HBM budget.
//
// Point schedule: a request starts with 2^14 points per replication; once a
// round is complete its standard errors predict how many points the target
// needs (error ~ n^-3/4, between the Monte Carlo and QMC rates), and the next
// round extends the point set to that power of two (Sobol points extend, so
// all earlier sums are kept), at least doubling, up to 2^22.
//
// Launch size: a launch carries at most ~kLaunchPathDates path-dates.  A
// large round is cut into point ranges (slices, at most kMaxSlicePoints
// points) that ride in successive launches, so a request that arrives behind
// it waits for one bounded launch rather than for the whole round.
//
// Device memory: the launches' workspaces are the server's only device
// buffers beyond the resident tables.  Each of the two slots may hold at
// most half the HBM budget; a launch is packed only with slices whose bytes
// (as the launch workspace lays them out) fit what is left of its slot, so
// the workspaces together never exceed the budget.  A queued request is
// admitted when its smallest slice (one QCPW_CHUNK of points) fits the
// launch being packed; one that cannot fit an empty slot is refused at
// submission.
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
#include <thread>
#include <vector>

#include "qcpw_host.h"

namespace qcpw {

static constexpr int64_t kFirstPoints = int64_t(1) << 14;
static constexpr int64_t kMaxPoints = int64_t(1) << 22;
static constexpr int64_t kMaxSlicePoints = kMaxPoints / 2;
static constexpr int kMaxBatchOptions = 8192;
static constexpr int kSlots = 2;
static constexpr double kLaunchPathDates = 2.0e10;   // ~25 ms of FP32-mixed work

enum ReqState { RQ_QUEUED, RQ_RUNNING, RQ_DONE, RQ_CANCELLED };

struct Request {
    uint64_t id = 0;
    std::vector<qcpw_option_spec> specs;
    int n_shifts = 0, path = 0;
    double target = 0.0;
    ReqState state = RQ_QUEUED;
    bool in_flight = false;
    int64_t n_done = 0;            // points per replication already summed
    int64_t n_target = 0;          // end of the current round
    int64_t n_issued = 0;          // points handed to launches (n_done <= n_issued <= n_target)
    int slices_in_flight = 0;
    double cost_per_point = 0.0;   // path-dates per point (all options, all replications)
    std::vector<double> S, Cc;     // [n_opts][L][4] compensated sums of F over points
    std::vector<double> greeks, stderr_;
    bool collected = false;        // cancelled and reported while a launch still held it
};

// Device bytes a slice of len points of request r adds to a launch: per
// option its constants, unit-prefix entry and per-replication means in the
// workspace, its outputs (greeks, standard errors, per-replication means),
// and 8 doubles per work unit (ws_layout and qcpw_unit_points give the
// units).
static int64_t slice_bytes(const Request *r, int64_t len)
{
    const bool pca_like = r->path == QCPW_PATH_PCA || r->path == QCPW_PATH_PCA_FULL;
    const int64_t up = pca_like ? QCPW_CHUNK : qcpw_unit_points(len);
    const int64_t n = (int64_t)r->specs.size(), L = r->n_shifts;
    const int64_t units = (len + up - 1) / up * L;
    return n * ((int64_t)sizeof(OptDev) + (int64_t)sizeof(int64_t) + 2 * L * 4 * (int64_t)sizeof(double) +
                2 * 4 * (int64_t)sizeof(double) + units * 8 * (int64_t)sizeof(double));
}

// Bytes of a launch that do not scale with its options: region alignment,
// the work-queue heads, the prefix's last entry, output alignment, and the
// FP64 full-covariance scratch tiles.
static int64_t launch_fixed_bytes(int path, int precision, int n_cu)
{
    int64_t b = 16 * 256 + QCPW_QUEUES * QCPW_QUEUE_STRIDE * 8 + 8;
    if (path == QCPW_PATH_PCA_FULL && precision == QCPW_FP64)
        b += (int64_t)2 * std::max(n_cu, 1) * 64 * QCPW_MAX_D_PCA_FULL * (int64_t)sizeof(double);
    return b;
}

struct Slot {
    hipStream_t stream = nullptr;
    Workspace ws;
    bool busy = false;
    int64_t bytes = 0;                 // accounted device bytes of the launch it holds
    std::vector<Request *> reqs;
    std::vector<int64_t> k0, len;      // point slice of each request in the launch
    std::vector<int> first_opt;        // first option of each request in the launch
    std::vector<double> per_shift;     // host copy [n][L][4]
    std::vector<double> g, e;
    double *d_g = nullptr, *d_e = nullptr, *d_ps = nullptr;
    int L = 0;
    int n = 0;
};

}  // namespace qcpw

struct qcpw_server {
    qcpw::Context *ctx = nullptr;
    qcpw_run_config cfg;
    int64_t budget = 0;                // device bytes of both slots' workspaces together
    int64_t in_use = 0, peak = 0;      // accounted bytes of the launches in flight
    int64_t n_admitted = 0, n_completed = 0, n_cancelled = 0, n_launches = 0;
    uint64_t next_id = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<uint64_t, std::unique_ptr<qcpw::Request>> reqs;
    std::deque<uint64_t> queue;       // admitted order of queued requests
    bool stop = false;
    std::thread worker;
    qcpw::Slot slots[qcpw::kSlots];
};

namespace qcpw {

static void finish_locked(qcpw_server *s, Request *r, ReqState st)
{
    // slices still in launches keep r->in_flight, and their bytes stay
    // accounted to the slot, until the launch is retired
    r->state = st;
    if (st == RQ_DONE) ++s->n_completed;
    if (st == RQ_CANCELLED) ++s->n_cancelled;
    s->cv_done.notify_all();
}

static int64_t slot_cap(const qcpw_server *s) { return s->budget / kSlots; }

// Pick the work of one launch (caller holds the lock): running requests
// with points left in their round, then newly admitted ones, each with one
// slice, until the launch's path-date budget or its slot's memory is used.
// A slice is as long as the round's remaining points, the path-date budget,
// kMaxSlicePoints and the slot's memory allow, a multiple of QCPW_CHUNK.
// All requests of a launch share path construction and replication count;
// the oldest runnable request decides which.  *bytes receives the launch's
// accounted device bytes.
static void pick_batch_locked(qcpw_server *s, std::vector<Request *> &out, std::vector<int64_t> &k0,
                              std::vector<int64_t> &len, int64_t *bytes)
{
    out.clear();
    k0.clear();
    len.clear();
    int group_path = -1, group_L = -1;
    int n_opts = 0;
    double budget = kLaunchPathDates;
    int64_t mem = 0;
    auto fits_group = [&](Request *r) {
        if (group_path < 0) {
            group_path = r->path;
            group_L = r->n_shifts;
            mem = slot_cap(s) - launch_fixed_bytes(r->path, s->cfg.precision, s->ctx->tab.n_cu);
        }
        return r->path == group_path && r->n_shifts == group_L;
    };
    // the longest slice of r that fits the path-date budget and the memory
    // left, 0 if not even one chunk fits the memory
    auto slice_len = [&](Request *r) -> int64_t {
        int64_t l = std::min(r->n_target - r->n_issued, kMaxSlicePoints);
        int64_t cap = (int64_t)(budget / r->cost_per_point) / QCPW_CHUNK * QCPW_CHUNK;
        l = std::min(l, std::max(cap, (int64_t)QCPW_CHUNK));
        while (l > QCPW_CHUNK && slice_bytes(r, l) > mem) l = std::max<int64_t>(QCPW_CHUNK, l / 2 / QCPW_CHUNK * QCPW_CHUNK);
        return slice_bytes(r, l) <= mem ? l : 0;
    };
    auto take = [&](Request *r, int64_t l) {
        out.push_back(r);
        k0.push_back(r->n_issued);
        len.push_back(l);
        r->n_issued += l;
        r->slices_in_flight += 1;
        r->in_flight = true;
        budget -= (double)l * r->cost_per_point;
        mem -= slice_bytes(r, l);
        n_opts += (int)r->specs.size();
    };
    for (auto &kv : s->reqs) {   // ids increase with arrival: FIFO
        Request *r = kv.second.get();
        if (budget <= 0.0) break;
        if (r->state != RQ_RUNNING || r->n_issued >= r->n_target) continue;
        if (!fits_group(r)) continue;
        if (n_opts + (int)r->specs.size() > kMaxBatchOptions && !out.empty()) break;
        const int64_t l = slice_len(r);
        if (l > 0) take(r, l);
    }
    while (!s->queue.empty() && budget > 0.0) {
        auto it = s->reqs.find(s->queue.front());
        if (it == s->reqs.end() || it->second->state != RQ_QUEUED) {
            s->queue.pop_front();
            continue;
        }
        Request *r = it->second.get();
        if (n_opts + (int)r->specs.size() > kMaxBatchOptions && !out.empty()) break;
        if (!fits_group(r)) break;
        r->n_target = kFirstPoints;
        const int64_t l = slice_len(r);
        if (l == 0) break;                                           // wait for memory
        s->queue.pop_front();
        r->state = RQ_RUNNING;
        ++s->n_admitted;
        take(r, l);
    }
    *bytes = out.empty() ? 0 : slot_cap(s) - mem;
}

static qcpw_status enqueue_slot(qcpw_server *s, Slot &sl, std::vector<Request *> &batch,
                                const std::vector<int64_t> &k0, const std::vector<int64_t> &len, int64_t bytes)
{
    std::vector<qcpw_option_spec> specs;
    std::vector<int64_t> kb;
    sl.reqs = batch;
    sl.k0 = k0;
    sl.len = len;
    sl.first_opt.clear();
    for (size_t bi = 0; bi < batch.size(); ++bi) {
        Request *r = batch[bi];
        sl.first_opt.push_back((int)specs.size());
        for (const auto &sp : r->specs) {
            qcpw_option_spec x = sp;
            x.n_points = len[bi];
            specs.push_back(x);
            kb.push_back(k0[bi]);
        }
    }
    const int n = (int)specs.size();
    const int L = batch[0]->n_shifts;
    LaunchPlan lp;
    qcpw_status st;
    {
        std::lock_guard<std::mutex> lk(s->ctx->mu);   // plan_launch may add PCA factors
        st = plan_launch(s->ctx, specs.data(), n, 0, 0, L, batch[0]->path, s->cfg.precision, s->cfg.pca_gemm,
                         s->cfg.block_threads, lp, kb.data(), (s->cfg.flags & QCPW_FLAG_OWEN) != 0);
    }
    if (st != QCPW_OK) return st;
    const size_t need = launch_workspace_bytes(lp);
    const size_t out_bytes = ((size_t)n * 4 * sizeof(double) + 255) / 256 * 256;
    const size_t ps_bytes = ((size_t)n * L * 4 * sizeof(double) + 255) / 256 * 256;
    const size_t total = need + 2 * out_bytes + ps_bytes;
    if ((int64_t)total > bytes)
        return fail(QCPW_ENOMEM, "launch needs " + std::to_string(total) + " bytes, " + std::to_string(bytes) +
                                     " were accounted");
    st = sl.ws.ensure(total, (size_t)slot_cap(s));   // never more than the slot's share of the budget
    if (st != QCPW_OK) return st;
    char *base = (char *)sl.ws.ptr;
    sl.d_g = (double *)(base + need);
    sl.d_e = (double *)(base + need + out_bytes);
    sl.d_ps = (double *)(base + need + 2 * out_bytes);
    sl.n = n;
    sl.L = L;
    st = enqueue_launch(s->ctx, lp, sl.stream, sl.d_g, sl.d_e, sl.d_ps, base, need);
    if (st != QCPW_OK) return st;
    sl.per_shift.resize((size_t)n * L * 4);
    QCPW_HIP(hipMemcpyAsync(sl.per_shift.data(), sl.d_ps, (size_t)n * L * 4 * sizeof(double),
                            hipMemcpyDeviceToHost, sl.stream));
    sl.busy = true;
    return QCPW_OK;
}

// Next round end after a complete round: the largest ratio of standard
// error to target predicts the points needed with error ~ n^-3/4.
static int64_t next_round_end(const Request *r, double worst_ratio)
{
    const double factor = std::pow(std::max(worst_ratio, 1.0), 4.0 / 3.0) * 1.2;
    int64_t n = 2 * r->n_done;
    while ((double)n < (double)r->n_done * factor && n < kMaxPoints) n *= 2;
    return std::min(n, kMaxPoints);
}

// Fold a finished launch into its requests (caller holds the lock).
static void absorb_slot_locked(qcpw_server *s, Slot &sl)
{
    for (size_t bi = 0; bi < sl.reqs.size(); ++bi) {
        Request *r = sl.reqs[bi];
        r->slices_in_flight -= 1;
        r->in_flight = r->slices_in_flight > 0;
        if (r->state == RQ_CANCELLED) {
            if (r->collected && !r->in_flight) s->reqs.erase(r->id);
            continue;
        }
        const int n = (int)r->specs.size(), L = r->n_shifts;
        const double len = (double)sl.len[bi];
        if (r->S.empty()) {
            r->S.assign((size_t)n * L * 4, 0.0);
            r->Cc.assign((size_t)n * L * 4, 0.0);
        }
        for (int i = 0; i < n; ++i)
            for (int l = 0; l < L; ++l)
                for (int k = 0; k < 4; ++k) {
                    const size_t src = ((size_t)(sl.first_opt[bi] + i) * L + l) * 4 + k;
                    const size_t dst = ((size_t)i * L + l) * 4 + k;
                    const double x = sl.per_shift[src] * len;
                    const double t = r->S[dst] + x, bp = t - r->S[dst];
                    r->Cc[dst] += (r->S[dst] - (t - bp)) + (x - bp);
                    r->S[dst] = t;
                }
        r->n_done += sl.len[bi];
        if (r->n_done < r->n_target) continue;   // round not complete yet
        // mean and standard error over replications
        r->greeks.assign((size_t)n * 4, 0.0);
        r->stderr_.assign((size_t)n * 4, 0.0);
        double worst = 0.0;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < 4; ++k) {
                double m = 0.0;
                for (int l = 0; l < L; ++l) {
                    const size_t id = ((size_t)i * L + l) * 4 + k;
                    m += (r->S[id] + r->Cc[id]) / (double)r->n_done;
                }
                m /= L;
                double v = 0.0;
                for (int l = 0; l < L; ++l) {
                    const size_t id = ((size_t)i * L + l) * 4 + k;
                    const double dv = (r->S[id] + r->Cc[id]) / (double)r->n_done - m;
                    v += dv * dv;
                }
                const double se = L >= 2 ? std::sqrt(v / ((double)L * (L - 1))) : NAN;
                r->greeks[(size_t)i * 4 + k] = m;
                r->stderr_[(size_t)i * 4 + k] = se;
                if (k >= 1) {
                    const double ratio = se / (r->target * std::max(1.0, std::fabs(m)));
                    worst = std::isnan(ratio) ? INFINITY : std::max(worst, ratio);
                }
            }
        if (worst <= 1.0 || r->n_done >= kMaxPoints) finish_locked(s, r, RQ_DONE);
        else r->n_target = next_round_end(r, std::min(worst, 1e6));
    }
    sl.reqs.clear();
    sl.busy = false;
    s->in_use -= sl.bytes;
    sl.bytes = 0;
    ++s->n_launches;
}

static void fail_slot_locked(qcpw_server *s, Slot &sl)
{
    for (Request *r : sl.reqs) {
        r->slices_in_flight -= 1;
        r->in_flight = r->slices_in_flight > 0;
        if (r->state == RQ_QUEUED || r->state == RQ_RUNNING) finish_locked(s, r, RQ_CANCELLED);
        if (r->collected && !r->in_flight) s->reqs.erase(r->id);
    }
    sl.reqs.clear();
    sl.busy = false;
    s->in_use -= sl.bytes;
    sl.bytes = 0;
}

static bool work_available_locked(qcpw_server *s)
{
    if (!s->queue.empty()) return true;
    for (auto &kv : s->reqs)
        if (kv.second->state == RQ_RUNNING && kv.second->n_issued < kv.second->n_target) return true;
    return false;
}

static void retire_slot(qcpw_server *s, Slot &sl)
{
    const hipError_t q = hipStreamSynchronize(sl.stream);
    std::lock_guard<std::mutex> lk(s->mu);
    if (q == hipSuccess) absorb_slot_locked(s, sl);
    else fail_slot_locked(s, sl);
}

static void worker_main(qcpw_server *s)
{
    // without its device the worker enqueues nothing and cancels every batch
    const bool dev_ok = hipSetDevice(s->ctx->tab.device) == hipSuccess;
    uint64_t seq = 0, slot_seq[kSlots] = {};
    for (;;) {
        std::vector<Request *> batch;
        std::vector<int64_t> bk0, blen;
        int64_t bytes = 0;
        int free_slot = -1, busy = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (auto &sl : s->slots) busy += sl.busy;
            if (busy == 0) {
                s->cv_work.wait(lk, [&] { return s->stop || work_available_locked(s); });
                if (s->stop) break;
            }
            if (s->stop) break;   // launches in flight are retired below
            for (int i = 0; i < kSlots; ++i)
                if (!s->slots[i].busy) {
                    free_slot = i;
                    break;
                }
            if (free_slot >= 0) {
                pick_batch_locked(s, batch, bk0, blen, &bytes);
                if (!batch.empty()) {
                    s->slots[free_slot].bytes = bytes;
                    s->in_use += bytes;
                    s->peak = std::max(s->peak, s->in_use);
                }
            }
        }
        if (!batch.empty()) {
            Slot &sl = s->slots[free_slot];
            if (dev_ok && enqueue_slot(s, sl, batch, bk0, blen, bytes) == QCPW_OK) {
                slot_seq[free_slot] = ++seq;
                ++busy;
            } else {
                std::lock_guard<std::mutex> lk(s->mu);
                sl.reqs = batch;
                fail_slot_locked(s, sl);
            }
        }
        // Wait for the oldest launch when every slot is busy, or when there is
        // nothing new to enqueue; otherwise go round and fill the free slot.
        if (busy == kSlots || (batch.empty() && busy > 0)) {
            int oldest = -1;
            for (int i = 0; i < kSlots; ++i)
                if (s->slots[i].busy && (oldest < 0 || slot_seq[i] < slot_seq[oldest])) oldest = i;
            if (oldest >= 0) retire_slot(s, s->slots[oldest]);
        }
    }
    for (int i = 0; i < kSlots; ++i)
        if (s->slots[i].busy) retire_slot(s, s->slots[i]);
}

}  // namespace qcpw

using namespace qcpw;

extern "C" {

qcpw_status qcpw_server_create(const qcpw_run_config *cfg, int64_t hbm_budget_bytes, qcpw_server **out)
{
    set_error("");
    if (!out) return fail(QCPW_EINVAL, "out is NULL");
    if (hbm_budget_bytes <= 0) return fail(QCPW_EINVAL, "hbm_budget_bytes must be > 0");
    qcpw_run_config c;
    memset(&c, 0, sizeof c);
    c.device = -1;
    if (cfg) c = *cfg;
    if (c.precision != QCPW_FP64 && c.precision != QCPW_FP32_MIXED) return fail(QCPW_EINVAL, "unknown precision");
    if (c.flags & ~QCPW_FLAG_OWEN) return fail(QCPW_EINVAL, "unknown flags for a server");
    if (!qcpw_block_threads_ok(c.block_threads))
        return fail(QCPW_EINVAL, "block_threads must be 0 or a multiple of 64 in [64, 1024]");
    Context *ctx = nullptr;
    qcpw_status st = get_context(c.device, &ctx);
    if (st != QCPW_OK) return st;
    if (c.block_threads == 0) {
        // tune the workgroup size of every lane-table bucket now, so that no
        // request pays for the autotuner's probe launches in its latency
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (int path : {QCPW_PATH_BB, QCPW_PATH_STANDARD})
            pretune_block_threads(ctx, path, c.precision, (c.flags & QCPW_FLAG_OWEN) != 0);
    }
    std::unique_ptr<qcpw_server> s(new qcpw_server());
    s->ctx = ctx;
    s->cfg = c;
    s->budget = hbm_budget_bytes;
    for (auto &sl : s->slots) QCPW_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    qcpw_server *raw = s.get();
    s->worker = std::thread(worker_main, raw);
    *out = s.release();
    return QCPW_OK;
}

qcpw_status qcpw_submit(qcpw_server *srv, const qcpw_option_spec *specs, int32_t n_opts, int32_t n_shifts,
                        int32_t path_construction, double target_stderr, uint64_t *request_id)
{
    set_error("");
    if (!srv || !request_id) return fail(QCPW_EINVAL, "NULL server or request_id");
    if (n_opts < 1 || n_opts > 4096) return fail(QCPW_EINVAL, "n_opts must be in [1, 4096]");
    if (!(target_stderr > 0) || !std::isfinite(target_stderr)) return fail(QCPW_EINVAL, "target_stderr must be > 0");
    qcpw_status st = validate_call(specs, n_opts, 0, kFirstPoints, n_shifts, path_construction, srv->cfg.precision,
                                   srv->cfg.pca_gemm, srv->cfg.block_threads);
    if (st != QCPW_OK) return st;
    if ((srv->cfg.flags & QCPW_FLAG_OWEN) && path_construction != QCPW_PATH_BB &&
        path_construction != QCPW_PATH_STANDARD)
        return fail(QCPW_EINVAL, "nested scrambling is available with the BB and STANDARD constructions");
    std::unique_ptr<Request> r(new Request());
    r->specs.assign(specs, specs + n_opts);
    r->n_shifts = n_shifts;
    r->path = path_construction;
    r->target = target_stderr;
    for (int i = 0; i < n_opts; ++i) {
        const bool basket = specs[i].type == QCPW_BASKET_ASIAN_CALL || specs[i].type == QCPW_BASKET_ASIAN_PUT;
        const int64_t ndims = (int64_t)(specs[i].d - 1) + (basket ? (int64_t)specs[i].n_assets * specs[i].d : 0);
        r->cost_per_point += (double)std::max<int64_t>(ndims, 1) * n_shifts;
    }
    if (slice_bytes(r.get(), QCPW_CHUNK) + launch_fixed_bytes(path_construction, srv->cfg.precision,
                                                              srv->ctx->tab.n_cu) > slot_cap(srv))
        return fail(QCPW_ENOMEM, "even the request's smallest slice exceeds half the HBM budget");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(QCPW_EINVAL, "server is shutting down");
    r->id = srv->next_id++;
    *request_id = r->id;
    srv->queue.push_back(r->id);
    srv->reqs[r->id] = std::move(r);
    srv->cv_work.notify_one();
    return QCPW_OK;
}

static qcpw_status take_result_locked(qcpw_server *srv, std::map<uint64_t, std::unique_ptr<Request>>::iterator it,
                                      double *g, double *e, int64_t *pts)
{
    Request *r = it->second.get();
    if (r->state == RQ_CANCELLED) {
        if (r->in_flight) r->collected = true;   // the launch that holds it erases it
        else srv->reqs.erase(it);
        return fail(QCPW_ECANCELLED, "request was cancelled");
    }
    if (g) memcpy(g, r->greeks.data(), r->greeks.size() * sizeof(double));
    if (e) memcpy(e, r->stderr_.data(), r->stderr_.size() * sizeof(double));
    if (pts) *pts = r->n_done;
    srv->reqs.erase(it);
    return QCPW_OK;
}

qcpw_status qcpw_poll(qcpw_server *srv, uint64_t request_id, double *out_greeks, double *out_stderr,
                      int64_t *out_points_used)
{
    set_error("");
    if (!srv) return fail(QCPW_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(request_id);
    if (it == srv->reqs.end() || it->second->collected) return fail(QCPW_ENOTFOUND, "unknown request id");
    if (it->second->state == RQ_QUEUED || it->second->state == RQ_RUNNING) return QCPW_EBUSY;
    return take_result_locked(srv, it, out_greeks, out_stderr, out_points_used);
}

qcpw_status qcpw_wait(qcpw_server *srv, uint64_t request_id, double *out_greeks, double *out_stderr,
                      int64_t *out_points_used)
{
    set_error("");
    if (!srv) return fail(QCPW_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(request_id);
    if (it == srv->reqs.end() || it->second->collected) return fail(QCPW_ENOTFOUND, "unknown request id");
    srv->cv_done.wait(lk, [&] {
        auto jt = srv->reqs.find(request_id);
        return jt == srv->reqs.end() || jt->second->state == RQ_DONE || jt->second->state == RQ_CANCELLED;
    });
    it = srv->reqs.find(request_id);
    if (it == srv->reqs.end() || it->second->collected)
        return fail(QCPW_ENOTFOUND, "request was collected by another caller");
    return take_result_locked(srv, it, out_greeks, out_stderr, out_points_used);
}

qcpw_status qcpw_cancel(qcpw_server *srv, uint64_t request_id)
{
    set_error("");
    if (!srv) return fail(QCPW_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(request_id);
    if (it == srv->reqs.end() || it->second->collected) return fail(QCPW_ENOTFOUND, "unknown request id");
    Request *r = it->second.get();
    if (r->state == RQ_QUEUED || r->state == RQ_RUNNING) finish_locked(srv, r, RQ_CANCELLED);
    return QCPW_OK;
}

qcpw_status qcpw_server_stats(qcpw_server *srv, int64_t out[8])
{
    if (!srv || !out) return fail(QCPW_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    int64_t queued = 0;
    for (auto &kv : srv->reqs) queued += kv.second->state == RQ_QUEUED;
    out[0] = srv->n_admitted;
    out[1] = srv->n_completed;
    out[2] = srv->n_cancelled;
    out[3] = srv->n_launches;
    out[4] = srv->in_use;
    out[5] = srv->peak;
    out[6] = queued;
    out[7] = 0;
    for (auto &sl : srv->slots) out[7] += (int64_t)sl.ws.bytes;
    return QCPW_OK;
}

qcpw_status qcpw_server_destroy(qcpw_server *srv)
{
    if (!srv) return fail(QCPW_EINVAL, "NULL server");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (auto &kv : srv->reqs)
            if (kv.second->state == RQ_QUEUED || kv.second->state == RQ_RUNNING)
                finish_locked(srv, kv.second.get(), RQ_CANCELLED);
    }
    for (auto &sl : srv->slots) {
        if (sl.ws.ptr) (void)hipFree(sl.ws.ptr);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete srv;
    return QCPW_OK;
}

}  // extern "C"
