// tvspec server: continuous batching of decomposition requests of mixed
// sizes on one device.
//
// Requests are grouped in size buckets (equal H, W, C, inner_iters).  A
// bucket is a slot table of the engine (engine.h) with its own stream: one
// bucket step is one ROF solve plus the fused outer step for every request
// in the table, so a request admitted at any step boundary simply joins the
// next step, and one whose flow is complete leaves after it.  Buckets step
// concurrently on their streams, which lets small images fill the device
// around large ones.
//
// The worker thread owns all device work.  Each pass it
//   retires requests whose completion event has fired (their pool range and
//       slot become free),
//   admits queued requests in FIFO order while the head request's working
//       state fits in the pool (slot descriptor and band rows are uploaded
//       through pinned staging, then the slot is initialised on the bucket's
//       stream); a request whose bucket already runs its cap -- as many
//       requests as fill the device on their own -- is passed over together
//       with the later requests of its bucket,
//   enqueues the next steps of every bucket with requests in flight -- up to
//       kMultiStep ROF solves in one graph replay, as many as every request of
//       the bucket still needs, so none idles inside the replay -- keeping at
//       most kDepthSteps steps per bucket ahead of the device, and finalises
//       (S, checks, report) the requests those steps complete.
// Every device operation of a request is on its bucket's stream, in order,
// so a slot index or table entry can be reused at the next step boundary;
// pool memory is only reused once the completion event of its previous owner
// has fired, since the next owner may be in another bucket.
//
// A run of bucket steps is captured once in a hipGraph per (table size,
// tile shape, temporal blocking factor, dual-field parity, number of steps)
// and replayed; the table size is the high-water mark of occupied slots
// rounded up, and inactive slots exit at once.  With iters_per_launch = 0
// the autotuner times kTuneSteps single steps of a bucket with each
// candidate (tile shape, blocking factor) -- 32 x 32 and 32 x 16 tiles,
// TB 4, 5 and 8 -- (events around the replay) and keeps the fastest;
// results do not depend on the choice.

#include <hip/hip_runtime.h>

#include <algorithm>
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

#include "engine.h"

namespace tvspec {
namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

constexpr int kDepthSteps = 8;    // bucket steps enqueued ahead of the device
constexpr int kMultiStep = 4;     // bucket steps per graph replay at most
constexpr int kFillPerCU = 16;    // workgroups per CU that fill the device (run cap; measured
                                  // 4 and 8 lose ~10% throughput to per-step fixed costs)
constexpr int kSlotCap = 128;     // slots per bucket table
constexpr int kTableRound = 4;    // table size rounded up to a multiple of this
constexpr int kTuneSteps = 3;     // steps timed per autotuner candidate
constexpr size_t kChunkMin = 64 << 10;
constexpr size_t kMinBudget = 1 << 20;


enum class State { Queued, Running, Finishing, Done, Failed };

struct Request {
    unsigned long long ticket = 0;
    tvspec_request r{};
    std::vector<int> edges;
    size_t scratch = 0;   // engine buffers (slot_scratch_bytes)
    size_t footprint = 0; // scratch + band rows + non-finite counter
    size_t off = 0;       // pool offset
    int bucket = -1, slot = -1;
    int steps_left = 0;
    hipEvent_t done = nullptr;
    State state = State::Queued;
    Clock::time_point t_submit, t_admit, t_done;
};

// Pinned staging for uploads; reusable once its event has fired.
struct Chunk {
    char *host = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool busy = false;
};

struct TuneCand {
    int tile, ipl;
};

struct TuneSample {
    TuneCand c;
    hipEvent_t a, b;
};

struct Bucket {
    int H = 0, W = 0, C = 0, iters = 0;
    StepConfig cfg{};
    hipStream_t st = nullptr;
    SlotDesc *table = nullptr;
    int cap = 0;
    int run_cap = 1;  // requests that fill the device on their own (see bucket_for)
    std::vector<Request *> slots;
    int in_use = 0;
    int parity = 0;
    std::deque<std::pair<hipEvent_t, int>> inflight; // one event per enqueued replay, and its steps
    int inflight_steps = 0;
    std::vector<hipEvent_t> spare;
    // graphs of the current (table size, tile shape, blocking factor), per
    // dual-field parity and number of steps
    hipGraphExec_t exec[2][kMultiStep + 1] = {};
    int exec_n = -1, exec_ipl = -1, exec_tile = -1;
    // autotuner
    bool tuning = false, collecting = false;
    std::vector<TuneCand> cand;
    int cand_i = 0, cand_steps = 0;
    std::vector<TuneSample> samples;
};

} // namespace
} // namespace tvspec

struct tvspec_server {
    int dev = 0;
    double tau = TVSPEC_DEFAULT_TAU;
    int warm = 0, precision = TVSPEC_DEFAULT_PRECISION, ipl = 0, use_graphs = 1;
    size_t budget = 0;
    char *pool = nullptr;
    tvspec::RangeAlloc alloc;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    int err = TVSPEC_OK;
    std::string err_msg;
    std::thread worker;

    unsigned long long next_ticket = 1;
    std::unordered_map<unsigned long long, std::unique_ptr<tvspec::Request>> reqs;
    std::deque<tvspec::Request *> queue;
    std::vector<tvspec::Request *> finishing;
    std::vector<std::unique_ptr<tvspec::Bucket>> buckets;
    std::vector<tvspec::Chunk> chunks;

    unsigned long long n_submitted = 0, n_admitted = 0, n_completed = 0, n_steps = 0, n_replays = 0, n_graphs = 0;
    int in_flight = 0, max_in_flight = 0;
};

namespace tvspec {
namespace {

// ---------------------------------------------------------------------------
// worker pieces; all run on the worker thread with srv->mu held

int get_chunk(tvspec_server *s, size_t bytes, Chunk **out)
{
    Chunk *best = nullptr;
    for (Chunk &c : s->chunks) {
        if (c.busy) {
            const hipError_t q = hipEventQuery(c.ev);
            if (q == hipSuccess)
                c.busy = false;
            else if (q != hipErrorNotReady)
                HIP_TRY(q);
        }
        if (!c.busy && c.bytes >= bytes && (!best || c.bytes < best->bytes))
            best = &c;
    }
    if (!best) {
        Chunk c;
        c.bytes = std::max(bytes, kChunkMin);
        HIP_TRY(hipHostMalloc((void **)&c.host, c.bytes, hipHostMallocDefault));
        HIP_TRY(hipEventCreateWithFlags(&c.ev, hipEventDisableTiming));
        s->chunks.push_back(c);
        best = &s->chunks.back();
    }
    *out = best;
    return TVSPEC_OK;
}

int bucket_for(tvspec_server *s, const Request &q, int *out)
{
    for (size_t i = 0; i < s->buckets.size(); ++i) {
        const Bucket &b = *s->buckets[i];
        if (b.H == q.r.H && b.W == q.r.W && b.C == q.r.C && b.iters == q.r.inner_iters) {
            *out = (int)i;
            return TVSPEC_OK;
        }
    }
    auto b = std::make_unique<Bucket>();
    b->H = q.r.H;
    b->W = q.r.W;
    b->C = q.r.C;
    b->iters = q.r.inner_iters;
    b->cfg = StepConfig{b->H, b->W, b->C, b->iters, s->tau, s->warm, s->ipl, s->precision};
    b->cfg.timed = 0;
    b->cap = std::min(kSlotCap, 65535 / b->C);
    // Run cap: a step of one request launches (tiles x C) workgroups per tile
    // launch; once the bucket's requests together fill the device
    // (kFillPerCU workgroups per CU), more of them only share it and each
    // finishes later, so the bucket admits at most that many at a time and
    // the rest wait in the queue in order.
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->dev) != hipSuccess || cus < 1)
            cus = 256;
        const long long wgs = (long long)((b->H + 31) / 32) * ((b->W + 31) / 32) * b->C;
        const long long fill = (long long)kFillPerCU * cus;
        b->run_cap = (int)std::max(1LL, std::min((long long)b->cap, (fill + wgs - 1) / wgs));
    }
    b->slots.assign(b->cap, nullptr);
    HIP_TRY(hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking));
    HIP_TRY(hipMalloc((void **)&b->table, (size_t)b->cap * sizeof(SlotDesc)));
    // every entry starts inactive (k_* kernels skip slots with active = 0)
    HIP_TRY(hipMemsetAsync(b->table, 0, (size_t)b->cap * sizeof(SlotDesc), b->st));
    if (s->ipl == 0) {
        b->tuning = true;
        const int big = s->precision == TVSPEC_PRECISION_F32 ? 16 : 5;
        for (int ipl : {4, big, 8})
            b->cand.push_back(TuneCand{kTileShapeSquare, ipl});
        for (int ipl : {4, 5, 8})
            b->cand.push_back(TuneCand{kTileShapeNarrow, ipl});
        b->cfg.tile = b->cand[0].tile;
        b->cfg.iters_per_launch = b->cand[0].ipl;
    }
    s->buckets.push_back(std::move(b));
    *out = (int)s->buckets.size() - 1;
    return TVSPEC_OK;
}

// Admit the queue's head if it fits; *admitted tells.
int try_admit(tvspec_server *s, Request *q, bool *admitted)
{
    *admitted = false;
    int bi = 0;
    TVSPEC_TRY(bucket_for(s, *q, &bi));
    Bucket &b = *s->buckets[bi];
    int slot = -1;
    for (int i = 0; i < b.cap; ++i)
        if (!b.slots[i]) {
            slot = i;
            break;
        }
    if (slot < 0)
        return TVSPEC_OK;
    size_t off = 0;
    if (!s->alloc.alloc(q->footprint, &off))
        return TVSPEC_OK;

    const int K = q->r.K;
    char *base = s->pool + off;
    SlotDesc d;
    std::memset(&d, 0, sizeof(d));
    slot_carve(d, base, s->precision, kSolverChambolle, b.H, b.W, b.C, K);
    int *d_rows = (int *)(base + q->scratch);
    unsigned int *d_nf = (unsigned int *)(base + q->scratch + align256((size_t)(K + 1) * sizeof(int)));
    d.band_rows = d_rows;
    d.nonfinite = d_nf;
    d.f = q->r.f;
    d.bands = q->r.bands;
    d.S = q->r.S;
    d.res = q->r.residual;
    d.stats = q->r.stats;
    d.dt = q->r.dt;
    d.nbands = q->r.n_bands;

    const size_t desc_bytes = align256(sizeof(SlotDesc));
    const size_t rows_bytes = (size_t)(K + 1) * sizeof(int);
    Chunk *c = nullptr;
    TVSPEC_TRY(get_chunk(s, desc_bytes + rows_bytes, &c));
    std::memcpy(c->host, &d, sizeof(SlotDesc));
    band_rows_of(q->edges.data(), q->r.n_bands, (int *)(c->host + desc_bytes));
    HIP_TRY(hipMemcpyAsync(b.table + slot, c->host, sizeof(SlotDesc), hipMemcpyHostToDevice, b.st));
    HIP_TRY(hipMemcpyAsync(d_rows, c->host + desc_bytes, rows_bytes, hipMemcpyHostToDevice, b.st));
    HIP_TRY(hipEventRecord(c->ev, b.st));
    c->busy = true;
    HIP_TRY(hipMemsetAsync(d_nf, 0, sizeof(unsigned int), b.st));
    TVSPEC_TRY(engine_init(b.cfg, b.table, slot, 1, b.st));
    HIP_TRY(hipEventCreateWithFlags(&q->done, hipEventDisableTiming));

    q->off = off;
    q->bucket = bi;
    q->slot = slot;
    q->steps_left = K + 1;
    q->state = State::Running;
    q->t_admit = Clock::now();
    b.slots[slot] = q;
    ++b.in_use;
    ++s->n_admitted;
    ++s->in_flight;
    s->max_in_flight = std::max(s->max_in_flight, s->in_flight);
    *admitted = true;
    return TVSPEC_OK;
}

void drop_graphs(Bucket &b)
{
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k <= kMultiStep; ++k)
            if (b.exec[p][k]) {
                (void)hipGraphExecDestroy(b.exec[p][k]);
                b.exec[p][k] = nullptr;
            }
}

// Pick the autotuner's winner once every timed step has completed.
int tune_collect(Bucket &b, bool *progressed)
{
    for (const TuneSample &t : b.samples) {
        const hipError_t q = hipEventQuery(t.b);
        if (q == hipErrorNotReady)
            return TVSPEC_OK;
        HIP_TRY(q);
    }
    std::map<std::pair<int, int>, float> best;
    for (const TuneSample &t : b.samples) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
        const std::pair<int, int> key(t.c.tile, t.c.ipl);
        auto it = best.find(key);
        if (it == best.end() || ms < it->second)
            best[key] = ms;
    }
    TuneCand pick = b.cand.back();
    float pick_ms = 0.f;
    bool first = true;
    for (const TuneCand &c : b.cand) {
        auto it = best.find(std::make_pair(c.tile, c.ipl));
        if (it != best.end() && (first || it->second < pick_ms)) {
            pick = c;
            pick_ms = it->second;
            first = false;
        }
    }
    for (const TuneSample &t : b.samples) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    b.samples.clear();
    b.cfg.tile = pick.tile;
    b.cfg.iters_per_launch = pick.ipl;
    b.collecting = false;
    *progressed = true;
    return TVSPEC_OK;
}

// Enqueue the next steps of bucket b and the finalisation of the requests
// they complete: one step while the autotuner times candidates, otherwise as
// many as every request of the bucket still needs, up to kMultiStep, in one
// replay.
int step_bucket(tvspec_server *s, Bucket &b)
{
    int hw = 0;
    int steps = kMultiStep;
    for (int i = 0; i < b.cap; ++i)
        if (b.slots[i]) {
            hw = i + 1;
            steps = std::min(steps, b.slots[i]->steps_left);
        }
    const int n = std::min(b.cap, (hw + kTableRound - 1) / kTableRound * kTableRound);
    const StepConfig cfg = b.cfg;
    const bool timing = b.tuning;
    if (timing)
        steps = 1;
    hipEvent_t ta = nullptr, tb = nullptr;
    if (timing) {
        HIP_TRY(hipEventCreate(&ta));
        HIP_TRY(hipEventCreate(&tb));
    }
    if (s->use_graphs) {
        if (b.exec_n != n || b.exec_ipl != cfg.iters_per_launch || b.exec_tile != cfg.tile) {
            drop_graphs(b);
            b.exec_n = n;
            b.exec_ipl = cfg.iters_per_launch;
            b.exec_tile = cfg.tile;
        }
        hipGraphExec_t &ex = b.exec[b.parity][steps];
        if (!ex) {
            HIP_TRY(hipStreamBeginCapture(b.st, hipStreamCaptureModeThreadLocal));
            int par = b.parity;
            int rc = TVSPEC_OK;
            for (int k = 0; k < steps && rc == TVSPEC_OK; ++k)
                rc = engine_step(cfg, b.table, n, &par, b.st, 0);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(b.st, &g);
            if (rc != TVSPEC_OK) {
                if (g)
                    (void)hipGraphDestroy(g);
                return rc;
            }
            HIP_TRY(e);
            const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIP_TRY(ei);
            ++s->n_graphs;
        }
        if (timing)
            HIP_TRY(hipEventRecord(ta, b.st));
        HIP_TRY(hipGraphLaunch(ex, b.st));
        b.parity ^= ((steps * tile_launches_per_step(cfg, n)) & 1);
    } else {
        if (timing)
            HIP_TRY(hipEventRecord(ta, b.st));
        for (int k = 0; k < steps; ++k)
            TVSPEC_TRY(engine_step(cfg, b.table, n, &b.parity, b.st, 0));
    }
    if (timing) {
        HIP_TRY(hipEventRecord(tb, b.st));
        b.samples.push_back(TuneSample{b.cand[b.cand_i], ta, tb});
        if (++b.cand_steps == kTuneSteps) {
            b.cand_steps = 0;
            if (++b.cand_i == (int)b.cand.size()) {
                b.tuning = false;
                b.collecting = true;
            } else {
                b.cfg.tile = b.cand[b.cand_i].tile;
                b.cfg.iters_per_launch = b.cand[b.cand_i].ipl;
            }
        }
    }
    hipEvent_t ev = nullptr;
    if (!b.spare.empty()) {
        ev = b.spare.back();
        b.spare.pop_back();
    } else {
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    HIP_TRY(hipEventRecord(ev, b.st));
    b.inflight.push_back(std::make_pair(ev, steps));
    b.inflight_steps += steps;
    s->n_steps += steps;
    ++s->n_replays;

    for (int i = 0; i < b.cap; ++i) {
        Request *q = b.slots[i];
        if (!q)
            continue;
        q->steps_left -= steps;
        if (q->steps_left > 0)
            continue;
        TVSPEC_TRY(engine_finalize(cfg, b.table, i, 1, q->r.K, b.st));
        HIP_TRY(hipEventRecord(q->done, b.st));
        q->state = State::Finishing;
        s->finishing.push_back(q);
        b.slots[i] = nullptr;
        --b.in_use;
    }
    return TVSPEC_OK;
}

// One pass of the worker; *progressed is set when anything moved, *busy
// when device work is in flight.
int worker_pass(tvspec_server *s, bool *progressed, bool *busy)
{
    *progressed = false;
    // retire
    for (size_t i = 0; i < s->finishing.size();) {
        Request *q = s->finishing[i];
        const hipError_t e = hipEventQuery(q->done);
        if (e == hipErrorNotReady) {
            ++i;
            continue;
        }
        HIP_TRY(e);
        s->alloc.release(q->off, q->footprint);
        (void)hipEventDestroy(q->done);
        q->done = nullptr;
        q->state = State::Done;
        q->t_done = Clock::now();
        --s->in_flight;
        ++s->n_completed;
        s->finishing[i] = s->finishing.back();
        s->finishing.pop_back();
        *progressed = true;
    }
    if (*progressed)
        s->cv_done.notify_all();
    // admit in FIFO order, passing over a request whose bucket already runs
    // its cap (and the later requests of that bucket, which keep their
    // order); the first request that does not fit in memory stops admission,
    // so no later request overtakes it for memory
    {
        std::vector<int> capped;
        for (auto it = s->queue.begin(); it != s->queue.end();) {
            Request *q = *it;
            int bi = 0;
            TVSPEC_TRY(bucket_for(s, *q, &bi));
            const Bucket &bk = *s->buckets[bi];
            if (std::find(capped.begin(), capped.end(), bi) != capped.end() || bk.in_use >= bk.run_cap) {
                capped.push_back(bi);
                ++it;
                continue;
            }
            bool ok = false;
            TVSPEC_TRY(try_admit(s, q, &ok));
            if (!ok)
                break;
            it = s->queue.erase(it);
            *progressed = true;
        }
    }
    // step
    for (auto &bp : s->buckets) {
        Bucket &b = *bp;
        while (!b.inflight.empty()) {
            const hipError_t e = hipEventQuery(b.inflight.front().first);
            if (e == hipErrorNotReady)
                break;
            HIP_TRY(e);
            b.spare.push_back(b.inflight.front().first);
            b.inflight_steps -= b.inflight.front().second;
            b.inflight.pop_front();
        }
        if (b.collecting)
            TVSPEC_TRY(tune_collect(b, progressed));
        if (b.in_use > 0 && b.inflight_steps < kDepthSteps) {
            TVSPEC_TRY(step_bucket(s, b));
            *progressed = true;
        }
    }
    *busy = !s->finishing.empty();
    for (auto &bp : s->buckets)
        *busy = *busy || !bp->inflight.empty();
    return TVSPEC_OK;
}

void fail_all(tvspec_server *s, int code, const std::string &msg)
{
    s->err = code;
    s->err_msg = msg;
    for (auto &kv : s->reqs)
        if (kv.second->state != State::Done)
            kv.second->state = State::Failed;
    s->queue.clear();
    s->cv_done.notify_all();
}

void worker_main(tvspec_server *s)
{
    if (hipSetDevice(s->dev) != hipSuccess) {
        std::lock_guard<std::mutex> lock(s->mu);
        fail_all(s, TVSPEC_EDEVICE, "server worker: hipSetDevice failed");
        return;
    }
    std::unique_lock<std::mutex> lock(s->mu);
    while (!s->stop) {
        bool progressed = false, busy = false;
        const int rc = worker_pass(s, &progressed, &busy);
        if (rc != TVSPEC_OK) {
            fail_all(s, rc, "server worker: " + g_last_error);
            return;
        }
        if (progressed)
            continue;
        if (busy) {
            // device work in flight: look again shortly
            lock.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lock.lock();
        } else {
            s->cv_work.wait_for(lock, std::chrono::milliseconds(5));
        }
    }
}

int result_of(tvspec_server *s, Request *q, tvspec_result *res)
{
    if (q->state == State::Failed) {
        g_last_error = s->err_msg;
        return s->err != TVSPEC_OK ? s->err : TVSPEC_EDEVICE;
    }
    if (q->state != State::Done)
        return TVSPEC_PENDING;
    if (res) {
        res->queue_ms = ms_between(q->t_submit, q->t_admit);
        res->latency_ms = ms_between(q->t_submit, q->t_done);
    }
    s->reqs.erase(q->ticket);
    return TVSPEC_OK;
}

} // namespace
} // namespace tvspec

using namespace tvspec;

// ---------------------------------------------------------------------------
// C ABI

extern "C" int tvspec_server_create(size_t budget_bytes, double tau, int warm_start, int precision,
                                    int iters_per_launch, int use_graphs, tvspec_server **out)
{
    g_last_error.clear();
    if (!out)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    *out = nullptr;
    if (budget_bytes < kMinBudget)
        return fail(TVSPEC_EINVAL, "budget_bytes must be >= 1 MiB");
    if (use_graphs != 0 && use_graphs != 1)
        return fail(TVSPEC_EINVAL, "use_graphs must be 0 or 1");
    TVSPEC_TRY(validate_opts(tau, warm_start, precision, iters_per_launch));
    auto s = std::make_unique<tvspec_server>();
    HIP_TRY(hipGetDevice(&s->dev));
    s->tau = tau;
    s->warm = warm_start;
    s->precision = precision;
    s->ipl = iters_per_launch;
    s->use_graphs = use_graphs;
    s->budget = align256(budget_bytes) - (align256(budget_bytes) == budget_bytes ? 0 : 256);
    HIP_TRY(hipMalloc((void **)&s->pool, s->budget));
    s->alloc.reset(s->budget);
    tvspec_server *raw = s.get();
    try {
        s->worker = std::thread(worker_main, raw);
    } catch (...) {
        (void)hipFree(s->pool);
        return fail(TVSPEC_ENOMEM, "could not start the server's worker thread");
    }
    *out = s.release();
    return TVSPEC_OK;
}

extern "C" int tvspec_submit(tvspec_server *srv, const tvspec_request *req, unsigned long long *ticket)
{
    g_last_error.clear();
    if (!srv || !req || !ticket)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    const tvspec_request &r = *req;
    if (!r.f || !r.band_edges || !r.bands || !r.S || !r.residual || !r.stats)
        return fail(TVSPEC_EINVAL, "null pointer in the request");
    TVSPEC_TRY(validate_shape(1, r.H, r.W, r.C, r.inner_iters));
    TVSPEC_TRY(validate_image(r.dt, r.K, r.band_edges, r.n_bands));
    auto q = std::make_unique<Request>();
    q->r = r;
    q->edges.assign(r.band_edges, r.band_edges + r.n_bands + 1);
    q->r.band_edges = nullptr;
    q->scratch = slot_scratch_bytes(srv->precision, kSolverChambolle, r.H, r.W, r.C, r.K);
    q->footprint = q->scratch + align256((size_t)(r.K + 1) * sizeof(int)) + 256;
    if (q->footprint > srv->budget)
        return fail(TVSPEC_EBUSY, "request needs " + std::to_string(q->footprint) +
                                      " bytes of working state, more than the server's budget of " +
                                      std::to_string(srv->budget));
    std::lock_guard<std::mutex> lock(srv->mu);
    if (srv->err != TVSPEC_OK)
        return fail(srv->err, srv->err_msg);
    if (srv->stop)
        return fail(TVSPEC_EINVAL, "server is shutting down");
    q->ticket = srv->next_ticket++;
    q->t_submit = Clock::now();
    *ticket = q->ticket;
    srv->queue.push_back(q.get());
    srv->reqs.emplace(q->ticket, std::move(q));
    ++srv->n_submitted;
    srv->cv_work.notify_one();
    return TVSPEC_OK;
}

extern "C" int tvspec_poll(tvspec_server *srv, unsigned long long ticket, tvspec_result *res)
{
    g_last_error.clear();
    if (!srv)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end())
        return fail(TVSPEC_EINVAL, "unknown ticket " + std::to_string(ticket));
    return result_of(srv, it->second.get(), res);
}

extern "C" int tvspec_wait(tvspec_server *srv, unsigned long long ticket, tvspec_result *res)
{
    g_last_error.clear();
    if (!srv)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    std::unique_lock<std::mutex> lock(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end())
        return fail(TVSPEC_EINVAL, "unknown ticket " + std::to_string(ticket));
    Request *q = it->second.get();
    srv->cv_done.wait(lock, [&] { return q->state == State::Done || q->state == State::Failed; });
    return result_of(srv, q, res);
}

extern "C" int tvspec_server_info(tvspec_server *srv, tvspec_server_stats *info)
{
    g_last_error.clear();
    if (!srv || !info)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    info->submitted = srv->n_submitted;
    info->admitted = srv->n_admitted;
    info->completed = srv->n_completed;
    info->steps = srv->n_steps;
    info->replays = srv->n_replays;
    info->graph_builds = srv->n_graphs;
    info->buckets = (int)srv->buckets.size();
    info->max_in_flight = srv->max_in_flight;
    info->budget_bytes = srv->budget;
    info->used_bytes = srv->alloc.used();
    info->peak_bytes = srv->alloc.peak();
    return srv->err;
}

extern "C" int tvspec_server_destroy(tvspec_server *srv)
{
    g_last_error.clear();
    if (!srv)
        return TVSPEC_OK;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable())
        srv->worker.join();
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(srv->dev);
    int rc = TVSPEC_OK;
    for (auto &bp : srv->buckets) {
        Bucket &b = *bp;
        if (b.st && hipStreamSynchronize(b.st) != hipSuccess)
            rc = fail(TVSPEC_EDEVICE, "server destroy: stream synchronisation failed");
        drop_graphs(b);
        for (const auto &e : b.inflight)
            (void)hipEventDestroy(e.first);
        for (hipEvent_t e : b.spare)
            (void)hipEventDestroy(e);
        for (const TuneSample &t : b.samples) {
            (void)hipEventDestroy(t.a);
            (void)hipEventDestroy(t.b);
        }
        if (b.table)
            (void)hipFree(b.table);
        if (b.st)
            (void)hipStreamDestroy(b.st);
    }
    for (auto &kv : srv->reqs)
        if (kv.second->done)
            (void)hipEventDestroy(kv.second->done);
    for (Chunk &c : srv->chunks) {
        (void)hipHostFree(c.host);
        (void)hipEventDestroy(c.ev);
    }
    if (srv->pool)
        (void)hipFree(srv->pool);
    (void)hipSetDevice(cur);
    delete srv;
    return rc;
}
