// Continuous-batching server for repeated solves against resident plans.
//
// Requests (plan, b, x) are queued by gltrsv_server_submit and admitted into
// device slots while the in-flight budget allows.  A worker thread runs the
// batched kernel in time quanta: waves claim chunks from every admitted
// request's open superstep and stop claiming at the quantum's deadline; a
// request's state word and done counters are consistent at the end of every
// launch, so it simply continues in the next one.  Between quanta the worker
// harvests finished requests (their superstep reached S), frees their slots
// and admits queued ones, so requests that arrive while others run join the
// device work at the next quantum.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

using namespace gltrsv;

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t ticket = 0;
    gltrsv_plan *plan = nullptr;
    const double *b = nullptr;
    double *x = nullptr;
    int64_t bytes = 0;
};

struct Slot {
    bool busy = false;
    bool fresh = false;     // descriptor changed since the last launch
    bool cancel = false;    // withdrawn: dropped at the next quantum boundary
    Request req;            // valid while busy only
    int32_t done_off = 0;
    // copied from the plan at admission, so a slot never reads a plan after
    // its request has left it (the caller may destroy the plan then)
    int32_t S = 0;          // supersteps = done counters held in the arena
    int64_t n = 0;
    int64_t chunks = 0;
    int64_t widest = 0;     // chunks of the plan's widest superstep
};

// First-fit allocator of per-superstep done counters inside one device array.
class CounterArena {
public:
    explicit CounterArena(int32_t words) { free_[0] = words; }
    int32_t take(int32_t n)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const int32_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                return off;
            }
        }
        return -1;
    }
    void give(int32_t off, int32_t n)
    {
        auto it = free_.emplace(off, n).first;
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

private:
    std::map<int32_t, int32_t> free_;
};

}  // namespace

struct gltrsv_server {
    gltrsv_server_opts opts{};
    int device = 0;
    hipStream_t stream = nullptr;
    int grid = 1;
    dev::SysDesc *d_desc = nullptr;
    unsigned long long *d_state = nullptr;
    uint32_t *d_done = nullptr;
    uint32_t *d_finished = nullptr;
    int32_t *d_err = nullptr;
    dev::SysDesc *h_desc = nullptr;          // pinned
    unsigned long long *h_state = nullptr;   // pinned
    CounterArena *arena = nullptr;

    std::mutex mu;
    std::condition_variable cv;        // wakes the worker (new request, stop)
    std::condition_variable cv_done;   // wakes cancel callers (a slot was released)
    std::deque<Request> queue;
    std::vector<Slot> slots;
    std::vector<std::pair<uint64_t, int64_t>> completed;
    int64_t inflight_bytes = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    int failure = 0;   // first error of the worker (GLTRSV_E*), sticky
    std::string failure_text;
    gltrsv_server_stats stats{};
    std::thread worker;
};

namespace {

int free_server_memory(gltrsv_server *sv)
{
    (void)hipFree(sv->d_desc);
    (void)hipFree(sv->d_state);
    (void)hipFree(sv->d_done);
    (void)hipFree(sv->d_finished);
    (void)hipFree(sv->d_err);
    if (sv->h_desc) (void)hipHostFree(sv->h_desc);
    if (sv->h_state) (void)hipHostFree(sv->h_state);
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    delete sv->arena;
    return GLTRSV_OK;
}

// One quantum: upload the descriptors of newly admitted requests, launch,
// read back every state word.  Runs on the worker thread without the lock.
int run_quantum(gltrsv_server *sv, int32_t used, int32_t busy)
{
    for (int32_t i = 0; i < used; i++) {
        Slot &sl = sv->slots[i];
        if (!sl.fresh) continue;
        sl.fresh = false;
        HIP_TRY(hipMemcpyAsync(sv->d_desc + i, sv->h_desc + i, sizeof(dev::SysDesc), hipMemcpyHostToDevice,
                               sv->stream));
        if (!sl.busy) continue;   // an emptied descriptor (S = 0) reads as finished
        HIP_TRY(hipMemsetAsync(sv->d_state + size_t(i) * dev::kStateStride, 0, sizeof(unsigned long long),
                               sv->stream));
        HIP_TRY(hipMemsetAsync(sv->d_done + sl.done_off, 0, sizeof(uint32_t) * size_t(std::max(1, sl.S)),
                               sv->stream));
        if (sv->opts.async_exec && sl.n > 0) {
            // semi-asynchronous: x starts as the not-yet-computed mark
            const unsigned blocks = unsigned(std::min<int64_t>(1024, (sl.n + dev::kBlock - 1) / dev::kBlock));
            hipLaunchKernelGGL(dev::fill_unready, dim3(blocks), dim3(dev::kBlock), 0, sv->stream,
                               reinterpret_cast<unsigned long long *>(sl.req.x), sl.n);
        }
    }
    HIP_TRY(hipMemsetAsync(sv->d_finished, 0, 2 * sizeof(uint32_t), sv->stream));
    int64_t widest = 0;
    for (int32_t i = 0; i < used; i++)
        if (sv->slots[i].busy) widest = std::max(widest, sv->slots[i].widest);
    const int64_t quantum = int64_t(sv->opts.quantum_us * 100.0);   // 100 MHz wall clock
    if (sv->opts.async_exec)
        hipLaunchKernelGGL(dev::trsv_batched_async, dim3(unsigned(sv->grid)), dim3(dev::kBlock), 0, sv->stream,
                           sv->d_desc, used, sv->d_state, sv->d_finished, sv->d_err, int64_t(5000000),
                           sv->opts.per_claim, std::max<int64_t>(quantum, 1));
    else
        hipLaunchKernelGGL(dev::trsv_batched, dim3(unsigned(sv->grid)), dim3(dev::kBlock), 0, sv->stream, sv->d_desc,
                           used, sv->d_state, sv->d_done, sv->d_finished, sv->d_err, int64_t(1000000000),
                           sv->opts.per_claim, busy, std::max<int64_t>(quantum, 1),
                           dev::keep_waves_for(widest, sv->opts.per_claim, sv->grid));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpy2DAsync(sv->h_state, sizeof(unsigned long long), sv->d_state,
                             sizeof(unsigned long long) * dev::kStateStride, sizeof(unsigned long long), size_t(used),
                             hipMemcpyDeviceToHost, sv->stream));
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, sv->d_err, sizeof(int32_t), hipMemcpyDeviceToHost, sv->stream));
    HIP_TRY(hipStreamSynchronize(sv->stream));
    if (err) return set_error(GLTRSV_ETIMEDOUT, "server: a wave went without work past the idle limit");
    return GLTRSV_OK;
}

// Frees slot i (caller holds the lock, no launch in flight): its budget and
// counters return, its descriptor is emptied (the next launch sees it
// finished) and its request is forgotten; the plan is not touched.
void free_slot(gltrsv_server *sv, int32_t i)
{
    Slot &sl = sv->slots[i];
    sv->inflight_bytes -= sl.req.bytes;
    sv->arena->give(sl.done_off, std::max(1, sl.S));
    sl.busy = false;
    sl.cancel = false;
    sl.req = Request();
    std::memset(&sv->h_desc[i], 0, sizeof(dev::SysDesc));
    sl.fresh = true;
}

// A withdrawn request leaves its slot; cancel callers waiting for it wake up.
void release_slot(gltrsv_server *sv, int32_t i)
{
    sv->stats.cancelled++;
    free_slot(sv, i);
    sv->cv_done.notify_all();
}

void worker_main(gltrsv_server *sv)
{
    if (hipSetDevice(sv->device) != hipSuccess) {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->failure = GLTRSV_EHIP;
        sv->failure_text = "server: hipSetDevice failed";
        return;
    }
    for (;;) {
        int32_t used = 0, busy = 0;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            // drop withdrawn requests: no chunk of theirs is in flight between quanta
            for (int32_t i = 0; i < int32_t(sv->slots.size()); i++)
                if (sv->slots[i].busy && sv->slots[i].cancel) release_slot(sv, i);
            // admit queued requests into the lowest free slots
            while (!sv->queue.empty()) {
                int32_t free_slot = -1;
                for (int32_t i = 0; i < int32_t(sv->slots.size()); i++)
                    if (!sv->slots[i].busy) {
                        free_slot = i;
                        break;
                    }
                if (free_slot < 0) break;
                Request &r = sv->queue.front();
                const int32_t off = sv->arena->take(std::max(1, r.plan->S));
                if (off < 0) break;
                Slot &sl = sv->slots[free_slot];
                sl.busy = true;
                sl.fresh = true;
                sl.cancel = false;
                sl.req = r;
                sl.done_off = off;
                sl.S = r.plan->S;
                sl.n = r.plan->n;
                sl.chunks = r.plan->chunks;
                sl.widest = r.plan->widest;
                dev::SysDesc &d = sv->h_desc[free_slot];
                d.word = r.plan->d_word;
                d.value = r.plan->d_value;
                d.chunk_base = r.plan->d_chunk_base;
                d.chunk_len = r.plan->d_chunk_len;
                d.super_chunk = r.plan->d_super_chunk;
                d.b = r.b;
                d.x = r.x;
                d.S = r.plan->S;
                d.done_off = off;
                d.nchunks = int32_t(r.plan->chunks);
                d.window = dev::async_window(r.plan->chunks, r.plan->S);
                d.n = r.plan->n;
                sv->queue.pop_front();
            }
            for (int32_t i = 0; i < int32_t(sv->slots.size()); i++)
                if (sv->slots[i].busy) {
                    busy++;
                    used = i + 1;
                }
            if (busy == 0) {
                if (sv->stop) return;
                sv->cv.wait_for(lk, std::chrono::milliseconds(1));
                continue;
            }
        }
        const int rc = run_quantum(sv, used, busy);
        const int64_t t = now_ns();
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stats.launches++;
        if (rc) {
            sv->failure = rc;
            sv->failure_text = gltrsv_last_error();
            // fail every request on the device and in the queue
            for (auto &sl : sv->slots)
                if (sl.busy) {
                    sl.busy = false;
                    sl.req = Request();
                    sv->stats.failed++;
                }
            sv->stats.failed += int64_t(sv->queue.size());
            sv->queue.clear();
            sv->inflight_bytes = 0;
            sv->cv_done.notify_all();
            return;
        }
        for (int32_t i = 0; i < used; i++) {
            Slot &sl = sv->slots[i];
            if (!sl.busy) continue;
            // complete: the open superstep passed S, or (semi-asynchronous) every chunk is done
            const int64_t hi = int64_t(sv->h_state[i] >> 32);
            if (sl.cancel) {
                release_slot(sv, i);   // withdrawn during the quantum: never reported
            } else if (sv->opts.async_exec ? hi >= sl.chunks : hi >= sl.S) {
                sv->completed.emplace_back(sl.req.ticket, t);
                sv->stats.completed++;
                sv->stats.rows_completed += sl.n;
                free_slot(sv, i);   // the emptied descriptor goes up with the next launch
            }
        }
    }
}

}  // namespace

extern "C" {

void gltrsv_default_server_opts(gltrsv_server_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->budget_bytes = int64_t(4) << 30;
    o->max_slots = 256;
    o->per_claim = 1;
    o->quantum_us = 200.0;
    o->counter_words = 1 << 22;
    o->grid_blocks = 0;
}

int gltrsv_server_create(const gltrsv_server_opts *opts, gltrsv_server **out)
{
    if (!out) return set_error(GLTRSV_EINVAL, "null argument");
    *out = nullptr;
    gltrsv_server_opts dflt;
    gltrsv_default_server_opts(&dflt);
    if (!opts) opts = &dflt;
    if (opts->budget_bytes <= 0 || opts->max_slots < 1 || opts->per_claim < 1 || !(opts->quantum_us > 0.0) ||
        opts->counter_words < 1 || opts->grid_blocks < 0 || (opts->async_exec != 0 && opts->async_exec != 1))
        return set_error(GLTRSV_EINVAL, "bad server options");
    gltrsv_server *sv = new (std::nothrow) gltrsv_server();
    if (!sv) return set_error(GLTRSV_ENOMEM, "host allocation");
    sv->opts = *opts;
    hipError_t e = hipGetDevice(&sv->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    const size_t ns = size_t(opts->max_slots);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&sv->d_desc), ns * sizeof(dev::SysDesc));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&sv->d_state), ns * dev::kStateStride * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&sv->d_done), size_t(opts->counter_words) * 4);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&sv->d_finished), 2 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&sv->d_err), sizeof(int32_t));
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&sv->h_desc), ns * sizeof(dev::SysDesc), 0);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&sv->h_state), ns * sizeof(unsigned long long), 0);
    if (e == hipSuccess) e = hipMemset(sv->d_err, 0, sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(sv->d_desc, 0, ns * sizeof(dev::SysDesc));
    // unused slots read as finished: S = 0 and superstep 0
    if (e == hipSuccess) e = hipMemset(sv->d_state, 0, ns * dev::kStateStride * sizeof(unsigned long long));
    int per_cu = 0, cus = 0;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dev::trsv_batched, dev::kBlock, 0);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, sv->device);
    if (e != hipSuccess) {
        free_server_memory(sv);
        delete sv;
        return set_error(e == hipErrorOutOfMemory ? GLTRSV_ENOMEM : GLTRSV_EHIP,
                         std::string("server creation: ") + hipGetErrorString(e));
    }
    std::memset(sv->h_desc, 0, ns * sizeof(dev::SysDesc));
    sv->grid = std::max(1, per_cu * cus);
    if (opts->grid_blocks > 0) sv->grid = std::min(sv->grid, opts->grid_blocks);
    sv->slots.resize(ns);
    sv->arena = new CounterArena(opts->counter_words);
    sv->worker = std::thread(worker_main, sv);
    *out = sv;
    return GLTRSV_OK;
}

int gltrsv_server_submit(gltrsv_server *sv, gltrsv_plan *plan, const double *b, double *x, uint64_t *ticket)
{
    if (!sv || !plan || !ticket || (plan->n && (!b || !x))) return set_error(GLTRSV_EINVAL, "null argument");
    if (plan->device != sv->device) return set_error(GLTRSV_EINVAL, "plan lives on another device");
    if (plan->S > sv->opts.counter_words) return set_error(GLTRSV_ERANGE, "plan has more supersteps than counters");
    if (sv->opts.async_exec && plan->n && b == x)
        return set_error(GLTRSV_EINVAL, "semi-asynchronous server: b must not alias x");
    const int64_t bytes = 16 * plan->n + 4 * int64_t(std::max(1, plan->S)) + 64;   // b, x, counters, slot
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->failure) return set_error(sv->failure, sv->failure_text);
    if (bytes > sv->opts.budget_bytes) return set_error(GLTRSV_ERANGE, "request larger than the whole budget");
    if (sv->inflight_bytes + bytes > sv->opts.budget_bytes)
        return set_error(GLTRSV_EAGAIN, "in-flight budget exhausted; retry after completions");
    *ticket = sv->next_ticket++;
    sv->stats.submitted++;
    if (plan->n == 0 || plan->S == 0) {
        sv->completed.emplace_back(*ticket, now_ns());
        sv->stats.completed++;
        return GLTRSV_OK;
    }
    Request r;
    r.ticket = *ticket;
    r.plan = plan;
    r.b = b;
    r.x = x;
    r.bytes = bytes;
    sv->inflight_bytes += bytes;
    sv->queue.push_back(r);
    sv->cv.notify_one();
    return GLTRSV_OK;
}

int gltrsv_server_poll(gltrsv_server *sv, uint64_t *tickets, int64_t *done_ns, int32_t max, int32_t *ndone)
{
    if (!sv || !ndone || max < 0 || (max > 0 && !tickets)) return set_error(GLTRSV_EINVAL, "bad poll arguments");
    std::lock_guard<std::mutex> g(sv->mu);
    const int32_t k = int32_t(std::min<size_t>(size_t(max), sv->completed.size()));
    for (int32_t i = 0; i < k; i++) {
        tickets[i] = sv->completed[i].first;
        if (done_ns) done_ns[i] = sv->completed[i].second;
    }
    sv->completed.erase(sv->completed.begin(), sv->completed.begin() + k);
    *ndone = k;
    if (sv->failure && k == 0) return set_error(sv->failure, sv->failure_text);
    return GLTRSV_OK;
}

int gltrsv_server_get_stats(gltrsv_server *sv, gltrsv_server_stats *out)
{
    if (!sv || !out) return set_error(GLTRSV_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(sv->mu);
    *out = sv->stats;
    out->queued = int64_t(sv->queue.size());
    out->inflight_bytes = sv->inflight_bytes;
    return GLTRSV_OK;
}

int gltrsv_server_cancel(gltrsv_server *sv, uint64_t ticket)
{
    if (!sv) return set_error(GLTRSV_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(sv->mu);
    for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it)
        if (it->ticket == ticket) {
            sv->inflight_bytes -= it->bytes;
            sv->stats.cancelled++;
            sv->queue.erase(it);
            return GLTRSV_OK;
        }
    for (size_t i = 0; i < sv->slots.size(); i++) {
        Slot &sl = sv->slots[i];
        if (sl.busy && !sl.cancel && sl.req.ticket == ticket) {
            // on the device: the worker drops it at the next quantum boundary;
            // wait for that, so b, x and the plan are free to go on return
            sl.cancel = true;
            sv->cv.notify_one();
            sv->cv_done.wait(lk, [&] { return !sl.busy || sl.req.ticket != ticket || sv->failure != 0; });
            return GLTRSV_OK;
        }
    }
    return set_error(GLTRSV_ENOENT, "no pending request with this ticket");
}

int64_t gltrsv_clock_ns(void) { return now_ns(); }

int gltrsv_server_destroy(gltrsv_server *sv)
{
    if (!sv) return GLTRSV_OK;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    free_server_memory(sv);
    delete sv;
    return GLTRSV_OK;
}

}  // extern "C"
