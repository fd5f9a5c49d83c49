// gltrsv host runtime and C ABI (include/gltrsv.h): option checks, plans
// (analysis, layouts, device upload), the single-system solve forms, the
// execution-form autotuner, batches and the measurement probes.  The kernels
// are in kernels.hip; the server is in serve.hip, device packing in pack.hip.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gltrsv.h"
#include "analysis.h"
#include "internal.h"

// ===========================================================================
// host runtime and C ABI
// ===========================================================================
using namespace gltrsv;

namespace {

thread_local std::string g_last_error = "no error";

}  // namespace

int gltrsv::set_error(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

namespace {

// True if the byte ranges [a, a + na) and [b, b + nb) share a byte.
bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return na && nb && pa < pb + nb && pb < pa + na;
}

// Launches a kernel whose workgroups wait for each other.  cooperative:
// hipLaunchCooperativeKernel (the runtime checks the grid against the
// device's co-resident capacity); otherwise a plain launch of the same
// occupancy-sized grid.  Measured on MI355X, neither keeps ordinary kernels
// on other streams from delaying some of the grid's workgroups, which is why
// the persistent kernels claim and steal their work (see trsv_persistent).
int launch_coresident(const void *kernel, dim3 grid, void **args, hipStream_t st, bool cooperative)
{
    if (cooperative) {
        HIP_TRY(hipLaunchCooperativeKernel(kernel, grid, dim3(dev::kBlock), args, 0, st));
    } else {
        HIP_TRY(hipLaunchKernel(kernel, grid, dim3(dev::kBlock), args, 0, st));
    }
    return GLTRSV_OK;
}

// Start ticket of a plan's semi-asynchronous kernel `which` (0 lane cores,
// 1 several right-hand sides, 2 wave cores).
unsigned long long *async_ticket(gltrsv_plan *p, int which)
{
    return reinterpret_cast<unsigned long long *>(p->d_bar + dev::kBarAsyncTicket + 32 * which);
}

CsrView view_of(const gltrsv_csr *A)
{
    CsrView v;
    v.n = A->n;
    v.nnz = A->nnz;
    v.row_ptr = A->row_ptr;
    v.col = A->col;
    v.val = A->val;
    return v;
}

int check_opts(const gltrsv_plan_opts *o)
{
    if (!o) return set_error(GLTRSV_EINVAL, "null options");
    if (o->schedule_kind != GLTRSV_SCHED_GROWLOCAL && o->schedule_kind != GLTRSV_SCHED_WAVEFRONT &&
        o->schedule_kind != GLTRSV_SCHED_AUTO)
        return set_error(GLTRSV_EINVAL, "unknown schedule kind");
    if (o->schedule_kind != GLTRSV_SCHED_WAVEFRONT) {
        if (o->k < 1) return set_error(GLTRSV_EINVAL, "k must be >= 1");
        if (!(o->alpha0 >= 1.0)) return set_error(GLTRSV_EINVAL, "alpha0 must be >= 1");
        if (!(o->growth > 1.0)) return set_error(GLTRSV_EINVAL, "growth must be > 1");
        if (!(o->L >= 0.0)) return set_error(GLTRSV_EINVAL, "L must be >= 0");
        if (!(o->accept > 0.0)) return set_error(GLTRSV_EINVAL, "accept must be > 0");
    }
    if (o->block_size != 0 && o->block_size != dev::kBlock)
        return set_error(GLTRSV_ENOTSUP, "block_size must be 0 or 256: the kernels are compiled for 256-thread workgroups");
    if (o->grid_blocks < 0) return set_error(GLTRSV_EINVAL, "grid_blocks must be >= 0");
    if (o->analysis_threads < 0 || o->analysis_threads > 64)
        return set_error(GLTRSV_EINVAL, "analysis_threads must be in 0..64");
    if (o->pack != GLTRSV_PACK_AUTO && o->pack != GLTRSV_PACK_HOST && o->pack != GLTRSV_PACK_DEVICE)
        return set_error(GLTRSV_EINVAL, "unknown pack mode");
    if (o->blocks < 0) return set_error(GLTRSV_EINVAL, "blocks must be >= 0");
    if (o->funnel_max_weight < 0) return set_error(GLTRSV_EINVAL, "funnel_max_weight must be >= 0");
    if (o->exec_hint < 0 || o->exec_hint > 2) return set_error(GLTRSV_EINVAL, "exec_hint must be 0, 1 or 2");
    if (o->exec_hint == 2) {
        if (o->core_width == 64) return set_error(GLTRSV_EINVAL, "exec_hint 2 (one workgroup) needs core_width 1");
        if (o->schedule_kind != GLTRSV_SCHED_WAVEFRONT && o->k > 64)
            return set_error(GLTRSV_EINVAL, "exec_hint 2 (one workgroup) needs k <= 64");
    }
    if (o->triangle != GLTRSV_LOWER && o->triangle != GLTRSV_UPPER)
        return set_error(GLTRSV_EINVAL, "triangle must be GLTRSV_LOWER or GLTRSV_UPPER");
    if (o->reorder != 0 && o->reorder != 1) return set_error(GLTRSV_EINVAL, "reorder must be 0 or 1");
    if (o->core_width != 0 && o->core_width != 1 && o->core_width != 64)
        return set_error(GLTRSV_EINVAL, "core_width must be 1 or 64");
    return GLTRSV_OK;
}

SchedParams params_of(const gltrsv_plan_opts *o)
{
    SchedParams p;
    p.k = o->k;
    p.L = o->L;
    p.alpha0 = o->alpha0;
    p.growth = o->growth;
    p.accept = o->accept;
    p.kind = o->schedule_kind;
    p.threads = o->analysis_threads;
    p.blocks = o->blocks;
    p.funnel_max_weight = o->funnel_max_weight;
    return p;
}

template <class T>
int upload_raw(T **dst, const T *src, size_t count, int64_t *bytes)
{
    const size_t nb = std::max<size_t>(1, count) * sizeof(T);
    HIP_TRY(hipMalloc(reinterpret_cast<void **>(dst), nb));
    if (count) HIP_TRY(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    *bytes += int64_t(nb);
    return GLTRSV_OK;
}

template <class T>
int upload(T **dst, const std::vector<T> &src, int64_t *bytes)
{
    return upload_raw(dst, src.data(), src.size(), bytes);
}

// Wave-core layouts (wave.h) of a plan, the record streams for W waves.
int upload_wave(gltrsv_plan *p, const gltrsv_csr *A, int64_t W, int64_t *bytes)
{
    WaveLayout L;
    build_wave_layout(view_of(A), p->upper, p->core.data(), p->superstep.data(), p->S, p->perm, W, &L);
    p->wsuper_host = L.wsuper;
    p->stream_w = W;
    p->ssize_host = std::move(L.ssize);
    int rc;
    if ((rc = upload(&p->d_wrow, L.wrow, bytes)) || (rc = upload(&p->d_wptr, L.wptr, bytes)) ||
        (rc = upload(&p->d_wdiag, L.wdiag, bytes)) || (rc = upload(&p->d_wcol, L.wcol, bytes)) ||
        (rc = upload(&p->d_wval, L.wval, bytes)) || (rc = upload(&p->d_wtask, L.wtask, bytes)) ||
        (rc = upload(&p->d_wsuper, L.wsuper, bytes)) || (rc = upload(&p->d_scol, L.scol, bytes)) ||
        (rc = upload(&p->d_sval, L.sval, bytes)) || (rc = upload(&p->d_sbeg, L.sbeg, bytes)) ||
        (rc = upload(&p->d_stask, L.stask, bytes)))
        return rc;
    return GLTRSV_OK;
}

// For plans kept in the caller's order too (opts.reorder = 0): the CSR as
// given, and the rows of every task, tasks of a superstep longest first.
int upload_unordered(gltrsv_plan *p, const gltrsv_csr *A, int64_t *bytes)
{
    const int64_t n = p->n;
    std::vector<int32_t> rows(static_cast<size_t>(n));
    std::vector<int64_t> off;
    std::vector<int32_t> super_task(size_t(p->S) + 1, 0);
    off.reserve(size_t(p->tasks) + 1);
    off.push_back(0);
    int64_t pos = 0;
    for (int32_t s = 0; s < p->S; s++) {
        // tasks of superstep s: runs of equal core in the order of Sec. 5
        std::vector<std::pair<int64_t, int64_t>> tasks;   // (first position, length)
        while (pos < n && p->superstep[size_t(p->perm[size_t(pos)])] == s) {
            const int32_t c = p->core[size_t(p->perm[size_t(pos)])];
            int64_t q = pos;
            while (q < n && p->superstep[size_t(p->perm[size_t(q)])] == s && p->core[size_t(p->perm[size_t(q)])] == c)
                q++;
            tasks.emplace_back(pos, q - pos);
            pos = q;
        }
        std::stable_sort(tasks.begin(), tasks.end(),
                         [](const std::pair<int64_t, int64_t> &a, const std::pair<int64_t, int64_t> &b) {
                             return a.second > b.second;
                         });
        for (const auto &tk : tasks) {
            for (int64_t q = 0; q < tk.second; q++) {
                const int32_t v = p->perm[size_t(tk.first + q)];
                rows[size_t(off.back() + q)] = p->upper ? int32_t(n - 1 - v) : v;   // original row
            }
            off.push_back(off.back() + tk.second);
        }
        super_task[size_t(s) + 1] = int32_t(off.size() - 1);
    }
    p->super_task_host = super_task;
    int rc;
    if ((rc = upload_raw(&p->d_csr_rp, A->row_ptr, size_t(n) + 1, bytes)) ||
        (rc = upload_raw(&p->d_csr_col, A->col, size_t(A->nnz), bytes)) ||
        (rc = upload_raw(&p->d_csr_val, A->val, size_t(A->nnz), bytes)) || (rc = upload(&p->d_urows, rows, bytes)) ||
        (rc = upload(&p->d_utask_off, off, bytes)))
        return rc;
    return GLTRSV_OK;
}

// GROWLOCAL, WAVEFRONT, or AUTO: both, keeping the lower predicted device
// time (ties go to GrowLocal).  Returns the order of Sec. 5 in *perm and the
// prediction in *cost_us.
Schedule build_schedule(const CsrView &V, const gltrsv_plan_opts *o, std::vector<int32_t> *perm, double *cost_us,
                        int32_t *chosen)
{
    const CostModel cm;
    auto predict = [&](const Schedule &sc, const std::vector<int32_t> &pm) {
        if (o->exec_hint == 2) return double(local_group_count(V, sc, pm)) * kLocalGroupUs;
        return o->exec_hint == 1 ? predict_async_us(V, sc, pm, cm) : predict_cost_us(V, sc, pm, cm);
    };
    // one workgroup: the levels dealt onto its 64 lanes
    auto wavefront = [&]() {
        Schedule w = schedule_wavefront(V);
        if (o->exec_hint == 2) fold_cores(w, 64);
        return w;
    };
    if (o->schedule_kind == GLTRSV_SCHED_WAVEFRONT) {
        Schedule w = wavefront();
        *perm = schedule_order(V.n, w.core.data(), w.superstep.data(), w.S);
        *cost_us = predict(w, *perm);
        *chosen = GLTRSV_SCHED_WAVEFRONT;
        return w;
    }
    Schedule g = schedule_growlocal(V, params_of(o));
    std::vector<int32_t> pg = schedule_order(V.n, g.core.data(), g.superstep.data(), g.S);
    const double cg = predict(g, pg);
    if (o->schedule_kind == GLTRSV_SCHED_AUTO) {
        Schedule w = wavefront();
        std::vector<int32_t> pw = schedule_order(V.n, w.core.data(), w.superstep.data(), w.S);
        const double cw = predict(w, pw);
        if (cw < cg) {
            *perm = std::move(pw);
            *cost_us = cw;
            *chosen = GLTRSV_SCHED_WAVEFRONT;
            return w;
        }
    }
    *perm = std::move(pg);
    *cost_us = cg;
    *chosen = GLTRSV_SCHED_GROWLOCAL;
    return g;
}

}  // namespace

struct gltrsv_batch {
    int32_t count = 0;                 // systems with n > 0
    std::vector<gltrsv_plan *> plans;
    std::vector<int32_t> slot;         // caller index of each kept system
    int32_t ncalls = 0;                // caller's count
    int device = 0;
    int grid = 0;
    int32_t per_claim = 1;
    int32_t ndone = 0;
    bool use_graph = true;
    dev::SysDesc *d_desc = nullptr;
    dev::SysDesc *h_desc[2] = {nullptr, nullptr};   // pinned staging, double-buffered
    hipEvent_t staged[2] = {nullptr, nullptr};
    int32_t flip = 0;
    unsigned long long *d_state = nullptr;
    uint32_t *d_done = nullptr;
    uint32_t *d_finished = nullptr;
    int32_t *d_err = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t graph_stream = nullptr;
    hipStream_t last_stream = nullptr;
    int64_t idle_ticks = 1000000000;   // 10 s of the 100 MHz wall clock
    int32_t keep_waves = 0;            // waves that never retire (see dev::kRetireTicks)
    bool async_exec = false;           // semi-asynchronous kernel (no barriers)
    bool wave = false;                 // ... on wavefront cores (every plan has core width 64)
    int64_t gtasks = 0;                // wave cores: tasks of the global order
    // wave cores: the batch as one system (see stream_rebase): its record
    // stream over the global task order, each system's first row there, and
    // the concatenated b and x
    uint32_t *d_bscol = nullptr;
    double *d_bsval = nullptr;
    int64_t *d_bbeg = nullptr;         // [4 grid + 1] first slot of each wave's stream
    int64_t *d_btask = nullptr;        // [gtasks] first slot of each global task
    int64_t *d_boff = nullptr;         // [count] first row of each system in bcat / xcat
    double *d_bcat = nullptr;
    double *d_xcat = nullptr;
    int64_t rows = 0;                  // rows of all systems
    bool row_dpp = false;              // DPP row subtraction (as for one system of all the rows)
    // wave cores: robbing of workgroups that have not started (start ticket,
    // kMaxGrid alive words, 4 kMaxGrid robbed-prefix words)
    unsigned long long *d_wticket = nullptr;
    uint32_t *d_walive = nullptr;
    unsigned long long *d_wvnext = nullptr;
};

// Semi-asynchronous batches of wavefront-core systems: the record stream of
// the global task order (gsys[g], gtask[g]) for the grid of the launch
// (at most `resident` workgroups, and grid_blocks if positive), built on the
// device from the systems' own streams with rows and columns shifted to
// the concatenated vectors; plus those vectors and the robbing words.
static int batch_stream(gltrsv_batch *bt, const std::vector<int32_t> &gsys, const std::vector<int32_t> &gtask,
                        int resident, int grid_blocks)
{
    const int64_t G = int64_t(gsys.size());
    if (G > INT32_MAX) return set_error(GLTRSV_ERANGE, "too many tasks in a wave-core batch");
    std::vector<int64_t> boff(size_t(bt->count) + 1, 0);
    for (int32_t i = 0; i < bt->count; i++) boff[size_t(i) + 1] = boff[size_t(i)] + bt->plans[size_t(i)]->n;
    bt->rows = boff.back();
    if (bt->rows > kMaxRows)
        return set_error(GLTRSV_ERANGE, "a semi-asynchronous wave-core batch holds at most 2^30 - 1 rows");
    int64_t grid = std::min<int64_t>(std::max(1, resident), dev::kMaxGrid);
    if (grid_blocks > 0) grid = std::min<int64_t>(grid, grid_blocks);
    grid = std::max<int64_t>(1, std::min<int64_t>(grid, (G + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock));
    bt->grid = int(grid);
    const int64_t W = grid * dev::kWavesPerBlock;
    const size_t ng = size_t(std::max<int64_t>(G, 1));
    std::vector<int64_t> bbeg(size_t(W) + 1), btask(ng, 0), bsize(ng, 0);
    int64_t so = 0;
    for (int64_t v = 0; v < W; v++) {
        bbeg[size_t(v)] = so;
        for (int64_t g = v; g < G; g += W) {
            btask[size_t(g)] = so;
            bsize[size_t(g)] = bt->plans[size_t(gsys[size_t(g)])]->ssize_host[size_t(gtask[size_t(g)])];
            so += bsize[size_t(g)];
        }
        so++;   // the slot's PAD
    }
    bbeg[size_t(W)] = so;
    std::vector<dev::StreamSrc> src(size_t(bt->count));
    for (int32_t i = 0; i < bt->count; i++) {
        const gltrsv_plan *pl = bt->plans[size_t(i)];
        src[size_t(i)] = dev::StreamSrc{pl->d_scol, pl->d_sval, pl->d_stask, boff[size_t(i)]};
    }
    boff.pop_back();
    int64_t bytes = 0;
    int rc;
    int32_t *d_gsys = nullptr, *d_gtask = nullptr;
    int64_t *d_bsize = nullptr;
    dev::StreamSrc *d_src = nullptr;
    std::vector<unsigned long long> ticket(16, 0ull), vnext(size_t(dev::kMaxGrid * dev::kWavesPerBlock), 0ull);
    std::vector<uint32_t> alive(size_t(dev::kMaxGrid), 0u);
    auto release = [&]() {
        (void)hipFree(d_gsys);
        (void)hipFree(d_gtask);
        (void)hipFree(d_bsize);
        (void)hipFree(d_src);
    };
    if ((rc = upload(&d_gsys, gsys, &bytes)) || (rc = upload(&d_gtask, gtask, &bytes)) ||
        (rc = upload(&d_bsize, bsize, &bytes)) || (rc = upload(&d_src, src, &bytes)) ||
        (rc = upload(&bt->d_bbeg, bbeg, &bytes)) || (rc = upload(&bt->d_btask, btask, &bytes)) ||
        (rc = upload(&bt->d_boff, boff, &bytes)) || (rc = upload(&bt->d_wticket, ticket, &bytes)) ||
        (rc = upload(&bt->d_walive, alive, &bytes)) || (rc = upload(&bt->d_wvnext, vnext, &bytes))) {
        release();
        return rc;
    }
    const size_t slots = size_t(so + kStreamPad);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&bt->d_bscol), slots * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&bt->d_bsval), slots * sizeof(double));
    const size_t vec = size_t(std::max<int64_t>(1, bt->rows)) * sizeof(double);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&bt->d_bcat), vec);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&bt->d_xcat), vec);
    // every slot starts as PAD (the slots' ends and the padding keep it)
    if (e == hipSuccess) e = hipMemset(bt->d_bscol, 0xFF, slots * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(bt->d_bsval, 0, slots * sizeof(double));
    if (e == hipSuccess && G > 0) {
        const int64_t blocks = std::min<int64_t>(4096, (G + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock);
        hipLaunchKernelGGL(dev::stream_rebase, dim3(unsigned(blocks)), dim3(dev::kBlock), 0, nullptr, d_src, d_gsys,
                           d_gtask, bt->d_btask, d_bsize, G, bt->d_bscol, bt->d_bsval);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    release();
    if (e != hipSuccess)
        return set_error(e == hipErrorOutOfMemory ? GLTRSV_ENOMEM : GLTRSV_EHIP,
                         std::string("batch stream: ") + hipGetErrorString(e));
    return GLTRSV_OK;
}

extern "C" {

const char *gltrsv_last_error(void) { return g_last_error.c_str(); }

const char *gltrsv_version(void) { return "0.1.0"; }

void gltrsv_default_opts(gltrsv_plan_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->k = 22;
    o->L = 500.0;
    o->alpha0 = 20.0;
    o->growth = 1.5;
    o->accept = 0.97;
    o->schedule_kind = GLTRSV_SCHED_GROWLOCAL;
    o->reorder = 1;
    o->block_size = 0;
    o->grid_blocks = 0;
    o->cooperative = 0;
    o->analysis_threads = 0;
    o->pack = GLTRSV_PACK_AUTO;
    o->blocks = 0;
    o->triangle = GLTRSV_LOWER;
    o->funnel_max_weight = 0;
    o->exec_hint = 0;
}

int gltrsv_check_csr(const gltrsv_csr *A)
{
    if (!A) return set_error(GLTRSV_EINVAL, "null matrix");
    std::string msg;
    const int rc = check_csr(view_of(A), A->val != nullptr, &msg);
    return rc ? set_error(rc, msg) : GLTRSV_OK;
}

int gltrsv_levels(const gltrsv_csr *A, int32_t *level, int32_t *nlevels)
{
    if (!A || !nlevels) return set_error(GLTRSV_EINVAL, "null argument");
    std::string msg;
    const int rc = check_csr(view_of(A), false, &msg);
    if (rc) return set_error(rc, msg);
    std::vector<int32_t> lv;
    *nlevels = wavefront_levels(view_of(A), lv);
    if (level && A->n) std::memcpy(level, lv.data(), sizeof(int32_t) * A->n);
    return GLTRSV_OK;
}

int gltrsv_schedule(const gltrsv_csr *A, const gltrsv_plan_opts *opts, int32_t *core, int32_t *superstep,
                    int32_t *S)
{
    if (!A || !core || !superstep || !S) return set_error(GLTRSV_EINVAL, "null argument");
    int rc = check_opts(opts);
    if (rc) return rc;
    std::string msg;
    const bool upper = opts->triangle == GLTRSV_UPPER;
    rc = upper ? check_csr_upper(view_of(A), false, &msg) : check_csr(view_of(A), false, &msg);
    if (rc) return set_error(rc, msg);
    Mirror mir;
    if (upper) mir = mirror_upper(view_of(A));
    std::vector<int32_t> perm;
    double cost = 0.0;
    int32_t chosen = 0;
    Schedule s = build_schedule(upper ? mir.view() : view_of(A), opts, &perm, &cost, &chosen);
    const int64_t n = A->n;
    for (int64_t i = 0; i < n; i++) {   // a backward solve's vertex v is row n-1-v
        core[i] = s.core[size_t(upper ? n - 1 - i : i)];
        superstep[i] = s.superstep[size_t(upper ? n - 1 - i : i)];
    }
    *S = s.S;
    return GLTRSV_OK;
}

int gltrsv_reorder(int64_t n, const int32_t *core, const int32_t *superstep, int32_t *perm)
{
    if (n < 0 || (n > 0 && (!core || !superstep || !perm))) return set_error(GLTRSV_EINVAL, "bad argument");
    int32_t S = 0;
    for (int64_t i = 0; i < n; i++) {
        if (core[i] < 0 || superstep[i] < 0) return set_error(GLTRSV_ERANGE, "negative core or superstep");
        S = std::max(S, superstep[i] + 1);
    }
    std::vector<int32_t> p = schedule_order(n, core, superstep, S);
    if (n) std::memcpy(perm, p.data(), sizeof(int32_t) * n);
    return GLTRSV_OK;
}

int gltrsv_local_layout(const gltrsv_csr *A, int32_t triangle, const int32_t *core, const int32_t *superstep,
                        void *rec, int64_t *rec_bytes, uint32_t *info, int64_t *records)
{
    if (!A || !rec_bytes || !records || (A->n > 0 && (!core || !superstep)))
        return set_error(GLTRSV_EINVAL, "null argument");
    if (triangle != GLTRSV_LOWER && triangle != GLTRSV_UPPER) return set_error(GLTRSV_EINVAL, "bad triangle");
    const bool upper = triangle == GLTRSV_UPPER;
    const CsrView V = view_of(A);
    std::string msg;
    int rc = upper ? check_csr_upper(V, true, &msg) : check_csr(V, true, &msg);
    if (rc) return set_error(rc, msg);
    Mirror mir;
    if (upper) mir = mirror_upper(V);
    const CsrView D = upper ? mir.view() : V;
    const int64_t n = A->n;
    Schedule s;
    s.core.resize(size_t(n));
    s.superstep.resize(size_t(n));
    for (int64_t v = 0; v < n; v++) {
        const int64_t row = upper ? n - 1 - v : v;
        s.core[size_t(v)] = core[row];
        s.superstep[size_t(v)] = superstep[row];
        s.S = std::max(s.S, superstep[row] + 1);
    }
    if ((rc = validate_schedule(D, s, &msg))) return set_error(rc, "schedule: " + msg);
    const std::vector<int32_t> perm = schedule_order(n, s.core.data(), s.superstep.data(), s.S);
    LocalLayout lay;
    if ((rc = build_local_layout(V, upper, s, perm, &lay, &msg))) return set_error(rc, msg);
    if (!rec || !info) {
        *rec_bytes = int64_t(lay.rec.size());
        *records = int64_t(lay.info.size());
        return GLTRSV_OK;
    }
    if (*rec_bytes != int64_t(lay.rec.size()) || *records != int64_t(lay.info.size()))
        return set_error(GLTRSV_EINVAL, "buffer sizes differ from the layout's (query them with null buffers)");
    if (!lay.rec.empty()) std::memcpy(rec, lay.rec.data(), lay.rec.size());
    if (!lay.info.empty()) std::memcpy(info, lay.info.data(), lay.info.size() * sizeof(LocalRec));
    return GLTRSV_OK;
}

int gltrsv_wave_streams(const gltrsv_csr *A, int32_t triangle, const int32_t *core, const int32_t *superstep,
                        int64_t waves, uint32_t *scol, double *sval, int64_t *sbeg, int64_t *stask, int64_t *slots,
                        int64_t *tasks)
{
    if (!A || !slots || !tasks || (A->n > 0 && (!core || !superstep))) return set_error(GLTRSV_EINVAL, "null argument");
    if (triangle != GLTRSV_LOWER && triangle != GLTRSV_UPPER) return set_error(GLTRSV_EINVAL, "bad triangle");
    if (waves < 1 || waves > int64_t(dev::kMaxGrid) * dev::kWavesPerBlock)
        return set_error(GLTRSV_EINVAL, "waves must be 1 .. 4 x the largest grid");
    const bool upper = triangle == GLTRSV_UPPER;
    const CsrView V = view_of(A);
    std::string msg;
    int rc = upper ? check_csr_upper(V, true, &msg) : check_csr(V, true, &msg);
    if (rc) return set_error(rc, msg);
    Mirror mir;
    if (upper) mir = mirror_upper(V);
    const CsrView D = upper ? mir.view() : V;
    const int64_t n = A->n;
    Schedule s;
    s.core.resize(size_t(n));
    s.superstep.resize(size_t(n));
    for (int64_t v = 0; v < n; v++) {
        const int64_t row = upper ? n - 1 - v : v;
        s.core[size_t(v)] = core[row];
        s.superstep[size_t(v)] = superstep[row];
        s.S = std::max(s.S, superstep[row] + 1);
    }
    if ((rc = validate_schedule(D, s, &msg))) return set_error(rc, "schedule: " + msg);
    const std::vector<int32_t> perm = schedule_order(n, s.core.data(), s.superstep.data(), s.S);
    WaveLayout L;
    build_wave_layout(V, upper, s.core.data(), s.superstep.data(), s.S, perm, waves, &L);
    if (!scol || !sval || !sbeg || !stask) {
        *slots = int64_t(L.scol.size());
        *tasks = int64_t(L.stask.size());
        return GLTRSV_OK;
    }
    if (*slots != int64_t(L.scol.size()) || *tasks != int64_t(L.stask.size()))
        return set_error(GLTRSV_EINVAL, "buffer sizes differ from the streams' (query them with null buffers)");
    std::memcpy(scol, L.scol.data(), L.scol.size() * sizeof(uint32_t));
    std::memcpy(sval, L.sval.data(), L.sval.size() * sizeof(double));
    std::memcpy(sbeg, L.sbeg.data(), L.sbeg.size() * sizeof(int64_t));
    if (!L.stask.empty()) std::memcpy(stask, L.stask.data(), L.stask.size() * sizeof(int64_t));
    return GLTRSV_OK;
}

int gltrsv_plan_destroy(gltrsv_plan *p)
{
    if (!p) return GLTRSV_OK;
    (void)hipFree(p->d_word);
    (void)hipFree(p->d_value);
    (void)hipFree(p->d_chunk_base);
    (void)hipFree(p->d_chunk_len);
    (void)hipFree(p->d_super_chunk);
    (void)hipFree(p->d_bar);
    (void)hipFree(p->d_claim);
    (void)hipFree(p->d_alive);
    (void)hipFree(p->d_aalive);
    (void)hipFree(p->d_vnext);
    (void)hipFree(p->d_wclaim);
    (void)hipFree(p->d_err);
    (void)hipFree(p->d_trace);
    (void)hipFree(p->d_bcopy);
    (void)hipFree(p->d_csr_rp);
    (void)hipFree(p->d_csr_col);
    (void)hipFree(p->d_csr_val);
    (void)hipFree(p->d_urows);
    (void)hipFree(p->d_utask_off);
    (void)hipFree(p->d_wrow);
    (void)hipFree(p->d_wptr);
    (void)hipFree(p->d_wdiag);
    (void)hipFree(p->d_wcol);
    (void)hipFree(p->d_wval);
    (void)hipFree(p->d_wtask);
    (void)hipFree(p->d_wsuper);
    (void)hipFree(p->d_scol);
    (void)hipFree(p->d_sval);
    (void)hipFree(p->d_sbeg);
    (void)hipFree(p->d_stask);
    (void)hipFree(p->d_lrec);
    (void)hipFree(p->d_linfo);
    delete p;
    return GLTRSV_OK;
}

static int plan_create_impl(const gltrsv_csr *A, const gltrsv_plan_opts *opts, const int32_t *core_in,
                            const int32_t *superstep_in, gltrsv_plan **out);

int gltrsv_plan_create(const gltrsv_csr *A, const gltrsv_plan_opts *opts, gltrsv_plan **out)
{
    return plan_create_impl(A, opts, nullptr, nullptr, out);
}

int gltrsv_plan_create_with_schedule(const gltrsv_csr *A, const gltrsv_plan_opts *opts, const int32_t *core,
                                     const int32_t *superstep, gltrsv_plan **out)
{
    if (!A || (A->n > 0 && (!core || !superstep))) return set_error(GLTRSV_EINVAL, "null schedule");
    return plan_create_impl(A, opts, core, superstep, out);
}

static int plan_create_impl(const gltrsv_csr *A, const gltrsv_plan_opts *opts, const int32_t *core_in,
                            const int32_t *superstep_in, gltrsv_plan **out)
{
    if (!A || !out) return set_error(GLTRSV_EINVAL, "null argument");
    *out = nullptr;
    int rc = check_opts(opts);
    if (rc) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    const CsrView V = view_of(A);
    const bool upper = opts->triangle == GLTRSV_UPPER;
    std::string msg;
    rc = upper ? check_csr_upper(V, true, &msg) : check_csr(V, true, &msg);
    if (rc) return set_error(rc, msg);
    // a backward solve is scheduled on its mirrored (lower) pattern
    Mirror mir;
    if (upper) mir = mirror_upper(V);
    const CsrView D = upper ? mir.view() : V;   // the DAG in the solve's direction

    gltrsv_plan *p = new (std::nothrow) gltrsv_plan();
    if (!p) return set_error(GLTRSV_ENOMEM, "host allocation");
    p->n = A->n;
    p->nnz = A->nnz;
    p->upper = upper;
    Schedule s;
    if (core_in) {
        // a schedule from an earlier analysis (per row; for a backward solve
        // vertex v is row n-1-v): checked against Definition 2.1
        const int64_t n = A->n;
        s.core.resize(size_t(n));
        s.superstep.resize(size_t(n));
        for (int64_t v = 0; v < n; v++) {
            const int64_t row = upper ? n - 1 - v : v;
            s.core[size_t(v)] = core_in[row];
            s.superstep[size_t(v)] = superstep_in[row];
            s.S = std::max(s.S, superstep_in[row] + 1);
        }
        if ((rc = validate_schedule(D, s, &msg))) {
            delete p;
            return set_error(rc, "given schedule: " + msg);
        }
        p->perm = schedule_order(n, s.core.data(), s.superstep.data(), s.S);
        const CostModel cm;
        if (opts->exec_hint == 2) {
            for (int64_t v = 0; v < n; v++)
                if (s.core[size_t(v)] >= 64) {
                    delete p;
                    return set_error(GLTRSV_EINVAL, "given schedule: exec_hint 2 (one workgroup) needs cores 0..63");
                }
            p->predicted_us = double(local_group_count(D, s, p->perm)) * kLocalGroupUs;
        } else {
            p->predicted_us =
                opts->exec_hint == 1 ? predict_async_us(D, s, p->perm, cm) : predict_cost_us(D, s, p->perm, cm);
        }
        p->schedule_kind = GLTRSV_SCHED_GIVEN;
    } else {
        s = build_schedule(D, opts, &p->perm, &p->predicted_us, &p->schedule_kind);
    }
    std::vector<int32_t> lv;
    p->wavefronts = wavefront_levels(D, lv);
    LocalLayout local;
    if (opts->exec_hint == 2 && (rc = build_local_layout(V, upper, s, p->perm, &local, &msg))) {
        delete p;
        return set_error(rc, msg);
    }
    const bool on_device =
        opts->pack == GLTRSV_PACK_DEVICE || (opts->pack == GLTRSV_PACK_AUTO && V.nnz >= (int64_t(1) << 20));
    PackLayout lay = pack_layout(D, s, p->perm);
    if (!on_device) {
        if (upper) pack_fill_upper(V, p->perm, lay);
        else pack_fill(V, s, p->perm, lay);
    }
    Packed &pk = lay.pk;
    p->S = s.S;
    p->core = std::move(s.core);
    p->superstep = std::move(s.superstep);
    p->tasks = pk.tasks;
    p->chunks = int64_t(pk.chunk_len.size());
    p->slots = pk.slots;
    p->max_task_rows = pk.max_task_rows;
    p->super_chunk_host = pk.super_chunk;
    p->key = pattern_key(V);

    HIP_TRY(hipGetDevice(&p->device));
    int64_t bytes = 0;
    if (on_device) {
        const size_t ns = size_t(std::max<int64_t>(1, pk.slots));
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&p->d_word), ns * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&p->d_value), ns * sizeof(double));
        if (e != hipSuccess) {
            gltrsv_plan_destroy(p);
            return set_error(e == hipErrorOutOfMemory ? GLTRSV_ENOMEM : GLTRSV_EHIP, "stream allocation");
        }
        bytes += int64_t(ns) * 12;
        if ((rc = dev::device_pack(V, p->perm, lay, upper, p->d_word, p->d_value))) {
            gltrsv_plan_destroy(p);
            return rc;
        }
    } else if ((rc = upload(&p->d_word, pk.word, &bytes)) || (rc = upload(&p->d_value, pk.value, &bytes))) {
        gltrsv_plan_destroy(p);
        return rc;
    }
    p->device_packed = on_device;
    p->exec_form = opts->exec_hint == 1 ? GLTRSV_EXEC_ASYNC : GLTRSV_EXEC_PERSISTENT;
    if (opts->exec_hint == 2) {
        if ((rc = upload(&p->d_lrec, local.rec, &bytes)) || (rc = upload(&p->d_linfo, local.info, &bytes))) {
            gltrsv_plan_destroy(p);
            return rc;
        }
        p->l_nrec = int32_t(local.info.size());
        p->l_bytes = int64_t(local.rec.size());
        p->l_groups = local.groups;
        p->l_far = local.far;
        p->exec_form = GLTRSV_EXEC_LOCAL;
    }
    if ((rc = upload(&p->d_chunk_base, pk.chunk_base, &bytes)) || (rc = upload(&p->d_chunk_len, pk.chunk_len, &bytes)) ||
        (rc = upload(&p->d_super_chunk, pk.super_chunk, &bytes))) {
        gltrsv_plan_destroy(p);
        return rc;
    }
    {
        std::vector<uint32_t> bar(dev::kBarWords, 0u);
        std::vector<int32_t> err(1, 0);
        std::vector<uint32_t> claim(size_t(std::max<int64_t>(1, p->chunks)), 0u);
        std::vector<uint32_t> alive(size_t(dev::kMaxGrid), 0u);
        std::vector<uint32_t> aalive(size_t(3 * dev::kMaxGrid), 0u);
        std::vector<unsigned long long> vnext(size_t(3 * dev::kMaxGrid * dev::kWavesPerBlock), 0ull);
        if ((rc = upload(&p->d_bar, bar, &bytes)) || (rc = upload(&p->d_err, err, &bytes)) ||
            (rc = upload(&p->d_claim, claim, &bytes)) || (rc = upload(&p->d_alive, alive, &bytes)) ||
            (rc = upload(&p->d_aalive, aalive, &bytes)) || (rc = upload(&p->d_vnext, vnext, &bytes))) {
            gltrsv_plan_destroy(p);
            return rc;
        }
    }
    if (opts->reorder == 0 && (rc = upload_unordered(p, A, &bytes))) {
        gltrsv_plan_destroy(p);
        return rc;
    }
    p->core_width = opts->core_width == 64 ? 64 : 1;
    p->row_dpp = p->core_width == 64 && p->n > 0 && p->nnz - p->n >= dev::kDppMinPerRow * p->n;
    if (p->core_width == 64) {
        // semi-asynchronous wave cores: at least two workgroups per CU, more
        // for large systems (about one wave per 1,024 rows), all co-resident.
        // Measured on MI355X: 512 workgroups were best for the n = 1e5 ER
        // and NB sets, the full 2,048 for n = 1e7.  The per-wave streams are
        // built for this grid.
        int per_cu_wa = 0, cus_wa = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu_wa,
            p->row_dpp ? reinterpret_cast<const void *>(dev::trsv_stream_async<true>)
                          : reinterpret_cast<const void *>(dev::trsv_stream_async<false>),
            dev::kBlock, 0);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus_wa, hipDeviceAttributeMultiprocessorCount, p->device);
        if (e != hipSuccess) {
            gltrsv_plan_destroy(p);
            return set_error(GLTRSV_EHIP, std::string("occupancy query: ") + hipGetErrorString(e));
        }
        per_cu_wa = std::min(per_cu_wa, dev::kStreamWgPerCu);   // (the query counts no scalar registers)
        int64_t gwa = std::min<int64_t>(int64_t(per_cu_wa) * cus_wa,
                                        std::max<int64_t>(2 * int64_t(cus_wa), (p->n + 4095) / 4096));
        if (opts->grid_blocks > 0) gwa = std::min<int64_t>(opts->grid_blocks, int64_t(per_cu_wa) * cus_wa);
        gwa = std::min<int64_t>(gwa, dev::kMaxGrid);
        p->grid_wave_async = int(std::max<int64_t>(
            1, std::min<int64_t>(gwa, (p->tasks + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock)));
        if ((rc = upload_wave(p, A, int64_t(p->grid_wave_async) * dev::kWavesPerBlock, &bytes))) {
            gltrsv_plan_destroy(p);
            return rc;
        }
        std::vector<uint32_t> wclaim(size_t(std::max(1, p->wsuper_host.back())), 0u);
        if ((rc = upload(&p->d_wclaim, wclaim, &bytes))) {
            gltrsv_plan_destroy(p);
            return rc;
        }
    }
    p->device_bytes = bytes;

    // persistent grid: every workgroup must be co-resident (cooperative launch)
    int per_cu = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dev::trsv_persistent, dev::kBlock, 0);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) {
        gltrsv_plan_destroy(p);
        return set_error(GLTRSV_EHIP, std::string("occupancy query: ") + hipGetErrorString(e));
    }
    int grid = std::min(per_cu * cus, dev::kMaxGrid);
    if (opts->grid_blocks > 0) grid = std::min(grid, opts->grid_blocks);
    p->cooperative = opts->cooperative != 0;
    // no more workgroups than the widest superstep can use
    int64_t widest = 0;
    for (int32_t q = 0; q < p->S; q++)
        widest = std::max<int64_t>(widest, p->super_chunk_host[q + 1] - p->super_chunk_host[q]);
    p->widest = widest;
    const int64_t useful = (widest + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock;
    grid = int(std::max<int64_t>(1, std::min<int64_t>(grid, useful)));
    p->grid = grid;
    // semi-asynchronous kernel: waves in flight = about four supersteps of
    // average width, at most one workgroup per CU (more waves only add
    // polling of not-yet-computed rows), all co-resident
    {
        int per_cu_a = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_a, dev::trsv_async, dev::kBlock, 0);
        if (e != hipSuccess) {
            gltrsv_plan_destroy(p);
            return set_error(GLTRSV_EHIP, std::string("occupancy query: ") + hipGetErrorString(e));
        }
        int64_t ga = std::min<int64_t>(int64_t(per_cu_a) * cus, cus);
        const int64_t avg_width = p->S > 0 ? (p->chunks + p->S - 1) / p->S : 1;
        ga = std::min<int64_t>(ga, avg_width);   // avg_width chunks x 4 waves per block = 4 supersteps
        if (opts->grid_blocks > 0) ga = opts->grid_blocks < per_cu_a * cus ? opts->grid_blocks : per_cu_a * cus;
        p->grid_async = int(std::max<int64_t>(
            1, std::min<int64_t>(ga, (p->chunks + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock)));
    }
    if (p->core_width == 64) {
        // wave cores: co-resident for the barrier, no more workgroups than
        // the superstep with the most tasks can use
        int per_cu_w = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu_w,
            p->row_dpp ? reinterpret_cast<const void *>(dev::trsv_wave<true>)
                       : reinterpret_cast<const void *>(dev::trsv_wave<false>),
            dev::kBlock, 0);
        if (e != hipSuccess) {
            gltrsv_plan_destroy(p);
            return set_error(GLTRSV_EHIP, std::string("occupancy query: ") + hipGetErrorString(e));
        }
        int64_t most = 1;
        for (int32_t q = 0; q < p->S; q++)
            most = std::max<int64_t>(most, p->wsuper_host[size_t(q) + 1] - p->wsuper_host[size_t(q)]);
        int64_t gw = std::min<int64_t>(int64_t(per_cu_w) * cus, dev::kMaxGrid);
        if (opts->grid_blocks > 0) gw = std::min<int64_t>(gw, opts->grid_blocks);
        p->grid_wave = int(std::max<int64_t>(1, std::min<int64_t>(gw, (most + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock)));
    }
#ifdef GLTRSV_TRACE
    {
        std::vector<int64_t> tr(size_t(p->S) * grid * 3, 0);
        if ((rc = upload(&p->d_trace, tr, &bytes))) {
            gltrsv_plan_destroy(p);
            return rc;
        }
    }
#endif
    p->analysis_ns =
        std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
    *out = p;
    return GLTRSV_OK;
}

int gltrsv_plan_info_get(const gltrsv_plan *p, gltrsv_plan_info *o)
{
    if (!p || !o) return set_error(GLTRSV_EINVAL, "null argument");
    std::memset(o, 0, sizeof(*o));
    o->n = p->n;
    o->nnz = p->nnz;
    o->supersteps = p->S;
    o->wavefronts = p->wavefronts;
    o->tasks = p->tasks;
    o->chunks = p->chunks;
    o->stream_slots = p->slots;
    o->device_bytes = p->device_bytes;
    o->analysis_ns = p->analysis_ns;
    o->pattern_key = p->key;
    o->grid_blocks = p->grid;
    o->block_size = dev::kBlock;
    o->max_task_rows = p->max_task_rows;
    o->schedule_kind = p->schedule_kind;
    o->predicted_us = p->predicted_us;
    o->device_packed = p->device_packed ? 1 : 0;
    o->async_grid_blocks = p->grid_async;
    o->exec_form = p->exec_form;
    o->core_width = p->core_width;
    o->local_groups = p->l_groups;
    o->local_records = p->l_nrec;
    o->local_far = p->l_far;
    o->row_dpp = p->row_dpp ? 1 : 0;
    return GLTRSV_OK;
}

int gltrsv_plan_schedule(const gltrsv_plan *p, int32_t *core, int32_t *superstep, int32_t *perm)
{
    if (!p) return set_error(GLTRSV_EINVAL, "null plan");
    const size_t nb = sizeof(int32_t) * size_t(p->n);
    if (!p->upper) {
        if (core && p->n) std::memcpy(core, p->core.data(), nb);
        if (superstep && p->n) std::memcpy(superstep, p->superstep.data(), nb);
        if (perm && p->n) std::memcpy(perm, p->perm.data(), nb);
        return GLTRSV_OK;
    }
    // backward solve: vertex v of the schedule is row n-1-v
    const int64_t n = p->n;
    for (int64_t i = 0; i < n; i++) {
        if (core) core[i] = p->core[size_t(n - 1 - i)];
        if (superstep) superstep[i] = p->superstep[size_t(n - 1 - i)];
        if (perm) perm[i] = int32_t(n - 1 - p->perm[size_t(i)]);
    }
    return GLTRSV_OK;
}

int gltrsv_solve_plain(gltrsv_plan *p, const double *b, double *x, void *stream)
{
    if (!p || (p->n && (!b || !x))) return set_error(GLTRSV_EINVAL, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->core_width == 64) {
        for (int32_t s = 0; s < p->S; s++) {
            const int32_t tasks = p->wsuper_host[size_t(s) + 1] - p->wsuper_host[size_t(s)];
            const int32_t blocks = (tasks + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock;
            if (blocks == 0) continue;
            hipLaunchKernelGGL(p->row_dpp ? dev::trsv_wave<true> : dev::trsv_wave<false>, dim3(blocks),
                               dim3(dev::kBlock), 0, st, p->d_wrow, p->d_wptr, p->d_wdiag, p->d_wcol, p->d_wval,
                               p->d_wtask, p->d_wsuper, s, s + 1, b, x, p->d_bar, static_cast<uint32_t *>(nullptr),
                               static_cast<uint32_t *>(nullptr), p->d_err, p->spin_limit, int64_t(0), int64_t(0));
        }
        HIP_TRY(hipGetLastError());
        p->last_stream = st;
        return GLTRSV_OK;
    }
    for (int32_t s = 0; s < p->S; s++) {
        const int32_t c0 = p->super_chunk_host[s], c1 = p->super_chunk_host[s + 1];
        const int32_t waves = c1 - c0;
        const int32_t blocks = (waves + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock;
        hipLaunchKernelGGL(dev::trsv_superstep_plain, dim3(blocks), dim3(dev::kBlock), 0, st, p->d_word,
                           p->d_value, p->d_chunk_base, p->d_chunk_len, c0, c1, b, x);
    }
    HIP_TRY(hipGetLastError());
    p->last_stream = st;
    return GLTRSV_OK;
}

int gltrsv_solve(gltrsv_plan *p, const double *b, double *x, void *stream)
{
    if (!p || (p->n && (!b || !x))) return set_error(GLTRSV_EINVAL, "null argument");
    if (p->n == 0) return GLTRSV_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->core_width == 64) {
        // all supersteps in one launch with the grid barrier between them
        const int32_t *wr = p->d_wrow, *ws = p->d_wsuper;
        const int64_t *wp = p->d_wptr, *wt = p->d_wtask;
        const double *wd = p->d_wdiag, *wv = p->d_wval;
        const uint32_t *wc = p->d_wcol;
        int32_t s0 = 0, s1 = p->S;
        uint32_t *bar = p->d_bar;
        uint32_t *alive = p->d_alive;
        uint32_t *claim = p->d_wclaim;
        int32_t *err = p->d_err;
        int64_t lim = p->spin_limit;
        int64_t steal = p->steal_ticks;
        int64_t delay = p->delay_ticks;
        void *args[] = {&wr, &wp, &wd, &wc, &wv, &wt, &ws, &s0, &s1, &b, &x, &bar, &alive, &claim, &err, &lim, &steal,
                        &delay};
        const void *kern = p->row_dpp ? reinterpret_cast<const void *>(dev::trsv_wave<true>)
                                      : reinterpret_cast<const void *>(dev::trsv_wave<false>);
        if (int rc = launch_coresident(kern, dim3(p->grid_wave), args, st, p->cooperative))
            return rc;
        p->last_stream = st;
        return GLTRSV_OK;
    }
    const uint32_t *w = p->d_word;
    const double *v = p->d_value;
    const int64_t *cb = p->d_chunk_base;
    const int32_t *cl = p->d_chunk_len;
    const int32_t *sc = p->d_super_chunk;
    int32_t S = p->S;
    uint32_t *bar = p->d_bar;
    uint32_t *alive = p->d_alive;
    uint32_t *claim = p->d_claim;
    int32_t *err = p->d_err;
    int64_t lim = p->spin_limit;
    int64_t steal = p->steal_ticks;
    int64_t delay = p->delay_ticks;
    int64_t *tr = p->d_trace;
    void *args[] = {&w, &v, &cb, &cl, &sc, &S, &b, &x, &bar, &alive, &claim, &err, &lim, &steal, &delay, &tr};
    // Without the cooperative launch the grid still fits the device's
    // co-resident capacity (occupancy query at plan creation), but should
    // other work keep workgroups from starting, the waiting ones reach the
    // spin limit and the solve reports GLTRSV_ETIMEDOUT.
    if (int rc = launch_coresident(reinterpret_cast<const void *>(dev::trsv_persistent), dim3(p->grid), args, st,
                                   p->cooperative))
        return rc;
    p->last_stream = st;
    return GLTRSV_OK;
}

int gltrsv_solve_async(gltrsv_plan *p, const double *b, double *x, void *stream)
{
    if (!p || (p->n && (!b || !x))) return set_error(GLTRSV_EINVAL, "null argument");
    if (p->n == 0) return GLTRSV_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t vec = sizeof(double) * size_t(p->n);
    if (b != x && overlap(b, vec, x, vec)) return set_error(GLTRSV_EINVAL, "b and x overlap without being equal");
    const double *bb = b;
    if (b == x) {   // x is about to be overwritten with the not-yet-computed mark
        if (!p->d_bcopy) HIP_TRY(hipMalloc(reinterpret_cast<void **>(&p->d_bcopy), sizeof(double) * size_t(p->n)));
        HIP_TRY(hipMemcpyAsync(p->d_bcopy, b, sizeof(double) * size_t(p->n), hipMemcpyDeviceToDevice, st));
        bb = p->d_bcopy;
    }
    const int64_t fill_blocks = std::min<int64_t>(4096, (p->n + dev::kBlock - 1) / dev::kBlock);
    hipLaunchKernelGGL(dev::fill_unready, dim3(unsigned(fill_blocks)), dim3(dev::kBlock), 0, st,
                       reinterpret_cast<unsigned long long *>(x), p->n);
    int64_t lim = p->spin_limit;
    int32_t *err = p->d_err;
    // static task orders; waves that wait long rob workgroups that have not
    // started, so no co-residency is needed (plain launches)
    if (p->core_width == 64) {
        hipLaunchKernelGGL(p->row_dpp ? dev::trsv_stream_async<true> : dev::trsv_stream_async<false>,
                           dim3(p->grid_wave_async), dim3(dev::kBlock), 0, st, p->d_scol, p->d_sval, p->d_sbeg,
                           p->d_stask, p->wsuper_host.back(), bb, x, err, lim, async_ticket(p, 2),
                           p->d_aalive + 2 * dev::kMaxGrid, p->d_vnext + 2 * dev::kMaxGrid * dev::kWavesPerBlock,
                           dev::kRobTicks, p->delay_ticks);
        HIP_TRY(hipGetLastError());
        p->last_stream = st;
        return GLTRSV_OK;
    }
    hipLaunchKernelGGL(dev::trsv_async, dim3(p->grid_async), dim3(dev::kBlock), 0, st, p->d_word, p->d_value,
                       p->d_chunk_base, p->d_chunk_len, int32_t(p->chunks), bb, x, err, lim, async_ticket(p, 0),
                       p->d_aalive, p->d_vnext, dev::kRobTicks, p->delay_ticks);
    HIP_TRY(hipGetLastError());
    p->last_stream = st;
    return GLTRSV_OK;
}

int gltrsv_solve_multi(gltrsv_plan *p, const double *b, double *x, int32_t nrhs, void *stream)
{
    if (!p || nrhs < 1 || (p->n && (!b || !x))) return set_error(GLTRSV_EINVAL, "bad argument");
    if (p->n == 0) return GLTRSV_OK;
    const int64_t total = p->n * int64_t(nrhs);
    if (overlap(b, sizeof(double) * size_t(total), x, sizeof(double) * size_t(total)))
        return set_error(GLTRSV_EINVAL, "B and X must not overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t fill_blocks = std::min<int64_t>(4096, (total + dev::kBlock - 1) / dev::kBlock);
    hipLaunchKernelGGL(dev::fill_unready, dim3(unsigned(fill_blocks)), dim3(dev::kBlock), 0, st,
                       reinterpret_cast<unsigned long long *>(x), total);
    const int32_t chunks = int32_t(p->chunks);
    const unsigned grid = unsigned(std::min<int64_t>(int64_t(p->grid_async) * dev::kWavesPerBlock, chunks));
    const int64_t ld = nrhs;
    unsigned long long *tk = async_ticket(p, 1);
    uint32_t *al = p->d_aalive + dev::kMaxGrid;
    unsigned long long *vn = p->d_vnext + dev::kMaxGrid * dev::kWavesPerBlock;
    for (int32_t r0 = 0; r0 < nrhs;) {
        const int32_t R = nrhs - r0 >= 4 ? 4 : (nrhs - r0 >= 2 ? 2 : 1);
        if (R == 4)
            hipLaunchKernelGGL(dev::trsv_async_multi<4>, dim3(grid), dim3(64), 0, st, p->d_word, p->d_value,
                               p->d_chunk_base, p->d_chunk_len, chunks, b + r0, x + r0, ld, p->d_err, p->spin_limit,
                               tk, al, vn, dev::kRobTicks, p->delay_ticks);
        else if (R == 2)
            hipLaunchKernelGGL(dev::trsv_async_multi<2>, dim3(grid), dim3(64), 0, st, p->d_word, p->d_value,
                               p->d_chunk_base, p->d_chunk_len, chunks, b + r0, x + r0, ld, p->d_err, p->spin_limit,
                               tk, al, vn, dev::kRobTicks, p->delay_ticks);
        else
            hipLaunchKernelGGL(dev::trsv_async_multi<1>, dim3(grid), dim3(64), 0, st, p->d_word, p->d_value,
                               p->d_chunk_base, p->d_chunk_len, chunks, b + r0, x + r0, ld, p->d_err, p->spin_limit,
                               tk, al, vn, dev::kRobTicks, p->delay_ticks);
        HIP_TRY(hipGetLastError());
        r0 += R;
    }
    p->last_stream = st;
    return GLTRSV_OK;
}

int gltrsv_copy_probe(const void *src, void *dst, int64_t bytes, void *stream)
{
    if (!src || !dst || bytes < 0 || (bytes % 16) != 0) return set_error(GLTRSV_EINVAL, "bad copy arguments");
    if (bytes == 0) return GLTRSV_OK;
    int cus = 0, dev_id = 0;
    HIP_TRY(hipGetDevice(&dev_id));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id));
    const int64_t n16 = bytes / 16;
    const int64_t blocks = std::min<int64_t>(int64_t(cus) * 8, (n16 + dev::kBlock - 1) / dev::kBlock);
    hipLaunchKernelGGL(dev::copy_probe, dim3(unsigned(blocks)), dim3(dev::kBlock), 0, static_cast<hipStream_t>(stream),
                       static_cast<const double2 *>(src), static_cast<double2 *>(dst), n16);
    HIP_TRY(hipGetLastError());
    return GLTRSV_OK;
}

int gltrsv_plan_stream(const gltrsv_plan *p, uint32_t *word, double *value, int64_t slots)
{
    if (!p || (p->slots && (!word || !value))) return set_error(GLTRSV_EINVAL, "null argument");
    if (slots != p->slots) return set_error(GLTRSV_EINVAL, "slots must equal the plan's stream_slots");
    if (slots == 0) return GLTRSV_OK;
    HIP_TRY(hipSetDevice(p->device));
    HIP_TRY(hipMemcpy(word, p->d_word, sizeof(uint32_t) * size_t(slots), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(value, p->d_value, sizeof(double) * size_t(slots), hipMemcpyDeviceToHost));
    return GLTRSV_OK;
}

int gltrsv_plan_gather_probe(gltrsv_plan *p, const double *x, double *y, void *stream)
{
    if (!p || (p->n && (!x || !y))) return set_error(GLTRSV_EINVAL, "null argument");
    if (p->chunks == 0) return GLTRSV_OK;
    HIP_TRY(hipSetDevice(p->device));
    const int64_t blocks = (p->chunks + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock;
    hipLaunchKernelGGL(dev::gather_probe, dim3(unsigned(blocks)), dim3(dev::kBlock), 0,
                       static_cast<hipStream_t>(stream), p->d_word, p->d_value, p->d_chunk_base, p->d_chunk_len,
                       p->chunks, x, y);
    HIP_TRY(hipGetLastError());
    return GLTRSV_OK;
}

// Trace builds only: copies S * grid * 3 timestamps (wall clock ticks) of the
// last persistent solve: start of work, end of work, end of barrier.
int gltrsv_debug_trace(gltrsv_plan *p, int64_t *out, int64_t count)
{
    if (!p || !out) return set_error(GLTRSV_EINVAL, "null argument");
    if (!p->d_trace) return set_error(GLTRSV_ENOTSUP, "not a trace build");
    const int64_t have = int64_t(p->S) * p->grid * 3;
    HIP_TRY(hipStreamSynchronize(p->last_stream));
    HIP_TRY(hipMemcpy(out, p->d_trace, sizeof(int64_t) * std::min(count, have), hipMemcpyDeviceToHost));
    return GLTRSV_OK;
}

int gltrsv_plan_device_status(gltrsv_plan *p, int32_t *status)
{
    if (!p || !status) return set_error(GLTRSV_EINVAL, "null argument");
    HIP_TRY(hipStreamSynchronize(p->last_stream));
    int32_t e = 0;
    HIP_TRY(hipMemcpy(&e, p->d_err, sizeof(int32_t), hipMemcpyDeviceToHost));
    *status = e;
    if (e) {
        // a solve stopped part way: clear its partial counts for the next
        // one (the start ticket keeps counting, so epochs stay unique)
        HIP_TRY(hipMemset(p->d_bar, 0, dev::kBarStart * sizeof(uint32_t)));
        HIP_TRY(hipMemset(p->d_err, 0, sizeof(int32_t)));
    }
    return GLTRSV_OK;
}

int gltrsv_plan_set_spin_limit(gltrsv_plan *p, int64_t polls)
{
    if (!p || polls < 1) return set_error(GLTRSV_EINVAL, "polls must be >= 1");
    p->spin_limit = polls;
    return GLTRSV_OK;
}

int gltrsv_plan_set_steal_wait(gltrsv_plan *p, int64_t microseconds)
{
    if (!p || microseconds < 0 || microseconds > (int64_t(1) << 40))
        return set_error(GLTRSV_EINVAL, "microseconds must be in 0..2^40");
    p->steal_ticks = microseconds * 100;   // the device wall clock runs at 100 MHz
    return GLTRSV_OK;
}

int gltrsv_plan_set_start_delay(gltrsv_plan *p, int64_t microseconds)
{
    if (!p || microseconds < 0 || microseconds > 10000000)
        return set_error(GLTRSV_EINVAL, "microseconds must be in 0..1e7");
    p->delay_ticks = microseconds * 100;
    return GLTRSV_OK;
}

int gltrsv_solve_unordered(gltrsv_plan *p, const double *b, double *x, void *stream)
{
    if (!p || (p->n && (!b || !x))) return set_error(GLTRSV_EINVAL, "null argument");
    if (p->n && !p->d_csr_rp) return set_error(GLTRSV_ENOTSUP, "plan was created with reorder = 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int32_t s = 0; s < p->S; s++) {
        const int32_t t0 = p->super_task_host[size_t(s)], t1 = p->super_task_host[size_t(s) + 1];
        const int32_t blocks = (t1 - t0 + dev::kBlock - 1) / dev::kBlock;
        if (blocks == 0) continue;
        hipLaunchKernelGGL(dev::trsv_superstep_unordered, dim3(blocks), dim3(dev::kBlock), 0, st, p->d_csr_rp,
                           p->d_csr_col, p->d_csr_val, p->d_urows, p->d_utask_off, t0, t1, p->upper ? 1 : 0, b, x);
    }
    HIP_TRY(hipGetLastError());
    p->last_stream = st;
    return GLTRSV_OK;
}

int gltrsv_solve_auto(gltrsv_plan *p, const double *b, double *x, void *stream)
{
    if (!p) return set_error(GLTRSV_EINVAL, "null plan");
    switch (p->exec_form) {
    case GLTRSV_EXEC_PLAIN: return gltrsv_solve_plain(p, b, x, stream);
    case GLTRSV_EXEC_ASYNC: return gltrsv_solve_async(p, b, x, stream);
    case GLTRSV_EXEC_LOCAL: return gltrsv_solve_local(p, b, x, stream);
    default: return gltrsv_solve(p, b, x, stream);
    }
}

int gltrsv_plan_set_exec(gltrsv_plan *p, int32_t form)
{
    if (!p) return set_error(GLTRSV_EINVAL, "null plan");
    if (form < 0 || form >= GLTRSV_EXEC_FORMS) return set_error(GLTRSV_EINVAL, "unknown execution form");
    if (form == GLTRSV_EXEC_LOCAL && !p->d_lrec)
        return set_error(GLTRSV_ENOTSUP, "the plan has no one-workgroup layout (create it with exec_hint 2)");
    p->exec_form = form;
    return GLTRSV_OK;
}

namespace {
// Event pair released on every return path.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};
}  // namespace

int gltrsv_plan_tune(gltrsv_plan *p, const double *b, double *x, int32_t reps, void *stream, double *us_out,
                     int32_t *best)
{
    if (!p || reps < 1) return set_error(GLTRSV_EINVAL, "null plan or reps < 1");
    if (p->n && (!b || !x)) return set_error(GLTRSV_EINVAL, "null argument");
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(b), x0 = reinterpret_cast<uintptr_t>(x);
    const uintptr_t len = uintptr_t(p->n) * sizeof(double);
    if (p->n && b0 < x0 + len && x0 < b0 + len) return set_error(GLTRSV_EINVAL, "b and x overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    using SolveFn = int (*)(gltrsv_plan *, const double *, double *, void *);
    const SolveFn forms[GLTRSV_EXEC_FORMS] = {gltrsv_solve, gltrsv_solve_plain, gltrsv_solve_async, gltrsv_solve_local};
    double us[GLTRSV_EXEC_FORMS] = {0.0, 0.0, 0.0, -1.0};
    const int nforms = p->d_lrec ? GLTRSV_EXEC_FORMS : GLTRSV_EXEC_FORMS - 1;
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    for (int f = 0; f < nforms; f++) {
        int rc = forms[f](p, b, x, stream);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(ev.a, st));
        for (int32_t r = 0; r < reps && rc == 0; r++) rc = forms[f](p, b, x, stream);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(ev.b, st));
        HIP_TRY(hipEventSynchronize(ev.b));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
        us[f] = 1000.0 * double(ms) / reps;
    }
    int32_t status = 0;
    int rc = gltrsv_plan_device_status(p, &status);
    if (rc) return rc;
    if (status) return set_error(GLTRSV_ETIMEDOUT, "a device-side wait ran out during tuning");
    int32_t f_best = 0;
    for (int32_t f = 1; f < nforms; f++)
        if (us[f] < us[f_best]) f_best = f;
    p->exec_form = f_best;
    if (us_out)
        for (int f = 0; f < GLTRSV_EXEC_FORMS; f++) us_out[f] = us[f];
    if (best) *best = f_best;
    return GLTRSV_OK;
}

void gltrsv_default_batch_opts(gltrsv_batch_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->per_claim = 1;
    o->grid_blocks = 0;
    o->use_graph = 1;
}

int gltrsv_batch_destroy(gltrsv_batch *bt)
{
    if (!bt) return GLTRSV_OK;
    if (bt->graph_exec) (void)hipGraphExecDestroy(bt->graph_exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    for (int k = 0; k < 2; k++) {
        if (bt->staged[k]) (void)hipEventDestroy(bt->staged[k]);
        if (bt->h_desc[k]) (void)hipHostFree(bt->h_desc[k]);
    }
    (void)hipFree(bt->d_desc);
    (void)hipFree(bt->d_state);
    (void)hipFree(bt->d_done);
    (void)hipFree(bt->d_finished);
    (void)hipFree(bt->d_err);
    (void)hipFree(bt->d_bscol);
    (void)hipFree(bt->d_bsval);
    (void)hipFree(bt->d_bbeg);
    (void)hipFree(bt->d_btask);
    (void)hipFree(bt->d_boff);
    (void)hipFree(bt->d_bcat);
    (void)hipFree(bt->d_xcat);
    (void)hipFree(bt->d_wticket);
    (void)hipFree(bt->d_walive);
    (void)hipFree(bt->d_wvnext);
    delete bt;
    return GLTRSV_OK;
}

int gltrsv_batch_create(gltrsv_plan *const *plans, int32_t count, const gltrsv_batch_opts *opts,
                        gltrsv_batch **out)
{
    if (!plans || !out || count < 0) return set_error(GLTRSV_EINVAL, "bad batch arguments");
    *out = nullptr;
    gltrsv_batch_opts dflt;
    gltrsv_default_batch_opts(&dflt);
    if (!opts) opts = &dflt;
    if (opts->per_claim < 1 || opts->grid_blocks < 0 || (opts->async_exec != 0 && opts->async_exec != 1))
        return set_error(GLTRSV_EINVAL, "bad batch options");
    int dev_id = 0;
    HIP_TRY(hipGetDevice(&dev_id));
    gltrsv_batch *bt = new (std::nothrow) gltrsv_batch();
    if (!bt) return set_error(GLTRSV_ENOMEM, "host allocation");
    bt->device = dev_id;
    bt->ncalls = count;
    bt->per_claim = opts->per_claim;
    bt->async_exec = opts->async_exec != 0;
    bt->use_graph = opts->use_graph != 0;
    for (int32_t i = 0; i < count; i++) {
        if (!plans[i]) {
            gltrsv_batch_destroy(bt);
            return set_error(GLTRSV_EINVAL, "null plan in batch");
        }
        if (plans[i]->device != dev_id) {
            gltrsv_batch_destroy(bt);
            return set_error(GLTRSV_EINVAL, "plans of a batch must live on the current device");
        }
        if (plans[i]->n == 0) continue;
        bt->plans.push_back(plans[i]);
        bt->slot.push_back(i);
        bt->ndone += plans[i]->S;
    }
    bt->count = int32_t(bt->plans.size());
    bt->wave = bt->async_exec && bt->count > 0;
    for (auto *pl : bt->plans) bt->wave = bt->wave && pl->core_width == 64;
    int64_t all_rows = 0, all_off = 0;
    for (auto *pl : bt->plans) {
        all_rows += pl->n;
        all_off += pl->nnz - pl->n;
    }
    bt->row_dpp = all_rows > 0 && all_off >= dev::kDppMinPerRow * all_rows;
    const size_t ndesc = std::max<size_t>(1, bt->plans.size());
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&bt->d_desc), ndesc * sizeof(dev::SysDesc));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&bt->d_state), ndesc * dev::kStateStride * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&bt->d_done), std::max(1, bt->ndone) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&bt->d_finished), 2 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&bt->d_err), sizeof(int32_t));
    for (int k = 0; k < 2 && e == hipSuccess; k++) {
        e = hipHostMalloc(reinterpret_cast<void **>(&bt->h_desc[k]), ndesc * sizeof(dev::SysDesc), hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->staged[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        gltrsv_batch_destroy(bt);
        return set_error(e == hipErrorOutOfMemory ? GLTRSV_ENOMEM : GLTRSV_EHIP,
                         std::string("batch allocation: ") + hipGetErrorString(e));
    }
    int32_t off = 0;
    for (int k = 0; k < 2; k++) {
        off = 0;
        for (int32_t i = 0; i < bt->count; i++) {
            const gltrsv_plan *pl = bt->plans[i];
            dev::SysDesc &d = bt->h_desc[k][i];
            d.word = pl->d_word;
            d.value = pl->d_value;
            d.chunk_base = pl->d_chunk_base;
            d.chunk_len = pl->d_chunk_len;
            d.super_chunk = pl->d_super_chunk;
            d.b = nullptr;
            d.x = nullptr;
            d.S = pl->S;
            d.done_off = off;
            d.nchunks = int32_t(pl->chunks);
            d.window = dev::async_window(pl->chunks, pl->S);
            d.n = pl->n;
            d.wrow = pl->d_wrow;
            d.wptr = pl->d_wptr;
            d.wdiag = pl->d_wdiag;
            d.wcol = pl->d_wcol;
            d.wval = pl->d_wval;
            d.wtask = pl->d_wtask;
            d.ntasks = pl->wsuper_host.empty() ? 0 : pl->wsuper_host.back();
            if (bt->wave) d.window = dev::async_window(d.ntasks, pl->S);
            off += pl->S;
        }
    }
    int per_cu = 0, cus = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu,
        bt->wave ? (bt->row_dpp ? reinterpret_cast<const void *>(dev::trsv_stream_async<true>)
                                   : reinterpret_cast<const void *>(dev::trsv_stream_async<false>))
                 : reinterpret_cast<const void *>(dev::trsv_batched),
        dev::kBlock, 0);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id);
    if (e != hipSuccess) {
        gltrsv_batch_destroy(bt);
        return set_error(GLTRSV_EHIP, std::string("occupancy query: ") + hipGetErrorString(e));
    }
    if (bt->wave) per_cu = std::min(per_cu, dev::kStreamWgPerCu);   // (see kStreamSgprs)
    int64_t chunks = 0;   // wave units of work: chunks, or tasks on wavefront cores
    for (auto *pl : bt->plans) chunks += bt->wave ? (pl->wsuper_host.empty() ? 0 : pl->wsuper_host.back()) : pl->chunks;
    if (bt->wave) {
        // global task order: the supersteps of all systems by relative depth
        // (s + 1/2) / S, so a system with many supersteps advances from the
        // start alongside the short ones instead of running alone at the
        // end; each system's own order is kept
        std::vector<std::pair<double, std::pair<int32_t, int32_t>>> steps;   // (depth, (system, superstep))
        for (int32_t i = 0; i < bt->count; i++) {
            const gltrsv_plan *pl = bt->plans[size_t(i)];
            for (int32_t s = 0; s < pl->S; s++) steps.push_back({(s + 0.5) / pl->S, {i, s}});
        }
        std::stable_sort(steps.begin(), steps.end(),
                         [](const std::pair<double, std::pair<int32_t, int32_t>> &a,
                            const std::pair<double, std::pair<int32_t, int32_t>> &b) { return a.first < b.first; });
        std::vector<int32_t> gsys, gtask;
        gsys.reserve(size_t(chunks));
        gtask.reserve(size_t(chunks));
        for (const auto &st : steps) {
            const int32_t i = st.second.first, s = st.second.second;
            const gltrsv_plan *pl = bt->plans[size_t(i)];
            for (int32_t t = pl->wsuper_host[size_t(s)]; t < pl->wsuper_host[size_t(s) + 1]; t++) {
                gsys.push_back(i);
                gtask.push_back(t);
            }
        }
        bt->gtasks = int64_t(gsys.size());
        if (int rc = batch_stream(bt, gsys, gtask, per_cu * cus, opts->grid_blocks)) {
            gltrsv_batch_destroy(bt);
            return rc;
        }
    }
    int grid = std::max(1, per_cu * cus);
    if (opts->grid_blocks > 0) grid = std::min(grid, opts->grid_blocks);
    grid = int(std::max<int64_t>(1, std::min<int64_t>(grid, (chunks + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock)));
    if (!bt->wave) bt->grid = grid;   // (wave cores: the grid the batch stream was built for)
    bt->keep_waves = dev::keep_waves_for(widest_of(bt->plans), bt->per_claim, grid);
    *out = bt;
    return GLTRSV_OK;
}

// The vectors of a batched solve: no null pointer; system i's x shares no
// byte with any other system's b or x; b[i] may equal x[i] (BSP execution
// only) but not overlap it partly.  Sorting the ranges keeps this
// O(count log count).
static int check_batch_vectors(const gltrsv_batch *bt, const double *const *b, double *const *x)
{
    struct Range {
        uintptr_t lo, hi;
        int32_t sys;
        bool is_x;
    };
    std::vector<Range> r;
    r.reserve(size_t(bt->count) * 2);
    for (int32_t i = 0; i < bt->count; i++) {
        const int32_t j = bt->slot[i];
        if (!b[j] || !x[j]) return set_error(GLTRSV_EINVAL, "null vector in batch");
        const uintptr_t len = uintptr_t(bt->plans[size_t(i)]->n) * sizeof(double);
        const uintptr_t pb = reinterpret_cast<uintptr_t>(b[j]), px = reinterpret_cast<uintptr_t>(x[j]);
        if (pb == px) {
            if (bt->async_exec) return set_error(GLTRSV_EINVAL, "semi-asynchronous batches need b and x apart");
            r.push_back({px, px + len, i, true});   // one range serves as both
        } else {
            r.push_back({pb, pb + len, i, false});
            r.push_back({px, px + len, i, true});
        }
    }
    std::sort(r.begin(), r.end(), [](const Range &a, const Range &c) { return a.lo < c.lo; });
    // any two overlapping ranges overlap a neighbour in this order, unless
    // both are b ranges (read-only, sharing is fine); track the x range that
    // reaches furthest and the furthest range of any kind
    uintptr_t far_any = 0, far_x = 0;
    bool any = false, anyx = false;
    for (const Range &q : r) {
        if (anyx && q.lo < far_x) return set_error(GLTRSV_EINVAL, "a batch's x overlaps another vector");
        if (q.is_x && any && q.lo < far_any)
            return set_error(GLTRSV_EINVAL, "a batch's x overlaps another vector");
        far_any = any ? std::max(far_any, q.hi) : q.hi;
        any = true;
        if (q.is_x) {
            far_x = anyx ? std::max(far_x, q.hi) : q.hi;
            anyx = true;
        }
    }
    return GLTRSV_OK;
}

static int batch_enqueue(gltrsv_batch *bt, hipStream_t st)
{
    if (bt->async_exec) {
        int64_t widest_n = 1;
        for (auto *pl : bt->plans) widest_n = std::max(widest_n, pl->n);
        const unsigned gx = unsigned(std::min<int64_t>(256, (widest_n + dev::kBlock - 1) / dev::kBlock));
        hipLaunchKernelGGL(dev::batch_reset, dim3(unsigned(std::max(1, (bt->count + dev::kBlock - 1) / dev::kBlock))),
                           dim3(dev::kBlock), 0, st, bt->d_state, bt->d_done, bt->count, 0, bt->d_finished,
                           bt->d_err);
        if (bt->wave) {
            // the batch as one system over the global task order (static;
            // waves that wait long rob workgroups that have not started, so
            // no co-residency is needed)
            const unsigned cx = gx;
            hipLaunchKernelGGL(dev::batch_concat, dim3(cx, unsigned(bt->count)), dim3(dev::kBlock), 0, st, bt->d_desc,
                               bt->d_boff, bt->d_bcat, true);
            const int64_t fb = std::min<int64_t>(4096, (bt->rows + dev::kBlock - 1) / dev::kBlock);
            hipLaunchKernelGGL(dev::fill_unready, dim3(unsigned(std::max<int64_t>(1, fb))), dim3(dev::kBlock), 0, st,
                               reinterpret_cast<unsigned long long *>(bt->d_xcat), bt->rows);
            hipLaunchKernelGGL(bt->row_dpp ? dev::trsv_stream_async<true> : dev::trsv_stream_async<false>,
                               dim3(unsigned(bt->grid)), dim3(dev::kBlock), 0, st,
                               bt->d_bscol, bt->d_bsval, bt->d_bbeg, bt->d_btask, int32_t(bt->gtasks), bt->d_bcat,
                               bt->d_xcat, bt->d_err, int64_t(5000000), bt->d_wticket, bt->d_walive, bt->d_wvnext,
                               dev::kRobTicks, int64_t(0));
            hipLaunchKernelGGL(dev::batch_concat, dim3(cx, unsigned(bt->count)), dim3(dev::kBlock), 0, st, bt->d_desc,
                               bt->d_boff, bt->d_xcat, false);
            HIP_TRY(hipGetLastError());
            return GLTRSV_OK;
        }
        hipLaunchKernelGGL(dev::fill_unready_sys, dim3(gx, unsigned(bt->count)), dim3(dev::kBlock), 0, st, bt->d_desc,
                           bt->count);
        hipLaunchKernelGGL(dev::trsv_batched_async, dim3(unsigned(bt->grid)), dim3(dev::kBlock), 0, st, bt->d_desc,
                           bt->count, bt->d_state, bt->d_finished, bt->d_err, int64_t(5000000), bt->per_claim,
                           int64_t(0));
        HIP_TRY(hipGetLastError());
        return GLTRSV_OK;
    }
    hipLaunchKernelGGL(dev::batch_reset, dim3(unsigned(std::max(1, (bt->count + dev::kBlock - 1) / dev::kBlock))),
                       dim3(dev::kBlock), 0, st, bt->d_state, bt->d_done, bt->count, bt->ndone, bt->d_finished,
                       bt->d_err);
    hipLaunchKernelGGL(dev::trsv_batched, dim3(unsigned(bt->grid)), dim3(dev::kBlock), 0, st, bt->d_desc, bt->count,
                       bt->d_state, bt->d_done, bt->d_finished, bt->d_err, bt->idle_ticks, bt->per_claim, bt->count,
                       int64_t(0), bt->keep_waves);
    HIP_TRY(hipGetLastError());
    return GLTRSV_OK;
}

int gltrsv_batch_solve(gltrsv_batch *bt, const double *const *b, double *const *x, void *stream)
{
    if (!bt || (bt->ncalls && (!b || !x))) return set_error(GLTRSV_EINVAL, "null argument");
    if (bt->count == 0) return GLTRSV_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int k = bt->flip;
    bt->flip ^= 1;
    // the copy issued from this staging buffer two calls ago has finished
    HIP_TRY(hipEventSynchronize(bt->staged[k]));
    if (int rc = check_batch_vectors(bt, b, x)) return rc;
    for (int32_t i = 0; i < bt->count; i++) {
        const int32_t j = bt->slot[i];
        bt->h_desc[k][i].b = b[j];
        bt->h_desc[k][i].x = x[j];
    }
    HIP_TRY(hipMemcpyAsync(bt->d_desc, bt->h_desc[k], sizeof(dev::SysDesc) * bt->count, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(bt->staged[k], st));
    if (bt->use_graph && st != nullptr) {   // the null stream cannot be captured
        if (!bt->graph_exec || bt->graph_stream != st) {
            if (bt->graph_exec) {
                HIP_TRY(hipGraphExecDestroy(bt->graph_exec));
                bt->graph_exec = nullptr;
            }
            if (bt->graph) {
                HIP_TRY(hipGraphDestroy(bt->graph));
                bt->graph = nullptr;
            }
            HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            const int rc = batch_enqueue(bt, st);
            hipGraph_t g = nullptr;
            const hipError_t ce = hipStreamEndCapture(st, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (ce != hipSuccess) return set_error(GLTRSV_EHIP, std::string("graph capture: ") + hipGetErrorString(ce));
            bt->graph = g;
            HIP_TRY(hipGraphInstantiate(&bt->graph_exec, bt->graph, nullptr, nullptr, 0));
            bt->graph_stream = st;
        }
        HIP_TRY(hipGraphLaunch(bt->graph_exec, st));
    } else {
        const int rc = batch_enqueue(bt, st);
        if (rc) return rc;
    }
    bt->last_stream = st;
    return GLTRSV_OK;
}

int gltrsv_batch_status(gltrsv_batch *bt, int32_t *status)
{
    if (!bt || !status) return set_error(GLTRSV_EINVAL, "null argument");
    HIP_TRY(hipStreamSynchronize(bt->last_stream));
    int32_t e = 0;
    HIP_TRY(hipMemcpy(&e, bt->d_err, sizeof(int32_t), hipMemcpyDeviceToHost));
    *status = e;
    return GLTRSV_OK;
}

int gltrsv_batch_info(const gltrsv_batch *bt, int32_t *systems, int32_t *grid_blocks)
{
    if (!bt) return set_error(GLTRSV_EINVAL, "null batch");
    if (systems) *systems = bt->count;
    if (grid_blocks) *grid_blocks = bt->grid;
    return GLTRSV_OK;
}

int gltrsv_solve_batched(gltrsv_plan *const *plans, const double *const *b, double *const *x, int32_t count,
                         void *stream)
{
    gltrsv_batch_opts o;
    gltrsv_default_batch_opts(&o);
    o.use_graph = 0;
    gltrsv_batch *bt = nullptr;
    int rc = gltrsv_batch_create(plans, count, &o, &bt);
    if (rc) return rc;
    rc = gltrsv_batch_solve(bt, b, x, stream);
    if (rc == GLTRSV_OK) {
        const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (e != hipSuccess) rc = set_error(GLTRSV_EHIP, std::string("batched solve: ") + hipGetErrorString(e));
    }
    int32_t status = 0;
    if (rc == GLTRSV_OK && (rc = gltrsv_batch_status(bt, &status)) == GLTRSV_OK && status)
        rc = set_error(GLTRSV_ETIMEDOUT, "batched solve: a wave found no work for longer than the idle limit");
    gltrsv_batch_destroy(bt);
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched solve without allocation (gltrsv_solve_batched_noalloc): the device
// state of gltrsv_solve_batched -- system descriptors, superstep state words,
// per-superstep done counters, the finished and error words -- lives in one
// fixed file-scope device array instead of buffers the library allocates.
// Host code never uses the array's name as an address: the address is taken
// once per device with hipGetSymbolAddress and kept.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr int32_t kScratchSystems = 1024;   // descriptors staged in host memory
constexpr int kScratchDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchSlot {
    std::mutex mu;                          // one call at a time per device
    unsigned char *ptr = nullptr;           // device address of `scratch`
    dev::SysDesc desc[kScratchSystems];     // host staging of the descriptors
};

std::mutex g_scratch_setup;
ScratchSlot g_scratch[kScratchDevices];

// The device's scratch slot; its address is looked up on the first call on
// that device (with the device current).
int scratch_slot(int device, ScratchSlot **out)
{
    if (device < 0 || device >= kScratchDevices)
        return set_error(GLTRSV_ENOTSUP, "device index beyond the no-allocation table");
    ScratchSlot &sl = g_scratch[device];
    std::lock_guard<std::mutex> g(g_scratch_setup);
    if (!sl.ptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(GLTRSV_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        sl.ptr = static_cast<unsigned char *>(p);
    }
    *out = &sl;
    return GLTRSV_OK;
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// The rule of check_batch_vectors for BSP batches, pairwise, without
// allocating: x of one system shares no byte with another system's b or x,
// and b may equal x but not overlap it partly.
int check_vectors_noalloc(gltrsv_plan *const *plans, const double *const *b, double *const *x, int32_t count)
{
    for (int32_t i = 0; i < count; i++) {
        if (!plans[i] || plans[i]->n == 0) continue;
        const size_t li = sizeof(double) * size_t(plans[i]->n);
        if (!b[i] || !x[i]) return set_error(GLTRSV_EINVAL, "null vector in batch");
        if (b[i] != x[i] && overlap(b[i], li, x[i], li))
            return set_error(GLTRSV_EINVAL, "b and x of a system overlap without being equal");
        for (int32_t j = 0; j < count; j++) {
            if (j == i || !plans[j] || plans[j]->n == 0 || !b[j] || !x[j]) continue;
            const size_t lj = sizeof(double) * size_t(plans[j]->n);
            if (overlap(x[i], li, b[j], lj) || overlap(x[i], li, x[j], lj))
                return set_error(GLTRSV_EINVAL, "a batch's x overlaps another vector");
        }
    }
    return GLTRSV_OK;
}

}  // namespace

extern "C" {

int gltrsv_solve_batched_noalloc(gltrsv_plan *const *plans, const double *const *b, double *const *x, int32_t count,
                                 void *stream)
{
    if (!plans || count < 0 || (count > 0 && (!b || !x))) return set_error(GLTRSV_EINVAL, "bad batch arguments");
    int dev_id = 0;
    HIP_TRY(hipGetDevice(&dev_id));
    int32_t systems = 0, ndone = 0;
    int64_t chunks = 0, widest = 0;
    for (int32_t i = 0; i < count; i++) {
        if (!plans[i]) return set_error(GLTRSV_EINVAL, "null plan in batch");
        if (plans[i]->device != dev_id) return set_error(GLTRSV_EINVAL, "plans of a batch must live on the current device");
        if (plans[i]->n == 0) continue;
        systems++;
        if (int64_t(ndone) + plans[i]->S > INT32_MAX) return set_error(GLTRSV_ERANGE, "too many supersteps");
        ndone += plans[i]->S;
        chunks += plans[i]->chunks;
        widest = std::max(widest, plans[i]->widest);
    }
    if (int rc = check_vectors_noalloc(plans, b, x, count)) return rc;
    if (systems == 0) return GLTRSV_OK;
    // scratch layout: descriptors | state words | done counters | finished[2] | error word
    const size_t off_state = round_up(sizeof(dev::SysDesc) * size_t(systems), 256);
    const size_t off_done = off_state + round_up(sizeof(unsigned long long) * dev::kStateStride * size_t(systems), 256);
    const size_t off_fin = off_done + round_up(sizeof(uint32_t) * size_t(ndone), 256);
    const size_t off_err = off_fin + 256;
    const size_t need = off_err + 256;
    if (systems > kScratchSystems || need > kScratchBytes)
        return set_error(GLTRSV_ERANGE, "batch too large for the no-allocation scratch (" + std::to_string(systems) +
                                            " systems, " + std::to_string(need) + " bytes; at most " +
                                            std::to_string(kScratchSystems) + " systems and " +
                                            std::to_string(kScratchBytes) + " bytes)");
    ScratchSlot *sl = nullptr;
    if (int rc = scratch_slot(dev_id, &sl)) return rc;
    std::lock_guard<std::mutex> g(sl->mu);
    int per_cu = 0, cus = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dev::trsv_batched, dev::kBlock, 0));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id));
    int32_t off = 0, k = 0;
    for (int32_t i = 0; i < count; i++) {
        const gltrsv_plan *pl = plans[i];
        if (pl->n == 0) continue;
        dev::SysDesc &d = sl->desc[k++];
        std::memset(&d, 0, sizeof(d));
        d.word = pl->d_word;
        d.value = pl->d_value;
        d.chunk_base = pl->d_chunk_base;
        d.chunk_len = pl->d_chunk_len;
        d.super_chunk = pl->d_super_chunk;
        d.b = b[i];
        d.x = x[i];
        d.S = pl->S;
        d.done_off = off;
        d.nchunks = int32_t(pl->chunks);
        d.window = dev::async_window(pl->chunks, pl->S);
        d.n = pl->n;
        off += pl->S;
    }
    unsigned char *base = sl->ptr;
    auto *d_desc = reinterpret_cast<dev::SysDesc *>(base);
    auto *d_state = reinterpret_cast<unsigned long long *>(base + off_state);
    auto *d_done = reinterpret_cast<uint32_t *>(base + off_done);
    auto *d_fin = reinterpret_cast<uint32_t *>(base + off_fin);
    auto *d_err = reinterpret_cast<int32_t *>(base + off_err);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(d_desc, sl->desc, sizeof(dev::SysDesc) * size_t(systems), hipMemcpyHostToDevice, st));
    // the array keeps the previous call's contents: the reset kernel clears
    // the state words, the done counters and the finished and error words
    hipLaunchKernelGGL(dev::batch_reset, dim3(unsigned(std::max(1, (systems + dev::kBlock - 1) / dev::kBlock))),
                       dim3(dev::kBlock), 0, st, d_state, d_done, systems, ndone, d_fin, d_err);
    int grid = std::max(1, per_cu * cus);
    grid = int(std::max<int64_t>(1, std::min<int64_t>(grid, (chunks + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock)));
    const int32_t keep = dev::keep_waves_for(widest, 1, grid);
    hipLaunchKernelGGL(dev::trsv_batched, dim3(unsigned(grid)), dim3(dev::kBlock), 0, st, d_desc, systems, d_state,
                       d_done, d_fin, d_err, int64_t(1000000000), int32_t(1), systems, int64_t(0), keep);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    int32_t e = 0;
    HIP_TRY(hipMemcpy(&e, d_err, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (e) return set_error(GLTRSV_ETIMEDOUT, "batched solve: a wave found no work for longer than the idle limit");
    return GLTRSV_OK;
}

}  // extern "C"
