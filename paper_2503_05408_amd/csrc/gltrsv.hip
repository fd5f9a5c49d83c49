// gltrsv: GrowLocal-scheduled sparse lower-triangular solve for gfx950.
//
// Device side: every BSP core of the schedule (Definition 2.1) is one lane
// of a 64-wide wavefront.  A lane walks the rows of its (superstep, core)
// task in the order of Sec. 5, each row as the forward substitution of
// Eq. (2.1): acc <- b_i, acc <- acc - A_ij * x_j over the stored
// off-diagonals (no fused multiply-add), x_i <- acc / A_ii.  Tasks of one
// superstep never read each other's results (Def. 2.1), so the only
// synchronisation is the barrier between supersteps: the kernel boundary in
// the plain form, a device-scope counter in the persistent form.
//
// Host side: the C ABI of include/gltrsv.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gltrsv.h"
#include "analysis.h"

#pragma clang fp contract(off)

namespace gltrsv {
namespace dev {

constexpr uint32_t HDR = 0x80000000u;
constexpr uint32_t INTL = 0x40000000u;
constexpr uint32_t MASK = 0x3FFFFFFFu;
constexpr uint32_t PAD = 0xFFFFFFFFu;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kUnroll = 8;
constexpr int kGenOffset = 32;   // the generation word sits 128 B after the count

// One lane processes the packed entries of its task: words at
// word[base + 64 t + lane], t < len.
__device__ __forceinline__ void run_lane(const uint32_t *__restrict__ word, const double *__restrict__ value,
                                         int64_t base, int32_t len, int lane, const double *b, double *x)
{
    double acc = 0.0, diag = 1.0, last_y = 0.0;
    int32_t cur = -1, last = -1;
    const uint32_t *wp = word + base + lane;
    const double *vp = value + base + lane;
    for (int32_t t0 = 0; t0 < len; t0 += kUnroll) {
        uint32_t w[kUnroll];
        double v[kUnroll], g[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; j++) {
            if (t0 + j < len) {
                w[j] = __builtin_nontemporal_load(wp + int64_t(t0 + j) * 64);
                v[j] = __builtin_nontemporal_load(vp + int64_t(t0 + j) * 64);
            } else {
                w[j] = PAD;
                v[j] = 0.0;
            }
        }
        // operands that are final before this superstep: columns of earlier
        // supersteps and the right-hand side of each new row
#pragma unroll
        for (int j = 0; j < kUnroll; j++) {
            const uint32_t c = w[j];
            if ((c & (HDR | INTL)) == 0) g[j] = x[c];
            else if ((c & HDR) && c != PAD) g[j] = b[c & MASK];
            else g[j] = 0.0;
        }
#pragma unroll
        for (int j = 0; j < kUnroll; j++) {
            const uint32_t c = w[j];
            if (c & HDR) {
                if (cur >= 0) {
                    const double y = acc / diag;
                    x[cur] = y;
                    last = cur;
                    last_y = y;
                }
                if (c == PAD) {
                    cur = -1;
                } else {
                    cur = int32_t(c & MASK);
                    diag = v[j];
                    acc = g[j];
                }
            } else {
                double xv;
                if (c & INTL) {
                    // computed earlier on this lane in this superstep
                    const int32_t cc = int32_t(c & MASK);
                    xv = (cc == last) ? last_y : x[cc];
                } else {
                    xv = g[j];
                }
                const double prod = v[j] * xv;
                acc = acc - prod;
            }
        }
    }
    if (cur >= 0) x[cur] = acc / diag;
}

__global__ __launch_bounds__(kBlock) void trsv_superstep_plain(
    const uint32_t *__restrict__ word, const double *__restrict__ value, const int64_t *__restrict__ chunk_base,
    const int32_t *__restrict__ chunk_len, int32_t c0, int32_t c1, const double *b, double *x)
{
    const int32_t c = c0 + int32_t((blockIdx.x * kBlock + threadIdx.x) >> 6);
    if (c >= c1) return;
    run_lane(word, value, chunk_base[c], chunk_len[c], threadIdx.x & 63, b, x);
}

// Barrier over all workgroups of the grid.  bar[0] counts arrivals,
// bar[kGenOffset] is a generation number; the last arrival resets the count
// and advances the generation.  Returns false if the spin limit was hit or
// another workgroup reported an error; then the whole workgroup must exit.
__device__ __forceinline__ bool grid_barrier(uint32_t *bar, int32_t *err, int64_t spin_limit)
{
    __shared__ int32_t ok;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t *count = bar;
        uint32_t *gen = bar + kGenOffset;
        const uint32_t g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t old = __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int32_t good = 1;
        if (old == gridDim.x - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            int64_t it = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(1);
                if (++it > spin_limit) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
                if ((it & 1023) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    good = 0;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok = good;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok != 0;
}

__global__ __launch_bounds__(kBlock) void trsv_persistent(
    const uint32_t *__restrict__ word, const double *__restrict__ value, const int64_t *__restrict__ chunk_base,
    const int32_t *__restrict__ chunk_len, const int32_t *__restrict__ super_chunk, int32_t S, const double *b,
    double *x, uint32_t *bar, int32_t *err, int64_t spin_limit)
{
    const int32_t waves = int32_t(gridDim.x) * kWavesPerBlock;
    const int32_t wave = int32_t(blockIdx.x) * kWavesPerBlock + int32_t(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int32_t s = 0; s < S; s++) {
        const int32_t c1 = super_chunk[s + 1];
        for (int32_t c = super_chunk[s] + wave; c < c1; c += waves)
            run_lane(word, value, chunk_base[c], chunk_len[c], lane, b, x);
        if (s + 1 < S && !grid_barrier(bar, err, spin_limit)) return;
    }
}

}  // namespace dev
}  // namespace gltrsv

// ===========================================================================
// host runtime and C ABI
// ===========================================================================
using namespace gltrsv;

namespace {

thread_local std::string g_last_error = "no error";

int set_error(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return set_error(e_ == hipErrorOutOfMemory ? GLTRSV_ENOMEM : GLTRSV_EHIP,                   \
                             std::string(#expr) + ": " + hipGetErrorString(e_));                        \
    } while (0)

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
    if (o->schedule_kind != GLTRSV_SCHED_GROWLOCAL && o->schedule_kind != GLTRSV_SCHED_WAVEFRONT)
        return set_error(GLTRSV_EINVAL, "unknown schedule kind");
    if (o->schedule_kind == GLTRSV_SCHED_GROWLOCAL) {
        if (o->k < 1) return set_error(GLTRSV_EINVAL, "k must be >= 1");
        if (!(o->alpha0 >= 1.0)) return set_error(GLTRSV_EINVAL, "alpha0 must be >= 1");
        if (!(o->growth > 1.0)) return set_error(GLTRSV_EINVAL, "growth must be > 1");
        if (!(o->L >= 0.0)) return set_error(GLTRSV_EINVAL, "L must be >= 0");
        if (!(o->accept > 0.0)) return set_error(GLTRSV_EINVAL, "accept must be > 0");
    }
    if (o->block_size != 0 && o->block_size != dev::kBlock)
        return set_error(GLTRSV_ENOTSUP, "block_size must be 0 or 256 in this build");
    if (o->grid_blocks < 0) return set_error(GLTRSV_EINVAL, "grid_blocks must be >= 0");
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
    return p;
}

template <class T>
int upload(T **dst, const std::vector<T> &src, int64_t *bytes)
{
    const size_t nb = std::max<size_t>(1, src.size()) * sizeof(T);
    HIP_TRY(hipMalloc(reinterpret_cast<void **>(dst), nb));
    if (!src.empty()) HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    *bytes += int64_t(nb);
    return GLTRSV_OK;
}

}  // namespace

struct gltrsv_plan {
    int64_t n = 0, nnz = 0;
    int32_t S = 0, wavefronts = 0;
    int64_t tasks = 0, chunks = 0, slots = 0, max_task_rows = 0;
    int64_t analysis_ns = 0, device_bytes = 0;
    uint64_t key = 0;
    int device = 0;
    int grid = 0;
    std::vector<int32_t> core, superstep, perm, super_chunk_host;
    uint32_t *d_word = nullptr;
    double *d_value = nullptr;
    int64_t *d_chunk_base = nullptr;
    int32_t *d_chunk_len = nullptr;
    int32_t *d_super_chunk = nullptr;
    uint32_t *d_bar = nullptr;   // barrier words (256 B)
    int32_t *d_err = nullptr;
    hipStream_t last_stream = nullptr;
    int64_t spin_limit = 20000000;
};

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
    rc = check_csr(view_of(A), false, &msg);
    if (rc) return set_error(rc, msg);
    Schedule s = opts->schedule_kind == GLTRSV_SCHED_WAVEFRONT ? schedule_wavefront(view_of(A))
                                                               : schedule_growlocal(view_of(A), params_of(opts));
    if (A->n) {
        std::memcpy(core, s.core.data(), sizeof(int32_t) * A->n);
        std::memcpy(superstep, s.superstep.data(), sizeof(int32_t) * A->n);
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

int gltrsv_plan_destroy(gltrsv_plan *p)
{
    if (!p) return GLTRSV_OK;
    (void)hipFree(p->d_word);
    (void)hipFree(p->d_value);
    (void)hipFree(p->d_chunk_base);
    (void)hipFree(p->d_chunk_len);
    (void)hipFree(p->d_super_chunk);
    (void)hipFree(p->d_bar);
    (void)hipFree(p->d_err);
    delete p;
    return GLTRSV_OK;
}

int gltrsv_plan_create(const gltrsv_csr *A, const gltrsv_plan_opts *opts, gltrsv_plan **out)
{
    if (!A || !out) return set_error(GLTRSV_EINVAL, "null argument");
    *out = nullptr;
    int rc = check_opts(opts);
    if (rc) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    const CsrView V = view_of(A);
    std::string msg;
    rc = check_csr(V, true, &msg);
    if (rc) return set_error(rc, msg);

    gltrsv_plan *p = new (std::nothrow) gltrsv_plan();
    if (!p) return set_error(GLTRSV_ENOMEM, "host allocation");
    p->n = A->n;
    p->nnz = A->nnz;
    Schedule s = opts->schedule_kind == GLTRSV_SCHED_WAVEFRONT ? schedule_wavefront(V)
                                                               : schedule_growlocal(V, params_of(opts));
    std::vector<int32_t> lv;
    p->wavefronts = wavefront_levels(V, lv);
    p->perm = schedule_order(A->n, s.core.data(), s.superstep.data(), s.S);
    Packed pk = pack_stream(V, s, p->perm);
    p->S = s.S;
    p->core = std::move(s.core);
    p->superstep = std::move(s.superstep);
    p->tasks = pk.tasks;
    p->chunks = int64_t(pk.chunk_len.size());
    p->slots = int64_t(pk.word.size());
    p->max_task_rows = pk.max_task_rows;
    p->super_chunk_host = pk.super_chunk;
    p->key = pattern_key(V);

    HIP_TRY(hipGetDevice(&p->device));
    int64_t bytes = 0;
    if ((rc = upload(&p->d_word, pk.word, &bytes)) || (rc = upload(&p->d_value, pk.value, &bytes)) ||
        (rc = upload(&p->d_chunk_base, pk.chunk_base, &bytes)) || (rc = upload(&p->d_chunk_len, pk.chunk_len, &bytes)) ||
        (rc = upload(&p->d_super_chunk, pk.super_chunk, &bytes))) {
        gltrsv_plan_destroy(p);
        return rc;
    }
    {
        std::vector<uint32_t> bar(64, 0u);
        std::vector<int32_t> err(1, 0);
        if ((rc = upload(&p->d_bar, bar, &bytes)) || (rc = upload(&p->d_err, err, &bytes))) {
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
    int grid = per_cu * cus;
    if (opts->grid_blocks > 0) grid = std::min(grid, opts->grid_blocks);
    // no more workgroups than the widest superstep can use
    int64_t widest = 0;
    for (int32_t q = 0; q < p->S; q++)
        widest = std::max<int64_t>(widest, p->super_chunk_host[q + 1] - p->super_chunk_host[q]);
    const int64_t useful = (widest + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock;
    grid = int(std::max<int64_t>(1, std::min<int64_t>(grid, useful)));
    p->grid = grid;
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
    return GLTRSV_OK;
}

int gltrsv_plan_schedule(const gltrsv_plan *p, int32_t *core, int32_t *superstep, int32_t *perm)
{
    if (!p) return set_error(GLTRSV_EINVAL, "null plan");
    const size_t nb = sizeof(int32_t) * size_t(p->n);
    if (core && p->n) std::memcpy(core, p->core.data(), nb);
    if (superstep && p->n) std::memcpy(superstep, p->superstep.data(), nb);
    if (perm && p->n) std::memcpy(perm, p->perm.data(), nb);
    return GLTRSV_OK;
}

int gltrsv_solve_plain(gltrsv_plan *p, const double *b, double *x, void *stream)
{
    if (!p || (p->n && (!b || !x))) return set_error(GLTRSV_EINVAL, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
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
    const uint32_t *w = p->d_word;
    const double *v = p->d_value;
    const int64_t *cb = p->d_chunk_base;
    const int32_t *cl = p->d_chunk_len;
    const int32_t *sc = p->d_super_chunk;
    int32_t S = p->S;
    uint32_t *bar = p->d_bar;
    int32_t *err = p->d_err;
    int64_t lim = p->spin_limit;
    void *args[] = {&w, &v, &cb, &cl, &sc, &S, &b, &x, &bar, &err, &lim};
    HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(dev::trsv_persistent), dim3(p->grid),
                                       dim3(dev::kBlock), args, 0, st));
    p->last_stream = st;
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
        // a workgroup left the barrier early: clear the words for the next solve
        HIP_TRY(hipMemset(p->d_bar, 0, 64 * sizeof(uint32_t)));
        HIP_TRY(hipMemset(p->d_err, 0, sizeof(int32_t)));
    }
    return GLTRSV_OK;
}

}  // extern "C"
