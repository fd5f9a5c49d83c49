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
#include "internal.h"

#pragma clang fp contract(off)

namespace gltrsv {
namespace dev {

constexpr uint32_t HDR = 0x80000000u;
constexpr uint32_t INTL = 0x40000000u;
constexpr uint32_t MASK = 0x3FFFFFFFu;
constexpr uint32_t PAD = 0xFFFFFFFFu;
// Entries per batch (below).  A short batch shortens a lane's serial path,
// since each batch waits for its own gathers; a long one keeps more gathers
// in flight per lane.  Measured on MI355X: 4 is fastest for the single-system
// kernels and BSP batches, 8 for semi-asynchronous batches and several
// right-hand sides.
#ifndef GLTRSV_UNROLL
#define GLTRSV_UNROLL 4
#endif
#ifndef GLTRSV_UNROLL_WIDE
#define GLTRSV_UNROLL_WIDE 8
#endif
constexpr int kUnroll = GLTRSV_UNROLL;
constexpr int kUnrollWide = GLTRSV_UNROLL_WIDE;
using gltrsv::kRing;

// One lane processes the packed entries of its task: entry t at
// word/value[base + 64 t + lane], t < len.  Entries are handled in batches of
// U (kUnroll or kUnrollWide) through a two-deep pipeline:
//   while batch i is processed, the gathers of batch i+1 and the words and
//   values of batch i+2 are in flight;
//   every operand that is final before batch i+1 starts (x of an earlier
//   superstep, b of a new row, a row of this task at least kRing rows back)
//   is gathered from memory; rows of this task fewer than kRing rows back come
//   from an on-chip ring (a register for the previous row, LDS for older);
//   the x values finished in a batch are stored after the batch, so no store
//   sits in front of a wait.
// A row read from memory by batch j finished at least kRing >= 2 U
// entries earlier, i.e. in batch j-2 or before, whose stores precede the
// gathers of batch j in the lane's program order.
// Loads are issued unconditionally (padding slots re-read the chunk's first
// slot, non-gathered operands re-read b[0]) so their count per iteration is
// fixed and the compiler can wait for exactly the batch it needs.
static_assert(2 * kUnroll <= gltrsv::kRing && 2 * kUnrollWide <= gltrsv::kRing,
              "the ring must cover two batches");

template <int U>
struct Batch {
    uint32_t w[U];
    double v[U];
};

// Cross-workgroup data protocol.  x is the only array written during a
// solve.  Every access to it (and to b, which may alias it) is an agent-scope
// atomic access; on this GPU family those are the L2-coherent (sc1) loads and
// stores, so a value stored by any XCD is what any other XCD loads once the
// store has completed.  The barrier therefore needs no L2 write-back or
// invalidation: an arrival waits for the workgroup's stores to complete, and
// the gathers of the next superstep are issued after the new generation has
// been observed.  (Plain accesses with agent-scope release/acquire fences
// at the barrier are slower: each fence writes back or invalidates the XCD's
// whole L2, and plain random gathers are no faster than coherent ones.)
__device__ __forceinline__ double load_x(const double *p)
{
    const unsigned long long u =
        __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double(static_cast<long long>(u));
}

__device__ __forceinline__ void store_x(double *p, double v)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                       static_cast<unsigned long long>(__double_as_longlong(v)), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

struct LaneCursor {
    const uint32_t *wp;   // word + base + lane
    const double *vp;
    int32_t len;
};

__device__ __forceinline__ LaneCursor make_cursor(const uint32_t *__restrict__ word, const double *__restrict__ value,
                                                  int64_t base, int32_t len, int lane)
{
    LaneCursor c;
    c.wp = word + base + lane;
    c.vp = value + base + lane;
    c.len = len;
    return c;
}

template <int U>
__device__ __forceinline__ void load_batch(const LaneCursor &c, int32_t t0, Batch<U> &B)
{
#pragma unroll
    for (int j = 0; j < U; j++) {
        const bool in = t0 + j < c.len;
        const int64_t off = in ? int64_t(t0 + j) * 64 : 0;
        const uint32_t w = __builtin_nontemporal_load(c.wp + off);
        const double v = __builtin_nontemporal_load(c.vp + off);
        B.w[j] = in ? w : PAD;
        B.v[j] = v;
    }
}

template <int U>
__device__ __forceinline__ void gather_batch(const Batch<U> &B, const double *b, const double *x, double (&g)[U])
{
#pragma unroll
    for (int j = 0; j < U; j++) {
        const uint32_t c = B.w[j];
        const bool ext = (c & (HDR | INTL)) == 0;
        const bool hdr = (c & HDR) && c != PAD;
        const double *src = ext ? x + c : (hdr ? b + (c & MASK) : b);
        g[j] = load_x(src);
    }
}

struct LaneState {
    double acc, diag, last_y;
    int32_t cur;
    uint32_t pos;
};

// Ring of the lane's recent rows in LDS: slot r % kRing holds row r of the
// task; slot kRing takes the writes of entries that finish no row, so the
// write needs no branch.
using Ring = double (*)[kBlock];

// Handles U entries in order.  Every entry runs the same instruction
// sequence: the division that closes a row is evaluated for every entry and
// kept only at row headers, so the wave never splits on the entry kind.
template <int U>
__device__ __forceinline__ void process_batch(const Batch<U> &B, const double (&g)[U], LaneState &st, double *x,
                                              Ring ring)
{
    double ys[U];
    int32_t yrow[U];
#pragma unroll
    for (int j = 0; j < U; j++) {
        const uint32_t c = B.w[j];
        const bool hdr = (c & HDR) != 0;           // row header or padding
        const bool intl = (c >> 30) == 1u;         // same task, a few rows back
        const bool fin = hdr && st.cur >= 0;       // closes the current row
        const double y = st.acc / st.diag;
        ys[j] = y;
        yrow[j] = fin ? st.cur : -1;
        st.last_y = fin ? y : st.last_y;
        ring[fin ? (st.pos % kRing) : kRing][threadIdx.x] = y;
        st.pos += fin ? 1u : 0u;
        const uint32_t back = c & MASK;
        double xv = g[j];
        if (intl && back >= 2u) xv = ring[(st.pos - back) % kRing][threadIdx.x];
        xv = (intl && back == 1u) ? st.last_y : xv;
        const double prod = B.v[j] * xv;
        const double nacc = st.acc - prod;
        st.acc = hdr ? g[j] : nacc;
        st.diag = hdr ? B.v[j] : st.diag;
        st.cur = hdr ? (c == PAD ? -1 : int32_t(back)) : st.cur;
    }
#pragma unroll
    for (int j = 0; j < U; j++)
        if (yrow[j] >= 0) store_x(x + yrow[j], ys[j]);
}

// Semi-asynchronous execution: x starts filled with kUnready, a signalling
// NaN.  Every value the solve stores is the result of a division, which never
// yields a signalling NaN, so a gathered kUnready means "not computed yet":
// the gather is repeated until the value arrives.
constexpr unsigned long long kUnready = 0x7FF4A5A5A5A5A5A5ull;
#ifndef GLTRSV_AWAIT_NAP_MAX
#define GLTRSV_AWAIT_NAP_MAX 1
#endif
constexpr int kAwaitNapMax = GLTRSV_AWAIT_NAP_MAX;   // longest pause between re-reads, in s_sleep(1) units

__device__ __forceinline__ bool unready(uint32_t c, double g)
{
    return (c & (HDR | INTL)) == 0 && static_cast<unsigned long long>(__double_as_longlong(g)) == kUnready;
}

// Waits until every gathered column of the batch holds a computed value.
// Gives up after spin_limit rounds (setting *err) or once another wave has
// set *err; the solve's status then reports the failure.
template <int U>
__device__ __forceinline__ void await_batch(const Batch<U> &B, double (&g)[U], const double *x, int32_t *err,
                                            int64_t spin_limit)
{
    bool miss = false;
#pragma unroll
    for (int j = 0; j < U; j++) miss |= unready(B.w[j], g[j]);
    if (__ballot(miss) == 0ull) return;
    int32_t nap = 1;
    for (int64_t spins = 1;; spins++) {
        for (int32_t k = 0; k < nap; k++) __builtin_amdgcn_s_sleep(1);
        nap = min(2 * nap, int32_t(kAwaitNapMax));
#pragma unroll
        for (int j = 0; j < U; j++)
            if (unready(B.w[j], g[j])) g[j] = load_x(x + B.w[j]);
        miss = false;
#pragma unroll
        for (int j = 0; j < U; j++) miss |= unready(B.w[j], g[j]);
        if (__ballot(miss) == 0ull) return;
        if (spins > spin_limit) {
            if ((threadIdx.x & 63) == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        if ((spins & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    }
}

// One pipeline step: gathers of `nxt`, words/values of the batch after it
// into `fut`, then the work of `now` (in the semi-asynchronous form, once
// every operand of `now` has been computed).
#define GLTRSV_STEP(NOW, GNOW, NXT, GNXT, FUT, T0)                                                       \
    do {                                                                                                 \
        gather_batch(NXT, b, x, GNXT);                                                                   \
        load_batch(cur, (T0) + 2 * U, FUT);                                                              \
        if constexpr (kAsync) await_batch(NOW, GNOW, x, err, spin_limit);                                \
        process_batch(NOW, GNOW, st, x, ring);                                                           \
    } while (0)

// Runs one lane's task.  b0/b1 hold the task's first two batches (already
// loaded by the caller, possibly before the superstep's barrier).  The loop
// is unrolled three times so the three batch buffers change roles without
// register copies.
template <int U, bool kAsync = false>
__device__ __forceinline__ void run_lane(const LaneCursor &cur, Batch<U> &b0, Batch<U> &b1, const double *b,
                                         double *x, Ring ring, int32_t *err = nullptr, int64_t spin_limit = 0)
{
    LaneState st;
    st.acc = 0.0;
    st.diag = 1.0;
    st.last_y = 0.0;
    st.cur = -1;
    st.pos = 0;
    Batch<U> b2;
    double g0[U], g1[U], g2[U];
    gather_batch(b0, b, x, g0);
    int32_t t0 = 0;
    for (;;) {
        GLTRSV_STEP(b0, g0, b1, g1, b2, t0);
        t0 += U;
        if (t0 >= cur.len) break;
        GLTRSV_STEP(b1, g1, b2, g2, b0, t0);
        t0 += U;
        if (t0 >= cur.len) break;
        GLTRSV_STEP(b2, g2, b0, g0, b1, t0);
        t0 += U;
        if (t0 >= cur.len) break;
    }
    if (st.cur >= 0) store_x(x + st.cur, st.acc / st.diag);
}
#undef GLTRSV_STEP

__global__ __launch_bounds__(kBlock) void trsv_superstep_plain(
    const uint32_t *__restrict__ word, const double *__restrict__ value, const int64_t *__restrict__ chunk_base,
    const int32_t *__restrict__ chunk_len, int32_t c0, int32_t c1, const double *b, double *x)
{
    __shared__ double ring[kRing + 1][kBlock];
    const int32_t c = c0 + int32_t((blockIdx.x * kBlock + threadIdx.x) >> 6);
    if (c >= c1) return;
    const LaneCursor cur = make_cursor(word, value, chunk_base[c], chunk_len[c], threadIdx.x & 63);
    Batch<kUnroll> b0, b1;
    load_batch(cur, 0, b0);
    load_batch(cur, kUnroll, b1);
    run_lane(cur, b0, b1, b, x, ring);
}

// The schedule executed without the reorder of Sec. 5 (the ablation of the
// paper's locality study): the matrix stays in the caller's CSR order and
// each lane walks the rows of its task through the row pointers.  One launch
// per superstep; lane t of the launch runs task t0 + t (tasks of a superstep
// longest first, as in the packed layout).  Per row the same operations in
// the same order as every other form: acc = b_i, then acc - a_ij x_j over
// the stored off-diagonals in stored order, then one division.  A row of
// the same task read from x was stored earlier by this lane (same address,
// program order); rows of other tasks come from earlier supersteps.
__global__ __launch_bounds__(kBlock) void trsv_superstep_unordered(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const double *__restrict__ val,
    const int32_t *__restrict__ rows, const int64_t *__restrict__ task_off, int32_t t0, int32_t t1, int32_t upper,
    const double *b, double *x)
{
    const int32_t t = t0 + int32_t(blockIdx.x * kBlock + threadIdx.x);
    if (t >= t1) return;
    for (int64_t k = task_off[t]; k < task_off[t + 1]; k++) {
        const int32_t r = rows[k];
        const int64_t beg = row_ptr[r], end = row_ptr[r + 1];
        const int64_t d = upper ? beg : end - 1;   // the diagonal: first (upper) or last (lower) entry
        int64_t e = upper ? beg + 1 : beg;
        const int64_t e_end = upper ? end : end - 1;
        double acc = load_x(b + r);
        // four entries at a time: their loads first, then the subtractions in order
        for (; e + 4 <= e_end; e += 4) {
            int32_t c[4];
            double v[4], g[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                c[j] = col[e + j];
                v[j] = val[e + j];
            }
#pragma unroll
            for (int j = 0; j < 4; j++) g[j] = load_x(x + c[j]);
#pragma unroll
            for (int j = 0; j < 4; j++) acc = acc - v[j] * g[j];
        }
        for (; e < e_end; e++) acc = acc - val[e] * load_x(x + col[e]);
        store_x(x + r, acc / val[d]);
    }
}

// Barrier over all workgroups of the grid, in two halves so that work that
// does not depend on other workgroups can run while waiting.  Arrivals are
// counted in two levels: workgroups of a group of kGroup count on the group's
// word; the last of each group counts on the top word; the last of those
// advances the generation word that every workgroup waits on.  No word sees
// more than max(kGroup, groups) arrivals, and every word sits on its own
// 128-byte line.  Each last arrival resets the word it completed before
// moving up, so the words are ready for the next barrier.
constexpr int kGroup = 16;
constexpr int kBarGen = 0;          // word index of the generation
constexpr int kBarTop = 32;         // word index of the top count
constexpr int kBarGroups = 64;      // group g counts at kBarGroups + 32 g
constexpr int kBarWords = kBarGroups + 32 * 128;   // up to 128 groups

struct BarrierTicket {
    uint32_t gen;
    bool last;
};

__device__ __forceinline__ BarrierTicket barrier_arrive(uint32_t *bar)
{
    // Every wave waits until its own (coherent) stores have completed.
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    __shared__ uint32_t s_gen;
    __shared__ int32_t s_last;
    if (threadIdx.x == 0) {
        const uint32_t G = gridDim.x;
        const uint32_t grp = blockIdx.x / kGroup;
        const uint32_t groups = (G + kGroup - 1) / kGroup;
        const uint32_t gsize = min(uint32_t(kGroup), G - grp * kGroup);
        uint32_t *gen = bar + kBarGen;
        uint32_t *top = bar + kBarTop;
        uint32_t *cnt = bar + kBarGroups + 32 * grp;
        const uint32_t g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool last = false;
        const uint32_t old = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == gsize - 1) {
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t old2 = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (old2 == groups - 1) {
                __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                last = true;
            }
        }
        s_gen = g;
        s_last = last;
    }
    __syncthreads();
    BarrierTicket t;
    t.gen = s_gen;
    t.last = s_last != 0;
    return t;
}

// Returns false if the spin limit was hit or another workgroup reported an
// error; then the whole workgroup must exit.
__device__ __forceinline__ bool barrier_wait(uint32_t *bar, BarrierTicket t, int32_t *err, int64_t spin_limit)
{
    __shared__ int32_t ok;
    if (threadIdx.x == 0) {
        int32_t good = 1;
        if (!t.last) {
            const uint32_t *gen = bar + kBarGen;
            int64_t it = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == t.gen) {
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
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

__global__ __launch_bounds__(kBlock) void trsv_persistent(
    const uint32_t *__restrict__ word, const double *__restrict__ value, const int64_t *__restrict__ chunk_base,
    const int32_t *__restrict__ chunk_len, const int32_t *__restrict__ super_chunk, int32_t S, const double *b,
    double *x, uint32_t *bar, int32_t *err, int64_t spin_limit, int64_t *trace)
{
    const int32_t waves = int32_t(gridDim.x) * kWavesPerBlock;
    // wave slot: the i-th wave of workgroup g is slot i G + g.  Chunks of a
    // superstep are sorted longest first, so every workgroup (one per CU)
    // takes one chunk from each quarter of that order, and a narrow
    // superstep spreads over as many CUs as it has chunks, instead of
    // filling the first CUs with the longest chunks four at a time.
    const int32_t wave = int32_t(threadIdx.x >> 6) * int32_t(gridDim.x) + int32_t(blockIdx.x);
    const int lane = threadIdx.x & 63;
    __shared__ double ring[kRing + 1][kBlock];
    // first chunk of this wave in superstep 0, and its first two batches
    int32_t c = super_chunk[0] + wave;
    int32_t c_end = super_chunk[1];
    LaneCursor cur = make_cursor(word, value, c < c_end ? chunk_base[c] : 0, c < c_end ? chunk_len[c] : 0, lane);
    Batch<kUnroll> b0, b1;
    load_batch(cur, 0, b0);
    load_batch(cur, kUnroll, b1);
    for (int32_t s = 0; s < S; s++) {
#ifdef GLTRSV_TRACE
        if (threadIdx.x == 0) trace[(int64_t(s) * gridDim.x + blockIdx.x) * 3 + 0] = wall_clock64();
#endif
        while (c < c_end) {
            run_lane(cur, b0, b1, b, x, ring);
            c += waves;
            if (c < c_end) {
                cur = make_cursor(word, value, chunk_base[c], chunk_len[c], lane);
                load_batch(cur, 0, b0);
                load_batch(cur, kUnroll, b1);
            }
        }
#ifdef GLTRSV_TRACE
        if (threadIdx.x == 0) trace[(int64_t(s) * gridDim.x + blockIdx.x) * 3 + 1] = wall_clock64();
#endif
        if (s + 1 < S) {
            const BarrierTicket t = barrier_arrive(bar);
            // the matrix stream of the next superstep does not depend on x:
            // fetch it while the other workgroups finish
            c = super_chunk[s + 1] + wave;
            c_end = super_chunk[s + 2];
            cur = make_cursor(word, value, c < c_end ? chunk_base[c] : 0, c < c_end ? chunk_len[c] : 0, lane);
            load_batch(cur, 0, b0);
            load_batch(cur, kUnroll, b1);
            if (!barrier_wait(bar, t, err, spin_limit)) return;
        }
#ifdef GLTRSV_TRACE
        if (threadIdx.x == 0) trace[(int64_t(s) * gridDim.x + blockIdx.x) * 3 + 2] = wall_clock64();
#endif
    }
}

// ---------------------------------------------------------------------------
// Wavefront cores (opts.core_width = 64): a BSP core is a whole wavefront.
// The task's rows run one after another; for each row the 64 lanes load 64
// of its off-diagonals at once, gather x and form the products, and the wave
// subtracts them from acc = b_i in stored order (one lane's product at a
// time, broadcast with readlane), so every row sees exactly the operations
// of the one-lane form.  The next 64 entries are loaded and gathered while
// the current ones are subtracted.  Columns among the task's last kWaveRing
// rows are marked in the layout and read from a per-wave LDS ring; older
// rows of the task were stored before the wave's last full memory wait,
// which it takes every kWaveRing rows.
// ---------------------------------------------------------------------------
constexpr int kWaveRing = 64;

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u)), l));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u >> 32)), l));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// value of entry e (if e < e1) of the current row: a column from memory or
// from the ring; the product is formed by the caller.  c receives the word
// (kPadWord past the row's end).
__device__ __forceinline__ void wave_load(const uint32_t *__restrict__ wcol, const double *__restrict__ wval,
                                          int64_t e, int64_t e1, const double *x, const double *ring, int32_t q,
                                          double &v, double &g, uint32_t &c)
{
    v = 0.0;
    g = 0.0;
    c = PAD;
    if (e < e1) {
        c = wcol[e];
        v = wval[e];
        g = (c & INTL) ? ring[(q - int32_t(c & MASK)) & (kWaveRing - 1)] : load_x(x + c);
    }
}

// Semi-asynchronous wave cores: gathers that returned the not-yet-computed
// mark are read again until every lane holds a computed value.  Returns
// false once the spin limit is hit (setting *err) or another wave failed.
__device__ __forceinline__ bool wave_await(uint32_t c, double &g, const double *x, int32_t *err, int64_t spin_limit)
{
    bool miss = (c & (HDR | INTL)) == 0 && static_cast<unsigned long long>(__double_as_longlong(g)) == kUnready;
    if (__ballot(miss) == 0ull) return true;
    for (int64_t spins = 1;; spins++) {
        __builtin_amdgcn_s_sleep(1);
        if (miss) {
            g = load_x(x + c);
            miss = static_cast<unsigned long long>(__double_as_longlong(g)) == kUnready;
        }
        if (__ballot(miss) == 0ull) return true;
        if (spins > spin_limit) {
            if ((threadIdx.x & 63) == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if ((spins & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    }
}

template <bool kAsync>
__device__ __forceinline__ bool wave_task(const int32_t *__restrict__ wrow, const int64_t *__restrict__ wptr,
                                          const double *__restrict__ wdiag, const uint32_t *__restrict__ wcol,
                                          const double *__restrict__ wval, int64_t t0, int64_t t1, const double *b,
                                          double *x, double *ring, int32_t *err, int64_t spin_limit)
{
    const int lane = threadIdx.x & 63;
    for (int64_t t = t0; t < t1; t++) {
        const int32_t q = int32_t(t - t0);   // row index within the task
        if (q > 0 && (q & (kWaveRing - 1)) == 0) __builtin_amdgcn_s_waitcnt(0);   // older rows are in memory
        const int32_t row = wrow[t];
        double acc = load_x(b + row);
        const int64_t e0 = wptr[t], e1 = wptr[t + 1];
        double v, g;
        uint32_t c;
        wave_load(wcol, wval, e0 + lane, e1, x, ring, q, v, g, c);
        for (int64_t base = e0; base < e1; base += 64) {
            double vn, gn;
            uint32_t cn;
            wave_load(wcol, wval, base + 64 + lane, e1, x, ring, q, vn, gn, cn);
            if constexpr (kAsync)
                if (!wave_await(c, g, x, err, spin_limit)) return false;
            const double p = v * g;
            const int cnt = int(min<int64_t>(64, e1 - base));
            for (int l = 0; l < cnt; l++) acc = acc - readlane_f64(p, l);
            v = vn;
            g = gn;
            c = cn;
        }
        const double y = acc / wdiag[t];
        if (lane == 0) {
            ring[q & (kWaveRing - 1)] = y;
            store_x(x + row, y);
        }
        __builtin_amdgcn_wave_barrier();
    }
    return true;
}

// Supersteps [s0, s1) of a wave-core plan.  With s1 - s0 > 1 the grid is
// co-resident and the device-scope barrier separates the supersteps; a
// single superstep per launch needs none.  The i-th wave of workgroup g is
// slot i G + g (tasks of a superstep sorted longest first).
__global__ __launch_bounds__(kBlock) void trsv_wave(
    const int32_t *__restrict__ wrow, const int64_t *__restrict__ wptr, const double *__restrict__ wdiag,
    const uint32_t *__restrict__ wcol, const double *__restrict__ wval, const int64_t *__restrict__ wtask,
    const int32_t *__restrict__ wsuper, int32_t s0, int32_t s1, const double *b, double *x, uint32_t *bar,
    int32_t *err, int64_t spin_limit)
{
    __shared__ double ring[kWavesPerBlock][kWaveRing];
    const int32_t waves = int32_t(gridDim.x) * kWavesPerBlock;
    const int32_t slot = int32_t(threadIdx.x >> 6) * int32_t(gridDim.x) + int32_t(blockIdx.x);
    double *my_ring = ring[threadIdx.x >> 6];
    for (int32_t s = s0; s < s1; s++) {
        for (int32_t t = wsuper[s] + slot; t < wsuper[s + 1]; t += waves)
            wave_task<false>(wrow, wptr, wdiag, wcol, wval, wtask[t], wtask[t + 1], b, x, my_ring, err, spin_limit);
        if (s + 1 < s1) {
            const BarrierTicket tk = barrier_arrive(bar);
            if (!barrier_wait(bar, tk, err, spin_limit)) return;
        }
    }
}

// Semi-asynchronous wave cores: x holds the not-yet-computed mark at the
// start; wave w runs tasks w, w + W, ... in their global order (superstep by
// superstep) and waits only for the values it gathers.  Progress as for
// trsv_async: the earliest unfinished task depends only on finished tasks
// and its wave has finished its own earlier tasks (all waves co-resident).
__global__ __launch_bounds__(kBlock) void trsv_wave_async(
    const int32_t *__restrict__ wrow, const int64_t *__restrict__ wptr, const double *__restrict__ wdiag,
    const uint32_t *__restrict__ wcol, const double *__restrict__ wval, const int64_t *__restrict__ wtask,
    int32_t tasks, const double *b, double *x, int32_t *err, int64_t spin_limit)
{
    __shared__ double ring[kWavesPerBlock][kWaveRing];
    const int32_t waves = int32_t(gridDim.x) * kWavesPerBlock;
    const int32_t w = int32_t(blockIdx.x) * kWavesPerBlock + int32_t(threadIdx.x >> 6);
    double *my_ring = ring[threadIdx.x >> 6];
    for (int32_t t = w; t < tasks; t += waves)
        if (!wave_task<true>(wrow, wptr, wdiag, wcol, wval, wtask[t], wtask[t + 1], b, x, my_ring, err, spin_limit))
            return;
}

// ---------------------------------------------------------------------------
// Semi-asynchronous solve: no barriers.  Wave w runs chunks w, w + W, w + 2W,
// ... in order (chunks are numbered superstep by superstep), and a lane waits
// only for the columns it reads (await_batch).  Progress: the earliest
// unfinished chunk depends only on chunks of earlier supersteps, which are
// finished, and its wave has finished its own earlier chunks, so it is
// running it; hence every chunk completes provided all W waves are resident
// (the grid is sized to the device's co-resident capacity, as for the
// persistent kernel, and a wave kept from starting ends the solve with the
// spin-limit error instead of a hang).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void fill_unready(unsigned long long *x, int64_t n)
{
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) x[i] = kUnready;
}

__global__ __launch_bounds__(kBlock) void trsv_async(const uint32_t *__restrict__ word,
                                                     const double *__restrict__ value,
                                                     const int64_t *__restrict__ chunk_base,
                                                     const int32_t *__restrict__ chunk_len, int32_t chunks,
                                                     const double *b, double *x, int32_t *err, int64_t spin_limit)
{
    __shared__ double ring[kRing + 1][kBlock];
    const int32_t waves = int32_t(gridDim.x) * kWavesPerBlock;
    const int lane = threadIdx.x & 63;
    for (int32_t c = int32_t(blockIdx.x) * kWavesPerBlock + int32_t(threadIdx.x >> 6); c < chunks; c += waves) {
        const LaneCursor cur = make_cursor(word, value, chunk_base[c], chunk_len[c], lane);
        Batch<kUnroll> b0, b1;
        load_batch(cur, 0, b0);
        load_batch(cur, kUnroll, b1);
        run_lane<kUnroll, true>(cur, b0, b1, b, x, ring, err, spin_limit);
    }
}

// ---------------------------------------------------------------------------
// Several right-hand sides at once (SpTRSM): B and X are row-major n x ld,
// a launch handles R consecutive columns.  Each lane runs its task once for
// all R columns: one pass over the stream, and the R values of a gathered
// column lie next to each other in memory.  Per column the operations and
// their order are exactly those of the one-column solve.  Semi-asynchronous
// (per-row readiness, as trsv_async); one wave per workgroup keeps the
// R-column ring of recent rows within LDS.
// ---------------------------------------------------------------------------
template <int R>
struct MultiState {
    double acc[R], last_y[R];
    double diag;
    int32_t cur;
    uint32_t pos;
};

template <int R>
using MultiRing = double (*)[R][64];

template <int R>
__device__ __forceinline__ void gather_multi(const Batch<kUnrollWide> &B, const double *b, const double *x,
                                             int64_t ld, double (&g)[kUnrollWide][R])
{
#pragma unroll
    for (int j = 0; j < kUnrollWide; j++) {
        const uint32_t c = B.w[j];
        const bool ext = (c & (HDR | INTL)) == 0;
        const bool hdr = (c & HDR) && c != PAD;
        const double *src = ext ? x + int64_t(c) * ld : (hdr ? b + int64_t(c & MASK) * ld : b);
#pragma unroll
        for (int r = 0; r < R; r++) g[j][r] = load_x(src + r);
    }
}

template <int R>
__device__ __forceinline__ void await_multi(const Batch<kUnrollWide> &B, double (&g)[kUnrollWide][R], const double *x,
                                            int64_t ld, int32_t *err, int64_t spin_limit)
{
    bool miss = false;
#pragma unroll
    for (int j = 0; j < kUnrollWide; j++)
#pragma unroll
        for (int r = 0; r < R; r++) miss |= unready(B.w[j], g[j][r]);
    if (__ballot(miss) == 0ull) return;
    for (int64_t spins = 1;; spins++) {
        __builtin_amdgcn_s_sleep(1);
        miss = false;
#pragma unroll
        for (int j = 0; j < kUnrollWide; j++)
#pragma unroll
            for (int r = 0; r < R; r++) {
                if (unready(B.w[j], g[j][r])) g[j][r] = load_x(x + int64_t(B.w[j]) * ld + r);
                miss |= unready(B.w[j], g[j][r]);
            }
        if (__ballot(miss) == 0ull) return;
        if (spins > spin_limit) {
            if ((threadIdx.x & 63) == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        if ((spins & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    }
}

// process_batch for R columns: the same branch-free sequence per column.
template <int R>
__device__ __forceinline__ void process_multi(const Batch<kUnrollWide> &B, const double (&g)[kUnrollWide][R],
                                              MultiState<R> &st, double *x, int64_t ld, MultiRing<R> ring)
{
    const int lane = threadIdx.x & 63;
    double ys[kUnrollWide][R];
    int32_t yrow[kUnrollWide];
#pragma unroll
    for (int j = 0; j < kUnrollWide; j++) {
        const uint32_t c = B.w[j];
        const bool hdr = (c & HDR) != 0;
        const bool intl = (c >> 30) == 1u;
        const bool fin = hdr && st.cur >= 0;
        const uint32_t slot = fin ? (st.pos % kRing) : kRing;
        yrow[j] = fin ? st.cur : -1;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const double y = st.acc[r] / st.diag;
            ys[j][r] = y;
            st.last_y[r] = fin ? y : st.last_y[r];
            ring[slot][r][lane] = y;
        }
        st.pos += fin ? 1u : 0u;
        const uint32_t back = c & MASK;
        const uint32_t rs = (st.pos - back) % kRing;
#pragma unroll
        for (int r = 0; r < R; r++) {
            double xv = g[j][r];
            if (intl && back >= 2u) xv = ring[rs][r][lane];
            xv = (intl && back == 1u) ? st.last_y[r] : xv;
            const double prod = B.v[j] * xv;
            const double nacc = st.acc[r] - prod;
            st.acc[r] = hdr ? g[j][r] : nacc;
        }
        st.diag = hdr ? B.v[j] : st.diag;
        st.cur = hdr ? (c == PAD ? -1 : int32_t(back)) : st.cur;
    }
#pragma unroll
    for (int j = 0; j < kUnrollWide; j++)
        if (yrow[j] >= 0)
#pragma unroll
            for (int r = 0; r < R; r++) store_x(x + int64_t(yrow[j]) * ld + r, ys[j][r]);
}

template <int R>
__device__ __forceinline__ void run_lane_multi(const LaneCursor &cur, const double *b, double *x, int64_t ld,
                                               MultiRing<R> ring, int32_t *err, int64_t spin_limit)
{
    MultiState<R> st;
#pragma unroll
    for (int r = 0; r < R; r++) {
        st.acc[r] = 0.0;
        st.last_y[r] = 0.0;
    }
    st.diag = 1.0;
    st.cur = -1;
    st.pos = 0;
    Batch<kUnrollWide> now, nxt;
    double gnow[kUnrollWide][R], gnxt[kUnrollWide][R];
    load_batch(cur, 0, now);
    gather_multi<R>(now, b, x, ld, gnow);
    for (int32_t t0 = 0; t0 < cur.len; t0 += kUnrollWide) {
        load_batch(cur, t0 + kUnrollWide, nxt);
        gather_multi<R>(nxt, b, x, ld, gnxt);
        await_multi<R>(now, gnow, x, ld, err, spin_limit);
        process_multi<R>(now, gnow, st, x, ld, ring);
        now = nxt;
#pragma unroll
        for (int j = 0; j < kUnrollWide; j++)
#pragma unroll
            for (int r = 0; r < R; r++) gnow[j][r] = gnxt[j][r];
    }
    if (st.cur >= 0)
#pragma unroll
        for (int r = 0; r < R; r++) store_x(x + int64_t(st.cur) * ld + r, st.acc[r] / st.diag);
}

template <int R>
__global__ __launch_bounds__(64) void trsv_async_multi(const uint32_t *__restrict__ word,
                                                       const double *__restrict__ value,
                                                       const int64_t *__restrict__ chunk_base,
                                                       const int32_t *__restrict__ chunk_len, int32_t chunks,
                                                       const double *b, double *x, int64_t ld, int32_t *err,
                                                       int64_t spin_limit)
{
    __shared__ double ring[kRing + 1][R][64];
    const int lane = threadIdx.x & 63;
    for (int32_t c = int32_t(blockIdx.x); c < chunks; c += int32_t(gridDim.x)) {
        const LaneCursor cur = make_cursor(word, value, chunk_base[c], chunk_len[c], lane);
        run_lane_multi<R>(cur, b, x, ld, ring, err, spin_limit);
    }
}

template __global__ void trsv_async_multi<1>(const uint32_t *, const double *, const int64_t *, const int32_t *,
                                             int32_t, const double *, double *, int64_t, int32_t *, int64_t);
template __global__ void trsv_async_multi<2>(const uint32_t *, const double *, const int64_t *, const int32_t *,
                                             int32_t, const double *, double *, int64_t, int32_t *, int64_t);
template __global__ void trsv_async_multi<4>(const uint32_t *, const double *, const int64_t *, const int32_t *,
                                             int32_t, const double *, double *, int64_t, int32_t *, int64_t);

// ---------------------------------------------------------------------------
// Batched solve: many independent systems in one launch.
//
// Every system i has a 64-bit state word: high half = its open superstep,
// low half = chunks of that superstep claimed so far.  A wave claims chunks
// with one atomic add on the state word; a claim whose low half is beyond the
// superstep's chunk count finds no work.  The wave that completes the last
// chunk of superstep s (per-superstep done counters) publishes s+1 by
// exchanging the state word to (s+1, 0): increments that land before the
// exchange belonged to the exhausted superstep, those after it are claims of
// s+1.  Systems never wait for each other, and a wave only waits for chunks
// that running waves hold, so the grid needs no co-residency.
// ---------------------------------------------------------------------------


__device__ __forceinline__ unsigned long long *state_word(unsigned long long *state, int32_t i)
{
    return state + int64_t(i) * kStateStride;
}

// One claim of up to per_claim chunks of system i: valid iff the claimed
// index lies inside the superstep the word held at that moment (it may have
// advanced since it was read).
__device__ __forceinline__ int32_t try_claim(const SysDesc *__restrict__ sys, unsigned long long *state, int32_t i,
                                             int32_t per_claim, int32_t *gs_out, int32_t *c0, int32_t *c1)
{
    const unsigned long long got = __hip_atomic_fetch_add(state_word(state, i), (unsigned long long)per_claim,
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t gs = int32_t(got >> 32);
    const int64_t gc = int64_t(got & 0xffffffffull);
    if (gs >= sys[i].S) return 0;
    const int32_t *sc = sys[i].super_chunk;
    const int32_t n2 = sc[gs + 1] - sc[gs];
    if (gc >= n2) return 0;
    *gs_out = gs;
    *c0 = sc[gs] + int32_t(gc);
    *c1 = sc[gs] + int32_t(min<int64_t>(gc + per_claim, n2));
    return 1;
}

__global__ __launch_bounds__(kBlock) void batch_reset(unsigned long long *state, uint32_t *done, int32_t count,
                                                      int32_t ndone, uint32_t *finished, int32_t *err)
{
    const int32_t i = int32_t(blockIdx.x) * kBlock + int32_t(threadIdx.x);
    if (i < count) *state_word(state, i) = 0ull;
    for (int32_t j = i; j < ndone; j += int32_t(gridDim.x) * kBlock) done[j] = 0u;
    if (i == 0) {
        finished[0] = 0u;
        finished[1] = 0u;
        *err = 0;
    }
}

// spin_limit: wall-clock ticks a wave may go without finding work.
// target: the launch ends once `finished` reaches it (systems completed in
// this launch).  quantum: wall-clock ticks after which waves stop claiming
// (<= 0: no limit); claimed chunks are always completed, so every state word
// is consistent when the launch ends and a later launch continues from it.
__global__ __launch_bounds__(kBlock) void trsv_batched(const SysDesc *__restrict__ sys, int32_t count,
                                                       unsigned long long *state, uint32_t *done,
                                                       uint32_t *finished, int32_t *err, int64_t spin_limit,
                                                       int32_t per_claim, int32_t target, int64_t quantum,
                                                       int32_t keep_waves)
{
    __shared__ double ring[kRing + 1][kBlock];
    __shared__ uint32_t done_mask[kMaskSystems / 32];   // systems seen finished
    for (int q = threadIdx.x; q < kMaskSystems / 32; q += kBlock) done_mask[q] = 0u;
    __syncthreads();
    const int32_t total_waves = int32_t(gridDim.x) * kWavesPerBlock;
    const int lane = threadIdx.x & 63;
    const int32_t wave = int32_t(blockIdx.x) * kWavesPerBlock + int32_t(threadIdx.x >> 6);
    int32_t home = count > 0 ? wave % count : 0;
    int64_t idle_since = -1;   // wall-clock tick when this wave last found no work
    const int64_t deadline = quantum > 0 ? int64_t(wall_clock64()) + quantum : -1;
    int32_t nap = 1;           // idle back-off, in units of s_sleep(2)
    int32_t idle = 0;          // consecutive scans without work
    bool may_retire = true;
    for (;;) {
        // lane 0 walks the systems from `home` on and claims from the first
        // one with an unclaimed chunk; `live` counts the unfinished ones seen
        int32_t found = -1, fs = 0, c0 = 0, c1 = 0, live = 0;
        const bool late = deadline >= 0 && int64_t(wall_clock64()) > deadline;
        if (lane == 0) {
            for (int32_t t = 0; t < count && found < 0 && !late; t++) {
                const int32_t i = home + t < count ? home + t : home + t - count;
                if (i < kMaskSystems && (done_mask[i >> 5] >> (i & 31)) & 1u) continue;
                const unsigned long long st = __hip_atomic_load(state_word(state, i), __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                const int32_t s = int32_t(st >> 32);
                if (s >= sys[i].S) {
                    if (i < kMaskSystems) atomicOr(&done_mask[i >> 5], 1u << (i & 31));
                    continue;
                }
                live++;
                const int32_t *sc = sys[i].super_chunk;
                if (int64_t(st & 0xffffffffull) >= int64_t(sc[s + 1] - sc[s])) continue;
                if (try_claim(sys, state, i, per_claim, &fs, &c0, &c1)) found = i;
            }
        }
        found = __shfl(found, 0);
        if (found < 0) {
            int32_t quit = 0;
            idle++;
            if (lane == 0) {
                // every system finished (a full scan saw none open), the
                // quantum is over, or (checked now and then) the target is
                // met or another wave failed
                quit = late || live == 0;
                if (!quit && (idle & 15) == 0)
                    quit = __hip_atomic_load(finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= uint32_t(target) ||
                           __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            }
            if (lane == 0 && !quit) {
                for (int32_t k = 0; k < nap; k++) __builtin_amdgcn_s_sleep(2);
                nap = min(2 * nap, int32_t(kIdleNapMax));
                const int64_t now = int64_t(wall_clock64());
                if (idle_since < 0) {
                    idle_since = now;
                } else if (now - idle_since > spin_limit) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else if (may_retire && now - idle_since > kRetireTicks) {
                    // retire unless that would leave keep_waves or fewer; a
                    // wave refused once stays for the rest of the launch
                    const uint32_t r = __hip_atomic_fetch_add(finished + 1, 1u, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
                    if (int64_t(total_waves) - int64_t(r) - 1 >= int64_t(keep_waves)) {
                        quit = 1;
                    } else {
                        __hip_atomic_fetch_sub(finished + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        may_retire = false;
                    }
                }
            }
            if (__shfl(quit, 0)) return;
            continue;
        }
        fs = __shfl(fs, 0);
        c0 = __shfl(c0, 0);
        c1 = __shfl(c1, 0);
        idle = 0;
        nap = 1;
        idle_since = -1;
        home = found;
        const SysDesc d = sys[found];
        for (int32_t c = c0; c < c1; c++) {
            const LaneCursor cur = make_cursor(d.word, d.value, d.chunk_base[c], d.chunk_len[c], lane);
            Batch<kUnroll> b0, b1;
            load_batch(cur, 0, b0);
            load_batch(cur, kUnroll, b1);
            run_lane(cur, b0, b1, d.b, d.x, ring);
        }
        // the chunks' x stores are complete before they are counted as done
        __builtin_amdgcn_s_waitcnt(0);
        if (lane == 0) {
            const int32_t nch = d.super_chunk[fs + 1] - d.super_chunk[fs];
            const uint32_t old = __hip_atomic_fetch_add(done + d.done_off + fs, uint32_t(c1 - c0),
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (int64_t(old) + (c1 - c0) == nch) {
                __hip_atomic_exchange(state_word(state, found), (unsigned long long)(fs + 1) << 32, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                if (fs + 1 == d.S)
                    __hip_atomic_fetch_add(finished, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// The solve's memory traffic without its dependencies: one wave per chunk
// streams the chunk's words and values and gathers x at every column the
// solve reads from memory; a header closes the previous row with y[row] =
// the running sum, in stored order, of value * x (1.0 stands in for x at
// entries the solve takes from its on-chip ring).  No barrier, no division,
// no row waits for another: the floor one solve's bytes can reach.
__global__ __launch_bounds__(kBlock) void gather_probe(const uint32_t *__restrict__ word,
                                                       const double *__restrict__ value,
                                                       const int64_t *__restrict__ chunk_base,
                                                       const int32_t *__restrict__ chunk_len, int64_t chunks,
                                                       const double *__restrict__ x, double *__restrict__ y)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = int64_t(blockIdx.x) * kWavesPerBlock + int64_t(threadIdx.x >> 6);
    if (c >= chunks) return;
    const LaneCursor cur = make_cursor(word, value, chunk_base[c], chunk_len[c], lane);
    double acc = 0.0;
    int32_t row = -1;
    Batch<kUnrollWide> now, nxt;
    load_batch(cur, 0, now);
    for (int32_t t0 = 0; t0 < cur.len; t0 += kUnrollWide) {
        load_batch(cur, t0 + kUnrollWide, nxt);
        double g[kUnrollWide];
#pragma unroll
        for (int j = 0; j < kUnrollWide; j++) {
            const uint32_t w = now.w[j];
            const bool ext = (w & (HDR | INTL)) == 0;
            const double gx = load_x(ext ? x + w : x);
            g[j] = ext ? gx : 1.0;
        }
#pragma unroll
        for (int j = 0; j < kUnrollWide; j++) {
            const uint32_t w = now.w[j];
            if (w & HDR) {
                if (row >= 0) y[row] = acc;
                acc = 0.0;
                row = w == PAD ? -1 : int32_t(w & MASK);
            } else {
                acc = acc + now.v[j] * g[j];
            }
        }
        now = nxt;
    }
    if (row >= 0) y[row] = acc;
}

// ---------------------------------------------------------------------------
// Semi-asynchronous batched solve.  Per system one 64-bit word: low half =
// chunks claimed, high half = chunks completed.  Chunks are claimed in order
// (an atomic add on the low half), at most `window` ahead of the completed
// ones, and run with per-row readiness (await_batch) instead of barriers.
// Progress needs no co-residency: the earliest unfinished chunk of a system
// depends only on finished chunks and is held by a running wave, since claims
// are made by running waves in order and a wave runs its claims in order.
// A wave leaves when no system has an unclaimed chunk (its claimed chunks are
// done by then), or once the quantum has passed (claimed chunks are always
// completed, so a later launch continues from the words).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void fill_unready_sys(const SysDesc *__restrict__ sys, int32_t count)
{
    const int32_t i = int32_t(blockIdx.y);
    if (i >= count) return;
    unsigned long long *x = reinterpret_cast<unsigned long long *>(sys[i].x);
    const int64_t n = sys[i].n;
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x; r < n; r += stride) x[r] = kUnready;
}

__global__ __launch_bounds__(kBlock) void trsv_batched_async(const SysDesc *__restrict__ sys, int32_t count,
                                                             unsigned long long *state, uint32_t *finished,
                                                             int32_t *err, int64_t spin_limit, int32_t per_claim,
                                                             int64_t quantum)
{
    __shared__ double ring[kRing + 1][kBlock];
    __shared__ uint32_t done_mask[kMaskSystems / 32];   // systems with every chunk claimed
    for (int q = threadIdx.x; q < kMaskSystems / 32; q += kBlock) done_mask[q] = 0u;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int32_t wave = int32_t(blockIdx.x) * kWavesPerBlock + int32_t(threadIdx.x >> 6);
    int32_t home = count > 0 ? wave % count : 0;
    const int64_t deadline = quantum > 0 ? int64_t(wall_clock64()) + quantum : -1;
    int32_t nap = 1;
    int64_t idle = 0;
    for (;;) {
        int32_t found = -1, c0 = 0, c1 = 0, open = 0;
        const bool late = deadline >= 0 && int64_t(wall_clock64()) > deadline;
        if (lane == 0) {
            for (int32_t t = 0; t < count && found < 0 && !late; t++) {
                const int32_t i = home + t < count ? home + t : home + t - count;
                if (i < kMaskSystems && (done_mask[i >> 5] >> (i & 31)) & 1u) continue;
                const int32_t nch = sys[i].nchunks;
                const unsigned long long st = __hip_atomic_load(state_word(state, i), __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                const int64_t claimed = int64_t(st & 0xffffffffull), done = int64_t(st >> 32);
                if (claimed >= nch) {
                    if (i < kMaskSystems) atomicOr(&done_mask[i >> 5], 1u << (i & 31));
                    continue;
                }
                open++;
                if (claimed - done >= sys[i].window) continue;   // far enough ahead
                const unsigned long long got = __hip_atomic_fetch_add(
                    state_word(state, i), (unsigned long long)per_claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int64_t g = int64_t(got & 0xffffffffull);
                if (g < nch) {
                    found = i;
                    c0 = int32_t(g);
                    c1 = int32_t(min<int64_t>(g + per_claim, nch));
                }
            }
        }
        found = __shfl(found, 0);
        if (found < 0) {
            int32_t quit = 0;
            if (lane == 0) {
                quit = late || open == 0 || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
                if (!quit) {   // every open system is a window ahead: wait for completions
                    for (int32_t k = 0; k < nap; k++) __builtin_amdgcn_s_sleep(2);
                    nap = min(2 * nap, int32_t(kIdleNapMax));
                    if (++idle > spin_limit) {
                        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        quit = 1;
                    }
                }
            }
            if (__shfl(quit, 0)) return;
            continue;
        }
        c0 = __shfl(c0, 0);
        c1 = __shfl(c1, 0);
        nap = 1;
        idle = 0;
        home = found;
        const SysDesc d = sys[found];
        for (int32_t c = c0; c < c1; c++) {
            const LaneCursor cur = make_cursor(d.word, d.value, d.chunk_base[c], d.chunk_len[c], lane);
            Batch<kUnrollWide> b0, b1;
            load_batch(cur, 0, b0);
            load_batch(cur, kUnrollWide, b1);
            run_lane<kUnrollWide, true>(cur, b0, b1, d.b, d.x, ring, err, spin_limit);
        }
        // the chunks' x stores are complete before they are counted as done
        __builtin_amdgcn_s_waitcnt(0);
        if (lane == 0) {
            const unsigned long long old = __hip_atomic_fetch_add(
                state_word(state, found), (unsigned long long)(c1 - c0) << 32, __ATOMIC_RELAXED,
                __HIP_MEMORY_SCOPE_AGENT);
            if (int64_t(old >> 32) + (c1 - c0) == d.nchunks)
                __hip_atomic_fetch_add(finished, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Plain copy of 16-byte elements, grid-stride: the achievable-bandwidth
// reference and the calibration kernel of the memory-traffic counters.
__global__ __launch_bounds__(kBlock) void copy_probe(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                     int64_t n16)
{
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace dev
}  // namespace gltrsv

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
        return set_error(GLTRSV_ENOTSUP, "block_size must be 0 or 256 in this build");
    if (o->grid_blocks < 0) return set_error(GLTRSV_EINVAL, "grid_blocks must be >= 0");
    if (o->analysis_threads < 0 || o->analysis_threads > 64)
        return set_error(GLTRSV_EINVAL, "analysis_threads must be in 0..64");
    if (o->pack != GLTRSV_PACK_AUTO && o->pack != GLTRSV_PACK_HOST && o->pack != GLTRSV_PACK_DEVICE)
        return set_error(GLTRSV_EINVAL, "unknown pack mode");
    if (o->blocks < 0) return set_error(GLTRSV_EINVAL, "blocks must be >= 0");
    if (o->funnel_max_weight < 0) return set_error(GLTRSV_EINVAL, "funnel_max_weight must be >= 0");
    if (o->exec_hint != 0 && o->exec_hint != 1) return set_error(GLTRSV_EINVAL, "exec_hint must be 0 or 1");
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

// Wave-core layout (opts.core_width = 64): positions in the order of Sec. 5,
// tasks of a superstep longest first; per position the original row, its
// off-diagonals in stored order (a column among the task's last kWaveRing
// rows as kIntBit | rows back) and its diagonal.
int upload_wave(gltrsv_plan *p, const gltrsv_csr *A, int64_t *bytes)
{
    const int64_t n = p->n;
    const bool up = p->upper;
    std::vector<std::pair<int64_t, int64_t>> tasks;   // (first position in perm, length)
    std::vector<int32_t> wsuper(size_t(p->S) + 1, 0);
    int64_t pos = 0;
    for (int32_t s = 0; s < p->S; s++) {
        const size_t first = tasks.size();
        while (pos < n && p->superstep[size_t(p->perm[size_t(pos)])] == s) {
            const int32_t c = p->core[size_t(p->perm[size_t(pos)])];
            int64_t q = pos;
            while (q < n && p->superstep[size_t(p->perm[size_t(q)])] == s && p->core[size_t(p->perm[size_t(q)])] == c)
                q++;
            tasks.emplace_back(pos, q - pos);
            pos = q;
        }
        std::stable_sort(tasks.begin() + std::ptrdiff_t(first), tasks.end(),
                         [](const std::pair<int64_t, int64_t> &a, const std::pair<int64_t, int64_t> &b) {
                             return a.second > b.second;
                         });
        wsuper[size_t(s) + 1] = int32_t(tasks.size());
    }
    // new position of every row, and the task of every new position
    const size_t un = static_cast<size_t>(n);
    std::vector<int32_t> wrow(un), task_of(un);
    std::vector<int64_t> wtask(tasks.size() + 1, 0), newpos(un);
    int64_t np = 0;
    for (size_t t = 0; t < tasks.size(); t++) {
        wtask[t] = np;
        for (int64_t q = 0; q < tasks[t].second; q++, np++) {
            const int32_t v = p->perm[size_t(tasks[t].first + q)];
            const int32_t row = up ? int32_t(n - 1 - v) : v;
            wrow[size_t(np)] = row;
            task_of[size_t(np)] = int32_t(t);
            newpos[size_t(row)] = np;
        }
    }
    wtask[tasks.size()] = np;
    const int64_t noff = A->nnz - n;
    std::vector<int64_t> wptr(size_t(n) + 1, 0);
    const size_t uoff = static_cast<size_t>(std::max<int64_t>(noff, 0));
    std::vector<double> wdiag(un);
    std::vector<uint32_t> wcol(uoff);
    std::vector<double> wval(uoff);
    int64_t e = 0;
    for (int64_t t = 0; t < n; t++) {
        const int32_t row = wrow[size_t(t)];
        const int64_t beg = A->row_ptr[row], end = A->row_ptr[row + 1];
        const int64_t d = up ? beg : end - 1;
        wdiag[size_t(t)] = A->val[d];
        wptr[size_t(t)] = e;
        for (int64_t k = up ? beg + 1 : beg; k < (up ? end : end - 1); k++, e++) {
            const int32_t c = A->col[k];
            const int64_t pc = newpos[size_t(c)];
            const int64_t back = t - pc;
            const bool same = task_of[size_t(pc)] == task_of[size_t(t)] && back > 0 && back < dev::kWaveRing;
            wcol[size_t(e)] = same ? (kIntBit | uint32_t(back)) : uint32_t(c);
            wval[size_t(e)] = A->val[k];
        }
    }
    wptr[size_t(n)] = e;
    p->wsuper_host = wsuper;
    int rc;
    if ((rc = upload(&p->d_wrow, wrow, bytes)) || (rc = upload(&p->d_wptr, wptr, bytes)) ||
        (rc = upload(&p->d_wdiag, wdiag, bytes)) || (rc = upload(&p->d_wcol, wcol, bytes)) ||
        (rc = upload(&p->d_wval, wval, bytes)) || (rc = upload(&p->d_wtask, wtask, bytes)) ||
        (rc = upload(&p->d_wsuper, wsuper, bytes)))
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
        return o->exec_hint == 1 ? predict_async_us(V, sc, pm, cm) : predict_cost_us(V, sc, pm, cm);
    };
    if (o->schedule_kind == GLTRSV_SCHED_WAVEFRONT) {
        Schedule w = schedule_wavefront(V);
        *perm = schedule_order(V.n, w.core.data(), w.superstep.data(), w.S);
        *cost_us = predict(w, *perm);
        *chosen = GLTRSV_SCHED_WAVEFRONT;
        return w;
    }
    Schedule g = schedule_growlocal(V, params_of(o));
    std::vector<int32_t> pg = schedule_order(V.n, g.core.data(), g.superstep.data(), g.S);
    const double cg = predict(g, pg);
    if (o->schedule_kind == GLTRSV_SCHED_AUTO) {
        Schedule w = schedule_wavefront(V);
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
        p->predicted_us = opts->exec_hint == 1 ? predict_async_us(D, s, p->perm, cm) : predict_cost_us(D, s, p->perm, cm);
        p->schedule_kind = GLTRSV_SCHED_GIVEN;
    } else {
        s = build_schedule(D, opts, &p->perm, &p->predicted_us, &p->schedule_kind);
    }
    std::vector<int32_t> lv;
    p->wavefronts = wavefront_levels(D, lv);
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
    if ((rc = upload(&p->d_chunk_base, pk.chunk_base, &bytes)) || (rc = upload(&p->d_chunk_len, pk.chunk_len, &bytes)) ||
        (rc = upload(&p->d_super_chunk, pk.super_chunk, &bytes))) {
        gltrsv_plan_destroy(p);
        return rc;
    }
    {
        std::vector<uint32_t> bar(dev::kBarWords, 0u);
        std::vector<int32_t> err(1, 0);
        if ((rc = upload(&p->d_bar, bar, &bytes)) || (rc = upload(&p->d_err, err, &bytes))) {
            gltrsv_plan_destroy(p);
            return rc;
        }
    }
    if (opts->reorder == 0 && (rc = upload_unordered(p, A, &bytes))) {
        gltrsv_plan_destroy(p);
        return rc;
    }
    p->core_width = opts->core_width == 64 ? 64 : 1;
    if (p->core_width == 64 && (rc = upload_wave(p, A, &bytes))) {
        gltrsv_plan_destroy(p);
        return rc;
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
    int grid = std::min(per_cu * cus, dev::kGroup * 128);
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
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_w, dev::trsv_wave, dev::kBlock, 0);
        if (e != hipSuccess) {
            gltrsv_plan_destroy(p);
            return set_error(GLTRSV_EHIP, std::string("occupancy query: ") + hipGetErrorString(e));
        }
        int64_t most = 1;
        for (int32_t q = 0; q < p->S; q++)
            most = std::max<int64_t>(most, p->wsuper_host[size_t(q) + 1] - p->wsuper_host[size_t(q)]);
        int64_t gw = std::min<int64_t>(int64_t(per_cu_w) * cus, dev::kGroup * 128);
        if (opts->grid_blocks > 0) gw = std::min<int64_t>(gw, opts->grid_blocks);
        p->grid_wave = int(std::max<int64_t>(1, std::min<int64_t>(gw, (most + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock)));
        // semi-asynchronous: at least two workgroups per CU, more for large
        // systems (about one wave per 1,024 rows: each wave has one row in
        // flight), all co-resident.  Measured on MI355X: 512 workgroups were
        // best for the n = 1e5 ER and NB sets, the full 2,048 for n = 1e7.
        int per_cu_wa = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_wa, dev::trsv_wave_async, dev::kBlock, 0);
        if (e != hipSuccess) {
            gltrsv_plan_destroy(p);
            return set_error(GLTRSV_EHIP, std::string("occupancy query: ") + hipGetErrorString(e));
        }
        const int64_t wtasks = p->wsuper_host.empty() ? 0 : p->wsuper_host.back();
        int64_t gwa = std::min<int64_t>(int64_t(per_cu_wa) * cus,
                                        std::max<int64_t>(2 * int64_t(cus), (p->n + 4095) / 4096));
        if (opts->grid_blocks > 0) gwa = std::min<int64_t>(opts->grid_blocks, int64_t(per_cu_wa) * cus);
        p->grid_wave_async = int(std::max<int64_t>(
            1, std::min<int64_t>(gwa, (wtasks + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock)));
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
            hipLaunchKernelGGL(dev::trsv_wave, dim3(blocks), dim3(dev::kBlock), 0, st, p->d_wrow, p->d_wptr,
                               p->d_wdiag, p->d_wcol, p->d_wval, p->d_wtask, p->d_wsuper, s, s + 1, b, x,
                               p->d_bar, p->d_err, p->spin_limit);
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
        // all supersteps in one launch; the grid fits the co-resident capacity
        hipLaunchKernelGGL(dev::trsv_wave, dim3(p->grid_wave), dim3(dev::kBlock), 0, st, p->d_wrow, p->d_wptr,
                           p->d_wdiag, p->d_wcol, p->d_wval, p->d_wtask, p->d_wsuper, 0, p->S, b, x, p->d_bar,
                           p->d_err, p->spin_limit);
        HIP_TRY(hipGetLastError());
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
    int32_t *err = p->d_err;
    int64_t lim = p->spin_limit;
    int64_t *tr = p->d_trace;
    void *args[] = {&w, &v, &cb, &cl, &sc, &S, &b, &x, &bar, &err, &lim, &tr};
    if (p->cooperative) {
        HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(dev::trsv_persistent), dim3(p->grid),
                                           dim3(dev::kBlock), args, 0, st));
    } else {
        // The grid fits the device's co-resident capacity (occupancy query at
        // plan creation).  Should other work on the device keep workgroups
        // from starting, the waiting ones reach the spin limit and the solve
        // reports GLTRSV_ETIMEDOUT through gltrsv_plan_device_status.
        hipLaunchKernelGGL(dev::trsv_persistent, dim3(p->grid), dim3(dev::kBlock), 0, st, w, v, cb, cl, sc, S, b, x,
                           bar, err, lim, tr);
        HIP_TRY(hipGetLastError());
    }
    p->last_stream = st;
    return GLTRSV_OK;
}

int gltrsv_solve_async(gltrsv_plan *p, const double *b, double *x, void *stream)
{
    if (!p || (p->n && (!b || !x))) return set_error(GLTRSV_EINVAL, "null argument");
    if (p->n == 0) return GLTRSV_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double *bb = b;
    if (b == x) {   // x is about to be overwritten with the not-yet-computed mark
        if (!p->d_bcopy) HIP_TRY(hipMalloc(reinterpret_cast<void **>(&p->d_bcopy), sizeof(double) * size_t(p->n)));
        HIP_TRY(hipMemcpyAsync(p->d_bcopy, b, sizeof(double) * size_t(p->n), hipMemcpyDeviceToDevice, st));
        bb = p->d_bcopy;
    }
    const int64_t fill_blocks = std::min<int64_t>(4096, (p->n + dev::kBlock - 1) / dev::kBlock);
    hipLaunchKernelGGL(dev::fill_unready, dim3(unsigned(fill_blocks)), dim3(dev::kBlock), 0, st,
                       reinterpret_cast<unsigned long long *>(x), p->n);
    if (p->core_width == 64) {
        const int32_t wtasks = p->wsuper_host.back();
        hipLaunchKernelGGL(dev::trsv_wave_async, dim3(p->grid_wave_async), dim3(dev::kBlock), 0, st, p->d_wrow,
                           p->d_wptr, p->d_wdiag, p->d_wcol, p->d_wval, p->d_wtask, wtasks, bb, x, p->d_err,
                           p->spin_limit);
        HIP_TRY(hipGetLastError());
        p->last_stream = st;
        return GLTRSV_OK;
    }
    const int32_t chunks = int32_t(p->chunks);
    int64_t lim = p->spin_limit;
    if (p->cooperative) {
        const uint32_t *w = p->d_word;
        const double *v = p->d_value;
        const int64_t *cb = p->d_chunk_base;
        const int32_t *cl = p->d_chunk_len;
        int32_t *err = p->d_err;
        int32_t nch = chunks;
        void *args[] = {&w, &v, &cb, &cl, &nch, &bb, &x, &err, &lim};
        HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(dev::trsv_async), dim3(p->grid_async),
                                           dim3(dev::kBlock), args, 0, st));
    } else {
        hipLaunchKernelGGL(dev::trsv_async, dim3(p->grid_async), dim3(dev::kBlock), 0, st, p->d_word, p->d_value,
                           p->d_chunk_base, p->d_chunk_len, chunks, bb, x, p->d_err, lim);
    }
    HIP_TRY(hipGetLastError());
    p->last_stream = st;
    return GLTRSV_OK;
}

int gltrsv_solve_multi(gltrsv_plan *p, const double *b, double *x, int32_t nrhs, void *stream)
{
    if (!p || nrhs < 1 || (p->n && (!b || !x))) return set_error(GLTRSV_EINVAL, "bad argument");
    if (p->n == 0) return GLTRSV_OK;
    const int64_t total = p->n * int64_t(nrhs);
    if (b < x + total && x < b + total) return set_error(GLTRSV_EINVAL, "B and X must not overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t fill_blocks = std::min<int64_t>(4096, (total + dev::kBlock - 1) / dev::kBlock);
    hipLaunchKernelGGL(dev::fill_unready, dim3(unsigned(fill_blocks)), dim3(dev::kBlock), 0, st,
                       reinterpret_cast<unsigned long long *>(x), total);
    const int32_t chunks = int32_t(p->chunks);
    const unsigned grid = unsigned(std::min<int64_t>(int64_t(p->grid_async) * dev::kWavesPerBlock, chunks));
    const int64_t ld = nrhs;
    for (int32_t r0 = 0; r0 < nrhs;) {
        const int32_t R = nrhs - r0 >= 4 ? 4 : (nrhs - r0 >= 2 ? 2 : 1);
        if (R == 4)
            hipLaunchKernelGGL(dev::trsv_async_multi<4>, dim3(grid), dim3(64), 0, st, p->d_word, p->d_value,
                               p->d_chunk_base, p->d_chunk_len, chunks, b + r0, x + r0, ld, p->d_err, p->spin_limit);
        else if (R == 2)
            hipLaunchKernelGGL(dev::trsv_async_multi<2>, dim3(grid), dim3(64), 0, st, p->d_word, p->d_value,
                               p->d_chunk_base, p->d_chunk_len, chunks, b + r0, x + r0, ld, p->d_err, p->spin_limit);
        else
            hipLaunchKernelGGL(dev::trsv_async_multi<1>, dim3(grid), dim3(64), 0, st, p->d_word, p->d_value,
                               p->d_chunk_base, p->d_chunk_len, chunks, b + r0, x + r0, ld, p->d_err, p->spin_limit);
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
        // a workgroup left the barrier early: clear the words for the next solve
        HIP_TRY(hipMemset(p->d_bar, 0, dev::kBarWords * sizeof(uint32_t)));
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
    default: return gltrsv_solve(p, b, x, stream);
    }
}

int gltrsv_plan_set_exec(gltrsv_plan *p, int32_t form)
{
    if (!p) return set_error(GLTRSV_EINVAL, "null plan");
    if (form != GLTRSV_EXEC_PERSISTENT && form != GLTRSV_EXEC_PLAIN && form != GLTRSV_EXEC_ASYNC)
        return set_error(GLTRSV_EINVAL, "unknown execution form");
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
    const SolveFn forms[3] = {gltrsv_solve, gltrsv_solve_plain, gltrsv_solve_async};
    double us[3] = {0.0, 0.0, 0.0};
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    for (int f = 0; f < 3; f++) {
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
    for (int32_t f = 1; f < 3; f++)
        if (us[f] < us[f_best]) f_best = f;
    p->exec_form = f_best;
    if (us_out)
        for (int f = 0; f < 3; f++) us_out[f] = us[f];
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
            off += pl->S;
        }
    }
    int per_cu = 0, cus = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dev::trsv_batched, dev::kBlock, 0);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id);
    if (e != hipSuccess) {
        gltrsv_batch_destroy(bt);
        return set_error(GLTRSV_EHIP, std::string("occupancy query: ") + hipGetErrorString(e));
    }
    int64_t chunks = 0;
    for (auto *pl : bt->plans) chunks += pl->chunks;
    int grid = std::max(1, per_cu * cus);
    if (opts->grid_blocks > 0) grid = std::min(grid, opts->grid_blocks);
    grid = int(std::max<int64_t>(1, std::min<int64_t>(grid, (chunks + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock)));
    bt->grid = grid;
    bt->keep_waves = dev::keep_waves_for(widest_of(bt->plans), bt->per_claim, grid);
    *out = bt;
    return GLTRSV_OK;
}

static int batch_enqueue(gltrsv_batch *bt, hipStream_t st)
{
    if (bt->async_exec) {
        int64_t widest_n = 1;
        for (auto *pl : bt->plans) widest_n = std::max(widest_n, pl->n);
        const unsigned gx = unsigned(std::min<int64_t>(256, (widest_n + dev::kBlock - 1) / dev::kBlock));
        hipLaunchKernelGGL(dev::fill_unready_sys, dim3(gx, unsigned(bt->count)), dim3(dev::kBlock), 0, st, bt->d_desc,
                           bt->count);
        hipLaunchKernelGGL(dev::batch_reset, dim3(unsigned(std::max(1, (bt->count + dev::kBlock - 1) / dev::kBlock))),
                           dim3(dev::kBlock), 0, st, bt->d_state, bt->d_done, bt->count, 0, bt->d_finished,
                           bt->d_err);
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
    for (int32_t i = 0; i < bt->count; i++) {
        const int32_t j = bt->slot[i];
        if (!b[j] || !x[j]) return set_error(GLTRSV_EINVAL, "null vector in batch");
        if (bt->async_exec && b[j] == x[j])
            return set_error(GLTRSV_EINVAL, "semi-asynchronous batches need b and x apart");
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
            if (rc) return rc;
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
