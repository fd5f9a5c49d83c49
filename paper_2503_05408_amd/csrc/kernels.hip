// gltrsv device kernels for gfx950 (the host runtime and C ABI are in
// gltrsv.hip, serve.hip and pack.hip).
//
// Every BSP core of the schedule (Definition 2.1) is one lane of a 64-wide
// wavefront, or, with core width 64, a whole wavefront.  A core walks the
// rows of its (superstep, core) task in the order of Sec. 5, each row as the
// forward substitution of Eq. (2.1): acc <- b_i, acc <- acc - A_ij * x_j over
// the stored off-diagonals (no fused multiply-add), x_i <- acc / A_ii.
// Tasks of one superstep never read each other's results (Def. 2.1), so the
// only synchronisation is the barrier between supersteps: the kernel
// boundary in the plain form, a device-scope counter in the persistent form,
// per-row readiness in the semi-asynchronous form.
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

// Robbing in the semi-asynchronous kernels (see trsv_async): a wave that has
// waited rob_ticks for values while some workgroup of the launch has not
// started abandons its chunk.  alive == nullptr: never abandon.
struct AsyncRob {
    const uint32_t *alive;   // per workgroup: epoch of its start
    uint32_t epoch;
    int64_t rob_ticks;
};

// True in every lane if some workgroup of the launch has not started in
// this epoch.
__device__ __forceinline__ bool any_not_started(AsyncRob rob)
{
    const int lane = threadIdx.x & 63;
    for (uint32_t base = 0; base < gridDim.x; base += 64) {
        const uint32_t g = base + uint32_t(lane);
        const bool late = g < gridDim.x &&
                          __hip_atomic_load(rob.alive + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != rob.epoch;
        if (__ballot(late)) return true;
    }
    return false;
}

enum AwaitResult { kReady = 0, kAbandon = 1, kFailed = 2 };

// Waits until every gathered column of the batch holds a computed value.
// Gives up after spin_limit rounds (setting *err) or once another wave has
// set *err (kFailed: the solve's status reports the failure), or returns
// kAbandon once it has waited rob.rob_ticks while a workgroup has not
// started.
template <int U>
__device__ __forceinline__ int await_batch(const Batch<U> &B, double (&g)[U], const double *x, int32_t *err,
                                           int64_t spin_limit, AsyncRob rob)
{
    bool miss = false;
#pragma unroll
    for (int j = 0; j < U; j++) miss |= unready(B.w[j], g[j]);
    if (__ballot(miss) == 0ull) return kReady;
    int32_t nap = 1;
    int64_t since = -1;   // wall clock at the first rob check
    for (int64_t spins = 1;; spins++) {
        for (int32_t k = 0; k < nap; k++) __builtin_amdgcn_s_sleep(1);
        nap = min(2 * nap, int32_t(kAwaitNapMax));
#pragma unroll
        for (int j = 0; j < U; j++)
            if (unready(B.w[j], g[j])) g[j] = load_x(x + B.w[j]);
        miss = false;
#pragma unroll
        for (int j = 0; j < U; j++) miss |= unready(B.w[j], g[j]);
        if (__ballot(miss) == 0ull) return kReady;
        if (spins > spin_limit) {
            if ((threadIdx.x & 63) == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return kFailed;
        }
        if ((spins & 255) == 0) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return kFailed;
            if (rob.alive) {
                const int64_t now = int64_t(wall_clock64());
                if (since < 0) {
                    since = now;
                } else if (now - since > rob.rob_ticks) {
                    if (any_not_started(rob)) return kAbandon;
                    since = now;
                }
            }
        }
    }
}

// Per-launch epoch from the start ticket (as bsp_start; launches of this
// kernel on a plan take their tickets from their own word), announced in
// the alive table.
__device__ __forceinline__ uint32_t async_start(unsigned long long *ticket, uint32_t *alive, int64_t delay_ticks)
{
    __shared__ uint32_t s_epoch;
    if (threadIdx.x == 0) {
        if (delay_ticks > 0 && blockIdx.x % 7 == 3) {   // diagnostic: a late start
            const int64_t until = int64_t(wall_clock64()) + delay_ticks;
            while (int64_t(wall_clock64()) < until) __builtin_amdgcn_s_sleep(8);
        }
        const unsigned long long t = __hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t e = (uint32_t(t / gridDim.x) % 0x7FFFFFFFu) + 1u;
        __hip_atomic_store(alive + blockIdx.x, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_epoch = e;
    }
    __syncthreads();
    return s_epoch;
}

// Minimum over the wave of a 64-bit key, in every lane.
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long o = static_cast<unsigned long long>(__shfl_xor(static_cast<long long>(v), d, 64));
        v = o < v ? o : v;
    }
    return v;
}

// The earliest item (of a static order: wave slot v -- the (v mod w)-th wave
// of workgroup v / w, w waves per workgroup -- runs items v + k W, W = w G)
// of a not-started workgroup's waves that no thief has taken; taken
// for the caller if it precedes `before`.  vnext[v] = (epoch << 32) | items
// of slot v taken by thieves.  Returns the item, or -1.
__device__ __forceinline__ int64_t rob_item(AsyncRob rob, unsigned long long *vnext, int64_t items,
                                            int64_t before)
{
    const int lane = threadIdx.x & 63;
    const uint32_t G = gridDim.x;
    const uint32_t wpg = blockDim.x >> 6;   // waves per workgroup
    const int64_t W = int64_t(G) * wpg;
    unsigned long long best = ~0ull;   // (item << 16) | slot
    for (uint32_t base = 0; base < G; base += 64) {
        const uint32_t g = base + uint32_t(lane);
        if (g >= G) continue;
        if (__hip_atomic_load(rob.alive + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == rob.epoch) continue;
        for (uint32_t j = 0; j < wpg; j++) {
            const uint32_t v = g * wpg + j;
            const unsigned long long w = __hip_atomic_load(vnext + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int64_t k = uint32_t(w >> 32) == rob.epoch ? int64_t(uint32_t(w)) : 0;
            const int64_t item = int64_t(v) + k * W;
            if (item < items && item < before) {
                const unsigned long long key = (static_cast<unsigned long long>(item) << 16) | v;
                best = key < best ? key : best;
            }
        }
    }
    best = wave_min_u64(best);
    if (best == ~0ull) return -1;
    const uint32_t v = uint32_t(best & 0xFFFFu);
    const int64_t item = int64_t(best >> 16);
    int32_t got = 0;
    if (lane == 0) {
        const int64_t k = (item - int64_t(v)) / W;
        unsigned long long expect = __hip_atomic_load(vnext + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t kk = uint32_t(expect >> 32) == rob.epoch ? int64_t(uint32_t(expect)) : 0;
        if (kk == k)
            got = __hip_atomic_compare_exchange_strong(
                vnext + v, &expect, (static_cast<unsigned long long>(rob.epoch) << 32) | uint32_t(k + 1),
                __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return __builtin_amdgcn_readfirstlane(got) ? item : -1;
}

// One pipeline step: gathers of `nxt`, words/values of the batch after it
// into `fut`, then the work of `now` (in the semi-asynchronous form, once
// every operand of `now` has been computed).
#define GLTRSV_STEP(NOW, GNOW, NXT, GNXT, FUT, T0)                                                       \
    do {                                                                                                 \
        gather_batch(NXT, b, x, GNXT);                                                                   \
        load_batch(cur, (T0) + 2 * U, FUT);                                                              \
        if constexpr (kAsync)                                                                            \
            if (await_batch(NOW, GNOW, x, err, spin_limit, rob) == kAbandon) return false;              \
        process_batch(NOW, GNOW, st, x, ring);                                                           \
    } while (0)

// Runs one lane's task.  b0/b1 hold the task's first two batches (already
// loaded by the caller, possibly before the superstep's barrier).  The loop
// is unrolled three times so the three batch buffers change roles without
// register copies.  Returns false if the semi-asynchronous form abandoned
// the chunk (the whole wave does; the rows stored so far are final).
__device__ __forceinline__ AsyncRob no_rob() { return AsyncRob{nullptr, 0u, 0}; }

template <int U, bool kAsync = false>
__device__ __forceinline__ bool run_lane(const LaneCursor &cur, Batch<U> &b0, Batch<U> &b1, const double *b,
                                         double *x, Ring ring, int32_t *err = nullptr, int64_t spin_limit = 0,
                                         AsyncRob rob = AsyncRob{nullptr, 0u, 0})
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
    return true;
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

// ---------------------------------------------------------------------------
// Supersteps of one system in one launch, without relying on co-residency.
//
// The items of superstep s (chunks of 64 lane-cores, or wavefront-core
// tasks) are numbered k = 0 .. m_s - 1; the wave in slot v = i G + g (the
// i-th wave of workgroup g) owns items v, v + W, v + 2W, ... (W = 4 G), so
// item k belongs to workgroup k mod G.
//
// Superstep s is complete when its m_s items are counted as done.  Counts
// go to one word for grids of up to kFlatMax workgroups; larger grids count
// per group of kGroup workgroups (the group of an item's owner) and count
// completed groups on a top word.  The arrival that completes a word resets
// it, waits for the reset to land and then counts one level up; the last
// one publishes progress = (epoch, s + 1).  Words are reused by every
// superstep: they are zero again before the progress that allows the next
// superstep's counts is published.
//
// Workgroups that cannot start (other work holds the device) would stall
// the solve, so a workgroup whose wait for a superstep exceeds steal_ticks
// robs the workgroups that have not started yet: it marks one robbed in the
// alive table (a compare-and-swap that fails once the owner has started),
// then claims and runs that owner's items of the superstep, one exchange of
// an item's claim word each.  A workgroup announces itself at its start by
// exchanging its alive word for the epoch; if it finds itself robbed it
// claims its items of its first superstep (thieves may still be at work on
// that one; later supersteps are never robbed), otherwise it runs its items
// without claims.  It starts at the published progress.  So the solve
// advances whenever any workgroup runs, and with every workgroup resident
// (the normal case) nothing is claimed or scanned.
//
// The epoch comes from a ticket every workgroup takes at its start: solves
// on a plan do not overlap and each launches G workgroups, so tickets
// [j G, (j + 1) G) belong to the plan's j-th solve -- also when the launch
// is replayed from a graph.  Epochs use 31 bits; the top bit of an alive
// word marks "robbed in that epoch".
// ---------------------------------------------------------------------------

constexpr uint32_t kRobbed = 0x80000000u;

struct BspStart {
    uint32_t epoch;
    int32_t first;   // supersteps already completed when the workgroup started
    bool robbed;     // thieves ran (or may be running) items of superstep `first`
};

__device__ __forceinline__ BspStart bsp_start(uint32_t *bar, uint32_t *alive, int64_t delay_ticks)
{
    __shared__ uint32_t s_epoch;
    __shared__ int32_t s_first;
    __shared__ int32_t s_robbed;
    if (threadIdx.x == 0) {
        if (delay_ticks > 0 && blockIdx.x % 7 == 3) {   // diagnostic: a late start
            const int64_t until = int64_t(wall_clock64()) + delay_ticks;
            while (int64_t(wall_clock64()) < until) __builtin_amdgcn_s_sleep(8);
        }
        const unsigned long long t = __hip_atomic_fetch_add(reinterpret_cast<unsigned long long *>(bar + kBarStart),
                                                            1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t e = (uint32_t(t / gridDim.x) % 0x7FFFFFFFu) + 1u;
        const uint32_t old = __hip_atomic_exchange(alive + blockIdx.x, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long p = __hip_atomic_load(reinterpret_cast<unsigned long long *>(bar + kBarProg),
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_epoch = e;
        s_first = uint32_t(p >> 32) == e ? int32_t(uint32_t(p)) : 0;
        s_robbed = old == (e | kRobbed);
    }
    __syncthreads();
    BspStart st;
    st.epoch = s_epoch;
    st.first = s_first;
    st.robbed = s_robbed != 0;
    return st;
}

// Supersteps completed in this solve, from a progress word.
__device__ __forceinline__ int32_t bsp_completed(unsigned long long p, uint32_t epoch)
{
    return uint32_t(p >> 32) == epoch ? int32_t(uint32_t(p)) : 0;
}

// One lane claims item `item` for the solve; the whole wave gets the answer.
__device__ __forceinline__ bool claim_item(uint32_t *claim, int32_t item, uint32_t epoch)
{
    uint32_t got = 0;
    if ((threadIdx.x & 63) == 0)
        got = __hip_atomic_exchange(claim + item, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch ? 1u : 0u;
    return __builtin_amdgcn_readfirstlane(got) != 0;
}

// Items of group q (workgroups [q kGroup, q kGroup + kGroup)) among m items
// owned by workgroup k mod G.
__device__ __forceinline__ uint32_t group_items(uint32_t m, uint32_t G, uint32_t q)
{
    const uint32_t lo = q * uint32_t(kGroup), hi = min(G, lo + uint32_t(kGroup));
    const uint32_t full = m / G, rem = m % G;
    return (hi - lo) * full + (rem > lo ? min(rem, hi) - lo : 0u);
}

// Counts k done items of superstep s owned by workgroup `owner`; the count
// that completes the superstep publishes it.  Called by one lane; the
// caller's x stores have completed.
__device__ __forceinline__ void bsp_done(uint32_t *bar, uint32_t epoch, int32_t s, uint32_t m, uint32_t owner,
                                         uint32_t k)
{
    const uint32_t G = gridDim.x;
    const bool flat = G <= uint32_t(kFlatMax);
    const uint32_t q = flat ? 0u : owner / uint32_t(kGroup);
    uint32_t *cnt = bar + kBarGroups + 32 * q;
    const uint32_t want = flat ? m : group_items(m, G, q);
    const uint32_t old = __hip_atomic_fetch_add(cnt, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + k != want) return;
    __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    if (!flat) {
        uint32_t *top = bar + kBarTop;
        const uint32_t groups = (min(m, G) + uint32_t(kGroup) - 1) / uint32_t(kGroup);
        const uint32_t old2 = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old2 + 1 != groups) return;
        __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);
    }
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(bar + kBarProg),
                       (static_cast<unsigned long long>(epoch) << 32) | uint32_t(s + 1), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// End of a workgroup's own items of superstep s: every wave has waited for
// its x stores and added its count to *s_done; one add for the workgroup.
__device__ __forceinline__ void bsp_count_own(uint32_t *bar, uint32_t epoch, int32_t s, uint32_t m, uint32_t mine,
                                              uint32_t *s_done)
{
    __builtin_amdgcn_s_waitcnt(0);
    if ((threadIdx.x & 63) == 0 && mine) atomicAdd(s_done, mine);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t k = *s_done;
        *s_done = 0;
        if (k) bsp_done(bar, epoch, s, m, blockIdx.x, k);
    }
}

// Waits until superstep s is complete.  Every steal_ticks of waiting (100
// MHz wall clock) each wave runs steal(s).  Returns false if the spin limit
// was hit or another workgroup failed; then the whole workgroup must leave.
template <class Steal>
__device__ __forceinline__ bool bsp_wait(uint32_t *bar, uint32_t epoch, int32_t s, int32_t *err, int64_t spin_limit,
                                         int64_t steal_ticks, Steal steal)
{
    __shared__ int32_t s_state;   // 0 waiting, 1 complete, 2 failed, 3 steal now
    const unsigned long long *prog = reinterpret_cast<const unsigned long long *>(bar + kBarProg);
    int64_t next_steal = int64_t(wall_clock64()) + steal_ticks;
    for (int64_t it = 0;; it++) {
        if (threadIdx.x == 0) {
            int32_t st = bsp_completed(__hip_atomic_load(prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), epoch) > s;
            if (!st) {
                if (it > spin_limit) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    st = 2;
                } else if ((it & 1023) == 1023 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    st = 2;
                } else if (int64_t(wall_clock64()) >= next_steal) {
                    st = 3;
                    next_steal = int64_t(wall_clock64()) + steal_ticks;
                }
            }
            s_state = st;
        }
        __syncthreads();
        const int32_t st = s_state;
        __syncthreads();   // s_state is written again in the next round
        if (st == 1) return true;
        if (st == 2) return false;
        if (st == 3)
            steal(s);
        else
            __builtin_amdgcn_s_sleep(1);
    }
}

// A wave's steal pass over superstep s (items [i0, i0 + m)): the victims
// are the workgroups v = r, r + 4, ... (from a start spread over the
// thieves) that have not started; each is marked robbed (compare-and-swap
// of its alive word), then its items of s are claimed and run (run(item))
// and counted for it.
template <class Run>
__device__ __forceinline__ void steal_items(uint32_t *bar, uint32_t *alive, uint32_t *claim, uint32_t epoch,
                                            int32_t s, int32_t i0, uint32_t m, Run run)
{
    const int lane = threadIdx.x & 63;
    const uint32_t G = gridDim.x;
    const uint32_t first = (blockIdx.x * uint32_t(kWavesPerBlock) + (threadIdx.x >> 6)) % G;
    for (uint32_t base = 0; base < G; base += 64 * kWavesPerBlock) {
        const uint32_t r = base + uint32_t(lane) * kWavesPerBlock;   // this lane's candidate, relative to `first`
        const uint32_t v = (first + r) % G;
        bool victim = false;
        if (r < G && v < m) {   // owners of no item in s need no robbing
            uint32_t a = __hip_atomic_load(alive + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a != epoch) {
                victim = a == (epoch | kRobbed);
                if (!victim) {
                    uint32_t expect = a;
                    victim = __hip_atomic_compare_exchange_strong(alive + v, &expect, epoch | kRobbed, __ATOMIC_RELAXED,
                                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                             expect == (epoch | kRobbed);
                }
            }
        }
        unsigned long long cand = __ballot(victim);
        while (cand) {
            const int l = __builtin_ctzll(cand);
            cand &= cand - 1;
            const uint32_t vv = (first + base + uint32_t(l) * kWavesPerBlock) % G;
            for (uint32_t k = vv; k < m; k += G) {
                if (!claim_item(claim, i0 + int32_t(k), epoch)) continue;
                run(i0 + int32_t(k));
                __builtin_amdgcn_s_waitcnt(0);
                if (lane == 0) bsp_done(bar, epoch, s, m, vv, 1u);
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void trsv_persistent(
    const uint32_t *__restrict__ word, const double *__restrict__ value, const int64_t *__restrict__ chunk_base,
    const int32_t *__restrict__ chunk_len, const int32_t *__restrict__ super_chunk, int32_t S, const double *b,
    double *x, uint32_t *bar, uint32_t *alive, uint32_t *claim, int32_t *err, int64_t spin_limit,
    int64_t steal_ticks, int64_t delay_ticks, int64_t *trace)
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
    __shared__ uint32_t s_done;
    if (threadIdx.x == 0) s_done = 0;
    const BspStart bs = bsp_start(bar, alive, delay_ticks);
    int32_t s = bs.first;
    if (s >= S) return;
    bool claiming = bs.robbed;   // only a robbed workgroup's first superstep is contested
    // this wave's first chunk and its first two batches
    int32_t c = super_chunk[s] + wave, c_end = super_chunk[s + 1];
    bool have = c < c_end && (!claiming || claim_item(claim, c, bs.epoch));
    LaneCursor cur = make_cursor(word, value, have ? chunk_base[c] : 0, have ? chunk_len[c] : 0, lane);
    Batch<kUnroll> b0, b1;
    load_batch(cur, 0, b0);
    load_batch(cur, kUnroll, b1);
    auto run_chunk = [&](int32_t cc) {
        const LaneCursor sc = make_cursor(word, value, chunk_base[cc], chunk_len[cc], lane);
        Batch<kUnroll> s0, s1;
        load_batch(sc, 0, s0);
        load_batch(sc, kUnroll, s1);
        run_lane(sc, s0, s1, b, x, ring);
    };
    for (; s < S; s++) {
#ifdef GLTRSV_TRACE
        if (threadIdx.x == 0) trace[(int64_t(s) * gridDim.x + blockIdx.x) * 3 + 0] = wall_clock64();
#endif
        const int32_t c0 = super_chunk[s];
        const uint32_t m = uint32_t(c_end - c0);
        uint32_t mine = 0;
        for (;;) {
            if (have) {
                run_lane(cur, b0, b1, b, x, ring);
                mine++;
            }
            c += waves;
            if (c >= c_end) break;
            have = !claiming || claim_item(claim, c, bs.epoch);
            if (have) {
                cur = make_cursor(word, value, chunk_base[c], chunk_len[c], lane);
                load_batch(cur, 0, b0);
                load_batch(cur, kUnroll, b1);
            }
        }
        claiming = false;
#ifdef GLTRSV_TRACE
        if (threadIdx.x == 0) trace[(int64_t(s) * gridDim.x + blockIdx.x) * 3 + 1] = wall_clock64();
#endif
        bsp_count_own(bar, bs.epoch, s, m, mine, &s_done);
        if (s + 1 < S) {
            // the next superstep's stream does not depend on x: fetch its
            // first batches while waiting
            c = super_chunk[s + 1] + wave;
            c_end = super_chunk[s + 2];
            have = c < c_end;
            cur = make_cursor(word, value, have ? chunk_base[c] : 0, have ? chunk_len[c] : 0, lane);
            load_batch(cur, 0, b0);
            load_batch(cur, kUnroll, b1);
        }
        if (!bsp_wait(bar, bs.epoch, s, err, spin_limit, steal_ticks,
                      [&](int32_t ss) { steal_items(bar, alive, claim, bs.epoch, ss, c0, m, run_chunk); }))
            return;
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

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u)), l));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u >> 32)), l));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// acc minus the products of lanes [l, e), one after another in lane order
// (l and e the same in every lane, acc too).  The plain form reads each
// product out with readlane and subtracts it: three VALU instructions an
// entry.  The DPP form takes each product to the accumulator with the
// data-parallel-primitive broadcast of its lane within its 16-lane row
// (row_newbcast) folded into a fused multiply-add by -1: one instruction an
// entry, and as the product by -1 is exact the single rounding is that of
// the subtraction, so the bits are those of acc - p.  It runs a 16-lane row
// at a time: every row of the wave executes the same instructions, the one
// holding the entries gets the result, and readlane hands that to all lanes
// before the next row.  Its entry point into a row is picked by a branch
// tree on the first lane, and the row ends after lane e - 1; that fixed
// cost makes it slower than the plain form on rows of few entries.
#define GLTRSV_DPP_PAIR(a, b) "s_bitcmp1_b32 %3, 0\n s_cbranch_scc1 .Ls" #b "_%=\n s_branch .Ls" #a "_%=\n"
#define GLTRSV_DPP_NODE(bit, hi) "s_bitcmp1_b32 %3, " #bit "\n s_cbranch_scc1 .Ln" #hi "_%=\n"
#define GLTRSV_DPP_SUB(k) "v_fmac_f64_dpp %0, %1, %2 row_newbcast:" #k " row_mask:0xf bank_mask:0xf\n"
#define GLTRSV_DPP_STEP(k, n) ".Ls" #k "_%=:\n " GLTRSV_DPP_SUB(k) " s_cmp_eq_u32 %4, " #n "\n s_cbranch_scc1 .Lend_%=\n"

template <bool kDpp>
__device__ __forceinline__ double subtract_lanes(double acc, const double prod, const int l, const int e)
{
    if constexpr (!kDpp) {
        for (int j = l; j < e; j++) acc = acc - readlane_f64(prod, j);
        return acc;
    } else {
        const double m1 = -1.0;
        for (int rb = l >> 4; l < e && (rb << 4) < e; rb++) {
            // lanes [k0, k1) of row rb, 0 <= k0 < k1 <= 16
            const int k0 = __builtin_amdgcn_readfirstlane(max(l - (rb << 4), 0));
            const int k1 = __builtin_amdgcn_readfirstlane(min(e - (rb << 4), 16));
            double a = acc;
            // (the leading s_nop: two wait states between the VALU write of
            // the products and their first DPP read)
            asm volatile("s_nop 1\n"
                         GLTRSV_DPP_NODE(3, 8) GLTRSV_DPP_NODE(2, 4) GLTRSV_DPP_NODE(1, 2) GLTRSV_DPP_PAIR(0, 1)
                         ".Ln2_%=:\n" GLTRSV_DPP_PAIR(2, 3)
                         ".Ln4_%=:\n" GLTRSV_DPP_NODE(1, 6) GLTRSV_DPP_PAIR(4, 5)
                         ".Ln6_%=:\n" GLTRSV_DPP_PAIR(6, 7)
                         ".Ln8_%=:\n" GLTRSV_DPP_NODE(2, 12) GLTRSV_DPP_NODE(1, 10) GLTRSV_DPP_PAIR(8, 9)
                         ".Ln10_%=:\n" GLTRSV_DPP_PAIR(10, 11)
                         ".Ln12_%=:\n" GLTRSV_DPP_NODE(1, 14) GLTRSV_DPP_PAIR(12, 13)
                         ".Ln14_%=:\n" GLTRSV_DPP_PAIR(14, 15)
                         GLTRSV_DPP_STEP(0, 1) GLTRSV_DPP_STEP(1, 2) GLTRSV_DPP_STEP(2, 3) GLTRSV_DPP_STEP(3, 4)
                         GLTRSV_DPP_STEP(4, 5) GLTRSV_DPP_STEP(5, 6) GLTRSV_DPP_STEP(6, 7) GLTRSV_DPP_STEP(7, 8)
                         GLTRSV_DPP_STEP(8, 9) GLTRSV_DPP_STEP(9, 10) GLTRSV_DPP_STEP(10, 11)
                         GLTRSV_DPP_STEP(11, 12) GLTRSV_DPP_STEP(12, 13) GLTRSV_DPP_STEP(13, 14)
                         GLTRSV_DPP_STEP(14, 15)
                         ".Ls15_%=:\n " GLTRSV_DPP_SUB(15)
                         ".Lend_%=:\n"
                         : "+v"(a)
                         : "v"(prod), "v"(m1), "s"(k0), "s"(k1)
                         : "scc");
            acc = readlane_f64(a, rb << 4);
        }
        return acc;
    }
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

// Scalar registers of the wave-core kernels.  Measured on MI355X: with 88 or
// more only 7 of their 256-thread workgroups are resident per CU (both the
// compiler and the occupancy query report 8), with 80 or fewer all 8 are.
// 64 makes the wave-core semi-asynchronous solve of an n = 1e7 system 17%
// slower than 80 (5.70 against 4.88 ms).
#ifndef GLTRSV_WAVE_SGPRS
#define GLTRSV_WAVE_SGPRS 80
#endif
constexpr int kWaveSgprs = GLTRSV_WAVE_SGPRS;

// Runs one wave-core task: the rows at positions [t0, t1) of the layout.
// kDpp: the DPP form of the row subtraction (see subtract_lanes).
template <bool kDpp>
__device__ __forceinline__ void wave_task(const int32_t *__restrict__ wrow, const int64_t *__restrict__ wptr,
                                          const double *__restrict__ wdiag, const uint32_t *__restrict__ wcol,
                                          const double *__restrict__ wval, int64_t t0, int64_t t1, const double *b,
                                          double *x, double *ring)
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
            const double p = v * g;
            // (the same in every lane: a scalar loop, see stream_run)
            const int cnt = __builtin_amdgcn_readfirstlane(int(min<int64_t>(64, e1 - base)));
            acc = subtract_lanes<kDpp>(acc, p, 0, cnt);
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
}

// Supersteps [s0, s1) of a wave-core plan.  One superstep per launch needs
// no synchronisation (claim = nullptr); several run as in trsv_persistent
// (counted completion, robbing of workgroups that have not started), so no
// co-residency is needed.  The i-th wave of workgroup g is slot i G + g
// (tasks of a superstep sorted longest first).  kDpp: the DPP form of the
// row subtraction (see subtract_lanes), for systems of long rows.
template <bool kDpp>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_num_sgpr(kWaveSgprs))) void trsv_wave(
    const int32_t *__restrict__ wrow, const int64_t *__restrict__ wptr, const double *__restrict__ wdiag,
    const uint32_t *__restrict__ wcol, const double *__restrict__ wval, const int64_t *__restrict__ wtask,
    const int32_t *__restrict__ wsuper, int32_t s0, int32_t s1, const double *b, double *x, uint32_t *bar,
    uint32_t *alive, uint32_t *claim, int32_t *err, int64_t spin_limit, int64_t steal_ticks, int64_t delay_ticks)
{
    __shared__ double ring[kWavesPerBlock][kWaveRing];
    __shared__ uint32_t s_done;
    const int32_t waves = int32_t(gridDim.x) * kWavesPerBlock;
    const int32_t slot = int32_t(threadIdx.x >> 6) * int32_t(gridDim.x) + int32_t(blockIdx.x);
    double *my_ring = ring[threadIdx.x >> 6];
    auto run_task = [&](int32_t t) { wave_task<kDpp>(wrow, wptr, wdiag, wcol, wval, wtask[t], wtask[t + 1], b, x, my_ring); };
    if (!claim) {   // one superstep, no other workgroup to wait for
        for (int32_t t = wsuper[s0] + slot; t < wsuper[s0 + 1]; t += waves) run_task(t);
        return;
    }
    if (threadIdx.x == 0) s_done = 0;
    const BspStart bs = bsp_start(bar, alive, delay_ticks);
    bool claiming = bs.robbed;
    for (int32_t s = s0 + bs.first; s < s1; s++) {
        const int32_t t0 = wsuper[s];
        const uint32_t m = uint32_t(wsuper[s + 1] - t0);
        uint32_t mine = 0;
        for (int32_t t = t0 + slot; t < wsuper[s + 1]; t += waves)
            if (!claiming || claim_item(claim, t, bs.epoch)) {
                run_task(t);
                mine++;
            }
        claiming = false;
        bsp_count_own(bar, bs.epoch, s - s0, m, mine, &s_done);
        if (!bsp_wait(bar, bs.epoch, s - s0, err, spin_limit, steal_ticks,
                      [&](int32_t ss) { steal_items(bar, alive, claim, bs.epoch, ss, t0, m, run_task); }))
            return;
    }
}
template __global__ void trsv_wave<false>(const int32_t *, const int64_t *, const double *, const uint32_t *,
                                          const double *, const int64_t *, const int32_t *, int32_t, int32_t,
                                          const double *, double *, uint32_t *, uint32_t *, uint32_t *, int32_t *,
                                          int64_t, int64_t, int64_t);
template __global__ void trsv_wave<true>(const int32_t *, const int64_t *, const double *, const uint32_t *,
                                         const double *, const int64_t *, const int32_t *, int32_t, int32_t,
                                         const double *, double *, uint32_t *, uint32_t *, uint32_t *, int32_t *,
                                         int64_t, int64_t, int64_t);

// ---------------------------------------------------------------------------
// Per-wave record streams (semi-asynchronous wave cores; layout in wave.h).
// Tasks are numbered superstep by superstep; wave slot v (the i-th wave of
// workgroup g is v = 4 g + i) runs tasks v, v + W, v + 2W, ... (W waves)
// and waits only for the values it gathers.  Slot v's stream holds the rows
// of those tasks one after another as records: a header slot (word HDR |
// row, INTL set on a task's first row; value the diagonal) and then the
// row's off-diagonal entries in stored order (word the column, or INTL |
// distance to one of the task's last kWaveRing rows; value A_ij).  A wave
// reads its stream as 64-slot windows: one load brings a short row's header
// and entries, and often the next rows' too, so a row waits for its gathers
// only.  Per row the operations and their order are those of wave_task
// (Eq. (2.1)).
// ---------------------------------------------------------------------------

// Loads need no branch and no select on their result (either makes the
// compiler wait for every load in flight at once): every slot's stream ends
// with a PAD word, and the arrays hold kStreamPad PAD slots past the last
// stream, so any window a wave reads is in bounds, and lanes past its
// stream's PAD (the next slot's records) are never used.
__device__ __forceinline__ void stream_load(const uint32_t *__restrict__ scol, const double *__restrict__ sval,
                                            int64_t o, uint32_t &w, double &v)
{
    const int64_t e = o + (threadIdx.x & 63);
    w = scol[e];
    v = sval[e];
}

// b_i for a header, x_j for an entry whose column is read from memory; any
// other lane loads b[0] and its value is not used (ring entries are read
// at their row's turn).
__device__ __forceinline__ double stream_gather(uint32_t w, const double *b, const double *x)
{
    const bool hdr = (w & HDR) && w != PAD;
    const bool mem = (w & (HDR | INTL)) == 0;
    return load_x(hdr ? b + (w & MASK) : (mem ? x + w : b));   // b is not written during the solve
}

// First lane >= l (l <= 64) whose bit is set in m, else 64.
__device__ __forceinline__ int first_from(unsigned long long m, int l)
{
    const unsigned long long r = l >= 64 ? 0ull : (m >> l) << l;
    return r ? __builtin_ctzll(r) : 64;
}

// Records of [o, end) of a stream, o at the first record of task t and end
// at a header or at the stream's PAD.  Returns kReady at `end`; kAbandon or
// kFailed from a wait, with (o, t) set to the first record of the task
// being run and its number (that task is run again from its start: the
// ring holds rows of the running task only).  The stream is read in chunks
// of kStreamSub 64-slot windows: a chunk's words and values arrive while
// the chunk before it is worked on; its gathers are issued together and
// waited for together, and the next chunk's loads go out behind them.
template <bool kDpp>
__device__ __forceinline__ int stream_run(const uint32_t *__restrict__ scol, const double *__restrict__ sval,
                                          int64_t &o, int64_t end, int32_t &t, int32_t W, const double *b, double *x,
                                          double *ring, int32_t *err, int64_t spin_limit, const AsyncRob &rob)
{
    constexpr int kMore = 3;   // the window is used up, the stream goes on
    const int lane = threadIdx.x & 63;
    // the row being worked on (open) and the task bookkeeping
    bool open = false;
    uint32_t hw = 0;
    double diag = 0.0, acc = 0.0;
    int32_t q = -1;        // the row's position within its task
    int32_t tt = t - W;    // task of the last task-first header seen
    int64_t task_o = o;
    // rows of window [wb, wb + 64) whose words, values and gathers are wc, vc, gc
    auto step = [&](const uint32_t wc, const double vc, double gc, const int64_t wb) -> int {
        const unsigned long long stop = __ballot((wc & HDR) != 0);   // headers and PAD
        int l = 0;
        for (;;) {
            if (open) {
                // the row's entries here are lanes [l, e); both are the same
                // in every lane, which the compiler is told so that the
                // subtraction loop below runs on scalar registers
                l = __builtin_amdgcn_readfirstlane(l);
                const int e = __builtin_amdgcn_readfirstlane(first_from(stop, l));
                const bool in = lane >= l && lane < e;
                const bool ring_in = in && (wc & INTL);
                if (__ballot(ring_in)) {
                    if (ring_in) gc = ring[(q - int32_t(wc & MASK)) & (kWaveRing - 1)];
                }
                bool miss = in && unready(wc, gc);
                if (__ballot(miss)) {
                    int64_t since = -1;   // wall clock at the first rob check
                    for (int64_t spins = 1;; spins++) {
                        __builtin_amdgcn_s_sleep(1);
                        if (miss) {
                            gc = load_x(x + wc);
                            miss = unready(wc, gc);
                        }
                        if (__ballot(miss) == 0ull) break;
                        int r = kReady;
                        if (spins > spin_limit) {
                            if (lane == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            r = kFailed;
                        } else if ((spins & 255) == 0) {
                            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                                r = kFailed;
                            } else if (rob.alive) {
                                const int64_t now = int64_t(wall_clock64());
                                if (since < 0) {
                                    since = now;
                                } else if (now - since > rob.rob_ticks) {
                                    if (any_not_started(rob)) r = kAbandon;
                                    since = now;
                                }
                            }
                        }
                        if (r != kReady) return r;
                    }
                }
                acc = subtract_lanes<kDpp>(acc, vc * gc, l, e);
                if (e == 64) return kMore;   // the row goes on in the next window
                const double y = acc / diag;
                if (lane == 0) {
                    ring[q & (kWaveRing - 1)] = y;
                    store_x(x + (hw & MASK), y);
                }
                __builtin_amdgcn_wave_barrier();
                open = false;
                l = e;
            }
            if (l == 64) return kMore;
            // a header (or the end) at lane l
            if (wb + l >= end) return kReady;
            hw = uint32_t(__builtin_amdgcn_readlane(int(wc), l));
            diag = readlane_f64(vc, l);
            acc = readlane_f64(gc, l);
            if (hw & INTL) {
                tt += W;
                task_o = wb + l;
                q = 0;
            } else {
                q++;
            }
            open = true;
            l++;
        }
    };
    int64_t cb = o;   // first slot of the chunk
    uint32_t w[kStreamSub];
    double v[kStreamSub];
#pragma unroll
    for (int j = 0; j < kStreamSub; j++) stream_load(scol, sval, cb + 64 * j, w[j], v[j]);
    int r;
    for (;;) {
        double g[kStreamSub];
#pragma unroll
        for (int j = 0; j < kStreamSub; j++) g[j] = stream_gather(w[j], b, x);
        uint32_t wn[kStreamSub];
        double vn[kStreamSub];
#pragma unroll
        for (int j = 0; j < kStreamSub; j++) stream_load(scol, sval, cb + kStreamChunk + 64 * j, wn[j], vn[j]);
        r = kMore;
#pragma unroll 1
        for (int j = 0; j < kStreamSub && r == kMore; j++) {
            // window j of the chunk, picked by selects (no copy of a register
            // whose load is in flight)
            uint32_t wc = w[0];
            double vc = v[0], gc = g[0];
#pragma unroll
            for (int i = 1; i < kStreamSub; i++) {
                wc = j == i ? w[i] : wc;
                vc = j == i ? v[i] : vc;
                gc = j == i ? g[i] : gc;
            }
            r = step(wc, vc, gc, cb + 64 * j);
        }
        if (r != kMore) break;
#pragma unroll
        for (int j = 0; j < kStreamSub; j++) {
            w[j] = wn[j];
            v[j] = vn[j];
        }
        cb += kStreamChunk;
    }
    if (r == kReady) {
        o = end;
        t = tt;
    } else {
        o = task_o;
        t = tt;
    }
    return r;
}

// Semi-asynchronous wave cores over per-wave record streams: slot v's
// records are [sbeg[v], sbeg[v + 1] - 1), its PAD at sbeg[v + 1] - 1; task
// t's first record is at stask[t]; the grid is the one the streams were
// built for (W = 4 x grid).  Progress: the earliest unfinished task depends
// only on earlier tasks, which are finished or running, and its wave has
// finished its own earlier tasks.  Waves blocked for long while some
// workgroup has not started rob that workgroup's tasks in order (see
// trsv_async); a robbed task runs from stask[k] to the first record of its
// slot's next task.  kDpp: the DPP form of the row subtraction (see
// subtract_lanes), for systems of long rows.
template <bool kDpp>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_num_sgpr(kStreamSgprs))) void trsv_stream_async(
    const uint32_t *__restrict__ scol, const double *__restrict__ sval, const int64_t *__restrict__ sbeg,
    const int64_t *__restrict__ stask, int32_t tasks, const double *b, double *x, int32_t *err,
    int64_t spin_limit, unsigned long long *ticket, uint32_t *alive, unsigned long long *vnext, int64_t rob_ticks,
    int64_t delay_ticks)
{
    __shared__ double ring[kWavesPerBlock][kWaveRing];
    // the robbing context lives in LDS: it is only read on the rare slow
    // path, and keeping it in scalar registers across the subtraction loop
    // costs residency (see kWaveSgprs)
    __shared__ AsyncRob s_rob, s_norob;
    const uint32_t epoch = async_start(ticket, alive, delay_ticks);
    if (threadIdx.x == 0) {
        s_rob = AsyncRob{alive, epoch, rob_ticks};
        s_norob = AsyncRob{nullptr, 0u, 0};
    }
    __syncthreads();
    const int32_t W = int32_t(gridDim.x) * kWavesPerBlock;
    const int32_t v = int32_t(blockIdx.x) * kWavesPerBlock + int32_t(threadIdx.x >> 6);
    double *my_ring = ring[threadIdx.x >> 6];
    const int64_t mine_end = sbeg[v + 1] - 1;
    int64_t o = sbeg[v];
    int32_t t = v;
    // one call site of the row loop: a robbed task runs in the turn after
    // the own stream was abandoned, the abandoned task again after it
    int64_t ro = -1, rend = 0;
    int32_t rt = 0;
    for (;;) {
        const bool robbed = ro >= 0;
        if (!robbed && o >= mine_end) return;
        int64_t oo = robbed ? ro : o;
        int32_t tt = robbed ? rt : t;
        const int r = stream_run<kDpp>(scol, sval, oo, robbed ? rend : mine_end, tt, W, b, x, my_ring, err, spin_limit,
                                 robbed ? s_norob : s_rob);
        if (r == kFailed) return;   // a wait ran out: *err is set, the other waves leave too
        if (robbed) {
            ro = -1;   // (a robbed task is never abandoned)
            continue;
        }
        o = oo;
        t = tt;
        if (r == kReady) return;
        const int64_t k = rob_item(s_rob, vnext, tasks, t);
        if (k >= 0) {
            ro = stask[k];
            rt = int32_t(k);
            rend = k + W < tasks ? stask[k + W] : sbeg[(k % W) + 1] - 1;
        }
    }
}
template __global__ void trsv_stream_async<false>(const uint32_t *, const double *, const int64_t *, const int64_t *,
                                                  int32_t, const double *, double *, int32_t *, int64_t,
                                                  unsigned long long *, uint32_t *, unsigned long long *, int64_t,
                                                  int64_t);
template __global__ void trsv_stream_async<true>(const uint32_t *, const double *, const int64_t *, const int64_t *,
                                                 int32_t, const double *, double *, int32_t *, int64_t,
                                                 unsigned long long *, uint32_t *, unsigned long long *, int64_t,
                                                 int64_t);

// ---------------------------------------------------------------------------
// Semi-asynchronous solve: no barriers.  Chunks are numbered superstep by
// superstep and run with per-row readiness (await_batch): a lane gathering
// a column that still holds the not-computed mark reads it again.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void fill_unready(unsigned long long *x, int64_t n)
{
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) x[i] = kUnready;
}

// Static order with robbing.  Wave w (w = 4 g + i for the i-th wave of
// workgroup g: neighbouring chunks on one CU, as their gathers overlap) runs
// chunks w, w + W, w + 2W, ... in order (W waves), so every wave is only a
// little ahead of the others and no claims are made.  The earliest
// unfinished chunk depends only on finished chunks and its wave has finished
// its earlier ones, so the solve advances as long as that wave runs -- which
// needs every workgroup to have started.  Other work on the device can keep
// workgroups from starting, so a wave that has waited rob_ticks for values
// while some workgroup has not started abandons its chunk (the rows it
// stored are final: every x_i has one value, so running a chunk again
// stores the same bits), runs the earliest chunk of a not-started workgroup
// that no one has taken yet if that chunk comes before its own (taking it
// by advancing that wave's robbed-prefix word), and then runs its own chunk
// again.  A robbed chunk depends only on chunks before it, which are done or
// running, so it completes; the solve therefore advances whenever any
// workgroup runs.  A late workgroup runs all of its chunks (robbed ones a
// second time, with the same bits).
__global__ __launch_bounds__(kBlock) void trsv_async(const uint32_t *__restrict__ word,
                                                     const double *__restrict__ value,
                                                     const int64_t *__restrict__ chunk_base,
                                                     const int32_t *__restrict__ chunk_len, int32_t chunks,
                                                     const double *b, double *x, int32_t *err, int64_t spin_limit,
                                                     unsigned long long *ticket, uint32_t *alive,
                                                     unsigned long long *vnext, int64_t rob_ticks, int64_t delay_ticks)
{
    __shared__ double ring[kRing + 1][kBlock];
    const int lane = threadIdx.x & 63;
    const AsyncRob rob = {alive, async_start(ticket, alive, delay_ticks), rob_ticks};
    const int32_t W = int32_t(gridDim.x) * kWavesPerBlock;
    auto run_chunk = [&](int32_t c, AsyncRob r) {
        const LaneCursor cur = make_cursor(word, value, chunk_base[c], chunk_len[c], lane);
        Batch<kUnroll> b0, b1;
        load_batch(cur, 0, b0);
        load_batch(cur, kUnroll, b1);
        return run_lane<kUnroll, true>(cur, b0, b1, b, x, ring, err, spin_limit, r);
    };
    for (int32_t c = int32_t(blockIdx.x) * kWavesPerBlock + int32_t(threadIdx.x >> 6); c < chunks;) {
        if (run_chunk(c, rob)) {
            c += W;
            continue;
        }
        const int64_t r = rob_item(rob, vnext, chunks, c);
        if (r >= 0) run_chunk(int32_t(r), no_rob());
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
__device__ __forceinline__ int await_multi(const Batch<kUnrollWide> &B, double (&g)[kUnrollWide][R], const double *x,
                                           int64_t ld, int32_t *err, int64_t spin_limit, AsyncRob rob)
{
    bool miss = false;
#pragma unroll
    for (int j = 0; j < kUnrollWide; j++)
#pragma unroll
        for (int r = 0; r < R; r++) miss |= unready(B.w[j], g[j][r]);
    if (__ballot(miss) == 0ull) return kReady;
    int64_t since = -1;   // wall clock at the first rob check
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
        if (__ballot(miss) == 0ull) return kReady;
        if (spins > spin_limit) {
            if ((threadIdx.x & 63) == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return kFailed;
        }
        if ((spins & 255) == 0) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return kFailed;
            if (rob.alive) {
                const int64_t now = int64_t(wall_clock64());
                if (since < 0) {
                    since = now;
                } else if (now - since > rob.rob_ticks) {
                    if (any_not_started(rob)) return kAbandon;
                    since = now;
                }
            }
        }
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
__device__ __forceinline__ bool run_lane_multi(const LaneCursor &cur, const double *b, double *x, int64_t ld,
                                               MultiRing<R> ring, int32_t *err, int64_t spin_limit, AsyncRob rob)
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
        if (await_multi<R>(now, gnow, x, ld, err, spin_limit, rob) == kAbandon) return false;
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
    return true;
}

// Static order with robbing, as trsv_async; one wave per workgroup (wave g
// runs chunks g, g + G, ...), whose R-column ring fills a quarter of the
// LDS at R = 4.
template <int R>
__global__ __launch_bounds__(64) void trsv_async_multi(const uint32_t *__restrict__ word,
                                                           const double *__restrict__ value,
                                                           const int64_t *__restrict__ chunk_base,
                                                           const int32_t *__restrict__ chunk_len, int32_t chunks,
                                                           const double *b, double *x, int64_t ld, int32_t *err,
                                                           int64_t spin_limit, unsigned long long *ticket,
                                                           uint32_t *alive, unsigned long long *vnext,
                                                           int64_t rob_ticks, int64_t delay_ticks)
{
    __shared__ double ring[kRing + 1][R][64];
    const int lane = threadIdx.x & 63;
    const AsyncRob rob = {alive, async_start(ticket, alive, delay_ticks), rob_ticks};
    const int32_t W = int32_t(gridDim.x);
    auto run_chunk = [&](int32_t c, AsyncRob r) {
        const LaneCursor cur = make_cursor(word, value, chunk_base[c], chunk_len[c], lane);
        return run_lane_multi<R>(cur, b, x, ld, ring, err, spin_limit, r);
    };
    for (int32_t c = int32_t(blockIdx.x); c < chunks;) {
        if (run_chunk(c, rob)) {
            c += W;
            continue;
        }
        const int64_t r = rob_item(rob, vnext, chunks, c);
        if (r >= 0) run_chunk(int32_t(r), no_rob());
    }
}

template __global__ void trsv_async_multi<1>(const uint32_t *, const double *, const int64_t *, const int32_t *,
                                             int32_t, const double *, double *, int64_t, int32_t *, int64_t,
                                             unsigned long long *, uint32_t *, unsigned long long *, int64_t, int64_t);
template __global__ void trsv_async_multi<2>(const uint32_t *, const double *, const int64_t *, const int32_t *,
                                             int32_t, const double *, double *, int64_t, int32_t *, int64_t,
                                             unsigned long long *, uint32_t *, unsigned long long *, int64_t, int64_t);
template __global__ void trsv_async_multi<4>(const uint32_t *, const double *, const int64_t *, const int32_t *,
                                             int32_t, const double *, double *, int64_t, int32_t *, int64_t,
                                             unsigned long long *, uint32_t *, unsigned long long *, int64_t, int64_t);

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

// Semi-asynchronous batches of wavefront-core systems run as one system: the
// systems' b are copied into one vector, their rows and columns shifted by
// the system's first row there (off[i]), and trsv_stream_async runs over a
// stream of the batch's global task order; x is copied back at the end.
// stream_rebase copies task g (task gtask[g] of system gsys[g]) from that
// system's own stream to boff[g] of the batch stream, one wave per task.
__global__ __launch_bounds__(kBlock) void stream_rebase(const StreamSrc *__restrict__ src,
                                                        const int32_t *__restrict__ gsys,
                                                        const int32_t *__restrict__ gtask,
                                                        const int64_t *__restrict__ boff,
                                                        const int64_t *__restrict__ bsize, int64_t ntasks,
                                                        uint32_t *__restrict__ scol, double *__restrict__ sval)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = int64_t(gridDim.x) * kWavesPerBlock;
    for (int64_t g = int64_t(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6); g < ntasks; g += waves) {
        const StreamSrc S = src[gsys[g]];
        const int64_t from = S.stask[gtask[g]], to = boff[g], len = bsize[g];
        const uint32_t off = uint32_t(S.off);
        for (int64_t k = lane; k < len; k += 64) {
            uint32_t w = S.scol[from + k];
            if (w & HDR)
                w = (w & (HDR | INTL)) | ((w & MASK) + off);   // a row header
            else if (!(w & INTL))
                w += off;                                     // a column read from memory
            scol[to + k] = w;
            sval[to + k] = S.sval[from + k];
        }
    }
}

// b of system blockIdx.y into cat[off[y] ...] (in = true), or cat back into
// its x (in = false).
__global__ __launch_bounds__(kBlock) void batch_concat(const SysDesc *__restrict__ sys,
                                                       const int64_t *__restrict__ off, double *cat, bool in)
{
    const SysDesc &d = sys[blockIdx.y];
    const int64_t o = off[blockIdx.y];
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < d.n; i += stride) {
        if (in)
            cat[o + i] = d.b[i];
        else
            d.x[i] = cat[o + i];
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
