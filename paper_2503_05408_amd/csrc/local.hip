// Single-workgroup execution (the layout is described in local.h): one
// computing wave whose lanes are the BSP cores, and one helper wave that
// moves data between global memory and LDS.
#include <hip/hip_runtime.h>

#include "local.h"
#include "internal.h"

#pragma clang fp contract(off)

namespace gltrsv {
namespace dev {

namespace {

constexpr int kStaged = 0, kComputed = 1, kDrained = 2, kAbort = 3;
// records whose copy the helper keeps in flight ahead of the staged ones
constexpr int kCopyAhead = 4;

__device__ __forceinline__ double load_xg(const double *p)
{
    const unsigned long long u =
        __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double(static_cast<long long>(u));
}

__device__ __forceinline__ void store_xg(double *p, double v)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                       static_cast<unsigned long long>(__double_as_longlong(v)), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t ctl_load(const uint32_t *c)
{
    return __hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Makes every earlier access of the wave complete (global stores, copies
// into LDS, LDS writes), then publishes v.
__device__ __forceinline__ void ctl_publish(uint32_t *c, uint32_t v)
{
    __builtin_amdgcn_s_waitcnt(0);
    __hip_atomic_store(c, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void local_abort(uint32_t *ctl, int32_t *err, int32_t code = 1)
{
    __hip_atomic_store(&ctl[kAbort], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_store(err, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until ctl[i] >= target; false after spin_limit polls or an abort.
__device__ __forceinline__ bool ctl_wait(uint32_t *ctl, int i, uint32_t target, int32_t *err, int64_t spin_limit)
{
    for (int64_t spins = 0;; spins++) {
        if (ctl_load(&ctl[i]) >= target) return true;
        if (ctl_load(&ctl[kAbort])) return false;
        if (spins >= spin_limit) {
            local_abort(ctl, err);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

typedef __attribute__((address_space(3))) void lds_void;

// Slot s (one binary64) lives in LDS words slot_word(s) (low half) and
// slot_word(s) + 64 (high half); see local.h.
__device__ __forceinline__ uint32_t slot_word(uint32_t s) { return s + (s & ~63u); }

__device__ __forceinline__ double read_slot(const uint32_t *w, uint32_t s)
{
    const uint32_t i = slot_word(s);
    return __hiloint2double(int(w[i + 64]), int(w[i]));
}

__device__ __forceinline__ void write_slot(uint32_t *w, uint32_t s, double v)
{
    const uint32_t i = slot_word(s);
    w[i] = uint32_t(__double2loint(v));
    w[i + 64] = uint32_t(__double2hiint(v));
}

struct GroupData {
    double2 v01, v23;
    uint2 o;
};

__device__ __forceinline__ GroupData read_group(const char *gp, int lane)
{
    GroupData d;
    d.v01 = *reinterpret_cast<const double2 *>(gp + 16 * lane);
    d.v23 = *reinterpret_cast<const double2 *>(gp + 1024 + 16 * lane);
    d.o = *reinterpret_cast<const uint2 *>(gp + 2048 + 8 * lane);
    return d;
}

// The computing wave: every group of every record, in order.  The next
// group's values and operand slots are read before the current group's
// division (they are record bytes, which no result overwrites).
__device__ __forceinline__ void local_compute(uint32_t *ldsw, uint32_t *ctl, int32_t nrec, int32_t *err,
                                              int64_t spin_limit)
{
    const int lane = threadIdx.x;
    const char *fifo = reinterpret_cast<const char *>(ldsw + 2 * kLocalFifoSlot0);
    double acc = 0.0, diag = 1.0;
    uint32_t off = 0, ring = 0;
    for (int32_t t = 0; t < nrec; t++) {
        if (!ctl_wait(ctl, kStaged, uint32_t(t) + 1, err, spin_limit)) return;
        const LocalHdr *h = reinterpret_cast<const LocalHdr *>(fifo + off);
        const uint32_t ng = h->ngroups, next = h->next_off;
        if (ng > uint32_t(kLocalRingGroups) || next >= uint32_t(kLocalFifoBytes) || (next & uint32_t(kLocalAlign - 1)) ||
            off + kLocalHdrBytes + ng * uint32_t(kLocalGroupBytes) > uint32_t(kLocalFifoBytes)) {
            local_abort(ctl, err, 2);
            return;
        }
        if (!ctl_wait(ctl, kDrained, h->need_drain, err, spin_limit)) return;
        const char *gp = fifo + off + kLocalHdrBytes;
        GroupData nx = read_group(gp, lane);
        for (uint32_t i = 0; i < ng; i++) {
            const GroupData g = nx;
            gp += kLocalGroupBytes;
            if (i + 1 < ng) nx = read_group(gp, lane);
            const uint32_t o0 = g.o.x & 0xFFFFu, o1 = g.o.x >> 16, o2 = g.o.y & 0xFFFFu, o3 = g.o.y >> 16;
            const double x0 = read_slot(ldsw, o0 & kLocalSlotMask);
            const double x1 = read_slot(ldsw, o1 & kLocalSlotMask);
            const double x2 = read_slot(ldsw, o2);
            const double x3 = read_slot(ldsw, o3);
            const bool start = (o0 & kLocalStartBit) != 0;
            const bool end = (o1 & kLocalEndBit) != 0;
            // Eq. (2.1): a header sets acc = b_i and takes the diagonal;
            // every other entry subtracts its product
            double a = start ? x0 : acc - g.v01.x * x0;
            diag = start ? g.v01.x : diag;
            a = a - g.v01.y * x1;
            a = a - g.v23.x * x2;
            a = a - g.v23.y * x3;
            acc = a;
            if (__ballot(end)) write_slot(ldsw, ring * 64 + lane, a / diag);
            ring = ring + 1 == uint32_t(kLocalRingGroups) ? 0u : ring + 1;
        }
        ctl_publish(&ctl[kComputed], uint32_t(t) + 1);
        off = next;
    }
}

// Publishes v once the wave's LDS accesses are done, without waiting for
// its global stores (only LDS slots are handed over).
__device__ __forceinline__ void ctl_publish_lds(uint32_t *c, uint32_t v)
{
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0), vmcnt and expcnt left running
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __hip_atomic_store(c, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

constexpr int kDrainU = 8;            // drains per lane per batch
constexpr int kFillBlocks = 8;        // blocks of 64 fills issued per helper iteration
constexpr uint32_t kNoRow = 0xFFFFFFFFu;

// The helper wave, a pipeline with one wait per iteration.  At the top it
// waits for everything issued in the previous iteration (record copies,
// fill copies, drain stores); then it publishes the records whose fills
// have landed, drains the records computed since, reads the fill entries
// of records whose copy has landed (up to kFillBlocks blocks of 64) and
// then issues their fills (two four-byte copies per block, into the split
// slots), and issues the copies of the next records (kCopyAhead ahead of
// the staged ones, each once the records whose FIFO bytes it reuses are
// computed).  Every LDS read of an iteration comes before its first copy
// into LDS: a read after such a copy waits for it (the compiler cannot
// tell the two apart), which would serialise the pipeline.  The FIFO
// offsets of the records in flight are kept in lanes (record r in lane
// r mod 64), not in LDS.  Far fills read x only from records drained
// before the previous wait, so those stores have completed.  Rows read
// from a record are checked against n before they are used; a bad record
// ends the solve with the error word set to 2.
__device__ __forceinline__ void local_helper(uint32_t *ldsw, uint32_t *ctl, const uint8_t *rec, const LocalRec *info,
                                             int32_t nrec, int64_t n, const double *b, double *x, int32_t *err,
                                             int64_t spin_limit)
{
    const int lane = threadIdx.x - 64;
    const uint32_t n32 = uint32_t(n);   // n < 2^30
    char *fifo = reinterpret_cast<char *>(ldsw + 2 * kLocalFifoSlot0);
    const uint32_t fifo_byte0 = uint32_t(kLocalFifoSlot0) * 8;
    int32_t staged = 0, filled = 0, issued = 0, drained = 0;
    uint32_t fblock = 0;       // next fill block of record `filled`
    uint64_t src = 0;          // byte offset of record `issued` in rec
    int64_t idle = 0;
    uint32_t off_v = 0, fill_v = 0;   // lane r mod 64: FIFO offset / first fill byte of record r
    uint4 win = make_uint4(0u, 0u, 0u, 0u);   // lane l: info[wb + l]
    int32_t wb = -64;
    while (drained < nrec) {
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const int32_t landed = issued, safe = drained;
        bool busy = false;
        if (issued < nrec && issued >= wb + 64) {   // next 64 records' copy data (waits once per 64)
            wb = issued & ~63;
            if (wb + lane < nrec) win = *reinterpret_cast<const uint4 *>(info + wb + lane);
            __builtin_amdgcn_s_waitcnt(0);
        }
        // 1. records whose fills were issued last time are complete
        if (filled != staged) {
            staged = filled;
            ctl_publish_lds(&ctl[kStaged], uint32_t(staged));
            busy = true;
        }
        // 2. drains
        const int32_t comp = int32_t(ctl_load(&ctl[kComputed]));
        if (comp > drained) {
            bool bad = false;
            for (int32_t r = drained; r < comp; r++) {
                const char *hp = fifo + uint32_t(__builtin_amdgcn_readlane(int(off_v), r & 63));
                const LocalHdr *h = reinterpret_cast<const LocalHdr *>(hp);
                const uint32_t nd = h->ndrain;
                const uint2 *dl = reinterpret_cast<const uint2 *>(hp + kLocalHdrBytes + size_t(h->ngroups) * kLocalGroupBytes +
                                                                  size_t(h->nfill) * 8);
                // branch-free reads (indices clamped into range), then the stores
                for (uint32_t base = 0; base < nd; base += 64 * kDrainU) {
                    double dv[kDrainU];
                    uint32_t drow[kDrainU];
#pragma unroll
                    for (int j = 0; j < kDrainU; j++) {
                        const uint32_t e = base + uint32_t(j * 64 + lane);
                        const uint2 d = dl[min(e, nd - 1)];
                        const bool ok = d.x < uint32_t(kLocalRingSlots) && d.y < n32;
                        bad |= e < nd && !ok;
                        drow[j] = (e < nd && ok) ? d.y : kNoRow;
                        dv[j] = read_slot(ldsw, min(d.x, uint32_t(kLocalRingSlots - 1)));
                    }
#pragma unroll
                    for (int j = 0; j < kDrainU; j++)
                        if (drow[j] != kNoRow) store_xg(x + drow[j], dv[j]);
                }
            }
            if (__ballot(bad)) {
                local_abort(ctl, err, 2);
                return;
            }
            drained = comp;
            ctl_publish_lds(&ctl[kDrained], uint32_t(comp));
            busy = true;
        }
        // 3. fills of landed records: read the entries of up to kFillBlocks
        // blocks, then issue their copies
        uint2 fe[kFillBlocks];
        uint32_t fdst[kFillBlocks];
        bool fact[kFillBlocks];
        bool bad = false;
        int32_t fill_to = filled;
        uint32_t nf = 0;
        const uint2 *fl = nullptr;
        bool have = false;   // nf / fl describe record fill_to
#pragma unroll
        for (int j = 0; j < kFillBlocks; j++) {
            fact[j] = false;
            fdst[j] = 0;
            fe[j] = make_uint2(0u, 0u);
            while (fill_to < landed) {
                if (!have) {
                    const char *hp = fifo + uint32_t(__builtin_amdgcn_readlane(int(off_v), fill_to & 63));
                    const LocalHdr *h = reinterpret_cast<const LocalHdr *>(hp);
                    if (h->ngroups > uint32_t(kLocalRingGroups) || uint64_t(h->nfill) + h->ndrain > uint64_t(kLocalFifoBytes / 8)) {
                        bad = true;
                        break;
                    }
                    if (uint32_t(safe) < h->need_far) break;   // its far rows are not all in x yet
                    nf = h->nfill;
                    fl = reinterpret_cast<const uint2 *>(hp + kLocalHdrBytes + size_t(h->ngroups) * kLocalGroupBytes);
                    have = true;
                }
                if (fblock * 64 < nf) break;
                fill_to++;        // every block of this record is issued
                fblock = 0;
                have = false;
            }
            if (!have || bad || fblock * 64 >= nf) continue;
            const uint32_t i = fblock * 64 + uint32_t(lane);
            fe[j] = fl[min(i, nf - 1)];
            bad |= i < nf && fe[j].y >= n32;
            if (i >= nf) fe[j] = make_uint2(0u, 0u);   // b[0], into an unused slot
            fdst[j] = uint32_t(__builtin_amdgcn_readlane(int(fill_v), fill_to & 63)) + fblock * uint32_t(kLocalAlign);
            fact[j] = true;
            fblock++;
        }
        if (have && fblock * 64 >= nf) {   // the last block read completes its record
            fill_to++;
            fblock = 0;
        }
        if (__ballot(bad)) {
            local_abort(ctl, err, 2);
            return;
        }
#pragma unroll
        for (int j = 0; j < kFillBlocks; j++) {
            if (!fact[j]) continue;
            const double *from = ((fe[j].x & kLocalFillX) ? x : b) + fe[j].y;
            const uint32_t *w = reinterpret_cast<const uint32_t *>(from);
            char *dst = reinterpret_cast<char *>(ldsw) + fdst[j];
            __builtin_amdgcn_global_load_lds(w, (lds_void *)dst, 4, 0, 0);
            __builtin_amdgcn_global_load_lds(w + 1, (lds_void *)(dst + 256), 4, 0, 0);
            busy = true;
        }
        if (fill_to != filled) {
            filled = fill_to;
            busy = true;
        }
        // 4. copies of the next records (no LDS reads from here on)
        while (issued < nrec && issued - staged < kCopyAhead && issued < wb + 64) {
            const int l = issued - wb;
            const uint32_t bytes = uint32_t(__builtin_amdgcn_readlane(int(win.x), l));
            const uint32_t foff = uint32_t(__builtin_amdgcn_readlane(int(win.y), l));
            const uint32_t wait = uint32_t(__builtin_amdgcn_readlane(int(win.z), l));
            if (uint32_t(comp) < wait) break;   // its FIFO bytes are still in use
            const uint32_t fill_off = foff + ((bytes + kLocalAlign - 1) & ~uint32_t(kLocalAlign - 1));
            if (fill_off > uint32_t(kLocalFifoBytes) || (foff & uint32_t(kLocalAlign - 1)) || (bytes & 15u)) {
                local_abort(ctl, err, 2);
                return;
            }
            off_v = lane == (issued & 63) ? foff : off_v;
            fill_v = lane == (issued & 63) ? fifo_byte0 + fill_off : fill_v;
            const uint8_t *from = rec + src;
            char *to = fifo + foff;
            for (uint32_t o = 0; o < bytes; o += 1024) {
                if (o + 16 * uint32_t(lane) < bytes)
                    __builtin_amdgcn_global_load_lds(from + o + 16 * lane, (lds_void *)(to + o), 16, 0, 0);
            }
            src += bytes;
            issued++;
            busy = true;
        }
        if (busy) {
            idle = 0;
            continue;
        }
        if (ctl_load(&ctl[kAbort])) return;
        if (++idle >= spin_limit) {
            local_abort(ctl, err);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

__device__ __forceinline__ void local_run(const uint8_t *rec, const LocalRec *info, int32_t nrec, int64_t n,
                                          const double *b, double *x, int32_t *err, int64_t spin_limit)
{
    __shared__ __align__(16) uint32_t ldsw[2 * kLocalLdsSlots];
    __shared__ uint32_t ctl[4];
    if (threadIdx.x < 4) ctl[threadIdx.x] = 0u;
    if (threadIdx.x == 0) write_slot(ldsw, kLocalZeroSlot, 0.0);
    __syncthreads();
    if (threadIdx.x < 64) local_compute(ldsw, ctl, nrec, err, spin_limit);
    else local_helper(ldsw, ctl, rec, info, nrec, n, b, x, err, spin_limit);
}

}  // namespace

__global__ __launch_bounds__(128) void trsv_local(const uint8_t *rec, const LocalRec *info, int32_t nrec, int64_t n,
                                                  const double *b, double *x, int32_t *err, int64_t spin_limit)
{
    local_run(rec, info, nrec, n, b, x, err, spin_limit);
}

__global__ __launch_bounds__(128) void trsv_local_batched(const LocalSys *sys, int32_t count, int32_t *err,
                                                          int64_t spin_limit)
{
    const LocalSys &s = sys[blockIdx.x];
    local_run(s.rec, s.info, s.nrec, s.n, s.b, s.x, err, spin_limit);
}

}  // namespace dev
}  // namespace gltrsv

// ===========================================================================
using namespace gltrsv;

extern "C" {

int gltrsv_solve_local(gltrsv_plan *p, const double *b, double *x, void *stream)
{
    if (!p || (p->n && (!b || !x))) return set_error(GLTRSV_EINVAL, "null argument");
    if (!p->d_lrec) return set_error(GLTRSV_ENOTSUP, "the plan has no one-workgroup layout (create it with exec_hint 2)");
    if (p->n == 0) return GLTRSV_OK;
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(b), x0 = reinterpret_cast<uintptr_t>(x);
    const uintptr_t len = uintptr_t(p->n) * sizeof(double);
    // in place is fine: b[i] is staged before x[i] is written
    if (b0 != x0 && b0 < x0 + len && x0 < b0 + len) return set_error(GLTRSV_EINVAL, "b and x overlap without being equal");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(dev::trsv_local, dim3(1), dim3(128), 0, st, p->d_lrec, p->d_linfo, p->l_nrec, p->n, b, x,
                       p->d_err, p->spin_limit);
    HIP_TRY(hipGetLastError());
    p->last_stream = st;
    return GLTRSV_OK;
}

int gltrsv_plan_local_size(const gltrsv_plan *p, int64_t *rec_bytes, int64_t *records)
{
    if (!p || !rec_bytes || !records) return set_error(GLTRSV_EINVAL, "null argument");
    if (!p->d_lrec) return set_error(GLTRSV_ENOTSUP, "the plan has no one-workgroup layout");
    *rec_bytes = p->l_bytes;
    *records = p->l_nrec;
    return GLTRSV_OK;
}

int gltrsv_plan_local_records(const gltrsv_plan *p, void *rec, int64_t rec_bytes, uint32_t *info, int64_t records)
{
    if (!p || !rec || !info) return set_error(GLTRSV_EINVAL, "null argument");
    if (!p->d_lrec) return set_error(GLTRSV_ENOTSUP, "the plan has no one-workgroup layout");
    if (rec_bytes != p->l_bytes || records != p->l_nrec)
        return set_error(GLTRSV_EINVAL, "sizes must equal gltrsv_plan_local_size");
    HIP_TRY(hipSetDevice(p->device));
    HIP_TRY(hipMemcpy(rec, p->d_lrec, size_t(rec_bytes), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(info, p->d_linfo, sizeof(LocalRec) * size_t(records), hipMemcpyDeviceToHost));
    return GLTRSV_OK;
}

}  // extern "C"
