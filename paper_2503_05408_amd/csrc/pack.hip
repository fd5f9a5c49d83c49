// Device packing of the lane-interleaved stream (the reorder of Sec. 5 and
// the packed layout the solve kernels read), after the host has laid out
// tasks, chunks and lanes:
//   1. per position t of the schedule order: the row perm[t], its inverse,
//      and its stream length (stored entries of the row);
//   2. an exclusive prefix sum of the lengths: each workgroup stages 2048
//      lengths through LDS, every thread sums 8 consecutive ones, the
//      64-lane wavefronts scan those sums with lane shuffles, and the four
//      wave totals are combined through LDS; one more workgroup scans the
//      workgroup totals;
//   3. the scatter: a row's entries start at (its prefix - the prefix of its
//      task's first row) entries into its lane, so entry j lands at
//      slot(lane) + 64 * (that offset + j).  Words are encoded as the host
//      packer does: header, a column of the same task fewer than kRing rows
//      back as "rows back", any other column as itself.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/gltrsv.h"
#include "analysis.h"
#include "internal.h"

namespace gltrsv {
namespace dev {
namespace {

constexpr int kScanItems = 8;                      // per thread
constexpr int kScanTile = kBlock * kScanItems;     // per workgroup

// perm lists vertices; for an upper-triangular matrix vertex v is row n-1-v.
__global__ __launch_bounds__(kBlock) void pack_rows(const int32_t *__restrict__ perm,
                                                    const int64_t *__restrict__ row_ptr, int64_t n, int32_t upper,
                                                    int32_t *__restrict__ inv, int64_t *__restrict__ len)
{
    const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= n) return;
    const int32_t v = perm[t];
    const int64_t row = upper ? n - 1 - v : v;
    inv[v] = int32_t(t);
    len[t] = row_ptr[row + 1] - row_ptr[row];
}

__device__ __forceinline__ int64_t wave_inclusive_scan(int64_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Exclusive scan of one tile of `data` in place; returns the tile's total
// (valid in every thread).
__device__ __forceinline__ int64_t scan_tile(int64_t *data, int64_t n, int64_t base, int64_t *tile, int64_t *wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const int64_t i = base + int64_t(k) * kBlock + tid;
        tile[k * kBlock + tid] = i < n ? data[i] : 0;
    }
    __syncthreads();
    int64_t own[kScanItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        own[k] = sum;
        sum += tile[tid * kScanItems + k];
    }
    const int64_t incl = wave_inclusive_scan(sum, lane);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int64_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; w++) {
        before += w < wave ? wsum[w] : 0;
        total += wsum[w];
    }
    const int64_t first = before + incl - sum;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) tile[tid * kScanItems + k] = first + own[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const int64_t i = base + int64_t(k) * kBlock + tid;
        if (i < n) data[i] = tile[k * kBlock + tid];
    }
    __syncthreads();   // tile and wsum are reused by the caller's next tile
    return total;
}

__global__ __launch_bounds__(kBlock) void scan_tiles(int64_t *__restrict__ data, int64_t n, int64_t *__restrict__ tops)
{
    __shared__ int64_t tile[kScanTile];
    __shared__ int64_t wsum[kWavesPerBlock];
    const int64_t total = scan_tile(data, n, int64_t(blockIdx.x) * kScanTile, tile, wsum);
    if (threadIdx.x == 0) tops[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the tile totals, tile after tile.
__global__ __launch_bounds__(kBlock) void scan_tops(int64_t *__restrict__ tops, int64_t m)
{
    __shared__ int64_t tile[kScanTile];
    __shared__ int64_t wsum[kWavesPerBlock];
    int64_t carry = 0;
    for (int64_t base = 0; base < m; base += kScanTile) {
        const int64_t total = scan_tile(tops, m, base, tile, wsum);
        for (int64_t i = base + threadIdx.x; i < min(m, base + kScanTile); i += kBlock) tops[i] += carry;
        __syncthreads();
        carry += total;
    }
}

__global__ __launch_bounds__(kBlock) void pack_scatter(
    const int32_t *__restrict__ perm, const int32_t *__restrict__ inv, const int64_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col, const double *__restrict__ val, const int64_t *__restrict__ pre,
    const int64_t *__restrict__ tops, const int64_t *__restrict__ slot, const int32_t *__restrict__ task0, int64_t n,
    int32_t upper, int64_t slots, uint32_t *__restrict__ word, double *__restrict__ value, int32_t *__restrict__ err)
{
    const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= n) return;
    const int32_t v = perm[t];
    const int64_t row = upper ? n - 1 - v : v;
    const int32_t t0 = task0[t];
    const int64_t off = (pre[t] + tops[t / kScanTile]) - (pre[t0] + tops[t0 / kScanTile]);
    // off-diagonals [lo, hi) in stored order, diagonal at dg
    const int64_t lo = upper ? row_ptr[row] + 1 : row_ptr[row];
    const int64_t hi = upper ? row_ptr[row + 1] : row_ptr[row + 1] - 1;
    const int64_t dg = upper ? row_ptr[row] : row_ptr[row + 1] - 1;
    const int64_t base = slot[t] + int64_t(kLanes) * off;
    if (off < 0 || t0 > t || base < 0 || base + int64_t(kLanes) * (hi - lo) >= slots) {
        *err = 1;   // inconsistent layout: write nothing
        return;
    }
    word[base] = kHdrBit | uint32_t(row);
    value[base] = val[dg];
    for (int64_t e = lo; e < hi; e++) {
        const int32_t c = col[e];
        const int32_t ic = inv[upper ? n - 1 - c : c];
        uint32_t w = uint32_t(c);
        // a parent inside the schedule order's task range is in this task
        if (ic >= t0 && t - ic < kRing) w = kIntBit | uint32_t(t - ic);
        const int64_t at = base + int64_t(kLanes) * (1 + e - lo);
        word[at] = w;
        value[at] = val[e];
    }
}

// Device buffers of one packing, released on every exit path.
struct Scratch {
    std::vector<void *> p;
    hipStream_t st = nullptr;
    ~Scratch()
    {
        if (st) (void)hipStreamSynchronize(st);
        for (void *q : p) (void)hipFree(q);
        if (st) (void)hipStreamDestroy(st);
    }
    template <class T>
    hipError_t alloc(T **out, size_t count)
    {
        void *q = nullptr;
        const hipError_t e = hipMalloc(&q, std::max<size_t>(1, count) * sizeof(T));
        if (e == hipSuccess) p.push_back(q);
        *out = static_cast<T *>(q);
        return e;
    }
};

}  // namespace

int device_pack(const CsrView &A, const std::vector<int32_t> &perm, const PackLayout &lay, bool upper,
                uint32_t *d_word, double *d_value)
{
    const int64_t n = A.n, nnz = A.nnz, slots = lay.pk.slots;
    if (n == 0 || slots == 0) return GLTRSV_OK;
    Scratch s;
    HIP_TRY(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
    int64_t *d_rp, *d_pre, *d_tops, *d_slot;
    int32_t *d_col, *d_perm, *d_inv, *d_t0, *d_err;
    double *d_val;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    HIP_TRY(s.alloc(&d_rp, size_t(n + 1)));
    HIP_TRY(s.alloc(&d_col, size_t(nnz)));
    HIP_TRY(s.alloc(&d_val, size_t(nnz)));
    HIP_TRY(s.alloc(&d_perm, size_t(n)));
    HIP_TRY(s.alloc(&d_inv, size_t(n)));
    HIP_TRY(s.alloc(&d_pre, size_t(n)));
    HIP_TRY(s.alloc(&d_tops, size_t(tiles)));
    HIP_TRY(s.alloc(&d_slot, size_t(n)));
    HIP_TRY(s.alloc(&d_t0, size_t(n)));
    HIP_TRY(s.alloc(&d_err, 1));
    HIP_TRY(hipMemsetAsync(d_err, 0, sizeof(int32_t), s.st));
    HIP_TRY(hipMemcpyAsync(d_rp, A.row_ptr, sizeof(int64_t) * size_t(n + 1), hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemcpyAsync(d_col, A.col, sizeof(int32_t) * size_t(nnz), hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemcpyAsync(d_val, A.val, sizeof(double) * size_t(nnz), hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemcpyAsync(d_perm, perm.data(), sizeof(int32_t) * size_t(n), hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemcpyAsync(d_slot, lay.pos_slot.data(), sizeof(int64_t) * size_t(n), hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemcpyAsync(d_t0, lay.pos_task0.data(), sizeof(int32_t) * size_t(n), hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemsetAsync(d_word, 0xFF, sizeof(uint32_t) * size_t(slots), s.st));   // padding words
    HIP_TRY(hipMemsetAsync(d_value, 0, sizeof(double) * size_t(slots), s.st));
    const unsigned rows_grid = unsigned((n + kBlock - 1) / kBlock);
    const int32_t up = upper ? 1 : 0;
    hipLaunchKernelGGL(pack_rows, dim3(rows_grid), dim3(kBlock), 0, s.st, d_perm, d_rp, n, up, d_inv, d_pre);
    hipLaunchKernelGGL(scan_tiles, dim3(unsigned(tiles)), dim3(kBlock), 0, s.st, d_pre, n, d_tops);
    hipLaunchKernelGGL(scan_tops, dim3(1), dim3(kBlock), 0, s.st, d_tops, tiles);
    hipLaunchKernelGGL(pack_scatter, dim3(rows_grid), dim3(kBlock), 0, s.st, d_perm, d_inv, d_rp, d_col, d_val, d_pre,
                       d_tops, d_slot, d_t0, n, up, slots, d_word, d_value, d_err);
    HIP_TRY(hipGetLastError());
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, s.st));
    HIP_TRY(hipStreamSynchronize(s.st));
    if (err) return set_error(GLTRSV_EINVAL, "device packing: inconsistent stream layout");
    return GLTRSV_OK;
}

}  // namespace dev
}  // namespace gltrsv
