// Device packing of the lane-interleaved stream (the reorder of Sec. 5 and
// the packed layout the solve kernels read), after the host has laid out
// tasks, chunks and lanes:
//   1. per position t of the schedule order: the inverse of the order,
//      inv[perm[t]] = t;
//   2. the fill: a wavefront per chunk, lane l walking the rows of the
//      chunk's l-th task in order, all lanes on the same entry index at
//      each step, so every step stores 64 consecutive words and values;
//      each lane reads its own rows' columns and values one after another.
//      Words are encoded as the host packer does: header, a column of the
//      same task fewer than kRing rows back as "rows back", any other column
//      as itself.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/gltrsv.h"
#include "analysis.h"
#include "internal.h"

namespace gltrsv {
namespace dev {
namespace {

// Waves of the fill kernel per compute unit.  Every wave keeps about two
// lines per lane in use (its lanes' current rows), so more waves hide more
// latency but push those lines out of L2 before the lanes' next steps reuse
// them.  Measured on MI355X for the n = 1e7 ER stream (1.2e8 slots): 1, 2,
// 4 and 8 waves per CU took 13.5, 7.0, 3.9 and 5.6 ms and read 1.31e8,
// 1.38e8, 1.69e8 and 2.98e8 128-byte requests beyond L2.
#ifndef GLTRSV_PACK_WAVES_PER_CU
#define GLTRSV_PACK_WAVES_PER_CU 4
#endif
constexpr int kPackWavesPerCU = GLTRSV_PACK_WAVES_PER_CU;

// perm lists vertices; for an upper-triangular matrix vertex v is row n-1-v.
__global__ __launch_bounds__(kBlock) void pack_inverse(const int32_t *__restrict__ perm, int64_t n,
                                                       int32_t *__restrict__ inv)
{
    const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (t < n) inv[perm[t]] = int32_t(t);
}

// Grid-stride over chunks, one wavefront per chunk at a time (a bounded
// number of waves keeps the lanes' row reads resident in L2).  Lane l
// emits entry k of its task at every step k < chunk_len: a row header (the
// original row, value = the diagonal) when it starts a row, else the row's
// next off-diagonal in stored order.
__global__ __launch_bounds__(kBlock) void pack_chunks(
    const int32_t *__restrict__ perm, const int32_t *__restrict__ inv, const int64_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col, const double *__restrict__ val, const int64_t *__restrict__ chunk_base,
    const int32_t *__restrict__ chunk_len, const int32_t *__restrict__ lane_first,
    const int32_t *__restrict__ lane_rows, int64_t chunks, int64_t n, int32_t upper, int64_t slots,
    uint32_t *__restrict__ word, double *__restrict__ value, int32_t *__restrict__ err)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = int64_t(gridDim.x) * kWavesPerBlock;
    for (int64_t c = int64_t(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6); c < chunks; c += waves) {
        const int64_t base = chunk_base[c] + lane;
        const int32_t len = chunk_len[c];
        const int32_t p0 = lane_first[c * kLanes + lane], nr = lane_rows[c * kLanes + lane];
        if (base + int64_t(kLanes) * len > slots + lane || p0 < 0 || int64_t(p0) + nr > n) {
            *err = 1;   // inconsistent layout: write nothing
            continue;
        }
        int32_t q = 0;                 // rows started
        int64_t t = p0, e = 0, hi = 0; // current position, next entry, end of its off-diagonals
        for (int32_t k = 0; k < len; k++) {
            const bool start = e >= hi;   // the previous row is complete
            if (start && q >= nr) continue;   // this lane's task is done (padding was stored before)
            uint32_t w;
            double v;
            if (start) {
                t = int64_t(p0) + q++;
                const int32_t vx = perm[t];
                const int64_t row = upper ? n - 1 - vx : vx;
                // off-diagonals [e, hi) in stored order, diagonal at dg
                e = upper ? row_ptr[row] + 1 : row_ptr[row];
                hi = upper ? row_ptr[row + 1] : row_ptr[row + 1] - 1;
                const int64_t dg = upper ? row_ptr[row] : row_ptr[row + 1] - 1;
                w = kHdrBit | uint32_t(row);
                v = val[dg];
            } else {
                const int32_t cl = col[e];
                const int32_t ic = inv[upper ? n - 1 - cl : cl];
                w = uint32_t(cl);
                // a parent inside the task's range of the order is in this task
                if (ic >= p0 && t - ic < kRing) w = kIntBit | uint32_t(t - ic);
                v = val[e];
                e++;
            }
            word[base + int64_t(kLanes) * k] = w;
            value[base + int64_t(kLanes) * k] = v;
        }
        if (e < hi || q < nr) *err = 1;   // the task did not fit its chunk length
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
    const int64_t chunks = int64_t(lay.pk.chunk_len.size());
    if (n == 0 || slots == 0) return GLTRSV_OK;
    Scratch s;
    HIP_TRY(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
    int64_t *d_rp, *d_base;
    int32_t *d_col, *d_perm, *d_inv, *d_len, *d_first, *d_rows, *d_err;
    double *d_val;
    HIP_TRY(s.alloc(&d_rp, size_t(n + 1)));
    HIP_TRY(s.alloc(&d_col, size_t(nnz)));
    HIP_TRY(s.alloc(&d_val, size_t(nnz)));
    HIP_TRY(s.alloc(&d_perm, size_t(n)));
    HIP_TRY(s.alloc(&d_inv, size_t(n)));
    HIP_TRY(s.alloc(&d_base, size_t(chunks)));
    HIP_TRY(s.alloc(&d_len, size_t(chunks)));
    HIP_TRY(s.alloc(&d_first, size_t(chunks) * kLanes));
    HIP_TRY(s.alloc(&d_rows, size_t(chunks) * kLanes));
    HIP_TRY(s.alloc(&d_err, 1));
    HIP_TRY(hipMemsetAsync(d_err, 0, sizeof(int32_t), s.st));
    HIP_TRY(hipMemcpyAsync(d_rp, A.row_ptr, sizeof(int64_t) * size_t(n + 1), hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemcpyAsync(d_col, A.col, sizeof(int32_t) * size_t(nnz), hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemcpyAsync(d_val, A.val, sizeof(double) * size_t(nnz), hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemcpyAsync(d_perm, perm.data(), sizeof(int32_t) * size_t(n), hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemcpyAsync(d_base, lay.pk.chunk_base.data(), sizeof(int64_t) * size_t(chunks), hipMemcpyHostToDevice,
                           s.st));
    HIP_TRY(hipMemcpyAsync(d_len, lay.pk.chunk_len.data(), sizeof(int32_t) * size_t(chunks), hipMemcpyHostToDevice,
                           s.st));
    HIP_TRY(hipMemcpyAsync(d_first, lay.lane_first.data(), sizeof(int32_t) * size_t(chunks) * kLanes,
                           hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemcpyAsync(d_rows, lay.lane_rows.data(), sizeof(int32_t) * size_t(chunks) * kLanes,
                           hipMemcpyHostToDevice, s.st));
    HIP_TRY(hipMemsetAsync(d_word, 0xFF, sizeof(uint32_t) * size_t(slots), s.st));   // padding words
    HIP_TRY(hipMemsetAsync(d_value, 0, sizeof(double) * size_t(slots), s.st));
    const int32_t up = upper ? 1 : 0;
    hipLaunchKernelGGL(pack_inverse, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s.st, d_perm, n,
                       d_inv);
    int cus = 0, dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(int64_t(cus) * kPackWavesPerCU / kWavesPerBlock,
                                                                (chunks + kWavesPerBlock - 1) / kWavesPerBlock));
    hipLaunchKernelGGL(pack_chunks, dim3(unsigned(grid)), dim3(kBlock), 0, s.st, d_perm, d_inv, d_rp, d_col, d_val,
                       d_base, d_len, d_first, d_rows, chunks, n, up, slots, d_word, d_value, d_err);
    HIP_TRY(hipGetLastError());
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, s.st));
    HIP_TRY(hipStreamSynchronize(s.st));
    if (err) return set_error(GLTRSV_EINVAL, "device packing: inconsistent stream layout");
    return GLTRSV_OK;
}

}  // namespace dev
}  // namespace gltrsv
