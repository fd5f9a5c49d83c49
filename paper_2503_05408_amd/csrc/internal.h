// Declarations shared by the library's HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <algorithm>
#include <vector>

#include "../../include/gltrsv.h"
#include "analysis.h"
#include "local.h"
#include "wave.h"

namespace gltrsv {

// Records `msg` as the calling thread's last error and returns `code`.
int set_error(int code, const std::string &msg);

namespace dev {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;

// Words of the persistent kernels' superstep synchronisation, one 128-byte
// line each: the progress word (64-bit: epoch of the solve, supersteps
// completed), the top count, one count per group of workgroups (up to 128
// groups), and the 64-bit start ticket.  A grid of at most kFlatMax
// workgroups counts on group 0's word only; larger grids count per group of
// kGroup workgroups and then on the top word.  Measured on MI355X: one level
// up to 256 workgroups beat groups of 16 (27-point grid 11.47 against
// 11.96 ms, equal on C2), while at 2,048 workgroups groups of 16 beat groups
// of 256 (15.3 against 11.8 ms with wavefront cores).
constexpr int kGroup = 16;
constexpr int kFlatMax = 256;
constexpr int kBarProg = 0;         // word index of the 64-bit progress word
constexpr int kBarTop = 32;         // word index of the top count
constexpr int kBarGroups = 64;      // group g counts at kBarGroups + 32 g
constexpr int kBarStart = kBarGroups + 32 * 128;   // 64-bit start ticket
// 64-bit start tickets of the semi-asynchronous kernels (lane cores, several
// right-hand sides, wavefront cores), one line each
constexpr int kBarAsyncTicket = kBarStart + 32;
constexpr int kBarWords = kBarAsyncTicket + 3 * 32;
// A semi-asynchronous wave that has waited this long for values (100 MHz
// ticks, 200 us) looks for workgroups of its launch that have not started.
constexpr int64_t kRobTicks = 20000;
constexpr int kMaxGrid = kGroup * 128;   // workgroups of a persistent launch at most
// A workgroup that has waited this long for a superstep (ticks of the
// 100 MHz wall clock, 200 us) starts claiming that superstep's unclaimed
// items: far above the imbalance waits of normal runs, so the steals only
// act when some workgroup cannot start or has stalled.
constexpr int64_t kStealTicks = 20000;

// (Wavefront cores: kWaveRing and the record-stream constants are in
// wave.h.)
// Scalar registers of the record-stream kernel (trsv_stream_async): with 96
// it needs no spills (92 used; at 80 it spilled 19 into vector lanes), and
// MI355X then holds 7 of its 256-thread workgroups per CU, although the
// occupancy query reports 8.  Measured: grids of 7 per CU were 2-4% faster
// than the 80-register build at 8 per CU (27-point 216^3 3.96 against 4.08
// ms, the 64-system batch 6.05 against 6.28 ms); a grid of 8 per CU with 96
// registers waited on workgroups that could not start (3.5 s per solve).
// So the kernel's grids are capped at kStreamWgPerCu per CU.
#ifndef GLTRSV_STREAM_SGPRS
#define GLTRSV_STREAM_SGPRS 96
#endif
constexpr int kStreamSgprs = GLTRSV_STREAM_SGPRS;
constexpr int kStreamWgPerCu = kStreamSgprs > 80 ? 7 : 8;
// The wave-core kernels subtract a row's products with the DPP form
// (subtract_lanes) when the system averages at least this many stored
// off-diagonals per row.  Measured on MI355X, the semi-asynchronous
// record-stream kernel with that form against readlane for every system:
// 27-point 216^3 (13 a row) 3.75 against 3.97 ms, ER n = 1e7 (11) 2.71
// against 2.76; NB n = 1e5, p = 0.03, B = 42 (about 1.3) 1.22 against 1.11,
// the 64-system batch (4.3) 6.51 against 6.05.  The BSP wave-core kernel
// (persistent / one launch per superstep): ER n = 1e5, p = 2e-3 (about 100
// a row) 7.57 / 7.56 against 10.62 / 11.07 ms, 27-point 12.35 / 10.08
// against 12.76 / 10.64; NB n = 1e5, p = 0.05, B = 20 0.530 / 0.353
// against 0.520 / 0.357.
#ifndef GLTRSV_DPP_MIN_PER_ROW
#define GLTRSV_DPP_MIN_PER_ROW 8
#endif
constexpr int64_t kDppMinPerRow = GLTRSV_DPP_MIN_PER_ROW;

// Batched launches: the state word of system i sits at state[i * kStateStride]
// (one per 256 bytes, so waves polling different systems do not queue on
// one line); an idle wave sleeps 1, 2, 4, ... up to kIdleNapMax short naps
// between scans.
#ifndef GLTRSV_STATE_STRIDE
#define GLTRSV_STATE_STRIDE 32
#endif
#ifndef GLTRSV_IDLE_NAP_MAX
#define GLTRSV_IDLE_NAP_MAX 64
#endif
constexpr int kStateStride = GLTRSV_STATE_STRIDE;
constexpr int kIdleNapMax = GLTRSV_IDLE_NAP_MAX;
// A wave idle for kRetireTicks of the 100 MHz wall clock leaves the launch
// while more than keep_waves waves remain, so a long tail of narrow
// supersteps is not slowed by thousands of pollers.  The first kMaskSystems
// systems have a bit in a per-workgroup mask once seen finished, so scans
// skip them.
#ifndef GLTRSV_RETIRE_TICKS
#define GLTRSV_RETIRE_TICKS 2000
#endif
constexpr int64_t kRetireTicks = GLTRSV_RETIRE_TICKS;
constexpr int kMaskSystems = 1024;

// Waves kept by a batched launch: enough for the widest superstep of any of
// its systems, at least 256, at most the whole grid.
inline int32_t keep_waves_for(int64_t widest_chunks, int32_t per_claim, int grid)
{
    const int64_t w = std::max<int64_t>(256, (widest_chunks + per_claim - 1) / std::max(1, per_claim));
    return int32_t(std::min<int64_t>(w, int64_t(grid) * kWavesPerBlock));
}

// One system of a batched launch: its plan's device arrays, its vectors, its
// superstep count and the index of its first per-superstep done counter.
struct SysDesc {
    const uint32_t *word;
    const double *value;
    const int64_t *chunk_base;
    const int32_t *chunk_len;
    const int32_t *super_chunk;
    const double *b;
    double *x;
    int32_t S;
    int32_t done_off;   // first per-superstep done counter of this system
    int32_t nchunks;    // chunks of all supersteps
    int32_t window;     // semi-asynchronous launches: chunks (or tasks) claimed ahead of the completed ones
    int64_t n;          // rows
    // wavefront-core systems (semi-asynchronous batches of core-width-64 plans);
    // ntasks is unused there (the launch runs a global task order)
    const int32_t *wrow;
    const int64_t *wptr;
    const double *wdiag;
    const uint32_t *wcol;
    const double *wval;
    const int64_t *wtask;
    int32_t ntasks;
};

// A system's record stream and its first row in a batch (stream_rebase).
struct StreamSrc {
    const uint32_t *scol;
    const double *sval;
    const int64_t *stask;
    int64_t off;
};
__global__ void stream_rebase(const StreamSrc *src, const int32_t *gsys, const int32_t *gtask, const int64_t *boff,
                              const int64_t *bsize, int64_t ntasks, uint32_t *scol, double *sval);
__global__ void batch_concat(const SysDesc *sys, const int64_t *off, double *cat, bool in);

// Chunks a semi-asynchronous batched launch lets one system have in flight:
// about four supersteps of its average width.
inline int32_t async_window(int64_t chunks, int32_t S)
{
    const int64_t avg = S > 0 ? (chunks + S - 1) / S : 1;
    return int32_t(std::max<int64_t>(8, std::min<int64_t>(int64_t(1) << 30, 4 * avg)));
}

__global__ void batch_reset(unsigned long long *state, uint32_t *done, int32_t count, int32_t ndone,
                            uint32_t *finished, int32_t *err);
// Semi-asynchronous batched launches: x of every system filled with the
// not-yet-computed mark, then chunks claimed in order per system.
// state[i * kStateStride]: low half = chunks claimed, high half = chunks done.
__global__ void fill_unready_sys(const SysDesc *__restrict__ sys, int32_t count);
__global__ void trsv_batched_async(const SysDesc *__restrict__ sys, int32_t count, unsigned long long *state,
                                   uint32_t *finished, int32_t *err, int64_t spin_limit, int32_t per_claim,
                                   int64_t quantum);
// x[0, n) = the not-yet-computed mark
__global__ void fill_unready(unsigned long long *x, int64_t n);

// Fills the plan's stream (d_word, d_value: lay.pk.slots entries) on the
// device from A, the schedule order and the host layout; synchronous.
// upper: A is upper-triangular and perm lists vertices of its mirror (row
// n-1-v), as for pack_fill_upper.
int device_pack(const CsrView &A, const std::vector<int32_t> &perm, const PackLayout &lay, bool upper,
                uint32_t *d_word, double *d_value);

// Single-system kernels (kernels.hip).  Lane cores, one launch per
// superstep, chunks [c0, c1):
__global__ void trsv_superstep_plain(const uint32_t *word, const double *value, const int64_t *chunk_base,
                                     const int32_t *chunk_len, int32_t c0, int32_t c1, const double *b, double *x);
// the same without the reorder of Sec. 5 (tasks [t0, t1) over the caller's CSR)
__global__ void trsv_superstep_unordered(const int64_t *row_ptr, const int32_t *col, const double *val,
                                         const int32_t *rows, const int64_t *task_off, int32_t t0, int32_t t1,
                                         int32_t upper, const double *b, double *x);
// lane cores, every superstep in one launch; superstep completion counted
// on `bar`, workgroups that have not started robbed (alive: one word per
// workgroup, claim: one word per chunk)
__global__ void trsv_persistent(const uint32_t *word, const double *value, const int64_t *chunk_base,
                                const int32_t *chunk_len, const int32_t *super_chunk, int32_t S, const double *b,
                                double *x, uint32_t *bar, uint32_t *alive, uint32_t *claim, int32_t *err,
                                int64_t spin_limit, int64_t steal_ticks, int64_t delay_ticks, int64_t *trace);
// wavefront cores: supersteps [s0, s1) (claim = nullptr for a single
// superstep, else one word per task as in trsv_persistent), and the
// semi-asynchronous form over all tasks
template <bool kDpp>
__global__ void trsv_wave(const int32_t *wrow, const int64_t *wptr, const double *wdiag, const uint32_t *wcol,
                          const double *wval, const int64_t *wtask, const int32_t *wsuper, int32_t s0, int32_t s1,
                          const double *b, double *x, uint32_t *bar, uint32_t *alive, uint32_t *claim,
                          int32_t *err, int64_t spin_limit, int64_t steal_ticks, int64_t delay_ticks);
template <bool kDpp>
__global__ void trsv_stream_async(const uint32_t *scol, const double *sval, const int64_t *sbeg, const int64_t *stask,
                                  int32_t tasks, const double *b, double *x, int32_t *err, int64_t spin_limit,
                                  unsigned long long *ticket, uint32_t *alive, unsigned long long *vnext,
                                  int64_t rob_ticks, int64_t delay_ticks);
// lane cores, semi-asynchronous; R right-hand sides (row-major, leading dimension ld)
// (static chunk order; ticket/alive/vnext: the robbing of workgroups that
// have not started, a start ticket, kMaxGrid alive words and 4 kMaxGrid
// robbed-prefix words per kernel)
__global__ void trsv_async(const uint32_t *word, const double *value, const int64_t *chunk_base,
                           const int32_t *chunk_len, int32_t chunks, const double *b, double *x, int32_t *err,
                           int64_t spin_limit, unsigned long long *ticket, uint32_t *alive, unsigned long long *vnext,
                           int64_t rob_ticks, int64_t delay_ticks);
template <int R>
__global__ void trsv_async_multi(const uint32_t *word, const double *value, const int64_t *chunk_base,
                                 const int32_t *chunk_len, int32_t chunks, const double *b, double *x, int64_t ld,
                                 int32_t *err, int64_t spin_limit, unsigned long long *ticket, uint32_t *alive,
                                 unsigned long long *vnext, int64_t rob_ticks, int64_t delay_ticks);
// single-workgroup execution (local.h): one workgroup of 128 threads per
// system; sys[blockIdx.x] in the batched form
struct LocalSys {
    const uint8_t *rec;
    const LocalRec *info;
    const double *b;
    double *x;
    int64_t n;
    int32_t nrec;
};
__global__ void trsv_local(const uint8_t *rec, const LocalRec *info, int32_t nrec, int64_t n, const double *b,
                           double *x, int32_t *err, int64_t spin_limit);
__global__ void trsv_local_batched(const LocalSys *sys, int32_t count, int32_t *err, int64_t spin_limit);
// measurement probes
__global__ void gather_probe(const uint32_t *word, const double *value, const int64_t *chunk_base,
                             const int32_t *chunk_len, int64_t chunks, const double *x, double *y);
__global__ void copy_probe(const double2 *src, double2 *dst, int64_t n16);

// finished[0] = systems completed in the launch, finished[1] = waves retired
__global__ void trsv_batched(const SysDesc *__restrict__ sys, int32_t count, unsigned long long *state,
                             uint32_t *done, uint32_t *finished, int32_t *err, int64_t spin_limit, int32_t per_claim,
                             int32_t target, int64_t quantum, int32_t keep_waves);

}  // namespace dev
}  // namespace gltrsv

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return ::gltrsv::set_error(e_ == hipErrorOutOfMemory ? GLTRSV_ENOMEM : GLTRSV_EHIP,         \
                                       std::string(#expr) + ": " + hipGetErrorString(e_));              \
    } while (0)

struct gltrsv_plan {
    int64_t n = 0, nnz = 0;
    int32_t S = 0, wavefronts = 0;
    int64_t tasks = 0, chunks = 0, slots = 0, max_task_rows = 0;
    int64_t analysis_ns = 0, device_bytes = 0;
    uint64_t key = 0;
    int device = 0;
    int grid = 0;
    int64_t widest = 0;             // chunks of the widest superstep
    std::vector<int32_t> core, superstep, perm, super_chunk_host;
    uint32_t *d_word = nullptr;
    double *d_value = nullptr;
    int64_t *d_chunk_base = nullptr;
    int32_t *d_chunk_len = nullptr;
    int32_t *d_super_chunk = nullptr;
    uint32_t *d_bar = nullptr;   // superstep synchronisation words (dev::kBarWords)
    uint32_t *d_alive = nullptr; // per persistent-kernel workgroup: epoch of its last start (+ robbed bit)
    uint32_t *d_claim = nullptr; // per chunk: epoch of the solve that claimed it (persistent kernel)
    uint32_t *d_wclaim = nullptr;// per wave-core task: the same for the wave-core persistent kernel
    // robbing in the semi-asynchronous kernels: alive words (3 x kMaxGrid:
    // lane cores, several right-hand sides, wave cores) and robbed-prefix
    // words (3 x 4 kMaxGrid)
    uint32_t *d_aalive = nullptr;
    unsigned long long *d_vnext = nullptr;
    int32_t *d_err = nullptr;
    int64_t *d_trace = nullptr;  // per-superstep timestamps (trace builds only)
    hipStream_t last_stream = nullptr;
    int64_t spin_limit = 5000000;   // polls of a device-side wait before ETIMEDOUT (0.7-5 s)
    int64_t steal_ticks = gltrsv::dev::kStealTicks;   // superstep wait before robbing (100 MHz ticks)
    int64_t delay_ticks = 0;        // diagnostic late start of every 7th persistent workgroup
    int32_t schedule_kind = 0;      // the schedule actually built
    double predicted_us = 0.0;      // cost-model prediction of one solve
    bool device_packed = false;     // stream filled by the packing kernels
    bool upper = false;             // backward solve: vertex v of core/superstep/perm is row n-1-v
    int grid_async = 0;             // workgroups of the semi-asynchronous kernel
    double *d_bcopy = nullptr;      // b when a semi-asynchronous solve runs in place
    int cooperative = 0;
    int32_t exec_form = 0;          // preferred form of gltrsv_solve_auto (GLTRSV_EXEC_*)
    // opts.reorder = 0: the matrix in the caller's order as well, for gltrsv_solve_unordered
    int64_t *d_csr_rp = nullptr;
    int32_t *d_csr_col = nullptr;
    double *d_csr_val = nullptr;
    int32_t *d_urows = nullptr;         // original rows of every task, task after task
    int64_t *d_utask_off = nullptr;     // [tasks + 1] offsets into d_urows
    std::vector<int32_t> super_task_host;   // [S + 1] task range of each superstep
    // opts.core_width = 64: a core is a wavefront (see trsv_wave)
    int32_t core_width = 1;
    int32_t *d_wrow = nullptr;          // [n] original row at each position of the wave layout
    int64_t *d_wptr = nullptr;          // [n + 1] off-diagonal entries of each position
    double *d_wdiag = nullptr;          // [n]
    uint32_t *d_wcol = nullptr;         // [nnz - n] column, or kIntBit | rows back within the task
    double *d_wval = nullptr;           // [nnz - n]
    int64_t *d_wtask = nullptr;         // [wave tasks + 1] first position of each task
    int32_t *d_wsuper = nullptr;        // [S + 1] task range of each superstep
    std::vector<int32_t> wsuper_host;   // [S + 1] task range of each superstep
    int grid_wave = 0;                  // workgroups of the persistent wave kernel
    int grid_wave_async = 0;            // workgroups of the semi-asynchronous wave kernel
    // per-wave record streams of the semi-asynchronous wave kernel (trsv_stream_async)
    uint32_t *d_scol = nullptr;         // [sbeg[W] + kStreamPad] header, column or ring word
    double *d_sval = nullptr;           // [sbeg[W] + kStreamPad] diagonal or A_ij
    int64_t *d_sbeg = nullptr;          // [W + 1] first slot of each wave's stream
    int64_t *d_stask = nullptr;         // [wave tasks] first slot of each task
    int64_t stream_w = 0;               // W: waves the streams were built for (4 x grid_wave_async)
    bool row_dpp = false;               // wave cores: DPP row subtraction (see kDppMinPerRow)
    std::vector<int64_t> ssize_host;    // [wave tasks] slots of each task's records
    // one-workgroup layout (opts.exec_hint = 2, local.h)
    uint8_t *d_lrec = nullptr;          // the records
    gltrsv::LocalRec *d_linfo = nullptr;   // [l_nrec]
    int32_t l_nrec = 0;
    int64_t l_bytes = 0, l_groups = 0, l_far = 0;
};

inline int64_t widest_of(const std::vector<gltrsv_plan *> &plans)
{
    int64_t w = 0;
    for (const gltrsv_plan *p : plans) w = std::max(w, p->widest);
    return w;
}
