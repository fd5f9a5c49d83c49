// Wavefront cores (opts.core_width = 64): the layouts the host builds
// (wave.cpp) and the wave-core kernels read (kernels.hip).
//
// Wave layout (superstep-barrier kernel trsv_wave): the rows in the order
// of Sec. 5 with the tasks of a superstep longest first; per position the
// original row, its diagonal and its off-diagonals in stored order.  A
// column among the task's last kWaveRing rows is stored as kIntBit | rows
// back (the kernel reads it from a per-wave LDS ring), any other column as
// itself.
//
// Per-wave record streams (semi-asynchronous kernel trsv_stream_async):
// tasks are numbered superstep by superstep in the order above and wave
// slot v (of W) runs tasks v, v + W, v + 2W, ...; slot v's stream holds the
// rows of those tasks one after another as records: a header slot (word
// kHdrBit | row, with kIntBit on a task's first row; value the diagonal)
// and then the row's off-diagonals as in the wave layout (word the column
// or kIntBit | rows back; value A_ij).  Slot v's records take
// [sbeg[v], sbeg[v + 1] - 1) and a kPadWord ends them at sbeg[v + 1] - 1;
// task t's first record is at stask[t] and takes ssize[t] slots.  The
// arrays hold kStreamPad kPadWord slots (value 0) past sbeg[W], since the
// kernel reads whole windows ahead of its records.
#pragma once

#include <cstdint>
#include <vector>

#include "analysis.h"

namespace gltrsv {

// Rows of the same task this many back or fewer come from the LDS ring.
constexpr int kWaveRing = 64;
// The stream kernel reads chunks of kStreamSub 64-slot windows; a chunk and
// the one after it are read from a chunk that starts at or before a
// stream's PAD, hence the padding.  Measured on MI355X (wavefront
// schedules, n = 1e7): one window a chunk keeps the kernel at 55 VGPRs and
// eight waves per SIMD, and was fastest (27-point grid 4.72 ms, ER 3.38 ms;
// two windows 4.96 / 3.45 ms at 71 VGPRs, four 5.31 / 3.62 ms at 87).
#ifndef GLTRSV_STREAM_SUB
#define GLTRSV_STREAM_SUB 1
#endif
constexpr int kStreamSub = GLTRSV_STREAM_SUB;
constexpr int64_t kStreamChunk = 64 * kStreamSub;
constexpr int64_t kStreamPad = 2 * kStreamChunk;

struct WaveLayout {
    // wave layout
    std::vector<int32_t> wrow;      // [n] original row at each position
    std::vector<int64_t> wptr;      // [n + 1] off-diagonal entries of each position
    std::vector<double> wdiag;      // [n]
    std::vector<uint32_t> wcol;     // [nnz - n]
    std::vector<double> wval;       // [nnz - n]
    std::vector<int64_t> wtask;     // [tasks + 1] first position of each task
    std::vector<int32_t> wsuper;    // [S + 1] task range of each superstep
    // per-wave record streams for W waves
    int64_t waves = 0;
    std::vector<uint32_t> scol;     // [sbeg[W] + kStreamPad]
    std::vector<double> sval;       // [sbeg[W] + kStreamPad]
    std::vector<int64_t> sbeg;      // [W + 1]
    std::vector<int64_t> stask;     // [tasks]
    std::vector<int64_t> ssize;     // [tasks]
};

// Both layouts of a checked matrix A (the stored triangle: upper = rows
// mirrored as in the plan, vertex v of core/superstep/perm is row n-1-v)
// under a schedule with S supersteps, its order perm (Sec. 5), for W >= 1
// waves.
void build_wave_layout(const CsrView &A, bool upper, const int32_t *core, const int32_t *superstep, int32_t S,
                       const std::vector<int32_t> &perm, int64_t W, WaveLayout *out);

}  // namespace gltrsv
