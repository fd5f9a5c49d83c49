// Host-side analysis of a sparse lower-triangular matrix: checks, wavefronts,
// the GrowLocal schedule (Algorithm 3.1), the schedule order of Sec. 5 and the
// packed device layout the solve kernels read.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace gltrsv {

// Stream word encoding of the packed layout (see pack_stream):
//   bit 31 set            -> row header; bits 0..29 = original row index and
//                            the paired value is the diagonal A_ii.
//   0xFFFFFFFF            -> padding / end of a lane's rows.
//   bit 30 set (31 clear) -> off-diagonal whose column is one of the last
//                            kRing rows computed earlier in the same
//                            (superstep, core) task; bits 0..29 = how many
//                            rows back (1 = the previous row).
//   otherwise             -> off-diagonal whose value is already in memory
//                            when the lane's current batch starts (an earlier
//                            superstep, or a row of the same task at least
//                            kRing rows back); the word is the column.
constexpr uint32_t kHdrBit = 0x80000000u;
constexpr uint32_t kIntBit = 0x40000000u;
constexpr uint32_t kIdxMask = 0x3FFFFFFFu;
constexpr uint32_t kPadWord = 0xFFFFFFFFu;
#ifndef GLTRSV_RING
#define GLTRSV_RING 16
#endif
constexpr int kRing = GLTRSV_RING;  // recent rows of a lane kept on chip
constexpr int64_t kMaxRows = (int64_t(1) << 30) - 1;
constexpr int kLanes = 64;  // tasks per chunk = lanes of a wavefront

struct CsrView {
    int64_t n = 0, nnz = 0;
    const int64_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
    const double *val = nullptr;
};

struct SchedParams {
    int32_t k = 22;
    double L = 500.0, alpha0 = 20.0, growth = 1.5, accept = 0.97;
    int32_t kind = 0;  // 0 GrowLocal, 1 wavefront
    int32_t threads = 0;  // GrowLocal workers, 0 = automatic
    int32_t blocks = 0;   // > 1: block-parallel scheduling over that many diagonal blocks
    int64_t funnel_max_weight = 0;   // > 0: Funnel coarsening first, parts up to this weight
    int32_t exec_hint = 0;           // AUTO predicts 0: persistent execution, 1: semi-asynchronous
};

struct Schedule {
    std::vector<int32_t> core, superstep;
    int32_t S = 0;
};

// Returns 0 or a negative GLTRSV_E* code; msg receives a description.
int check_csr(const CsrView &A, bool need_values, std::string *msg);

// Upper-triangular layout (backward substitution): in every row the
// diagonal is the first stored entry and the other columns rise above it.
int check_csr_upper(const CsrView &A, bool need_values, std::string *msg);

// J U J for an upper-triangular U (J = the reversal i -> n-1-i): the
// lower-triangular pattern of the same DAG with vertex n-1-i for row i,
// columns rising, no values.  Scheduling it schedules the backward solve in
// its own direction.
struct Mirror {
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    CsrView view() const
    {
        CsrView v;
        v.n = int64_t(row_ptr.size()) - 1;
        v.nnz = v.n >= 0 ? row_ptr.back() : 0;
        v.row_ptr = row_ptr.data();
        v.col = col.data();
        return v;
    }
};
Mirror mirror_upper(const CsrView &U);

// level[i] in 1..; returns the number of wavefronts.
int32_t wavefront_levels(const CsrView &A, std::vector<int32_t> &level);

Schedule schedule_wavefront(const CsrView &A);

// Definition 2.1 for a given schedule: cores >= 0, supersteps in [0, S), and
// for every edge (j, i) either sigma(j) < sigma(i), or the same superstep on
// the same core.  Returns 0 or GLTRSV_EINVAL with a description.
int validate_schedule(const CsrView &A, const Schedule &s, std::string *msg);
Schedule schedule_growlocal(const CsrView &A, const SchedParams &p);
// Funnel coarsening (Sec. 4).  The approximate transitive reduction keeps
// the parents of each vertex except those u with u -> v -> w for another
// parent v (a long edge of a triangle); parents rising.
struct ReducedDag {
    std::vector<int64_t> beg;   // [n+1]
    std::vector<int32_t> par;
};
ReducedDag transitive_reduction(const CsrView &A);
// Algorithm 4.1 on the reduced DAG: vertices in reverse topological order,
// the largest vertex popped first, a parent joins once all its children are
// in the part, a vertex that would lift the part weight (stored entries)
// above max_weight stays out.  part[v], parts numbered by root, rising.
std::vector<int32_t> funnel_partition(const CsrView &A, const ReducedDag &r, int64_t max_weight, int32_t *nparts);

// Row bounds of the diagonal blocks of block-parallel scheduling (Sec. 3.1):
// block b = rows [floor(b n / B), floor((b+1) n / B)).
std::vector<int64_t> block_bounds(int64_t n, int32_t nblocks);
// Workers GrowLocal uses for n rows when `requested` (0 = automatic) is given.
int growlocal_workers(int64_t n, int32_t requested);

// perm[t] = row at position t in (superstep, core, index) order.
std::vector<int32_t> schedule_order(int64_t n, const int32_t *core, const int32_t *superstep, int32_t S);

// Device layout.  Tasks of a superstep are sorted by length (longest first)
// and grouped 64 at a time into chunks; chunk c occupies stream slots
// [chunk_base[c], chunk_base[c] + 64 * chunk_len[c]), entry t of lane l at
// chunk_base[c] + 64 * t + l.
struct Packed {
    int32_t S = 0;
    std::vector<int32_t> super_chunk;   // [S+1] chunk range of each superstep
    std::vector<int64_t> chunk_base;    // [C]
    std::vector<int32_t> chunk_len;     // [C]
    std::vector<uint32_t> word;         // [slots]
    std::vector<double> value;          // [slots]
    int64_t tasks = 0;
    int64_t max_task_rows = 0;
    int64_t slots = 0;
};

// Layout part of the packing (O(n + tasks)): tasks, their chunk and lane,
// chunk lengths and bases, and for every position t of the order the stream
// slot of its lane (chunk base + lane) and the first position of its task.
struct PackLayout {
    Packed pk;                         // everything but word/value
    std::vector<int64_t> pos_slot;     // [n]
    std::vector<int32_t> pos_task0;    // [n]
    // per (chunk, lane), chunk-major: the task's first position in the order
    // and its row count (0 for a lane without a task)
    std::vector<int32_t> lane_first, lane_rows;
};
PackLayout pack_layout(const CsrView &A, const Schedule &sch, const std::vector<int32_t> &perm);

// Fills word/value of `pk` (already sized) on the host, O(nnz).
void pack_fill(const CsrView &A, const Schedule &sch, const std::vector<int32_t> &perm, PackLayout &lay);

// Host fill for an upper-triangular U scheduled through mirror_upper(U):
// perm lists vertices (row n-1-v); headers and columns carry U's row and
// column numbers and each row's entries follow U's stored order.
void pack_fill_upper(const CsrView &U, const std::vector<int32_t> &perm, PackLayout &lay);

// Layout + host fill.
Packed pack_stream(const CsrView &A, const Schedule &sch, const std::vector<int32_t> &perm);

// Predicted device time of one solve under `sch`, in microseconds: per
// superstep a fixed cost (barrier and one dependent memory round trip) plus
// the larger of the longest task (one lane walks it entry by entry) and the
// superstep's entries at the device's entry throughput.
struct CostModel {
    double superstep_us = 3.0;     // barrier + first gather round trip
    double entry_us = 0.18;        // one lane, one stored entry
    double entries_per_us = 4.0e4; // whole device, random gathers
    double hop_us = 1.5;           // a value passed between lanes through memory (semi-asynchronous)
    double launch_us = 10.0;       // fill of x + launch (semi-asynchronous)
};
// Persistent (barrier) execution: per superstep, the barrier plus the larger
// of its longest task and its entries at the device rate.
double predict_cost_us(const CsrView &A, const Schedule &sch, const std::vector<int32_t> &perm, const CostModel &cm);
// Semi-asynchronous execution: the larger of the critical path (rows of a
// task one after another in their lane, a parent in another task adding a
// memory hop) and all entries at the device rate.
double predict_async_us(const CsrView &A, const Schedule &sch, const std::vector<int32_t> &perm, const CostModel &cm);

uint64_t pattern_key(const CsrView &A);

}  // namespace gltrsv
