// Single-workgroup execution of a BSP schedule with at most 64 cores
// (Definition 2.1): the layout the host builds (local.cpp) and the kernel
// reads (local.hip).
//
// One wavefront is the machine: lane c is core c, and the wave's program
// order is the barrier between supersteps, since a value one lane writes to
// LDS is seen by every later LDS read of the wave.  The work of each lane is
// cut into groups of four stream entries; a row starts on the first entry of
// a group (its header: the diagonal and b_i) and may run over several
// groups, and the wave steps through the groups of every lane together.
// Each group ends with the division of Eq. (2.1) in every lane where a row
// ends there.
//
// The result of the row ending in global group g on lane c goes to LDS slot
// (g mod kLocalRingGroups) * 64 + c, a ring that keeps it for the next
// kLocalRingGroups groups.  A later row reads it from there when it runs
// within that window, and otherwise ("far") from a copy of x that a second
// wave stages next to the group.  That helper wave also stages b_i for
// every row header and copies every result to x in global memory.  So the
// computing wave only ever touches LDS.
//
// A slot holds one binary64 value, split: slots come in blocks of 64, and
// slot 64 q + l keeps its low word at LDS word 128 q + l and its high word
// at 128 q + 64 + l (so one read of two words, 64 apart, fetches any slot).
// That is the layout in which the hardware's copy from global memory into
// LDS (four bytes per lane, lane l at word l of the destination) can stage
// 64 values with two instructions.
//
// The groups are cut into records of at most kLocalRecMax bytes.  The
// helper copies each record into an LDS FIFO at an offset the host fixed,
// then fills the record's staging slots, then marks it staged.  Every
// ordering between the two waves is a host-computed count: records
// computed, staged, drained.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "analysis.h"

namespace gltrsv {

constexpr int kLocalAlignBytes = 512;                            // records and fill blocks: 64 slots
constexpr int kLocalRingGroups = 128;
constexpr int kLocalRingSlots = kLocalRingGroups * 64;          // 8 bytes each
constexpr int kLocalZeroSlot = kLocalRingSlots;                  // holds +0.0 (operand of padding)
constexpr int kLocalFifoSlot0 = kLocalRingSlots + 64;            // first FIFO slot (block-aligned)
constexpr int kLocalFifoBytes = 189 * kLocalAlignBytes;
constexpr int kLocalLdsSlots = kLocalFifoSlot0 + kLocalFifoBytes / 8;
constexpr int kLocalRecMax = kLocalFifoBytes / 6;                // FIFO bytes of one record at most
constexpr int kLocalAlign = kLocalAlignBytes;
constexpr int kLocalGroupBytes = 2560;
constexpr int kLocalHdrBytes = 32;
constexpr uint32_t kLocalStartBit = 0x8000u;                     // entry 0: a row header
constexpr uint32_t kLocalEndBit = 0x8000u;                       // entry 1: a row ends in the group
constexpr uint32_t kLocalSlotMask = 0x7FFFu;
constexpr uint32_t kLocalFillX = 0x80000000u;                    // fill from x (else from b)
static_assert(kLocalLdsSlots <= int(kLocalSlotMask) + 1, "slot indices fit 15 bits");
static_assert(kLocalLdsSlots * 8 + 1024 <= 163840, "LDS of one workgroup (with the control words)");

// Record layout (16-byte aligned, copied verbatim into the FIFO):
//   header, kLocalHdrBytes: ngroups, nfill, ndrain, need_drain (records the
//     helper must have drained before the computing wave starts this one:
//     their ring slots are overwritten here), next_off (FIFO byte offset of
//     the next record), need_far (records the helper must have drained
//     before its fills: the rows it reads from x), 2 unused words;
//   ngroups groups of kLocalGroupBytes: values as f64 pairs [2][64][2]
//     (lane l, entries 2h and 2h+1 at byte 1024 h + 16 l), then operand
//     slots as u16 [64][4] at byte 2048 + 8 l;
//   nfill fill entries {u32 slot | kLocalFillX, i32 row}: slot <- b[row] or
//     x[row] (rows in the caller's numbering);
//   ndrain drain entries {u32 slot, i32 row}: x[row] <- slot, after the
//     record is computed;
//   padding to 16 bytes.
// Records start at multiples of kLocalAlign bytes in the FIFO; the nfill
// staging slots follow the copied part in whole blocks of 64 slots from
// the next multiple of kLocalAlign (not copied; the fills write them, fill
// i into the i-th slot).
struct LocalHdr {
    uint32_t ngroups, nfill, ndrain, need_drain, next_off, need_far, unused[2];
};
static_assert(sizeof(LocalHdr) == kLocalHdrBytes, "header size");

// Per record, for the helper's copy: bytes copied, FIFO byte offset, and
// the records that must be computed first (those whose FIFO bytes it
// reuses).
struct LocalRec {
    uint32_t bytes, fifo_off, wait, unused;
};

struct LocalLayout {
    std::vector<uint8_t> rec;         // the records, one after another
    std::vector<LocalRec> info;       // [records]
    int64_t groups = 0;               // groups of all records
    int64_t far = 0;                  // operands staged from x
    int64_t entries = 0;              // group entries (4 per lane and group)
};

// Groups one lane steps through under `sch` (cores < 64): per superstep
// the busiest lane's sum of ceil(entries / 4) over its rows.  D holds the
// rows in the solve's direction (vertex v's stored entries); this is the
// serial path of the one-workgroup solve.
int64_t local_group_count(const CsrView &D, const Schedule &sch, const std::vector<int32_t> &perm);

// The wavefront schedule dealt onto 64 cores: row r of a level (core r)
// goes to core r mod 64.
void fold_cores(Schedule &sch, int32_t cores);

// Predicted one-workgroup solve time: groups at kLocalGroupUs each.
constexpr double kLocalGroupUs = 0.1;

// Builds the layout for `sch` (cores < 64) in the order `perm` of Sec. 5.
// A is the caller's matrix; with upper, vertex v of the schedule is row
// n-1-v (the backward solve, scheduled on the mirrored DAG).  Returns 0, or
// GLTRSV_EINVAL with msg when a core is 64 or more.
int build_local_layout(const CsrView &A, bool upper, const Schedule &sch, const std::vector<int32_t> &perm,
                       LocalLayout *out, std::string *msg);

}  // namespace gltrsv
