// Declarations shared by the library's HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/gltrsv.h"
#include "analysis.h"

namespace gltrsv {

// Records `msg` as the calling thread's last error and returns `code`.
int set_error(int code, const std::string &msg);

namespace dev {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;

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
};

__global__ void batch_reset(unsigned long long *state, uint32_t *done, int32_t count, int32_t ndone,
                            uint32_t *finished, int32_t *err);
__global__ void trsv_batched(const SysDesc *__restrict__ sys, int32_t count, unsigned long long *state,
                             uint32_t *done, uint32_t *finished, int32_t *err, int64_t spin_limit, int32_t per_claim,
                             int32_t target, int64_t quantum);

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
    std::vector<int32_t> core, superstep, perm, super_chunk_host;
    uint32_t *d_word = nullptr;
    double *d_value = nullptr;
    int64_t *d_chunk_base = nullptr;
    int32_t *d_chunk_len = nullptr;
    int32_t *d_super_chunk = nullptr;
    uint32_t *d_bar = nullptr;   // barrier words (dev::kBarWords)
    int32_t *d_err = nullptr;
    int64_t *d_trace = nullptr;  // per-superstep timestamps (trace builds only)
    hipStream_t last_stream = nullptr;
    int64_t spin_limit = 5000000;
    int32_t schedule_kind = 0;      // the schedule actually built
    double predicted_us = 0.0;      // cost-model prediction of one solve   // about 5 s of polling
    int cooperative = 0;
};
