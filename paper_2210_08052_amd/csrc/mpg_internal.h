// Internal declarations shared by the host runtime and the HIP kernels of the
// spliced protein-to-genome DP library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpg.h"

namespace mpg {

// Sentinel for "unreachable" (-infinity).  Reachable values are bounded by
// |v| < 2^24 (checked on the host); traceback kernels store 16*v + nibble, so
// reachable scaled values stay inside (-2^28, 2^28) and everything derived
// from the sentinel stays below -2^29 without wrapping.
constexpr int kNeg = -(1 << 30);
constexpr int kUnreachable = -(1 << 29);  // anything below is -infinity

// Row descriptor table covers rows [-kDescLo, nsteps + kDescHi).
constexpr int kDescLo = 128;
constexpr int kDescHi = 64;
// Boundary column buffer covers rows [-kBndLo, nsteps + kBndHi).
constexpr int kBndLo = 64;
constexpr int kBndHi = 128;
// Bytes of traceback storage per 64-step block and per column-in-lane:
// 8 nibble dwords x 64 lanes (2048 B) + 5 states x 64 steps x 8 B (2560 B).
constexpr int kTbBlockBytes = 4608;

// Scoring parameters passed by value to the kernels.
struct DevParams {
    int32_t q, e, f, r;
    int32_t mode, flags;
    int8_t mat[24 * 24];
    uint8_t gcode[64];
    uint8_t donor[128];
    uint8_t acceptor[128];
};

// Per-pair launch plan (device copy; 80 bytes).
struct PairJob {
    int32_t n, m;        // genome rows, protein columns
    int32_t res;         // index of the result record
    int32_t tb;          // 1: store direction bits and emit an op string
    int64_t dna_off;     // offset of the region's letters in the DNA buffer
    int64_t prot_off;    // offset of the protein's letters
    int64_t desc_off;    // byte offset of descriptor row -kDescLo
    int64_t bnd_off;     // int2 index of boundary row -kBndLo
    int64_t tb_off;      // byte offset of this pair's direction bits
    int64_t ops_off;     // byte offset of this pair's op string
    int32_t nchunks;     // 64-step chunks per strip (steps = 64 * nchunks >= n + 64)
    int32_t nstrips;     // strips of 64*K columns covering columns 0..m
    int32_t K;           // columns per lane
    int32_t status;      // host pre-check status (MPG_OK or MPG_E_RANGE)
    int32_t prog_off;    // index of strip 0's progress counter
    int32_t _pad;
};

// Bytes of per-pair shared state of the DP launch (end-cell key, counters).
constexpr int kPairStateBytes = 24;

// Kernel launch helpers implemented in mpg_kernels.hip.
hipError_t launch_prepass(hipStream_t s, const PairJob* jobs, const int64_t* row_start,
                          int npairs, int64_t total_rows, const uint8_t* dna, uint8_t* desc,
                          const DevParams& P);

// One DP launch of persistent wavefronts over the work items (job index,
// strip) of pairs that share K and traceback; all pairs of a call share mode
// and flags.  The grid holds as many wavefronts as `ncu` compute units run at
// once for this kernel, capped at the item count.  qhead must be zero, pst
// and prog zeroed by launch_init.
hipError_t launch_dp(hipStream_t s, int K, bool tb, int ncu, const DevParams& P,
                     const PairJob* jobs, const int2* items, int nitems, int* qhead, void* pst,
                     int* prog, const uint8_t* prot, const uint8_t* desc, int2* bnd,
                     uint8_t* tbbuf, mpg_dev_result* out);

// Zero the per-pair state, the strips' progress counters and the queue heads.
hipError_t launch_init(hipStream_t s, const PairJob* jobs, int npairs, void* pst, int* prog,
                       int* qheads, int nq, int gsc_init);

hipError_t launch_walk(hipStream_t s, const PairJob* jobs, const int32_t* order, int count,
                       const uint8_t* tbbuf, mpg_dev_result* out, char* ops);

hipError_t launch_status(hipStream_t s, const PairJob* jobs, int npairs, mpg_dev_result* out);

// Dynamic LDS bytes of one DP wavefront.
int dp_lds_bytes(int K, bool tb);

}  // namespace mpg
