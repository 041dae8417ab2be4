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
// 8 nibble dwords x 64 lanes (2048 B: the H winner of 8 steps per dword) +
// 5 states x 2 halves x 64 lanes x 4 B (2560 B: one extension bit per step).
constexpr int kTbBlockBytes = 4608;
// Kernel variant for calls with per-pair boundary modes (not LOCAL): each
// item runs the EXTEND code or the fixed-end code (GLOBAL, EXTEND_LEFT) by
// its pair's mode, so such a call needs one launch per strip width.
constexpr int kModeMixed = 8;

// Scoring parameters passed by value to the kernels.
struct DevParams {
    int32_t q, e, f, r;
    int32_t mode, flags;
    int8_t mat[24 * 24];
    uint8_t gcode[64];
    uint8_t donor[128];
    uint8_t acceptor[128];
    int32_t max_polls;  // polls of a bounded wait before it gives up (kMaxPolls)
};
static_assert(offsetof(DevParams, mat) % 4 == 0, "the DP kernel copies mat in dwords");
// A strip waits for its left neighbour's progress for at most this many
// polls (well under a second) before the pair reports MPG_E_DEVICE.
constexpr int32_t kMaxPolls = 1 << 18;

// Per-pair launch plan (device copy; 96 bytes).
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
    int32_t i16;         // 1: runs in a packed int16 job (see PackJob)
    int32_t mode;        // boundary mode of this pair (MPG_LOCAL ... MPG_EXTEND_LEFT)
    int32_t _pad;
};
static_assert(sizeof(PairJob) == 96, "PairJob layout");

// Two LOCAL score-only pairs run together by the lane-packed int16 kernel:
// pair a in the low 16 bits of every lane value, pair b in the high 16 bits
// (b < 0: the high half idles).  Both follow one schedule of nchunks steps
// per strip and nstrips strips (the larger of the two pairs').
struct PackJob {
    int32_t a, b;        // job indices
    int32_t n;           // rows: the larger region
    int32_t nchunks;     // 64-step chunks per strip
    int32_t nstrips;     // strips of 64*K columns
    int32_t K;           // columns per lane
    int32_t prog_off;    // index of strip 0's progress counter
    int32_t _pad;
    int64_t desc_off;    // byte offset of packed descriptor row -kDescLo (16 B per row)
    int64_t bnd_off;     // int2 index of boundary row -kBndLo
};

// A position-specific query block (see the public header): the m x 24 int8
// scores, padded to 8 bytes, then the (m+1) x 4 int16 gap costs.
__host__ __device__ constexpr int64_t prof_gap_offset(int64_t m) { return (24 * m + 7) & ~(int64_t)7; }
__host__ __device__ constexpr int64_t prof_block_bytes(int64_t m) {
    return prof_gap_offset(m) + 8 * (m + 1);
}
__host__ __device__ inline const int8_t* prof_scores(const uint8_t* blk) {
    return (const int8_t*)blk;
}
__host__ __device__ inline const int16_t* prof_gaps(const uint8_t* blk, int64_t m) {
    return (const int16_t*)(blk + prof_gap_offset(m));
}

// Bytes of per-pair shared state of the DP launch (end-cell key, counters).
constexpr int kPairStateBytes = 24;

// Where the DP kernels leave their results.  A record's status field is
// written last; with `system` set the fields reach host memory before it
// (records and op strings may then live in host-mapped memory that the host
// polls while the kernel runs).  With `walk` set, the wavefront that finishes
// a traceback pair walks it at once (results complete pair by pair);
// otherwise the walk kernel runs after the DP.
struct DpSink {
    mpg_dev_result* out;  // result records, indexed by PairJob::res
    char* ops;            // op-string buffer, slots at PairJob::ops_off
    int32_t walk;
    int32_t system;
};

// Status of a record not yet written (records are preset to it when the host
// polls them); never a value of MPG_OK or an MPG_E_* code.
constexpr int32_t kPending = 1;

// Kernel launch helpers implemented in mpg_kernels.hip.
hipError_t launch_prepass(hipStream_t s, const PairJob* jobs, const int64_t* row_start,
                          int npairs, int64_t total_rows, const uint8_t* dna, uint8_t* desc,
                          const DevParams& P);

// One DP launch of persistent wavefronts over the work items (job index,
// strip) of pairs that share K and traceback; all pairs of a call share mode
// and flags.  The grid holds as many wavefronts as `ncu` compute units run at
// once for this kernel, capped at the item count.  qhead must be zero, pst
// and prog zeroed by launch_init.
// pro: the pairs are position-specific queries (prot points at their
// profile blocks; K must be 1 or 2).
hipError_t launch_dp(hipStream_t s, int K, bool tb, bool pro, int ncu, const DevParams& P,
                     const PairJob* jobs, const int2* items, int nitems, int* qhead, void* pst,
                     int* prog, const uint8_t* prot, const uint8_t* desc, int2* bnd,
                     uint8_t* tbbuf, const DpSink& sink);

// Zero the per-pair state, the strips' progress counters and the queue heads.
hipError_t launch_init(hipStream_t s, const PairJob* jobs, int npairs, void* pst, int* prog,
                       int* qheads, int nq, int gsc_init);

hipError_t launch_walk(hipStream_t s, const PairJob* jobs, const int32_t* order, int count,
                       const uint8_t* tbbuf, mpg_dev_result* out, char* ops);

hipError_t launch_status(hipStream_t s, const PairJob* jobs, int npairs, const DpSink& sink);

// One chain of anchor runs (device copy; 56 bytes).  Its pieces are
// consecutive in the piece results: the left extension, the gaps between
// consecutive runs, then the right extension (nruns + 1 pieces).
struct ChainJob {
    int32_t piece0;    // index of the left piece's result record
    int32_t nruns;     // anchor runs, at runs[run0 .. run0 + nruns) as (x, y, len, 0)
    int32_t run0;
    int32_t tb;        // 1: assemble the op string
    int64_t prot_off;  // the chain's letters in the device buffers
    int64_t dna_off;
    int64_t ops_off;   // the chain's op-string slot
    int64_t ops_cap;   // bytes of that slot
    int32_t res;       // index of the chain's result record
    int32_t status;    // MPG_OK, or the chain's host-side error (it has no pieces then)
};
static_assert(sizeof(ChainJob) == 56, "ChainJob layout");

// One wavefront per chain: add the runs' codon scores to the pieces' optima,
// take the end coordinates from the last run and the right piece, and (tb)
// concatenate the pieces' op strings with the runs as M tokens, merging
// adjacent M tokens.  A chain whose piece failed gets that piece's status.
hipError_t launch_stitch(hipStream_t s, const ChainJob* chains, int nchains, const int4* runs,
                         const mpg_dev_result* pres, const char* pops, const uint8_t* prot,
                         const uint8_t* dna, const DevParams& P, mpg_dev_result* out,
                         char* ops);

// Dynamic LDS bytes of one DP wavefront.
int dp_lds_bytes(int K, bool tb);

// Pseudogene guard (mpg_kernels.hip).  One traced pair's coding-sequence cut:
// its op string, the region from the alignment's first base, and where the
// cut goes.
struct CdsJob {
    int64_t ops_off;  // op string in the ops buffer
    int64_t dna_off;  // region base g_beg in the DNA buffer
    int64_t cds_off;  // output slot in the coding-sequence buffer
    int32_t ops_len;
    int32_t cap;      // g_end - g_beg: bases the path consumes
    int32_t plen;     // p_end - p_beg: residues the path consumes
    int32_t _pad;
};
// One wavefront per job: info[k] = {coding length, introns, MPG_OK or
// MPG_E_INVAL for an op string that does not span exactly cap x plen}.
hipError_t launch_cds(hipStream_t s, const CdsJob* jobs, int n, const char* ops, const uint8_t* dna,
                      uint8_t* cds, int4* info);
// Per pair: the first pass's status if it failed, else the coding-sequence
// cut's, else the second alignment's; score = second score, minus r when the
// path had no intron; exons = introns + 1.  j2[k] indexes res2 (-1: none).
hipError_t launch_rescore_finish(hipStream_t s, int n, const mpg_dev_result* res1,
                                 const int4* info, const int32_t* j2, const mpg_dev_result* res2,
                                 int r, int32_t* score, int32_t* exons, int32_t* status);

// Chaining (mpg_chain.hip): one wavefront per anchor set.
struct ChainSetJob {
    int64_t off;     // first anchor of the set (in anchors, f, pred, idx and the records)
    int32_t n;       // anchors
    int32_t status;  // MPG_OK, or the set's error (the kernel writes it to ntop)
    int32_t id;      // the set's index in the call (its ntop and top slots)
    int32_t _pad;
};
// LDS of the chaining kernel (at most 64 KB): the reduction slots, then per
// anchor the used flag (1 byte), f (8) when it fits, and the anchor (8) and
// its predecessor (4) when those fit too.
constexpr int kChainRedBytes = 64;
constexpr int kChainLdsBytes = 65536;
struct ChainCfg {
    int32_t k, G, binned, max_chains;
    int32_t max_n;   // largest set of the launch (sizes the LDS)
    int32_t stage;   // 1: anchors and predecessors also staged in LDS
    int32_t f_lds;   // 1: f in LDS; 0: f read and written in the f output
    int32_t waves;   // wavefronts per set: 1 or 4
    double beta;
};
inline size_t chain_lds_bytes(const ChainCfg& c) {
    const size_t n = (size_t)c.max_n;
    return (kChainRedBytes + (c.f_lds ? 8 * n : 0) + (c.stage ? 12 * n : 0) + n + 15) &
           ~(size_t)15;
}
struct ChainRec {    // one extracted chain (scratch)
    double score;
    int32_t first, len;
};
hipError_t launch_chain(hipStream_t st, const ChainSetJob* sets, int nsets, const int2* anchors,
                        const ChainCfg& cfg, double* f, int* pred, ChainRec* recs, int* idx,
                        mpg_chain_out* top, int* ntop);

// Lane-packed int16 path (mpg_dp16.hip): packed row descriptors of every
// PackJob (rows [-kDescLo, 64*nchunks + kDescHi), pack k's first row at
// global row row_start[k]; also zeroes the packs' progress counters), and the
// DP launch over (pack, strip) items.
hipError_t launch_prepass16(hipStream_t s, const PairJob* jobs, const PackJob* packs,
                            const int64_t* row_start, int npacks, int64_t total_rows,
                            const uint8_t* dna, uint8_t* desc, int* prog, const DevParams& P);
hipError_t launch_dp16(hipStream_t s, int K, int ncu, const DevParams& P, const PairJob* jobs,
                       const PackJob* packs, const int2* items, int nitems, int* qhead, void* pst,
                       int* prog, const uint8_t* prot, const uint8_t* desc, int2* bnd,
                       const DpSink& sink);
int dp16_lds_bytes(int K);

// The fixed scratch array of the allocation-free batch entry point, on the
// current device: its device address (taken with hipGetSymbolAddress once
// per device, with that device current, and kept) and its size.
hipError_t scratch_address(int device, uint8_t** ptr);
constexpr size_t kScratchBytes = MPG_NOALLOC_SCRATCH_BYTES;

}  // namespace mpg
