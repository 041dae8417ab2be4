// Device helpers and the templated DP kernel, shared by the per-K
// translation units (mpg_dp_k1/k2/k4.hip) and the other kernels.
#pragma once

#include <climits>

#include "mpg_internal.h"
#include "mpg_walk.h"

// Occupancy targets of the DP kernels (waves per SIMD; 1 = no cap).  The
// score-only kernels of width <= 2 run four waves per SIMD (128 VGPRs; 3.4%
// faster than three waves on the 10k batch); the width-2 traceback kernels
// run three (4.9% on the traceback batch), which their LDS also caps.  Width 1
// with traceback and width 4 keep the registers they need (about 320 and 400
// with traceback: one wave per SIMD; width 4 at two waves slows the long-tail
// batch 279 -> 343 ms: its long pairs' strip pipelines are the critical path,
// and a second wave halves each strip's own pace).
#ifndef MPG_SCORE_WAVES
#define MPG_SCORE_WAVES 4
#endif
#ifndef MPG_TB_WAVES
#define MPG_TB_WAVES 3
#endif
// A scheduling barrier between the steps of a chunk keeps each step's
// instructions together (bounding the registers the unrolled chunk needs):
// kept in the score-only kernels, left out of the traceback ones, which run
// 2% faster with neighbouring steps interleaved (timed on the 10k batch).
#ifndef MPG_STEP_BARRIER
#define MPG_STEP_BARRIER 1
#endif
#ifndef MPG_TB_STEP_BARRIER
#define MPG_TB_STEP_BARRIER 0
#endif
#ifndef MPG_K4_WAVES
#define MPG_K4_WAVES 1
#endif
template <int K, bool TB>
struct WavesPerEu {
    static constexpr int value =
        K > 2 ? MPG_K4_WAVES : (TB ? (K == 2 ? MPG_TB_WAVES : 1) : MPG_SCORE_WAVES);
};

namespace mpg {
namespace dev {


constexpr int kShr1 = 0x138;  // DPP wave_shr:1
constexpr int kShl1 = 0x130;  // DPP wave_shl:1

static __constant__ uint8_t kAaOfLetter[26] = {0,  20, 4,  3,  6,  13, 7,  8,  9,  22, 11, 10, 12,
                                        2,  22, 14, 5,  1,  15, 16, 22, 19, 17, 22, 18, 21};

__device__ __forceinline__ int dna_code(uint32_t ch) {
    switch (ch | 0x20u) {
        case 'a': return 0;
        case 'c': return 1;
        case 'g': return 2;
        case 't': return 3;
        default: return 4;
    }
}

__device__ __forceinline__ int aa_code(uint32_t ch) {
    if (ch == '*') return 23;
    uint32_t u = (ch | 0x20u) - 'a';
    return u < 26u ? kAaOfLetter[u] : 22;
}

__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int imax3(int a, int b, int c) { return imax(imax(a, b), c); }

__device__ __forceinline__ int shr1(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, kShr1, 0xF, 0xF, false);
}
__device__ __forceinline__ int shl1(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, kShl1, 0xF, 0xF, false);
}

// max(x of lane - 1, v) with the lane shift as the max's own operand (one
// instruction instead of a move and a max); lane 0 keeps `old`.  The s_nop
// gives the two wait states a DPP read needs after a VALU write of x.
__device__ __forceinline__ int max_from_left(int old, int x, int v) {
    int r = old;
    asm("s_nop 1\n\tv_max_i32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf"
        : "+v"(r)
        : "v"(x), "v"(v));
    return r;
}
// (x of lane - 1) - v, likewise; lane 0 keeps `old`
__device__ __forceinline__ int sub_from_left(int old, int x, int v) {
    int r = old;
    asm("s_nop 1\n\tv_sub_u32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf"
        : "+v"(r)
        : "v"(x), "v"(v));
    return r;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
        uint32_t olo = __shfl_xor((int)lo, o, 64), ohi = __shfl_xor((int)hi, o, 64);
        uint64_t w = ((uint64_t)ohi << 32) | olo;
        v = w > v ? w : v;
    }
    return v;
}

// End-cell key: larger is better; score desc, then row asc, then column asc.
__device__ __forceinline__ uint64_t end_key(int score, int row, int col) {
    return ((uint64_t)(uint32_t)(score + (1 << 27)) << 36) |
           ((uint64_t)(uint32_t)((1 << 21) - 1 - row) << 15) | (uint64_t)((1 << 15) - 1 - col);
}

// Modes whose H floors at 0 in every cell (a path may start anywhere), and
// modes read at the single end cell (n, m).
__host__ __device__ constexpr bool floor_mode(int mode) {
    return mode == MPG_LOCAL || mode == MPG_EXTEND_LEFT;
}
__host__ __device__ constexpr bool fixed_end_mode(int mode) {
    return mode == MPG_GLOBAL || mode == MPG_EXTEND_LEFT;
}

__device__ __forceinline__ int neg_for(int mode, bool tb) {
    return floor_mode(mode) ? (tb ? -(1 << 29) : -(1 << 25)) : -(1 << 30);
}

// ------------------------------------------------------------ prepasses
// Rows per thread: a block covers 256 * kPrepassRows consecutive rows, so its
// owner search and table staging are shared by that many rows, and a thread
// reads one window of bases for its consecutive rows.
constexpr int kPrepassRows = 4;
static_assert(64 % kPrepassRows == 0 && kDescLo % kPrepassRows == 0 &&
                  kDescHi % kPrepassRows == 0,
              "a thread's rows must lie in one pair");

// The last index p in [0, n) with start[p] <= g (start ascending, start[0] <=
// g), found by wave 0 of the block 64 probes at a time: each round reads 64
// positions spread over the remaining range at once and keeps the part between
// the last probe at or below g and the next one, so 10^5 entries take 3 rounds
// of dependent loads instead of 17.  Must be called by all 64 lanes of a wave.
__device__ __forceinline__ int wave_find_owner(const int64_t* __restrict__ start, int n, int64_t g) {
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = n - 1;  // start[lo] <= g; the answer is in [lo, hi]
    while (hi > lo) {
        const int64_t span = hi - lo;
        // probe l: lo + ceil(span * (l + 1) / 64), ascending in l, probe 63 = hi
        const int pl = lo + (int)((span * (lane + 1) + 63) / 64);
        const unsigned long long ok = __ballot(start[pl] <= g);
        const int nk = __popcll(ok);  // ok holds for probes 0 .. nk-1
        const int nlo = nk ? lo + (int)((span * nk + 63) / 64) : lo;
        const int nhi = nk < 64 ? lo + (int)((span * (nk + 1) + 63) / 64) - 1 : hi;
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// ---------------------------------------------------------------------- DP
//
// Score-only layout (TB = false): plain values, descriptor {tr, z, r+d(i+1),
// a(i)}; r+d(i), r+d(i-1), a(i-1), a(i-2) are carried in registers.
// Traceback layout (TB = true): H is 16*H; I, D, A, B, C are 16*v + their
// fixed nibble (13, 12, 7, 6, 5); descriptor {tr, z+15, 5-16(r+d(i+1)),
// 16a(i)}, the same rows carried: C opens at H - 16(r+d(i+1)) + 5, B at
// H - 16(r+d(i)) + 6 (the previous row's field plus one), A at
// H - 16(r+d(i-1)) + 7 (the field of two rows up plus two), one three-input
// add each.
// H winner codes: 0 start, 1 M, 2 I, 3 D, 4 F1, 5 F2, 6 G1, 7 G2, 8 A, 9 B,
// 10 C; nibble = 15 - code.

// SEG: the kernel also runs two pairs' last strips on lane segments of one
// wavefront; the second pair's descriptor ring follows the other areas, and
// its incoming boundary takes the outgoing boundary's area (a last strip
// publishes no boundary).
template <int K, bool TB, bool SEG = false>
struct LdsLayout {
    static constexpr int DS = 16;              // descriptor bytes per row
    static constexpr int PS = TB ? 2 : 1;      // profile entry bytes
    static constexpr int SW = 64 * K;          // strip width
    static constexpr int RING = 128 * DS;      // two chunks of descriptors
    static constexpr int PROF = 25 * SW * PS;  // profile: 24 aa + poison row
    static constexpr int IN = 64 * 8;          // incoming boundary of the chunk
    // outgoing boundary, then the other lanes' dummy slots (one per lane and
    // step at width 2, one per lane otherwise)
    static constexpr int OUT = (K == 2 ? 192 : 128) * 8;
    static constexpr int MAT = 640;            // substitution matrix, then the letter codes
    static constexpr int RING2 = RING + PROF + IN + OUT + MAT;  // SEG: second ring
    static constexpr int WAVE = RING2 + (SEG ? RING : 0);
};

// Sentinels per layout.  The floor modes keep -infinity small enough that a
// shifted end-tracking key of any sentinel-derived value stays negative.
template <int MODE, bool TB>
struct Sentinel {
    static constexpr int NEG = floor_mode(MODE) ? (TB ? -(1 << 29) : -(1 << 25)) : -(1 << 30);
    static constexpr int UNREACH = floor_mode(MODE) ? NEG / 2 : -(1 << 29);
};

// a + b + k in one instruction (left to itself, the compiler shares b + k
// between a lane's columns and spends two)
template <int k>
__device__ __forceinline__ int add3k(int a, int b) {
    int r;
    asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "i"(k));
    return r;
}

// acc = 2*acc + (diff < 0) in every lane, one funnel shift: the choice of a
// gap or intron state, one bit per step, most recent step in bit 0.  diff =
// extension - opening, so the bit is 1 where the state opened (opening
// strictly better: extension wins ties).  All values lie within 2^31 of each
// other (planner's score bound), so the difference never overflows.
__device__ __forceinline__ uint32_t push_open(uint32_t acc, int diff) {
    return __builtin_amdgcn_alignbit(acc, (uint32_t)diff, 31);
}

// Per-pair state shared by the waves that work on the pair's strips.
struct PairState {
    unsigned long long key;  // best end-cell key over the finished strips
    int done;                // strips finished
    int gsc;                 // GLOBAL: H(n, m)
    int bad;                 // a bounded wait gave up
    int pad;
};

// Device-scope relaxed atomics: coherent across every CU and XCD without
// cache-wide fences (loads and stores carry the device-scope cache bits).
__device__ __forceinline__ int ld_dev(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int2 ld_dev2(const int2* p) {
    const unsigned long long v = __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
    return make_int2((int)(uint32_t)v, (int)(uint32_t)(v >> 32));
}
__device__ __forceinline__ void st_dev2(int2* p, int2 v) {
    const unsigned long long u = (unsigned long long)(uint32_t)v.x |
                                 ((unsigned long long)(uint32_t)v.y << 32);
    __hip_atomic_store((unsigned long long*)p, u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// s_waitcnt encoding (gfx9 family): vmcnt in bits 3:0 and 15:14, expcnt in
// 6:4, lgkmcnt in 11:8.  vmcnt(1) with the other counters left free: every
// vector memory operation but the most recent one has completed (they retire
// in issue order).
constexpr int kWaitVm1 = 0x0F71;

// Write a result record, its status last (after a system-scope fence when the
// record lives in host memory that the host polls).
__device__ __forceinline__ void publish(mpg_dev_result* rec, const mpg_dev_result& R, int system) {
    rec->score = R.score;
    rec->g_beg = R.g_beg;
    rec->g_end = R.g_end;
    rec->p_beg = R.p_beg;
    rec->p_end = R.p_end;
    rec->ops_off = R.ops_off;
    rec->ops_len = R.ops_len;
    rec->_pad = 0;
    if (system) {
        __threadfence_system();
        __hip_atomic_store(&rec->status, R.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    } else {
        // read only after the kernel has ended (by later kernels or the
        // host): no fence
        rec->status = R.status;
    }
}

// Bounded wait until the left strip has published `target` chunks.  Gives up
// after `limit` polls (kMaxPolls: well under a second) so no wave can spin
// forever; the pair then reports MPG_E_DEVICE.  A limit of 0 gives up at
// once (the host sets it to exercise that path).
// The polled value goes through readfirstlane: the loop exit is then uniform
// for the compiler too, so the wave never runs it in divergent form.
__device__ __forceinline__ bool wait_prog(const int* flag, int target, int limit) {
    for (int it = 0; it < limit; ++it) {
        if (__builtin_amdgcn_readfirstlane(ld_dev(flag)) >= target) return true;
        __builtin_amdgcn_s_sleep(2);
    }
    return false;
}

// Result record of a LOCAL score-only pair from its end key (score, -i, -j).
__device__ __forceinline__ void local_record(mpg_dev_result& R, const PairJob& J,
                                             unsigned long long ku, bool bad) {
    R.g_beg = -1;
    R.p_beg = -1;
    R.ops_off = J.ops_off;
    R.ops_len = 0;
    R._pad = 0;
    if (bad) {
        R.status = MPG_E_DEVICE;
        R.score = 0;
        R.g_end = -1;
        R.p_end = -1;
    } else {
        R.status = MPG_OK;
        R.score = (int)(ku >> 36) - (1 << 27);
        R.g_end = (1 << 21) - 1 - (int)((ku >> 15) & ((1u << 21) - 1));
        R.p_end = (1 << 15) - 1 - (int)(ku & ((1u << 15) - 1));
    }
}

// Two LOCAL pairs' last strips on lane segments of one wavefront (a strip
// that fills only part of its lanes leaves the rest idle for all its steps).
// item = (pair A, -1 - (pair B << 6 | split)): pair A's last strip in lanes
// [0, split), pair B's in [split, 64); both strips run the same number of
// chunks.  Each lane works on its own pair's rows (the segment's lane k at
// step s on row s - k), reads its pair's descriptors from that pair's LDS
// ring and takes its left neighbour's H and I by the same DPP shift as a
// whole-wave strip; the first lane of each segment takes them from its pair's
// incoming boundary instead (one select per value and step).  A pair of one
// strip starts from the -infinity column; otherwise its previous strip
// streams the boundary through HBM as for any strip.  With traceback (batch
// calls, walked afterwards by the walk kernel) each lane stores its direction
// bits into its own pair's block of the strip at its lane within the
// segment: the layout of a whole-wave strip.
template <int K, bool TB, bool NOI, bool NOF>
__device__ __forceinline__ void seg_item(const int2 item, const PairJob* __restrict__ jobs,
                                         PairState* __restrict__ pst, int* __restrict__ prog_g,
                                         const uint8_t* __restrict__ prot,
                                         const uint8_t* __restrict__ desc, int2* __restrict__ bnd,
                                         uint8_t* __restrict__ tbbuf, const DpSink& sink,
                                         const DevParams& P, uint8_t* smem, const int8_t* smat,
                                         const uint8_t* saa) {
    using LY = LdsLayout<K, TB, true>;
    constexpr int NEG = Sentinel<MPG_LOCAL, TB>::NEG;
    constexpr int UNREACH = Sentinel<MPG_LOCAL, TB>::UNREACH;
    const int lane = threadIdx.x & 63;
    const int code = -1 - item.y;
    const int ja = item.x, jb = code >> 6, split = code & 63;
    const PairJob JA = jobs[ja], JB = jobs[jb];
    const bool sg = lane >= split;            // lane of pair B
    const bool first = lane == 0 || lane == split;
    const int kk = sg ? lane - split : lane;  // lane within its segment
    const int nA = JA.n, nB = JB.n;
    const int n_l = sg ? nB : nA, m_l = sg ? JB.m : JA.m;
    const int nchunks = JA.nchunks;
    const int stripA = JA.nstrips - 1, stripB = JB.nstrips - 1;
    const int col0 = (sg ? stripB : stripA) * LY::SW + kk * K;
    const uint8_t* dscA = desc + JA.desc_off;
    const uint8_t* dscB = desc + JB.desc_off;
    const uint8_t* dsc_l = sg ? dscB : dscA;
    const uint8_t* Pa = prot + (sg ? JB.prot_off : JA.prot_off);
    const int2* bndA = bnd + JA.bnd_off;
    const int2* bndB = bnd + JB.bnd_off;
    const int* progA = prog_g + JA.prog_off;
    const int* progB = prog_g + JB.prog_off;
    const bool leftA = stripA > 0, leftB = stripB > 0;
    // traceback: this lane's direction-bit blocks (its pair's last strip)
    uint8_t* tb_l = TB ? tbbuf + (sg ? JB.tb_off : JA.tb_off) +
                             (int64_t)(sg ? stripB : stripA) * nchunks * (kTbBlockBytes * K)
                       : nullptr;
    uint8_t* ringA = smem;
    uint8_t* ringB = smem + LY::RING2;
    uint8_t* prof = smem + LY::RING;
    int2* inbA = (int2*)(smem + LY::RING + LY::PROF);
    int2* inbB = (int2*)(smem + LY::RING + LY::PROF + LY::IN);
    // penalties in the layout of the variant (as in the whole-wave strips)
    const int cq = TB ? 16 * (P.q + P.e) - 13 : P.q;
    const int cqD = TB ? 16 * (P.q + P.e) - 12 : P.q;
    const int ce = TB ? 16 * P.e : P.e;
    const int cf = TB ? 16 * P.f : P.f;
    int cf11 = cf - 11, cf9 = cf - 9;
    asm volatile("" : "+s"(cf11), "+s"(cf9));
    const int2 neg2 = make_int2(NEG, NEG);

    // profile of this lane's columns (its own pair's residues)
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const int j = col0 + c;
        int pc = -1;
        if (j >= 1 && j <= m_l) {
            const uint32_t ch = Pa[j - 1];
            const uint32_t u = (ch | 0x20u) - 'a';
            pc = ch == '*' ? 23 : (u < 26u ? saa[u] : 22);
        }
        int sv[24];
#pragma unroll
        for (int tr = 0; tr < 24; ++tr) sv[tr] = pc < 0 ? 0 : (int)smat[tr * 24 + pc];
#pragma unroll
        for (int tr = 0; tr < 25; ++tr) {
            const bool poison = pc < 0 || tr == 24;
            const int v = tr < 24 ? sv[tr < 24 ? tr : 0] : 0;
            if (TB)
                ((int16_t*)prof)[(c * 25 + tr) * 64 + lane] =
                    (int16_t)(poison ? -32768 : 16 * v + 14);
            else
                ((int8_t*)prof)[(c * 25 + tr) * 64 + lane] = (int8_t)(poison ? -128 : v);
        }
    }
    int h1[K], h2[K], h3[K], d1[K], d2[K], d3[K], a1[K], b1[K], c1[K];
    int best[K], bstep[K], bk[K], fp[K];
    uint32_t nacc[K], xacc[5][K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        h1[c] = h2[c] = h3[c] = NEG;
        d1[c] = d2[c] = d3[c] = NEG;
        a1[c] = b1[c] = c1[c] = NEG;
        best[c] = NEG;
        bstep[c] = 0;
        bk[c] = INT_MIN;
        fp[c] = TB ? NEG - cf11 : NEG - cf;
        nacc[c] = 0;
#pragma unroll
        for (int x = 0; x < 5; ++x) xacc[x][c] = 0;
    }
    int hl1 = NEG, hl2 = NEG, hl3 = NEG;
    int Hout = NEG, Iout = NEG;
    int dd0, ddm1, aam1, aam2;
    {
        const int4 u = *(const int4*)(dsc_l + (int64_t)(-kk - 1 + kDescLo) * LY::DS);
        const int4 v = *(const int4*)(dsc_l + (int64_t)(-kk - 2 + kDescLo) * LY::DS);
        dd0 = u.z; aam1 = u.w; ddm1 = v.z; aam2 = v.w;
    }
    // both rings: rows -64..-1 then 0..63 of each pair
    {
        const int4 a0 = *(const int4*)(dscA + (int64_t)(lane - 64 + kDescLo) * LY::DS);
        const int4 a1v = *(const int4*)(dscA + (int64_t)(lane + kDescLo) * LY::DS);
        const int4 b0 = *(const int4*)(dscB + (int64_t)(lane - 64 + kDescLo) * LY::DS);
        const int4 b1v = *(const int4*)(dscB + (int64_t)(lane + kDescLo) * LY::DS);
        *(int4*)(ringA + lane * LY::DS) = a0;
        *(int4*)(ringA + (64 + lane) * LY::DS) = a1v;
        *(int4*)(ringB + lane * LY::DS) = b0;
        *(int4*)(ringB + (64 + lane) * LY::DS) = b1v;
    }
    inbA[lane] = neg2;
    inbB[lane] = neg2;
    bool failed = false;
    int2 nbA = neg2, nbB = neg2;
    int seenA = 0, seenB = 0;
    if (leftA) {
        if (!wait_prog(&progA[stripA - 1], nchunks < 2 ? nchunks : 2, P.max_polls)) failed = true;
        nbA = ld_dev2(&bndA[kBndLo + lane]);
        seenA = ld_dev(&progA[stripA - 1]);
    }
    if (leftB) {
        if (!wait_prog(&progB[stripB - 1], nchunks < 2 ? nchunks : 2, P.max_polls)) failed = true;
        nbB = ld_dev2(&bndB[kBndLo + lane]);
        seenB = ld_dev(&progB[stripB - 1]);
    }
    int4 pfA = make_int4(0, 0, 0, 0), pfB = make_int4(0, 0, 0, 0);
    // this lane's ring and incoming rows; at width 2 as one LDS offset each,
    // opaque to the compiler: a select of the two pairs' areas is distributed
    // over the steps' addresses, which are invariant across chunks, and the
    // compiler hoists all of them into registers, which width 2 spills (the
    // widths that run one wave per SIMD hold them; see the outgoing rows)
    int ring_off = sg ? LY::RING2 : 0;
    int inb_off = sg ? LY::RING + LY::PROF + LY::IN : LY::RING + LY::PROF;
    if constexpr (K == 2) asm volatile("" : "+v"(ring_off), "+v"(inb_off));
    const uint8_t* ring_l = K != 2 ? (sg ? ringB : ringA) : smem + ring_off;
    const int2* inb_l = K != 2 ? (sg ? inbB : inbA) : (const int2*)(smem + inb_off);

    for (int ch = 0; ch < nchunks && !failed; ++ch) {
        // incoming boundary rows ch*64 .. ch*64+63 of each pair with a left strip
        if (leftA) {
            inbA[lane] = ch * 64 + lane > nA ? neg2 : nbA;
            if (ch + 1 < nchunks) {
                const int need = ch + 3 < nchunks ? ch + 3 : nchunks;
                if (__builtin_amdgcn_readfirstlane(seenA) < need &&
                    !wait_prog(&progA[stripA - 1], need, P.max_polls)) {
                    failed = true;
                    break;
                }
                nbA = ld_dev2(&bndA[kBndLo + (ch + 1) * 64 + lane]);
                seenA = ld_dev(&progA[stripA - 1]);
            }
        }
        if (leftB) {
            inbB[lane] = ch * 64 + lane > nB ? neg2 : nbB;
            if (ch + 1 < nchunks) {
                const int need = ch + 3 < nchunks ? ch + 3 : nchunks;
                if (__builtin_amdgcn_readfirstlane(seenB) < need &&
                    !wait_prog(&progB[stripB - 1], need, P.max_polls)) {
                    failed = true;
                    break;
                }
                nbB = ld_dev2(&bndB[kBndLo + (ch + 1) * 64 + lane]);
                seenB = ld_dev(&progB[stripB - 1]);
            }
        }
        if (ch > 0) {
            const int4 oA = *(const int4*)(ringA + (64 + lane) * LY::DS);
            const int4 oB = *(const int4*)(ringB + (64 + lane) * LY::DS);
            *(int4*)(ringA + lane * LY::DS) = oA;
            *(int4*)(ringA + (64 + lane) * LY::DS) = pfA;
            *(int4*)(ringB + lane * LY::DS) = oB;
            *(int4*)(ringB + (64 + lane) * LY::DS) = pfB;
        }
        pfA = *(const int4*)(dscA + (int64_t)((ch + 1) * 64 + lane + kDescLo) * LY::DS);
        pfB = *(const int4*)(dscB + (int64_t)((ch + 1) * 64 + lane + kDescLo) * LY::DS);
        const uint8_t* rb = ring_l + (64 - kk) * LY::DS;
        auto ld_prof = [&](const int4& x0, int* scv) {
            if (TB) {
                const int16_t* pr = (const int16_t*)prof + x0.x * 64 + lane;
#pragma unroll
                for (int c = 0; c < K; ++c) scv[c] = pr[c * 25 * 64];
            } else {
                const int8_t* pr = (const int8_t*)prof + x0.x * 64 + lane;
#pragma unroll
                for (int c = 0; c < K; ++c) scv[c] = pr[c * 25 * 64];
            }
        };
        uint8_t* tbblk = TB ? tb_l + (int64_t)ch * (kTbBlockBytes * K) : nullptr;
        int4 cd0 = *(const int4*)(rb), nd0 = *(const int4*)(rb + LY::DS);
        int csc[K];
        ld_prof(cd0, csc);
        int2 cin = inb_l[0];
#pragma unroll
        for (int t = 0; t < 64; ++t) {
            int4 fd0 = make_int4(0, 0, 0, 0);
            if (t + 2 < 64) fd0 = *(const int4*)(rb + (t + 2) * LY::DS);
            int nsc[K];
            int2 nin = make_int2(0, 0);
            if (t + 1 < 64) {
                ld_prof(nd0, nsc);
                nin = inb_l[t + 1];
            }
            const int4 ds0 = cd0;
            // a segment's first lane takes its own pair's boundary (the
            // shift's own lane 0 value is replaced too, so the shift needs no
            // copy of the boundary value as its old operand)
            int hl0, il0;
            if constexpr (K == 2) {
                hl0 = __builtin_amdgcn_mov_dpp(Hout, kShr1, 0xF, 0xF, true);
                il0 = __builtin_amdgcn_mov_dpp(Iout, kShr1, 0xF, 0xF, true);
            } else {
                hl0 = shr1(cin.x, Hout);
                il0 = shr1(cin.y, Iout);
            }
            hl0 = first ? cin.x : hl0;
            il0 = first ? cin.y : il0;
            const int z = ds0.y;
            int Hn[K], In[K], Dn[K], An[K], Bn[K], Cn[K];
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const int L0 = c ? Hn[c - 1] : hl0;
                const int IL = c ? In[c - 1] : il0;
                const int L1 = c ? h1[c - 1] : hl1;
                const int L3 = c ? h3[c - 1] : hl3;
                if (!TB) {
                    const int D = imax(h3[c] - cq, d3[c]) - ce;
                    const int I = imax(L0 - cq, IL) - ce;
                    const int M = L3 + csc[c];
                    int pf = 0;
                    if (!NOF) {
                        pf = imax(L1, h1[c]) - cf;
                        asm("" : "+v"(pf));
                    }
                    int H;
                    if (!NOI) {
                        const int A = imax(h1[c] - ddm1, a1[c]);
                        const int B = imax(L1 - dd0, b1[c]);
                        const int C = imax(L1 - ds0.z, c1[c]);
                        An[c] = A; Bn[c] = B; Cn[c] = C;
                        const int x = imax3(D, A - ds0.w, B - aam2);
                        if (!NOF) H = imax3(x, imax3(C - aam1, pf, fp[c]), imax3(M, I, z));
                        else H = imax3(x, imax3(C - aam1, M, I), z);
                    } else {
                        if (!NOF) H = imax(imax3(D, pf, fp[c]), imax3(M, I, z));
                        else H = imax(imax3(D, M, I), z);
                    }
                    if (!NOF) fp[c] = pf;
                    Hn[c] = H; In[c] = I; Dn[c] = D;
                } else {
                    const int oD = h3[c] - cqD, xD = d3[c] - ce;
                    xacc[1][c] = push_open(xacc[1][c], xD - oD);
                    int D = imax(oD, xD);
                    const int oI = L0 - cq, xI = IL - ce;
                    xacc[0][c] = push_open(xacc[0][c], xI - oI);
                    int I = imax(oI, xI);
                    const int M = L3 + csc[c];
                    int p1 = 0, p2 = 0;
                    if (!NOF) {
                        p1 = imax(L1 - cf11, h1[c] - cf9);
                        asm("" : "+v"(p1));
                        p2 = fp[c] - 1;
                        fp[c] = p1;
                    }
                    asm("" : "+v"(D), "+v"(I));
                    int Hk;
                    if (!NOI) {
                        const int oA = add3k<2>(h1[c], ddm1);
                        xacc[2][c] = push_open(xacc[2][c], a1[c] - oA);
                        int A = imax(oA, a1[c]);
                        const int oB = add3k<1>(L1, dd0);
                        xacc[3][c] = push_open(xacc[3][c], b1[c] - oB);
                        int B = imax(oB, b1[c]);
                        const int oC = L1 + ds0.z;
                        xacc[4][c] = push_open(xacc[4][c], c1[c] - oC);
                        int C = imax(oC, c1[c]);
                        asm("" : "+v"(A), "+v"(B), "+v"(C));
                        An[c] = A; Bn[c] = B; Cn[c] = C;
                        const int x = imax3(D, A - ds0.w, B - aam2);
                        if (!NOF) Hk = imax3(x, imax3(C - aam1, p1, p2), imax3(M, I, z));
                        else Hk = imax3(x, imax3(C - aam1, M, I), z);
                    } else {
                        if (!NOF) Hk = imax(imax3(D, p1, p2), imax3(M, I, z));
                        else Hk = imax(imax3(D, M, I), z);
                    }
                    nacc[c] = __builtin_amdgcn_alignbit(Hk, nacc[c], 4);
                    Hn[c] = Hk & ~15;
                    In[c] = I; Dn[c] = D;
                }
            }
#pragma unroll
            for (int c = 0; c < K; ++c)
                bk[c] = imax(bk[c], (Hn[c] << (TB ? 2 : 6)) | (63 - t));
            if (TB && (t & 7) == 7) {
#pragma unroll
                for (int c = 0; c < K; ++c)
                    *(uint32_t*)(tbblk + (((t >> 3) * K + c) * 64 + kk) * 4) = nacc[c];
            }
            if (TB && (t & 31) == 31) {
#pragma unroll
                for (int x = 0; x < 5; ++x) {
                    if (NOI && x >= 2) continue;
#pragma unroll
                    for (int c = 0; c < K; ++c)
                        *(uint32_t*)(tbblk + 2048 * K +
                                     (((x * K + c) * 2 + (t >> 5)) * 64 + kk) * 4) = xacc[x][c];
                }
            }
            hl3 = hl2; hl2 = hl1; hl1 = hl0;
#pragma unroll
            for (int c = 0; c < K; ++c) {
                h3[c] = h2[c]; h2[c] = h1[c]; h1[c] = Hn[c];
                d3[c] = d2[c]; d2[c] = d1[c]; d1[c] = Dn[c];
                if (!NOI) { a1[c] = An[c]; b1[c] = Bn[c]; c1[c] = Cn[c]; }
            }
            ddm1 = dd0; dd0 = ds0.z; aam2 = aam1; aam1 = ds0.w;
            Hout = Hn[K - 1];
            Iout = In[K - 1];
            cd0 = nd0; nd0 = fd0;
#pragma unroll
            for (int c = 0; c < K; ++c) csc[c] = nsc[c];
            cin = nin;
            if (TB ? MPG_TB_STEP_BARRIER : MPG_STEP_BARRIER) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int c = 0; c < K; ++c) {
            int v = bk[c] >> 6;
            const int tt = 63 - (bk[c] & 63);
            if (TB) v <<= 4;  // back to 16*H units
            if (v > best[c]) { best[c] = v; bstep[c] = ch * 64 + tt; }
            bk[c] = INT_MIN;
        }
    }

    // each pair's best cell over its own lanes, folded into the pair
    uint64_t key = 0;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const int row = bstep[c] - kk, col = col0 + c;
        if (col <= m_l && row >= 0 && row <= n_l && best[c] > UNREACH) {
            const uint64_t k2 = end_key(TB ? (best[c] >> 4) : best[c], row, col);
            key = k2 > key ? k2 : key;
        }
    }
    const uint64_t keyA = wave_max_u64(sg ? 0 : key), keyB = wave_max_u64(sg ? key : 0);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const PairJob& J = q ? JB : JA;
        PairState* ps = pst + (q ? jb : ja);
        const unsigned long long k = q ? keyB : keyA;
        const bool solo = J.nstrips == 1;
        int done = 0;
        if (!solo) {
            if (lane == 0) {
                if (failed) atomicMax(&ps->bad, 1);
                else if (k) atomicMax(&ps->key, k);
            }
            __builtin_amdgcn_s_waitcnt(0);
            if (lane == 0)
                done = __hip_atomic_fetch_add(&ps->done, 1, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
            done = __builtin_amdgcn_readfirstlane(done);
        }
        if (done == J.nstrips - 1) {
            const unsigned long long kf =
                solo ? k : __hip_atomic_load(&ps->key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool bad =
                solo ? failed : __builtin_amdgcn_readfirstlane(ld_dev(&ps->bad)) != 0;
            const uint32_t khi = __builtin_amdgcn_readfirstlane((uint32_t)(kf >> 32));
            const uint32_t klo = __builtin_amdgcn_readfirstlane((uint32_t)kf);
            mpg_dev_result R;
            local_record(R, J, ((unsigned long long)khi << 32) | klo, bad);
            if (lane == 0) publish(sink.out + J.res, R, sink.system);
        }
    }
}

// The DP kernel.  Persistent single-wavefront workgroups take (pair, strip)
// work items from one queue ordered longest pair first, strips in order.  A
// strip streams its left boundary (H and I of the previous strip's last
// column) from HBM as the previous strip publishes it chunk by chunk, so the
// strips of a long pair run as a pipeline spread over many CUs, and every
// wavefront slot stays busy until the queue is empty.  Dependencies only point
// to items taken earlier by running wavefronts, so the waits always end.
// PRO: the query is a position-specific profile block (prof_scores /
// prof_gaps) instead of protein letters and one matrix.
template <int K, int MODE, bool TB, bool NOI, bool NOF, bool PRO>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(WavesPerEu<K, TB>::value)))
dp_kernel(const PairJob* __restrict__ jobs, const int2* __restrict__ items, int nitems,
          int* __restrict__ qhead, PairState* __restrict__ pst, int* __restrict__ prog_g,
          const uint8_t* __restrict__ prot, const uint8_t* __restrict__ desc,
          int2* __restrict__ bnd, uint8_t* __restrict__ tbbuf, DpSink sink, DevParams P) {
    // LOCAL launches also run lane-segment items (two pairs' last strips in
    // one wavefront)
    constexpr bool SEGOK = MODE == MPG_LOCAL && !PRO;
    using LY = LdsLayout<K, TB, SEGOK>;
    // the mixed variant runs EXTEND and fixed-end pairs (per-pair modes)
    constexpr bool MIXED = MODE == kModeMixed;
    constexpr int SM = MIXED ? (int)MPG_GLOBAL : MODE;  // mode of the sentinels and the floor
    constexpr int NEG = Sentinel<SM, TB>::NEG;
    constexpr int UNREACH = Sentinel<SM, TB>::UNREACH;
    constexpr int ZN = TB ? 15 : 0;  // nibble of the start candidate
    // The first column's I term takes the left lane's I as a DPP operand of
    // the max (score-only) or subtraction (traceback) that consumes it.
    // Timed on the 10k batch: 3% faster at one column per lane, 1% with
    // traceback, not faster in the score-only kernels of wider lanes.
    constexpr bool FUSE_I = TB || K == 1;
    extern __shared__ __align__(16) uint8_t smem[];
    const int lane = threadIdx.x & 63;
    uint8_t* ring = smem;
    uint8_t* prof = smem + LY::RING;
    int2* inb = (int2*)(smem + LY::RING + LY::PROF);
    int2* outb = (int2*)(smem + LY::RING + LY::PROF + LY::IN);
    // step t's outgoing row: lane 63 writes slot t, lane l < 63 a dummy slot,
    // never read.  A per-step select of the slot is invariant across chunks,
    // and the compiler hoists all 64 of them into registers.  Width 2 (three
    // or four waves per SIMD) spills them, and every reload waited for the
    // chunk's direction-bit stores, so it writes slot 64 + l + t through one
    // base per lane with the step in the store's immediate offset (traceback
    // batch DP 26.3 -> 25.4 ms with the packed strips' offsets below).  The
    // other widths keep the select: built without the hoisted registers they
    // run more waves per SIMD, which slows the long-tail batch (280 -> 331 ms)
    // and doubles the serving latency (p50 1.9 -> 3.9 ms).
    int2* const outw = outb + (lane == 63 ? 0 : 64 + lane);
    int8_t* smat = (int8_t*)(smem + LY::RING + LY::PROF + LY::IN + LY::OUT);
    uint8_t* saa = (uint8_t*)(smat + 24 * 24);
    // the matrix and the letter codes, read with per-lane indices when a
    // strip's profile is built, are staged in LDS once per launch
    for (int k = lane; k < 24 * 24 / 4; k += 64)
        ((int*)smat)[k] = ((const int*)P.mat)[k];  // 4-byte aligned in both
    if (lane < 26) saa[lane] = kAaOfLetter[lane];
    __syncthreads();
    auto aa_lds = [&](uint32_t ch) -> int {
        if (ch == '*') return 23;
        const uint32_t u = (ch | 0x20u) - 'a';
        return u < 26u ? saa[u] : 22;
    };

    // penalties in the layout of this variant
    const int cq = TB ? 16 * (P.q + P.e) - 13 : P.q;   // I open  (TB: nibble 13)
    const int cqD = TB ? 16 * (P.q + P.e) - 12 : P.q;  // D open  (TB: nibble 12)
    const int ce = TB ? 16 * P.e : P.e;
    const int cf = TB ? 16 * P.f : P.f;
    // traceback: the F1 and G1 candidates' offsets (16f less their nibbles),
    // kept opaque so that the compiler does not share H - 16f between them
    // and add each nibble with a separate instruction
    int cf11 = cf - 11, cf9 = cf - 9;
    asm volatile("" : "+s"(cf11), "+s"(cf9));

    // Items are taken when the previous one is done (claiming ahead would
    // hold a strip that the next strip of its pair then waits for).
    for (;;) {
        // take the next item without a divergent branch: lane 0 adds 1, the
        // other lanes add 0, so lane 0 always receives the old head; its value
        // through readfirstlane is wave-uniform, which keeps the loop exit
        // uniform, so no cross-lane operation below ever runs with part of
        // the wave masked off
        const int it = __builtin_amdgcn_readfirstlane(atomicAdd(qhead, lane == 0 ? 1 : 0));
        if (it >= nitems) break;
        const int2 item = items[it];
        if constexpr (SEGOK) {
            if (item.y < 0) {
                seg_item<K, TB, NOI, NOF>(item, jobs, pst, prog_g, prot, desc, bnd, tbbuf, sink,
                                          P, smem, smat, saa);
                continue;
            }
        }
        const PairJob J = jobs[item.x];
        const int strip = item.y;
        const int n = J.n, m = J.m;
        const int nchunks = J.nchunks, nstrips = J.nstrips;
        const uint8_t* dsc_g = desc + J.desc_off;  // row r at (r + kDescLo) * DS
        int2* bnd_g = bnd + J.bnd_off;             // row r at r + kBndLo
        const uint8_t* Pa = prot + J.prot_off;
        uint8_t* tbp = tbbuf + J.tb_off;
        int* prog = prog_g + J.prog_off;           // chunks published, per strip
        PairState* ps = pst + item.x;
        const bool has_next = strip + 1 < nstrips;
        const int col0 = strip * LY::SW + lane * K;  // DP column of this lane's first column
        const bool act = true;
        bool failed = false;
        uint64_t best_key = 0;

        // ---- strip set-up: profile, registers, first descriptors and boundary
        if (act) {
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const int j = col0 + c;
                const int pc = (j >= 1 && j <= m) ? (PRO ? 0 : aa_lds(Pa[j - 1])) : -1;
                // all 24 entries are read before any is stored, so the reads
                // overlap
                int sv[24];
#pragma unroll
                for (int tr = 0; tr < 24; ++tr)
                    sv[tr] = pc < 0 ? 0
                                    : (PRO ? (int)prof_scores(Pa)[24 * (j - 1) + tr]
                                           : (int)smat[tr * 24 + pc]);
#pragma unroll
                for (int tr = 0; tr < 25; ++tr) {
                    const bool poison = pc < 0 || tr == 24;
                    const int v = tr < 24 ? sv[tr < 24 ? tr : 0] : 0;
                    // column c of every lane in a row of its own, so that each
                    // step reads one sign-extended entry per column
                    if (TB)
                        ((int16_t*)prof)[(c * 25 + tr) * 64 + lane] =
                            (int16_t)(poison ? -32768 : 16 * v + 14);
                    else
                        ((int8_t*)prof)[(c * 25 + tr) * 64 + lane] = (int8_t)(poison ? -128 : v);
                }
            }
        }

        // gap costs of this lane's columns in the layout of the variant (a
        // profile's own per column; columns beyond m take column m's)
        int cqv[K], cqDv[K], cev[K], ceDv[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            if (PRO) {
                const int16_t* g = prof_gaps(Pa, m) + 4 * imin(col0 + c, m);
                const int oi = g[0], ei = g[1], od = g[2], ed = g[3];
                cqv[c] = TB ? 16 * (oi + ei) - 13 : oi;
                cev[c] = TB ? 16 * ei : ei;
                cqDv[c] = TB ? 16 * (od + ed) - 12 : od;
                ceDv[c] = TB ? 16 * ed : ed;
            } else {
                cqv[c] = cq;
                cev[c] = ce;
                cqDv[c] = cqD;
                ceDv[c] = ce;
            }
        }
        // With FUSE_I the incoming boundary rows are kept with their I part
        // pre-combined for the first column of the strip, as lane 0 needs it
        // (the other lanes take the same terms from their left neighbour
        // within the step): score-only max(H - q, I), traceback I less the
        // extension.
        const int cq0 = __builtin_amdgcn_readfirstlane(cqv[0]);
        const int ce0 = __builtin_amdgcn_readfirstlane(cev[0]);
        auto in_row = [&](int2 w) {
            if (!FUSE_I) return w;
            return make_int2(w.x, TB ? w.y - ce0 : imax(w.x - cq0, w.y));
        };
        if (act) inb[lane] = in_row(make_int2(NEG, NEG));
        int h1[K], h2[K], h3[K], d1[K], d2[K], d3[K], a1[K], b1[K], c1[K];
        int zl[K], best[K], bstep[K], bk[K], bkt[K], hn[K];
        int fp[K];  // previous row's frameshift term (F1/G1 maximum)
        uint32_t nacc[K];
        uint32_t xacc[5][K];  // extension decisions of the last steps, per lane
        // The fixed-end kernel also runs EXTEND_LEFT pairs: their start term
        // is the row's own (0 on every valid row), so the column term is
        // lifted out of the minimum.
        const bool floor0 = (MIXED || fixed_end_mode(MODE)) && J.mode == MPG_EXTEND_LEFT;
        // the pair ends at (n, m) (a compile-time constant but in the mixed variant)
        const bool fixed = MIXED ? J.mode != MPG_EXTEND : fixed_end_mode(MODE);
#pragma unroll
        for (int c = 0; c < K; ++c) {
            h1[c] = h2[c] = h3[c] = NEG;
            d1[c] = d2[c] = d3[c] = NEG;
            a1[c] = b1[c] = c1[c] = NEG;
            zl[c] = floor0 ? INT_MAX : ((col0 + c == 0) ? ZN : NEG + ZN);
            best[c] = NEG;
            bstep[c] = 0;
            bk[c] = INT_MIN;
            bkt[c] = 0;
            hn[c] = NEG;
            // the frameshift term of the row above the strip's first (every
            // H there is -infinity)
            fp[c] = TB ? NEG - cf11 : NEG - cf;
            nacc[c] = 0;
#pragma unroll
            for (int x = 0; x < 5; ++x) xacc[x][c] = 0;
        }
        int hl1 = NEG, hl2 = NEG, hl3 = NEG;
        int Hout = NEG, Iout = NEG;
        // registers carrying the previous two rows' donor and acceptor fields
        // (score-only: r+d(i), r+d(i-1), a(i-1), a(i-2))
        int dd0 = 0, ddm1 = 0, aam1 = 0, aam2 = 0;
        if (act) {
            const int4 u = *(const int4*)(dsc_g + (int64_t)(-lane - 1 + kDescLo) * LY::DS);
            const int4 v = *(const int4*)(dsc_g + (int64_t)(-lane - 2 + kDescLo) * LY::DS);
            dd0 = u.z; aam1 = u.w; ddm1 = v.z; aam2 = v.w;
        }
        // descriptor ring: rows -64..-1 then 0..63
        int4 pf0 = make_int4(0, 0, 0, 0);
        if (act) {
            // all loads first, then the stores
            const uint8_t* src = dsc_g + (int64_t)(lane - 64 + kDescLo) * LY::DS;
            const uint8_t* src2 = dsc_g + (int64_t)(lane + kDescLo) * LY::DS;
            const int4 r0 = *(const int4*)src, r2 = *(const int4*)src2;
            *(int4*)(ring + lane * LY::DS) = r0;
            *(int4*)(ring + (64 + lane) * LY::DS) = r2;
        }
        int2 nb = make_int2(NEG, NEG);
        // the left strip's last column arrives from HBM as that strip
        // publishes it; rows of chunk c need its chunks c and c+1.  Its
        // progress counter is read one chunk ahead, so the check at a chunk
        // start normally finds the value loaded long before and never waits.
        const bool from_left = strip > 0;
        int seen = 0;
        if (from_left) {
            if (!wait_prog(&prog[strip - 1], nchunks < 2 ? nchunks : 2, P.max_polls))
                failed = true;
            nb = ld_dev2(&bnd_g[kBndLo + lane]);
            seen = ld_dev(&prog[strip - 1]);
        }

        for (int ch = 0; ch < nchunks && !failed; ++ch) {
            {
                // incoming boundary rows ch*64 .. ch*64+63 (rows beyond n hold
                // garbage-row values or were never written: -infinity)
                const bool beyond = ch * 64 + lane > n;
                if (from_left) {
                    inb[lane] = in_row(beyond ? make_int2(NEG, NEG) : nb);
                    if (ch + 1 < nchunks) {
                        const int need = ch + 3 < nchunks ? ch + 3 : nchunks;
                        if (__builtin_amdgcn_readfirstlane(seen) < need &&
                            !wait_prog(&prog[strip - 1], need, P.max_polls)) {
                            failed = true;
                            break;
                        }
                        nb = ld_dev2(&bnd_g[kBndLo + (ch + 1) * 64 + lane]);
                        seen = ld_dev(&prog[strip - 1]);
                    }
                }
                if (ch > 0) {
                    // slide the descriptor ring: current chunk -> previous half
                    const int4 o0 = *(const int4*)(ring + (64 + lane) * LY::DS);
                    *(int4*)(ring + lane * LY::DS) = o0;
                    *(int4*)(ring + (64 + lane) * LY::DS) = pf0;
                }
                pf0 = *(const int4*)(dsc_g + (int64_t)((ch + 1) * 64 + lane + kDescLo) * LY::DS);
                const uint8_t* rb = ring + (64 - lane) * LY::DS;
                uint8_t* tbblk = tbp + ((int64_t)strip * nchunks + ch) * (kTbBlockBytes * K);
                const int srow_n = ch * 64 - n;  // GLOBAL: lane == t + srow_n  <=>  row == n

                // Software pipeline: descriptors are read two steps ahead, the
                // profile entries and the incoming boundary value one step ahead.
                auto ld_desc = [&](int tt, int4& x0) { x0 = *(const int4*)(rb + tt * LY::DS); };
                auto ld_prof = [&](const int4& x0, int* scv) {
                    if (TB) {
                        const int16_t* pr = (const int16_t*)prof + x0.x * 64 + lane;
#pragma unroll
                        for (int c = 0; c < K; ++c) scv[c] = pr[c * 25 * 64];
                    } else {
                        const int8_t* pr = (const int8_t*)prof + x0.x * 64 + lane;
#pragma unroll
                        for (int c = 0; c < K; ++c) scv[c] = pr[c * 25 * 64];
                    }
                };
                int4 cd0, nd0;
                ld_desc(0, cd0);
                ld_desc(1, nd0);
                int csc[K];
                ld_prof(cd0, csc);
                int2 cin = inb[0];

#pragma unroll
                for (int t = 0; t < 64; ++t) {
                    // ---- prefetch for steps t+1 and t+2
                    int4 fd0 = make_int4(0, 0, 0, 0);
                    if (t + 2 < 64) ld_desc(t + 2, fd0);
                    int nsc[K];
                    int2 nin = make_int2(0, 0);
                    if (t + 1 < 64) {
                        ld_prof(nd0, nsc);
                        nin = inb[t + 1];
                    }
                    const int4 ds0 = cd0;
                    const int hl0 = shr1(cin.x, Hout);
                    const int il0 = FUSE_I ? 0 : shr1(cin.y, Iout);
                    const int zr = ds0.y;
                    int Hn[K], In[K], Dn[K], An[K], Bn[K], Cn[K];
#pragma unroll
                    for (int c = 0; c < K; ++c) {
                        const int L0 = c ? Hn[c - 1] : hl0;
                        const int IL = c ? In[c - 1] : il0;
                        const int L1 = c ? h1[c - 1] : hl1;
                        const int L2 = c ? h2[c - 1] : hl2;
                        const int L3 = c ? h3[c - 1] : hl3;
                        const int z = floor_mode(SM) ? zr : imin(zr, zl[c]);
                        if (!TB) {
                            const int D = imax(h3[c] - cqDv[c], d3[c]) - ceDv[c];
                            // column 0 takes I(i, j-1) from the left lane inside
                            // the max (lane 0 from the boundary row)
                            const int I = (c || !FUSE_I ? imax(L0 - cqv[c], IL)
                                                        : max_from_left(cin.y, Iout, L0 - cqv[c])) -
                                          cev[c];
                            const int M = L3 + csc[c];
                            // frameshifts: F1 and G1 of this row cost f each, and F2,
                            // G2 are the previous row's F1, G1 (H two rows up is the
                            // history one row up), so one max per cell covers all four
                            int pf = 0;
                            if (!NOF) {
                                pf = imax(L1, h1[c]) - cf;
                                // opaque to the next row: the compiler would otherwise
                                // expand fp - ... back into four candidates there
                                asm("" : "+v"(pf));
                            }
                            int H;
                            if (!NOI) {
                                const int A = imax(h1[c] - ddm1, a1[c]);
                                const int B = imax(L1 - dd0, b1[c]);
                                const int C = imax(L1 - ds0.z, c1[c]);
                                An[c] = A; Bn[c] = B; Cn[c] = C;
                                const int x = imax3(D, A - ds0.w, B - aam2);
                                if (!NOF) H = imax3(x, imax3(C - aam1, pf, fp[c]), imax3(M, I, z));
                                else H = imax3(x, imax3(C - aam1, M, I), z);
                            } else {
                                if (!NOF) H = imax(imax3(D, pf, fp[c]), imax3(M, I, z));
                                else H = imax(imax3(D, M, I), z);
                            }
                            if (!NOF) fp[c] = pf;
                            Hn[c] = H; In[c] = I; Dn[c] = D;
                        } else {
                            const int oD = h3[c] - cqDv[c], xD = d3[c] - ceDv[c];
                            xacc[1][c] = push_open(xacc[1][c], xD - oD);
                            int D = imax(oD, xD);
                            const int oI = L0 - cqv[c];
                            const int xI = c || !FUSE_I ? IL - cev[c]
                                                        : sub_from_left(cin.y, Iout, cev[c]);
                            xacc[0][c] = push_open(xacc[0][c], xI - oI);
                            int I = imax(oI, xI);
                            const int M = L3 + csc[c];
                            // F1 (nibble 11) and G1 (9) of this row; F2 (10) and G2
                            // (8) are the previous row's F1 and G1 less one, so their
                            // maximum is the previous row's maximum less one
                            int p1 = 0, p2 = 0;
                            if (!NOF) {
                                p1 = imax(L1 - cf11, h1[c] - cf9);
                                // opaque to the next row: the compiler would otherwise
                                // expand fp - 1 back into four candidates there
                                asm("" : "+v"(p1));
                                p2 = fp[c] - 1;
                                fp[c] = p1;
                            }
                            // the states enter H's maximum as they are: left visible,
                            // the compiler may also build H from their two halves in a
                            // second tree (seen at one column per lane)
                            asm("" : "+v"(D), "+v"(I));
                            int Hk;
                            if (!NOI) {
                                const int oA = add3k<2>(h1[c], ddm1);
                                xacc[2][c] = push_open(xacc[2][c], a1[c] - oA);
                                int A = imax(oA, a1[c]);
                                const int oB = add3k<1>(L1, dd0);
                                xacc[3][c] = push_open(xacc[3][c], b1[c] - oB);
                                int B = imax(oB, b1[c]);
                                const int oC = L1 + ds0.z;
                                xacc[4][c] = push_open(xacc[4][c], c1[c] - oC);
                                int C = imax(oC, c1[c]);
                                asm("" : "+v"(A), "+v"(B), "+v"(C));
                                An[c] = A; Bn[c] = B; Cn[c] = C;
                                const int x = imax3(D, A - ds0.w, B - aam2);
                                if (!NOF) Hk = imax3(x, imax3(C - aam1, p1, p2), imax3(M, I, z));
                                else Hk = imax3(x, imax3(C - aam1, M, I), z);
                            } else {
                                if (!NOF) Hk = imax(imax3(D, p1, p2), imax3(M, I, z));
                                else Hk = imax(imax3(D, M, I), z);
                            }
                            nacc[c] = __builtin_amdgcn_alignbit(Hk, nacc[c], 4);
                            Hn[c] = Hk & ~15;
                            In[c] = I; Dn[c] = D;
                        }
                    }
                    // end-cell tracking (chunk-local, merged after the chunk)
                    if constexpr (MIXED) {
                        // the best cell, over every cell (EXTEND) or the
                        // cells of row n (fixed end)
                        const bool take = !fixed || lane == t + srow_n;
#pragma unroll
                        for (int c = 0; c < K; ++c) {
                            const int v = take ? Hn[c] : NEG;
                            const bool gt = v > bk[c];
                            bk[c] = gt ? v : bk[c];
                            bkt[c] = gt ? t : bkt[c];
                        }
                    } else if (fixed_end_mode(MODE)) {
                        const bool at_n = (lane == t + srow_n);
#pragma unroll
                        for (int c = 0; c < K; ++c) {
                            hn[c] = at_n ? Hn[c] : hn[c];
                            // keep the select in this step: left free, the
                            // compiler defers all 64 of them to the chunk's
                            // end, holding every step's H and mask live
                            // (about 100 more VGPRs, one wave per SIMD)
                            asm volatile("" : "+v"(hn[c]));
                        }
                    } else if (MODE == MPG_LOCAL) {
#pragma unroll
                        for (int c = 0; c < K; ++c)
                            bk[c] = imax(bk[c], (Hn[c] << (TB ? 2 : 6)) | (63 - t));
                    } else {
#pragma unroll
                        for (int c = 0; c < K; ++c) {
                            const bool gt = Hn[c] > bk[c];
                            bk[c] = gt ? Hn[c] : bk[c];
                            bkt[c] = gt ? t : bkt[c];
                        }
                    }
                    if (TB && (t & 7) == 7) {
#pragma unroll
                        for (int c = 0; c < K; ++c)
                            *(uint32_t*)(tbblk + (((t >> 3) * K + c) * 64 + lane) * 4) = nacc[c];
                    }
                    if (TB && (t & 31) == 31) {
                        // each lane's state choices of the last 32 steps, bit
                        // 31 - (t & 31) for step t, 1 = opened
#pragma unroll
                        for (int x = 0; x < 5; ++x) {
                            if (NOI && x >= 2) continue;
#pragma unroll
                            for (int c = 0; c < K; ++c)
                                *(uint32_t*)(tbblk + 2048 * K +
                                             (((x * K + c) * 2 + (t >> 5)) * 64 + lane) * 4) =
                                    xacc[x][c];
                        }
                    }
                    // shift histories
                    hl3 = hl2; hl2 = hl1; hl1 = hl0;
#pragma unroll
                    for (int c = 0; c < K; ++c) {
                        h3[c] = h2[c]; h2[c] = h1[c]; h1[c] = Hn[c];
                        d3[c] = d2[c]; d2[c] = d1[c]; d1[c] = Dn[c];
                        if (!NOI) { a1[c] = An[c]; b1[c] = Bn[c]; c1[c] = Cn[c]; }
                    }
                    ddm1 = dd0; dd0 = ds0.z; aam2 = aam1; aam1 = ds0.w;
                    Hout = Hn[K - 1];
                    Iout = In[K - 1];
                    // lane 63 records the row; the other lanes write to slots
                    // of their own, so the store needs no branch (a branch
                    // splits the step's scheduling region and costs spills)
                    if constexpr (K == 2) outw[t] = make_int2(Hout, Iout);
                    else outb[lane == 63 ? t : 64 + lane] = make_int2(Hout, Iout);
                    // rotate the pipeline
                    cd0 = nd0; nd0 = fd0;
#pragma unroll
                    for (int c = 0; c < K; ++c) csc[c] = nsc[c];
                    cin = nin;
                    if (TB ? MPG_TB_STEP_BARRIER : MPG_STEP_BARRIER)
                        __builtin_amdgcn_sched_barrier(0);
                }  // steps

                // merge the chunk's best into the strip's best (first maximum)
                if (MIXED || !fixed_end_mode(MODE)) {
#pragma unroll
                    for (int c = 0; c < K; ++c) {
                        int v, tt;
                        if (MODE == MPG_LOCAL) { v = bk[c] >> 6; tt = 63 - (bk[c] & 63); }
                        else { v = bk[c]; tt = bkt[c]; }
                        if (TB && MODE == MPG_LOCAL) v <<= 4;  // back to 16*H units
                        if (v > best[c]) { best[c] = v; bstep[c] = ch * 64 + tt; }
                        bk[c] = INT_MIN;
                    }
                }
                // publish the strip's last column for rows ch*64-63+lane.  The
                // counter lags one chunk: once every memory operation but this
                // store has completed, the previous chunk's rows are at the
                // coherence point, so chunks 0..ch-1 are announced without
                // waiting for the store just issued.
                if (has_next) {
                    const int orow = ch * 64 - 63 + lane;
                    st_dev2(&bnd_g[kBndLo + orow], outb[lane]);
                    __builtin_amdgcn_s_waitcnt(kWaitVm1);
                    if (lane == 0 && ch > 0) st_dev(&prog[strip], ch);
                }
            }
        }  // chunks
        if (has_next && !failed) {
            __builtin_amdgcn_s_waitcnt(0);  // the last chunk's rows, then the count
            if (lane == 0) st_dev(&prog[strip], nchunks);
        }
        if (failed) {
            // let the strips to the right drain quickly; the pair reports an error
            if (lane == 0) {
                st_dev(&prog[strip], nchunks);
                atomicMax(&ps->bad, 1);
            }
        }

        // ---- strip epilogue: best cell of the strip, folded into the pair.
        // A pair of one strip keeps it in registers: no pair state, no
        // atomics.
        const bool solo = nstrips == 1;
        unsigned long long solo_key = 0;
        int solo_gsc = NEG;
        if (!failed) {
            if (fixed) {
                // H(n, m): tracked on its own, or (mixed variant) the best
                // cell of row n
                int hv[K];
#pragma unroll
                for (int c = 0; c < K; ++c) hv[c] = MIXED ? best[c] : hn[c];
                if (solo) {
                    int v = NEG;
#pragma unroll
                    for (int c = 0; c < K; ++c)
                        if (col0 + c == m) v = hv[c];
                    // one lane holds column m
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) v = imax(v, __shfl_xor(v, o, 64));
                    solo_gsc = v;
                } else {
#pragma unroll
                    for (int c = 0; c < K; ++c)
                        if (col0 + c == m) st_dev(&ps->gsc, hv[c]);
                }
            } else {
                uint64_t key = 0;
#pragma unroll
                for (int c = 0; c < K; ++c) {
                    const int row = bstep[c] - lane;
                    const int col = col0 + c;
                    const int v = TB ? (best[c] >> 4) : best[c];
                    if (col <= m && row >= 0 && row <= n && best[c] > UNREACH) {
                        const uint64_t k2 = end_key(v, row, col);
                        key = k2 > key ? k2 : key;
                    }
                }
                key = wave_max_u64(key);
                best_key = key > best_key ? key : best_key;
                if (solo) solo_key = best_key;
                else if (lane == 0 && best_key)
                    atomicMax(&ps->key, (unsigned long long)best_key);
            }
        }
        // the wave that finishes the pair's last strip writes the result.
        // Its end key and H(n, m) are device-scope atomics that completed
        // before the count (the wait), so the finishing wave reads them
        // after its own count; when the traceback is walked in this kernel
        // the count is also acquire-release, so that the walking wave sees
        // every strip's direction bits.
        int done = 0;
        if (!solo) {
            __builtin_amdgcn_s_waitcnt(0);
            if (lane == 0)
                done = (TB && sink.walk)
                           ? __hip_atomic_fetch_add(&ps->done, 1, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT)
                           : __hip_atomic_fetch_add(&ps->done, 1, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
            done = __builtin_amdgcn_readfirstlane(done);
        }
        if (done == nstrips - 1) {
            const unsigned long long k =
                solo ? solo_key
                     : __hip_atomic_load(&ps->key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int gv =
                __builtin_amdgcn_readfirstlane(solo ? solo_gsc : ld_dev(&ps->gsc));
            const int bad = solo ? 0 : __builtin_amdgcn_readfirstlane(ld_dev(&ps->bad));
            mpg_dev_result R;
            R.g_beg = -1;
            R.p_beg = -1;
            R.ops_off = J.ops_off;
            R.ops_len = 0;
            R._pad = 0;
            if (bad) {
                R.status = MPG_E_DEVICE;
                R.score = 0;
                R.g_end = -1;
                R.p_end = -1;
            } else if (fixed) {
                if (gv < UNREACH) {
                    R.status = MPG_E_NOALN;
                    R.score = 0;
                    R.g_end = -1;
                    R.p_end = -1;
                } else {
                    R.status = MPG_OK;
                    R.score = TB ? (gv >> 4) : gv;
                    R.g_end = n;
                    R.p_end = m;
                }
            } else {
                const uint32_t khi = __builtin_amdgcn_readfirstlane((uint32_t)(k >> 32));
                const uint32_t klo = __builtin_amdgcn_readfirstlane((uint32_t)k);
                const unsigned long long ku = ((unsigned long long)khi << 32) | klo;
                R.status = MPG_OK;
                R.score = (int)(ku >> 36) - (1 << 27);
                R.g_end = (1 << 21) - 1 - (int)((ku >> 15) & ((1u << 21) - 1));
                R.p_end = (1 << 15) - 1 - (int)(ku & ((1u << 15) - 1));
            }
            if (TB && sink.walk) {
                if (solo) {
                    // this wave's own direction bits: complete, then read
                    // past the vector cache
                    __builtin_amdgcn_s_waitcnt(0);
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
                // walk the traceback now: the pair completes without a second kernel
                char* txt = sink.ops + J.ops_off;
                if (R.status == MPG_OK) {
                    const TbView V{tbbuf + J.tb_off, J.K, J.nchunks};
                    const int64_t end = 2LL * (n + m);
                    OpWriter W{txt, end};
                    int bi = -1, bj = -1;
                    const bool ok = walk_wave(V, R.g_end, R.p_end, n, m, W, lane, bi, bj);
                    if (!ok || W.overflow) {
                        R.status = MPG_E_DEVICE;
                        if (lane == 0) txt[0] = 0;
                    } else {
                        if (lane == 0) txt[end] = 0;
                        R.g_beg = bi;
                        R.p_beg = bj;
                        R.ops_off = J.ops_off + W.pos;
                        R.ops_len = (int32_t)(end - W.pos);
                    }
                } else if (lane == 0) {
                    txt[0] = 0;
                }
            }
            if (lane == 0) publish(sink.out + J.res, R, sink.system);
        }
    }  // queue
}

template <int K, int MODE, bool TB, bool PRO>
hipError_t launch_dp_t(hipStream_t s, int ncu, const DevParams& P, const PairJob* jobs,
                       const int2* items, int nitems, int* qhead, PairState* pst, int* prog,
                       const uint8_t* prot, const uint8_t* desc, int2* bnd, uint8_t* tbbuf,
                       const DpSink& sink) {
    const bool noi = (P.flags & MPG_NO_INTRON) != 0;
    const bool nof = (P.flags & MPG_NO_FRAMESHIFT) != 0;
    const size_t lds = (size_t)LdsLayout<K, TB, MODE == MPG_LOCAL && !PRO>::WAVE;
    dim3 b(64);
    // persistent grid: as many waves as ncu compute units hold at once for
    // this kernel, never more than there are items
#define MPG_LAUNCH(NI, NF)                                                                      \
    do {                                                                                        \
        static int per_cu = 0;                                                                  \
        if (per_cu <= 0 &&                                                                      \
            hipOccupancyMaxActiveBlocksPerMultiprocessor(                                       \
                &per_cu, dp_kernel<K, MODE, TB, NI, NF, PRO>, 64, lds) != hipSuccess)           \
            per_cu = 0;                                                                         \
        const int waves = per_cu > 0 ? per_cu * ncu : 8 * ncu;                                \
        dim3 g(nitems < waves ? nitems : waves);                                                \
        hipLaunchKernelGGL((dp_kernel<K, MODE, TB, NI, NF, PRO>), g, b, lds, s, jobs, items,   \
                           nitems, qhead, pst, prog, prot, desc, bnd, tbbuf, sink, P);          \
    } while (0)
    if (!noi && !nof) MPG_LAUNCH(false, false);
    else if (noi && !nof) MPG_LAUNCH(true, false);
    else if (!noi && nof) MPG_LAUNCH(false, true);
    else MPG_LAUNCH(true, true);
#undef MPG_LAUNCH
    return hipGetLastError();
}

template <int K, bool PRO>
hipError_t launch_dp_k(hipStream_t s, int ncu, bool tb, const DevParams& P, const PairJob* jobs,
                       const int2* items, int nitems, int* qhead, PairState* pst, int* prog,
                       const uint8_t* prot, const uint8_t* desc, int2* bnd, uint8_t* tbbuf,
                       const DpSink& sink) {
#define MPG_MODE(M)                                                                             \
    return tb ? launch_dp_t<K, M, true, PRO>(s, ncu, P, jobs, items, nitems, qhead, pst, prog, \
                                             prot, desc, bnd, tbbuf, sink)                      \
              : launch_dp_t<K, M, false, PRO>(s, ncu, P, jobs, items, nitems, qhead, pst, prog, \
                                              prot, desc, bnd, tbbuf, sink)
    switch (P.mode) {
        case MPG_LOCAL: MPG_MODE(MPG_LOCAL);
        case MPG_EXTEND: MPG_MODE(MPG_EXTEND);
        case kModeMixed:
            if constexpr (!PRO) MPG_MODE(kModeMixed);
            return hipErrorInvalidValue;  // profile queries come in one mode per call
        default: MPG_MODE(MPG_GLOBAL);  // GLOBAL and EXTEND_LEFT (per-pair start term)
    }
#undef MPG_MODE
}

}  // namespace dev
}  // namespace mpg
