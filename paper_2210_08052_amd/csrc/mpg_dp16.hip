// Lane-packed int16 variant of the DP for LOCAL score-only pairs (Eq. (full)
// of Li 2022, "DP for protein-to-genome alignment"; the paper's own CPU
// kernel also scores in 16-bit lanes, as the closing paragraph of that
// subsection states).
//
// Two pairs share one wavefront: every 32-bit lane register holds pair A's
// value in its low half and pair B's in its high half, and one packed
// instruction (v_pk_add_i16 / v_pk_max_i16, saturating) advances both cells.
// The two pairs run the same anti-diagonal schedule as the int32 kernel
// (lane k computes row s-k at step s, strips of 64*K columns, left boundary
// streamed through HBM behind a progress counter), so the host pairs
// eligible pairs of similar size.  Saturation keeps -infinity fixed at
// -32768; the host admits a pair only when every reachable value provably
// fits: in LOCAL mode H >= 0, so the smallest value is bounded by the largest
// penalty sum (at most 8,192 is admitted), and the largest by the protein
// length times the largest matrix entry (m * max(mat) <= 32,511 is
// admitted): each residue adds at most one substitution score to a path.
#include "mpg_dp.h"

namespace mpg {
namespace dev {

typedef short s2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s2 as_s2(int v) { return __builtin_bit_cast(s2, v); }
__device__ __forceinline__ int as_i(s2 v) { return __builtin_bit_cast(int, v); }
__device__ __forceinline__ s2 pmax(s2 a, s2 b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ s2 psub(s2 a, s2 b) { return __builtin_elementwise_sub_sat(a, b); }
__device__ __forceinline__ s2 padd(s2 a, s2 b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ s2 splat(int v) {
    const int c = v > 32767 ? 32767 : (v < -32768 ? -32768 : v);
    s2 r;
    r.x = (short)c;
    r.y = (short)c;
    return r;
}
__device__ __forceinline__ int pack16(int lo, int hi) {
    return (int)(((uint32_t)lo & 0xFFFFu) | ((uint32_t)hi << 16));
}

constexpr int kNeg16 = -32768;
constexpr int kNeg2 = (int)0x80008000u;  // both halves -infinity

template <int K>
struct Lds16 {
    static constexpr int SW = 64 * K;          // strip width
    static constexpr int RING = 128 * 16;      // two chunks of packed descriptors
    static constexpr int HALF = 25 * SW * 2;   // one pair's int16 profile
    static constexpr int PROF = 2 * HALF;      // A then B
    static constexpr int IN = 64 * 8;
    static constexpr int OUT = 128 * 8;  // rows 0..63, then one dummy slot per lane
    static constexpr int WAVE = RING + PROF + IN + OUT;
};

// Packed descriptor of row r (16 bytes): {profile byte offset of A's row |
// B's offset << 16, z, r + d(r+1), a(r)}, the last three as int16 pairs.
__global__ void __launch_bounds__(256) prepass16_kernel(const PairJob* __restrict__ jobs,
                                                        const PackJob* __restrict__ packs,
                                                        const int64_t* __restrict__ row_start,
                                                        int npacks, int64_t total_rows,
                                                        const uint8_t* __restrict__ dna,
                                                        uint8_t* __restrict__ desc,
                                                        int* __restrict__ prog, DevParams P) {
    // the owner of the block's first row, then each thread steps forward (a
    // pack owns at least 256 rows, so a block spans few packs)
    __shared__ int first_owner;
    // the codon and splice tables, looked up with per-thread indices, in LDS
    __shared__ uint8_t s_gcode[64], s_donor[128], s_acceptor[128];
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x * kPrepassRows;
    if (threadIdx.x < 64) s_gcode[threadIdx.x] = P.gcode[threadIdx.x];
    if (threadIdx.x < 125) {
        s_donor[threadIdx.x] = P.donor[threadIdx.x];
        s_acceptor[threadIdx.x] = P.acceptor[threadIdx.x];
    }
    if (threadIdx.x < 64) {
        const int o = wave_find_owner(row_start, npacks, g0);
        if (threadIdx.x == 0) first_owner = o;
    }
    __syncthreads();
    // kPrepassRows consecutive rows per thread, all of one pack (a pack's rows
    // start at a multiple of 64 and number a multiple of 64)
    const int64_t q = g0 + (int64_t)threadIdx.x * kPrepassRows;
    if (q >= total_rows) return;
    int lo = first_owner;
    while (lo + 1 < npacks && row_start[lo + 1] <= q) ++lo;
    const PackJob& X = packs[lo];
    const int i0 = (int)(q - row_start[lo]) - kDescLo;
    if (i0 == -kDescLo)
        for (int s = 0; s < X.nstrips; ++s) prog[X.prog_off + s] = 0;
    constexpr int W = kPrepassRows + 8;
    int f[kPrepassRows][2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int jx = h ? X.b : X.a;
        const int n = jx >= 0 ? jobs[jx].n : -1;  // an idle half has no valid row
        const uint8_t* T = dna + (jx >= 0 ? jobs[jx].dna_off : 0);
        int b[W];  // bases i0-4 .. i0+kPrepassRows+3
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int x = i0 - 4 + k;
            b[k] = (x >= 1 && x <= n) ? dna_code(T[x - 1]) : 4;
        }
#pragma unroll
        for (int rr = 0; rr < kPrepassRows; ++rr) {
            const int i = i0 + rr;
            const int* bb = b + rr;  // bb[k] = T[i-4+k]
            int tr;
            if (i > n || i < 0) tr = 24;
            else if (i < 3 || bb[2] == 4 || bb[3] == 4 || bb[4] == 4) tr = 22;
            else tr = s_gcode[16 * bb[2] + 4 * bb[3] + bb[4]];
            // d(i+1) reads T[i+2..i+4]; a(i) reads T[i-2..i]
            const int dn = s_donor[25 * bb[6] + 5 * bb[7] + bb[8]];
            const int ac = s_acceptor[25 * bb[2] + 5 * bb[3] + bb[4]];
            f[rr][h][0] = tr;
            f[rr][h][1] = (i >= 0 && i <= n) ? 0 : kNeg16;
            f[rr][h][2] = P.r + dn;
            f[rr][h][3] = ac;
        }
    }
    // profile offsets in bytes from the start of the profile area; B's table
    // follows A's
    const int sw2 = (int)(X.K * 64 * 2);
    int4* out = (int4*)(desc + X.desc_off + (int64_t)(i0 + kDescLo) * 16);
#pragma unroll
    for (int rr = 0; rr < kPrepassRows; ++rr) {
        const int offA = f[rr][0][0] * sw2;
        const int offB = 25 * sw2 + f[rr][1][0] * sw2;
        out[rr] = make_int4(pack16(offA, offB), pack16(f[rr][0][1], f[rr][1][1]),
                            pack16(f[rr][0][2], f[rr][1][2]), pack16(f[rr][0][3], f[rr][1][3]));
    }
}

// Waves per SIMD the register allocation of the int16 kernel aims at.
#ifndef MPG_I16_WAVES
#define MPG_I16_WAVES 3
#endif

template <int K, bool NOI, bool NOF>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MPG_I16_WAVES)))
dp16_kernel(const PairJob* __restrict__ jobs, const PackJob* __restrict__ packs,
            const int2* __restrict__ items, int nitems, int* __restrict__ qhead,
            PairState* __restrict__ pst, int* __restrict__ prog_g,
            const uint8_t* __restrict__ prot, const uint8_t* __restrict__ desc,
            int2* __restrict__ bnd, DpSink sink, DevParams P) {
    using LY = Lds16<K>;
    extern __shared__ __align__(16) uint8_t smem[];
    const int lane = threadIdx.x & 63;
    uint8_t* ring = smem;
    uint8_t* prof = smem + LY::RING;
    int2* inb = (int2*)(smem + LY::RING + LY::PROF);
    int2* outb = (int2*)(smem + LY::RING + LY::PROF + LY::IN);
    const s2 ce = splat(P.e), cf = splat(P.f);
    const s2 cqe = splat(P.q + P.e);  // open and first extension
    const s2 neg2 = as_s2(kNeg2);

    for (;;) {
        const int it = __builtin_amdgcn_readfirstlane(atomicAdd(qhead, lane == 0 ? 1 : 0));
        if (it >= nitems) break;
        const int2 item = items[it];
        const PackJob X = packs[item.x];
        const int strip = item.y;
        const bool hasB = X.b >= 0;
        const PairJob JA = jobs[X.a];
        const PairJob JB = jobs[hasB ? X.b : X.a];
        const int nA = JA.n, mA = JA.m;
        const int nB = hasB ? JB.n : -1, mB = hasB ? JB.m : -1;
        const int nchunks = X.nchunks;
        const uint8_t* dsc_g = desc + X.desc_off;
        int2* bnd_g = bnd + X.bnd_off;
        int* prog = prog_g + X.prog_off;
        const bool has_next = strip + 1 < X.nstrips;
        const int col0 = strip * LY::SW + lane * K;
        bool failed = false;

        // ---- profiles of both pairs for this strip's columns
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const PairJob& J = h ? JB : JA;
            const int m = h ? mB : mA;
            const uint8_t* Pa = prot + J.prot_off;
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const int j = col0 + c;
                const int pc = (j >= 1 && j <= m) ? aa_code(Pa[j - 1]) : -1;
                int16_t* pr = (int16_t*)(prof + h * LY::HALF) + lane * K + c;
                for (int tr = 0; tr < 25; ++tr)
                    pr[tr * LY::SW] = (int16_t)((pc < 0 || tr == 24) ? kNeg16 : P.mat[tr * 24 + pc]);
            }
        }
        inb[lane] = make_int2(kNeg2, kNeg2);

        s2 h1[K], h2[K], h3[K], d1[K], d2[K], d3[K], a1[K], b1[K], c1[K];
        int kA[K], kB[K], bestA[K], bestB[K], stA[K], stB[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            h1[c] = h2[c] = h3[c] = neg2;
            d1[c] = d2[c] = d3[c] = neg2;
            a1[c] = b1[c] = c1[c] = neg2;
            kA[c] = kB[c] = INT_MIN;
            bestA[c] = bestB[c] = kNeg16;
            stA[c] = stB[c] = 0;
        }
        s2 hl1 = neg2, hl2 = neg2, hl3 = neg2;
        int Hout = kNeg2, Iout = kNeg2;
        // r+d(i), r+d(i-1), a(i-1), a(i-2) of the two pairs, carried in registers
        s2 dd0, ddm1, aam1, aam2;
        {
            const int4 u = *(const int4*)(dsc_g + (int64_t)(-lane - 1 + kDescLo) * 16);
            const int4 v = *(const int4*)(dsc_g + (int64_t)(-lane - 2 + kDescLo) * 16);
            dd0 = as_s2(u.z); aam1 = as_s2(u.w); ddm1 = as_s2(v.z); aam2 = as_s2(v.w);
        }
        int4 pf0;
        {
            *(int4*)(ring + lane * 16) = *(const int4*)(dsc_g + (int64_t)(lane - 64 + kDescLo) * 16);
            *(int4*)(ring + (64 + lane) * 16) = *(const int4*)(dsc_g + (int64_t)(lane + kDescLo) * 16);
        }
        int2 nb = make_int2(kNeg2, kNeg2);
        // left boundary and the left strip's progress, read one chunk ahead
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
                // rows beyond a pair's region are -infinity in that half
                const int row = ch * 64 + lane;
                if (from_left) {
                    const uint32_t mlo = row > nA ? 0xFFFFu : 0u;
                    const uint32_t mhi = row > nB ? 0xFFFF0000u : 0u;
                    const uint32_t msk = mlo | mhi;
                    const int hx = (int)(((uint32_t)nb.x & ~msk) | ((uint32_t)kNeg2 & msk));
                    const int ix = (int)(((uint32_t)nb.y & ~msk) | ((uint32_t)kNeg2 & msk));
                    inb[lane] = make_int2(hx, ix);
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
                    const int4 o0 = *(const int4*)(ring + (64 + lane) * 16);
                    *(int4*)(ring + lane * 16) = o0;
                    *(int4*)(ring + (64 + lane) * 16) = pf0;
                }
                pf0 = *(const int4*)(dsc_g + (int64_t)((ch + 1) * 64 + lane + kDescLo) * 16);
                const uint8_t* rb = ring + (64 - lane) * 16;
                const uint8_t* pbase = prof + lane * K * 2;

                auto ld_prof = [&](const int4& x0, s2* scv) {
                    const int16_t* pa = (const int16_t*)(pbase + (x0.x & 0xFFFF));
                    const int16_t* pb = (const int16_t*)(pbase + ((uint32_t)x0.x >> 16));
#pragma unroll
                    for (int c = 0; c < K; ++c) {
                        s2 v;
                        v.x = pa[c];
                        v.y = pb[c];
                        scv[c] = v;
                    }
                };
                int4 cd0 = *(const int4*)(rb);
                int4 nd0 = *(const int4*)(rb + 16);
                s2 csc[K];
                ld_prof(cd0, csc);
                int2 cin = inb[0];

#pragma unroll
                for (int t = 0; t < 64; ++t) {
                    int4 fd0 = make_int4(0, 0, 0, 0);
                    if (t + 2 < 64) fd0 = *(const int4*)(rb + (t + 2) * 16);
                    s2 nsc[K];
                    int2 nin = make_int2(0, 0);
                    if (t + 1 < 64) {
                        ld_prof(nd0, nsc);
                        nin = inb[t + 1];
                    }
                    const int4 ds0 = cd0;
                    const s2 hl0 = as_s2(shr1(cin.x, Hout));
                    const s2 il0 = as_s2(shr1(cin.y, Iout));
                    const s2 z = as_s2(ds0.y);
                    const s2 rdn = as_s2(ds0.z);  // r + d(i+1)
                    const s2 acc = as_s2(ds0.w);  // a(i)
                    s2 Hn[K], In[K], Dn[K], An[K], Bn[K], Cn[K];
#pragma unroll
                    for (int c = 0; c < K; ++c) {
                        const s2 L0 = c ? Hn[c - 1] : hl0;
                        const s2 IL = c ? In[c - 1] : il0;
                        const s2 L1 = c ? h1[c - 1] : hl1;
                        const s2 L2 = c ? h2[c - 1] : hl2;
                        const s2 L3 = c ? h3[c - 1] : hl3;
                        // every candidate but I is known before the left
                        // neighbour's H of this row: fold them in two
                        // independent trees, so that dependent packed
                        // instructions rarely follow each other
                        // max(x - q, y) - e as max(x - (q+e), y - e): no
                        // value reachable here saturates, so both are exact
                        const s2 D = pmax(psub(h3[c], cqe), psub(d3[c], ce));
                        s2 t0 = pmax(D, z);
                        s2 t1 = padd(L3, csc[c]);
                        if (!NOI) {
                            const s2 A = pmax(psub(h1[c], ddm1), a1[c]);
                            const s2 B = pmax(psub(L1, dd0), b1[c]);
                            const s2 C = pmax(psub(L1, rdn), c1[c]);
                            t0 = pmax(t0, psub(A, acc));
                            t1 = pmax(t1, pmax(psub(B, aam2), psub(C, aam1)));
                            An[c] = A; Bn[c] = B; Cn[c] = C;
                        }
                        if (!NOF) t0 = pmax(t0, psub(pmax(pmax(L1, L2), pmax(h1[c], h2[c])), cf));
                        const s2 I = pmax(psub(L0, cqe), psub(IL, ce));
                        const s2 H = pmax(pmax(t0, t1), I);
                        Hn[c] = H; In[c] = I; Dn[c] = D;
                        // end-cell keys: value in the high half, 63 - step below
                        const int hv = as_i(H);
                        kA[c] = imax(kA[c], (int)(((uint32_t)hv << 16) | (uint32_t)(63 - t)));
                        kB[c] = imax(kB[c], (int)(((uint32_t)hv & 0xFFFF0000u) | (uint32_t)(63 - t)));
                    }
                    hl3 = hl2; hl2 = hl1; hl1 = hl0;
#pragma unroll
                    for (int c = 0; c < K; ++c) {
                        h3[c] = h2[c]; h2[c] = h1[c]; h1[c] = Hn[c];
                        d3[c] = d2[c]; d2[c] = d1[c]; d1[c] = Dn[c];
                        if (!NOI) { a1[c] = An[c]; b1[c] = Bn[c]; c1[c] = Cn[c]; }
                    }
                    ddm1 = dd0; dd0 = rdn; aam2 = aam1; aam1 = acc;
                    Hout = as_i(Hn[K - 1]);
                    Iout = as_i(In[K - 1]);
                    // lane 63 records the row; the other lanes write to slots of
                    // their own, so the store needs no branch (a branch would
                    // split the step's scheduling region)
                    outb[lane == 63 ? t : 64 + lane] = make_int2(Hout, Iout);
                    cd0 = nd0; nd0 = fd0;
#pragma unroll
                    for (int c = 0; c < K; ++c) csc[c] = nsc[c];
                    cin = nin;
                    // (no scheduling barrier between steps: the next step's
                    // independent terms fill the wait states of this step's
                    // dependent packed instructions)
                }  // steps

                // fold the chunk's best of each half into the strip's best
#pragma unroll
                for (int c = 0; c < K; ++c) {
                    const int va = kA[c] >> 16, vb = kB[c] >> 16;
                    if (va > bestA[c]) { bestA[c] = va; stA[c] = ch * 64 + 63 - (kA[c] & 63); }
                    if (vb > bestB[c]) { bestB[c] = vb; stB[c] = ch * 64 + 63 - (kB[c] & 63); }
                    kA[c] = kB[c] = INT_MIN;
                }
                // publish with a one-chunk lag (see the int32 kernel)
                if (has_next) {
                    const int orow = ch * 64 - 63 + lane;
                    st_dev2(&bnd_g[kBndLo + orow], outb[lane]);
                    __builtin_amdgcn_s_waitcnt(kWaitVm1);
                    if (lane == 0 && ch > 0) st_dev(&prog[strip], ch);
                }
            }
        }  // chunks
        if (has_next && !failed) {
            __builtin_amdgcn_s_waitcnt(0);
            if (lane == 0) st_dev(&prog[strip], nchunks);
        }
        if (failed && lane == 0) {
            st_dev(&prog[strip], nchunks);
            atomicMax(&pst[X.a].bad, 1);
            if (hasB) atomicMax(&pst[X.b].bad, 1);
        }
        // ---- strip epilogue: best cell of each pair in this strip
        if (!failed) {
            uint64_t keyA = 0, keyB = 0;
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const int col = col0 + c;
                const int ra = stA[c] - lane, rbw = stB[c] - lane;
                if (col <= mA && ra >= 0 && ra <= nA && bestA[c] >= 0) {
                    const uint64_t k2 = end_key(bestA[c], ra, col);
                    keyA = k2 > keyA ? k2 : keyA;
                }
                if (col <= mB && rbw >= 0 && rbw <= nB && bestB[c] >= 0) {
                    const uint64_t k2 = end_key(bestB[c], rbw, col);
                    keyB = k2 > keyB ? k2 : keyB;
                }
            }
            keyA = wave_max_u64(keyA);
            keyB = wave_max_u64(keyB);
            if (lane == 0) {
                if (keyA) atomicMax(&pst[X.a].key, (unsigned long long)keyA);
                if (hasB && keyB) atomicMax(&pst[X.b].key, (unsigned long long)keyB);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        // the wave that finishes a pair's last strip writes its result; the
        // end keys are device-scope atomics completed before the count (the
        // wait), and nothing else of the other strips is read here, so the
        // count needs no cache-wide release or acquire
        if (lane == 0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h && !hasB) continue;
                const PairJob& J = h ? JB : JA;
                const int jx = h ? X.b : X.a;
                if (strip >= J.nstrips) continue;
                PairState* ps = pst + jx;
                const int done = __hip_atomic_fetch_add(&ps->done, 1, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
                if (done != J.nstrips - 1) continue;
                mpg_dev_result R;
                R.g_beg = -1;
                R.p_beg = -1;
                R.ops_off = J.ops_off;
                R.ops_len = 0;
                R._pad = 0;
                const unsigned long long k = __hip_atomic_load(&ps->key, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                if (ld_dev(&ps->bad)) {
                    R.status = MPG_E_DEVICE;
                    R.score = 0;
                    R.g_end = -1;
                    R.p_end = -1;
                } else {
                    R.status = MPG_OK;
                    R.score = (int)(k >> 36) - (1 << 27);
                    R.g_end = (1 << 21) - 1 - (int)((k >> 15) & ((1u << 21) - 1));
                    R.p_end = (1 << 15) - 1 - (int)(k & ((1u << 15) - 1));
                }
                publish(sink.out + J.res, R, sink.system);
            }
        }
    }  // queue
}

template <int K>
hipError_t launch_dp16_t(hipStream_t s, int ncu, const DevParams& P, const PairJob* jobs,
                         const PackJob* packs, const int2* items, int nitems, int* qhead,
                         PairState* pst, int* prog, const uint8_t* prot, const uint8_t* desc,
                         int2* bnd, const DpSink& sink) {
    const bool noi = (P.flags & MPG_NO_INTRON) != 0;
    const bool nof = (P.flags & MPG_NO_FRAMESHIFT) != 0;
    const size_t lds = (size_t)Lds16<K>::WAVE;
    dim3 b(64);
#define MPG_LAUNCH16(NI, NF)                                                                    \
    do {                                                                                        \
        static int per_cu = 0;                                                                  \
        if (per_cu <= 0 && hipOccupancyMaxActiveBlocksPerMultiprocessor(                        \
                               &per_cu, dp16_kernel<K, NI, NF>, 64, lds) != hipSuccess)         \
            per_cu = 0;                                                                         \
        const int waves = per_cu > 0 ? per_cu * ncu : 8 * ncu;                                  \
        dim3 g(nitems < waves ? nitems : waves);                                                \
        hipLaunchKernelGGL((dp16_kernel<K, NI, NF>), g, b, lds, s, jobs, packs, items, nitems,  \
                           qhead, pst, prog, prot, desc, bnd, sink, P);                         \
    } while (0)
    if (!noi && !nof) MPG_LAUNCH16(false, false);
    else if (noi && !nof) MPG_LAUNCH16(true, false);
    else if (!noi && nof) MPG_LAUNCH16(false, true);
    else MPG_LAUNCH16(true, true);
#undef MPG_LAUNCH16
    return hipGetLastError();
}

}  // namespace dev

hipError_t launch_prepass16(hipStream_t s, const PairJob* jobs, const PackJob* packs,
                            const int64_t* row_start, int npacks, int64_t total_rows,
                            const uint8_t* dna, uint8_t* desc, int* prog, const DevParams& P) {
    if (total_rows <= 0) return hipSuccess;
    const int64_t per_block = 256 * dev::kPrepassRows;
    const int64_t blocks = (total_rows + per_block - 1) / per_block;
    hipLaunchKernelGGL(dev::prepass16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, jobs, packs,
                       row_start, npacks, total_rows, dna, desc, prog, P);
    return hipGetLastError();
}

hipError_t launch_dp16(hipStream_t s, int K, int ncu, const DevParams& P, const PairJob* jobs,
                       const PackJob* packs, const int2* items, int nitems, int* qhead, void* pst,
                       int* prog, const uint8_t* prot, const uint8_t* desc, int2* bnd,
                       const DpSink& sink) {
    if (nitems <= 0) return hipSuccess;
    if (P.mode != MPG_LOCAL) return hipErrorInvalidValue;
    switch (K) {
        case 1:
            return dev::launch_dp16_t<1>(s, ncu, P, jobs, packs, items, nitems, qhead,
                                         (dev::PairState*)pst, prog, prot, desc, bnd, sink);
        case 2:
            return dev::launch_dp16_t<2>(s, ncu, P, jobs, packs, items, nitems, qhead,
                                         (dev::PairState*)pst, prog, prot, desc, bnd, sink);
        default: return hipErrorInvalidValue;
    }
}

int dp16_lds_bytes(int K) { return K == 1 ? dev::Lds16<1>::WAVE : dev::Lds16<2>::WAVE; }

}  // namespace mpg
