// HIP kernels of the spliced protein-to-genome DP for gfx950 (CDNA4).
//
// The recurrence is Eq. (full) of Li 2022 (Methods, "DP for
// protein-to-genome alignment"): states H, I, D and the intron states A, B, C
// per cell (i = genome row, j = protein column), with the match term read as
// H(i-3,j-1)+s(i,j) (the codon ending at i against residue j; the printed
// H(i-3,j) consumes no residue), frameshift terms of Eq. (fs) and the splice
// penalties of "Splice models" supplied as 3-mer tables.
//
// Data layout and schedule:
//  * prepass: one thread per genome row writes a row descriptor: the amino
//    acid of the codon ending at the row, the start/floor value z(i) and the
//    splice penalties the row needs (all rows -128 .. steps+64, with poison
//    values outside 0..n);
//  * dp: one wavefront owns a strip of 64*K consecutive protein columns, lane
//    k holding K adjacent columns.  At step s lane k computes row s-k, so the
//    anti-diagonal order satisfies every dependency (rows i-1..i-3 of its own
//    columns live in registers; the left neighbour's H and I of the same row
//    arrive by a DPP wave_shr:1).  Lane 0 takes the left strip's last column
//    from HBM, where the wavefront running the left strip publishes it 64
//    rows at a time behind a progress counter; the kernel is persistent and
//    takes (pair, strip) items from one queue, longest pair first;
//  * traceback variant: every value is kept as 16*v + nibble, where the
//    nibble encodes the H winner (15 - code) so one max3 chain yields the
//    value and the first-maximum tie-break together; gap/intron extension
//    choices are shifted into a per-lane bit register (compare + add with
//    carry).  Both go to HBM as coalesced 256 B writes;
//  * walk: one wavefront per traced pair follows the stored choices back from
//    the end cell, reading each run of the path in parallel, and writes the
//    run-length op string.
#include <mutex>

#include "mpg_dp.h"

namespace mpg {

using namespace dev;

namespace dev {

// ----------------------------------------------------------------- prepass
__global__ void __launch_bounds__(256) prepass_kernel(const PairJob* __restrict__ jobs,
                                                      const int64_t* __restrict__ row_start,
                                                      int npairs, int64_t total_rows,
                                                      const uint8_t* __restrict__ dna,
                                                      uint8_t* __restrict__ desc, DevParams P) {
    // the owner of the block's first row, then each thread steps forward from
    // there (a pair owns at least 192 rows, so a block spans few pairs)
    __shared__ int first_owner;
    // the codon and splice tables, looked up with per-thread indices, in LDS
    __shared__ uint8_t s_gcode[64], s_donor[128], s_acceptor[128];
    // The block's rows are one contiguous byte range of the descriptor table
    // (pairs are laid out in row order).  Each thread writes its rows here,
    // then the block copies the range out in consecutive 16-byte pieces, so
    // the stores coalesce although a thread owns several consecutive rows.
    __shared__ __align__(16) uint8_t s_out[256 * kPrepassRows * 16];
    __shared__ int64_t s_base;  // byte offset in desc of the block's first row
    __shared__ int s_len;       // bytes of the block's rows
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x * kPrepassRows;
    if (threadIdx.x < 64) {
        const int o = wave_find_owner(row_start, npairs, g0);
        if (threadIdx.x == 0) {
            first_owner = o;
            const PairJob& J0 = jobs[o];
            s_base = J0.desc_off + (g0 - row_start[o]) * 16;
            s_len = 0;
        }
    }
    if (threadIdx.x < 64) s_gcode[threadIdx.x] = P.gcode[threadIdx.x];
    if (threadIdx.x < 125) {
        s_donor[threadIdx.x] = P.donor[threadIdx.x];
        s_acceptor[threadIdx.x] = P.acceptor[threadIdx.x];
    }
    __syncthreads();
    // kPrepassRows consecutive rows per thread: a pair's rows start at a
    // multiple of 64 and number a multiple of 64, so they share one pair, one
    // window of bases and one run of stores
    const int64_t q = g0 + (int64_t)threadIdx.x * kPrepassRows;
    const bool active = q < total_rows;
    if (active) {
        int lo = first_owner;
        while (lo + 1 < npairs && row_start[lo + 1] <= q) ++lo;
        const PairJob& J = jobs[lo];
        const int i0 = (int)(q - row_start[lo]) - kDescLo;
        const int n = J.n;
        const uint8_t* T = dna + J.dna_off;
        constexpr int W = kPrepassRows + 8;
        int b[W];  // bases i0-4 .. i0+kPrepassRows+3 (code 4 outside 1..n)
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int x = i0 - 4 + k;
            b[k] = (x >= 1 && x <= n) ? dna_code(T[x - 1]) : 4;
        }
        const int neg = neg_for(J.mode, J.tb != 0);
        const bool floor = floor_mode(J.mode);
        const int64_t at = J.desc_off + (int64_t)(i0 + kDescLo) * 16 - s_base;
        uint8_t* rowp = s_out + at;
#pragma unroll
        for (int rr = 0; rr < kPrepassRows; ++rr) {
            const int i = i0 + rr;
            const int* bb = b + rr;  // bb[k] = T[i-4+k]
            // codon ending at i: T[i-2..i]
            int tr;
            if (i > n || i < 0) tr = 24;  // poison row
            else if (i < 3 || bb[2] == 4 || bb[3] == 4 || bb[4] == 4) tr = 22;
            else tr = s_gcode[16 * bb[2] + 4 * bb[3] + bb[4]];
            // d(x) uses T[x+1..x+3], a(x) uses T[x-2..x]
            auto dpen = [&](int x) -> int {  // x in i-1 .. i+1
                const int o = x - i + 4;
                return s_donor[25 * bb[o + 1] + 5 * bb[o + 2] + bb[o + 3]];
            };
            auto apen = [&](int x) -> int {  // x in i-2 .. i
                const int o = x - i + 4;
                return s_acceptor[25 * bb[o - 2] + 5 * bb[o - 1] + bb[o]];
            };
            const bool valid = (i >= 0 && i <= n);
            const int z = floor ? (valid ? 0 : neg) : (i == 0 ? 0 : neg);
            // traceback layout: the start candidate's nibble, and the donor
            // term negated and offset by C's nibble (the kernel adds B's and
            // A's nibble differences when it reads the row again one and two
            // rows later)
            if (!J.tb)
                ((int4*)rowp)[rr] = make_int4(tr, z, P.r + dpen(i + 1), apen(i));
            else
                ((int4*)rowp)[rr] = make_int4(tr, z + 15, 5 - 16 * (P.r + dpen(i + 1)),
                                              16 * apen(i));
        }
        atomicMax(&s_len, (int)at + kPrepassRows * 16);
    }
    __syncthreads();
    const int len = s_len;
    for (int off = threadIdx.x * 16; off < len; off += 256 * 16)
        *(int4*)(desc + s_base + off) = *(const int4*)(s_out + off);
}

// ------------------------------------------------------------------- init
__global__ void init_kernel(const PairJob* __restrict__ jobs, int npairs, PairState* __restrict__ pst,
                            int* __restrict__ prog, int* __restrict__ qheads, int nq, int gsc_init) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nq) qheads[k] = 0;
    if (k >= npairs) return;
    const PairJob& J = jobs[k];
    pst[k].key = 0;
    pst[k].done = 0;
    pst[k].gsc = gsc_init;
    pst[k].bad = 0;
    pst[k].pad = 0;
    if (J.status != MPG_OK || J.i16) return;
    for (int s = 0; s < J.nstrips; ++s) prog[J.prog_off + s] = 0;
}

// ------------------------------------------------------------------- walk

// One wavefront (block) per traced pair.  The op string ends at the last
// byte but one of the pair's slot (2(n+m)+1 bytes, enough for any path) and
// the record's ops_off points at its first byte.
__global__ void __launch_bounds__(64) walk_kernel(const PairJob* __restrict__ jobs,
                                                  const int32_t* __restrict__ order, int count,
                                                  const uint8_t* __restrict__ tbbuf,
                                                  mpg_dev_result* __restrict__ out,
                                                  char* __restrict__ ops) {
    const int w = blockIdx.x;
    if (w >= count) return;
    const int lane = threadIdx.x;
    const PairJob J = jobs[order[w]];
    mpg_dev_result R = out[J.res];
    char* txt = ops + J.ops_off;
    if (J.status != MPG_OK || R.status != MPG_OK) {
        if (lane == 0) txt[0] = 0;
        return;
    }
    const TbView V{tbbuf + J.tb_off, J.K, J.nchunks};
    const int64_t end = 2LL * (J.n + J.m);
    OpWriter W{txt, end};
    int bi = -1, bj = -1;
    const bool ok = walk_wave(V, R.g_end, R.p_end, J.n, J.m, W, lane, bi, bj);
    if (lane == 0) {
        if (!ok || W.overflow) {
            R.status = MPG_E_DEVICE;
            txt[0] = 0;
        } else {
            txt[end] = 0;
            R.g_beg = bi;
            R.p_beg = bj;
            R.ops_off = J.ops_off + W.pos;
            R.ops_len = (int32_t)(end - W.pos);
        }
        out[J.res] = R;
    }
}

// Records for pairs the host rejected before launch.
__global__ void status_kernel(const PairJob* __restrict__ jobs, int npairs, DpSink sink) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npairs) return;
    const PairJob J = jobs[k];
    if (J.status == MPG_OK) return;
    mpg_dev_result R;
    R.status = J.status;
    R.score = 0;
    R.g_beg = R.g_end = R.p_beg = R.p_end = -1;
    R.ops_off = J.ops_off;
    R.ops_len = 0;
    R._pad = 0;
    publish(sink.out + J.res, R, sink.system);
}

// ------------------------------------------------------------------ stitch
// First token "<len><op>" of s[beg, end): returns the op, sets *len and *next.
__device__ __forceinline__ char head_token(const char* s, int beg, int end, int* len, int* next) {
    int v = 0, i = beg;
    while (i < end && s[i] >= '0' && s[i] <= '9') v = v * 10 + (s[i++] - '0');
    *len = v;
    *next = i + 1;
    return i < end ? s[i] : 0;
}

__global__ void __launch_bounds__(64) stitch_kernel(const ChainJob* __restrict__ chains,
                                                    int nchains, const int4* __restrict__ runs,
                                                    const mpg_dev_result* __restrict__ pres,
                                                    const char* __restrict__ pops,
                                                    const uint8_t* __restrict__ prot,
                                                    const uint8_t* __restrict__ dna, DevParams P,
                                                    mpg_dev_result* __restrict__ out,
                                                    char* __restrict__ ops) {
    const int c = blockIdx.x;
    if (c >= nchains) return;
    const int lane = threadIdx.x;
    const ChainJob C = chains[c];
    mpg_dev_result R;
    R.status = MPG_OK;
    R.score = 0;
    R.g_beg = R.g_end = R.p_beg = R.p_end = -1;
    R.ops_off = C.ops_off;
    R.ops_len = 0;
    R._pad = 0;
    if (C.status != MPG_OK) R.status = C.status;
    for (int t = 0; t <= C.nruns && R.status == MPG_OK; ++t) {
        const int st = pres[C.piece0 + t].status;
        if (st != MPG_OK) {
            R.status = st;
            break;
        }
    }
    char* txt = ops + C.ops_off;
    if (R.status != MPG_OK) {
        if (lane == 0) {
            out[C.res] = R;
            if (C.tb && C.ops_cap > 0) txt[0] = 0;
        }
        return;
    }
    // the runs' M steps: codon x+3u .. x+3u+2 against residue y+u, lanes over u
    int acc = 0;
    const uint8_t* T = dna + C.dna_off;
    const uint8_t* Pa = prot + C.prot_off;
    for (int r = 0; r < C.nruns; ++r) {
        const int4 X = runs[C.run0 + r];
        for (int u = lane; u < X.z; u += 64) {
            const int g = X.x + 3 * u;
            const int b1 = dna_code(T[g]), b2 = dna_code(T[g + 1]), b3 = dna_code(T[g + 2]);
            const int tr = (b1 == 4 || b2 == 4 || b3 == 4) ? 22 : P.gcode[16 * b1 + 4 * b2 + b3];
            acc += P.mat[tr * 24 + aa_code(Pa[X.y + u])];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    for (int t = 0; t <= C.nruns; ++t) acc += pres[C.piece0 + t].score;
    const mpg_dev_result L = pres[C.piece0];
    const mpg_dev_result Rt = pres[C.piece0 + C.nruns];
    const int4 last = runs[C.run0 + C.nruns - 1];
    R.score = acc;
    R.g_end = last.x + 3 * last.z + Rt.g_end;
    R.p_end = last.y + last.z + Rt.p_end;
    if (C.tb) {
        R.g_beg = L.g_beg;
        R.p_beg = L.p_beg;
        // concatenate: left piece, then (run, following piece) per run; an M
        // token at either end of a piece joins the pending M run
        int64_t pos = 0;
        int pend = 0;
        bool overflow = false;
        const int64_t room = (int64_t)C.ops_cap - 1;  // the NUL
        auto emit_m = [&]() {
            if (pend == 0) return;
            const int nd = ndigits(pend);
            if (pos + nd + 1 > room) {
                overflow = true;
                return;
            }
            if (lane == 0) {
                int v = pend;
                for (int d = nd - 1; d >= 0; --d) {
                    txt[pos + d] = (char)('0' + v % 10);
                    v /= 10;
                }
                txt[pos + nd] = 'M';
            }
            pos += nd + 1;
            pend = 0;
        };
        for (int t = 0; t <= C.nruns && !overflow; ++t) {
            if (t > 0) pend += runs[C.run0 + t - 1].z;
            const mpg_dev_result& Q = pres[C.piece0 + t];
            const char* s = pops + Q.ops_off;
            const int len = Q.ops_len;
            if (len <= 0) continue;
            int v, nx;
            int beg = 0;
            if (head_token(s, 0, len, &v, &nx) == 'M') {
                pend += v;
                beg = nx;
            }
            if (beg >= len) continue;
            // last token: digits back from the op letter
            int end = len, tail = 0;
            if (s[len - 1] == 'M') {
                int j = len - 2;
                while (j >= beg && s[j] >= '0' && s[j] <= '9') --j;
                int w = 0;
                for (int q = j + 1; q < len - 1; ++q) w = w * 10 + (s[q] - '0');
                end = j + 1;
                tail = w;
            }
            emit_m();
            if (overflow || pos + (end - beg) > room) {
                overflow = true;
                break;
            }
            for (int q = beg + lane; q < end; q += 64) txt[pos + q - beg] = s[q];
            pos += end - beg;
            pend = tail;
        }
        emit_m();  // what is still pending after the right piece
        if (overflow) {
            R.status = MPG_E_DEVICE;
            pos = 0;
        }
        if (lane == 0 && C.ops_cap > 0) txt[pos] = 0;
        R.ops_len = (int32_t)pos;
    }
    __syncthreads();
    if (lane == 0) out[C.res] = R;
}

// ------------------------------------------------------------------ coding sequence
// Methods, "Avoiding pseudogenes": the genome bases the path consumes, in
// order, without the interior of any intron.  M/D/F/G tokens copy their
// bases, N copies none, U copies the split codon's first base and last two,
// V its first two and last one (a U/V token shorter than a codon copies its
// bases).  Lane 0 reads the tokens; every lane copies each run of bases.
__global__ void __launch_bounds__(64) cds_kernel(const CdsJob* __restrict__ jobs, int n,
                                                 const char* __restrict__ ops,
                                                 const uint8_t* __restrict__ dna,
                                                 uint8_t* __restrict__ cds,
                                                 int4* __restrict__ info) {
    const int k = blockIdx.x;
    if (k >= n) return;
    const int lane = threadIdx.x;
    const CdsJob J = jobs[k];
    const char* s = ops + J.ops_off;
    const uint8_t* T = dna + J.dna_off;
    uint8_t* out = cds + J.cds_off;
    int pos = 0, g = 0, res = 0, introns = 0, bad = 0;
    int i = 0;
    for (;;) {
        // lane 0 reads the next token and names up to two runs to copy
        int src0 = 0, len0 = 0, src1 = 0, len1 = 0, fin = 0;
        if (lane == 0) {
            if (i >= J.ops_len || bad) {
                fin = 1;
            } else {
                int L = 0, d0 = i;
                while (i < J.ops_len && s[i] >= '0' && s[i] <= '9' && L <= (1 << 27))
                    L = L * 10 + (s[i++] - '0');
                const char op = i < J.ops_len ? s[i++] : 0;
                int nt = 0, aa = 0;
                if (i - 1 == d0 || L <= 0) bad = 1;  // no length digits
                switch (op) {
                    case 'M': nt = 3 * L; aa = L; src0 = g; len0 = nt; break;
                    case 'D': nt = 3 * L; src0 = g; len0 = nt; break;
                    case 'I': aa = L; break;
                    case 'F': nt = L; aa = 1; src0 = g; len0 = nt; break;
                    case 'G': nt = L; src0 = g; len0 = nt; break;
                    case 'N': nt = L; ++introns; break;
                    case 'U':
                    case 'V':
                        nt = L;
                        aa = 1;
                        ++introns;
                        if (L < 3) {
                            src0 = g;
                            len0 = L;
                        } else {
                            const int head = op == 'U' ? 1 : 2;
                            src0 = g;
                            len0 = head;
                            src1 = g + L - (3 - head);
                            len1 = 3 - head;
                        }
                        break;
                    default: bad = 1;
                }
                if (g + nt > J.cap || res + aa > J.plen) bad = 1;
                if (bad) len0 = len1 = 0;
                g += nt;
                res += aa;
            }
        }
        fin = __shfl(fin, 0);
        if (fin) break;
        src0 = __shfl(src0, 0);
        len0 = __shfl(len0, 0);
        src1 = __shfl(src1, 0);
        len1 = __shfl(len1, 0);
        for (int q = lane; q < len0; q += 64) out[pos + q] = T[src0 + q];
        for (int q = lane; q < len1; q += 64) out[pos + len0 + q] = T[src1 + q];
        pos += len0 + len1;
    }
    if (lane == 0) {
        if (g != J.cap || res != J.plen) bad = 1;
        info[k] = make_int4(bad ? 0 : pos, introns, bad ? MPG_E_INVAL : MPG_OK, 0);
    }
}

__global__ void rescore_finish_kernel(int n, const mpg_dev_result* __restrict__ res1,
                                      const int4* __restrict__ info, const int32_t* __restrict__ j2,
                                      const mpg_dev_result* __restrict__ res2, int r,
                                      int32_t* __restrict__ score, int32_t* __restrict__ exons,
                                      int32_t* __restrict__ status) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int st = res1[k].status, sc = 0, ex = 0;
    if (st == MPG_OK) {
        const int4 c = info[k];
        ex = c.y + 1;
        st = c.z;
        if (st == MPG_OK) {
            const mpg_dev_result& R = res2[j2[k]];
            st = R.status;
            if (st == MPG_OK) sc = R.score - (ex == 1 ? r : 0);
        }
    }
    score[k] = sc;
    exons[k] = ex;
    status[k] = st;
}

}  // namespace dev

hipError_t launch_dp_k1(hipStream_t, int, bool, const DevParams&, const PairJob*, const int2*, int,
                        int*, void*, int*, const uint8_t*, const uint8_t*, int2*, uint8_t*,
                        const DpSink&);
hipError_t launch_dp_k2(hipStream_t, int, bool, const DevParams&, const PairJob*, const int2*, int,
                        int*, void*, int*, const uint8_t*, const uint8_t*, int2*, uint8_t*,
                        const DpSink&);
hipError_t launch_dp_k4(hipStream_t, int, bool, const DevParams&, const PairJob*, const int2*, int,
                        int*, void*, int*, const uint8_t*, const uint8_t*, int2*, uint8_t*,
                        const DpSink&);
hipError_t launch_dp_p1(hipStream_t, int, bool, const DevParams&, const PairJob*, const int2*, int,
                        int*, void*, int*, const uint8_t*, const uint8_t*, int2*, uint8_t*,
                        const DpSink&);
hipError_t launch_dp_p2(hipStream_t, int, bool, const DevParams&, const PairJob*, const int2*, int,
                        int*, void*, int*, const uint8_t*, const uint8_t*, int2*, uint8_t*,
                        const DpSink&);

int dp_lds_bytes(int K, bool tb) {
    if (K == 1) return tb ? LdsLayout<1, true>::WAVE : LdsLayout<1, false>::WAVE;
    if (K == 2) return tb ? LdsLayout<2, true>::WAVE : LdsLayout<2, false>::WAVE;
    return tb ? LdsLayout<4, true>::WAVE : LdsLayout<4, false>::WAVE;
}

hipError_t launch_prepass(hipStream_t s, const PairJob* jobs, const int64_t* row_start, int npairs,
                          int64_t total_rows, const uint8_t* dna, uint8_t* desc, const DevParams& P) {
    if (total_rows <= 0) return hipSuccess;
    const int64_t per_block = 256 * dev::kPrepassRows;
    const int64_t blocks = (total_rows + per_block - 1) / per_block;
    hipLaunchKernelGGL(prepass_kernel, dim3((unsigned)blocks), dim3(256), 0, s, jobs, row_start,
                       npairs, total_rows, dna, desc, P);
    return hipGetLastError();
}

hipError_t launch_dp(hipStream_t s, int K, bool tb, bool pro, int ncu, const DevParams& P,
                     const PairJob* jobs, const int2* items, int nitems, int* qhead, void* pst,
                     int* prog, const uint8_t* prot, const uint8_t* desc, int2* bnd,
                     uint8_t* tbbuf, const DpSink& sink) {
    if (nitems <= 0) return hipSuccess;
    if (pro) {
        switch (K) {
            case 1: return launch_dp_p1(s, ncu, tb, P, jobs, items, nitems, qhead, pst, prog, prot, desc, bnd, tbbuf, sink);
            case 2: return launch_dp_p2(s, ncu, tb, P, jobs, items, nitems, qhead, pst, prog, prot, desc, bnd, tbbuf, sink);
            default: return hipErrorInvalidValue;
        }
    }
    switch (K) {
        case 1: return launch_dp_k1(s, ncu, tb, P, jobs, items, nitems, qhead, pst, prog, prot, desc, bnd, tbbuf, sink);
        case 2: return launch_dp_k2(s, ncu, tb, P, jobs, items, nitems, qhead, pst, prog, prot, desc, bnd, tbbuf, sink);
        case 4: return launch_dp_k4(s, ncu, tb, P, jobs, items, nitems, qhead, pst, prog, prot, desc, bnd, tbbuf, sink);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(hipStream_t s, const PairJob* jobs, int npairs, void* pst, int* prog,
                       int* qheads, int nq, int gsc_init) {
    if (npairs <= 0 && nq <= 0) return hipSuccess;
    const int n = npairs > nq ? npairs : nq;
    hipLaunchKernelGGL(init_kernel, dim3((n + 255) / 256), dim3(256), 0, s, jobs, npairs,
                       (PairState*)pst, prog, qheads, nq, gsc_init);
    return hipGetLastError();
}

hipError_t launch_walk(hipStream_t s, const PairJob* jobs, const int32_t* order, int count,
                       const uint8_t* tbbuf, mpg_dev_result* out, char* ops) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(walk_kernel, dim3(count), dim3(64), 0, s, jobs, order, count,
                       tbbuf, out, ops);
    return hipGetLastError();
}

hipError_t launch_stitch(hipStream_t s, const ChainJob* chains, int nchains, const int4* runs,
                         const mpg_dev_result* pres, const char* pops, const uint8_t* prot,
                         const uint8_t* dna, const DevParams& P, mpg_dev_result* out,
                         char* ops) {
    if (nchains <= 0) return hipSuccess;
    hipLaunchKernelGGL(stitch_kernel, dim3(nchains), dim3(64), 0, s, chains, nchains, runs, pres,
                       pops, prot, dna, P, out, ops);
    return hipGetLastError();
}

hipError_t launch_cds(hipStream_t s, const CdsJob* jobs, int n, const char* ops, const uint8_t* dna,
                      uint8_t* cds, int4* info) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(cds_kernel, dim3(n), dim3(64), 0, s, jobs, n, ops, dna, cds, info);
    return hipGetLastError();
}

hipError_t launch_rescore_finish(hipStream_t s, int n, const mpg_dev_result* res1,
                                 const int4* info, const int32_t* j2, const mpg_dev_result* res2,
                                 int r, int32_t* score, int32_t* exons, int32_t* status) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(rescore_finish_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, res1,
                       info, j2, res2, r, score, exons, status);
    return hipGetLastError();
}

hipError_t launch_status(hipStream_t s, const PairJob* jobs, int npairs, const DpSink& sink) {
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(status_kernel, dim3((npairs + 255) / 256), dim3(256), 0, s, jobs, npairs,
                       sink);
    return hipGetLastError();
}

// ------------------------------------------------------ fixed scratch array
// Device memory of the allocation-free batch entry point: every buffer of
// such a call beyond the caller's inputs and outputs is carved out of this
// array.  Each GPU holds its own copy from the time the library's code is
// loaded on it until the process ends.  In host code `scratch` only names
// the symbol: its device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is ever passed
// to a kernel or a copy.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(int device, uint8_t** ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller sets the device
        void* a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !a) {
            (void)hipGetLastError();
            return e != hipSuccess ? e : hipErrorInvalidSymbol;
        }
        g_scratch_ptr[device] = (uint8_t*)a;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace mpg
