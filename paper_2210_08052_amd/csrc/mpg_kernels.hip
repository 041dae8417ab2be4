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
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_rows) return;
    int lo = 0, hi = npairs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_start[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    const PairJob& J = jobs[lo];
    const int i = (int)(g - row_start[lo]) - kDescLo;
    const int n = J.n;
    const uint8_t* T = dna + J.dna_off;
    auto base = [&](int x) -> int { return (x >= 1 && x <= n) ? dna_code(T[x - 1]) : 4; };
    int b[9];  // bases i-4 .. i+4
#pragma unroll
    for (int k = 0; k < 9; ++k) b[k] = base(i - 4 + k);
    // codon ending at i: T[i-2..i]
    int tr;
    if (i > n || i < 0) tr = 24;  // poison row
    else if (i < 3 || b[2] == 4 || b[3] == 4 || b[4] == 4) tr = 22;
    else tr = P.gcode[16 * b[2] + 4 * b[3] + b[4]];
    // d(x) uses T[x+1..x+3], a(x) uses T[x-2..x]; b[k] = T[i-4+k]
    auto dpen = [&](int x) -> int {  // x in i-1 .. i+1
        const int o = x - i + 4;
        return P.donor[25 * b[o + 1] + 5 * b[o + 2] + b[o + 3]];
    };
    auto apen = [&](int x) -> int {  // x in i-2 .. i
        const int o = x - i + 4;
        return P.acceptor[25 * b[o - 2] + 5 * b[o - 1] + b[o]];
    };
    const bool valid = (i >= 0 && i <= n);
    int z;
    const int neg = neg_for(J.mode, J.tb != 0);
    if (floor_mode(J.mode)) z = valid ? 0 : neg;
    else z = (i == 0) ? 0 : neg;
    int4* out = (int4*)(desc + J.desc_off + (int64_t)(i + kDescLo) * (J.tb ? 32 : 16));
    if (!J.tb) {
        out[0] = make_int4(tr, z, P.r + dpen(i + 1), apen(i));
    } else {
        out[0] = make_int4(tr, z + 15, 16 * (P.r + dpen(i - 1)) - 7, 16 * (P.r + dpen(i)) - 6);
        out[1] = make_int4(16 * (P.r + dpen(i + 1)) - 5, 16 * apen(i), 16 * apen(i - 2),
                           16 * apen(i - 1));
    }
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

int dp_lds_bytes(int K, bool tb) {
    if (K == 1) return tb ? LdsLayout<1, true>::WAVE : LdsLayout<1, false>::WAVE;
    if (K == 2) return tb ? LdsLayout<2, true>::WAVE : LdsLayout<2, false>::WAVE;
    return tb ? LdsLayout<4, true>::WAVE : LdsLayout<4, false>::WAVE;
}

hipError_t launch_prepass(hipStream_t s, const PairJob* jobs, const int64_t* row_start, int npairs,
                          int64_t total_rows, const uint8_t* dna, uint8_t* desc, const DevParams& P) {
    if (total_rows <= 0) return hipSuccess;
    const int64_t blocks = (total_rows + 255) / 256;
    hipLaunchKernelGGL(prepass_kernel, dim3((unsigned)blocks), dim3(256), 0, s, jobs, row_start,
                       npairs, total_rows, dna, desc, P);
    return hipGetLastError();
}

hipError_t launch_dp(hipStream_t s, int K, bool tb, int ncu, const DevParams& P,
                     const PairJob* jobs, const int2* items, int nitems, int* qhead, void* pst,
                     int* prog, const uint8_t* prot, const uint8_t* desc, int2* bnd,
                     uint8_t* tbbuf, const DpSink& sink) {
    if (nitems <= 0) return hipSuccess;
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

hipError_t launch_status(hipStream_t s, const PairJob* jobs, int npairs, const DpSink& sink) {
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(status_kernel, dim3((npairs + 255) / 256), dim3(256), 0, s, jobs, npairs,
                       sink);
    return hipGetLastError();
}

}  // namespace mpg
