// Chaining of seed anchors on gfx950 (Methods, "Chaining" of Li 2022):
// Eq. (gap) on a genome binned in 256-bp bins (or, in the second round, the
// base-resolution gap 3*dy - dx), the chaining recurrence
//   f(j) = max(k, max_{i<j} f(i) + min(y_j - y_i, k) - gamma(g(i,j)))
// with the gap penalty of Eq. (gap-pen), then the extraction of chains and
// their ranking.
//
// One workgroup per anchor set: one wavefront, or four when the launch's
// largest set has 512 anchors or more (its candidate loops are the launch's
// critical path).  f of the set's anchors lives in LDS (fp64), or, for a set
// too large for it, in the f output in HBM, read and written with
// device-scope atomics so that no wavefront reads a stale copy from its
// vector cache.  For anchor j the workgroup's threads take the candidates
// i < j in a strided loop, keep their best (value, first index), and a wave
// reduction, then (several wavefronts) a reduction over the wavefronts' bests
// in LDS, picks the maximum (ties: smaller i).  Extraction repeats an arg-max
// over the unused anchors and lets thread 0 follow the predecessors; ranking
// repeats an arg-max over the extracted chains.
#include "mpg_internal.h"

namespace mpg {
namespace dev {

// Eq. (gap) (binned) or 3*dy - dx (base resolution).
__device__ __forceinline__ long long chain_gap(long long dx, long long dy, int binned) {
    if (!binned) return 3 * dy - dx;
    const long long lo = 256 * (dx - 1), hi = 256 * (dx + 1);
    if (3 * dy < lo) return 3 * dy - lo;
    if (3 * dy > hi) return 3 * dy - hi;
    return 0;
}

// Eq. (gap-pen) for |g| < G.  Each operation rounds on its own (no fused
// multiply-add), in the order the equation is written.
__device__ __forceinline__ double chain_gamma(long long g, double beta) {
#pragma clang fp contract(off)
    if (g == 0) return 0.0;
    const double a = (double)(g < 0 ? -g : g);
    const double third = a / 3.0;
    const double lg = beta * log2(a + 1.0);
    if (g > 0) return third + lg;
    return third < lg ? third : lg;
}

// Wave-wide arg-max of (v, i): the larger v, ties the smaller i (i < 0: none).
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(v, o);
        const int i2 = __shfl_xor(i, o);
        const bool take = i2 >= 0 && (i < 0 || v2 > v || (v2 == v && i2 < i));
        v = take ? v2 : v;
        i = take ? i2 : i;
    }
}

// Arg-max of (v, i) over the workgroup's W wavefronts (the larger v, ties
// the smaller i); every thread receives it.  rv, ri: W slots in LDS.
template <int W>
__device__ __forceinline__ void block_argmax(double& v, int& i, double* rv, int* ri) {
    wave_argmax(v, i);
    if constexpr (W > 1) {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            rv[w] = v;
            ri[w] = i;
        }
        __syncthreads();
        v = rv[0];
        i = ri[0];
#pragma unroll
        for (int q = 1; q < W; ++q) {
            const double v2 = rv[q];
            const int i2 = ri[q];
            const bool take = i2 >= 0 && (i < 0 || v2 > v || (v2 == v && i2 < i));
            v = take ? v2 : v;
            i = take ? i2 : i;
        }
        __syncthreads();  // the slots are free again
    }
}

__device__ __forceinline__ double ld_f64_dev(const double* p) {
    const unsigned long long u = __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)u);
}
__device__ __forceinline__ void st_f64_dev(double* p, double v) {
    __hip_atomic_store((unsigned long long*)p, (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int W>
__global__ void __launch_bounds__(64 * W) chain_kernel(const ChainSetJob* __restrict__ sets,
                                                       int nsets, const int2* __restrict__ anchors,
                                                       ChainCfg cfg, double* __restrict__ f_out,
                                                       int* __restrict__ pred_out,
                                                       ChainRec* __restrict__ recs,
                                                       int* __restrict__ idx_out,
                                                       mpg_chain_out* __restrict__ top,
                                                       int* __restrict__ ntop) {
    constexpr int NT = 64 * W;
    if ((int)blockIdx.x >= nsets) return;
    const int tid = threadIdx.x;
    // the jobs come largest set first (the launch's makespan is the largest
    // sets' sequential work); id is the set's own index
    const ChainSetJob S = sets[blockIdx.x];
    const int s = S.id;
    const int n = S.n;
    extern __shared__ __align__(16) uint8_t smem[];
    // LDS: the reduction slots, then f (if it fits), then (staged) the
    // anchors and the predecessors, then the used flags.  The anchor reads
    // of the candidate loop and the predecessor walk of the extraction are on
    // the set's sequential path, so staging them takes a global-memory
    // latency off every step of it.
    const bool f_lds = cfg.f_lds != 0;
    const bool stage = cfg.stage != 0;
    double* rv = (double*)smem;
    int* ri = (int*)(smem + 8 * W);
    size_t off = kChainRedBytes;
    double* f = (double*)(smem + off);
    if (f_lds) off += 8 * (size_t)cfg.max_n;
    int2* sA = (int2*)(smem + off);
    int* spo = (int*)(smem + off + 8 * (size_t)cfg.max_n);
    if (stage) off += 12 * (size_t)cfg.max_n;
    uint8_t* used = smem + off;
    const int2* A = anchors + S.off;
    double* fo = f_out + S.off;
    int* po = pred_out + S.off;
    auto fget = [&](int i) -> double { return f_lds ? f[i] : ld_f64_dev(fo + i); };
    if (S.status != MPG_OK) {
        if (tid == 0) ntop[s] = S.status;
        return;
    }
    if (stage) {
        for (int i = tid; i < n; i += NT) sA[i] = A[i];
        __syncthreads();
    }
    const int2* AA = stage ? (const int2*)sA : A;
    const double kd = (double)cfg.k;
    // ---- the DP, anchor by anchor
    for (int j = 0; j < n; ++j) {
        const int2 aj = AA[j];
        double bv = 0.0;
        int bi = -1;
        for (int i = tid; i < j; i += NT) {
            const int2 ai = AA[i];
            const long long dx = (long long)aj.x - ai.x, dy = (long long)aj.y - ai.y;
            if (dx < 0 || dy <= 0) continue;
            const long long g = chain_gap(dx, dy, cfg.binned);
            if (g >= cfg.G || -g >= cfg.G) continue;
            const double v = (fget(i) + (double)(dy < cfg.k ? dy : cfg.k)) - chain_gamma(g, cfg.beta);
            if (bi < 0 || v > bv) {
                bv = v;
                bi = i;
            }
        }
        block_argmax<W>(bv, bi, rv, ri);
        if (tid == 0) {
            const bool link = bi >= 0 && bv > kd;
            const double fj = link ? bv : kd;
            if (f_lds) {
                f[j] = fj;
                fo[j] = fj;
            } else {
                st_f64_dev(fo + j, fj);
            }
            po[j] = link ? bi : -1;
            if (stage) spo[j] = link ? bi : -1;
        }
        __syncthreads();
    }
    // ---- extraction: the unused anchor of largest f starts a chain that
    // follows the predecessors until -1 or a used anchor
    for (int i = tid; i < n; i += NT) used[i] = 0;
    __syncthreads();
    ChainRec* R = recs + S.off;  // at most n chains
    int* idx = idx_out + S.off;
    int* slen = ri + W;  // one more slot: the chain's length for every thread
    int nc = 0, pos = 0;
    for (;;) {
        double bv = 0.0;
        int bi = -1;
        for (int i = tid; i < n; i += NT)
            if (!used[i]) {
                const double fi = fget(i);
                if (bi < 0 || fi > bv) {
                    bv = fi;
                    bi = i;
                }
            }
        block_argmax<W>(bv, bi, rv, ri);
        if (bi < 0) break;
        if (tid == 0) {
            int len = 0;
            int t = bi;
            const int* P = stage ? (const int*)spo : po;
            while (t >= 0 && !used[t]) {
                used[t] = 1;
                ++len;
                t = P[t];
            }
            // indices ascending: write from the end of the chain's range
            int u = bi;
            for (int q = len - 1; q >= 0; --q) {
                idx[pos + q] = u;
                u = P[u];
            }
            ChainRec c;
            c.score = fget(bi) - (t >= 0 ? fget(t) : 0.0);
            c.first = pos;
            c.len = len;
            R[nc] = c;
            *slen = len;
        }
        __syncthreads();
        pos += *slen;
        ++nc;
        __syncthreads();  // slen is written again by the next chain
    }
    // ---- ranking: the max_chains best chains (ties: extracted first)
    const int keep = nc < cfg.max_chains ? nc : cfg.max_chains;
    for (int r = 0; r < keep; ++r) {
        double bv = 0.0;
        int bi = -1;
        for (int c = tid; c < nc; c += NT)
            if (R[c].len > 0 && (bi < 0 || R[c].score > bv)) {
                bv = R[c].score;
                bi = c;
            }
        block_argmax<W>(bv, bi, rv, ri);
        if (tid == 0) {
            mpg_chain_out o;
            o.score = R[bi].score;
            o.first = R[bi].first;
            o.len = R[bi].len;
            top[(int64_t)s * cfg.max_chains + r] = o;
            R[bi].len = -R[bi].len - 1;  // taken
        }
        __syncthreads();
    }
    if (tid == 0) ntop[s] = keep;
}

}  // namespace dev

hipError_t launch_chain(hipStream_t st, const ChainSetJob* sets, int nsets, const int2* anchors,
                        const ChainCfg& cfg, double* f, int* pred, ChainRec* recs, int* idx,
                        mpg_chain_out* top, int* ntop) {
    if (nsets <= 0) return hipSuccess;
    const size_t lds = chain_lds_bytes(cfg);
    if (cfg.waves == 4)
        hipLaunchKernelGGL(dev::chain_kernel<4>, dim3(nsets), dim3(256), lds, st, sets, nsets,
                           anchors, cfg, f, pred, recs, idx, top, ntop);
    else
        hipLaunchKernelGGL(dev::chain_kernel<1>, dim3(nsets), dim3(64), lds, st, sets, nsets,
                           anchors, cfg, f, pred, recs, idx, top, ntop);
    return hipGetLastError();
}

}  // namespace mpg
