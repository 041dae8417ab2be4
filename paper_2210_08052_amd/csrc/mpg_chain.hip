// Chaining of seed anchors on gfx950 (Methods, "Chaining" of Li 2022):
// Eq. (gap) on a genome binned in 256-bp bins (or, in the second round, the
// base-resolution gap 3*dy - dx), the chaining recurrence
//   f(j) = max(k, max_{i<j} f(i) + min(y_j - y_i, k) - gamma(g(i,j)))
// with the gap penalty of Eq. (gap-pen), then the extraction of chains and
// their ranking.
//
// One wavefront per anchor set.  f of the set's anchors lives in LDS (fp64);
// for anchor j the 64 lanes take the candidates i < j in a strided loop, keep
// their best (value, first index), and a wave reduction picks the maximum
// (ties: smaller i).  Extraction repeats a wave-wide arg-max over the unused
// anchors and lets lane 0 follow the predecessors; ranking repeats a
// wave-wide arg-max over the extracted chains.
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

__global__ void __launch_bounds__(64) chain_kernel(const ChainSetJob* __restrict__ sets,
                                                   int nsets, const int2* __restrict__ anchors,
                                                   ChainCfg cfg, double* __restrict__ f_out,
                                                   int* __restrict__ pred_out,
                                                   ChainRec* __restrict__ recs,
                                                   int* __restrict__ idx_out,
                                                   mpg_chain_out* __restrict__ top,
                                                   int* __restrict__ ntop) {
    if ((int)blockIdx.x >= nsets) return;
    const int lane = threadIdx.x;
    // the jobs come largest set first (the launch's makespan is the largest
    // sets' sequential work); id is the set's own index
    const ChainSetJob S = sets[blockIdx.x];
    const int s = S.id;
    const int n = S.n;
    extern __shared__ __align__(16) uint8_t smem[];
    // LDS: f, then (staged) the anchors and the predecessors, then the used
    // flags.  The anchor reads of the candidate loop and the predecessor walk
    // of the extraction are on the set's sequential path, so staging them
    // takes a global-memory latency off every step of it.
    const bool stage = cfg.stage != 0;
    double* f = (double*)smem;
    int2* sA = (int2*)(smem + 8 * (size_t)cfg.max_n);
    int* spo = (int*)(smem + 16 * (size_t)cfg.max_n);
    uint8_t* used = smem + (stage ? 20 : 8) * (size_t)cfg.max_n;
    const int2* A = anchors + S.off;
    double* fo = f_out + S.off;
    int* po = pred_out + S.off;
    if (S.status != MPG_OK) {
        if (lane == 0) ntop[s] = S.status;
        return;
    }
    if (stage) {
        for (int i = lane; i < n; i += 64) sA[i] = A[i];
        __syncthreads();
    }
    const int2* AA = stage ? (const int2*)sA : A;
    const double kd = (double)cfg.k;
    // ---- the DP, anchor by anchor
    for (int j = 0; j < n; ++j) {
        const int2 aj = AA[j];
        double bv = 0.0;
        int bi = -1;
        for (int i = lane; i < j; i += 64) {
            const int2 ai = AA[i];
            const long long dx = (long long)aj.x - ai.x, dy = (long long)aj.y - ai.y;
            if (dx < 0 || dy <= 0) continue;
            const long long g = chain_gap(dx, dy, cfg.binned);
            if (g >= cfg.G || -g >= cfg.G) continue;
            const double v = (f[i] + (double)(dy < cfg.k ? dy : cfg.k)) - chain_gamma(g, cfg.beta);
            if (bi < 0 || v > bv) {
                bv = v;
                bi = i;
            }
        }
        wave_argmax(bv, bi);
        if (lane == 0) {
            const bool link = bi >= 0 && bv > kd;
            f[j] = link ? bv : kd;
            fo[j] = f[j];
            po[j] = link ? bi : -1;
            if (stage) spo[j] = link ? bi : -1;
        }
        __syncthreads();
    }
    // ---- extraction: the unused anchor of largest f starts a chain that
    // follows the predecessors until -1 or a used anchor
    for (int i = lane; i < n; i += 64) used[i] = 0;
    __syncthreads();
    ChainRec* R = recs + S.off;  // at most n chains
    int* idx = idx_out + S.off;
    int nc = 0, pos = 0;
    for (;;) {
        double bv = 0.0;
        int bi = -1;
        for (int i = lane; i < n; i += 64)
            if (!used[i] && (bi < 0 || f[i] > bv)) {
                bv = f[i];
                bi = i;
            }
        wave_argmax(bv, bi);
        if (bi < 0) break;
        int len = 0;
        if (lane == 0) {
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
            c.score = f[bi] - (t >= 0 ? f[t] : 0.0);
            c.first = pos;
            c.len = len;
            R[nc] = c;
        }
        len = __shfl(len, 0);
        __syncthreads();
        pos += len;
        ++nc;
    }
    // ---- ranking: the max_chains best chains (ties: extracted first)
    const int keep = nc < cfg.max_chains ? nc : cfg.max_chains;
    for (int r = 0; r < keep; ++r) {
        double bv = 0.0;
        int bi = -1;
        for (int c = lane; c < nc; c += 64)
            if (R[c].len > 0 && (bi < 0 || R[c].score > bv)) {
                bv = R[c].score;
                bi = c;
            }
        wave_argmax(bv, bi);
        if (lane == 0) {
            mpg_chain_out o;
            o.score = R[bi].score;
            o.first = R[bi].first;
            o.len = R[bi].len;
            top[(int64_t)s * cfg.max_chains + r] = o;
            R[bi].len = -R[bi].len - 1;  // taken
        }
        __syncthreads();
    }
    if (lane == 0) ntop[s] = keep;
}

}  // namespace dev

hipError_t launch_chain(hipStream_t st, const ChainSetJob* sets, int nsets, const int2* anchors,
                        const ChainCfg& cfg, double* f, int* pred, ChainRec* recs, int* idx,
                        mpg_chain_out* top, int* ntop) {
    if (nsets <= 0) return hipSuccess;
    const size_t lds =
        ((size_t)(cfg.stage ? kChainStageBytes : kChainBaseBytes) * cfg.max_n + 15) & ~(size_t)15;
    hipLaunchKernelGGL(dev::chain_kernel, dim3(nsets), dim3(64), lds, st, sets, nsets, anchors,
                       cfg, f, pred, recs, idx, top, ntop);
    return hipGetLastError();
}

}  // namespace mpg
