// Traceback walk shared by the walk kernel and the DP kernels (which run it
// in the wavefront that finishes a pair when results are published per pair).
#pragma once

#include "mpg_internal.h"

namespace mpg {
namespace dev {

struct TbView {
    const uint8_t* base;
    int K, nchunks;
    __device__ __forceinline__ const uint8_t* blk(int i, int j, int& k, int& c, int& t) const {
        const int SW = 64 * K;
        const int S = j / SW;
        const int jj = j - S * SW;
        k = jj / K;
        c = jj - k * K;
        const int s = i + k;
        t = s & 63;
        return base + ((int64_t)S * nchunks + (s >> 6)) * (kTbBlockBytes * K);
    }
    __device__ __forceinline__ int code(int i, int j) const {
        int k, c, t;
        const uint8_t* b = blk(i, j, k, c, t);
        const uint32_t w = *(const uint32_t*)(b + (((t >> 3) * K + c) * 64 + k) * 4);
        return 15 - (int)((w >> ((t & 7) * 4)) & 15u);
    }
    // 1 if state x (I, D, A, B, C) extended at (i, j); the stored bit is 1
    // where the state opened
    __device__ __forceinline__ int ext(int x, int i, int j) const {
        int k, c, t;
        const uint8_t* b = blk(i, j, k, c, t);
        const uint32_t w =
            *(const uint32_t*)(b + 2048 * K + (((x * K + c) * 2 + (t >> 5)) * 64 + k) * 4);
        return (int)((~w >> (31 - (t & 31))) & 1u);
    }
};

__device__ __forceinline__ int ndigits(int v) {
    int d = 1;
    while (v >= 10) { v /= 10; ++d; }
    return d;
}

// Op-string writer: tokens are produced last-to-first and written backwards
// from the end of the pair's slot; lane 0 stores the bytes.  M, I and D runs
// are merged into one token, F, G, N, U and V never.
struct OpWriter {
    char* txt;
    int64_t pos;   // first byte written so far
    char pop = 0;  // pending (not yet written) token
    int plen = 0;
    bool overflow = false;
    __device__ void flush(int lane) {
        if (!pop) return;
        const int nd = ndigits(plen);
        if (pos < nd + 1) {
            overflow = true;
            pop = 0;
            return;
        }
        if (lane == 0) {
            txt[pos - 1] = pop;
            int v = plen;
            for (int d = 2; d <= nd + 1; ++d) {
                txt[pos - d] = (char)('0' + v % 10);
                v /= 10;
            }
        }
        pos -= nd + 1;
        pop = 0;
    }
    __device__ void emit(char op, int l, bool merge, int lane) {
        if (merge && pop == op) {
            plen += l;
            return;
        }
        flush(lane);
        pop = op;
        plen = l;
        if (!merge) flush(lane);
    }
};

// Walks one pair back from its end cell, one wavefront per pair.  The
// choices along the path are read speculatively 64 at a time: in state H the
// lanes read the H codes down the diagonal (a run of codon:residue steps),
// in a gap state the extension bits along the gap, and in an intron state
// the extension bits of 4 consecutive rows each (256 rows per round); a
// ballot finds where the run ends.  Every round is then one memory round
// trip for up to 64-256 steps of the path.  Returns the start cell in
// (bi, bj), or false on an inconsistent path (never expected).
__device__ bool walk_wave(const TbView& V, int i, int j, int n, int m, OpWriter& W, int lane,
                          int& bi, int& bj) {
    int st = 0;  // 0 H, 1 I, 2 D, 3 A, 4 B, 5 C
    int kend = 0;
    const int64_t guard = 4LL * (n + m) + 64;
    for (int64_t it = 0; it < guard; ++it) {
        if (i < 0 || j < 0 || i > n || j > m) return false;
        if (st == 0) {
            const int ii = i - 3 * lane, jj = j - lane;
            const bool ok = ii >= 0 && jj >= 0;
            const int hc = ok ? V.code(ii, jj) : -1;
            const uint64_t stop = __ballot(hc != 1);
            if (stop == 0) {
                W.emit('M', 64, true, lane);
                i -= 192;
                j -= 64;
                continue;
            }
            const int l = __builtin_ctzll(stop);
            if (l) W.emit('M', l, true, lane);
            i -= 3 * l;
            j -= l;
            const int c = __builtin_amdgcn_readlane(hc, l);
            switch (c) {
                case 0:
                    W.flush(lane);
                    bi = i;
                    bj = j;
                    return true;
                case 2: st = 1; break;
                case 3: st = 2; break;
                case 4: W.emit('F', 1, false, lane); i -= 1; j -= 1; break;
                case 5: W.emit('F', 2, false, lane); i -= 2; j -= 1; break;
                case 6: W.emit('G', 1, false, lane); i -= 1; break;
                case 7: W.emit('G', 2, false, lane); i -= 2; break;
                case 8: st = 3; kend = i; break;
                case 9: st = 4; kend = i; break;
                case 10: st = 5; kend = i; break;
                default: return false;
            }
        } else if (st <= 2) {
            // gap run: I moves left along the row, D up by one codon
            const int ii = st == 1 ? i : i - 3 * lane;
            const int jj = st == 1 ? j - lane : j;
            const bool ok = ii >= 0 && jj >= 0;
            const int bit = ok ? V.ext(st - 1, ii, jj) : 0;
            const uint64_t endm = __ballot(!ok || !bit);
            if (endm == 0) {
                W.emit(st == 1 ? 'I' : 'D', 64, true, lane);
                if (st == 1) j -= 64; else i -= 192;
                continue;
            }
            const int l = __builtin_ctzll(endm);
            if (!__builtin_amdgcn_readlane((int)ok, l)) return false;
            W.emit(st == 1 ? 'I' : 'D', l + 1, true, lane);
            if (st == 1) j -= l + 1; else i -= 3 * (l + 1);
            st = 0;
        } else {
            // intron run: rows i - (4*lane + r), r = 0..3
            int first = 4;
            bool bad = false;
#pragma unroll
            for (int r = 3; r >= 0; --r) {
                const int ii = i - 4 * lane - r;
                if (ii < 0) {
                    first = r;
                    bad = true;
                } else if (!V.ext(st - 1, ii, j)) {
                    first = r;
                    bad = false;
                }
            }
            const uint64_t endm = __ballot(first < 4);
            if (endm == 0) {
                i -= 256;
                continue;
            }
            const int l = __builtin_ctzll(endm);
            if (__builtin_amdgcn_readlane((int)bad, l)) return false;
            const int f = 4 * l + __builtin_amdgcn_readlane(first, l);
            const int k = i - f;
            W.emit(st == 3 ? 'N' : st == 4 ? 'U' : 'V', kend - k + 1, false, lane);
            if (st != 3) j -= 1;
            i = k - 1;
            st = 0;
        }
    }
    return false;
}

}  // namespace dev
}  // namespace mpg
