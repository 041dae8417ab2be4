// Host runtime of the spliced protein-to-genome DP library: parameters,
// validation, planning, device memory, batch entry points and the serving
// loop.  All DP arithmetic runs in the HIP kernels of mpg_kernels.hip; this
// file only marshals arguments, sizes buffers and orders launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mpg_internal.h"

using namespace mpg;

namespace {

// ---------------------------------------------------------------- defaults
// BLOSUM62 (Henikoff & Henikoff 1992) in the order ARNDCQEGHILKMFPSTWYVBZX*.
const int8_t kBlosum62[24][24] = {
    {4, -1, -2, -2, 0, -1, -1, 0, -2, -1, -1, -1, -1, -2, -1, 1, 0, -3, -2, 0, -2, -1, 0, -4},
    {-1, 5, 0, -2, -3, 1, 0, -2, 0, -3, -2, 2, -1, -3, -2, -1, -1, -3, -2, -3, -1, 0, -1, -4},
    {-2, 0, 6, 1, -3, 0, 0, 0, 1, -3, -3, 0, -2, -3, -2, 1, 0, -4, -2, -3, 3, 0, -1, -4},
    {-2, -2, 1, 6, -3, 0, 2, -1, -1, -3, -4, -1, -3, -3, -1, 0, -1, -4, -3, -3, 4, 1, -1, -4},
    {0, -3, -3, -3, 9, -3, -4, -3, -3, -1, -1, -3, -1, -2, -3, -1, -1, -2, -2, -1, -3, -3, -2, -4},
    {-1, 1, 0, 0, -3, 5, 2, -2, 0, -3, -2, 1, 0, -3, -1, 0, -1, -2, -1, -2, 0, 3, -1, -4},
    {-1, 0, 0, 2, -4, 2, 5, -2, 0, -3, -3, 1, -2, -3, -1, 0, -1, -3, -2, -2, 1, 4, -1, -4},
    {0, -2, 0, -1, -3, -2, -2, 6, -2, -4, -4, -2, -3, -3, -2, 0, -2, -2, -3, -3, -1, -2, -1, -4},
    {-2, 0, 1, -1, -3, 0, 0, -2, 8, -3, -3, -1, -2, -1, -2, -1, -2, -2, 2, -3, 0, 0, -1, -4},
    {-1, -3, -3, -3, -1, -3, -3, -4, -3, 4, 2, -3, 1, 0, -3, -2, -1, -3, -1, 3, -3, -3, -1, -4},
    {-1, -2, -3, -4, -1, -2, -3, -4, -3, 2, 4, -2, 2, 0, -3, -2, -1, -2, -1, 1, -4, -3, -1, -4},
    {-1, 2, 0, -1, -3, 1, 1, -2, -1, -3, -2, 5, -1, -3, -1, 0, -1, -3, -2, -2, 0, 1, -1, -4},
    {-1, -1, -2, -3, -1, 0, -2, -3, -2, 1, 2, -1, 5, 0, -2, -1, -1, -1, -1, 1, -3, -1, -1, -4},
    {-2, -3, -3, -3, -2, -3, -3, -3, -1, 0, 0, -3, 0, 6, -4, -2, -2, 1, 3, -1, -3, -3, -1, -4},
    {-1, -2, -2, -1, -3, -1, -1, -2, -2, -3, -3, -1, -2, -4, 7, -1, -1, -4, -3, -2, -2, -1, -2, -4},
    {1, -1, 1, 0, -1, 0, 0, 0, -1, -2, -2, 0, -1, -2, -1, 4, 1, -3, -2, -2, 0, 0, 0, -4},
    {0, -1, 0, -1, -1, -1, -1, -2, -2, -1, -1, -1, -1, -2, -1, 1, 5, -2, -2, 0, -1, -1, 0, -4},
    {-3, -3, -4, -4, -2, -2, -3, -2, -2, -3, -2, -3, -1, 1, -4, -3, -2, 11, 2, -3, -4, -3, -2, -4},
    {-2, -2, -2, -3, -2, -1, -2, -3, 2, -1, -1, -2, -1, 3, -3, -2, -2, 2, 7, -1, -3, -2, -1, -4},
    {0, -3, -3, -3, -1, -2, -2, -3, -3, 3, 1, -2, 1, -1, -2, -2, 0, -3, -1, 4, -3, -2, -1, -4},
    {-2, -1, 3, 4, -3, 0, 1, -1, 0, -3, -4, 0, -3, -3, -2, 0, -1, -4, -3, -3, 4, 1, -1, -4},
    {-1, 0, 0, 1, -3, 3, 4, -2, 0, -3, -3, 1, -1, -3, -1, 0, -1, -3, -2, -2, 1, 4, -1, -4},
    {0, -1, -1, -1, -2, -1, -1, -1, -1, -1, -1, -1, -1, -1, -2, 0, 0, -2, -1, -1, -1, -1, -1, -4},
    {-4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, 1},
};

const char kAlphabet[] = "ARNDCQEGHILKMFPSTWYVBZX*";
// Standard genetic code, codons in A,C,G,T nesting order (AAA, AAC, ..., TTT).
const char kCodeACGT[] = "KNKNTTTTRSRSIIMIQHQHPPPPRRRRLLLLEDEDAAAAGGGGVVVV*Y*YSSSS*CWCLFLF";

// Final splice model ("Splice models"): donor penalty from the intron's first
// three bases, acceptor penalty from its last three; N and out-of-range bases
// never match a listed pattern.
int donor_pen(int b1, int b2, int b3) {
    enum { A = 0, C = 1, G = 2, T = 3 };
    if (b1 == G && b2 == T && (b3 == A || b3 == G)) return 0;
    if (b1 == G && b2 == T && (b3 == C || b3 == T)) return 8;
    if (b1 == G && b2 == C) return 15;
    if (b1 == A && b2 == T) return 21;
    return 30;
}
int acceptor_pen(int b1, int b2, int b3) {
    enum { A = 0, C = 1, G = 2, T = 3 };
    if ((b1 == C || b1 == T) && b2 == A && b3 == G) return 0;
    if ((b1 == A || b1 == G) && b2 == A && b3 == G) return 8;
    if (b2 == A && b3 == C) return 21;
    return 30;
}

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ------------------------------------------------------------- device memory
// Where device workspace memory comes from: the caller's allocator set with
// mpg_set_allocator, else hipMalloc / hipFree.  A block goes back through
// the allocator that made it.
struct DevAlloc {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*release)(void*, void*) = nullptr;
    void* user = nullptr;
};

void free_dev(void* q, const DevAlloc& a) {
    if (!q) return;
    if (a.release) a.release(q, a.user);
    else (void)hipFree(q);
}

// Buffers outgrown while other work may be running.  hipFree and hipHostFree
// wait for the whole device, and a caller's allocator may hand a block to
// other work at once, so a serving workspace must not free while batches run
// on other streams: it parks outgrown buffers here, and the scheduler frees
// them when no batch is on the device.
struct Retired {
    std::mutex mu;
    std::vector<std::pair<void*, DevAlloc>> dev;
    std::vector<void*> host;
    void flush() {
        std::lock_guard<std::mutex> g(mu);
        for (auto& q : dev) free_dev(q.first, q.second);
        for (void* q : host) (void)hipHostFree(q);
        dev.clear();
        host.clear();
    }
};

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    Retired* later = nullptr;      // set: park outgrown buffers instead of freeing
    const DevAlloc* src = nullptr;  // allocator of new blocks (NULL or empty: hipMalloc)
    DevAlloc owner;                 // allocator of the current block
    // One block of `bytes` from the allocator in effect; MPG_E_INVAL if a
    // caller's allocator returns a block that is not 256-byte aligned.
    int grab(size_t bytes) {
        if (src && src->alloc) {
            void* q = src->alloc(bytes, src->user);
            if (!q) return MPG_E_NOMEM;
            if ((uintptr_t)q & 255) {
                src->release(q, src->user);
                return MPG_E_INVAL;
            }
            p = q;
            owner = *src;
            return MPG_OK;
        }
        if (hipMalloc(&p, bytes) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return MPG_E_NOMEM;
        }
        owner = DevAlloc{};
        return MPG_OK;
    }
    int ensure(size_t bytes) {
        if (bytes <= cap) return MPG_OK;
        if (p && later) {
            std::lock_guard<std::mutex> g(later->mu);
            later->dev.push_back({p, owner});
        } else if (p) {
            free_dev(p, owner);
        }
        p = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(bytes, 256);
        want = want + want / 4;
        int rc = grab(want);
        if (rc == MPG_E_NOMEM) {
            rc = grab(bytes);
            want = bytes;
        }
        if (rc != MPG_OK) {
            p = nullptr;
            return rc;
        }
        cap = want;
        return MPG_OK;
    }
    void release() {
        free_dev(p, owner);
        p = nullptr;
        cap = 0;
    }
};

struct HostBuf {  // pinned host memory
    void* p = nullptr;
    size_t cap = 0;
    // coherent: device writes become visible to the host while a kernel runs
    // (result records and op strings that the host polls)
    unsigned flags = hipHostMallocDefault;
    Retired* later = nullptr;  // set: park outgrown buffers instead of freeing
    int ensure(size_t bytes) {
        if (bytes <= cap) return MPG_OK;
        if (p && later) {
            std::lock_guard<std::mutex> g(later->mu);
            later->host.push_back(p);
        } else if (p) {
            hipHostFree(p);
        }
        p = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(bytes, 4096);
        want = want + want / 4;
        if (hipHostMalloc(&p, want, flags) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return MPG_E_NOMEM;
        }
        cap = want;
        return MPG_OK;
    }
    void release() {
        if (p) hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
};

// One DP launch: the strips of every pair sharing (K, traceback, kernel
// mode), as a queue of (job, strip) items, longest pair first, strips in
// order.  The int16 group's items are (pack, strip).
struct Group {
    int K;
    bool tb;
    bool i16;
    int mode;  // kernel variant of the group's pairs (EXTEND_LEFT pairs run in GLOBAL's)
    size_t off, cnt;  // its work items in Plan::items
};

struct Plan {
    std::vector<int2> items;  // work items of every group, group after group
    // lane-segment packs: per job, the partner whose last strip shares its
    // wavefront (-1: none), and per job whether it carries the pack item
    std::vector<int32_t> seg_mate;
    std::vector<uint8_t> seg_emit;
    std::vector<int32_t> seg_key;  // per job: pack class and lanes, or -1
    std::vector<std::pair<int64_t, int32_t>> seg_cand;
    // planning scratch: per job group key, traceback and strips; the queue
    // orders and the sort's buffers
    std::vector<uint32_t> ginfo;
    std::vector<std::pair<int64_t, int32_t>> bysize, e16, sort_tmp;
    std::vector<uint32_t> sort_cnt;
    std::vector<PairJob> jobs;
    std::vector<int64_t> row_start;
    std::vector<Group> groups;
    std::vector<int32_t> walk;
    std::vector<PackJob> packs;
    std::vector<int64_t> pack_row_start;
    int64_t desc_bytes = 0, bnd_elems = 0, tb_bytes = 0;
    int64_t total_rows = 0, pack_rows = 0;
    int64_t nprog = 0;
};

// Everything one in-flight batch needs on the device.  The DP launches of a
// batch (one per kernel variant) run concurrently on side streams forked
// from the batch stream and joined back with events.
constexpr int kSideStreams = 8;
struct Workspace {
    DevBuf jobs, row_start, order, desc, bnd, tb, seq, out, ops, state, chain, piece_out,
        piece_ops, cset, cio;
    HostBuf hplan, hseq, hout, hops, hchain, hcset;
    HostBuf prec, pops;  // serving: host-mapped records and op strings the host polls
    // host-side planning storage kept from call to call, so that large plans
    // reuse memory that is already mapped instead of faulting in new pages
    Plan plan_cache;
    std::vector<mpg_seg> psegs;
    std::vector<int8_t> pmodes;
    std::vector<int4> cruns;
    std::vector<ChainJob> cjobs;
    std::vector<int64_t> wave_ops_off;
    std::vector<int32_t> wave_idx;
    void use_allocator(const DevAlloc* a) {
        DevBuf* d[] = {&jobs, &row_start, &order, &desc, &bnd, &tb, &seq, &out, &ops, &state,
                       &chain, &piece_out, &piece_ops, &cset, &cio};
        for (auto* b : d) b->src = a;
    }
    void defer_frees(Retired* r) {
        DevBuf* d[] = {&jobs, &row_start, &order, &desc, &bnd, &tb, &seq, &out, &ops, &state,
                       &chain, &piece_out, &piece_ops, &cset, &cio};
        for (auto* b : d) b->later = r;
        HostBuf* h[] = {&hplan, &hseq, &hout, &hops, &prec, &pops, &hchain, &hcset};
        for (auto* b : h) b->later = r;
    }
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kSideStreams] = {};
    bool streams_ready = false;
    int ensure_streams() {
        if (streams_ready) return MPG_OK;
        for (int k = 0; k < kSideStreams; ++k) {
            if (hipStreamCreateWithFlags(&side[k], hipStreamNonBlocking) != hipSuccess)
                return MPG_E_DEVICE;
            if (hipEventCreateWithFlags(&join_ev[k], hipEventDisableTiming) != hipSuccess)
                return MPG_E_DEVICE;
        }
        if (hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming) != hipSuccess)
            return MPG_E_DEVICE;
        streams_ready = true;
        return MPG_OK;
    }
    void release() {
        DevBuf* d[] = {&jobs, &row_start, &order, &desc, &bnd, &tb, &seq, &out, &ops, &state,
                       &chain, &piece_out, &piece_ops, &cset, &cio};
        for (auto* b : d) b->release();
        HostBuf* h[] = {&hplan, &hseq, &hout, &hops, &prec, &pops, &hchain, &hcset};
        for (auto* b : h) b->release();
        if (streams_ready) {
            for (int k = 0; k < kSideStreams; ++k) {
                hipStreamSynchronize(side[k]);
                hipStreamDestroy(side[k]);
                hipEventDestroy(join_ev[k]);
            }
            hipEventDestroy(fork_ev);
            streams_ready = false;
        }
    }
};

// ------------------------------------------------------------------ planning

int g_max_lds = 65536;

// Debug-only override (tests use it to reach every kernel variant on small
// inputs): MPG_FORCE_K = columns per lane.
int env_int(const char* name) {
    const char* v = std::getenv(name);
    return v ? std::atoi(v) : 0;
}

// Debug overrides are read once per call (getenv per pair is too slow).
struct Overrides {
    int K = 0, K16 = 0;
    bool no_seg = false;  // MPG_NO_SEG_PACK=1: every last strip in a wavefront of its own
    Overrides()
        : K(env_int("MPG_FORCE_K")), K16(env_int("MPG_FORCE_K16")),
          no_seg(env_int("MPG_NO_SEG_PACK") != 0) {}
};

// Planning choices made by mpg_autotune from timed runs (0: not tuned).
struct Tuning {
    int K = 0;       // int32 kernels
    int K16 = 0;     // int16 kernel
    int narrow = 0;  // pairs of at most this many columns run one column per lane (64)
    int seg = -1;    // lane-segment packs: 1 on, 0 off, -1 not tuned (on)
};

// Columns per lane: one width for the pairs of a call wider than 64 columns
// (pairs of one width share a launch; mixed widths would split the device
// between concurrent persistent launches): a forced width, else the tuned
// one, else 2.  Pairs of at most 64 columns take width 1.
struct KChoice {
    int K[2] = {2, 2};  // [traceback]
};

KChoice choose_widths(const Overrides& ov, const Tuning* tu, int force) {
    KChoice kc;
    int K = 2;
    if (ov.K == 1 || ov.K == 2 || ov.K == 4) K = ov.K;
    else if (force) K = force;
    else if (tu && tu->K) K = tu->K;
    kc.K[0] = kc.K[1] = K;
    return kc;
}

// Columns per lane of the int16 kernel (one width for a whole call: pairs of
// a pack share it).
int choose_K16(const Overrides& ov, const Tuning* tu, int force = 0) {
    if (ov.K16 == 1 || ov.K16 == 2) return ov.K16;
    if (force) return force;
    if (tu && tu->K16) return tu->K16;
    return 2;
}

int g_num_cu = 256;  // compute units of the device (the DP grid is sized per CU)

// Steps every strip of a pair runs (a multiple of 64).  Lane L reaches row
// n at step n + L: a pair of one strip stops once the lane of column m has,
// the strips of a wider pair run all 64 lanes to row n.
int pair_nsteps(int n, int m, int K) {
    const int nstrips = (m + 1 + 64 * K - 1) / (64 * K);
    const int lanes = nstrips == 1 ? m / K + 1 : 64;
    return ((n + lanes + 63) / 64) * 64;
}

int64_t tb_bytes_of(int n, int m, int K) {
    const int nsteps = pair_nsteps(n, m, K);
    const int nstrips = (m + 1 + 64 * K - 1) / (64 * K);
    return (int64_t)nstrips * (nsteps / 64) * kTbBlockBytes * K;
}

// Direction-bit bytes of a pair at the width that needs most.
int64_t tb_bytes_max(int n, int m) {
    return std::max({tb_bytes_of(n, m, 1), tb_bytes_of(n, m, 2), tb_bytes_of(n, m, 4)});
}

// Bound on |value| of reachable cells (see the public header): the largest
// match score times the protein length, and (EXTEND/GLOBAL, whose H has no 0
// floor) the largest per-unit penalty times the number of units a path can
// consume.
struct BoundInfo {
    int64_t maxpos = 0, pmax = 0;
    int64_t pfix = 0;  // the penalties a profile does not replace: f, r + d + a
    explicit BoundInfo(const mpg_params* p) {
        int mp = 0, mn = 0;
        for (int a = 0; a < 24; ++a)
            for (int b = 0; b < 24; ++b) {
                mp = std::max<int>(mp, p->mat[a][b]);
                mn = std::min<int>(mn, p->mat[a][b]);
            }
        int dmax = 0, amax = 0;
        for (int k = 0; k < 125; ++k) {
            dmax = std::max<int>(dmax, p->donor[k]);
            amax = std::max<int>(amax, p->acceptor[k]);
        }
        maxpos = mp;
        pfix = std::max<int64_t>((int64_t)p->f, (int64_t)p->r + dmax + amax);
        pmax = std::max<int64_t>({(int64_t)p->q + p->e, pfix, (int64_t)-mn});
    }
    // the same bound for a position-specific query whose largest score is
    // smax and whose largest gap cost or negated score is gmax
    BoundInfo profile(int64_t smax, int64_t gmax) const {
        BoundInfo b = *this;
        b.maxpos = std::max<int64_t>(0, smax);
        b.pmax = std::max(pfix, gmax);
        return b;
    }
    bool ok(int64_t n, int64_t m, int mode) const {
        const int64_t lim = (int64_t)1 << 24;
        if (maxpos * (m + 1) >= lim) return false;
        if (mode == MPG_LOCAL || mode == MPG_EXTEND_LEFT) return pmax * 4 < lim;
        return (n + m + 4) * pmax < lim;
    }
    // int16 lanes (LOCAL only): H >= 0 everywhere, so reachable values lie in
    // [-(the largest penalty sum), the best score]; the best score of a
    // protein of m residues is at most m times the largest matrix entry.
    // Both must stay clear of the int16 range with room to spare.
    bool ok16(int64_t m, int mode) const {
        return mode == MPG_LOCAL && maxpos * m <= 32767 - 256 && pmax <= 8192;
    }
};

bool score_bound_ok(const mpg_params* p, int64_t n, int64_t m) {
    return BoundInfo(p).ok(n, m, p->mode);
}

void make_dev_params(const mpg_params* p, DevParams* d) {
    std::memset(d, 0, sizeof(*d));
    d->q = p->q;
    d->e = p->e;
    d->f = p->f;
    d->r = p->r;
    d->mode = p->mode;
    d->flags = (int32_t)p->flags;
    std::memcpy(d->mat, p->mat, sizeof(d->mat));
    std::memcpy(d->gcode, p->gcode, 64);
    std::memcpy(d->donor, p->donor, 125);
    std::memcpy(d->acceptor, p->acceptor, 125);
    d->max_polls = kMaxPolls;
    // debug override for tests of the failure path: MPG_DEBUG_WAIT_POLLS=0
    // makes every bounded wait between strips give up at once (its pairs
    // report MPG_E_DEVICE; every kernel still runs to its end)
    if (const char* v = std::getenv("MPG_DEBUG_WAIT_POLLS"))
        d->max_polls = std::max(0, std::min(std::atoi(v), (int)kMaxPolls));
}

struct Timer;

// How a call runs on the device.
struct RunCfg {
    uint64_t tb_budget = 0;
    Timer* tm = nullptr;
    int ncu = 256;      // compute units the DP grid may fill
    bool serve = false; // results pair by pair: the finishing wavefront walks
                        // the traceback and publishes the record (status
                        // last) to memory the host polls; shortest pairs first
    const Tuning* tune = nullptr;  // measured costs for choosing K
    int force_K = 0, force_K16 = 0;  // calibration runs: one width for all
    const int8_t* modes = nullptr;   // per pair of the call: its boundary mode
                                     // (NULL: params.mode for every pair)
    bool pro = false;                // position-specific queries (prot_off: profile block)
    const int32_t* pro_bounds = nullptr;  // per pair: largest score, largest cost
    // set: the workspace is free once this event has completed, so the host
    // waits for it instead of for the whole stream (and plans while earlier
    // work still runs); it covers the call's first use of the workspace only
    hipEvent_t ws_ready = nullptr;
};

// Wait until the workspace may be reused: its readiness event when the call
// has one, else everything on the stream.
int wait_workspace(hipStream_t st, const RunCfg& cfg) {
    const hipError_t e = cfg.ws_ready ? hipEventSynchronize(cfg.ws_ready) : hipStreamSynchronize(st);
    return e == hipSuccess ? MPG_OK : MPG_E_DEVICE;
}

// Stable sort of (key, index) entries by key, ascending or descending; the
// entries arrive in index order, so equal keys stay in index order (the
// order a comparison sort with an index tie-break gives).  LSD radix over
// 16-bit digits: planning sorts up to ~10^5 entries per call.
void sort_by_key(std::vector<std::pair<int64_t, int32_t>>& v, bool descending,
                 std::vector<std::pair<int64_t, int32_t>>& tmp, std::vector<uint32_t>& cnt) {
    if (v.size() < 2) return;
    int64_t lo = v[0].first, hi = v[0].first;
    for (const auto& e : v) {
        lo = std::min(lo, e.first);
        hi = std::max(hi, e.first);
    }
    auto digit_key = [&](int64_t k) -> uint64_t {
        return descending ? (uint64_t)(hi - k) : (uint64_t)(k - lo);
    };
    const uint64_t span = (uint64_t)(hi - lo);
    tmp.resize(v.size());
    // 16-bit digits for large inputs, 8-bit ones below 16k entries (where
    // clearing and scanning 65,536 counters per pass would dominate)
    const int bits = v.size() < 16384 ? 8 : 16;
    const uint64_t mask = (1u << bits) - 1;
    cnt.resize((size_t)mask + 2);
    for (int sh = 0; sh < 64 && (span >> sh) != 0; sh += bits) {
        std::fill(cnt.begin(), cnt.end(), 0u);
        for (const auto& e : v) ++cnt[((digit_key(e.first) >> sh) & mask) + 1];
        for (uint64_t d = 0; d <= mask; ++d) cnt[d + 1] += cnt[d];
        for (const auto& e : v) tmp[cnt[(digit_key(e.first) >> sh) & mask]++] = e;
        v.swap(tmp);
    }
}

// Build the plan for the pairs idx[0..cnt) of a call with n pairs.  Each
// job writes result record idx[k] and its op string at ops_off[idx[k]].
void plan_pairs(const mpg_params* p, const mpg_seg* segs, const int32_t* idx, int32_t cnt,
                const std::vector<int64_t>& ops_off, Plan& P, const RunCfg& cfg) {
    const uint64_t tb_budget = cfg.tb_budget;
    const bool shortest_first = cfg.serve;
    P.jobs.assign(cnt, PairJob{});
    P.row_start.assign(cnt, 0);
    P.groups.clear();
    P.items.clear();
    P.walk.clear();
    P.packs.clear();
    P.pack_row_start.clear();
    P.desc_bytes = P.bnd_elems = P.tb_bytes = P.total_rows = 0;
    P.pack_rows = P.nprog = 0;
    std::vector<std::pair<int64_t, int32_t>>& bysize = P.bysize;
    bysize.clear();
    bysize.reserve(cnt);
    const Overrides ov;
    const BoundInfo bound(p);
    const bool allow16 = (p->flags & MPG_ALLOW_I16) != 0 && !cfg.pro;
    const int K16 = choose_K16(ov, cfg.tune, cfg.force_K16);
    const KChoice kc = choose_widths(ov, cfg.tune, cfg.force_K);
    std::vector<std::pair<int64_t, int32_t>>& e16 = P.e16;
    e16.clear();
    // One group per (width, traceback, kernel mode), in order of first
    // appearance in the queue order, its items counted first and then written
    // in place.  The two fixed-end modes share a kernel (EXTEND_LEFT's start term is read
    // per pair); with per-pair modes every mode but LOCAL runs in the mixed
    // kernel, so a chain's three piece kinds fill one group per width.
    const bool per_pair = cfg.modes != nullptr && !cfg.pro;
    auto gmode = [&](int mode) {
        if (per_pair && mode != MPG_LOCAL) return kModeMixed;
        return mode == MPG_EXTEND_LEFT ? (int)MPG_GLOBAL : mode;
    };
    auto gkey = [&](const PairJob& J) {
        const int gm = gmode(J.mode) == kModeMixed ? 3 : gmode(J.mode);  // 0, 1, 2 or 3
        return ((J.K == 1 ? 0 : J.K == 2 ? 1 : 2) * 2 + (J.tb ? 1 : 0)) * 4 + gm;
    };
    // per job: group key << 24 | traceback << 23 | strips (a compact copy for
    // the passes in queue order, which visit the jobs out of order)
    P.ginfo.resize(cnt);
    P.seg_key.assign(cnt, -1);
    // lanes the last strip of a pair needs
    auto last_lanes = [](const PairJob& J) {
        if (J.nstrips == 1) return J.m / J.K + 1;
        return (J.m + 1 - (J.nstrips - 1) * 64 * J.K + J.K - 1) / J.K;
    };
    const bool seg_pref = !(cfg.tune && cfg.tune->seg == 0);
    const bool seg_on = seg_pref && !ov.no_seg && !cfg.pro && cnt < (1 << 24);
    // pairs this narrow run one column per lane: a single strip of at most 64
    // lanes by default; the autotuner may move the cutover
    const int narrow = cfg.tune && cfg.tune->narrow > 0 ? cfg.tune->narrow : 64;
    for (int32_t k = 0; k < cnt; ++k) {
        const mpg_seg& s = segs[idx[k]];
        PairJob& J = P.jobs[k];
        J.n = s.dlen;
        J.m = s.plen;
        J.res = idx[k];
        J.tb = ((s.flags | p->flags) & MPG_WANT_TB) ? 1 : 0;
        J.dna_off = s.dna_off;
        J.prot_off = s.prot_off;
        J.status = MPG_OK;
        J.mode = cfg.modes ? cfg.modes[idx[k]] : p->mode;
        J._pad = 0;
        const BoundInfo bk = cfg.pro ? bound.profile(cfg.pro_bounds[2 * idx[k]],
                                                     cfg.pro_bounds[2 * idx[k] + 1])
                                     : bound;
        if (s.dlen < 0 || s.plen < 0 || s.dlen > MPG_MAX_DNA || s.plen > MPG_MAX_PROT ||
            !bk.ok(s.dlen, s.plen, J.mode))
            J.status = MPG_E_RANGE;
        const bool want_tb = ((s.flags | p->flags) & MPG_WANT_TB) != 0;
        const int nn = std::max(0, J.n), mm = std::max(0, J.m);
        // a pair whose columns fit one strip of 64 takes one column per lane:
        // wider lanes would only add idle columns to every step
        int K = (mm + 1 <= narrow && !ov.K && !cfg.force_K) ? 1 : kc.K[want_tb ? 1 : 0];
        if (cfg.pro && K > 2) K = 2;  // profile kernels come in widths 1 and 2
        J.K = K;
        const int nsteps = pair_nsteps(nn, mm, K);
        J.nchunks = nsteps / 64;
        J.nstrips = (mm + 1 + 64 * K - 1) / (64 * K);
        if (J.tb && J.status == MPG_OK && (uint64_t)tb_bytes_of(nn, mm, K) > tb_budget)
            J.status = MPG_E_RANGE;
        J.ops_off = ops_off[idx[k]];
        J.i16 = 0;
        if (J.status != MPG_OK) continue;
        if (allow16 && !J.tb && bound.ok16(mm, J.mode)) {
            J.i16 = 1;
            J.K = K16;
            J.nstrips = (mm + 1 + 64 * K16 - 1) / (64 * K16);
            J.nchunks = pair_nsteps(nn, mm, K16) / 64;
            // pairs are matched by shape: strips first, then chunks
            e16.push_back({(int64_t)J.nstrips * (1LL << 32) + J.nchunks, k});
            continue;
        }
        J.desc_off = P.desc_bytes;
        const int64_t rows = (int64_t)nsteps + kDescLo + kDescHi;
        P.row_start[k] = P.total_rows;
        P.total_rows += rows;
        P.desc_bytes += rows * 16;
        J.bnd_off = P.bnd_elems;
        P.bnd_elems += (int64_t)nsteps + kBndLo + kBndHi;
        J.tb_off = P.tb_bytes;
        if (J.tb) P.tb_bytes += tb_bytes_of(nn, mm, K);
        J.prog_off = (int32_t)P.nprog;
        P.nprog += J.nstrips;
        P.ginfo[k] = (uint32_t)gkey(J) << 24 | (uint32_t)(J.tb ? 1 : 0) << 23 | (uint32_t)J.nstrips;
        // lane-segment class (traceback, width, chunks), then lanes
        // descending; a pair has fewer than 2^15 chunks (genome rows are
        // below 2^21).  Traced pairs only in batch calls (serving walks each
        // pair in the wavefront that finishes it).
        P.seg_key[k] = -1;
        if (seg_on && J.status == MPG_OK && (!J.tb || !cfg.serve) &&
            gmode(J.mode) == MPG_LOCAL) {
            const int u = last_lanes(J);
            if (u >= 1 && u <= 63)
                P.seg_key[k] = (J.tb << 23) | ((K == 1 ? 0 : K == 2 ? 1 : 2) << 21) |
                               (J.nchunks << 6) | (63 - u);
        }
        bysize.push_back({(int64_t)J.nstrips * J.nchunks, k});
    }
    // batches: longest pair first (the last pairs to finish are the short
    // ones); serving: shortest first (short results are out early)
    sort_by_key(bysize, !shortest_first, P.sort_tmp, P.sort_cnt);
    int gidx[24];
    int64_t gcount[24] = {0};
    std::fill(gidx, gidx + 24, -1);
    int64_t nwalk = 0;
    for (auto& e : bysize) {
        const uint32_t gi = P.ginfo[e.second];
        const int key = (int)(gi >> 24);
        if (gidx[key] < 0) {
            const PairJob& J = P.jobs[e.second];
            gidx[key] = (int)P.groups.size();
            P.groups.push_back(Group{J.K, J.tb != 0, false, gmode(J.mode), 0, 0});
        }
        gcount[gidx[key]] += gi & 0x7FFFFF;
        nwalk += (gi >> 23) & 1;
    }
    // Lane-segment packs.  A pair's last strip fills only the lanes its
    // remaining columns need and idles the rest for all its steps.  Two
    // LOCAL pairs of one width and kind (score-only or traced) whose strips
    // run the same number of chunks and whose last strips need at most 64
    // lanes together share one wavefront: the pair with more lanes first, the other from lane `split`.
    // Within each (width, chunks) class the widest remaining last strip is
    // matched with the narrowest that fits.  The pack's item goes where the
    // later pair's last strip would be, so it follows both pairs' other
    // strips in the queue and its waits point to items taken earlier.
    P.seg_mate.assign(cnt, -1);
    P.seg_emit.assign(cnt, 0);
    if (seg_on) {
        std::vector<std::pair<int64_t, int32_t>>& cand = P.seg_cand;
        cand.clear();
        for (size_t q = 0; q < bysize.size(); ++q) {
            const int32_t key = P.seg_key[bysize[q].second];
            if (key >= 0) cand.push_back({key, (int32_t)q});
        }
        sort_by_key(cand, false, P.sort_tmp, P.sort_cnt);
        for (size_t r0 = 0; r0 < cand.size();) {
            size_t r1 = r0;
            while (r1 < cand.size() && (cand[r1].first >> 6) == (cand[r0].first >> 6)) ++r1;
            size_t lo = r0, hi = r1;  // [lo, hi): widest first
            while (hi - lo >= 2) {
                const int ua = 63 - (int)(cand[lo].first & 63);
                const int ub = 63 - (int)(cand[hi - 1].first & 63);
                if (ua + ub <= 64) {
                    const int32_t qa = cand[lo].second, qb = cand[hi - 1].second;
                    const int32_t a = bysize[qa].second, b = bysize[qb].second;
                    P.seg_mate[a] = b;
                    P.seg_mate[b] = a;
                    P.seg_emit[qa > qb ? a : b] = 1;
                    --gcount[gidx[P.ginfo[a] >> 24]];
                    --hi;
                }
                ++lo;
            }
            r0 = r1;
        }
    }
    size_t total = 0;
    for (size_t g = 0; g < P.groups.size(); ++g) {
        P.groups[g].off = total;
        total += (size_t)gcount[g];
    }
    P.items.resize(total);
    P.walk.reserve(nwalk);
    for (auto& e : bysize) {
        const uint32_t gi = P.ginfo[e.second];
        Group& g = P.groups[gidx[gi >> 24]];
        const int ns = (int)(gi & 0x7FFFFF);
        const int32_t mate = P.seg_mate[e.second];
        for (int st = 0; st < ns; ++st) {
            if (st == ns - 1 && mate >= 0) {
                if (!P.seg_emit[e.second]) continue;
                // the pair with more lanes in [0, split)
                int32_t a = e.second, b = mate;
                const int ua = 63 - (P.seg_key[a] & 63), ub = 63 - (P.seg_key[b] & 63);
                if (ua < ub) std::swap(a, b);
                P.items[g.off + g.cnt++] = make_int2(a, -1 - ((b << 6) | (ua < ub ? ub : ua)));
                continue;
            }
            P.items[g.off + g.cnt++] = make_int2(e.second, st);
        }
        if ((gi >> 23) & 1) P.walk.push_back(e.second);
    }
    // int16 pairs: neighbours in size order share a pack
    if (!e16.empty()) {
        sort_by_key(e16, true, P.sort_tmp, P.sort_cnt);
        P.groups.push_back(Group{K16, false, true, MPG_LOCAL, P.items.size(), 0});
        for (size_t q = 0; q < e16.size(); q += 2) {
            const PairJob& A = P.jobs[e16[q].second];
            const bool hasB = q + 1 < e16.size();
            const PairJob& B = P.jobs[hasB ? e16[q + 1].second : e16[q].second];
            PackJob X{};
            X.a = e16[q].second;
            X.b = hasB ? e16[q + 1].second : -1;
            X.n = std::max(A.n, hasB ? B.n : 0);
            X.nchunks = std::max(A.nchunks, hasB ? B.nchunks : 0);
            X.nstrips = std::max(A.nstrips, hasB ? B.nstrips : 0);
            X.K = K16;
            const int64_t nsteps = (int64_t)X.nchunks * 64;
            X.desc_off = P.desc_bytes;
            P.pack_row_start.push_back(P.pack_rows);
            P.pack_rows += nsteps + kDescLo + kDescHi;
            P.desc_bytes += (nsteps + kDescLo + kDescHi) * 16;
            X.bnd_off = P.bnd_elems;
            P.bnd_elems += nsteps + kBndLo + kBndHi;
            X.prog_off = (int32_t)P.nprog;
            P.nprog += X.nstrips;
            P.packs.push_back(X);
        }
        // queue order: longest pack first
        std::vector<int32_t> ord(P.packs.size());
        for (size_t q = 0; q < ord.size(); ++q) ord[q] = (int32_t)q;
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
            return (int64_t)P.packs[a].nstrips * P.packs[a].nchunks >
                   (int64_t)P.packs[b].nstrips * P.packs[b].nchunks;
        });
        Group& g = P.groups.back();
        for (int32_t xi : ord)
            for (int st = 0; st < P.packs[xi].nstrips; ++st) {
                P.items.push_back(make_int2(xi, st));
                ++g.cnt;
            }
    }
}

}  // namespace

// ------------------------------------------------------------------ context
struct mpg_ctx {
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    uint64_t tb_budget = 64ull << 30;
    // device memory of every workspace of the context (mpg_set_allocator)
    DevAlloc alloc;
    Workspace ws;
    // allocation-free entry point: the device's fixed scratch array (its
    // address taken at creation) and the host storage its calls reuse
    uint8_t* scratch = nullptr;
    int scratch_rc = MPG_E_DEVICE;
    struct NoAllocHost {
        Plan plan;
        std::vector<uint8_t> stage;
        std::vector<int64_t> ops_off;
        std::vector<int32_t> idx;
    } noalloc;
    // anchor-driven calls in sub-batches: two workspaces, each with the event
    // that marks the end of its last use
    Workspace chain_ws[2];
    hipEvent_t chain_ev[2] = {nullptr, nullptr};
    std::mutex batch_mu;
    // optional kernel timing (hipEvents on the batch stream)
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pre, ev_dp, ev_walk;
    std::vector<hipEvent_t> ev_pool;
    double t_pre = 0, t_dp = 0, t_walk = 0, t_host = 0;
    uint64_t n_dp = 0, n_calls = 0, n_i16 = 0, n_cells = 0, n_seg = 0;

    // ---- serving
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool params_set = false;
    mpg_params sparams;
    struct Job {
        uint64_t id;
        std::string prot, dna;
        uint32_t flags;
        int64_t t_arrive;
        int64_t tb_bytes;
        int64_t cells;
    };
    // pending jobs by class: 2*long + traceback (long = more than kLongCells)
    static constexpr int64_t kLongCells = 200000000LL;
    std::deque<Job> pending[4];
    size_t npending = 0;
    std::deque<mpg_result> done;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread sched;
    bool sched_running = false;
    size_t max_pending = 1 << 20;
    // slots 0..nshort-1 run short micro-batches, the rest long batches
    int nshort = 3, nlong = 4;
    int64_t short_cells = 2000000000LL;   // cells per short batch
    int64_t long_cells = 60000000000LL;   // cells per long batch
    double long_share = 1.0;              // device share of one long batch's grid
    // serving strip widths: the narrowest strips give the shortest critical
    // path per pair and, with long pairs split into more strips, the best
    // overlap of long pairs in flight
    int serve_K_short = 1, serve_K_long = 1;
    int max_jobs_per_batch = 4096;
    mpg_stats stats{};
    uint64_t tb_in_use = 0;
    Tuning tune;  // measured kernel costs (mpg_autotune)
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? MPG_OK : MPG_E_DEVICE; }

// Records hipEvent pairs around the prepass (0), DP (1) and walk (2) launches
// of a batch; resolved lazily by mpg_get_timing.
struct Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>>* ev[3];
    std::vector<hipEvent_t>* pool;
    double* host_ms;  // wall time spent planning and enqueuing on the host
    uint64_t* i16 = nullptr;  // pairs run in the int16 kernel
    uint64_t* cells = nullptr;  // DP cells (n*m) of the pairs run
    uint64_t* segs = nullptr;   // lane-segment packs run
    hipEvent_t open[3] = {nullptr, nullptr, nullptr};
    hipEvent_t get() {
        hipEvent_t e = nullptr;
        if (!pool->empty()) {
            e = pool->back();
            pool->pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
    void begin(hipStream_t st, int k) {
        open[k] = get();
        if (open[k]) hipEventRecord(open[k], st);
    }
    void end(hipStream_t st, int k) {
        if (!open[k]) return;
        hipEvent_t e = get();
        if (!e) return;
        hipEventRecord(e, st);
        ev[k]->push_back({open[k], e});
        open[k] = nullptr;
    }
};


// A planned call: the plan, its device copies and where everything lives.
struct Prepared {
    Plan P;
    DevParams DP;
    int32_t cnt = 0;
    size_t npjobs = 0, npacks = 0;
    std::vector<size_t> goff;  // first item of each group
    PairJob *d_jobs = nullptr, *d_pjobs = nullptr;
    PackJob* d_packs = nullptr;
    int64_t *d_starts = nullptr, *d_pkstarts = nullptr;
    int2* d_items = nullptr;
    int32_t* d_walk = nullptr;
    void* d_pst = nullptr;
    int *d_qhead = nullptr, *d_prog = nullptr;
    uint8_t *d_desc = nullptr, *d_tb = nullptr;
    int2* d_bnd = nullptr;
    const uint8_t *d_prot = nullptr, *d_dna = nullptr;
    mpg_dev_result* d_out = nullptr;
    char* d_ops = nullptr;
};

// The fixed scratch array of the allocation-free entry point, and the
// context's pageable host storage the plan is staged in for it.
struct FixedScratch {
    uint8_t* dev = nullptr;
    size_t cap = 0;
    std::vector<uint8_t>* stage = nullptr;
};

// Host part of a call: plan the pairs idx[0..cnt), size the workspace and
// upload the plan (asynchronously on st).  Waits for earlier work on st,
// since the staging buffer and workspace may still be in use.  With `fx` the
// device buffers are carved out of the fixed scratch array instead of the
// workspace's (MPG_E_RANGE if they do not fit) and the plan is staged in
// fx's host storage: nothing is allocated on the device or pinned.
int prepare(hipStream_t st, Workspace& ws, const mpg_params* p, const uint8_t* d_prot,
            const uint8_t* d_dna, const mpg_seg* segs, const int32_t* idx, int32_t cnt,
            const std::vector<int64_t>& ops_off, mpg_dev_result* d_out, char* d_ops,
            const RunCfg& cfg, Prepared& X, const FixedScratch* fx = nullptr) {
    Timer* tm = cfg.tm;
    const auto th0 = std::chrono::steady_clock::now();
    struct HostClock {
        Timer* tm;
        std::chrono::steady_clock::time_point t0;
        ~HostClock() {
            if (tm && tm->host_ms)
                *tm->host_ms += std::chrono::duration<double, std::milli>(
                                    std::chrono::steady_clock::now() - t0)
                                    .count();
        }
    } host_clock{tm, th0};
    Plan& P = X.P;
    plan_pairs(p, segs, idx, cnt, ops_off, P, cfg);
    make_dev_params(p, &X.DP);
    X.cnt = cnt;
    X.d_prot = d_prot;
    X.d_dna = d_dna;
    X.d_out = d_out;
    X.d_ops = d_ops;
    // prepass list: planned pairs only, row_start ascending; when every pair
    // is planned in int32 lanes, the job list itself
    bool all_int32 = true;
    for (int32_t k = 0; k < cnt && all_int32; ++k)
        all_int32 = P.jobs[k].status == MPG_OK && !P.jobs[k].i16;
    std::vector<PairJob> pjobs;
    std::vector<int64_t> pstarts;
    if (!all_int32) {
        pjobs.reserve(cnt);
        pstarts.reserve(cnt);
        for (int32_t k = 0; k < cnt; ++k)
            if (P.jobs[k].status == MPG_OK && !P.jobs[k].i16) {
                pjobs.push_back(P.jobs[k]);
                pstarts.push_back(P.row_start[k]);
            }
    }
    X.npjobs = all_int32 ? (size_t)cnt : pjobs.size();
    const size_t npacks = P.packs.size();
    X.npacks = npacks;
    if (tm && tm->i16)
        for (const PackJob& Q : P.packs) *tm->i16 += Q.b >= 0 ? 2 : 1;
    if (tm && tm->segs)
        for (const int2& it : P.items) *tm->segs += it.y < 0 ? 1 : 0;
    if (tm && tm->cells)
        for (const PairJob& J : P.jobs)
            if (J.status == MPG_OK) *tm->cells += (uint64_t)J.n * (uint64_t)J.m;
    // work items of every launch, then the walk order (local job indices)
    const std::vector<int2>& items = P.items;
    X.goff.clear();
    for (auto& g : P.groups) X.goff.push_back(g.off);
    if (P.groups.size() > 15) return MPG_E_INVAL;

    const size_t jobs_b = sizeof(PairJob) * (size_t)cnt;
    const size_t pj_b = sizeof(PairJob) * pjobs.size();
    const size_t ps_b = sizeof(int64_t) * X.npjobs;
    const size_t it_b = sizeof(int2) * items.size();
    const size_t wk_b = sizeof(int32_t) * P.walk.size();
    const size_t pk_b = sizeof(PackJob) * npacks;
    const size_t pks_b = sizeof(int64_t) * npacks;
    int rc;
    // the wait is device time, not host time
    const auto tw0 = std::chrono::steady_clock::now();
    if ((rc = wait_workspace(st, cfg)) != MPG_OK) return rc;
    host_clock.t0 += std::chrono::steady_clock::now() - tw0;
    const size_t b_jobs = jobs_b + pj_b + pk_b + 256, b_rs = ps_b + pks_b + 64,
                 b_order = it_b + wk_b + 64, b_desc = (size_t)P.desc_bytes + 64,
                 b_bnd = sizeof(int2) * (size_t)P.bnd_elems + 64,
                 b_tb = (size_t)P.tb_bytes + 64,
                 b_state = (size_t)kPairStateBytes * cnt + sizeof(int) * (P.nprog + 64);
    // staging layout: jobs, prepass jobs, packs | row starts, pack row
    // starts | items, walk list
    const size_t plan_b = jobs_b + pj_b + pk_b + ps_b + pks_b + it_b + wk_b + 1024;
    uint8_t *p_jobs, *p_rs, *p_order, *p_desc, *p_bnd, *p_tb, *p_state;
    uint8_t* h;
    if (fx) {
        size_t off = 0;
        auto carve = [&](size_t bytes) {
            uint8_t* q = fx->dev + off;
            off += (bytes + 255) & ~(size_t)255;
            return q;
        };
        p_jobs = carve(b_jobs);
        p_rs = carve(b_rs);
        p_order = carve(b_order);
        p_desc = carve(b_desc);
        p_bnd = carve(b_bnd);
        p_tb = carve(b_tb);
        p_state = carve(b_state);
        if (off > fx->cap) return MPG_E_RANGE;
        if (fx->stage->size() < plan_b) fx->stage->resize(plan_b);
        h = fx->stage->data();
    } else {
        if ((rc = ws.jobs.ensure(b_jobs)) != MPG_OK) return rc;
        if ((rc = ws.row_start.ensure(b_rs)) != MPG_OK) return rc;
        if ((rc = ws.order.ensure(b_order)) != MPG_OK) return rc;
        if ((rc = ws.desc.ensure(b_desc)) != MPG_OK) return rc;
        if ((rc = ws.bnd.ensure(b_bnd)) != MPG_OK) return rc;
        if ((rc = ws.tb.ensure(b_tb)) != MPG_OK) return rc;
        if ((rc = ws.state.ensure(b_state)) != MPG_OK) return rc;
        if ((rc = ws.hplan.ensure(plan_b)) != MPG_OK) return rc;
        p_jobs = (uint8_t*)ws.jobs.p;
        p_rs = (uint8_t*)ws.row_start.p;
        p_order = (uint8_t*)ws.order.p;
        p_desc = (uint8_t*)ws.desc.p;
        p_bnd = (uint8_t*)ws.bnd.p;
        p_tb = (uint8_t*)ws.tb.p;
        p_state = (uint8_t*)ws.state.p;
        h = (uint8_t*)ws.hplan.p;
    }
    std::memcpy(h, P.jobs.data(), jobs_b);
    if (pj_b) std::memcpy(h + jobs_b, pjobs.data(), pj_b);
    std::memcpy(h + jobs_b + pj_b, P.packs.data(), pk_b);
    uint8_t* h2 = h + jobs_b + pj_b + pk_b;
    std::memcpy(h2, all_int32 ? P.row_start.data() : pstarts.data(), ps_b);
    std::memcpy(h2 + ps_b, P.pack_row_start.data(), pks_b);
    uint8_t* h3 = h2 + ps_b + pks_b;
    std::memcpy(h3, items.data(), it_b);
    std::memcpy(h3 + it_b, P.walk.data(), wk_b);
    X.d_jobs = (PairJob*)p_jobs;
    X.d_pjobs = all_int32 ? (PairJob*)p_jobs : (PairJob*)(p_jobs + jobs_b);
    X.d_packs = (PackJob*)(p_jobs + jobs_b + pj_b);
    X.d_starts = (int64_t*)p_rs;
    X.d_pkstarts = (int64_t*)(p_rs + ps_b);
    X.d_items = (int2*)p_order;
    X.d_walk = (int32_t*)(p_order + it_b);
    X.d_desc = p_desc;
    X.d_bnd = (int2*)p_bnd;
    X.d_tb = p_tb;
    X.d_pst = p_state;
    X.d_qhead = (int*)(p_state + (size_t)kPairStateBytes * cnt);  // one per launch
    X.d_prog = X.d_qhead + 16;
    hipError_t e = hipSuccess;
    if (jobs_b + pj_b + pk_b)
        e = hipMemcpyAsync(p_jobs, h, jobs_b + pj_b + pk_b, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && ps_b + pks_b)
        e = hipMemcpyAsync(X.d_starts, h2, ps_b + pks_b, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && it_b + wk_b)
        e = hipMemcpyAsync(p_order, h3, it_b + wk_b, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return MPG_E_DEVICE;
    return MPG_OK;
}

// Device part of a call: only kernel launches (and, with `fork`, event
// record/wait to run the kernel variants concurrently on side streams), no
// host synchronisation, allocation or memset, so it may be captured into a
// graph (with fork = false).
int enqueue(hipStream_t st, Workspace& ws, const Prepared& X, const RunCfg& cfg, bool fork) {
    Timer* tm = cfg.tm;
    const Plan& P = X.P;
    const DevParams& DP = X.DP;
    const size_t ngroups = P.groups.size();
    int rc;
    const DpSink sink{X.d_out, X.d_ops, cfg.serve ? 1 : 0, cfg.serve ? 1 : 0};
    if (launch_status(st, X.d_jobs, X.cnt, sink) != hipSuccess) return MPG_E_DEVICE;
    const int neg_init = -(1 << 30);
    if (launch_init(st, X.d_jobs, X.cnt, X.d_pst, X.d_prog, X.d_qhead, 16, neg_init) !=
        hipSuccess)
        return MPG_E_DEVICE;
    if (tm) tm->begin(st, 0);
    if (launch_prepass(st, X.d_pjobs, X.d_starts, (int)X.npjobs, P.total_rows, X.d_dna,
                       X.d_desc, DP) != hipSuccess)
        return MPG_E_DEVICE;
    if (X.npacks &&
        launch_prepass16(st, X.d_jobs, X.d_packs, X.d_pkstarts, (int)X.npacks, P.pack_rows,
                         X.d_dna, X.d_desc, X.d_prog, DP) != hipSuccess)
        return MPG_E_DEVICE;
    if (tm) tm->end(st, 0);
    if (tm) tm->begin(st, 1);
    auto launch_group = [&](hipStream_t s2, size_t g) -> hipError_t {
        const Group& G = P.groups[g];
        const int nit = (int)G.cnt;
        DevParams DG = DP;
        DG.mode = G.mode;
        if (G.i16)
            return launch_dp16(s2, G.K, cfg.ncu, DG, X.d_jobs, X.d_packs, X.d_items + X.goff[g],
                               nit, X.d_qhead + g, X.d_pst, X.d_prog, X.d_prot,
                               X.d_desc, X.d_bnd, sink);
        return launch_dp(s2, G.K, G.tb, cfg.pro, cfg.ncu, DG, X.d_jobs, X.d_items + X.goff[g],
                         nit,
                         X.d_qhead + g, X.d_pst, X.d_prog, X.d_prot, X.d_desc, X.d_bnd,
                         X.d_tb, sink);
    };
    if (ngroups == 1 || (ngroups > 1 && !fork)) {
        for (size_t g = 0; g < ngroups; ++g)
            if (launch_group(st, g) != hipSuccess) return MPG_E_DEVICE;
    } else if (ngroups > 1) {
        // fork: every variant's launch starts after the prepass, concurrently;
        // the first runs on the batch stream itself (one hardware queue fewer
        // to share with the side streams)
        if ((rc = ws.ensure_streams()) != MPG_OK) return rc;
        if (hipEventRecord(ws.fork_ev, st) != hipSuccess) return MPG_E_DEVICE;
        const int ng = (int)std::min<size_t>(ngroups - 1, kSideStreams);
        for (int k = 0; k < ng; ++k)
            if (hipStreamWaitEvent(ws.side[k], ws.fork_ev, 0) != hipSuccess) return MPG_E_DEVICE;
        if (launch_group(st, 0) != hipSuccess) return MPG_E_DEVICE;
        for (size_t g = 1; g < ngroups; ++g)
            if (launch_group(ws.side[(g - 1) % kSideStreams], g) != hipSuccess)
                return MPG_E_DEVICE;
        // join
        for (int k = 0; k < ng; ++k) {
            if (hipEventRecord(ws.join_ev[k], ws.side[k]) != hipSuccess) return MPG_E_DEVICE;
            if (hipStreamWaitEvent(st, ws.join_ev[k], 0) != hipSuccess) return MPG_E_DEVICE;
        }
    }
    if (tm) tm->end(st, 1);
    if (!P.walk.empty() && !cfg.serve) {
        if (tm) tm->begin(st, 2);
        if (launch_walk(st, X.d_jobs, X.d_walk, (int)P.walk.size(), X.d_tb,
                        X.d_out, X.d_ops) != hipSuccess)
            return MPG_E_DEVICE;
        if (tm) tm->end(st, 2);
    }
    return MPG_OK;
}

// Enqueue the pairs idx[0..cnt) of a call whose letters are on the device.
int run_dev(hipStream_t st, Workspace& ws, const mpg_params* p, const uint8_t* d_prot,
            const uint8_t* d_dna, const mpg_seg* segs, const int32_t* idx, int32_t cnt,
            const std::vector<int64_t>& ops_off, mpg_dev_result* d_out, char* d_ops,
            const RunCfg& cfg) {
    Prepared X;
    // plan in the workspace's storage, handed back on every return
    struct Lend {
        Plan& a;
        Plan& b;
        Lend(Plan& x, Plan& y) : a(x), b(y) { std::swap(a, b); }
        ~Lend() { std::swap(a, b); }
    } lend(X.P, ws.plan_cache);
    int rc = prepare(st, ws, p, d_prot, d_dna, segs, idx, cnt, ops_off, d_out, d_ops, cfg, X);
    if (rc != MPG_OK) return rc;
    return enqueue(st, ws, X, cfg, true);
}

bool seg_tb(const mpg_seg& s, const mpg_params* p) {
    return ((s.flags | p->flags) & MPG_WANT_TB) != 0;
}

// Run all n pairs.  Traceback pairs whose direction bits together exceed the
// budget are split into waves that reuse the same buffer one after another on
// the stream; each wave writes straight into the caller's records and ops.
int run_dev_waves(hipStream_t st, Workspace& ws, const mpg_params* p, const uint8_t* d_prot,
                  const uint8_t* d_dna, const mpg_seg* segs, int32_t n, mpg_dev_result* d_out,
                  char* d_ops, const RunCfg& cfg_in) {
    RunCfg cfg = cfg_in;  // after the first wave, later waves wait for the stream
    const uint64_t tb_budget = cfg.tb_budget;
    std::vector<int64_t>& ops_off = ws.wave_ops_off;
    ops_off.resize(n);
    int64_t o = 0;
    for (int32_t k = 0; k < n; ++k) {
        ops_off[k] = o;
        o += seg_tb(segs[k], p) ? 2 * ((int64_t)std::max(0, segs[k].dlen) +
                                       std::max(0, segs[k].plen)) + 1
                                : 1;
    }
    std::vector<int32_t>& idx = ws.wave_idx;
    idx.clear();
    idx.reserve(n);
    int64_t acc = 0;
    // waves are sized with each pair's largest direction-bit need over the
    // widths (the width is chosen per wave and cannot make it larger)
    for (int32_t k = 0; k < n; ++k) {
        const mpg_seg& s = segs[k];
        const int64_t b = (seg_tb(s, p) && s.plen >= 0 && s.dlen >= 0)
                              ? tb_bytes_max(s.dlen, s.plen)
                              : 0;
        if (b <= (int64_t)tb_budget && acc + b > (int64_t)tb_budget && !idx.empty()) {
            int rc = run_dev(st, ws, p, d_prot, d_dna, segs, idx.data(), (int32_t)idx.size(),
                             ops_off, d_out, d_ops, cfg);
            if (rc != MPG_OK) return rc;
            cfg.ws_ready = nullptr;
            idx.clear();
            acc = 0;
        }
        idx.push_back(k);
        if (b <= (int64_t)tb_budget) acc += b;
    }
    if (idx.empty()) return MPG_OK;
    return run_dev(st, ws, p, d_prot, d_dna, segs, idx.data(), (int32_t)idx.size(), ops_off,
                   d_out, d_ops, cfg);
}

int params_check_impl(const mpg_params* p) {
    if (!p) return MPG_E_INVAL;
    if (p->q < 0 || p->e < 0 || p->f < 0 || p->r < 0 || p->q + p->e <= 0) return MPG_E_INVAL;
    if (p->mode < MPG_LOCAL || p->mode > MPG_EXTEND_LEFT) return MPG_E_INVAL;
    if (p->flags & ~(uint32_t)(MPG_NO_INTRON | MPG_NO_FRAMESHIFT | MPG_WANT_TB | MPG_ALLOW_I16))
        return MPG_E_INVAL;
    for (int k = 0; k < 64; ++k)
        if (p->gcode[k] >= 24) return MPG_E_INVAL;
    if (p->q > (1 << 20) || p->e > (1 << 20) || p->f > (1 << 20) || p->r > (1 << 20))
        return MPG_E_RANGE;
    return MPG_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* mpg_strerror(int status) {
    switch (status) {
        case MPG_OK: return "ok";
        case MPG_E_INVAL: return "invalid argument";
        case MPG_E_RANGE:
            return "out of range: a length, the score bound, the traceback budget, the ops buffer "
                   "or the fixed scratch size";
        case MPG_E_NOMEM: return "out of memory";
        case MPG_E_AGAIN: return "queue full, try again";
        case MPG_E_DEVICE: return "device error";
        case MPG_E_NOALN: return "no alignment reaches the end cell";
        case MPG_E_CANCELLED: return "cancelled";
        default: return "unknown status";
    }
}

void mpg_params_default(mpg_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->q = 11;
    p->e = 1;
    p->f = 23;
    p->r = 29;
    p->flags = 0;
    p->mode = MPG_LOCAL;
    std::memcpy(p->mat, kBlosum62, sizeof(p->mat));
    for (int k = 0; k < 64; ++k) {
        const char* hit = std::strchr(kAlphabet, kCodeACGT[k]);
        p->gcode[k] = (uint8_t)(hit - kAlphabet);
    }
    for (int b1 = 0; b1 < 5; ++b1)
        for (int b2 = 0; b2 < 5; ++b2)
            for (int b3 = 0; b3 < 5; ++b3) {
                p->donor[25 * b1 + 5 * b2 + b3] = (uint8_t)donor_pen(b1, b2, b3);
                p->acceptor[25 * b1 + 5 * b2 + b3] = (uint8_t)acceptor_pen(b1, b2, b3);
            }
}

int mpg_params_check(const mpg_params* p, int32_t max_plen, int32_t max_dlen) {
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    if (max_plen < 0 || max_dlen < 0) return MPG_E_INVAL;
    if (max_plen > MPG_MAX_PROT || max_dlen > MPG_MAX_DNA) return MPG_E_RANGE;
    if (!score_bound_ok(p, max_dlen, max_plen)) return MPG_E_RANGE;
    return MPG_OK;
}

int mpg_ctx_create(mpg_ctx** out, int device, uint64_t tb_budget_bytes, uint32_t flags) {
    if (!out) return MPG_E_INVAL;
    *out = nullptr;
    if (flags != 0) return MPG_E_INVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return MPG_E_DEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return MPG_E_DEVICE;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
            hipSuccess &&
        lds > 0)
        g_max_lds = lds;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        ncu > 0)
        g_num_cu = ncu;
    mpg_ctx* c = new (std::nothrow) mpg_ctx();
    if (!c) return MPG_E_NOMEM;
    c->device = device;
    if (tb_budget_bytes) c->tb_budget = tb_budget_bytes;
    // serving knobs (tuning only): lanes, micro-batch size, long-batch share
    if (const int v = env_int("MPG_SRV_NSHORT")) c->nshort = std::max(1, std::min(v, 4));
    if (const int v = env_int("MPG_SRV_NLONG")) c->nlong = std::max(1, std::min(v, 4));
    if (const int v = env_int("MPG_SRV_SHORT_MCELLS")) c->short_cells = (int64_t)v * 1000000;
    if (const int v = env_int("MPG_SRV_LONG_SHARE_PCT")) c->long_share = std::min(v, 100) / 100.0;
    if (const int v = env_int("MPG_SRV_MAX_JOBS")) c->max_jobs_per_batch = std::max(1, v);
    if (const int v = env_int("MPG_SRV_MAX_PENDING")) c->max_pending = (size_t)std::max(1, v);
    if (const int v = env_int("MPG_SRV_K_SHORT")) c->serve_K_short = (v == 1 || v == 2 || v == 4) ? v : 1;
    if (const int v = env_int("MPG_SRV_K_LONG")) c->serve_K_long = (v == 1 || v == 2 || v == 4) ? v : 2;
    // streams beyond the process's hardware queues share a queue and run
    // one after another: keep no more serving streams than queues (HIP's
    // default is 4), fewer long lanes first, at least one of each
    {
        const int hwq = env_int("GPU_MAX_HW_QUEUES") > 0 ? env_int("GPU_MAX_HW_QUEUES") : 4;
        if (c->nshort + c->nlong > hwq) c->nlong = std::max(1, hwq - c->nshort);
        if (c->nshort + c->nlong > hwq) c->nshort = std::max(1, hwq - c->nlong);
    }
    if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return MPG_E_DEVICE;
    }
    c->stream = c->own_stream;
    c->stats.tb_budget = c->tb_budget;
    c->stats.short_streams = (uint64_t)c->nshort;
    c->stats.long_streams = (uint64_t)c->nlong;
    c->ws.use_allocator(&c->alloc);
    for (auto& w : c->chain_ws) w.use_allocator(&c->alloc);
    // the fixed scratch array of the allocation-free entry point, with this
    // device current (its address is taken once per device and kept)
    c->scratch_rc = scratch_address(device, &c->scratch) == hipSuccess ? MPG_OK : MPG_E_DEVICE;
    *out = c;
    return MPG_OK;
}

int mpg_set_allocator(mpg_ctx* ctx, void* (*alloc)(size_t, void*),
                      void (*release)(void*, void*), void* user) {
    if (!ctx || (!alloc) != (!release)) return MPG_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    std::lock_guard<std::mutex> lk2(ctx->mu);
    // the serving threads read the allocator without a lock
    if (ctx->sched_running) return MPG_E_INVAL;
    ctx->alloc.alloc = alloc;
    ctx->alloc.release = release;
    ctx->alloc.user = alloc ? user : nullptr;
    return MPG_OK;
}

int mpg_set_stream(mpg_ctx* ctx, void* s) {
    if (!ctx) return MPG_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    ctx->stream = s ? (hipStream_t)s : ctx->own_stream;
    return MPG_OK;
}

int mpg_sync(mpg_ctx* ctx) {
    if (!ctx) return MPG_E_INVAL;
    hipSetDevice(ctx->device);
    return hip_status(hipStreamSynchronize(ctx->stream));
}

int64_t mpg_ops_capacity(const mpg_seg* segs, int32_t n) {
    if (!segs || n < 0) return -1;
    int64_t o = 0;
    for (int32_t k = 0; k < n; ++k) {
        const bool tb = (segs[k].flags & MPG_WANT_TB) != 0;
        o += tb ? 2 * ((int64_t)std::max(0, segs[k].dlen) + std::max(0, segs[k].plen)) + 1 : 1;
    }
    return o;
}

int mpg_align_batch_dev(mpg_ctx* ctx, const mpg_params* p, const uint8_t* d_prot,
                        const uint8_t* d_dna, const mpg_seg* segs, int32_t n,
                        mpg_dev_result* d_out, char* d_ops, int64_t ops_cap) {
    if (!ctx || !p || (n > 0 && (!segs || !d_out))) return MPG_E_INVAL;
    if (n < 0) return MPG_E_INVAL;
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    if (n == 0) return MPG_OK;
    // capacity needed with params.flags applied
    int64_t need = 0;
    for (int32_t k = 0; k < n; ++k) {
        const bool tb = ((segs[k].flags | p->flags) & MPG_WANT_TB) != 0;
        need += tb ? 2 * ((int64_t)std::max(0, segs[k].dlen) + std::max(0, segs[k].plen)) + 1 : 1;
    }
    if (need > 0 && (!d_ops || ops_cap < need)) return MPG_E_RANGE;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    Timer tm{{&ctx->ev_pre, &ctx->ev_dp, &ctx->ev_walk}, &ctx->ev_pool, &ctx->t_host, &ctx->n_i16,
             &ctx->n_cells, &ctx->n_seg};
    ctx->n_calls++;
    RunCfg cfg;
    cfg.tb_budget = ctx->tb_budget;
    cfg.tm = ctx->timing ? &tm : nullptr;
    cfg.ncu = g_num_cu;
    cfg.tune = &ctx->tune;
    return run_dev_waves(ctx->stream, ctx->ws, p, d_prot, d_dna, segs, n, d_out, d_ops, cfg);
}

int mpg_align_batch_dev_noalloc(mpg_ctx* ctx, const mpg_params* p, const uint8_t* d_prot,
                                const uint8_t* d_dna, const mpg_seg* segs, int32_t n,
                                mpg_dev_result* d_out, char* d_ops, int64_t ops_cap) {
    if (!ctx || !p || (n > 0 && (!segs || !d_out))) return MPG_E_INVAL;
    if (n < 0) return MPG_E_INVAL;
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    if (n == 0) return MPG_OK;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    if (ctx->scratch_rc != MPG_OK || !ctx->scratch) return MPG_E_DEVICE;
    mpg_ctx::NoAllocHost& na = ctx->noalloc;
    // op-string slots in input order, as mpg_align_batch_dev lays them out
    na.ops_off.resize(n);
    na.idx.resize(n);
    int64_t need = 0;
    for (int32_t k = 0; k < n; ++k) {
        na.ops_off[k] = need;
        na.idx[k] = k;
        need += seg_tb(segs[k], p) ? 2 * ((int64_t)std::max(0, segs[k].dlen) +
                                          std::max(0, segs[k].plen)) + 1
                                   : 1;
    }
    if (need > 0 && (!d_ops || ops_cap < need)) return MPG_E_RANGE;
    hipSetDevice(ctx->device);
    RunCfg cfg;
    cfg.tb_budget = ctx->tb_budget;
    cfg.ncu = g_num_cu;
    cfg.tune = &ctx->tune;
    Prepared X;
    std::swap(X.P, na.plan);  // plan in the context's storage, handed back below
    const FixedScratch fx{ctx->scratch, kScratchBytes, &na.stage};
    rc = prepare(ctx->stream, ctx->ws, p, d_prot, d_dna, segs, na.idx.data(), n, na.ops_off,
                 d_out, d_ops, cfg, X, &fx);
    // every kernel variant on the context's stream, one after another
    if (rc == MPG_OK) rc = enqueue(ctx->stream, ctx->ws, X, cfg, false);
    std::swap(X.P, na.plan);
    return rc;
}

}  // extern "C"

namespace {

// Copy the records (and op strings) of a finished call from ws.out / ws.ops
// into out[], duplicating each op string for the caller.
int download_results(hipStream_t st, Workspace& ws, const mpg_params* p, const mpg_seg* segs,
                     int32_t n, int64_t ops_cap, mpg_result* out) {
    int rc;
    if (hipMemcpyAsync(ws.hout.p, ws.out.p, sizeof(mpg_dev_result) * (size_t)n,
                       hipMemcpyDeviceToHost, st) != hipSuccess)
        return MPG_E_DEVICE;
    bool any_tb = false;
    for (int32_t k = 0; k < n; ++k) any_tb |= ((segs[k].flags | p->flags) & MPG_WANT_TB) != 0;
    if (any_tb) {
        if ((rc = ws.hops.ensure((size_t)ops_cap + 64)) != MPG_OK) return rc;
        if (hipMemcpyAsync(ws.hops.p, ws.ops.p, (size_t)ops_cap, hipMemcpyDeviceToHost, st) !=
            hipSuccess)
            return MPG_E_DEVICE;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return MPG_E_DEVICE;
    const mpg_dev_result* R = (const mpg_dev_result*)ws.hout.p;
    for (int32_t k = 0; k < n; ++k) {
        mpg_result& o = out[k];
        std::memset(&o, 0, sizeof(o));
        o.status = R[k].status;
        o.score = R[k].score;
        o.g_beg = R[k].g_beg;
        o.g_end = R[k].g_end;
        o.p_beg = R[k].p_beg;
        o.p_end = R[k].p_end;
        o.job_id = (uint64_t)k;
        o.ops = nullptr;
        o.ops_len = 0;
        if (((segs[k].flags | p->flags) & MPG_WANT_TB) && o.status == MPG_OK) {
            char* sdup = (char*)std::malloc((size_t)R[k].ops_len + 1);
            if (!sdup) return MPG_E_NOMEM;
            std::memcpy(sdup, (const char*)ws.hops.p + R[k].ops_off, (size_t)R[k].ops_len);
            sdup[R[k].ops_len] = 0;
            o.ops = sdup;
            o.ops_len = R[k].ops_len;
        }
    }
    return MPG_OK;
}

// Synchronous host-memory batch on a given stream/workspace; fills out[].
int align_host(hipStream_t st, Workspace& ws, const mpg_params* p, const mpg_pair* pairs,
               int32_t n, mpg_result* out, const RunCfg& cfg) {
    std::vector<mpg_seg> segs(n);
    int64_t pbytes = 0, dbytes = 0;
    for (int32_t k = 0; k < n; ++k) {
        if (pairs[k].plen < 0 || pairs[k].dlen < 0 || (pairs[k].plen && !pairs[k].prot) ||
            (pairs[k].dlen && !pairs[k].dna))
            return MPG_E_INVAL;
        segs[k].prot_off = pbytes;
        segs[k].plen = pairs[k].plen;
        segs[k].dna_off = dbytes;
        segs[k].dlen = pairs[k].dlen;
        segs[k].flags = pairs[k].flags | (p->flags & MPG_WANT_TB);
        segs[k]._pad = 0;
        pbytes += pairs[k].plen;
        dbytes += pairs[k].dlen;
    }
    const int64_t ops_cap = mpg_ops_capacity(segs.data(), n);
    int rc;
    if ((rc = ws.seq.ensure((size_t)(pbytes + dbytes) + 64)) != MPG_OK) return rc;
    if ((rc = ws.out.ensure(sizeof(mpg_dev_result) * (size_t)n + 64)) != MPG_OK) return rc;
    if ((rc = ws.ops.ensure((size_t)ops_cap + 64)) != MPG_OK) return rc;
    if ((rc = ws.hseq.ensure((size_t)(pbytes + dbytes) + 64)) != MPG_OK) return rc;
    if ((rc = ws.hout.ensure(sizeof(mpg_dev_result) * (size_t)n + 64)) != MPG_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return MPG_E_DEVICE;
    uint8_t* hs = (uint8_t*)ws.hseq.p;
    for (int32_t k = 0; k < n; ++k) {
        if (pairs[k].plen) std::memcpy(hs + segs[k].prot_off, pairs[k].prot, pairs[k].plen);
        if (pairs[k].dlen) std::memcpy(hs + pbytes + segs[k].dna_off, pairs[k].dna, pairs[k].dlen);
    }
    uint8_t* d_seq = (uint8_t*)ws.seq.p;
    if (pbytes + dbytes > 0 &&
        hipMemcpyAsync(d_seq, hs, (size_t)(pbytes + dbytes), hipMemcpyHostToDevice, st) !=
            hipSuccess)
        return MPG_E_DEVICE;
    rc = run_dev_waves(st, ws, p, d_seq, d_seq + pbytes, segs.data(), n,
                       (mpg_dev_result*)ws.out.p, (char*)ws.ops.p, cfg);
    if (rc != MPG_OK) return rc;
    return download_results(st, ws, p, segs.data(), n, ops_cap, out);
}

// ------------------------------------------------------------------ serving
// One serving batch: stage the sequences, launch with per-pair publication
// into host-mapped records, and deliver every result as soon as its pair's
// record is published.  Returns once all pairs are delivered (or the stream
// failed; then the rest complete with MPG_E_DEVICE).
template <typename Deliver>
int serve_batch(hipStream_t st, Workspace& ws, const mpg_params* p, const mpg_pair* pairs,
                int32_t n, uint64_t tb_budget, int ncu, const Tuning* tune, int force_K,
                Deliver deliver) {
    std::vector<mpg_seg> segs(n);
    int64_t pbytes = 0, dbytes = 0;
    for (int32_t k = 0; k < n; ++k) {
        segs[k].prot_off = pbytes;
        segs[k].plen = pairs[k].plen;
        segs[k].dna_off = dbytes;
        segs[k].dlen = pairs[k].dlen;
        segs[k].flags = pairs[k].flags | (p->flags & MPG_WANT_TB);
        segs[k]._pad = 0;
        pbytes += pairs[k].plen;
        dbytes += pairs[k].dlen;
    }
    const int64_t ops_cap = mpg_ops_capacity(segs.data(), n);
    volatile mpg_dev_result* rec = nullptr;
    // stage, launch; a failure anywhere here completes every pair with it
    int rc = [&]() -> int {
        int r;
        ws.prec.flags = ws.pops.flags = hipHostMallocMapped | hipHostMallocCoherent;
        if ((r = ws.seq.ensure((size_t)(pbytes + dbytes) + 64)) != MPG_OK) return r;
        if ((r = ws.hseq.ensure((size_t)(pbytes + dbytes) + 64)) != MPG_OK) return r;
        if ((r = ws.prec.ensure(sizeof(mpg_dev_result) * (size_t)n + 64)) != MPG_OK) return r;
        if ((r = ws.pops.ensure((size_t)ops_cap + 64)) != MPG_OK) return r;
        if (hipStreamSynchronize(st) != hipSuccess) return MPG_E_DEVICE;
        uint8_t* hs = (uint8_t*)ws.hseq.p;
        for (int32_t k = 0; k < n; ++k) {
            if (pairs[k].plen) std::memcpy(hs + segs[k].prot_off, pairs[k].prot, pairs[k].plen);
            if (pairs[k].dlen)
                std::memcpy(hs + pbytes + segs[k].dna_off, pairs[k].dna, pairs[k].dlen);
        }
        rec = (volatile mpg_dev_result*)ws.prec.p;
        for (int32_t k = 0; k < n; ++k) rec[k].status = kPending;
        std::atomic_thread_fence(std::memory_order_seq_cst);
        uint8_t* d_seq = (uint8_t*)ws.seq.p;
        if (pbytes + dbytes > 0 &&
            hipMemcpyAsync(d_seq, hs, (size_t)(pbytes + dbytes), hipMemcpyHostToDevice, st) !=
                hipSuccess)
            return MPG_E_DEVICE;
        RunCfg cfg;
        cfg.tb_budget = tb_budget;
        cfg.ncu = ncu;
        cfg.serve = true;
        cfg.tune = tune;
        cfg.force_K = force_K;
        return run_dev_waves(st, ws, p, d_seq, d_seq + pbytes, segs.data(), n,
                             (mpg_dev_result*)ws.prec.p, (char*)ws.pops.p, cfg);
    }();
    std::vector<char> got(n, 0);
    int32_t left = n;
    auto harvest = [&]() {
        int32_t found = 0;
        for (int32_t k = 0; k < n; ++k) {
            if (got[k] || rec[k].status == kPending) continue;
            std::atomic_thread_fence(std::memory_order_acquire);
            mpg_dev_result R;
            R.status = rec[k].status;
            R.score = rec[k].score;
            R.g_beg = rec[k].g_beg;
            R.g_end = rec[k].g_end;
            R.p_beg = rec[k].p_beg;
            R.p_end = rec[k].p_end;
            R.ops_off = rec[k].ops_off;
            R.ops_len = rec[k].ops_len;
            const char* ops = (segs[k].flags & MPG_WANT_TB) && R.status == MPG_OK
                                  ? (const char*)ws.pops.p + R.ops_off
                                  : nullptr;
            deliver(k, R, ops);
            got[k] = 1;
            --left;
            ++found;
        }
        return found;
    };
    if (rc == MPG_OK) {
        // poll the records while the device works; the stream's state tells
        // when nothing more can arrive
        for (;;) {
            const int32_t f = harvest();
            if (!left) break;
            const hipError_t q = hipStreamQuery(st);
            if (q == hipSuccess) {
                harvest();
                break;
            }
            if (q != hipErrorNotReady) {
                rc = MPG_E_DEVICE;
                break;
            }
            if (!f) std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    // wait for whatever was enqueued before the records are given up
    if (hipStreamSynchronize(st) != hipSuccess && rc == MPG_OK) rc = MPG_E_DEVICE;
    if (left) {
        // set-up or the device failed, or a record was never published:
        // every pair not yet delivered completes with that status
        if (rc == MPG_OK) rc = MPG_E_DEVICE;
        for (int32_t k = 0; k < n; ++k) {
            if (got[k]) continue;
            mpg_dev_result R{};
            R.status = rc;
            R.g_beg = R.g_end = R.p_beg = R.p_end = -1;
            deliver(k, R, nullptr);
        }
    }
    return rc;
}

// One scheduler thread admits pending jobs into batches while a slot (stream
// + workspace) and traceback budget are free.  Jobs are queued by class
// (short/long x score-only/traceback); every batch holds one class, so it is
// a single DP launch.  Short jobs go to small micro-batches on the short
// slots; long jobs (whose serial strip pipeline runs for tens of ms) are
// gathered into batches of their own on the long slots, so short results
// never wait behind a long pair.  Batches on different slots overlap on the
// device, and jobs that arrive meanwhile join the next batch of their class.
void scheduler(mpg_ctx* c) {
    hipSetDevice(c->device);
    const int nsh = std::max(1, c->nshort);
    const int ns = nsh + std::max(1, c->nlong);
    std::vector<hipStream_t> streams(ns);
    std::vector<Workspace> wss(ns);
    std::vector<bool> busy(ns, false);
    std::vector<std::thread> workers(ns);
    Retired retired;
    for (int k = 0; k < ns; ++k) {
        hipStreamCreateWithFlags(&streams[k], hipStreamNonBlocking);
        wss[k].defer_frees(&retired);
        wss[k].use_allocator(&c->alloc);
    }
    std::unique_lock<std::mutex> lk(c->mu);
    for (;;) {
        bool any_busy = false;
        for (int k = 0; k < ns; ++k) any_busy |= busy[k];
        if (c->stop && c->npending == 0 && !any_busy) break;
        if (!any_busy) {
            // nothing on the device: outgrown buffers can go now
            lk.unlock();
            retired.flush();
            lk.lock();
        }
        int slot = -1, cls = -1;
        for (int k = 0; k < ns && cls < 0; ++k) {
            if (busy[k]) continue;
            const int lane = k < nsh ? 0 : 2;
            // the class of this lane whose oldest job arrived first
            int best = -1;
            for (int q = lane; q < lane + 2; ++q)
                if (!c->pending[q].empty() &&
                    (best < 0 || c->pending[q].front().t_arrive < c->pending[best].front().t_arrive))
                    best = q;
            if (best >= 0) {
                slot = k;
                cls = best;
            }
        }
        if (cls < 0) {
            c->cv_work.wait_for(lk, std::chrono::milliseconds(20));
            continue;
        }
        std::deque<mpg_ctx::Job>& Q = c->pending[cls];
        const int64_t cap_cells = cls >= 2 ? c->long_cells : c->short_cells;
        std::vector<mpg_ctx::Job> batch;
        int64_t cells = 0, tb = 0;
        while (!Q.empty() && (int)batch.size() < c->max_jobs_per_batch) {
            mpg_ctx::Job& j = Q.front();
            if (!batch.empty() && cells + j.cells > cap_cells) break;
            // long batches leave a reserve of the budget to short jobs
            const uint64_t limit = cls >= 2 ? c->tb_budget - c->tb_budget / 8 : c->tb_budget;
            if (c->tb_in_use + tb + (uint64_t)j.tb_bytes > limit) break;
            cells += j.cells;
            tb += j.tb_bytes;
            batch.push_back(std::move(j));
            Q.pop_front();
        }
        c->npending -= batch.size();
        if (batch.empty()) {
            // traceback budget exhausted: wait for a batch to finish
            c->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            continue;
        }
        busy[slot] = true;
        c->tb_in_use += (uint64_t)tb;
        c->stats.tb_bytes_in_use = c->tb_in_use;
        c->stats.tb_bytes_peak = std::max<uint64_t>(c->stats.tb_bytes_peak, c->tb_in_use);
        c->stats.in_flight += batch.size();
        c->stats.queue_depth = c->npending;
        c->stats.batches += 1;
        if (workers[slot].joinable()) workers[slot].join();
        mpg_params params = c->sparams;
        // a long batch's persistent grid is held to a share of the device, so
        // short micro-batches always find free wavefront slots
        const int ncu = cls >= 2 ? std::max(1, (int)(g_num_cu * c->long_share)) : g_num_cu;
        const int K = cls >= 2 ? c->serve_K_long : c->serve_K_short;
        workers[slot] = std::thread([c, slot, tb, ncu, K, params, &streams, &wss, &busy,
                                     b = std::move(batch)]() mutable {
            hipSetDevice(c->device);
            std::vector<mpg_pair> pairs(b.size());
            for (size_t k = 0; k < b.size(); ++k) {
                pairs[k].prot = b[k].prot.data();
                pairs[k].plen = (int32_t)b[k].prot.size();
                pairs[k].dna = b[k].dna.data();
                pairs[k].dlen = (int32_t)b[k].dna.size();
                pairs[k].flags = b[k].flags;
            }
            params.flags &= ~(uint32_t)MPG_WANT_TB;
            // every result goes to the poll queue the moment its pair is done
            auto deliver = [&](int32_t k, const mpg_dev_result& R, const char* ops) {
                mpg_result r;
                std::memset(&r, 0, sizeof(r));
                r.status = R.status;
                r.score = R.score;
                r.g_beg = R.g_beg;
                r.g_end = R.g_end;
                r.p_beg = R.p_beg;
                r.p_end = R.p_end;
                if (ops) {
                    char* d = (char*)std::malloc((size_t)R.ops_len + 1);
                    if (d) {
                        std::memcpy(d, ops, (size_t)R.ops_len);
                        d[R.ops_len] = 0;
                        r.ops = d;
                        r.ops_len = R.ops_len;
                    } else {
                        r.status = MPG_E_NOMEM;
                    }
                }
                r.job_id = b[k].id;
                r.t_arrive_ns = b[k].t_arrive;
                r.t_done_ns = now_ns();
                std::lock_guard<std::mutex> g(c->mu);
                c->done.push_back(r);
                c->stats.cells += (uint64_t)b[k].cells;
                c->stats.completed += 1;
                c->stats.in_flight -= 1;
                c->cv_done.notify_all();
            };
            serve_batch(streams[slot], wss[slot], &params, pairs.data(), (int32_t)pairs.size(),
                        (uint64_t)tb + 1, ncu, &c->tune, K, deliver);
            std::lock_guard<std::mutex> g(c->mu);
            c->tb_in_use -= (uint64_t)tb;
            c->stats.tb_bytes_in_use = c->tb_in_use;
            busy[slot] = false;
            c->cv_work.notify_all();
        });
    }
    lk.unlock();
    for (auto& w : workers)
        if (w.joinable()) w.join();
    retired.flush();
    for (auto& w : wss) {
        w.defer_frees(nullptr);
        w.release();
    }
    for (auto& s : streams) hipStreamDestroy(s);
}

}  // namespace

// Anchor runs of one chain (Methods, opening paragraph: the DP closes the
// gaps between the anchors of a chain and extends from its terminal ones).
// Anchors arrive in genome order; one on the current run's diagonal that
// overlaps or abuts it extends the run, one at or after the run's end in
// both sequences starts a new run, any other is dropped.  Returns false for
// an anchor outside the sequences.
constexpr int64_t kMaxChainDna = (int64_t)1 << 30;  // longest region of one chain

bool chain_runs(const mpg_chain_seg& ch, std::vector<int4>& runs) {
    runs.clear();
    const int64_t k = ch.k;
    for (int32_t a = 0; a < ch.nanchors; ++a) {
        const int64_t x = ch.anchors[2 * a], y = ch.anchors[2 * a + 1];
        if (x < 0 || y < 0 || x + 3 * k > ch.dlen || y + k > ch.plen) return false;
        if (!runs.empty()) {
            int4& R = runs.back();
            if (x - R.x == 3 * (y - R.y) && y >= R.y && y <= (int64_t)R.y + R.z) {
                R.z = (int)std::max<int64_t>(R.z, y + k - R.y);
                continue;
            }
            if (!(x >= (int64_t)R.x + 3 * R.z && y >= (int64_t)R.y + R.z)) continue;
        }
        runs.push_back(make_int4((int)x, (int)y, (int)k, 0));
    }
    return true;
}

bool chain_tb(const mpg_chain_seg& c, const mpg_params* p) {
    return ((c.flags | p->flags) & MPG_WANT_TB) != 0;
}

// A chain's fields, and every anchor inside the sequences (what chain_runs
// checks as it goes).
bool chain_valid(const mpg_chain_seg& ch) {
    if (ch.plen < 0 || ch.dlen < 0 || ch.prot_off < 0 || ch.dna_off < 0 || ch.k <= 0 ||
        ch.nanchors <= 0 || !ch.anchors)
        return false;
    const int64_t k = ch.k;
    for (int32_t a = 0; a < ch.nanchors; ++a) {
        const int64_t x = ch.anchors[2 * a], y = ch.anchors[2 * a + 1];
        if (x < 0 || y < 0 || x + 3 * k > ch.dlen || y + k > ch.plen) return false;
    }
    return true;
}

// Enqueue the alignment of n chains whose letters are on the device: plan
// the runs and pieces, run every piece in one batch (per-pair modes), then
// the stitch kernel writes chain c's record d_out[c] and op string (slot at
// ops_base plus the prefix sum of mpg_chain_ops_capacity).  Waits for the
// workspace (cfg.ws_ready, else earlier work on st) before reusing it.
int chains_dev(hipStream_t st, Workspace& ws, const mpg_params* p, const uint8_t* d_prot,
               const uint8_t* d_dna, const mpg_chain_seg* chains, int32_t n,
               mpg_dev_result* d_out, char* d_ops, int64_t ops_cap, RunCfg cfg,
               int64_t ops_base = 0) {
    std::vector<int4> cr;
    std::vector<int4>& runs = ws.cruns;
    std::vector<ChainJob>& cj = ws.cjobs;
    std::vector<mpg_seg>& psegs = ws.psegs;
    std::vector<int8_t>& modes = ws.pmodes;
    runs.clear();
    cj.resize(n);
    psegs.clear();
    modes.clear();
    int64_t cops = ops_base;
    for (int32_t c = 0; c < n; ++c) {
        const mpg_chain_seg& ch = chains[c];
        if (ch.plen < 0 || ch.dlen < 0 || ch.prot_off < 0 || ch.dna_off < 0 || ch.k <= 0 ||
            ch.nanchors <= 0 || !ch.anchors)
            return MPG_E_INVAL;
        if (!chain_runs(ch, cr)) return MPG_E_INVAL;
        const bool tb = chain_tb(ch, p);
        ChainJob& J = cj[c];
        J.piece0 = (int32_t)psegs.size();
        J.nruns = 0;
        J.run0 = (int32_t)runs.size();
        J.tb = tb ? 1 : 0;
        J.prot_off = ch.prot_off;
        J.dna_off = ch.dna_off;
        J.ops_off = cops;
        J.ops_cap = tb ? 2 * ((int64_t)ch.plen + ch.dlen) + 1 : 1;
        J.res = c;
        J.status = MPG_OK;
        cops += J.ops_cap;
        if (ch.plen > MPG_MAX_PROT || ch.dlen > kMaxChainDna) {
            J.status = MPG_E_RANGE;
            continue;
        }
        J.nruns = (int32_t)cr.size();
        auto piece = [&](int64_t p0, int64_t p1, int64_t d0, int64_t d1, int mode) {
            mpg_seg s;
            s.prot_off = ch.prot_off + p0;
            s.plen = (int32_t)(p1 - p0);
            s.dna_off = ch.dna_off + d0;
            s.dlen = (int32_t)(d1 - d0);
            s.flags = tb ? MPG_WANT_TB : 0;
            s._pad = 0;
            psegs.push_back(s);
            modes.push_back((int8_t)mode);
        };
        piece(0, cr[0].y, 0, cr[0].x, MPG_EXTEND_LEFT);
        for (size_t t = 0; t + 1 < cr.size(); ++t)
            piece(cr[t].y + cr[t].z, cr[t + 1].y, cr[t].x + 3 * (int64_t)cr[t].z, cr[t + 1].x,
                  MPG_GLOBAL);
        const int4& L = cr.back();
        piece(L.y + L.z, ch.plen, L.x + 3 * (int64_t)L.z, ch.dlen, MPG_EXTEND);
        runs.insert(runs.end(), cr.begin(), cr.end());
    }
    if (cops > ops_cap) return MPG_E_RANGE;
    const int32_t np = (int32_t)psegs.size();
    const int64_t pops_cap = mpg_ops_capacity(psegs.data(), np);
    const size_t cj_b = sizeof(ChainJob) * (size_t)n, run_b = sizeof(int4) * runs.size();
    int rc;
    if ((rc = wait_workspace(st, cfg)) != MPG_OK) return rc;
    if ((rc = ws.piece_out.ensure(sizeof(mpg_dev_result) * (size_t)np + 64)) != MPG_OK) return rc;
    if ((rc = ws.piece_ops.ensure((size_t)pops_cap + 64)) != MPG_OK) return rc;
    if ((rc = ws.chain.ensure(cj_b + run_b + 64)) != MPG_OK) return rc;
    if ((rc = ws.hchain.ensure(cj_b + run_b + 64)) != MPG_OK) return rc;
    std::memcpy(ws.hchain.p, cj.data(), cj_b);
    if (run_b) std::memcpy((uint8_t*)ws.hchain.p + cj_b, runs.data(), run_b);
    if (hipMemcpyAsync(ws.chain.p, ws.hchain.p, cj_b + run_b, hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return MPG_E_DEVICE;
    mpg_dev_result* d_pres = (mpg_dev_result*)ws.piece_out.p;
    char* d_pops = (char*)ws.piece_ops.p;
    cfg.modes = modes.data();
    if (np > 0) {
        rc = run_dev_waves(st, ws, p, d_prot, d_dna, psegs.data(), np, d_pres, d_pops, cfg);
        if (rc != MPG_OK) return rc;
    }
    DevParams DP;
    make_dev_params(p, &DP);
    const ChainJob* d_cj = (const ChainJob*)ws.chain.p;
    const int4* d_runs = (const int4*)((const uint8_t*)ws.chain.p + cj_b);
    if (launch_stitch(st, d_cj, n, d_runs, d_pres, d_pops, d_prot, d_dna, DP, d_out, d_ops) !=
        hipSuccess)
        return MPG_E_DEVICE;
    return MPG_OK;
}

// Largest score (at least 0) and largest gap cost or negated score of a
// position-specific query; false if a cost is outside [0, 8191] or an open +
// extend pair is 0 (costs enter the traceback layout as 16 * cost - nibble).
bool profile_bounds(const int8_t* S, const int16_t* gap, int32_t m, int32_t* smax,
                    int32_t* gmax) {
    int32_t hi = 0, g = 0;
    for (int64_t k = 0; k < 24 * (int64_t)m; ++k) {
        hi = std::max<int32_t>(hi, S[k]);
        g = std::max<int32_t>(g, -S[k]);
    }
    for (int64_t j = 0; j <= m; ++j) {
        const int16_t* c = gap + 4 * j;
        for (int t = 0; t < 4; ++t)
            if (c[t] < 0 || c[t] > 8191) return false;
        if (c[2] + c[3] < 1 || (j >= 1 && c[0] + c[1] < 1)) return false;
        g = std::max<int32_t>(g, std::max(c[0] + c[1], c[2] + c[3]));
    }
    *smax = hi;
    *gmax = g;
    return true;
}

int chaining_params_check(const mpg_chaining_params* cp) {
    if (!cp || cp->k < 1 || cp->G < 1 || !(cp->beta >= 0.0) || cp->max_chains < 1 ||
        (cp->binned != 0 && cp->binned != 1))
        return MPG_E_INVAL;
    return MPG_OK;
}

// Enqueue the chaining of nsets sets whose anchors are on the device.
int chain_sets_dev(hipStream_t st, Workspace& ws, const mpg_chaining_params* cp,
                   const int32_t* d_anchors, const int64_t* set_off, int32_t nsets, double* d_f,
                   int32_t* d_pred, int32_t* d_idx, mpg_chain_out* d_top, int32_t* d_ntop) {
    std::vector<ChainSetJob> jobs(nsets);
    int32_t max_n = 1;
    for (int32_t t = 0; t < nsets; ++t) {
        const int64_t n = set_off[t + 1] - set_off[t];
        if (set_off[t] < 0 || n < 0) return MPG_E_INVAL;
        jobs[t].off = set_off[t];
        jobs[t].n = (int32_t)std::min<int64_t>(n, MPG_MAX_ANCHORS);
        jobs[t].status = n > MPG_MAX_ANCHORS ? MPG_E_RANGE : MPG_OK;
        jobs[t].id = t;
        jobs[t]._pad = 0;
        if (jobs[t].status == MPG_OK) max_n = std::max<int32_t>(max_n, (int32_t)n);
    }
    // largest sets first: a set's work is sequential over its anchors, so the
    // launch lasts at least as long as its largest set, which should start at
    // once (stable: equal sizes keep their order)
    std::stable_sort(jobs.begin(), jobs.end(), [](const ChainSetJob& a, const ChainSetJob& b) {
        return a.n > b.n;
    });
    const int64_t total = set_off[nsets];
    const size_t jb = sizeof(ChainSetJob) * (size_t)nsets;
    const size_t rb = sizeof(ChainRec) * (size_t)std::max<int64_t>(total, 1);
    int rc;
    if (hipStreamSynchronize(st) != hipSuccess) return MPG_E_DEVICE;
    if ((rc = ws.cset.ensure(((jb + 15) & ~(size_t)15) + rb + 64)) != MPG_OK) return rc;
    if ((rc = ws.hcset.ensure(jb + 64)) != MPG_OK) return rc;
    std::memcpy(ws.hcset.p, jobs.data(), jb);
    if (hipMemcpyAsync(ws.cset.p, ws.hcset.p, jb, hipMemcpyHostToDevice, st) != hipSuccess)
        return MPG_E_DEVICE;
    ChainCfg cfg;
    cfg.k = cp->k;
    cfg.G = cp->G;
    cfg.binned = cp->binned;
    cfg.max_chains = cp->max_chains;
    cfg.max_n = max_n;
    // f in LDS when it fits beside the used flags; anchors and predecessors
    // too when they also fit; four wavefronts per set once the largest set's
    // candidate loops are long enough to share
    cfg.f_lds = kChainRedBytes + 9 * (int64_t)max_n + 16 <= kChainLdsBytes ? 1 : 0;
    cfg.stage = cfg.f_lds && kChainRedBytes + 21 * (int64_t)max_n + 16 <= kChainLdsBytes ? 1 : 0;
    cfg.waves = max_n >= 512 ? 4 : 1;
    cfg.beta = cp->beta;
    ChainRec* recs = (ChainRec*)((uint8_t*)ws.cset.p + ((jb + 15) & ~(size_t)15));
    if (launch_chain(st, (const ChainSetJob*)ws.cset.p, nsets, (const int2*)d_anchors, cfg, d_f,
                     d_pred, recs, d_idx, d_top, d_ntop) != hipSuccess)
        return MPG_E_DEVICE;
    return MPG_OK;
}

// Pseudogene guard on the device: cut each traced pair's coding sequence
// (cds_kernel), align the aligned protein segment to it end to end without
// intron states, score only, and finish the scores (rescore_finish_kernel).
// The coding lengths come back to the host once, to plan the second batch.
int rescore_dev(hipStream_t st, Workspace& ws, const mpg_params* p, const uint8_t* d_prot,
                const uint8_t* d_dna, const mpg_seg* segs, int32_t n, const mpg_dev_result* d_res,
                const char* d_ops, int32_t* d_score, int32_t* d_exons, int32_t* d_status,
                RunCfg cfg) {
    std::vector<mpg_dev_result> rec(n);
    if (hipMemcpyAsync(rec.data(), d_res, sizeof(mpg_dev_result) * (size_t)n,
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MPG_E_DEVICE;
    std::vector<CdsJob> jobs(n);
    int64_t cbytes = 0;
    for (int32_t k = 0; k < n; ++k) {
        const mpg_dev_result& r = rec[k];
        CdsJob& J = jobs[k];
        std::memset(&J, 0, sizeof(J));
        J.cds_off = cbytes;
        if (r.status != MPG_OK) continue;
        if (r.g_beg < 0 || r.p_beg < 0 || r.g_end < r.g_beg || r.p_end < r.p_beg ||
            r.g_end > segs[k].dlen || r.p_end > segs[k].plen || r.ops_len < 0)
            return MPG_E_INVAL;  // not a traced result of these pairs
        J.ops_off = r.ops_off;
        J.ops_len = r.ops_len;
        J.dna_off = segs[k].dna_off + r.g_beg;
        J.cap = r.g_end - r.g_beg;
        J.plen = r.p_end - r.p_beg;
        cbytes += J.cap;
    }
    const size_t jb = sizeof(CdsJob) * (size_t)n, ib = sizeof(int4) * (size_t)n;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_j = 0, o_i = al(jb), o_c = o_i + al(ib), o_2 = o_c + al((size_t)cbytes),
                 o_m = o_2 + al(sizeof(mpg_dev_result) * (size_t)n), tot = o_m + al(4 * (size_t)n);
    int rc;
    if ((rc = ws.cset.ensure(tot + 64)) != MPG_OK) return rc;
    if ((rc = ws.hcset.ensure(jb + 64)) != MPG_OK) return rc;
    std::memcpy(ws.hcset.p, jobs.data(), jb);
    uint8_t* d = (uint8_t*)ws.cset.p;
    if (hipMemcpyAsync(d + o_j, ws.hcset.p, jb, hipMemcpyHostToDevice, st) != hipSuccess)
        return MPG_E_DEVICE;
    int4* d_info = (int4*)(d + o_i);
    uint8_t* d_cds = d + o_c;
    if (launch_cds(st, (const CdsJob*)(d + o_j), n, d_ops, d_dna, d_cds, d_info) != hipSuccess)
        return MPG_E_DEVICE;
    std::vector<int4> info(n);
    if (hipMemcpyAsync(info.data(), d_info, ib, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MPG_E_DEVICE;
    // the second alignment: end to end, no intron states, score only
    mpg_params p2 = *p;
    p2.mode = MPG_GLOBAL;
    p2.flags = (p->flags | MPG_NO_INTRON) & ~(uint32_t)(MPG_WANT_TB | MPG_ALLOW_I16);
    std::vector<mpg_seg> s2;
    std::vector<int32_t> j2(n, -1);
    for (int32_t k = 0; k < n; ++k) {
        if (rec[k].status != MPG_OK || info[k].z != MPG_OK) continue;
        mpg_seg q;
        q.prot_off = segs[k].prot_off + rec[k].p_beg;
        q.plen = jobs[k].plen;
        q.dna_off = jobs[k].cds_off;
        q.dlen = info[k].x;
        q.flags = 0;
        q._pad = 0;
        j2[k] = (int32_t)s2.size();
        s2.push_back(q);
    }
    mpg_dev_result* d_res2 = (mpg_dev_result*)(d + o_2);
    int32_t* d_j2 = (int32_t*)(d + o_m);
    if ((rc = ws.hchain.ensure(4 * (size_t)n + 64)) != MPG_OK) return rc;
    std::memcpy(ws.hchain.p, j2.data(), 4 * (size_t)n);
    if (hipMemcpyAsync(d_j2, ws.hchain.p, 4 * (size_t)n, hipMemcpyHostToDevice, st) != hipSuccess)
        return MPG_E_DEVICE;
    if (!s2.empty()) {
        char* d_ops2 = nullptr;  // score only: one byte per pair
        if ((rc = ws.piece_ops.ensure(s2.size() + 64)) != MPG_OK) return rc;
        d_ops2 = (char*)ws.piece_ops.p;
        rc = run_dev_waves(st, ws, &p2, d_prot, d_cds, s2.data(), (int32_t)s2.size(), d_res2,
                           d_ops2, cfg);
        if (rc != MPG_OK) return rc;
    }
    if (launch_rescore_finish(st, n, d_res, d_info, d_j2, d_res2, p->r, d_score, d_exons,
                              d_status) != hipSuccess)
        return MPG_E_DEVICE;
    return MPG_OK;
}

extern "C" {

int mpg_align_batch(mpg_ctx* ctx, const mpg_params* p, const mpg_pair* pairs, int32_t n,
                    mpg_result* out) {
    if (!ctx || !p || n < 0 || (n > 0 && (!pairs || !out))) return MPG_E_INVAL;
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    if (n == 0) return MPG_OK;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    Timer tm{{&ctx->ev_pre, &ctx->ev_dp, &ctx->ev_walk}, &ctx->ev_pool, &ctx->t_host, &ctx->n_i16,
             &ctx->n_cells, &ctx->n_seg};
    ctx->n_calls++;
    RunCfg cfg;
    cfg.tb_budget = ctx->tb_budget;
    cfg.tm = ctx->timing ? &tm : nullptr;
    cfg.ncu = g_num_cu;
    cfg.tune = &ctx->tune;
    return align_host(ctx->stream, ctx->ws, p, pairs, n, out, cfg);
}

int64_t mpg_chain_ops_capacity(const mpg_params* p, const mpg_chain_seg* chains, int32_t n) {
    if (!p || n < 0 || (n > 0 && !chains)) return 0;
    int64_t o = 0;
    for (int32_t c = 0; c < n; ++c)
        o += chain_tb(chains[c], p)
                 ? 2 * ((int64_t)std::max(0, chains[c].plen) + std::max(0, chains[c].dlen)) + 1
                 : 1;
    return o;
}

int mpg_align_chains_dev(mpg_ctx* ctx, const mpg_params* p, const uint8_t* d_prot,
                         const uint8_t* d_dna, const mpg_chain_seg* chains, int32_t n,
                         mpg_dev_result* d_out, char* d_ops, int64_t ops_cap) {
    if (!ctx || !p || n < 0 || (n > 0 && (!chains || !d_out || !d_ops))) return MPG_E_INVAL;
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    if (n == 0) return MPG_OK;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    Timer tm{{&ctx->ev_pre, &ctx->ev_dp, &ctx->ev_walk}, &ctx->ev_pool, &ctx->t_host, &ctx->n_i16,
             &ctx->n_cells, &ctx->n_seg};
    ctx->n_calls++;
    RunCfg cfg;
    cfg.tb_budget = ctx->tb_budget;
    cfg.tm = ctx->timing ? &tm : nullptr;
    cfg.ncu = g_num_cu;
    cfg.tune = &ctx->tune;
    // Large calls run as two sub-batches on two workspaces of their own: the
    // host plans the second while the device runs the first (each waits only
    // for its workspace's previous use, marked by an event).  Both go to the
    // context stream in order; every chain is checked before either is
    // enqueued, so an invalid call does no work.  (Four sub-batches cost more
    // in the tails of their DP launches than the overlap gains.)
    const int nsub = n >= 2048 ? 2 : 1;
    if (nsub == 1)
        return chains_dev(ctx->stream, ctx->ws, p, d_prot, d_dna, chains, n, d_out, d_ops,
                          ops_cap, cfg);
    for (int32_t c = 0; c < n; ++c)
        if (!chain_valid(chains[c])) return MPG_E_INVAL;
    if (mpg_chain_ops_capacity(p, chains, n) > ops_cap) return MPG_E_RANGE;
    for (int k = 0; k < 2; ++k)
        if (!ctx->chain_ev[k] &&
            hipEventCreateWithFlags(&ctx->chain_ev[k], hipEventDisableTiming) != hipSuccess)
            return MPG_E_DEVICE;
    int64_t ops_base = 0;
    for (int sb = 0; sb < nsub; ++sb) {
        const int32_t lo = (int32_t)((int64_t)n * sb / nsub);
        const int32_t hi = (int32_t)((int64_t)n * (sb + 1) / nsub);
        Workspace& w = ctx->chain_ws[sb & 1];
        RunCfg c = cfg;
        c.ws_ready = ctx->chain_ev[sb & 1];  // never recorded yet: complete
        rc = chains_dev(ctx->stream, w, p, d_prot, d_dna, chains + lo, hi - lo, d_out + lo, d_ops,
                        ops_cap, c, ops_base);
        if (rc != MPG_OK) return rc;
        if (hipEventRecord(ctx->chain_ev[sb & 1], ctx->stream) != hipSuccess) return MPG_E_DEVICE;
        ops_base += mpg_chain_ops_capacity(p, chains + lo, hi - lo);
    }
    return MPG_OK;
}

int mpg_align_chains(mpg_ctx* ctx, const mpg_params* p, const mpg_chain* chains, int32_t n,
                     mpg_result* out) {
    if (!ctx || !p || n < 0 || (n > 0 && (!chains || !out))) return MPG_E_INVAL;
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    if (n == 0) return MPG_OK;
    std::vector<mpg_chain_seg> cs(n);
    int64_t pbytes = 0, dbytes = 0;
    for (int32_t c = 0; c < n; ++c) {
        const mpg_chain& ch = chains[c];
        if (ch.plen < 0 || ch.dlen < 0 || (ch.plen && !ch.prot) || (ch.dlen && !ch.dna))
            return MPG_E_INVAL;
        cs[c].prot_off = pbytes;
        cs[c].dna_off = dbytes;
        cs[c].plen = ch.plen;
        cs[c].dlen = ch.dlen;
        cs[c].anchors = ch.anchors;
        cs[c].nanchors = ch.nanchors;
        cs[c].k = ch.k;
        cs[c].flags = ch.flags;
        cs[c]._pad = 0;
        pbytes += ch.plen;
        dbytes += ch.dlen;
    }
    const int64_t cops = mpg_chain_ops_capacity(p, cs.data(), n);
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    Timer tm{{&ctx->ev_pre, &ctx->ev_dp, &ctx->ev_walk}, &ctx->ev_pool, &ctx->t_host, &ctx->n_i16,
             &ctx->n_cells, &ctx->n_seg};
    ctx->n_calls++;
    RunCfg cfg;
    cfg.tb_budget = ctx->tb_budget;
    cfg.tm = ctx->timing ? &tm : nullptr;
    cfg.ncu = g_num_cu;
    cfg.tune = &ctx->tune;
    Workspace& ws = ctx->ws;
    hipStream_t st = ctx->stream;
    if (hipStreamSynchronize(st) != hipSuccess) return MPG_E_DEVICE;
    if ((rc = ws.seq.ensure((size_t)(pbytes + dbytes) + 64)) != MPG_OK) return rc;
    if ((rc = ws.out.ensure(sizeof(mpg_dev_result) * (size_t)n + 64)) != MPG_OK) return rc;
    if ((rc = ws.ops.ensure((size_t)cops + 64)) != MPG_OK) return rc;
    if ((rc = ws.hseq.ensure((size_t)(pbytes + dbytes) + 64)) != MPG_OK) return rc;
    if ((rc = ws.hout.ensure(sizeof(mpg_dev_result) * (size_t)n + 64)) != MPG_OK) return rc;
    uint8_t* hs = (uint8_t*)ws.hseq.p;
    for (int32_t c = 0; c < n; ++c) {
        if (chains[c].plen) std::memcpy(hs + cs[c].prot_off, chains[c].prot, chains[c].plen);
        if (chains[c].dlen) std::memcpy(hs + pbytes + cs[c].dna_off, chains[c].dna, chains[c].dlen);
    }
    uint8_t* d_seq = (uint8_t*)ws.seq.p;
    if (pbytes + dbytes > 0 &&
        hipMemcpyAsync(d_seq, hs, (size_t)(pbytes + dbytes), hipMemcpyHostToDevice, st) !=
            hipSuccess)
        return MPG_E_DEVICE;
    mpg_dev_result* d_cres = (mpg_dev_result*)ws.out.p;
    char* d_cops = (char*)ws.ops.p;
    rc = chains_dev(st, ws, p, d_seq, d_seq + pbytes, cs.data(), n, d_cres, d_cops, cops, cfg);
    if (rc != MPG_OK) return rc;
    if (hipMemcpyAsync(ws.hout.p, d_cres, sizeof(mpg_dev_result) * (size_t)n,
                       hipMemcpyDeviceToHost, st) != hipSuccess)
        return MPG_E_DEVICE;
    bool any_tb = false;
    for (int32_t c = 0; c < n; ++c) any_tb |= chain_tb(cs[c], p);
    if (any_tb) {
        if ((rc = ws.hops.ensure((size_t)cops + 64)) != MPG_OK) return rc;
        if (hipMemcpyAsync(ws.hops.p, d_cops, (size_t)cops, hipMemcpyDeviceToHost, st) !=
            hipSuccess)
            return MPG_E_DEVICE;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return MPG_E_DEVICE;
    const mpg_dev_result* R = (const mpg_dev_result*)ws.hout.p;
    for (int32_t c = 0; c < n; ++c) {
        mpg_result& o = out[c];
        std::memset(&o, 0, sizeof(o));
        o.job_id = (uint64_t)c;
        o.status = R[c].status;
        o.score = R[c].score;
        o.g_beg = R[c].g_beg;
        o.g_end = R[c].g_end;
        o.p_beg = R[c].p_beg;
        o.p_end = R[c].p_end;
        if (chain_tb(cs[c], p) && o.status == MPG_OK) {
            char* sdup = (char*)std::malloc((size_t)R[c].ops_len + 1);
            if (!sdup) return MPG_E_NOMEM;
            std::memcpy(sdup, (const char*)ws.hops.p + R[c].ops_off, (size_t)R[c].ops_len);
            sdup[R[c].ops_len] = 0;
            o.ops = sdup;
            o.ops_len = R[c].ops_len;
        }
    }
    return MPG_OK;
}

int64_t mpg_profile_bytes(int32_t m) { return m < 0 ? 0 : prof_block_bytes(m); }

int mpg_align_profiles_dev(mpg_ctx* ctx, const mpg_params* p, const uint8_t* d_prof,
                           const uint8_t* d_dna, const mpg_profile_seg* segs, int32_t n,
                           mpg_dev_result* d_out, char* d_ops, int64_t ops_cap) {
    if (!ctx || !p || n < 0 || (n > 0 && (!segs || !d_out))) return MPG_E_INVAL;
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    if (n == 0) return MPG_OK;
    std::vector<mpg_seg> ps(n);
    std::vector<int32_t> bounds(2 * (size_t)n);
    int64_t need = 0;
    for (int32_t k = 0; k < n; ++k) {
        const mpg_profile_seg& g = segs[k];
        if (g.prof_off < 0 || (g.prof_off & 7) || g.dna_off < 0 || g.smax < 0 || g.pmax < 0)
            return MPG_E_INVAL;
        ps[k].prot_off = g.prof_off;
        ps[k].dna_off = g.dna_off;
        ps[k].plen = g.m;
        ps[k].dlen = g.dlen;
        ps[k].flags = g.flags;
        ps[k]._pad = 0;
        bounds[2 * k] = g.smax;
        bounds[2 * k + 1] = g.pmax;
        const bool tb = ((g.flags | p->flags) & MPG_WANT_TB) != 0;
        need += tb ? 2 * ((int64_t)std::max(0, g.dlen) + std::max(0, g.m)) + 1 : 1;
    }
    if (need > 0 && (!d_ops || ops_cap < need)) return MPG_E_RANGE;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    Timer tm{{&ctx->ev_pre, &ctx->ev_dp, &ctx->ev_walk}, &ctx->ev_pool, &ctx->t_host, &ctx->n_i16,
             &ctx->n_cells, &ctx->n_seg};
    ctx->n_calls++;
    RunCfg cfg;
    cfg.tb_budget = ctx->tb_budget;
    cfg.tm = ctx->timing ? &tm : nullptr;
    cfg.ncu = g_num_cu;
    cfg.tune = &ctx->tune;
    cfg.pro = true;
    cfg.pro_bounds = bounds.data();
    return run_dev_waves(ctx->stream, ctx->ws, p, d_prof, d_dna, ps.data(), n, d_out, d_ops, cfg);
}

int mpg_align_profiles(mpg_ctx* ctx, const mpg_params* p, const mpg_profile_pair* pairs,
                       int32_t n, mpg_result* out) {
    if (!ctx || !p || n < 0 || (n > 0 && (!pairs || !out))) return MPG_E_INVAL;
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    if (n == 0) return MPG_OK;
    std::vector<mpg_seg> ps(n);
    std::vector<int32_t> bounds(2 * (size_t)n);
    int64_t fbytes = 0, dbytes = 0;
    for (int32_t k = 0; k < n; ++k) {
        const mpg_profile_pair& q = pairs[k];
        if (q.m < 0 || q.dlen < 0 || !q.gap || (q.m && !q.score) || (q.dlen && !q.dna))
            return MPG_E_INVAL;
        if (q.m <= MPG_MAX_PROT &&
            !profile_bounds(q.score, q.gap, q.m, &bounds[2 * k], &bounds[2 * k + 1]))
            return MPG_E_INVAL;
        ps[k].prot_off = fbytes;
        ps[k].dna_off = dbytes;
        ps[k].plen = q.m;
        ps[k].dlen = q.dlen;
        ps[k].flags = q.flags | (p->flags & MPG_WANT_TB);
        ps[k]._pad = 0;
        fbytes += q.m <= MPG_MAX_PROT ? prof_block_bytes(q.m) : 0;
        dbytes += q.dlen;
    }
    const int64_t ops_cap = mpg_ops_capacity(ps.data(), n);
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    Timer tm{{&ctx->ev_pre, &ctx->ev_dp, &ctx->ev_walk}, &ctx->ev_pool, &ctx->t_host, &ctx->n_i16,
             &ctx->n_cells, &ctx->n_seg};
    ctx->n_calls++;
    RunCfg cfg;
    cfg.tb_budget = ctx->tb_budget;
    cfg.tm = ctx->timing ? &tm : nullptr;
    cfg.ncu = g_num_cu;
    cfg.tune = &ctx->tune;
    cfg.pro = true;
    cfg.pro_bounds = bounds.data();
    Workspace& ws = ctx->ws;
    hipStream_t st = ctx->stream;
    const size_t tot = (size_t)(fbytes + dbytes);
    if ((rc = ws.seq.ensure(tot + 64)) != MPG_OK) return rc;
    if ((rc = ws.out.ensure(sizeof(mpg_dev_result) * (size_t)n + 64)) != MPG_OK) return rc;
    if ((rc = ws.ops.ensure((size_t)ops_cap + 64)) != MPG_OK) return rc;
    if ((rc = ws.hseq.ensure(tot + 64)) != MPG_OK) return rc;
    if ((rc = ws.hout.ensure(sizeof(mpg_dev_result) * (size_t)n + 64)) != MPG_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return MPG_E_DEVICE;
    uint8_t* hs = (uint8_t*)ws.hseq.p;
    for (int32_t k = 0; k < n; ++k) {
        const mpg_profile_pair& q = pairs[k];
        if (q.m <= MPG_MAX_PROT) {
            uint8_t* blk = hs + ps[k].prot_off;
            std::memset(blk, 0, (size_t)prof_block_bytes(q.m));
            if (q.m) std::memcpy(blk, q.score, (size_t)24 * q.m);
            std::memcpy(blk + prof_gap_offset(q.m), q.gap, (size_t)8 * (q.m + 1));
        }
        if (q.dlen) std::memcpy(hs + fbytes + ps[k].dna_off, q.dna, (size_t)q.dlen);
    }
    uint8_t* d_seq = (uint8_t*)ws.seq.p;
    if (tot && hipMemcpyAsync(d_seq, hs, tot, hipMemcpyHostToDevice, st) != hipSuccess)
        return MPG_E_DEVICE;
    mpg_dev_result* d_out = (mpg_dev_result*)ws.out.p;
    rc = run_dev_waves(st, ws, p, d_seq, d_seq + fbytes, ps.data(), n, d_out, (char*)ws.ops.p,
                       cfg);
    if (rc != MPG_OK) return rc;
    return download_results(st, ws, p, ps.data(), n, ops_cap, out);
}

void mpg_chaining_params_default(mpg_chaining_params* cp) {
    if (!cp) return;
    cp->k = 6;
    cp->G = 200000;
    cp->beta = 0.75;
    cp->binned = 1;
    cp->max_chains = 30;
}

int mpg_chain_anchors_dev(mpg_ctx* ctx, const mpg_chaining_params* cp, const int32_t* d_anchors,
                          const int64_t* set_off, int32_t nsets, double* d_f, int32_t* d_pred,
                          int32_t* d_idx, mpg_chain_out* d_top, int32_t* d_ntop) {
    if (!ctx || nsets < 0 || (nsets > 0 && (!set_off || !d_top || !d_ntop))) return MPG_E_INVAL;
    int rc = chaining_params_check(cp);
    if (rc != MPG_OK) return rc;
    if (nsets == 0) return MPG_OK;
    if (set_off[0] != 0) return MPG_E_INVAL;
    if (set_off[nsets] > 0 && (!d_anchors || !d_f || !d_pred || !d_idx)) return MPG_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    return chain_sets_dev(ctx->stream, ctx->ws, cp, d_anchors, set_off, nsets, d_f, d_pred, d_idx,
                          d_top, d_ntop);
}

int mpg_chain_anchors(mpg_ctx* ctx, const mpg_chaining_params* cp, const int32_t* anchors,
                      const int64_t* set_off, int32_t nsets, double* f, int32_t* pred,
                      int32_t* idx, mpg_chain_out* top, int32_t* ntop) {
    if (!ctx || nsets < 0 || (nsets > 0 && (!set_off || !top || !ntop))) return MPG_E_INVAL;
    int rc = chaining_params_check(cp);
    if (rc != MPG_OK) return rc;
    if (nsets == 0) return MPG_OK;
    if (set_off[0] != 0) return MPG_E_INVAL;
    const int64_t total = set_off[nsets];
    if (total > 0 && (!anchors || !f || !pred || !idx)) return MPG_E_INVAL;
    for (int32_t t = 0; t < nsets; ++t) {
        if (set_off[t + 1] < set_off[t]) return MPG_E_INVAL;
        for (int64_t a = set_off[t] + 1; a < set_off[t + 1]; ++a) {
            const int32_t* u = anchors + 2 * (a - 1);
            const int32_t* v = anchors + 2 * a;
            if (v[0] < u[0] || (v[0] == u[0] && v[1] < u[1])) return MPG_E_INVAL;
        }
    }
    const size_t ab = 8 * (size_t)total, fb = 8 * (size_t)total, ib = 4 * (size_t)total;
    const size_t tb = sizeof(mpg_chain_out) * (size_t)nsets * cp->max_chains, nb = 4 * (size_t)nsets;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_a = 0, o_f = al(ab), o_p = o_f + al(fb), o_i = o_p + al(ib), o_t = o_i + al(ib),
                 o_n = o_t + al(tb), tot = o_n + al(nb);
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    Workspace& ws = ctx->ws;
    hipStream_t st = ctx->stream;
    if (hipStreamSynchronize(st) != hipSuccess) return MPG_E_DEVICE;
    if ((rc = ws.cio.ensure(tot + 64)) != MPG_OK) return rc;
    uint8_t* d = (uint8_t*)ws.cio.p;
    if (ab && hipMemcpyAsync(d + o_a, anchors, ab, hipMemcpyHostToDevice, st) != hipSuccess)
        return MPG_E_DEVICE;
    rc = chain_sets_dev(st, ws, cp, (const int32_t*)(d + o_a), set_off, nsets,
                        (double*)(d + o_f), (int32_t*)(d + o_p), (int32_t*)(d + o_i),
                        (mpg_chain_out*)(d + o_t), (int32_t*)(d + o_n));
    if (rc != MPG_OK) return rc;
    hipError_t e = hipSuccess;
    if (fb) e = hipMemcpyAsync(f, d + o_f, fb, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && ib) e = hipMemcpyAsync(pred, d + o_p, ib, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && ib) e = hipMemcpyAsync(idx, d + o_i, ib, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(top, d + o_t, tb, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ntop, d + o_n, nb, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return MPG_E_DEVICE;
    return MPG_OK;
}

int mpg_rescore_spliced_dev(mpg_ctx* ctx, const mpg_params* p, const uint8_t* d_prot,
                            const uint8_t* d_dna, const mpg_seg* segs, int32_t n,
                            const mpg_dev_result* d_res, const char* d_ops, int32_t* d_score,
                            int32_t* d_exons, int32_t* d_status) {
    if (!ctx || !p || n < 0 || (n > 0 && (!segs || !d_res || !d_score || !d_exons || !d_status)))
        return MPG_E_INVAL;
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    if (n == 0) return MPG_OK;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    Timer tm{{&ctx->ev_pre, &ctx->ev_dp, &ctx->ev_walk}, &ctx->ev_pool, &ctx->t_host, &ctx->n_i16,
             &ctx->n_cells, &ctx->n_seg};
    ctx->n_calls++;
    RunCfg cfg;
    cfg.tb_budget = ctx->tb_budget;
    cfg.tm = ctx->timing ? &tm : nullptr;
    cfg.ncu = g_num_cu;
    cfg.tune = &ctx->tune;
    return rescore_dev(ctx->stream, ctx->ws, p, d_prot, d_dna, segs, n, d_res, d_ops, d_score,
                       d_exons, d_status, cfg);
}

int mpg_rescore_spliced(mpg_ctx* ctx, const mpg_params* p, const mpg_pair* pairs,
                        const mpg_result* res, int32_t n, int32_t* score, int32_t* exons,
                        int32_t* status) {
    if (!ctx || !p || n < 0 || (n > 0 && (!pairs || !res || !score || !exons || !status)))
        return MPG_E_INVAL;
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    if (n == 0) return MPG_OK;
    // stage letters, first-pass records and op strings as the device entry
    // point takes them
    std::vector<mpg_seg> segs(n);
    std::vector<mpg_dev_result> rec(n);
    int64_t pbytes = 0, dbytes = 0, obytes = 0;
    for (int32_t k = 0; k < n; ++k) {
        const mpg_pair& q = pairs[k];
        if (q.plen < 0 || q.dlen < 0 || (q.plen && !q.prot) || (q.dlen && !q.dna)) return MPG_E_INVAL;
        const mpg_result& r = res[k];
        if (r.status == MPG_OK &&
            (!r.ops || r.ops_len < 0 || r.g_beg < 0 || r.p_beg < 0 || r.g_beg > r.g_end ||
             r.p_beg > r.p_end || r.g_end > q.dlen || r.p_end > q.plen))
            return MPG_E_INVAL;
        segs[k].prot_off = pbytes;
        segs[k].dna_off = dbytes;
        segs[k].plen = q.plen;
        segs[k].dlen = q.dlen;
        segs[k].flags = 0;
        segs[k]._pad = 0;
        mpg_dev_result& d = rec[k];
        d.status = r.status;
        d.score = r.score;
        d.g_beg = r.g_beg;
        d.g_end = r.g_end;
        d.p_beg = r.p_beg;
        d.p_end = r.p_end;
        d.ops_off = obytes;
        d.ops_len = r.status == MPG_OK ? r.ops_len : 0;
        d._pad = 0;
        pbytes += q.plen;
        dbytes += q.dlen;
        obytes += d.ops_len;
    }
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    Timer tm{{&ctx->ev_pre, &ctx->ev_dp, &ctx->ev_walk}, &ctx->ev_pool, &ctx->t_host, &ctx->n_i16,
             &ctx->n_cells, &ctx->n_seg};
    ctx->n_calls++;
    RunCfg cfg;
    cfg.tb_budget = ctx->tb_budget;
    cfg.tm = ctx->timing ? &tm : nullptr;
    cfg.ncu = g_num_cu;
    cfg.tune = &ctx->tune;
    Workspace& ws = ctx->ws;
    hipStream_t st = ctx->stream;
    const size_t rb = sizeof(mpg_dev_result) * (size_t)n, ob = 12 * (size_t)n;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_p = 0, o_d = al(pbytes), o_r = o_d + al(dbytes), o_o = o_r + al(rb),
                 o_f = o_o + al(obytes), tot = o_f + al(ob);
    if (hipStreamSynchronize(st) != hipSuccess) return MPG_E_DEVICE;
    if ((rc = ws.seq.ensure(tot + 64)) != MPG_OK) return rc;
    if ((rc = ws.hseq.ensure(tot + 64)) != MPG_OK) return rc;
    uint8_t* h = (uint8_t*)ws.hseq.p;
    for (int32_t k = 0; k < n; ++k) {
        if (pairs[k].plen) std::memcpy(h + o_p + segs[k].prot_off, pairs[k].prot, pairs[k].plen);
        if (pairs[k].dlen) std::memcpy(h + o_d + segs[k].dna_off, pairs[k].dna, pairs[k].dlen);
        if (rec[k].ops_len)
            std::memcpy(h + o_o + rec[k].ops_off, res[k].ops, (size_t)rec[k].ops_len);
    }
    std::memcpy(h + o_r, rec.data(), rb);
    uint8_t* d = (uint8_t*)ws.seq.p;
    if (hipMemcpyAsync(d, h, o_f, hipMemcpyHostToDevice, st) != hipSuccess) return MPG_E_DEVICE;
    int32_t* d_fin = (int32_t*)(d + o_f);
    rc = rescore_dev(st, ws, p, d + o_p, d + o_d, segs.data(), n, (const mpg_dev_result*)(d + o_r),
                     (const char*)(d + o_o), d_fin, d_fin + n, d_fin + 2 * n, cfg);
    if (rc != MPG_OK) return rc;
    std::vector<int32_t> fin(3 * (size_t)n);
    if (hipMemcpyAsync(fin.data(), d_fin, ob, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MPG_E_DEVICE;
    for (int32_t k = 0; k < n; ++k) {
        // a malformed op string is the caller's error
        if (res[k].status == MPG_OK && fin[2 * n + k] == MPG_E_INVAL) return MPG_E_INVAL;
        score[k] = fin[k];
        exons[k] = fin[n + k];
        status[k] = fin[2 * n + k];
    }
    return MPG_OK;
}

int mpg_submit(mpg_ctx* ctx, const mpg_params* p, const mpg_pair* pair, uint64_t* job_id) {
    if (!ctx || !p || !pair || !job_id) return MPG_E_INVAL;
    if (pair->plen < 0 || pair->dlen < 0 || (pair->plen && !pair->prot) ||
        (pair->dlen && !pair->dna))
        return MPG_E_INVAL;
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    std::unique_lock<std::mutex> lk(ctx->mu);
    if (!ctx->params_set) {
        ctx->sparams = *p;
        ctx->params_set = true;
    } else if (std::memcmp(&ctx->sparams, p, sizeof(*p)) != 0) {
        return MPG_E_INVAL;
    }
    const bool tb = ((pair->flags | p->flags) & MPG_WANT_TB) != 0;
    const int64_t tbb = tb ? tb_bytes_max(pair->dlen, pair->plen) : 0;
    const int64_t cells = (int64_t)(pair->dlen + 64) * (pair->plen + 1);
    // a long job must fit the part of the budget long batches may use
    const uint64_t tb_limit = cells > mpg_ctx::kLongCells ? ctx->tb_budget - ctx->tb_budget / 8
                                                          : ctx->tb_budget;
    if (pair->dlen > MPG_MAX_DNA || pair->plen > MPG_MAX_PROT || (uint64_t)tbb > tb_limit ||
        !score_bound_ok(p, pair->dlen, pair->plen)) {
        ctx->stats.rejected_range++;
        return MPG_E_RANGE;
    }
    if (ctx->npending >= ctx->max_pending) {
        ctx->stats.rejected_again++;
        return MPG_E_AGAIN;
    }
    mpg_ctx::Job j;
    j.id = ctx->next_id++;
    j.prot.assign(pair->prot ? pair->prot : "", (size_t)pair->plen);
    j.dna.assign(pair->dna ? pair->dna : "", (size_t)pair->dlen);
    j.flags = tb ? (uint32_t)MPG_WANT_TB : 0u;
    j.t_arrive = now_ns();
    j.tb_bytes = tbb;
    j.cells = cells;
    *job_id = j.id;
    const int cls = (j.cells > mpg_ctx::kLongCells ? 2 : 0) + (tb ? 1 : 0);
    ctx->pending[cls].push_back(std::move(j));
    ctx->npending++;
    ctx->stats.submitted++;
    ctx->stats.queue_depth = ctx->npending;
    if (!ctx->sched_running) {
        ctx->stop = false;
        ctx->sched = std::thread(scheduler, ctx);
        ctx->sched_running = true;
    }
    lk.unlock();
    ctx->cv_work.notify_one();
    return MPG_OK;
}

int mpg_poll(mpg_ctx* ctx, mpg_result* out, int32_t max_results, int32_t timeout_us) {
    if (!ctx || (max_results > 0 && !out) || max_results < 0) return MPG_E_INVAL;
    std::unique_lock<std::mutex> lk(ctx->mu);
    if (ctx->done.empty() && timeout_us > 0)
        ctx->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                              [ctx] { return !ctx->done.empty(); });
    int k = 0;
    const int64_t t = now_ns();
    while (k < max_results && !ctx->done.empty()) {
        out[k] = ctx->done.front();
        if (out[k].t_done_ns == 0) out[k].t_done_ns = t;
        ctx->done.pop_front();
        ++k;
    }
    return k;
}

int mpg_cancel(mpg_ctx* ctx, uint64_t job_id) {
    if (!ctx) return MPG_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto& Q : ctx->pending) {
        for (auto it = Q.begin(); it != Q.end(); ++it) {
            if (it->id != job_id) continue;
            mpg_result r;
            std::memset(&r, 0, sizeof(r));
            r.status = MPG_E_CANCELLED;
            r.g_beg = r.g_end = r.p_beg = r.p_end = -1;
            r.job_id = job_id;
            r.t_arrive_ns = it->t_arrive;
            r.t_done_ns = now_ns();
            Q.erase(it);
            ctx->npending--;
            ctx->done.push_back(r);
            ctx->stats.cancelled++;
            ctx->stats.queue_depth = ctx->npending;
            ctx->cv_done.notify_all();
            return MPG_OK;
        }
    }
    return MPG_E_INVAL;
}

int mpg_enable_timing(mpg_ctx* ctx, int on) {
    if (!ctx) return MPG_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    ctx->timing = on != 0;
    return MPG_OK;
}

int mpg_autotune(mpg_ctx* ctx, const mpg_params* p, const uint8_t* d_prot, const uint8_t* d_dna,
                 const mpg_seg* segs, int32_t n, mpg_tuning* out) {
    if (!ctx || n < 0 || (n > 0 && (!p || !segs))) return MPG_E_INVAL;
    if (p && params_check_impl(p) != MPG_OK) return MPG_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    Workspace ws;
    ws.use_allocator(&ctx->alloc);
    int rc = MPG_OK;
    hipStream_t st = ctx->stream;
    mpg_params prm;
    std::vector<mpg_seg> sg;
    if (n > 0) {
        prm = *p;
        sg.assign(segs, segs + n);
    } else {
        // built-in sample: 1,024 pairs of 511 residues (no column padding at
        // any width) against 4,096 nucleotides, half of them with traceback,
        // letters from a fixed linear congruential sequence
        const int32_t np = 1024, m = 511, len = 4096;
        std::vector<uint8_t> seq((size_t)np * (m + len));
        uint32_t x = 12345u;
        const char* aa = "ARNDCQEGHILKMFPSTWYV";
        for (size_t k = 0; k < (size_t)np * m; ++k) {
            x = x * 1664525u + 1013904223u;
            seq[k] = (uint8_t)aa[(x >> 16) % 20];
        }
        for (size_t k = (size_t)np * m; k < seq.size(); ++k) {
            x = x * 1664525u + 1013904223u;
            seq[k] = (uint8_t)"ACGT"[(x >> 16) & 3];
        }
        if ((rc = ws.seq.ensure(seq.size())) != MPG_OK) return rc;
        if (hipMemcpyAsync(ws.seq.p, seq.data(), seq.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess) {
            ws.release();
            return MPG_E_DEVICE;
        }
        d_prot = (const uint8_t*)ws.seq.p;
        d_dna = d_prot + (size_t)np * m;
        sg.resize(np);
        for (int32_t k = 0; k < np; ++k) {
            sg[k].prot_off = (int64_t)k * m;
            sg[k].dna_off = (int64_t)k * len;
            sg[k].plen = m;
            sg[k].dlen = len;
            sg[k].flags = (k & 1) ? MPG_WANT_TB : 0;
            sg[k]._pad = 0;
        }
        mpg_params_default(&prm);
        n = np;
    }
    double cells = 0;
    for (const auto& q : sg) cells += (double)std::max(0, q.plen) * std::max(0, q.dlen);
    const int64_t ops_cap = mpg_ops_capacity(sg.data(), n);
    if ((rc = ws.out.ensure(sizeof(mpg_dev_result) * (size_t)n + 64)) != MPG_OK ||
        (rc = ws.ops.ensure((size_t)ops_cap + 64)) != MPG_OK) {
        ws.release();
        return rc;
    }
    // DP time of the sample at one width (the second of two runs)
    // DP time of the sample at one width (K > 0, all pairs), or with the
    // planning choices of t (K = 0): a warm-up run, then the faster of two
    // timed runs (single runs differ by 1-2%, as much as some choices do)
    auto run = [&](int K, int K16, double& ms_out, const Tuning* t = nullptr) -> int {
        RunCfg cfg;
        cfg.tb_budget = ctx->tb_budget;
        cfg.ncu = g_num_cu;
        cfg.force_K = K;
        cfg.force_K16 = K16;
        cfg.tune = t;
        double best_ms = 0;
        for (int rep = 0; rep < 3; ++rep) {
            std::vector<std::pair<hipEvent_t, hipEvent_t>> e3[3];
            std::vector<hipEvent_t> pool;
            double host = 0;
            uint64_t i16 = 0;
            Timer tm{{&e3[0], &e3[1], &e3[2]}, &pool, &host, &i16};
            cfg.tm = rep ? &tm : nullptr;
            int r = run_dev_waves(st, ws, &prm, d_prot, d_dna, sg.data(), n,
                                  (mpg_dev_result*)ws.out.p, (char*)ws.ops.p, cfg);
            if (r == MPG_OK && hipStreamSynchronize(st) != hipSuccess) r = MPG_E_DEVICE;
            double ms = 0;
            for (auto& pr : e3[1]) {
                float f = 0.f;
                if (r == MPG_OK && hipEventElapsedTime(&f, pr.first, pr.second) != hipSuccess)
                    r = MPG_E_DEVICE;
                ms += f;
            }
            for (auto& v : e3)
                for (auto& pr : v) {
                    hipEventDestroy(pr.first);
                    hipEventDestroy(pr.second);
                }
            for (auto e : pool) hipEventDestroy(e);
            if (r != MPG_OK) return r;
            if (rep && (best_ms == 0 || ms < best_ms)) best_ms = ms;
        }
        ms_out = best_ms;
        return MPG_OK;
    };
    Tuning tu;
    mpg_tuning res{};
    const int Ks[3] = {1, 2, 4};
    double best = 0;
    for (int q = 0; q < 3 && rc == MPG_OK; ++q) {
        double ms = 0;
        rc = run(Ks[q], 2, ms);
        if (rc != MPG_OK || ms <= 0) break;
        res.gcups[q] = cells / (ms * 1e-3) / 1e9;
        if (best == 0 || ms < best) {
            best = ms;
            tu.K = Ks[q];
        }
    }
    // at that width: the narrow-pair cutover (pairs of at most 64, 128 or 192
    // columns in strips of one column per lane: the one-wavefront strip of a
    // narrow pair against more, cheaper strips; or none, 1: narrow pairs at
    // the width too, two of them sharing a wavefront), then lane-segment packs
    // on and off
    tu.narrow = 64;
    tu.seg = 1;
    double best_c = 0;
    const int cuts[4] = {64, 128, 192, 1};
    for (int q = 0; q < 4 && rc == MPG_OK && (q == 0 || tu.K > 1); ++q) {
        Tuning t = tu;
        t.narrow = cuts[q];
        double ms = 0;
        rc = run(0, 2, ms, &t);
        if (rc != MPG_OK || ms <= 0) break;
        res.narrow_gcups[q] = cells / (ms * 1e-3) / 1e9;
        if (best_c == 0 || ms < best_c) {
            best_c = ms;
            tu.narrow = cuts[q];
        }
    }
    if (rc == MPG_OK && best_c > 0) {
        Tuning t = tu;
        t.seg = 0;
        double ms = 0;
        rc = run(0, 2, ms, &t);
        if (rc == MPG_OK && ms > 0) {
            res.seg_gcups[0] = cells / (ms * 1e-3) / 1e9;
            res.seg_gcups[1] = cells / (best_c * 1e-3) / 1e9;
            if (ms < best_c) tu.seg = 0;
        }
    }
    if (rc == MPG_OK && (prm.flags & MPG_ALLOW_I16)) {
        double b16 = 0;
        for (int q = 0; q < 2 && rc == MPG_OK; ++q) {
            double ms = 0;
            rc = run(0, q + 1, ms, &tu);
            if (rc != MPG_OK || ms <= 0) break;
            res.i16_gcups[q] = cells / (ms * 1e-3) / 1e9;
            if (b16 == 0 || ms < b16) {
                b16 = ms;
                tu.K16 = q + 1;
            }
        }
    }
    hipStreamSynchronize(st);
    ws.release();
    if (rc != MPG_OK) return rc;
    ctx->tune = tu;
    res.K = tu.K;
    res.K16 = tu.K16;
    res.narrow_cols = tu.narrow;
    res.seg_packs = tu.seg;
    if (out) *out = res;
    return MPG_OK;
}

// ---- planned batches (graph capture and replay)
}  // extern "C"

struct mpg_plan {
    mpg_ctx* ctx = nullptr;
    Workspace ws;
    Prepared X;
    RunCfg cfg;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int mpg_plan_create(mpg_ctx* ctx, const mpg_params* p, const uint8_t* d_prot,
                    const uint8_t* d_dna, const mpg_seg* segs, int32_t n, mpg_dev_result* d_out,
                    char* d_ops, int64_t ops_cap, mpg_plan** plan) {
    if (!ctx || !p || !plan || n < 0 || (n > 0 && (!segs || !d_out))) return MPG_E_INVAL;
    *plan = nullptr;
    int rc = params_check_impl(p);
    if (rc != MPG_OK) return rc;
    const int64_t need = mpg_ops_capacity(segs, n);
    if (need > 0 && (!d_ops || ops_cap < need)) return MPG_E_RANGE;
    std::vector<int64_t> ops_off(n);
    int64_t o = 0, tbb = 0;
    for (int32_t k = 0; k < n; ++k) {
        ops_off[k] = o;
        const bool tb = seg_tb(segs[k], p);
        o += tb ? 2 * ((int64_t)std::max(0, segs[k].dlen) + std::max(0, segs[k].plen)) + 1 : 1;
        if (tb && segs[k].plen >= 0 && segs[k].dlen >= 0) tbb += tb_bytes_max(segs[k].dlen, segs[k].plen);
    }
    // one launch sequence: all direction bits must fit the budget at once
    if ((uint64_t)tbb > ctx->tb_budget) return MPG_E_RANGE;
    mpg_plan* pl = new (std::nothrow) mpg_plan();
    if (!pl) return MPG_E_NOMEM;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    pl->ctx = ctx;
    pl->ws.use_allocator(&ctx->alloc);
    pl->cfg.tb_budget = ctx->tb_budget;
    pl->cfg.ncu = g_num_cu;
    pl->cfg.tune = &ctx->tune;
    std::vector<int32_t> idx(n);
    for (int32_t k = 0; k < n; ++k) idx[k] = k;
    rc = prepare(ctx->stream, pl->ws, p, d_prot, d_dna, segs, idx.data(), n, ops_off, d_out,
                 d_ops, pl->cfg, pl->X);
    if (rc == MPG_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) rc = MPG_E_DEVICE;
    if (rc != MPG_OK) {
        pl->ws.release();
        delete pl;
        return rc;
    }
    *plan = pl;
    return MPG_OK;
}

int mpg_plan_launch(mpg_plan* plan, void* hip_stream) {
    if (!plan) return MPG_E_INVAL;
    hipSetDevice(plan->ctx->device);
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : plan->ctx->stream;
    if (plan->exec) return hipGraphLaunch(plan->exec, st) == hipSuccess ? MPG_OK : MPG_E_DEVICE;
    return enqueue(st, plan->ws, plan->X, plan->cfg, false);
}

int mpg_plan_graph(mpg_plan* plan, void* hip_stream) {
    if (!plan || !hip_stream) return MPG_E_INVAL;
    if (plan->exec) return MPG_OK;
    hipSetDevice(plan->ctx->device);
    hipStream_t st = (hipStream_t)hip_stream;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return MPG_E_DEVICE;
    const int rc = enqueue(st, plan->ws, plan->X, plan->cfg, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != MPG_OK || e != hipSuccess || !g) {
        if (g) hipGraphDestroy(g);
        return rc != MPG_OK ? rc : MPG_E_DEVICE;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(g);
        return MPG_E_DEVICE;
    }
    plan->graph = g;
    plan->exec = x;
    return MPG_OK;
}

void mpg_plan_destroy(mpg_plan* plan) {
    if (!plan) return;
    hipSetDevice(plan->ctx->device);
    hipStreamSynchronize(plan->ctx->stream);
    if (plan->exec) hipGraphExecDestroy(plan->exec);
    if (plan->graph) hipGraphDestroy(plan->graph);
    hipDeviceSynchronize();
    plan->ws.release();
    delete plan;
}

int mpg_get_timing(mpg_ctx* ctx, mpg_timing* t, int reset) {
    if (!ctx || !t) return MPG_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipSetDevice(ctx->device);
    auto drain = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, double& acc,
                     uint64_t* cnt) -> int {
        for (auto& pr : v) {
            if (hipEventSynchronize(pr.second) != hipSuccess) return MPG_E_DEVICE;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess) return MPG_E_DEVICE;
            acc += ms;
            if (cnt) ++*cnt;
            ctx->ev_pool.push_back(pr.first);
            ctx->ev_pool.push_back(pr.second);
        }
        v.clear();
        return MPG_OK;
    };
    int rc;
    if ((rc = drain(ctx->ev_pre, ctx->t_pre, nullptr)) != MPG_OK) return rc;
    if ((rc = drain(ctx->ev_dp, ctx->t_dp, &ctx->n_dp)) != MPG_OK) return rc;
    if ((rc = drain(ctx->ev_walk, ctx->t_walk, nullptr)) != MPG_OK) return rc;
    t->prepass_ms = ctx->t_pre;
    t->dp_ms = ctx->t_dp;
    t->walk_ms = ctx->t_walk;
    t->dp_spans = ctx->n_dp;
    t->calls = ctx->n_calls;
    t->host_ms = ctx->t_host;
    t->i16_pairs = ctx->n_i16;
    t->cells = ctx->n_cells;
    t->seg_packs = ctx->n_seg;
    if (reset) {
        ctx->t_pre = ctx->t_dp = ctx->t_walk = ctx->t_host = 0;
        ctx->n_dp = ctx->n_calls = ctx->n_i16 = ctx->n_cells = ctx->n_seg = 0;
    }
    return MPG_OK;
}

int mpg_get_stats(mpg_ctx* ctx, mpg_stats* st) {
    if (!ctx || !st) return MPG_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    *st = ctx->stats;
    st->tb_budget = ctx->tb_budget;
    return MPG_OK;
}

void mpg_result_release(mpg_ctx* ctx, mpg_result* r, int32_t n) {
    (void)ctx;
    if (!r) return;
    for (int32_t k = 0; k < n; ++k) {
        std::free((void*)r[k].ops);
        r[k].ops = nullptr;
        r[k].ops_len = 0;
    }
}

void mpg_ctx_destroy(mpg_ctx* ctx) {
    if (!ctx) return;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->stop = true;
    }
    ctx->cv_work.notify_all();
    if (ctx->sched_running && ctx->sched.joinable()) ctx->sched.join();
    hipSetDevice(ctx->device);
    if (ctx->own_stream) {
        hipStreamSynchronize(ctx->own_stream);
        hipStreamDestroy(ctx->own_stream);
    }
    ctx->ws.release();
    for (int k = 0; k < 2; ++k) {
        ctx->chain_ws[k].release();
        if (ctx->chain_ev[k]) hipEventDestroy(ctx->chain_ev[k]);
    }
    for (auto* v : {&ctx->ev_pre, &ctx->ev_dp, &ctx->ev_walk})
        for (auto& pr : *v) {
            hipEventDestroy(pr.first);
            hipEventDestroy(pr.second);
        }
    for (auto e : ctx->ev_pool) hipEventDestroy(e);
    for (auto& r : ctx->done) std::free((void*)r.ops);
    delete ctx;
}

}  // extern "C"
