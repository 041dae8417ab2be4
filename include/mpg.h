/*
 * mpg.h -- spliced protein-to-genome DP on AMD Instinct MI355X (gfx950).
 *
 * The library aligns a protein to a genomic region with the dynamic program of
 * Li 2022, "Protein-to-genome alignment with miniprot" (Methods, subsection
 * "DP for protein-to-genome alignment", Eq. (full)): codon translation scored
 * by a 24x24 substitution matrix, affine gaps (a gap of g residues or codons
 * costs q + e*g), frameshifts (penalty f; "DP for protein-to-DNA alignment",
 * Eq. (fs)) and phase-0/1/2 introns (penalty r plus splice-signal penalties
 * d() and a(); "Splice models").  Tools of this kind take a protein and a
 * nucleotide sequence and return a spliced alignment between them
 * (Introduction); the DP is used to close gaps between anchors and to extend
 * from terminal anchors (Methods, opening paragraph and "Residue alignment
 * with dynamic programming").  All DP work runs in HIP kernels on the GPU;
 * there is no CPU fallback.
 *
 * Conventions for every call:
 *  - functions return MPG_OK (0) or a negative MPG_E_* status; no exception
 *    crosses the ABI;
 *  - genome rows i = 1..n are nucleotides, protein columns j = 1..m residues;
 *    coordinates returned are 0-based half-open: the alignment covers genome
 *    [g_beg, g_end) and protein [p_beg, p_end); g_end / p_end are the DP row
 *    and column of the end cell;
 *  - scores are exact integers (int32 storage; mpg_params_check proves that
 *    every reachable value fits with room for packed tie-break keys);
 *  - only the forward strand is aligned: the caller passes the reverse
 *    complement for the other strand (the paper indexes each strand as a
 *    separate sequence, "Indexing the genome").
 */
#ifndef MPG_H
#define MPG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    MPG_OK = 0,
    MPG_E_INVAL = -1,     /* bad argument: NULL pointer, bad params, bad flags */
    MPG_E_RANGE = -2,     /* a length or the score bound exceeds the limits */
    MPG_E_NOMEM = -3,     /* device or host allocation failed */
    MPG_E_AGAIN = -4,     /* serving queue full; retry later */
    MPG_E_DEVICE = -5,    /* a HIP call failed */
    MPG_E_NOALN = -6,     /* GLOBAL: the end cell (n,m) is unreachable */
    MPG_E_CANCELLED = -7  /* serving: job cancelled before it ran */
};

/* ---- boundary modes (sources and sinks of the DP) ---------------------- */
enum {
    MPG_LOCAL = 0,      /* start and end anywhere; H never drops below 0 */
    MPG_EXTEND = 1,     /* start at H(0,0)=0 (an anchor), end anywhere: rightward extension */
    MPG_GLOBAL = 2,     /* start at H(0,0)=0, end at (n,m): closing a gap between anchors */
    MPG_EXTEND_LEFT = 3 /* start anywhere (H never drops below 0), end at (n,m) (an anchor):
                           leftward extension */
};

/* ---- flags -------------------------------------------------------------- */
enum {
    MPG_NO_INTRON = 1u,     /* drop the intron states A, B, C (Eq. (fs)) */
    MPG_NO_FRAMESHIFT = 2u, /* drop the four frameshift terms */
    MPG_WANT_TB = 4u,       /* per pair (or for all pairs in params.flags): op string */
    MPG_ALLOW_I16 = 8u      /* LOCAL score-only pairs may run in the int16 kernel */
};

#define MPG_MAX_DNA 1040000 /* longest genomic region (nucleotides) */
#define MPG_MAX_PROT 32000  /* longest protein (residues) */

/*
 * Scoring parameters (Eq. (full) and "Splice models").
 * Amino-acid order of mat: "ARNDCQEGHILKMFPSTWYVBZX*"; row = translated codon,
 * column = protein residue.  gcode maps the codon 16*b1 + 4*b2 + b3 with
 * A,C,G,T = 0..3 to an amino-acid index.  donor[25*b1+5*b2+b3] is d(i) for
 * the 3-mer T[i+1..i+3] over A,C,G,T,N = 0..4 (the first three intron bases);
 * acceptor[...] is a(i) for T[i-2..i] (the last three intron bases).  Bases
 * outside the region count as N.  Penalties are non-negative, q + e > 0.
 */
typedef struct {
    int32_t q, e, f, r;   /* gap open, gap extend, frameshift, intron */
    uint32_t flags;       /* MPG_NO_INTRON | MPG_NO_FRAMESHIFT | MPG_WANT_TB | MPG_ALLOW_I16 */
    int32_t mode;         /* MPG_LOCAL / MPG_EXTEND / MPG_GLOBAL */
    int8_t mat[24][24];
    uint8_t gcode[64];
    uint8_t donor[125];
    uint8_t acceptor[125];
    uint8_t _pad[2];
} mpg_params;

/* One pair in host memory.  Letters are ASCII, case-insensitive; DNA letters
 * other than ACGT are N, protein letters outside the alphabet are X. */
typedef struct {
    const char *prot;
    int32_t plen;
    const char *dna;
    int32_t dlen;
    uint32_t flags; /* MPG_WANT_TB for this pair (OR-ed with params.flags) */
} mpg_pair;

/* One result.  beg fields are -1 and ops is NULL for score-only pairs. */
typedef struct {
    int32_t status;   /* MPG_OK, MPG_E_RANGE, MPG_E_NOALN, MPG_E_CANCELLED */
    int32_t score;
    int32_t g_beg, g_end, p_beg, p_end;
    const char *ops;  /* run-length op string, owned by the library until released */
    int32_t ops_len;
    int32_t _pad;
    uint64_t job_id;       /* serving: the id returned by mpg_submit; batch: pair index */
    int64_t t_arrive_ns;   /* serving: submit time (CLOCK_MONOTONIC) */
    int64_t t_done_ns;     /* serving: time the result became visible to mpg_poll */
} mpg_result;
/*
 * Op string: tokens "<len><op>" in forward order.  M codon:residue (len =
 * codons), I residues against no genome (len = residues), D codons against no
 * residue (len = codons), F frameshift substitution (len = 1 or 2 nt, one
 * residue), G frameshift insertion (len = 1 or 2 nt), N phase-0 intron (len =
 * nt), U / V phase-1 / phase-2 intron with its split codon (len = total nt
 * consumed, one residue).  M, I and D runs are merged; F, G, N, U, V never.
 * Symbols follow the paper's worked alignment ("Residue alignment with
 * dynamic programming"): F is its "$", G its "+".
 */

typedef struct mpg_ctx mpg_ctx;

/* Create a context on HIP device `device`.  tb_budget_bytes caps the device
 * memory used for traceback direction bits at any time (0 = 64 GiB); larger
 * batches are run in waves under the cap.  flags: reserved, pass 0. */
int mpg_ctx_create(mpg_ctx **ctx, int device, uint64_t tb_budget_bytes, uint32_t flags);

/* Destroy a context; waits for its device work and frees everything. */
void mpg_ctx_destroy(mpg_ctx *ctx);

/* Use an existing hipStream_t for all batch work of this context (NULL =
 * the context's own stream).  The stream stays owned by the caller. */
int mpg_set_stream(mpg_ctx *ctx, void *hip_stream);

/*
 * Take the device memory of every workspace of this context (plans, row
 * descriptors, strip boundaries, direction bits, staging of sequences and
 * results, serving batches) from the caller's allocator instead of
 * hipMalloc/hipFree -- for example PyTorch's caching allocator, so that the
 * library and the caller share one pool of device memory.  The computation
 * itself stays in the library's kernels.
 *  - alloc(bytes, user) returns a block of at least `bytes` bytes of device
 *    memory on the context's device, 256-byte aligned, or NULL (the call
 *    then fails with MPG_E_NOMEM; a misaligned block is given back and the
 *    call fails with MPG_E_INVAL);
 *  - release(ptr, user) takes back a block that alloc returned.  The library
 *    calls it only when none of its own work that uses the block can still
 *    be running: batch calls wait for the context's stream before a
 *    workspace grows, serving parks outgrown blocks until no serving batch
 *    is on the device, and the rest are released by mpg_ctx_destroy (or
 *    mpg_plan_destroy) after the device work has finished.
 * Both callbacks NULL: back to hipMalloc/hipFree for new blocks.  A block is
 * always given back through the allocator that made it, so earlier callbacks
 * and their `user` must stay valid until the context (and every plan made
 * from it) is destroyed.  The callbacks may be called from the library's
 * serving threads.  MPG_E_INVAL: ctx NULL, exactly one callback NULL, or the
 * context has already served a job (mpg_submit): set the allocator before. */
int mpg_set_allocator(mpg_ctx *ctx, void *(*alloc)(size_t bytes, void *user),
                      void (*release)(void *ptr, void *user), void *user);

/* Fill *p with the defaults: q=11, e=1, f=23, r=29, BLOSUM62, the standard
 * genetic code, the final splice model of "Splice models", LOCAL mode. */
void mpg_params_default(mpg_params *p);

/* Check params for pairs up to max_plen residues and max_dlen nucleotides.
 * MPG_E_INVAL: negative penalty, q+e == 0, bad mode/flags or gcode entry.
 * MPG_E_RANGE: lengths beyond MPG_MAX_*, or the bound on |score| for these
 * lengths is not provably below 2^24. */
int mpg_params_check(const mpg_params *p, int32_t max_plen, int32_t max_dlen);

/*
 * Align n pairs held in host memory; synchronous.  `pairs` and the strings
 * are borrowed for the call only.  out[k] receives pair k; its ops string is
 * owned by the library until mpg_result_release(ctx, out, n).  Per-pair
 * failures (MPG_E_RANGE, MPG_E_NOALN) are reported in out[k].status; the
 * call itself fails only for MPG_E_INVAL / MPG_E_NOMEM / MPG_E_DEVICE.  A
 * strip whose wait for its left neighbour gives up (bounded, so that no
 * kernel can hang) reports MPG_E_DEVICE for its pair, and for the pair whose
 * last strip shares its wavefront, if any (two LOCAL pairs' ragged last
 * strips may share one).
 */
int mpg_align_batch(mpg_ctx *ctx, const mpg_params *p, const mpg_pair *pairs, int32_t n,
                    mpg_result *out);

/* ---- device-resident batch ---------------------------------------------- */

/* One pair whose letters already sit in device memory (offsets into the
 * caller's concatenated device buffers). */
typedef struct {
    int64_t prot_off;
    int64_t dna_off;
    int32_t plen;
    int32_t dlen;
    uint32_t flags; /* MPG_WANT_TB */
    int32_t _pad;
} mpg_seg;

/* Device-side result record written by mpg_align_batch_dev (40 bytes). */
typedef struct {
    int32_t status, score, g_beg, g_end, p_beg, p_end;
    int64_t ops_off; /* byte offset of this pair's NUL-terminated op string in the ops
                        buffer; it lies inside the pair's slot (see mpg_ops_capacity) */
    int32_t ops_len;
    int32_t _pad;
} mpg_dev_result;

/* Bytes of op-string buffer that mpg_align_batch_dev needs for these pairs:
 * pairs take consecutive slots in input order, 2*(plen+dlen)+1 bytes for a
 * traceback pair (enough for any path: every token consumes at least one
 * residue or nucleotide per two characters) and 1 byte otherwise. */
int64_t mpg_ops_capacity(const mpg_seg *segs, int32_t n);

/*
 * Enqueue the alignment of n pairs whose letters are in device memory
 * (d_prot, d_dna) on the context's stream and return without waiting.
 * segs (host memory, n entries) gives offsets and lengths; d_out (device,
 * n records) and d_ops (device, ops_cap bytes, NUL-terminated strings) receive
 * the results.  The device buffers must stay valid until the stream has
 * finished the work.  Returns MPG_E_RANGE if ops_cap is too small.
 */
int mpg_align_batch_dev(mpg_ctx *ctx, const mpg_params *p, const uint8_t *d_prot,
                        const uint8_t *d_dna, const mpg_seg *segs, int32_t n,
                        mpg_dev_result *d_out, char *d_ops, int64_t ops_cap);

/* Wait for all work enqueued on the context's stream. */
int mpg_sync(mpg_ctx *ctx);

/* Bytes of the fixed device scratch array behind mpg_align_batch_dev_noalloc
 * (one per GPU, reserved when the library's code is loaded on that GPU and
 * held until the process ends). */
#define MPG_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * For callers that cannot allocate device memory (code that runs under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * mpg_align_batch_dev without any allocation.  Arguments, layouts, ownership
 * and results are those of mpg_align_batch_dev, and the results are
 * identical.  Every device buffer of the call beyond the caller's inputs and
 * outputs (the uploaded plan, row descriptors, strip boundaries, progress
 * counters, pair states, traceback direction bits) is carved out of the
 * GPU's fixed scratch array of MPG_NOALLOC_SCRATCH_BYTES; the call allocates
 * no device or pinned host memory (host planning storage of the context is
 * reused from call to call), creates no stream, and runs all its kernels on
 * the context's stream.
 *  - MPG_E_RANGE: the call needs more scratch than MPG_NOALLOC_SCRATCH_BYTES
 *    (about 24 bytes per genome row of each score-only pair and 1.2 bytes
 *    per cell of each traceback pair, plus ~100 bytes per pair), or ops_cap
 *    is too small; nothing is enqueued then.  Traceback pairs are never split
 *    into waves here.
 *  - MPG_E_DEVICE: the scratch array's address could not be obtained when
 *    the context was created, or a HIP call failed.
 * The call waits for earlier work on the context's stream before it reuses
 * the scratch array, and clears the counters and states that must start at
 * zero with a kernel.  All calls on one GPU share its array: calls that
 * overlap in time on one GPU (other streams, contexts or threads, or work of
 * this call still running while another context calls it) race and give
 * wrong results. */
int mpg_align_batch_dev_noalloc(mpg_ctx *ctx, const mpg_params *p, const uint8_t *d_prot,
                                const uint8_t *d_dna, const mpg_seg *segs, int32_t n,
                                mpg_dev_result *d_out, char *d_ops, int64_t ops_cap);

/*
 * Pseudogene guard (Methods, "Avoiding pseudogenes").  An unspliced copy of a
 * gene pays no intron penalty and can outscore the real, spliced gene; the
 * paper therefore aligns the protein a second time against the coding
 * sequence with the introns taken out, and charges a single-exon alignment
 * the intron penalty r once more.  For each k with res[k].status == MPG_OK
 * (res[k] a traced result of pairs[k], as mpg_align_batch returns it, with
 * params p), this call:
 *  - cuts the coding sequence out of the pair's region along res[k].ops, on
 *    the GPU: the bases of M, D, F and G tokens in path order, nothing of an
 *    N token, and of a U (V) token the split codon's first base and last two
 *    (first two and last one); a U/V token shorter than three bases keeps all
 *    of them;
 *  - aligns the protein segment [p_beg, p_end) to it end to end (MPG_GLOBAL)
 *    with the intron states removed (Eq. (fs)) and p's other scoring, in
 *    the GPU kernels, score only;
 *  - writes score[k] = that optimum, minus p->r when the path has no intron,
 *    exons[k] = number of N/U/V tokens + 1, status[k] = MPG_OK or the second
 *    alignment's status (MPG_E_NOALN when the end cell is unreachable, e.g.
 *    frameshifts off and a coding length not a multiple of 3).
 * Other k get status[k] = res[k].status, score 0, exons 0.  pairs, res and
 * the three output arrays (n entries each) are host memory, borrowed for the
 * call.  MPG_E_INVAL if an MPG_OK result has no op string or its op string
 * does not span exactly its [g_beg, g_end) x [p_beg, p_end); synchronous.
 */
int mpg_rescore_spliced(mpg_ctx *ctx, const mpg_params *p, const mpg_pair *pairs,
                        const mpg_result *res, int32_t n, int32_t *score, int32_t *exons,
                        int32_t *status);

/* As mpg_rescore_spliced for a traced batch still in device memory: the
 * letters and segments given to mpg_align_batch_dev and its d_out / d_ops;
 * score, exons and status are device arrays of n entries.  The coding
 * sequences are cut on the GPU (one wavefront per pair); the call waits for
 * the stream twice (the first pass's records and the coding lengths come to
 * the host to plan the second alignment) and returns with the second
 * alignment and the final scores enqueued.  A malformed op string gives
 * status MPG_E_INVAL for its pair. */
int mpg_rescore_spliced_dev(mpg_ctx *ctx, const mpg_params *p, const uint8_t *d_prot,
                            const uint8_t *d_dna, const mpg_seg *segs, int32_t n,
                            const mpg_dev_result *d_res, const char *d_ops, int32_t *d_score,
                            int32_t *d_exons, int32_t *d_status);

/* ---- anchor-driven alignment ------------------------------------------- */

/* One chain: a protein, its genomic region and the anchors that chaining put
 * on them.  Anchor a is the seed hit anchors[2a] = x, anchors[2a+1] = y: the k
 * codons of the region starting at base x (0-based) against residues
 * y .. y+k-1, one to one. */
typedef struct {
    const char *prot;
    int32_t plen;
    const char *dna;
    int32_t dlen;           /* up to 2^30 nucleotides: each DP piece has its own limit */
    const int32_t *anchors; /* nanchors (x, y) pairs in genome order */
    int32_t nanchors;       /* >= 1 */
    int32_t k;              /* residues per anchor, >= 1 */
    uint32_t flags;         /* MPG_WANT_TB for this chain (OR-ed with params.flags) */
    int32_t _pad;
} mpg_chain;

/*
 * Align n chains (Methods, opening paragraph; "Residue alignment with dynamic
 * programming"): the DP closes the gaps between consecutive anchors and
 * extends from the first and the last anchor.  Per chain:
 *  - anchors become runs: an anchor on the current run's diagonal
 *    (x - x0 == 3 (y - y0)) that overlaps or abuts it extends the run; one
 *    that starts at or after the run's end in both sequences starts a new
 *    run; any other anchor is dropped;
 *  - every run is aligned as M steps (codon against residue, scored by the
 *    matrix); the pieces between are DP calls of their own, all chains'
 *    pieces in one batch: P[0, y_1) x T[0, x_1) in MPG_EXTEND_LEFT, each gap
 *    P[y_t + l_t, y_{t+1}) x T[x_t + 3 l_t, x_{t+1}) in MPG_GLOBAL, and
 *    P[y_R + l_R, m) x T[x_R + 3 l_R, n) in MPG_EXTEND, with p's scoring
 *    (p->mode is not used; bases outside a piece count as N);
 *  - out[c]: the sum of the runs' and the pieces' scores, the alignment from
 *    the left piece's start (traceback only, else -1) to the right piece's
 *    end in the chain's coordinates, and (traceback) the joined op string,
 *    adjacent M tokens merged.  A piece that fails fails the chain with its
 *    status (MPG_E_NOALN: a gap with no end-to-end path; MPG_E_RANGE: a piece
 *    beyond the limits or the traceback budget, or a protein longer than
 *    MPG_MAX_PROT).
 * The call fails with MPG_E_INVAL for a chain without anchors, k < 1 or an
 * anchor outside its sequences.  Synchronous; strings and anchors are
 * borrowed for the call; ops strings are released with mpg_result_release.
 */
int mpg_align_chains(mpg_ctx *ctx, const mpg_params *p, const mpg_chain *chains, int32_t n,
                     mpg_result *out);

/* One chain whose letters already sit in device memory (offsets into the
 * caller's concatenated device buffers, as mpg_seg); the anchors stay in host
 * memory. */
typedef struct {
    int64_t prot_off;
    int64_t dna_off;
    int32_t plen;
    int32_t dlen;
    const int32_t *anchors; /* host memory: nanchors (x, y) pairs in genome order */
    int32_t nanchors;
    int32_t k;
    uint32_t flags;         /* MPG_WANT_TB */
    int32_t _pad;
} mpg_chain_seg;

/* Bytes of op-string buffer mpg_align_chains_dev needs: chains take
 * consecutive slots in input order, 2*(plen+dlen)+1 bytes for a traceback
 * chain (params.flags or the chain's flags) and 1 byte otherwise. */
int64_t mpg_chain_ops_capacity(const mpg_params *p, const mpg_chain_seg *chains, int32_t n);

/* As mpg_align_chains for chains whose letters are in device memory: plans on
 * the host, enqueues everything on the context's stream and returns without
 * waiting.  d_out (device, n records) and d_ops (device, ops_cap bytes)
 * receive the results; each record's ops_off locates its op string.  The
 * device buffers must stay valid until the stream has finished; the anchors
 * are read before the call returns.  MPG_E_RANGE if ops_cap is too small.
 * A call of 2,048 chains or more runs in two halves on two workspaces of its
 * own: the host plans the second half while the device runs the first, and
 * waits only for the previous call's use of each workspace, not for the whole
 * stream.  Every chain is checked before any work is enqueued. */
int mpg_align_chains_dev(mpg_ctx *ctx, const mpg_params *p, const uint8_t *d_prot,
                         const uint8_t *d_dna, const mpg_chain_seg *chains, int32_t n,
                         mpg_dev_result *d_out, char *d_ops, int64_t ops_cap);

/* ---- position-specific (profile) queries ---------------------------------- */

/*
 * A query given as a profile instead of a protein and one matrix: the
 * position-specific substitution and gap costs that the paper's Discussion
 * names for profile queries (HMMER families).  For columns j = 1..m:
 *   score[24*(j-1) + a]  the score of a codon translating to amino acid a
 *                        (order of mpg_params.mat) at column j;
 *   gap[4*j + 0], [4*j + 1]  open and extend cost of column j's residue
 *                        against no genome: I(i,j) = max(H(i,j-1) - open,
 *                        I(i,j-1)) - extend;
 * and for columns j = 0..m:
 *   gap[4*j + 2], [4*j + 3]  open and extend cost of codons against no
 *                        residue after column j: D(i,j) = max(H(i-3,j) - open,
 *                        D(i-3,j)) - extend.
 * (gap[0], gap[1] are unused.)  Costs lie in [0, 8191], and each used
 * open + extend pair is at least 1.  f, r, the splice tables, the genetic
 * code, the mode and the flags come from mpg_params; its q, e and mat are not
 * used.  A profile made of the matrix rows of a protein's residues with
 * uniform costs q, e gives exactly the protein's results.
 */
typedef struct {
    const int8_t *score;  /* m x 24 */
    const int16_t *gap;   /* (m + 1) x 4 */
    int32_t m;
    const char *dna;
    int32_t dlen;
    uint32_t flags;       /* MPG_WANT_TB for this pair (OR-ed with params.flags) */
} mpg_profile_pair;

/* Align n profile queries to their regions (as mpg_align_batch; the int16
 * kernel is not used).  MPG_E_INVAL for a cost outside the rules above. */
int mpg_align_profiles(mpg_ctx *ctx, const mpg_params *p, const mpg_profile_pair *pairs,
                       int32_t n, mpg_result *out);

/* Bytes of the device layout of one profile: the m x 24 scores, zero-padded
 * to a multiple of 8 bytes, then the (m + 1) x 4 gap costs. */
int64_t mpg_profile_bytes(int32_t m);

/* A profile query already in device memory. */
typedef struct {
    int64_t prof_off;  /* byte offset of the profile (mpg_profile_bytes layout) in d_prof;
                          a multiple of 8 */
    int64_t dna_off;   /* offset of the region in d_dna */
    int32_t m;
    int32_t dlen;
    uint32_t flags;    /* MPG_WANT_TB */
    int32_t smax;      /* >= every score entry, >= 0 */
    int32_t pmax;      /* >= every used open + extend pair and >= -(every score entry) */
    int32_t _pad;
} mpg_profile_seg;

/* As mpg_align_batch_dev for profile queries in device memory.  The library
 * cannot read them before the launch: smax and pmax are taken as given (they
 * size the score-bound check), and the cost rules above are the caller's to
 * keep; values outside them give wrong results, never a fault. */
int mpg_align_profiles_dev(mpg_ctx *ctx, const mpg_params *p, const uint8_t *d_prof,
                           const uint8_t *d_dna, const mpg_profile_seg *segs, int32_t n,
                           mpg_dev_result *d_out, char *d_ops, int64_t ops_cap);

/* ---- chaining ------------------------------------------------------------- */

/*
 * Chaining of seed anchors (Methods, "Chaining").  Anchor (x, y): genome
 * position x (a 256-bp bin when binned, else a base) and residue y.  For
 * anchors sorted by x, then y, with dx = x_j - x_i, dy = y_j - y_i (i may
 * precede j only if dx >= 0 and dy > 0):
 *   g(i,j) = 3dy - 256(dx-1) if 3dy < 256(dx-1); 3dy - 256(dx+1) if
 *            3dy > 256(dx+1); else 0 (Eq. (gap), binned); 3dy - dx otherwise
 *            (the base-resolution second round);
 *   gamma(g) = 0 (g = 0), infinite (|g| >= G), g/3 + beta log2(g+1) (g > 0),
 *            min(|g|/3, beta log2(|g|+1)) (g < 0) (Eq. (gap-pen));
 *   f(j) = max(k, max_i f(i) + min(dy, k) - gamma(g(i,j))), pred(j) the first
 *          i reaching it or -1.
 * All in fp64.  Chains: the unused anchor of largest f (ties: smaller index)
 * starts a chain that follows pred until -1 or a used anchor; its score is
 * f(end) minus f(that anchor) (or 0).  Chains are ranked by score (ties: the
 * earlier extracted) and the first max_chains are reported.
 */
typedef struct {
    int32_t k;          /* anchor length in residues (6) */
    int32_t G;          /* largest gap (200,000) */
    double beta;        /* weight of the log term (0.75) */
    int32_t binned;     /* 1: x in 256-bp bins; 0: x in bases */
    int32_t max_chains; /* chains reported per set (30) */
} mpg_chaining_params;

void mpg_chaining_params_default(mpg_chaining_params *cp);

/* One reported chain: its score and its anchors idx[first .. first+len) of
 * the set's range of idx (anchor indices within the set, ascending). */
typedef struct {
    double score;
    int32_t first;
    int32_t len;
} mpg_chain_out;

#define MPG_MAX_ANCHORS 65536 /* anchors of one set */

/*
 * Chain nsets anchor sets on the GPU.  anchors: 2 int32 per anchor (x, y), all
 * sets concatenated; set s is anchors[set_off[s] .. set_off[s+1]) (set_off has
 * nsets + 1 ascending entries, set_off[0] = 0), sorted by x then y.  Outputs
 * are indexed like the anchors: f and pred (pred relative to the set), idx
 * (the extracted chains' anchors); top holds max_chains records per set and
 * ntop[s] the number reported, or MPG_E_RANGE for a set of more than
 * MPG_MAX_ANCHORS anchors.  The call fails with MPG_E_INVAL for a set that is
 * not sorted or bad parameters (k < 1, G < 1, beta < 0, max_chains < 1).
 * Host memory, synchronous.
 */
int mpg_chain_anchors(mpg_ctx *ctx, const mpg_chaining_params *cp, const int32_t *anchors,
                      const int64_t *set_off, int32_t nsets, double *f, int32_t *pred,
                      int32_t *idx, mpg_chain_out *top, int32_t *ntop);

/* As mpg_chain_anchors with anchors and every output in device memory
 * (set_off stays in host memory); enqueued on the context's stream.  Sets
 * are not checked for order: an unsorted set gives unspecified chains. */
int mpg_chain_anchors_dev(mpg_ctx *ctx, const mpg_chaining_params *cp, const int32_t *d_anchors,
                          const int64_t *set_off, int32_t nsets, double *d_f, int32_t *d_pred,
                          int32_t *d_idx, mpg_chain_out *d_top, int32_t *d_ntop);

/* ---- serving ------------------------------------------------------------ */

/*
 * Submit one job.  The sequences are copied before the call returns.  All
 * jobs of one context must use the same params (the first submit fixes them;
 * a different set returns MPG_E_INVAL).  A job whose traceback bytes exceed
 * the traceback budget returns MPG_E_RANGE (for a long job, more than 2e8
 * cells, 7/8 of the budget: the rest is kept for short jobs); a full queue
 * returns MPG_E_AGAIN.  *job_id receives the job's id.  Thread-safe against
 * mpg_poll.
 *
 * Scheduling: short and long jobs, with and without traceback, wait in four
 * queues.  Short jobs run in batches of up to 2e9 cells on three streams;
 * long jobs are gathered into batches of their own on four more streams, so
 * a short job never shares a launch with a long pair, and new long pairs
 * start while earlier ones still run.  Within a batch every pair completes on
 * its own: the wavefront that finishes a pair's last strip walks its
 * traceback and publishes the result to host-mapped memory, and the result
 * is in mpg_poll at once, while the rest of the batch still runs.  Streams
 * run concurrently only with hardware queues of their own: the context keeps
 * no more serving streams than the process's GPU_MAX_HW_QUEUES (HIP's
 * default is 4: three short lanes and one long lane; start the process with
 * GPU_MAX_HW_QUEUES of at least 8 for all seven), reported in mpg_stats.
 * A batch that fails (device memory, a HIP call, a bounded wait that gives
 * up) completes each of its jobs with that status; none is lost.
 */
int mpg_submit(mpg_ctx *ctx, const mpg_params *p, const mpg_pair *pair, uint64_t *job_id);

/* Move up to max_results finished jobs into out, in completion order, waiting
 * at most timeout_us microseconds for the first one (0 = do not wait).
 * Returns the number of results (>= 0) or a negative status.  Each result's
 * ops string is owned by the library until mpg_result_release. */
int mpg_poll(mpg_ctx *ctx, mpg_result *out, int32_t max_results, int32_t timeout_us);

/* Cancel a job that has not been admitted to the device yet; it completes
 * with status MPG_E_CANCELLED.  MPG_E_INVAL if unknown or already running. */
int mpg_cancel(mpg_ctx *ctx, uint64_t job_id);

/* Serving statistics (all counters since ctx creation). */
typedef struct {
    uint64_t submitted, completed, cancelled, rejected_again, rejected_range;
    uint64_t batches, cells;
    uint64_t queue_depth;   /* jobs submitted but not yet admitted */
    uint64_t in_flight;     /* jobs admitted to the device, not yet completed */
    uint64_t tb_bytes_in_use, tb_bytes_peak, tb_budget;
    uint64_t short_streams, long_streams; /* serving lanes in use (capped by the process's
                                             hardware queues, GPU_MAX_HW_QUEUES) */
} mpg_stats;
int mpg_get_stats(mpg_ctx *ctx, mpg_stats *st);

/* ---- kernel timing ------------------------------------------------------- */

/* Cumulative device time of the batch calls of this context, measured with
 * hipEvents on the context's stream around the prepass kernel, the DP kernels
 * and the traceback walk (only while timing is enabled). */
typedef struct {
    double prepass_ms, dp_ms, walk_ms;
    uint64_t dp_spans; /* number of timed DP spans (one per batch wave) */
    uint64_t calls;    /* batch calls since the last reset */
    double host_ms;    /* host wall time planning and enqueuing the device work */
    uint64_t i16_pairs; /* pairs that ran in the lane-packed int16 kernel */
    uint64_t cells;     /* DP cells (genome length x protein length) of the pairs run */
    uint64_t seg_packs; /* wavefronts that ran two pairs' last strips side by side */
} mpg_timing;

/* Turn event timing of batch calls on (1) or off (0). */
int mpg_enable_timing(mpg_ctx *ctx, int on);

/* Wait for the timed work, fill *t, and zero the counters if reset != 0. */
int mpg_get_timing(mpg_ctx *ctx, mpg_timing *t, int reset);

/* ---- planned batches: graph capture and replay ------------------------------ */

typedef struct mpg_plan mpg_plan;

/*
 * Plan a device-resident batch once (as mpg_align_batch_dev, and bound to the
 * same buffers: d_prot, d_dna, d_out, d_ops), so that it can be run many
 * times with no host work.  All planning, allocation and uploads happen
 * here; the plan owns its device workspace.  The direction bits of all
 * traceback pairs must fit the context's traceback budget at once
 * (MPG_E_RANGE otherwise).  Each run recomputes everything from the bound
 * inputs, so the caller may change the letters in d_prot/d_dna between runs
 * as long as the lengths stay the same.
 */
int mpg_plan_create(mpg_ctx *ctx, const mpg_params *p, const uint8_t *d_prot, const uint8_t *d_dna,
                    const mpg_seg *segs, int32_t n, mpg_dev_result *d_out, char *d_ops,
                    int64_t ops_cap, mpg_plan **plan);

/* Run a plan on hip_stream (NULL = the context's stream): kernel launches
 * only, no host synchronisation, allocation or memset, so the call may
 * itself be captured into a caller's graph.  Once mpg_plan_graph has
 * succeeded, the captured graph is replayed instead. */
int mpg_plan_launch(mpg_plan *plan, void *hip_stream);

/* Capture one run of the plan on hip_stream (a stream the caller created;
 * not the null stream) into a hipGraph and instantiate it; later
 * mpg_plan_launch calls replay it with one hipGraphLaunch. */
int mpg_plan_graph(mpg_plan *plan, void *hip_stream);

/* Wait for the plan's work and free it. */
void mpg_plan_destroy(mpg_plan *plan);

/* ---- autotuning ----------------------------------------------------------- */

/* DP rates (GCUPS) of a sample batch under each planning choice tried, and
 * the choices kept. */
typedef struct {
    double gcups[3];     /* int32 kernels at 1, 2, 4 columns per lane (every pair) */
    double i16_gcups[2]; /* int16 lanes at 1, 2 columns per lane (0 if not tried) */
    int32_t K, K16;      /* the widths this context uses from now on */
    int32_t narrow_cols; /* pairs of at most this many columns (residues + 1) run one
                            column per lane (1: none but the empty protein) */
    int32_t seg_packs;   /* 1: two pairs' ragged last strips may share a wavefront */
    double narrow_gcups[4]; /* at width K with the cutover at 64, 128, 192 and 1 columns
                               (0 if not tried: at K = 1 it changes nothing) */
    double seg_gcups[2];    /* at width K and the kept cutover, packs off and on */
} mpg_tuning;

/*
 * Run a sample of the caller's workload at every kernel width, then, at the
 * fastest width, with the narrow-pair cutover at 64, 128, 192 and 1 columns and
 * with lane-segment packs off and on, and keep the fastest choices for the
 * batch calls of this context.  The sample is given like
 * mpg_align_batch_dev's input (letters in device memory, n segments, params
 * p; MPG_ALLOW_I16 in p also tunes the int16 width); with n = 0 a built-in
 * sample is used (1,024 pairs of 511 residues x 4,096 nucleotides, half with
 * traceback; p, d_prot, d_dna and segs may then be NULL).  Each choice runs
 * three times and the faster of the last two DP times counts.  Results never
 * depend on these choices.  Serving uses its own width (the narrowest, for the shortest per-pair
 * critical path).  Call it while no other work of the context is in flight.
 * out may be NULL.
 */
int mpg_autotune(mpg_ctx *ctx, const mpg_params *p, const uint8_t *d_prot, const uint8_t *d_dna,
                 const mpg_seg *segs, int32_t n, mpg_tuning *out);

/* Release the ops strings of n results returned by this context. */
void mpg_result_release(mpg_ctx *ctx, mpg_result *r, int32_t n);

const char *mpg_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* MPG_H */
