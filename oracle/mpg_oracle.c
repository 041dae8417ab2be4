/*
 * Oracle for the spliced protein-to-genome DP -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously-correct CPU reference against which
 * the GPU library is checked.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU library.
 *
 * What it computes (Li 2022, "Protein-to-genome alignment with miniprot",
 * Methods, subsection "DP for protein-to-genome alignment", Eq. (full)):
 * a full (n+1) x (m+1) matrix DP over genome rows i and protein columns j with
 * six states per cell, in int64 arithmetic:
 *
 *   I(i,j) = max{ H(i,j-1) - q, I(i,j-1) } - e
 *   D(i,j) = max{ H(i-3,j) - q, D(i-3,j) } - e
 *   A(i,j) = max{ H(i-1,j) - r - d(i-1), A(i-1,j) }
 *   B(i,j) = max{ H(i-1,j-1) - r - d(i), B(i-1,j) }
 *   C(i,j) = max{ H(i-1,j-1) - r - d(i+1), C(i-1,j) }
 *   H(i,j) = max{ H(i-3,j-1) + s(i,j), I, D, H(i-1,j-1)-f, H(i-2,j-1)-f,
 *                 H(i-1,j)-f, H(i-2,j)-f, A-a(i), B-a(i-2), C-a(i-1) }
 *
 * Readings of the paper that this file follows:
 *  - the printed match term H(i-3,j)+s(i,j) consumes no residue and would
 *    duplicate D at zero gap cost; the codon:residue step is H(i-3,j-1)+s(i,j)
 *    (the AE86 form, Eq. (ae86), uses H(i-1,j-1)+s, and the worked alignment
 *    in the same subsection pairs every codon with one residue);
 *  - s(i,j) scores the codon ending at genome position i, T[i-2..i], translated
 *    by the genetic code, against P[j]; a codon containing N translates to X;
 *  - d(x) is a table over the 3-mer T[x+1..x+3] and a(x) over T[x-2..x]
 *    (the splice models of the "Splice models" subsection), bases outside
 *    [1,n] count as N;
 *  - four boundary modes: LOCAL (0 floor at every cell, free end), EXTEND
 *    (start at H(0,0)=0, free end), GLOBAL (start at H(0,0)=0, end (n,m)) and
 *    EXTEND_LEFT (0 floor at every cell, end (n,m)).  The DP closes gaps
 *    between anchors (GLOBAL) and extends from terminal anchors (Methods,
 *    opening paragraph; "Residue alignment with dynamic programming"): to
 *    the right an extension starts at the anchor and ends anywhere
 *    (EXTEND); to the left it starts anywhere and ends at the anchor
 *    (EXTEND_LEFT);
 *  - ties: H takes the first maximum in the order
 *    [start, M, I, D, F1, F2, G1, G2, A, B, C]; I/D/A/B/C prefer extension
 *    over opening on ties; the end cell is the first maximum in row-major
 *    order (smallest i, then smallest j);
 *  - traceback stops at the first H cell whose winner is "start".
 *
 * Sentinel: unreachable values are exactly NEG; pen()/addsc() keep NEG fixed.
 *
 * Parity unpinned: the paper fixes neither the tie-break order above, nor the
 * op-string format, nor the default q/e/f/r and matrix, nor how the DP is
 * bounded at its start and end.  The optimal score of every mode is pinned
 * (brute force over the segment grammar, textbook Gotoh reduction, the worked
 * alignment of "Residue alignment with dynamic programming"); which of several optimal paths
 * and end cells is reported, and how it is spelled, follows the choices above
 * and is checked only for validity (rescoring) and against itself.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NEG (-((int64_t)1 << 62))

/* H winner codes, in tie-break order. */
enum { C_START = 0, C_M, C_I, C_D, C_F1, C_F2, C_G1, C_G2, C_A, C_B, C_C };
/* extension bits stored above the 4-bit H code */
#define X_I (1u << 4)
#define X_D (1u << 5)
#define X_A (1u << 6)
#define X_B (1u << 7)
#define X_C (1u << 8)

enum { ORC_LOCAL = 0, ORC_EXTEND = 1, ORC_GLOBAL = 2, ORC_EXTEND_LEFT = 3 };
enum { ORC_NO_INTRON = 1, ORC_NO_FS = 2 };

static const char ORC_AA[] = "ARNDCQEGHILKMFPSTWYVBZX*";

/* ---- encodings (case-insensitive; unknown DNA -> N=4, unknown aa -> X) -- */
int orc_dna_code(int ch)
{
    switch (ch) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return 4;
    }
}

int orc_aa_code(int ch)
{
    int k;
    if (ch >= 'a' && ch <= 'z') ch -= 32;
    for (k = 0; k < 24; ++k)
        if (ORC_AA[k] == ch) return k;
    return 22; /* X */
}

typedef struct {
    int64_t q, e, f, r;
    int no_intron, no_fs, mode;
    const int8_t *mat;       /* 24 x 24, mat[a * 24 + b] */
    const uint8_t *gcode;    /* codon 16*b1+4*b2+b3 (ACGT = 0..3) -> aa code */
    const uint8_t *donor;    /* 125, index 25*b1+5*b2+b3 over ACGTN */
    const uint8_t *acceptor; /* 125 */
    const uint8_t *T;        /* genome codes, T[1..n] (T[0] unused) */
    const uint8_t *P;        /* protein codes, P[1..m] */
    int n, m;
} orc_ctx;

static int base_at(const orc_ctx *c, long x)
{
    return (x >= 1 && x <= c->n) ? c->T[x] : 4;
}

/* amino acid of the codon ending at row i (T[i-2..i]); X if any base is N */
static int tr_at(const orc_ctx *c, long i)
{
    int b1 = base_at(c, i - 2), b2 = base_at(c, i - 1), b3 = base_at(c, i);
    if (b1 == 4 || b2 == 4 || b3 == 4) return 22;
    return c->gcode[16 * b1 + 4 * b2 + b3];
}

/* donor penalty d(x): 3-mer T[x+1..x+3] */
static int64_t d_at(const orc_ctx *c, long x)
{
    return c->donor[25 * base_at(c, x + 1) + 5 * base_at(c, x + 2) + base_at(c, x + 3)];
}

/* acceptor penalty a(x): 3-mer T[x-2..x] */
static int64_t a_at(const orc_ctx *c, long x)
{
    return c->acceptor[25 * base_at(c, x - 2) + 5 * base_at(c, x - 1) + base_at(c, x)];
}

static int64_t pen(int64_t v, int64_t c) { return v == NEG ? NEG : v - c; }
static int64_t addsc(int64_t v, int64_t s) { return v == NEG ? NEG : v + s; }

/* rolling row storage: 4 rows, row i lives in slot i & 3 */
typedef struct {
    int64_t *H, *I, *D, *A, *B, *C;
    int w; /* m + 1 */
} rows_t;

#define AT(arr, i, j) ((arr)[(size_t)((i) & 3) * (size_t)rw.w + (size_t)(j)])

static int64_t getH(const rows_t *r, long i, long j)
{
    if (i < 0 || j < 0) return NEG;
    return r->H[(size_t)(i & 3) * (size_t)r->w + (size_t)j];
}
static int64_t getS(const int64_t *a, const rows_t *r, long i, long j)
{
    if (i < 0 || j < 0) return NEG;
    return a[(size_t)(i & 3) * (size_t)r->w + (size_t)j];
}

/* one token of the op string, kept in reverse order during the walk */
typedef struct { char op; int64_t len; } tok_t;

static int emit(tok_t **v, int64_t *nv, int64_t *cap, char op, int64_t len, int mergeable)
{
    if (mergeable && *nv > 0 && (*v)[*nv - 1].op == op) {
        (*v)[*nv - 1].len += len;
        return 0;
    }
    if (*nv == *cap) {
        int64_t nc = *cap ? *cap * 2 : 64;
        tok_t *nb = (tok_t *)realloc(*v, (size_t)nc * sizeof(tok_t));
        if (!nb) return -1;
        *v = nb;
        *cap = nc;
    }
    (*v)[*nv].op = op;
    (*v)[*nv].len = len;
    ++*nv;
    return 0;
}

/*
 * orc_align: align protein P (ASCII, length m) to genome T (ASCII, length n).
 * out[0..4] = score, g_beg, g_end, p_beg, p_end (begins are -1 without traceback).
 * ops: buffer for the run-length op string (NUL-terminated), ops_cap bytes.
 * Returns 0, -6 (GLOBAL end unreachable), -3 (out of memory), -2 (ops buffer
 * too small) or -1 (unknown mode).
 */
static int align_core(const char *prot, int32_t m, const char *dna, int32_t n,
                      int64_t q, int64_t e, int64_t f, int64_t r, int32_t flags, int32_t mode,
                      const int8_t *mat, const int8_t *S, const int16_t *gap,
                      const uint8_t *gcode, const uint8_t *donor, const uint8_t *acceptor,
                      int32_t want_tb, int64_t *out, char *ops, int64_t ops_cap,
                      int64_t *ops_len);

int orc_align(const char *prot, int32_t m, const char *dna, int32_t n,
              int64_t q, int64_t e, int64_t f, int64_t r, int32_t flags, int32_t mode,
              const int8_t *mat, const uint8_t *gcode, const uint8_t *donor,
              const uint8_t *acceptor, int32_t want_tb,
              int64_t *out, char *ops, int64_t ops_cap, int64_t *ops_len)
{
    return align_core(prot, m, dna, n, q, e, f, r, flags, mode, mat, NULL, NULL, gcode, donor,
                      acceptor, want_tb, out, ops, ops_cap, ops_len);
}

/*
 * orc_align_profile: the same DP with a position-specific query of m columns
 * in place of a protein and one matrix (the paper's outlook on profile
 * queries: position-specific substitution and gap costs, Discussion).
 *   S[24*(j-1) + a]  score of a codon translating to a at column j (1..m);
 *   gap[4*j + 0, 1]  I open and extend at column j (1..m): residue j against
 *                    no genome, I(i,j) = max(H(i,j-1) - o, I(i,j-1)) - x;
 *   gap[4*j + 2, 3]  D open and extend at column j (0..m): codons against no
 *                    residue after column j, D(i,j) = max(H(i-3,j) - o, D(i-3,j)) - x.
 * f, r and the splice tables are those of the uniform DP.
 */
int orc_align_profile(const int8_t *S, const int16_t *gap, int32_t m, const char *dna, int32_t n,
                      int64_t f, int64_t r, int32_t flags, int32_t mode, const uint8_t *gcode,
                      const uint8_t *donor, const uint8_t *acceptor, int32_t want_tb,
                      int64_t *out, char *ops, int64_t ops_cap, int64_t *ops_len)
{
    return align_core(NULL, m, dna, n, 0, 0, f, r, flags, mode, NULL, S, gap, gcode, donor,
                      acceptor, want_tb, out, ops, ops_cap, ops_len);
}

static int align_core(const char *prot, int32_t m, const char *dna, int32_t n,
                      int64_t q, int64_t e, int64_t f, int64_t r, int32_t flags, int32_t mode,
                      const int8_t *mat, const int8_t *S, const int16_t *gap,
                      const uint8_t *gcode, const uint8_t *donor, const uint8_t *acceptor,
                      int32_t want_tb, int64_t *out, char *ops, int64_t ops_cap,
                      int64_t *ops_len)
{
    orc_ctx c;
    rows_t rw;
    uint16_t *code = NULL;
    uint8_t *T = NULL, *P = NULL;
    int64_t best = NEG;
    long bi = 0, bj = 0;
    long i, j;
    int status = 0;
    const int64_t w = (int64_t)m + 1;

    if (mode < ORC_LOCAL || mode > ORC_EXTEND_LEFT) return -1;
    const int floor0 = mode == ORC_LOCAL || mode == ORC_EXTEND_LEFT;
    const int fixed_end = mode == ORC_GLOBAL || mode == ORC_EXTEND_LEFT;
    memset(&c, 0, sizeof c);
    c.q = q; c.e = e; c.f = f; c.r = r;
    c.no_intron = (flags & ORC_NO_INTRON) != 0;
    c.no_fs = (flags & ORC_NO_FS) != 0;
    c.mode = mode;
    c.mat = mat; c.gcode = gcode; c.donor = donor; c.acceptor = acceptor;
    c.n = n; c.m = m;

    T = (uint8_t *)malloc((size_t)n + 1);
    P = (uint8_t *)malloc((size_t)m + 1);
    rw.w = (int)w;
    rw.H = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)w);
    rw.I = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)w);
    rw.D = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)w);
    rw.A = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)w);
    rw.B = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)w);
    rw.C = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)w);
    if (want_tb) code = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)(n + 1) * (size_t)w);
    if (!T || !P || !rw.H || !rw.I || !rw.D || !rw.A || !rw.B || !rw.C || (want_tb && !code)) {
        status = -3;
        goto done;
    }
    for (i = 1; i <= n; ++i) T[i] = (uint8_t)orc_dna_code((unsigned char)dna[i - 1]);
    for (j = 1; j <= m; ++j) P[j] = S ? 0 : (uint8_t)orc_aa_code((unsigned char)prot[j - 1]);
    c.T = T; c.P = P;

    for (i = 0; i <= n; ++i) {
        const int64_t dm1 = d_at(&c, i - 1), d0 = d_at(&c, i), dp1 = d_at(&c, i + 1);
        const int64_t a0 = a_at(&c, i), am1 = a_at(&c, i - 1), am2 = a_at(&c, i - 2);
        const int tri = tr_at(&c, i);
        for (j = 0; j <= m; ++j) {
            uint16_t cc = 0;
            int64_t Iv = NEG, Dv = NEG, Av = NEG, Bv = NEG, Cv = NEG;
            int64_t cand[11];
            int64_t h;
            int k, win;

            /* I: one residue against no genome */
            if (j >= 1) {
                int64_t op = pen(getH(&rw, i, j - 1), gap ? gap[4 * j] : q);
                int64_t ex = getS(rw.I, &rw, i, j - 1);
                if (ex >= op) { Iv = ex; cc |= X_I; } else Iv = op;
                Iv = pen(Iv, gap ? gap[4 * j + 1] : e);
            }
            /* D: one codon (3 nt) against no residue */
            if (i >= 3) {
                int64_t op = pen(getH(&rw, i - 3, j), gap ? gap[4 * j + 2] : q);
                int64_t ex = getS(rw.D, &rw, i - 3, j);
                if (ex >= op) { Dv = ex; cc |= X_D; } else Dv = op;
                Dv = pen(Dv, gap ? gap[4 * j + 3] : e);
            }
            if (!c.no_intron && i >= 1) {
                /* A: phase-0 intron, opened from H(i-1,j) */
                {
                    int64_t op = pen(getH(&rw, i - 1, j), r + dm1);
                    int64_t ex = getS(rw.A, &rw, i - 1, j);
                    if (ex >= op) { Av = ex; cc |= X_A; } else Av = op;
                }
                /* B: phase-1 intron, opened from H(i-1,j-1) */
                {
                    int64_t op = pen(getH(&rw, i - 1, j - 1), r + d0);
                    int64_t ex = getS(rw.B, &rw, i - 1, j);
                    if (ex >= op) { Bv = ex; cc |= X_B; } else Bv = op;
                }
                /* C: phase-2 intron, opened from H(i-1,j-1) */
                {
                    int64_t op = pen(getH(&rw, i - 1, j - 1), r + dp1);
                    int64_t ex = getS(rw.C, &rw, i - 1, j);
                    if (ex >= op) { Cv = ex; cc |= X_C; } else Cv = op;
                }
            }

            /* H candidates in tie-break order */
            if (floor0) cand[C_START] = 0;
            else cand[C_START] = (i == 0 && j == 0) ? 0 : NEG;
            cand[C_M] = (i >= 3 && j >= 1)
                ? addsc(getH(&rw, i - 3, j - 1), S ? S[24 * (j - 1) + tri] : mat[tri * 24 + P[j]])
                : NEG;
            cand[C_I] = Iv;
            cand[C_D] = Dv;
            if (!c.no_fs) {
                cand[C_F1] = pen(getH(&rw, i - 1, j - 1), f);
                cand[C_F2] = pen(getH(&rw, i - 2, j - 1), f);
                cand[C_G1] = pen(getH(&rw, i - 1, j), f);
                cand[C_G2] = pen(getH(&rw, i - 2, j), f);
            } else {
                cand[C_F1] = cand[C_F2] = cand[C_G1] = cand[C_G2] = NEG;
            }
            cand[C_A] = pen(Av, a0);
            cand[C_B] = pen(Bv, am2);
            cand[C_C] = pen(Cv, am1);
            h = cand[0];
            win = 0;
            for (k = 1; k < 11; ++k)
                if (cand[k] > h) { h = cand[k]; win = k; }
            cc |= (uint16_t)win;

            AT(rw.H, i, j) = h;
            AT(rw.I, i, j) = Iv;
            AT(rw.D, i, j) = Dv;
            AT(rw.A, i, j) = Av;
            AT(rw.B, i, j) = Bv;
            AT(rw.C, i, j) = Cv;
            if (want_tb) code[(size_t)i * (size_t)w + (size_t)j] = cc;

            if (!fixed_end && h > best) { best = h; bi = i; bj = j; }
        }
    }
    if (fixed_end) {
        best = getH(&rw, n, m);
        bi = n; bj = m;
        if (best == NEG) { status = -6; goto done; }
    }

    out[0] = best; out[1] = -1; out[2] = bi; out[3] = -1; out[4] = bj;
    if (ops_len) *ops_len = 0;
    if (want_tb) {
        /* walk back from the end cell in state H */
        tok_t *tv = NULL;
        int64_t nt = 0, tcap = 0, pos = 0, t;
        long ci = bi, cj = bj, kend = 0;
        int st = 0; /* 0 = H, 1 = I, 2 = D, 3 = A, 4 = B, 5 = C */
        int err = 0;
        for (;;) {
            uint16_t cc = code[(size_t)ci * (size_t)w + (size_t)cj];
            if (st == 0) {
                int hc = cc & 15;
                if (hc == C_START) break;
                switch (hc) {
                case C_M: err |= emit(&tv, &nt, &tcap, 'M', 1, 1); ci -= 3; cj -= 1; break;
                case C_I: st = 1; break;
                case C_D: st = 2; break;
                case C_F1: err |= emit(&tv, &nt, &tcap, 'F', 1, 0); ci -= 1; cj -= 1; break;
                case C_F2: err |= emit(&tv, &nt, &tcap, 'F', 2, 0); ci -= 2; cj -= 1; break;
                case C_G1: err |= emit(&tv, &nt, &tcap, 'G', 1, 0); ci -= 1; break;
                case C_G2: err |= emit(&tv, &nt, &tcap, 'G', 2, 0); ci -= 2; break;
                case C_A: st = 3; kend = ci; break;
                case C_B: st = 4; kend = ci; break;
                default: st = 5; kend = ci; break;
                }
            } else if (st == 1) {
                err |= emit(&tv, &nt, &tcap, 'I', 1, 1);
                if (!(cc & X_I)) st = 0;
                cj -= 1;
            } else if (st == 2) {
                err |= emit(&tv, &nt, &tcap, 'D', 1, 1);
                if (!(cc & X_D)) st = 0;
                ci -= 3;
            } else {
                uint16_t xb = st == 3 ? X_A : st == 4 ? X_B : X_C;
                if (!(cc & xb)) {
                    /* opened here: the intron (plus split codon) spans rows ci..kend */
                    char op = st == 3 ? 'N' : st == 4 ? 'U' : 'V';
                    err |= emit(&tv, &nt, &tcap, op, (int64_t)(kend - ci + 1), 0);
                    if (st != 3) cj -= 1;
                    st = 0;
                }
                ci -= 1;
            }
            if (err) break;
            if (ci < 0 || cj < 0) { err = 1; break; } /* cannot happen on a valid path */
        }
        if (err) { free(tv); status = -3; goto done; }
        out[1] = ci; out[3] = cj;
        /* format tokens in forward order */
        for (t = nt - 1; t >= 0; --t) {
            char buf[32];
            int bl = 0, k2;
            int64_t L = tv[t].len;
            char tmp[24];
            int tl = 0;
            do { tmp[tl++] = (char)('0' + (int)(L % 10)); L /= 10; } while (L > 0);
            for (k2 = tl - 1; k2 >= 0; --k2) buf[bl++] = tmp[k2];
            buf[bl++] = tv[t].op;
            if (pos + bl + 1 > ops_cap) { free(tv); status = -2; goto done; }
            memcpy(ops + pos, buf, (size_t)bl);
            pos += bl;
        }
        if (ops_cap > 0) ops[pos] = 0;
        if (ops_len) *ops_len = pos;
        free(tv);
    }

done:
    free(T); free(P);
    free(rw.H); free(rw.I); free(rw.D); free(rw.A); free(rw.B); free(rw.C);
    free(code);
    return status;
}
