/*
 * CPU ORACLE for the PanDelos-plus best-hit path -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately literal implementation of what the paper defines:
 *   - k-mer windows, occurrences and multiplicities (Basic notions, Eqs.
 *     kmer_dictionary, kmer_occurrences, kmer_multiplicity);
 *   - the k rule of phase (a) (Eq. k_length);
 *   - the multiplicity vector of one gene (Multiplicity vector building phase,
 *     Alg. 1);
 *   - the generalised Jaccard similarity (Eq. jaccard_k), with both the sum of
 *     minima over the intersection and the sum of maxima over the union
 *     computed literally by merging two sorted multiplicity vectors;
 *   - the best hits of a gene in another genome, ties included (Eq. best_hit,
 *     Alg. 2), compared as exact rationals by 128-bit cross-multiplication;
 *   - bidirectional best hits by their set definition (Eq.
 *     bidirectional_best_hit) and, as a second path that must agree, by the
 *     column-maximum procedure of Alg. 3.
 *
 * Readings of passages the paper leaves silent or garbled (all documented with
 * the tests that pin them):
 *   - a gene of length L has max(0, L-k+1) windows g[p..p+k-1] (the count and
 *     indices that Alg. 1 uses);
 *   - J := 0 when both genes have no window (0/0);
 *   - a gene whose row maximum is J = 0 has no best hit (the BH set needs a
 *     maximum above zero, as the predecessor's minimum-overlap preselection
 *     implies);
 *   - the second condition of the BBH equation is read with genome G_i, as the
 *     sentence defining BBH says;
 *   - the k rule sums residues over the dataset and rounds up, computed in
 *     integers (smallest k with |alphabet|^k >= total); rounding down is mode 1.
 *
 * The paper's genes are strings over a nucleotide or an amino-acid alphabet
 * (Basic notions); both are supported: the 20 standard amino acids
 * ACDEFGHIKLMNPQRSTVWY (alphabet 0) and the four nucleotides ACGT (alphabet 1).
 * The k-mer identifier f used here is the base-|alphabet| value of the window,
 * each letter taking its index in the alphabet string below, first letter most
 * significant.  Best hits do not depend on the choice of f; only the order
 * inside a multiplicity vector does.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * use this file.  It shares nothing with the GPU library.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const char *const ORC_ALPHABETS[2] = {"ACDEFGHIKLMNPQRSTVWY", "ACGT"};
static const uint32_t ORC_SIGMA[2] = {20u, 4u};

/* Index of byte c in alphabet a (0: amino acids, 1: nucleotides), or -1 for any
 * other byte. */
static int orc_residue(unsigned char c, uint32_t a) {
    for (int i = 0; i < (int)ORC_SIGMA[a]; ++i)
        if ((unsigned char)ORC_ALPHABETS[a][i] == c) return i;
    return -1;
}

/* Largest k whose identifiers all fit 64 bits (|alphabet|^k <= 2^64), 0 for an
 * unknown alphabet. */
uint32_t orc_k_max(uint32_t a) {
    if (a > 1) return 0;
    uint32_t k = 0;
    unsigned __int128 p = 1;
    while (p * ORC_SIGMA[a] <= ((unsigned __int128)1 << 64)) { p *= ORC_SIGMA[a]; ++k; }
    return k;
}

/* ---------------------------------------------------------------- phase (a) */

/* Eq. k_length: k = log_{|alphabet|}(total).  mode 0: smallest k with
 * alphabet^k >= total; mode 1: largest k with alphabet^k <= total.  k >= 1.
 * Returns 0, or -1 for alphabet < 2. */
int orc_k_rule(uint64_t total, uint32_t alphabet, int mode, uint32_t *k_out) {
    if (alphabet < 2) return -1;
    uint32_t k = 0;
    unsigned __int128 p = 1; /* alphabet^k */
    if (mode == 0) {
        while (p < total) { p *= alphabet; ++k; }
    } else {
        while (p * alphabet <= total) { p *= alphabet; ++k; }
    }
    if (k < 1) k = 1;
    *k_out = k;
    return 0;
}

/* ------------------------------------------------------- multiplicity vectors */

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Number of windows of a gene of length len: max(0, len-k+1). */
int64_t orc_n_windows(int64_t len, uint32_t k) {
    return len >= (int64_t)k ? len - (int64_t)k + 1 : 0;
}

/* Alg. 1 for one gene over alphabet a: every window g[p..p+k-1] gets the
 * identifier f(alpha) (its base-|alphabet| value); the identifiers are grouped
 * by sorting, and each group becomes one (id, multiplicity) pair, ascending by
 * id.  ids/cnt must hold orc_n_windows(len, k) entries.  Returns the number of
 * distinct k-mers, -1 if a byte outside the alphabet occurs (its offset goes to
 * *bad), or -2 for an unknown alphabet or k outside 1..orc_k_max(a). */
int64_t orc_mv(const unsigned char *s, int64_t len, uint32_t k, uint32_t a, uint64_t *ids, uint32_t *cnt, int64_t *bad) {
    if (a > 1 || k < 1 || k > orc_k_max(a)) return -2;
    for (int64_t p = 0; p < len; ++p) {
        if (orc_residue(s[p], a) < 0) { if (bad) *bad = p; return -1; }
    }
    int64_t nw = orc_n_windows(len, k);
    if (nw == 0) return 0;
    uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nw);
    for (int64_t p = 0; p < nw; ++p) {
        uint64_t id = 0;
        for (uint32_t i = 0; i < k; ++i) id = id * ORC_SIGMA[a] + (uint64_t)orc_residue(s[p + i], a);
        w[p] = id;
    }
    qsort(w, (size_t)nw, sizeof(uint64_t), cmp_u64);
    int64_t d = 0;
    for (int64_t p = 0; p < nw; ++p) {
        if (d > 0 && ids[d - 1] == w[p]) {
            cnt[d - 1] += 1;
        } else {
            ids[d] = w[p];
            cnt[d] = 1;
            ++d;
        }
    }
    free(w);
    return d;
}

/* All multiplicity vectors of one genome, in CSR form. */
typedef struct {
    uint32_t n, k;
    uint64_t *ptr;   /* n+1 */
    uint64_t *ids;   /* ptr[n] */
    uint32_t *cnt;   /* ptr[n] */
    uint64_t *nwin;  /* n: windows of each gene */
    uint64_t *len;   /* n: residues of each gene (Eq. length_threshold compares these) */
} orc_genome;

void orc_genome_free(orc_genome *g) {
    if (!g) return;
    free(g->ptr); free(g->ids); free(g->cnt); free(g->nwin); free(g->len); free(g);
}

/* Builds the multiplicity vector of every gene (genes are residues[off[i]..off[i+1])) over
 * alphabet a.  Returns NULL on a byte outside the alphabet (*bad = its offset in residues)
 * or on an unknown alphabet or k outside 1..orc_k_max(a) (*bad = -2). */
orc_genome *orc_genome_new(const unsigned char *residues, const uint64_t *off, uint32_t n, uint32_t k, uint32_t a,
                           int64_t *bad) {
    if (a > 1 || k < 1 || k > orc_k_max(a)) {
        if (bad) *bad = -2;
        return NULL;
    }
    orc_genome *g = (orc_genome *)calloc(1, sizeof(orc_genome));
    g->n = n; g->k = k;
    g->ptr = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    g->nwin = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    g->len = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    uint64_t cap = 0;
    for (uint32_t i = 0; i < n; ++i) {
        g->len[i] = off[i + 1] - off[i];
        g->nwin[i] = (uint64_t)orc_n_windows((int64_t)(off[i + 1] - off[i]), k);
        cap += g->nwin[i];
    }
    g->ids = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(cap + 1));
    g->cnt = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cap + 1));
    uint64_t pos = 0;
    for (uint32_t i = 0; i < n; ++i) {
        g->ptr[i] = pos;
        int64_t b = -1;
        int64_t d = orc_mv(residues + off[i], (int64_t)(off[i + 1] - off[i]), k, a, g->ids + pos, g->cnt + pos, &b);
        if (d < 0) {
            if (bad) *bad = (int64_t)off[i] + b;
            orc_genome_free(g);
            return NULL;
        }
        pos += (uint64_t)d;
    }
    g->ptr[n] = pos;
    return g;
}

uint32_t orc_genome_n(const orc_genome *g) { return g->n; }
uint64_t orc_genome_entries(const orc_genome *g) { return g->ptr[g->n]; }
const uint64_t *orc_genome_ptr(const orc_genome *g) { return g->ptr; }
const uint64_t *orc_genome_ids(const orc_genome *g) { return g->ids; }
const uint32_t *orc_genome_cnt(const orc_genome *g) { return g->cnt; }
const uint64_t *orc_genome_nwin(const orc_genome *g) { return g->nwin; }

/* ---------------------------------------------------------- Eq. jaccard_k */

/* Numerator and denominator of the generalised Jaccard similarity of two
 * genes given by ascending multiplicity vectors: *smin = sum over k-mers in
 * both dictionaries of min(mult_a, mult_b); *smax = sum over k-mers in either
 * dictionary of max(mult_a, mult_b) (a k-mer absent from a gene has
 * multiplicity 0 there). */
void orc_jaccard_terms(const uint64_t *ia, const uint32_t *ca, uint64_t na,
                       const uint64_t *ib, const uint32_t *cb, uint64_t nb,
                       uint64_t *smin, uint64_t *smax) {
    uint64_t i = 0, j = 0, mn = 0, mx = 0;
    while (i < na || j < nb) {
        if (j >= nb || (i < na && ia[i] < ib[j])) {
            mx += ca[i];               /* only in a */
            ++i;
        } else if (i >= na || ib[j] < ia[i]) {
            mx += cb[j];               /* only in b */
            ++j;
        } else {                       /* in both */
            mn += ca[i] < cb[j] ? ca[i] : cb[j];
            mx += ca[i] > cb[j] ? ca[i] : cb[j];
            ++i; ++j;
        }
    }
    *smin = mn;
    *smax = mx;
}

/* Three-way comparison of J1 = m1/d1 and J2 = m2/d2, with J = 0 when d = 0. */
static int orc_cmp_j(uint64_t m1, uint64_t d1, uint64_t m2, uint64_t d2) {
    if (d1 == 0) { m1 = 0; d1 = 1; }
    if (d2 == 0) { m2 = 0; d2 = 1; }
    unsigned __int128 l = (unsigned __int128)m1 * d2, r = (unsigned __int128)m2 * d1;
    return (l > r) - (l < r);
}

int orc_compare_j(uint64_t m1, uint64_t d1, uint64_t m2, uint64_t d2) { return orc_cmp_j(m1, d1, m2, d2); }

void orc_pair_terms(const orc_genome *q, uint32_t a, const orc_genome *t, uint32_t b, uint64_t *smin, uint64_t *smax) {
    orc_jaccard_terms(q->ids + q->ptr[a], q->cnt + q->ptr[a], q->ptr[a + 1] - q->ptr[a],
                      t->ids + t->ptr[b], t->cnt + t->ptr[b], t->ptr[b + 1] - t->ptr[b], smin, smax);
}

/* ------------------------------------------- Eqs. length_threshold, directional_jaccard */

/* Numerators of the two directional similarities of Eq. directional_jaccard:
 * *occ_a = sum over k-mers present in both genes of the k-mer's occurrences in a,
 * *occ_b = the same with b's occurrences.  p(a -> b) = occ_a / (|a| - k + 1). */
void orc_directional_terms(const uint64_t *ia, const uint32_t *ca, uint64_t na,
                           const uint64_t *ib, const uint32_t *cb, uint64_t nb,
                           uint64_t *occ_a, uint64_t *occ_b) {
    uint64_t i = 0, j = 0, sa = 0, sb = 0;
    while (i < na && j < nb) {
        if (ia[i] < ib[j]) ++i;
        else if (ib[j] < ia[i]) ++j;
        else { sa += ca[i]; sb += cb[j]; ++i; ++j; }
    }
    *occ_a = sa;
    *occ_b = sb;
}

/* Candidate filters (theta = theta_n / theta_d, tau = tau_n / tau_d; a zero
 * denominator switches that filter off).  Eq. length_threshold: both lengths at
 * least theta times the other.  Eq. directional_jaccard: both directional
 * similarities at least tau (p = 0 for a gene without windows). */
static int orc_candidate(const orc_genome *q, uint32_t a, const orc_genome *t, uint32_t b,
                         uint64_t theta_n, uint64_t theta_d, uint64_t tau_n, uint64_t tau_d) {
    if (theta_d) {
        const unsigned __int128 la = q->len[a], lb = t->len[b];
        if (la * theta_d < (unsigned __int128)theta_n * lb || lb * theta_d < (unsigned __int128)theta_n * la) return 0;
    }
    if (tau_d) {
        uint64_t oa, ob;
        orc_directional_terms(q->ids + q->ptr[a], q->cnt + q->ptr[a], q->ptr[a + 1] - q->ptr[a],
                              t->ids + t->ptr[b], t->cnt + t->ptr[b], t->ptr[b + 1] - t->ptr[b], &oa, &ob);
        const uint64_t wa = q->nwin[a], wb = t->nwin[b];
        /* p >= tau  <=>  occ * tau_d >= tau_n * windows (both sides non-negative) */
        if (wa == 0 ? tau_n > 0 : (unsigned __int128)oa * tau_d < (unsigned __int128)tau_n * wa) return 0;
        if (wb == 0 ? tau_n > 0 : (unsigned __int128)ob * tau_d < (unsigned __int128)tau_n * wb) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------ Eq. best_hit */

/* BH(a, T): the genes b of T whose J(a,b) equals the maximum of row a,
 * provided that maximum is above zero; ascending b.  col/num/den must hold
 * t->n entries.  Returns the number of best hits. */
int64_t orc_bh_row_f(const orc_genome *q, uint32_t a, const orc_genome *t, uint32_t *col, uint64_t *num, uint64_t *den,
                     uint64_t theta_n, uint64_t theta_d, uint64_t tau_n, uint64_t tau_d) {
    uint32_t n = t->n;
    if (n == 0) return 0;
    uint64_t *m = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * n);
    char *cand = (char *)malloc(n);
    int have = 0;
    uint32_t best = 0;
    for (uint32_t b = 0; b < n; ++b) {
        orc_pair_terms(q, a, t, b, &m[b], &d[b]);
        cand[b] = (char)orc_candidate(q, a, t, b, theta_n, theta_d, tau_n, tau_d);
        if (!cand[b]) continue;  /* a filtered pair is no best-hit candidate */
        if (!have || orc_cmp_j(m[b], d[b], m[best], d[best]) > 0) best = b;
        have = 1;
    }
    int64_t c = 0;
    if (have && orc_cmp_j(m[best], d[best], 0, 1) > 0) {
        for (uint32_t b = 0; b < n; ++b) {
            if (cand[b] && orc_cmp_j(m[b], d[b], m[best], d[best]) == 0) {
                col[c] = b; num[c] = m[b]; den[c] = d[b]; ++c;
            }
        }
    }
    free(m);
    free(d);
    free(cand);
    return c;
}

int64_t orc_bh_row(const orc_genome *q, uint32_t a, const orc_genome *t, uint32_t *col, uint64_t *num, uint64_t *den) {
    return orc_bh_row_f(q, a, t, col, num, den, 0, 0, 0, 0);
}

/* Best hits of many rows of q against t, rows handed to a pool of threads
 * one at a time (each row is an independent unit of work, as in Alg. 2). */
typedef struct {
    uint32_t nrows;
    uint64_t *ptr;   /* nrows+1 */
    uint32_t *col;
    uint64_t *num, *den;
} orc_bh;

typedef struct {
    const orc_genome *q, *t;
    uint64_t theta_n, theta_d, tau_n, tau_d;
    const uint32_t *rows;
    uint32_t nrows;
    uint32_t next;          /* shared row counter */
    uint32_t **rc;          /* per-row results */
    uint64_t **rn, **rd;
    int64_t *rcount;
} orc_bh_job;

static void *orc_bh_worker(void *arg) {
    orc_bh_job *J = (orc_bh_job *)arg;
    uint32_t n = J->t->n ? J->t->n : 1;
    uint32_t *col = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint64_t *num = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint64_t *den = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (;;) {
        uint32_t r = __atomic_fetch_add(&J->next, 1u, __ATOMIC_RELAXED);
        if (r >= J->nrows) break;
        uint32_t a = J->rows ? J->rows[r] : r;
        int64_t c = orc_bh_row_f(J->q, a, J->t, col, num, den, J->theta_n, J->theta_d, J->tau_n, J->tau_d);
        J->rcount[r] = c;
        J->rc[r] = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(c + 1));
        J->rn[r] = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(c + 1));
        J->rd[r] = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(c + 1));
        memcpy(J->rc[r], col, sizeof(uint32_t) * (size_t)c);
        memcpy(J->rn[r], num, sizeof(uint64_t) * (size_t)c);
        memcpy(J->rd[r], den, sizeof(uint64_t) * (size_t)c);
    }
    free(col); free(num); free(den);
    return NULL;
}

/* rows == NULL means every row of q, in order.  The filters as in orc_candidate. */
orc_bh *orc_bh_rows_f(const orc_genome *q, const orc_genome *t, const uint32_t *rows, uint32_t nrows, int nthreads,
                      uint64_t theta_n, uint64_t theta_d, uint64_t tau_n, uint64_t tau_d) {
    if (!rows) nrows = q->n;
    if (nthreads < 1) nthreads = 1;
    orc_bh_job J;
    memset(&J, 0, sizeof(J));
    J.q = q; J.t = t; J.rows = rows; J.nrows = nrows; J.next = 0;
    J.theta_n = theta_n; J.theta_d = theta_d; J.tau_n = tau_n; J.tau_d = tau_d;
    J.rc = (uint32_t **)calloc((size_t)nrows + 1, sizeof(void *));
    J.rn = (uint64_t **)calloc((size_t)nrows + 1, sizeof(void *));
    J.rd = (uint64_t **)calloc((size_t)nrows + 1, sizeof(void *));
    J.rcount = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int i = 0; i < nthreads; ++i) pthread_create(&th[i], NULL, orc_bh_worker, &J);
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    free(th);
    orc_bh *o = (orc_bh *)calloc(1, sizeof(orc_bh));
    o->nrows = nrows;
    o->ptr = (uint64_t *)calloc((size_t)nrows + 1, sizeof(uint64_t));
    for (uint32_t r = 0; r < nrows; ++r) o->ptr[r + 1] = o->ptr[r] + (uint64_t)J.rcount[r];
    uint64_t nnz = o->ptr[nrows];
    o->col = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nnz + 1));
    o->num = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nnz + 1));
    o->den = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nnz + 1));
    for (uint32_t r = 0; r < nrows; ++r) {
        uint64_t p = o->ptr[r], c = (uint64_t)J.rcount[r];
        memcpy(o->col + p, J.rc[r], sizeof(uint32_t) * (size_t)c);
        memcpy(o->num + p, J.rn[r], sizeof(uint64_t) * (size_t)c);
        memcpy(o->den + p, J.rd[r], sizeof(uint64_t) * (size_t)c);
        free(J.rc[r]); free(J.rn[r]); free(J.rd[r]);
    }
    free(J.rc); free(J.rn); free(J.rd); free(J.rcount);
    return o;
}

orc_bh *orc_bh_rows(const orc_genome *q, const orc_genome *t, const uint32_t *rows, uint32_t nrows, int nthreads) {
    return orc_bh_rows_f(q, t, rows, nrows, nthreads, 0, 0, 0, 0);
}

void orc_bh_free(orc_bh *o) {
    if (!o) return;
    free(o->ptr); free(o->col); free(o->num); free(o->den); free(o);
}
uint32_t orc_bh_nrows(const orc_bh *o) { return o->nrows; }
const uint64_t *orc_bh_ptr(const orc_bh *o) { return o->ptr; }
const uint32_t *orc_bh_col(const orc_bh *o) { return o->col; }
const uint64_t *orc_bh_num(const orc_bh *o) { return o->num; }
const uint64_t *orc_bh_den(const orc_bh *o) { return o->den; }

/* ------------------------------------------------ Eq. bidirectional_best_hit */

typedef struct {
    uint64_t n;
    uint32_t *a, *b;
    uint64_t *num, *den;
} orc_pairs;

static int orc_row_has(const orc_bh *o, uint32_t row, uint32_t x) {
    for (uint64_t p = o->ptr[row]; p < o->ptr[row + 1]; ++p)
        if (o->col[p] == x) return 1;
    return 0;
}

static orc_pairs *orc_pairs_new(uint64_t cap) {
    orc_pairs *P = (orc_pairs *)calloc(1, sizeof(orc_pairs));
    P->a = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cap + 1));
    P->b = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cap + 1));
    P->num = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(cap + 1));
    P->den = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(cap + 1));
    return P;
}

/* BBH(G_i, G_j) = {(a, b) : b in BH(a, G_j) and a in BH(b, G_i)}, in (a, b)
 * order.  ab must hold every row of G_i, ba every row of G_j. */
orc_pairs *orc_bbh(const orc_bh *ab, const orc_bh *ba) {
    orc_pairs *P = orc_pairs_new(ab->ptr[ab->nrows]);
    for (uint32_t a = 0; a < ab->nrows; ++a) {
        for (uint64_t p = ab->ptr[a]; p < ab->ptr[a + 1]; ++p) {
            uint32_t b = ab->col[p];
            if (b < ba->nrows && orc_row_has(ba, b, a)) {
                P->a[P->n] = a; P->b[P->n] = b; P->num[P->n] = ab->num[p]; P->den[P->n] = ab->den[p];
                P->n++;
            }
        }
    }
    return P;
}

/* Alg. 3, taken step by step: the relevant columns are those named in A_ij;
 * for each relevant column b and each row a whose best hits contain b, keep
 * (a, b) when S[a][b] equals the maximum of column b and a is among the best
 * hits A_ji of b.  The column maximum is recomputed from the similarities. */
orc_pairs *orc_bbh_alg3(const orc_genome *gi, const orc_genome *gj, const orc_bh *ab, const orc_bh *ba) {
    uint32_t nb = gj->n;
    char *relevant = (char *)calloc((size_t)nb + 1, 1);
    for (uint64_t p = 0; p < ab->ptr[ab->nrows]; ++p) relevant[ab->col[p]] = 1;
    orc_pairs *P = orc_pairs_new(ab->ptr[ab->nrows]);
    /* the pairs are gathered column by column, then put in (a, b) order */
    for (uint32_t b = 0; b < nb; ++b) {
        if (!relevant[b]) continue;
        uint64_t cm = 0, cd = 1; /* column maximum, as a rational */
        for (uint32_t r = 0; r < gi->n; ++r) {
            uint64_t m, d;
            orc_pair_terms(gi, r, gj, b, &m, &d);
            if (orc_cmp_j(m, d, cm, cd) > 0) { cm = m; cd = d; }
        }
        for (uint32_t a = 0; a < ab->nrows; ++a) {
            for (uint64_t p = ab->ptr[a]; p < ab->ptr[a + 1]; ++p) {
                if (ab->col[p] != b) continue;
                if (orc_cmp_j(ab->num[p], ab->den[p], cm, cd) == 0 && orc_row_has(ba, b, a)) {
                    P->a[P->n] = a; P->b[P->n] = b; P->num[P->n] = ab->num[p]; P->den[P->n] = ab->den[p];
                    P->n++;
                }
            }
        }
    }
    free(relevant);
    /* insertion sort by (a, b): the set definition lists pairs in that order */
    for (uint64_t i = 1; i < P->n; ++i) {
        uint32_t a = P->a[i], b = P->b[i];
        uint64_t nu = P->num[i], de = P->den[i];
        uint64_t j = i;
        while (j > 0 && (P->a[j - 1] > a || (P->a[j - 1] == a && P->b[j - 1] > b))) {
            P->a[j] = P->a[j - 1]; P->b[j] = P->b[j - 1]; P->num[j] = P->num[j - 1]; P->den[j] = P->den[j - 1];
            --j;
        }
        P->a[j] = a; P->b[j] = b; P->num[j] = nu; P->den[j] = de;
    }
    return P;
}

void orc_pairs_free(orc_pairs *P) {
    if (!P) return;
    free(P->a); free(P->b); free(P->num); free(P->den); free(P);
}
uint64_t orc_pairs_n(const orc_pairs *P) { return P->n; }
const uint32_t *orc_pairs_a(const orc_pairs *P) { return P->a; }
const uint32_t *orc_pairs_b(const orc_pairs *P) { return P->b; }
const uint64_t *orc_pairs_num(const orc_pairs *P) { return P->num; }
const uint64_t *orc_pairs_den(const orc_pairs *P) { return P->den; }

/* ===================================================== sparse exact oracle (O2)
 *
 * The same best hits as orc_bh_rows_f, computed without visiting gene pairs that share
 * nothing, so that whole genome-scale workloads can be checked in full.  It is still
 * plain: for the target genome a hash map sends each k-mer identifier to its postings
 * (gene, multiplicity), in gene order; for a query gene a, every k-mer w of MV(a) adds
 * min(mult_a(w), mult_b(w)) to the accumulator of each gene b posted under w (Eq.
 * jaccard_k's sum of minima over D(a) and D(b) together).  A gene b never touched shares
 * no k-mer with a, so J(a,b) = 0 and b is no best hit (the maximum must be above zero).
 * For a touched b the sum of maxima over the union is n_a + n_b - m: per k-mer,
 * max(x,y) = x + y - min(x,y), with x or y = 0 for a k-mer in one gene only, and the
 * multiplicities of a gene sum to its window count.  The dense oracle computes that sum
 * literally; the tests pin this one to it (and to brute force) on shared inputs.  The
 * row maximum and its ties follow Eq. best_hit exactly as in orc_bh_row_f, with the same
 * candidate filters (the directional sums of Eq. directional_jaccard accumulate beside the
 * minima: occurrences in a and in b of every shared k-mer).
 */

/* One slot of the map: an identifier and the range of its postings; len 0 marks a free
 * slot (every identifier present has at least one posting). */
typedef struct {
    uint64_t key;
    uint32_t start, len;
} orc_slot;

typedef struct {
    uint64_t mask;       /* slots - 1 (slots a power of two) */
    orc_slot *slot;
    uint32_t *gene;      /* postings */
    uint32_t *cnt;
} orc_index;

static uint64_t orc_hash(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

/* The slot holding id, or the free slot where it would go (linear probing). */
static orc_slot *orc_index_slot(const orc_index *ix, uint64_t id) {
    uint64_t s = orc_hash(id) & ix->mask;
    while (ix->slot[s].len && ix->slot[s].key != id) s = (s + 1) & ix->mask;
    return &ix->slot[s];
}

/* Map from identifier to postings over every gene of t (at most 2^32 - 1 entries). */
orc_index *orc_index_new(const orc_genome *t) {
    const uint64_t e = t->ptr[t->n];
    if (e >= 0xffffffffull) return NULL;
    uint64_t slots = 16;
    while (slots < e + e / 2) slots <<= 1;  /* distinct identifiers <= e: load at most 2/3 */
    orc_index *ix = (orc_index *)calloc(1, sizeof(orc_index));
    ix->mask = slots - 1;
    ix->slot = (orc_slot *)calloc((size_t)slots, sizeof(orc_slot));
    ix->gene = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(e + 1));
    ix->cnt = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(e + 1));
    /* pass 1: postings per identifier */
    for (uint64_t p = 0; p < e; ++p) {
        orc_slot *s = orc_index_slot(ix, t->ids[p]);
        s->key = t->ids[p];
        s->len += 1;
    }
    uint32_t run = 0;
    for (uint64_t s = 0; s < slots; ++s) { ix->slot[s].start = run; run += ix->slot[s].len; }
    /* pass 2: fill, genes ascending inside each identifier (start advances, then is restored) */
    for (uint32_t b = 0; b < t->n; ++b)
        for (uint64_t p = t->ptr[b]; p < t->ptr[b + 1]; ++p) {
            orc_slot *s = orc_index_slot(ix, t->ids[p]);
            ix->gene[s->start] = b;
            ix->cnt[s->start] = t->cnt[p];
            s->start += 1;
        }
    for (uint64_t s = 0; s < slots; ++s) ix->slot[s].start -= ix->slot[s].len;
    return ix;
}

void orc_index_free(orc_index *ix) {
    if (!ix) return;
    free(ix->slot); free(ix->gene); free(ix->cnt); free(ix);
}

/* Scratch of one worker: accumulators over the target's genes and the touched list. */
typedef struct {
    uint64_t *m, *oa, *ob;
    uint32_t *touched;
} orc_acc;

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* Best hits of row a of q in t through t's index; same contract as orc_bh_row_f. */
static int64_t orc_bh_row_sparse(const orc_genome *q, uint32_t a, const orc_genome *t, const orc_index *ix,
                                 orc_acc *A, uint32_t *col, uint64_t *num, uint64_t *den,
                                 uint64_t theta_n, uint64_t theta_d, uint64_t tau_n, uint64_t tau_d) {
    uint32_t nt = 0;
    for (uint64_t p = q->ptr[a]; p < q->ptr[a + 1]; ++p) {
        const orc_slot *s = orc_index_slot(ix, q->ids[p]);
        if (!s->len) continue;  /* a k-mer no gene of t has */
        const uint32_t ca = q->cnt[p];
        for (uint64_t x = s->start; x < (uint64_t)s->start + s->len; ++x) {
            const uint32_t b = ix->gene[x], cb = ix->cnt[x];
            if (A->m[b] == 0) A->touched[nt++] = b;
            A->m[b] += ca < cb ? ca : cb;
            A->oa[b] += ca;
            A->ob[b] += cb;
        }
    }
    qsort(A->touched, nt, sizeof(uint32_t), cmp_u32);
    const uint64_t na = q->nwin[a];
    int have = 0;
    uint64_t bm = 0, bd = 1;
    int64_t c = 0;
    /* the candidates' maximum, then every candidate at it, ascending b */
    for (int pass = 0; pass < 2; ++pass) {
        for (uint32_t i = 0; i < nt; ++i) {
            const uint32_t b = A->touched[i];
            const uint64_t m = A->m[b], d = na + t->nwin[b] - m;
            int ok = 1;
            if (theta_d) {
                const unsigned __int128 la = q->len[a], lb = t->len[b];
                if (la * theta_d < (unsigned __int128)theta_n * lb || lb * theta_d < (unsigned __int128)theta_n * la) ok = 0;
            }
            if (ok && tau_d) {
                if ((unsigned __int128)A->oa[b] * tau_d < (unsigned __int128)tau_n * na) ok = 0;
                if ((unsigned __int128)A->ob[b] * tau_d < (unsigned __int128)tau_n * t->nwin[b]) ok = 0;
            }
            if (!ok) continue;
            if (pass == 0) {
                if (!have || orc_cmp_j(m, d, bm, bd) > 0) { bm = m; bd = d; }
                have = 1;
            } else if (orc_cmp_j(m, d, bm, bd) == 0) {
                col[c] = b; num[c] = m; den[c] = d; ++c;
            }
        }
        if (pass == 0 && !(have && orc_cmp_j(bm, bd, 0, 1) > 0)) break;
    }
    for (uint32_t i = 0; i < nt; ++i) {
        const uint32_t b = A->touched[i];
        A->m[b] = 0; A->oa[b] = 0; A->ob[b] = 0;
    }
    return c;
}

typedef struct {
    const orc_genome *q, *t;
    const orc_index *ix;
    uint64_t theta_n, theta_d, tau_n, tau_d;
    const uint32_t *rows;
    uint32_t nrows;
    uint32_t next;
    uint32_t **rc;
    uint64_t **rn, **rd;
    int64_t *rcount;
} orc_sparse_job;

static void *orc_sparse_worker(void *arg) {
    orc_sparse_job *J = (orc_sparse_job *)arg;
    const uint32_t n = J->t->n ? J->t->n : 1;
    orc_acc A;
    A.m = (uint64_t *)calloc(n, sizeof(uint64_t));
    A.oa = (uint64_t *)calloc(n, sizeof(uint64_t));
    A.ob = (uint64_t *)calloc(n, sizeof(uint64_t));
    A.touched = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *col = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint64_t *num = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint64_t *den = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (;;) {
        const uint32_t r = __atomic_fetch_add(&J->next, 1u, __ATOMIC_RELAXED);
        if (r >= J->nrows) break;
        const uint32_t a = J->rows ? J->rows[r] : r;
        const int64_t c = orc_bh_row_sparse(J->q, a, J->t, J->ix, &A, col, num, den, J->theta_n, J->theta_d,
                                            J->tau_n, J->tau_d);
        J->rcount[r] = c;
        J->rc[r] = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(c + 1));
        J->rn[r] = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(c + 1));
        J->rd[r] = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(c + 1));
        memcpy(J->rc[r], col, sizeof(uint32_t) * (size_t)c);
        memcpy(J->rn[r], num, sizeof(uint64_t) * (size_t)c);
        memcpy(J->rd[r], den, sizeof(uint64_t) * (size_t)c);
    }
    free(A.m); free(A.oa); free(A.ob); free(A.touched);
    free(col); free(num); free(den);
    return NULL;
}

/* Best hits of the given rows of q (every row when rows == NULL) in t, whose index is ix;
 * rows go to a pool of threads one at a time.  Returns the same structure as
 * orc_bh_rows_f, so orc_bbh applies to it. */
orc_bh *orc_bh_sparse(const orc_genome *q, const orc_genome *t, const orc_index *ix, const uint32_t *rows,
                      uint32_t nrows, int nthreads, uint64_t theta_n, uint64_t theta_d, uint64_t tau_n,
                      uint64_t tau_d) {
    if (!rows) nrows = q->n;
    if (nthreads < 1) nthreads = 1;
    orc_sparse_job J;
    memset(&J, 0, sizeof(J));
    J.q = q; J.t = t; J.ix = ix; J.rows = rows; J.nrows = nrows;
    J.theta_n = theta_n; J.theta_d = theta_d; J.tau_n = tau_n; J.tau_d = tau_d;
    J.rc = (uint32_t **)calloc((size_t)nrows + 1, sizeof(void *));
    J.rn = (uint64_t **)calloc((size_t)nrows + 1, sizeof(void *));
    J.rd = (uint64_t **)calloc((size_t)nrows + 1, sizeof(void *));
    J.rcount = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int i = 0; i < nthreads; ++i) pthread_create(&th[i], NULL, orc_sparse_worker, &J);
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    free(th);
    orc_bh *o = (orc_bh *)calloc(1, sizeof(orc_bh));
    o->nrows = nrows;
    o->ptr = (uint64_t *)calloc((size_t)nrows + 1, sizeof(uint64_t));
    for (uint32_t r = 0; r < nrows; ++r) o->ptr[r + 1] = o->ptr[r] + (uint64_t)J.rcount[r];
    const uint64_t nnz = o->ptr[nrows];
    o->col = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nnz + 1));
    o->num = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nnz + 1));
    o->den = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nnz + 1));
    for (uint32_t r = 0; r < nrows; ++r) {
        const uint64_t p = o->ptr[r], c = (uint64_t)J.rcount[r];
        memcpy(o->col + p, J.rc[r], sizeof(uint32_t) * (size_t)c);
        memcpy(o->num + p, J.rn[r], sizeof(uint64_t) * (size_t)c);
        memcpy(o->den + p, J.rd[r], sizeof(uint64_t) * (size_t)c);
        free(J.rc[r]); free(J.rn[r]); free(J.rd[r]);
    }
    free(J.rc); free(J.rn); free(J.rd); free(J.rcount);
    return o;
}
