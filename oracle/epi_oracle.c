/*
 * CPU oracle for the exhaustive k-order epistasis scan.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may build, load or
 * call it.  It shares no code, table or helper with the GPU library.
 *
 * What it computes (paper: Section 2 and Algorithm 1):
 *   - every combination c_1 < ... < c_k of k SNPs out of M, exactly once,
 *     visited in lexicographic order (Section 2.4, Algorithm 1 enumerates the
 *     same set depth-first);
 *   - its contingency table: for each class (cases, controls) and each of the
 *     3^k genotype combinations, the number of individuals of that class with
 *     that genotype combination (Sections 2.1-2.2).  The oracle walks the
 *     individuals one by one; it never builds bitsets.  Cell index
 *     x = sum_t g_t * 3^(k-t), first SNP most significant, which is the
 *     row index i*3+j the paper uses when a SNP is added to a table;
 *   - its mutual information MI = H(X) + H(Y) - H(X,Y) (Section 2.3,
 *     Equations 1-3) in double precision with natural logarithms, where every
 *     probability is a count divided by the total number of individuals m and
 *     zero counts contribute nothing;
 *   - the best `top_k` combinations: larger MI first, ties broken by the
 *     lexicographically smaller combination (the paper keeps only the
 *     combinations with the highest MI, Section 2.4);
 *   - a completeness digest: the number of combinations of a rank range and
 *     the sum of a hash of each combination and its table (the definition is
 *     at oracle_digest), against which a GPU scan that visits the
 *     combinations in its own order can show that it scored every one of
 *     them exactly once, each with its table.
 *
 * Inputs: genotypes G (uint8, M rows of N individuals, row stride ld, values
 * 0/1/2 = homozygous dominant / heterozygous / homozygous recessive, the three
 * genotype-table rows of Section 2.1) and phenotype y (uint8, 1 = case,
 * 0 = control).
 *
 * Build: plain C99 + pthreads, no intrinsics, no bit tricks.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORACLE_MAX_ORDER 8

/* ---- combinatorics ------------------------------------------------------ */

/* Binomial coefficient C(n, k) computed exactly (n, k small enough that the
 * result fits in 64 bits); returns 0 when k < 0 or k > n. */
uint64_t oracle_binomial(int64_t n, int64_t k)
{
    if (k < 0 || n < 0 || k > n)
        return 0;
    if (k > n - k)
        k = n - k;
    unsigned __int128 r = 1;
    for (int64_t i = 0; i < k; i++) {
        r = r * (unsigned __int128)(n - i);
        r = r / (unsigned __int128)(i + 1);
    }
    return (uint64_t)r;
}

/* The combination at position `rank` of the lexicographic order of all
 * k-subsets of {0..M-1}: choose each position's smallest value whose block of
 * completions still contains `rank`. */
static void lex_unrank(uint64_t rank, int32_t M, int32_t k, int32_t *c)
{
    int32_t v = 0;
    for (int32_t t = 0; t < k; t++) {
        for (;;) {
            uint64_t block = oracle_binomial(M - 1 - v, k - 1 - t);
            if (rank < block)
                break;
            rank -= block;
            v++;
        }
        c[t] = v;
        v++;
    }
}

/* Advance c to the next combination in lexicographic order; returns 0 when c
 * was the last one. */
static int lex_next(int32_t *c, int32_t M, int32_t k)
{
    int32_t t = k - 1;
    while (t >= 0 && c[t] == M - k + t)
        t--;
    if (t < 0)
        return 0;
    c[t]++;
    for (int32_t u = t + 1; u < k; u++)
        c[u] = c[u - 1] + 1;
    return 1;
}

/* Number of combinations visited by walking the lexicographic order from the
 * first combination to the last (an enumeration, not a formula). */
uint64_t oracle_enumerate_count(int32_t M, int32_t k)
{
    if (k < 1 || k > M)
        return 0;
    int32_t c[64];
    for (int32_t t = 0; t < k; t++)
        c[t] = t;
    uint64_t n = 1;
    while (lex_next(c, M, k))
        n++;
    return n;
}

/* ---- contingency table -------------------------------------------------- */

static int64_t pow3(int32_t k)
{
    int64_t p = 1;
    for (int32_t t = 0; t < k; t++)
        p *= 3;
    return p;
}

/* table[cls * 3^k + x], cls 0 = cases, 1 = controls.  Walks the N individuals
 * one at a time.  Returns -1 if a genotype is outside {0,1,2}. */
int oracle_count_table(const uint8_t *G, int64_t ld, const uint8_t *y, int32_t N,
                       const int32_t *combo, int32_t k, uint64_t *table)
{
    const int64_t P = pow3(k);
    for (int64_t i = 0; i < 2 * P; i++)
        table[i] = 0;
    for (int32_t s = 0; s < N; s++) {
        int64_t x = 0;
        for (int32_t t = 0; t < k; t++) {
            uint8_t g = G[(int64_t)combo[t] * ld + s];
            if (g > 2)
                return -1;
            x = x * 3 + g;
        }
        int cls = y[s] ? 0 : 1;
        table[cls * P + x] += 1;
    }
    return 0;
}

/* Genotype table of a combination (Section 2.1: one row of individuals per
 * genotype combination, built by Algorithm 1's combine step one SNP at a
 * time).  Row x of class cls is a bitset over that class's individuals in
 * input order: bit b of word w stands for the class's individual 32 w + b.
 * rows[x * (words0 + words1) + (cls ? words0 : 0) + w], words_cls words per
 * class (at least enough for the class; bits past its size are 0).  Walks the
 * individuals one at a time.  Returns -1 if a genotype is outside {0,1,2} or
 * a class does not fit its words. */
int oracle_genotype_rows(const uint8_t *G, int64_t ld, const uint8_t *y, int32_t N,
                         const int32_t *combo, int32_t k, int32_t words0, int32_t words1, uint32_t *rows)
{
    const int64_t P = pow3(k);
    const int64_t W = (int64_t)words0 + words1;
    for (int64_t i = 0; i < P * W; i++)
        rows[i] = 0;
    int32_t pos[2] = {0, 0};
    for (int32_t s = 0; s < N; s++) {
        int64_t row = 0;
        for (int32_t t = 0; t < k; t++) {
            uint8_t geno = G[(int64_t)combo[t] * ld + s];
            if (geno > 2)
                return -1;
            row = 3 * row + geno;
        }
        int cl = y[s] ? 0 : 1;
        int32_t b = pos[cl]++;
        if (b >= 32 * (cl ? words1 : words0))
            return -1;
        rows[row * W + (cl ? words0 : 0) + b / 32] |= (uint32_t)1 << (b % 32);
    }
    return 0;
}

/* ---- mutual information (Equations 1-3) --------------------------------- */

/* MI of a 2 x 3^k table, natural logarithm, probabilities = count / m with m
 * the total number of individuals in the table. */
double oracle_mi(const uint64_t *table, int32_t k)
{
    const int64_t P = pow3(k);
    double m = 0.0;
    for (int64_t i = 0; i < 2 * P; i++)
        m += (double)table[i];
    if (m <= 0.0)
        return 0.0;
    double h_xy = 0.0, h_x = 0.0, h_y = 0.0;
    double n_y[2] = {0.0, 0.0};
    for (int64_t x = 0; x < P; x++) {
        double n_x = 0.0;
        for (int cls = 0; cls < 2; cls++) {
            double n = (double)table[cls * P + x];
            if (n > 0.0) {
                double p = n / m;
                h_xy -= p * log(p);
            }
            n_x += n;
            n_y[cls] += n;
        }
        if (n_x > 0.0) {
            double p = n_x / m;
            h_x -= p * log(p);
        }
    }
    for (int cls = 0; cls < 2; cls++) {
        if (n_y[cls] > 0.0) {
            double p = n_y[cls] / m;
            h_y -= p * log(p);
        }
    }
    return h_x + h_y - h_xy;
}

/* ---- top-K scan --------------------------------------------------------- */

typedef struct {
    double mi;
    int32_t c[ORACLE_MAX_ORDER];
} entry_t;

static int lex_less(const int32_t *a, const int32_t *b, int32_t k)
{
    for (int32_t t = 0; t < k; t++) {
        if (a[t] != b[t])
            return a[t] < b[t];
    }
    return 0;
}

/* a ranks before b: larger MI, then lexicographically smaller combination */
static int ranks_before(const entry_t *a, const entry_t *b, int32_t k)
{
    if (a->mi != b->mi)
        return a->mi > b->mi;
    return lex_less(a->c, b->c, k);
}

/* Insert e into list (sorted best first, length *n, capacity K). */
static void topk_insert(entry_t *list, int32_t *n, int32_t K, const entry_t *e, int32_t k)
{
    int32_t len = *n;
    if (len == K && !ranks_before(e, &list[len - 1], k))
        return;
    int32_t pos = (len < K) ? len : K - 1;
    while (pos > 0 && ranks_before(e, &list[pos - 1], k)) {
        list[pos] = list[pos - 1];
        pos--;
    }
    list[pos] = *e;
    if (len < K)
        *n = len + 1;
}

typedef struct {
    const uint8_t *G;
    int64_t ld;
    const uint8_t *y;
    int32_t M, N, k, K;
    uint64_t begin, end;
    entry_t *list;
    int32_t n;
    uint64_t *table;
    int status;
} job_t;

static void *scan_range(void *arg)
{
    job_t *j = (job_t *)arg;
    j->n = 0;
    j->status = 0;
    if (j->begin >= j->end)
        return NULL;
    entry_t e;
    memset(&e, 0, sizeof(e));
    lex_unrank(j->begin, j->M, j->k, e.c);
    for (uint64_t r = j->begin; r < j->end; r++) {
        if (oracle_count_table(j->G, j->ld, j->y, j->N, e.c, j->k, j->table) != 0) {
            j->status = -1;
            return NULL;
        }
        e.mi = oracle_mi(j->table, j->k);
        topk_insert(j->list, &j->n, j->K, &e, j->k);
        if (r + 1 < j->end)
            lex_next(e.c, j->M, j->k);
    }
    return NULL;
}

/*
 * Scan the lexicographic rank range [rank_begin, rank_end) (rank_end is
 * clamped to C(M,k)) with `nthreads` threads (<= 0: all online cores) and
 * return the best `top_k` combinations of that range, best first.
 *
 * out_combos: top_k * k int32; out_scores: top_k doubles; out_tables
 * (nullable): top_k * 2 * 3^k counts.  *n_out = number written.
 * Returns 0, or -1 on invalid arguments / genotype values.
 */
int oracle_scan(const uint8_t *G, int64_t ld, const uint8_t *y, int32_t M, int32_t N, int32_t k,
                int32_t top_k, uint64_t rank_begin, uint64_t rank_end, int32_t nthreads,
                int32_t *out_combos, double *out_scores, uint64_t *out_tables, int32_t *n_out,
                int32_t *threads_used)
{
    *n_out = 0;
    if (k < 1 || k > ORACLE_MAX_ORDER || k > M || top_k < 1 || N < 1)
        return -1;
    uint64_t total = oracle_binomial(M, k);
    if (rank_end > total)
        rank_end = total;
    if (rank_begin >= rank_end)
        return 0;
    if (nthreads <= 0)
        nthreads = (int32_t)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1)
        nthreads = 1;
    uint64_t span = rank_end - rank_begin;
    if ((uint64_t)nthreads > span)
        nthreads = (int32_t)span;
    if (threads_used)
        *threads_used = nthreads;
    const int64_t P = pow3(k);
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    int rc = 0;
    for (int32_t t = 0; t < nthreads; t++) {
        job_t *j = &jobs[t];
        j->G = G;
        j->ld = ld;
        j->y = y;
        j->M = M;
        j->N = N;
        j->k = k;
        j->K = top_k;
        j->begin = rank_begin + span * (uint64_t)t / (uint64_t)nthreads;
        j->end = rank_begin + span * (uint64_t)(t + 1) / (uint64_t)nthreads;
        j->list = (entry_t *)calloc((size_t)top_k, sizeof(entry_t));
        j->table = (uint64_t *)calloc((size_t)(2 * P), sizeof(uint64_t));
    }
    for (int32_t t = 1; t < nthreads; t++)
        pthread_create(&tids[t], NULL, scan_range, &jobs[t]);
    scan_range(&jobs[0]);
    for (int32_t t = 1; t < nthreads; t++)
        pthread_join(tids[t], NULL);

    entry_t *best = (entry_t *)calloc((size_t)top_k, sizeof(entry_t));
    int32_t nb = 0;
    for (int32_t t = 0; t < nthreads; t++) {
        if (jobs[t].status != 0)
            rc = -1;
        for (int32_t i = 0; i < jobs[t].n; i++)
            topk_insert(best, &nb, top_k, &jobs[t].list[i], k);
    }
    if (rc == 0) {
        for (int32_t i = 0; i < nb; i++) {
            for (int32_t t = 0; t < k; t++)
                out_combos[i * k + t] = best[i].c[t];
            out_scores[i] = best[i].mi;
            if (out_tables)
                oracle_count_table(G, ld, y, N, best[i].c, k, out_tables + (int64_t)i * 2 * P);
        }
        *n_out = nb;
    }
    for (int32_t t = 0; t < nthreads; t++) {
        free(jobs[t].list);
        free(jobs[t].table);
    }
    free(best);
    free(jobs);
    free(tids);
    return rc;
}

/* ---- completeness digest (Algorithm 1 visits every combination once;
 *      Section 2.2 gives each its table) --------------------------------- */

/* Output function of SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), arithmetic modulo 2^64. */
static uint64_t splitmix_out(uint64_t z)
{
    z = (z ^ (z >> 30)) * UINT64_C(0xbf58476d1ce4e5b9);
    z = (z ^ (z >> 27)) * UINT64_C(0x94d049bb133111eb);
    return z ^ (z >> 31);
}

/* Contribution of one combination c[0] < ... < c[k-1] with table
 * table[cls * 3^k + x]: the indices folded one at a time,
 * h = mix(h + c_t + 1) from h = 0; the counts weighted per cell,
 * s = sum table[cls][x] * mix(2 x + cls + 1); the contribution mix(h ^ s). */
static uint64_t digest_term(const int32_t *c, int32_t k, const uint64_t *table)
{
    const int64_t P = pow3(k);
    uint64_t h = 0;
    for (int32_t t = 0; t < k; t++)
        h = splitmix_out(h + (uint64_t)c[t] + 1);
    uint64_t s = 0;
    for (int cls = 0; cls < 2; cls++)
        for (int64_t x = 0; x < P; x++)
            s += table[cls * P + x] * splitmix_out(2 * (uint64_t)x + (uint64_t)cls + 1);
    return splitmix_out(h ^ s);
}

typedef struct {
    const uint8_t *G;
    int64_t ld;
    const uint8_t *y;
    int32_t M, N, k;
    uint64_t begin, end, count, sum;
    uint64_t *table;
    int status;
} digest_job_t;

static void *digest_range(void *arg)
{
    digest_job_t *j = (digest_job_t *)arg;
    j->count = 0;
    j->sum = 0;
    j->status = 0;
    if (j->begin >= j->end)
        return NULL;
    int32_t c[64];
    lex_unrank(j->begin, j->M, j->k, c);
    for (uint64_t r = j->begin; r < j->end; r++) {
        if (oracle_count_table(j->G, j->ld, j->y, j->N, c, j->k, j->table) != 0) {
            j->status = -1;
            return NULL;
        }
        j->sum += digest_term(c, j->k, j->table);
        j->count++;
        if (r + 1 < j->end)
            lex_next(c, j->M, j->k);
    }
    return NULL;
}

/*
 * Number of combinations in the lexicographic rank range [rank_begin,
 * rank_end) (clamped to C(M,k)) and the sum modulo 2^64 of their digest
 * contributions, each table counted one individual at a time, with
 * `nthreads` threads (<= 0: all online cores).  Returns 0, or -1 on invalid
 * arguments / genotype values.
 */
int oracle_digest(const uint8_t *G, int64_t ld, const uint8_t *y, int32_t M, int32_t N, int32_t k,
                  uint64_t rank_begin, uint64_t rank_end, int32_t nthreads, uint64_t *count, uint64_t *digest)
{
    *count = 0;
    *digest = 0;
    if (k < 1 || k > ORACLE_MAX_ORDER || k > M || N < 1)
        return -1;
    uint64_t total = oracle_binomial(M, k);
    if (rank_end > total)
        rank_end = total;
    if (rank_begin >= rank_end)
        return 0;
    if (nthreads <= 0)
        nthreads = (int32_t)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1)
        nthreads = 1;
    uint64_t span = rank_end - rank_begin;
    if ((uint64_t)nthreads > span)
        nthreads = (int32_t)span;
    const int64_t P = pow3(k);
    digest_job_t *jobs = (digest_job_t *)calloc((size_t)nthreads, sizeof(digest_job_t));
    pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int32_t t = 0; t < nthreads; t++) {
        digest_job_t *j = &jobs[t];
        j->G = G;
        j->ld = ld;
        j->y = y;
        j->M = M;
        j->N = N;
        j->k = k;
        j->begin = rank_begin + span * (uint64_t)t / (uint64_t)nthreads;
        j->end = rank_begin + span * (uint64_t)(t + 1) / (uint64_t)nthreads;
        j->table = (uint64_t *)calloc((size_t)(2 * P), sizeof(uint64_t));
    }
    for (int32_t t = 1; t < nthreads; t++)
        pthread_create(&tids[t], NULL, digest_range, &jobs[t]);
    digest_range(&jobs[0]);
    for (int32_t t = 1; t < nthreads; t++)
        pthread_join(tids[t], NULL);
    int rc = 0;
    for (int32_t t = 0; t < nthreads; t++) {
        if (jobs[t].status != 0)
            rc = -1;
        *count += jobs[t].count;
        *digest += jobs[t].sum;
        free(jobs[t].table);
    }
    free(jobs);
    free(tids);
    return rc;
}

/* Tables and MI of an explicit list of combinations (n x k indices). */
int oracle_score_list(const uint8_t *G, int64_t ld, const uint8_t *y, int32_t N, int32_t k,
                      const int32_t *combos, int32_t n, double *out_scores, uint64_t *out_tables)
{
    const int64_t P = pow3(k);
    uint64_t *table = (uint64_t *)calloc((size_t)(2 * P), sizeof(uint64_t));
    int rc = 0;
    for (int32_t i = 0; i < n && rc == 0; i++) {
        uint64_t *t = out_tables ? out_tables + (int64_t)i * 2 * P : table;
        if (oracle_count_table(G, ld, y, N, combos + (int64_t)i * k, k, t) != 0)
            rc = -1;
        else
            out_scores[i] = oracle_mi(t, k);
    }
    free(table);
    return rc;
}
