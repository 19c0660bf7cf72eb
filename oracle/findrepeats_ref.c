/*
 * Reference (oracle) implementation of FindRepeats -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain CPU oracle that the GPU library is checked against.
 * Nothing in the product path may link, load or call it: only the tests, the
 * smoke check and the benchmark's CPU-baseline leg use it.  It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * What it computes: Algorithm 2 ("Non-overlapping repeated sub-strings") of
 * Yadav et al., "Automatic Tracing in Task-Based Runtime Systems" (ASPLOS'25),
 * Section 4.2, with the O(n log n) realisation the same section describes in
 * its implementation paragraph (mark array for the intersection test, a
 * per-substring ID in the sort key so deduplication happens during selection).
 *
 * Readings of points the paper leaves open (each also listed in the design notes):
 *   - tokens are ordered as unsigned integers; substrings lexicographically;
 *   - a suffix that is a proper prefix of another sorts first;
 *   - LCP[i] is the common prefix of suffixes SA[i] and SA[i+1] (length n-1);
 *   - (p+d)/2 is floor division; the overlap branch uses base = min(s1,s2);
 *   - candidates shorter than min_len are dropped (min_len >= 1, inclusive);
 *   - duplicate (length, start) candidates are kept (the copy always loses);
 *   - the substring ID of a candidate from pair i with length l is
 *     1 + max{ j < i : LCP[j] < l } (0 if none), i.e. the suffix-array left
 *     boundary of the l-interval holding pair i.  For equal l this orders
 *     candidates exactly as comparing the substrings does;
 *   - the intersection test looks at positions s and s+l-1;
 *   - output: accepted occurrences in acceptance order, plus one row per
 *     distinct substring (first accepted start, length, count) in order of
 *     first acceptance.
 *
 * Every step is the textbook method, written for clarity, not speed:
 *   suffix array : prefix doubling (Karp-Miller-Rosenberg / Manber-Myers),
 *                  each round a pair of stable counting sorts;
 *   LCP          : Kasai et al. (2001);
 *   IDs          : one left-to-right sweep with a monotone stack of
 *                  previous-smaller LCP values and a binary search per query;
 *   sort         : qsort with an explicit (length desc, ID asc, start asc)
 *                  comparator;
 *   selection    : the mark-array greedy.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t len;
    int64_t id;
    int64_t start;
    int64_t pair;
} ref_cand;

/* ------------------------------------------------------------------ */
/* Suffix array (Section 4.2: SuffixArray(S)).                         */
/* ------------------------------------------------------------------ */

typedef struct { uint64_t tok; int64_t idx; } tok_idx;

static int cmp_tok_idx(const void *a, const void *b)
{
    const tok_idx *x = (const tok_idx *)a, *y = (const tok_idx *)b;
    if (x->tok < y->tok) return -1;
    if (x->tok > y->tok) return 1;
    if (x->idx < y->idx) return -1;
    if (x->idx > y->idx) return 1;
    return 0;
}

/*
 * Dense token rank: rank[i] = 1 + #{distinct token values < t[i]}.
 * Returns sigma (number of distinct values).  0 is kept for "past the end".
 */
int64_t ref_token_ranks(const uint64_t *t, int64_t n, int64_t *rank)
{
    if (n <= 0) return 0;
    tok_idx *v = (tok_idx *)malloc(sizeof(tok_idx) * (size_t)n);
    if (!v) return -1;
    for (int64_t i = 0; i < n; i++) { v[i].tok = t[i]; v[i].idx = i; }
    qsort(v, (size_t)n, sizeof(tok_idx), cmp_tok_idx);
    int64_t r = 0;
    for (int64_t k = 0; k < n; k++) {
        if (k == 0 || v[k].tok != v[k - 1].tok) r++;
        rank[v[k].idx] = r;
    }
    free(v);
    return r;
}

/*
 * Suffix array by prefix doubling.  Round h sorts suffixes by the pair
 * (rank_h[i], rank_h[i+h]) (0 past the end) with two stable counting sorts
 * (second key first), then renumbers ranks densely.  Stops once every rank is
 * distinct.  `active_per_round`, when non-NULL, receives the number of
 * suffixes that still share their h-prefix with another suffix at the start
 * of each round (room for 64 rounds); the return value is the number of
 * rounds run, or -1 on allocation failure.
 */
int64_t ref_suffix_array(const uint64_t *t, int64_t n, int64_t *sa,
                         int64_t *active_per_round)
{
    if (n <= 0) return 0;
    int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *nr = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 2));
    if (!rank || !tmp || !nr || !cnt) {
        free(rank); free(tmp); free(nr); free(cnt);
        return -1;
    }
    int64_t maxr = ref_token_ranks(t, n, rank);
    /* initial order: by first token (counting sort on rank, stable by index) */
    memset(cnt, 0, sizeof(int64_t) * (size_t)(n + 2));
    for (int64_t i = 0; i < n; i++) cnt[rank[i]]++;
    for (int64_t r = 1; r <= n + 1; r++) cnt[r] += cnt[r - 1];
    for (int64_t i = n - 1; i >= 0; i--) sa[--cnt[rank[i]]] = i;

    int64_t rounds = 0;
    for (int64_t h = 1; maxr < n; h *= 2) {
        if (active_per_round && rounds < 64) {
            /* suffixes in groups of size >= 2 (groups are runs of equal rank in sa order) */
            int64_t act = 0;
            for (int64_t k = 0; k < n; k++) {
                int same_prev = k > 0 && rank[sa[k]] == rank[sa[k - 1]];
                int same_next = k + 1 < n && rank[sa[k]] == rank[sa[k + 1]];
                if (same_prev || same_next) act++;
            }
            active_per_round[rounds] = act;
        }
        rounds++;
        /* stable counting sort by second key rank[i+h] (0 past the end) */
        memset(cnt, 0, sizeof(int64_t) * (size_t)(n + 2));
        for (int64_t i = 0; i < n; i++) cnt[i + h < n ? rank[i + h] : 0]++;
        for (int64_t r = 1; r <= n + 1; r++) cnt[r] += cnt[r - 1];
        for (int64_t i = n - 1; i >= 0; i--) tmp[--cnt[i + h < n ? rank[i + h] : 0]] = i;
        /* stable counting sort by first key rank[i] */
        memset(cnt, 0, sizeof(int64_t) * (size_t)(n + 2));
        for (int64_t i = 0; i < n; i++) cnt[rank[i]]++;
        for (int64_t r = 1; r <= n + 1; r++) cnt[r] += cnt[r - 1];
        for (int64_t k = n - 1; k >= 0; k--) sa[--cnt[rank[tmp[k]]]] = tmp[k];
        /* dense renumbering */
        int64_t r = 0;
        for (int64_t k = 0; k < n; k++) {
            int64_t a = sa[k];
            if (k == 0) r = 1;
            else {
                int64_t b = sa[k - 1];
                int64_t a2 = a + h < n ? rank[a + h] : 0;
                int64_t b2 = b + h < n ? rank[b + h] : 0;
                if (rank[a] != rank[b] || a2 != b2) r++;
            }
            nr[a] = r;
        }
        memcpy(rank, nr, sizeof(int64_t) * (size_t)n);
        maxr = r;
    }
    free(rank); free(tmp); free(nr); free(cnt);
    return rounds;
}

/* ------------------------------------------------------------------ */
/* LCP array, Kasai et al.  lcp[i] = lcp(SA[i], SA[i+1]), i < n-1.      */
/* ------------------------------------------------------------------ */
int ref_lcp(const uint64_t *t, int64_t n, const int64_t *sa, int64_t *lcp)
{
    if (n < 2) return 0;
    int64_t *inv = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!inv) return -1;
    for (int64_t k = 0; k < n; k++) inv[sa[k]] = k;
    int64_t h = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t k = inv[i];
        if (k + 1 < n) {
            int64_t j = sa[k + 1];
            while (i + h < n && j + h < n && t[i + h] == t[j + h]) h++;
            lcp[k] = h;
            if (h > 0) h--;
        } else {
            h = 0;
        }
    }
    free(inv);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Candidate generation (the loop over adjacent suffix-array pairs).    */
/* ------------------------------------------------------------------ */

/*
 * Emits, for every adjacent pair i, the two candidates of the paper's loop
 * body, keeping those with length >= min_len.  Each candidate also gets the
 * substring ID described in the header.  `out` needs room for 2(n-1)
 * entries; returns the number written.
 */
int64_t ref_candidates(const uint64_t *t, int64_t n, const int64_t *sa,
                       const int64_t *lcp, int64_t min_len, ref_cand *out)
{
    (void)t;
    if (n < 2) return 0;
    /* stack of pair indices j < i whose LCP is smaller than every LCP after them */
    int64_t *stk = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!stk) return -1;
    int64_t top = 0; /* number of entries */
    int64_t m = 0;
    for (int64_t i = 0; i + 1 < n; i++) {
        int64_t s1 = sa[i], s2 = sa[i + 1], p = lcp[i];
        int64_t lo = s1 < s2 ? s1 : s2, hi = s1 < s2 ? s2 : s1;
        int64_t l, a, b;
        if (lo + p <= hi) {
            /* [s1,s1+p) and [s2,s2+p) are disjoint */
            l = p; a = s1; b = s2;
        } else {
            int64_t d = hi - lo;
            l = (p + d) / 2;
            l -= l % d;
            a = lo; b = lo + l;
        }
        if (l >= min_len) {
            /* ID: 1 + last j < i with lcp[j] < l; stack LCPs increase bottom->top */
            int64_t L = 0, R = top; /* find count of stack entries with lcp < l */
            while (L < R) {
                int64_t mid = (L + R) / 2;
                if (lcp[stk[mid]] < l) L = mid + 1; else R = mid;
            }
            int64_t id = L == 0 ? 0 : stk[L - 1] + 1;
            out[m].len = l; out[m].id = id; out[m].start = a; out[m].pair = i; m++;
            out[m].len = l; out[m].id = id; out[m].start = b; out[m].pair = i; m++;
        }
        while (top > 0 && lcp[stk[top - 1]] >= p) top--;
        stk[top++] = i;
    }
    free(stk);
    return m;
}

static int cmp_cand(const void *x, const void *y)
{
    const ref_cand *a = (const ref_cand *)x, *b = (const ref_cand *)y;
    if (a->len != b->len) return a->len > b->len ? -1 : 1;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    if (a->start != b->start) return a->start < b->start ? -1 : 1;
    if (a->pair != b->pair) return a->pair < b->pair ? -1 : 1;
    return 0;
}

/* Sort(C): decreasing length, increasing substring (via ID), increasing start. */
void ref_sort_candidates(ref_cand *c, int64_t m)
{
    if (m > 1) qsort(c, (size_t)m, sizeof(ref_cand), cmp_cand);
}

/* ------------------------------------------------------------------ */
/* Whole algorithm.                                                     */
/* ------------------------------------------------------------------ */

/*
 * FindRepeats(S).  Outputs (caller-allocated, capacity n each):
 *   occ_start/occ_len/occ_row : accepted occurrences, acceptance order;
 *   row_start/row_len/row_count : one row per distinct accepted substring,
 *                                 first-acceptance order.
 * stats[0..7] (if non-NULL): candidates kept (length >= min_len), rounds of
 * doubling, sum over rounds of active suffixes, coverage (sum of accepted
 * lengths), number of occurrences, number of rows, max LCP, distinct tokens.
 * Returns 0, -1 on bad arguments, -2 on allocation failure.
 */
int ref_find_repeats(const uint64_t *t, int64_t n, int64_t min_len,
                     int64_t *occ_start, int64_t *occ_len, int64_t *occ_row, int64_t *n_occ,
                     int64_t *row_start, int64_t *row_len, int64_t *row_count, int64_t *n_rows,
                     int64_t *stats)
{
    if (min_len < 1 || n < 0 || !n_occ || !n_rows) return -1;
    *n_occ = 0; *n_rows = 0;
    if (stats) memset(stats, 0, sizeof(int64_t) * 8);
    if (n < 2) return 0;
    int rc = 0;
    int64_t *sa = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *lcp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    ref_cand *c = (ref_cand *)malloc(sizeof(ref_cand) * (size_t)(2 * n));
    unsigned char *mark = (unsigned char *)calloc((size_t)n, 1);
    int64_t act[64];
    memset(act, 0, sizeof(act));
    if (!sa || !lcp || !c || !mark) { rc = -2; goto done; }
    int64_t rounds = ref_suffix_array(t, n, sa, act);
    if (rounds < 0) { rc = -2; goto done; }
    if (ref_lcp(t, n, sa, lcp) != 0) { rc = -2; goto done; }
    int64_t m = ref_candidates(t, n, sa, lcp, min_len, c);
    if (m < 0) { rc = -2; goto done; }
    ref_sort_candidates(c, m);

    int64_t no = 0, nrow = 0, cov = 0;
    int64_t cur_len = -1, cur_id = -1;
    for (int64_t k = 0; k < m; k++) {
        int64_t s = c[k].start, l = c[k].len;
        if (mark[s] || mark[s + l - 1]) continue;
        for (int64_t x = s; x < s + l; x++) mark[x] = 1;
        if (c[k].len != cur_len || c[k].id != cur_id) {
            cur_len = c[k].len; cur_id = c[k].id;
            if (row_start) row_start[nrow] = s;
            if (row_len) row_len[nrow] = l;
            if (row_count) row_count[nrow] = 0;
            nrow++;
        }
        if (row_count) row_count[nrow - 1]++;
        if (occ_start) occ_start[no] = s;
        if (occ_len) occ_len[no] = l;
        if (occ_row) occ_row[no] = nrow - 1;
        no++;
        cov += l;
    }
    *n_occ = no; *n_rows = nrow;
    if (stats) {
        int64_t sum_act = 0, maxl = 0;
        for (int r = 0; r < 64 && r < rounds; r++) sum_act += act[r];
        for (int64_t i = 0; i + 1 < n; i++) if (lcp[i] > maxl) maxl = lcp[i];
        stats[0] = m; stats[1] = rounds; stats[2] = sum_act; stats[3] = cov;
        stats[4] = no; stats[5] = nrow; stats[6] = maxl;
        int64_t *rk = sa; /* reuse: distinct-token count */
        stats[7] = ref_token_ranks(t, n, rk);
    }
done:
    free(sa); free(lcp); free(c); free(mark);
    return rc;
}

/* Per-stage entry points for stage-by-stage parity checks. */
int64_t ref_sorted_candidates(const uint64_t *t, int64_t n, int64_t min_len,
                              int64_t *len, int64_t *id, int64_t *start, int64_t *pair)
{
    if (n < 2) return 0;
    int64_t *sa = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *lcp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    ref_cand *c = (ref_cand *)malloc(sizeof(ref_cand) * (size_t)(2 * n));
    int64_t m = -2;
    if (sa && lcp && c && ref_suffix_array(t, n, sa, NULL) >= 0 && ref_lcp(t, n, sa, lcp) == 0) {
        m = ref_candidates(t, n, sa, lcp, min_len, c);
        if (m >= 0) {
            ref_sort_candidates(c, m);
            for (int64_t k = 0; k < m; k++) {
                len[k] = c[k].len; id[k] = c[k].id; start[k] = c[k].start; pair[k] = c[k].pair;
            }
        }
    }
    free(sa); free(lcp); free(c);
    return m;
}
