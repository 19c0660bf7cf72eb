/* Runs every entry point of the C oracle on small seeded inputs (random over
 * small alphabets, constant runs, periodic strings, the empty and one-token
 * strings, extreme token values) for a sanitizer build.  Exits non-zero if
 * an entry point reports an error or an invariant of its output fails. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t ref_token_ranks(const uint64_t *t, int64_t n, int64_t *rank);
int64_t ref_suffix_array(const uint64_t *t, int64_t n, int64_t *sa, int64_t *active);
int ref_lcp(const uint64_t *t, int64_t n, const int64_t *sa, int64_t *lcp);
int ref_find_repeats(const uint64_t *t, int64_t n, int64_t min_len, int64_t *occ_start, int64_t *occ_len,
                     int64_t *occ_row, int64_t *n_occ, int64_t *row_start, int64_t *row_len, int64_t *row_count,
                     int64_t *n_rows, int64_t *stats);
int64_t ref_sorted_candidates(const uint64_t *t, int64_t n, int64_t min_len, int64_t *len, int64_t *id,
                              int64_t *start, int64_t *pair);

static uint64_t state = 88172645463325252ull;
static uint64_t next(void) {
    state ^= state << 13; state ^= state >> 7; state ^= state << 17;
    return state;
}

static int run(const uint64_t *t, int64_t n) {
    int64_t cap = n > 0 ? n : 1;
    int64_t *a = malloc(sizeof(int64_t) * (size_t)cap * 2), *b = malloc(sizeof(int64_t) * (size_t)cap * 2);
    int64_t *c = malloc(sizeof(int64_t) * (size_t)cap * 2), *d = malloc(sizeof(int64_t) * (size_t)cap * 2);
    int64_t *e = malloc(sizeof(int64_t) * (size_t)cap), *f = malloc(sizeof(int64_t) * (size_t)cap);
    int64_t act[64], stats[8], no = 0, nr = 0;
    int bad = 0;
    if (ref_token_ranks(t, n, e) < 0) bad = 1;
    int64_t rounds = ref_suffix_array(t, n, a, act);
    if (rounds < 0) bad = 1;
    if (n >= 2) {
        if (ref_lcp(t, n, a, b) != 0) bad = 1;
        for (int64_t i = 0; i + 1 < n; i++)
            if (b[i] < 0 || b[i] > n) bad = 1;
    }
    for (int64_t m = 1; m <= 9; m += 4) {
        if (ref_sorted_candidates(t, n, m, a, b, c, d) < 0) bad = 1;
        if (ref_find_repeats(t, n, m, a, b, c, &no, d, e, f, &nr, stats) != 0) bad = 1;
        int64_t cov = 0;
        for (int64_t k = 0; k < no; k++) {
            if (a[k] < 0 || a[k] + b[k] > n || b[k] < m) bad = 1;
            cov += b[k];
        }
        if (cov > n || nr > no) bad = 1;
    }
    free(a); free(b); free(c); free(d); free(e); free(f);
    return bad;
}

int main(void) {
    int bad = 0;
    static uint64_t t[6000];
    bad |= run(t, 0);
    t[0] = 5;
    bad |= run(t, 1);
    for (int trial = 0; trial < 60; trial++) {
        int64_t n = 1 + (int64_t)(next() % 3000);
        uint64_t alpha = 1 + next() % 6;
        for (int64_t i = 0; i < n; i++) t[i] = next() % alpha;
        bad |= run(t, n);
    }
    for (int64_t i = 0; i < 5000; i++) t[i] = 7;
    bad |= run(t, 5000);
    for (int64_t i = 0; i < 6000; i++) t[i] = (uint64_t)(i % 41) * 0x9E3779B97F4A7C15ull;
    bad |= run(t, 6000);
    for (int64_t i = 0; i < 3000; i++) t[i] = (i % 3 == 0) ? UINT64_MAX : (i % 3 == 1) ? 0 : (1ull << 63);
    bad |= run(t, 3000);
    if (bad) {
        fprintf(stderr, "oracle driver: an entry point failed\n");
        return 1;
    }
    printf("oracle driver ok\n");
    return 0;
}
