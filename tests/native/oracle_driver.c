/*
 * Driver of the oracle for a sanitizer build (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host code only): random tables of every kind,
 * call sequences with push / pop under every branch policy, the fast mode
 * against the plain mode, a fixpoint, then everything destroyed.  Exits
 * non-zero on any disagreement; the sanitizers abort on a memory or
 * undefined-behaviour error.  Test infrastructure only.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct cto_table cto_table;
int cto_create(const int32_t *, int64_t, int32_t, const int32_t *, const int32_t *, const uint64_t *, cto_table **);
int cto_create_fast(const int32_t *, int64_t, int32_t, const int32_t *, const int32_t *, const uint64_t *,
                    cto_table **);
int cto_create_kind(const int32_t *, int64_t, int32_t, const int32_t *, const int32_t *, const uint64_t *, int32_t,
                    cto_table **);
void cto_destroy(cto_table *);
int cto_layout(const cto_table *, int32_t *, int64_t *, int32_t *, int32_t *);
int cto_get_state(const cto_table *, uint64_t *, uint64_t *, int32_t *);
int cto_propagate(cto_table *, const uint64_t *, uint64_t *, uint64_t *, int32_t);
int cto_push(cto_table *);
int cto_pop(cto_table *);
int cto_last_stats(const cto_table *, int64_t *, int32_t);
int cto_fixpoint(int32_t, cto_table **, const int32_t *, const int32_t *, int32_t, const int32_t *,
                 const uint64_t *, int32_t, uint64_t *, const int32_t *, int32_t, int64_t *);

static uint64_t rs = 88172645463325252ull;
static uint64_t rnd(void) {
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return rs;
}

static int run_table(int kind, int fast) {
    int n = 1 + (int)(rnd() % 5);
    int32_t lo[5], ds[5];
    for (int i = 0; i < n; i++) {
        lo[i] = (int32_t)(rnd() % 5) - 2;
        ds[i] = 1 + (int32_t)(rnd() % 70);
    }
    int64_t t = (int64_t)(rnd() % 300);
    int32_t *tup = (int32_t *)malloc(sizeof(int32_t) * (size_t)(t * n + 1));
    int64_t k = 0;
    for (int64_t j = 0; j < t; j++) {
        for (int i = 0; i < n; i++) {
            int32_t v = lo[i] + (int32_t)(rnd() % (uint64_t)(ds[i] + 1));
            if (kind == 0 && rnd() % 8 == 0) v = (int32_t)0x80000000; /* star */
            tup[k * n + i] = v;
        }
        /* a negative table lists distinct tuples: drop a repeat */
        int dup = 0;
        for (int64_t p = 0; kind == 1 && p < k && !dup; p++)
            dup = memcmp(tup + p * n, tup + k * n, sizeof(int32_t) * n) == 0;
        if (!dup) k++;
    }
    t = k;
    cto_table *T = NULL, *P = NULL;
    int st = fast ? cto_create_fast(tup, t, n, lo, ds, NULL, &T) : cto_create_kind(tup, t, n, lo, ds, NULL, kind, &T);
    int sp = cto_create_kind(tup, t, n, lo, ds, NULL, kind, &P);
    free(tup);
    if (st != sp) return 1;
    if (!T) return st == 1 ? 0 : (st < 0 ? 0 : 1);
    int32_t D = 0, rows = 0, depth = 0;
    int64_t W = 0;
    cto_layout(T, &D, &W, &rows, &depth);
    uint64_t *dom = calloc((size_t)D + 1, 8), *out1 = calloc((size_t)D + 1, 8), *out2 = calloc((size_t)D + 1, 8);
    uint64_t *c1 = calloc((size_t)W + 1, 8), *c2 = calloc((size_t)W + 1, 8);
    int32_t f = 0;
    int bad = 0;
    for (int step = 0; step < 40 && !bad; step++) {
        cto_get_state(P, dom, NULL, &f);
        if (f) break;
        for (int q = 0; q < D; q++) dom[q] &= rnd() | rnd();
        int mode = (int)(rnd() % 3);
        if (cto_push(T) != cto_push(P)) bad = 1;
        int a = cto_propagate(T, dom, out1, c1, mode);
        int b = cto_propagate(P, dom, out2, c2, mode);
        int64_t stats[16];
        cto_last_stats(T, stats, 16);
        if (a != b) bad = 1;
        if (a == 0 && (memcmp(out1, out2, 8 * (size_t)D) || memcmp(c1, c2, 8 * (size_t)W))) bad = 1;
        if (a != 0 || rnd() % 3 == 0) {
            if (cto_pop(T) != cto_pop(P)) bad = 1;
        }
    }
    /* errors: stray bits, not a subset, pop at depth 0 */
    while (cto_pop(T) == 0) cto_pop(P);
    free(dom); free(out1); free(out2); free(c1); free(c2);
    cto_destroy(T);
    cto_destroy(P);
    return bad;
}

static int run_fixpoint(void) {
    enum { NP = 8, NT = 5 };
    int32_t pool_ds[NP], pool_off[NP];
    int words = 0;
    for (int v = 0; v < NP; v++) {
        pool_ds[v] = 2 + (int32_t)(rnd() % 6);
        pool_off[v] = words++;
    }
    cto_table *tabs[NT];
    int32_t scope_off[NT + 1], scopes[NT * 3];
    scope_off[0] = 0;
    for (int c = 0; c < NT; c++) {
        int32_t lo[3] = {0, 0, 0}, ds[3], sc[3];
        for (int i = 0; i < 3; i++) {
            sc[i] = (int32_t)((c + 2 * i) % NP);
            ds[i] = pool_ds[sc[i]];
            scopes[3 * c + i] = sc[i];
        }
        scope_off[c + 1] = 3 * (c + 1);
        int32_t tup[3 * 20];
        for (int j = 0; j < 20; j++)
            for (int i = 0; i < 3; i++) tup[3 * j + i] = (int32_t)(rnd() % (uint64_t)ds[i]);
        if (cto_create_fast(tup, 20, 3, lo, ds, NULL, &tabs[c]) < 0 || !tabs[c]) return 1;
    }
    uint64_t pin[NP], pout[NP];
    for (int v = 0; v < NP; v++) pin[v] = (1ull << pool_ds[v]) - 1;
    int64_t props = 0;
    int32_t seed[2] = {1, 3};
    cto_fixpoint(NT, tabs, scope_off, scopes, NP, pool_off, pin, NP, pout, NULL, -1, &props);
    cto_fixpoint(NT, tabs, scope_off, scopes, NP, pool_off, pin, NP, pout, seed, 2, &props);
    for (int c = 0; c < NT; c++) cto_destroy(tabs[c]);
    return 0;
}

int main(void) {
    int bad = 0;
    for (int r = 0; r < 300 && !bad; r++) bad |= run_table((int)(r % 2), r % 3 == 0 && r % 2 == 0);
    for (int r = 0; r < 20 && !bad; r++) bad |= run_fixpoint();
    printf(bad ? "oracle driver: disagreement\n" : "oracle driver: ok\n");
    return bad;
}
