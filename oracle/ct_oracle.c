/*
 * ct_oracle.c -- plain serial Compact-Table (CT) propagation for the positive
 * table constraint.  TEST INFRASTRUCTURE ONLY: this file is the oracle that
 * the GPU library is checked against.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark load it; the product path never does.
 * It shares no code, header or constant table with the HIP library.
 *
 * Source: E. Santi, F. Tardivo, A. Dovier, A. Formisano, "GPU Accelerated
 * Compact-Table Propagation" (arXiv 2507.18413):
 *   - supports / currTable / valid tuple: Sec. 2, definitions after Alg. 2;
 *   - enforceGAC: Alg. 1;  updateTable: Alg. 2;  filterDomains: Alg. 3;
 *   - supportJmp / variablesOffsets indexing and the constructor's
 *     satisfiability check: Sec. 3 ("Data structures", "Procedures");
 *   - GAC and propagation to a fixpoint: Sec. 2, first paragraphs.
 *
 * The plain mode is dense and direct: one uint64 word holds 64 tuples (tuple
 * j is bit j%64 of word j/64), every support row has W = ceil(t/64) words, no
 * sparse word list, no residues, and backtracking keeps a full snapshot of
 * the propagator state per level.  The fast mode (cto_create_fast) reaches
 * the same results with CT's economies -- the list of non-zero currTable
 * words, residues checked first by filterDomains (Sec. 2), a trail of
 * currTable words -- and serves as the timed serial baseline; both modes
 * count the work of each call (cto_last_stats).  Readings of points the
 * paper leaves open:
 *   - the incremental branch (OR over the removed values, then complement) is
 *     taken iff |Delta_i| < |dom(x_i)| (strict, as printed in Alg. 2); the
 *     branch labels printed as comments in Alg. 2 are swapped relative to the
 *     prose, and the code lines and prose are followed;
 *   - dom(x_i) in Alg. 2/3 is the domain after the removals in Delta;
 *   - Delta_i is the set of values present after the previous call of this
 *     propagator (its output domains) and absent from the new input;
 *   - at creation every variable takes the reset branch over its initial
 *     domain, so tuples holding values outside a domain are never valid;
 *   - a failed state accepts only pop; pop below depth 0 is an error.
 *
 * parity unpinned: none of the functions.  Results of both modes are pinned
 * by the tests against brute-force GAC, the paper's Table 1 and closed-form
 * invariants; the fast mode also against the plain mode call by call; the
 * work counters by hand counts on Table 1 and by counts taken from the
 * previous call's currTable.
 */
#define _GNU_SOURCE /* qsort_r */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CTO_OK 0
#define CTO_FAIL 1
#define CTO_E_INVALID (-1)
#define CTO_E_NOT_SUBSET (-2)
#define CTO_E_STATE (-3)
#define CTO_E_NOMEM (-4)

#define CTO_KIND_POSITIVE 0    /* the tuples list the allowed combinations */
#define CTO_KIND_NEGATIVE 1    /* the tuples list the forbidden combinations */
#define CTO_STAR ((int32_t)0x80000000)  /* a cell of a short table: any value */

#define CTO_MODE_AUTO 0        /* Alg. 2's branch rule */
#define CTO_MODE_RESET 1       /* always OR over dom(x_i)  */
#define CTO_MODE_INCREMENTAL 2 /* always OR over Delta_i, complement */

/* per-call work counters (cto_last_stats) */
enum {
    CTO_ST_NZ_WORDS = 0,  /* non-zero currTable words at entry */
    CTO_ST_ROWS_OR,       /* support rows OR-ed by updateTable (up to Alg. 2's break) */
    CTO_ST_SVAL,          /* |s_val| */
    CTO_ST_SSUP,          /* |s_sup| */
    CTO_ST_NZ_GRANULES,   /* 64-word groups of currTable holding a non-zero word at entry */
    CTO_ST_ROWS_SEL,      /* rows Alg. 2's branch rule selects over all of s_val:
                             sum of |Delta_i| (incremental) or |dom(x_i)| (reset) */
    CTO_ST_RES_CHECKS,    /* fast mode: values tested by filterDomains */
    CTO_ST_RES_MISSES,    /* fast mode: residue word no longer intersecting */
    CTO_ST_SCAN_WORDS,    /* fast mode: words scanned after residue misses */
    CTO_ST_UPD_WORDS,     /* support words read by updateTable */
    CTO_NSTATS
};

typedef struct {
    int n;
    int64_t t, W;
    int rows, D;
    int32_t *lo, *dsz, *row_start, *dom_off, *dom_words;
    int kind;           /* CTO_KIND_POSITIVE or CTO_KIND_NEGATIVE */
    int has_star;       /* a short table: some cell holds CTO_STAR */
    uint64_t *S;        /* rows x W: supports[x_i, v] (Sec. 2); a star cell
                           supports every value of its column */
    uint64_t *S_strict; /* short tables only: the cells that name v itself */
    uint64_t *ct;       /* W: currTable */
    uint64_t *last_dom; /* D: domains after the previous call */
    int32_t *last_sizes;/* n: lastSizes of Alg. 1 */
    int failed;
    /* snapshot stack for push/pop */
    int depth, cap;
    uint64_t *snap_ct, *snap_dom;
    int32_t *snap_sizes, *snap_failed;
    /* counters of the last propagate call (work done, not results) */
    int64_t st[CTO_NSTATS];
    /* fast mode (cto_create_fast): the sparse form of currTable, residues
     * and a word trail instead of snapshots of currTable */
    int fast;
    int32_t *idx;        /* W: permutation of the word ids; idx[0..limit) are
                            the non-zero words of ct */
    int64_t limit;
    int32_t *res;        /* rows: residue word of each (x_i, a) */
    uint64_t *fmask;     /* W: mask scratch */
    int32_t *stamp;      /* W: serial of the level that last saved the word */
    int32_t serial, next_serial;
    int64_t tr_top, tr_cap;
    int32_t *tr_w;       /* trail: word id and old value */
    uint64_t *tr_v;
    int64_t *lv_top, *lv_limit;  /* per level: trail top, limit, serial */
    int32_t *lv_serial;
} cto_table;

static int popc(uint64_t x) { return __builtin_popcountll(x); }

static int var_size(const cto_table *T, const uint64_t *dom, int i) {
    int s = 0;
    for (int k = 0; k < T->dom_words[i]; k++) s += popc(dom[T->dom_off[i] + k]);
    return s;
}

static int has_value(const cto_table *T, const uint64_t *dom, int i, int a) {
    return (int)((dom[T->dom_off[i] + a / 64] >> (a % 64)) & 1u);
}

static uint64_t *row_ptr(const cto_table *T, int i, int a) {
    /* supportJmp[i] + (v - variablesOffsets[i]) of Sec. 3, with a = v - lo_i */
    return T->S + (int64_t)(T->row_start[i] + a) * T->W;
}

/* the row OR-ed by the incremental branch: a removed value invalidates only
 * the tuples that name it (a star cell keeps its tuple valid while the
 * column's domain is not empty) */
static uint64_t *strict_row_ptr(const cto_table *T, int i, int a) {
    if (!T->S_strict) return row_ptr(T, i, a);
    return T->S_strict + (int64_t)(T->row_start[i] + a) * T->W;
}

static int any_word(const uint64_t *x, int64_t W) {
    for (int64_t w = 0; w < W; w++)
        if (x[w]) return 1;
    return 0;
}

/* 64-word groups of x holding a non-zero word (a work count) */
static int64_t nonzero_granules(const uint64_t *x, int64_t W) {
    int64_t g = 0;
    for (int64_t w0 = 0; w0 < W; w0 += 64) {
        int64_t e = w0 + 64 < W ? w0 + 64 : W;
        if (any_word(x + w0, e - w0)) g++;
    }
    return g;
}

/* tail bits of each variable's last word must be zero */
static int stray_bits(const cto_table *T, const uint64_t *dom) {
    for (int i = 0; i < T->n; i++) {
        int d = T->dsz[i];
        int last = T->dom_off[i] + T->dom_words[i] - 1;
        int used = d - 64 * (T->dom_words[i] - 1);
        if (used < 64 && (dom[last] >> used) != 0) return 1;
    }
    return 0;
}

/* filterDomains (Alg. 3) over the variables flagged in s_sup; dom is edited */
static void filter_domains(cto_table *T, uint64_t *dom, const char *s_sup) {
    for (int i = 0; i < T->n; i++) {
        if (!s_sup[i]) continue;
        for (int a = 0; a < T->dsz[i]; a++) {
            if (!has_value(T, dom, i, a)) continue;
            const uint64_t *r = row_ptr(T, i, a);
            int supported = 0;
            for (int64_t w = 0; w < T->W; w++)
                if (T->ct[w] & r[w]) { supported = 1; break; }
            if (!supported) dom[T->dom_off[i] + a / 64] &= ~(1ull << (a % 64));
        }
        T->last_sizes[i] = var_size(T, dom, i);
    }
}

void cto_destroy(cto_table *T) {
    if (!T) return;
    free(T->lo); free(T->dsz); free(T->row_start); free(T->dom_off); free(T->dom_words);
    free(T->S); free(T->S_strict); free(T->ct); free(T->last_dom); free(T->last_sizes);
    free(T->snap_ct); free(T->snap_dom); free(T->snap_sizes); free(T->snap_failed);
    free(T->idx); free(T->res); free(T->fmask); free(T->stamp); free(T->tr_w); free(T->tr_v);
    free(T->lv_top); free(T->lv_limit); free(T->lv_serial);
    free(T);
}

/*
 * Build supports (Sec. 2: cell ([x_i, v], j) is 1 iff tau_j[i] = v) and run
 * the root propagation (Sec. 3, constructor).  Returns CTO_OK, CTO_FAIL (the
 * handle exists, in the failed state), or an error with *out = NULL.
 */
/* qsort_r comparator of tuple indices by their rows */
static int cmp_rows(const void *pa, const void *pb, void *arg) {
    const int32_t *tup = (const int32_t *)((void **)arg)[0];
    const int n = *(const int *)((void **)arg)[1];
    const int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    for (int i = 0; i < n; i++) {
        int32_t x = tup[a * n + i], y = tup[b * n + i];
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

/* 1 if two tuples are equal (sort of the indices) */
static int has_duplicates(const int32_t *tuples, int64_t t, int n) {
    if (t < 2) return 0;
    int64_t *ix = (int64_t *)malloc(sizeof(int64_t) * t);
    if (!ix) return -1;
    for (int64_t j = 0; j < t; j++) ix[j] = j;
    int nn = n;
    void *arg[2] = {(void *)tuples, &nn};
    qsort_r(ix, (size_t)t, sizeof(int64_t), cmp_rows, arg);
    int dup = 0;
    for (int64_t j = 1; j < t && !dup; j++) dup = cmp_rows(&ix[j - 1], &ix[j], arg) == 0;
    free(ix);
    return dup;
}

static int filter_negative(cto_table *T, uint64_t *dom);

static int create_impl(const int32_t *tuples, int64_t t, int32_t n, const int32_t *lo,
                       const int32_t *dsz, const uint64_t *init_dom, int32_t kind, cto_table **out) {
    *out = NULL;
    if (n < 1 || t < 0 || !lo || !dsz || (t > 0 && !tuples)) return CTO_E_INVALID;
    if (kind != CTO_KIND_POSITIVE && kind != CTO_KIND_NEGATIVE) return CTO_E_INVALID;
    for (int i = 0; i < n; i++)
        if (dsz[i] < 1) return CTO_E_INVALID;
    int star = 0;
    for (int64_t k = 0; k < t * n && !star; k++) star = tuples[k] == CTO_STAR;
    /* a negative table lists distinct combinations and has no star cell */
    if (kind == CTO_KIND_NEGATIVE && (star || has_duplicates(tuples, t, n) != 0)) return CTO_E_INVALID;
    cto_table *T = (cto_table *)calloc(1, sizeof(cto_table));
    if (!T) return CTO_E_NOMEM;
    T->kind = kind;
    T->has_star = star;
    T->n = n;
    T->t = t;
    T->W = (t + 63) / 64;
    T->lo = (int32_t *)malloc(sizeof(int32_t) * n);
    T->dsz = (int32_t *)malloc(sizeof(int32_t) * n);
    T->row_start = (int32_t *)malloc(sizeof(int32_t) * n);
    T->dom_off = (int32_t *)malloc(sizeof(int32_t) * n);
    T->dom_words = (int32_t *)malloc(sizeof(int32_t) * n);
    T->last_sizes = (int32_t *)malloc(sizeof(int32_t) * n);
    if (!T->lo || !T->dsz || !T->row_start || !T->dom_off || !T->dom_words || !T->last_sizes) {
        cto_destroy(T);
        return CTO_E_NOMEM;
    }
    int rows = 0, D = 0;
    for (int i = 0; i < n; i++) {
        T->lo[i] = lo[i];
        T->dsz[i] = dsz[i];
        T->row_start[i] = rows;
        T->dom_off[i] = D;
        T->dom_words[i] = (dsz[i] + 63) / 64;
        rows += dsz[i];
        D += T->dom_words[i];
    }
    T->rows = rows;
    T->D = D;
    int64_t Wa = T->W > 0 ? T->W : 1;
    T->S = (uint64_t *)calloc((size_t)rows * (size_t)Wa, sizeof(uint64_t));
    T->ct = (uint64_t *)calloc((size_t)Wa, sizeof(uint64_t));
    T->last_dom = (uint64_t *)calloc((size_t)D, sizeof(uint64_t));
    if (star) T->S_strict = (uint64_t *)calloc((size_t)rows * (size_t)Wa, sizeof(uint64_t));
    if (!T->S || !T->ct || !T->last_dom || (star && !T->S_strict)) {
        cto_destroy(T);
        return CTO_E_NOMEM;
    }
    for (int64_t j = 0; j < t; j++) {
        for (int i = 0; i < n; i++) {
            if (tuples[j * n + i] == CTO_STAR) { /* short table: every value of x_i */
                for (int a = 0; a < dsz[i]; a++) row_ptr(T, i, a)[j / 64] |= 1ull << (j % 64);
                continue;
            }
            int64_t v = (int64_t)tuples[j * n + i] - lo[i];
            if (v < 0 || v >= dsz[i]) continue; /* value outside dom0: no row */
            row_ptr(T, i, (int)v)[j / 64] |= 1ull << (j % 64);
            if (star) strict_row_ptr(T, i, (int)v)[j / 64] |= 1ull << (j % 64);
        }
    }
    /* initial domains */
    if (init_dom) {
        memcpy(T->last_dom, init_dom, sizeof(uint64_t) * D);
        if (stray_bits(T, T->last_dom)) {
            cto_destroy(T);
            return CTO_E_INVALID;
        }
    } else {
        for (int i = 0; i < n; i++)
            for (int a = 0; a < dsz[i]; a++) T->last_dom[T->dom_off[i] + a / 64] |= 1ull << (a % 64);
    }
    /* currTable = AND_i OR_{a in dom0_i} supports[x_i, a] (reset branch for all) */
    for (int64_t j = 0; j < t; j++) T->ct[j / 64] |= 1ull << (j % 64);
    uint64_t *mask = (uint64_t *)malloc(sizeof(uint64_t) * Wa);
    char *s_sup = (char *)calloc((size_t)n, 1);
    if (!mask || !s_sup) {
        free(mask); free(s_sup);
        cto_destroy(T);
        return CTO_E_NOMEM;
    }
    for (int i = 0; i < n; i++) {
        memset(mask, 0, sizeof(uint64_t) * Wa);
        for (int a = 0; a < dsz[i]; a++) {
            if (!has_value(T, T->last_dom, i, a)) continue;
            const uint64_t *r = row_ptr(T, i, a);
            for (int64_t w = 0; w < T->W; w++) mask[w] |= r[w];
        }
        for (int64_t w = 0; w < T->W; w++) T->ct[w] &= mask[w];
    }
    free(mask);
    for (int i = 0; i < n; i++) T->last_sizes[i] = var_size(T, T->last_dom, i);
    if (kind == CTO_KIND_NEGATIVE) {
        free(s_sup);
        int st = filter_negative(T, T->last_dom);
        if (st == CTO_FAIL) T->failed = 1;
        *out = T;
        return st;
    }
    if (!any_word(T->ct, T->W)) {
        T->failed = 1;
        free(s_sup);
        *out = T;
        return CTO_FAIL;
    }
    for (int i = 0; i < n; i++) s_sup[i] = T->last_sizes[i] > 1;
    filter_domains(T, T->last_dom, s_sup);
    free(s_sup);
    *out = T;
    return CTO_OK;
}

/*
 * Build supports (Sec. 2: cell ([x_i, v], j) is 1 iff tau_j[i] = v; a star
 * cell of a short table -- the paper's footnote on short tables, Sec. 2 --
 * supports every value of its column) and run the root propagation (Sec. 3,
 * constructor).  Returns CTO_OK, CTO_FAIL (the handle exists, in the failed
 * state), or an error with *out = NULL.
 */
int cto_create(const int32_t *tuples, int64_t t, int32_t n, const int32_t *lo,
               const int32_t *dsz, const uint64_t *init_dom, cto_table **out) {
    return create_impl(tuples, t, n, lo, dsz, init_dom, CTO_KIND_POSITIVE, out);
}

/* cto_create for a positive (kind 0) or negative (kind 1) table.  A negative
 * table lists forbidden combinations (the paper's footnote, Sec. 2): the
 * valid tuples are the combinations of the domains that it does not list;
 * its tuples must be distinct and hold no star (CTO_E_INVALID). */
int cto_create_kind(const int32_t *tuples, int64_t t, int32_t n, const int32_t *lo,
                    const int32_t *dsz, const uint64_t *init_dom, int32_t kind, cto_table **out) {
    return create_impl(tuples, t, n, lo, dsz, init_dom, kind, out);
}

/*
 * filterDomains of a negative table.  currTable holds the listed (forbidden)
 * tuples whose every value is in the current domains.  Value a of x_i has a
 * valid (allowed) tuple iff fewer than prod_{k != i} |dom(x_k)| of the
 * combinations with x_i = a are listed, i.e. iff
 * popcount(currTable & supports[x_i, a]) < prod_{k != i} |dom(x_k)|.
 * Every variable is filtered (a singleton too: its value may have no
 * allowed tuple), each decision on the input domains.  Removing unsupported
 * values removes no allowed tuple, so one pass reaches GAC.  The listed
 * tuples naming a removed value then leave currTable, so that currTable
 * stays the listed tuples valid under the output domains.  CTO_FAIL iff a
 * domain is empty.
 */
static int filter_negative(cto_table *T, uint64_t *dom) {
    const int n = T->n;
    const int64_t cap = T->t + 1; /* a count never exceeds t */
    int32_t *size = (int32_t *)malloc(sizeof(int32_t) * n);
    uint64_t *out = (uint64_t *)malloc(sizeof(uint64_t) * T->D);
    if (!size || !out) {
        free(size); free(out);
        return CTO_E_NOMEM;
    }
    for (int i = 0; i < n; i++) size[i] = var_size(T, dom, i);
    memcpy(out, dom, sizeof(uint64_t) * T->D);
    for (int i = 0; i < n; i++) {
        int64_t prod = 1;
        for (int k = 0; k < n; k++) {
            if (k == i) continue;
            prod *= size[k];
            if (prod > cap) prod = cap;
        }
        for (int a = 0; a < T->dsz[i]; a++) {
            if (!has_value(T, dom, i, a)) continue;
            const uint64_t *r = row_ptr(T, i, a);
            int64_t cnt = 0;
            for (int64_t w = 0; w < T->W; w++) cnt += popc(T->ct[w] & r[w]);
            if (cnt == prod) out[T->dom_off[i] + a / 64] &= ~(1ull << (a % 64));
        }
    }
    int empty = 0;
    for (int i = 0; i < n; i++) {
        for (int a = 0; a < T->dsz[i]; a++) {
            if (!has_value(T, dom, i, a) || has_value(T, out, i, a)) continue;
            const uint64_t *r = row_ptr(T, i, a);
            for (int64_t w = 0; w < T->W; w++) T->ct[w] &= ~r[w];
        }
        T->last_sizes[i] = var_size(T, out, i);
        if (T->last_sizes[i] == 0) empty = 1;
    }
    memcpy(dom, out, sizeof(uint64_t) * T->D);
    free(size); free(out);
    return empty ? CTO_FAIL : CTO_OK;
}

int cto_layout(const cto_table *T, int32_t *D, int64_t *W, int32_t *rows, int32_t *depth) {
    if (!T) return CTO_E_INVALID;
    if (D) *D = T->D;
    if (W) *W = T->W;
    if (rows) *rows = T->rows;
    if (depth) *depth = T->depth;
    return CTO_OK;
}

int cto_get_state(const cto_table *T, uint64_t *dom_out, uint64_t *ct_out, int32_t *failed) {
    if (!T) return CTO_E_INVALID;
    if (dom_out) memcpy(dom_out, T->last_dom, sizeof(uint64_t) * T->D);
    if (ct_out) memcpy(ct_out, T->ct, sizeof(uint64_t) * T->W);
    if (failed) *failed = T->failed;
    return CTO_OK;
}

int cto_support_row(const cto_table *T, int32_t row, uint64_t *out) {
    if (!T || row < 0 || row >= T->rows) return CTO_E_INVALID;
    memcpy(out, T->S + (int64_t)row * T->W, sizeof(uint64_t) * T->W);
    return CTO_OK;
}

/*
 * One propagation: Alg. 1 (enforceGAC) calling Alg. 2 and Alg. 3.
 * dom_in: the solver's current domains (must be a subset of the domains this
 * propagator returned last).  dom_out may alias dom_in.
 */
/* Alg. 2's branch: incremental iff |Delta_i| < |dom(x_i)| (or forced); an
 * emptied domain always takes the reset branch (OR over no value: no tuple
 * survives -- with star cells the incremental branch would keep the tuples
 * holding a star in that column). */
static int branch_incremental(int32_t mode, int delta, int size) {
    if (size == 0) return 0;
    return mode == CTO_MODE_INCREMENTAL || (mode == CTO_MODE_AUTO && delta < size);
}

static int propagate_fast(cto_table *T, const uint64_t *dom_in, uint64_t *dom_out, uint64_t *ct_out,
                          int32_t mode);

int cto_propagate(cto_table *T, const uint64_t *dom_in, uint64_t *dom_out, uint64_t *ct_out,
                  int32_t mode) {
    if (!T || !dom_in) return CTO_E_INVALID;
    if (T->fast) return propagate_fast(T, dom_in, dom_out, ct_out, mode);
    if (T->failed) return CTO_E_STATE;
    if (stray_bits(T, dom_in)) return CTO_E_INVALID;
    for (int k = 0; k < T->D; k++)
        if (dom_in[k] & ~T->last_dom[k]) return CTO_E_NOT_SUBSET;
    int n = T->n;
    int64_t W = T->W, Wa = W > 0 ? W : 1;
    uint64_t *dom = (uint64_t *)malloc(sizeof(uint64_t) * T->D);
    uint64_t *mask = (uint64_t *)malloc(sizeof(uint64_t) * Wa);
    int32_t *size = (int32_t *)malloc(sizeof(int32_t) * n);
    char *s_val = (char *)calloc((size_t)n, 1), *s_sup = (char *)calloc((size_t)n, 1);
    if (!dom || !mask || !size || !s_val || !s_sup) {
        free(dom); free(mask); free(size); free(s_val); free(s_sup);
        return CTO_E_NOMEM;
    }
    memcpy(dom, dom_in, sizeof(uint64_t) * T->D);
    memset(T->st, 0, sizeof(T->st));
    for (int64_t w = 0; w < W; w++) T->st[CTO_ST_NZ_WORDS] += T->ct[w] != 0;
    T->st[CTO_ST_NZ_GRANULES] = nonzero_granules(T->ct, W);

    /* Alg. 1: Delta, s_val, s_sup */
    for (int i = 0; i < n; i++) {
        size[i] = var_size(T, dom, i);
        if (size[i] != T->last_sizes[i]) {
            s_val[i] = 1;
            T->last_sizes[i] = size[i];
            T->st[CTO_ST_SVAL]++;
        }
        if (size[i] > 1) {
            s_sup[i] = 1;
            T->st[CTO_ST_SSUP]++;
        }
    }
    /* rows the branch rule selects over all of s_val (work count only) */
    for (int i = 0; i < n; i++) {
        if (!s_val[i]) continue;
        int delta = 0;
        for (int k = 0; k < T->dom_words[i]; k++)
            delta += popc(T->last_dom[T->dom_off[i] + k] & ~dom[T->dom_off[i] + k]);
        int incremental = branch_incremental(mode, delta, size[i]);
        T->st[CTO_ST_ROWS_SEL] += incremental ? delta : size[i];
    }
    /* Alg. 2: updateTable */
    for (int i = 0; i < n; i++) {
        if (!s_val[i]) continue;
        int delta = 0;
        for (int k = 0; k < T->dom_words[i]; k++)
            delta += popc(T->last_dom[T->dom_off[i] + k] & ~dom[T->dom_off[i] + k]);
        int incremental = branch_incremental(mode, delta, size[i]);
        memset(mask, 0, sizeof(uint64_t) * Wa);
        for (int a = 0; a < T->dsz[i]; a++) {
            int was = has_value(T, T->last_dom, i, a), is = has_value(T, dom, i, a);
            int take = incremental ? (was && !is) : is;
            if (!take) continue;
            const uint64_t *r = incremental ? strict_row_ptr(T, i, a) : row_ptr(T, i, a);
            for (int64_t w = 0; w < W; w++) mask[w] |= r[w];
            T->st[CTO_ST_ROWS_OR]++;
            T->st[CTO_ST_UPD_WORDS] += W;
        }
        if (incremental)
            for (int64_t w = 0; w < W; w++) mask[w] = ~mask[w];
        for (int64_t w = 0; w < W; w++) T->ct[w] &= mask[w];
        /* Alg. 2's break (a negative table has no early failure: an empty
         * currTable means no combination is forbidden) */
        if (T->kind == CTO_KIND_POSITIVE && !any_word(T->ct, W)) break;
    }
    if (T->kind == CTO_KIND_NEGATIVE) {
        int st = filter_negative(T, dom);
        if (st == CTO_FAIL) {
            T->failed = 1;
            if (ct_out) memset(ct_out, 0, sizeof(uint64_t) * W);
        } else if (st == CTO_OK) {
            memcpy(T->last_dom, dom, sizeof(uint64_t) * T->D);
            if (dom_out) memcpy(dom_out, dom, sizeof(uint64_t) * T->D);
            if (ct_out) memcpy(ct_out, T->ct, sizeof(uint64_t) * W);
        }
        free(dom); free(mask); free(size); free(s_val); free(s_sup);
        return st;
    }
    /* Alg. 1: failure test */
    if (!any_word(T->ct, W)) {
        T->failed = 1;
        if (ct_out) memset(ct_out, 0, sizeof(uint64_t) * W);
        free(dom); free(mask); free(size); free(s_val); free(s_sup);
        return CTO_FAIL;
    }
    /* Alg. 1 goes on to filterDomains (Alg. 3) */
    filter_domains(T, dom, s_sup);
    memcpy(T->last_dom, dom, sizeof(uint64_t) * T->D);
    if (dom_out) memcpy(dom_out, dom, sizeof(uint64_t) * T->D);
    if (ct_out) memcpy(ct_out, T->ct, sizeof(uint64_t) * W);
    free(dom); free(mask); free(size); free(s_val); free(s_sup);
    return CTO_OK;
}

/* Work counters of the last propagate call: the first min(n, CTO_NSTATS)
 * entries of the CTO_ST_* list.  Returns CTO_NSTATS. */
int cto_last_stats(const cto_table *T, int64_t *out, int32_t n) {
    for (int k = 0; k < n && k < CTO_NSTATS; k++) out[k] = T->st[k];
    return CTO_NSTATS;
}

static int push_fast(cto_table *T);
static int pop_fast(cto_table *T);

/* push: snapshot of currTable, last domains, lastSizes and the failed flag */
int cto_push(cto_table *T) {
    if (!T) return CTO_E_INVALID;
    if (T->fast) return push_fast(T);
    if (T->failed) return CTO_E_STATE;
    if (T->depth == T->cap) {
        int nc = T->cap ? 2 * T->cap : 16;
        int64_t Wa = T->W > 0 ? T->W : 1;
        uint64_t *a = (uint64_t *)realloc(T->snap_ct, sizeof(uint64_t) * (size_t)Wa * nc);
        if (!a) return CTO_E_NOMEM;
        T->snap_ct = a;
        uint64_t *b = (uint64_t *)realloc(T->snap_dom, sizeof(uint64_t) * (size_t)T->D * nc);
        if (!b) return CTO_E_NOMEM;
        T->snap_dom = b;
        int32_t *c = (int32_t *)realloc(T->snap_sizes, sizeof(int32_t) * (size_t)T->n * nc);
        if (!c) return CTO_E_NOMEM;
        T->snap_sizes = c;
        int32_t *d = (int32_t *)realloc(T->snap_failed, sizeof(int32_t) * nc);
        if (!d) return CTO_E_NOMEM;
        T->snap_failed = d;
        T->cap = nc;
    }
    int64_t Wa = T->W > 0 ? T->W : 1;
    memcpy(T->snap_ct + (int64_t)T->depth * Wa, T->ct, sizeof(uint64_t) * Wa);
    memcpy(T->snap_dom + (int64_t)T->depth * T->D, T->last_dom, sizeof(uint64_t) * T->D);
    memcpy(T->snap_sizes + (int64_t)T->depth * T->n, T->last_sizes, sizeof(int32_t) * T->n);
    T->snap_failed[T->depth] = T->failed;
    T->depth++;
    return CTO_OK;
}

int cto_pop(cto_table *T) {
    if (!T) return CTO_E_INVALID;
    if (T->fast) return pop_fast(T);
    if (T->depth == 0) return CTO_E_STATE;
    T->depth--;
    int64_t Wa = T->W > 0 ? T->W : 1;
    memcpy(T->ct, T->snap_ct + (int64_t)T->depth * Wa, sizeof(uint64_t) * Wa);
    memcpy(T->last_dom, T->snap_dom + (int64_t)T->depth * T->D, sizeof(uint64_t) * T->D);
    memcpy(T->last_sizes, T->snap_sizes + (int64_t)T->depth * T->n, sizeof(int32_t) * T->n);
    T->failed = T->snap_failed[T->depth];
    return CTO_OK;
}

/* ========================================================================
 * Fast mode: the same results by CT's own economies (Sec. 2: the sparse
 * bitset of non-zero currTable words, residues checked first by
 * filterDomains; reversible state by a trail of currTable words).  It exists
 * to time a competent serial CT beside the GPU and to count the work CT
 * does; every call agrees with the plain mode (tested call by call).
 * ===================================================================== */

/* Builds the fast-mode structures from the state left by cto_create. */
static int fast_init(cto_table *T) {
    int64_t Wa = T->W > 0 ? T->W : 1;
    T->idx = (int32_t *)malloc(sizeof(int32_t) * Wa);
    T->res = (int32_t *)calloc((size_t)(T->rows > 0 ? T->rows : 1), sizeof(int32_t));
    T->fmask = (uint64_t *)malloc(sizeof(uint64_t) * Wa);
    T->stamp = (int32_t *)calloc((size_t)Wa, sizeof(int32_t));
    if (!T->idx || !T->res || !T->fmask || !T->stamp) return CTO_E_NOMEM;
    int64_t k = 0;
    for (int64_t w = 0; w < T->W; w++)
        if (T->ct[w]) T->idx[k++] = (int32_t)w;
    T->limit = T->failed ? 0 : k;
    for (int64_t w = 0; w < T->W; w++)
        if (!T->ct[w]) T->idx[k++] = (int32_t)w;
    T->serial = 0;
    T->next_serial = 0;
    T->fast = 1;
    return CTO_OK;
}

/* cto_create with the fast-mode state: same arguments and statuses. */
int cto_create_fast(const int32_t *tuples, int64_t t, int32_t n, const int32_t *lo,
                    const int32_t *dsz, const uint64_t *init_dom, cto_table **out) {
    int st = cto_create(tuples, t, n, lo, dsz, init_dom, out);
    if (!*out) return st;
    if (fast_init(*out) != CTO_OK) {
        cto_destroy(*out);
        *out = NULL;
        return CTO_E_NOMEM;
    }
    return st;
}

/* saves word w on the trail before its first change in the current level */
static int trail_word(cto_table *T, int32_t w) {
    if (T->depth == 0 || T->stamp[w] == T->serial) return CTO_OK;
    if (T->tr_top == T->tr_cap) {
        int64_t nc = T->tr_cap ? 2 * T->tr_cap : 1024;
        int32_t *a = (int32_t *)realloc(T->tr_w, sizeof(int32_t) * nc);
        if (!a) return CTO_E_NOMEM;
        T->tr_w = a;
        uint64_t *b = (uint64_t *)realloc(T->tr_v, sizeof(uint64_t) * nc);
        if (!b) return CTO_E_NOMEM;
        T->tr_v = b;
        T->tr_cap = nc;
    }
    T->tr_w[T->tr_top] = w;
    T->tr_v[T->tr_top] = T->ct[w];
    T->tr_top++;
    T->stamp[w] = T->serial;
    return CTO_OK;
}

static int propagate_fast(cto_table *T, const uint64_t *dom_in, uint64_t *dom_out, uint64_t *ct_out,
                          int32_t mode) {
    if (T->failed) return CTO_E_STATE;
    if (stray_bits(T, dom_in)) return CTO_E_INVALID;
    for (int k = 0; k < T->D; k++)
        if (dom_in[k] & ~T->last_dom[k]) return CTO_E_NOT_SUBSET;
    const int n = T->n;
    const int64_t W = T->W;
    uint64_t *dom = (uint64_t *)malloc(sizeof(uint64_t) * T->D);
    int32_t *size = (int32_t *)malloc(sizeof(int32_t) * n);
    char *s_val = (char *)calloc((size_t)n, 1), *s_sup = (char *)calloc((size_t)n, 1);
    if (!dom || !size || !s_val || !s_sup) {
        free(dom); free(size); free(s_val); free(s_sup);
        return CTO_E_NOMEM;
    }
    memcpy(dom, dom_in, sizeof(uint64_t) * T->D);
    memset(T->st, 0, sizeof(T->st));
    T->st[CTO_ST_NZ_WORDS] = T->limit;
    {   /* granules: distinct w / 64 among the listed words */
        int64_t last = -1, g = 0;
        char *seen = (char *)calloc((size_t)(W / 64 + 1), 1);
        if (!seen) {
            free(dom); free(size); free(s_val); free(s_sup);
            return CTO_E_NOMEM;
        }
        for (int64_t k = 0; k < T->limit; k++) {
            int64_t gr = T->idx[k] / 64;
            if (!seen[gr]) { seen[gr] = 1; g++; }
            last = gr;
        }
        (void)last;
        free(seen);
        T->st[CTO_ST_NZ_GRANULES] = g;
    }
    /* Alg. 1: s_val, s_sup */
    for (int i = 0; i < n; i++) {
        size[i] = var_size(T, dom, i);
        if (size[i] != T->last_sizes[i]) {
            s_val[i] = 1;
            T->last_sizes[i] = size[i];
            T->st[CTO_ST_SVAL]++;
        }
        if (size[i] > 1) {
            s_sup[i] = 1;
            T->st[CTO_ST_SSUP]++;
        }
    }
    /* Alg. 2 over the listed (non-zero) words only */
    int rc = CTO_OK;
    for (int i = 0; i < n; i++) {
        if (!s_val[i]) continue;
        int delta = 0;
        for (int k = 0; k < T->dom_words[i]; k++)
            delta += popc(T->last_dom[T->dom_off[i] + k] & ~dom[T->dom_off[i] + k]);
        int incremental = branch_incremental(mode, delta, size[i]);
        T->st[CTO_ST_ROWS_SEL] += incremental ? delta : size[i];
        if (T->limit == 0) continue;  /* past Alg. 2's break: selected, not read */
        for (int64_t k = 0; k < T->limit; k++) T->fmask[T->idx[k]] = 0;
        for (int a = 0; a < T->dsz[i]; a++) {
            int was = has_value(T, T->last_dom, i, a), is = has_value(T, dom, i, a);
            if (!(incremental ? (was && !is) : is)) continue;
            const uint64_t *r = incremental ? strict_row_ptr(T, i, a) : row_ptr(T, i, a);
            for (int64_t k = 0; k < T->limit; k++) T->fmask[T->idx[k]] |= r[T->idx[k]];
            T->st[CTO_ST_ROWS_OR]++;
            T->st[CTO_ST_UPD_WORDS] += T->limit;
        }
        /* intersect; a word that becomes zero leaves the list (swapped with
         * the last listed word: the listed set of an earlier limit is kept) */
        for (int64_t k = T->limit - 1; k >= 0; k--) {
            const int32_t w = T->idx[k];
            const uint64_t nw = T->ct[w] & (incremental ? ~T->fmask[w] : T->fmask[w]);
            if (nw == T->ct[w]) continue;
            if ((rc = trail_word(T, w)) != CTO_OK) break;
            T->ct[w] = nw;
            if (nw == 0) {
                T->idx[k] = T->idx[T->limit - 1];
                T->idx[T->limit - 1] = w;
                T->limit--;
            }
        }
        if (rc != CTO_OK) break;
    }
    if (rc == CTO_OK && T->limit == 0) {  /* Alg. 1: failure test */
        T->failed = 1;
        if (ct_out) memset(ct_out, 0, sizeof(uint64_t) * W);
        rc = CTO_FAIL;
    } else if (rc == CTO_OK) {
        /* Alg. 3 with residues: the residue word first, then the listed words */
        for (int i = 0; i < n; i++) {
            if (!s_sup[i]) continue;
            for (int a = 0; a < T->dsz[i]; a++) {
                if (!has_value(T, dom, i, a)) continue;
                const int row = T->row_start[i] + a;
                const uint64_t *r = row_ptr(T, i, a);
                T->st[CTO_ST_RES_CHECKS]++;
                if (T->ct[T->res[row]] & r[T->res[row]]) continue;
                T->st[CTO_ST_RES_MISSES]++;
                int found = 0;
                for (int64_t k = 0; k < T->limit; k++) {
                    const int32_t w = T->idx[k];
                    T->st[CTO_ST_SCAN_WORDS]++;
                    if (T->ct[w] & r[w]) {
                        T->res[row] = w;
                        found = 1;
                        break;
                    }
                }
                if (!found) dom[T->dom_off[i] + a / 64] &= ~(1ull << (a % 64));
            }
            T->last_sizes[i] = var_size(T, dom, i);
        }
        memcpy(T->last_dom, dom, sizeof(uint64_t) * T->D);
        if (dom_out) memcpy(dom_out, dom, sizeof(uint64_t) * T->D);
        if (ct_out) memcpy(ct_out, T->ct, sizeof(uint64_t) * W);
    }
    free(dom); free(size); free(s_val); free(s_sup);
    return rc;
}

static int push_fast(cto_table *T) {
    if (T->failed) return CTO_E_STATE;
    if (T->depth == T->cap) {
        int nc = T->cap ? 2 * T->cap : 16;
        uint64_t *b = (uint64_t *)realloc(T->snap_dom, sizeof(uint64_t) * (size_t)T->D * nc);
        if (!b) return CTO_E_NOMEM;
        T->snap_dom = b;
        int32_t *c = (int32_t *)realloc(T->snap_sizes, sizeof(int32_t) * (size_t)T->n * nc);
        if (!c) return CTO_E_NOMEM;
        T->snap_sizes = c;
        int32_t *d = (int32_t *)realloc(T->snap_failed, sizeof(int32_t) * nc);
        if (!d) return CTO_E_NOMEM;
        T->snap_failed = d;
        int64_t *e = (int64_t *)realloc(T->lv_top, sizeof(int64_t) * nc);
        if (!e) return CTO_E_NOMEM;
        T->lv_top = e;
        int64_t *f = (int64_t *)realloc(T->lv_limit, sizeof(int64_t) * nc);
        if (!f) return CTO_E_NOMEM;
        T->lv_limit = f;
        int32_t *g = (int32_t *)realloc(T->lv_serial, sizeof(int32_t) * nc);
        if (!g) return CTO_E_NOMEM;
        T->lv_serial = g;
        T->cap = nc;
    }
    memcpy(T->snap_dom + (int64_t)T->depth * T->D, T->last_dom, sizeof(uint64_t) * T->D);
    memcpy(T->snap_sizes + (int64_t)T->depth * T->n, T->last_sizes, sizeof(int32_t) * T->n);
    T->snap_failed[T->depth] = T->failed;
    T->lv_top[T->depth] = T->tr_top;
    T->lv_limit[T->depth] = T->limit;
    T->lv_serial[T->depth] = T->serial;
    T->depth++;
    T->serial = ++T->next_serial;
    return CTO_OK;
}

static int pop_fast(cto_table *T) {
    if (T->depth == 0) return CTO_E_STATE;
    T->depth--;
    for (int64_t e = T->tr_top - 1; e >= T->lv_top[T->depth]; e--) T->ct[T->tr_w[e]] = T->tr_v[e];
    T->tr_top = T->lv_top[T->depth];
    T->limit = T->lv_limit[T->depth];
    T->serial = T->lv_serial[T->depth];
    memcpy(T->last_dom, T->snap_dom + (int64_t)T->depth * T->D, sizeof(uint64_t) * T->D);
    memcpy(T->last_sizes, T->snap_sizes + (int64_t)T->depth * T->n, sizeof(int32_t) * T->n);
    T->failed = T->snap_failed[T->depth];
    return CTO_OK;
}

/*
 * Propagation to a fixpoint over several tables sharing pool variables
 * (Sec. 2: propagation repeats until GAC holds for every constraint or a
 * domain wipe-out is found).  FIFO queue of tables (AC-3 style); a table is
 * re-queued when another table shrinks a variable of its scope.  The pool
 * layout is per-variable 64-bit segments at pool_off[v]; table c's column k
 * is pool variable scopes[scope_off[c] + k] and must have the same initial
 * domain size and lo.  A table's input is the pool restricted to its scope
 * and intersected with the domains it returned last: values it removed
 * before were unsupported under larger domains and stay unsupported, so the
 * closure is unchanged, and the input is always a subset of its state.
 * `order` (nullable) gives the initial queue: its first n_init entries
 * (n_init < 0: all n_tables; without `order`, tables 0..n_init-1).  Starting
 * from a state that was already a fixpoint, a queue holding only the tables
 * whose scope contains a variable that pool_in changed reaches the same
 * closure (the others are still GAC).
 * Returns CTO_OK with pool_out = the GAC closure, or CTO_FAIL.
 */
int cto_fixpoint(int32_t n_tables, cto_table **tabs, const int32_t *scope_off,
                 const int32_t *scopes, int32_t n_pool, const int32_t *pool_off,
                 const uint64_t *pool_in, int32_t pool_words, uint64_t *pool_out,
                 const int32_t *order, int32_t n_init, int64_t *n_props) {
    memcpy(pool_out, pool_in, sizeof(uint64_t) * pool_words);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (n_tables + 1));
    char *inq = (char *)calloc((size_t)n_tables + 1, 1);
    /* var -> tables index */
    int32_t *vcount = (int32_t *)calloc((size_t)n_pool + 1, sizeof(int32_t));
    int64_t total = scope_off[n_tables];
    int32_t *vstart = (int32_t *)calloc((size_t)n_pool + 1, sizeof(int32_t));
    int32_t *vtabs = (int32_t *)malloc(sizeof(int32_t) * (total + 1));
    uint64_t *buf_in = NULL, *buf_out = NULL;
    int maxD = 1;
    for (int c = 0; c < n_tables; c++) if (tabs[c]->D > maxD) maxD = tabs[c]->D;
    buf_in = (uint64_t *)malloc(sizeof(uint64_t) * maxD);
    buf_out = (uint64_t *)malloc(sizeof(uint64_t) * maxD);
    if (!queue || !inq || !vcount || !vstart || !vtabs || !buf_in || !buf_out) {
        free(queue); free(inq); free(vcount); free(vstart); free(vtabs); free(buf_in); free(buf_out);
        return CTO_E_NOMEM;
    }
    for (int64_t k = 0; k < total; k++) vcount[scopes[k]]++;
    for (int v = 0; v < n_pool; v++) vstart[v + 1] = vstart[v] + vcount[v];
    memset(vcount, 0, sizeof(int32_t) * (n_pool + 1));
    for (int c = 0; c < n_tables; c++)
        for (int k = scope_off[c]; k < scope_off[c + 1]; k++) {
            int v = scopes[k];
            vtabs[vstart[v] + vcount[v]++] = c;
        }
    int head = 0, tail = 0, size = 0, cap = n_tables + 1;
    if (n_init < 0 || n_init > n_tables) n_init = n_tables;
    for (int c = 0; c < n_init; c++) {
        int cc = order ? order[c] : c;
        if (inq[cc]) continue;
        queue[tail] = cc; tail = (tail + 1) % cap; size++;
        inq[cc] = 1;
    }
    int rc = CTO_OK;
    int64_t props = 0;
    while (size > 0) {
        int c = queue[head]; head = (head + 1) % cap; size--;
        inq[c] = 0;
        cto_table *T = tabs[c];
        for (int k = 0; k < T->n; k++) {
            int v = scopes[scope_off[c] + k];
            for (int q = 0; q < T->dom_words[k]; q++)
                buf_in[T->dom_off[k] + q] = pool_out[pool_off[v] + q] & T->last_dom[T->dom_off[k] + q];
        }
        int st = cto_propagate(T, buf_in, buf_out, NULL, CTO_MODE_AUTO);
        props++;
        if (st == CTO_FAIL) { rc = CTO_FAIL; break; }
        if (st != CTO_OK) { rc = st; break; }
        for (int k = 0; k < T->n; k++) {
            int v = scopes[scope_off[c] + k];
            int changed = 0;
            for (int q = 0; q < T->dom_words[k]; q++)
                if (pool_out[pool_off[v] + q] != buf_out[T->dom_off[k] + q]) changed = 1;
            if (!changed) continue;
            memcpy(pool_out + pool_off[v], buf_out + T->dom_off[k], sizeof(uint64_t) * T->dom_words[k]);
            for (int e = vstart[v]; e < vstart[v + 1]; e++) {
                int c2 = vtabs[e];
                if (c2 == c || inq[c2]) continue;
                queue[tail] = c2; tail = (tail + 1) % cap; size++;
                inq[c2] = 1;
            }
        }
    }
    if (n_props) *n_props = props;
    free(queue); free(inq); free(vcount); free(vstart); free(vtabs); free(buf_in); free(buf_out);
    return rc;
}
