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
 * Everything is dense and direct: one uint64 word holds 64 tuples (tuple j is
 * bit j%64 of word j/64), every support row has W = ceil(t/64) words, no
 * sparse word list, no residues.  Backtracking keeps a full snapshot of the
 * propagator state per level.  Readings of points the paper leaves open:
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
 * parity unpinned: none of the functions (each result is pinned by the tests
 * against brute-force GAC, the paper's Table 1 and closed-form invariants).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CTO_OK 0
#define CTO_FAIL 1
#define CTO_E_INVALID (-1)
#define CTO_E_NOT_SUBSET (-2)
#define CTO_E_STATE (-3)
#define CTO_E_NOMEM (-4)

#define CTO_MODE_AUTO 0        /* Alg. 2's branch rule */
#define CTO_MODE_RESET 1       /* always OR over dom(x_i)  */
#define CTO_MODE_INCREMENTAL 2 /* always OR over Delta_i, complement */

typedef struct {
    int n;
    int64_t t, W;
    int rows, D;
    int32_t *lo, *dsz, *row_start, *dom_off, *dom_words;
    uint64_t *S;        /* rows x W: supports[x_i, v] (Sec. 2) */
    uint64_t *ct;       /* W: currTable */
    uint64_t *last_dom; /* D: domains after the previous call */
    int32_t *last_sizes;/* n: lastSizes of Alg. 1 */
    int failed;
    /* snapshot stack for push/pop */
    int depth, cap;
    uint64_t *snap_ct, *snap_dom;
    int32_t *snap_sizes, *snap_failed;
    /* counters of the last propagate call (work done, not results) */
    int64_t st_nonzero_words_in; /* non-zero currTable words at entry */
    int64_t st_update_rows;      /* support rows OR-ed by updateTable */
    int64_t st_sval, st_ssup;
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

static int any_word(const uint64_t *x, int64_t W) {
    for (int64_t w = 0; w < W; w++)
        if (x[w]) return 1;
    return 0;
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
    free(T->S); free(T->ct); free(T->last_dom); free(T->last_sizes);
    free(T->snap_ct); free(T->snap_dom); free(T->snap_sizes); free(T->snap_failed);
    free(T);
}

/*
 * Build supports (Sec. 2: cell ([x_i, v], j) is 1 iff tau_j[i] = v) and run
 * the root propagation (Sec. 3, constructor).  Returns CTO_OK, CTO_FAIL (the
 * handle exists, in the failed state), or an error with *out = NULL.
 */
int cto_create(const int32_t *tuples, int64_t t, int32_t n, const int32_t *lo,
               const int32_t *dsz, const uint64_t *init_dom, cto_table **out) {
    *out = NULL;
    if (n < 1 || t < 0 || !lo || !dsz || (t > 0 && !tuples)) return CTO_E_INVALID;
    for (int i = 0; i < n; i++)
        if (dsz[i] < 1) return CTO_E_INVALID;
    cto_table *T = (cto_table *)calloc(1, sizeof(cto_table));
    if (!T) return CTO_E_NOMEM;
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
    if (!T->S || !T->ct || !T->last_dom) {
        cto_destroy(T);
        return CTO_E_NOMEM;
    }
    for (int64_t j = 0; j < t; j++) {
        for (int i = 0; i < n; i++) {
            int64_t v = (int64_t)tuples[j * n + i] - lo[i];
            if (v < 0 || v >= dsz[i]) continue; /* value outside dom0: no row */
            row_ptr(T, i, (int)v)[j / 64] |= 1ull << (j % 64);
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
int cto_propagate(cto_table *T, const uint64_t *dom_in, uint64_t *dom_out, uint64_t *ct_out,
                  int32_t mode) {
    if (!T || !dom_in) return CTO_E_INVALID;
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
    T->st_nonzero_words_in = 0;
    for (int64_t w = 0; w < W; w++) T->st_nonzero_words_in += T->ct[w] != 0;
    T->st_update_rows = 0;
    T->st_sval = 0;
    T->st_ssup = 0;

    /* Alg. 1: Delta, s_val, s_sup */
    for (int i = 0; i < n; i++) {
        size[i] = var_size(T, dom, i);
        if (size[i] != T->last_sizes[i]) {
            s_val[i] = 1;
            T->last_sizes[i] = size[i];
            T->st_sval++;
        }
        if (size[i] > 1) {
            s_sup[i] = 1;
            T->st_ssup++;
        }
    }
    /* Alg. 2: updateTable */
    for (int i = 0; i < n; i++) {
        if (!s_val[i]) continue;
        int delta = 0;
        for (int k = 0; k < T->dom_words[i]; k++)
            delta += popc(T->last_dom[T->dom_off[i] + k] & ~dom[T->dom_off[i] + k]);
        int incremental = mode == CTO_MODE_INCREMENTAL || (mode == CTO_MODE_AUTO && delta < size[i]);
        memset(mask, 0, sizeof(uint64_t) * Wa);
        for (int a = 0; a < T->dsz[i]; a++) {
            int was = has_value(T, T->last_dom, i, a), is = has_value(T, dom, i, a);
            int take = incremental ? (was && !is) : is;
            if (!take) continue;
            const uint64_t *r = row_ptr(T, i, a);
            for (int64_t w = 0; w < W; w++) mask[w] |= r[w];
            T->st_update_rows++;
        }
        if (incremental)
            for (int64_t w = 0; w < W; w++) mask[w] = ~mask[w];
        for (int64_t w = 0; w < W; w++) T->ct[w] &= mask[w];
        if (!any_word(T->ct, W)) break;
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

void cto_last_stats(const cto_table *T, int64_t *out4) {
    out4[0] = T->st_nonzero_words_in;
    out4[1] = T->st_update_rows;
    out4[2] = T->st_sval;
    out4[3] = T->st_ssup;
}

/* push: snapshot of currTable, last domains, lastSizes and the failed flag */
int cto_push(cto_table *T) {
    if (!T) return CTO_E_INVALID;
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
    if (T->depth == 0) return CTO_E_STATE;
    T->depth--;
    int64_t Wa = T->W > 0 ? T->W : 1;
    memcpy(T->ct, T->snap_ct + (int64_t)T->depth * Wa, sizeof(uint64_t) * Wa);
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
 * `order` (nullable) gives the initial queue order.
 * Returns CTO_OK with pool_out = the GAC closure, or CTO_FAIL.
 */
int cto_fixpoint(int32_t n_tables, cto_table **tabs, const int32_t *scope_off,
                 const int32_t *scopes, int32_t n_pool, const int32_t *pool_off,
                 const uint64_t *pool_in, int32_t pool_words, uint64_t *pool_out,
                 const int32_t *order, int64_t *n_props) {
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
    for (int c = 0; c < n_tables; c++) {
        int cc = order ? order[c] : c;
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
