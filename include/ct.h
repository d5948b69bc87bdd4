/*
 * ct.h -- C ABI of the MI355X Compact-Table (CT) propagation library.
 *
 * Method: Compact-Table propagation for the positive table constraint,
 * after E. Santi, F. Tardivo, A. Dovier, A. Formisano, "GPU Accelerated
 * Compact-Table Propagation" (arXiv 2507.18413).  Definitions of supports,
 * currTable and valid tuples: Sec. 2; enforceGAC / updateTable /
 * filterDomains: Alg. 1-3; constructor check and indexing: Sec. 3.
 *
 * Conventions shared by every call
 * --------------------------------
 * Tables.  A table has `arity` columns x_0..x_{n-1} and `n_tuples` rows; the
 * tuples are int32, row-major (`tuples[j * arity + i]` = tau_j[i]).  Column i
 * has the initial domain [dom_lo[i], dom_lo[i] + dom_size[i]).  Duplicate
 * tuples are kept (each has its own currTable bit); a tuple holding a value
 * outside an initial domain is never valid.
 *
 * Domain bitmaps.  Variable i owns ceil(dom_size[i] / 64) consecutive uint64
 * words starting at word dom_off[i] = sum of the word counts of variables
 * 0..i-1; value v is bit (v - dom_lo[i]) % 64 of word
 * dom_off[i] + (v - dom_lo[i]) / 64, least significant bit first, 1 = present.
 * Bits at or beyond dom_size[i] must be zero ("stray bits").  D is the total
 * word count.
 *
 * currTable.  ceil(n_tuples / 64) uint64 words; tuple j is bit j % 64 of word
 * j / 64; bit set = the tuple is valid under the current domains (Sec. 2).
 * Tail bits past n_tuples are zero.
 *
 * Slots.  A table owns one or more independent reversible propagator states
 * ("slots", e.g. one per search or search node).  Slot 0 exists after
 * ct_create; every slot starts as a copy of the root state (the state after
 * the root propagation in ct_create).
 *
 * Status codes: CT_OK, CT_FAIL (domain wipe-out: no valid tuple, Alg. 1's
 * failure test), or a negative error.  No call throws; after an error ct_last_error()
 * returns a message for the calling thread.  A ct_table may be used by one
 * thread at a time; distinct tables are independent.
 */
#ifndef CT_H
#define CT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CT_OK 0
#define CT_FAIL 1
#define CT_E_INVALID (-1)    /* malformed argument or stray domain bits */
#define CT_E_NOT_SUBSET (-2) /* dom_in holds a value the slot's domains lack */
#define CT_E_STATE (-3)      /* slot failed (only pop allowed) / pop at depth 0 */
#define CT_E_NOMEM (-4)      /* device or host allocation, trail or depth capacity */
#define CT_E_DEVICE (-5)     /* HIP error or device-side timeout; handle is poisoned */

/* update branch policy (Alg. 2's branch choice): AUTO takes the incremental branch
 * (OR over the removed values, complemented) iff |Delta_i| < |dom(x_i)|,
 * else the reset branch (OR over the remaining values).  Both give the same
 * currTable; the forced modes exist for testing and ablation. */
#define CT_BRANCH_AUTO 0
#define CT_BRANCH_RESET 1
#define CT_BRANCH_INCREMENTAL 2

typedef struct ct_table ct_table;

/* How a propagation is spread over the GPU: SOLO runs a whole call in one
 * workgroup (no hand-off between workgroups; best for small tables and for
 * batches of many jobs), SPLIT spreads updateTable over workgroups of 8
 * granules and filterDomains over workgroups of 4 domain words.  NODES is the
 * search-node schedule of ct_propagate_batch: when every job of a batch is a
 * CT_JOB_FROM_ROOT propagation of the same table of at most 256 support rows
 * (sum of the domain sizes), one workgroup per (one or two granules, up to
 * 64 jobs) stages those granules of every support row in LDS and evaluates
 * updateTable for its jobs from there, so the supports are read once per
 * group of jobs; other batches and single calls fall back to AUTO.  AUTO picks SOLO for tables of at most 4
 * granules (16,384 tuples) and at most 16 domain words (wider tables spread
 * filterDomains over workgroups) and for batches of at least 256 jobs, and
 * NODES for eligible batches of at least 64 jobs.  A batch whose jobs are all
 * CT_JOB_ROOT on AUTO tables runs as two launches: one wave per (job,
 * granule) streams every support row of its granule once, then one
 * workgroup per job partitions and filters.  On an AUTO table of more than
 * 64 and at most 256 domain words whose update is one SPLIT item (at most 8
 * granules), with variables of at most 31 domain words, plain synchronous
 * calls on slot 0 (no currTable copy, no counters) go to the resident split
 * schedule: the SPLIT schedule's update workgroup and its filter workgroups
 * as one persistent launch that takes calls from a mailbox in pinned host
 * memory, as the resident engine does (it exits after 2 ms without a call
 * and before any other operation on the table's device state).  Results are
 * identical. */
#define CT_SCHED_AUTO 0
#define CT_SCHED_SOLO 1
#define CT_SCHED_SPLIT 2
#define CT_SCHED_NODES 3
/* RESIDENT: synchronous calls on slot 0 (ct_propagate, ct_propagate_slot
 * with slot 0) go to a resident engine: one persistent workgroup that keeps
 * the slot's currTable, granule index, stamps, residues and domains in LDS
 * and takes calls from a mailbox in pinned host memory, so a call costs no
 * launch and few round trips to HBM.  Used when that state fits one
 * workgroup's LDS (currTable of up to roughly a million tuples), the table
 * has at most 65,535 support rows and D <= 512; AUTO does the same for
 * D <= 64 (on wider tables the launched schedules spread filterDomains over
 * many workgroups and are faster).  Results are identical to the launched
 * schedules.  The
 * engine writes the state back and exits after 2 ms without a call (the
 * next call starts it again) and before any other operation on the table's
 * device state; one engine runs per process (see ct_quiesce). */
#define CT_SCHED_RESIDENT 4

typedef struct {
    int32_t branch_policy; /* CT_BRANCH_*; default AUTO */
    int32_t max_depth;     /* push levels per slot; default 256 */
    int32_t schedule;      /* CT_SCHED_*; default AUTO */
} ct_config;

typedef struct {
    int32_t n_vars;
    int32_t D;          /* domain bitmap words */
    int64_t W;          /* currTable words = ceil(n_tuples / 64) */
    int64_t n_tuples;
    int32_t rows;       /* support rows = sum of dom_size */
    int32_t n_slots;
    int32_t granules;   /* 64-word groups of currTable tracked by the sparse index */
    int32_t root_failed;/* 1 if the root propagation found no valid tuple */
    int32_t resident;   /* synchronous calls on slot 0: 1 = the resident engine,
                           2 = the resident split schedule (AUTO), 0 = launched */
    int32_t kind;       /* CT_KIND_POSITIVE, CT_KIND_SHORT (positive with star cells) or
                           CT_KIND_NEGATIVE */
} ct_layout_info;

/* Cumulative per-slot work counters (never reset; take differences). */
typedef struct {
    int64_t jobs;             /* propagate jobs executed */
    int64_t granules_in;      /* sum over jobs of active granules at entry */
    int64_t rows_or;          /* support rows OR-ed by updateTable (sum of k_i) */
    int64_t granule_rows;     /* granule x row loads issued by updateTable */
    int64_t trail_granules;   /* granules saved on the trail */
    int64_t residue_checks;   /* values tested by filterDomains */
    int64_t residue_misses;   /* of those, residue word no longer intersecting */
    int64_t scan_granules;    /* granules scanned after residue misses */
} ct_stats;

/*
 * ct_create -- copy the tuples to the device, build the support bitsets
 * (supports[x_i, v] bit j = 1 iff tau_j[i] = v, Sec. 2) and run the root
 * propagation: every variable takes the reset branch over its initial domain,
 * then every non-singleton variable is filtered (the constructor's check of
 * Sec. 3, read as root GAC).  init_dom (host, nullable) restricts the initial
 * domains; NULL = full intervals.  cfg is nullable.  All inputs are host
 * pointers owned by the caller and not retained.
 * Returns CT_OK, or CT_FAIL with *out valid but its root state failed, or
 * CT_E_INVALID (arity < 1 or > 256, n_tuples < 0, dom_size < 1, more than
 * 2^22 support rows (sum of dom_size) or 65,536 domain words, more than
 * 33,554,432 tuples, stray init_dom bits), CT_E_NOMEM, CT_E_DEVICE with
 * *out = NULL.
 */
int ct_create(const int32_t *tuples, int64_t n_tuples, int32_t arity, const int32_t *dom_lo,
              const int32_t *dom_size, const uint64_t *init_dom, const ct_config *cfg,
              ct_table **out);

/*
 * ct_create_table -- ct_create for a table of a given kind (the table kinds
 * of the paper's footnote on Sec. 2):
 *   CT_KIND_POSITIVE: the tuples are the allowed combinations.  A cell may
 *     hold CT_STAR, standing for every value of its column (a short table;
 *     INT32_MIN is therefore not a value).  A star cell is in the support
 *     row of every value of its column; a short table's updateTable takes
 *     the reset branch of Alg. 2 for every changed variable (OR over the
 *     remaining values: a star tuple stays valid while its column's domain is
 *     not empty), so CT_BRANCH_INCREMENTAL is refused (CT_E_INVALID).
 *   CT_KIND_NEGATIVE: the tuples are the forbidden combinations, distinct
 *     and without stars, with at most 8,192 support rows and 1,024 domain
 *     words (CT_E_INVALID otherwise).  The valid tuples are the
 *     combinations of the domains that the table does not list; currTable
 *     holds the listed tuples whose every value is in the slot's domains.
 *     A value of x_i stays iff fewer than prod_{k != i} |dom(x_k)| listed
 *     tuples with x_i = a are in currTable; every variable is filtered; the
 *     listed tuples of removed values then leave currTable; CT_FAIL iff a
 *     domain is empty (an empty currTable is no failure).  Calls run in one
 *     workgroup each (CT_SCHED_SOLO), never on the resident engine, the
 *     search-node or the root-stream schedules; the split propagators refuse
 *     negative tables.
 * Everything else is ct_create's contract.
 */
#define CT_KIND_POSITIVE 0
#define CT_KIND_NEGATIVE 1
#define CT_KIND_SHORT 2 /* reported by ct_layout only */
#define CT_STAR ((int32_t)0x80000000)
int ct_create_table(const int32_t *tuples, int64_t n_tuples, int32_t arity, const int32_t *dom_lo,
                    const int32_t *dom_size, const uint64_t *init_dom, const ct_config *cfg, int32_t kind,
                    ct_table **out);

/* Frees every device and host resource of the table; NULL is ignored. */
void ct_destroy(ct_table *t);

/* Sizes of the table; dom_off (host, nullable, n_vars entries) receives the
 * first bitmap word of every variable. */
int ct_layout(const ct_table *t, ct_layout_info *info, int32_t *dom_off);

/* Copies n_rows support rows starting at row_begin (row of value v of x_i =
 * sum_{k<i} dom_size[k] + v - dom_lo[i], the supportJmp / variablesOffsets
 * indexing of Sec. 3) to host memory, W words each. */
int ct_get_supports(ct_table *t, int32_t row_begin, int32_t n_rows, uint64_t *out);

/*
 * ct_propagate / ct_propagate_slot -- one call of enforceGAC (Alg. 1): Delta
 * and s_val from the slot's last domains, updateTable (Alg. 2) on the device,
 * fail if currTable = 0, filterDomains (Alg. 3) with residues.  Host pointers,
 * synchronous.  dom_in (D words) must be a subset of the slot's current
 * domains (the dom_out of its previous call, or the root domains); dom_out
 * (D words, may alias dom_in) receives the pruned domains; ct_out (nullable,
 * W words) receives currTable; st (nullable) receives the slot's cumulative
 * counters after the call.
 * CT_OK: dom_out = GAC domains, ct_out = exactly the tuples valid under them.
 * CT_FAIL: no valid tuple; dom_out untouched, ct_out zeros; the slot is
 *   failed until popped.
 * CT_E_NOT_SUBSET / CT_E_INVALID (stray bits) / CT_E_STATE (failed slot):
 *   nothing changes.  CT_E_DEVICE: the handle is poisoned.
 */
int ct_propagate(ct_table *t, const uint64_t *dom_in, uint64_t *dom_out, uint64_t *ct_out,
                 ct_stats *st);
int ct_propagate_slot(ct_table *t, int32_t slot, const uint64_t *dom_in, uint64_t *dom_out,
                      uint64_t *ct_out, ct_stats *st);

/*
 * ct_push / ct_pop -- backtracking.  CT's state is reversible: the solver
 * saves and restores it when the search backtracks (Sec. 3, the propagator's
 * state is managed by the solver; Sec. 5.2.1, backtracking phases that grow
 * domains and valid tuples again).  push records a level; pop restores the
 * slot's currTable, domains and failed flag exactly as they were at the
 * matching push.  push on a failed slot -> CT_E_STATE; push beyond max_depth
 * -> CT_E_NOMEM; pop at depth 0 -> CT_E_STATE.  Both are cheap host calls;
 * the device work is folded into the slot's next device operation.
 */
int ct_push(ct_table *t);
int ct_pop(ct_table *t);
int ct_push_slot(ct_table *t, int32_t slot);
int ct_pop_slot(ct_table *t, int32_t slot);

/* Current domains (D words; the domains the slot's last propagation
 * returned, Alg. 3's output) and currTable (W words; the tuples valid under
 * them, Sec. 2) of a slot, host pointers, both nullable.  A failed slot
 * reports its domains at the failure's input and a zero currTable. */
int ct_get_state(ct_table *t, int32_t slot, uint64_t *dom_out, uint64_t *ct_out);

/* Adds n slots with consecutive ids, each a copy of the root state (the
 * state after the constructor's root propagation, Sec. 3) with room for
 * max_depth push levels (negative = the table's default; 0 = no levels, for
 * slots that are only reset by CT_JOB_FROM_ROOT jobs or never pushed).
 * Synchronous.  *first_slot receives the first id.  The first run of n
 * consecutive slots released by ct_slots_free whose trails hold max_depth
 * levels is reused (reset to the root state); otherwise new slots are
 * allocated on the device (CT_E_NOMEM if that fails). */
int ct_slots_alloc(ct_table *t, int32_t n, int32_t max_depth, int32_t *first_slot);

/* Releases slots first .. first + n - 1 (slot 0, the table's own, cannot be
 * released).  A released slot answers every call that names it (propagate,
 * push, pop, get_state, slot_stats, batch jobs) with CT_E_INVALID until
 * ct_slots_alloc hands it out again.  Its device memory stays with the table
 * (freed by ct_destroy) and is reused by ct_slots_alloc.  The caller releases
 * a slot only after every batch that names it has completed.  CT_E_INVALID
 * for a range outside the table, slot 0, or a slot already released. */
int ct_slots_free(ct_table *t, int32_t first, int32_t n);

/* Cumulative counters of a slot (host pointer). */
int ct_slot_stats(ct_table *t, int32_t slot, ct_stats *st);

/* ------------------------------------------------------------------------
 * Batched propagation (device pointers, asynchronous)
 * --------------------------------------------------------------------- */
#define CT_JOB_PROPAGATE 1u /* run enforceGAC after the pops and pushes */
#define CT_JOB_FROM_ROOT 2u /* reset the slot to the root state (depth 0) first */
/* Recompute the root state from scratch into the slot, as at creation (Alg. 1
 * with every variable on the reset branch of Alg. 2, starting from all
 * tuples; Sec. 3, "Procedures"): dom_in = the table's initial domains, or any
 * domains without stray bits; the slot ends at depth 0 holding GAC of dom_in.
 * Streams every support row once.  Needs CT_JOB_PROPAGATE; no pops/pushes;
 * not with CT_JOB_FROM_ROOT. */
#define CT_JOB_ROOT 4u

typedef struct {
    ct_table *table;
    int32_t slot;
    uint32_t flags;      /* CT_JOB_* */
    int32_t n_pop;       /* levels popped first (<= the slot's depth) */
    int32_t n_push;      /* levels pushed after the pops */
    const uint64_t *dom_in; /* device-accessible (device memory or mapped pinned
                               host memory), D words of the table (PROPAGATE) */
    uint64_t *dom_out;      /* device-accessible, D words (PROPAGATE; may alias dom_in) */
    uint64_t *ct_out;       /* device-accessible, W words, nullable */
} ct_job;

/*
 * ct_propagate_batch -- runs every job in one persistent launch on `stream`
 * (a hipStream_t; NULL = the null stream) driven by a device work queue.
 * Each job's result equals that of the same pops, pushes and ct_propagate on
 * its slot alone.  status_dev (device-accessible, n_jobs int32) receives each job's
 * status (CT_OK, CT_FAIL, CT_E_NOT_SUBSET, CT_E_INVALID, CT_E_STATE,
 * CT_E_NOMEM).  Returns immediately after queueing; CT_E_INVALID for a
 * malformed batch (two jobs on one slot, pop below depth 0, FROM_ROOT with
 * pops or pushes), CT_E_NOMEM (push beyond max_depth).  In a batch a push on
 * a failed slot is allowed (the level records the failed flag).  A FROM_ROOT
 * or ROOT job whose input is rejected (CT_E_INVALID, CT_E_NOT_SUBSET,
 * CT_E_STATE) still resets its slot, which then holds the table's root state
 * at depth 0.  The tables must not be used from another stream until the
 * batch completes.
 */
int ct_propagate_batch(const ct_job *jobs, int32_t n_jobs, void *stream, int32_t *status_dev);

/*
 * ct_propagate_batch_noalloc -- ct_propagate_batch for callers that cannot
 * allocate memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same jobs, statuses and results,
 * but no device, pinned or host allocation.  The work-queue counters, the
 * staged job descriptors and the search-node schedule's records live in a
 * static device array of 16 MiB that each GPU holds until the process ends
 * (set up on the device's first call), and the descriptors are built in
 * static host arrays.  Limits: at most 8,192 jobs, at most 2 MiB of staged
 * descriptors (about 88 bytes per job plus the root tasks of a batch of
 * CT_JOB_ROOT jobs: one per 4 granules), and for a batch on the search-node
 * schedule at most 14 MiB of node records and flags (per job about 8 x
 * (4 + (rows + 3 x arity + 3) / 4) + granules bytes); a batch beyond them is
 * refused with CT_E_INVALID before anything changes.  Every no-allocation
 * call on one GPU shares that array and the host arrays: calls are
 * serialized on the host, and calls whose batches overlap on the GPU (on
 * different streams, or before an earlier one has completed on another
 * stream) race and give undefined results; batches queued on one stream
 * run in order and are safe.  Each call clears the queue counters first
 * (a small kernel on `stream`).  Device-side errors are reported by
 * ct_batch_status on the stream of the last no-allocation call.
 */
int ct_propagate_batch_noalloc(const ct_job *jobs, int32_t n_jobs, void *stream, int32_t *status_dev);

/* ------------------------------------------------------------------------
 * Many tables sharing variables: propagation to a fixpoint
 * --------------------------------------------------------------------- */
/*
 * A model is a pool of variables plus tables whose columns are pool
 * variables (a CSP whose constraints are table constraints, Sec. 2).  Its
 * fixpoint is the largest set of sub-domains of the pool that is GAC for
 * every table (propagation repeated until nothing changes, Sec. 2), or a
 * failure.  Each table takes part through its slot 0; a table may belong to
 * one model.  The pool bitmap uses the per-variable 64-bit segments of the
 * domain bitmaps above, over all pool variables.  A table column must have
 * the same dom_lo and dom_size as its pool variable.
 */
typedef struct ct_model ct_model;

/* n_vars pool variables with initial domains [dom_lo[i], dom_lo[i] + dom_size[i]). */
int ct_model_create(int32_t n_vars, const int32_t *dom_lo, const int32_t *dom_size, ct_model **out);
void ct_model_destroy(ct_model *m);

/* Adds a table; scope (host, arity entries) names the pool variable of each
 * column, all distinct.  *index (nullable) receives the table's index. */
int ct_model_add(ct_model *m, ct_table *t, const int32_t *scope, int32_t *index);

/* Word offset of each pool variable in the pool bitmap (host, n_vars) and the
 * total word count. */
int ct_model_layout(const ct_model *m, int32_t *pool_off, int32_t *pool_words);

/*
 * Runs propagation rounds from pool_in (device, pool words) until no domain
 * changes: every round propagates, in one persistent launch, each table one
 * of whose variables changed in the previous round (in the first round: each
 * table from whose last domains pool_in removes a value) on the pool
 * intersected with its own last domains, and ANDs the results into the
 * pool.  Rounds are captured in a hipGraph, `rounds_per_graph`
 * at a time, and replayed until the device reports convergence or failure.
 * Synchronous on `stream` (NULL = the model's own stream).  pool_out (device)
 * receives the fixpoint (undefined after CT_FAIL).  n_props (nullable)
 * receives the number of table propagations, n_rounds (nullable) the rounds.
 * Returns CT_OK or CT_FAIL.  After CT_FAIL the failed tables must be popped
 * (ct_model_pop) before the next fixpoint.
 */
int ct_model_fixpoint(ct_model *m, const uint64_t *pool_in, uint64_t *pool_out, void *stream,
                      int64_t *n_props, int64_t *n_rounds);

/* Push / pop one level on slot 0 of every table of the model (one launch,
 * queued on the model's stream; the next fixpoint reports a device-side error
 * of it, and any other call on one of the tables first waits for it). */
int ct_model_push(ct_model *m);
int ct_model_pop(ct_model *m);

/* Scheduling knob of the model's rounds: tables of at most solo_max_granules
 * granules run in one workgroup each, larger ones are split over workgroups
 * (see CT_SCHED_*); rounds_per_graph rounds are captured per graph.  A
 * fixpoint's first two launches are one-round graphs (most search steps
 * converge in a round or two), the launches after them take rounds_per_graph
 * rounds.  The
 * default is chosen by ct_model_autotune or is (4, 8). */
int ct_model_set_schedule(ct_model *m, int32_t solo_max_granules, int32_t rounds_per_graph);

/* Autotuner of the rounds' schedule.  Tables are grouped in classes by
 * floor(log4) of their granule count and of their support-row count; each
 * class gets a schedule: solo (one workgroup per table, 4 granules of 64
 * words per wavefront per step) or split (update items spread over
 * workgroups) with a tile of 2, 4 or 8 granules per wavefront per item.
 * Classes are tuned one after the other, those with the most granules in all
 * first, each candidate timed as the median of 3 fixpoints from pool_in
 * (device pointer), every table restored between trials with a push / pop;
 * every candidate must reach the same fixpoint (CT_E_DEVICE otherwise).
 * cache_path (nullable): a JSON file of choices keyed by the device
 * architecture and the class buckets ("gfx950 g2 r3": [solo, tile]); when
 * it holds every class of the model, those choices are applied without
 * timing anything (*from_cache = 1), otherwise the tuned choices are merged
 * into it.  *timed (nullable) receives the number of candidates timed.
 * Classes the tuner never saw follow ct_model_set_schedule's threshold with
 * the default tile (2). */
int ct_model_autotune(ct_model *m, const uint64_t *pool_in, const char *cache_path, int32_t *from_cache,
                      int32_t *timed);
/* Effective schedule of table `table` (index from ct_model_add) in the
 * model's rounds: *solo = 1 for one workgroup per table, *tile = granules
 * per wavefront per update step (solo) or item (split). */
int ct_model_get_choice(const ct_model *m, int32_t table, int32_t *solo, int32_t *tile);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of propagate requests from many searches
 * --------------------------------------------------------------------- */
/*
 * A server owns a thread that takes requests from many concurrent searches
 * (each bound to one table), batches the requests of searches that have no
 * request in flight into one ct_propagate_batch launch per free stream, and
 * returns completions while later requests are already being batched: a
 * request that arrives while others run on the GPU joins the next launch.
 * Requests of one search run in submission order, one at a time.
 * A search holds a slot of its table from its first request to its finishing
 * request; slots are admitted against a device-memory budget (bytes of slot
 * state; one search is always admitted), and a search waits, queued, while
 * the budget is exhausted.  The
 * server keeps each search's domain stack on the host, so a request names
 * only the values to remove.  Results do not depend on what else is in the
 * batch.  The tables must not be used by anything else while the server runs.
 */
typedef struct ct_server ct_server;

typedef struct {
    int64_t mem_budget;  /* bytes of slot state admitted at once; <= 0: unlimited */
    int32_t max_batch;   /* requests per launch; <= 0: 1024 */
    int32_t streams;     /* launches in flight; <= 0: 2 */
} ct_server_cfg;

#define CT_REQ_FINISH 1u /* the search ends after this request; its slot is released */

typedef struct {
    int32_t search;          /* id from ct_server_add_search */
    uint32_t flags;          /* CT_REQ_* */
    int32_t n_pop;           /* levels popped first */
    int32_t push;            /* 1: push a level after the pops */
    const uint64_t *remove;  /* host, D words of the search's table: values removed
                                from the current domains (NULL: none); copied */
    uint64_t *dom_out;       /* host, D words, written before completion (nullable) */
    uint64_t tag;            /* returned in the completion */
} ct_request;

typedef struct {
    uint64_t tag;
    int32_t search;
    int32_t status;          /* as ct_propagate; CT_E_NOMEM if the search's depth
                                would exceed its max_depth */
    double t_submit, t_launch, t_done;  /* seconds, steady clock of the process */
} ct_completion;

int ct_server_create(const ct_server_cfg *cfg, ct_server **out);
/* Stops the thread after the requests in flight and returns every slot its
 * searches still hold to their tables (ct_slots_free; the tables keep the
 * memory and reuse the slots). */
void ct_server_destroy(ct_server *s);
/* Registers a search on table t with room for max_depth levels (all searches
 * of one table use the same max_depth); it starts at the table's root state
 * when its first request is admitted.  Searches are registered before the
 * first ct_server_submit (CT_E_STATE afterwards); a registration that races
 * the first submit from another thread is serialized with it (one of the two
 * comes first under the server's lock).  The first request of a
 * search (and the first after a CT_REQ_FINISH) has n_pop = 0 and push = 0. */
int ct_server_add_search(ct_server *s, ct_table *t, int32_t max_depth, int32_t *search);
/* Thread-safe. */
int ct_server_submit(ct_server *s, const ct_request *req);
/* Up to max completions, waiting up to wait_us microseconds for the first;
 * returns the number written (>= 0) or a negative error. */
int ct_server_poll(ct_server *s, ct_completion *out, int32_t max, int32_t wait_us);
/* Counters, the first min(n, CT_SERVER_NSTATS) written to out (host):
 * [0] requests done, [1] launches, [2] admission waits (times a ready request
 * could not get a slot), [3] slot bytes in use, [4] peak slot bytes, [5]
 * slots allocated (new ones; a slot freed by a finished search is reused),
 * [6] launches that carried two or more requests, [7] launches whose
 * requests named two or more tables, [8] the largest batch launched. */
#define CT_SERVER_NSTATS 9
int ct_server_stats(ct_server *s, int64_t *out, int32_t n);
/* The steady clock the timestamps use (seconds). */
double ct_server_now(void);

/*
 * Split propagators -- the two variants of Sec. 4 that run only one of CT's
 * procedures on the device (Sec. 4.1 and 4.2), for comparison with
 * ct_propagate, which runs all of enforceGAC (Alg. 1) there.  A split
 * propagator starts from the table's root state, keeps its own currTable,
 * domains and levels on the host (the table's slots are untouched) and uses
 * the table's device supports, which must outlive it.
 *   CT_SPLIT_UPDATE: updateTable's mask (Alg. 2) on the device; the host
 *     ANDs it into currTable and runs filterDomains (Alg. 3, residues).
 *   CT_SPLIT_FILTER: updateTable on the host; filterDomains on the device
 *     over the words of the variables with more than one value.
 * Each call is one host-to-device copy and one launch whose results the
 * device writes into pinned host memory; synchronous.  ct_split_propagate has ct_propagate's contract (host
 * pointers; dom_in a subset of the current domains, no stray bits; CT_OK
 * with the GAC domains and currTable, CT_FAIL with dom_out untouched and
 * ct_out zeroed and the propagator failed until popped; CT_E_NOT_SUBSET /
 * CT_E_INVALID / CT_E_STATE change nothing; CT_E_DEVICE poisons it) and the
 * same results; the table's branch policy applies.  push / pop save and
 * restore the whole host state (no depth limit); push on a failed
 * propagator and pop at depth 0 return CT_E_STATE.  ct_split_create returns
 * CT_E_INVALID for an unknown mode, CT_E_NOMEM when the host copy of the
 * supports (rows x W words) or a buffer cannot be allocated.
 */
#define CT_SPLIT_UPDATE 1
#define CT_SPLIT_FILTER 2
typedef struct ct_split ct_split;
int ct_split_create(ct_table *t, int32_t mode, ct_split **out);
int ct_split_propagate(ct_split *s, const uint64_t *dom_in, uint64_t *dom_out, uint64_t *ct_out);
int ct_split_push(ct_split *s);
int ct_split_pop(ct_split *s);
/* Frees the propagator; NULL is ignored. */
void ct_split_destroy(ct_split *s);

/* Synchronizes `stream` and reports whether a batch launched on it hit a
 * device-side error (a bounded wait that expired): CT_OK or CT_E_DEVICE (the
 * error is cleared; the slots of the affected jobs are undefined). */
int ct_batch_status(void *stream);

/* Kernel timing of the synchronous calls (ct_propagate*, flushes of
 * ct_push/ct_pop): when on, every launch measures itself on the GPU's
 * constant-rate wall clock (earliest workgroup start to latest workgroup
 * end) and adds the duration to a device counter; no host events are
 * inserted into the stream.  ct_get_timing synchronizes the table's stream
 * and returns the cumulative kernel milliseconds and launch count since
 * timing was last switched on. */
int ct_set_timing(ct_table *t, int32_t on);
int ct_get_timing(ct_table *t, double *kernel_ms, int64_t *launches);
/* Lifetimes of the kernel launches that served the synchronous calls since
 * timing was switched on, on the same device clock: for launched calls the
 * same figures as ct_get_timing; for the resident engine, each launch's
 * whole lifetime from its start to its exit (the polling between calls
 * included), counting the launches started while timing was on.  Ends a
 * running engine first (so its lifetime is known).  Synchronous. */
int ct_get_dispatch_timing(ct_table *t, double *dispatch_ms, int64_t *dispatches);

/* Thread-local message of the last error ("" if none). */
const char *ct_last_error(void);

/* Test hook for the callers' error paths: the nth device or pinned host
 * allocation the library makes from now on (tables, slots, batch staging,
 * models) fails as if the memory were exhausted, and the call that made it
 * returns CT_E_NOMEM after releasing what it had allocated; nth <= 0 turns
 * the hook off.  Returns the previous setting (allocations still to go). */
int ct_debug_fail_alloc(int32_t nth);

/* Ends the resident engine of any table (CT_SCHED_RESIDENT, or the resident
 * split schedule of an AUTO table) after it has written its state back to
 * the device: call before the process exits, or
 * before work on the GPU that must not wait up to 2 ms behind an idle engine.
 * Synchronous; CT_OK or CT_E_DEVICE. */
int ct_quiesce(void);

#ifdef __cplusplus
}
#endif
#endif /* CT_H */
