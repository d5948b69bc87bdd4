// ct_kernels.hip -- HIP kernels of the CT library for gfx950 (CDNA4).
//
// Work is exact bitwise integer arithmetic on uint64 words; nothing here is
// a dense contraction, so there is no MFMA: the kernels are built around
// coalesced 512-byte granule loads (one word per lane of a wave64), wave
// ballots and LDS.
//
// One persistent kernel executes a batch of propagation jobs as a list of
// work items.  A job runs either in solo mode -- one item, one workgroup,
// the whole of Alg. 1-3 with no hand-off between workgroups (small tables,
// large batches) -- or in split mode, as items in this order:
//   prep   (jobs that pop, and pure push/pop jobs)  backtrack restore, pushes
//   update (nUpd per job)   updateTable (Alg. 2) over 8 granules each, with the
//                           Delta / s_val / s_sup prologue of Alg. 1 recomputed
//                           per item in LDS; the last update item of a job
//                           records the job's pushes, partitions the sparse
//                           index and decides FAIL (Alg. 1's failure test)
//   filter (nFilt per job)  filterDomains (Alg. 3), one domain word per wave,
//                           residue word first, then a scan of active granules
// Workgroup b starts with item b; when the grid is smaller than the item
// count the remaining items are taken from a device queue in increasing
// order.  An item only waits for earlier items of its own job (update waits
// for prep when the job pops; filter waits for the job's last update item).
// Waits are bounded: on expiry the kernel records a device error and the
// remaining work of the launch is skipped.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ct_device.h"

namespace ctk {

constexpr int NGW = 2;                 // granules per wave per update step (split mode)
constexpr int NGS = 4;                 // default granules per wave per step (solo mode)
constexpr int LANE_SCAN = 16;          // words each missing lane checks before the wave scan
constexpr int FULL_SCAN_GRAN = 4;      // at most this many active granules: misses test every active word
constexpr int FULL_SCAN_VALS = 8;      //   for this many values per round trip
constexpr int ROW_UNROLL = 8;          // support rows loaded per batch
constexpr int ROWS_CHUNK = 8192;       // row-list entries staged in LDS at a time
constexpr uint32_t SPIN_LIMIT = 1u << 22;
constexpr int32_t STAR_CELL = (int32_t)0x80000000;  // a short table's cell: every value of its column

// Steps of NGW granules a wave takes per update item for a job's tile
// (granules per wave per item: 2, 4 or 8; 0 = 2).
__host__ __device__ __forceinline__ int tile_reps(int tile) { return tile == 8 ? 4 : tile == 4 ? 2 : 1; }

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / WAVE; }

__device__ __forceinline__ void st_release(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed(int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A word of the slot's previous domains (JF_COHLAST: read at device scope,
// around this XCD's L2)
__device__ __forceinline__ uint64_t ld_last(const CT_G uint64_t* p, bool coh) {
  return coh ? __hip_atomic_load(const_cast<CT_G uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *p;
}

// The slot's array addresses (they never change), loaded together: an item
// that reads them early has them when its first loads from the arrays go.
struct SlotPtrs {
  CT_G uint64_t* ct;
  CT_G int32_t* idx[2];
  CT_G int32_t* stamp;
  CT_G int32_t* nzFlag;
  CT_G uint64_t* trailWords;
  CT_G TrailHdr* trailHdr;
  int64_t trailCap;
};

struct Shared {
  int32_t item, ok, isLast, status, noop, nseg, nrows, limit, serial, depth, bad_stray, bad_sub;
  int64_t trailTop;
  int32_t size[MAX_ARITY];
  int32_t dcnt[MAX_ARITY];
  int32_t segOf[MAX_ARITY];   // var -> segment, -1 if not in s_val
  int32_t segEnd[MAX_ARITY];  // exclusive end of segment rows
  int32_t segInc[MAX_ARITY];
  int32_t wsum[WAVES];
  int32_t trailCount;          // trail entries of a job run by one workgroup
  uint64_t din[MAX_D];         // the job's first MAX_D domain words (the rest are read from memory)
  uint64_t dout[MAX_D];        // negative tables: the filtered domains, published if no domain empties
  uint32_t rows[ROWS_CHUNK];   // entries [k0, k0 + ROWS_CHUNK) of the job's row list
  uint8_t nz[MAX_GRAN];        // granule non-zero flags of a job run by one workgroup
  uint16_t gidx[MAX_GRAN];     // granule list of a job run by one workgroup
  unsigned long long fcnt[3];  // a filter item's counters (residue checks, misses, scans)
  int32_t cur;                 // the slot's index buffer in use at the job's start (prologue)
  SlotPtrs sp;                 // the slot's array addresses (prologue)
  int32_t seOp, seNPop, seNPush, seSerial, seDepth;  // resident split schedule: the call's header
};

__device__ __forceinline__ SlotPtrs slot_ptrs(const SlotDesc* s) {
  SlotPtrs p;
  p.ct = s->ct;
  p.idx[0] = s->idx[0];
  p.idx[1] = s->idx[1];
  p.stamp = s->stamp;
  p.nzFlag = s->nzFlag;
  p.trailWords = s->trailWords;
  p.trailHdr = s->trailHdr;
  p.trailCap = s->trailCap;
  return p;
}

// Record a device error: the host sees it through hostErr (pinned) and the
// other workgroups of the launch stop waiting.
__device__ void raise_error(const KArgs& a, int code) {
  atomicExch(&a.queue[3], code);
  if (a.hostErr) {
    __hip_atomic_store(a.hostErr, code, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Thread 0 spins until *flag == want; the result is broadcast to the block.
// The spin reads the flag relaxed and takes one acquire fence once it holds:
// an acquire load per poll would invalidate the L2 on every iteration (an
// agent-scope acquire does on this chip), under the feet of the workgroup
// being waited for.
__device__ bool block_wait(const KArgs& a, int32_t* flag, int32_t want, Shared& sh) {
  if (threadIdx.x == 0) {
    int ok = 1;
    for (uint32_t it = 0;; ++it) {
      if (ld_relaxed(flag) == want) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        break;
      }
      if (ld_relaxed(&a.queue[3])) { ok = 0; break; }
      if (it > SPIN_LIMIT) { raise_error(a, 1); ok = 0; break; }
      __builtin_amdgcn_s_sleep(1);
    }
    sh.ok = ok;
  }
  __syncthreads();
  const int ok = sh.ok;
  __syncthreads();
  return ok != 0;
}

// Workgroup barrier that orders LDS only: global stores still in flight
// need not complete here (__syncthreads waits for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Inclusive prefix sum over the 64 lanes (every lane active), with DPP
// moves (VALU, no LDS round trips): shifts within rows of 16 lanes, then
// the row broadcasts of lanes 15 and 31.
__device__ __forceinline__ int wave_scan_incl(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Exclusive prefix sum over the block; *total receives the sum.
// (LDS_ONLY: its barriers order LDS only, so global stores still in flight
// need not complete there)
template <bool LDS_ONLY = false>
__device__ int block_scan_excl(int v, int* total, Shared& sh) {
  const int lane = lane_id(), w = wave_id();
  const int x = wave_scan_incl(v);
  if (lane == WAVE - 1) sh.wsum[w] = x;
  if (LDS_ONLY) lds_barrier();
  else __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < WAVES; ++k) {
    const int s = sh.wsum[k];
    if (k < w) off += s;
    tot += s;
  }
  if (LDS_ONLY) lds_barrier();
  else __syncthreads();
  *total = tot;
  return off + x - v;
}

// The job descriptor by value: from the batch array (global memory) or from
// the kernel arguments; a reference chosen between the two would be a flat
// pointer and turn every field access into a flat load.
__device__ __forceinline__ DevJob job_of(const KArgs& a, int j) {
  DevJob J;
  if (a.jobs) J = a.jobs[j];
  else J = a.job;
  return J;
}

__device__ __forceinline__ uint64_t job_din(const KArgs& a, const DevJob& J, int k) {
  return (J.flags & JF_INLINE_DOM) ? a.inl[k] : J.dom_in[k];
}

// Domain word q of the job's input: the prologue's LDS copy for the first
// MAX_D words, memory beyond (inline inputs have at most INLINE_WORDS words,
// all in the copy).
__device__ __forceinline__ uint64_t din_at(const DevJob& J, const Shared& sh, int q) {
  return q < MAX_D ? sh.din[q] : J.dom_in[q];
}

// Word w of the set of all tuples (the starting currTable of a root state
// recomputed from scratch): ones up to the last tuple, zero past it.
__device__ __forceinline__ uint64_t all_tuples_word(const TabDesc* T, int64_t w) {
  if (w >= T->W) return 0ull;
  if (w < T->W - 1 || T->tailBits >= 64) return ~0ull;
  return (1ull << T->tailBits) - 1ull;
}

// Job status for the caller.  Outputs in host memory are published with a
// system-scope release after a system-scope fence, so a host that sees the
// status also sees the domain words written before it.
__device__ __forceinline__ void ll_put(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ void publish_status(const DevJob& J, int st) {
  if (J.flags & JF_LL) {  // a flagged slot: no fence (see JF_LL)
    ll_put(J.ll, eng_slot((uint32_t)st, (uint32_t)J.seq));
    return;
  }
  if (!J.status_out) return;
  if (J.flags & JF_HOST_OUT) {
    __threadfence_system();
    __hip_atomic_store(J.status_out, st, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  } else {
    *J.status_out = st;
  }
}

__device__ __forceinline__ void item_fence(const DevJob& J) {
  if (J.flags & JF_HOST_OUT) __threadfence_system();
  else __threadfence();
}

// Before a job's status is published or its last item is counted: the host
// reads a synchronous call's outputs (pinned memory, JF_HOST_OUT) as soon as
// the status changes, so they must be visible first; a batch's statuses and
// outputs are read after the launch has ended, which makes them visible.  A
// device-scope fence here costs an L2 write-back and invalidate per job (per
// search node: thousands per batch), so batch jobs take none.
__device__ __forceinline__ void status_fence(const DevJob& J) {
  if (J.flags & JF_HOST_OUT) __threadfence_system();
}

// largest j with off[j] <= x  (off has n + 1 entries, off[0] = 0)
__device__ int find_job(const CT_G int32_t* off, int n, int x) {
  int lo = 0, hi = n;  // off[lo] <= x < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// Push nPush levels recording (trailTop, limit, failed, serial, domains);
// the k-th new level continues with serial serialBase + k.  Whole block.
__device__ void push_levels(const DevJob& J, SlotDesc* s, int depth0, int64_t trailTop, int limit,
                            int failed, int serial0, int D) {
  for (int k = 0; k < J.nPush; ++k) {
    const int d = depth0 + k;
    for (int q = threadIdx.x; q < D; q += BLOCK)
      s->levelDom[(int64_t)d * D + q] = ld_last(&s->lastDom[q], J.flags & JF_COHLAST);
    if (threadIdx.x == 0) {
      Level L;
      L.trailTop = trailTop;
      L.limit = limit;
      L.failed = failed;
      L.serial = k == 0 ? serial0 : J.serialBase + k - 1;
      L.pad = 0;
      s->levels[d] = L;
    }
  }
}

// ---------------------------------------------------------------------------
// prep: pops then pushes (whole block), for jobs that pop or only push/pop
// ---------------------------------------------------------------------------
__device__ void apply_pops_pushes(const DevJob& J, Shared& sh) {
  SlotDesc* s = J.slot;
  const int D = J.tab->D;
  for (int p = 0; p < J.nPop; ++p) {
    if (threadIdx.x == 0) {
      sh.depth = s->depth - 1;
      sh.trailTop = s->trailTop;
    }
    __syncthreads();
    const int d = sh.depth;
    const Level L = s->levels[d];
    const int64_t top = sh.trailTop;
    // entries of one level name distinct granules: restore 4 per wave at once
    for (int64_t e0 = L.trailTop + 4 * wave_id(); e0 < top; e0 += 4 * WAVES) {
      TrailHdr h[4];
      uint64_t w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t e = e0 + j;
        if (e < top) {
          h[j] = s->trailHdr[e];
          w[j] = s->trailWords[e * GW + lane_id()];
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (e0 + j < top) {
          s->ct[(int64_t)h[j].gran * GW + lane_id()] = w[j];
          if (lane_id() == 0) s->stamp[h[j].gran] = h[j].oldStamp;
        }
      }
    }
    for (int q = threadIdx.x; q < D; q += BLOCK) s->lastDom[q] = s->levelDom[(int64_t)d * D + q];
    __syncthreads();
    if (threadIdx.x == 0) {
      s->trailTop = L.trailTop;
      s->limit = L.limit;
      s->failed = L.failed;
      s->serial = L.serial;
      s->depth = d;
    }
    __syncthreads();
  }
  if (J.nPush > 0) {
    if (threadIdx.x == 0) {
      sh.depth = s->depth;
      sh.trailTop = s->trailTop;
      sh.limit = s->limit;
      sh.status = s->failed;
      sh.serial = s->serial;
    }
    __syncthreads();
    push_levels(J, s, sh.depth, sh.trailTop, sh.limit, sh.status, sh.serial, D);
    __syncthreads();
    if (threadIdx.x == 0) {
      s->depth = sh.depth + J.nPush;
      s->serial = J.serialBase + J.nPush - 1;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void do_prep(const KArgs& a, const DevJob& J, Shared& sh) {
  apply_pops_pushes(J, sh);
  if (threadIdx.x == 0) {
    // (the barrier at the end of apply_pops_pushes orders the block's
    // writes before thread 0's release)
    if (!(J.flags & JF_PROPAGATE)) publish_status(J, ST_OK);
    else st_release(&J.slot->prepDone, 1);  // consumed (and reset) by the job's last update item
  }
}

__device__ void stage_rows(const DevJob& J, Shared& sh, int k0, const CT_G uint64_t* lastArr = nullptr,
                           const CT_G WordDesc* wordsArr = nullptr);

// ---------------------------------------------------------------------------
// prologue of Alg. 1 for one job (every update item recomputes it in LDS).
// Its barriers order LDS only: what it stores to memory (pushed levels) is
// read by later calls.  stageGidx: the job's granule list into sh.gidx as
// well (a job run by one workgroup), loaded with the domain words.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void prologue(const KArgs& a, const DevJob& J, Shared& sh, bool pushHere, bool stageGidx) {
  const TabDesc* T = J.tab;
  SlotDesc* s = J.slot;
  const bool fromRoot = J.flags & JF_FROM_ROOT;
  const bool root = J.flags & JF_ROOT;
  const bool scratch = J.flags & JF_SCRATCH;
  const int n = T->n, D = T->D;
  // read before the first barrier (a load after one waits its round trip):
  // the table's and slot's addresses, this thread's first domain word with
  // its record and previous word, and its entry of both index buffers (the
  // one in use is known after the barrier); addresses are clamped, values
  // selected afterwards
  const int policy = T->policy;
  const int nGran = T->nGran;
  const CT_G WordDesc* words = T->words;
  const CT_G uint64_t* last = fromRoot ? T->dom0 : s->lastDom;
  const int q0 = min((int)threadIdx.x, D - 1);
  const uint64_t din0 = job_din(a, J, q0);
  const WordDesc wd0 = words[q0];
  const bool coh = J.flags & JF_COHLAST;
  const uint64_t ld0 = ld_last(last + q0, coh);
  const int p0 = min((int)threadIdx.x, nGran - 1);
  int ga = 0, gb = 0;
  if (stageGidx && !scratch) {
    ga = (fromRoot ? T->idx0 : s->idx[0])[p0];
    gb = fromRoot ? ga : s->idx[1][p0];
  }
  if (threadIdx.x == 0) {
    sh.bad_stray = 0;
    sh.bad_sub = 0;
    if (scratch) {  // every tuple, every granule
      sh.limit = T->nGran;
      sh.status = ST_OK;
    } else if (fromRoot) {
      sh.limit = T->limit0;
      sh.status = T->rootFailed ? ST_STATE : ST_OK;
    } else {
      sh.limit = s->limit;
      sh.status = s->failed ? ST_STATE : ST_OK;
    }
    sh.trailTop = s->trailTop;
    sh.cur = s->cur;
    sh.sp = slot_ptrs(s);
    sh.serial = J.nPush > 0 ? J.serialBase + J.nPush - 1 : s->serial;
    if (pushHere) {
      // this job's pushes record the state before it (levels of push_levels)
      const int d0 = s->depth;
      const int failed = s->failed;
      for (int k = 0; k < J.nPush; ++k) {
        Level L;
        L.trailTop = sh.trailTop;
        L.limit = sh.limit;
        L.failed = failed;
        L.serial = k == 0 ? s->serial : J.serialBase + k - 1;
        L.pad = 0;
        s->levels[d0 + k] = L;
      }
      sh.depth = d0;
      s->depth = d0 + J.nPush;
      s->serial = J.serialBase + J.nPush - 1;
    }
  }
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    sh.size[i] = 0;
    sh.dcnt[i] = 0;
  }
  lds_barrier();
  // one domain word per thread and pass: validation, Delta, |dom| per
  // variable; the first pass takes the words loaded above, and wider tables
  // load PRE_PASSES passes at once (one round trip, not one per pass: the
  // input may be in host memory)
  constexpr int PRE_PASSES = 4;
  uint64_t dinK = 0, dlK = 0;  // this thread's word and Delta word (D <= BLOCK)
  for (int qg = threadIdx.x; qg < D; qg += PRE_PASSES * BLOCK) {
    uint64_t dv[PRE_PASSES], lv[PRE_PASSES];
    WordDesc wv[PRE_PASSES];
#pragma unroll
    for (int g = 0; g < PRE_PASSES; ++g) {
      const int q = min(qg + g * BLOCK, D - 1);
      const bool first = g == 0 && qg == (int)threadIdx.x;
      if (g > 0 && D <= BLOCK) break;  // (one pass: nothing more to load)
      dv[g] = first ? din0 : job_din(a, J, q);
      wv[g] = first ? wd0 : words[q];
      lv[g] = first ? ld0 : ld_last(last + q, coh);
    }
#pragma unroll
    for (int g = 0; g < PRE_PASSES; ++g) {
      const int q = qg + g * BLOCK;
      if (q >= D) break;
      const uint64_t din = dv[g];
      const int i = wv[g].var;
      const VarDesc v = wv[g].v;
      const int used = v.dsize - 64 * (q - v.domOff);
      if (used < 64 && (din >> used) != 0) sh.bad_stray = 1;
      uint64_t dl = 0;
      if (!root) {
        const uint64_t ld = lv[g];
        if (din & ~ld) sh.bad_sub = 1;
        dl = ld & ~din;
        if (pushHere)
          for (int k = 0; k < J.nPush; ++k) s->levelDom[(int64_t)(sh.depth + k) * D + q] = ld;
      }
      if (q < MAX_D) sh.din[q] = din;
      if (q == (int)threadIdx.x) {
        dinK = din;
        dlK = dl;
      }
      atomicAdd(&sh.size[i], __popcll(din));
      atomicAdd(&sh.dcnt[i], __popcll(dl));
    }
  }
  if (stageGidx) {
    if ((int)threadIdx.x < nGran) sh.gidx[threadIdx.x] = (uint16_t)(scratch ? (int)threadIdx.x : sh.cur ? gb : ga);
    const CT_G int32_t* gsrc = fromRoot ? T->idx0 : sh.sp.idx[sh.cur];
    for (int p = threadIdx.x + BLOCK; p < nGran; p += BLOCK) sh.gidx[p] = (uint16_t)(scratch ? p : gsrc[p]);
  }
  lds_barrier();
  if (threadIdx.x < WAVE) {
    // wave 0: the segments of s_val in variable order (prefix sums over the
    // variables, 64 at a time)
    const int lane = threadIdx.x;
    int nseg = 0, nrows = 0;
    for (int i0 = 0; i0 < n; i0 += WAVE) {
      const int i = i0 + lane;
      bool inSval = false;
      int inc = 0, cnt = 0;
      if (i < n) {
        inSval = root || sh.dcnt[i] > 0;  // |dom| changed since the last call
        if (inSval) {
          inc = root ? 0 : (policy == 2 ? 1 : policy == 1 ? 0 : (sh.dcnt[i] < sh.size[i] ? 1 : 0));
          cnt = inc ? sh.dcnt[i] : sh.size[i];
        }
      }
      const int segIncl = wave_scan_incl(inSval ? 1 : 0);
      const int rowsIncl = wave_scan_incl(cnt);
      if (i < n) {
        if (inSval) {
          const int sg = nseg + segIncl - 1;
          sh.segOf[i] = sg;
          sh.segInc[sg] = inc;
          sh.segEnd[sg] = nrows + rowsIncl;
        } else {
          sh.segOf[i] = -1;
        }
      }
      nseg += __builtin_amdgcn_readlane(segIncl, WAVE - 1);
      nrows += __builtin_amdgcn_readlane(rowsIncl, WAVE - 1);
    }
    if (lane == 0) {
      if (sh.status == ST_OK) {
        if (sh.bad_stray) sh.status = ST_INVALID;
        else if (sh.bad_sub) sh.status = ST_NOT_SUBSET;
      }
      sh.nseg = nseg;
      sh.nrows = nrows;
      sh.noop = (nseg == 0) && !fromRoot;
    }
  }
  lds_barrier();
  if (sh.status != ST_OK || sh.noop) return;
  if (D <= BLOCK && sh.nrows <= ROWS_CHUNK) {
    // the row list from the words in registers: segments follow variable
    // order and a variable's words are consecutive, so a word's first entry
    // is the exclusive prefix sum of the selected bits of the words before it
    const int q = threadIdx.x;
    const int sg = q < D ? sh.segOf[wd0.var] : -1;
    const bool inc = sg >= 0 && sh.segInc[sg];
    uint64_t bits = sg < 0 ? 0ull : inc ? dlK : dinK;
    int tot = 0;
    int off = block_scan_excl<true>(__popcll(bits), &tot, sh);
    const int base = wd0.v.rowStart + (q - wd0.v.domOff) * 64;
    while (bits) {
      const int b = __ffsll((unsigned long long)bits) - 1;
      bits &= bits - 1;
      sh.rows[off++] = (uint32_t)(base + b);
    }
  } else {
    stage_rows(J, sh, 0, last, words);
  }
  lds_barrier();
}

// Entries [k0, k0 + ROWS_CHUNK) of the job's row list into sh.rows: the
// selected rows of every segment, in segment order; word q of variable i
// contributes the set bits of its Delta word (incremental) or domain word
// (reset) in ascending order.  Whole block; a barrier must follow.
// (lastArr, wordsArr: the previous domains and the word records as the
// caller read their addresses, else read here)
__device__ void stage_rows(const DevJob& J, Shared& sh, int k0, const CT_G uint64_t* lastArr,
                           const CT_G WordDesc* wordsArr) {
  const TabDesc* T = J.tab;
  const CT_G uint64_t* last = lastArr ? lastArr : (J.flags & JF_FROM_ROOT) ? T->dom0 : J.slot->lastDom;
  const bool coh = J.flags & JF_COHLAST;
  const CT_G WordDesc* words = wordsArr ? wordsArr : T->words;
  const int k1 = k0 + ROWS_CHUNK;
  for (int q = threadIdx.x; q < T->D; q += BLOCK) {
    const WordDesc wd = words[q];
    const int sg = sh.segOf[wd.var];
    if (sg < 0) continue;
    const VarDesc v = wd.v;
    const int inc = sh.segInc[sg];
    int off = sg == 0 ? 0 : sh.segEnd[sg - 1];
    for (int k = v.domOff; k < q && off < k1; ++k) {
      const uint64_t dk = din_at(J, sh, k);
      off += __popcll(inc ? (ld_last(last + k, coh) & ~dk) : dk);
    }
    const uint64_t dq = din_at(J, sh, q);
    uint64_t bits = inc ? (ld_last(last + q, coh) & ~dq) : dq;
    if (off >= k1 || off + __popcll(bits) <= k0) continue;
    const int base = v.rowStart + (q - v.domOff) * 64;
    while (bits && off < k1) {
      const int b = __ffsll((unsigned long long)bits) - 1;
      bits &= bits - 1;
      if (off >= k0) sh.rows[off - k0] = (uint32_t)(base + b);
      ++off;
    }
  }
}

// ---------------------------------------------------------------------------
// updateTable (Alg. 2) for NG granules per wave starting at position p0,
// RU support rows in flight per granule.  Granule flags go to LDS (whole job
// in one workgroup) or to global memory.
// ---------------------------------------------------------------------------
template <int NG, int RU = ROW_UNROLL>
__device__ __forceinline__ void update_granules(const KArgs& a, const DevJob& J, Shared& sh, int p0, bool lds,
                                int* trailCounter, const SlotPtrs* sp = nullptr) {
  const TabDesc* T = J.tab;
  SlotDesc* s = J.slot;
  const bool fromRoot = J.flags & JF_FROM_ROOT;
  const bool root = J.flags & JF_ROOT;
  // levels exist only above depth 0: nothing is saved at depth 0
  const bool trailOn = !fromRoot && !root && J.depthAfter > 0;
  const int nGran = T->nGran;
  const int64_t stride = T->stride;
  const int64_t W = T->W;
  const int limit = sh.limit;
  const int status = sh.status;
  const int noop = sh.noop;
  const int nseg = sh.nseg, nrows = sh.nrows;
  const int serial = sh.serial;
  const int lane = lane_id();
  const bool scratch = J.flags & JF_SCRATCH;
  // the slot's arrays as the prologue read them (sp, in LDS), or from the
  // descriptor
  const CT_G uint64_t* srcCt = fromRoot ? T->ct0 : sp ? sp->ct : s->ct;
  const CT_G int32_t* srcIdx = fromRoot ? T->idx0 : sp ? sp->idx[sh.cur] : s->idx[s->cur];
  const CT_G int32_t* stampArr = sp ? sp->stamp : s->stamp;
  const int64_t trailTop = sh.trailTop;

  // Loads below are unconditional, from clamped (always valid) addresses, and
  // their results are selected afterwards: a load under a branch is followed
  // by a wait for it, which would serialize the round trips to memory.
  unsigned long long nAct = 0;
  int pos[NG], g[NG], gs[NG], stv[NG];
  bool act[NG];
  uint64_t old[NG], m[NG], acc[NG];
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    pos[u] = p0 + u;
    const int pc = min(pos[u], nGran - 1);
    g[u] = scratch ? pc : lds ? (int)sh.gidx[pc] : srcIdx[pc];
    if (pos[u] >= nGran) g[u] = -1;
    act[u] = pos[u] < limit && status == ST_OK;
    gs[u] = act[u] ? g[u] : 0;
    const uint64_t o = scratch ? all_tuples_word(T, (int64_t)gs[u] * GW + lane) : srcCt[(int64_t)gs[u] * GW + lane];
    const int sv = stampArr[gs[u]];
    old[u] = act[u] ? o : 0ull;
    stv[u] = (act[u] && trailOn && !noop) ? sv : serial;
    m[u] = ~0ull;
    acc[u] = 0ull;
    nAct += act[u] ? 1 : 0;
  }
  // a row list longer than the LDS chunk is staged chunk by chunk, with the
  // whole block (every wave runs this loop the same number of times)
  const bool work = status == ST_OK && !noop;
  const bool chunked = nrows > ROWS_CHUNK;
  int seg = 0;
  int segEnd = nseg > 0 ? sh.segEnd[0] : 0;
  for (int c0 = 0; work && c0 < nrows; c0 += ROWS_CHUNK) {
    if (chunked) {
      __syncthreads();
      stage_rows(J, sh, c0);
      __syncthreads();
    }
    if (nAct == 0) continue;
    const int c1 = min(nrows, c0 + ROWS_CHUNK);
    for (int k0 = c0; k0 < c1; k0 += RU) {
      uint64_t v[RU][NG];
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const int k = k0 + j;
        const int r = k < c1 ? (int)sh.rows[k - c0] : 0;  // rows past the end are never used
#pragma unroll
        for (int u = 0; u < NG; ++u) v[j][u] = T->S[(int64_t)r * stride + (int64_t)gs[u] * GW + lane];
      }
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const int k = k0 + j;
        if (k >= c1) break;
        while (k >= segEnd) {
          const int inc = sh.segInc[seg];
#pragma unroll
          for (int u = 0; u < NG; ++u) {
            m[u] &= inc ? ~acc[u] : acc[u];
            acc[u] = 0ull;
          }
          ++seg;
          segEnd = sh.segEnd[seg];
        }
#pragma unroll
        for (int u = 0; u < NG; ++u) acc[u] |= v[j][u];
      }
    }
  }
  if (work && nAct > 0) {
    while (seg < nseg) {  // remaining segments (an empty reset segment gives 0)
      const int inc = sh.segInc[seg];
#pragma unroll
      for (int u = 0; u < NG; ++u) {
        m[u] &= inc ? ~acc[u] : acc[u];
        acc[u] = 0ull;
      }
      ++seg;
    }
  }
  // new words, and which granules need saving on the trail (first change in
  // this level); one trail allocation per wave
  uint64_t nw[NG];
  bool need[NG], wr[NG];
  int nNeed = 0;
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    nw[u] = noop ? old[u] : (old[u] & m[u]);
    const bool changed = act[u] && (__ballot(nw[u] != old[u]) != 0ull);
    need[u] = changed && trailOn && stv[u] != serial;
    nNeed += need[u] ? 1 : 0;
    wr[u] = act[u] && (changed || fromRoot || root);
  }
  int tbase = 0;
  // the slot's arrays, read once: the stores below could otherwise force a
  // reload (and a wait) of the descriptor before each of them
  const SlotPtrs P = sp ? *sp : slot_ptrs(s);
  const int64_t trailCap = P.trailCap;
  CT_G uint64_t* const sCt = P.ct;
  CT_G uint64_t* const sTrailWords = P.trailWords;
  CT_G TrailHdr* const sTrailHdr = P.trailHdr;
  CT_G int32_t* const sStamp = P.stamp;
  CT_G int32_t* const sNz = P.nzFlag;
  CT_G uint64_t* const ctOut = J.ct_out;
  if (nNeed) {
    if (lane == 0) tbase = atomicAdd(trailCounter, nNeed);
    tbase = __shfl(tbase, 0);
  }
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    if (pos[u] >= nGran || status != ST_OK) continue;
    const int64_t w = (int64_t)g[u] * GW + lane;
    if (pos[u] >= limit) {
      // inactive granule (all zero by invariant)
      if (fromRoot) sCt[w] = 0ull;
      if (ctOut && w < W) ctOut[w] = 0ull;
      continue;
    }
    if (need[u]) {
      const int64_t tp = trailTop + tbase++;
      if (tp < trailCap) {
        sTrailWords[tp * GW + lane] = old[u];
        if (lane == 0) {
          TrailHdr h;
          h.gran = g[u];
          h.oldStamp = stv[u];
          sTrailHdr[tp] = h;
          sStamp[g[u]] = serial;
        }
      } else if (lane == 0) {
        raise_error(a, 2);  // capacity is sized so that this cannot happen
      }
    }
    if (wr[u]) sCt[w] = nw[u];
    if (ctOut && w < W) ctOut[w] = nw[u];
    const bool nz = __ballot(nw[u] != 0ull) != 0ull;
    if (lane == 0) {
      if (lds) sh.nz[pos[u]] = nz ? 1 : 0;
      else sNz[pos[u]] = nz ? 1 : 0;
    }
  }
  if (lane == 0 && status == ST_OK) {
    if (nAct && !noop) atomicAdd(&s->stats[S_GRAN_ROWS], nAct * (unsigned long long)nrows);
    if (nNeed) atomicAdd(&s->stats[S_TRAIL], (unsigned long long)nNeed);
  }
}

// ---------------------------------------------------------------------------
// A job that resets its slot to the root (depth 0) and then rejects its input
// still performs the reset: the slot becomes a copy of the table's root state
// (threads tid of nthr, a workgroup or a wave; a rare path, so the whole
// currTable is copied).
// ---------------------------------------------------------------------------
__device__ void slot_reset_root(const TabDesc* T, SlotDesc* s, int serial, int tid, int nthr) {
  for (int64_t w = tid; w < T->stride; w += nthr) s->ct[w] = T->ct0[w];
  for (int p = tid; p < T->nGran; p += nthr) s->idx[0][p] = T->idx0[p];
  for (int q = tid; q < T->D; q += nthr) s->lastDom[q] = T->dom0[q];
  if (tid == 0) {
    s->cur = 0;
    s->limit = T->limit0;
    s->failed = T->rootFailed;
    s->depth = 0;
    s->trailTop = 0;
    s->serial = serial;
  }
}

// ---------------------------------------------------------------------------
// End of updateTable for a job (one workgroup): stable partition of the
// active granule list (survivors first), new limit, trail top, FAIL when no
// granule survives (Alg. 1's failure test).  Returns the job status.
// ---------------------------------------------------------------------------
__device__ int finalize_update(const DevJob& J, Shared& sh, bool ldsFlags, int jobTrail, bool count = true) {
  const TabDesc* T = J.tab;
  // a negative table's currTable holds forbidden tuples: empty means no
  // combination is forbidden, not a failure
  const bool negative = T->kind != 0;
  SlotDesc* s = J.slot;
  const bool fromRoot = J.flags & JF_FROM_ROOT;
  const int limit = sh.limit;
  const int nGran = T->nGran;
  int st = sh.status;
  if (st == ST_OK && !sh.noop) {
    const bool scratch = J.flags & JF_SCRATCH;  // index = identity
    // the index buffers and flags as the prologue read them (sh.sp, sh.cur)
    const CT_G int32_t* src = fromRoot ? T->idx0 : sh.sp.idx[sh.cur];
    const int dstBuf = fromRoot ? 0 : 1 - sh.cur;
    CT_G int32_t* dst = sh.sp.idx[dstBuf];
    const CT_G int32_t* nzf = sh.sp.nzFlag;
    const int per = (limit + BLOCK - 1) / BLOCK;
    const int b = min((int)threadIdx.x * per, limit);
    const int e = min(b + per, limit);
    int cnt = 0;
    for (int p = b; p < e; ++p) cnt += ldsFlags ? sh.nz[p] : nzf[p];
    int nSurv = 0;
    int sv = block_scan_excl<true>(cnt, &nSurv, sh);
    int zr = nSurv + (b - sv);
    for (int p = b; p < e; ++p) {
      const int gid = scratch ? p : ldsFlags ? (int)sh.gidx[p] : src[p];
      const int f = ldsFlags ? sh.nz[p] : nzf[p];
      if (f) dst[sv++] = gid; else dst[zr++] = gid;
    }
    for (int p = limit + threadIdx.x; p < nGran; p += BLOCK)
      dst[p] = scratch ? p : ldsFlags ? (int)sh.gidx[p] : src[p];
    if (nSurv == 0 && !negative) st = ST_FAIL;
    if (threadIdx.x == 0) {
      s->cur = dstBuf;
      sh.cur = dstBuf;  // a second pass over the job (negative tables) reads it
      s->limit = nSurv;
      if (fromRoot) {
        s->depth = 0;
        s->trailTop = 0;
        s->serial = J.serialBase;
        s->failed = 0;
      } else {
        s->trailTop = sh.trailTop + jobTrail;
      }
      if (nSurv == 0 && !negative) s->failed = 1;
    }
  } else if (fromRoot && st != ST_OK) {
    slot_reset_root(T, s, J.serialBase, threadIdx.x, blockDim.x);
  }
  if (threadIdx.x == 0) {
    s->status = st;
    s->pad2 = sh.noop;
    if (count && (st == ST_OK || st == ST_FAIL)) {
      atomicAdd(&s->stats[S_JOBS], 1ull);
      atomicAdd(&s->stats[S_GRAN_IN], (unsigned long long)limit);
      atomicAdd(&s->stats[S_ROWS], (unsigned long long)(sh.noop ? 0 : sh.nrows));
    }
  }
  __syncthreads();
  return st;
}

// ---------------------------------------------------------------------------
// filterDomains (Alg. 3) for domain word q, by one wave: residue word first,
// then the active granules in index order until a support is found.
// ---------------------------------------------------------------------------
// What filterDomains reads for domain word q before currTable is final: the
// word, its variable's size, and per value (lane) the residue and the support
// word at the residue (supports and residues do not change during the
// update), so a filter that waits for the update has them loaded meanwhile.
struct FilterPre {
  uint64_t din, sres;
  VarDesc v;
  int size, rl, rw0;
};

// (din: the input word q, size: the size of its variable's input domain)
__device__ __forceinline__ FilterPre filter_pre_of(const DevJob& J, int q, const VarDesc& v, uint64_t din,
                                                   int size) {
  const TabDesc* T = J.tab;
  const int lane = lane_id();
  FilterPre f;
  f.v = v;
  f.din = din;
  f.size = size;
  const int rowBase = f.v.rowStart + (q - f.v.domOff) * 64;
  // these loads run before the job's input is validated: a lane past the
  // variable's last value (a stray bit) takes the word's first row, and the
  // residue is clamped to the row, so every address is inside the table
  const int used = f.v.dsize - 64 * (q - f.v.domOff);
  const bool present = lane < used && ((f.din >> lane) & 1ull);
  // unconditional loads from valid addresses (row of the word's first value
  // for absent lanes), results selected afterwards
  f.rl = present ? rowBase + lane : rowBase;
  f.rw0 = min(max(J.slot->res[f.rl], 0), (int)T->stride - 1);
  f.sres = T->S[(int64_t)f.rl * T->stride + f.rw0];
  return f;
}

__device__ __forceinline__ FilterPre filter_pre(const KArgs& a, const DevJob& J, int q) {
  const VarDesc v = J.tab->words[q].v;
  int size = 0;
  for (int k = v.domOff; k < v.domOff + v.domWords; ++k) size += __popcll(job_din(a, J, k));
  return filter_pre_of(J, q, v, job_din(a, J, q), size);
}

__device__ __forceinline__ void filter_word(const KArgs& a, const DevJob& J, int q, int noop, int lim,
                                            const CT_G int32_t* idx, unsigned long long* cnt, const FilterPre& f,
                            bool haveCtRes = false, uint64_t ctRes = 0ull, CT_G uint64_t* ctArr = nullptr,
                            CT_G int32_t* resArr = nullptr, const int* idxHead = nullptr,
                            const uint64_t* ctHead = nullptr, bool phys = false) {
  const TabDesc* T = J.tab;
  SlotDesc* slot = J.slot;
  // the slot's arrays, read once (see update_granules), or as the caller
  // read them
  struct {
    CT_G uint64_t* ct;
    CT_G int32_t* res;
  } sv{ctArr ? ctArr : slot->ct, resArr ? resArr : slot->res}, *s = &sv;
  const int lane = lane_id();
  const VarDesc v = f.v;
  const uint64_t din = f.din;
  const int size = f.size;
  uint64_t dout = din;
  if (!noop && size > 1) {  // s_sup: non-singleton variables
    const int64_t stride = T->stride;
    const int rowBase = v.rowStart + (q - v.domOff) * 64;
    const bool present = (din >> lane) & 1ull;
    const int rl = f.rl;
    const int rw0 = f.rw0;
    // the currTable word at the residue (loaded by the caller with those of
    // other words, or here)
    const uint64_t cr = haveCtRes ? ctRes : s->ct[rw0];
    const bool hit = present && (cr & f.sres) != 0ull;
    unsigned long long miss = __ballot(present && !hit);
    cnt[0] += __popcll(__ballot(present));
    cnt[1] += __popcll(miss);
    uint64_t unsup = 0;
    // phys: the caller loaded every granule of a table of at most
    // FULL_SCAN_GRAN granules into ctHead (physical order; inactive ones are
    // all zero)
    if (miss && lim > 0 && (phys || lim <= FULL_SCAN_GRAN)) {
      // few active granules: each missing value tests every active word at
      // once (FULL_SCAN_VALS values per round trip, one word per lane and
      // granule); a value with no supported word among them has no support
      int gg[FULL_SCAN_GRAN];
      uint64_t c[FULL_SCAN_GRAN];
      const int nG = T->nGran;
#pragma unroll
      for (int j = 0; j < FULL_SCAN_GRAN; ++j) {
        if (phys) {
          gg[j] = j < nG ? j : -1;
          c[j] = j < nG ? ctHead[j] : 0ull;
          continue;
        }
        // the first FULL_SCAN_GRAN entries of the index as the caller read
        // them, or from memory
        const int gv = idxHead ? idxHead[j] : idx[min(j, lim - 1)];
        gg[j] = j < lim ? gv : -1;
        const uint64_t cv = s->ct[(int64_t)gv * GW + lane];
        c[j] = j < lim ? cv : 0ull;
      }
      uint64_t todo = miss;
      while (todo) {
        int ls[FULL_SCAN_VALS];
#pragma unroll
        for (int v = 0; v < FULL_SCAN_VALS; ++v) {
          ls[v] = todo ? __ffsll((unsigned long long)todo) - 1 : -1;
          todo &= todo - 1;
        }
        uint64_t x[FULL_SCAN_VALS][FULL_SCAN_GRAN];
#pragma unroll
        for (int v = 0; v < FULL_SCAN_VALS; ++v) {
          const CT_G uint64_t* row = T->S + (int64_t)(rowBase + max(ls[v], 0)) * stride;
#pragma unroll
          for (int j = 0; j < FULL_SCAN_GRAN; ++j) x[v][j] = row[(int64_t)max(gg[j], 0) * GW + lane] & c[j];
        }
#pragma unroll
        for (int v = 0; v < FULL_SCAN_VALS; ++v) {
          if (ls[v] < 0) continue;
          cnt[2] += (unsigned long long)lim;
          bool found = false;
#pragma unroll
          for (int j = 0; j < FULL_SCAN_GRAN; ++j) {
            const unsigned long long bm = __ballot(x[v][j] != 0ull);
            if (bm) {
              if (lane == 0) s->res[rowBase + ls[v]] = gg[j] * GW + (__ffsll(bm) - 1);
              found = true;
              break;
            }
          }
          if (!found) unsup |= 1ull << ls[v];
        }
      }
    } else {
      if (miss) {
        // every missing lane first walks the words after its old residue
        // (wrapping at the end of the table): a value's supports are spread
        // over the whole table, so a nearby word usually still holds one
        const bool mine = (miss >> lane) & 1ull;
        const int r = rl;
        const int64_t words = (int64_t)T->nGran * GW;
        int64_t w = mine ? (int64_t)rw0 : 0;
        bool found = false;
  #pragma unroll 1
        for (int step = 0; step < LANE_SCAN; step += 8) {
          uint64_t x[8];
          int64_t ww[8];
  #pragma unroll
          for (int j = 0; j < 8; ++j) {
            ww[j] = w + 1 + step + j;
            if (ww[j] >= words) ww[j] -= words;
            const uint64_t y = s->ct[ww[j]] & T->S[(int64_t)r * stride + ww[j]];
            x[j] = (mine && !found) ? y : 0ull;
          }
  #pragma unroll
          for (int j = 0; j < 8; ++j) {
            if (!found && x[j]) {
              found = true;
              s->res[r] = (int)ww[j];
            }
          }
          if (!__ballot(mine && !found)) break;
        }
        cnt[2] += __popcll(__ballot(mine));
        miss = __ballot(mine && !found);
      }
      // the values still without a support scan the active granules in index
      // order together: each step loads 4 currTable granules once and tests
      // them against the rows of up to 3 values at a time; a value leaves the
      // scan at its first supported word (its new residue)
      uint64_t todo = miss;
      for (int p = 0; p < lim && todo; p += 4) {
        int gg[4];
        uint64_t c[4];
  #pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int gv = idx[min(p + j, lim - 1)];
          gg[j] = (p + j < lim) ? gv : -1;
          const uint64_t cv = s->ct[(int64_t)gv * GW + lane];
          c[j] = gg[j] >= 0 ? cv : 0ull;
        }
        cnt[2] += (unsigned long long)min(4, lim - p) * (unsigned long long)__popcll(todo);
        uint64_t t = todo;
        while (t) {
          int ls[3];
  #pragma unroll
          for (int v = 0; v < 3; ++v) {
            ls[v] = t ? __ffsll((unsigned long long)t) - 1 : -1;
            t &= t - 1;
          }
          uint64_t x[3][4];
  #pragma unroll
          for (int v = 0; v < 3; ++v) {
            const CT_G uint64_t* row = T->S + (int64_t)(rowBase + max(ls[v], 0)) * stride;
  #pragma unroll
            for (int j = 0; j < 4; ++j) {
              const uint64_t y = c[j] & row[(int64_t)max(gg[j], 0) * GW + lane];
              x[v][j] = (ls[v] >= 0 && gg[j] >= 0) ? y : 0ull;
            }
          }
  #pragma unroll
          for (int v = 0; v < 3; ++v) {
            if (ls[v] < 0) continue;
  #pragma unroll
            for (int j = 0; j < 4; ++j) {
              const unsigned long long bm = __ballot(x[v][j] != 0ull);
              if (bm) {
                if (lane == 0) s->res[rowBase + ls[v]] = gg[j] * GW + (__ffsll(bm) - 1);
                todo &= ~(1ull << ls[v]);
                break;
              }
            }
          }
        }
      }
      unsup = todo;
    }
    dout = din & ~unsup;
  }
  if (J.flags & JF_LL) {
    if (lane < 2) ll_put(J.ll + 2 + 2 * q + lane, eng_slot((uint32_t)(lane ? dout >> 32 : dout), (uint32_t)J.seq));
  } else if (lane == 0) {
    J.dom_out[q] = dout;
  }
  if (lane == 0) slot->lastDom[q] = dout;
}

__device__ __forceinline__ void filter_word(const KArgs& a, const DevJob& J, int q, int noop, int lim,
                                            const CT_G int32_t* idx, unsigned long long* cnt) {
  filter_word(a, J, q, noop, lim, idx, cnt, filter_pre(a, J, q));
}

__device__ void add_filter_stats(SlotDesc* s, const unsigned long long* cnt) {
  if (lane_id() == 0 && (cnt[0] | cnt[1] | cnt[2])) {
    atomicAdd(&s->stats[S_RES_CHECK], cnt[0]);
    atomicAdd(&s->stats[S_RES_MISS], cnt[1]);
    atomicAdd(&s->stats[S_SCAN], cnt[2]);
  }
}

// ---------------------------------------------------------------------------
// split mode: one update item of a job (the last one finalizes the job)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void do_update(const KArgs& a, const DevJob& J, int chunk, Shared& sh) {
  SlotDesc* s = J.slot;
  if (J.nPop > 0) {
    if (!block_wait(a, &s->prepDone, 1, sh)) return;
  }
  // a job of one update item runs the whole update in this workgroup, as
  // in solo mode: pushes in the prologue (unless the prep item made them),
  // granule list, flags and trail count in LDS, no global round trip
  // between the update and the partition (one call site each of the
  // prologue and the update: a second would take the kernel arguments'
  // address)
  const bool one = J.nUpd == 1;
  if (one && threadIdx.x == 0) sh.trailCount = 0;
  prologue(a, J, sh, one && J.nPop == 0 && J.nPush > 0, one);
  // the job's tile: each wave takes tile granules of the item, NGW at a
  // time (the item covers WAVES x tile granules)
  if (one && J.tab->nGran <= WAVES) {
    // at most one granule per wave: twice the rows in flight instead
    update_granules<1, 2 * ROW_UNROLL>(a, J, sh, wave_id(), true, &sh.trailCount, &sh.sp);
  } else {
    const int reps = tile_reps(J.tile);
    for (int r = 0; r < reps; ++r)
      update_granules<NGW>(a, J, sh, ((chunk * reps + r) * WAVES + wave_id()) * NGW, one,
                           one ? &sh.trailCount : &s->jobTrail, &sh.sp);
  }
  if (one) {
    lds_barrier();
    if (J.nPop > 0 && threadIdx.x == 0) s->prepDone = 0;  // the prep item also did the pushes
    const int st = finalize_update(J, sh, true, sh.trailCount);
    if (threadIdx.x == 0) {
      if (st != ST_OK) publish_status(J, st);
      // finalize_update ends with a full barrier: the block's writes are
      // ordered before this release; a currTable copy in host memory is
      // made visible before the filter publishes the status
      if (J.ct_out) status_fence(J);
      // consumed (and reset) by the job's last filter item, or a flagged
      // job's number
      st_release(&s->updDone, (J.flags & JF_LL) ? ll_gen(J.seq) : 1);
    }
    return;
  }

  // count finished items; the last one finalizes the job
  __syncthreads();
  if (threadIdx.x == 0) {
    item_fence(J);
    const int prev = atomicAdd(&s->updCount, 1);
    sh.isLast = prev == J.nUpd - 1;
    if (sh.isLast) {
      s->updCount = 0;
      __threadfence();
    }
  }
  __syncthreads();
  if (!sh.isLast) return;

  if (J.nPop > 0) {
    if (threadIdx.x == 0) s->prepDone = 0;  // the prep item also did the pushes
  } else if (J.nPush > 0) {
    // pushes record the state before this job
    if (threadIdx.x == 0) {
      sh.depth = s->depth;
      sh.bad_sub = s->failed;
      sh.item = s->serial;
    }
    __syncthreads();
    push_levels(J, s, sh.depth, sh.trailTop, sh.limit, sh.bad_sub, sh.item, J.tab->D);
    __syncthreads();
    if (threadIdx.x == 0) {
      s->depth = sh.depth + J.nPush;
      s->serial = J.serialBase + J.nPush - 1;
    }
  }
  if (threadIdx.x == 0) sh.trailCount = s->jobTrail;
  __syncthreads();
  const int st = finalize_update(J, sh, false, sh.trailCount);
  if (threadIdx.x == 0) {
    s->jobTrail = 0;
    if (st != ST_OK) publish_status(J, st);
    // finalize_update ends with a barrier: the block's writes are ordered
    // before this release
    st_release(&s->updDone, (J.flags & JF_LL) ? ll_gen(J.seq) : 1);
  }
}

// split mode: one filter item (one domain word per wave)
__device__ __forceinline__ void do_filter(const KArgs& a, const DevJob& J, int chunk, Shared& sh) {
  SlotDesc* s = J.slot;
  const int q = chunk * WAVES + wave_id();
  const int qc = min(q, J.tab->D - 1);
  // in flight while the update runs: what filterDomains needs of the input
  // (filter_pre) and the slot's array addresses, which never change
  CT_G uint64_t* const sct = s->ct;
  CT_G int32_t* const sres = s->res;
  CT_G int32_t* const idx0 = s->idx[0];
  CT_G int32_t* const idx1 = s->idx[1];
  const FilterPre pre = filter_pre(a, J, qc);
  if (threadIdx.x < 3) sh.fcnt[threadIdx.x] = 0ull;
  const bool ll = J.flags & JF_LL;
  if (!block_wait(a, &s->updDone, ll ? ll_gen(J.seq) : 1, sh)) return;
  // one round trip: the job's state after the update, per value the
  // currTable word at its residue, and the head of both index buffers (the
  // one in use is known with the state)
  const int jobStatus = s->status, noop = s->pad2, lim = s->limit, cur = s->cur;
  const uint64_t cr = sct[pre.rw0];
  const int nG = J.tab->nGran;
  int h0[FULL_SCAN_GRAN], h1[FULL_SCAN_GRAN], head[FULL_SCAN_GRAN];
#pragma unroll
  for (int j = 0; j < FULL_SCAN_GRAN; ++j) {
    h0[j] = idx0[min(j, nG - 1)];
    h1[j] = idx1[min(j, nG - 1)];
  }
#pragma unroll
  for (int j = 0; j < FULL_SCAN_GRAN; ++j) head[j] = cur ? h1[j] : h0[j];
  // a table of at most FULL_SCAN_GRAN granules: all of currTable, in the
  // same round trip
  uint64_t cth[FULL_SCAN_GRAN];
#pragma unroll
  for (int j = 0; j < FULL_SCAN_GRAN; ++j) cth[j] = sct[(int64_t)min(j, nG - 1) * GW + lane_id()];
  unsigned long long cnt[3] = {0, 0, 0};
  if (q < J.tab->D && jobStatus == ST_OK)
    filter_word(a, J, q, noop, lim, cur ? idx1 : idx0, cnt, pre, true, cr, sct, sres, head, cth,
                nG <= FULL_SCAN_GRAN);
  // the item's counts, summed in LDS: one set of counter atomics per item
  if (lane_id() == 0 && (cnt[0] | cnt[1] | cnt[2]))
    for (int k = 0; k < 3; ++k) atomicAdd(&sh.fcnt[k], cnt[k]);
  // the last filter item of the job reports OK
  __syncthreads();
  if (threadIdx.x == 0) add_filter_stats(s, sh.fcnt);
  if (ll) return;  // the host counts the domain words itself
  if (threadIdx.x == 0) {
    status_fence(J);  // no other item reads this one's outputs
    const int prev = atomicAdd(&s->filtCount, 1);
    if (prev == J.nFilt - 1) {
      s->filtCount = 0;
      s->updDone = 0;
      if (jobStatus == ST_OK) publish_status(J, ST_OK);
    }
  }
}

// ---------------------------------------------------------------------------
// filterDomains of a negative table for domain word q (one wave; whole job
// in one workgroup).  currTable holds the forbidden tuples whose values are
// all in the input domains; value a of x_i has an allowed tuple iff fewer
// than prod_{k != i} |dom(x_k)| (sh.dcnt[i], capped above the tuple count)
// of them have x_i = a.  Each lane counts its value's row against the
// active granules (currTable words are the same for every lane).  Returns
// the filtered word.
// ---------------------------------------------------------------------------
__device__ uint64_t neg_filter_word(const DevJob& J, int q, int lim, const CT_G int32_t* idx, const Shared& sh) {
  const TabDesc* T = J.tab;
  const CT_G uint64_t* ct = J.slot->ct;
  const int i = T->wordVar[q];
  const VarDesc v = T->vars[i];
  const uint64_t din = sh.din[q];
  const int64_t prod = sh.dcnt[i];
  // no count can reach the product: every value keeps an allowed tuple
  if (din == 0ull || prod > (int64_t)lim * GW * 64) return din;
  const int lane = lane_id();
  const bool present = (din >> lane) & 1ull;
  const int row = v.rowStart + (q - v.domOff) * 64 + (present ? lane : 0);
  const CT_G uint64_t* srow = T->S + (int64_t)row * T->stride;
  int64_t cnt = 0;
  for (int p = 0; p < lim; ++p) {
    const int64_t base = (int64_t)idx[p] * GW;
#pragma unroll 8
    for (int k = 0; k < GW; ++k) cnt += __popcll(ct[base + k] & srow[base + k]);
  }
  return din & ~__ballot(present && cnt == prod);
}

// A negative table's filterDomains in one workgroup, after updateTable and
// its partition (st: the job status so far): per-variable products,
// every variable filtered into sh.dout, failure iff a domain empties.  On
// success the removed values' rows are listed as one incremental segment
// (in word order) for a second update pass that takes their tuples out of
// currTable.  Returns the status; *rows2 receives the listed rows.
__device__ int neg_filter(const DevJob& J, Shared& sh, int st, int* rows2) {
  SlotDesc* s = J.slot;
  const TabDesc* T = J.tab;
  const int n = T->n, D = T->D;
  *rows2 = 0;
  if (st != ST_OK) return st;
  const int64_t cap = (int64_t)T->nGran * GW * 64 + 1;
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    int64_t prod = 1;
    for (int k = 0; k < n; ++k) {
      if (k == i) continue;
      prod = min(prod * (int64_t)sh.size[k], cap);
    }
    sh.dcnt[i] = (int32_t)prod;
  }
  if (threadIdx.x == 0) sh.bad_sub = 0;
  __syncthreads();
  {
    const int lim = s->limit;
    const CT_G int32_t* idx = s->idx[s->cur];
    for (int q = wave_id(); q < D; q += WAVES) {
      const uint64_t dout = sh.noop ? sh.din[q] : neg_filter_word(J, q, lim, idx, sh);
      if (lane_id() == 0) sh.dout[q] = dout;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    const VarDesc v = T->vars[i];
    uint64_t any = 0ull;
    for (int k = 0; k < v.domWords; ++k) any |= sh.dout[v.domOff + k];
    if (!any) sh.bad_sub = 1;
  }
  __syncthreads();
  if (sh.bad_sub) {
    if (threadIdx.x == 0) {
      s->failed = 1;
      s->status = ST_FAIL;
    }
    return ST_FAIL;
  }
  if (sh.noop) return ST_OK;
  const int per = (D + BLOCK - 1) / BLOCK;
  const int b = min((int)threadIdx.x * per, D), e = min(b + per, D);
  int cnt = 0;
  for (int q = b; q < e; ++q) cnt += __popcll(sh.din[q] & ~sh.dout[q]);
  int total = 0;
  int off = block_scan_excl(cnt, &total, sh);
  for (int q = b; q < e; ++q) {
    const VarDesc v = T->vars[T->wordVar[q]];
    const int base = v.rowStart + (q - v.domOff) * 64;
    uint64_t bits = sh.din[q] & ~sh.dout[q];
    while (bits) {
      const int k = __ffsll((unsigned long long)bits) - 1;
      bits &= bits - 1;
      sh.rows[off++] = (uint32_t)(base + k);
    }
  }
  if (total > 0) {
    // the second pass reads the slot's own (updated) currTable and granule
    // list; its trail entries follow the first pass's
    if (threadIdx.x == 0) {
      sh.nseg = 1;
      sh.segEnd[0] = total;
      sh.segInc[0] = 1;
      sh.nrows = total;
      sh.status = ST_OK;
      sh.limit = s->limit;
      sh.trailTop = s->trailTop;
      sh.trailCount = 0;
    }
    __syncthreads();
    const CT_G int32_t* idx = s->idx[s->cur];
    for (int p = threadIdx.x; p < sh.limit; p += BLOCK) sh.gidx[p] = (uint16_t)idx[p];
    __syncthreads();
  }
  *rows2 = total;
  return ST_OK;
}

// ---------------------------------------------------------------------------
// solo mode: the whole job in one workgroup -- pops/pushes, prologue, all
// granules, partition, filter -- with no hand-off between workgroups.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void do_solo(const KArgs& a, const DevJob& J0, Shared& sh) {
  // a negative table filters before its update is complete (its second
  // pass takes the removed values' tuples out) and writes currTable out at
  // the end of the call
  const bool negative = J0.tab->kind != 0;
  DevJob J = J0;
  if (negative) J.ct_out = nullptr;
  SlotDesc* s = J.slot;
  const bool pushHere = J.nPop == 0 && J.nPush > 0;
  if (!pushHere) apply_pops_pushes(J, sh);
  // (the job's granule list is read once, in the prologue: each update step
  // is then a single round of independent loads)
  prologue(a, J, sh, pushHere, true);
  if (threadIdx.x == 0) sh.trailCount = 0;
  const int nGran = J.tab->nGran;
  int span = sh.status == ST_OK ? nGran : 0;
  __syncthreads();
  int st = ST_OK;
  for (int pass = 0;; ++pass) {
    for (int c = 0; c < span; c += WAVES * NGS) {
      update_granules<NGS>(a, J, sh, c + wave_id() * NGS, true, &sh.trailCount);
    }
    __syncthreads();
    st = finalize_update(J, sh, true, sh.trailCount, pass == 0);
    if (!negative || pass == 1) break;
    int rows2 = 0;
    st = neg_filter(J, sh, st, &rows2);
    if (rows2 == 0) break;
    span = sh.limit;
    J.flags &= ~(JF_FROM_ROOT | JF_ROOT | JF_SCRATCH);
  }
  if (negative) {
    __syncthreads();
    const TabDesc* T = J.tab;
    if (st == ST_OK) {
      for (int q = threadIdx.x; q < T->D; q += BLOCK) {
        J0.dom_out[q] = sh.dout[q];
        s->lastDom[q] = sh.dout[q];
      }
    }
    if (J0.ct_out && (st == ST_OK || st == ST_FAIL))
      for (int64_t w = threadIdx.x; w < T->W; w += BLOCK) J0.ct_out[w] = st == ST_OK ? s->ct[w] : 0ull;
  } else if (st == ST_OK) {
    unsigned long long cnt[3] = {0, 0, 0};
    const int lim = s->limit;
    const CT_G int32_t* idx = s->idx[s->cur];
    const int noop = sh.noop;
    for (int q = wave_id(); q < J.tab->D; q += WAVES) filter_word(a, J, q, noop, lim, idx, cnt);
    add_filter_stats(s, cnt);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    status_fence(J);
    publish_status(J, st);
  }
}

// ---------------------------------------------------------------------------
// Granule-major schedule of search nodes (jobs that all propagate one table
// from its root state).  The per-job schedules read every selected support
// row of a node from memory; here a workgroup stages one granule of every
// support row in LDS once and evaluates a group of nodes against it, so the
// supports cross the memory hierarchy once per group and HBM mostly sees the
// nodes' currTable writes.
//   nodes_prep:   one workgroup per node: Alg. 1 prologue -> encoded row list
//   nodes_update: one workgroup per (granule, node group): Alg. 2 from LDS
//   nodes_finish: one workgroup per node: partition, FAIL, Alg. 3, status
// ---------------------------------------------------------------------------
constexpr int NODES_MAX_ROWS = 256;  // LDS tile of the update kernel: rows x 512 B at least
constexpr int XCDS = 8;

// Orders this wave's LDS accesses: a wave's LDS operations complete in issue
// order, so only the compiler has to be kept from moving accesses across.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// One wave per node: the Alg. 1 prologue of a root reset.  Per variable the
// number of values of dom_in (|dom|) and of removed root values (|Delta|)
// decide membership of s_val and the branch of Alg. 2 (incremental when
// |Delta| < |dom|, or as the table's policy fixes it); the node's row list
// holds one segment with the rows of Delta of every incremental variable,
// then per reset variable of s_val a segment with the rows of dom, each
// segment padded to a multiple of 4 rows with the zero row and its first
// entry tagged.
__global__ void __launch_bounds__(BLOCK) nodes_prep_kernel(KArgs a, NodesDesc N) {
  __shared__ int32_t shSize[WAVES][MAX_ARITY];
  __shared__ int32_t shDcnt[WAVES][MAX_ARITY];
  __shared__ int32_t shSeg[WAVES][MAX_ARITY];  // first list entry | inc << 30, or -1 (not in s_val)
  __shared__ int32_t shWcnt[WAVES][MAX_D];     // popcount of Delta << 8 | popcount of dom, per word
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int j = blockIdx.x * WAVES + wv;
  if (j >= N.nJobs) return;  // no workgroup barrier below
  const int lane = lane_id();
  const DevJob J = N.jobs[j];
  const TabDesc* T = J.tab;
  const int n = T->n, D = T->D;
  const uint16_t zeroRow = (uint16_t)T->rows;
  int32_t* size = shSize[wv];
  int32_t* dcnt = shDcnt[wv];
  int32_t* seg = shSeg[wv];
  int32_t* wcnt = shWcnt[wv];
  for (int i = lane; i < n; i += WAVE) {
    size[i] = 0;
    dcnt[i] = 0;
  }
  wave_lds_sync();
  bool stray = false, notSub = false;
  for (int q = lane; q < D; q += WAVE) {
    const uint64_t din = J.dom_in[q];
    const uint64_t ld = T->dom0[q];
    const int i = T->wordVar[q];
    const VarDesc v = T->vars[i];
    const int used = v.dsize - 64 * (q - v.domOff);
    if (used < 64 && (din >> used) != 0) stray = true;
    if (din & ~ld) notSub = true;
    const int cs = __popcll(din), cd = __popcll(ld & ~din);
    wcnt[q] = (cd << 8) | cs;
    atomicAdd(&size[i], cs);
    atomicAdd(&dcnt[i], cd);
  }
  int st = T->rootFailed ? ST_STATE
           : __ballot(stray) ? ST_INVALID
           : __ballot(notSub) ? ST_NOT_SUBSET : ST_OK;
  wave_lds_sync();
  // segments.  Alg. 2's incremental masks AND together into the complement
  // of one OR over every removed value of those variables (De Morgan), so the
  // incremental variables of s_val share one segment, first, padded once to
  // a multiple of 4; each reset variable follows with a segment of its own,
  // padded the same way
  int total = 0, incTotal = 0;
  bool emptyReset = false;
  const int policy = T->policy;
  auto branch = [&](int i, bool* in, int* inc, int* cnt) {
    *in = false;
    *inc = 0;
    *cnt = 0;
    if (i >= n) return;
    const int sz = size[i], dc = dcnt[i];
    *in = dc > 0;  // |dom| changed since the root
    *inc = policy == 2 ? 1 : policy == 1 ? 0 : (dc < sz ? 1 : 0);
    *cnt = *in ? (*inc ? dc : sz) : 0;
  };
  for (int i0 = 0; i0 < n; i0 += WAVE) {
    const int i = i0 + lane;
    bool in;
    int inc, cnt;
    branch(i, &in, &inc, &cnt);
    const int c = (in && inc) ? cnt : 0;
    const int incl = wave_scan_incl(c);
    if (i < n) seg[i] = (in && inc) ? ((incTotal + incl - c) | (1 << 30)) : -1;
    incTotal += __builtin_amdgcn_readlane(incl, WAVE - 1);
  }
  const int incPadded = (incTotal + 3) & ~3;
  int padded = incPadded;
  total = incTotal;
  for (int i0 = 0; i0 < n; i0 += WAVE) {
    const int i = i0 + lane;
    bool in;
    int inc, cnt;
    branch(i, &in, &inc, &cnt);
    const bool rs = in && !inc;
    if (rs && cnt == 0) emptyReset = true;  // a reset segment of an empty domain
    const int c = rs ? cnt : 0;
    const int groups = (c + 3) >> 2;
    const int inclRows = wave_scan_incl(c);
    const int inclPad = wave_scan_incl(4 * groups);
    if (rs) seg[i] = padded + inclPad - 4 * groups;
    total += __builtin_amdgcn_readlane(inclRows, WAVE - 1);
    padded += __builtin_amdgcn_readlane(inclPad, WAVE - 1);
  }
  if (st == ST_OK && __ballot(emptyReset)) st = ST_FAIL;
  wave_lds_sync();
  if (st == ST_OK) {
    CT_G uint16_t* out = (CT_G uint16_t*)(N.nodes + (int64_t)j * N.nodeWords + sizeof(NodeInfo) / 8);
    for (int q = lane; q < D; q += WAVE) {
      const int i = T->wordVar[q];
      const int sg = seg[i];
      if (sg < 0) continue;
      const int inc = sg >> 30;
      const int start = sg & 0x3FFFFFFF;
      const VarDesc v = T->vars[i];
      int off = start;
      for (int k = v.domOff; k < q; ++k) off += inc ? (wcnt[k] >> 8) : (wcnt[k] & 0xFF);
      const uint64_t din = J.dom_in[q];
      uint64_t bits = inc ? (T->dom0[q] & ~din) : din;
      const int base = v.rowStart + (q - v.domOff) * 64;
      while (bits) {
        const int b = __ffsll((unsigned long long)bits) - 1;
        bits &= bits - 1;
        uint32_t e = (uint32_t)(base + b);
        // the first entry of the shared incremental segment, or of a reset
        // variable's segment, carries the segment tag
        if (inc ? off == 0 : off == start) e |= 0x8000u | (inc ? 0x4000u : 0u);
        out[off++] = (uint16_t)e;
      }
      // a reset variable's last word pads its segment
      if (!inc && q == v.domOff + v.domWords - 1)
        while (off & 3) out[off++] = zeroRow;
    }
    // the padding of the shared incremental segment
    if (lane < incPadded - incTotal) out[incTotal + lane] = zeroRow;
  }
  if (lane == 0) {
    NodeInfo I;
    I.status = st;
    I.nrows = (st == ST_OK || st == ST_FAIL) ? total : 0;
    I.groups = st == ST_OK ? padded / 4 : 0;
    I.pad = 0;
    I.ct = J.slot->ct;
    I.ct_out = J.ct_out;
    *(CT_G NodeInfo*)(N.nodes + (int64_t)j * N.nodeWords) = I;
  }
}

// A tile is TW consecutive granules (a span of 64·TW words) of the table for
// one group of nodes.  LDS holds that span of every support row (rows x 64·TW
// words) and a zero row, then the group's node records (NodeInfo and row
// list); a node then costs only LDS reads and its currTable store.  A list is
// read 8 rows per step: the row numbers come from registers by readlane (one
// group of 4 per lane), the rows are independent LDS reads OR-ed in.  With
// TW = 2 a lane holds two consecutive words and every row read is one 16-byte
// load per lane (1 KB per wave): LDS serves 16-byte loads at about twice the
// rate of 8-byte ones.  TW = 2 is used when the doubled tile fits a CU's LDS
// (one 16-wave workgroup per CU), else TW = 1 (8-wave workgroups, two per CU).
//
// Persistent workgroups (as many as fit at once) walk the tiles: while one
// tile is evaluated from LDS, the next one's words are already on their way
// into registers, so the memory latency of staging is hidden.  Block b runs on
// XCD b % 8 (round-robin dispatch) and works on the spans s with
// s % 8 == b % 8 (they stay in that XCD's L2): the XCD's tiles, span-major,
// are cut into one contiguous range per block, so a block keeps a span's
// rows in LDS across its groups and restages only the node records.
constexpr int NODES_TPF = 16;  // tile words per thread prefetched (rows <= 128)
constexpr int NODES_NPF = 5;   // node-record words per thread prefetched

template <int TW>
struct NodesCfg {
  static constexpr int SPAN = GW * TW;           // words per row of a tile
  static constexpr int BLOCKT = TW == 2 ? 1024 : 512;
  static constexpr int WAVEST = BLOCKT / WAVE;
  static constexpr int RSTEP = BLOCKT / SPAN;    // rows staged per pass (8)
};

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

struct NodesTile {
  int g, node0, nG, nodeTotal;  // g: first granule of the span
  u64x2 root;                   // the root's words of this lane (TW = 1: .x)
};

template <int TW>
__device__ __forceinline__ NodesTile nodes_tile(const NodesDesc& N, int xcd, int t) {
  NodesTile x;
  x.g = ((t / N.groups) * XCDS + xcd) * TW;
  x.node0 = (t % N.groups) * N.groupSize;
  x.nG = min(N.groupSize, N.nJobs - x.node0);
  x.nodeTotal = x.nG * N.nodeWords;
  const int64_t w = (int64_t)x.g * GW + TW * lane_id();
  if (TW == 2) {
    // a span past the last granule reads as zero
    x.root = w < N.stride ? *(const CT_G u64x2*)(N.ct0 + w) : u64x2{0ull, 0ull};
  } else {
    x.root = u64x2{N.ct0[w], 0ull};
  }
  return x;
}

// Staging of a tile: thread t holds words t % SPAN of tile rows t / SPAN + 8u
// and the words t + BLOCKT·u of the group's node records.
template <int TW>
__device__ __forceinline__ void nodes_stage_issue(const NodesDesc& N, const NodesTile& x, uint64_t* vt,
                                                  uint64_t* vn, bool rows) {
  using C = NodesCfg<TW>;
  const int r0 = (int)threadIdx.x / C::SPAN, l = (int)threadIdx.x % C::SPAN;
  const int64_t w = (int64_t)x.g * GW + l;
  const bool inRow = w < N.stride;  // words past the last granule are not loaded
  const CT_G uint64_t* S = N.S + (int64_t)r0 * N.stride + w;
  if (rows) {
#pragma unroll
    for (int u = 0; u < NODES_TPF; ++u)
      if (r0 + C::RSTEP * u < N.rows) vt[u] = inRow ? S[(int64_t)(C::RSTEP * u) * N.stride] : 0ull;
  }
  const CT_G uint64_t* src = N.nodes + (int64_t)x.node0 * N.nodeWords + threadIdx.x;
#pragma unroll
  for (int u = 0; u < NODES_NPF; ++u)
    if ((int)threadIdx.x + C::BLOCKT * u < x.nodeTotal) vn[u] = src[C::BLOCKT * u];
}

// Stores the prefetched words (and loads and stores any beyond them) and
// resets the tile's node counter; the caller synchronizes the workgroup
// afterwards.  The support rows are staged only for a new span.
template <int TW>
__device__ __forceinline__ void nodes_stage_commit(const NodesDesc& N, const NodesTile& x, const uint64_t* vt,
                                                   const uint64_t* vn, uint64_t* lds, bool rows, int* next) {
  using C = NodesCfg<TW>;
  const int r0 = (int)threadIdx.x / C::SPAN, l = (int)threadIdx.x % C::SPAN;
  const int64_t w = (int64_t)x.g * GW + l;
  const bool inRow = w < N.stride;
  if (rows) {
#pragma unroll
    for (int u = 0; u < NODES_TPF; ++u)
      if (r0 + C::RSTEP * u < N.rows) lds[(r0 + C::RSTEP * u) * C::SPAN + l] = vt[u];
    for (int r = r0 + C::RSTEP * NODES_TPF; r < N.rows; r += C::RSTEP)
      lds[r * C::SPAN + l] = inRow ? N.S[(int64_t)r * N.stride + w] : 0ull;
  }
  if (threadIdx.x == 0) *next = 0;
  uint64_t* dst = lds + (size_t)(N.rows + 1) * C::SPAN;  // the zero row sits between
#pragma unroll
  for (int u = 0; u < NODES_NPF; ++u) {
    const int i = (int)threadIdx.x + C::BLOCKT * u;
    if (i < x.nodeTotal) dst[i] = vn[u];
  }
  const CT_G uint64_t* src = N.nodes + (int64_t)x.node0 * N.nodeWords;
  for (int i = (int)threadIdx.x + C::BLOCKT * NODES_NPF; i < x.nodeTotal; i += C::BLOCKT) dst[i] = src[i];
}

// Row r of the tile for this lane: its word (TW = 1) or its two words (TW = 2).
template <int TW>
__device__ __forceinline__ u64x2 nodes_row(const char* tileBytes, uint32_t r, uint32_t laneOff) {
  if (TW == 2) return *(const u64x2*)(tileBytes + (r << 10) + laneOff);
  return u64x2{*(const uint64_t*)(tileBytes + (r << 9) + laneOff), 0ull};
}

template <int TW>
__device__ __forceinline__ void nodes_eval_tile(const NodesDesc& N, const NodesTile& x, const uint64_t* lds,
                                                int* next) {
  using C = NodesCfg<TW>;
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const uint64_t* recs = lds + (size_t)(N.rows + 1) * C::SPAN;
  const uint32_t laneOff = (uint32_t)lane * 8u * TW;
  const char* tileBytes = (const char*)lds;
  const int64_t w = (int64_t)x.g * GW + TW * lane;
  // the waves take the group's nodes one at a time from the tile's counter:
  // nodes differ in row count, so a fixed share per wave would leave waves
  // idle at the tile's barrier.  Every lane adds one, so a wave's fetch moves
  // the counter by 64 and the node is the value any lane got divided by 64:
  // no branch on the lane precedes the wave-uniform exit test (a
  // lane-0-only atomic followed by a shuffle let the compiler send the other
  // lanes back to the test with a stale node id, so they never left the loop)
  for (;;) {
    const int p = __builtin_amdgcn_readfirstlane(atomicAdd(next, 1)) >> 6;
    if (p >= x.nG) break;
    const NodeInfo* info = (const NodeInfo*)(recs + p * N.nodeWords);
    // the record is the same for every lane: scalar registers, uniform loops
    const int status = __builtin_amdgcn_readfirstlane(info->status);
    if (status != ST_OK && status != ST_FAIL) continue;  // rejected input: nothing changes
    const int ng = __builtin_amdgcn_readfirstlane(info->groups);
    const uint64_t* rl = (const uint64_t*)(info + 1);  // 4 entries per word
    const uint64_t m0 = status == ST_OK ? ~0ull : 0ull;
    u64x2 m = {m0, m0};
    u64x2 acc = {0ull, 0ull};
    bool inc = false, open = false;
    // the list, 64 groups of 4 row numbers at a time, one group per lane;
    // two groups (8 rows) per step, taken from the lanes by readlane, so the
    // row reads of a step never wait for an LDS read of row numbers; a missing
    // second group reads the zero row
    const uint64_t zeroGroup = (uint64_t)N.rows * 0x0001000100010001ull;
    for (int c0 = 0; c0 < ng; c0 += WAVE) {
      const uint64_t mine = c0 + lane < ng ? rl[c0 + lane] : zeroGroup;
      const uint32_t mlo = (uint32_t)mine, mhi = (uint32_t)(mine >> 32);
      const int cn = min(WAVE, ng - c0);
      for (int q = 0; q < cn; q += 2) {
        const uint32_t a0 = __builtin_amdgcn_readlane(mlo, q);
        const uint32_t a1 = __builtin_amdgcn_readlane(mhi, q);
        const uint32_t b0 = __builtin_amdgcn_readlane(mlo, q + 1);  // q + 1 <= 63
        const uint32_t b1 = __builtin_amdgcn_readlane(mhi, q + 1);
        // 8 rows in flight (TW = 1), or 4 when each is 16 bytes per lane
        u64x2 v[4], u[4];
        v[0] = nodes_row<TW>(tileBytes, a0 & 0x3FFFu, laneOff);
        v[1] = nodes_row<TW>(tileBytes, a0 >> 16, laneOff);
        v[2] = nodes_row<TW>(tileBytes, a1 & 0xFFFFu, laneOff);
        v[3] = nodes_row<TW>(tileBytes, a1 >> 16, laneOff);
        if (TW == 1) {
          u[0] = nodes_row<TW>(tileBytes, b0 & 0x3FFFu, laneOff);
          u[1] = nodes_row<TW>(tileBytes, b0 >> 16, laneOff);
          u[2] = nodes_row<TW>(tileBytes, b1 & 0xFFFFu, laneOff);
          u[3] = nodes_row<TW>(tileBytes, b1 >> 16, laneOff);
        }
        if (a0 & 0x8000u) {  // a segment starts with the first group
          if (open) m &= inc ? ~acc : acc;
          acc = u64x2{0ull, 0ull};
          inc = (a0 & 0x4000u) != 0;
          open = true;
        }
        acc |= (v[0] | v[1]) | (v[2] | v[3]);
        if (TW == 2) {
          u[0] = nodes_row<TW>(tileBytes, b0 & 0x3FFFu, laneOff);
          u[1] = nodes_row<TW>(tileBytes, b0 >> 16, laneOff);
          u[2] = nodes_row<TW>(tileBytes, b1 & 0xFFFFu, laneOff);
          u[3] = nodes_row<TW>(tileBytes, b1 >> 16, laneOff);
        }
        if (b0 & 0x8000u) {  // ... or with the second
          m &= inc ? ~acc : acc;
          acc = u64x2{0ull, 0ull};
          inc = (b0 & 0x4000u) != 0;
        }
        acc |= (u[0] | u[1]) | (u[2] | u[3]);
      }
    }
    if (open) m &= inc ? ~acc : acc;
    const u64x2 nw = x.root & m;
    CT_G uint64_t* ct = info->ct;
    CT_G uint64_t* ctOut = info->ct_out;
    const unsigned long long nzl = __ballot((nw.x | nw.y) != 0ull);
    if (TW == 2) {
      // lanes 0-31 hold granule g, lanes 32-63 granule g + 1 (when it exists)
      if (w < N.stride) *(CT_G u64x2*)(ct + w) = nw;
      if (ctOut) {
        if (w + 1 < N.W) {
          ctOut[w] = nw.x;
          ctOut[w + 1] = nw.y;
        } else if (w < N.W) {
          ctOut[w] = nw.x;
        }
      }
      if (lane == 0) {
        CT_G uint8_t* nz = N.nz + (int64_t)(x.node0 + p) * N.nGran + x.g;
        nz[0] = (nzl & 0xFFFFFFFFull) ? 1 : 0;
        if (x.g + 1 < N.nGran) nz[1] = (nzl >> 32) ? 1 : 0;
      }
    } else {
      ct[w] = nw.x;
      if (ctOut && w < N.W) ctOut[w] = nw.x;
      if (lane == 0) N.nz[(int64_t)(x.node0 + p) * N.nGran + x.g] = nzl ? 1 : 0;
    }
  }
}

template <int TW>
__global__ void __launch_bounds__(NodesCfg<TW>::BLOCKT, 4) nodes_update_kernel(KArgs a, NodesDesc N) {
  // the tile (16-byte row reads need the array at LDS offset 0: no static
  // LDS in this kernel), the group's node records, then the node counter
  extern __shared__ uint64_t lds[];
  using C = NodesCfg<TW>;
  int* next = (int*)(lds + (size_t)(N.rows + 1) * C::SPAN + (size_t)N.groupSize * N.nodeWords);
  const int xcd = blockIdx.x % XCDS;
  const int perX = gridDim.x / XCDS;  // the grid is a multiple of 8
  const int spans = (N.nGran + TW - 1) / TW;
  const int tilesX = (spans - xcd + XCDS - 1) / XCDS * N.groups;
  // the XCD's tiles, span by span with the groups of a span in a row, are
  // cut into one contiguous range per block: a block stages a span's rows
  // once and then only the next group's node records
  const int k = blockIdx.x / XCDS;
  const int hi = (int)((int64_t)(k + 1) * tilesX / perX);
  int t = (int)((int64_t)k * tilesX / perX);
  if (t >= hi) return;
  if (threadIdx.x < C::SPAN) lds[N.rows * C::SPAN + threadIdx.x] = 0ull;  // the zero row
  uint64_t vt[NODES_TPF], vn[NODES_NPF];
  NodesTile cur = nodes_tile<TW>(N, xcd, t);
  nodes_stage_issue<TW>(N, cur, vt, vn, true);
  nodes_stage_commit<TW>(N, cur, vt, vn, lds, true, next);
  __syncthreads();
  for (;;) {
    const int tn = t + 1;
    const bool more = tn < hi;
    NodesTile nxt;
    bool rows = false;
    if (more) {
      nxt = nodes_tile<TW>(N, xcd, tn);
      rows = nxt.g != cur.g;  // the same for every thread
      nodes_stage_issue<TW>(N, nxt, vt, vn, rows);  // in flight during the evaluation
    }
    nodes_eval_tile<TW>(N, cur, lds, next);
    __syncthreads();  // every wave is done with this tile's LDS
    if (!more) break;
    nodes_stage_commit<TW>(N, nxt, vt, vn, lds, rows, next);
    __syncthreads();
    t = tn;
    cur = nxt;
  }
}

// One wave per node, four nodes per workgroup, so the nodes of a batch are
// resident at once: the stable partition of the root's granule list by the
// non-zero flags (survivors first) and FAIL (Alg. 1), then filterDomains
// (Alg. 3) over the node's domain words.  The residue and support-word loads
// of FINISH_PRE domain words are issued before the partition and the node's
// currTable words at those residues together after it, so a node's chain of
// dependent memory rounds does not grow with its domain words.
constexpr int FINISH_BLOCK = 256;
constexpr int FINISH_NODES = FINISH_BLOCK / WAVE;
constexpr int FINISH_PRE = 4;

__global__ void __launch_bounds__(FINISH_BLOCK) nodes_finish_kernel(KArgs a, NodesDesc N) {
  const int j = blockIdx.x * FINISH_NODES + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  if (j >= N.nJobs) return;
  const int lane = lane_id();
  const DevJob J = N.jobs[j];
  const TabDesc* T = J.tab;
  SlotDesc* s = J.slot;
  const CT_G NodeInfo* rec = (const CT_G NodeInfo*)(N.nodes + (int64_t)j * N.nodeWords);
  const int st0 = rec->status;
  const int nrows = rec->nrows;
  const bool run = st0 == ST_OK || st0 == ST_FAIL;
  // the residues and support words of the first FINISH_PRE domain words:
  // independent of the partition, so their loads run meanwhile (they clamp
  // every address, so a rejected node's loads are harmless too)
  const int D = T->D;
  FilterPre pre[FINISH_PRE];
#pragma unroll
  for (int u = 0; u < FINISH_PRE; ++u) pre[u] = filter_pre(a, J, min(u, D - 1));
  int nSurv = 0;
  if (run) {
    const int limit0 = T->limit0, nGran = T->nGran;
    const CT_G uint8_t* nz = N.nz + (int64_t)j * nGran;
    const CT_G int32_t* src = T->idx0;
    CT_G int32_t* dst = s->idx[0];
    const uint64_t below = (1ull << lane) - 1ull;
    // granule ids and flags of 4 x 64 positions per round trip
    for (int p0 = 0; p0 < limit0; p0 += 4 * WAVE) {
      int gid[4];
      bool f[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = p0 + u * WAVE + lane;
        gid[u] = p < limit0 ? src[p] : -1;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) f[u] = gid[u] >= 0 && nz[gid[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u) nSurv += __popcll(__ballot(f[u]));
    }
    int sv = 0, zr = nSurv;
    for (int p0 = 0; p0 < limit0; p0 += 4 * WAVE) {
      int gid[4];
      bool f[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = p0 + u * WAVE + lane;
        gid[u] = p < limit0 ? src[p] : -1;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) f[u] = gid[u] >= 0 && nz[gid[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint64_t bs = __ballot(f[u]), bz = __ballot(gid[u] >= 0 && !f[u]);
        if (f[u]) dst[sv + __popcll(bs & below)] = gid[u];
        else if (gid[u] >= 0) dst[zr + __popcll(bz & below)] = gid[u];
        sv += __popcll(bs);
        zr += __popcll(bz);
      }
    }
    for (int p = limit0 + lane; p < nGran; p += WAVE) dst[p] = src[p];
    if (lane == 0) {
      s->cur = 0;
      s->limit = nSurv;
      s->depth = 0;
      s->trailTop = 0;
      s->serial = J.serialBase;
      s->failed = nSurv ? 0 : 1;
      atomicAdd(&s->stats[S_JOBS], 1ull);
      atomicAdd(&s->stats[S_GRAN_IN], (unsigned long long)limit0);
      atomicAdd(&s->stats[S_ROWS], (unsigned long long)nrows);
      if (nrows) atomicAdd(&s->stats[S_GRAN_ROWS], (unsigned long long)limit0 * (unsigned long long)nrows);
    }
    __threadfence_block();  // the index written by the lanes is read by the filter's scans
  } else {
    slot_reset_root(T, s, J.serialBase, lane, WAVE);
  }
  const int st = run ? (nSurv ? ST_OK : ST_FAIL) : st0;
  if (st == ST_OK) {
    unsigned long long cnt[3] = {0, 0, 0};
    const CT_G uint64_t* ct = s->ct;
    for (int q0 = 0; q0 < D; q0 += FINISH_PRE) {
      if (q0 > 0) {
#pragma unroll
        for (int u = 0; u < FINISH_PRE; ++u) pre[u] = filter_pre(a, J, min(q0 + u, D - 1));
      }
      // the node's currTable words at the residues, all in flight together
      uint64_t cr[FINISH_PRE];
#pragma unroll
      for (int u = 0; u < FINISH_PRE; ++u) cr[u] = ct[pre[u].rw0];
#pragma unroll
      for (int u = 0; u < FINISH_PRE; ++u)
        if (q0 + u < D) filter_word(a, J, q0 + u, 0, nSurv, s->idx[0], cnt, pre[u], true, cr[u]);
    }
    add_filter_stats(s, cnt);
  }
  if (lane == 0) {
    s->status = st;
    s->pad2 = 0;
    status_fence(J);
    publish_status(J, st);
  }
}

// ---------------------------------------------------------------------------
// Batches whose jobs all recompute a root from scratch.  Stream: one wave per
// (job, granule); a currTable word is the AND over the variables of the OR
// of the support rows of the values in dom_in, starting from all tuples
// (Alg. 2 with every variable on the reset branch).  A granule's words are
// final once its wave ends, so the stream has no hand-offs; support rows are
// fetched ROOT_UNROLL at a time, each as one coalesced 512-byte non-temporal
// load of the wave (read once: kept out of the caches' way).  Finish (next launch): one workgroup per job validates dom_in,
// partitions the granules (survivors first; Alg. 1's FAIL when none), sets
// the slot to depth 0 and runs filterDomains (Alg. 3).  The launch boundary
// orders the two; a hand-off inside one launch would need a release per wave
// (an L2 write-back on this chip), which costs more than the second launch.
// ---------------------------------------------------------------------------
constexpr int ROOT_UNROLL = 4;

__global__ void __launch_bounds__(BLOCK) root_stream_kernel(KArgs a, RootDesc R) {
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const DevJob J = a.jobs[R.tasks[2 * blockIdx.x]];
  const int g = R.tasks[2 * blockIdx.x + 1] + wv;
  const TabDesc* T = J.tab;
  if (g >= T->nGran) return;
  const unsigned lane = (unsigned)lane_id();
  const int64_t stride = T->stride;
  const int64_t gOff = (int64_t)g * GW;
  uint64_t acc = all_tuples_word(T, gOff + lane);
  for (int i = 0; i < T->n; ++i) {
    const VarDesc v = T->vars[i];
    uint64_t orv = 0;
    for (int k = 0; k < v.domWords; ++k) {
      const int used = v.dsize - 64 * k;
      uint64_t bits = job_din(a, J, v.domOff + k);  // uniform
      if (used < 64) bits &= (1ull << used) - 1ull;  // stray bits: the finish rejects the job
      const CT_G uint64_t* rows = T->S + (int64_t)(v.rowStart + 64 * k) * stride + gOff;
      int b = 0;
      while (bits) {
        // past the last value the previous row is fetched again (OR is
        // idempotent, the load hits the cache)
        uint64_t x[ROOT_UNROLL];
#pragma unroll
        for (int u = 0; u < ROOT_UNROLL; ++u) {
          if (bits) {
            b = __ffsll((unsigned long long)bits) - 1;
            bits &= bits - 1;
          }
          x[u] = __builtin_nontemporal_load(rows + (int64_t)b * stride + lane);
        }
#pragma unroll
        for (int u = 0; u < ROOT_UNROLL; ++u) orv |= x[u];
      }
    }
    acc &= orv;
    if (__ballot(acc != 0ull) == 0ull) break;  // the granule is already empty
  }
  SlotDesc* s = J.slot;
  s->ct[gOff + lane] = acc;
  if (J.ct_out && gOff + lane < T->W) J.ct_out[gOff + lane] = acc;
  const bool nz = __ballot(acc != 0ull) != 0ull;
  if (lane == 0) {
    s->nzFlag[g] = nz ? 1 : 0;
    if (nz) atomicAdd(&s->nzCount, 1);
  }
}

__global__ void __launch_bounds__(BLOCK) root_finish_kernel(KArgs a) {
  __shared__ int32_t shSurv, shStray, shRows;
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const DevJob J = a.jobs[blockIdx.x];
  const TabDesc* T = J.tab;
  SlotDesc* s = J.slot;
  // the filter's first two words per wave: their residue loads are in
  // flight during the validation and the partition (their addresses stay in
  // the table whatever the input)
  const int D = T->D;
  const FilterPre pre0 = filter_pre(a, J, min(wv, D - 1));
  const FilterPre pre1 = filter_pre(a, J, min(wv + WAVES, D - 1));
  if (threadIdx.x == 0) {
    shStray = 0;
    shRows = 0;
    shSurv = s->nzCount;  // counted by the stream
    s->nzCount = 0;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < T->D; q += BLOCK) {
    const uint64_t din = job_din(a, J, q);
    const VarDesc v = T->vars[T->wordVar[q]];
    const int used = v.dsize - 64 * (q - v.domOff);
    if (used < 64 && (din >> used) != 0) shStray = 1;
    atomicAdd(&shRows, __popcll(din));
  }
  __syncthreads();
  int st;
  if (shStray) {
    slot_reset_root(T, s, J.serialBase, threadIdx.x, BLOCK);  // the reset still happens
    st = ST_INVALID;
  } else {
    if (wv == 0) {
      const int nGran = T->nGran;
      const CT_G int32_t* nzf = s->nzFlag;
      CT_G int32_t* dst = s->idx[0];
      const uint64_t below = (1ull << lane) - 1ull;
      const int nSurv = shSurv;
      int sv = 0, zr = nSurv;
      for (int p0 = 0; p0 < nGran; p0 += WAVE) {
        const int p = p0 + lane;
        const bool in = p < nGran;
        const bool f = in && nzf[min(p, nGran - 1)] != 0;
        const uint64_t bs = __ballot(f), bz = __ballot(in && !f);
        if (f) dst[sv + __popcll(bs & below)] = p;
        else if (in) dst[zr + __popcll(bz & below)] = p;
        sv += __popcll(bs);
        zr += __popcll(bz);
      }
      if (lane == 0) {
        s->cur = 0;
        s->limit = nSurv;
        s->depth = 0;
        s->trailTop = 0;
        s->serial = J.serialBase;
        s->failed = nSurv ? 0 : 1;
        const unsigned long long rows = (unsigned long long)shRows;
        atomicAdd(&s->stats[S_JOBS], 1ull);
        atomicAdd(&s->stats[S_GRAN_IN], (unsigned long long)nGran);
        atomicAdd(&s->stats[S_ROWS], rows);
        if (rows) atomicAdd(&s->stats[S_GRAN_ROWS], (unsigned long long)nGran * rows);
      }
    }
    __syncthreads();
    st = shSurv ? ST_OK : ST_FAIL;
    if (st == ST_OK) {
      unsigned long long cnt[3] = {0, 0, 0};
      for (int q = wv, k = 0; q < D; q += WAVES, ++k) {
        if (k < 2) filter_word(a, J, q, 0, shSurv, s->idx[0], cnt, k == 0 ? pre0 : pre1);
        else filter_word(a, J, q, 0, shSurv, s->idx[0], cnt);
      }
      add_filter_stats(s, cnt);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s->status = st;
    s->pad2 = 0;
    if (J.flags & JF_HOST_OUT) __threadfence_system();
    publish_status(J, st);
  }
}

// Device-clock duration of a launch: first workgroup start to last end.
__device__ void clock_begin(const KArgs& a) {
  if (a.clock && threadIdx.x == 0) atomicMin(&a.clock[0], wall_clock64());
}

__device__ void clock_end(const KArgs& a) {
  if (!a.clock || threadIdx.x != 0) return;
  const unsigned long long now = wall_clock64();
  atomicMax(&a.clock[1], now);
  __threadfence();
  const unsigned long long prev = atomicAdd(&a.clock[2], 1ull);
  if (prev == gridDim.x - 1) {
    const unsigned long long t0 = atomicOr(&a.clock[0], 0ull);
    const unsigned long long t1 = atomicOr(&a.clock[1], 0ull);
    atomicAdd(&a.clock[3], t1 > t0 ? t1 - t0 : 0ull);
    atomicAdd(&a.clock[4], 1ull);
    a.clock[0] = ~0ull;
    a.clock[1] = 0ull;
    a.clock[2] = 0ull;
    __threadfence();
  }
}

__global__ void __launch_bounds__(BLOCK) propagate_kernel(KArgs a) {
  __shared__ Shared sh;
  int32_t* q = a.queue;
  const int total = a.nPrep + a.nUpd + a.nFilt;
  const bool dynamic = (int)gridDim.x < total;
  clock_begin(a);
  int item = blockIdx.x;
  while (item < total) {
    if (item < a.nPrep) {
      const int j = a.jobs ? a.prepList[item] : 0;
      const DevJob J = job_of(a, j);
      if (!J.active || *J.active) do_prep(a, J, sh);
    } else if (item < a.nPrep + a.nUpd) {
      const int x = item - a.nPrep;
      const int j = a.jobs ? find_job(a.updOff, a.nJobs, x) : 0;
      const DevJob J = job_of(a, j);
      if (J.active && !*J.active) {
        // a clean job of a model round: nothing to do
      } else if (J.flags & JF_SOLO) {
        do_solo(a, J, sh);
      } else {
        const int c = a.jobs ? x - a.updOff[j] : x;
        do_update(a, J, c, sh);
      }
    } else {
      const int x = item - a.nPrep - a.nUpd;
      const int j = a.jobs ? find_job(a.filtOff, a.nJobs, x) : 0;
      const int c = a.jobs ? x - a.filtOff[j] : x;
      const DevJob J = job_of(a, j);
      if (!J.active || *J.active) do_filter(a, J, c, sh);
    }
    if (!dynamic) break;
    __syncthreads();
    if (threadIdx.x == 0) sh.item = (int)gridDim.x + atomicAdd(&q[0], 1);
    __syncthreads();
    item = sh.item;
  }
  __syncthreads();
  clock_end(a);
  if (!dynamic) return;
  // the last workgroup out resets the queue for the next launch
  if (threadIdx.x == 0) {
    __threadfence();
    const int prev = atomicAdd(&q[1], 1);
    if (prev == (int)gridDim.x - 1) {
      q[0] = 0;
      q[1] = 0;
      q[2] += 1;  // dynamic launches completed (diagnostics)
      __threadfence();
    }
  }
}

// ---------------------------------------------------------------------------
// Resident split schedule of slot 0, for synchronous calls on tables whose
// update is one item: the split schedule's update item and filter items as
// one persistent launch that takes calls from the resident engine's mailbox
// (pinned host memory), so a call pays no kernel launch.  Workgroup 0 polls
// the mailbox, rings the doorbell ctl[SE_CALL] once a whole call is there,
// runs the call's pops, pushes, prologue, updateTable and partition, writes
// the status slot and hands over to the filters with the call's generation in
// updDone.  Filter workgroup c (filter item c) waits for the doorbell, reads
// its domain words from the mailbox itself, so its residue loads are in
// flight during the update; after the hand-over it filters and answers with
// flagged domain slots, then counts the call in ctl[SE_DONE] behind a
// release: workgroup 0 waits for that count before the next call reads the
// slot's domains.  The other workgroups of XCD 0 stay empty and workgroup 0
// takes no acquire between calls (JF_COHLAST), so its L2 keeps the table
// and the slot.  Workgroup 0 alone stops (a stop command, or no call for
// idleTicks) and sets ctl[SE_STOP], the word every wait of the launch
// watches, so the filters end too.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mb_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Workgroup 0's wave 0: waits for call `want` in the mailbox, copies its
// input words into ka.inl and its header into sh.se*; sh.seOp is 0 when no
// call came within idleTicks.  It polls the op slot alone (written last by
// the host: the lines the host is still writing are not read meanwhile),
// two loads in flight, then reads the whole command, U chunks of 64 slots
// per round trip.  Every lane loads (lanes past the command re-read its
// last slot): a load under a lane condition would be waited for before the
// test after it.
__device__ __forceinline__ void se_take_call(const EngDesc& E, KArgs& ka, Shared& sh, uint32_t want, int D) {
  constexpr int U = 8;
  const int l = lane_id();
  const uint64_t* slots = E.cmd->slot;
  const int nS = EC_DOM + 2 * D;
  uint32_t* in32 = (uint32_t*)ka.inl;
  const unsigned long long t0 = wall_clock64();
  bool seen = false;
  {
    uint64_t p0 = mb_load(slots + EC_OP);
    for (;;) {
      const uint64_t p1 = mb_load(slots + EC_OP);
      if (__builtin_amdgcn_readfirstlane((uint32_t)p0) == want) {
        seen = true;
        break;
      }
      p0 = mb_load(slots + EC_OP);
      if (__builtin_amdgcn_readfirstlane((uint32_t)p1) == want) {
        seen = true;
        break;
      }
      if ((long long)(wall_clock64() - t0) > E.idleTicks) break;
    }
  }
  uint32_t hv = 0;
  for (int c0 = 0; seen && c0 < nS; c0 += U * WAVE) {
    for (;;) {  // written before the op slot: normally present at once
      uint64_t w[U];
      bool ok = true;
#pragma unroll
      for (int u = 0; u < U; ++u) w[u] = mb_load(slots + min(c0 + u * WAVE + l, nS - 1));
#pragma unroll
      for (int u = 0; u < U; ++u) ok = ok && (uint32_t)w[u] == want;
      if (__all(ok)) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = c0 + u * WAVE + l;
          if (i >= EC_DOM && i < nS) in32[i - EC_DOM] = (uint32_t)(w[u] >> 32);
        }
        if (c0 == 0) hv = (uint32_t)(w[0] >> 32);
        break;
      }
      if ((long long)(wall_clock64() - t0) > E.idleTicks) {
        seen = false;
        break;
      }
    }
  }
  const int h0 = __shfl((int)hv, EC_OP), h1 = __shfl((int)hv, EC_NPOP), h2 = __shfl((int)hv, EC_NPUSH);
  const int h3 = __shfl((int)hv, EC_SERIAL), h4 = __shfl((int)hv, EC_DEPTH);
  if (l == 0) {
    sh.seOp = seen ? h0 : 0;
    sh.seNPop = h1;
    sh.seNPush = h2;
    sh.seSerial = h3;
    sh.seDepth = h4;
    // the filters' doorbell: the whole call is in the mailbox (a release: a
    // relaxed store can wait in this XCD's L2 until the next release, and
    // polls of one word at system scope from every filter workgroup queue
    // up at the memory)
    if (seen && h0 == ENG_OP_PROPAGATE) st_release(&E.ctl[SE_CALL], (int32_t)want);
  }
}

// A filter workgroup's input of call `want`.  Wave 0 waits for the doorbell
// (device memory: the host's lines are read by workgroup 0 alone) while the
// others wait at the barrier; then each wave reads the input slots of its
// variable's words (at most SE_MAX_VAR_WORDS, one slot per lane; the lanes
// past them re-read the last one, so a wave reads one or two lines of host
// memory) from the mailbox.  Returns false once the launch stops; else the
// word q and the size of its variable's input.
__device__ __forceinline__ bool se_filter_input(const EngDesc& E, Shared& sh, const VarDesc& v, int q,
                                                uint32_t want, uint64_t* din, int* size) {
  const int l = lane_id();
  const unsigned long long t0 = wall_clock64();
  if (wave_id() == 0) {
    int go = 0;
    for (;;) {
      if ((uint32_t)ld_relaxed(&E.ctl[SE_CALL]) == want) {
        go = 1;
        break;
      }
      // the launch has stopped, or (a bound that is never reached while
      // workgroup 0 runs) nothing has come for far longer than it waits
      if (ld_relaxed(&E.ctl[SE_STOP]) != 0 || (long long)(wall_clock64() - t0) > 8 * E.idleTicks) break;
      __builtin_amdgcn_s_sleep(1);
    }
    if (l == 0) sh.ok = go;
  }
  lds_barrier();
  if (!sh.ok) return false;
  const int nW = 2 * v.domWords;
  const uint64_t* mine = E.cmd->slot + EC_DOM + 2 * v.domOff + min(l, nW - 1);
  uint64_t x;
  for (;;) {  // all there once workgroup 0 rang
    x = mb_load(mine);
    if (__all((uint32_t)x == want)) break;
    if (ld_relaxed(&E.ctl[SE_STOP]) != 0 || (long long)(wall_clock64() - t0) > 8 * E.idleTicks) return false;
  }
  const uint32_t p = (uint32_t)(x >> 32);
  *size = __builtin_amdgcn_readlane(wave_scan_incl(l < nW ? __popc(p) : 0), WAVE - 1);
  const int k = 2 * (q - v.domOff);
  const uint32_t lo = (uint32_t)__shfl((int)p, k), hi = (uint32_t)__shfl((int)p, k + 1);
  *din = ((uint64_t)hi << 32) | lo;
  return true;
}

// Workgroup 0 waits until the filters have counted `want` calls (bounded:
// false on a device error or when the wait runs out).
__device__ __forceinline__ bool se_wait_done(const EngDesc& E, int want, Shared& sh) {
  if (threadIdx.x == 0) {
    int ok = 1;
    for (uint32_t it = 0;; ++it) {
      if (ld_relaxed(&E.ctl[SE_DONE]) == want) break;
      if (ld_relaxed(&E.ctl[SE_STOP]) > 0) { ok = 0; break; }
      if (it > SPIN_LIMIT) {
        atomicExch(&E.ctl[SE_STOP], 1);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    sh.ok = ok;
  }
  lds_barrier();
  const int ok = sh.ok;
  lds_barrier();
  return ok != 0;
}

// One call's update on workgroup 0: pops and pushes, prologue, updateTable
// and partition, then the hand-over to the filters.  Returns the status.
__device__ __forceinline__ int se_update(const KArgs& a, const DevJob& J, Shared& sh) {
  SlotDesc* s = J.slot;
  if (J.nPop > 0) apply_pops_pushes(J, sh);  // the pops, then the pushes
  if (threadIdx.x == 0) sh.trailCount = 0;
  prologue(a, J, sh, J.nPop == 0 && J.nPush > 0, true);
  if (J.tab->nGran <= WAVES)  // at most one granule per wave: twice the rows in flight
    update_granules<1, 2 * ROW_UNROLL>(a, J, sh, wave_id(), true, &sh.trailCount, &sh.sp);
  else
    update_granules<NGW>(a, J, sh, wave_id() * NGW, true, &sh.trailCount, &sh.sp);
  lds_barrier();
  const int st = finalize_update(J, sh, true, sh.trailCount);
  // finalize_update ends with a full barrier: the block's writes are ordered
  // before this release
  if (threadIdx.x == 0) st_release(&s->updDone, ll_gen(J.seq));
  return st;
}

__global__ void __launch_bounds__(BLOCK) split_engine_kernel(EngDesc E) {
  __shared__ Shared sh;
  __shared__ KArgs ka;  // the calls' view of the launched schedule's arguments
  const CT_G TabDesc* T = E.tab;
  CT_G SlotDesc* s = E.slot;
  const int D = T->D;
  if (threadIdx.x == 0) {
    ka.jobs = nullptr;
    ka.nJobs = 1;
    ka.queue = E.ctl;  // queue[3] = ctl[SE_STOP]: raise_error and block_wait use it
    ka.hostErr = nullptr;
    ka.clock = nullptr;
  }
  __syncthreads();
  DevJob J = {};
  J.tab = T;
  J.slot = s;
  J.flags = JF_PROPAGATE | JF_LL | JF_INLINE_DOM | JF_COHLAST;
  J.nUpd = 1;
  J.nFilt = E.nFilt;
  J.ll = E.res->slot + ER_DOM - 2;  // domain word q in slots ER_DOM + 2q, + 1
  uint32_t last = (uint32_t)E.startSeq;
  if (blockIdx.x == 0) {
    const unsigned long long tLife = wall_clock64();
    for (int served = 0;; ++served) {
      const uint32_t want = last + 1;
      if (threadIdx.x < WAVE) se_take_call(E, ka, sh, want, D);
      lds_barrier();
      if (sh.seOp != ENG_OP_PROPAGATE) break;
      // the filters' writes of the previous call (the slot's domains) first;
      // no acquire (it would invalidate this XCD's L2, which holds the table
      // and the slot between calls): those domains are read at device scope
      if (served > 0 && !se_wait_done(E, served * E.nFilt, sh)) {
        if (threadIdx.x == 0) ll_put(&E.res->slot[ER_STATUS], eng_slot((uint32_t)ST_DEVICE, want));
        last = want;
        break;
      }
      const unsigned long long tStart = wall_clock64();
      J.nPop = sh.seNPop;
      J.nPush = sh.seNPush;
      J.serialBase = sh.seSerial;
      J.depthAfter = sh.seDepth;
      J.seq = (int32_t)want;
      int st = se_update(ka, J, sh);
      if (threadIdx.x == 0) {
        if (ld_relaxed(&E.ctl[SE_STOP]) > 0) st = ST_DEVICE;
        const unsigned long long ticks = wall_clock64() - tStart;
        ll_put(&E.res->slot[ER_TICKS], eng_slot((uint32_t)min(ticks, 0xffffffffull), want));
        ll_put(&E.res->slot[ER_STATUS], eng_slot((uint32_t)st, want));
      }
      last = want;
      lds_barrier();
    }
    if (threadIdx.x == 0) {
      atomicCAS(&E.ctl[SE_STOP], 0, -1);
      E.res->exitSeq = (int32_t)last;
      E.res->lifeTicks = wall_clock64() - tLife;
      __threadfence_system();
      __hip_atomic_store(&E.res->alive, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    return;
  }
  // filter workgroup c: the workgroups of XCD 0 (every eighth, in the
  // dispatch order's round robin) are left to workgroup 0 and end here, so
  // the filters' acquires never invalidate its L2
  if (blockIdx.x % 8 == 0) return;
  const int c = (int)blockIdx.x - 1 - (int)blockIdx.x / 8;
  if (c >= E.nFilt) return;
  const int q = c * WAVES + wave_id();
  const int qc = min(q, D - 1);
  const VarDesc v = T->words[qc].v;
  CT_G uint64_t* const sct = s->ct;
  CT_G int32_t* const sres = s->res;
  CT_G int32_t* const idx0 = s->idx[0];
  CT_G int32_t* const idx1 = s->idx[1];
  const int nG = T->nGran;
  for (;;) {
    const uint32_t want = last + 1;
    uint64_t din = 0;
    int size = 0;
    const bool go = se_filter_input(E, sh, v, qc, want, &din, &size);
    if (lane_id() == 0) sh.wsum[wave_id()] = go ? 1 : 0;
    if (threadIdx.x < 3) sh.fcnt[threadIdx.x] = 0ull;
    lds_barrier();
    bool all = true;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) all = all && sh.wsum[w] != 0;
    if (!all) break;
    J.seq = (int32_t)want;
    const FilterPre pre = filter_pre_of(J, qc, v, din, size);
    if (!block_wait(ka, &s->updDone, ll_gen(J.seq), sh)) break;
    // as do_filter: the state after the update, the currTable word at each
    // value's residue and the head of both index buffers in one round trip
    const int jobStatus = s->status, noop = s->pad2, lim = s->limit, cur = s->cur;
    const uint64_t cr = sct[pre.rw0];
    int h0[FULL_SCAN_GRAN], h1[FULL_SCAN_GRAN], head[FULL_SCAN_GRAN];
#pragma unroll
    for (int j = 0; j < FULL_SCAN_GRAN; ++j) {
      h0[j] = idx0[min(j, nG - 1)];
      h1[j] = idx1[min(j, nG - 1)];
    }
#pragma unroll
    for (int j = 0; j < FULL_SCAN_GRAN; ++j) head[j] = cur ? h1[j] : h0[j];
    uint64_t cth[FULL_SCAN_GRAN];
#pragma unroll
    for (int j = 0; j < FULL_SCAN_GRAN; ++j) cth[j] = sct[(int64_t)min(j, nG - 1) * GW + lane_id()];
    unsigned long long cnt[3] = {0, 0, 0};
    if (q < D && jobStatus == ST_OK)
      filter_word(ka, J, q, noop, lim, cur ? idx1 : idx0, cnt, pre, true, cr, sct, sres, head, cth,
                  nG <= FULL_SCAN_GRAN);
    if (lane_id() == 0 && (cnt[0] | cnt[1] | cnt[2]))
      for (int k = 0; k < 3; ++k) atomicAdd(&sh.fcnt[k], cnt[k]);
    // every wave's stores of the slot's domains complete at the barrier; the
    // release makes them visible to workgroup 0 before the call is counted
    __syncthreads();
    if (threadIdx.x == 0) {
      add_filter_stats(s, sh.fcnt);
      __threadfence();
      atomicAdd(&E.ctl[SE_DONE], 1);
    }
    last = want;
  }
}

// ---------------------------------------------------------------------------
// support bitset builder: one wave per 64 tuples (one word column); for each
// column of the table every distinct row among the wave's lanes is written
// once with the ballot of the lanes holding that value (no atomics, each
// (row, word) has exactly one writer).  S must be zeroed beforehand.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BLOCK) build_supports_kernel(const int32_t* tuples, int64_t t,
                                                               int n, const VarDesc* vars,
                                                               const int32_t* lo, uint64_t* S,
                                                               int64_t stride, int64_t W) {
  const int64_t w = (int64_t)blockIdx.x * WAVES + wave_id();
  if (w >= W) return;
  const int lane = lane_id();
  const int64_t j = w * 64 + lane;
  for (int i = 0; i < n; ++i) {
    const VarDesc v = vars[i];
    int r = -1;
    bool star = false;
    if (j < t) {
      const int32_t raw = tuples[j * n + i];
      star = raw == STAR_CELL;
      const int64_t val = (int64_t)raw - lo[i];
      if (!star && val >= 0 && val < v.dsize) r = v.rowStart + (int)val;
    }
    // a star cell (short table) is in every row of its column: each row
    // word is the ballot of its lanes or'ed with the star lanes, written once
    const unsigned long long starMask = __ballot(star);
    if (starMask) {
      for (int k = 0; k < v.dsize; ++k) {
        const unsigned long long m = __ballot(r == v.rowStart + k) | starMask;
        if (lane == 0) S[(int64_t)(v.rowStart + k) * stride + w] = m;
      }
      continue;
    }
    bool pending = r >= 0;
    for (;;) {
      const unsigned long long act = __ballot(pending);
      if (!act) break;
      const int leader = __ffsll(act) - 1;
      const int rl = __shfl(r, leader);
      const unsigned long long mask = __ballot(pending && r == rl);
      if (lane == leader) S[(int64_t)rl * stride + w] = mask;
      if (r == rl) pending = false;
    }
  }
}

// copy the root state into n fresh slots (one workgroup per slot)
__global__ void __launch_bounds__(BLOCK) init_slots_kernel(const TabDesc* T, SlotDesc* slots,
                                                           int n, const int32_t* rootRes) {
  const int k = blockIdx.x;
  if (k >= n) return;
  SlotDesc* s = slots + k;
  const int64_t words = T->stride;
  for (int64_t w = threadIdx.x; w < words; w += BLOCK) s->ct[w] = T->ct0[w];
  for (int p = threadIdx.x; p < T->nGran; p += BLOCK) {
    s->idx[0][p] = T->idx0[p];
    s->idx[1][p] = T->idx0[p];
    s->stamp[p] = 0;
    s->nzFlag[p] = 0;
  }
  for (int q = threadIdx.x; q < T->D; q += BLOCK) s->lastDom[q] = T->dom0[q];
  for (int r = threadIdx.x; r < T->rows; r += BLOCK) s->res[r] = rootRes[r];
  if (threadIdx.x == 0) {
    s->trailTop = 0;
    s->cur = 0;
    s->limit = T->limit0;
    s->failed = T->rootFailed;
    s->depth = 0;
    s->serial = 0;
    s->updCount = 0;
    s->filtCount = 0;
    s->jobTrail = 0;
    s->prepDone = 0;
    s->updDone = 0;
    s->status = 0;
    s->nzCount = 0;
    s->pad2 = 0;
    for (int x = 0; x < 8; ++x) s->stats[x] = 0;
  }
}

// ---------------------------------------------------------------------------
// Propagation rounds of a multi-table model.  One round = gather -> propagate
// (every dirty table, one persistent launch) -> merge -> changed -> mark.
// All state lives on the device, so rounds can be captured in a graph; once
// nothing is dirty (or a table failed) the remaining rounds do no work.
// ---------------------------------------------------------------------------
// input of every dirty table: pool restricted to its scope, intersected with
// the domains the table returned last; poolNext starts as a copy of pool
__global__ void __launch_bounds__(BLOCK) model_gather_kernel(ModelDesc M) {
  const int stride = gridDim.x * BLOCK;
  for (int w = blockIdx.x * BLOCK + threadIdx.x; w < M.poolWords; w += stride) M.poolNext[w] = M.pool[w];
  if (M.flags[1]) return;
  for (int e = blockIdx.x * BLOCK + threadIdx.x; e < M.nEntries; e += stride) {
    const int c = M.scopeTab[e];
    if (!M.dirty[c]) continue;
    const int v = M.scopeVar[e];
    const int po = M.poolOff[v], nw = M.poolNW[v];
    const int to = M.entDomOff[e];
    const CT_G uint64_t* last = M.lastDom[c];
    CT_G uint64_t* din = M.domIn + M.bufOff[c];
    for (int q = 0; q < nw; ++q) din[to + q] = M.pool[po + q] & last[to + q];
  }
}

// Seeding the first round.  Every table's earlier pruning holds under the
// (smaller) input pool, so the pool is first ANDed with the domains each
// table returned last; a table then runs iff that pool removes a value from
// its domains.
__global__ void __launch_bounds__(BLOCK) model_seed_and_kernel(ModelDesc M) {
  const int stride = gridDim.x * BLOCK;
  for (int e = blockIdx.x * BLOCK + threadIdx.x; e < M.nEntries; e += stride) {
    const int c = M.scopeTab[e];
    const int v = M.scopeVar[e];
    const int po = M.poolOff[v], nw = M.poolNW[v], to = M.entDomOff[e];
    const CT_G uint64_t* last = M.lastDom[c];
    for (int q = 0; q < nw; ++q) atomicAnd((unsigned long long*)&M.poolNext[po + q], (unsigned long long)last[to + q]);
  }
}

__global__ void __launch_bounds__(BLOCK) model_seed_mark_kernel(ModelDesc M) {
  const int stride = gridDim.x * BLOCK;
  int any = 0, cnt = 0;
  for (int c = blockIdx.x * BLOCK + threadIdx.x; c < M.nTables; c += stride) {
    const CT_G uint64_t* last = M.lastDom[c];
    int d = 0;
    for (int e = M.tabScope[c]; e < M.tabScope[c + 1] && !d; ++e) {
      const int v = M.scopeVar[e];
      const int po = M.poolOff[v], nw = M.poolNW[v], to = M.entDomOff[e];
      for (int q = 0; q < nw; ++q)
        if (last[to + q] & ~M.poolNext[po + q]) d = 1;
    }
    M.dirty[c] = d;
    any |= d;
    cnt += d;
  }
  if (any) atomicOr(&M.flags[0], 1);
  if (cnt) atomicAdd(&M.flags[3], cnt);
}

// (kernel parameters never carry the address-space qualifier: host and device
// passes must mangle the kernel's name identically)
__global__ void __launch_bounds__(BLOCK) model_copy_kernel(uint64_t* dst, const uint64_t* src, int n) {
  CT_G uint64_t* d = (CT_G uint64_t*)dst;
  const CT_G uint64_t* sc = (const CT_G uint64_t*)src;
  for (int w = blockIdx.x * BLOCK + threadIdx.x; w < n; w += gridDim.x * BLOCK) d[w] = sc[w];
}

// AND every successful table's output into poolNext; a failure stops the model
__global__ void __launch_bounds__(BLOCK) model_merge_kernel(ModelDesc M) {
  const int stride = gridDim.x * BLOCK;
  for (int e = blockIdx.x * BLOCK + threadIdx.x; e < M.nEntries; e += stride) {
    const int c = M.scopeTab[e];
    if (!M.dirty[c]) continue;
    const int st = M.status[c];
    if (st != ST_OK) {
      if (e == M.tabScope[c]) atomicExch(&M.flags[1], st == ST_FAIL ? 1 : 2);
      continue;
    }
    const int v = M.scopeVar[e];
    const int po = M.poolOff[v], nw = M.poolNW[v];
    const CT_G uint64_t* dout = M.domOut + M.bufOff[c] + M.entDomOff[e];
    for (int q = 0; q < nw; ++q) atomicAnd((unsigned long long*)&M.poolNext[po + q], (unsigned long long)dout[q]);
  }
}

// variables whose pool domain shrank in this round; pool <- poolNext
__global__ void __launch_bounds__(BLOCK) model_changed_kernel(ModelDesc M) {
  const int stride = gridDim.x * BLOCK;
  if (blockIdx.x == 0 && threadIdx.x == 0) M.flags[0] = 0;
  for (int v = blockIdx.x * BLOCK + threadIdx.x; v < M.nPool; v += stride) {
    const int po = M.poolOff[v], nw = M.poolNW[v];
    int ch = 0;
    for (int q = 0; q < nw; ++q) {
      const uint64_t nx = M.poolNext[po + q];
      if (nx != M.pool[po + q]) ch = 1;
      M.pool[po + q] = nx;
    }
    M.changed[v] = ch;
  }
}

// a table is dirty in the next round iff a variable of its scope changed
__global__ void __launch_bounds__(BLOCK) model_mark_kernel(ModelDesc M) {
  const int stride = gridDim.x * BLOCK;
  const bool failed = M.flags[1] != 0;
  int any = 0, cnt = 0;
  for (int c = blockIdx.x * BLOCK + threadIdx.x; c < M.nTables; c += stride) {
    int d = 0;
    if (!failed)
      for (int e = M.tabScope[c]; e < M.tabScope[c + 1]; ++e) d |= M.changed[M.scopeVar[e]];
    M.dirty[c] = d;
    any |= d;
    cnt += d;
  }
  if (any) atomicOr(&M.flags[0], 1);
  if (cnt) atomicAdd(&M.flags[3], cnt);
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&M.flags[2], 1);
}

}  // namespace ctk

// ---------------------------------------------------------------------------
// launch wrappers used by the host runtime
// ---------------------------------------------------------------------------
namespace ctk {

// update items of a split job: WAVES x (granules per wave of its tile) granules each
int propagate_items_per_job_update(int nGran, int tile) {
  const int gpi = WAVES * NGW * tile_reps(tile);
  return (nGran + gpi - 1) / gpi;
}
int propagate_items_per_job_filter(int D) { return (D + WAVES - 1) / WAVES; }

// Workgroups of the propagate kernel that are resident at once on the whole
// device: the grid never exceeds it, so every workgroup that holds an item
// is running and every wait in the kernel can end.
int propagate_max_grid() {
  static int cached = 0;
  if (cached) return cached;
  int dev = 0, cus = 0, perCu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&perCu, propagate_kernel, BLOCK, 0) != hipSuccess ||
      perCu < 1)
    perCu = 1;
  cached = cus * perCu;
  return cached;
}

hipError_t launch_split_engine(const EngDesc& E, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(split_engine_kernel, dim3(grid), dim3(BLOCK), 0, stream, E);
  return hipGetLastError();
}

hipError_t launch_propagate(const KArgs& a, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(propagate_kernel, dim3(grid), dim3(BLOCK), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_build_supports(const int32_t* tuples, int64_t t, int n, const VarDesc* vars,
                                 const int32_t* lo, uint64_t* S, int64_t stride, int64_t W,
                                 hipStream_t stream) {
  if (W <= 0) return hipSuccess;
  const int64_t blocks = (W + WAVES - 1) / WAVES;
  hipLaunchKernelGGL(build_supports_kernel, dim3((unsigned)blocks), dim3(BLOCK), 0, stream, tuples,
                     t, n, vars, lo, S, stride, W);
  return hipGetLastError();
}

hipError_t launch_model_round(const ModelDesc& M, const KArgs& a, int grid, hipStream_t stream) {
  const int gb = 256;
  hipLaunchKernelGGL(model_gather_kernel, dim3(gb), dim3(BLOCK), 0, stream, M);
  hipLaunchKernelGGL(propagate_kernel, dim3(grid), dim3(BLOCK), 0, stream, a);
  hipLaunchKernelGGL(model_merge_kernel, dim3(gb), dim3(BLOCK), 0, stream, M);
  hipLaunchKernelGGL(model_changed_kernel, dim3(gb), dim3(BLOCK), 0, stream, M);
  hipLaunchKernelGGL(model_mark_kernel, dim3(gb), dim3(BLOCK), 0, stream, M);
  return hipGetLastError();
}

// M.pool holds the input; leaves pool = input AND every table's domains and
// the dirty flags of the first round.
int nodes_max_rows() { return NODES_MAX_ROWS; }

// Row-list entries per node (every segment padded to a multiple of 4, the
// list to a multiple of 4 entries).
int nodes_list_cap(int rows, int n) { return (rows + 3 * n + 3) & ~3; }

// Words of a node's record: its NodeInfo and its row list.
int nodes_node_words(int rows, int n) {
  return (int)(sizeof(NodeInfo) / 8) + nodes_list_cap(rows, n) / 4;
}

// Dynamic LDS of the update kernel for groups of `groupSize` nodes and tiles
// of `tw` granules: the tile with its zero row, the records, the node counter.
size_t nodes_update_lds(int rows, int n, int groupSize, int tw) {
  return (size_t)(rows + 1) * GW * tw * sizeof(uint64_t) +
         (size_t)groupSize * nodes_node_words(rows, n) * sizeof(uint64_t) + 16;
}

int nodes_update_block(int tw) { return tw == 2 ? NodesCfg<2>::BLOCKT : NodesCfg<1>::BLOCKT; }

// Persistent workgroups of the update kernel: as many as fit at once, a
// multiple of the XCD count.
template <int TW>
int nodes_update_grid(size_t ldsBytes) {
  int dev = 0, cus = 0, perCu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return XCDS;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&perCu, nodes_update_kernel<TW>, NodesCfg<TW>::BLOCKT,
                                                   ldsBytes) != hipSuccess ||
      perCu < 1)
    perCu = 1;
  return std::max(XCDS, cus * perCu / XCDS * XCDS);
}

hipError_t launch_nodes(const KArgs& a, const NodesDesc& N, int n, hipStream_t stream) {
  hipLaunchKernelGGL(nodes_prep_kernel, dim3((N.nJobs + WAVES - 1) / WAVES), dim3(BLOCK), 0, stream, a, N);
  const size_t lds = nodes_update_lds(N.rows, n, N.groupSize, N.tw);
  if (N.tw == 2)
    hipLaunchKernelGGL(nodes_update_kernel<2>, dim3(nodes_update_grid<2>(lds)), dim3(NodesCfg<2>::BLOCKT), lds,
                       stream, a, N);
  else
    hipLaunchKernelGGL(nodes_update_kernel<1>, dim3(nodes_update_grid<1>(lds)), dim3(NodesCfg<1>::BLOCKT), lds,
                       stream, a, N);
  hipLaunchKernelGGL(nodes_finish_kernel, dim3((N.nJobs + FINISH_NODES - 1) / FINISH_NODES), dim3(FINISH_BLOCK), 0,
                     stream, a, N);
  return hipGetLastError();
}

hipError_t launch_roots(const KArgs& a, const RootDesc& R, hipStream_t stream) {
  if (R.nTasks > 0)
    hipLaunchKernelGGL(root_stream_kernel, dim3(R.nTasks), dim3(BLOCK), 0, stream, a, R);
  hipLaunchKernelGGL(root_finish_kernel, dim3(a.nJobs), dim3(BLOCK), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_model_seed(const ModelDesc& M, hipStream_t stream) {
  hipLaunchKernelGGL(model_copy_kernel, dim3(64), dim3(BLOCK), 0, stream, (uint64_t*)M.poolNext,
                     (const uint64_t*)M.pool, M.poolWords);
  hipLaunchKernelGGL(model_seed_and_kernel, dim3(64), dim3(BLOCK), 0, stream, M);
  hipLaunchKernelGGL(model_seed_mark_kernel, dim3(64), dim3(BLOCK), 0, stream, M);
  hipLaunchKernelGGL(model_copy_kernel, dim3(64), dim3(BLOCK), 0, stream, (uint64_t*)M.pool,
                     (const uint64_t*)M.poolNext, M.poolWords);
  return hipGetLastError();
}

hipError_t launch_init_slots(const TabDesc* T, SlotDesc* slots, int n, const int32_t* rootRes,
                             hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(init_slots_kernel, dim3(n), dim3(BLOCK), 0, stream, T, slots, n, rootRes);
  return hipGetLastError();
}

}  // namespace ctk
