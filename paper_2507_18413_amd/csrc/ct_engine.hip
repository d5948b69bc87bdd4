// ct_engine.hip -- resident engine for synchronous calls on a table's primary
// slot (include/ct.h, CT_SCHED_RESIDENT).
//
// A synchronous call (ct_propagate) is a chain of dependent steps -- apply
// pops and pushes, the Alg. 1 prologue, updateTable (Alg. 2) over the active
// granules, the sparse-bitset compaction, filterDomains (Alg. 3) with its
// residues -- over a few hundred KB.  Launched per call, every step pays a
// round trip to memory and the call pays a launch.  Here one persistent
// workgroup of 16 waves keeps the slot's currTable, granule index, stamps,
// residues and last domains in LDS for as long as calls keep coming: only
// the support rows (read-only) and the trail (written on changes, read on
// pops) stay in HBM.  Calls arrive in a mailbox in coherent pinned host
// memory (EngCmd) and results leave the same way (EngRes).  The engine
// writes its state back to the slot and exits on a stop command or after
// `idleTicks` of device clock without a call, so every launch ends.
#include <hip/hip_runtime.h>

#include <cstddef>

#include "ct_device.h"

namespace ctk {
namespace {

constexpr int EBLOCK = 1024;
constexpr int EWAVES = EBLOCK / WAVE;
constexpr int E_NG = 4;          // granules per wave per update step
constexpr int E_ROWS = 6;        // support rows loaded per batch (even: row ids are read in pairs)
constexpr int E_LANE_SCAN = 16;  // words each missing lane checks after its residue
constexpr int E_POP_U = 8;       // granules per wave per step of a pop
constexpr int E_CMD_U = 8;       // 64-slot chunks of a long command loaded per round trip

struct EngState {
  int32_t op, seq, lastSeq, nPop, nPush, serialBase, depthAfter, wantCt, wantStats, pad3;
  int32_t limit, failed, depth, serial, cur, status, noop, nseg;
  int32_t nrows, badStray, badSub, trailCount, nSurv, devErr, nMiss, nLeft;
  int64_t trailTop, lvTrailTop;
  int64_t trLo;  // trail entries [trLo, trailTop) have their headers in the LDS ring
  int32_t lvLimit, lvFailed, lvSerial;
  int32_t lvLo;  // levels [lvLo, depth) have their records and domains in the LDS ring
  int32_t waveSum[EWAVES];
  unsigned long long stat[8];
};

// Dynamic LDS regions, in this order, each 8-byte aligned.
enum { R_CT, R_IDX0, R_IDX1, R_STAMP, R_NZ, R_FIRST, R_RES, R_LAST, R_DIN, R_ROWS, R_WVAR, R_VARS, R_VSIZE,
       R_VDCNT, R_SEGOF, R_SEGEND, R_SEGINC, R_WCNT, R_MSLOT, R_LEFT, R_MFOUND, R_STATE, R_TRH, R_LVR, R_LVD,
       R_END };

// LDS of one workgroup on gfx950; what the regions above leave of it holds
// rings that mirror the newest trail headers and level records (a pop then
// reads its headers, its level's record and its domains from LDS and only
// the saved words from HBM).
constexpr size_t E_LDS = 160 * 1024;
constexpr int E_TRH_MAX = 4096;  // trail headers mirrored (a power of two)
constexpr int E_LVR_MAX = 64;    // levels mirrored (a power of two)

// Tables of at most this many domain words filter one word per wave (one
// pass, no barrier); wider ones filter flat over the value slots.
constexpr int E_NARROW_D = 16;
// The flat filter keeps the values whose residue word missed in a list of at
// most this many entries (a domain slot fits 16 bits: ENG_MAX_D x 64 slots);
// wider domains are filtered in chunks of slots.
constexpr int E_MISS_CAP = 16384;
static_assert(ENG_MAX_D * 64 <= 65536, "domain slots fit 16 bits");
static_assert(E_ROWS % 2 == 0, "a batch starts on a pair of row ids");
static_assert(E_NG % 2 == 0, "the update takes granules in pairs");

__host__ __device__ inline size_t eng_align(size_t x) { return (x + 7) & ~(size_t)7; }

__host__ __device__ inline int eng_miss_cap(int D) { return D * 64 < E_MISS_CAP ? D * 64 : E_MISS_CAP; }

__host__ __device__ inline void eng_layout(int n, int D, int nGran, int rows, size_t* off, int* mirror = nullptr) {
  size_t sz[R_END];
  sz[R_CT] = (size_t)nGran * GW * 8;
  sz[R_IDX0] = sz[R_IDX1] = (size_t)nGran * 2;
  sz[R_STAMP] = (size_t)nGran * 4;
  sz[R_NZ] = (size_t)nGran;
  sz[R_FIRST] = (size_t)nGran * 4;
  sz[R_RES] = (size_t)rows * 4;
  sz[R_LAST] = sz[R_DIN] = (size_t)D * 8;
  sz[R_ROWS] = ((size_t)rows + 16) * 2;  // batches read up to 16 entries past the end
  sz[R_WVAR] = (size_t)D * 4;
  sz[R_VARS] = (size_t)n * sizeof(VarDesc);
  sz[R_VSIZE] = sz[R_VDCNT] = sz[R_SEGOF] = sz[R_SEGEND] = sz[R_SEGINC] = (size_t)n * 4;
  sz[R_WCNT] = (size_t)D * 4;
  const int cap = D > E_NARROW_D ? eng_miss_cap(D) : 0;
  sz[R_MSLOT] = sz[R_LEFT] = (size_t)cap * 2;
  sz[R_MFOUND] = (size_t)cap;
  sz[R_STATE] = sizeof(EngState);
  size_t o = 0;
  for (int r = 0; r < R_TRH; ++r) {
    off[r] = o;
    o += eng_align(sz[r]);
  }
  // the rings, each a power of two entries: levels first (up to half of
  // what is left), then trail headers, at least a call's worth (nGran)
  const size_t spare = o < E_LDS ? E_LDS - o : 0;
  const size_t lvBytes = (size_t)D * 8 + sizeof(Level);
  int lr = E_LVR_MAX;
  while (lr >= 4 && (size_t)lr * lvBytes > spare / 2) lr >>= 1;
  if (lr < 4) lr = 0;
  const size_t left = spare - (size_t)lr * lvBytes;
  int trh = 0;
  for (int t = E_TRH_MAX; t >= nGran && t > 0; t >>= 1)
    if ((size_t)t * sizeof(TrailHdr) <= left) {
      trh = t;
      break;
    }
  if (mirror) {
    mirror[0] = trh;
    mirror[1] = lr;
  }
  sz[R_TRH] = (size_t)trh * sizeof(TrailHdr);
  sz[R_LVR] = (size_t)lr * sizeof(Level);
  sz[R_LVD] = (size_t)lr * D * 8;
  for (int r = R_TRH; r < R_END; ++r) {
    off[r] = o;
    o += eng_align(sz[r]);
  }
  off[R_END] = o;
}

// Workgroup barrier that orders LDS only: outstanding global stores (trail,
// levels) need not complete here.  The end of every call has a full
// barrier, so a later call's waves see all of an earlier call's stores.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int e_lane() { return threadIdx.x & (WAVE - 1); }
// The thread index, opaque to the optimizer: a phase of the call loop
// computes its per-thread LDS addresses from it afresh, instead of keeping
// every phase's addresses live across the whole loop (which spilled them).
__device__ __forceinline__ int e_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}
// Flagged mailbox slots: 64-bit loads and stores at system scope (the
// pinned host buffers are read and written around the GPU's caches).
__device__ __forceinline__ uint64_t ll_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void ll_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ int e_wave() { return __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE); }

// Support rows through a buffer resource: one scalar descriptor, a scalar
// byte offset per (row, granule) and the lane's byte offset in one vector
// register shared by every load (loads past num_records return 0).
constexpr int BUF_DWORD3 = 0x00020000;  // raw buffer, gfx9 family

__device__ __forceinline__ uint64_t e_ld(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0);
  return (uint64_t)v[0] | ((uint64_t)v[1] << 32);
}

struct Eng {
  // table (read-only)
  __amdgpu_buffer_rsrc_t Sbuf;
  const CT_G uint64_t* S;
  int64_t stride, W;
  int n, D, nGran, rows, policy;
  // slot arrays in HBM
  CT_G SlotDesc* slot;
  CT_G TrailHdr* trailHdr;
  CT_G uint64_t* trailWords;
  CT_G Level* levels;
  CT_G uint64_t* levelDom;
  int64_t trailCap;
  // LDS
  uint64_t* ct;
  uint16_t* idx0;  // granule index ping-pong buffers (no array: a dynamically
  uint16_t* idx1;  // indexed member would put this struct in scratch)
  int32_t* stamp;
  uint8_t* nz;
  int32_t* first;  // per granule: its first trail entry among those undone by pops
  int32_t* res;
  uint64_t* last;
  uint64_t* din;
  uint16_t* rowList;
  int32_t* wordVar;
  VarDesc* vars;
  int32_t *vsize, *vdcnt, *segOf, *segEnd, *segInc;
  int32_t* wcnt;     // per domain word: popcount of Delta << 16 | popcount of dom_in (wide prologue)
  uint16_t* mSlot;   // filter misses: domain slot (word << 6 | bit)
  uint16_t* left;    //   misses the walk after the residue did not resolve
  uint8_t* mFound;   //   a support was found by the granule scans
  int missCap;
  TrailHdr* trRing;   // mirror of the newest trail headers (trh entries, 0: none)
  Level* lvRing;      // mirror of the newest level records (lr entries, 0: none)
  uint64_t* lvDomRing;  //   and their domains (lr x D words)
  int trh, lr;
  EngState* st;
};

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves (VALU,
// no LDS round trip): shifts by 1, 2, 4, 8 within each row of 16 lanes,
// then the last lane of row 0 / 2 added to rows 1 / 3 (row_bcast:15) and
// lane 31 added to rows 2 and 3 (row_bcast:31).  Lanes without a source
// add the `old` operand, 0.
__device__ __forceinline__ int e_wscan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// ---------------------------------------------------------------------------
// pops (all waves, every popped level at once) and pushes (wave 0; the
// trail and the levels stay in HBM)
// ---------------------------------------------------------------------------
__device__ void e_pops_pushes(Eng& E) {
  const int tid = e_tid();
  EngState* st = E.st;
  const int nPop = st->nPop, nPush = st->nPush;
  if (nPop > 0) {
    // all popped levels at once: the state of the level popped to is in
    // its Level record and domains; a granule saved on the trail after it
    // gets the words of its first entry there (the oldest save holds the
    // words of that level)
    const int dT = st->depth - nPop;
    const bool lvIn = E.lr > 0 && dT >= st->lvLo;  // level dT's record and domains are in LDS
    const int lvSlot = dT & (E.lr - 1);
    if (tid == 0) {
      const Level L = lvIn ? E.lvRing[lvSlot] : E.levels[dT];
      st->lvTrailTop = L.trailTop;
      st->lvLimit = L.limit;
      st->lvFailed = L.failed;
      st->lvSerial = L.serial;
    }
    for (int g = tid; g < E.nGran; g += EBLOCK) E.first[g] = 0x7fffffff;
    for (int q = tid; q < E.D; q += EBLOCK)
      E.last[q] = lvIn ? E.lvDomRing[(int64_t)lvSlot * E.D + q] : E.levelDom[(int64_t)dT * E.D + q];
    lds_barrier();
    const int64_t lo = st->lvTrailTop, top = st->trailTop, trLo = E.trh > 0 ? st->trLo : top;
    const int64_t trMask = E.trh - 1;
    for (int64_t e = lo + tid; e < top; e += EBLOCK)
      atomicMin(&E.first[(e >= trLo ? E.trRing[e & trMask] : E.trailHdr[e]).gran], (int)(e - lo));
    lds_barrier();
    // each granule saved since the level takes back the words of its first
    // entry: E_POP_U granules per wave per step, every load of a step issued
    // before any is used (the engine holds currTable in LDS, so a table has
    // a few hundred granules at most: one or a few steps)
    for (int g0 = e_wave() * E_POP_U; g0 < E.nGran; g0 += EWAVES * E_POP_U) {
      int f[E_POP_U];
      TrailHdr h[E_POP_U];
      uint64_t w[E_POP_U];
#pragma unroll
      for (int u = 0; u < E_POP_U; ++u) {
        f[u] = g0 + u < E.nGran ? E.first[g0 + u] : 0x7fffffff;  // the same on every lane
        if (f[u] != 0x7fffffff) {
          const int64_t e = lo + f[u];
          h[u] = e >= trLo ? E.trRing[e & trMask] : E.trailHdr[e];
          w[u] = E.trailWords[e * GW + e_lane()];
        }
      }
#pragma unroll
      for (int u = 0; u < E_POP_U; ++u) {
        if (f[u] != 0x7fffffff) {
          E.ct[(int64_t)(g0 + u) * GW + e_lane()] = w[u];
          if (e_lane() == 0) E.stamp[g0 + u] = h[u].oldStamp;
        }
      }
    }
    lds_barrier();
    if (tid == 0) {
      st->trailTop = lo;
      st->trLo = min(st->trLo, lo);
      st->limit = st->lvLimit;
      st->failed = st->lvFailed;
      st->serial = st->lvSerial;
      st->depth = dT;
      st->lvLo = min(st->lvLo, dT);
    }
    lds_barrier();
  }
  // each push records the state before this call's propagation (wave 0,
  // which also runs the prologue next: no barrier needed)
  if (tid < WAVE && nPush > 0) {
    const int lane = e_lane();
    for (int k = 0; k < nPush; ++k) {
      const int d = st->depth + k;
      const int slotL = d & (E.lr - 1);
      for (int q = lane; q < E.D; q += WAVE) {
        const uint64_t w = E.last[q];
        E.levelDom[(int64_t)d * E.D + q] = w;
        if (E.lr > 0) E.lvDomRing[(int64_t)slotL * E.D + q] = w;
      }
      if (lane == 0) {
        Level L;
        L.trailTop = st->trailTop;
        L.limit = st->limit;
        L.failed = st->failed;
        L.serial = k == 0 ? st->serial : st->serialBase + k - 1;
        L.pad = 0;
        E.levels[d] = L;
        if (E.lr > 0) E.lvRing[slotL] = L;
      }
    }
    if (lane == 0) {
      st->depth += nPush;
      st->serial = st->serialBase + nPush - 1;
      if (E.lr > 0) st->lvLo = max(st->lvLo, st->depth - E.lr);
    }
  }
}

// ---------------------------------------------------------------------------
// prologue of Alg. 1, by wave 0 with one domain word per lane (tables of at
// most 64 domain words): checks, |dom| and |Delta| per variable (prefix sums
// over the words), s_val, the branch of Alg. 2 per variable and the list of
// support rows to OR, segment by segment
// ---------------------------------------------------------------------------
__device__ void e_prologue_narrow(Eng& E) {
  const int tid = e_tid();
  EngState* st = E.st;
  if (tid < WAVE) {
    const int q = e_lane();
    const bool isWord = q < E.D;
    uint64_t din = 0, ld = 0;
    VarDesc v{};
    v.domOff = q;
    v.domWords = 1;
    v.dsize = 64;
    if (isWord) {
      din = E.din[q];
      ld = E.last[q];
      v = E.vars[E.wordVar[q]];
    }
    const int used = v.dsize - 64 * (q - v.domOff);
    const bool stray = isWord && used < 64 && (din >> used) != 0;
    const bool notSub = isWord && (din & ~ld) != 0;
    int status = st->failed ? ST_STATE : ST_OK;
    if (status == ST_OK) {
      if (__ballot(stray)) status = ST_INVALID;
      else if (__ballot(notSub)) status = ST_NOT_SUBSET;
    }
    // |dom| and |Delta| of the word's variable: prefix sums over the words
    const int first = v.domOff, lastW = v.domOff + v.domWords - 1;
    const int cs = isWord ? __popcll(din) : 0, cd = isWord ? __popcll(ld & ~din) : 0;
    const int scS = e_wscan(cs), scD = e_wscan(cd);
    const int befS = __shfl(scS, max(first - 1, 0)), befD = __shfl(scD, max(first - 1, 0));
    const int sz = __shfl(scS, lastW) - (first > 0 ? befS : 0);
    const int dc = __shfl(scD, lastW) - (first > 0 ? befD : 0);
    // decisions on each variable's first word
    const bool head = isWord && q == first;
    if (head) E.vsize[E.wordVar[q]] = sz;  // |dom(x_i)|: the filter's s_sup test
    const bool in = head && dc > 0;  // |dom| changed since the last call: in s_val
    const int policy = E.policy;
    const int inc = policy == 2 ? 1 : policy == 1 ? 0 : (dc < sz ? 1 : 0);
    const int cnt = in ? (inc ? dc : sz) : 0;
    const int scSeg = e_wscan(in ? 1 : 0), scCnt = e_wscan(cnt);
    const int nseg = __builtin_amdgcn_readlane(scSeg, WAVE - 1), nrows = __builtin_amdgcn_readlane(scCnt, WAVE - 1);
    if (in) {
      E.segEnd[scSeg - 1] = scCnt;
      E.segInc[scSeg - 1] = inc;
    }
    // rows of each word: at its variable's segment start plus the rows of
    // the variable's earlier words
    const int vIn = __shfl(in ? 1 : 0, first), vInc = __shfl(inc, first), vStart = __shfl(scCnt - cnt, first);
    const uint64_t bits = (isWord && vIn) ? (vInc ? (ld & ~din) : din) : 0ull;
    const int nb = __popcll(bits);
    const int scB = e_wscan(nb);
    const int befB = __shfl(scB, max(first - 1, 0));
    if (status == ST_OK && nseg > 0) {
      int off = vStart + (scB - nb) - (first > 0 ? befB : 0);
      const int base = v.rowStart + (q - v.domOff) * 64;
      uint64_t b = bits;
      while (b) {
        const int k = __ffsll((unsigned long long)b) - 1;
        b &= b - 1;
        E.rowList[off++] = (uint16_t)(base + k);
      }
    }
    if (q == 0) {
      st->status = status;
      st->nseg = nseg;
      st->nrows = nrows;
      st->noop = nseg == 0;
    }
  }
  lds_barrier();
}

// ---------------------------------------------------------------------------
// the same prologue for tables of more than 64 domain words: per-word checks
// and counts by every thread (LDS atomics per variable), the variables'
// decisions and segments by wave 0 (64 variables per step), then the row
// list by every thread, one domain word each
// ---------------------------------------------------------------------------
__device__ void e_prologue_wide(Eng& E) {
  EngState* st = E.st;
  const int tid = e_tid();
  for (int i = tid; i < E.n; i += EBLOCK) {
    E.vsize[i] = 0;
    E.vdcnt[i] = 0;
  }
  if (tid == 0) {
    st->badStray = 0;
    st->badSub = 0;
  }
  lds_barrier();
  int stray = 0, notSub = 0;
  for (int q = tid; q < E.D; q += EBLOCK) {
    const uint64_t din = E.din[q], ld = E.last[q];
    const int i = E.wordVar[q];
    const VarDesc v = E.vars[i];
    const int used = v.dsize - 64 * (q - v.domOff);
    if (used < 64 && (din >> used) != 0) stray = 1;
    if (din & ~ld) notSub = 1;
    const int cs = __popcll(din), cd = __popcll(ld & ~din);
    E.wcnt[q] = (cd << 16) | cs;
    atomicAdd(&E.vsize[i], cs);
    atomicAdd(&E.vdcnt[i], cd);
  }
  if (__ballot(stray) && e_lane() == 0) atomicOr(&st->badStray, 1);
  if (__ballot(notSub) && e_lane() == 0) atomicOr(&st->badSub, 1);
  lds_barrier();
  int status = st->failed ? ST_STATE : st->badStray ? ST_INVALID : st->badSub ? ST_NOT_SUBSET : ST_OK;
  if (threadIdx.x < WAVE) {
    const int lane = e_lane();
    const int policy = E.policy;
    int nseg = 0, nrows = 0;
    for (int i0 = 0; i0 < E.n; i0 += WAVE) {
      const int i = i0 + lane;
      int cnt = 0, inc = 0;
      bool in = false;
      if (i < E.n) {
        const int sz = E.vsize[i], dc = E.vdcnt[i];
        in = dc > 0;  // |dom| changed since the last call: in s_val
        inc = policy == 2 ? 1 : policy == 1 ? 0 : (dc < sz ? 1 : 0);
        cnt = in ? (inc ? dc : sz) : 0;
      }
      const int scSeg = e_wscan(in ? 1 : 0), scCnt = e_wscan(cnt);
      if (in) {
        E.segEnd[nseg + scSeg - 1] = nrows + scCnt;
        E.segInc[nseg + scSeg - 1] = inc;
      }
      if (i < E.n) E.segOf[i] = in ? ((nrows + scCnt - cnt) | (inc << 30)) : -1;
      nseg += __builtin_amdgcn_readlane(scSeg, WAVE - 1);
      nrows += __builtin_amdgcn_readlane(scCnt, WAVE - 1);
    }
    if (lane == 0) {
      st->status = status;
      st->nseg = nseg;
      st->nrows = nrows;
      st->noop = nseg == 0;
    }
  }
  lds_barrier();
  if (status == ST_OK && !st->noop) {
    for (int q = tid; q < E.D; q += EBLOCK) {
      const int i = E.wordVar[q];
      const int sg = E.segOf[i];
      if (sg < 0) continue;
      const int inc = sg >> 30;
      const VarDesc v = E.vars[i];
      int off = sg & 0x3FFFFFFF;
      for (int k = v.domOff; k < q; ++k) off += inc ? (E.wcnt[k] >> 16) : (E.wcnt[k] & 0xFFFF);
      uint64_t b = inc ? (E.last[q] & ~E.din[q]) : E.din[q];
      const int base = v.rowStart + (q - v.domOff) * 64;
      while (b) {
        const int k = __ffsll((unsigned long long)b) - 1;
        b &= b - 1;
        E.rowList[off++] = (uint16_t)(base + k);
      }
    }
  }
  lds_barrier();
}

__device__ __forceinline__ void e_prologue(Eng& E) {
  if (E.D <= WAVE) e_prologue_narrow(E);
  else e_prologue_wide(E);
}

// ---------------------------------------------------------------------------
// updateTable (Alg. 2) over the active granules: currTable in LDS, support
// rows from HBM; first changes of a level are saved on the trail.  A wave
// takes E_NG granules per step as pairs on its two half-waves: each lane
// owns two adjacent words of its half's granule and loads them with one
// 16-byte load (a half-wave reads a granule's 512 bytes; one CU moves about
// twice the bytes per second with 16-byte loads than with 8-byte ones)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void e_ld2(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, uint64_t* w) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, 0);
  w[0] = (uint64_t)v[0] | ((uint64_t)v[1] << 32);
  w[1] = (uint64_t)v[2] | ((uint64_t)v[3] << 32);
}

__device__ void e_update(Eng& E) {
  constexpr int NP = E_NG / 2;  // granule pairs per wave per step
  EngState* st = E.st;
  const int lane = e_lane();
  const int half = lane >> 5, hl = lane & 31;  // this lane: words 2hl, 2hl+1 of its half's granule
  const uint64_t halfMask = half ? 0xffffffff00000000ull : 0x00000000ffffffffull;
  const int limit = st->limit, nseg = st->nseg, nrows = st->nrows, serial = st->serial;
  const uint16_t* idxCur = st->cur ? E.idx1 : E.idx0;
  const bool trailOn = st->depthAfter > 0;  // levels exist only above depth 0
  const int64_t trailTop = st->trailTop;
  unsigned long long nAct = 0, nTrail = 0;
  for (int base = e_wave() * E_NG; base < limit; base += EWAVES * E_NG) {
    int pos[NP], gs[NP];
    bool act[NP];
    uint32_t voff[NP];
    uint64_t m[NP][2], acc[NP][2];
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      pos[s] = base + 2 * s + half;
      act[s] = pos[s] < limit;
      gs[s] = act[s] ? (int)idxCur[pos[s]] : 0;
      voff[s] = (uint32_t)gs[s] * (GW * 8) + (uint32_t)hl * 16;
      m[s][0] = m[s][1] = ~0ull;
      acc[s][0] = acc[s][1] = 0ull;
    }
    nAct += (unsigned long long)min(E_NG, limit - base);
    int seg = 0;
    int segEnd = nseg > 0 ? E.segEnd[0] : 0;
    for (int k0 = 0; k0 < nrows; k0 += E_ROWS) {
      uint64_t v[E_ROWS][NP][2];
      // the batch's row numbers, two per 32-bit LDS word, into scalar
      // registers (the same on every lane)
      uint32_t idw[(E_ROWS + 1) / 2];
      const uint32_t* lw = (const uint32_t*)(E.rowList + k0);  // k0 is even
#pragma unroll
      for (int i = 0; i < (E_ROWS + 1) / 2; ++i) idw[i] = __builtin_amdgcn_readfirstlane(lw[i]);
#pragma unroll
      for (int j = 0; j < E_ROWS; ++j) {
        const int k = k0 + j;
        const uint32_t id = (j & 1) ? (idw[j / 2] >> 16) : (idw[j / 2] & 0xFFFFu);
        const int r = k < nrows ? (int)id : 0;  // rows past the end are never used
        const uint32_t soff = (uint32_t)((int64_t)r * E.stride * 8);
#pragma unroll
        for (int s = 0; s < NP; ++s) e_ld2(E.Sbuf, voff[s], soff, v[j][s]);
      }
#pragma unroll
      for (int j = 0; j < E_ROWS; ++j) {
        const int k = k0 + j;
        if (k >= nrows) break;
        while (k >= segEnd) {
          const int inc = E.segInc[seg];
#pragma unroll
          for (int s = 0; s < NP; ++s)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              m[s][h] &= inc ? ~acc[s][h] : acc[s][h];
              acc[s][h] = 0ull;
            }
          ++seg;
          segEnd = E.segEnd[seg];
        }
#pragma unroll
        for (int s = 0; s < NP; ++s) {
          acc[s][0] |= v[j][s][0];
          acc[s][1] |= v[j][s][1];
        }
      }
    }
    while (seg < nseg) {  // remaining segments (an empty reset segment gives 0)
      const int inc = E.segInc[seg];
#pragma unroll
      for (int s = 0; s < NP; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          m[s][h] &= inc ? ~acc[s][h] : acc[s][h];
          acc[s][h] = 0ull;
        }
      ++seg;
    }
    // currTable and the stamps, read from LDS once the rows are in (fewer
    // registers live while the row loads are in flight)
    uint64_t old[NP][2], nw[NP][2];
    int stv[NP];
    bool changed[NP], need[NP];
    int myOff[NP];  // this half's granule's place among the wave's trail entries
    int nNeed = 0;
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      const int64_t wi = (int64_t)gs[s] * GW + 2 * hl;
      old[s][0] = E.ct[wi];
      old[s][1] = E.ct[wi + 1];
      stv[s] = E.stamp[gs[s]];
      nw[s][0] = old[s][0] & m[s][0];
      nw[s][1] = old[s][1] & m[s][1];
      const uint64_t bc = __ballot(act[s] && (nw[s][0] != old[s][0] || nw[s][1] != old[s][1]));
      changed[s] = (bc & halfMask) != 0ull;
      need[s] = changed[s] && trailOn && stv[s] != serial;
      const uint64_t bn = __ballot(need[s] && hl == 0);  // bits 0 and 32
      myOff[s] = nNeed + (half && (bn & 1ull) ? 1 : 0);
      nNeed += __popcll(bn);
    }
    int tb = 0;
    if (nNeed) {
      if (lane == 0) tb = atomicAdd(&st->trailCount, nNeed);
      tb = __shfl(tb, 0);
    }
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      if (need[s]) {
        const int64_t tp = trailTop + tb + myOff[s];
        if (tp < E.trailCap) {
          E.trailWords[tp * GW + 2 * hl] = old[s][0];
          E.trailWords[tp * GW + 2 * hl + 1] = old[s][1];
          if (hl == 0) {
            TrailHdr h;
            h.gran = gs[s];
            h.oldStamp = stv[s];
            E.trailHdr[tp] = h;
            if (E.trh > 0) E.trRing[tp & (E.trh - 1)] = h;
            E.stamp[gs[s]] = serial;
          }
        } else if (hl == 0) {
          st->devErr = 2;  // capacity is sized so that this cannot happen
        }
      }
      if (changed[s]) {
        const int64_t wi = (int64_t)gs[s] * GW + 2 * hl;
        E.ct[wi] = nw[s][0];
        E.ct[wi + 1] = nw[s][1];
      }
      const uint64_t bz = __ballot((nw[s][0] | nw[s][1]) != 0ull);
      if (act[s] && hl == 0) E.nz[pos[s]] = (bz & halfMask) != 0ull ? 1 : 0;
    }
    nTrail += nNeed;
  }
  if (lane == 0) {
    if (nAct) atomicAdd(&st->stat[S_GRAN_ROWS], nAct * (unsigned long long)nrows);
    if (nTrail) atomicAdd(&st->stat[S_TRAIL], nTrail);
  }
  lds_barrier();
}

// stable partition of the active granules (survivors first), new limit,
// FAIL when none survives (Alg. 1); wave 0, 64 positions per step
__device__ void e_partition(Eng& E) {
  const int tid = e_tid();
  EngState* st = E.st;
  if (tid < WAVE) {
    const int lane = e_lane();
    const int limit = st->limit, cur = st->cur, nGran = E.nGran;
    const uint16_t* src = cur ? E.idx1 : E.idx0;
    uint16_t* dst = cur ? E.idx0 : E.idx1;
    const uint64_t below = (1ull << lane) - 1ull;
    int nSurv = 0;
    for (int p0 = 0; p0 < limit; p0 += WAVE) {
      const int p = p0 + lane;
      nSurv += __popcll(__ballot(p < limit && E.nz[p]));
    }
    int sv = 0, zr = nSurv;
    for (int p0 = 0; p0 < limit; p0 += WAVE) {
      const int p = p0 + lane;
      const bool in = p < limit;
      const bool f = in && E.nz[p];
      const uint64_t bs = __ballot(f), bz = __ballot(in && !f);
      if (f) dst[sv + __popcll(bs & below)] = src[p];
      else if (in) dst[zr + __popcll(bz & below)] = src[p];
      sv += __popcll(bs);
      zr += __popcll(bz);
    }
    for (int p = limit + lane; p < nGran; p += WAVE) dst[p] = src[p];
    if (lane == 0) {
      st->cur = 1 - cur;
      st->limit = nSurv;
      st->trailTop += st->trailCount;
      st->trailCount = 0;
      if (E.trh > 0) st->trLo = max(st->trLo, st->trailTop - E.trh);
      if (nSurv == 0) {
        st->status = ST_FAIL;
        st->failed = 1;
      }
    }
  }
  lds_barrier();
}

// ---------------------------------------------------------------------------
// filterDomains (Alg. 3) of tables of at most E_NARROW_D domain words: one
// wave per domain word, all words at once, no workgroup barrier.  For word q:
// the residue first, then the words after it, then the active granules in
// index order
// ---------------------------------------------------------------------------
// The support word at a value's residue does not depend on currTable: it is
// loaded before updateTable (e_residue_word) and tested after it.
struct ResidueWord {
  int rl, rw0;
  uint64_t x;
};

__device__ __forceinline__ ResidueWord e_residue_word(const Eng& E, int q) {
  const int lane = e_lane();
  const VarDesc v = E.vars[E.wordVar[q]];
  const int rowBase = v.rowStart + (q - v.domOff) * 64;
  const bool present = (E.din[q] >> lane) & 1ull;
  ResidueWord r;
  r.rl = present ? rowBase + lane : rowBase;
  r.rw0 = E.res[r.rl];
  r.x = E.S[(int64_t)r.rl * E.stride + r.rw0];
  return r;
}

__device__ void e_filter_word(Eng& E, int q, unsigned long long* cnt, bool havePre, ResidueWord pre) {
  EngState* st = E.st;
  const int lane = e_lane();
  const int i = E.wordVar[q];
  const VarDesc v = E.vars[i];
  const uint64_t din = E.din[q];
  int size = 0;
  for (int k = v.domOff; k < v.domOff + v.domWords; ++k) size += __popcll(E.din[k]);
  uint64_t dout = din;
  if (!st->noop && size > 1) {  // s_sup: non-singleton variables
    const int64_t stride = E.stride;
    const int rowBase = v.rowStart + (q - v.domOff) * 64;
    const bool present = (din >> lane) & 1ull;
    const ResidueWord rwd = havePre ? pre : e_residue_word(E, q);
    const int rl = rwd.rl, rw0 = rwd.rw0;
    const bool hit = present && (E.ct[rw0] & rwd.x) != 0ull;
    unsigned long long miss = __ballot(present && !hit);
    cnt[0] += __popcll(__ballot(present));
    cnt[1] += __popcll(miss);
    if (miss) {
      const bool mine = (miss >> lane) & 1ull;
      const int64_t words = (int64_t)E.nGran * GW;
      bool found = false;
      const CT_G uint64_t* row = E.S + (int64_t)rl * stride;
      for (int j0 = 0; j0 < E_LANE_SCAN; j0 += 8) {
        uint64_t x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          int64_t w = rw0 + 1 + j0 + j;
          if (w >= words) w -= words;
          x[j] = row[w];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          int64_t w = rw0 + 1 + j0 + j;
          if (w >= words) w -= words;
          if (mine && !found && (E.ct[w] & x[j])) {
            found = true;
            E.res[rl] = (int)w;
          }
        }
        if (!__ballot(mine && !found)) break;
      }
      cnt[2] += __popcll(__ballot(mine));
      miss = __ballot(mine && !found);
    }
    // the values still without a support scan the active granules in index
    // order together, up to 3 values x 4 granules per step
    uint64_t todo = miss;
    const int lim = st->limit;
    const uint16_t* idx = st->cur ? E.idx1 : E.idx0;
    for (int p = 0; p < lim && todo; p += 4) {
      int gg[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) gg[j] = (p + j < lim) ? (int)idx[p + j] : -1;
      cnt[2] += (unsigned long long)min(4, lim - p) * (unsigned long long)__popcll(todo);
      uint64_t t = todo;
      while (t) {
        int ls[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          ls[u] = t ? __ffsll((unsigned long long)t) - 1 : -1;
          t &= t - 1;
        }
        uint64_t y[3][4];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          const CT_G uint64_t* row = E.S + (int64_t)(rowBase + max(ls[u], 0)) * stride;
#pragma unroll
          for (int j = 0; j < 4; ++j) y[u][j] = row[(int64_t)max(gg[j], 0) * GW + lane];
        }
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          if (ls[u] < 0) continue;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (gg[j] < 0) break;
            const unsigned long long bm = __ballot((E.ct[(int64_t)gg[j] * GW + lane] & y[u][j]) != 0ull);
            if (bm) {
              if (lane == 0) E.res[rowBase + ls[u]] = gg[j] * GW + (__ffsll(bm) - 1);
              todo &= ~(1ull << ls[u]);
              break;
            }
          }
        }
      }
    }
    dout = din & ~todo;
  }
  if (lane == 0) E.last[q] = dout;
}

// ---------------------------------------------------------------------------
// filterDomains (Alg. 3): every present value of a variable with two or more
// values (s_sup) keeps its place iff its support row meets currTable.  The
// work is flat over the domain slots (word << 6 | bit), so every wave takes
// part whatever the number of domain words:
//   A. one thread per slot tests the support word at the value's residue
//      (loaded before updateTable for the first EBLOCK slots: the residue
//      and the support rows do not change during it); misses go to a list;
//   B. one thread per miss reads the 16 words after the residue;
//   C. the misses still without a support scan the active granules, in
//      tasks of (value, 4 granules) shared by the waves;
//   values with no support found leave dom_out.
// Slots are taken in chunks of at most missCap (the miss list's size).
// ---------------------------------------------------------------------------
struct ResiduePre {
  int rw;      // the residue of the thread's first slot
  uint64_t x;  // the support word there
};

__device__ __forceinline__ int e_slot_row(const Eng& E, int slot) {
  const VarDesc v = E.vars[E.wordVar[slot >> 6]];
  return v.rowStart + ((slot >> 6) - v.domOff) * 64 + (slot & 63);
}

// the slot is a value filterDomains checks: present in dom_in, and its
// variable has two or more values
__device__ __forceinline__ bool e_checked(const Eng& E, int slot) {
  return ((E.din[slot >> 6] >> (slot & 63)) & 1ull) && E.vsize[E.wordVar[slot >> 6]] > 1;
}

// Residue word of slot `slot` (row 0 for a slot that is not checked: an
// unconditional load from a valid address).
__device__ __forceinline__ ResiduePre e_residue(const Eng& E, int slot, bool chk) {
  ResiduePre r;
  const int row = chk ? e_slot_row(E, slot) : 0;
  r.rw = E.res[row];
  r.x = E.S[(int64_t)row * E.stride + r.rw];
  return r;
}

constexpr int E_A_UNROLL = 4;  // residue loads per thread in flight (phase A)
constexpr int E_C_TASKS = 2;   // (value, 4 granules) tasks per wave step (phase C)

__device__ void e_filter(Eng& E, bool havePre, ResiduePre pre) {
  EngState* st = E.st;
  const int lane = e_lane();
  const int tid = e_tid();
  const int nSlots = E.D * 64;
  const int cap = E.missCap;
  const int64_t words = (int64_t)E.nGran * GW;
  const int lim = st->limit;
  const uint16_t* idx = st->cur ? E.idx1 : E.idx0;
  unsigned long long cChk = 0, cMiss = 0, cScan = 0;
  for (int base = 0; base < nSlots; base += cap) {
    const int end = min(nSlots, base + cap);
    if (tid == 0) {
      st->nMiss = 0;
      st->nLeft = 0;
    }
    lds_barrier();
    // A: residues
    for (int s0 = base + tid; s0 < end; s0 += EBLOCK * E_A_UNROLL) {
      bool chk[E_A_UNROLL];
      ResiduePre r[E_A_UNROLL];
      const bool usePre = havePre && s0 == tid;  // the first step of the first chunk
#pragma unroll
      for (int u = 0; u < E_A_UNROLL; ++u) {
        const int sl = s0 + u * EBLOCK;
        chk[u] = sl < end && e_checked(E, sl);
        if (u == 0 && usePre) r[u] = pre;
        else r[u] = e_residue(E, sl < end ? sl : 0, chk[u]);
      }
#pragma unroll
      for (int u = 0; u < E_A_UNROLL; ++u) {
        if (!chk[u]) continue;
        ++cChk;
        if ((E.ct[r[u].rw] & r[u].x) == 0ull) {
          const int k = atomicAdd(&st->nMiss, 1);
          E.mSlot[k] = (uint16_t)(s0 + u * EBLOCK);
          ++cMiss;
        }
      }
    }
    lds_barrier();
    // B: the 16 words after the residue, one thread per miss
    const int nMiss = st->nMiss;
    for (int k = tid; k < nMiss; k += EBLOCK) {
      const int row = e_slot_row(E, E.mSlot[k]);
      const int rw0 = E.res[row];  // the residue that missed (not changed since)
      const CT_G uint64_t* rp = E.S + (int64_t)row * E.stride;
      int found = -1;
      for (int j0 = 0; j0 < E_LANE_SCAN && found < 0; j0 += 8) {
        uint64_t x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          int w = rw0 + 1 + j0 + j;
          if (w >= words) w -= (int)words;
          x[j] = rp[w];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          int w = rw0 + 1 + j0 + j;
          if (w >= words) w -= (int)words;
          if (found < 0 && (E.ct[w] & x[j])) found = w;
        }
      }
      ++cScan;
      if (found >= 0) {
        E.res[row] = found;
      } else {
        const int j = atomicAdd(&st->nLeft, 1);
        E.left[j] = (uint16_t)k;
        E.mFound[j] = 0;
      }
    }
    lds_barrier();
    // C: the active granules, in index order per value; task t is value
    // t % nLeft, granules 4 (t / nLeft) .. +3, so every value's first
    // granules come first and a value found there skips the rest
    const int nLeft = st->nLeft;
    const int chunks = (lim + 3) / 4;
    const int nTasks = nLeft * chunks;
    for (int t0 = e_wave() * E_C_TASKS; t0 < nTasks; t0 += EWAVES * E_C_TASKS) {
      int jv[E_C_TASKS], row[E_C_TASKS], g[E_C_TASKS][4];
      bool live[E_C_TASKS];
      uint64_t y[E_C_TASKS][4];
#pragma unroll
      for (int u = 0; u < E_C_TASKS; ++u) {
        const int t = t0 + u;
        live[u] = t < nTasks;
        jv[u] = live[u] ? t % nLeft : 0;
        const int c = live[u] ? t / nLeft : 0;
        live[u] = live[u] && !E.mFound[jv[u]];
        // the same on every lane: scalar registers
        row[u] = __builtin_amdgcn_readfirstlane(live[u] ? e_slot_row(E, E.mSlot[E.left[jv[u]]]) : 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int p = 4 * c + q;
          g[u][q] = __builtin_amdgcn_readfirstlane((live[u] && p < lim) ? (int)idx[p] : -1);
          y[u][q] = E.S[(int64_t)row[u] * E.stride + (int64_t)max(g[u][q], 0) * GW + lane];
        }
      }
#pragma unroll
      for (int u = 0; u < E_C_TASKS; ++u) {
        if (!live[u]) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (g[u][q] < 0) break;
          cScan += lane == 0 ? 1 : 0;  // a wave's work, counted once
          const unsigned long long bm =
              __ballot((E.ct[(int64_t)g[u][q] * GW + lane] & y[u][q]) != 0ull);
          if (bm) {
            if (lane == 0) {
              E.mFound[jv[u]] = 1;
              E.res[row[u]] = g[u][q] * GW + (__ffsll(bm) - 1);
            }
            break;
          }
        }
      }
    }
    lds_barrier();
    // values with no support leave the domain
    for (int j = tid; j < nLeft; j += EBLOCK) {
      if (!E.mFound[j]) {
        const int sl = E.mSlot[E.left[j]];
        atomicAnd((unsigned long long*)&E.last[sl >> 6], ~(1ull << (sl & 63)));
      }
    }
    lds_barrier();
  }
  // the counters: summed over the wave first (every lane is active here)
  const int sChk = __builtin_amdgcn_readlane(e_wscan((int)cChk), WAVE - 1);
  const int sMiss = __builtin_amdgcn_readlane(e_wscan((int)cMiss), WAVE - 1);
  const int sScan = __builtin_amdgcn_readlane(e_wscan((int)cScan), WAVE - 1);
  if (lane == 0 && (sChk | sMiss | sScan)) {
    atomicAdd(&st->stat[S_RES_CHECK], (unsigned long long)sChk);
    atomicAdd(&st->stat[S_RES_MISS], (unsigned long long)sMiss);
    atomicAdd(&st->stat[S_SCAN], (unsigned long long)sScan);
  }
}

__device__ void e_load(Eng& E, const EngDesc& D) {
  const CT_G SlotDesc* s = E.slot;
  EngState* st = E.st;
  const int cur = s->cur;
  const CT_G uint64_t* ct = s->ct;
  const CT_G int32_t* idx = s->idx[cur];
  for (int64_t i = threadIdx.x; i < (int64_t)E.nGran * GW; i += EBLOCK) E.ct[i] = ct[i];
  for (int p = threadIdx.x; p < E.nGran; p += EBLOCK) {
    E.idx0[p] = (uint16_t)idx[p];
    E.stamp[p] = s->stamp[p];
  }
  for (int r = threadIdx.x; r < E.rows; r += EBLOCK) E.res[r] = s->res[r];
  for (int q = threadIdx.x; q < E.D; q += EBLOCK) {
    E.last[q] = s->lastDom[q];
    E.wordVar[q] = D.tab->wordVar[q];
  }
  for (int i = threadIdx.x; i < E.n; i += EBLOCK) E.vars[i] = D.tab->vars[i];
  if (threadIdx.x == 0) {
    st->lastSeq = D.startSeq;
    st->limit = s->limit;
    st->failed = s->failed;
    st->depth = s->depth;
    st->serial = s->serial;
    st->trailTop = s->trailTop;
    st->trLo = s->trailTop;  // the rings start empty
    st->lvLo = s->depth;
    st->cur = 0;
    st->trailCount = 0;
    st->devErr = 0;
  }
  if (threadIdx.x < 8) st->stat[threadIdx.x] = s->stats[threadIdx.x];
  __syncthreads();
}

__device__ void e_store(Eng& E) {
  CT_G SlotDesc* s = E.slot;
  EngState* st = E.st;
  CT_G uint64_t* ct = s->ct;
  CT_G int32_t* idx = s->idx[0];
  for (int64_t i = threadIdx.x; i < (int64_t)E.nGran * GW; i += EBLOCK) ct[i] = E.ct[i];
  for (int p = threadIdx.x; p < E.nGran; p += EBLOCK) {
    idx[p] = (st->cur ? E.idx1 : E.idx0)[p];
    s->stamp[p] = E.stamp[p];
  }
  for (int r = threadIdx.x; r < E.rows; r += EBLOCK) s->res[r] = E.res[r];
  for (int q = threadIdx.x; q < E.D; q += EBLOCK) s->lastDom[q] = E.last[q];
  if (threadIdx.x < 8) s->stats[threadIdx.x] = st->stat[threadIdx.x];
  if (threadIdx.x == 0) {
    s->cur = 0;
    s->limit = st->limit;
    s->failed = st->failed;
    s->depth = st->depth;
    s->serial = st->serial;
    s->trailTop = st->trailTop;
  }
  __threadfence();
  __syncthreads();
}

}  // namespace

__global__ void __launch_bounds__(EBLOCK) engine_kernel(EngDesc D) {
  extern __shared__ uint64_t ldsWords[];
  char* lds = (char*)ldsWords;
  const CT_G TabDesc* T = D.tab;
  Eng E;
  E.S = T->S;
  E.Sbuf = __builtin_amdgcn_make_buffer_rsrc((void*)T->S, (short)0,
                                             (int)min((int64_t)T->rows * T->stride * 8, (int64_t)0x7fffffff),
                                             BUF_DWORD3);
  E.stride = T->stride;
  E.W = T->W;
  E.n = T->n;
  E.D = T->D;
  E.nGran = T->nGran;
  E.rows = T->rows;
  E.policy = T->policy;
  E.slot = D.slot;
  E.trailHdr = D.slot->trailHdr;
  E.trailWords = D.slot->trailWords;
  E.levels = D.slot->levels;
  E.levelDom = D.slot->levelDom;
  E.trailCap = D.slot->trailCap;
  size_t off[R_END + 1];
  int mirror[2];
  eng_layout(E.n, E.D, E.nGran, E.rows, off, mirror);
  E.trh = mirror[0];
  E.lr = mirror[1];
  E.trRing = (TrailHdr*)(lds + off[R_TRH]);
  E.lvRing = (Level*)(lds + off[R_LVR]);
  E.lvDomRing = (uint64_t*)(lds + off[R_LVD]);
  E.ct = (uint64_t*)(lds + off[R_CT]);
  E.idx0 = (uint16_t*)(lds + off[R_IDX0]);
  E.idx1 = (uint16_t*)(lds + off[R_IDX1]);
  E.stamp = (int32_t*)(lds + off[R_STAMP]);
  E.nz = (uint8_t*)(lds + off[R_NZ]);
  E.first = (int32_t*)(lds + off[R_FIRST]);
  E.res = (int32_t*)(lds + off[R_RES]);
  E.last = (uint64_t*)(lds + off[R_LAST]);
  E.din = (uint64_t*)(lds + off[R_DIN]);
  E.rowList = (uint16_t*)(lds + off[R_ROWS]);
  E.wordVar = (int32_t*)(lds + off[R_WVAR]);
  E.vars = (VarDesc*)(lds + off[R_VARS]);
  E.vsize = (int32_t*)(lds + off[R_VSIZE]);
  E.vdcnt = (int32_t*)(lds + off[R_VDCNT]);
  E.segOf = (int32_t*)(lds + off[R_SEGOF]);
  E.segEnd = (int32_t*)(lds + off[R_SEGEND]);
  E.segInc = (int32_t*)(lds + off[R_SEGINC]);
  E.wcnt = (int32_t*)(lds + off[R_WCNT]);
  E.mSlot = (uint16_t*)(lds + off[R_MSLOT]);
  E.left = (uint16_t*)(lds + off[R_LEFT]);
  E.mFound = (uint8_t*)(lds + off[R_MFOUND]);
  E.missCap = eng_miss_cap(E.D);
  E.st = (EngState*)(lds + off[R_STATE]);
  EngState* st = E.st;
  EngCmd* cmd = D.cmd;
  EngRes* res = D.res;

  const unsigned long long tLife = wall_clock64();
  e_load(E, D);
  for (;;) {
    // wave 0 waits for a call (bounded: an idle engine exits): it polls the
    // command's first 64 slots with two wave-wide loads in flight and takes
    // the call once every slot carries the next sequence number; the rest
    // of a long command follows the same way
    if (threadIdx.x < WAVE) {
      const int l = e_tid();
      const uint32_t want = (uint32_t)(st->lastSeq + 1);
      const int nS = EC_DOM + 2 * E.D;
      const uint64_t* slots = cmd->slot;
      const unsigned long long t0 = wall_clock64();
      bool seen = false;
      uint64_t v = 0;
      {
        // every lane loads (lanes past the command re-read its last slot and
        // count as holding the number): loads under a branch would each be
        // waited for before the test, one poll in flight at a time
        const uint64_t* mine = slots + min(l, nS - 1);
#define E_POLL_LD ll_load(mine)
#define E_POLL_TEST(x)                                              \
  if (__all(l >= nS || (uint32_t)(x) == want)) {                    \
    v = (x);                                                        \
    seen = true;                                                    \
    break;                                                          \
  }                                                                 \
  if ((long long)(wall_clock64() - t0) > D.idleTicks) break;
        uint64_t p0 = E_POLL_LD;
        for (;;) {
          const uint64_t p1 = E_POLL_LD;
          E_POLL_TEST(p0)
          p0 = E_POLL_LD;
          E_POLL_TEST(p1)
        }
#undef E_POLL_TEST
#undef E_POLL_LD
      }
      uint32_t* din32 = (uint32_t*)E.din;
      if (seen) {
        if (l >= EC_DOM && l < nS) din32[l - EC_DOM] = (uint32_t)(v >> 32);
        // the rest, E_CMD_U chunks of 64 slots per round trip
        for (int c0 = WAVE; c0 < nS && seen; c0 += E_CMD_U * WAVE) {
          for (;;) {
            uint64_t w[E_CMD_U];
            bool ok = true;
#pragma unroll
            for (int u = 0; u < E_CMD_U; ++u) {  // unconditional loads, as above
              const int i = c0 + u * WAVE + l;
              w[u] = ll_load(slots + min(i, nS - 1));
            }
#pragma unroll
            for (int u = 0; u < E_CMD_U; ++u) ok = ok && (c0 + u * WAVE + l >= nS || (uint32_t)w[u] == want);
            if (__all(ok)) {
#pragma unroll
              for (int u = 0; u < E_CMD_U; ++u) {
                const int i = c0 + u * WAVE + l;
                if (i < nS) din32[i - EC_DOM] = (uint32_t)(w[u] >> 32);
              }
              break;
            }
            if ((long long)(wall_clock64() - t0) > D.idleTicks) {
              seen = false;
              break;
            }
          }
        }
      }
      if (l == 0) {
        const uint32_t hv = (uint32_t)(v >> 32);
        st->op = seen ? (int32_t)hv : 0;
        st->seq = (int32_t)want;
      }
      const int32_t h1 = __shfl((int32_t)(v >> 32), EC_NPOP), h2 = __shfl((int32_t)(v >> 32), EC_NPUSH);
      const int32_t h3 = __shfl((int32_t)(v >> 32), EC_SERIAL), h4 = __shfl((int32_t)(v >> 32), EC_DEPTH);
      const int32_t h5 = __shfl((int32_t)(v >> 32), EC_WANTCT), h6 = __shfl((int32_t)(v >> 32), EC_WANTST);
      if (l == 0) {
        st->nPop = h1;
        st->nPush = h2;
        st->serialBase = h3;
        st->depthAfter = h4;
        st->wantCt = h5;
        st->wantStats = h6;
      }
    }
    lds_barrier();
    if (st->op != ENG_OP_PROPAGATE) break;
    const unsigned long long tStart = wall_clock64();

    e_pops_pushes(E);
    e_prologue(E);
    // residue words in flight during the update: this wave's domain word
    // (narrow tables) or this thread's first value slot (wide tables)
    const bool narrow = E.D <= E_NARROW_D;
    ResidueWord preW{0, 0, 0ull};
    ResiduePre pre{0, 0ull};
    const bool havePre = st->status == ST_OK && !st->noop;
    if (havePre) {
      if (narrow) {
        if (e_wave() < E.D) preW = e_residue_word(E, e_wave());
      } else {
        const int tid = e_tid();
        const int sl = tid < E.D * 64 ? tid : 0;
        pre = e_residue(E, sl, tid < E.D * 64 && e_checked(E, sl));
      }
    }
    if (st->status == ST_OK && !st->noop) {
      const int limitIn = st->limit;
      e_update(E);
      e_partition(E);
      if (threadIdx.x == 0) {
        atomicAdd(&st->stat[S_JOBS], 1ull);
        atomicAdd(&st->stat[S_GRAN_IN], (unsigned long long)limitIn);
        atomicAdd(&st->stat[S_ROWS], (unsigned long long)st->nrows);
      }
    } else if (st->status == ST_OK && threadIdx.x == 0) {
      atomicAdd(&st->stat[S_JOBS], 1ull);
      atomicAdd(&st->stat[S_GRAN_IN], (unsigned long long)st->limit);
    }
    lds_barrier();
    if (st->status == ST_OK && narrow) {
      unsigned long long cnt[3] = {0, 0, 0};
      for (int q = e_wave(); q < E.D; q += EWAVES)
        e_filter_word(E, q, cnt, havePre && q == e_wave(), preW);
      if (e_lane() == 0 && (cnt[0] | cnt[1] | cnt[2])) {
        atomicAdd(&st->stat[S_RES_CHECK], cnt[0]);
        atomicAdd(&st->stat[S_RES_MISS], cnt[1]);
        atomicAdd(&st->stat[S_SCAN], cnt[2]);
      }
    } else if (st->status == ST_OK) {
      // dom_out starts as dom_in; the filter clears the values it removes
      for (int q = e_tid(); q < E.D; q += EBLOCK) E.last[q] = E.din[q];
      if (!st->noop) {
        lds_barrier();
        e_filter(E, havePre, pre);
      }
    }
    lds_barrier();
    // wave 0 writes the outputs to host memory: flagged result slots (the
    // domains and counters first, the status last; the host waits for
    // every slot it reads), and currTable before them behind a system-scope
    // release, for the calls that want it
    if (threadIdx.x < WAVE) {
      const int l = e_tid();
      const uint32_t sq = (uint32_t)st->seq;
      const int status = st->devErr ? ST_DEVICE : st->status;
      uint64_t* rs = res->slot;
      if (status == ST_OK && st->wantCt) {
        for (int64_t w = l; w < E.W; w += WAVE) D.ctOut[w] = E.ct[w];
        __threadfence_system();
      }
      if (status == ST_OK) {
        const uint32_t* out32 = (const uint32_t*)E.last;
        for (int i = l; i < 2 * E.D; i += WAVE) ll_store(rs + ER_DOM + i, eng_slot(out32[i], sq));
      }
      if (st->wantStats && l < 16) {
        const unsigned long long c = st->stat[l >> 1];
        ll_store(rs + ER_STATS + l, eng_slot((uint32_t)(l & 1 ? c >> 32 : c), sq));
      }
      if (l == 0) {
        const unsigned long long ticks = wall_clock64() - tStart;
        ll_store(rs + ER_TICKS, eng_slot((uint32_t)min(ticks, 0xffffffffull), sq));
        ll_store(rs + ER_STATUS, eng_slot((uint32_t)status, sq));
        st->lastSeq = st->seq;
      }
    }
    __syncthreads();
  }
  e_store(E);
  if (threadIdx.x == 0) {
    res->exitSeq = st->lastSeq;
    res->lifeTicks = wall_clock64() - tLife;
    __threadfence_system();
    __hip_atomic_store(&res->alive, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
size_t engine_lds_bytes(int n, int D, int nGran, int rows) {
  size_t off[R_END + 1];
  eng_layout(n, D, nGran, rows, off);
  return off[R_END];
}

hipError_t launch_engine(const EngDesc& D, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL(engine_kernel, dim3(1), dim3(EBLOCK), lds, stream, D);
  return hipGetLastError();
}

}  // namespace ctk
