// ct_runtime.cpp -- host runtime and C ABI of the CT library (include/ct.h).
//
// Owns device memory, streams and the host-side mirror of each slot's depth.
// Every step of propagation runs in the HIP kernels of ct_kernels.hip; the
// host only validates arguments, lays out job descriptors and moves the
// domain bitmaps across the boundary.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "ct.h"
#include "ct_device.h"

using namespace ctk;

namespace ctk {
int propagate_items_per_job_update(int nGran, int tile);
int propagate_items_per_job_filter(int D);
int propagate_max_grid();
hipError_t launch_propagate(const KArgs& a, int grid, hipStream_t stream);
size_t engine_lds_bytes(int n, int D, int nGran, int rows);
hipError_t launch_engine(const EngDesc& D, size_t lds, hipStream_t stream);
hipError_t launch_split_engine(const EngDesc& E, int grid, hipStream_t stream);
int nodes_max_rows();
int nodes_list_cap(int rows, int n);
int nodes_node_words(int rows, int n);
size_t nodes_update_lds(int rows, int n, int groupSize, int tw);
hipError_t launch_nodes(const KArgs& a, const NodesDesc& N, int n, hipStream_t stream);
hipError_t launch_roots(const KArgs& a, const RootDesc& R, hipStream_t stream);
hipError_t noalloc_scratch(char** ptr, size_t* bytes);
hipError_t launch_noalloc_reset(int32_t* q, hipStream_t stream);
hipError_t launch_build_supports(const int32_t* tuples, int64_t t, int n, const VarDesc* vars,
                                 const int32_t* lo, uint64_t* S, int64_t stride, int64_t W,
                                 hipStream_t stream);
hipError_t launch_init_slots(const TabDesc* T, SlotDesc* slots, int n, const int32_t* rootRes,
                             hipStream_t stream);
}  // namespace ctk

namespace {

// the calling thread's last error message, in a fixed buffer: reporting an
// error allocates nothing
thread_local char g_err[512];

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(CT_E_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                  __FILE__, __LINE__);                                                      \
  } while (0)

constexpr int32_t kStatusPending = 0x7fff0001;

// device-side errors of ct_propagate_batch_noalloc calls on `stream`
int noalloc_status(hipStream_t stream);

// Injected allocation failure (a test hook): the g_failAlloc-th allocation
// from now fails.
std::atomic<int32_t> g_failAlloc{0};

bool alloc_injected() {
  int32_t n = g_failAlloc.load();
  while (n > 0)
    if (g_failAlloc.compare_exchange_weak(n, n - 1)) return n == 1;
  return false;
}

// A device or pinned host allocation: CT_E_NOMEM when it fails (or when
// the injected failure fires on it).
#define ALLOCCHK(expr)                                                                      \
  do {                                                                                      \
    if (alloc_injected()) return fail(CT_E_NOMEM, "injected allocation failure: %s", #expr); \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      (void)hipGetLastError();                                                              \
      return fail(CT_E_NOMEM, "%s failed: %s", #expr, hipGetErrorString(e_));              \
    }                                                                                       \
  } while (0)

// failed flag as known on the host: 0 no, 1 yes, 2 unknown (after batches)
struct SlotHost {
  SlotDesc* dev = nullptr;
  int maxDepth = 0;
  int capDepth = 0;        // levels the slot's device trail was sized for
  bool freed = false;      // released by ct_slots_free (reused by ct_slots_alloc)
  int depth = 0;           // depth including pending operations
  int pendPop = 0, pendPush = 0;
  int8_t failed = 0;
  std::vector<int8_t> failedAt;  // failed flag recorded by each push
  uint64_t batchMark = 0;        // last batch that named this slot
};

struct DevBlock {
  void* ptr = nullptr;
};

// Device queue + staging for one stream.
struct QueueCtx {
  int32_t* queue = nullptr;   // 4 ints on the device
  int32_t* hostErr = nullptr; // pinned
  // batch staging: job descriptors, then (256-byte aligned) updOff | filtOff
  // | prepList | root tasks, sent in one copy; two pinned buffers in turn let
  // the host fill one while the other's copy is still queued
  char* dStage = nullptr;
  char* pStage[2] = {nullptr, nullptr};
  hipEvent_t staged[2] = {nullptr, nullptr};
  size_t capStage = 0;
  int turn = 0;
  // host scratch of a batch, kept between batches (no allocation per call)
  std::vector<DevJob> hJobs;
  std::vector<int32_t> updOff, filtOff, prep, rootTasks;
  std::vector<std::array<int32_t, 3>> rootKey;
  // search-node schedule scratch (node records | granule flags)
  void* dNodes = nullptr;
  size_t capNodes = 0;
};

int queue_init(QueueCtx& q) {
  ALLOCCHK(hipMalloc(&q.queue, 4 * sizeof(int32_t)));
  HIPCHK(hipMemset(q.queue, 0, 4 * sizeof(int32_t)));
  ALLOCCHK(hipHostMalloc((void**)&q.hostErr, sizeof(int32_t), hipHostMallocMapped | hipHostMallocCoherent));
  *q.hostErr = 0;
  for (int k = 0; k < 2; ++k) HIPCHK(hipEventCreateWithFlags(&q.staged[k], hipEventDisableTiming));
  return CT_OK;
}

void queue_free(QueueCtx& q) {
  if (q.queue) (void)hipFree(q.queue);
  if (q.hostErr) (void)hipHostFree(q.hostErr);
  if (q.dStage) (void)hipFree(q.dStage);
  for (int k = 0; k < 2; ++k) {
    if (q.pStage[k]) (void)hipHostFree(q.pStage[k]);
    if (q.staged[k]) (void)hipEventDestroy(q.staged[k]);
  }
  if (q.dNodes) (void)hipFree(q.dNodes);
  q = QueueCtx();
}

std::mutex g_qmu;
std::map<hipStream_t, QueueCtx*> g_queues;

}  // namespace

struct ct_table {
  // the fields every call reads first, together (a batch of thousands of
  // jobs touches them for every table)
  int n = 0;
  int64_t t = 0, W = 0, stride = 0;
  int rows = 0, D = 0, nGran = 0;
  ct_config cfg{};
  TabDesc* dTab = nullptr;
  std::vector<SlotHost> slots;
  int32_t serialCounter = 1;
  bool poisoned = false;
  bool tailPending = false;  // a synchronous call returned before its kernel ended
  bool engEligible = false, engOn = false;
  int kind = CT_KIND_POSITIVE;  // CT_KIND_POSITIVE or CT_KIND_NEGATIVE
  bool shortTab = false;        // a positive table with star cells
  int rootFailed = 0;
  hipStream_t stream = nullptr;
  uint64_t batchMark = 0;    // last batch that named this table
  hipStream_t pendStream = nullptr;  // a model's stream holding queued work on slot 0
  std::vector<int32_t> lo, dsz, domOff;
  std::vector<VarDesc> vars;
  std::vector<int32_t> wordVar;
  // device
  uint64_t* dS = nullptr;
  VarDesc* dVars = nullptr;
  int32_t* dWordVar = nullptr;
  WordDesc* dWords = nullptr;
  int32_t* dLo = nullptr;
  TabDesc hTab{};
  SlotDesc* dRoot = nullptr;
  SlotDesc hRoot{};
  std::vector<void*> blocks;  // device allocations to free
  QueueCtx q;
  // pinned staging of the synchronous calls
  uint64_t* pDomOut = nullptr;  // D words
  uint64_t* pLL = nullptr;      // result slots of flagged synchronous jobs (2 + 2D)
  uint64_t* pDomIn = nullptr;   // D words (used when D > INLINE_WORDS)
  uint64_t* pCt = nullptr;      // W words (lazily)
  int32_t* pStatus = nullptr;
  // optional kernel timing of synchronous launches, on the device clock
  // (no host events: they would add dispatch packets to every call)
  unsigned long long* dClock = nullptr;  // 5 words, see KArgs::clock
  bool timing = false;
  // resident engine of slot 0 (see ct_engine.hip; engEligible, engOn above)
  size_t engLds = 0;
  hipStream_t engStream = nullptr;
  EngCmd* pCmd = nullptr;   // coherent pinned mailbox
  EngRes* pRes = nullptr;
  int32_t engSeq = 0;  // call numbers of the mailbox and of flagged launched calls (one sequence)
  bool engSplit = false;    // the running engine is the resident split schedule
  int32_t* dCtl = nullptr;  // its control words (SE_CTL_WORDS)
  int seVarWords = -1;      // largest domain words of one variable (computed once)
  std::vector<uint64_t> engDom;        // the last call's output domains (D words)
  unsigned long long engStats[8] = {};  // the slot's counters after the last call
  bool engStatsFresh = false;  // engStats is from the last call
  unsigned long long engTicks = 0, engCalls = 0;  // timing of engine calls
  // lifetimes of the engine launches started while timing was on
  bool engTimed = false;
  unsigned long long engLifeTicks = 0, engLaunches = 0;
};

namespace {

int dev_alloc(ct_table* T, void** p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (alloc_injected()) return fail(CT_E_NOMEM, "injected allocation failure: hipMalloc(%zu)", bytes);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(CT_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  T->blocks.push_back(*p);
  return CT_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Allocate n slot descriptors and their arrays in one device block.
int alloc_slots(ct_table* T, int n, int maxDepth, SlotDesc** dSlots, std::vector<SlotDesc>& h) {
  const size_t ctB = align256(sizeof(uint64_t) * T->stride);
  const size_t idxB = align256(sizeof(int32_t) * T->nGran);
  const size_t domB = align256(sizeof(uint64_t) * T->D);
  const size_t resB = align256(sizeof(int32_t) * T->rows);
  const int64_t trailCap = (int64_t)maxDepth * T->nGran;
  const size_t thB = align256(sizeof(TrailHdr) * std::max<int64_t>(trailCap, 1));
  const size_t twB = align256(sizeof(uint64_t) * GW * std::max<int64_t>(trailCap, 1));
  const size_t lvB = align256(sizeof(Level) * std::max(maxDepth, 1));
  const size_t ldB = align256(sizeof(uint64_t) * T->D * std::max(maxDepth, 1));
  const size_t per = ctB + 4 * idxB + domB + resB + thB + twB + lvB + ldB;
  const size_t descB = align256(sizeof(SlotDesc) * n);
  char* base = nullptr;
  int rc = dev_alloc(T, (void**)&base, descB + per * (size_t)n);
  if (rc != CT_OK) return rc;
  *dSlots = (SlotDesc*)base;
  h.assign(n, SlotDesc{});
  char* p = base + descB;
  for (int k = 0; k < n; ++k) {
    SlotDesc& s = h[k];
    s.ct = (uint64_t*)p; p += ctB;
    s.idx[0] = (int32_t*)p; p += idxB;
    s.idx[1] = (int32_t*)p; p += idxB;
    s.stamp = (int32_t*)p; p += idxB;
    s.nzFlag = (int32_t*)p; p += idxB;
    s.lastDom = (uint64_t*)p; p += domB;
    s.res = (int32_t*)p; p += resB;
    s.trailHdr = (TrailHdr*)p; p += thB;
    s.trailWords = (uint64_t*)p; p += twB;
    s.levels = (Level*)p; p += lvB;
    s.levelDom = (uint64_t*)p; p += ldB;
    s.trailCap = trailCap;
    s.maxDepth = maxDepth;
  }
  HIPCHK(hipMemcpy(base, h.data(), sizeof(SlotDesc) * n, hipMemcpyHostToDevice));
  return CT_OK;
}

int check_poison(const ct_table* T) {
  if (!T) return fail(CT_E_INVALID, "null table");
  if (T->poisoned) return fail(CT_E_DEVICE, "table handle poisoned by an earlier device error");
  return CT_OK;
}

constexpr int SOLO_MAX_GRAN = 4;      // tables up to 16,384 tuples run solo ...
constexpr int SOLO_MAX_D = 16;        // ... unless filterDomains has more words than 4 waves take at once
constexpr int SOLO_MIN_BATCH = 256;   // batches this large run every job solo

constexpr int NODES_MIN_BATCH = 64;   // AUTO: batches of root resets this large run granule-major
constexpr int SCRATCH_SOLO_MAX_GRAN = 16;  // AUTO: roots recomputed solo up to 65,536 tuples

bool use_solo(const ct_table* T, int nJobs) {
  // a negative table's call filters and then removes the pruned values'
  // tuples, in one workgroup
  if (T->kind == CT_KIND_NEGATIVE || T->cfg.schedule == CT_SCHED_SOLO) return true;
  if (T->cfg.schedule == CT_SCHED_SPLIT) return false;
  return (T->nGran <= SOLO_MAX_GRAN && T->D <= SOLO_MAX_D) || nJobs >= SOLO_MIN_BATCH;
}

// The search-node schedule takes a batch whose jobs all reset slots of one
// table to the root and propagate (the slots are distinct: checked before).
// Largest LDS of one workgroup on the current device (0 if unknown).
int device_lds() {
  int dev = 0, lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 0;
  return lds;
}

// Tile of the node update kernel: nodes per group (a multiple of 8 up to 64)
// and granules per tile.  Two-granule tiles (16-byte LDS reads) when the tile
// and a group of at least 32 nodes fit one workgroup's LDS; else one-granule
// tiles with the largest group for which two workgroups fit a CU, else one.
struct NodesPlan {
  int groupSize = 0, tw = 1;
};

NodesPlan nodes_plan(const ct_table* T) {
  const size_t lds = (size_t)device_lds();
  NodesPlan p;
  for (int gs = 64; gs >= 32; gs -= 8)
    if (nodes_update_lds(T->rows, T->n, gs, 2) <= lds) {
      p.groupSize = gs;
      p.tw = 2;
      return p;
    }
  for (int per = 2; per >= 1; --per)
    for (int gs = 64; gs >= 8; gs -= 8)
      if (per * nodes_update_lds(T->rows, T->n, gs, 1) <= lds) {
        p.groupSize = gs;
        return p;
      }
  return p;
}

// Batches of roots recomputed from scratch run on their own streaming
// kernels when every job is a ROOT job of a table on the AUTO schedule.
bool use_roots(const ct_job* jobs, int n) {
  for (int j = 0; j < n; ++j)
    if (jobs[j].flags != (CT_JOB_PROPAGATE | CT_JOB_ROOT) || jobs[j].table->cfg.schedule != CT_SCHED_AUTO ||
        jobs[j].table->kind != CT_KIND_POSITIVE)
      return false;
  return true;
}

bool use_nodes(const ct_job* jobs, int n) {
  const ct_table* T = jobs[0].table;
  if (T->cfg.schedule != CT_SCHED_NODES && (T->cfg.schedule != CT_SCHED_AUTO || n < NODES_MIN_BATCH))
    return false;
  if (T->kind != CT_KIND_POSITIVE) return false;
  if (T->rows > nodes_max_rows() || T->nGran > MAX_GRAN) return false;
  // the update kernel's LDS holds one granule of every support row
  if (nodes_plan(T).groupSize == 0) return false;
  for (int j = 0; j < n; ++j)
    if (jobs[j].table != T || jobs[j].flags != (CT_JOB_PROPAGATE | CT_JOB_FROM_ROOT)) return false;
  return true;
}

// Fill item counts of a job: solo = one update item that does everything.
void job_counts(const ct_table* T, DevJob& J) {
  if (!(J.flags & JF_PROPAGATE)) {
    J.nUpd = 0;
    J.nFilt = 0;
  } else if (J.flags & JF_SOLO) {
    J.nUpd = 1;
    J.nFilt = 0;
  } else {
    J.nUpd = propagate_items_per_job_update(T->nGran, J.tile);
    J.nFilt = propagate_items_per_job_filter(T->D);
  }
}

bool needs_prep(const DevJob& J) {
  if (!(J.flags & JF_PROPAGATE)) return true;
  return !(J.flags & JF_SOLO) && J.nPop > 0;
}

// Run one job synchronously on the table's stream.
int quiesce(ct_table* T, hipStream_t same = nullptr);

uint64_t* pinned_dev64(ct_table* T, uint64_t* host);

int run_single(ct_table* T, DevJob& J, const uint64_t* dom_in_host) {
  int qrc = quiesce(T);
  if (qrc) return qrc;
  KArgs a{};
  a.jobs = nullptr;
  a.nJobs = 1;
  if ((J.flags & JF_PROPAGATE) && use_solo(T, 1)) J.flags |= JF_SOLO;
  job_counts(T, J);
  a.nPrep = needs_prep(J) ? 1 : 0;
  J.flags |= JF_HOST_OUT;
  // a split propagation answers through flagged slots (no currTable copy:
  // that one keeps the fenced, counted status)
  const bool ll = (J.flags & JF_PROPAGATE) && !(J.flags & JF_SOLO) && !J.ct_out && T->pLL;
  uint32_t sq = 0;
  if (ll) {
    J.flags |= JF_LL;
    J.seq = ++T->engSeq;
    if (J.seq == 0) J.seq = ++T->engSeq;  // (0 is the slots' initial flag)
    sq = (uint32_t)J.seq;
    if (!(J.ll = pinned_dev64(T, T->pLL))) return fail(CT_E_DEVICE, "no device address for the result slots");
  }
  a.nUpd = J.nUpd;
  a.nFilt = J.nFilt;
  a.queue = T->q.queue;
  a.hostErr = T->q.hostErr;
  if (dom_in_host) {
    if (T->D <= INLINE_WORDS) {
      memcpy(a.inl, dom_in_host, sizeof(uint64_t) * T->D);
      J.flags |= JF_INLINE_DOM;
    } else {
      memcpy(T->pDomIn, dom_in_host, sizeof(uint64_t) * T->D);
      uint64_t* dp = nullptr;
      HIPCHK(hipHostGetDevicePointer((void**)&dp, T->pDomIn, 0));
      J.dom_in = dp;
    }
  }
  a.job = J;
  const int total = a.nPrep + a.nUpd + a.nFilt;
  if (total == 0) return CT_OK;
  volatile int32_t* status = T->pStatus;
  *status = kStatusPending;
  a.clock = T->timing ? T->dClock : nullptr;
  HIPCHK(launch_propagate(a, std::min(total, propagate_max_grid()), T->stream));
  T->tailPending = true;
  if (ll) {
    // the status slot (a job that does not succeed) or every domain word
    const uint64_t* sl = T->pLL;
    const int nS = 2 * T->D;
    int got = 0;
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t spin = 0;; ++spin) {
      const uint64_t v = __atomic_load_n(&sl[0], __ATOMIC_ACQUIRE);
      if ((uint32_t)v == sq) {
        *status = (int32_t)(uint32_t)(v >> 32);
        break;
      }
      while (got < nS && (uint32_t)__atomic_load_n(&sl[2 + got], __ATOMIC_ACQUIRE) == sq) ++got;
      if (got == nS) {
        for (int q = 0; q < T->D; ++q)
          T->pDomOut[q] = ((uint64_t)(uint32_t)(sl[3 + 2 * q] >> 32) << 32) | (uint32_t)(sl[2 + 2 * q] >> 32);
        *status = CT_OK;
        break;
      }
      if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
        hipError_t e = hipStreamSynchronize(T->stream);
        if (e != hipSuccess) {
          T->poisoned = true;
          return fail(CT_E_DEVICE, "kernel failed: %s", hipGetErrorString(e));
        }
        T->poisoned = true;
        return fail(CT_E_DEVICE, "kernel finished without a result (device error %d)", *T->q.hostErr);
      }
    }
    if (*T->q.hostErr) {
      T->poisoned = true;
      return fail(CT_E_DEVICE, "device-side error %d (wait timeout or trail overflow)", *T->q.hostErr);
    }
    return CT_OK;
  }
  // The job publishes its status (and its outputs before it) to coherent
  // host memory with a system-scope release: wait for that word instead of
  // the whole kernel.  The kernel's tail finishes on the stream, which
  // orders it before the next launch.
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 0; *status == kStatusPending; ++spin) {
    if ((spin & 1023) == 1023 &&
        std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      hipError_t e = hipStreamSynchronize(T->stream);
      if (e != hipSuccess) {
        T->poisoned = true;
        return fail(CT_E_DEVICE, "kernel failed: %s", hipGetErrorString(e));
      }
      if (*status == kStatusPending) {
        T->poisoned = true;
        return fail(CT_E_DEVICE, "kernel finished without a status (device error %d)", *T->q.hostErr);
      }
    }
  }
  if (*T->q.hostErr) {
    T->poisoned = true;
    return fail(CT_E_DEVICE, "device-side error %d (wait timeout or trail overflow)", *T->q.hostErr);
  }
  return CT_OK;
}

int ensure_pinned_ct(ct_table* T);

// ---------------------------------------------------------------------------
// resident engine of a table's slot 0 (one engine alive per process: each
// holds a hardware queue while it waits for calls)
// ---------------------------------------------------------------------------
std::mutex g_engMu;
ct_table* g_engOwner = nullptr;
std::set<ct_table*> g_tables;  // live tables (for ct_quiesce)
constexpr double kEngineIdleMs = 2.0;  // an engine without calls for this long exits

int64_t engine_idle_ticks() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  return (int64_t)(kEngineIdleMs * khz);
}

// Waits for the engine of T to end (it has exited or was told to) and
// marks it stopped; its state is then back in the slot's device arrays.
int engine_join(ct_table* T) {
  const auto t0 = std::chrono::steady_clock::now();
  while (__atomic_load_n(&T->pRes->alive, __ATOMIC_ACQUIRE) != 0) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) break;
  }
  hipError_t e = hipStreamSynchronize(T->engStream);
  T->engOn = false;
  if (g_engOwner == T) g_engOwner = nullptr;
  if (e == hipSuccess && T->engTimed && T->timing) {
    T->engLifeTicks += T->pRes->lifeTicks;
    T->engLaunches += 1;
  }
  if (e != hipSuccess) {
    T->poisoned = true;
    return fail(CT_E_DEVICE, "engine failed: %s", hipGetErrorString(e));
  }
  return CT_OK;
}

// Writes a call into the mailbox: every command slot, flagged with the
// call's sequence number, the domain words first and the op last (the
// engine takes the call once all of them carry the number).
void engine_post(ct_table* T, int32_t seq, int32_t op, const DevJob* J, const uint64_t* dom_in, bool wantCt,
                 bool wantStats) {
  uint64_t* s = T->pCmd->slot;
  const uint32_t sq = (uint32_t)seq;
  for (int i = 0; i < 2 * T->D; ++i) {
    const uint32_t half = dom_in ? (uint32_t)(dom_in[i >> 1] >> (i & 1 ? 32 : 0)) : 0u;
    __atomic_store_n(&s[EC_DOM + i], eng_slot(half, sq), __ATOMIC_RELAXED);
  }
  const uint32_t hdr[EC_DOM] = {(uint32_t)op,
                                J ? (uint32_t)J->nPop : 0u,
                                J ? (uint32_t)J->nPush : 0u,
                                J ? (uint32_t)J->serialBase : 0u,
                                J ? (uint32_t)J->depthAfter : 0u,
                                wantCt ? 1u : 0u,
                                wantStats ? 1u : 0u,
                                0u};
  for (int i = EC_DOM - 1; i > 0; --i) __atomic_store_n(&s[i], eng_slot(hdr[i], sq), __ATOMIC_RELAXED);
  __atomic_store_n(&s[EC_OP], eng_slot(hdr[EC_OP], sq), __ATOMIC_RELEASE);
}

int engine_stop(ct_table* T) {
  if (!T || !T->engOn) return CT_OK;
  if (__atomic_load_n(&T->pRes->alive, __ATOMIC_ACQUIRE) != 0) engine_post(T, ++T->engSeq, ENG_OP_STOP, nullptr,
                                                                           nullptr, false, false);
  return engine_join(T);
}

bool engine_wanted(const ct_table* T);
bool split_engine_wanted(ct_table* T);

int engine_start(ct_table* T) {
  if (g_engOwner && g_engOwner != T) {
    int rc = engine_stop(g_engOwner);
    if (rc) return rc;
  }
  if (T->tailPending) {  // earlier launches on the slot end first
    HIPCHK(hipStreamSynchronize(T->stream));
    T->tailPending = false;
  }
  if (!T->engStream) HIPCHK(hipStreamCreateWithFlags(&T->engStream, hipStreamNonBlocking));
  if (!T->pCmd) {
    ALLOCCHK(hipHostMalloc((void**)&T->pCmd, sizeof(EngCmd), hipHostMallocMapped | hipHostMallocCoherent));
    ALLOCCHK(hipHostMalloc((void**)&T->pRes, sizeof(EngRes), hipHostMallocMapped | hipHostMallocCoherent));
    memset((void*)T->pCmd, 0, sizeof(EngCmd));
    memset((void*)T->pRes, 0, sizeof(EngRes));
  }
  int rc = ensure_pinned_ct(T);
  if (rc) return rc;
  EngDesc D{};
  D.tab = T->dTab;
  D.slot = T->slots[0].dev;
  HIPCHK(hipHostGetDevicePointer((void**)&D.cmd, T->pCmd, 0));
  HIPCHK(hipHostGetDevicePointer((void**)&D.res, T->pRes, 0));
  HIPCHK(hipHostGetDevicePointer((void**)&D.ctOut, T->pCt, 0));
  D.idleTicks = engine_idle_ticks();
  D.startSeq = T->engSeq;
  T->engTimed = T->timing;
  T->engSplit = !engine_wanted(T) && split_engine_wanted(T);
  if (T->engSplit) {
    if (!T->dCtl) {
      void* p = nullptr;
      ALLOCCHK(hipMalloc(&p, sizeof(int32_t) * SE_CTL_WORDS));
      T->blocks.push_back(p);
      T->dCtl = (int32_t*)p;
    }
    // (stream-ordered before the launch; never inside a captured graph)
    HIPCHK(hipMemsetAsync(T->dCtl, 0, sizeof(int32_t) * SE_CTL_WORDS, T->engStream));
    D.ctl = T->dCtl;
    D.nFilt = propagate_items_per_job_filter(T->D);
  }
  __atomic_store_n(&T->pRes->alive, 1, __ATOMIC_RELEASE);
  if (T->engSplit) {
    // workgroup 0, then the filter workgroups with every eighth workgroup
    // (XCD 0 in the dispatch round robin) left empty
    int grid = 1;
    for (int f = 0; f < D.nFilt; ++grid)
      if (grid % 8 != 0) ++f;
    HIPCHK(launch_split_engine(D, grid, T->engStream));
  }
  else HIPCHK(launch_engine(D, T->engLds, T->engStream));
  T->engOn = true;
  g_engOwner = T;
  return CT_OK;
}

// Waits for a result slot of call `sq` (written at most a few microseconds
// after its status) and returns its payload; false after two seconds.
bool engine_slot(const ct_table* T, int i, uint32_t sq, uint32_t* payload) {
  const uint64_t* p = &T->pRes->slot[i];
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 0;; ++spin) {
    const uint64_t v = __atomic_load_n(p, __ATOMIC_ACQUIRE);
    if ((uint32_t)v == sq) {
      *payload = (uint32_t)(v >> 32);
      return true;
    }
    if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) return false;
  }
}

// One call through the engine; *status receives the call's status and the
// outputs are in T->engDom, T->engStats (wantStats) and T->pCt (wantCt).
int engine_call(ct_table* T, const DevJob& J, const uint64_t* dom_in, bool wantCt, bool wantStats, int* status) {
  std::lock_guard<std::mutex> lk(g_engMu);
  int rc;
  if (T->engOn && __atomic_load_n(&T->pRes->alive, __ATOMIC_ACQUIRE) == 0 && (rc = engine_join(T))) return rc;
  if (!T->engOn && (rc = engine_start(T))) return rc;
  const int32_t seq = ++T->engSeq;
  const uint32_t sq = (uint32_t)seq;
  engine_post(T, seq, ENG_OP_PROPAGATE, &J, dom_in, wantCt, wantStats);
  const uint64_t* stSlot = &T->pRes->slot[ER_STATUS];
  const auto t0 = std::chrono::steady_clock::now();
  uint64_t sv = 0;
  for (uint32_t spin = 0;; ++spin) {
    if ((uint32_t)(sv = __atomic_load_n(stSlot, __ATOMIC_ACQUIRE)) == sq) break;
    if (__atomic_load_n(&T->pRes->alive, __ATOMIC_ACQUIRE) == 0) {
      if ((uint32_t)(sv = __atomic_load_n(stSlot, __ATOMIC_ACQUIRE)) == sq) break;
      // the engine went idle before it saw this call: start a new one (the
      // command stays in the mailbox)
      if ((rc = engine_join(T))) return rc;
      T->engSeq = seq - 1;
      if ((rc = engine_start(T))) return rc;
      T->engSeq = seq;
      continue;
    }
    if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      T->poisoned = true;
      return fail(CT_E_DEVICE, "engine did not answer");
    }
  }
  *status = (int32_t)(uint32_t)(sv >> 32);
  bool whole = true;
  if (*status == CT_OK) {
    // every domain slot carries the number (in order of arrival: one clock
    // read per poll round, not per slot)
    const uint64_t* sl = &T->pRes->slot[ER_DOM];
    const int nS = 2 * T->D;
    int got = 0;
    const auto t1 = std::chrono::steady_clock::now();
    for (uint32_t spin = 0;; ++spin) {
      while (got < nS && (uint32_t)__atomic_load_n(&sl[got], __ATOMIC_ACQUIRE) == sq) ++got;
      if (got == nS) break;
      if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t1 > std::chrono::seconds(2)) {
        whole = false;
        break;
      }
    }
    T->engDom.resize(T->D);
    for (int q = 0; q < T->D && whole; ++q)
      T->engDom[q] = ((uint64_t)(uint32_t)(sl[2 * q + 1] >> 32) << 32) | (uint32_t)(sl[2 * q] >> 32);
  }
  if (wantStats) {
    for (int k = 0; k < 8 && whole; ++k) {
      uint32_t lo = 0, hi = 0;
      whole = engine_slot(T, ER_STATS + 2 * k, sq, &lo) && engine_slot(T, ER_STATS + 2 * k + 1, sq, &hi);
      T->engStats[k] = ((unsigned long long)hi << 32) | lo;
    }
  }
  uint32_t ticks = 0;
  if (whole && T->timing) whole = engine_slot(T, ER_TICKS, sq, &ticks);
  if (!whole) {
    T->poisoned = true;
    return fail(CT_E_DEVICE, "engine answer incomplete");
  }
  T->engStatsFresh = wantStats;
  if (T->timing) {
    T->engTicks += ticks;
    T->engCalls += 1;
  }
  return CT_OK;
}

// AUTO takes the engine for tables of at most ENG_AUTO_D domain words: on
// wider tables one workgroup's filterDomains (a gather of one word per
// checked value) is slower than the launched schedules, which spread it over
// many workgroups; RESIDENT takes it up to ENG_MAX_D words.
constexpr int ENG_AUTO_D = 64;
bool engine_wanted(const ct_table* T) {
  return T->engEligible &&
         ((T->cfg.schedule == CT_SCHED_AUTO && T->D <= ENG_AUTO_D) || T->cfg.schedule == CT_SCHED_RESIDENT);
}

// AUTO takes the resident split schedule (split_engine_kernel) for the other
// positive tables whose split update is one item (at most 8 granules) and
// whose input fits the kernel-argument view (D <= INLINE_WORDS, so at most
// 64 filter workgroups, all resident at once), with variables of at most
// SE_MAX_VAR_WORDS domain words: plain synchronous calls on slot 0 then pay
// no kernel launch.  Calls that want currTable or counters, and the other
// slots, take the launched schedules.
bool split_engine_wanted(ct_table* T) {
  if (T->seVarWords < 0) {
    int m = 0;
    for (const VarDesc& v : T->vars) m = std::max(m, (int)v.domWords);
    T->seVarWords = m;
  }
  return T->cfg.schedule == CT_SCHED_AUTO && T->kind == CT_KIND_POSITIVE && !engine_wanted(T) &&
         !use_solo(T, 1) && propagate_items_per_job_update(T->nGran, 0) == 1 && T->D <= INLINE_WORDS &&
         T->D <= ENG_MAX_D && T->seVarWords <= SE_MAX_VAR_WORDS &&
         2 + (8 * propagate_items_per_job_filter(T->D)) / 7 <= propagate_max_grid();
}

// Before any other use of a table's device state (from `same`, nullable):
// work a model queued on slot 0 from another stream has ended, and the
// table's engine is stopped.
int quiesce(ct_table* T, hipStream_t same) {
  if (!T) return CT_OK;
  if (T->pendStream && T->pendStream != same) {
    HIPCHK(hipStreamSynchronize(T->pendStream));
    T->pendStream = nullptr;
  }
  if (!T->engOn) return CT_OK;
  std::lock_guard<std::mutex> lk(g_engMu);
  return engine_stop(T);
}

int32_t* pinned_dev(ct_table* T, int32_t* host) {
  int32_t* d = nullptr;
  if (hipHostGetDevicePointer((void**)&d, host, 0) != hipSuccess) return nullptr;
  return d;
}
uint64_t* pinned_dev64(ct_table* T, uint64_t* host) {
  uint64_t* d = nullptr;
  if (hipHostGetDevicePointer((void**)&d, host, 0) != hipSuccess) return nullptr;
  return d;
}

// Apply pending pushes/pops of a slot (device work) without propagating.
int flush_slot(ct_table* T, int slot) {
  SlotHost& S = T->slots[slot];
  if (S.pendPop == 0 && S.pendPush == 0) return CT_OK;
  DevJob J{};
  J.tab = T->dTab;
  J.slot = S.dev;
  J.flags = 0;
  J.nPop = S.pendPop;
  J.nPush = S.pendPush;
  J.serialBase = T->serialCounter;
  T->serialCounter += S.pendPush;
  J.depthAfter = S.depth;
  J.status_out = pinned_dev(T, T->pStatus);
  S.pendPop = S.pendPush = 0;
  return run_single(T, J, nullptr);
}

int ensure_pinned_ct(ct_table* T) {
  if (T->pCt) return CT_OK;
  ALLOCCHK(hipHostMalloc((void**)&T->pCt, sizeof(uint64_t) * std::max<int64_t>(T->W, 1),
                       hipHostMallocMapped | hipHostMallocCoherent));
  return CT_OK;
}

int check_slot(const ct_table* T, int slot) {
  if (slot < 0 || slot >= (int)T->slots.size())
    return fail(CT_E_INVALID, "slot %d out of range (%zu slots)", slot, T->slots.size());
  if (T->slots[slot].freed) return fail(CT_E_INVALID, "slot %d was freed", slot);
  return CT_OK;
}

// ---------------------------------------------------------------------------
// batch staging shared by ct_propagate_batch and ct_propagate_batch_static
// ---------------------------------------------------------------------------
// Validates every job (no state is touched before all pass; the marks that
// find a slot named twice carry no state), then waits for what the tables
// may still have in flight elsewhere (a model's queued work, the resident
// engine, the tail of a synchronous call).
int batch_validate_quiesce(const ct_job* jobs, int n_jobs, hipStream_t stream) {
  static std::atomic<uint64_t> batchCounter{0};
  const uint64_t mark = ++batchCounter;
  for (int j = 0; j < n_jobs; ++j) {
    const ct_job& cj = jobs[j];
    ct_table* T = cj.table;
    int rc = check_poison(T);
    if (rc) return rc;
    if ((rc = check_slot(T, cj.slot))) return rc;
    if (T->slots[cj.slot].batchMark == mark)
      return fail(CT_E_INVALID, "job %d: slot %d appears twice in the batch", j, cj.slot);
    T->slots[cj.slot].batchMark = mark;
    if (cj.flags & ~(CT_JOB_PROPAGATE | CT_JOB_FROM_ROOT | CT_JOB_ROOT))
      return fail(CT_E_INVALID, "job %d: unknown flags", j);
    if ((cj.flags & CT_JOB_ROOT) && (cj.flags & CT_JOB_FROM_ROOT))
      return fail(CT_E_INVALID, "job %d: ROOT and FROM_ROOT together", j);
    if ((cj.flags & CT_JOB_ROOT) && (cj.n_pop || cj.n_push || !(cj.flags & CT_JOB_PROPAGATE)))
      return fail(CT_E_INVALID, "job %d: ROOT needs PROPAGATE and no pops/pushes", j);
    if (cj.n_pop < 0 || cj.n_push < 0) return fail(CT_E_INVALID, "job %d: negative pops/pushes", j);
    const SlotHost& S = T->slots[cj.slot];
    if (cj.flags & CT_JOB_FROM_ROOT) {
      if (cj.n_pop || cj.n_push) return fail(CT_E_INVALID, "job %d: FROM_ROOT with pops/pushes", j);
      if (!(cj.flags & CT_JOB_PROPAGATE)) return fail(CT_E_INVALID, "job %d: FROM_ROOT needs PROPAGATE", j);
    } else {
      if (cj.n_pop > S.depth) return fail(CT_E_INVALID, "job %d: pop below depth 0", j);
      if (S.depth - cj.n_pop + cj.n_push > S.maxDepth)
        return fail(CT_E_NOMEM, "job %d: depth beyond max_depth", j);
    }
    if ((cj.flags & CT_JOB_PROPAGATE) && (!cj.dom_in || !cj.dom_out))
      return fail(CT_E_INVALID, "job %d: dom_in / dom_out is NULL", j);
  }
  // the synchronous calls of these tables may still be finishing their tail
  for (int j = 0; j < n_jobs; ++j) {
    ct_table* T = jobs[j].table;
    if (T->batchMark == mark) continue;
    T->batchMark = mark;
    int rc = quiesce(T, stream);
    if (rc) return rc;
    if (T->tailPending) {
      HIPCHK(hipStreamSynchronize(T->stream));
      T->tailPending = false;
    }
  }
  return CT_OK;
}

// Device descriptors of a validated batch, written into out[n_jobs], the
// item offsets updOff / filtOff (n_jobs + 1 entries, [0] = 0 on entry) and
// the prep list (up to n_jobs entries); returns the prep list's length.
// Applies the jobs' pops and pushes to the host mirror of each slot.
int batch_build(const ct_job* jobs, int n_jobs, int32_t* status_dev, bool nodes, DevJob* out,
                int32_t* updOff, int32_t* filtOff, int32_t* prep) {
  int nPrep = 0;
  updOff[0] = filtOff[0] = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const ct_job& cj = jobs[j];
    ct_table* T = cj.table;
    SlotHost& S = T->slots[cj.slot];
    DevJob& J = out[j];
    J = DevJob{};
    J.tab = T->dTab;
    J.slot = S.dev;
    J.dom_in = cj.dom_in;
    J.dom_out = cj.dom_out;
    J.ct_out = cj.ct_out;
    J.status_out = status_dev + j;
    J.flags = ((cj.flags & CT_JOB_PROPAGATE) ? JF_PROPAGATE : 0u) |
              ((cj.flags & CT_JOB_FROM_ROOT) ? JF_FROM_ROOT : 0u) |
              ((cj.flags & CT_JOB_ROOT) ? (JF_ROOT | JF_FROM_ROOT | JF_SCRATCH) : 0u);
    if (cj.flags & (CT_JOB_FROM_ROOT | CT_JOB_ROOT)) {
      S.pendPop = S.pendPush = 0;
      S.depth = 0;
      S.failedAt.clear();
      J.serialBase = T->serialCounter++;
      J.depthAfter = 0;
    } else {
      // pending single-call operations (pops P then pushes Q) come first
      int P = S.pendPop, Q = S.pendPush;
      if (cj.n_pop <= Q) {
        Q = Q - cj.n_pop + cj.n_push;
      } else {
        P += cj.n_pop - Q;
        Q = cj.n_push;
      }
      S.pendPop = S.pendPush = 0;
      J.nPop = P;
      J.nPush = Q;
      J.serialBase = T->serialCounter;
      T->serialCounter += Q;
      for (int k = 0; k < cj.n_pop; ++k) S.failedAt.pop_back();
      for (int k = 0; k < cj.n_push; ++k) S.failedAt.push_back(2);
      S.depth = S.depth - cj.n_pop + cj.n_push;
      J.depthAfter = S.depth;
    }
    S.failed = 2;
    // a root recomputed from scratch streams every support row: large
    // tables are split over workgroups (the queue balances them), small ones
    // run solo
    const bool solo = (J.flags & JF_SCRATCH) && T->cfg.schedule == CT_SCHED_AUTO && T->kind == CT_KIND_POSITIVE
                          ? T->nGran <= SCRATCH_SOLO_MAX_GRAN
                          : use_solo(T, n_jobs);
    if ((J.flags & JF_PROPAGATE) && !nodes && solo) J.flags |= JF_SOLO;
    job_counts(T, J);
    updOff[j + 1] = updOff[j] + J.nUpd;
    filtOff[j + 1] = filtOff[j] + J.nFilt;
    if (needs_prep(J)) prep[nPrep++] = j;
  }
  return nPrep;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* ct_last_error(void) { return g_err; }

int ct_debug_fail_alloc(int32_t nth) { return g_failAlloc.exchange(nth > 0 ? nth : 0); }

int ct_quiesce(void) {
  std::lock_guard<std::mutex> lk(g_engMu);
  return g_engOwner ? engine_stop(g_engOwner) : CT_OK;
}

void ct_destroy(ct_table* T) {
  if (!T) return;
  (void)quiesce(T);
  {
    std::lock_guard<std::mutex> lk(g_engMu);
    g_tables.erase(T);
  }
  if (T->pCmd) (void)hipHostFree(T->pCmd);
  if (T->pRes) (void)hipHostFree(T->pRes);
  if (T->engStream) (void)hipStreamDestroy(T->engStream);
  if (T->stream) (void)hipStreamSynchronize(T->stream);
  for (void* p : T->blocks) (void)hipFree(p);
  queue_free(T->q);
  if (T->pDomOut) (void)hipHostFree(T->pDomOut);
  if (T->pLL) (void)hipHostFree(T->pLL);
  if (T->pDomIn) (void)hipHostFree(T->pDomIn);
  if (T->pCt) (void)hipHostFree(T->pCt);
  if (T->pStatus) (void)hipHostFree(T->pStatus);
  if (T->stream) (void)hipStreamDestroy(T->stream);
  delete T;
}

// 1 if two tuples of the table are equal (hash of each row, then the rows
// with equal hashes compared)
bool has_duplicate_rows(const int32_t* tuples, int64_t t, int n) {
  std::vector<std::pair<uint64_t, int64_t>> h((size_t)t);
  for (int64_t j = 0; j < t; ++j) {
    uint64_t x = 1469598103934665603ull;
    for (int i = 0; i < n; ++i) x = (x ^ (uint32_t)tuples[j * n + i]) * 1099511628211ull;
    h[(size_t)j] = {x, j};
  }
  std::sort(h.begin(), h.end());
  for (size_t k = 1; k < h.size(); ++k)
    if (h[k].first == h[k - 1].first &&
        std::equal(tuples + h[k].second * n, tuples + h[k].second * n + n, tuples + h[k - 1].second * n))
      return true;
  return false;
}

static int create_impl(ct_table* T, const int32_t* tuples, int64_t t, int32_t n,
                       const int32_t* lo, const int32_t* dsz, const uint64_t* init_dom) {
  bool star = false;
  for (int64_t k = 0; k < t * n && !star; ++k) star = tuples[k] == CT_STAR;
  if (T->kind == CT_KIND_NEGATIVE) {
    if (star) return fail(CT_E_INVALID, "a negative table has no star cell");
    if (has_duplicate_rows(tuples, t, n)) return fail(CT_E_INVALID, "a negative table lists distinct tuples");
  }
  if (star) {
    // a star cell supports every value of its column: the update takes the
    // reset branch (OR over the remaining values), which needs no other rows
    if (T->cfg.branch_policy == CT_BRANCH_INCREMENTAL)
      return fail(CT_E_INVALID, "a short table's update takes the reset branch");
    T->cfg.branch_policy = CT_BRANCH_RESET;
    T->shortTab = true;
  }
  T->n = n;
  T->t = t;
  T->W = (t + 63) / 64;
  T->nGran = (int)std::max<int64_t>(1, (T->W + GW - 1) / GW);
  T->stride = (int64_t)T->nGran * GW;
  T->lo.assign(lo, lo + n);
  T->dsz.assign(dsz, dsz + n);
  int rows = 0, D = 0;
  for (int i = 0; i < n; ++i) {
    VarDesc v;
    v.rowStart = rows;
    v.dsize = dsz[i];
    v.domOff = D;
    v.domWords = (dsz[i] + 63) / 64;
    T->vars.push_back(v);
    T->domOff.push_back(D);
    for (int k = 0; k < v.domWords; ++k) T->wordVar.push_back(i);
    rows += dsz[i];
    D += v.domWords;
  }
  T->rows = rows;
  T->D = D;
  if (rows > MAX_TABLE_ROWS) return fail(CT_E_INVALID, "%d support rows exceed the limit %d", rows, MAX_TABLE_ROWS);
  if (D > MAX_TABLE_D) return fail(CT_E_INVALID, "%d domain words exceed the limit %d", D, MAX_TABLE_D);
  if (T->kind == CT_KIND_NEGATIVE && (rows > NEG_MAX_ROWS || D > MAX_D))
    return fail(CT_E_INVALID, "a negative table has at most %d support rows and %d domain words", NEG_MAX_ROWS,
                MAX_D);
  if (T->nGran > MAX_GRAN)
    return fail(CT_E_INVALID, "%lld tuples exceed the limit %lld", (long long)t,
                (long long)MAX_GRAN * GW * 64);
  // initial domains (validated on the host, before any device work)
  std::vector<uint64_t> dom0(D, 0);
  for (int i = 0; i < n; ++i) {
    const VarDesc& v = T->vars[i];
    for (int k = 0; k < v.domWords; ++k) {
      const int used = std::min(64, v.dsize - 64 * k);
      const uint64_t full = used == 64 ? ~0ull : ((1ull << used) - 1);
      if (init_dom) {
        if (init_dom[v.domOff + k] & ~full)
          return fail(CT_E_INVALID, "init_dom has stray bits in variable %d", i);
        dom0[v.domOff + k] = init_dom[v.domOff + k];
      } else {
        dom0[v.domOff + k] = full;
      }
    }
  }
  HIPCHK(hipStreamCreateWithFlags(&T->stream, hipStreamNonBlocking));
  int rc = queue_init(T->q);
  if (rc) return rc;
  // coherent (fine-grained) pinned buffers: the kernel's writes reach host
  // memory without waiting for the end of the kernel
  const unsigned kCoherent = hipHostMallocMapped | hipHostMallocCoherent;
  ALLOCCHK(hipHostMalloc((void**)&T->pDomOut, sizeof(uint64_t) * D, kCoherent));
  ALLOCCHK(hipHostMalloc((void**)&T->pLL, sizeof(uint64_t) * (2 + 2 * (size_t)D), kCoherent));
  memset(T->pLL, 0, sizeof(uint64_t) * (2 + 2 * (size_t)D));
  ALLOCCHK(hipHostMalloc((void**)&T->pDomIn, sizeof(uint64_t) * D, kCoherent));
  ALLOCCHK(hipHostMalloc((void**)&T->pStatus, sizeof(int32_t) * 4, kCoherent));

  // static data
  if ((rc = dev_alloc(T, (void**)&T->dS, sizeof(uint64_t) * (size_t)rows * T->stride))) return rc;
  if ((rc = dev_alloc(T, (void**)&T->dVars, sizeof(VarDesc) * n))) return rc;
  if ((rc = dev_alloc(T, (void**)&T->dWordVar, sizeof(int32_t) * D))) return rc;
  if ((rc = dev_alloc(T, (void**)&T->dWords, sizeof(WordDesc) * D))) return rc;
  if ((rc = dev_alloc(T, (void**)&T->dLo, sizeof(int32_t) * n))) return rc;
  if ((rc = dev_alloc(T, (void**)&T->dTab, sizeof(TabDesc)))) return rc;
  HIPCHK(hipMemcpy(T->dVars, T->vars.data(), sizeof(VarDesc) * n, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(T->dWordVar, T->wordVar.data(), sizeof(int32_t) * D, hipMemcpyHostToDevice));
  {
    std::vector<WordDesc> words(D);
    for (int q = 0; q < D; ++q) {
      words[q] = WordDesc{};
      words[q].v = T->vars[T->wordVar[q]];
      words[q].var = T->wordVar[q];
    }
    HIPCHK(hipMemcpy(T->dWords, words.data(), sizeof(WordDesc) * D, hipMemcpyHostToDevice));
  }
  HIPCHK(hipMemcpy(T->dLo, lo, sizeof(int32_t) * n, hipMemcpyHostToDevice));
  HIPCHK(hipMemsetAsync(T->dS, 0, sizeof(uint64_t) * (size_t)rows * T->stride, T->stream));
  if (t > 0) {
    int32_t* dTup = nullptr;
    ALLOCCHK(hipMalloc(&dTup, sizeof(int32_t) * (size_t)t * n));
    hipError_t e = hipMemcpyAsync(dTup, tuples, sizeof(int32_t) * (size_t)t * n,
                                  hipMemcpyHostToDevice, T->stream);
    if (e == hipSuccess)
      e = launch_build_supports(dTup, t, n, T->dVars, T->dLo, T->dS, T->stride, T->W, T->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(T->stream);
    (void)hipFree(dTup);
    if (e != hipSuccess) return fail(CT_E_DEVICE, "support build failed: %s", hipGetErrorString(e));
  }

  // root slot: currTable = all t tuples, every granule active, domains dom0
  std::vector<SlotDesc> hs;
  if ((rc = alloc_slots(T, 1, 0, &T->dRoot, hs))) return rc;
  T->hRoot = hs[0];
  {
    std::vector<uint64_t> ones(T->stride, 0);
    for (int64_t j = 0; j < T->W; ++j) {
      const int64_t left = t - 64 * j;
      ones[j] = left >= 64 ? ~0ull : ((1ull << left) - 1);
    }
    std::vector<int32_t> iota(T->nGran);
    for (int g = 0; g < T->nGran; ++g) iota[g] = g;
    std::vector<int32_t> zeros(std::max(rows, T->nGran), 0);
    HIPCHK(hipMemcpy(T->hRoot.ct, ones.data(), sizeof(uint64_t) * T->stride, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(T->hRoot.idx[0], iota.data(), sizeof(int32_t) * T->nGran, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(T->hRoot.idx[1], iota.data(), sizeof(int32_t) * T->nGran, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(T->hRoot.stamp, zeros.data(), sizeof(int32_t) * T->nGran, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(T->hRoot.nzFlag, zeros.data(), sizeof(int32_t) * T->nGran, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(T->hRoot.res, zeros.data(), sizeof(int32_t) * rows, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(T->hRoot.lastDom, dom0.data(), sizeof(uint64_t) * D, hipMemcpyHostToDevice));
    SlotDesc r = T->hRoot;
    r.limit = T->nGran;
    HIPCHK(hipMemcpy(T->dRoot, &r, sizeof(SlotDesc), hipMemcpyHostToDevice));
  }
  // TabDesc (root pointers filled after the root propagation)
  TabDesc& tb = T->hTab;
  tb.n = n;
  tb.rows = rows;
  tb.D = D;
  tb.nGran = T->nGran;
  tb.W = T->W;
  tb.stride = T->stride;
  tb.S = T->dS;
  tb.vars = T->dVars;
  tb.wordVar = T->dWordVar;
  tb.words = T->dWords;
  tb.policy = T->cfg.branch_policy;
  tb.tailBits = T->W > 0 ? (int32_t)(t - 64 * (T->W - 1)) : 0;
  tb.kind = T->kind;
  HIPCHK(hipMemcpy(T->dTab, &tb, sizeof(TabDesc), hipMemcpyHostToDevice));

  // root propagation: every variable takes the reset branch over dom0
  DevJob J{};
  J.tab = T->dTab;
  J.slot = T->dRoot;
  J.flags = JF_PROPAGATE | JF_ROOT;
  J.dom_out = pinned_dev64(T, T->pDomOut);
  J.status_out = pinned_dev(T, T->pStatus);
  J.depthAfter = 0;
  if ((rc = run_single(T, J, dom0.data()))) return rc;
  HIPCHK(hipStreamSynchronize(T->stream));
  const int st = *T->pStatus;
  SlotDesc r{};
  HIPCHK(hipMemcpy(&r, T->dRoot, sizeof(SlotDesc), hipMemcpyDeviceToHost));
  if (st != CT_OK && st != CT_FAIL) return fail(CT_E_DEVICE, "root propagation returned %d", st);
  T->rootFailed = st == CT_FAIL;
  tb.ct0 = T->hRoot.ct;
  tb.idx0 = r.idx[r.cur];
  tb.dom0 = T->hRoot.lastDom;
  tb.limit0 = r.limit;
  tb.rootFailed = T->rootFailed;
  if (T->rootFailed) {
    // the failed root keeps dom0 as its domains and no valid tuple
    HIPCHK(hipMemcpy(T->hRoot.lastDom, dom0.data(), sizeof(uint64_t) * D, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(T->hRoot.ct, 0, sizeof(uint64_t) * T->stride));
    tb.limit0 = 0;
  }
  HIPCHK(hipMemcpy(T->dTab, &tb, sizeof(TabDesc), hipMemcpyHostToDevice));
  int first = 0;
  if ((rc = ct_slots_alloc(T, 1, -1, &first))) return rc;
  // the resident engine holds the slot's state in one workgroup's LDS
  T->engLds = engine_lds_bytes(T->n, T->D, T->nGran, T->rows);
  int dev = 0, lds = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // (the engine lists rows with 16-bit ids)
  T->engEligible = T->D <= ENG_MAX_D && T->W > 0 && T->engLds <= (size_t)lds && T->kind == CT_KIND_POSITIVE &&
                   T->rows <= 65535;
  std::lock_guard<std::mutex> lk(g_engMu);
  g_tables.insert(T);
  return CT_OK;
}

int ct_create(const int32_t* tuples, int64_t n_tuples, int32_t arity, const int32_t* dom_lo,
              const int32_t* dom_size, const uint64_t* init_dom, const ct_config* cfg,
              ct_table** out) {
  return ct_create_table(tuples, n_tuples, arity, dom_lo, dom_size, init_dom, cfg, CT_KIND_POSITIVE, out);
}

int ct_create_table(const int32_t* tuples, int64_t n_tuples, int32_t arity, const int32_t* dom_lo,
                    const int32_t* dom_size, const uint64_t* init_dom, const ct_config* cfg, int32_t kind,
                    ct_table** out) {
  if (!out) return fail(CT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (kind != CT_KIND_POSITIVE && kind != CT_KIND_NEGATIVE) return fail(CT_E_INVALID, "kind %d", kind);
  if (arity < 1 || arity > MAX_ARITY) return fail(CT_E_INVALID, "arity %d not in [1, %d]", arity, MAX_ARITY);
  if (n_tuples < 0) return fail(CT_E_INVALID, "n_tuples < 0");
  if (n_tuples > 0 && !tuples) return fail(CT_E_INVALID, "tuples is NULL");
  if (!dom_lo || !dom_size) return fail(CT_E_INVALID, "dom_lo / dom_size is NULL");
  for (int i = 0; i < arity; ++i)
    if (dom_size[i] < 1) return fail(CT_E_INVALID, "dom_size[%d] < 1", i);
  ct_table* T = new (std::nothrow) ct_table();
  if (!T) return fail(CT_E_NOMEM, "host allocation failed");
  T->cfg.branch_policy = CT_BRANCH_AUTO;
  T->cfg.max_depth = 256;
  T->cfg.schedule = CT_SCHED_AUTO;
  T->kind = kind;
  if (cfg) {
    if (cfg->schedule < 0 || cfg->schedule > 4) {
      delete T;
      return fail(CT_E_INVALID, "schedule %d", cfg->schedule);
    }
    T->cfg.schedule = cfg->schedule;
    if (cfg->branch_policy < 0 || cfg->branch_policy > 2) {
      delete T;
      return fail(CT_E_INVALID, "branch_policy %d", cfg->branch_policy);
    }
    T->cfg.branch_policy = cfg->branch_policy;
    if (cfg->max_depth < 0) {
      delete T;
      return fail(CT_E_INVALID, "max_depth < 0");
    }
    T->cfg.max_depth = cfg->max_depth;
  }
  int rc = create_impl(T, tuples, n_tuples, arity, dom_lo, dom_size, init_dom);
  if (rc != CT_OK) {
    char msg[sizeof(g_err)];
    memcpy(msg, g_err, sizeof(g_err));
    ct_destroy(T);
    memcpy(g_err, msg, sizeof(g_err));
    return rc;
  }
  *out = T;
  return T->rootFailed ? CT_FAIL : CT_OK;
}

int ct_layout(const ct_table* T, ct_layout_info* info, int32_t* dom_off) {
  if (!T) return fail(CT_E_INVALID, "null table");
  if (info) {
    info->n_vars = T->n;
    info->D = T->D;
    info->W = T->W;
    info->n_tuples = T->t;
    info->rows = T->rows;
    info->n_slots = (int32_t)T->slots.size();
    info->granules = T->nGran;
    info->root_failed = T->rootFailed;
    info->resident = engine_wanted(T) ? 1 : split_engine_wanted(const_cast<ct_table*>(T)) ? 2 : 0;
    info->kind = T->kind == CT_KIND_NEGATIVE ? CT_KIND_NEGATIVE : T->shortTab ? CT_KIND_SHORT : CT_KIND_POSITIVE;
  }
  if (dom_off) memcpy(dom_off, T->domOff.data(), sizeof(int32_t) * T->n);
  return CT_OK;
}

int ct_get_supports(ct_table* T, int32_t row_begin, int32_t n_rows, uint64_t* out) {
  int rc = check_poison(T);
  if (rc) return rc;
  if (row_begin < 0 || n_rows < 0 || row_begin + n_rows > T->rows || (!out && n_rows))
    return fail(CT_E_INVALID, "rows [%d, %d) out of range", row_begin, row_begin + n_rows);
  if (T->W == 0) return CT_OK;
  HIPCHK(hipMemcpy2D(out, sizeof(uint64_t) * T->W, T->dS + (size_t)row_begin * T->stride,
                     sizeof(uint64_t) * T->stride, sizeof(uint64_t) * T->W, n_rows,
                     hipMemcpyDeviceToHost));
  return CT_OK;
}

int ct_slots_alloc(ct_table* T, int32_t n, int32_t max_depth, int32_t* first_slot) {
  int rc = check_poison(T);
  if (rc) return rc;
  if (n < 1) return fail(CT_E_INVALID, "n < 1");
  if ((rc = quiesce(T))) return rc;
  if (max_depth < 0) max_depth = T->cfg.max_depth;
  // reuse: the first run of n consecutive freed slots whose trails hold
  // max_depth levels; each is reset to the root state
  int run = 0, first = -1;
  for (int k = 0; k < (int)T->slots.size() && first < 0; ++k) {
    const SlotHost& S = T->slots[k];
    run = (S.freed && S.capDepth >= max_depth) ? run + 1 : 0;
    if (run == n) first = k - n + 1;
  }
  if (first >= 0) {
    for (int k = first; k < first + n; ++k)
      HIPCHK(launch_init_slots(T->dTab, T->slots[k].dev, 1, T->hRoot.res, T->stream));
    HIPCHK(hipStreamSynchronize(T->stream));
    for (int k = first; k < first + n; ++k) {
      SlotHost& S = T->slots[k];
      const int cap = S.capDepth;
      SlotDesc* dev = S.dev;
      S = SlotHost();
      S.dev = dev;
      S.capDepth = cap;
      S.maxDepth = max_depth;
      S.failed = T->rootFailed ? 1 : 0;
      S.failedAt.reserve(max_depth);
    }
    if (first_slot) *first_slot = first;
    return CT_OK;
  }
  SlotDesc* d = nullptr;
  std::vector<SlotDesc> h;
  if ((rc = alloc_slots(T, n, max_depth, &d, h))) return rc;
  HIPCHK(launch_init_slots(T->dTab, d, n, T->hRoot.res, T->stream));
  HIPCHK(hipStreamSynchronize(T->stream));
  if (first_slot) *first_slot = (int32_t)T->slots.size();
  for (int k = 0; k < n; ++k) {
    SlotHost s;
    s.dev = d + k;
    s.maxDepth = max_depth;
    s.capDepth = max_depth;
    s.failed = T->rootFailed ? 1 : 0;
    // a push never grows this vector past its capacity (no allocation per push)
    s.failedAt.reserve(max_depth);
    T->slots.push_back(s);
  }
  return CT_OK;
}

int ct_slots_free(ct_table* T, int32_t first, int32_t n) {
  int rc = check_poison(T);
  if (rc) return rc;
  if (n < 1 || first < 1 || first > (int)T->slots.size() - n)
    return fail(CT_E_INVALID, "slots [%d, %d) cannot be freed (%zu slots; slot 0 stays)", first, first + n,
                T->slots.size());
  for (int k = first; k < first + n; ++k)
    if (T->slots[k].freed) return fail(CT_E_INVALID, "slot %d is already free", k);
  // batches queued on other streams may still use the slots: the caller
  // frees a slot only after its last batch has completed
  if ((rc = quiesce(T))) return rc;
  for (int k = first; k < first + n; ++k) {
    SlotHost& S = T->slots[k];
    S.freed = true;
    S.depth = 0;
    S.pendPop = S.pendPush = 0;
    S.failedAt.clear();
  }
  return CT_OK;
}

int ct_push_slot(ct_table* T, int32_t slot) {
  int rc = check_poison(T);
  if (rc) return rc;
  if ((rc = check_slot(T, slot))) return rc;
  SlotHost& S = T->slots[slot];
  if (S.failed == 1) return fail(CT_E_STATE, "push on a failed slot");
  if (S.depth >= S.maxDepth) return fail(CT_E_NOMEM, "depth %d reaches max_depth", S.depth);
  S.failedAt.push_back(S.failed);
  S.depth++;
  S.pendPush++;
  return CT_OK;
}

int ct_pop_slot(ct_table* T, int32_t slot) {
  int rc = check_poison(T);
  if (rc) return rc;
  if ((rc = check_slot(T, slot))) return rc;
  SlotHost& S = T->slots[slot];
  if (S.depth == 0) return fail(CT_E_STATE, "pop at depth 0");
  S.depth--;
  S.failed = S.failedAt.back();
  S.failedAt.pop_back();
  if (S.pendPush > 0) S.pendPush--;
  else S.pendPop++;
  return CT_OK;
}

int ct_push(ct_table* T) { return ct_push_slot(T, 0); }
int ct_pop(ct_table* T) { return ct_pop_slot(T, 0); }

int ct_propagate_slot(ct_table* T, int32_t slot, const uint64_t* dom_in, uint64_t* dom_out,
                      uint64_t* ct_out, ct_stats* st) {
  int rc = check_poison(T);
  if (rc) return rc;
  if ((rc = check_slot(T, slot))) return rc;
  if (!dom_in || !dom_out) return fail(CT_E_INVALID, "dom_in / dom_out is NULL");
  SlotHost& S = T->slots[slot];
  DevJob J{};
  J.tab = T->dTab;
  J.slot = S.dev;
  J.flags = JF_PROPAGATE;
  J.nPop = S.pendPop;
  J.nPush = S.pendPush;
  J.serialBase = T->serialCounter;
  T->serialCounter += S.pendPush;
  J.depthAfter = S.depth;
  J.dom_out = pinned_dev64(T, T->pDomOut);
  J.status_out = pinned_dev(T, T->pStatus);
  if (ct_out) {
    if ((rc = ensure_pinned_ct(T))) return rc;
    J.ct_out = pinned_dev64(T, T->pCt);
  }
  S.pendPop = S.pendPush = 0;
  int status = CT_OK;
  const uint64_t* domRes = T->pDomOut;
  if (slot == 0 && engine_wanted(T)) {
    if ((rc = engine_call(T, J, dom_in, ct_out != nullptr, st != nullptr, &status))) return rc;
    domRes = T->engDom.data();
  } else if (slot == 0 && !ct_out && !st && split_engine_wanted(T)) {
    if ((rc = engine_call(T, J, dom_in, false, false, &status))) return rc;
    domRes = T->engDom.data();
  } else {
    if ((rc = run_single(T, J, dom_in))) return rc;
    status = *T->pStatus;
  }
  if (status == CT_OK) {
    memcpy(dom_out, domRes, sizeof(uint64_t) * T->D);
    if (ct_out) memcpy(ct_out, T->pCt, sizeof(uint64_t) * T->W);
  } else if (status == CT_FAIL) {
    S.failed = 1;
    if (ct_out) memset(ct_out, 0, sizeof(uint64_t) * T->W);
  }
  if (st) {
    if ((rc = ct_slot_stats(T, slot, st))) return rc;
  }
  switch (status) {
    case CT_OK:
    case CT_FAIL:
      return status;
    case CT_E_NOT_SUBSET:
      return fail(status, "dom_in is not a subset of the slot's domains");
    case CT_E_INVALID:
      return fail(status, "dom_in has stray bits");
    case CT_E_STATE:
      return fail(status, "slot is failed; only pop is allowed");
    default:
      T->poisoned = true;
      return fail(CT_E_DEVICE, "unexpected device status %d", status);
  }
}

int ct_propagate(ct_table* T, const uint64_t* dom_in, uint64_t* dom_out, uint64_t* ct_out,
                 ct_stats* st) {
  return ct_propagate_slot(T, 0, dom_in, dom_out, ct_out, st);
}

int ct_get_state(ct_table* T, int32_t slot, uint64_t* dom_out, uint64_t* ct_out) {
  int rc = check_poison(T);
  if (rc) return rc;
  if ((rc = check_slot(T, slot))) return rc;
  if ((rc = quiesce(T))) return rc;
  if ((rc = flush_slot(T, slot))) return rc;
  HIPCHK(hipStreamSynchronize(T->stream));
  SlotDesc s{};
  HIPCHK(hipMemcpy(&s, T->slots[slot].dev, sizeof(SlotDesc), hipMemcpyDeviceToHost));
  if (dom_out) HIPCHK(hipMemcpy(dom_out, s.lastDom, sizeof(uint64_t) * T->D, hipMemcpyDeviceToHost));
  if (ct_out && T->W > 0) {
    if (s.failed) {
      memset(ct_out, 0, sizeof(uint64_t) * T->W);
    } else {
      HIPCHK(hipMemcpy(ct_out, s.ct, sizeof(uint64_t) * T->W, hipMemcpyDeviceToHost));
    }
  }
  return CT_OK;
}

int ct_slot_stats(ct_table* T, int32_t slot, ct_stats* st) {
  int rc = check_poison(T);
  if (rc) return rc;
  if ((rc = check_slot(T, slot))) return rc;
  if (!st) return fail(CT_E_INVALID, "st is NULL");
  SlotDesc s{};
  if (slot == 0 && T->engOn && T->engStatsFresh && __atomic_load_n(&T->pRes->alive, __ATOMIC_ACQUIRE) != 0) {
    // the engine holds the counters: its snapshot after the last call
    for (int k = 0; k < 8; ++k) s.stats[k] = T->engStats[k];
  } else {
    if ((rc = quiesce(T))) return rc;
    HIPCHK(hipStreamSynchronize(T->stream));
    HIPCHK(hipMemcpy(&s, T->slots[slot].dev, sizeof(SlotDesc), hipMemcpyDeviceToHost));
  }
  st->jobs = (int64_t)s.stats[S_JOBS];
  st->granules_in = (int64_t)s.stats[S_GRAN_IN];
  st->rows_or = (int64_t)s.stats[S_ROWS];
  st->granule_rows = (int64_t)s.stats[S_GRAN_ROWS];
  st->trail_granules = (int64_t)s.stats[S_TRAIL];
  st->residue_checks = (int64_t)s.stats[S_RES_CHECK];
  st->residue_misses = (int64_t)s.stats[S_RES_MISS];
  st->scan_granules = (int64_t)s.stats[S_SCAN];
  return CT_OK;
}

int ct_batch_status(void* stream_v) {
  hipStream_t stream = (hipStream_t)stream_v;
  int rc = noalloc_status(stream);
  if (rc) return rc;
  QueueCtx* q = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_qmu);
    auto it = g_queues.find(stream);
    if (it == g_queues.end()) return CT_OK;
    q = it->second;
  }
  HIPCHK(hipStreamSynchronize(stream));
  const int32_t err = *(volatile int32_t*)q->hostErr;
  if (!err) return CT_OK;
  *q->hostErr = 0;
  HIPCHK(hipMemsetAsync(q->queue + 3, 0, sizeof(int32_t), stream));
  HIPCHK(hipStreamSynchronize(stream));
  return fail(CT_E_DEVICE, "device-side error %d in a batch on this stream (wait timeout or trail "
              "overflow); the slots of that batch are undefined", err);
}

static const unsigned long long kClockInit[5] = {~0ull, 0ull, 0ull, 0ull, 0ull};

int ct_set_timing(ct_table* T, int32_t on) {
  int rc = check_poison(T);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(T->stream));
  if (on && !T->dClock) {
    if ((rc = dev_alloc(T, (void**)&T->dClock, sizeof(kClockInit)))) return rc;
  }
  if (T->dClock) HIPCHK(hipMemcpy(T->dClock, kClockInit, sizeof(kClockInit), hipMemcpyHostToDevice));
  T->timing = on != 0;
  T->engTicks = 0;
  T->engCalls = 0;
  T->engLifeTicks = 0;
  T->engLaunches = 0;
  return CT_OK;
}

int ct_get_dispatch_timing(ct_table* T, double* dispatch_ms, int64_t* dispatches) {
  if (!T) return fail(CT_E_INVALID, "null table");
  unsigned long long c[5] = {0, 0, 0, 0, 0};
  if (T->dClock) {
    int rc = quiesce(T);  // also ends a running engine: its lifetime is then known
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(T->stream));
    HIPCHK(hipMemcpy(c, T->dClock, sizeof(c), hipMemcpyDeviceToHost));
  }
  int dev = 0, khz = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (dispatch_ms) *dispatch_ms = khz > 0 ? (double)(c[3] + T->engLifeTicks) / (double)khz : 0.0;
  if (dispatches) *dispatches = (int64_t)(c[4] + T->engLaunches);
  return CT_OK;
}

int ct_get_timing(ct_table* T, double* kernel_ms, int64_t* launches) {
  if (!T) return fail(CT_E_INVALID, "null table");
  unsigned long long c[5] = {0, 0, 0, 0, 0};
  if (T->dClock) {
    int rc = quiesce(T);  // launched calls on the table's stream have ended
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(T->stream));
    HIPCHK(hipMemcpy(c, T->dClock, sizeof(c), hipMemcpyDeviceToHost));
  }
  int dev = 0, khz = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  // launched calls, plus calls served by the resident engine (device time of
  // each call inside the engine)
  if (kernel_ms) *kernel_ms = khz > 0 ? (double)(c[3] + T->engTicks) / (double)khz : 0.0;
  if (launches) *launches = (int64_t)(c[4] + T->engCalls);
  return CT_OK;
}

}  // extern "C"

namespace {

// What a validated batch needs, before any slot's host state changes.
struct BatchPlan {
  bool nodes = false, roots = false;
  size_t nodesBytes = 0;   // search-node records and granule flags
  size_t nTaskInts = 0;    // root tasks, two ints each
  size_t offAt = 0;        // byte offset of the int section of the staging area
  size_t stageBytes = 0;   // staging bytes for the largest prep list
};

BatchPlan batch_plan(const ct_job* jobs, int n_jobs) {
  BatchPlan p;
  p.nodes = use_nodes(jobs, n_jobs);
  p.roots = !p.nodes && use_roots(jobs, n_jobs);
  if (p.nodes) {
    const ct_table* T = jobs[0].table;
    p.nodesBytes = align256(sizeof(uint64_t) * (size_t)n_jobs * nodes_node_words(T->rows, T->n)) +
                   align256((size_t)n_jobs * T->nGran);
  }
  if (p.roots) {
    size_t nTasks = 0;
    for (int j = 0; j < n_jobs; ++j) nTasks += (size_t)(jobs[j].table->nGran + WAVES - 1) / WAVES;
    p.nTaskInts = 2 * nTasks;
  }
  p.offAt = align256(sizeof(DevJob) * (size_t)n_jobs);
  // job descriptors, then updOff | filtOff | prep list | root tasks (even offset)
  p.stageBytes = p.offAt + sizeof(int32_t) * (2 * (size_t)(n_jobs + 1) + (size_t)n_jobs + 2 + p.nTaskInts);
  return p;
}

// Where a batch's scratch lives: device counters, staging and search-node
// scratch, and the host arrays the descriptors are built in.  Capacities
// must cover the batch's plan.
struct BatchRes {
  int32_t* queue = nullptr;     // device: [0] head, [1] exit count, [2] launches, [3] error
  int32_t* hostErr = nullptr;   // pinned, nullable
  char* dStage = nullptr;       // device staging
  char* hStage = nullptr;       // host staging (the source of the one copy)
  hipEvent_t staged = nullptr;  // nullable: recorded after the copy
  void* dNodes = nullptr;
  DevJob* hJobs = nullptr;      // n_jobs
  int32_t* updOff = nullptr;    // n_jobs + 1
  int32_t* filtOff = nullptr;   // n_jobs + 1
  int32_t* prep = nullptr;      // n_jobs
  int32_t* rootTasks = nullptr; // plan.nTaskInts
  std::array<int32_t, 3>* rootKey = nullptr;  // n_jobs
};

// Builds the descriptors of a validated batch (applying its pops and pushes
// to the slots' host mirrors), stages them in one copy and launches it.
int batch_launch(const ct_job* jobs, int n_jobs, hipStream_t stream, int32_t* status_dev, const BatchPlan& p,
                 const BatchRes& r) {
  // root streams: WAVES granules per task, tables with the most support rows
  // first (their tasks are the longest)
  if (p.roots) {
    for (int j = 0; j < n_jobs; ++j) {
      const ct_table* T = jobs[j].table;
      r.rootKey[j] = {-T->rows, -T->nGran, j};
    }
    std::sort(r.rootKey, r.rootKey + n_jobs);
    size_t at = 0;
    for (int k = 0; k < n_jobs; ++k)
      for (int g = 0; g < -r.rootKey[k][1]; g += WAVES) {
        r.rootTasks[at++] = r.rootKey[k][2];
        r.rootTasks[at++] = g;
      }
  }
  const int nPrep = batch_build(jobs, n_jobs, status_dev, p.nodes, r.hJobs, r.updOff, r.filtOff, r.prep);
  // stage to the device (the root tasks start at an even offset: int pairs)
  const size_t rootBase = (2 * (size_t)(n_jobs + 1) + (size_t)nPrep + 2) & ~(size_t)1;
  const size_t nOff = p.roots ? rootBase + p.nTaskInts : 2 * (size_t)(n_jobs + 1) + (size_t)nPrep + 1;
  const size_t stageBytes = p.offAt + sizeof(int32_t) * nOff;
  int32_t* pOff = (int32_t*)(r.hStage + p.offAt);
  memcpy(r.hStage, r.hJobs, sizeof(DevJob) * n_jobs);
  memcpy(pOff, r.updOff, sizeof(int32_t) * (n_jobs + 1));
  memcpy(pOff + (n_jobs + 1), r.filtOff, sizeof(int32_t) * (n_jobs + 1));
  if (nPrep) memcpy(pOff + 2 * (n_jobs + 1), r.prep, sizeof(int32_t) * nPrep);
  if (p.roots && p.nTaskInts) memcpy(pOff + rootBase, r.rootTasks, sizeof(int32_t) * p.nTaskInts);
  HIPCHK(hipMemcpyAsync(r.dStage, r.hStage, stageBytes, hipMemcpyHostToDevice, stream));
  if (r.staged) HIPCHK(hipEventRecord(r.staged, stream));
  DevJob* dJobs = (DevJob*)r.dStage;
  int32_t* dOff = (int32_t*)(r.dStage + p.offAt);
  KArgs a{};
  a.jobs = dJobs;
  a.updOff = dOff;
  a.filtOff = dOff + (n_jobs + 1);
  a.prepList = dOff + 2 * (n_jobs + 1);
  a.nJobs = n_jobs;
  a.nPrep = nPrep;
  a.nUpd = r.updOff[n_jobs];
  a.nFilt = r.filtOff[n_jobs];
  a.queue = r.queue;
  a.hostErr = r.hostErr;
  if (p.nodes) {
    const ct_table* T = jobs[0].table;
    NodesDesc N{};
    N.nJobs = n_jobs;
    N.listCap = nodes_list_cap(T->rows, T->n);
    const NodesPlan plan = nodes_plan(T);
    N.groupSize = plan.groupSize;
    N.tw = plan.tw;
    N.groups = (n_jobs + N.groupSize - 1) / N.groupSize;
    N.jobs = dJobs;
    char* base = (char*)r.dNodes;
    N.nodeWords = nodes_node_words(T->rows, T->n);
    N.nodes = (uint64_t*)base;
    base += align256(sizeof(uint64_t) * (size_t)n_jobs * N.nodeWords);
    N.nz = (uint8_t*)base;
    N.rows = T->rows;
    N.nGran = T->nGran;
    N.stride = T->stride;
    N.W = T->W;
    N.S = T->hTab.S;
    N.ct0 = T->hTab.ct0;
    HIPCHK(launch_nodes(a, N, T->n, stream));
    return CT_OK;
  }
  if (p.roots) {
    RootDesc R{};
    R.tasks = dOff + rootBase;
    R.nTasks = (int32_t)(p.nTaskInts / 2);
    HIPCHK(launch_roots(a, R, stream));
    return CT_OK;
  }
  const int total = a.nPrep + a.nUpd + a.nFilt;
  if (total > 0) HIPCHK(launch_propagate(a, std::min(total, propagate_max_grid()), stream));
  return CT_OK;
}

// ct_propagate_batch_noalloc: fixed limits of the static scratch (device
// array in ct_noalloc.hip) and of the host arrays the descriptors are built in
constexpr int NA_MAX_JOBS = 8192;
constexpr size_t NA_QUEUE_BYTES = 256;
constexpr size_t NA_STAGE_BYTES = (size_t)2 << 20;
constexpr size_t NA_MAX_TASK_INTS = (NA_STAGE_BYTES - (size_t)NA_MAX_JOBS * 128) / sizeof(int32_t);

struct NoAllocHost {
  std::mutex mu;  // the host arrays are shared by every caller
  bool used = false;
  hipStream_t lastStream = nullptr;  // the stream of the last call (ct_batch_status)
  DevJob jobs[NA_MAX_JOBS];
  int32_t updOff[NA_MAX_JOBS + 1], filtOff[NA_MAX_JOBS + 1], prep[NA_MAX_JOBS];
  std::array<int32_t, 3> rootKey[NA_MAX_JOBS];
  int32_t rootTasks[NA_MAX_TASK_INTS];
  alignas(256) char stage[NA_STAGE_BYTES];
};
NoAllocHost g_na;

int noalloc_status(hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_na.mu);
  if (!g_na.used || g_na.lastStream != stream) return CT_OK;
  char* scratch = nullptr;
  size_t bytes = 0;
  HIPCHK(noalloc_scratch(&scratch, &bytes));
  HIPCHK(hipStreamSynchronize(stream));
  int32_t w[2] = {0, 0};  // the error words of the last call and of an earlier one
  HIPCHK(hipMemcpy(w, scratch + 3 * sizeof(int32_t), sizeof(w), hipMemcpyDeviceToHost));
  if (!w[0] && !w[1]) return CT_OK;
  const int32_t zero[2] = {0, 0};
  HIPCHK(hipMemcpy(scratch + 3 * sizeof(int32_t), zero, sizeof(zero), hipMemcpyHostToDevice));
  return fail(CT_E_DEVICE, "device-side error %d in a ct_propagate_batch_noalloc call on this stream (wait "
              "timeout or trail overflow); the slots of that batch are undefined", w[0] ? w[0] : w[1]);
}

}  // namespace

extern "C" {

int ct_propagate_batch(const ct_job* jobs, int32_t n_jobs, void* stream_v, int32_t* status_dev) {
  if (n_jobs < 0 || (n_jobs > 0 && (!jobs || !status_dev)))
    return fail(CT_E_INVALID, "bad batch arguments");
  if (n_jobs == 0) return CT_OK;
  hipStream_t stream = (hipStream_t)stream_v;
  int rc = batch_validate_quiesce(jobs, n_jobs, stream);
  if (rc) return rc;
  QueueCtx* q = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_qmu);
    auto it = g_queues.find(stream);
    if (it == g_queues.end()) {
      q = new QueueCtx();
      int rc = queue_init(*q);
      if (rc) {
        queue_free(*q);
        delete q;
        return rc;
      }
      g_queues[stream] = q;
    } else {
      q = it->second;
    }
  }
  const BatchPlan p = batch_plan(jobs, n_jobs);
  // device and pinned scratch, grown before any slot's host state changes:
  // a failed allocation leaves the slots as they were
  if (p.nodes && q->capNodes < p.nodesBytes) {
    HIPCHK(hipStreamSynchronize(stream));
    if (q->dNodes) (void)hipFree(q->dNodes);
    q->dNodes = nullptr;
    q->capNodes = 0;
    ALLOCCHK(hipMalloc(&q->dNodes, p.nodesBytes));
    q->capNodes = p.nodesBytes;
  }
  if (q->capStage < p.stageBytes) {
    HIPCHK(hipStreamSynchronize(stream));
    if (q->dStage) (void)hipFree(q->dStage);
    for (int k = 0; k < 2; ++k)
      if (q->pStage[k]) (void)hipHostFree(q->pStage[k]);
    const size_t cap = std::max(p.stageBytes, 2 * q->capStage);
    q->dStage = nullptr;
    q->pStage[0] = q->pStage[1] = nullptr;
    q->capStage = 0;
    ALLOCCHK(hipMalloc(&q->dStage, cap));
    for (int k = 0; k < 2; ++k) ALLOCCHK(hipHostMalloc((void**)&q->pStage[k], cap, hipHostMallocDefault));
    q->capStage = cap;
  }
  q->hJobs.resize(n_jobs);
  q->updOff.assign(n_jobs + 1, 0);
  q->filtOff.assign(n_jobs + 1, 0);
  q->prep.resize(n_jobs);
  q->rootTasks.resize(p.nTaskInts);
  q->rootKey.resize(p.roots ? n_jobs : 0);
  // two pinned staging buffers in turn: the copy that last read this one
  // (two batches ago) has ended
  q->turn ^= 1;
  HIPCHK(hipEventSynchronize(q->staged[q->turn]));
  BatchRes r;
  r.queue = q->queue;
  r.hostErr = q->hostErr;
  r.dStage = q->dStage;
  r.hStage = q->pStage[q->turn];
  r.staged = q->staged[q->turn];
  r.dNodes = q->dNodes;
  r.hJobs = q->hJobs.data();
  r.updOff = q->updOff.data();
  r.filtOff = q->filtOff.data();
  r.prep = q->prep.data();
  r.rootTasks = q->rootTasks.data();
  r.rootKey = q->rootKey.data();
  return batch_launch(jobs, n_jobs, stream, status_dev, p, r);
}

int ct_propagate_batch_noalloc(const ct_job* jobs, int32_t n_jobs, void* stream_v, int32_t* status_dev) {
  if (n_jobs < 0 || (n_jobs > 0 && (!jobs || !status_dev)))
    return fail(CT_E_INVALID, "bad batch arguments");
  if (n_jobs == 0) return CT_OK;
  if (n_jobs > NA_MAX_JOBS)
    return fail(CT_E_INVALID, "ct_propagate_batch_noalloc: %d jobs, at most %d", n_jobs, NA_MAX_JOBS);
  for (int j = 0; j < n_jobs; ++j)
    if (!jobs[j].table) return fail(CT_E_INVALID, "job %d: table is NULL", j);
  char* scratch = nullptr;
  size_t scratchBytes = 0;
  HIPCHK(noalloc_scratch(&scratch, &scratchBytes));
  const size_t nodesCap = scratchBytes - NA_QUEUE_BYTES - NA_STAGE_BYTES;
  const BatchPlan p = batch_plan(jobs, n_jobs);
  if (p.stageBytes > NA_STAGE_BYTES || p.nTaskInts > NA_MAX_TASK_INTS)
    return fail(CT_E_INVALID, "ct_propagate_batch_noalloc: the batch needs %zu staging bytes, at most %zu",
                p.stageBytes, NA_STAGE_BYTES);
  if (p.nodes && p.nodesBytes > nodesCap)
    return fail(CT_E_INVALID, "ct_propagate_batch_noalloc: the search-node schedule needs %zu scratch bytes, "
                "at most %zu", p.nodesBytes, nodesCap);
  hipStream_t stream = (hipStream_t)stream_v;
  std::lock_guard<std::mutex> lk(g_na.mu);
  int rc = batch_validate_quiesce(jobs, n_jobs, stream);
  if (rc) return rc;
  BatchRes r;
  r.queue = (int32_t*)scratch;
  r.dStage = scratch + NA_QUEUE_BYTES;
  r.hStage = g_na.stage;
  r.dNodes = scratch + NA_QUEUE_BYTES + NA_STAGE_BYTES;
  r.hJobs = g_na.jobs;
  r.updOff = g_na.updOff;
  r.filtOff = g_na.filtOff;
  r.prep = g_na.prep;
  r.rootTasks = g_na.rootTasks;
  r.rootKey = g_na.rootKey;
  // the work queue's counters start at zero (an earlier call's error word
  // is kept for ct_batch_status)
  HIPCHK(launch_noalloc_reset(r.queue, stream));
  g_na.used = true;
  g_na.lastStream = stream;
  return batch_launch(jobs, n_jobs, stream, status_dev, p, r);
}


}  // extern "C"

// internal accessors used by the serving loop (ct_server.cpp)
namespace ctk {
int64_t slot_footprint(const ct_table* T, int maxDepth) {
  const int64_t trailCap = (int64_t)maxDepth * T->nGran;
  return (int64_t)(align256(sizeof(uint64_t) * T->stride) + 4 * align256(sizeof(int32_t) * T->nGran) +
                   align256(sizeof(uint64_t) * T->D) + align256(sizeof(int32_t) * T->rows) +
                   align256(sizeof(TrailHdr) * std::max<int64_t>(trailCap, 1)) +
                   align256(sizeof(uint64_t) * GW * std::max<int64_t>(trailCap, 1)) +
                   align256(sizeof(Level) * std::max(maxDepth, 1)) +
                   align256(sizeof(uint64_t) * T->D * std::max(maxDepth, 1)) + sizeof(SlotDesc));
}

int root_domains(ct_table* T, uint64_t* out) {
  HIPCHK(hipMemcpy(out, T->hRoot.lastDom, sizeof(uint64_t) * T->D, hipMemcpyDeviceToHost));
  return CT_OK;
}

void set_error(const char* msg) { snprintf(g_err, sizeof(g_err), "%s", msg); }

// Read-only view of a table for the split propagators (ct_split.cpp): the
// supports, the layout and the root state never change after ct_create.
int table_view(const ct_table* T, TableView* v) {
  int rc = check_poison(T);
  if (rc) return rc;
  v->S = T->dS;
  v->stride = T->stride;
  v->W = T->W;
  v->n = T->n;
  v->D = T->D;
  v->rows = T->rows;
  v->rootFailed = T->rootFailed;
  v->branchPolicy = T->cfg.branch_policy;
  v->kind = T->kind;
  v->vars = T->vars.data();
  v->rootCt = T->hRoot.ct;
  v->rootDom = T->hRoot.lastDom;
  return CT_OK;
}
}  // namespace ctk

// ===========================================================================
// Multi-table model: propagation rounds captured in a hipGraph
// ===========================================================================
namespace ctk {
hipError_t launch_model_round(const ModelDesc& M, const KArgs& a, int grid, hipStream_t stream);
hipError_t launch_model_seed(const ModelDesc& M, hipStream_t stream);
}

struct ct_model {
  int nPool = 0, poolWords = 0;
  std::vector<int32_t> lo, dsz, poolOff, poolNW;
  std::vector<ct_table*> tabs;
  std::vector<std::vector<int32_t>> scopes;
  hipStream_t stream = nullptr;
  QueueCtx q;
  int soloMax = 4, roundsPerGraph = 8;
  // schedule per class of tables (granule bucket, rows bucket), set by the
  // autotuner: solo or split, and the tile (granules per wave); classes
  // without an entry follow soloMax with the default tile
  std::map<std::pair<int, int>, std::pair<int, int>> choice;
  // device state, rebuilt when the table set or the schedule changes
  bool built = false;
  std::vector<void*> blocks;
  ModelDesc M{};
  DevJob* dJobs = nullptr;
  int32_t* dOff = nullptr;
  std::vector<DevJob> hJobs;
  KArgs a{};
  int grid = 1;
  hipGraphExec_t exec = nullptr;   // roundsPerGraph rounds
  hipGraphExec_t exec1 = nullptr;  // one round: a fixpoint's first launch
  int32_t* pFlags = nullptr;   // pinned copy of M.flags
  int32_t* dStatus = nullptr;  // statuses of push/pop batches
};

namespace {

int model_alloc(ct_model* m, void** p, size_t bytes) {
  if (alloc_injected()) return fail(CT_E_NOMEM, "injected allocation failure: hipMalloc(%zu)", bytes);
  hipError_t e = hipMalloc(p, bytes ? bytes : 8);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(CT_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  m->blocks.push_back(*p);
  return CT_OK;
}

void model_free_device(ct_model* m) {
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->exec1) (void)hipGraphExecDestroy(m->exec1);
  m->exec = nullptr;
  m->exec1 = nullptr;
  for (void* p : m->blocks) (void)hipFree(p);
  m->blocks.clear();
  m->dStatus = nullptr;
  m->dJobs = nullptr;
  m->dOff = nullptr;
  m->M = ModelDesc{};
  m->built = false;
}

template <class T>
int model_upload(ct_model* m, T** dst, const std::vector<T>& src) {
  int rc = model_alloc(m, (void**)dst, sizeof(T) * std::max<size_t>(src.size(), 1));
  if (rc) return rc;
  if (!src.empty()) HIPCHK(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
  return CT_OK;
}

// Class of a table for the autotuner: floor(log4) of its granule count and
// of its support-row count.
int log4_bucket(int64_t x) {
  int b = 0;
  while (x >= 4) {
    x /= 4;
    ++b;
  }
  return b;
}

std::pair<int, int> table_class(const ct_table* T) { return {log4_bucket(T->nGran), log4_bucket(T->rows)}; }

// (solo, tile) of a table's round job
std::pair<int, int> model_choice(const ct_model* m, const ct_table* T) {
  auto it = m->choice.find(table_class(T));
  if (it != m->choice.end()) return it->second;
  return {T->nGran <= m->soloMax ? 1 : 0, 0};
}

// Device arrays, one propagate job per table, and the graph of K rounds.
int model_build(ct_model* m) {
  model_free_device(m);
  const int nT = (int)m->tabs.size();
  std::vector<int32_t> scopeTab, scopeVar, entDomOff, tabScope(nT + 1, 0), bufOff(nT, 0);
  std::vector<const uint64_t*> lastDom(nT);
  int64_t words = 0;
  for (int c = 0; c < nT; ++c) {
    ct_table* T = m->tabs[c];
    for (int k = 0; k < T->n; ++k) {
      scopeTab.push_back(c);
      scopeVar.push_back(m->scopes[c][k]);
      entDomOff.push_back(T->domOff[k]);
    }
    tabScope[c + 1] = (int32_t)scopeTab.size();
    bufOff[c] = (int32_t)words;
    words += T->D;
    SlotDesc sd{};
    HIPCHK(hipMemcpy(&sd, T->slots[0].dev, sizeof(SlotDesc), hipMemcpyDeviceToHost));
    lastDom[c] = (const uint64_t*)sd.lastDom;
  }
  ModelDesc& M = m->M;
  M = ModelDesc{};
  M.nTables = nT;
  M.nPool = m->nPool;
  M.poolWords = m->poolWords;
  M.nEntries = (int32_t)scopeTab.size();
  int rc;
  int32_t* p32 = nullptr;
  if ((rc = model_upload(m, &p32, m->poolOff))) return rc;
  M.poolOff = p32;
  if ((rc = model_upload(m, &p32, m->poolNW))) return rc;
  M.poolNW = p32;
  if ((rc = model_upload(m, &p32, scopeTab))) return rc;
  M.scopeTab = p32;
  if ((rc = model_upload(m, &p32, scopeVar))) return rc;
  M.scopeVar = p32;
  if ((rc = model_upload(m, &p32, entDomOff))) return rc;
  M.entDomOff = p32;
  if ((rc = model_upload(m, &p32, tabScope))) return rc;
  M.tabScope = p32;
  if ((rc = model_upload(m, &p32, bufOff))) return rc;
  M.bufOff = p32;
  const uint64_t** pld = nullptr;
  if ((rc = model_upload(m, &pld, lastDom))) return rc;
  M.lastDom = pld;
  uint64_t* p64 = nullptr;
  if ((rc = model_alloc(m, (void**)&p64, sizeof(uint64_t) * std::max<int64_t>(words, 1)))) return rc;
  M.domIn = p64;
  if ((rc = model_alloc(m, (void**)&p64, sizeof(uint64_t) * std::max<int64_t>(words, 1)))) return rc;
  M.domOut = p64;
  if ((rc = model_alloc(m, (void**)&p64, sizeof(uint64_t) * m->poolWords))) return rc;
  M.pool = p64;
  if ((rc = model_alloc(m, (void**)&p64, sizeof(uint64_t) * m->poolWords))) return rc;
  M.poolNext = p64;
  if ((rc = model_alloc(m, (void**)&p32, sizeof(int32_t) * std::max(nT, 1)))) return rc;
  M.status = p32;
  if ((rc = model_alloc(m, (void**)&p32, sizeof(int32_t) * std::max(nT, 1)))) return rc;
  M.dirty = p32;
  if ((rc = model_alloc(m, (void**)&p32, sizeof(int32_t) * std::max(m->nPool, 1)))) return rc;
  M.changed = p32;
  if ((rc = model_alloc(m, (void**)&p32, sizeof(int32_t) * 8))) return rc;
  M.flags = p32;
  if ((rc = model_alloc(m, (void**)&m->dStatus, sizeof(int32_t) * std::max(nT, 1)))) return rc;
  // jobs: table c propagates slot 0 from domIn to domOut when dirty[c]
  m->hJobs.assign(nT, DevJob{});
  std::vector<int32_t> off(2 * (nT + 1) + 1, 0);
  for (int c = 0; c < nT; ++c) {
    ct_table* T = m->tabs[c];
    DevJob& J = m->hJobs[c];
    J.tab = T->dTab;
    J.slot = T->slots[0].dev;
    J.dom_in = M.domIn + bufOff[c];
    J.dom_out = M.domOut + bufOff[c];
    J.status_out = M.status + c;
    const auto ch = model_choice(m, T);
    J.flags = JF_PROPAGATE | (ch.first || T->kind == CT_KIND_NEGATIVE ? JF_SOLO : 0u);
    J.tile = ch.second;
    J.depthAfter = T->slots[0].depth;
    J.active = M.dirty + c;
    job_counts(T, J);
    off[c + 1] = off[c] + J.nUpd;
    off[(nT + 1) + c + 1] = off[(nT + 1) + c] + J.nFilt;
  }
  if ((rc = model_upload(m, &m->dJobs, m->hJobs))) return rc;
  if ((rc = model_upload(m, &m->dOff, off))) return rc;
  KArgs& a = m->a;
  a = KArgs{};
  a.jobs = m->dJobs;
  a.updOff = m->dOff;
  a.filtOff = m->dOff + (nT + 1);
  a.prepList = m->dOff + 2 * (nT + 1);
  a.nJobs = nT;
  a.nPrep = 0;
  a.nUpd = off[nT];
  a.nFilt = off[(nT + 1) + nT];
  a.queue = m->q.queue;
  a.hostErr = m->q.hostErr;
  const int total = a.nUpd + a.nFilt;
  m->grid = std::max(1, std::min(total, propagate_max_grid()));
  // capture a one-round graph (a fixpoint's first two launches: most search
  // steps converge in a round or two, and rounds after convergence cost
  // launches) and a rounds_per_graph-round graph for the launches after them
  for (int which = 0; which < 2; ++which) {
    const int rounds = which == 0 ? 1 : m->roundsPerGraph;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < rounds; ++r) {
      hipError_t e = launch_model_round(M, a, m->grid, m->stream);
      if (e != hipSuccess) {
        hipGraph_t dummy = nullptr;
        (void)hipStreamEndCapture(m->stream, &dummy);
        if (dummy) (void)hipGraphDestroy(dummy);
        return fail(CT_E_DEVICE, "model round capture failed: %s", hipGetErrorString(e));
      }
    }
    HIPCHK(hipStreamEndCapture(m->stream, &g));
    hipError_t e = hipGraphInstantiate(which == 0 ? &m->exec1 : &m->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(CT_E_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
  }
  m->built = true;
  return CT_OK;
}

// Bring every table's slot 0 up to date (pending pushes/pops) and refresh the
// depth each job trails at.
int model_sync_tables(ct_model* m) {
  bool changed = false;
  for (size_t c = 0; c < m->tabs.size(); ++c) {
    ct_table* T = m->tabs[c];
    int rc = check_poison(T);
    if (rc) return rc;
    if ((rc = flush_slot(T, 0))) return rc;
    if ((rc = quiesce(T, m->stream))) return rc;
    // only a synchronous call's unfinished tail can still be on the table's
    // stream (everything else on it is waited for where it is queued)
    if (T->tailPending) {
      HIPCHK(hipStreamSynchronize(T->stream));
      T->tailPending = false;
    }
    // a round's job only asks whether levels exist (depth > 0: trail the
    // words it changes), so the job array is sent again only when that flips
    if (m->built && (m->hJobs[c].depthAfter > 0) != (T->slots[0].depth > 0)) {
      m->hJobs[c].depthAfter = T->slots[0].depth;
      changed = true;
    }
  }
  if (changed)
    HIPCHK(hipMemcpy(m->dJobs, m->hJobs.data(), sizeof(DevJob) * m->hJobs.size(), hipMemcpyHostToDevice));
  return CT_OK;
}

int model_push_pop(ct_model* m, bool push) {
  const int nT = (int)m->tabs.size();
  if (nT == 0) return CT_OK;
  if (!m->dStatus) {
    int rc = model_alloc(m, (void**)&m->dStatus, sizeof(int32_t) * nT);
    if (rc) return rc;
  }
  std::vector<ct_job> jobs(nT);
  for (int c = 0; c < nT; ++c) {
    jobs[c] = ct_job{};
    jobs[c].table = m->tabs[c];
    jobs[c].slot = 0;
    jobs[c].flags = 0;
    jobs[c].n_pop = push ? 0 : 1;
    jobs[c].n_push = push ? 1 : 0;
  }
  // queued on the model's stream, ahead of the next fixpoint's rounds; a
  // device-side error of this batch is reported by that fixpoint, and any
  // other use of a table waits for it (quiesce)
  int rc = ct_propagate_batch(jobs.data(), nT, m->stream, m->dStatus);
  if (rc) return rc;
  for (ct_table* T : m->tabs) T->pendStream = m->stream;
  return CT_OK;
}

}  // namespace

extern "C" {

int ct_model_create(int32_t n_vars, const int32_t* dom_lo, const int32_t* dom_size, ct_model** out) {
  if (!out) return fail(CT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n_vars < 1 || !dom_lo || !dom_size) return fail(CT_E_INVALID, "bad model arguments");
  ct_model* m = new (std::nothrow) ct_model();
  if (!m) return fail(CT_E_NOMEM, "host allocation failed");
  m->nPool = n_vars;
  int w = 0;
  for (int i = 0; i < n_vars; ++i) {
    if (dom_size[i] < 1) {
      delete m;
      return fail(CT_E_INVALID, "dom_size[%d] < 1", i);
    }
    m->lo.push_back(dom_lo[i]);
    m->dsz.push_back(dom_size[i]);
    m->poolOff.push_back(w);
    m->poolNW.push_back((dom_size[i] + 63) / 64);
    w += (dom_size[i] + 63) / 64;
  }
  m->poolWords = w;
  hipError_t e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete m;
    return fail(CT_E_DEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
  }
  int rc = queue_init(m->q);
  if (rc == CT_OK) {
    e = hipHostMalloc((void**)&m->pFlags, sizeof(int32_t) * 8, hipHostMallocDefault);
    if (e != hipSuccess) rc = fail(CT_E_NOMEM, "pinned allocation failed");
  }
  if (rc) {
    ct_model_destroy(m);
    return rc;
  }
  *out = m;
  return CT_OK;
}

void ct_model_destroy(ct_model* m) {
  if (!m) return;
  model_free_device(m);  // waits for the model's stream
  {
    // the live tables no longer wait for this stream
    std::lock_guard<std::mutex> lk(g_engMu);
    for (ct_table* T : m->tabs)
      if (g_tables.count(T) && T->pendStream == m->stream) T->pendStream = nullptr;
  }
  queue_free(m->q);
  if (m->pFlags) (void)hipHostFree(m->pFlags);
  if (m->stream) (void)hipStreamDestroy(m->stream);
  delete m;
}

int ct_model_add(ct_model* m, ct_table* T, const int32_t* scope, int32_t* index) {
  if (!m || !scope) return fail(CT_E_INVALID, "bad arguments");
  int rc = check_poison(T);
  if (rc) return rc;
  std::vector<int32_t> sc(scope, scope + T->n);
  std::set<int32_t> seen;
  for (int k = 0; k < T->n; ++k) {
    const int v = sc[k];
    if (v < 0 || v >= m->nPool) return fail(CT_E_INVALID, "scope[%d] = %d out of range", k, v);
    if (!seen.insert(v).second) return fail(CT_E_INVALID, "variable %d twice in a scope", v);
    if (m->lo[v] != T->lo[k] || m->dsz[v] != T->dsz[k])
      return fail(CT_E_INVALID, "column %d does not match pool variable %d", k, v);
  }
  for (ct_table* u : m->tabs)
    if (u == T) return fail(CT_E_INVALID, "table already in the model");
  if (index) *index = (int32_t)m->tabs.size();
  m->tabs.push_back(T);
  m->scopes.push_back(sc);
  model_free_device(m);
  return CT_OK;
}

int ct_model_layout(const ct_model* m, int32_t* pool_off, int32_t* pool_words) {
  if (!m) return fail(CT_E_INVALID, "null model");
  if (pool_off) memcpy(pool_off, m->poolOff.data(), sizeof(int32_t) * m->nPool);
  if (pool_words) *pool_words = m->poolWords;
  return CT_OK;
}

int ct_model_set_schedule(ct_model* m, int32_t solo_max_granules, int32_t rounds_per_graph) {
  if (!m || solo_max_granules < 0 || rounds_per_graph < 1 || rounds_per_graph > 256)
    return fail(CT_E_INVALID, "bad schedule");
  if (solo_max_granules != m->soloMax || rounds_per_graph != m->roundsPerGraph) {
    m->soloMax = solo_max_granules;
    m->roundsPerGraph = rounds_per_graph;
    model_free_device(m);
  }
  return CT_OK;
}

int ct_model_fixpoint(ct_model* m, const uint64_t* pool_in, uint64_t* pool_out, void* stream_v,
                      int64_t* n_props, int64_t* n_rounds) {
  if (!m || !pool_in || !pool_out) return fail(CT_E_INVALID, "bad arguments");
  hipStream_t user = (hipStream_t)stream_v;
  if (user) HIPCHK(hipStreamSynchronize(user));
  int rc = model_sync_tables(m);
  if (rc) return rc;
  if (!m->built && (rc = model_build(m))) return rc;
  ModelDesc& M = m->M;
  HIPCHK(hipMemcpyAsync(M.pool, pool_in, sizeof(uint64_t) * m->poolWords, hipMemcpyDeviceToDevice, m->stream));
  // (eager, never inside the captured rounds)
  HIPCHK(hipMemsetAsync(M.flags, 0, sizeof(int32_t) * 8, m->stream));
  HIPCHK(launch_model_seed(M, m->stream));
  for (int replays = 0;; ++replays) {
    if (replays > 100000) return fail(CT_E_DEVICE, "fixpoint did not converge");
    HIPCHK(hipGraphLaunch(replays < 2 ? m->exec1 : m->exec, m->stream));
    // the pool is copied out with the flags: when they say done, it is there
    HIPCHK(hipMemcpyAsync(pool_out, M.pool, sizeof(uint64_t) * m->poolWords, hipMemcpyDeviceToDevice, m->stream));
    HIPCHK(hipMemcpyAsync(m->pFlags, M.flags, sizeof(int32_t) * 8, hipMemcpyDeviceToHost, m->stream));
    hipError_t e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
      for (ct_table* T : m->tabs) T->poisoned = true;
      return fail(CT_E_DEVICE, "model round failed: %s", hipGetErrorString(e));
    }
    if (*(volatile int32_t*)m->q.hostErr) {
      for (ct_table* T : m->tabs) T->poisoned = true;
      return fail(CT_E_DEVICE, "device-side error %d in a model round", *m->q.hostErr);
    }
    if (m->pFlags[1] || !m->pFlags[0]) break;
  }
  // the push / pop batches queued on the model's stream before these rounds
  // have ended with them
  for (ct_table* T : m->tabs)
    if (T->pendStream == m->stream) T->pendStream = nullptr;
  if ((rc = ct_batch_status(m->stream))) {
    for (ct_table* T : m->tabs) T->poisoned = true;
    return rc;
  }
  for (ct_table* T : m->tabs) T->slots[0].failed = 2;
  if (n_props) *n_props = m->pFlags[3];
  if (n_rounds) *n_rounds = m->pFlags[2];
  if (m->pFlags[1] == 2)
    return fail(CT_E_STATE, "a table of the model is in the failed state (pop it first)");
  if (m->pFlags[1]) return CT_FAIL;
  return CT_OK;
}

int ct_model_push(ct_model* m) {
  if (!m) return fail(CT_E_INVALID, "null model");
  return model_push_pop(m, true);
}

int ct_model_pop(ct_model* m) {
  if (!m) return fail(CT_E_INVALID, "null model");
  for (ct_table* T : m->tabs)
    if (T->slots[0].depth == 0) return fail(CT_E_STATE, "pop at depth 0");
  return model_push_pop(m, false);
}

int ct_model_get_choice(const ct_model* m, int32_t table, int32_t* solo, int32_t* tile) {
  if (!m || table < 0 || table >= (int)m->tabs.size()) return fail(CT_E_INVALID, "bad table index");
  const auto ch = model_choice(m, m->tabs[table]);
  if (solo) *solo = ch.first;
  if (tile) *tile = ch.first ? 4 : (ch.second == 0 ? 2 : ch.second);
  return CT_OK;
}

}  // extern "C"

namespace {

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string class_key(const std::string& arch, std::pair<int, int> c) {
  return arch + " g" + std::to_string(c.first) + " r" + std::to_string(c.second);
}

// The tuning cache: a JSON object, one entry per line,
//   "gfx950 g2 r3": [solo, tile],
// keyed by architecture, granule bucket and rows bucket.
std::map<std::string, std::pair<int, int>> cache_read(const char* path) {
  std::map<std::string, std::pair<int, int>> out;
  FILE* f = path ? fopen(path, "r") : nullptr;
  if (!f) return out;
  char line[256], key[128];
  int solo = 0, tile = 0;
  while (fgets(line, sizeof(line), f))
    if (sscanf(line, " \"%127[^\"]\": [%d, %d]", key, &solo, &tile) == 3) out[key] = {solo, tile};
  fclose(f);
  return out;
}

bool cache_write(const char* path, const std::map<std::string, std::pair<int, int>>& entries) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& e : entries)
    fprintf(f, "\"%s\": [%d, %d]%s\n", e.first.c_str(), e.second.first, e.second.second,
            ++k < entries.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
  return rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" {

int ct_model_autotune(ct_model* m, const uint64_t* pool_in, const char* cache_path, int32_t* from_cache,
                      int32_t* timed) {
  if (!m || !pool_in) return fail(CT_E_INVALID, "bad arguments");
  if (from_cache) *from_cache = 0;
  if (timed) *timed = 0;
  // classes present, the largest total granule count first
  std::map<std::pair<int, int>, int64_t> work;
  for (ct_table* T : m->tabs) work[table_class(T)] += T->nGran;
  std::vector<std::pair<int64_t, std::pair<int, int>>> order;
  for (const auto& w : work) order.push_back({-w.second, w.first});
  std::sort(order.begin(), order.end());
  const std::string arch = device_arch();
  auto cache = cache_read(cache_path);
  bool all = !order.empty();
  for (const auto& o : order) all = all && cache.count(class_key(arch, o.second));
  if (cache_path && all) {
    for (const auto& o : order) m->choice[o.second] = cache[class_key(arch, o.second)];
    model_free_device(m);
    if (from_cache) *from_cache = 1;
    return CT_OK;
  }
  uint64_t* scratch = nullptr;
  ALLOCCHK(hipMalloc(&scratch, sizeof(uint64_t) * m->poolWords));
  std::vector<uint64_t> ref(m->poolWords), got(m->poolWords);
  int refSt = -100, rc = CT_OK, nTimed = 0;
  // one candidate: the median of 3 timed fixpoints from pool_in, each
  // between a push and a pop; every candidate must reach the same fixpoint
  auto measure = [&](double* ms) -> int {
    model_free_device(m);
    std::vector<double> t;
    for (int rep = 0; rep < 3; ++rep) {
      int r;
      if ((r = ct_model_push(m))) return r;
      if ((r = model_sync_tables(m))) return r;
      if (!m->built && (r = model_build(m))) return r;
      const auto t0 = std::chrono::steady_clock::now();
      const int st = ct_model_fixpoint(m, pool_in, scratch, nullptr, nullptr, nullptr);
      t.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
      if (st != CT_OK && st != CT_FAIL) return st;
      if (st == CT_OK && hipMemcpy(got.data(), scratch, sizeof(uint64_t) * m->poolWords,
                                   hipMemcpyDeviceToHost) != hipSuccess)
        return fail(CT_E_DEVICE, "copy failed");
      if (refSt == -100) {
        refSt = st;
        ref = got;
      } else if (st != refSt || (st == CT_OK && got != ref)) {
        return fail(CT_E_DEVICE, "schedules disagree on the fixpoint");
      }
      if ((r = ct_model_pop(m))) return r;
    }
    std::sort(t.begin(), t.end());
    *ms = t[1];
    ++nTimed;
    return CT_OK;
  };
  // coordinate descent over the classes: solo (one workgroup; its step is
  // fixed) or split with 2, 4 or 8 granules per wave per update item
  const std::pair<int, int> opts[] = {{1, 0}, {0, 2}, {0, 4}, {0, 8}};
  for (const auto& o : order) {
    const auto cls = o.second;
    std::pair<int, int> best{0, 0};
    double bestMs = 1e30;
    for (const auto& opt : opts) {
      m->choice[cls] = opt;
      double ms = 0;
      if ((rc = measure(&ms))) break;
      if (ms < bestMs) {
        bestMs = ms;
        best = opt;
      }
    }
    if (rc) break;
    m->choice[cls] = best;
    cache[class_key(arch, cls)] = best;
  }
  (void)hipFree(scratch);
  model_free_device(m);
  if (timed) *timed = nTimed;
  if (rc) return rc;
  if (cache_path && !cache_write(cache_path, cache))
    return fail(CT_E_INVALID, "cannot write the tuning cache %s", cache_path);
  return CT_OK;
}

}  // extern "C"
