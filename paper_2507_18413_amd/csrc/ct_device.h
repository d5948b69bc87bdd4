// ct_device.h -- device-side data layout of the CT library (internal).
//
// Shared by the kernels (ct_kernels.hip) and the host runtime (ct_runtime.cpp);
// never by the oracle.
//
// Reversible sparse bitset for currTable, MI355X form.  The paper keeps a
// dense currTable (Sec. 3); the CT algorithm it builds on tracks the non-zero
// words in an index list so that zero words are skipped.  Here the unit of the
// index is a *granule* of 64 consecutive uint64 words -- one word per lane of
// a 64-wide wavefront -- so that every load of a granule is one coalesced
// 512-byte access:
//   ct[stride]             dense words, exact: words of inactive granules are 0
//   idx[2][nGran]          two permutations of the granule ids (ping-pong);
//                          idx[cur][0..limit) are the granules with a non-zero
//                          word.  A propagation writes the stable partition of
//                          idx[cur][0..limit) (survivors first) into the other
//                          buffer and copies the tail, so idx[cur][0..L) holds
//                          the same *set* for every earlier limit L: restoring
//                          `limit` on backtrack restores the set.
//   stamp[nGran]           serial of the level in which the granule was last
//                          saved on the trail (first write per level only)
//   trail                  (granule, old stamp) headers + 64 old words each
//   levels[maxDepth]       trail top, limit, failed, serial at each push
#pragma once
#include <stdint.h>

// Pointers inside the descriptors address global memory (device HBM or
// pinned host memory).  The device pass types them as address space 1 so
// that the compiler emits global_load/global_store rather than flat
// accesses, which would share the LDS wait counter and serialize the
// support-row loads behind every LDS read.  The host pass sees plain
// pointers; the layout is the same.
#if defined(__HIP_DEVICE_COMPILE__)
#define CT_G __attribute__((address_space(1)))
#else
#define CT_G
#endif

namespace ctk {

constexpr int WAVE = 64;
constexpr int GW = 64;             // words per granule
constexpr int BLOCK = 256;         // threads per workgroup of the propagate kernel
constexpr int WAVES = BLOCK / WAVE;
constexpr int MAX_ARITY = 256;
constexpr int MAX_TABLE_ROWS = 1 << 22;  // support rows per table (row lists are staged in chunks)
constexpr int MAX_TABLE_D = 1 << 16;     // domain words per table
constexpr int MAX_D = 1024;        // domain words of a job cached in LDS (the rest read from memory)
constexpr int NEG_MAX_ROWS = 8192; // negative tables: support rows (their second update pass lists
                                   // the removed values' rows in one LDS chunk)
constexpr int MAX_GRAN = 8192;     // granules per table (partition done in LDS)
constexpr int INLINE_WORDS = 256;  // dom_in words carried in kernel arguments
constexpr int ENG_MAX_D = 512;     // domain words of a table served by the resident engine

// status codes (same values as the public header)
constexpr int ST_OK = 0, ST_FAIL = 1, ST_INVALID = -1, ST_NOT_SUBSET = -2, ST_STATE = -3,
              ST_NOMEM = -4, ST_DEVICE = -5;

// job flags
constexpr uint32_t JF_PROPAGATE = 1u;
constexpr uint32_t JF_FROM_ROOT = 2u;
constexpr uint32_t JF_ROOT = 4u;      // creation: every variable takes the reset branch
constexpr uint32_t JF_INLINE_DOM = 8u;
constexpr uint32_t JF_HOST_OUT = 16u;   // status / outputs in host memory: system-scope release
constexpr uint32_t JF_SOLO = 32u;       // whole job in one workgroup
constexpr uint32_t JF_SCRATCH = 64u;    // with JF_ROOT | JF_FROM_ROOT: root state recomputed from all tuples
// A synchronous split job answers through flagged slots in host memory (`ll`:
// slot 0 the status of a job that does not succeed, slots 2 + 2q and 3 + 2q
// the halves of domain word q; every slot carries `seq`): no fence, no count
// of finished items, and the host takes the call once all its domain words
// carry the number (or the status slot does).
constexpr uint32_t JF_LL = 128u;
// The slot's previous domains are read around the L2 (resident split
// schedule: the filter workgroups on other XCDs write them, and workgroup 0
// takes no acquire between calls, so its L2 keeps the table and the slot)
constexpr uint32_t JF_COHLAST = 256u;

struct VarDesc {
  int32_t rowStart, dsize, domOff, domWords;
};

// A domain word's variable and its descriptor, in one record (one load
// where the variable index and then its descriptor would take two).
struct WordDesc {
  VarDesc v;
  int32_t var, pad0, pad1, pad2;
};

struct TabDesc {
  int32_t n, rows, D, nGran;
  int64_t W, stride;          // stride = nGran * 64 words per support row
  const CT_G uint64_t* S;          // rows x stride
  const CT_G VarDesc* vars;        // n
  const CT_G int32_t* wordVar;     // D: variable owning each domain word
  const CT_G WordDesc* words;      // D: the same with the variable's descriptor
  // root state, read-only after creation
  const CT_G uint64_t* ct0;
  const CT_G int32_t* idx0;
  const CT_G uint64_t* dom0;
  int32_t limit0, rootFailed;
  int32_t policy, tailBits;      // tailBits: tuples in the last currTable word (1..64)
  int32_t kind, pad;             // 0: positive (allowed tuples), 1: negative (forbidden tuples)
};

struct TrailHdr {
  int32_t gran, oldStamp;
};

struct Level {
  int64_t trailTop;
  int32_t limit, failed, serial, pad;
};

enum StatIdx { S_JOBS = 0, S_GRAN_IN, S_ROWS, S_GRAN_ROWS, S_TRAIL, S_RES_CHECK, S_RES_MISS, S_SCAN };

struct SlotDesc {
  // arrays
  CT_G uint64_t* ct;
  CT_G int32_t* idx[2];
  CT_G int32_t* stamp;
  CT_G uint64_t* lastDom;
  CT_G int32_t* res;           // residue word per support row
  CT_G TrailHdr* trailHdr;
  CT_G uint64_t* trailWords;   // trailCap x 64
  CT_G Level* levels;          // maxDepth
  CT_G uint64_t* levelDom;     // maxDepth x D
  CT_G int32_t* nzFlag;        // nGran: granule non-zero after the running job
  int64_t trailCap;
  int32_t maxDepth, pad0;
  // mutable state
  int64_t trailTop;
  int32_t cur, limit, failed, depth, serial, pad1;
  // per-job scratch
  int32_t updCount, filtCount, jobTrail, prepDone, updDone, status;
  int32_t nzCount;  // granules a root stream found non-empty (reset by its finish)
  int32_t pad2;
  unsigned long long stats[8];
};

struct DevJob {
  const CT_G TabDesc* tab;
  CT_G SlotDesc* slot;
  const CT_G uint64_t* dom_in;  // device pointer, or unused with JF_INLINE_DOM
  CT_G uint64_t* dom_out;
  CT_G uint64_t* ct_out;
  CT_G int32_t* status_out;
  uint32_t flags;
  int32_t nPop, nPush;
  int32_t serialBase;      // serial of the k-th pushed level = serialBase + k
  int32_t nUpd, nFilt;     // item counts of this job
  int32_t depthAfter;      // slot depth once the pops and pushes are applied
  int32_t tile;            // split jobs: granules per wave per update item (2, 4 or 8;
                           // 0 = 2); solo jobs step 4 granules per wave
  const CT_G int32_t* active;  // nullable: the job is skipped when *active == 0
  uint64_t* ll;             // JF_LL: the result slots (pinned host memory)
  int32_t seq, llPad;       // JF_LL: the call's number
};

// The update item's hand-over word of a JF_LL job: the call's number with
// bit 30 set (never 0 or 1, the values the counted protocol uses).
__host__ __device__ inline int32_t ll_gen(int32_t seq) { return (seq & 0x3fffffff) | 0x40000000; }

// Granule-major schedule of a batch of search nodes (jobs that all propagate
// one table from its root state).  Per node: the Alg. 1 prologue's outcome
// and its row list: one segment holding the removed values' rows of every
// incremental variable of s_val (the complement of their OR is the AND of
// their incremental masks), then one segment per reset variable, in
// variable order, each padded to a multiple of 4 rows with the all-zero row
// `rows` of the update kernel's tile, its first entry tagged 0x8000 (| 0x4000
// when incremental); per (node, granule) the non-zero flag of the new
// currTable granule.
struct NodeInfo {
  int32_t status, nrows;   // nrows: support rows OR-ed (without padding)
  int32_t groups, pad;     // groups: list length / 4
  CT_G uint64_t* ct;       // the node's slot currTable
  CT_G uint64_t* ct_out;   // optional copy (W words), may be null
};

// A node's record in memory: its NodeInfo, then its row list (listCap
// entries); records of consecutive nodes are contiguous (nodeWords words).
struct NodesDesc {
  int32_t nJobs, listCap, nodeWords, groups, groupSize;
  int32_t rows, nGran;       // the table's (copied: no dependent loads)
  int32_t tw;                // granules per tile of the update kernel (1 or 2)
  int64_t stride, W;
  const CT_G uint64_t* S;
  const CT_G uint64_t* ct0;
  const CT_G DevJob* jobs;
  CT_G uint64_t* nodes;    // nJobs x nodeWords
  CT_G uint8_t* nz;        // nJobs x nGran
};

// Batch of roots recomputed from scratch: one task per workgroup of the
// stream kernel, (job, first granule) pairs, each covering WAVES consecutive
// granules of the job (one per wave), largest tables first.
struct RootDesc {
  const CT_G int32_t* tasks;  // nTasks x 2
  int32_t nTasks, pad;
};

// Multi-table model: pool variables shared by tables (device side of a
// propagation round).  Scope entry e links column tabCol[e] of table
// scopeTab[e] to pool variable scopeVar[e].
struct ModelDesc {
  int32_t nTables, nPool, poolWords, nEntries;
  const CT_G int32_t* poolOff;    // nPool: first pool word of each variable
  const CT_G int32_t* poolNW;     // nPool: words of each variable
  const CT_G int32_t* scopeTab;   // nEntries
  const CT_G int32_t* scopeVar;   // nEntries
  const CT_G int32_t* entDomOff;  // nEntries: word offset of the column in its table's bitmap
  const CT_G int32_t* tabScope;   // nTables + 1: entries of table c are [tabScope[c], tabScope[c+1])
  const CT_G int32_t* bufOff;     // nTables: offset of table c's words in domIn / domOut
  const CT_G uint64_t* const CT_G* lastDom;  // nTables: slot-0 domains of each table
  CT_G uint64_t* domIn;
  CT_G uint64_t* domOut;
  CT_G int32_t* status;           // nTables: job status of the round
  CT_G int32_t* dirty;            // nTables: table runs in the round
  CT_G uint64_t* pool;            // poolWords
  CT_G uint64_t* poolNext;        // poolWords
  CT_G int32_t* changed;          // nPool
  CT_G int32_t* flags;            // [0] some table dirty, [1] failed, [2] rounds, [3] table runs
};

// Kernel argument block of the persistent propagate kernel.
struct KArgs {
  const CT_G DevJob* jobs;      // nullptr: single job in `job`
  const CT_G int32_t* updOff;   // nJobs + 1 prefix sums of update items (nullptr for one job)
  const CT_G int32_t* filtOff;  // nJobs + 1 prefix sums of filter items
  const CT_G int32_t* prepList; // jobs that need a prep item (pops, or only pushes/pops)
  int32_t nJobs, nPrep, nUpd, nFilt;
  int32_t* queue;          // [0] head, [1] exit count, [2] launches, [3] error
  int32_t* hostErr;        // nullable: error word copied here by the last block
  // nullable: kernel timing on the device clock (wall_clock64): [0] earliest
  // workgroup start, [1] latest end, [2] workgroups done, [3] summed
  // durations, [4] timed launches
  unsigned long long* clock;
  DevJob job;
  uint64_t inl[INLINE_WORDS];
};

// ---------------------------------------------------------------------------
// Resident engine of a table's primary slot (synchronous calls).  One
// persistent workgroup keeps the slot's currTable, granule index, stamps,
// residues and last domains in LDS and takes calls from a mailbox in
// coherent pinned host memory; results go back the same way.
//
// Both directions use flagged slots: every 8-byte slot holds 32 bits of
// payload (high half) and the call's sequence number (low half), written by
// one aligned 64-bit store and read by one aligned 64-bit load, which are
// single-copy atomic on the host CPU and on the GPU.  A reader takes a
// message once every slot it needs carries the call's number, so no fence
// orders the slots against each other and the reader needs no second round
// trip after it has seen the flag.
// ---------------------------------------------------------------------------
constexpr int ENG_OP_PROPAGATE = 1, ENG_OP_STOP = 2;

// command slots: op, nPop, nPush, serialBase, depthAfter, wantCt, wantStats,
// one spare, then each domain word as two slots (low half first)
enum { EC_OP, EC_NPOP, EC_NPUSH, EC_SERIAL, EC_DEPTH, EC_WANTCT, EC_WANTST, EC_SPARE, EC_DOM };
constexpr int ENG_CMD_SLOTS = EC_DOM + 2 * ENG_MAX_D;

// result slots: status, call ticks, the slot's 8 counters (two slots each,
// written on calls that want them), then the domain words (written on OK)
enum { ER_STATUS, ER_TICKS, ER_STATS, ER_DOM = ER_STATS + 16 };
constexpr int ENG_RES_SLOTS = ER_DOM + 2 * ENG_MAX_D;

__host__ __device__ inline uint64_t eng_slot(uint32_t payload, uint32_t seq) {
  return ((uint64_t)payload << 32) | seq;
}

struct EngCmd {             // written by the host (every slot of a call)
  uint64_t slot[ENG_CMD_SLOTS];
};

struct EngRes {             // written by the engine
  uint64_t slot[ENG_RES_SLOTS];
  int32_t alive, exitSeq;        // written at exit (release)
  unsigned long long lifeTicks;  // written at exit: the launch's lifetime (device clock)
};

struct EngDesc {
  const CT_G TabDesc* tab;
  CT_G SlotDesc* slot;
  EngCmd* cmd;              // device pointers of the pinned host buffers
  EngRes* res;
  uint64_t* ctOut;          // pinned host buffer of W words (calls that want currTable)
  int64_t idleTicks;        // exit after this long without a call (device clock)
  int32_t startSeq, pad;    // the last call seq already answered
  // resident split schedule only: its control words in device memory
  // (SE_*, zeroed before each launch) and the filter workgroups
  int32_t* ctl;
  int32_t nFilt, pad2;
};

// Control words of the resident split schedule: the filter workgroups'
// count of finished calls, the number of the call workgroup 0 has taken
// (the filters' doorbell: they read the call from the mailbox once it is
// there), and the word every wait of the launch watches (the launch's error
// word: -1 once workgroup 0 has stopped, > 0 on a device error).
enum { SE_DONE = 1, SE_CALL = 2, SE_STOP = 3, SE_CTL_WORDS = 4 };
constexpr int SE_MAX_VAR_WORDS = 31;  // a filter wave reads its variable's input slots in one load

// Read-only view of a table's immutable parts (host code only): device
// supports, layout, branch policy and the device root state.
struct TableView {
  const uint64_t* S;        // device, rows x stride
  int64_t stride, W;
  int32_t n, D, rows, rootFailed, branchPolicy, kind;
  const VarDesc* vars;      // host, n
  const uint64_t* rootCt;   // device, W words
  const uint64_t* rootDom;  // device, D words
};

}  // namespace ctk
