// ct_split.cpp -- the split propagators (include/ct.h, ct_split_*): the two
// variants of Sec. 4 that put only one CT procedure on the device, kept for
// comparison with the library's propagators, which run the whole of
// enforceGAC (Alg. 1) there.
//
// The host half of each variant is CT's serial procedure over a host copy of
// the supports: a sparse bitset (the currTable words and the index of the
// non-zero ones, compacted after every variable's update, Alg. 2) for the
// filter variant, filterDomains with host residues (Alg. 3) for the update
// variant.  A call makes one host-to-device copy (blocking: the inputs have
// landed before the launch) and one launch whose workgroups write their
// results into coherent pinned host memory and then each publish the call's
// sequence number; the host waits for the stream and for every flag: the
// round trip that the paper measures for these variants (Sec. 5.2).  Backtracking saves the host state
// whole at every push.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ct.h"
#include "ct_device.h"

namespace ctk {
int table_view(const ct_table* t, TableView* v);
void set_error(const char* msg);
int split_update_grid(int64_t W);
int split_filter_grid(int nWords);
hipError_t launch_split_update(const uint64_t* S, int64_t stride, int64_t W, const int32_t* segBegin,
                               int nSeg, const int32_t* rowList, uint64_t* mask, int32_t* flags, int32_t seq,
                               hipStream_t stream);
hipError_t launch_split_filter(const uint64_t* S, int64_t stride, int64_t W, const uint64_t* ct,
                               const uint64_t* dom, const int32_t* words, int nWords, const int32_t* wordRow,
                               int32_t* res, uint64_t* domOut, int32_t* flags, int32_t seq, hipStream_t stream);
}  // namespace ctk

using namespace ctk;

namespace {

int sfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  set_error(buf);
  return code;
}

#define SPLITCHK(expr)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      s->poisoned = true;                                                                       \
      return sfail(CT_E_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                   __LINE__);                                                                   \
    }                                                                                           \
  } while (0)

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

struct SavedLevel {
  std::vector<uint64_t> ct, dom;
  std::vector<int32_t> sizes;
  bool failed;
};

}  // namespace

struct ct_split {
  int mode = 0;
  TableView v{};
  std::vector<VarDesc> vars;
  uint64_t* S = nullptr;  // rows x W, host copy of the supports (pinned: copied without staging)
  // host CT state
  std::vector<uint64_t> ct, lastDom;
  std::vector<int32_t> lastSizes, nz, res;  // nz: indexes of the non-zero currTable words
  bool failed = false, poisoned = false;
  std::vector<SavedLevel> levels;
  // per-call host scratch
  std::vector<uint64_t> dom;
  std::vector<int32_t> size, rowList, segBegin, words;
  std::vector<char> sVal, sSup;
  // device
  hipStream_t stream = nullptr;
  char* dStage = nullptr;  // one call's inputs
  char* pStage = nullptr;  // pinned mirror
  size_t stageBytes = 0;
  // results: written by the kernel straight into coherent pinned memory,
  // then one flag per workgroup set to the call's sequence number
  uint64_t* pOut = nullptr;
  uint64_t* dOut = nullptr;  // device address of pOut
  int32_t* pFlags = nullptr;
  int32_t* dFlags = nullptr;
  int32_t seq = 0;
  int32_t* dWordRow = nullptr;
  int32_t* dRes = nullptr;

  ~ct_split() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (dStage) (void)hipFree(dStage);
    if (dWordRow) (void)hipFree(dWordRow);
    if (dRes) (void)hipFree(dRes);
    if (pStage) (void)hipHostFree(pStage);
    if (pOut) (void)hipHostFree(pOut);
    if (pFlags) (void)hipHostFree(pFlags);
    if (S) (void)hipHostFree(S);
    if (stream) (void)hipStreamDestroy(stream);
  }

  int32_t var_size(const uint64_t* d, int i) const {
    int32_t c = 0;
    for (int k = 0; k < vars[i].domWords; ++k) c += __builtin_popcountll(d[vars[i].domOff + k]);
    return c;
  }
  const uint64_t* row(int r) const { return S + (size_t)r * v.W; }
};

namespace {

// Alg. 2 on the host's sparse bitset: for each changed variable the mask of
// its rows (removed values on the incremental branch, kept ones on the
// reset branch) is ANDed into the non-zero words only, then the index is
// compacted; stops at an empty currTable.
void host_update(ct_split* s) {
  const int n = s->v.n;
  for (int i = 0; i < n; ++i) {
    if (!s->sVal[i]) continue;
    const VarDesc& x = s->vars[i];
    int32_t delta = 0;
    for (int k = 0; k < x.domWords; ++k)
      delta += __builtin_popcountll(s->lastDom[x.domOff + k] & ~s->dom[x.domOff + k]);
    const bool inc = s->v.branchPolicy == CT_BRANCH_INCREMENTAL ||
                     (s->v.branchPolicy == CT_BRANCH_AUTO && delta < s->size[i]);
    s->rowList.clear();
    for (int a = 0; a < x.dsize; ++a) {
      const int k = x.domOff + a / 64;
      const bool was = (s->lastDom[k] >> (a % 64)) & 1ull, is = (s->dom[k] >> (a % 64)) & 1ull;
      if (inc ? (was && !is) : is) s->rowList.push_back(x.rowStart + a);
    }
    size_t keep = 0;
    for (size_t j = 0; j < s->nz.size(); ++j) {
      const int32_t w = s->nz[j];
      uint64_t m = 0;
      for (int32_t r : s->rowList) m |= s->row(r)[w];
      const uint64_t c = s->ct[w] & (inc ? ~m : m);
      s->ct[w] = c;
      if (c) s->nz[keep++] = w;
    }
    s->nz.resize(keep);
    if (keep == 0) break;
  }
}

// Alg. 3 on the host: residue word first, then the non-zero words in order.
void host_filter(ct_split* s) {
  for (int i = 0; i < s->v.n; ++i) {
    if (!s->sSup[i]) continue;
    const VarDesc& x = s->vars[i];
    for (int a = 0; a < x.dsize; ++a) {
      const int k = x.domOff + a / 64;
      if (!((s->dom[k] >> (a % 64)) & 1ull)) continue;
      const int r = x.rowStart + a;
      const uint64_t* R = s->row(r);
      if (s->ct[s->res[r]] & R[s->res[r]]) continue;
      int32_t found = -1;
      for (int32_t w : s->nz)
        if (s->ct[w] & R[w]) {
          found = w;
          break;
        }
      if (found >= 0)
        s->res[r] = found;
      else
        s->dom[k] &= ~(1ull << (a % 64));
    }
    s->lastSizes[i] = s->var_size(s->dom.data(), i);
  }
}

// Waits (bounded) until every one of the call's `grid` workgroups has
// published its outputs.
bool wait_flags(ct_split* s, int grid) {
  const auto t0 = std::chrono::steady_clock::now();
  for (int b = 0; b < grid; ++b) {
    int spins = 0;
    while (__atomic_load_n(&s->pFlags[b], __ATOMIC_ACQUIRE) != s->seq) {
      if (++spins % 1024 == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) return false;
    }
  }
  return true;
}

void rebuild_index(ct_split* s) {
  s->nz.clear();
  for (int64_t w = 0; w < s->v.W; ++w)
    if (s->ct[w]) s->nz.push_back((int32_t)w);
}

}  // namespace

extern "C" {

int ct_split_create(ct_table* t, int32_t mode, ct_split** out) {
  if (!out) return sfail(CT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (mode != CT_SPLIT_UPDATE && mode != CT_SPLIT_FILTER) return sfail(CT_E_INVALID, "unknown split mode %d", mode);
  TableView v{};
  int rc = table_view(t, &v);
  if (rc) return rc;
  if (v.kind != 0) return sfail(CT_E_INVALID, "the split propagators take positive tables");
  ct_split* s = new (std::nothrow) ct_split;
  if (!s) return sfail(CT_E_NOMEM, "host allocation failed");
  s->mode = mode;
  s->v = v;
  const int64_t W = v.W, D = v.D;
  try {
    s->vars.assign(v.vars, v.vars + v.n);
    s->ct.resize((size_t)W);
    s->lastDom.resize((size_t)D);
    s->dom.resize((size_t)D);
    s->lastSizes.resize(v.n);
    s->size.resize(v.n);
    s->sVal.resize(v.n);
    s->sSup.resize(v.n);
    s->res.assign((size_t)v.rows, 0);
    s->segBegin.reserve(v.n + 1);
    s->rowList.reserve(v.rows);
    s->words.reserve(D);
  } catch (const std::bad_alloc&) {
    delete s;
    return sfail(CT_E_NOMEM, "host allocation of the split state failed");
  }
#define CREATECHK(expr)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      (void)hipGetLastError();                                                                \
      delete s;                                                                               \
      return sfail(e_ == hipErrorOutOfMemory ? CT_E_NOMEM : CT_E_DEVICE, "%s failed: %s", #expr, \
                   hipGetErrorString(e_));                                                    \
    }                                                                                         \
  } while (0)
  CREATECHK(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
  // blocking copies into pinned host memory (no staging through a bounce
  // buffer): each has landed when the call returns
  CREATECHK(hipHostMalloc((void**)&s->S, sizeof(uint64_t) * std::max<size_t>((size_t)v.rows * (size_t)W, 1),
                          hipHostMallocDefault));
  if (W > 0 && v.rows > 0)
    CREATECHK(hipMemcpy2D(s->S, sizeof(uint64_t) * W, v.S, sizeof(uint64_t) * v.stride, sizeof(uint64_t) * W,
                          v.rows, hipMemcpyDeviceToHost));
  // stage: update variant = segment starts + row list;
  //        filter variant = currTable + domains + word list
  const size_t upd = align16(sizeof(int32_t) * (v.n + 1)) + align16(sizeof(int32_t) * (v.rows + 1)) +
                     align16(sizeof(uint64_t) * std::max<int64_t>(W, 1));
  const size_t flt = align16(sizeof(uint64_t) * std::max<int64_t>(W, 1)) + align16(sizeof(uint64_t) * D) +
                     align16(sizeof(int32_t) * D);
  s->stageBytes = mode == CT_SPLIT_UPDATE ? upd : flt;
  CREATECHK(hipMalloc((void**)&s->dStage, s->stageBytes));
  // the inputs' pinned mirror (coherent pinned memory, like the library's
  // other host buffers that the device reads or writes)
  CREATECHK(hipHostMalloc((void**)&s->pStage, s->stageBytes, hipHostMallocMapped | hipHostMallocCoherent));
  // the root state, through the pinned stage (it holds W and D words in either layout)
  if (W > 0) {
    CREATECHK(hipMemcpy(s->pStage, v.rootCt, sizeof(uint64_t) * W, hipMemcpyDeviceToHost));
    memcpy(s->ct.data(), s->pStage, sizeof(uint64_t) * W);
  }
  CREATECHK(hipMemcpy(s->pStage, v.rootDom, sizeof(uint64_t) * D, hipMemcpyDeviceToHost));
  memcpy(s->lastDom.data(), s->pStage, sizeof(uint64_t) * D);
  {
    const int64_t outWords = std::max<int64_t>(mode == CT_SPLIT_UPDATE ? W : D, 1);
    const int grid = std::max(mode == CT_SPLIT_UPDATE ? split_update_grid(std::max<int64_t>(W, 1))
                                                      : split_filter_grid((int)D), 1);
    CREATECHK(hipHostMalloc((void**)&s->pOut, sizeof(uint64_t) * outWords, hipHostMallocMapped | hipHostMallocCoherent));
    CREATECHK(hipHostMalloc((void**)&s->pFlags, sizeof(int32_t) * grid, hipHostMallocMapped | hipHostMallocCoherent));
    memset(s->pFlags, 0, sizeof(int32_t) * grid);
    CREATECHK(hipHostGetDevicePointer((void**)&s->dOut, s->pOut, 0));
    CREATECHK(hipHostGetDevicePointer((void**)&s->dFlags, s->pFlags, 0));
  }
  if (mode == CT_SPLIT_FILTER) {
    std::vector<int32_t> wordRow((size_t)D, 0);
    for (const VarDesc& x : s->vars)
      for (int k = 0; k < x.domWords; ++k) wordRow[x.domOff + k] = x.rowStart + 64 * k;
    CREATECHK(hipMalloc((void**)&s->dWordRow, sizeof(int32_t) * std::max<int64_t>(D, 1)));
    CREATECHK(hipMalloc((void**)&s->dRes, sizeof(int32_t) * std::max(v.rows, 1)));
    memcpy(s->pStage, wordRow.data(), sizeof(int32_t) * D);  // pinned source, no staging
    CREATECHK(hipMemcpy(s->dWordRow, s->pStage, sizeof(int32_t) * D, hipMemcpyHostToDevice));
    CREATECHK(hipMemset(s->dRes, 0, sizeof(int32_t) * std::max(v.rows, 1)));
  }
  CREATECHK(hipStreamSynchronize(nullptr));  // the memset above
#undef CREATECHK
  for (int i = 0; i < v.n; ++i) s->lastSizes[i] = s->var_size(s->lastDom.data(), i);
  s->failed = v.rootFailed != 0;
  rebuild_index(s);
  *out = s;
  return CT_OK;
}

void ct_split_destroy(ct_split* s) { delete s; }

int ct_split_propagate(ct_split* s, const uint64_t* dom_in, uint64_t* dom_out, uint64_t* ct_out) {
  if (!s) return sfail(CT_E_INVALID, "null split propagator");
  if (s->poisoned) return sfail(CT_E_DEVICE, "split propagator poisoned by an earlier device error");
  if (!dom_in) return sfail(CT_E_INVALID, "dom_in is NULL");
  if (s->failed) return sfail(CT_E_STATE, "propagator failed; only pop is allowed");
  const int n = s->v.n;
  const int64_t W = s->v.W, D = s->v.D;
  for (int i = 0; i < n; ++i) {
    const VarDesc& x = s->vars[i];
    const int tail = x.dsize % 64;
    if (tail && (dom_in[x.domOff + x.domWords - 1] >> tail))
      return sfail(CT_E_INVALID, "stray bits in the domain of variable %d", i);
  }
  for (int64_t k = 0; k < D; ++k)
    if (dom_in[k] & ~s->lastDom[k]) return sfail(CT_E_NOT_SUBSET, "domain word %lld gains values", (long long)k);
  std::copy(dom_in, dom_in + D, s->dom.begin());
  // Alg. 1: s_val (size differs from lastSizes) and s_sup (more than one value)
  bool anyVal = false;
  for (int i = 0; i < n; ++i) {
    s->size[i] = s->var_size(s->dom.data(), i);
    s->sVal[i] = s->size[i] != s->lastSizes[i];
    s->sSup[i] = s->size[i] > 1;
    anyVal |= s->sVal[i] != 0;
  }
  if (s->mode == CT_SPLIT_UPDATE && anyVal) {
    // the row list of every changed variable, on the branch Alg. 2 takes
    s->segBegin.clear();
    s->rowList.clear();
    for (int i = 0; i < n; ++i) {
      if (!s->sVal[i]) continue;
      const VarDesc& x = s->vars[i];
      int32_t delta = 0;
      for (int k = 0; k < x.domWords; ++k)
        delta += __builtin_popcountll(s->lastDom[x.domOff + k] & ~s->dom[x.domOff + k]);
      const bool inc = s->v.branchPolicy == CT_BRANCH_INCREMENTAL ||
                       (s->v.branchPolicy == CT_BRANCH_AUTO && delta < s->size[i]);
      const int32_t b = (int32_t)s->rowList.size();
      s->segBegin.push_back(inc ? -1 - b : b);
      for (int a = 0; a < x.dsize; ++a) {
        const int k = x.domOff + a / 64;
        const bool was = (s->lastDom[k] >> (a % 64)) & 1ull, is = (s->dom[k] >> (a % 64)) & 1ull;
        if (inc ? (was && !is) : is) s->rowList.push_back(x.rowStart + a);
      }
    }
    const int nSeg = (int)s->segBegin.size();
    s->segBegin.push_back((int32_t)s->rowList.size());
    const size_t oSeg = 0, oRows = align16(sizeof(int32_t) * (n + 1));
    memcpy(s->pStage + oSeg, s->segBegin.data(), sizeof(int32_t) * s->segBegin.size());
    memcpy(s->pStage + oRows, s->rowList.data(), sizeof(int32_t) * s->rowList.size());
    const size_t inBytes = oRows + sizeof(int32_t) * s->rowList.size();
    SPLITCHK(hipMemcpy(s->dStage, s->pStage, inBytes, hipMemcpyHostToDevice));  // landed on return
    ++s->seq;
    SPLITCHK(launch_split_update(s->v.S, s->v.stride, W, (const int32_t*)(s->dStage + oSeg), nSeg,
                                 (const int32_t*)(s->dStage + oRows), s->dOut, s->dFlags, s->seq, s->stream));
    SPLITCHK(hipStreamSynchronize(s->stream));
    if (!wait_flags(s, split_update_grid(W))) {
      s->poisoned = true;
      return sfail(CT_E_DEVICE, "split update: results not published");
    }
    const uint64_t* mask = s->pOut;
    size_t keep = 0;
    for (size_t j = 0; j < s->nz.size(); ++j) {
      const int32_t w = s->nz[j];
      const uint64_t c = s->ct[w] & mask[w];
      s->ct[w] = c;
      if (c) s->nz[keep++] = w;
    }
    s->nz.resize(keep);
  } else if (s->mode == CT_SPLIT_FILTER) {
    host_update(s);
  }
  for (int i = 0; i < n; ++i)
    if (s->sVal[i]) s->lastSizes[i] = s->size[i];
  // Alg. 1: failure test
  if (s->nz.empty()) {
    s->failed = true;
    if (ct_out && W > 0) memset(ct_out, 0, sizeof(uint64_t) * W);
    return CT_FAIL;
  }
  if (s->mode == CT_SPLIT_UPDATE) {
    host_filter(s);
  } else {
    s->words.clear();
    for (int i = 0; i < n; ++i)
      if (s->sSup[i])
        for (int k = 0; k < s->vars[i].domWords; ++k) s->words.push_back(s->vars[i].domOff + k);
    if (!s->words.empty()) {
      const size_t oCt = 0, oDom = align16(sizeof(uint64_t) * W), oWords = oDom + align16(sizeof(uint64_t) * D);
      memcpy(s->pStage + oCt, s->ct.data(), sizeof(uint64_t) * W);
      memcpy(s->pStage + oDom, s->dom.data(), sizeof(uint64_t) * D);
      memcpy(s->pStage + oWords, s->words.data(), sizeof(int32_t) * s->words.size());
      const size_t inBytes = oWords + sizeof(int32_t) * s->words.size();
      SPLITCHK(hipMemcpy(s->dStage, s->pStage, inBytes, hipMemcpyHostToDevice));  // landed on return
      ++s->seq;
      SPLITCHK(launch_split_filter(s->v.S, s->v.stride, W, (const uint64_t*)(s->dStage + oCt),
                                   (const uint64_t*)(s->dStage + oDom), (const int32_t*)(s->dStage + oWords),
                                   (int)s->words.size(), s->dWordRow, s->dRes, s->dOut, s->dFlags, s->seq,
                                   s->stream));
      SPLITCHK(hipStreamSynchronize(s->stream));
      if (!wait_flags(s, split_filter_grid((int)s->words.size()))) {
        s->poisoned = true;
        return sfail(CT_E_DEVICE, "split filter: results not published");
      }
      for (int32_t k : s->words) s->dom[k] = s->pOut[k];
      for (int i = 0; i < n; ++i)
        if (s->sSup[i]) s->lastSizes[i] = s->var_size(s->dom.data(), i);
    }
  }
  s->lastDom = s->dom;
  if (dom_out) std::copy(s->dom.begin(), s->dom.end(), dom_out);
  if (ct_out && W > 0) std::copy(s->ct.begin(), s->ct.end(), ct_out);
  return CT_OK;
}

int ct_split_push(ct_split* s) {
  if (!s) return sfail(CT_E_INVALID, "null split propagator");
  if (s->failed) return sfail(CT_E_STATE, "push on a failed propagator");
  try {
    s->levels.push_back(SavedLevel{s->ct, s->lastDom, s->lastSizes, s->failed});
  } catch (const std::bad_alloc&) {
    return sfail(CT_E_NOMEM, "host allocation of a level failed");
  }
  return CT_OK;
}

int ct_split_pop(ct_split* s) {
  if (!s) return sfail(CT_E_INVALID, "null split propagator");
  if (s->levels.empty()) return sfail(CT_E_STATE, "pop at depth 0");
  SavedLevel& L = s->levels.back();
  s->ct.swap(L.ct);
  s->lastDom.swap(L.dom);
  s->lastSizes.swap(L.sizes);
  s->failed = L.failed;
  s->levels.pop_back();
  rebuild_index(s);
  return CT_OK;
}

}  // extern "C"
