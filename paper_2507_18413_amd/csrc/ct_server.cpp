// ct_server.cpp -- serving loop: continuous batching of propagate requests
// from many concurrent searches (include/ct.h, "Serving").
//
// Built only on the library's public C ABI: every propagation is a job of
// ct_propagate_batch.  One server thread moves requests from a submission
// queue to per-search FIFO queues, launches a batch on each free stream with
// the head request of every search that has none in flight (admitting new
// searches into slots while the memory budget allows), and harvests finished
// batches into the completion queue.  With two streams a batch is being
// built and launched while the previous one runs, so requests that arrive
// meanwhile join the next launch instead of waiting for a whole queue to
// drain.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ct.h"

namespace ctk {
// internal accessors of the runtime (ct_runtime.cpp)
int64_t slot_footprint(const ct_table* t, int max_depth);
int root_domains(ct_table* t, uint64_t* out);
void set_error(const char* msg);
}  // namespace ctk

namespace {

constexpr int DW = 64;  // domain words per request in the staging buffers
constexpr unsigned kPinned = hipHostMallocMapped | hipHostMallocCoherent;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SReq {
  ct_request r{};
  std::vector<uint64_t> remove;
  double tSubmit = 0;
};

struct Search {
  ct_table* T = nullptr;
  int maxDepth = 0, D = 0, tab = -1;
  int slot = -1;
  bool busy = false, fresh = true;
  int8_t failed = 0;
  std::vector<uint64_t> dom;
  std::vector<std::vector<uint64_t>> stack;
  std::vector<int8_t> failedAt;
  std::deque<SReq> q;
};

struct TableInfo {
  ct_table* T = nullptr;
  std::vector<uint64_t> root;
  int64_t slotBytes = 0;
  int maxDepth = 0;
};

struct Flight {
  bool busy = false;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  // pinned host buffers, read and written by the batch's kernels in place
  // (d* = their device addresses): no copies around a batch
  uint64_t *pIn = nullptr, *pOut = nullptr, *dIn = nullptr, *dOut = nullptr;
  int32_t *pStatus = nullptr, *dStatus = nullptr;
  std::vector<int> searches;
  std::vector<SReq> reqs;
  double tLaunch = 0;
};

}  // namespace

struct ct_server {
  ct_server_cfg cfg{};
  std::mutex mu;                 // submissions, completions, searches list
  std::condition_variable cvIn, cvOut;
  std::vector<SReq> incoming;
  std::deque<ct_completion> done;
  std::vector<Search> searches;  // grows only under mu; the thread reads sizes under mu
  std::vector<TableInfo> tables;
  std::map<ct_table*, int> tableIndex;
  std::vector<Flight> flights;
  std::thread th;
  std::atomic<bool> stop{false};
  std::atomic<bool> broken{false};
  std::atomic<int64_t> stats[CT_SERVER_NSTATS] = {};
  size_t rr = 0;  // round-robin start for fairness
  bool started = false;  // first request submitted: the search list is fixed
};

namespace {

void complete(ct_server* s, const SReq& q, int status, double tLaunch) {
  ct_completion c{};
  c.tag = q.r.tag;
  c.search = q.r.search;
  c.status = status;
  c.t_submit = q.tSubmit;
  c.t_launch = tLaunch;
  c.t_done = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  s->done.push_back(c);
  s->stats[0]++;
  s->cvOut.notify_all();
}

void release_slot(ct_server* s, Search& S) {
  if (S.slot < 0) return;
  TableInfo& ti = s->tables[S.tab];
  // the slot goes back to the table (ct_slots_alloc reuses it); its last
  // batch has completed (harvested)
  (void)ct_slots_free(ti.T, S.slot, 1);
  s->stats[3] -= ti.slotBytes;
  S.slot = -1;
  S.fresh = true;
  S.failed = 0;
  S.dom = ti.root;
  S.stack.clear();
  S.failedAt.clear();
}

// Slot for a search: a free slot of its table, or a new one within budget.
bool admit(ct_server* s, Search& S) {
  if (S.slot >= 0) return true;
  TableInfo& ti = s->tables[S.tab];
  const int64_t budget = s->cfg.mem_budget;
  // within budget, and always at least one search so that work can proceed
  if (budget > 0 && s->stats[3] > 0 && s->stats[3] + ti.slotBytes > budget) return false;
  // a slot freed by an earlier search of the table is reused
  ct_layout_info before{};
  if (ct_layout(ti.T, &before, nullptr) != CT_OK) return false;
  int32_t slot = -1;
  if (ct_slots_alloc(ti.T, 1, ti.maxDepth, &slot) != CT_OK) return false;
  if (slot >= before.n_slots) s->stats[5]++;
  S.slot = slot;
  s->stats[3] += ti.slotBytes;
  s->stats[4] = std::max(s->stats[4].load(), s->stats[3].load());
  S.fresh = true;
  S.dom = ti.root;
  return true;
}

void harvest(ct_server* s, Flight& f) {
  for (size_t i = 0; i < f.searches.size(); ++i) {
    Search& S = s->searches[f.searches[i]];
    const SReq& q = f.reqs[i];
    const int st = f.pStatus[i];
    if (st == CT_OK) {
      memcpy(S.dom.data(), f.pOut + (size_t)i * DW, sizeof(uint64_t) * S.D);
      if (q.r.dom_out) memcpy(q.r.dom_out, S.dom.data(), sizeof(uint64_t) * S.D);
    } else if (st == CT_FAIL) {
      S.failed = 1;
    }
    S.busy = false;
    if (q.r.flags & CT_REQ_FINISH) release_slot(s, S);
    complete(s, q, st, f.tLaunch);
  }
  f.searches.clear();
  f.reqs.clear();
  f.busy = false;
}

// Build and launch one batch on flight f; returns the number of requests.
int launch(ct_server* s, Flight& f) {
  const int maxBatch = s->cfg.max_batch;
  std::vector<ct_job> jobs;
  const size_t nS = s->searches.size();
  for (size_t k = 0; k < nS && (int)jobs.size() < maxBatch; ++k) {
    const size_t si = (s->rr + k) % nS;
    Search& S = s->searches[si];
    if (S.busy || S.q.empty()) continue;
    SReq& q = S.q.front();
    if (S.slot < 0 && !admit(s, S)) {
      s->stats[2]++;
      continue;
    }
    // host mirror of the search's domain stack: pops, then the push
    const int n_pop = q.r.n_pop, push = q.r.push ? 1 : 0;
    int bad = CT_OK;
    if (n_pop < 0 || n_pop > (int)S.stack.size()) bad = CT_E_STATE;
    else if (S.fresh && (n_pop || push)) bad = CT_E_INVALID;
    else if ((int)S.stack.size() - n_pop + push > S.maxDepth) bad = CT_E_NOMEM;
    if (bad != CT_OK) {
      SReq r = q;
      S.q.pop_front();
      if (r.r.flags & CT_REQ_FINISH) release_slot(s, S);
      complete(s, r, bad, now_s());
      continue;
    }
    for (int p = 0; p < n_pop; ++p) {
      S.dom = S.stack.back();
      S.stack.pop_back();
      S.failed = S.failedAt.back();
      S.failedAt.pop_back();
    }
    if (push) {
      S.stack.push_back(S.dom);
      S.failedAt.push_back(S.failed);
    }
    const size_t i = jobs.size();
    uint64_t* in = f.pIn + i * DW;
    for (int w = 0; w < S.D; ++w) in[w] = S.dom[w] & (q.remove.empty() ? ~0ull : ~q.remove[w]);
    ct_job j{};
    j.table = S.T;
    j.slot = S.slot;
    j.flags = CT_JOB_PROPAGATE | (S.fresh ? CT_JOB_FROM_ROOT : 0u);
    j.n_pop = S.fresh ? 0 : n_pop;
    j.n_push = S.fresh ? 0 : push;
    j.dom_in = f.dIn + i * DW;
    j.dom_out = f.dOut + i * DW;
    j.ct_out = nullptr;
    jobs.push_back(j);
    S.fresh = false;
    S.busy = true;
    f.searches.push_back((int)si);
    f.reqs.push_back(std::move(q));
    S.q.pop_front();
  }
  s->rr = nS ? (s->rr + 1) % nS : 0;
  const int n = (int)jobs.size();
  if (n == 0) return 0;
  f.tLaunch = now_s();
  int rc = ct_propagate_batch(jobs.data(), n, f.stream, f.dStatus);
  if (rc == CT_OK && hipEventRecord(f.ev, f.stream) != hipSuccess) rc = CT_E_DEVICE;
  if (rc != CT_OK) {
    s->broken = true;
    for (size_t k = 0; k < f.reqs.size(); ++k) {
      s->searches[f.searches[k]].busy = false;
      complete(s, f.reqs[k], rc, f.tLaunch);
    }
    f.searches.clear();
    f.reqs.clear();
    return 0;
  }
  f.busy = true;
  s->stats[1]++;
  if (n >= 2) {
    s->stats[6]++;
    for (int k = 1; k < n; ++k)
      if (jobs[k].table != jobs[0].table) {
        s->stats[7]++;
        break;
      }
  }
  s->stats[8] = std::max<int64_t>(s->stats[8].load(), n);
  return n;
}

void server_loop(ct_server* s) {
  // the search list is fixed once the first request arrives
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cvIn.wait(lk, [&] { return s->started || s->stop.load(); });
  }
  for (;;) {
    std::vector<SReq> in;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      in.swap(s->incoming);
    }
    for (SReq& q : in) s->searches[q.r.search].q.push_back(std::move(q));
    bool progress = !in.empty();
    bool inFlight = false;
    for (Flight& f : s->flights) {
      if (f.busy && hipEventQuery(f.ev) == hipSuccess) {
        harvest(s, f);
        progress = true;
      }
    }
    if (!s->broken) {
      for (Flight& f : s->flights)
        if (!f.busy && launch(s, f) > 0) progress = true;
    }
    for (Flight& f : s->flights) inFlight |= f.busy;
    if (s->stop && !inFlight) break;
    if (!progress) {
      if (inFlight) {
        // a batch is running: poll its event again at once (a timed wait
        // would sleep for the kernel's timer slack, tens of microseconds,
        // after the batch ends)
        std::this_thread::yield();
        continue;
      }
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->incoming.empty() && !s->stop) s->cvIn.wait_for(lk, std::chrono::microseconds(200));
    }
  }
}

}  // namespace

extern "C" {

double ct_server_now(void) { return now_s(); }

int ct_server_create(const ct_server_cfg* cfg, ct_server** out) {
  if (!out) return CT_E_INVALID;
  *out = nullptr;
  ct_server* s = new (std::nothrow) ct_server();
  if (!s) return CT_E_NOMEM;
  if (cfg) s->cfg = *cfg;
  if (s->cfg.max_batch <= 0) s->cfg.max_batch = 1024;
  if (s->cfg.streams <= 0) s->cfg.streams = 2;
  s->flights.resize(s->cfg.streams);
  const size_t words = (size_t)DW * s->cfg.max_batch;
  for (Flight& f : s->flights) {
    bool ok = hipStreamCreateWithFlags(&f.stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&f.ev, hipEventDisableTiming) == hipSuccess &&
              hipHostMalloc((void**)&f.pIn, sizeof(uint64_t) * words, kPinned) == hipSuccess &&
              hipHostMalloc((void**)&f.pOut, sizeof(uint64_t) * words, kPinned) == hipSuccess &&
              hipHostMalloc((void**)&f.pStatus, sizeof(int32_t) * s->cfg.max_batch, kPinned) == hipSuccess &&
              hipHostGetDevicePointer((void**)&f.dIn, f.pIn, 0) == hipSuccess &&
              hipHostGetDevicePointer((void**)&f.dOut, f.pOut, 0) == hipSuccess &&
              hipHostGetDevicePointer((void**)&f.dStatus, f.pStatus, 0) == hipSuccess;
    if (!ok) {
      ct_server_destroy(s);
      ctk::set_error("server resource allocation failed");
      return CT_E_NOMEM;
    }
  }
  s->th = std::thread(server_loop, s);
  *out = s;
  return CT_OK;
}

void ct_server_destroy(ct_server* s) {
  if (!s) return;
  s->stop = true;
  s->cvIn.notify_all();
  if (s->th.joinable()) s->th.join();
  for (Flight& f : s->flights)
    if (f.stream) (void)hipStreamSynchronize(f.stream);
  // slots still held by searches go back to their tables
  for (Search& S : s->searches)
    if (S.slot >= 0) (void)ct_slots_free(S.T, S.slot, 1);
  for (Flight& f : s->flights) {
    if (f.pIn) (void)hipHostFree(f.pIn);
    if (f.pOut) (void)hipHostFree(f.pOut);
    if (f.pStatus) (void)hipHostFree(f.pStatus);
    if (f.ev) (void)hipEventDestroy(f.ev);
    if (f.stream) (void)hipStreamDestroy(f.stream);
  }
  delete s;
}

int ct_server_add_search(ct_server* s, ct_table* t, int32_t max_depth, int32_t* search) {
  if (!s || !t || max_depth < 0) return CT_E_INVALID;
  // the lock is held from the check of `started` to the end: a first submit
  // on another thread cannot slip in between (the server thread reads the
  // search list without the lock once started)
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->started) {
    ctk::set_error("searches are added before the first request");
    return CT_E_STATE;
  }
  ct_layout_info info{};
  int rc = ct_layout(t, &info, nullptr);
  if (rc) return rc;
  if (info.D > DW) {
    ctk::set_error("tables served must have at most 64 domain words");
    return CT_E_INVALID;
  }
  auto it = s->tableIndex.find(t);
  int tab;
  if (it == s->tableIndex.end()) {
    TableInfo ti;
    ti.T = t;
    ti.maxDepth = max_depth;
    ti.root.assign(info.D, 0);
    if ((rc = ctk::root_domains(t, ti.root.data()))) return rc;
    ti.slotBytes = ctk::slot_footprint(t, max_depth);
    tab = (int)s->tables.size();
    s->tables.push_back(ti);
    s->tableIndex[t] = tab;
  } else {
    tab = it->second;
    if (s->tables[tab].maxDepth != max_depth) {
      ctk::set_error("all searches of a table share one max_depth");
      return CT_E_INVALID;
    }
  }
  Search S;
  S.T = t;
  S.tab = tab;
  S.maxDepth = max_depth;
  S.D = info.D;
  S.dom = s->tables[tab].root;
  if (search) *search = (int32_t)s->searches.size();
  s->searches.push_back(std::move(S));
  return CT_OK;
}

int ct_server_submit(ct_server* s, const ct_request* req) {
  if (!s || !req) return CT_E_INVALID;
  SReq q;
  q.r = *req;
  q.tSubmit = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  s->started = true;
  if (req->search < 0 || req->search >= (int)s->searches.size()) {
    ctk::set_error("unknown search");
    return CT_E_INVALID;
  }
  if (req->remove) q.remove.assign(req->remove, req->remove + s->searches[req->search].D);
  q.r.remove = nullptr;
  s->incoming.push_back(std::move(q));
  s->cvIn.notify_one();
  return CT_OK;
}

int ct_server_poll(ct_server* s, ct_completion* out, int32_t max, int32_t wait_us) {
  if (!s || (max > 0 && !out)) return CT_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_us > 0)
    s->cvOut.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return !s->done.empty(); });
  int n = 0;
  while (n < max && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.pop_front();
  }
  return n;
}

int ct_server_stats(ct_server* s, int64_t* out, int32_t n) {
  if (!s || !out || n < 0) return CT_E_INVALID;
  for (int k = 0; k < n && k < CT_SERVER_NSTATS; ++k) out[k] = s->stats[k].load();
  return CT_OK;
}

}  // extern "C"
