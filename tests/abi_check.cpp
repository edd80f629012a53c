// Host-side check of the C ABI's argument handling, built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host code of the library's entry-point
// files (device code is built as usual) and run on a machine with or without a
// GPU: every entry point is called with NULL handles, NULL pointers and
// out-of-range sizes, and must return its documented status without a memory
// error or undefined behaviour. Exit status 0 when every expectation holds.
// Built and run by tests/test_abi_sanitized.py.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "ftcg.h"

static int failures = 0;

#define EXPECT(call, want)                                                          \
  do {                                                                              \
    const ftcg_status got_ = (call);                                                \
    if (got_ != (want)) {                                                           \
      fprintf(stderr, "FAIL %s:%d %s -> %d, want %d\n", __FILE__, __LINE__, #call, \
              (int)got_, (int)(want));                                              \
      ++failures;                                                                   \
    }                                                                               \
  } while (0)

// a plan when the machine has a GPU, else NULL (creation then fails cleanly)
static ftcg_plan try_plan(int dim, int64_t n, ftcg_dtype dt, ftcg_wmode wm) {
  int64_t nn[2] = {n, n};
  ftcg_plan p = NULL;
  const ftcg_status s = ftcg_plan_create(&p, dim, nn, 6, 2.0, dt, wm, 8.0, NULL);
  if (s != FTCG_OK) {
    if (p != NULL) {
      fprintf(stderr, "FAIL plan handle set although creation failed (%d)\n", (int)s);
      ++failures;
    }
    return NULL;
  }
  return p;
}

int main() {
  // status strings: every code and an unknown one
  for (int s = -1; s <= 6; ++s) {
    const char* str = ftcg_status_string((ftcg_status)s);
    if (!str || !strlen(str)) {
      fprintf(stderr, "FAIL empty status string %d\n", s);
      ++failures;
    }
  }
  int64_t n[2] = {64, 64};
  ftcg_plan p = NULL;
  // plan creation: argument checks come before any device work
  EXPECT(ftcg_plan_create(NULL, 2, n, 6, 2.0, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, NULL, 6, 2.0, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 3, n, 6, 2.0, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  int64_t odd[2] = {63, 63}, tiny[2] = {4, 4}, huge[2] = {16384, 16384}, uneq[2] = {64, 32};
  EXPECT(ftcg_plan_create(&p, 2, odd, 6, 2.0, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, tiny, 6, 2.0, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, huge, 6, 2.0, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, uneq, 6, 2.0, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EUNSUPPORTED);
  EXPECT(ftcg_plan_create(&p, 2, n, 1, 2.0, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, n, 9, 2.0, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, n, 6, 1.0, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, n, 6, 0.0 / 0.0, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, n, 6, 1.7, FTCG_F32, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, n, 6, 2.0, (ftcg_dtype)7, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, n, 6, 2.0, FTCG_F32, (ftcg_wmode)9, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, n, 6, 2.0, FTCG_F32, FTCG_W_PLAIN, 0.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 2, n, 6, 2.0, FTCG_F32, FTCG_W_PLAIN, 65.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_plan_create(&p, 1, n, 6, 2.0, FTCG_F32, FTCG_W_LEARNED, 8.0, NULL), FTCG_EUNSUPPORTED);
  if (p != NULL) {
    fprintf(stderr, "FAIL plan handle set by a rejected creation\n");
    ++failures;
  }
  // every plan call with a NULL plan
  double d = 0.0;
  int i = 0;
  int64_t l = 0;
  char buf[64];
  EXPECT(ftcg_plan_destroy(NULL), FTCG_EINVAL);
  EXPECT(ftcg_set_points(NULL, 4, &d), FTCG_EINVAL);
  EXPECT(ftcg_set_weights(NULL, &d), FTCG_EINVAL);
  EXPECT(ftcg_get_weights(NULL, &d, &i), FTCG_EINVAL);
  EXPECT(ftcg_execute(NULL, buf, buf), FTCG_EINVAL);
  EXPECT(ftcg_forward(NULL, buf, buf), FTCG_EINVAL);
  EXPECT(ftcg_frame_approx(NULL, 4, &d, buf, buf), FTCG_EINVAL);
  EXPECT(ftcg_plan_set_density_iterations(NULL, 5), FTCG_EINVAL);
  EXPECT(ftcg_plan_set_band(NULL, 2), FTCG_EINVAL);
  EXPECT(ftcg_get_band(NULL, &d, &i), FTCG_EINVAL);
  EXPECT(ftcg_spread_only(NULL, buf, buf), FTCG_EINVAL);
  EXPECT(ftcg_grid_to_image(NULL, buf, buf), FTCG_EINVAL);
  EXPECT(ftcg_plan_info(NULL, &l, &l, &l, &i), FTCG_EINVAL);
  EXPECT(ftcg_plan_set_tuning(NULL, 32, 0, 1), FTCG_EINVAL);
  EXPECT(ftcg_plan_set_weight_tuning(NULL, 0, 0), FTCG_EINVAL);
  EXPECT(ftcg_plan_set_spread_layout(NULL, 0), FTCG_EINVAL);
  EXPECT(ftcg_plan_enable_timing(NULL, 1), FTCG_EINVAL);
  EXPECT(ftcg_plan_timing(NULL, &d, &l), FTCG_EINVAL);
  EXPECT(ftcg_plan_set_mlp(NULL, NULL, 1e-4, 16), FTCG_EINVAL);
  EXPECT(ftcg_plan_learned_report(NULL, &d, &i), FTCG_EINVAL);
  // the allocation-free call: argument checks and the workspace limit come first
  EXPECT(ftcg_grid_to_image_noalloc(2, 64, 6, 2.0, FTCG_F32, NULL, buf, NULL), FTCG_EINVAL);
  EXPECT(ftcg_grid_to_image_noalloc(3, 64, 6, 2.0, FTCG_F32, buf, buf, NULL), FTCG_EINVAL);
  EXPECT(ftcg_grid_to_image_noalloc(2, 2048, 6, 2.0, FTCG_F32, buf, buf, NULL), FTCG_EUNSUPPORTED);
  EXPECT(ftcg_grid_to_image_noalloc(2, 64, 6, 1.5, FTCG_F32, buf, buf, NULL), FTCG_EUNSUPPORTED);
  // networks and batches
  ftcg_mlp net = NULL;
  EXPECT(ftcg_mlp_create(NULL, NULL), FTCG_EINVAL);
  EXPECT(ftcg_mlp_destroy(NULL), FTCG_EINVAL);
  EXPECT(ftcg_mlp_set_params(NULL, (const float*)buf, FTCG_MLP_NPARAM), FTCG_EINVAL);
  EXPECT(ftcg_mlp_get_params(NULL, (float*)buf, FTCG_MLP_NPARAM), FTCG_EINVAL);
  size_t sz = 0;
  EXPECT(ftcg_mlp_save(NULL, NULL, &sz), FTCG_EINVAL);
  EXPECT(ftcg_mlp_load(NULL, buf, 8), FTCG_EINVAL);
  EXPECT(ftcg_mlp_forward(NULL, 1, (const float*)buf, (float*)buf), FTCG_EINVAL);
  ftcg_batch b = NULL;
  EXPECT(ftcg_batch_create(NULL, 1, n, 6, 2.0, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_batch_create(&b, 0, n, 6, 2.0, FTCG_W_PLAIN, 8.0, NULL), FTCG_EINVAL);
  EXPECT(ftcg_batch_create(&b, 1, n, 6, 2.0, FTCG_W_BAND, 8.0, NULL), FTCG_EUNSUPPORTED);
  EXPECT(ftcg_batch_create(&b, 1, n, 6, 2.0, FTCG_W_DENSITY, 8.0, NULL), FTCG_EUNSUPPORTED);
  EXPECT(ftcg_batch_destroy(NULL), FTCG_EINVAL);
  EXPECT(ftcg_batch_info(NULL, &l, &l, &l, &l), FTCG_EINVAL);
  EXPECT(ftcg_batch_execute(NULL, buf, buf), FTCG_EINVAL);
  // with a device: a real plan's state errors (no GPU: creation fails cleanly)
  ftcg_plan q = try_plan(2, 64, FTCG_F32, FTCG_W_PLAIN);
  if (q) {
    EXPECT(ftcg_execute(q, buf, buf), FTCG_ESTATE);
    EXPECT(ftcg_forward(q, buf, buf), FTCG_ESTATE);
    EXPECT(ftcg_set_weights(q, &d), FTCG_ESTATE);
    EXPECT(ftcg_plan_set_band(q, 2), FTCG_ESTATE);
    EXPECT(ftcg_plan_set_density_iterations(q, 5), FTCG_ESTATE);
    EXPECT(ftcg_set_points(q, 0, &d), FTCG_EINVAL);
    EXPECT(ftcg_plan_set_tuning(q, 48, 0, 1), FTCG_EINVAL);
    EXPECT(ftcg_plan_set_tuning(q, 32, 2, 1), FTCG_EINVAL);
    EXPECT(ftcg_plan_set_weight_tuning(q, 3, 0), FTCG_EINVAL);
    EXPECT(ftcg_plan_set_spread_layout(q, 2), FTCG_EINVAL);
    EXPECT(ftcg_plan_set_spread_layout(q, -1), FTCG_EINVAL);
    EXPECT(ftcg_frame_approx(q, 4, &d, buf, buf), FTCG_EUNSUPPORTED);   // float32 plan
    EXPECT(ftcg_plan_destroy(q), FTCG_OK);
  }
  (void)net;
  printf("abi_check: %d failure(s)\n", failures);
  return failures == 0 ? 0 : 1;
}
