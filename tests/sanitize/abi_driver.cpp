// Host-only driver of the C ABI, built with AddressSanitizer and UndefinedBehaviorSanitizer
// on the host side: every call below is rejected (or answered) before any device work, so
// it runs without a GPU.  Prints "ok" and exits 0 when every status is the expected one.
#include <stdio.h>
#include <string.h>

#include "ccm.h"

static int g_fail = 0;

static void expect(const char* what, ccm_status got, ccm_status want) {
  if (got != want) {
    printf("FAIL %s: status %d, expected %d (%s)\n", what, got, want, ccm_last_error());
    g_fail = 1;
  }
}

int main() {
  // fake, never dereferenced: every call below fails its argument checks first
  float* fp = (float*)0x1000;
  int32_t* ip = (int32_t*)0x2000;
  double* dp = (double*)0x3000;
  size_t bytes = 0;

  for (int op = CCM_OP_EMBED; op <= CCM_OP_CROSSMAP_TARGET_E; ++op) {
    expect("workspace_size", ccm_workspace_size(op, 1600, 512, 101729, 21, &bytes), CCM_OK);
    expect("workspace_size long", ccm_workspace_size(op, CCM_L_MAX, 64, 1000, 21, &bytes), CCM_OK);
  }
  expect("workspace_size null", ccm_workspace_size(CCM_OP_KNN, 10, 1, 1, 2, NULL), CCM_EINVAL);
  expect("workspace_size neg", ccm_workspace_size(CCM_OP_KNN, -1, 1, 1, 2, &bytes), CCM_EINVAL);
  expect("workspace_size op", ccm_workspace_size(99, 10, 1, 1, 2, &bytes), CCM_EINVAL);

  expect("embed null", ccm_embed(NULL, 4, 100, ip, 1, 2, 1, fp, NULL), CCM_EINVAL);
  expect("embed E", ccm_embed(fp, 4, 100, ip, 1, 21, 1, fp, NULL), CCM_ERANGE);
  expect("embed short", ccm_embed(fp, 4, 10, ip, 1, 6, 2, fp, NULL), CCM_ERANGE);
  expect("embed L", ccm_embed(fp, 4, CCM_L_MAX + 1, ip, 1, 2, 1, fp, NULL), CCM_ERANGE);

  expect("knn k_max", ccm_knn(fp, 4, 100, ip, ip, 1, 1, 0, 1, ip, fp, NULL, NULL, 0, NULL),
         CCM_EINVAL);
  expect("knn Tp", ccm_knn(fp, 4, 100, ip, ip, 1, 1, 100, 4, ip, fp, NULL, NULL, 0, NULL),
         CCM_EINVAL);
  expect("knn tau", ccm_knn(fp, 4, 100, ip, ip, 1, 0, 0, 4, ip, fp, NULL, NULL, 0, NULL),
         CCM_ERANGE);
  expect("knn_subset mask", ccm_knn_subset(fp, 4, 100, ip, ip, 1, 1, 0, 4, NULL, ip, fp, NULL,
                                           NULL, 0, NULL), CCM_EINVAL);

  expect("optE mode", ccm_simplex_optE(fp, 4, 100, ip, 1, 1, 5, 1, 1, 7, ip, fp, dp, 1 << 20,
                                       NULL), CCM_EINVAL);
  expect("optE range", ccm_simplex_optE(fp, 4, 100, ip, 1, 6, 5, 1, 1, 0, ip, fp, dp, 1 << 20,
                                        NULL), CCM_ERANGE);
  expect("optE points", ccm_simplex_optE(fp, 4, 30, ip, 1, 1, 20, 1, 1, 0, ip, fp, dp, 1 << 20,
                                         NULL), CCM_ERANGE);
  expect("optE ws", ccm_simplex_optE(fp, 4, 100, ip, 1, 1, 5, 1, 1, 0, ip, fp, dp, 8, NULL),
         CCM_EWORKSPACE);
  expect("optE noalloc size", ccm_simplex_optE_noalloc(fp, 4, 100, ip, CCM_NOALLOC_MAX_SERIES + 1,
                                                       1, 5, 1, 1, 0, ip, fp, NULL),
         CCM_ERANGE);
  expect("optE noalloc mode", ccm_simplex_optE_noalloc(fp, 4, 100, ip, 1, 1, 5, 1, 1, 7, ip, fp,
                                                       NULL),
         CCM_EINVAL);
  expect("optE noalloc empty", ccm_simplex_optE_noalloc(fp, 4, 100, ip, 0, 1, 5, 1, 1, 0, ip, fp,
                                                        NULL),
         CCM_OK);

  expect("crossmap precision", ccm_crossmap_rho(fp, 4, 100, ip, fp, ip, 1, 4, 1, 0, 4, 9, fp,
                                                NULL, dp, 1 << 20, NULL), CCM_EINVAL);
  expect("crossmap ld", ccm_crossmap_rho(fp, 4, 100, ip, fp, ip, 1, 4, 1, 2, 4, 0, fp, NULL, dp,
                                         1 << 20, NULL), CCM_EINVAL);
  expect("crossmap ws", ccm_crossmap_rho(fp, 4, 100, ip, fp, ip, 1, 4, 1, 0, 4, 0, fp, NULL, dp,
                                         8, NULL), CCM_EWORKSPACE);
  expect("crossmap ws bf16", ccm_crossmap_rho(fp, 4, 100, ip, fp, ip, 1, 4, 1, 0, 4, 1, fp, NULL,
                                              dp, 8, NULL), CCM_EWORKSPACE);
  // long series: 1 MB covers the tables but not the global copy of two 32-target tiles
  expect("crossmap long ws", ccm_crossmap_rho(fp, 64, CCM_L_MAX, ip, fp, ip, 1, 4, 1, 0, 64, 0,
                                              fp, NULL, dp, 1 << 20, NULL), CCM_EWORKSPACE);

  expect("target_E range", ccm_crossmap_rho_target_E(fp, 4, 100, ip, fp, 1, 0, 3, 4, 1, ip, 0, 4,
                                                     fp, NULL, dp, 1 << 20, NULL), CCM_ERANGE);
  expect("target_E k_max", ccm_crossmap_rho_target_E(fp, 4, 100, ip, fp, 1, 1, 5, 4, 1, ip, 0, 4,
                                                     fp, NULL, dp, 1 << 20, NULL), CCM_ERANGE);
  expect("target_E ws", ccm_crossmap_rho_target_E(fp, 4, 100, ip, fp, 1, 1, 3, 4, 1, ip, 0, 4,
                                                  fp, NULL, dp, 8, NULL), CCM_EWORKSPACE);

  expect("backward grads", ccm_crossmap_rho_backward(fp, 4, 100, fp, ip, fp, ip, 1, 4, 1, ip, ip,
                                                     fp, 1, NULL, NULL, dp, 1 << 20, NULL),
         CCM_EINVAL);
  expect("backward ws", ccm_crossmap_rho_backward(fp, 4, 100, fp, ip, fp, ip, 1, 4, 1, ip, ip,
                                                  fp, 1, fp, fp, dp, 8, NULL), CCM_EWORKSPACE);

  // the debug switch does not move the argument checks
  expect("check_finite on", ccm_set_check_finite(1), CCM_OK);
  expect("knn k_max (debug)", ccm_knn(fp, 4, 100, ip, ip, 1, 1, 0, 1, ip, fp, NULL, NULL, 0,
                                      NULL), CCM_EINVAL);
  expect("check_finite off", ccm_set_check_finite(0), CCM_OK);

  for (int s = 0; s <= 6; ++s)
    if (!ccm_status_string(s) || !strlen(ccm_status_string(s))) g_fail = 1;
  if (!ccm_last_error() || strncmp(ccm_version(), "ccm-gfx950", 10) != 0) g_fail = 1;
  if (!g_fail) printf("ok\n");
  return g_fail;
}
