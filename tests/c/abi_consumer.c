/* A plain C99 consumer of the library: compiles against the public header only and
 * exercises the entry points that need no GPU (status text, sizes, FLOP counts,
 * defaults and argument checks). */
#include <stdio.h>
#include <string.h>

#include "riccsd.h"

static int fails = 0;
#define CHECK(cond)                                              \
  do {                                                           \
    if (!(cond)) {                                               \
      fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      ++fails;                                                   \
    }                                                            \
  } while (0)

int main(void) {
  ri_ccsd_opts opts;
  double dummy = 0.0;
  CHECK(strcmp(ri_status_str(RI_OK), "ok") == 0);
  CHECK(ri_ppl_flops(16, 256, 768) > 3.8e12 && ri_ppl_flops(16, 256, 768) < 3.9e12);
  CHECK(ri_ppl_flops(0, 256, 768) == 0.0);
  CHECK(ri_ppl_workspace_bytes(4, 24, 96, RI_PREC_FP64) > 0);
  CHECK(ri_ppl_workspace_bytes(4, 24, 96, RI_PREC_FP32) > 0);
  CHECK(ri_ppl_workspace_bytes(4, 24, 96, RI_PREC_BF16X3) > 0);
  CHECK(ri_ppl_workspace_bytes(4, 24, 96, 99) == 0);
  /* argument errors are reported before any device work */
  CHECK(ri_ppl(NULL, NULL, 2, 3, 4, NULL, NULL) == RI_E_ARG);
  CHECK(strlen(ri_last_error_msg()) > 0);
  CHECK(ri_ppl_shard(&dummy, &dummy, 2, 3, 4, &dummy, RI_PREC_FP64, 2, 2, NULL, 0, NULL) == RI_E_ARG);
  ri_ccsd_default_opts(&opts);
  CHECK(opts.max_iter == 100 && opts.diis_size == 6 && opts.guess == RI_GUESS_MP2);
  CHECK(opts.ppl_precision == RI_PREC_FP64 && opts.polish_precision == RI_PREC_FP64);
  CHECK(opts.other_precision == RI_PREC_FP64 && opts.mlp == NULL);
  CHECK(ri_ccsd_iterate(NULL, NULL, NULL, &opts, NULL, NULL) == RI_E_ARG);
  CHECK(ri_mlp_load("/nonexistent/net.bin") == NULL);
  if (fails) return 1;
  printf("c consumer ok\n");
  return 0;
}
