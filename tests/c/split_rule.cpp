// Host check of the contraction's split-count rule (no GPU): the launch model is a
// number of rounds of resident workgroups, each as long as one split's k range.
#include <cstdio>
#include <cstdlib>

#include "../../paper_1810_08142_amd/csrc/ppl_shared.h"

using ri::ppl::balance_splits;

static int fails = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::printf("FAILED at line %d: %s\n", __LINE__, #c);       \
      ++fails;                                                    \
    }                                                             \
  } while (0)

// modelled duration of a launch of nwg workgroups per split, `slots` resident at once
static double model(long nwg, long slots, long K, long step, long z) {
  long kz = (K + z - 1) / z;
  kz = (kz + step - 1) / step * step;
  const long launched = (K + kz - 1) / kz;
  const long rounds = (nwg * launched + slots - 1) / slots;
  return static_cast<double>(rounds) * kz;
}

int main() {
  const long K = 301056;  // cd slots of o=48 v=768 naux=2304
  // tau+ split contraction: 135 workgroups per split, one per CU; 19 splits leave a last
  // round of 5 workgroups, 24 splits fill 13 rounds to 97%
  CHECK(balance_splits(135, 256, K, 32, 19, 294) == 24);
  // tau- (already 11 nearly full rounds) keeps its count
  CHECK(balance_splits(162, 256, K, 32, 17, 294) == 17);
  // FP64 tau+: 208 workgroups per split, two per CU: 37 splits leave 16 in a last round
  CHECK(balance_splits(208, 512, K, 16, 37, 588) == 39);
  // the count never leaves [z0, zmax]
  CHECK(balance_splits(1000, 256, 4096, 32, 3, 3) == 3);
  CHECK(balance_splits(1, 256, 1 << 20, 32, 1, 1) == 1);
  // over a sweep: within the searched range, never slower than z0, within 3% of the
  // best of the range, and the smallest such count
  for (long nwg = 1; nwg <= 400; nwg += 7)
    for (long slots : {256L, 512L, 768L})
      for (long Kx : {34816L, 140032L, 301056L})
        for (long z0 : {1L, 4L, 17L, 37L}) {
          const long step = 32, zmax = Kx / (32 * step);
          if (z0 > zmax) continue;
          const long z = balance_splits(nwg, slots, Kx, step, z0, zmax);
          const long hi = zmax < (2 * z0 > z0 + 8 ? 2 * z0 : z0 + 8) ? zmax : (2 * z0 > z0 + 8 ? 2 * z0 : z0 + 8);
          CHECK(z >= z0 && z <= hi);
          double best = model(nwg, slots, Kx, step, z0);
          for (long y = z0; y <= hi; ++y)
            if (model(nwg, slots, Kx, step, y) < best) best = model(nwg, slots, Kx, step, y);
          CHECK(model(nwg, slots, Kx, step, z) <= model(nwg, slots, Kx, step, z0));
          CHECK(model(nwg, slots, Kx, step, z) <= 1.03 * best);
          for (long y = z0; y < z; ++y) CHECK(model(nwg, slots, Kx, step, y) > 1.03 * best);
        }
  if (fails == 0) std::printf("split rule ok\n");
  return fails == 0 ? 0 : 1;
}
