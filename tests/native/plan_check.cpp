// Host check of the force-pass plan (plan_layout in csrc/common.h): for a
// grid of cluster sizes, block sizes, slicing targets and thresholds, the
// 32-bit and 64-bit forms agree wherever the 32-bit form is taken, and every
// plan covers its block and its cluster exactly once within the row budget.
// Prints "ok" and exits 0, or names the first failing case and exits 1.
#include <stdio.h>
#include <stdint.h>
#include "common.h"

using namespace nb;

static int fail(const char* what, int64_t na, int64_t nn, int64_t tgt) {
  printf("FAIL %s: na=%lld nn=%lld target=%lld\n", what, (long long)na, (long long)nn, (long long)tgt);
  return 1;
}

static bool same(const Plan& a, const Plan& b) {
  return a.n_act == b.n_act && a.variant == b.variant && a.chunks == b.chunks && a.slices == b.slices &&
         a.slice_len == b.slice_len && a.red_tp == b.red_tp;
}

int main() {
  const int64_t big = (int64_t)1 << 30;
  const int32_t th_default[9] = {1024, 1024, 48, 12, (int32_t)big, (int32_t)big, 24, 6, 16384};
  const int32_t th_all[9] = {1, 1, 1, 1, 1, 1, 1, 1, 0};
  const int32_t th_split[9] = {(int32_t)big, (int32_t)big, 8, 2, (int32_t)big, (int32_t)big, 8, 2, 0};
  const int32_t* ths[3] = {th_default, th_all, th_split};
  // up to the library's limit on the particle count (kMaxParticles)
  const int64_t sizes[] = {1, 2, 255, 256, 257, 1000, 4096, 65536, 262144, ((int64_t)1 << 26) - 1,
                           (int64_t)1 << 26, kMaxParticles - 1, kMaxParticles};
  const int64_t targets[] = {1, 8, 2048, 16384};
  long cases = 0;
  for (const int32_t* th : ths)
    for (int64_t nn : sizes)
      for (int64_t tgt : targets)
        for (int64_t na : {(int64_t)0, (int64_t)1, (int64_t)5, (int64_t)47, (int64_t)1023, (int64_t)4096, nn / 3,
                           nn - 1, nn}) {
          if (na < 0 || na > nn) continue;
          Plan P{}, Q{};
          plan_layout(na, nn, tgt, th, P);
          plan_layout_t<int64_t>(na, nn, tgt, th, Q);
          ++cases;
          if (!same(P, Q)) return fail("32-bit and 64-bit plans differ", na, nn, tgt);
          if (P.n_act != na) return fail("block size", na, nn, tgt);
          if (P.variant < 0 || P.variant >= kNumVariants) return fail("layout", na, nn, tgt);
          const int64_t iwg = variant_iwg(P.variant);
          if ((int64_t)P.chunks * iwg < na || (na > 0 && (int64_t)(P.chunks - 1) * iwg >= na))
            return fail("i-chunks do not cover the block exactly", na, nn, tgt);
          if (P.slices < 1 || P.slice_len < kTile || P.slice_len % kTile != 0)
            return fail("slice shape", na, nn, tgt);
          if ((int64_t)P.slices * P.slice_len < nn || (int64_t)(P.slices - 1) * P.slice_len >= nn)
            return fail("j-slices do not cover the cluster exactly", na, nn, tgt);
          if ((int64_t)P.slices * na > kRowsPerParticle * nn + kRowsPerCluster)
            return fail("partial rows over budget", na, nn, tgt);
          if (P.red_tp < 1 || P.red_tp > 256 || (P.red_tp & (P.red_tp - 1)) != 0 ||
              (na < kReduceSerialBlock && P.red_tp < 256 && P.red_tp < P.slices) ||
              (na >= kReduceSerialBlock && P.red_tp != 1))
            return fail("reduce lanes", na, nn, tgt);
          const int64_t epw = 256 / P.red_tp;
          if (plan_units(P) * epw < na || (na > 0 && (plan_units(P) - 1) * epw >= na))
            return fail("reduce units do not cover the block exactly", na, nn, tgt);
        }
  printf("ok %ld cases\n", cases);
  return 0;
}
