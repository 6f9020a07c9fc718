// Host-side check of the output walk's step-end test (past_step in
// rtcdf_device.h) for output positions near 2^32: the step starting at p
// covers [p, p + span); a value end e >= p lies at or past the step's end iff
// e >= p + span in exact (64-bit) arithmetic.  The 32-bit form e <= p + span - 1
// that the walks used before wraps for p > 2^32 - span; the check counts its
// disagreements too, so the test shows the case it guards against.
#include <cstdint>
#include <cstdio>

#include "../../paper_2609_00843_amd/csrc/rtcdf_device.h"

int main() {
  const uint64_t top = 1ull << 32;
  uint64_t checked = 0, wrong = 0, old_wrong = 0;
  for (uint32_t span : {256u, 512u, 1024u}) {
    for (uint64_t p = top - 4 * span; p < top; ++p) {
      // every end position from p to 2^32 - 1, stepping densely near the step end
      for (uint64_t e = p; e < top; e += (e >= p + span - 2 && e <= p + span + 2) ? 1 : 7) {
        const bool want = e >= p + span;
        const bool got = rtcdf::dev::past_step((uint32_t)e, (uint32_t)p, span);
        const bool old_form = !((uint32_t)e <= (uint32_t)p + (span - 1));
        ++checked;
        wrong += got != want;
        old_wrong += old_form != want;
      }
    }
  }
  std::printf("checked %llu wrong %llu old_form_wrong %llu\n", (unsigned long long)checked,
              (unsigned long long)wrong, (unsigned long long)old_wrong);
  return wrong == 0 && old_wrong > 0 ? 0 : 1;
}
