// cpu_parallel.cc -- multi-threaded CPU counting sort, a measurement baseline.
//
// TEST AND MEASUREMENT INFRASTRUCTURE ONLY: the benchmark times it on the host
// cores beside the single-core oracle, and the tests check it against the
// oracle (rtcdf_oracle.c).  It checks nothing itself and shares no code with
// the HIP path or with the oracle.
//
// It computes the sort of Sec. 2.1 (counts c_v, then every value v written
// over its output interval [s_v, s_v + c_v), s_v the exclusive prefix sum of
// the counts) with std::thread in three phases, each a fork/join:
//   1. count   -- thread t counts its contiguous slice of the input into its
//                 own histogram (no atomics, no sharing);
//   2. merge   -- thread t sums the per-thread histograms over its slice of
//                 the values, then the interval starts s_v are formed from a
//                 short serial scan of the slice totals;
//   3. fill    -- thread t writes output positions [tn/T, (t+1)n/T): it finds
//                 the value whose interval holds its first position by binary
//                 search over s, then writes whole runs.
#include <stdint.h>

#include <algorithm>
#include <thread>
#include <vector>

namespace {

constexpr int kOk = 0;
constexpr int kInvalidArgument = 1;
constexpr int kKeyOutOfRange = 2;

// Per-thread histograms may use at most this many bytes in total; above it the
// thread count is lowered (a range of 2^18 values allows 512 threads).
constexpr uint64_t kHistBudgetBytes = 1ull << 30;

template <class F>
void fork_join(int threads, F&& f) {
  std::vector<std::thread> pool;
  pool.reserve(threads - 1);
  for (int t = 1; t < threads; t++) pool.emplace_back(f, t);
  f(0);
  for (auto& th : pool) th.join();
}

}  // namespace

extern "C" {

// Sorts A[0, n) with every key in [minVal, maxVal) into B[0, n) using
// `threads` threads (at least 1; lowered when the per-thread histograms would
// exceed 1 GiB).  Returns 0, 1 for invalid arguments (empty or out-of-int32
// range, null pointers with n > 0, threads < 1) or 2 when a key lies outside
// the range; B is then unspecified.  *used (may be null) receives the thread
// count actually used.
int cpu_parallel_sort(const int32_t* A, uint64_t n, int64_t minVal, int64_t maxVal, int threads,
                      int32_t* B, int* used) {
  if (maxVal <= minVal || minVal < (int64_t)INT32_MIN || maxVal > (int64_t)INT32_MAX + 1)
    return kInvalidArgument;
  if (threads < 1 || (n > 0 && (A == nullptr || B == nullptr))) return kInvalidArgument;
  const uint64_t R = (uint64_t)(maxVal - minVal);
  const uint32_t min_u = (uint32_t)minVal;
  uint64_t T = (uint64_t)threads;
  T = std::min<uint64_t>(T, std::max<uint64_t>(1, kHistBudgetBytes / (8 * R)));
  T = std::min<uint64_t>(T, std::max<uint64_t>(1, n));  // no thread without keys
  if (used) *used = (int)T;
  if (n == 0) return kOk;

  std::vector<std::vector<uint64_t>> hist(T);
  std::vector<int> bad(T, 0);
  fork_join((int)T, [&](int t) {
    std::vector<uint64_t>& h = hist[t];
    h.assign(R, 0);
    const uint64_t i0 = n * t / T, i1 = n * (t + 1) / T;
    for (uint64_t i = i0; i < i1; i++) {
      const uint32_t x = (uint32_t)A[i] - min_u;  // v = A[i] - minVal, modulo 2^32
      if (x >= R) {
        bad[t] = 1;
        return;
      }
      h[x] += 1;
    }
  });
  for (uint64_t t = 0; t < T; t++)
    if (bad[t]) return kKeyOutOfRange;

  // s has R + 1 entries: s[v] = sum of c_u for u < v, s[R] = n.
  std::vector<uint64_t> s(R + 1);
  std::vector<uint64_t> part(T + 1, 0);
  fork_join((int)T, [&](int t) {
    const uint64_t v0 = R * t / T, v1 = R * (t + 1) / T;
    uint64_t run = 0;
    for (uint64_t v = v0; v < v1; v++) {
      uint64_t c = 0;
      for (uint64_t u = 0; u < T; u++) c += hist[u][v];
      s[v] = run;  // prefix within the slice; the slice base is added below
      run += c;
    }
    part[t + 1] = run;
  });
  for (uint64_t t = 0; t < T; t++) part[t + 1] += part[t];
  s[R] = part[T];
  hist.clear();
  hist.shrink_to_fit();
  fork_join((int)T, [&](int t) {
    const uint64_t v0 = R * t / T, v1 = R * (t + 1) / T;
    for (uint64_t v = v0; v < v1; v++) s[v] += part[t];
  });

  fork_join((int)T, [&](int t) {
    const uint64_t p0 = n * t / T, p1 = n * (t + 1) / T;
    if (p0 == p1) return;
    // the value whose interval [s_v, s_{v+1}) holds p0: the last v with s_v <= p0
    uint64_t v = (uint64_t)(std::upper_bound(s.begin(), s.begin() + R, p0) - s.begin()) - 1;
    uint64_t pos = p0;
    while (pos < p1) {
      const uint64_t end = std::min(s[v + 1], p1);
      std::fill(B + pos, B + end, (int32_t)(minVal + (int64_t)v));
      pos = end;
      v++;
    }
  });
  return kOk;
}

}  // extern "C"
