// Replayed against the HIP stand-in (asan_hip_stub.cpp): the same batch
// (square m = 2..14, n = m + 1, 80 q x 8 primes) submitted again and again on
// one workspace must be captured once; every later call replays the cached
// graph.  Prints the number of captures.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <hip/hip_runtime_api.h>
#include "chromstrip.h"
extern "C" long hip_stub_captures(void);

int main() {
  const uint32_t primes[8] = {2147483647u, 998244353u, 1000000007u, 2147483629u,
                              2147483587u, 1000000009u, 998244853u, 2147483563u};
  std::vector<uint32_t> q(80);
  for (int k = 0; k < 80; ++k) q[k] = k + 1;
  std::vector<chrom_job> jobs;
  std::vector<void*> outs;
  for (int m = 2; m <= 14; ++m) {
    void* o = nullptr;
    if (hipMalloc(&o, static_cast<size_t>(m + 1) * 640 * 4) != hipSuccess) return 1;
    outs.push_back(o);
    jobs.push_back(chrom_job{CHROM_SQUARE, m, m + 1, q.data(), 80, primes, 8, static_cast<uint32_t*>(o)});
  }
  chrom_tuning t{};
  t.lanes_v = 2; t.targets_per_wave = 8; t.waves_per_block = 4; t.xcd_order = 4; t.unroll = 4; t.fuse = 2;
  t.stage = 6;
  const size_t bytes = chromatic_batch_workspace_bytes(jobs.data(), static_cast<int>(jobs.size()), &t);
  void* ws = nullptr;
  if (!bytes || hipMalloc(&ws, bytes) != hipSuccess) return 1;
  for (int r = 0; r < 40; ++r) {
    // stack traffic between the calls, as a caller's own work would leave
    volatile char junk[4096];
    for (int k = 0; k < 4096; ++k) junk[k] = static_cast<char>(r * 31 + k);
    if (chromatic_batch(jobs.data(), static_cast<int>(jobs.size()), &t, ws, bytes, nullptr) != CHROM_OK) {
      printf("batch: %s\n", chromatic_last_error());
      return 1;
    }
  }
  printf("captures %ld\n", hip_stub_captures());
  return 0;
}
