// Replayed under ThreadSanitizer against the HIP stand-in (asan_hip_stub.cpp,
// which aborts when a capture begins on a stream that is already capturing):
// three host threads, each with its own workspaces, queue strips that the
// library captures into graphs -- graph-mode strips, grouped strips and
// coefficient-form strips -- with a new strip height every round, so every
// call captures.  Argument: rounds.
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>
#include <hip/hip_runtime_api.h>
#include "chromstrip.h"

static void* dmalloc(size_t n) {
  void* p = nullptr;
  if (hipMalloc(&p, n) != hipSuccess) abort();
  return p;
}

static int strips(int mode, int rounds, int* failed) {
  const uint32_t primes[2] = {1084098661u, 1848443263u};
  std::vector<uint32_t> q(12);
  for (int k = 0; k < 12; ++k) q[k] = k + 1;
  chrom_tuning t{};
  t.lanes_v = 1;
  t.streams = mode == CHROM_MODE_GRAPH ? 2 : 1;
  for (int r = 0; r < rounds; ++r)
    for (int m = 3; m <= 5; ++m) {
      const int n_max = 3 + r;
      const size_t bytes = chromatic_workspace_bytes(CHROM_SQUARE, m, n_max, 12, 2, mode, &t);
      if (!bytes) { printf("workspace: %s\n", chromatic_last_error()); *failed = 1; return 1; }
      void* ws = dmalloc(bytes);
      void* out = dmalloc(static_cast<size_t>(n_max) * 24 * 4);
      for (int k = 0; k < 2; ++k)
        if (chromatic_strip_async(CHROM_SQUARE, m, n_max, q.data(), 12, primes, 2, mode, &t, ws, bytes, nullptr,
                                  static_cast<uint32_t*>(out)) != CHROM_OK) {
          printf("strip mode %d: %s\n", mode, chromatic_last_error());
          *failed = 1;
          return 1;
        }
      (void)hipFree(out);
      (void)hipFree(ws);
    }
  return 0;
}

static int series(int rounds, int* failed) {
  const uint32_t primes[2] = {1084098661u, 1848443263u};
  for (int r = 0; r < rounds; ++r)
    for (int m = 3; m <= 5; ++m) {
      const int n_max = 3 + r, d_max = 30;
      const size_t bytes = chromatic_series_workspace_bytes(CHROM_SQUARE, m, n_max, 2, d_max, CHROM_MODE_GRAPH, nullptr);
      if (!bytes) { printf("series workspace: %s\n", chromatic_last_error()); *failed = 1; return 1; }
      void* ws = dmalloc(bytes);
      void* out = dmalloc(static_cast<size_t>(n_max) * 2 * (d_max + 1) * 4);
      if (chromatic_series_async(CHROM_SQUARE, m, n_max, d_max, primes, 2, CHROM_MODE_GRAPH, nullptr, ws, bytes,
                                 nullptr, static_cast<uint32_t*>(out)) != CHROM_OK) {
        printf("series: %s\n", chromatic_last_error());
        *failed = 1;
        return 1;
      }
      (void)hipFree(out);
      (void)hipFree(ws);
    }
  return 0;
}

int main(int argc, char** argv) {
  const int rounds = argc > 1 ? atoi(argv[1]) : 6;
  for (int m = 3; m <= 5; ++m)
    if (chromatic_prepare(CHROM_SQUARE, m) != CHROM_OK || chromatic_prepare_series(CHROM_SQUARE, m) != CHROM_OK) {
      printf("prepare: %s\n", chromatic_last_error());
      return 1;
    }
  int failed[3] = {0, 0, 0};
  std::thread a([&] { strips(CHROM_MODE_GRAPH, rounds, &failed[0]); });
  std::thread b([&] { strips(CHROM_MODE_GROUPED, rounds, &failed[1]); });
  std::thread c([&] { series(rounds, &failed[2]); });
  a.join();
  b.join();
  c.join();
  if (failed[0] || failed[1] || failed[2]) return 1;
  printf("done\n");
  return 0;
}
