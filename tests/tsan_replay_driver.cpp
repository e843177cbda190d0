// Replayed under ThreadSanitizer against the HIP stand-in (asan_hip_stub.cpp):
// one host thread builds the coefficient form's host maps of widths 2..m_hi
// (chromatic_prepare_host) while the main thread runs coefficient-form strips
// of widths 1..m_hi (host-built maps, uploaded), as the finite-lattice driver
// once did with a second thread.  Arguments: lattice, m_hi.
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>
#include <hip/hip_runtime_api.h>
#include "chromstrip.h"
int main(int argc, char** argv) {
  setenv("CHROMSTRIP_HOST_MAPS", "1", 1);
  const int lat = argc > 1 ? atoi(argv[1]) : CHROM_SQUARE;
  const int m_hi = argc > 2 ? atoi(argv[2]) : 11;
  const uint32_t primes[3] = {1084098661u, 1848443263u, 1135934141u};
  std::thread prep([&] {
    for (int m = 2; m <= m_hi; ++m)
      if (chromatic_prepare_host(lat, m, 1) != CHROM_OK) printf("prepare %d: %s\n", m, chromatic_last_error());
  });
  for (int m = 1; m <= m_hi; ++m) {
    const int n_max = m + 2, d_max = 40;   // any sizes: the stand-in runs no kernel
    size_t bytes = chromatic_series_workspace_bytes(lat, m, n_max, 3, d_max, CHROM_MODE_GRAPH, nullptr);
    if (!bytes) { printf("ws %d: %s\n", m, chromatic_last_error()); return 1; }
    void* ws = nullptr; void* out = nullptr;
    (void)hipMalloc(&ws, bytes);
    (void)hipMalloc(&out, (size_t)n_max * 3 * (d_max + 1) * 4);
    for (int r = 0; r < 2; ++r)
      if (chromatic_series_async(lat, m, n_max, d_max, primes, 3, CHROM_MODE_GRAPH, nullptr, ws, bytes, nullptr,
                                 static_cast<uint32_t*>(out)) != CHROM_OK) {
        printf("series %d: %s\n", m, chromatic_last_error());
        return 1;
      }
    printf("series m %d ok\n", m);
    fflush(stdout);
    (void)hipFree(out); (void)hipFree(ws);
  }
  prep.join();
  printf("done\n");
  return 0;
}
