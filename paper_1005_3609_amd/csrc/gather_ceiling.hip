// Ceiling of the factor kernel's memory access pattern on this GPU: gathers
// of whole 512-byte rows (64 lanes x 8 bytes, one instance chunk of a state)
// at given row indices, nothing computed but an XOR.  Each wavefront reads K
// rows, U at a time, and stores one row.  Three index patterns over a
// 57346 x 5-row buffer (the input vector of a square m = 14 fused-pair launch
// with 640 instances, 147 MB): uniformly random rows, random rows within a
// sliding window of 4096 (locality like the factor maps' reader order), and
// near-sequential rows.  Prints one line per (pattern, wavefronts, U) with
// the time per launch and the gathered bytes per second.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#define CHECK(x)                                                                   \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                        \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                                \
    }                                                                              \
  } while (0)

template <int U>
__global__ void __launch_bounds__(256) gather_rows(const uint2* __restrict__ in, const int* __restrict__ idx, int K,
                                                   uint2* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int* mine = idx + static_cast<long>(wave) * K;
  uint2 acc = make_uint2(0, 0);
  for (int k = 0; k < K; k += U) {
    uint2 x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = __builtin_amdgcn_readfirstlane(mine[k + u]);
      x[u] = in[static_cast<long>(r) * 64 + lane];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc.x ^= x[u].x;
      acc.y ^= x[u].y;
    }
  }
  out[static_cast<long>(wave) * 64 + lane] = acc;
}

int main() {
  const long nrows = 57346L * 5;
  const long N = 1240000;  // gathers per launch (wavefront-entries of one fused launch)
  uint2* in = nullptr;
  CHECK(hipMalloc(&in, nrows * 512));
  CHECK(hipMemset(in, 1, nrows * 512));
  std::mt19937 rng(7);
  const char* names[3] = {"uniform", "window4096", "sequential"};
  for (int pattern = 0; pattern < 3; ++pattern) {
    std::vector<int> h(N);
    for (long i = 0; i < N; ++i) {
      if (pattern == 0) {
        h[i] = static_cast<int>(rng() % nrows);
      } else if (pattern == 1) {
        const long c = (i * nrows) / N, lo = std::max(0L, c - 2048);
        h[i] = static_cast<int>(std::min(nrows - 1, lo + static_cast<long>(rng() % 4096)));
      } else {
        h[i] = static_cast<int>((i * nrows) / N);
      }
      if (h[i] < 0 || h[i] >= nrows) {
        std::fprintf(stderr, "index out of range\n");
        return 1;
      }
    }
    int* idx = nullptr;
    CHECK(hipMalloc(&idx, N * 4));
    CHECK(hipMemcpy(idx, h.data(), N * 4, hipMemcpyHostToDevice));
    for (int nw : {8192, 16384, 32768, 77500}) {
      for (int U : {4, 8, 16}) {
        const int K = static_cast<int>(N / nw) / U * U;  // nw * K <= N: every index read is in idx
        if (K < U) continue;
        uint2* out = nullptr;
        CHECK(hipMalloc(&out, static_cast<long>(nw) * 512));
        auto launch = [&]() {
          const dim3 grid(nw / 4), block(256);
          if (U == 4) hipLaunchKernelGGL(gather_rows<4>, grid, block, 0, 0, in, idx, K, out);
          if (U == 8) hipLaunchKernelGGL(gather_rows<8>, grid, block, 0, 0, in, idx, K, out);
          if (U == 16) hipLaunchKernelGGL(gather_rows<16>, grid, block, 0, 0, in, idx, K, out);
        };
        hipEvent_t a, b;
        CHECK(hipEventCreate(&a));
        CHECK(hipEventCreate(&b));
        launch();
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(a));
        for (int it = 0; it < 10; ++it) launch();
        CHECK(hipEventRecord(b));
        CHECK(hipEventSynchronize(b));
        float ms = 0;
        CHECK(hipEventElapsedTime(&ms, a, b));
        const double us = ms * 100.0;
        const double bytes = static_cast<double>(nw) * K * 512;
        std::printf("%-10s wavefronts %6d U %2d rows/wave %4d: %7.1f us/launch %6.2f TB/s gathered\n", names[pattern],
                    nw, U, K, us, bytes / us / 1e6);
        std::fflush(stdout);
        CHECK(hipEventDestroy(a));
        CHECK(hipEventDestroy(b));
        CHECK(hipFree(out));
      }
    }
    CHECK(hipFree(idx));
  }
  CHECK(hipFree(in));
  return 0;
}
