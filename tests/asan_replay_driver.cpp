// Replays host call sequences of the library against the HIP stand-in
// (asan_hip_stub.cpp) under AddressSanitizer:
//  1. the batch autotuner's candidate sequence over the square m = 2..14
//     sweep (80 q x 8 primes): lanes_v, targets per wave, waves per block,
//     fusion and 1-3 chunk groups, each candidate once plus `steps` replays
//     on a fresh workspace, freed before the next (as the tuner's tensors);
//  2. graph-mode strips of square m = 14 with 1-3 chunk groups over the
//     target orders of stages 0, 4 and 6, single factors and fused pairs;
//  3. lanes_v 4 strips split into a job of 512 and one of 128 instances
//     (graph and batched modes, with the factor launches alone);
//  4. resident strips (triangular m = 12, square m = 10) in both arithmetic
//     forms, and the strip entry point that allocates nothing.
// Prints one line per case; exits non-zero on the first library error.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "chromstrip.h"

static void* dmalloc(size_t n) {
  void* p = nullptr;
  if (hipMalloc(&p, n) != hipSuccess) abort();
  return p;
}

int main(int argc, char** argv) {
  const int steps = argc > 1 ? atoi(argv[1]) : 3;
  const uint32_t primes[8] = {1084098661u, 1848443263u, 1135934141u, 1516637251u,
                              2135061679u, 2056503863u, 1256711527u, 1751345737u};
  std::vector<uint32_t> q(80);
  for (int i = 0; i < 80; ++i) q[i] = static_cast<uint32_t>(i + 1);
  std::vector<chrom_job> jobs;
  for (int m = 2; m <= 14; ++m) jobs.push_back(chrom_job{CHROM_SQUARE, m, m + 1, q.data(), 80, primes, 8, nullptr});
  int n = 0;
  for (int v : {1, 2})
    for (int tpw : {4, 8})
      for (int wpb : {4, 8})
        for (int f : {1, 2})
          for (int s : {1, 2, 3}) {
            chrom_tuning t{};
            t.lanes_v = v; t.targets_per_wave = tpw; t.waves_per_block = wpb; t.xcd_order = 1; t.unroll = 4;
            t.fuse = f; t.streams = s;
            const size_t bytes = chromatic_batch_workspace_bytes(jobs.data(), static_cast<int>(jobs.size()), &t);
            if (!bytes) { printf("batch workspace: %s\n", chromatic_last_error()); return 1; }
            void* ws = dmalloc(bytes);
            std::vector<void*> outs;
            for (chrom_job& j : jobs) {
              outs.push_back(dmalloc(static_cast<size_t>(j.n_max) * j.nq * j.np * 4));
              j.d_out = static_cast<uint32_t*>(outs.back());
            }
            for (int r = 0; r < 1 + steps; ++r)
              if (chromatic_batch(jobs.data(), static_cast<int>(jobs.size()), &t, ws, bytes, nullptr) != CHROM_OK) {
                printf("batch: %s\n", chromatic_last_error());
                return 1;
              }
            printf("batch %2d lanes_v %d tpw %d wpb %d fuse %d streams %d ok\n", ++n, v, tpw, wpb, f, s);
            for (void* o : outs) (void)hipFree(o);
            (void)hipFree(ws);
          }
  // graph-mode strips (the headline's fork/join of chunk groups)
  for (int stage : {0, 4, 6})
    for (int f : {1, 2})
      for (int s : {1, 2, 3}) {
        chrom_tuning t{};
        t.lanes_v = 2; t.targets_per_wave = 16; t.waves_per_block = 8; t.xcd_order = 1; t.unroll = 4;
        t.streams = s; t.fuse = f; t.stage = stage;
        const size_t bytes = chromatic_workspace_bytes(CHROM_SQUARE, 14, 15, 80, 8, CHROM_MODE_GRAPH, &t);
        if (!bytes) { printf("graph workspace: %s\n", chromatic_last_error()); return 1; }
        void* ws = dmalloc(bytes);
        void* out = dmalloc(15u * 640u * 4u);
        for (int r = 0; r < 1 + steps; ++r)
          if (chromatic_strip_async(CHROM_SQUARE, 14, 15, q.data(), 80, primes, 8, CHROM_MODE_GRAPH, &t, ws, bytes,
                                    nullptr, static_cast<uint32_t*>(out)) != CHROM_OK) {
            printf("graph strip: %s\n", chromatic_last_error());
            return 1;
          }
        printf("graph strip stage %d fuse %d streams %d ok\n", stage, f, s);
        (void)hipFree(out);
        (void)hipFree(ws);
      }
  // lanes_v 4 at 640 instances: a job of 512 and one of 128 (graph: one
  // graph with two branches; batched: a forked library stream)
  for (int mode : {CHROM_MODE_GRAPH, CHROM_MODE_BATCHED})
    for (int stage : {0, 6})
      for (int s : {1, 2}) {
        chrom_tuning t{};
        t.lanes_v = 4; t.targets_per_wave = 8; t.waves_per_block = 4; t.xcd_order = 4; t.unroll = 4;
        t.streams = s; t.fuse = 2; t.stage = stage;
        const size_t bytes = chromatic_workspace_bytes(CHROM_SQUARE, 14, 15, 80, 8, mode, &t);
        if (!bytes) { printf("split workspace: %s\n", chromatic_last_error()); return 1; }
        void* ws = dmalloc(bytes);
        void* out = dmalloc(15u * 640u * 4u);
        for (int r = 0; r < 1 + steps; ++r)
          if (chromatic_strip_async(CHROM_SQUARE, 14, 15, q.data(), 80, primes, 8, mode, &t, ws, bytes, nullptr,
                                    static_cast<uint32_t*>(out)) != CHROM_OK) {
            printf("split strip: %s\n", chromatic_last_error());
            return 1;
          }
        if (chromatic_factor_launches(CHROM_SQUARE, 14, q.data(), 80, primes, 8, 2, &t, ws, bytes, nullptr) !=
            CHROM_OK) {
          printf("split factor launches: %s\n", chromatic_last_error());
          return 1;
        }
        printf("split strip mode %d stage %d streams %d ok\n", mode, stage, s);
        (void)hipFree(out);
        (void)hipFree(ws);
      }
  // resident strips, both arithmetic forms
  const int res[2][3] = {{CHROM_TRIANGULAR, 12, 13}, {CHROM_SQUARE, 10, 11}};
  for (const auto& r : res)
    for (int stage : {0, 1})
      for (int v : {1, 2}) {
        chrom_tuning t{};
        t.lanes_v = v; t.waves_per_block = 16; t.fuse = 2; t.stage = stage;
        const size_t bytes = chromatic_workspace_bytes(r[0], r[1], r[2], 48, 6, CHROM_MODE_RESIDENT, &t);
        if (!bytes) { printf("resident workspace: %s\n", chromatic_last_error()); return 1; }
        void* ws = dmalloc(bytes);
        void* out = dmalloc(static_cast<size_t>(r[2]) * 288 * 4);
        for (int k = 0; k < 1 + steps; ++k)
          if (chromatic_strip_async(r[0], r[1], r[2], q.data(), 48, primes, 6, CHROM_MODE_RESIDENT, &t, ws, bytes,
                                    nullptr, static_cast<uint32_t*>(out)) != CHROM_OK) {
            printf("resident strip: %s\n", chromatic_last_error());
            return 1;
          }
        printf("resident lattice %d m %d stage %d lanes_v %d ok\n", r[0], r[1], stage, v);
        (void)hipFree(out);
        (void)hipFree(ws);
      }
  // the strip that allocates nothing, a larger call then a smaller one
  for (int m : {12, 9}) {
    void* out = dmalloc(static_cast<size_t>(m + 1) * 640 * 4);
    if (chromatic_strip_noalloc(CHROM_SQUARE, m, m + 1, q.data(), 80, primes, 8, nullptr, nullptr,
                                static_cast<uint32_t*>(out)) != CHROM_OK) {
      printf("noalloc strip: %s\n", chromatic_last_error());
      return 1;
    }
    printf("noalloc strip m %d ok\n", m);
    (void)hipFree(out);
  }
  printf("done\n");
  return 0;
}
