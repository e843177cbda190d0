// Pipelined staged tiles: each workgroup runs a range of tiles in turn and
// requests the next tile's data while it computes the current one.
//
// A tile (maps.hpp: build_staged, build_clustered) is a set of target rows
// with the list of distinct source rows they read.  For tile t the
// workgroup needs the source rows (W*4 bytes each), the tile's entry words
// (slot | code), row pointers and target rows.  All of them are requested
// one tile ahead into registers -- the source ids themselves two tiles ahead,
// since the row requests depend on them -- and copied to LDS between two
// barriers at the tile boundary, so the loads of tile t+1 are in flight
// while the wavefronts compute tile t from LDS.  A tile's shared sources are
// read from memory once; the coefficient handling and row finishing are
// those of gather_tile.
#pragma once

#include "kernels.hpp"

namespace cs {

constexpr int kPipeSlotsPerWave = 16;   // source rows one wavefront requests per tile
constexpr int kPipeMaxEnt = 1024;       // entries of one tile
constexpr int kPipeMaxRows = 64;        // target rows of one tile
// LDS words before the source rows: entry words, row pointers, target rows
// (rounded up so the rows that follow are 64-byte aligned)
constexpr int kPipeMetaWords = (kPipeMaxEnt + 2 * kPipeMaxRows + 1 + 15) / 16 * 16;

__host__ __device__ inline size_t pipe_lds_bytes(int max_slots, int W) {
  return 4u * (static_cast<size_t>(kPipeMetaWords) + static_cast<size_t>(max_slots) * W);
}

// Workgroup `range` of chunk `chunk`: tiles [range * tiles_per_block, ...).
// Needs stage_cap <= kPipeSlotsPerWave * waves (slots past the cap are read
// from memory), rows <= kPipeMaxRows and rows + 1 <= threads, entries <=
// kPipeMaxEnt and <= 2 x threads (each thread copies two entry words), and
// tiles_per_block < 64 (checked on the host).
template <int V, int U, bool G>
__device__ void stage_range(const GatherArgs& a, int chunk, int range, uint32_t* lds) {
  constexpr int W = 64 * V;
  constexpr int R = kPipeSlotsPerWave;
  const int lane = lane_id(), wave = wave_id();
  const int nw = static_cast<int>(blockDim.x) >> 6;
  const int nt = static_cast<int>(blockDim.x), tid = static_cast<int>(threadIdx.x);
  const int tb = range * a.tiles_per_block;
  const int te = min(tb + a.tiles_per_block, a.n_tiles);
  if (tb >= te) return;
  const int inst0 = chunk * W + lane * V;
  const uint32_t boff = static_cast<uint32_t>(lane) * (4u * V);
  const uint32_t* in = a.in + chunk * a.in_cstride;
  uint32_t* out = a.out + chunk * a.out_cstride;
  uint32_t* m_ent = lds;
  int* m_rp = reinterpret_cast<int*>(lds + kPipeMaxEnt);
  int* m_tg = m_rp + kPipeMaxRows + 1;
  uint32_t* slots = lds + kPipeMetaWords;
  uint32_t p[V], tv[V], ts_[V];
  load_v<V>(a.ic.p + inst0, p);
  load_v<V>(a.ic.tv + inst0, tv);
  load_v<V>(a.ic.ts + inst0, ts_);
  const int pw = a.ic.poly[lane];
  const int pm = a.ic.poly[kCodes + lane];
  // bounds of every tile of the range (lane k: tile tb + k)
  const int span = te - tb;
  const int trv = lane <= span ? a.tile_row0[tb + lane] : 0;
  const int tsv = lane <= span ? a.tile_src0[tb + lane] : 0;
  const int tev = lane <= span ? a.tile_ent0[tb + lane] : 0;
  auto rows0 = [&](int t) { return __builtin_amdgcn_readlane(trv, t - tb); };
  auto rows1 = [&](int t) { return __builtin_amdgcn_readlane(trv, t - tb + 1); };
  auto src0 = [&](int t) { return __builtin_amdgcn_readlane(tsv, t - tb); };
  auto src1 = [&](int t) { return __builtin_amdgcn_readlane(tsv, t - tb + 1); };
  auto ent0 = [&](int t) { return __builtin_amdgcn_readlane(tev, t - tb); };
  auto ent1 = [&](int t) { return __builtin_amdgcn_readlane(tev, t - tb + 1); };
  // lane u < R: source of this wavefront's u-th slot of tile t
  auto load_sid = [&](int t) {
    const int s0 = src0(t), ns = min(src1(t) - s0, a.stage_cap);   // a tile of rows without entries has no sources
    return (lane < R && ns > 0) ? a.tile_src[s0 + min(wave + lane * nw, ns - 1)] : 0;
  };
  // prefetched tile: source rows, entry words, row pointers, target rows
  uint32_t x[R][V];
  uint32_t me0 = 0, me1 = 0;
  int mrp = 0, mtg = 0, p_ns = 0, p_ne = 0, p_nrows = 0;
  auto request = [&](int t, int sid) {
    const int ns = min(src1(t) - src0(t), a.stage_cap);
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (wave + u * nw < ns) {
        const uint32_t src = static_cast<uint32_t>(__builtin_amdgcn_readlane(sid, u));
        load_row<V>(in, src * (4u * W) + boff, x[u]);
      }
    }
    const int e0 = ent0(t), ne = ent1(t) - e0;
    const int r0 = rows0(t), nrows = rows1(t) - r0;
    me0 = tid < ne ? a.csr.ent[e0 + tid] : 0u;
    me1 = tid + nt < ne ? a.csr.ent[e0 + tid + nt] : 0u;
    mrp = tid <= nrows ? a.csr.row_ptr[r0 + tid] - e0 : 0;
    mtg = tid < nrows ? (a.tile_tgt ? a.tile_tgt[r0 + tid] : r0 + tid) : 0;
    p_ns = ns;
    p_ne = ne;
    p_nrows = nrows;
  };
  auto commit = [&]() {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int k = wave + u * nw;
      if (k < p_ns) {
#pragma unroll
        for (int j = 0; j < V; ++j) slots[k * W + lane * V + j] = x[u][j];
      }
    }
    if (tid < p_ne) m_ent[tid] = me0;
    if (tid + nt < p_ne) m_ent[tid + nt] = me1;
    if (tid <= p_nrows) m_rp[tid] = mrp;
    if (tid < p_nrows) m_tg[tid] = mtg;
  };
  int sid = load_sid(tb);
  request(tb, sid);
  sid = tb + 1 < te ? load_sid(tb + 1) : 0;
  for (int t = tb; t < te; ++t) {
    __syncthreads();   // every wavefront is done with tile t - 1
    commit();
    __syncthreads();
    const int nrows = p_nrows;
    const int s0t = src0(t), nst = src1(t) - s0t;
    if (t + 1 < te) request(t + 1, sid);
    if (t + 2 < te) sid = load_sid(t + 2);
    // tile t from LDS: wavefront w takes a contiguous share of its rows
    const int per = (nrows + nw - 1) / nw;
    const int r0 = min(wave * per, nrows), r1 = min(r0 + per, nrows);
    const int nr = r1 - r0;
    if (nr > 0) {
      const int rp = lane <= nr ? m_rp[r0 + lane] : 0;
      const int tg = lane < nr ? m_tg[r0 + lane] : 0;
      uint32_t A[4][V];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < V; ++j) A[k][j] = 0;
      int deg = 0;
      const int beg = __builtin_amdgcn_readlane(rp, 0);
      const int end = __builtin_amdgcn_readlane(rp, nr);
      int row = r0;
      int row_end = __builtin_amdgcn_readlane(rp, 1);
      auto flush = [&]() {
        uint32_t v[V];
        horner<V>(v, A, deg, tv, ts_, p);
        const int dst = __builtin_amdgcn_readlane(tg, row - r0);
        store_row<V>(out, static_cast<uint32_t>(dst) * (4u * W) + boff, v);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k <= deg) {
#pragma unroll
            for (int j = 0; j < V; ++j) A[k][j] = 0;
          }
        deg = 0;
        ++row;
        if (row < r1) row_end = __builtin_amdgcn_readlane(rp, row - r0 + 1);
      };
      for (int base = beg; base < end; base += 64) {
        const int n = min(64, end - base);
        const uint32_t ev = lane < n ? m_ent[base + lane] : 0u;
        for (int k = 0; k < n; k += U) {
          uint32_t w[U], xs[U][V];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            w[u] = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(ev), min(k + u, n - 1)));
            const uint32_t slot = w[u] & kEntSrcMask;
            if (slot < static_cast<uint32_t>(a.stage_cap)) {
              const uint32_t* sl = slots + slot * W + lane * V;
#pragma unroll
              for (int j = 0; j < V; ++j) xs[u][j] = sl[j];
            } else {   // past the LDS slots: straight from memory
              const uint32_t src = static_cast<uint32_t>(a.tile_src[s0t + min(static_cast<int>(slot), nst - 1)]);
              load_row<V>(in, src * (4u * W) + boff, xs[u]);
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (k + u < n) {
              while (base + k + u >= row_end) flush();
              accumulate<V, G>(A, xs[u], w[u] >> kEntSrcBits, p, pw, pm, deg);
            }
          }
        }
      }
      while (row < r1) flush();
    }
  }
}

// grid (ranges, chunks); dynamic LDS: pipe_lds_bytes(max_slots, 64 V)
template <int V, int U, bool G>
__global__ void __launch_bounds__(512) k_stage_pipe(GatherArgs a, int xcd, int chunk0) {
  extern __shared__ uint32_t pipe_lds[];
  int range, chunk;
  tile_chunk(xcd, chunk0, range, chunk);
  stage_range<V, U, G>(a, chunk, range, pipe_lds);
}

}  // namespace cs
