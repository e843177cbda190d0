// Op-stream gather: the factor apply for unit-coefficient factors of the
// evaluation form (every code's polynomial in t = q - s has digits
// d_0..d_2 in {-1, 0, +1} and no t^3 term -- the square lattice's single
// factors and fused pairs).
//
// The factor's map is re-encoded as one stream of 32-bit op words in target
// row order: bits 0..22 the source state, bits 24..29 the entry's
// coefficient as signed unit digits (bit 24 + 2k: d_k = +1, bit 25 + 2k:
// d_k = -1), bit 31 set on the last word of a row.  A row with no entries
// has a single word without coefficient bits.  A wavefront's rows are one
// contiguous range of the stream, so the kernel needs no row pointers
// beyond the range's ends, and the words are uniform across the wavefront:
// they arrive through the scalar data cache sixteen at a time (one
// s_load_dwordx16 per four groups of four entries), straight into scalar
// registers.  Sources are read with buffer loads whose scalar offset is the
// source row's offset and whose vector offset is the lane's, so forming an
// address costs one scalar shift.  Every gather is issued unconditionally,
// four groups in flight, so the compiler's wait counts stay exact (loads
// complete in issue order): entries past a wavefront's range, up to three
// groups of them at its end, read its first source row again (cache hits).
// The buffer's range (2^31 - 1 bytes) bounds every access to the chunk's
// input region plus 2 GiB.
#pragma once

#include "kernels.hpp"

namespace cs {

constexpr uint32_t kOpSrcBits = 23;
constexpr uint32_t kOpSrcMask = (1u << kOpSrcBits) - 1;
constexpr uint32_t kOpRowEnd = 0x80000000u;
// A wavefront reads up to 36 words past its range (the blocks requested
// ahead); the stream carries this many zero words after its last row.
constexpr int kOpPad = 64;
// Buffer range: every offset (source row plus lane) stays below 2^31 (the
// host checks a chunk's vector).
constexpr int kOpRange = 0x7fffffff;
// gfx9 buffer resource, third dword (raw 32-bit data)
constexpr int kBufWord3 = 0x00020000;

typedef const __attribute__((address_space(4))) uint32_t* op_cptr;

// Adds or subtracts the source row x into A_0..A_2 as the digits say.  The
// common single-digit words take one compare each; real (uniform) branches.
template <int V>
__device__ __forceinline__ void op_accumulate(uint32_t (&A)[3][V], const uint32_t (&x)[V], uint32_t d,
                                              const uint32_t (&p)[V]) {
  if (d == 0x1u) {
    asm volatile("");
#pragma unroll
    for (int j = 0; j < V; ++j) A[0][j] = add_mod(A[0][j], x[j], p[j]);
  } else if (d == 0x2u) {
    asm volatile("");
#pragma unroll
    for (int j = 0; j < V; ++j) A[0][j] = sub_mod(A[0][j], x[j], p[j]);
  } else if (d == 0x4u) {
    asm volatile("");
#pragma unroll
    for (int j = 0; j < V; ++j) A[1][j] = add_mod(A[1][j], x[j], p[j]);
  } else if (d == 0x8u) {
    asm volatile("");
#pragma unroll
    for (int j = 0; j < V; ++j) A[1][j] = sub_mod(A[1][j], x[j], p[j]);
  } else if (d != 0u) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (d & (1u << (2 * k))) {
        asm volatile("");
#pragma unroll
        for (int j = 0; j < V; ++j) A[k][j] = add_mod(A[k][j], x[j], p[j]);
      }
      if (d & (2u << (2 * k))) {
        asm volatile("");
#pragma unroll
        for (int j = 0; j < V; ++j) A[k][j] = sub_mod(A[k][j], x[j], p[j]);
      }
    }
  }
}

// One wavefront computes target rows [r0, r1) of one chunk.
template <int V>
__device__ void op_tile(const GatherArgs& a, int chunk, int tile, uint32_t* lds) {
  static_assert(V == 1 || V == 2, "op-stream gathers take lanes_v 1 or 2");
  constexpr int W = 64 * V;
  constexpr int U = 4;        // entries per group
  constexpr int B = 16;       // words per scalar block (four groups)
  const int lane = lane_id(), wave = wave_id();
  const int inst0 = chunk * W + lane * V;
  const uint32_t boff = static_cast<uint32_t>(lane) * (4u * V);
  uint32_t p[V], tv[V], ts[V];
  load_v<V>(a.ic.p + inst0, p);
  load_v<V>(a.ic.tv + inst0, tv);
  load_v<V>(a.ic.ts + inst0, ts);
  uint32_t* out = a.out + chunk * a.out_cstride;
  const bool fused = a.w != nullptr;
  const uint32_t* wv = fused ? a.w + chunk * a.w_cstride : nullptr;
  uint32_t pinv[V];
  if (fused) load_v<V>(a.ic.pinv + inst0, pinv);
  uint32_t red[V];
#pragma unroll
  for (int j = 0; j < V; ++j) red[j] = 0;
  const int nw = blockDim.x >> 6;
  const int r0 = (tile * nw + wave) * a.rows_per_wave;
  const int r1 = min(r0 + a.rows_per_wave, a.csr.n_rows);
  if (r0 < r1) {
    const op_cptr rows = (op_cptr)(a.op_row);
    const op_cptr ops = (op_cptr)(a.ops);
    const int beg = static_cast<int>(rows[r0]);
    const int end = static_cast<int>(rows[r1]);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(a.in + chunk * a.in_cstride), 0, kOpRange, kBufWord3);
    const uint32_t first = ops[beg] & kOpSrcMask;
    uint32_t A[3][V];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < V; ++j) A[k][j] = 0;
    uint32_t used = 0;
    int row = r0;
    const int ng = (end - beg + U - 1) / U;   // groups holding entries
    // words of two blocks (even and odd); in blocks reaching past `end`, the
    // words past it become the wavefront's first source with no digits
    uint32_t wb[2][B];
    auto fetch = [&](int blk, uint32_t (&w)[B]) {
      const int e0 = beg + blk * B;
#pragma unroll
      for (int i = 0; i < B; ++i) w[i] = ops[e0 + i];
    };
    auto clamp = [&](int blk, uint32_t (&w)[B]) {
      const int e0 = beg + blk * B;
      if (e0 + B > end) {
#pragma unroll
        for (int i = 0; i < B; ++i) w[i] = (e0 + i < end) ? w[i] : first;
      }
    };
    uint32_t xq[4][U][V];
    auto issue = [&](const uint32_t (&w)[B], int q, uint32_t (&x)[U][V]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int so = static_cast<int>((w[q * U + u] & kOpSrcMask) * (4u * W));
        if constexpr (V == 2) {
          const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, static_cast<int>(boff), so, 0);
          x[u][0] = v[0];
          x[u][1] = v[1];
        } else {
          x[u][0] = __builtin_amdgcn_raw_buffer_load_b32(rs, static_cast<int>(boff), so, 0);
        }
        // loads stay in issue order (waits count completions in that order)
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    auto flush = [&]() {
      uint32_t v[V];
      if (used & 0x30u) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
          v[j] = add_mod(mul_shoup(A[2][j], tv[j], ts[j], p[j]), A[1][j], p[j]);
          v[j] = add_mod(mul_shoup(v[j], tv[j], ts[j], p[j]), A[0][j], p[j]);
        }
      } else if (used & 0x0cu) {
#pragma unroll
        for (int j = 0; j < V; ++j) v[j] = add_mod(mul_shoup(A[1][j], tv[j], ts[j], p[j]), A[0][j], p[j]);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j) v[j] = A[0][j];
      }
      store_row<V>(out, static_cast<uint32_t>(row) * (4u * W) + boff, v);
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < V; ++j) A[k][j] = 0;
      used = 0;
      ++row;
    };
    auto consume = [&](const uint32_t (&w)[B], int q, const uint32_t (&x)[U][V]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t word = w[q * U + u];
        const uint32_t d = (word >> 24) & 0x3fu;
        used |= d;
        op_accumulate<V>(A, x[u], d, p);
        if (word & kOpRowEnd) flush();
      }
    };
    // Prologue: blocks 0 and 1 requested, groups 0..2 issued.
    fetch(0, wb[0]);
    fetch(1, wb[1]);
    clamp(0, wb[0]);
    issue(wb[0], 0, xq[0]);
    issue(wb[0], 1, xq[1]);
    issue(wb[0], 2, xq[2]);
    // Steady state, eight groups (blocks 2i and 2i + 1) per iteration: slot
    // s consumes group g + s and issues group g + s + 3.  Block 2i + 2 is
    // requested into the even buffer once block 2i's last group is consumed,
    // block 2i + 3 into the odd one once block 2i + 1's is; a block is
    // clamped just before its first group is issued.
    for (int g = 0;; g += 8) {
      const int b = g / 4;
      if (g >= ng) break;
      issue(wb[0], 3, xq[3]);
      consume(wb[0], 0, xq[0]);
      if (g + 1 >= ng) break;
      clamp(b + 1, wb[1]);
      issue(wb[1], 0, xq[0]);
      consume(wb[0], 1, xq[1]);
      if (g + 2 >= ng) break;
      issue(wb[1], 1, xq[1]);
      consume(wb[0], 2, xq[2]);
      if (g + 3 >= ng) break;
      issue(wb[1], 2, xq[2]);
      consume(wb[0], 3, xq[3]);
      fetch(b + 2, wb[0]);
      if (g + 4 >= ng) break;
      issue(wb[1], 3, xq[3]);
      consume(wb[1], 0, xq[0]);
      if (g + 5 >= ng) break;
      clamp(b + 2, wb[0]);
      issue(wb[0], 0, xq[0]);
      consume(wb[1], 1, xq[1]);
      if (g + 6 >= ng) break;
      issue(wb[0], 1, xq[1]);
      consume(wb[1], 2, xq[2]);
      if (g + 7 >= ng) break;
      issue(wb[0], 2, xq[2]);
      consume(wb[1], 3, xq[3]);
      fetch(b + 3, wb[1]);
    }
    // Fused read-out, after the stream: each lane reads back its own
    // just-stored rows (cache-resident) with their weights, four rows per
    // wait.
    if (fused) {
      for (int r = r0; r < r1; r += 4) {
        uint32_t xo[4][V], wr[4][V];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t off = static_cast<uint32_t>(min(r + i, r1 - 1)) * (4u * W) + boff;
          load_row<V>(out, off, xo[i]);
          load_row<V>(wv, off, wr[i]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (r + i < r1) {
#pragma unroll
            for (int j = 0; j < V; ++j) red[j] = add_mod(red[j], mul_redc(xo[i][j], wr[i][j], p[j], pinv[j]), p[j]);
          }
      }
    }
  }
  if (fused) block_reduce_store<V>(red, p, a.partial + chunk * a.p_cstride + static_cast<long>(tile) * W, lds);
}

template <int V>
__global__ void __launch_bounds__(512) k_gather_ops(GatherArgs a, int xcd, int chunk0) {
  __shared__ uint32_t lds[8 * 64 * V];
  int tile, chunk;
  tile_chunk(xcd, chunk0, tile, chunk);
  op_tile<V>(a, chunk, tile, lds);
}

}  // namespace cs
