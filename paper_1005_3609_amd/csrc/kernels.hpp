// HIP kernels (gfx950, wave64) applying the per-site transfer-matrix
// factors of arXiv 1005.3609 to residue vectors.
//
// Layouts.
//   plain    one instance (q, p): vector [S] of uint32 residues.
//   batched  instances in chunks of W = 64 V: [chunk][S][W]; a wavefront owns
//            one chunk's row of a state, lane l holding instances l V .. l V+V-1,
//            so every row read or written is one coalesced W*4-byte segment.
// A factor is a target-major CSR matrix (gather form): out[t] = sum over the
// row's entries of coef(code) * in[src].  Every lane of a wavefront works on
// the same row and entry, so the row bounds and entry words are scalar loads
// and the branch on the coefficient code is uniform.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.hpp"

namespace cs {

constexpr uint32_t kEntSrcBits = 26;
constexpr uint32_t kEntSrcMask = (1u << kEntSrcBits) - 1;
constexpr int kCodes = 64;

// ---------------------------------------------------------------------------
// Vector helpers
// ---------------------------------------------------------------------------
// V = 1, 2, 4 or 8 consecutive words per lane (8: the coefficient form's
// widest rows, two 16-byte accesses).
template <int V>
__device__ __forceinline__ void load_v(const uint32_t* ptr, uint32_t (&x)[V]) {
  static_assert(V == 1 || V == 2 || V == 4 || V == 8, "V must be 1, 2, 4 or 8");
  if constexpr (V == 1) {
    x[0] = *ptr;
  } else if constexpr (V == 2) {
    uint2 t = *reinterpret_cast<const uint2*>(ptr);
    x[0] = t.x;
    x[1] = t.y;
  } else {
#pragma unroll
    for (int h = 0; h < V / 4; ++h) {
      uint4 t = *reinterpret_cast<const uint4*>(ptr + 4 * h);
      x[4 * h] = t.x;
      x[4 * h + 1] = t.y;
      x[4 * h + 2] = t.z;
      x[4 * h + 3] = t.w;
    }
  }
}

template <int V>
__device__ __forceinline__ void store_v(uint32_t* ptr, const uint32_t (&x)[V]) {
  static_assert(V == 1 || V == 2 || V == 4 || V == 8, "V must be 1, 2, 4 or 8");
  if constexpr (V == 1) {
    *ptr = x[0];
  } else if constexpr (V == 2) {
    *reinterpret_cast<uint2*>(ptr) = make_uint2(x[0], x[1]);
  } else {
#pragma unroll
    for (int h = 0; h < V / 4; ++h)
      *reinterpret_cast<uint4*>(ptr + 4 * h) = make_uint4(x[4 * h], x[4 * h + 1], x[4 * h + 2], x[4 * h + 3]);
  }
}

// Row access as a wave-uniform base plus a 32-bit byte offset (the row's
// offset plus the lane's): the form the scalar-base global load/store
// instructions take.  A chunk's vector stays below 4 GiB (checked on the host).
template <int V>
__device__ __forceinline__ void load_row(const uint32_t* base, uint32_t off, uint32_t (&x)[V]) {
  load_v<V>(reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(base) + off), x);
}

template <int V>
__device__ __forceinline__ void store_row(uint32_t* base, uint32_t off, const uint32_t (&x)[V]) {
  store_v<V>(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(base) + off), x);
}

// The same with the non-temporal hint (rows of vectors far larger than the
// caches, written once and read a launch later).
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
template <int V>
__device__ __forceinline__ void store_row_nt(uint32_t* base, uint32_t off, const uint32_t (&x)[V]) {
  char* p = reinterpret_cast<char*>(base) + off;
  if constexpr (V == 1) {
    __builtin_nontemporal_store(x[0], reinterpret_cast<uint32_t*>(p));
  } else if constexpr (V == 2) {
    __builtin_nontemporal_store(u32x2_t{x[0], x[1]}, reinterpret_cast<u32x2_t*>(p));
  } else {
#pragma unroll
    for (int h = 0; h < V / 4; ++h)
      __builtin_nontemporal_store(u32x4_t{x[4 * h], x[4 * h + 1], x[4 * h + 2], x[4 * h + 3]},
                                  reinterpret_cast<u32x4_t*>(p + 16 * h));
  }
}

// Row base for vectors whose chunk exceeds 4 GiB: the 64-bit address of row
// `row` formed in scalar registers (readfirstlane keeps the compiler from
// folding it into per-lane 64-bit addresses), so every access is that base
// plus the lane's 32-bit offset.
template <int W>
__device__ __forceinline__ uint32_t* wide_row(const uint32_t* base, uint32_t row) {
  const uint64_t a = reinterpret_cast<uint64_t>(base) + static_cast<uint64_t>(row) * (4u * W);
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(static_cast<uint32_t>(a))));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(static_cast<uint32_t>(a >> 32))));
  return reinterpret_cast<uint32_t*>((static_cast<uint64_t>(hi) << 32) | lo);
}

// Workgroups are handed to the 8 XCDs round-robin in dispatch order.  This
// bijection on [0, nb) gives each XCD one contiguous range of ids instead, so
// neighbouring target rows -- which share many source rows -- run under the
// same L2.
__device__ __forceinline__ int xcd_contiguous(int b, int nb) {
  constexpr int X = 8;
  const int per = (nb + X - 1) / X;
  const int tall = nb - (per - 1) * X;  // XCDs that receive `per` workgroups
  const int xcd = b % X, local = b / X;
  return xcd < tall ? xcd * per + local : tall * per + (xcd - tall) * (per - 1) + local;
}

// Block-id remaps (all bijections on [0, nb)): mode 1 gives each XCD one
// contiguous range; modes 2..5 give each XCD runs of 4, 16, 64 or 256
// consecutive ids, the runs dealt round-robin (neighbouring tiles share an
// L2 while the XCDs together sweep one region of the launch); ids past the
// last whole round stay.
__device__ __forceinline__ int xcd_remap(int b, int nb, int mode) {
  if (mode == 1) return xcd_contiguous(b, nb);
  constexpr int X = 8;
  const int G = 1 << (2 * (mode - 1));
  const int nfull = nb / (X * G) * (X * G);
  if (b >= nfull) return b;
  const int x = b % X, k = b / X;
  return ((k / G) * X + x) * G + k % G;
}

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
}
__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x) & 63; }

// ---------------------------------------------------------------------------
// Argument blocks
// ---------------------------------------------------------------------------
struct DevCsr {
  const int32_t* row_ptr;
  const uint32_t* ent;
  int n_rows;
  int n_cols;
};

// Per-instance constants of a batch, instance index inst = chunk W + lane V + j.
//   p[inst], pinv[inst] = -p^{-1} mod 2^32, tv[inst] = t mod p with
//   t = q - s for the job's basis shift s, ts[inst] = floor(tv 2^32 / p).
// Coefficient codes: poly[code] holds the integer coefficients d0..d3 of the
// code's polynomial written in powers of t, d0 + d1 t + d2 t^2 + d3 t^3, as
// four signed bytes (d_k in byte k); poly[64 + code] holds the same as masks
// (see accumulate); 2 x 64 words, unused codes zero.  Code 0 is +1 and code
// 1 is -1 (constants, so the same in every basis).
struct InstConsts {
  const uint32_t* p;
  const uint32_t* pinv;
  const uint32_t* tv;
  const uint32_t* ts;
  const int32_t* poly;
};

struct GatherArgs {
  DevCsr csr;
  const uint32_t* in;      // chunk 0, row 0
  uint32_t* out;
  long in_cstride;         // elements from one chunk to the next
  long out_cstride;
  InstConsts ic;
  // Fused read-out (w == nullptr: none): partial[chunk*pc_stride + tile*W + lane V + j]
  // = sum over the tile's rows of out * w (w in Montgomery form).
  const uint32_t* w;
  long w_cstride;
  uint32_t* partial;
  long p_cstride;
  int rows_per_wave;
  // Staged tiles (tile_row0 == nullptr: direct gathers).  Entry words then
  // hold a slot of the tile's source list instead of a source state.
  // Clustered tiles (tile_tgt != nullptr): tile positions are not rows;
  // position k writes row tile_tgt[k] (csr.row_ptr is then in tile order).
  const int32_t* tile_row0;
  const int32_t* tile_src0;
  const int32_t* tile_src;
  const int32_t* tile_tgt;
  // Pipelined staging (stage_range): first entry of every tile, the tile
  // count and the tiles one workgroup runs in turn.
  const int32_t* tile_ent0;
  int n_tiles, tiles_per_block;
  // Slots a staged tile keeps in LDS: a tile with more sources (a row of
  // exceptional fan-in forms a tile of its own) reads the rest from memory.
  int stage_cap;
  // Coefficient form with 512-slot rows, degree bound (deg_step == 0: none;
  // narrower rows ignore it).  The state being
  // gathered belongs to output row r (r = *deg_row when deg_row is set, a
  // device counter advanced by graph replays, else deg_row0) and has degree
  // below deg_step (r + 2) in x, deg_step being the sites of one row.
  int deg_step;
  int deg_row0;
  const int* deg_row;
  // Op-stream gather (opgather.hpp; ops == nullptr: none): the factor's op
  // words and the first word of every row.
  const uint32_t* ops;
  const int32_t* op_row;
  // Evaluation form: store target rows with the non-temporal hint.
  int nt_store;
};

struct DotArgs {
  const uint32_t* x;
  const uint32_t* w;
  long x_cstride;
  long w_cstride;
  int n_rows;
  InstConsts ic;
  uint32_t* partial;
  long p_cstride;
  int rows_per_wave;
};

struct FillArgs {
  uint32_t* x;
  long cstride;
  int n_rows;              // rows to write: row 0 = v0, the rest 0
  const uint32_t* v0;      // per instance (nullptr: 1)
  int rows_per_wave;
};

// Coefficient-form read-out: copies coefficients 0 .. dlen-1 of state 0 of
// every chunk (one prime each) to dst[chunk][dlen] of the output row.
struct EmitArgs {
  const uint32_t* src;     // chunk 0, state 0
  long src_cstride;
  uint32_t* dst;           // output row
  int dlen;
};

// Two-level read-out reduction.  Level 1: workgroup g of a chunk sums the
// partials [g*per, (g+1)*per) into part2[chunk][g][W]; level 2 sums the
// n_groups level-1 results into out[inst].
struct ReduceArgs {
  const uint32_t* partial;
  long p_cstride;
  int n_parts;
  InstConsts ic;
  uint32_t* part2;         // [chunk][n_groups][W]
  long p2_cstride;
  int n_groups;
  uint32_t* out;           // out[inst] for inst < n_valid (this row)
  int n_valid;
};

// ---------------------------------------------------------------------------
// Tile bodies (one workgroup, rows [row0, row0 + waves*rows_per_wave))
// ---------------------------------------------------------------------------
template <int V>
__device__ __forceinline__ void block_reduce_store(uint32_t (&red)[V], const uint32_t (&p)[V],
                                                   uint32_t* dst, uint32_t* lds) {
  const int lane = lane_id(), wave = wave_id(), nw = blockDim.x >> 6;
  constexpr int W = 64 * V;
#pragma unroll
  for (int j = 0; j < V; ++j) lds[wave * W + lane * V + j] = red[j];
  __syncthreads();
  if (wave == 0) {
    for (int k = 1; k < nw; ++k)
#pragma unroll
      for (int j = 0; j < V; ++j) red[j] = add_mod(red[j], lds[k * W + lane * V + j], p[j]);
    store_v<V>(dst + lane * V, red);
  }
  __syncthreads();
}

// A += c x mod p for a small wave-uniform integer c != 0: |c| x by
// left-to-right binary doubling (no steps for |c| = 1), then one modular add
// or subtract.
template <int V>
__device__ __forceinline__ void add_multiple(uint32_t (&A)[V], const uint32_t (&x)[V], int c,
                                             const uint32_t (&p)[V]) {
  const int n = c < 0 ? -c : c;
  uint32_t y[V];
#pragma unroll
  for (int j = 0; j < V; ++j) y[j] = x[j];
  for (int b = 30 - __builtin_clz(static_cast<unsigned>(n)); b >= 0; --b) {
#pragma unroll
    for (int j = 0; j < V; ++j) y[j] = add_mod(y[j], y[j], p[j]);
    if ((n >> b) & 1) {
#pragma unroll
      for (int j = 0; j < V; ++j) y[j] = add_mod(y[j], x[j], p[j]);
    }
  }
  if (c > 0) {
#pragma unroll
    for (int j = 0; j < V; ++j) A[j] = add_mod(A[j], y[j], p[j]);
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) A[j] = sub_mod(A[j], y[j], p[j]);
  }
}

// Coefficient accumulation without multiplications.  A factor entry's
// coefficient is an integer polynomial in q, written in powers of t = q - s
// (the host picks the shift s that makes the coefficients smallest, e.g.
// q - 2 = t), c = sum_k d_k t^k, so a target row's value sum_e c_e x_e equals
// sum_k t^k A_k with A_k = sum_e d_{e,k} x_e.  Each entry adds small
// multiples of its source row to the A_k (modular adds only); the row is
// finished by Horner's rule in t (at most three Shoup products).
//
// The wavefront keeps two copies of the code table, one word per lane:
// `pm` (lane c: code c's small coefficients as masks -- bit k for d_k = +1,
// bit 4+k for d_k = -1 -- bit 8 when some |d_k| > 1, degree in bits 12-13)
// and `pw` (lane c: d_0..d_3 as signed bytes, for the rare codes with bit 8).
// Every branch below updates one A_k in place, so the common paths compile
// to the modular additions alone.  Launches whose codes all have unit
// coefficients use the G = false instance, which has no general path at all
// (its merges would cost register copies on every entry).
//
// The coefficient-form instances (CF) also take |d_k| = 2, 3 on the fast
// path: such a d_k is written as +-2 (bit 16+k for +2, 20+k for -2) plus
// the +-1 bits, and only |d_k| > 3 (bit 9) needs the general path.  The
// normalised single factors never have one, so their launches run G = false.
constexpr uint32_t kMaskGeneral = 0x100u;
constexpr uint32_t kMaskGeneralCF = 0x200u;

template <int V, bool G, bool CF = false>
__device__ __forceinline__ void accumulate(uint32_t (&A)[4][V], const uint32_t (&x)[V], uint32_t code,
                                           const uint32_t (&p)[V], int pw, int pm, int& deg) {
  const uint32_t m = static_cast<uint32_t>(__builtin_amdgcn_readlane(pm, static_cast<int>(code)));
  if (G && (m & (CF ? kMaskGeneralCF : kMaskGeneral))) {
    const int cw = __builtin_amdgcn_readlane(pw, static_cast<int>(code));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = static_cast<int>(static_cast<int8_t>(static_cast<uint32_t>(cw) >> (8 * k)));
      if (c != 0) add_multiple<V>(A[k], x, c, p);
    }
  } else {
    // Real (uniform) branches, up to the code's own degree: the empty
    // volatile statements keep the compiler from computing every arm and
    // selecting.
    const int dc = static_cast<int>((m >> 12) & 3u);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k > dc) break;
      if (m & (1u << k)) {
        asm volatile("");
#pragma unroll
        for (int j = 0; j < V; ++j) A[k][j] = add_mod(A[k][j], x[j], p[j]);
      }
      if (m & (16u << k)) {
        asm volatile("");
#pragma unroll
        for (int j = 0; j < V; ++j) A[k][j] = sub_mod(A[k][j], x[j], p[j]);
      }
      if constexpr (CF) {
        if (m & (0x10000u << k)) {
          asm volatile("");
#pragma unroll
          for (int j = 0; j < V; ++j) A[k][j] = add_mod(A[k][j], add_mod(x[j], x[j], p[j]), p[j]);
        }
        if (m & (0x100000u << k)) {
          asm volatile("");
#pragma unroll
          for (int j = 0; j < V; ++j) A[k][j] = sub_mod(A[k][j], add_mod(x[j], x[j], p[j]), p[j]);
        }
      }
    }
  }
  const int dk = static_cast<int>((m >> 12) & 3u);
  deg = deg > dk ? deg : dk;
}

// sum_k t^k A_k mod p by Horner's rule; A_k = 0 for k > deg.
template <int V>
__device__ __forceinline__ void horner(uint32_t (&v)[V], const uint32_t (&A)[4][V], int deg,
                                       const uint32_t (&tv)[V], const uint32_t (&ts)[V],
                                       const uint32_t (&p)[V]) {
#pragma unroll
  for (int j = 0; j < V; ++j) v[j] = A[3][j];
#pragma unroll
  for (int k = 2; k >= 0; --k) {
    if (deg > k) {
#pragma unroll
      for (int j = 0; j < V; ++j) v[j] = add_mod(mul_shoup(v[j], tv[j], ts[j], p[j]), A[k][j], p[j]);
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j) v[j] = A[k][j];
    }
  }
}

// Coefficient form: a chunk holds one prime's truncated coefficient array
// of a polynomial in x = 1/q, coefficient k = lane V + j.  Multiplying by x
// moves every coefficient up one place (the top one drops out of the
// truncation); across lanes by one shuffle per wavefront.
template <int V>
__device__ __forceinline__ void shift_up(uint32_t (&v)[V]) {
  const uint32_t carry = static_cast<uint32_t>(__shfl_up(static_cast<int>(v[V - 1]), 1, 64));
#pragma unroll
  for (int j = V - 1; j > 0; --j) v[j] = v[j - 1];
  v[0] = (lane_id() == 0) ? 0u : carry;
}

// sum_k x^k A_k by Horner's rule on coefficient arrays; A_k = 0 for k > deg.
template <int V>
__device__ __forceinline__ void horner_cf(uint32_t (&v)[V], const uint32_t (&A)[4][V], int deg,
                                          const uint32_t (&p)[V]) {
#pragma unroll
  for (int j = 0; j < V; ++j) v[j] = A[3][j];
#pragma unroll
  for (int k = 2; k >= 0; --k) {
    if (deg > k) {
      shift_up<V>(v);
#pragma unroll
      for (int j = 0; j < V; ++j) v[j] = add_mod(v[j], A[k][j], p[j]);
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j) v[j] = A[k][j];
    }
  }
}

// One wavefront computes target rows [r0, r1) of one chunk.  Its row
// pointers (lane j holds row_ptr[r0 + j]) and its entry words (64 per
// register, lane l holding one) arrive with coalesced vector loads and are
// broadcast with readlane; source rows are loaded U entries at a time, P
// groups ahead of the group being consumed, so up to P U W*4-byte gathers
// are in flight per wavefront.  The inner loop loads nothing else: coefficients
// come from registers (see accumulate), so the only waits are for the source
// rows themselves, oldest first.  Row boundaries are uniform, so each
// finished row is stored without divergence; rows with no entries are stored
// as zero.
template <int V, int U, bool G, bool CF, bool WIDE = false>
__device__ void gather_tile(const GatherArgs& a, int chunk, int tile, uint32_t* lds) {
  constexpr int W = 64 * V;
  const int lane = lane_id(), wave = wave_id();
  const int inst0 = chunk * W + lane * V;
  const uint32_t boff = static_cast<uint32_t>(lane) * (4u * V);
  uint32_t p[V], tv[V], ts[V];
  load_v<V>(a.ic.p + inst0, p);
  load_v<V>(a.ic.tv + inst0, tv);
  load_v<V>(a.ic.ts + inst0, ts);
  const int pw = a.ic.poly[lane];
  const int pm = a.ic.poly[kCodes + lane];
  const uint32_t* in = a.in + chunk * a.in_cstride;     // uniform bases
  uint32_t* out = a.out + chunk * a.out_cstride;
  const bool fused = a.w != nullptr;
  const uint32_t* wv = fused ? a.w + chunk * a.w_cstride : nullptr;
  uint32_t pinv[V];
  if (fused) load_v<V>(a.ic.pinv + inst0, pinv);
  uint32_t red[V], A[4][V];
#pragma unroll
  for (int j = 0; j < V; ++j) red[j] = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int j = 0; j < V; ++j) A[k][j] = 0;
  int deg = 0;
  const int nw = blockDim.x >> 6;
  const int r0 = (tile * nw + wave) * a.rows_per_wave;
  const int r1 = min(r0 + a.rows_per_wave, a.csr.n_rows);
  // Coefficient form with 512-slot rows: a state of a strip whose rows so far
  // hold n sites has degree below n in x (each x pays for one merge of two
  // components, and there are fewer merges than sites), so the lanes whose
  // slots all lie above deg_step (r + 2) hold zeros.  They neither load nor
  // store: the vectors start zeroed, and a lane becomes live before any of
  // its slots can be non-zero.  Narrower rows fill up within a few rows, and
  // there the masking costs more than it saves.
  constexpr bool kBound = CF && V == 8;
  bool live = true;
  if constexpr (kBound) {
    if (a.deg_step) {
      const int row = a.deg_row ? *a.deg_row : a.deg_row0;
      live = lane <= a.deg_step * (row + 2) / V;
    }
  }
  if (r0 < r1) {
    const int nrows = r1 - r0;
    const int rp = (lane <= nrows) ? a.csr.row_ptr[r0 + lane] : 0;
    // rows in clustered order (evaluation form, never the read-out factor):
    // position r writes target row tile_tgt[r]
    const int tg = (!CF && a.tile_tgt && lane < nrows) ? a.tile_tgt[r0 + lane] : 0;
    const int beg = __builtin_amdgcn_readlane(rp, 0);
    const int end = __builtin_amdgcn_readlane(rp, nrows);
    int row = r0;
    int row_end = __builtin_amdgcn_readlane(rp, 1);
    auto flush = [&]() {
      uint32_t v[V];
      if constexpr (CF)
        horner_cf<V>(v, A, deg, p);
      else
        horner<V>(v, A, deg, tv, ts, p);
      if (!kBound || live) {
        if constexpr (WIDE) {
          store_row<V>(wide_row<W>(out, static_cast<uint32_t>(row)), boff, v);
        } else if constexpr (!CF) {
          const int dst = a.tile_tgt ? __builtin_amdgcn_readlane(tg, row - r0) : row;
          if (a.nt_store)
            store_row_nt<V>(out, static_cast<uint32_t>(dst) * (4u * W) + boff, v);
          else
            store_row<V>(out, static_cast<uint32_t>(dst) * (4u * W) + boff, v);
        } else {
          store_row<V>(out, static_cast<uint32_t>(row) * (4u * W) + boff, v);
        }
      }
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
    // One continuous entry stream [beg, end) in groups of U.  P groups are in
    // flight: group g + P - 1 is issued before group g is consumed, and every
    // issue is unconditional (slots past `end` repeat the last entry, a cache
    // hit), so each wait is for a fixed count of newer loads.  Entry words
    // come through a window of 128 (ev0: [base, base + 64), ev1: the next
    // 64); the window moves when the issue point leaves ev0, and the next
    // words are requested then, a full window ahead of their use.  U divides
    // 64, so no group straddles the two halves.
    constexpr int P = (U == 4) ? 3 : 2;
    int base = beg;
    uint32_t ev0 = (base + lane < end) ? a.csr.ent[base + lane] : 0u;
    uint32_t ev1 = (base + 64 + lane < end) ? a.csr.ent[base + 64 + lane] : 0u;
    uint32_t wq[P][U];
    uint32_t xq[P][U][V];
    auto issue = [&](int g, uint32_t (&w)[U], uint32_t (&x)[U][V]) {
      const int e0 = beg + g * U;
      if (e0 - base >= 64 && base + 64 < end) {
        base += 64;
        ev0 = ev1;
        ev1 = (base + 64 + lane < end) ? a.csr.ent[base + 64 + lane] : 0u;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        w[u] = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(ev0), min(e0 + u, end - 1) - base));
        if (!kBound || live) {
          if constexpr (WIDE)
            load_row<V>(wide_row<W>(in, w[u] & kEntSrcMask), boff, x[u]);
          else
            load_row<V>(in, (w[u] & kEntSrcMask) * (4u * W) + boff, x[u]);
        } else {
#pragma unroll
          for (int j = 0; j < V; ++j) x[u][j] = 0;
        }
        // Keep the loads in entry order: completions are counted in issue
        // order, so entry u must not be issued after entry u + 1.
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    auto consume = [&](int g, const uint32_t (&w)[U], const uint32_t (&x)[U][V]) {
      const int e0 = beg + g * U;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (e0 + u < end) {
          while (e0 + u >= row_end) flush();
          accumulate<V, G, CF>(A, x[u], w[u] >> kEntSrcBits, p, pw, pm, deg);
        }
      }
    };
    if (beg < end) {
#pragma unroll
      for (int s = 0; s < P - 1; ++s) issue(s, wq[s], xq[s]);
      for (int g = 0;;) {
        bool done = false;
#pragma unroll
        for (int s = 0; s < P; ++s) {
          if (!done) {
            issue(g + P - 1, wq[(s + P - 1) % P], xq[(s + P - 1) % P]);
            consume(g, wq[s], xq[s]);
            ++g;
            done = beg + g * U >= end;
          }
        }
        if (done) break;
      }
    }
    while (row < r1) flush();
    // Fused read-out, after the entry stream so that its loads never sit
    // behind in-flight gathers: each lane reads back its own just-stored
    // rows (cache-resident) with their weights, four rows per wait (with a
    // target list, the rows it stored at their targets).
    if (fused) {
      for (int r = r0; r < r1; r += 4) {
        uint32_t xo[4][V], wr[4][V];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rr = min(r + i, r1 - 1);
          const int dst = (!CF && a.tile_tgt) ? __builtin_amdgcn_readlane(tg, rr - r0) : rr;
          const uint32_t off = static_cast<uint32_t>(dst) * (4u * W) + boff;
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

// Staged variant of gather_tile: the workgroup first copies the distinct
// source rows of its tile (one W*4-byte row per slot, listed ascending) into
// LDS with independent loads spread over its wavefronts, then each
// wavefront computes a contiguous share of the tile's rows reading its
// sources from LDS.  Sources shared by several rows of the tile are read
// from memory once; the coefficient handling and row finishing are those of
// gather_tile.  `slots` is the LDS area (max_slots rows of W words).  With
// clustered tiles the tile's positions are written to the rows tile_tgt
// lists (targets grouped by the sources they share).
template <int V, int U, bool G>
__device__ void stage_tile(const GatherArgs& a, int chunk, int tile, uint32_t* slots) {
  constexpr int W = 64 * V;
  const int lane = lane_id(), wave = wave_id();
  const int nw = blockDim.x >> 6;
  const int inst0 = chunk * W + lane * V;
  const uint32_t boff = static_cast<uint32_t>(lane) * (4u * V);
  const uint32_t* in = a.in + chunk * a.in_cstride;
  uint32_t* out = a.out + chunk * a.out_cstride;
  // tile bounds (lanes 0/1 read the two ends, broadcast)
  const int tr = a.tile_row0[tile + (lane & 1)];
  const int ts = a.tile_src0[tile + (lane & 1)];
  const int row0 = __builtin_amdgcn_readlane(tr, 0), row1 = __builtin_amdgcn_readlane(tr, 1);
  const int s0 = __builtin_amdgcn_readlane(ts, 0), ns = __builtin_amdgcn_readlane(ts, 1) - s0;
  // this wavefront's rows, and its row pointers and first entry words,
  // requested before the staging loads so their latency overlaps them
  const int per = (row1 - row0 + nw - 1) / nw;
  const int r0 = min(row0 + wave * per, row1), r1 = min(r0 + per, row1);
  const int nrows = r1 - r0;
  const int rp = (lane <= nrows) ? a.csr.row_ptr[r0 + lane] : 0;
  const int tg = (a.tile_tgt && lane < nrows) ? a.tile_tgt[r0 + lane] : 0;
  uint32_t p[V], tv[V], ts_[V];
  load_v<V>(a.ic.p + inst0, p);
  load_v<V>(a.ic.tv + inst0, tv);
  load_v<V>(a.ic.ts + inst0, ts_);
  const int pw = a.ic.poly[lane];
  const int pm = a.ic.poly[kCodes + lane];
  // phase 1: slot k of the tile goes to wavefront k % nw; a wavefront
  // requests up to R of its slots at once (one round trip for a tile of up
  // to R nw sources), then writes them to LDS in order
  constexpr int R = 16;
  const int nsl = min(ns, a.stage_cap);
  for (int k0 = wave; k0 < nsl; k0 += nw * R) {
    const int sid = (lane < R) ? a.tile_src[s0 + min(k0 + lane * nw, nsl - 1)] : 0;
    uint32_t x[R][V];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (k0 + u * nw < nsl) {
        const uint32_t src = static_cast<uint32_t>(__builtin_amdgcn_readlane(sid, u));
        load_row<V>(in, src * (4u * W) + boff, x[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int k = k0 + u * nw;
      if (k < nsl) {
#pragma unroll
        for (int j = 0; j < V; ++j) slots[k * W + lane * V + j] = x[u][j];
      }
    }
  }
  __syncthreads();
  // phase 2
  if (nrows > 0) {
    uint32_t A[4][V];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < V; ++j) A[k][j] = 0;
    int deg = 0;
    const int beg = __builtin_amdgcn_readlane(rp, 0);
    const int end = __builtin_amdgcn_readlane(rp, nrows);
    int row = r0;
    int row_end = __builtin_amdgcn_readlane(rp, 1);
    auto flush = [&]() {
      uint32_t v[V];
      horner<V>(v, A, deg, tv, ts_, p);
      const int dst = a.tile_tgt ? __builtin_amdgcn_readlane(tg, row - r0) : row;
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
      const uint32_t ev = (lane < n) ? a.csr.ent[base + lane] : 0u;
      for (int k = 0; k < n; k += U) {
        uint32_t w[U], x[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          w[u] = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(ev), min(k + u, n - 1)));
          const uint32_t slot = w[u] & kEntSrcMask;
          if (slot < static_cast<uint32_t>(a.stage_cap)) {
            const uint32_t* sl = slots + slot * W + lane * V;
#pragma unroll
            for (int j = 0; j < V; ++j) x[u][j] = sl[j];
          } else {   // past the LDS slots: straight from memory
            const uint32_t src = static_cast<uint32_t>(a.tile_src[s0 + min(static_cast<int>(slot), ns - 1)]);
            load_row<V>(in, src * (4u * W) + boff, x[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (k + u < n) {
            while (base + k + u >= row_end) flush();
            accumulate<V, G>(A, x[u], w[u] >> kEntSrcBits, p, pw, pm, deg);
          }
        }
      }
    }
    while (row < r1) flush();
  }
}

template <int V>
__device__ void dot_tile(const DotArgs& a, int chunk, int tile, uint32_t* lds) {
  constexpr int W = 64 * V;
  const int lane = lane_id(), wave = wave_id();
  const int inst0 = chunk * W + lane * V;
  uint32_t p[V], pinv[V];
  load_v<V>(a.ic.p + inst0, p);
  load_v<V>(a.ic.pinv + inst0, pinv);
  const uint32_t* x = a.x + chunk * a.x_cstride + lane * V;
  const uint32_t* w = a.w + chunk * a.w_cstride + lane * V;
  const int nw = blockDim.x >> 6;
  int r0 = (tile * nw + wave) * a.rows_per_wave;
  int r1 = min(r0 + a.rows_per_wave, a.n_rows);
  uint32_t red[V];
#pragma unroll
  for (int j = 0; j < V; ++j) red[j] = 0;
  for (int r = r0; r < r1; ++r) {
    uint32_t xv[V], wv[V];
    load_v<V>(x + static_cast<size_t>(r) * W, xv);
    load_v<V>(w + static_cast<size_t>(r) * W, wv);
#pragma unroll
    for (int j = 0; j < V; ++j) red[j] = add_mod(red[j], mul_redc(xv[j], wv[j], p[j], pinv[j]), p[j]);
  }
  block_reduce_store<V>(red, p, a.partial + chunk * a.p_cstride + static_cast<long>(tile) * W, lds);
}

template <int V>
__device__ void fill_tile(const FillArgs& a, int chunk, int tile) {
  constexpr int W = 64 * V;
  const int lane = lane_id(), wave = wave_id();
  const int nw = blockDim.x >> 6;
  uint32_t* x = a.x + chunk * a.cstride + lane * V;
  int r0 = (tile * nw + wave) * a.rows_per_wave;
  int r1 = min(r0 + a.rows_per_wave, a.n_rows);
  for (int r = r0; r < r1; ++r) {
    uint32_t v[V];
#pragma unroll
    for (int j = 0; j < V; ++j) v[j] = 0;
    if (r == 0) {
      if (a.v0)
        load_v<V>(a.v0 + chunk * W + lane * V, v);
      else
#pragma unroll
        for (int j = 0; j < V; ++j) v[j] = 1;
    }
    store_v<V>(x + static_cast<size_t>(r) * W, v);
  }
}

template <int V>
__device__ void reduce1_tile(const ReduceArgs& a, int chunk, int g, uint32_t* lds) {
  constexpr int W = 64 * V;
  const int nt = blockDim.x, tid = threadIdx.x;
  const int per = (a.n_parts + a.n_groups - 1) / a.n_groups;
  const int k0 = g * per, k1 = min(k0 + per, a.n_parts);
  const int span = nt >= W ? W : nt;      // threads sharing one pass over the instances
  const int G = nt >= W ? nt / W : 1;     // groups splitting the parts
  const int grp = tid / span;
  const uint32_t* src = a.partial + chunk * a.p_cstride;
  for (int j = tid % span; j < W; j += span) {
    const uint32_t p = a.ic.p[chunk * W + j];
    uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int k = k0 + grp;
    for (; k + 3 * G < k1; k += 4 * G) {
      s0 = add_mod(s0, src[static_cast<long>(k) * W + j], p);
      s1 = add_mod(s1, src[static_cast<long>(k + G) * W + j], p);
      s2 = add_mod(s2, src[static_cast<long>(k + 2 * G) * W + j], p);
      s3 = add_mod(s3, src[static_cast<long>(k + 3 * G) * W + j], p);
    }
    for (; k < k1; k += G) s0 = add_mod(s0, src[static_cast<long>(k) * W + j], p);
    lds[grp * W + j] = add_mod(add_mod(s0, s1, p), add_mod(s2, s3, p), p);
  }
  __syncthreads();
  for (int j = tid; j < W; j += nt) {
    const uint32_t p = a.ic.p[chunk * W + j];
    uint32_t s = 0;
    for (int q = 0; q < G; ++q) s = add_mod(s, lds[q * W + j], p);
    a.part2[chunk * a.p2_cstride + static_cast<long>(g) * W + j] = s;
  }
  __syncthreads();
}

template <int V>
__device__ void reduce2_tile(const ReduceArgs& a, int chunk, uint32_t* out) {
  constexpr int W = 64 * V;
  for (int j = threadIdx.x; j < W; j += blockDim.x) {
    const int inst = chunk * W + j;
    const uint32_t p = a.ic.p[inst];
    const uint32_t* src = a.part2 + chunk * a.p2_cstride + j;
    uint32_t s = 0;
    for (int k = 0; k < a.n_groups; ++k) s = add_mod(s, src[static_cast<long>(k) * W], p);
    if (inst < a.n_valid) out[inst] = s;
  }
}

// ---------------------------------------------------------------------------
// Eager kernels: grid.x = tiles, grid.y = chunks
// ---------------------------------------------------------------------------
// Block (x, y) = (tile, chunk0 + y); with xcd != 0 the linear block id is
// first remapped so each XCD sweeps a contiguous range.
__device__ __forceinline__ void tile_chunk(int xcd, int chunk0, int& tile, int& chunk) {
  int b = blockIdx.y * gridDim.x + blockIdx.x;
  if (xcd) b = xcd_remap(b, gridDim.x * gridDim.y, xcd);
  tile = b % gridDim.x;
  chunk = chunk0 + b / gridDim.x;
}

template <int V, int U, bool G, bool CF, bool WIDE = false>
__global__ void __launch_bounds__(512) k_gather(GatherArgs a, int xcd, int chunk0) {
  __shared__ uint32_t lds[8 * 64 * V];
  int tile, chunk;
  tile_chunk(xcd, chunk0, tile, chunk);
  gather_tile<V, U, G, CF, WIDE>(a, chunk, tile, lds);
}

// The coefficient form's 512-slot rows (V = 8, U = 4).  The form never fuses
// the read-out into a gather (it applies T_last instead), so this instance
// has no read-out and no LDS, and asks for three wavefronts per SIMD (at
// most 168 VGPRs).  Rows below their degree bound leave most lanes idle, and
// such launches wait on load latency rather than bandwidth: the third
// wavefront takes 26 % off the first six rows of a square m = 20 strip.
template <bool G, bool WIDE>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3)))
k_gather_cf8(GatherArgs a, int xcd, int chunk0) {
  int tile, chunk;
  tile_chunk(xcd, chunk0, tile, chunk);
  a.w = nullptr;
  gather_tile<8, 4, G, true, WIDE>(a, chunk, tile, nullptr);
}

// grid (tiles, chunks); dynamic LDS: max_slots * 64 V words
template <int V, int U, bool G>
__global__ void __launch_bounds__(512) k_stage(GatherArgs a, int xcd, int chunk0) {
  extern __shared__ uint32_t stage_lds[];
  int tile, chunk;
  tile_chunk(xcd, chunk0, tile, chunk);
  stage_tile<V, U, G>(a, chunk, tile, stage_lds);
}

template <int V>
__global__ void __launch_bounds__(512) k_dot(DotArgs a, int xcd, int chunk0) {
  __shared__ uint32_t lds[8 * 64 * V];
  int tile, chunk;
  tile_chunk(xcd, chunk0, tile, chunk);
  dot_tile<V>(a, chunk, tile, lds);
}

template <int V>
__global__ void __launch_bounds__(512) k_fill(FillArgs a, int chunk0) {
  fill_tile<V>(a, chunk0 + blockIdx.y, blockIdx.x);
}

// grid (n_groups, chunks)
template <int V>
__global__ void __launch_bounds__(512) k_reduce1(ReduceArgs a, int chunk0) {
  __shared__ uint32_t lds[8 * 64 * V];
  reduce1_tile<V>(a, chunk0 + blockIdx.y, blockIdx.x, lds);
}

// grid (chunks)
template <int V>
__global__ void __launch_bounds__(512) k_reduce2(ReduceArgs a, int chunk0) {
  reduce2_tile<V>(a, chunk0 + blockIdx.x, a.out);
}

// Level 2 whose output row is taken from a device counter (hipGraph replays
// write successive rows); k_bump advances the counter afterwards.
template <int V>
__global__ void __launch_bounds__(512) k_reduce2_counted(ReduceArgs a, int chunk0, const int* row, long row_stride) {
  reduce2_tile<V>(a, chunk0 + blockIdx.x, a.out + static_cast<long>(*row) * row_stride);
}

// grid (chunks)
__global__ void __launch_bounds__(256) k_emit(EmitArgs a, int chunk0) {
  const int chunk = chunk0 + blockIdx.x;
  for (int k = threadIdx.x; k < a.dlen; k += blockDim.x)
    a.dst[static_cast<long>(chunk) * a.dlen + k] = a.src[chunk * a.src_cstride + k];
}

// Output row taken from a device counter (hipGraph replays), as k_reduce2_counted.
__global__ void __launch_bounds__(256) k_emit_counted(EmitArgs a, int chunk0, const int* row, long row_stride) {
  const int chunk = chunk0 + blockIdx.x;
  uint32_t* dst = a.dst + static_cast<long>(*row) * row_stride;
  for (int k = threadIdx.x; k < a.dlen; k += blockDim.x)
    dst[static_cast<long>(chunk) * a.dlen + k] = a.src[chunk * a.src_cstride + k];
}

__global__ void k_bump(int* row) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *row += 1;
}

__global__ void k_set_int(int* dst, int value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = value;
}

// ---------------------------------------------------------------------------
// Plain (one instance) kernels
// ---------------------------------------------------------------------------
struct PlainConsts {
  uint32_t p, pinv;
  uint32_t cval[kCodes];
  uint32_t cshp[kCodes];
};

__global__ void __launch_bounds__(256) k_gather_plain(DevCsr csr, const uint32_t* __restrict__ in,
                                                      uint32_t* __restrict__ out, PlainConsts c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= csr.n_rows) return;
  const int beg = csr.row_ptr[r], end = csr.row_ptr[r + 1];
  uint32_t acc = 0;
  for (int e = beg; e < end; ++e) {
    const uint32_t w = csr.ent[e];
    const uint32_t x = in[w & kEntSrcMask];
    const uint32_t code = w >> kEntSrcBits;
    if (code == 0)
      acc = add_mod(acc, x, c.p);
    else if (code == 1)
      acc = sub_mod(acc, x, c.p);
    else
      acc = add_mod(acc, mul_shoup(x, c.cval[code], c.cshp[code], c.p), c.p);
  }
  out[r] = acc;
}

__global__ void __launch_bounds__(256) k_fill_plain(uint32_t* x, int n, uint32_t v0) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) x[r] = (r == 0) ? v0 : 0u;
}

// Z = sum_s x[s] w[s] mod p with w in Montgomery form; one workgroup of
// 256 threads.  Each lane strides over the states, then the wavefront folds
// its 64 partial sums with cross-lane shuffles, and the four wavefront sums
// meet in LDS.  The ragged tail is masked by a ballot of the lanes that own
// a state.
__global__ void __launch_bounds__(256) k_dot_plain(const uint32_t* __restrict__ x,
                                                   const uint32_t* __restrict__ w, int n,
                                                   uint32_t p, uint32_t pinv, uint32_t* out) {
  __shared__ uint32_t part[4];
  uint32_t s = 0;
  const int base_full = (n / blockDim.x) * blockDim.x;
  for (int i = threadIdx.x; i < base_full; i += blockDim.x) s = add_mod(s, mul_redc(x[i], w[i], p, pinv), p);
  const int i = base_full + threadIdx.x;
  const unsigned long long owners = __ballot(i < n);
  if (owners != 0ull && i < n) s = add_mod(s, mul_redc(x[i], w[i], p, pinv), p);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s = add_mod(s, __shfl_xor(s, off, 64), p);
  if (lane_id() == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < static_cast<int>(blockDim.x >> 6); ++k) t = add_mod(t, part[k], p);
    *out = t;
  }
}

// ---------------------------------------------------------------------------
// Grouped launches: one launch runs one step of many (job, chunk) items
// ---------------------------------------------------------------------------
enum StepOp : int { kOpFill = 0, kOpGather = 1, kOpDot = 2, kOpReduce1 = 3, kOpReduce2 = 4, kOpEmit = 5 };

struct Step {
  int op;
  int ntiles;
  int chunk;               // chunk index handed to the tile body
  int general;             // gather: needs the general coefficient path (host-side kernel choice)
  int lds_bytes;           // staged gather: dynamic LDS of the launch
  int cf;                  // gather: coefficient form (polynomials in x = 1/q); 2: also wide rows
  union {
    GatherArgs g;
    DotArgs d;
    FillArgs f;
    EmitArgs e;
    ReduceArgs r;
  } u;
};

// Workgroup b runs tile (b - tile_start[k]) of steps[k], k the largest index
// with tile_start[k] <= b.  Items of one launch never share buffers, and the
// launches of a sweep run in stream order, so no workgroup waits on another.
struct GroupArgs {
  const Step* steps;
  const int* tile_start;   // nsteps + 1 prefix sums of ntiles
  int nsteps;
  int xcd;                 // block-id remap mode (xcd_remap)
};

template <int V, int U, bool G>
__global__ void __launch_bounds__(512) k_grouped(GroupArgs g) {
  __shared__ uint32_t lds[8 * 64 * V];
  const int b = g.xcd ? xcd_remap(blockIdx.x, gridDim.x, g.xcd) : static_cast<int>(blockIdx.x);
  int lo = 0, hi = g.nsteps - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.tile_start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const int k = __builtin_amdgcn_readfirstlane(lo);
  const int tile = __builtin_amdgcn_readfirstlane(b - g.tile_start[k]);
  const Step& st = g.steps[k];
  switch (st.op) {
    case kOpGather: gather_tile<V, U, G, false>(st.u.g, st.chunk, tile, lds); break;
    case kOpDot: dot_tile<V>(st.u.d, st.chunk, tile, lds); break;
    case kOpFill: fill_tile<V>(st.u.f, st.chunk, tile); break;
    case kOpReduce1: reduce1_tile<V>(st.u.r, st.chunk, tile, lds); break;
    case kOpReduce2: reduce2_tile<V>(st.u.r, st.chunk, st.u.r.out); break;
  }
}

}  // namespace cs
