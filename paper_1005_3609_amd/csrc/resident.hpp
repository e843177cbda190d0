// Whole-strip kernel with the state vectors resident in LDS (gfx950: up to
// 160 KiB per workgroup).
//
// One launch runs every step of a strip -- the read-out vector's build
// (eqs. T_last, T_last_i), x = e0 (eq. Z_from_T), and for every row the m
// per-site factors (Sec. 3.2-3.3) followed by the row's read-out -- for
// every instance (q, p) of one or more jobs.  Workgroup g owns K instances
// of one job: their two state vectors live in LDS as x[state][K] and every
// step ends with a workgroup barrier, so no workgroup ever waits for another
// and nothing but the factor maps, the per-instance constants, the read-out
// vector and the output touches global memory.  This is the tier for the
// small widths, whose vectors (kilobytes to tens of kilobytes per instance)
// make the per-launch cost of the batched path dominate: square m <= 12 and
// triangular m <= 13 fit at K = 1.
//
// Arithmetic.  A factor entry's coefficient is an integer polynomial in q
// (a code); for one instance it is a fixed integer c(q).  Two forms:
//  * exact double accumulation (the default wherever its bound holds): a
//    target row is sum_e c_e(q) x_e over its entries, with x_e < p < 2^31 the
//    source residues and |c_e(q)| small, so when (row length) x max |c(q)|
//    <= 2^21 every product and partial sum is an integer below 2^52 in
//    magnitude and double arithmetic computes it exactly: one conversion and
//    one fused multiply-add per entry and instance, then one reduction mod p
//    per row (floor(T / p) from the rounded reciprocal, off by at most one,
//    then a conditional subtraction);
//  * modular integer arithmetic: c(q) mod p per entry, one Shoup product
//    c x mod p (the host precomputes c and floor(c 2^32 / p) per code and
//    instance) and one modular addition.  Its 32-bit multiplies issue at a
//    quarter of the rate of the double operations above.
// The host picks the first form per job when the bound holds for every map
// of the strip and every instance (tuning stage 0), else, or on request
// (stage 1), the second.
//
// Work split.  Half of a single factor's target rows hold one entry and a
// few hold ten or more, so with one thread per row in map order most lanes
// of a wavefront would idle while one finished a long row.  The maps run
// here in sliced-ELL form: rows sorted by their number of entries and cut
// into slices of 64 (one per wavefront pass, lane l taking the slice's l-th
// row), each slice's entries padded to its longest row and stored
// column-major, so a wavefront's loop counts are uniform and its entry loads
// coalesced.  For the modular form a slice keeps the entries with
// coefficient +1 or -1 in columns of their own, ahead of the others: those
// cost one modular addition or subtraction, the others a Shoup product as
// well.  The double form costs the same per entry whatever the coefficient,
// so its maps keep every entry in one group (fewer padded columns).  Padding
// entries read a row kept at zero past the end of each vector.
#pragma once

#include "kernels.hpp"

namespace cs {

constexpr int kResMaxM = 20;
constexpr int kResMaxWaves = 16;

// A gather-form factor map (entry word = source | code << 26) in sliced-ELL
// form.  Slice s holds the rows perm[64 s .. 64 s + 63] (-1 past the last
// row) and slice[s] = (offset, unit columns, other columns, 0): column u of
// lane l's row is ent[offset + 64 u + l], the unit columns (codes 0 = +1 and
// 1 = -1) first.  Missing entries are padding: source n_zero (a row of zeros)
// with code 0.
struct DevSell {
  const int32_t* perm;
  const int32_t* slice;    // 4 ints per slice
  const uint32_t* ent;
  int n_rows, n_cols, nslice;
};

// One job of a resident launch.
struct ResidentJob {
  DevSell fac[kResMaxM];   // forward factors F_1 .. F_nf of one row (single sites or fused products)
  DevSell last[kResMaxM];  // read-out maps: last[i-1] is applied as a gather for i = m .. 1
  int nf, m;
  int s_nc, s_max;         // NCNNN states, largest space (LDS rows per vector)
  int n_max;               // output rows (rectangles m x 1 .. m x n_max)
  int I, ncodes;           // instances, codes of the code table
  int g0, ngroups;         // first workgroup of the job, workgroups (instance groups of K)
  const uint32_t* coef;    // [I][ncodes]: code c at instance i, mod p_i
  const uint32_t* coefs;   // [I][ncodes]: its Shoup quotient
  const double* coff;      // [I][ncodes]: code c at instance i as an integer (double form)
  const double* rcp;       // [I]: 1 / p_i rounded to double (double form)
  const uint32_t* p;       // [I]
  const uint32_t* pinv;    // [I]: -p^{-1} mod 2^32
  const uint32_t* r1;      // [I]: 2^32 mod p
  uint32_t* w;             // [I][s_nc] read-out vector (Montgomery form), written by the kernel
  uint32_t* out;           // [n_max][I]
  int exact;               // 1: exact double accumulation (maps in one group), 0: modular
};

// LDS bytes of a workgroup: two vectors of s_max + 1 rows of K words (row
// s_max stays zero: the padding entries' source), the code table (value and
// quotient per code and instance, or the value as a double) and the
// reduction slots.
__host__ __device__ inline size_t resident_lds_bytes(int s_max, int ncodes, int K) {
  return 4u * (2u * (static_cast<size_t>(s_max) + 1) * K + 2u * static_cast<size_t>(ncodes) * K +
               static_cast<size_t>(kResMaxWaves) * K);
}

// Map arrays are global memory; loads through these pointers compile to
// global (not flat) loads, whose completion the LDS traffic does not wait on.
typedef const uint32_t __attribute__((address_space(1)))* gu32;
typedef const int32_t __attribute__((address_space(1)))* gi32;

// c x mod p for one entry's source row and code; the code table holds, per
// code, K (value, quotient) pairs.
template <int K>
__device__ __forceinline__ void res_product(uint32_t (&v)[K], uint32_t w, const uint32_t* in, const uint32_t* cc,
                                            const uint32_t (&p)[K]) {
  const uint32_t src = w & kEntSrcMask;
  const uint32_t code = w >> kEntSrcBits;
  uint32_t x[K];
  load_v<K>(in + src * K, x);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint2 c = *reinterpret_cast<const uint2*>(cc + (code * K + k) * 2);
    v[k] = mul_shoup(x[k], c.x, c.y, p[k]);
  }
}

// acc += (+-1) in[src] for one unit entry (code 0 = +1, 1 = -1).
template <int K>
__device__ __forceinline__ void res_unit(uint32_t (&acc)[K], uint32_t w, const uint32_t* in, const uint32_t (&p)[K]) {
  uint32_t x[K];
  load_v<K>(in + (w & kEntSrcMask) * K, x);
  const bool neg = (w >> kEntSrcBits) != 0u;
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = add_mod(acc[k], neg ? p[k] - x[k] : x[k], p[k]);
}

// G columns starting at `e` (the lane's word of the first): the loads first,
// then the arithmetic.
template <int K, bool UNIT, int G>
__device__ __forceinline__ void res_cols(uint32_t (&acc)[K], gu32 e, const uint32_t* in, const uint32_t* cc,
                                         const uint32_t (&p)[K]) {
  uint32_t w[G];
#pragma unroll
  for (int i = 0; i < G; ++i) w[i] = e[i * 64];
  if constexpr (UNIT) {
#pragma unroll
    for (int i = 0; i < G; ++i) res_unit<K>(acc, w[i], in, p);
  } else {
    uint32_t v[G][K];
#pragma unroll
    for (int i = 0; i < G; ++i) res_product<K>(v[i], w[i], in, cc, p);
#pragma unroll
    for (int i = 0; i < G; ++i)
#pragma unroll
      for (int k = 0; k < K; ++k) acc[k] = add_mod(acc[k], v[i][k], p[k]);
  }
}

// n columns: four at a time, then two, then one.
template <int K, bool UNIT>
__device__ __forceinline__ void res_columns(uint32_t (&acc)[K], gu32 e, int n, const uint32_t* in,
                                            const uint32_t* cc, const uint32_t (&p)[K]) {
  int u = 0;
  for (; u + 4 <= n; u += 4) res_cols<K, UNIT, 4>(acc, e + u * 64, in, cc, p);
  if (u + 2 <= n) {
    res_cols<K, UNIT, 2>(acc, e + u * 64, in, cc, p);
    u += 2;
  }
  if (u < n) res_cols<K, UNIT, 1>(acc, e + u * 64, in, cc, p);
}

// out <- c in for one map, ending with the workgroup barrier.  Wavefront w
// takes slices w, w + waves, ...; every loop count in a slice is uniform.
template <int K>
__device__ __forceinline__ void res_apply(const DevSell& c, const uint32_t* in, uint32_t* out, const uint32_t* cc,
                                          const uint32_t (&p)[K]) {
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int nw = static_cast<int>(blockDim.x) >> 6;
  const gi32 slices = (gi32)c.slice;
  const gi32 perm = (gi32)c.perm;
  for (int s = wave_id(); s < c.nslice; s += nw) {
    const int off = slices[4 * s], nu = slices[4 * s + 1], ng = slices[4 * s + 2];
    const int row = perm[s * 64 + lane];
    const gu32 e = (gu32)c.ent + off + lane;
    uint32_t acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0;
    res_columns<K, true>(acc, e, nu, in, cc, p);
    res_columns<K, false>(acc, e + nu * 64, ng, in, cc, p);
    if (row >= 0) store_v<K>(out + static_cast<uint32_t>(row) * K, acc);
  }
  __syncthreads();
}

// T mod p for an integer T held exactly in a double, |T| / p < 2^21 (the
// double form's bound): the quotient estimate floor(T / p - 1/2) from the
// rounded reciprocal is floor(T / p) or one less, so r = T - estimate x p
// (one fused multiply-add, exact: an integer in [0, 2p)) needs at most one
// subtraction.
__device__ __forceinline__ uint32_t reduce_exact(double t, double pf, double rcp, uint32_t p) {
  const double qe = __builtin_floor(__builtin_fma(t, rcp, -0.5));
  const uint32_t r = static_cast<uint32_t>(__builtin_fma(-qe, pf, t));
  return min(r, r - p);
}

// Sum of G entries (words w) into acc in the double form: source rows and
// coefficients (code table cf[code][K]) first, then the products.
template <int K, int G>
__device__ __forceinline__ void res_words_exact(double (&acc)[K], const uint32_t (&w)[G], const uint32_t* in,
                                                const double* cf) {
  uint32_t x[G][K];
  double c[G][K];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    load_v<K>(in + (w[i] & kEntSrcMask) * K, x[i]);
    const double* ci = cf + (w[i] >> kEntSrcBits) * K;
#pragma unroll
    for (int k = 0; k < K; ++k) c[i][k] = ci[k];
  }
#pragma unroll
  for (int i = 0; i < G; ++i)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = __builtin_fma(c[i][k], static_cast<double>(x[i][k]), acc[k]);
}

// G columns starting at `e` (the lane's word of the first).
template <int K, int G>
__device__ __forceinline__ void res_cols_exact(double (&acc)[K], gu32 e, const uint32_t* in, const double* cf) {
  uint32_t w[G];
#pragma unroll
  for (int i = 0; i < G; ++i) w[i] = e[i * 64];
  res_words_exact<K, G>(acc, w, in, cf);
}

// out <- c in for one map in the double form (one column group per slice),
// ending with the workgroup barrier.  Wavefront w takes slices w, w + waves,
// ...; every loop count in a slice is uniform.  (Requesting the next slice's
// entry words ahead of the current slice's sum was measured slower.)
template <int K>
__device__ __forceinline__ void res_apply_exact(const DevSell& c, const uint32_t* in, uint32_t* out, const double* cf,
                                                const uint32_t (&p)[K], const double (&pf)[K],
                                                const double (&rcp)[K]) {
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int nw = static_cast<int>(blockDim.x) >> 6;
  const gi32 slices = (gi32)c.slice;
  const gi32 perm = (gi32)c.perm;
  for (int s = wave_id(); s < c.nslice; s += nw) {
    const int off = slices[4 * s], n = slices[4 * s + 1] + slices[4 * s + 2];
    const int row = perm[s * 64 + lane];
    const gu32 e = (gu32)c.ent + off + lane;
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    int u = 0;
    for (; u + 4 <= n; u += 4) res_cols_exact<K, 4>(acc, e + u * 64, in, cf);
    if (u + 2 <= n) {
      res_cols_exact<K, 2>(acc, e + u * 64, in, cf);
      u += 2;
    }
    if (u < n) res_cols_exact<K, 1>(acc, e + u * 64, in, cf);
    if (row >= 0) {
      uint32_t v[K];
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = reduce_exact(acc[k], pf[k], rcp[k], p[k]);
      store_v<K>(out + static_cast<uint32_t>(row) * K, v);
    }
  }
  __syncthreads();
}

// Row read-out: out_row[k] = sum_s w_k[s] x[s][k] mod p_k over the NCNNN
// states, w in Montgomery form.  Ends with the workgroup barrier.
template <int K>
__device__ __forceinline__ void res_dot(const uint32_t* x, const uint32_t* const (&wk)[K], int s_nc,
                                        const uint32_t (&p)[K], const uint32_t (&pinv)[K], uint32_t* red,
                                        uint32_t* out_row, int nvalid) {
  uint32_t acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0;
  for (int s = threadIdx.x; s < s_nc; s += blockDim.x) {
    uint32_t xv[K];
    load_v<K>(x + static_cast<uint32_t>(s) * K, xv);
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = add_mod(acc[k], mul_redc(wk[k][s], xv[k], p[k], pinv[k]), p[k]);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int k = 0; k < K; ++k)
      acc[k] = add_mod(acc[k], static_cast<uint32_t>(__shfl_xor(static_cast<int>(acc[k]), off, 64)), p[k]);
  const int wave = static_cast<int>(threadIdx.x) >> 6, nw = static_cast<int>(blockDim.x) >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[wave * K + k] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x < static_cast<unsigned>(nvalid)) {
    const int k = static_cast<int>(threadIdx.x);
    uint32_t pk = 0, s = 0;
#pragma unroll
    for (int kk = 0; kk < K; ++kk)
      if (kk == k) pk = p[kk];
    for (int v = 0; v < nw; ++v) s = add_mod(s, red[v * K + k], pk);
    out_row[k] = s;
  }
  __syncthreads();
}

template <int K>
__global__ void __launch_bounds__(64 * kResMaxWaves) k_resident(const ResidentJob* __restrict__ jobs, int njobs) {
  extern __shared__ uint32_t res_lds[];
  // the job of this workgroup: the last with g0 <= blockIdx.x
  int lo = 0, hi = njobs - 1;
  const int b = static_cast<int>(blockIdx.x);
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].g0 <= b) lo = mid; else hi = mid - 1;
  }
  const ResidentJob& J = jobs[lo];
  const int g = b - J.g0;
  if (g >= J.ngroups || J.n_max < 1) return;
  const int i0 = g * K;
  const int nvalid = min(K, J.I - i0);
  uint32_t* xa = res_lds;
  uint32_t* xb = xa + (static_cast<size_t>(J.s_max) + 1) * K;
  uint32_t* cc = xb + (static_cast<size_t>(J.s_max) + 1) * K;
  uint32_t* red = cc + 2 * J.ncodes * K;
  // Instances past the job's last (a ragged final group) repeat its
  // constants; their results are never written.
  uint32_t p[K], pinv[K];
  const uint32_t* wk[K];
  int ik[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ik[k] = min(i0 + k, J.I - 1);
    p[k] = J.p[ik[k]];
    pinv[k] = J.pinv[ik[k]];
    wk[k] = J.w + static_cast<size_t>(ik[k]) * J.s_nc;
  }
  if (threadIdx.x < static_cast<unsigned>(K)) {   // the zero rows read by padding entries
    xa[static_cast<size_t>(J.s_max) * K + threadIdx.x] = 0u;
    xb[static_cast<size_t>(J.s_max) * K + threadIdx.x] = 0u;
  }
  // code table: (value, quotient) pairs, or in the double form the value as
  // a double at the same place (cc is 8-byte aligned: 2 (s_max + 1) K words
  // in; 16-byte for K >= 2)
  const bool exact = J.exact != 0;
  double* cf = reinterpret_cast<double*>(cc);
  double pf[K], rcp[K];
  for (int idx = threadIdx.x; idx < J.ncodes * K; idx += blockDim.x) {
    const int code = idx / K, k = idx % K;
    const int inst = min(i0 + k, J.I - 1);
    if (exact) {
      cf[idx] = J.coff[static_cast<size_t>(inst) * J.ncodes + code];
    } else {
      cc[2 * idx] = J.coef[static_cast<size_t>(inst) * J.ncodes + code];
      cc[2 * idx + 1] = J.coefs[static_cast<size_t>(inst) * J.ncodes + code];
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    pf[k] = static_cast<double>(p[k]);
    rcp[k] = exact ? J.rcp[ik[k]] : 0.0;
  }
  auto apply = [&](const DevSell& c, const uint32_t* in, uint32_t* out) {
    if (exact)
      res_apply_exact<K>(c, in, out, cf, p, pf, rcp);
    else
      res_apply<K>(c, in, out, cc, p);
  };
  // Read-out vector: R e0 on the first read-out space, then T_m^last ..
  // T_1^last in gather form (transposed), ending on the NCNNN space.
  const int n0 = J.last[J.m - 1].n_cols;
  for (int idx = threadIdx.x; idx < n0 * K; idx += blockDim.x) {
    const int k = idx % K;
    xa[idx] = (idx < K) ? J.r1[min(i0 + k, J.I - 1)] : 0u;
  }
  __syncthreads();
  uint32_t* cur = xa;
  uint32_t* oth = xb;
  for (int i = J.m; i >= 1; --i) {
    apply(J.last[i - 1], cur, oth);
    uint32_t* t = cur;
    cur = oth;
    oth = t;
  }
  for (int s = threadIdx.x; s < J.s_nc; s += blockDim.x) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < nvalid) J.w[static_cast<size_t>(i0 + k) * J.s_nc + s] = cur[static_cast<uint32_t>(s) * K + k];
  }
  // (cur is xa when m is even: every copy must be done before xa changes)
  __syncthreads();
  // x = e0 on the NCNNN space; row 1 (the path of m sites) is its read-out.
  for (int idx = threadIdx.x; idx < J.s_nc * K; idx += blockDim.x) xa[idx] = (idx < K) ? 1u : 0u;
  __syncthreads();
  res_dot<K>(xa, wk, J.s_nc, p, pinv, red, J.out + i0, nvalid);
  cur = xa;
  oth = xb;
  for (int r = 1; r < J.n_max; ++r) {
    for (int f = 0; f < J.nf; ++f) {
      apply(J.fac[f], cur, oth);
      uint32_t* t = cur;
      cur = oth;
      oth = t;
    }
    res_dot<K>(cur, wk, J.s_nc, p, pinv, red, J.out + static_cast<size_t>(r) * J.I + i0, nvalid);
  }
}

}  // namespace cs
