// Runtime and C ABI of the chromatic-strip library.
//
// Evaluation form: the sweep computes P of the m x r rectangles, r =
// 1..n_max, as Z_r = <w, x_r>, x_1 = e_0, x_{r+1} = T_m ... T_1 x_r, and
// w = (T_1^last)^T ... (T_m^last)^T e_0 (arXiv 1005.3609, eqs. Z_from_T,
// T_sq_decomp, T_last).  w is built once per instance set on the device and
// kept in Montgomery form so the read-out is a plain dot product.
//
// Coefficient form (eq. Z_modified, Sec. 3.5): the states carry truncated
// polynomials in x = 1/q mod p, and T_last is applied to every row's state
// (a polynomial read-out vector would need a convolution per state).  Its
// factor maps are built on the device (devexpand.hpp, the k_dx_* kernels).
//
// Sections: device copies of the maps and the device map build; constants
// and job layouts; step programs (setup, rows, read-out); launches, chunk
// groups on parallel streams and hipGraph row replay; grouped launches for
// batches and the server; the resident mode (a whole strip per launch, the
// state vectors in LDS); the plain per-instance path; the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/chromstrip.h"
#include "devexpand.hpp"
#include "kernels.hpp"
#include "maps.hpp"
#include "opgather.hpp"
#include "pipeline.hpp"
#include "resident.hpp"
#include "states.hpp"

namespace cs {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct MemError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIPX(expr)                                                                  \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw HipError(std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const ArgError& e) {
    return fail(CHROM_EINVAL, e.what());
  } catch (const MemError& e) {
    return fail(CHROM_ENOMEM, e.what());
  } catch (const HipError& e) {
    return fail(CHROM_EDEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(CHROM_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(CHROM_EUNSUPPORTED, e.what());
  }
}

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Device copies of the factor maps, one per (device, lattice, m)
// ---------------------------------------------------------------------------
// A factor's staged tiles on the device (see StagedCsr).
struct DevStaged {
  DevCsr csr;                 // entries hold slots; row pointers the plain map's (clustered: tile order)
  const int32_t* tile_row0 = nullptr;
  const int32_t* tile_src0 = nullptr;
  const int32_t* src = nullptr;
  const int32_t* tgt = nullptr;   // clustered tiles: row written by each tile position
  const int32_t* tile_ent0 = nullptr;
  const uint32_t* ent_src = nullptr;   // clustered: entry words with sources, tile order
  int n_tiles = 0, max_slots = 0, max_rows = 0, max_ent = 0;
};
struct DevStagedSet {
  void* base = nullptr;
  std::vector<DevStaged> fac;
};
// A family's factors and the read-out maps in sliced-ELL form (resident.hpp).
struct DevSellSet {
  void* base = nullptr;
  std::vector<DevSell> fac, last;
  int max_row = 0;   // entries of the longest row over all maps
};

// A family's factors as op streams (opgather.hpp).
struct DevOps {
  const uint32_t* ops = nullptr;
  const int32_t* op_row = nullptr;
  int64_t n_cols = 0;
};
struct DevOpSet {
  void* base = nullptr;
  std::vector<DevOps> fac;
};

struct DevFamily {
  int k = 1;
  void* base = nullptr;
  std::vector<DevCsr> fac;
  std::vector<Poly> codes;   // extends the base table
  int shift = 0;             // kernels expand the codes in powers of t = q - shift
  bool general = false;      // some coefficient its factors use exceeds the fast path (|d| > 1; > 3 in the coefficient form)
  // staged copies, one set per (kind: 1 consecutive rows, 2 clustered;
  // slot limit; rows per tile), built on first use
  mutable std::mutex st_mu;
  mutable std::map<std::tuple<int, int, int>, std::unique_ptr<DevStagedSet>> staged;
  // sliced-ELL copies of the factors and read-out maps (resident mode), built
  // on first use: +-1 entries in their own columns (modular form) or every
  // entry in one group (double form)
  mutable std::unique_ptr<struct DevSellSet> sell, sell_one;
  // op streams of the factors (stage 5), built on first use
  mutable std::unique_ptr<DevOpSet> ops;
};

struct DevMaps {
  void* base = nullptr;
  size_t bytes = 0;
  DevCsr fwd[kMaxM];
  DevCsr last[kMaxM];
  DevCsr last_fwd[kMaxM];    // normalised sets: T_i^last in gather form
  bool normalised = false;
  int64_t l_max = 0;         // normalised sets: largest read-out space L_1 .. L_m
  std::vector<Poly> codes;   // base table of fwd and last
  int64_t s_nc = 0;    // NCNNN states
  int64_t s_max = 0;   // largest space
  int lattice = 0, m = 0;
  // built on the device (coefficient form): the per-factor allocations, and
  // whether some coefficient needs the general kernel path (|d| > 3)
  bool on_device = false;
  bool general_cf = false;
  std::vector<void*> allocs;
  // fused families (k >= 2), uploaded on first use
  mutable std::mutex fam_mu;
  mutable std::map<int, std::unique_ptr<DevFamily>> fam;
};

size_t csr_bytes(const Csr& c) { return align_up(c.row_ptr.size() * 4) + align_up(std::max<size_t>(c.ent.size(), 1) * 4); }

// Copies one CSR into device memory at `cur` (advanced).
void upload_csr(const Csr& c, DevCsr& d, char*& cur) {
  int32_t* rp = reinterpret_cast<int32_t*>(cur);
  HIPX(hipMemcpy(rp, c.row_ptr.data(), c.row_ptr.size() * 4, hipMemcpyHostToDevice));
  cur += align_up(c.row_ptr.size() * 4);
  uint32_t* en = reinterpret_cast<uint32_t*>(cur);
  if (!c.ent.empty()) HIPX(hipMemcpy(en, c.ent.data(), c.ent.size() * 4, hipMemcpyHostToDevice));
  cur += align_up(std::max<size_t>(c.ent.size(), 1) * 4);
  d.row_ptr = rp;
  d.ent = en;
  d.n_rows = static_cast<int>(c.n_rows);
  d.n_cols = static_cast<int>(c.n_cols);
}


// ---------------------------------------------------------------------------
// Coefficient-form maps built on the device.  Every source state of a
// factor is expanded by one thread (devexpand.hpp: unrank, the factor's
// single-edge operators, rank of each target); the gather-form CSR then
// follows from atomic row counts, a prefix sum, atomic row cursors and a
// per-row sort, so it does not depend on the schedule.  Two passes: the
// first only collects the coefficient keys of every factor (they fix the
// code table, numbered as the host builder numbers it), the second writes
// each factor's CSR with final codes.  States keep the paper's order.
// ---------------------------------------------------------------------------
constexpr int kKeyWords = (dx::kKeys + 31) / 32;

__global__ void __launch_bounds__(256, 8) k_dx_keys(dx::Factor f, const dx::Tables* tab, int64_t nin, uint32_t* keybits,
                                                 int* err) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nin) return;
  int32_t tg[dx::kTerms], ky[dx::kTerms];
  const int n = dx::expand_source(*tab, f, r, tg, ky);
  if (n < 0) {
    atomicOr(err, 1);
    return;
  }
  // Few distinct keys exist, so almost every bit is already set: a plain
  // read first keeps the atomics (all on a handful of words) rare.
  for (int j = 0; j < n; ++j) {
    const uint32_t bit = 1u << (ky[j] & 31);
    if (!(keybits[ky[j] >> 5] & bit)) atomicOr(&keybits[ky[j] >> 5], bit);  // a stale read only costs an atomic
  }
}

// Per source: up to kTerms (target, code) pairs, target -1 for unused slots.
__global__ void __launch_bounds__(256, 8) k_dx_expand(dx::Factor f, const dx::Tables* tab, int64_t nin,
                                                   const int8_t* code_of_key, int32_t* tgt, uint8_t* code,
                                                   int32_t* cnt, int* err) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nin) return;
  int32_t tg[dx::kTerms], ky[dx::kTerms];
  int n = dx::expand_source(*tab, f, r, tg, ky);
  if (n < 0) {
    atomicOr(err, 1);
    n = 0;
  }
  for (int j = 0; j < dx::kTerms; ++j) {
    const int c = j < n ? code_of_key[ky[j]] : 0;
    if (j < n && c < 0) atomicOr(err, 2);
    const bool use = j < n && c >= 0;
    tgt[r * dx::kTerms + j] = use ? tg[j] : -1;
    code[r * dx::kTerms + j] = static_cast<uint8_t>(use ? c : 0);
    if (use) atomicAdd(&cnt[tg[j]], 1);
  }
}

__global__ void __launch_bounds__(256) k_set_fill(int32_t* a, int64_t n, int32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Exclusive prefix sum, first level: blocks of 1024 counts scanned in LDS;
// block totals to sums[block].
__global__ void __launch_bounds__(1024) k_dx_scan_blocks(const int32_t* cnt, int64_t n, int32_t* out, int32_t* sums) {
  __shared__ int32_t s[1024];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 1024 + threadIdx.x;
  const int32_t v = i < n ? cnt[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t add = threadIdx.x >= static_cast<unsigned>(off) ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  if (i < n) out[i] = s[threadIdx.x] - v;
  if (threadIdx.x == 1023) sums[blockIdx.x] = s[1023];
}

__global__ void __launch_bounds__(1024) k_dx_scan_add(int32_t* out, int64_t n, const int32_t* offs) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 1024 + threadIdx.x;
  if (i < n) out[i] += offs[blockIdx.x];
}

__global__ void __launch_bounds__(256) k_dx_fill(const int32_t* tgt, const uint8_t* code, int64_t nslots,
                                                 const int32_t* row_ptr, int32_t* cur, uint32_t* ent) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nslots) return;
  const int32_t t = tgt[e];
  if (t < 0) return;
  const int32_t pos = row_ptr[t] + atomicAdd(&cur[t], 1);
  ent[pos] = static_cast<uint32_t>(e / dx::kTerms) | (static_cast<uint32_t>(code[e]) << kSrcBits);
}

// Each row's entries by source, then code (insertion sort: rows are short).
__global__ void __launch_bounds__(256) k_dx_sort_rows(const int32_t* row_ptr, int64_t nrows, uint32_t* ent) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int32_t a0 = row_ptr[r], a1 = row_ptr[r + 1];
  for (int32_t a = a0 + 1; a < a1; ++a) {
    const uint32_t v = ent[a];
    int32_t b = a;
    while (b > a0) {
      const uint32_t u = ent[b - 1];
      const bool after = (u & kSrcMask) > (v & kSrcMask) || ((u & kSrcMask) == (v & kSrcMask) && u > v);
      if (!after) break;
      ent[b] = u;
      --b;
    }
    ent[b] = v;
  }
}

// Codes in the host builder's numbering: +1, -1, then every other key seen,
// ascending.  code_of_key: kKeys entries, -1 for keys not seen.
std::vector<Poly> codes_from_keys(const std::vector<uint32_t>& keybits, std::vector<int8_t>& code_of_key) {
  auto poly_of = [](int key) {
    Poly p;
    for (int k = 0; k <= kMaxDeg; ++k) {
      p.c[k] = key % dx::kKeyBase - dx::kKeyOff;
      key /= dx::kKeyBase;
    }
    return p;
  };
  auto key_of = [](int c0) {
    int8_t c[4] = {static_cast<int8_t>(c0), 0, 0, 0};
    return dx::coef_key(c);
  };
  code_of_key.assign(dx::kKeys, -1);
  std::vector<Poly> codes;
  auto add = [&](int key) {
    if (code_of_key[key] >= 0) return;
    if (static_cast<int>(codes.size()) >= kMaxCodes) throw std::runtime_error("too many distinct coefficients");
    code_of_key[key] = static_cast<int8_t>(codes.size());
    codes.push_back(poly_of(key));
  };
  add(key_of(1));
  add(key_of(-1));
  for (int k = 0; k < dx::kKeys; ++k)
    if ((keybits[k >> 5] >> (k & 31)) & 1u) add(k);
  return codes;
}

// Temporary device buffer of the builder.
struct DxBuf {
  void* p = nullptr;
  explicit DxBuf(size_t n) {
    if (n && hipMalloc(&p, n) != hipSuccess) throw MemError("device allocation of " + std::to_string(n) + " bytes failed");
  }
  ~DxBuf() {
    if (p) (void)hipFree(p);
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

unsigned dx_blocks(int64_t n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

// out[0..n] = exclusive prefix sums of in[0..n-1] (out[n] = total), on the
// device; block totals are combined on the host.  `sums` holds at least
// dx_blocks(n, 1024) words.  Returns the total.
int64_t dx_exclusive_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* sums) {
  const unsigned nb = dx_blocks(std::max<int64_t>(n, 1), 1024);
  hipLaunchKernelGGL(k_dx_scan_blocks, dim3(nb), dim3(1024), 0, nullptr, in, n, out, sums);
  HIPX(hipGetLastError());
  std::vector<int32_t> hs(nb);
  HIPX(hipMemcpy(hs.data(), sums, nb * 4, hipMemcpyDeviceToHost));
  int64_t total = 0;
  for (unsigned b = 0; b < nb; ++b) {
    const int64_t v = hs[b];
    hs[b] = static_cast<int32_t>(total);
    total += v;
    if (total > INT32_MAX) throw std::runtime_error("prefix sum beyond 32 bits");
  }
  const int32_t t32 = static_cast<int32_t>(total);
  HIPX(hipMemcpy(sums, hs.data(), nb * 4, hipMemcpyHostToDevice));
  HIPX(hipMemcpy(out + n, &t32, 4, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_dx_scan_add, dim3(nb), dim3(1024), 0, nullptr, out, n, sums);
  HIPX(hipGetLastError());
  return total;
}

// Reader order on the device (the host builder's rule): going backwards
// over the forward factors, the states between F_k and F_{k+1} are ordered
// by the first row of F_{k+1}, in its own new order, that reads them (ties
// by old rank), unread states last.  first[s] = that row (nrows if none).
__global__ void __launch_bounds__(256) k_ro_first(const int32_t* row_ptr, const uint32_t* ent, int64_t nrows,
                                                  const int32_t* perm_rows, int32_t* first) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int32_t nr = perm_rows ? perm_rows[r] : static_cast<int32_t>(r);
  for (int32_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) atomicMin(&first[ent[e] & kSrcMask], nr);
}

// cnt[row] = states first read by that (new) row; unread[s] = 1 for states no row reads.
__global__ void __launch_bounds__(256) k_ro_count(const int32_t* first, int64_t ns, int64_t nrows, int32_t* cnt,
                                                  int32_t* unread) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const int32_t f = first[s];
  unread[s] = f >= nrows ? 1 : 0;
  if (f < nrows) atomicAdd(&cnt[f], 1);
}

// A row's first-read states, in column (old rank) order, take consecutive
// positions from its bucket's start.
__global__ void __launch_bounds__(256) k_ro_assign(const int32_t* row_ptr, const uint32_t* ent, int64_t nrows,
                                                   const int32_t* perm_rows, const int32_t* first,
                                                   const int32_t* start, int32_t* perm) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int32_t nr = perm_rows ? perm_rows[r] : static_cast<int32_t>(r);
  int32_t j = start[nr];
  for (int32_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
    const uint32_t s = ent[e] & kSrcMask;
    if (first[s] == nr) perm[s] = j++;
  }
}

__global__ void __launch_bounds__(256) k_ro_unread(const int32_t* first, int64_t ns, int64_t nrows,
                                                   const int32_t* upos, int32_t base, int32_t* perm) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  if (first[s] >= nrows) perm[s] = base + upos[s];
}

// Renumbering of one factor: new row lengths, then entries copied with new
// columns (rows sorted afterwards by k_dx_sort_rows).
__global__ void __launch_bounds__(256) k_rn_len(const int32_t* row_ptr, int64_t nrows, const int32_t* perm_rows,
                                                int32_t* len) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  len[perm_rows ? perm_rows[r] : r] = row_ptr[r + 1] - row_ptr[r];
}

__global__ void __launch_bounds__(256) k_rn_fill(const int32_t* row_ptr, const uint32_t* ent, int64_t nrows,
                                                 const int32_t* perm_rows, const int32_t* perm_cols,
                                                 const int32_t* new_row_ptr, uint32_t* new_ent) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int32_t w = new_row_ptr[perm_rows ? perm_rows[r] : r];
  for (int32_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
    const uint32_t c = ent[e] & kSrcMask, code = ent[e] & ~kSrcMask;
    new_ent[w++] = (perm_cols ? static_cast<uint32_t>(perm_cols[c]) : c) | code;
  }
}

// Applies the reader order to the forward factors of a device-built set:
// fwd[k] (F_{k+1}) has rows in space k+1 and columns in space k; spaces 0
// and m (NCNNN, before and after the row) keep the paper's order.
void device_reader_order(DevMaps& dm, int m) {
  if (m < 2) return;
  std::vector<DxBuf*> perm(m + 1, nullptr);   // perm[k][old] = new, space after F_k
  std::vector<std::unique_ptr<DxBuf>> own;
  int64_t big = 1;
  for (int k = 0; k < m; ++k) big = std::max<int64_t>(big, std::max(dm.fwd[k].n_rows, dm.fwd[k].n_cols));
  DxBuf first((big + 1) * 4), cnt((big + 1) * 4), start((big + 2) * 4), unread((big + 1) * 4),
      upos((big + 2) * 4), sums(dx_blocks(big + 1, 1024) * 4 + 64);
  for (int k = m - 1; k >= 1; --k) {
    const DevCsr& t = dm.fwd[k];   // F_{k+1}
    const int64_t ns = t.n_cols, nrows = t.n_rows;
    const int32_t* prow = perm[k + 1] ? perm[k + 1]->as<int32_t>() : nullptr;
    hipLaunchKernelGGL(k_set_fill, dim3(dx_blocks(ns, 256)), dim3(256), 0, nullptr, first.as<int32_t>(), ns,
                       static_cast<int32_t>(nrows));
    hipLaunchKernelGGL(k_ro_first, dim3(dx_blocks(nrows, 256)), dim3(256), 0, nullptr, t.row_ptr, t.ent, nrows, prow,
                       first.as<int32_t>());
    HIPX(hipMemset(cnt.p, 0, nrows * 4));
    hipLaunchKernelGGL(k_ro_count, dim3(dx_blocks(ns, 256)), dim3(256), 0, nullptr, first.as<int32_t>(), ns, nrows,
                       cnt.as<int32_t>(), unread.as<int32_t>());
    const int64_t nread = dx_exclusive_scan(cnt.as<int32_t>(), nrows, start.as<int32_t>(), sums.as<int32_t>());
    (void)dx_exclusive_scan(unread.as<int32_t>(), ns, upos.as<int32_t>(), sums.as<int32_t>());
    own.push_back(std::make_unique<DxBuf>(ns * 4));
    perm[k] = own.back().get();
    hipLaunchKernelGGL(k_ro_assign, dim3(dx_blocks(nrows, 256)), dim3(256), 0, nullptr, t.row_ptr, t.ent, nrows,
                       prow, first.as<int32_t>(), start.as<int32_t>(), perm[k]->as<int32_t>());
    hipLaunchKernelGGL(k_ro_unread, dim3(dx_blocks(ns, 256)), dim3(256), 0, nullptr, first.as<int32_t>(), ns, nrows,
                       upos.as<int32_t>(), static_cast<int32_t>(nread), perm[k]->as<int32_t>());
    HIPX(hipGetLastError());
  }
  for (int k = 0; k < m; ++k) {
    DevCsr& c = dm.fwd[k];
    const int64_t nrows = c.n_rows;
    const int32_t* prow = perm[k + 1] ? perm[k + 1]->as<int32_t>() : nullptr;
    const int32_t* pcol = perm[k] ? perm[k]->as<int32_t>() : nullptr;
    hipLaunchKernelGGL(k_rn_len, dim3(dx_blocks(nrows, 256)), dim3(256), 0, nullptr, c.row_ptr, nrows, prow,
                       cnt.as<int32_t>());
    void* rp = nullptr;
    void* ep = nullptr;
    if (hipMalloc(&rp, (nrows + 1) * 4) != hipSuccess) throw MemError("device allocation of factor maps failed");
    dm.allocs.push_back(rp);
    const int64_t nnz = dx_exclusive_scan(cnt.as<int32_t>(), nrows, static_cast<int32_t*>(rp), sums.as<int32_t>());
    if (hipMalloc(&ep, std::max<int64_t>(nnz, 1) * 4) != hipSuccess)
      throw MemError("device allocation of factor maps failed");
    dm.allocs.push_back(ep);
    hipLaunchKernelGGL(k_rn_fill, dim3(dx_blocks(nrows, 256)), dim3(256), 0, nullptr, c.row_ptr, c.ent, nrows, prow,
                       pcol, static_cast<int32_t*>(rp), static_cast<uint32_t*>(ep));
    hipLaunchKernelGGL(k_dx_sort_rows, dim3(dx_blocks(nrows, 256)), dim3(256), 0, nullptr,
                       static_cast<const int32_t*>(rp), nrows, static_cast<uint32_t*>(ep));
    HIPX(hipGetLastError());
    HIPX(hipDeviceSynchronize());
    // the old arrays go
    for (auto it = dm.allocs.begin(); it != dm.allocs.end();) {
      if (*it == static_cast<const void*>(c.row_ptr) || *it == static_cast<const void*>(c.ent)) {
        (void)hipFree(*it);
        it = dm.allocs.erase(it);
      } else {
        ++it;
      }
    }
    c.row_ptr = static_cast<const int32_t*>(rp);
    c.ent = static_cast<const uint32_t*>(ep);
  }
}

// Builds the forward and read-out maps of the coefficient form of
// (lattice, m) on the current device.
std::unique_ptr<DevMaps> build_dev_maps_cf(int lattice, int m) {
  dx::Tables th;
  dx::make_tables(th);
  std::vector<dx::Factor> fac;
  for (int i = 1; i <= m; ++i) fac.push_back(dx::forward_factor(lattice, m, i, true));
  for (int i = 1; i <= m; ++i) fac.push_back(dx::last_factor(lattice, m, i, true));
  int64_t in_max = 1, out_max = 1;
  for (const dx::Factor& f : fac) {
    in_max = std::max(in_max, dx::space_size(th, f.in));
    out_max = std::max(out_max, dx::space_size(th, f.out));
  }
  if (in_max > static_cast<int64_t>(kSrcMask) || out_max > static_cast<int64_t>(kSrcMask))
    throw std::runtime_error("state space too large for 26-bit ranks");
  DxBuf tab(sizeof(dx::Tables)), keybits(kKeyWords * 4), err(4), code_map(dx::kKeys);
  HIPX(hipMemcpy(tab.p, &th, sizeof th, hipMemcpyHostToDevice));
  HIPX(hipMemset(keybits.p, 0, kKeyWords * 4));
  HIPX(hipMemset(err.p, 0, 4));
  // pass 1: coefficient keys of every factor
  for (const dx::Factor& f : fac) {
    const int64_t nin = dx::space_size(th, f.in);
    hipLaunchKernelGGL(k_dx_keys, dim3(dx_blocks(nin, 256)), dim3(256), 0, nullptr, f, tab.as<dx::Tables>(), nin,
                       keybits.as<uint32_t>(), err.as<int>());
  }
  HIPX(hipGetLastError());
  std::vector<uint32_t> kb(kKeyWords);
  int herr = 0;
  HIPX(hipMemcpy(kb.data(), keybits.p, kKeyWords * 4, hipMemcpyDeviceToHost));
  HIPX(hipMemcpy(&herr, err.p, 4, hipMemcpyDeviceToHost));
  if (herr) throw std::runtime_error("device map build: an expansion left the supported coefficient range");
  std::vector<int8_t> cok;
  auto dm = std::make_unique<DevMaps>();
  dm->codes = codes_from_keys(kb, cok);
  HIPX(hipMemcpy(code_map.p, cok.data(), cok.size(), hipMemcpyHostToDevice));
  for (const Poly& c : dm->codes)
    for (int k = 0; k <= kMaxDeg; ++k) dm->general_cf = dm->general_cf || c.c[k] > 3 || c.c[k] < -3;
  // pass 2: one factor at a time
  const int64_t nslots_max = in_max * dx::kTerms;
  DxBuf tgt(nslots_max * 4), code(nslots_max), cnt(out_max * 4), cur(out_max * 4),
      sums(dx_blocks(out_max, 1024) * 4);
  try {
    for (size_t fi = 0; fi < fac.size(); ++fi) {
      const dx::Factor& f = fac[fi];
      const int64_t nin = dx::space_size(th, f.in), nout = dx::space_size(th, f.out);
      HIPX(hipMemset(cnt.p, 0, nout * 4));
      hipLaunchKernelGGL(k_dx_expand, dim3(dx_blocks(nin, 256)), dim3(256), 0, nullptr, f, tab.as<dx::Tables>(), nin,
                         code_map.as<int8_t>(), tgt.as<int32_t>(), code.as<uint8_t>(), cnt.as<int32_t>(), err.as<int>());
      void* rp = nullptr;
      if (hipMalloc(&rp, (nout + 1) * 4) != hipSuccess) throw MemError("device allocation of factor maps failed");
      dm->allocs.push_back(rp);
      int32_t* row_ptr = static_cast<int32_t*>(rp);
      const int32_t nnz = static_cast<int32_t>(dx_exclusive_scan(cnt.as<int32_t>(), nout, row_ptr, sums.as<int32_t>()));
      HIPX(hipMemcpy(&herr, err.p, 4, hipMemcpyDeviceToHost));
      if (herr) throw std::runtime_error("device map build: an expansion failed");
      void* ep = nullptr;
      if (hipMalloc(&ep, std::max<int64_t>(nnz, 1) * 4) != hipSuccess)
        throw MemError("device allocation of factor maps failed");
      dm->allocs.push_back(ep);
      uint32_t* ent = static_cast<uint32_t*>(ep);
      HIPX(hipMemset(cur.p, 0, nout * 4));
      hipLaunchKernelGGL(k_dx_fill, dim3(dx_blocks(nin * dx::kTerms, 256)), dim3(256), 0, nullptr, tgt.as<int32_t>(),
                         code.as<uint8_t>(), nin * dx::kTerms, row_ptr, cur.as<int32_t>(), ent);
      hipLaunchKernelGGL(k_dx_sort_rows, dim3(dx_blocks(nout, 256)), dim3(256), 0, nullptr, row_ptr, nout, ent);
      HIPX(hipGetLastError());
      HIPX(hipDeviceSynchronize());
      DevCsr d{row_ptr, ent, static_cast<int>(nout), static_cast<int>(nin)};
      if (fi < static_cast<size_t>(m)) {
        dm->fwd[fi] = d;
      } else {
        dm->last_fwd[fi - m] = d;
        dm->l_max = std::max<int64_t>(dm->l_max, nout);
      }
    }
    const char* order = std::getenv("CHROMSTRIP_STATE_ORDER");
    if (!(order && std::string(order) == "paper")) device_reader_order(*dm, m);
  } catch (...) {
    (void)hipDeviceSynchronize();
    for (void* a : dm->allocs) (void)hipFree(a);
    throw;
  }
  dm->normalised = true;
  dm->on_device = true;
  dm->lattice = lattice;
  dm->m = m;
  dm->s_nc = ncnnn_count(m);
  dm->s_max = (lattice == kSquare && m >= 2) ? ncnnn_count(m) + ncnnn_count(m - 1) : ncnnn_count(m);
  return dm;
}

// The builder's expansion and CSR assembly run on the host (same functions,
// same order of operations) and compared with the host builder's maps in
// the paper's state order: every forward factor, and for the coefficient
// form every read-out factor in gather form.  Returns "" or the first
// difference.
std::string check_expansion(int lattice, int m, bool normalised) {
  dx::Tables th;
  dx::make_tables(th);
  std::unique_ptr<MapSet> ms = build_maps(lattice, m, 0, normalised, true);
  std::vector<dx::Factor> fac;
  for (int i = 1; i <= m; ++i) fac.push_back(dx::forward_factor(lattice, m, i, normalised));
  if (normalised)
    for (int i = 1; i <= m; ++i) fac.push_back(dx::last_factor(lattice, m, i, normalised));
  std::vector<uint32_t> kb(kKeyWords, 0u);
  int32_t tg[dx::kTerms], ky[dx::kTerms];
  for (const dx::Factor& f : fac) {
    const int64_t nin = dx::space_size(th, f.in);
    for (int64_t r = 0; r < nin; ++r) {
      const int n = dx::expand_source(th, f, r, tg, ky);
      if (n < 0) return "expansion failed for a source state";
      for (int j = 0; j < n; ++j) kb[ky[j] >> 5] |= 1u << (ky[j] & 31);
    }
  }
  std::vector<int8_t> cok;
  std::vector<Poly> codes = codes_from_keys(kb, cok);
  if (!normalised) {
    // the host's evaluation-form table also holds the read-out factors' codes
    if (codes.size() > ms->codes.size()) return "code table larger than the host's";
  } else if (codes.size() != ms->codes.size()) {
    return "code table size differs";
  }
  for (size_t c = 0; c < codes.size(); ++c)
    for (int k = 0; k <= kMaxDeg; ++k)
      if (codes[c].c[k] != ms->codes[c].c[k] && normalised) return "code table differs";
  for (size_t fi = 0; fi < fac.size(); ++fi) {
    const dx::Factor& f = fac[fi];
    const Csr& h = fi < static_cast<size_t>(m) ? ms->fwd[fi] : ms->last_fwd[fi - m];
    const int64_t nin = dx::space_size(th, f.in), nout = dx::space_size(th, f.out);
    if (h.n_rows != nout || h.n_cols != nin) return "space sizes differ at factor " + std::to_string(fi);
    std::vector<std::vector<uint32_t>> rows(nout);
    for (int64_t r = 0; r < nin; ++r) {
      const int n = dx::expand_source(th, f, r, tg, ky);
      for (int j = 0; j < n; ++j) {
        // codes by the host table's numbering (same keys, same order)
        const Poly want = codes[cok[ky[j]]];
        int hc = -1;
        for (size_t c = 0; c < ms->codes.size() && hc < 0; ++c) {
          bool eq = true;
          for (int k = 0; k <= kMaxDeg; ++k) eq = eq && ms->codes[c].c[k] == want.c[k];
          if (eq) hc = static_cast<int>(c);
        }
        if (hc < 0) return "coefficient missing from the host table";
        rows[tg[j]].push_back(static_cast<uint32_t>(r) | (static_cast<uint32_t>(hc) << kSrcBits));
      }
    }
    for (int64_t t = 0; t < nout; ++t) {
      std::vector<uint32_t>& v = rows[t];
      std::sort(v.begin(), v.end(), [](uint32_t a, uint32_t b) {
        return (a & kSrcMask) != (b & kSrcMask) ? (a & kSrcMask) < (b & kSrcMask) : a < b;
      });
      const int64_t a0 = h.row_ptr[t], a1 = h.row_ptr[t + 1];
      if (a1 - a0 != static_cast<int64_t>(v.size())) return "row length differs at factor " + std::to_string(fi);
      for (int64_t a = a0; a < a1; ++a)
        if (h.ent[a] != v[a - a0]) return "entry differs at factor " + std::to_string(fi);
    }
  }
  return "";
}

std::mutex g_dev_mu;
std::map<std::tuple<int, int, int, int>, std::unique_ptr<DevMaps>> g_dev;

// Where the coefficient form's maps are built: on the device unless
// CHROMSTRIP_HOST_MAPS=1 (host build and upload, reader order).
bool cf_maps_on_device() {
  const char* v = std::getenv("CHROMSTRIP_HOST_MAPS");
  return !(v && std::string(v) == "1");
}

// Device copy of the maps of (lattice, m) in the un-normalised (evaluation)
// or normalised (coefficient) form.
const DevMaps& dev_maps(int lattice, int m, bool normalised = false) {
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto key = std::make_tuple(dev, lattice, m, normalised ? 1 : 0);
  auto it = g_dev.find(key);
  if (it != g_dev.end()) return *it->second;
  if (normalised && cf_maps_on_device()) {
    auto dm = build_dev_maps_cf(lattice, m);
    const DevMaps& ref = *dm;
    g_dev.emplace(key, std::move(dm));
    return ref;
  }
  const MapSet& ms = get_maps(lattice, m, normalised);
  auto dm = std::make_unique<DevMaps>();
  size_t bytes = 0;
  for (int i = 0; i < m; ++i) bytes += csr_bytes(ms.fwd[i]) + (normalised ? 0 : csr_bytes(ms.last[i]));
  for (const Csr& c : ms.last_fwd) bytes += csr_bytes(c);
  void* base = nullptr;
  if (hipMalloc(&base, bytes) != hipSuccess) throw MemError("device allocation of factor maps failed");
  char* cur = static_cast<char*>(base);
  for (int i = 0; i < m; ++i) {
    upload_csr(ms.fwd[i], dm->fwd[i], cur);
    if (!normalised) upload_csr(ms.last[i], dm->last[i], cur);
  }
  for (size_t i = 0; i < ms.last_fwd.size(); ++i) {
    upload_csr(ms.last_fwd[i], dm->last_fwd[i], cur);
    dm->l_max = std::max<int64_t>(dm->l_max, ms.last_fwd[i].n_rows);
  }
  dm->normalised = normalised;
  dm->base = base;
  dm->bytes = bytes;
  dm->codes = ms.codes;
  dm->lattice = lattice;
  dm->m = m;
  dm->s_nc = ncnnn_count(m);
  dm->s_max = ms.max_states();
  const DevMaps& ref = *dm;
  g_dev.emplace(key, std::move(dm));
  return ref;
}

// Coefficients of c(q) in powers of t = q - s: d_j = sum_{k >= j} c_k C(k, j) s^(k-j).
Poly shift_basis(const Poly& c, int s) {
  static const int64_t binom[kMaxDeg + 1][kMaxDeg + 1] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
  Poly d;
  for (int j = 0; j <= kMaxDeg; ++j) {
    int64_t acc = 0, sp = 1;
    for (int k = j; k <= kMaxDeg; ++k) {
      acc += c.c[k] * binom[k][j] * sp;
      sp *= s;
    }
    d.c[j] = acc;
  }
  return d;
}

// Modular additions the factor kernel spends on one entry with code
// polynomial d: a coefficient of magnitude n costs floor(log2 n) doublings,
// popcount(n) - 1 further additions and the final one.
int64_t entry_cost(const Poly& d) {
  int64_t ops = 0;
  for (int k = 0; k <= kMaxDeg; ++k) {
    const int64_t n = d.c[k] < 0 ? -d.c[k] : d.c[k];
    if (n == 0) continue;
    if (n > 127) return -1;   // outside the packed table
    ops += (63 - __builtin_clzll(static_cast<uint64_t>(n))) + __builtin_popcountll(static_cast<uint64_t>(n));
  }
  return ops;
}

// Basis shift for a family: one under which every coefficient its factors
// use is 0 or +-1 if there is one (their launches then run the factor kernel
// without its general path), else any; among those, the fewest modular
// additions over the family's entries, ties to the smallest |s|.  Every code
// of the table (also those only the read-out factors use) must fit the
// packed range.
int choose_shift(const std::vector<Poly>& codes, const std::vector<Csr>& fac, bool& general) {
  std::vector<int64_t> count(codes.size(), 0);
  for (const Csr& c : fac)
    for (uint32_t e : c.ent) ++count[e >> kSrcBits];
  int best = 0;
  int64_t best_cost = -1;
  bool best_general = true;
  for (int s : {0, 1, -1, 2, -2, 3, -3, 4, -4}) {
    int64_t cost = 0;
    bool ok = true, gen = false;
    for (size_t c = 0; c < codes.size() && ok; ++c) {
      const Poly d = shift_basis(codes[c], s);
      const int64_t e = entry_cost(d);
      if (e < 0) ok = false;
      cost += e * count[c];
      if (count[c] > 0)
        for (int k = 0; k <= kMaxDeg; ++k) gen = gen || d.c[k] > 1 || d.c[k] < -1;
    }
    if (!ok) continue;
    const bool better = best_cost < 0 || (best_general && !gen) || (best_general == gen && cost < best_cost);
    if (better) {
      best = s;
      best_cost = cost;
      best_general = gen;
    }
  }
  if (best_cost < 0) throw std::runtime_error("no basis shift keeps the coefficient polynomials in the packed range");
  general = best_general;
  return best;
}

// Device copy of fused family k (k = 1: the single factors).
const DevFamily& dev_family(const DevMaps& dm, int k) {
  std::lock_guard<std::mutex> lk(dm.fam_mu);
  auto it = dm.fam.find(k);
  if (it != dm.fam.end()) return *it->second;
  auto df = std::make_unique<DevFamily>();
  df->k = k;
  if (dm.normalised) {
    // coefficient form: the kernels' Horner variable is x itself (no shift)
    if (k != 1) throw ArgError("the coefficient form runs single factors only (fuse 1)");
    df->fac.assign(dm.fwd, dm.fwd + dm.m);
    df->codes = dm.codes;
    df->shift = 0;
    if (dm.on_device) {
      df->general = dm.general_cf;
      const DevFamily& r = *df;
      dm.fam.emplace(k, std::move(df));
      return r;
    }
    const MapSet& ms = get_maps(dm.lattice, dm.m, true);
    std::vector<bool> used(dm.codes.size(), false);
    for (const Csr& c : ms.fwd)
      for (uint32_t e : c.ent) used[e >> kSrcBits] = true;
    for (const Csr& c : ms.last_fwd)
      for (uint32_t e : c.ent) used[e >> kSrcBits] = true;
    // the coefficient-form kernels take |d| <= 3 on their fast path
    for (size_t c = 0; c < dm.codes.size(); ++c)
      for (int d = 0; d <= kMaxDeg && used[c]; ++d)
        df->general = df->general || dm.codes[c].c[d] > 3 || dm.codes[c].c[d] < -3;
  } else if (k == 1) {
    df->fac.assign(dm.fwd, dm.fwd + dm.m);
    df->codes = dm.codes;
    df->shift = choose_shift(dm.codes, get_maps(dm.lattice, dm.m).fwd, df->general);
  } else {
    const Family& f = get_maps(dm.lattice, dm.m).family(k);
    size_t bytes = 0;
    for (const Csr& c : f.fac) bytes += csr_bytes(c);
    if (hipMalloc(&df->base, bytes) != hipSuccess) throw MemError("device allocation of fused maps failed");
    char* cur = static_cast<char*>(df->base);
    df->fac.resize(f.fac.size());
    for (size_t i = 0; i < f.fac.size(); ++i) upload_csr(f.fac[i], df->fac[i], cur);
    df->codes = f.codes;
    df->shift = choose_shift(f.codes, f.fac, df->general);
  }
  const DevFamily& ref = *df;
  dm.fam.emplace(k, std::move(df));
  return ref;
}

// Slot limit of a staged tile: 48 KiB of LDS (rows of 64 V words).
int stage_slots(int V) { return 48 * 1024 / (256 * V); }
constexpr int kStageMaxLds = 64 * 1024;
constexpr size_t kPipeMaxLds = 64 * 1024;

// Tiles per workgroup of the pipelined staging: about 8, fewer where that
// would leave under 2048 workgroups over all chunks; at most 63.
int pipe_tiles_per_block(int n_tiles, int nchunk) {
  const long total = static_cast<long>(n_tiles) * std::max(nchunk, 1);
  return static_cast<int>(std::max<long>(1, std::min<long>(8, total / 2048)));
}

// Device copies of family fam's factors cut into staged tiles: kind 1 runs
// of consecutive rows, kind 2 clustered tiles (build_clustered; the factors
// are clustered on parallel host threads).
const DevStagedSet& dev_staged(const DevMaps& dm, const DevFamily& fam, int slots, int rows, int kind = 1) {
  std::lock_guard<std::mutex> lk(fam.st_mu);
  auto key = std::make_tuple(kind, slots, rows);
  auto it = fam.staged.find(key);
  if (it != fam.staged.end()) return *it->second;
  const MapSet& ms = get_maps(dm.lattice, dm.m);
  const std::vector<Csr>& host = (fam.k == 1) ? ms.fwd : ms.family(fam.k).fac;
  std::vector<StagedCsr> st(host.size());
  if (kind == 3) {
    // interleaved order: `slots` carries the wavefronts per workgroup; the
    // last factor's targets, the NCNNN states in the paper's order, are
    // first taken in their natural-label order (its readers' sources then
    // lie close together, as the site order does for the other spaces)
    const std::vector<int32_t> nat = ncnnn_natural_order(dm.m);
    for (size_t i = 0; i < host.size(); ++i)
      st[i] = build_interleaved(host[i], rows, slots, i + 1 == host.size() ? &nat : nullptr);
  } else if (kind == 2) {
    std::vector<std::thread> th;
    std::vector<std::string> err(host.size());
    for (size_t i = 0; i < host.size(); ++i)
      th.emplace_back([&, i] {
        try {
          st[i] = build_clustered(host[i], slots, rows, kPipeMaxEnt);
        } catch (const std::exception& e) {
          err[i] = e.what();
        }
      });
    for (auto& t : th) t.join();
    for (const std::string& e : err)
      if (!e.empty()) throw std::runtime_error(e);
  } else {
    for (size_t i = 0; i < host.size(); ++i) st[i] = build_staged(host[i], slots, rows);
  }
  size_t bytes = 0;
  for (size_t i = 0; i < host.size(); ++i)
    bytes += align_up(st[i].ent.size() * 4 + 4) + align_up(st[i].tile_row0.size() * 4 + 4) +
             align_up(st[i].tile_src0.size() * 4 + 4) + align_up(st[i].src.size() * 4 + 4) +
             align_up(st[i].tgt.size() * 4 + 4) + align_up(st[i].row_ptr.size() * 4 + 4) +
             align_up(st[i].tile_ent0.size() * 4 + 4) + align_up(st[i].ent_src.size() * 4 + 4);
  auto set = std::make_unique<DevStagedSet>();
  if (hipMalloc(&set->base, bytes) != hipSuccess) throw MemError("device allocation of staged maps failed");
  char* cur = static_cast<char*>(set->base);
  auto put = [&](const void* src, size_t n) {
    void* dst = cur;
    if (n) HIPX(hipMemcpy(dst, src, n, hipMemcpyHostToDevice));
    cur += align_up(n + 4);
    return dst;
  };
  set->fac.resize(host.size());
  for (size_t i = 0; i < host.size(); ++i) {
    DevStaged& d = set->fac[i];
    d.csr = fam.fac[i];
    d.csr.ent = static_cast<const uint32_t*>(put(st[i].ent.data(), st[i].ent.size() * 4));
    d.tile_row0 = static_cast<const int32_t*>(put(st[i].tile_row0.data(), st[i].tile_row0.size() * 4));
    d.tile_src0 = static_cast<const int32_t*>(put(st[i].tile_src0.data(), st[i].tile_src0.size() * 4));
    d.src = static_cast<const int32_t*>(put(st[i].src.data(), st[i].src.size() * 4));
    if (kind >= 2) {
      d.tgt = static_cast<const int32_t*>(put(st[i].tgt.data(), st[i].tgt.size() * 4));
      d.csr.row_ptr = static_cast<const int32_t*>(put(st[i].row_ptr.data(), st[i].row_ptr.size() * 4));
      d.ent_src = static_cast<const uint32_t*>(put(st[i].ent_src.data(), st[i].ent_src.size() * 4));
    }
    d.tile_ent0 = static_cast<const int32_t*>(put(st[i].tile_ent0.data(), st[i].tile_ent0.size() * 4));
    d.n_tiles = st[i].n_tiles();
    d.max_slots = st[i].max_slots;
    d.max_rows = st[i].max_rows;
    d.max_ent = st[i].max_ent;
  }
  const DevStagedSet& ref = *set;
  fam.staged.emplace(key, std::move(set));
  return ref;
}

// Op stream of one factor (opgather.hpp): one word per entry, source |
// unit digits of its coefficient in powers of t = q - shift << 24 | row end
// << 31, one digit-less word for a row without entries, kOpPad zero words
// after the last row; rows[r] = the first word of row r (n_rows + 1).
// ArgError when a code the factor uses has a digit outside -1..1 or a t^3
// term, or a source state does not fit the word.
void build_op_stream(const Csr& c, const std::vector<Poly>& codes, int shift, std::vector<uint32_t>& w,
                     std::vector<int32_t>& rp) {
  uint32_t digits[kMaxCodes];
  bool unit[kMaxCodes];
  for (size_t k = 0; k < codes.size(); ++k) {
    const Poly d = shift_basis(codes[k], shift);
    unit[k] = d.c[3] == 0;
    digits[k] = 0;
    for (int j = 0; j < 3; ++j) {
      if (d.c[j] > 1 || d.c[j] < -1) unit[k] = false;
      if (d.c[j] == 1) digits[k] |= 1u << (2 * j);
      if (d.c[j] == -1) digits[k] |= 2u << (2 * j);
    }
  }
  if (c.n_cols > static_cast<int64_t>(kOpSrcMask)) throw ArgError("op-stream gathers: source space too large");
  w.clear();
  w.reserve(c.ent.size() + static_cast<size_t>(c.n_rows) + kOpPad);
  rp.assign(c.n_rows + 1, 0);
  for (int64_t r = 0; r < c.n_rows; ++r) {
    rp[r] = static_cast<int32_t>(w.size());
    const int32_t e0 = c.row_ptr[r], e1 = c.row_ptr[r + 1];
    if (e0 == e1) w.push_back(kOpRowEnd);
    for (int32_t e = e0; e < e1; ++e) {
      const uint32_t code = c.ent[e] >> kSrcBits;
      if (code >= codes.size() || !unit[code])
        throw ArgError("op-stream gathers need unit coefficients in powers of t, up to t^2");
      w.push_back((c.ent[e] & kSrcMask) | (digits[code] << 24) | (e + 1 == e1 ? kOpRowEnd : 0u));
    }
  }
  rp[c.n_rows] = static_cast<int32_t>(w.size());
  if (w.size() + kOpPad > static_cast<size_t>(INT32_MAX)) throw ArgError("op-stream gathers: too many entries");
  w.resize(w.size() + kOpPad, 0u);
}

// Op streams of a family's factors (stage 5), built on first use.
// Evaluation form only.
const DevOpSet& dev_ops(const DevMaps& dm, const DevFamily& fam) {
  std::lock_guard<std::mutex> lk(fam.st_mu);
  if (fam.ops) return *fam.ops;
  if (dm.normalised) throw ArgError("op-stream gathers are for the evaluation form");
  const MapSet& ms = get_maps(dm.lattice, dm.m);
  const std::vector<Csr>& host = (fam.k == 1) ? ms.fwd : ms.family(fam.k).fac;
  std::vector<std::vector<uint32_t>> words(host.size());
  std::vector<std::vector<int32_t>> rows(host.size());
  for (size_t i = 0; i < host.size(); ++i) build_op_stream(host[i], fam.codes, fam.shift, words[i], rows[i]);
  size_t bytes = 0;
  for (size_t i = 0; i < host.size(); ++i) bytes += align_up(words[i].size() * 4) + align_up(rows[i].size() * 4);
  auto set = std::make_unique<DevOpSet>();
  if (hipMalloc(&set->base, bytes) != hipSuccess) throw MemError("device allocation of op streams failed");
  char* cur = static_cast<char*>(set->base);
  set->fac.resize(host.size());
  for (size_t i = 0; i < host.size(); ++i) {
    HIPX(hipMemcpy(cur, words[i].data(), words[i].size() * 4, hipMemcpyHostToDevice));
    set->fac[i].ops = reinterpret_cast<const uint32_t*>(cur);
    cur += align_up(words[i].size() * 4);
    HIPX(hipMemcpy(cur, rows[i].data(), rows[i].size() * 4, hipMemcpyHostToDevice));
    set->fac[i].op_row = reinterpret_cast<const int32_t*>(cur);
    cur += align_up(rows[i].size() * 4);
    set->fac[i].n_cols = host[i].n_cols;
  }
  fam.ops = std::move(set);
  return *fam.ops;
}

struct Sizes {
  int64_t s_nc, s_max;
};
Sizes space_sizes(int lattice, int m) {
  Sizes s;
  s.s_nc = ncnnn_count(m);
  s.s_max = (lattice == kSquare && m >= 2) ? ncnnn_count(m) + ncnnn_count(m - 1) : ncnnn_count(m);
  return s;
}

// Sliced-ELL form of a gather-form map (resident.hpp).  With `split`: rows
// sorted by their entries with coefficient other than +-1, then by their +-1
// entries (most first, ties in row order), slices of 64 rows; a slice stores
// its rows' +-1 entries column-major, padded to the slice's most, then the
// others likewise.  Without: rows sorted by their entry count, every entry in
// the first group.  Padding entries read row `zero_row` with code 0.
struct HostSell {
  std::vector<int32_t> perm, slice;   // slice: (offset, unit columns, other columns, 0)
  std::vector<uint32_t> ent;
  int nslice = 0;
};

HostSell build_sell(const Csr& c, uint32_t zero_row, bool split) {
  HostSell h;
  const int64_t n = c.n_rows;
  auto unit = [split](uint32_t w) { return !split || (w >> kEntSrcBits) <= 1u; };
  std::vector<int32_t> nu(n, 0), ng(n, 0);
  for (int64_t r = 0; r < n; ++r)
    for (int32_t e = c.row_ptr[r]; e < c.row_ptr[r + 1]; ++e) (unit(c.ent[e]) ? nu[r] : ng[r]) += 1;
  std::vector<int32_t> order(n);
  for (int64_t r = 0; r < n; ++r) order[r] = static_cast<int32_t>(r);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return ng[a] != ng[b] ? ng[a] > ng[b] : nu[a] > nu[b]; });
  h.nslice = static_cast<int>((n + 63) / 64);
  h.perm.assign(static_cast<size_t>(h.nslice) * 64, -1);
  const uint32_t pad = zero_row;   // code 0
  for (int s = 0; s < h.nslice; ++s) {
    const int64_t r0 = static_cast<int64_t>(s) * 64;
    int U = 0, G = 0;
    for (int l = 0; l < 64 && r0 + l < n; ++l) {
      h.perm[r0 + l] = order[r0 + l];
      U = std::max(U, nu[order[r0 + l]]);
      G = std::max(G, ng[order[r0 + l]]);
    }
    h.slice.insert(h.slice.end(), {static_cast<int32_t>(h.ent.size()), U, G, 0});
    for (int pass = 0; pass < 2; ++pass) {
      const int cols = pass == 0 ? U : G;
      const size_t base = h.ent.size();
      h.ent.resize(base + static_cast<size_t>(cols) * 64, pad);
      for (int l = 0; l < 64; ++l) {
        const int32_t r = h.perm[r0 + l];
        if (r < 0) continue;
        int u = 0;
        for (int32_t e = c.row_ptr[r]; e < c.row_ptr[r + 1]; ++e)
          if (unit(c.ent[e]) == (pass == 0)) h.ent[base + static_cast<size_t>(u++) * 64 + l] = c.ent[e];
      }
    }
  }
  if (h.ent.size() >= (size_t(1) << 31)) throw std::runtime_error("sliced-ELL map too large");
  return h;
}

// The family's forward factors and the read-out maps of (lattice, m) in
// sliced-ELL form on the device, padding entries reading row s_max (kept at
// zero by the resident kernel).
const DevSellSet& dev_sell(const DevMaps& dm, const DevFamily& fam, bool split) {
  std::lock_guard<std::mutex> lk(fam.st_mu);
  std::unique_ptr<DevSellSet>& slot = split ? fam.sell : fam.sell_one;
  if (slot) return *slot;
  if (dm.normalised) throw std::runtime_error("resident mode runs the evaluation form only");
  const MapSet& ms = get_maps(dm.lattice, dm.m);
  const std::vector<Csr>& fwd = (fam.k == 1) ? ms.fwd : ms.family(fam.k).fac;
  std::vector<HostSell> hs;
  std::vector<const Csr*> src;
  for (const Csr& c : fwd) src.push_back(&c);
  for (int i = 0; i < dm.m; ++i) src.push_back(&ms.last[i]);
  size_t bytes = 0;
  for (const Csr* c : src) {
    hs.push_back(build_sell(*c, static_cast<uint32_t>(space_sizes(dm.lattice, dm.m).s_max), split));
    const HostSell& h = hs.back();
    bytes += align_up(h.perm.size() * 4 + 4) + align_up(h.slice.size() * 4 + 4) + align_up(h.ent.size() * 4 + 4);
  }
  auto set = std::make_unique<DevSellSet>();
  for (const Csr* c : src)
    for (int64_t r = 0; r < c->n_rows; ++r) set->max_row = std::max(set->max_row, c->row_ptr[r + 1] - c->row_ptr[r]);
  if (hipMalloc(&set->base, bytes) != hipSuccess) throw MemError("device allocation of sliced-ELL maps failed");
  char* cur = static_cast<char*>(set->base);
  auto put = [&](const void* data, size_t n) {
    void* dst = cur;
    if (n) HIPX(hipMemcpy(dst, data, n, hipMemcpyHostToDevice));
    cur += align_up(n + 4);
    return dst;
  };
  for (size_t i = 0; i < src.size(); ++i) {
    const HostSell& h = hs[i];
    DevSell d{};
    d.perm = static_cast<const int32_t*>(put(h.perm.data(), h.perm.size() * 4));
    d.slice = static_cast<const int32_t*>(put(h.slice.data(), h.slice.size() * 4));
    d.ent = static_cast<const uint32_t*>(put(h.ent.data(), h.ent.size() * 4));
    d.n_rows = static_cast<int>(src[i]->n_rows);
    d.n_cols = static_cast<int>(src[i]->n_cols);
    d.nslice = h.nslice;
    (i < fwd.size() ? set->fac : set->last).push_back(d);
  }
  slot = std::move(set);
  return *slot;
}

// Host-side sizes without building device copies.
// ---------------------------------------------------------------------------
// Pinned staging buffers for host-to-device uploads on a stream
// ---------------------------------------------------------------------------
struct StageBuf {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool in_use = false;
};
std::mutex g_stage_mu;
std::vector<std::unique_ptr<StageBuf>> g_stage;

// Copies `bytes` from `src` to device `dst` on `stream` through a pinned
// buffer that is recycled once the copy has completed.  The buffer is filled
// and its copy and completion event queued under the lock: a buffer counts as
// free when its last event has completed, so another thread must not see it
// between the claim and the new event.
void upload(void* dst, const void* src, size_t bytes, hipStream_t stream) {
  if (bytes == 0) return;
  StageBuf* sb = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    for (auto& b : g_stage) {
      if (b->bytes < bytes) continue;
      if (b->in_use && hipEventQuery(b->done) != hipSuccess) continue;
      sb = b.get();
      break;
    }
    if (!sb) {
      auto nb = std::make_unique<StageBuf>();
      nb->bytes = std::max<size_t>(align_up(bytes, 1 << 16), 1 << 20);
      HIPX(hipHostMalloc(&nb->host, nb->bytes, hipHostMallocDefault));
      HIPX(hipEventCreateWithFlags(&nb->done, hipEventDisableTiming));
      sb = nb.get();
      g_stage.push_back(std::move(nb));
    }
    sb->in_use = true;
    std::memcpy(sb->host, src, bytes);
    HIPX(hipMemcpyAsync(dst, sb->host, bytes, hipMemcpyHostToDevice, stream));
    HIPX(hipEventRecord(sb->done, stream));
  }
}

// ---------------------------------------------------------------------------
// Per-instance constants
// ---------------------------------------------------------------------------
uint32_t neg_inv_2_32(uint32_t p) {
  uint32_t inv = p;  // correct to 3 bits for odd p
  for (int k = 0; k < 5; ++k) inv *= 2u - p * inv;
  return 0u - inv;
}

struct Inst {
  uint32_t q, p;
};

std::vector<Inst> make_instances(const uint32_t* q, int nq, const uint32_t* p, int np) {
  if (nq < 1 || np < 1) throw ArgError("need at least one q point and one prime");
  if (!q || !p) throw ArgError("null q_points or primes");
  std::vector<Inst> v;
  v.reserve(static_cast<size_t>(nq) * np);
  for (int b = 0; b < np; ++b)
    if (p[b] <= 2u || p[b] >= (1u << 31) || (p[b] & 1u) == 0u)
      throw ArgError("each prime must be odd with 2 < p < 2^31");
  for (int a = 0; a < nq; ++a)
    for (int b = 0; b < np; ++b) v.push_back({q[a] % p[b], p[b]});
  return v;
}

// c0 + c1 q + c2 q^2 + c3 q^3 mod p (Horner, every step reduced).
uint32_t coef_mod(const Poly& c, uint32_t q, uint32_t p) {
  uint64_t acc = 0;
  for (int k = kMaxDeg; k >= 0; --k) {
    int64_t ck = c.c[k] % static_cast<int64_t>(p);
    if (ck < 0) ck += p;
    acc = (acc * q + static_cast<uint64_t>(ck)) % p;
  }
  return static_cast<uint32_t>(acc);
}

uint32_t shoup_of(uint32_t c, uint32_t p) {
  return static_cast<uint32_t>((static_cast<uint64_t>(c) << 32) / p);
}

// ---------------------------------------------------------------------------
// Tuning and workspace layout
// ---------------------------------------------------------------------------
struct Tune {
  int V = 2, rpw = 8, wpb = 4, xcd = 0, U = 4, streams = 1, fuse = 1, stage = 0;
};

// lanes_v 8 (512 coefficient slots per row) exists for the coefficient form
// only: `series` admits it.
// Resident mode (`resident`): lanes_v is the number of instances per
// workgroup (1, 2 or 4), waves_per_block may also be 16, and stage selects
// the arithmetic: 0 exact double accumulation where its bound holds, 1
// modular throughout.
Tune resolve(const chrom_tuning* t, bool series = false, bool resident = false) {
  Tune r;
  if (!t) return r;
  if (t->lanes_v) r.V = t->lanes_v;
  if (t->targets_per_wave) r.rpw = t->targets_per_wave;
  if (t->waves_per_block) r.wpb = t->waves_per_block;
  if (t->xcd_order < 0 || t->xcd_order > 6) throw ArgError("xcd_order must be in 0..6");
  if (t->xcd_order) r.xcd = t->xcd_order - 1;
  if (t->unroll) r.U = t->unroll;
  if (t->streams) r.streams = t->streams;
  if (r.U != 4 && r.U != 8) throw ArgError("unroll must be 4 or 8");
  if (r.streams < 1 || r.streams > 4) throw ArgError("streams must be in 1..4");
  if (t->fuse) r.fuse = t->fuse;
  if (r.fuse < 1 || r.fuse > kMaxFuse) throw ArgError("fuse must be in 1..3");
  if (t->stage < 0 || t->stage > 6) throw ArgError("stage must be in 0..6");
  r.stage = t->stage;
  if (series && r.V == 8) {
    if (r.U != 4) throw ArgError("lanes_v 8 runs with unroll 4");
  } else if (r.V != 1 && r.V != 2 && r.V != 4) {
    throw ArgError(series ? "lanes_v must be 1, 2, 4 or 8" : "lanes_v must be 1, 2 or 4");
  }
  if (r.rpw < 1 || r.rpw > 63) throw ArgError("targets_per_wave must be in 1..63");
  if (r.stage == 5 && r.V > 2) throw ArgError("stage 5 (op-stream gathers) takes lanes_v 1 or 2");
  if (resident && r.stage > 1) throw ArgError("resident mode takes stage 0 (exact double accumulation) or 1 (modular)");
  if (r.wpb != 1 && r.wpb != 2 && r.wpb != 4 && r.wpb != 8 && !(resident && r.wpb == 16))
    throw ArgError(resident ? "waves_per_block must be 1, 2, 4, 8 or 16" : "waves_per_block must be 1, 2, 4 or 8");
  return r;
}

// Batched layout of one strip's device state.
struct JobLayout {
  int lattice = 0, m = 0, I = 0, V = 2, W = 128, nchunk = 0, ipad = 0, ncodes = 0;
  int rows_tile = 32;    // rows per workgroup tile
  int64_t s_nc = 0, s_max = 0;
  int nparts = 0;        // read-out partial tiles per chunk
  int ngroups = 0;       // level-1 reduction groups per chunk
  size_t x0 = 0, x1 = 0, w = 0, part = 0, part2 = 0, p = 0, pinv = 0, r1 = 0, tv = 0, ts = 0, poly = 0, bytes = 0;
  // coefficient form: one chunk per prime, lane V + j = coefficient of x^k
  bool cf = false;
  bool wide = false;     // a chunk's vector reaches 4 GiB: kernels form 64-bit row bases
  int dlen = 0;          // coefficients emitted per row and prime (d_max + 1)
  int64_t l_max = 0;     // largest read-out space
  size_t ra = 0, rb = 0, e0 = 0;
};

// Level-1 groups: about 32 partials each, at most 64 groups.
int reduce_groups(int nparts) { return std::max(1, std::min(64, (nparts + 31) / 32)); }

JobLayout job_layout(int lattice, int m, int I, const Tune& t, int ncodes, int rows_tile) {
  JobLayout L;
  L.lattice = lattice;
  L.m = m;
  L.I = I;
  L.V = t.V;
  L.W = 64 * t.V;
  L.nchunk = (I + L.W - 1) / L.W;
  L.ipad = L.nchunk * L.W;
  L.ncodes = ncodes;
  L.rows_tile = rows_tile;
  Sizes s = space_sizes(lattice, m);
  L.s_nc = s.s_nc;
  L.s_max = s.s_max;
  L.nparts = static_cast<int>((L.s_nc + rows_tile - 1) / rows_tile);
  L.ngroups = reduce_groups(L.nparts);
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += align_up(b);
    return o;
  };
  // Kernels address a chunk's rows with 32-bit byte offsets.
  if (static_cast<uint64_t>(L.s_max) * L.W * 4 >= (uint64_t(1) << 32))
    throw ArgError("one chunk's state vector would exceed 4 GiB; use fewer lanes_v");
  const size_t vec = static_cast<size_t>(L.nchunk) * L.s_max * L.W * 4;
  L.x0 = take(vec);
  L.x1 = take(vec);
  L.w = take(static_cast<size_t>(L.nchunk) * L.s_nc * L.W * 4);
  L.part = take(static_cast<size_t>(L.nchunk) * L.nparts * L.W * 4);
  L.part2 = take(static_cast<size_t>(L.nchunk) * L.ngroups * L.W * 4);
  L.p = take(L.ipad * 4);
  L.pinv = take(L.ipad * 4);
  L.r1 = take(L.ipad * 4);
  L.tv = take(L.ipad * 4);
  L.ts = take(L.ipad * 4);
  L.poly = take(static_cast<size_t>(kMaxCodes) * 8);
  L.bytes = off;
  return L;
}

// Layout of a coefficient-form strip: np chunks (one per prime) of W = 64 V
// coefficients, the two state vectors, the read-out ping-pong pair and the
// constants.  No read-out vector, partials or reductions.
JobLayout job_layout_series(int lattice, int m, int np, int d_max, const Tune& t, int64_t l_max) {
  JobLayout L;
  L.lattice = lattice;
  L.m = m;
  L.V = t.V;
  L.W = 64 * t.V;
  if (d_max < 0 || d_max >= L.W) throw ArgError("d_max must be in 0 .. 64 * lanes_v - 1");
  L.cf = true;
  L.dlen = d_max + 1;
  L.nchunk = np;
  L.I = np * L.W;
  L.ipad = L.I;
  L.ncodes = kMaxCodes;
  L.rows_tile = t.rpw * t.wpb;
  Sizes s = space_sizes(lattice, m);
  L.s_nc = s.s_nc;
  L.s_max = s.s_max;
  L.l_max = std::max<int64_t>(l_max, 1);
  L.wide = static_cast<uint64_t>(std::max(L.s_max, L.l_max)) * L.W * 4 >= (uint64_t(1) << 32);
  // CHROMSTRIP_WIDE_ROWS=1 takes the 64-bit row-base path for any size
  // (same results; lets small cases exercise it).
  const char* wide_env = std::getenv("CHROMSTRIP_WIDE_ROWS");
  if (wide_env && std::string(wide_env) == "1") L.wide = true;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += align_up(b);
    return o;
  };
  const size_t vec = static_cast<size_t>(L.nchunk) * L.s_max * L.W * 4;
  L.x0 = take(vec);
  L.x1 = take(vec);
  L.ra = take(static_cast<size_t>(L.nchunk) * L.l_max * L.W * 4);
  L.rb = take(static_cast<size_t>(L.nchunk) * L.l_max * L.W * 4);
  L.w = L.part = L.part2 = off;
  L.p = take(L.ipad * 4);
  L.pinv = take(L.ipad * 4);
  L.r1 = take(L.ipad * 4);
  L.tv = take(L.ipad * 4);
  L.ts = take(L.ipad * 4);
  L.poly = take(static_cast<size_t>(kMaxCodes) * 8);
  L.e0 = take(2 * static_cast<size_t>(L.ipad) * 4);   // e_0, then zeros
  L.bytes = off;
  return L;
}

// Code table word: the coefficients d0..d3 as signed bytes, d_k in byte k.
uint32_t pack_poly(const Poly& c) {
  uint32_t w = 0;
  for (int k = 0; k <= kMaxDeg; ++k) {
    if (c.c[k] < -127 || c.c[k] > 127) throw std::runtime_error("coefficient polynomial out of the packed range");
    w |= (static_cast<uint32_t>(c.c[k]) & 0xffu) << (8 * k);
  }
  return w;
}

// Mask word of a code (kernel side: accumulate): bit 8 when some |d_k| > 1,
// bit 9 when some |d_k| > 3, the degree in bits 12-13; every d_k with
// |d_k| <= 3 as +-2 (bit 16+k for +2, 20+k for -2) plus +-1 (bit k for +1,
// 4+k for -1).  The evaluation-form kernels read the +-1 bits only when bit
// 8 is clear (all |d_k| <= 1), the coefficient-form kernels all of them
// unless bit 9 is set.
uint32_t pack_mask(const Poly& d) {
  uint32_t m = 0;
  int deg = 0;
  for (int k = 0; k <= kMaxDeg; ++k) {
    const int64_t c = d.c[k];
    if (c == 0) continue;
    deg = k;
    const int64_t a = c < 0 ? -c : c;
    if (a > 1) m |= 0x100u;
    if (a > 3) {
      m |= 0x200u;
    } else {
      if (a & 1) m |= (c > 0 ? 1u : 16u) << k;
      if (a & 2) m |= (c > 0 ? 0x10000u : 0x100000u) << k;
    }
  }
  return m | (static_cast<uint32_t>(deg) << 12);
}

// Constants of a job: p, pinv, r1, tv = (q - shift) mod p and its Shoup
// constant over the padded instances, and the code table in powers of
// t = q - shift, as one host image laid out like the workspace region
// [p .. poly].
std::vector<uint32_t> const_image(const JobLayout& L, const std::vector<Inst>& inst,
                                  const std::vector<Poly>& codes, int shift) {
  const size_t base = L.p;
  if (codes.size() < 2 || !(codes[0].c[0] == 1 && codes[1].c[0] == -1))
    throw std::runtime_error("code table must start with +1 and -1");
  std::vector<uint32_t> img((L.poly + static_cast<size_t>(kMaxCodes) * 8 - base) / 4, 0);
  auto at = [&](size_t off) { return img.data() + (off - base) / 4; };
  uint32_t* p = at(L.p);
  uint32_t* pinv = at(L.pinv);
  uint32_t* r1 = at(L.r1);
  uint32_t* tv = at(L.tv);
  uint32_t* ts = at(L.ts);
  uint32_t* poly = at(L.poly);
  for (size_t c = 0; c < codes.size(); ++c) {
    const Poly d = shift_basis(codes[c], shift);
    poly[c] = pack_poly(d);
    poly[kMaxCodes + c] = pack_mask(d);
  }
  for (int k = 0; k < L.ipad; ++k) {
    const Inst& in = inst[k < L.I ? k : 0];
    p[k] = in.p;
    pinv[k] = neg_inv_2_32(in.p);
    r1[k] = static_cast<uint32_t>((uint64_t(1) << 32) % in.p);
    const int64_t sm = ((static_cast<int64_t>(shift) % in.p) + in.p) % in.p;
    tv[k] = static_cast<uint32_t>((static_cast<int64_t>(in.q % in.p) + in.p - sm) % in.p);
    ts[k] = shoup_of(tv[k], in.p);
  }
  return img;
}

// Pointers of one job's device state.
struct JobPtrs {
  uint32_t *x0, *x1, *w, *part, *part2, *p, *pinv, *r1, *tv, *ts, *poly;
  uint32_t *ra = nullptr, *rb = nullptr, *e0 = nullptr;   // coefficient form
  InstConsts ic() const { return InstConsts{p, pinv, tv, ts, reinterpret_cast<const int32_t*>(poly)}; }
};

JobPtrs job_ptrs(const JobLayout& L, void* base) {
  char* b = static_cast<char*>(base);
  JobPtrs j;
  j.x0 = reinterpret_cast<uint32_t*>(b + L.x0);
  j.x1 = reinterpret_cast<uint32_t*>(b + L.x1);
  j.w = reinterpret_cast<uint32_t*>(b + L.w);
  j.part = reinterpret_cast<uint32_t*>(b + L.part);
  j.part2 = reinterpret_cast<uint32_t*>(b + L.part2);
  j.p = reinterpret_cast<uint32_t*>(b + L.p);
  j.pinv = reinterpret_cast<uint32_t*>(b + L.pinv);
  j.r1 = reinterpret_cast<uint32_t*>(b + L.r1);
  j.tv = reinterpret_cast<uint32_t*>(b + L.tv);
  j.ts = reinterpret_cast<uint32_t*>(b + L.ts);
  j.poly = reinterpret_cast<uint32_t*>(b + L.poly);
  if (L.cf) {
    j.ra = reinterpret_cast<uint32_t*>(b + L.ra);
    j.rb = reinterpret_cast<uint32_t*>(b + L.rb);
    j.e0 = reinterpret_cast<uint32_t*>(b + L.e0);
  }
  return j;
}


void check_mode(int mode) {
  if (mode < CHROM_MODE_PLAIN || mode > CHROM_MODE_GROUPED) throw ArgError("unknown mode");
}

void check_args(int lattice, int m, int n_max) {
  if (lattice != CHROM_SQUARE && lattice != CHROM_TRIANGULAR) throw ArgError("lattice must be CHROM_SQUARE or CHROM_TRIANGULAR");
  if (m < 1 || m > CHROM_MAX_M) throw ArgError("m must be in 1..CHROM_MAX_M");
  if (n_max < 0) throw ArgError("n_max must be >= 0");
}


// ---------------------------------------------------------------------------
// Programs: a strip's work as an ordered list of steps over one job's buffers
// ---------------------------------------------------------------------------
struct PStep {
  Step s;       // op, ntiles, args (chunk filled in per item)
  int dep[2];   // local indices of steps that must be complete (-1: none)
};

struct Program {
  std::vector<PStep> steps;
  int nchunk = 0;
};

struct JobCtx {
  const DevMaps* dm;
  const DevFamily* fam;   // forward factors (single or fused) and their code table
  const DevStagedSet* stg = nullptr;   // staged tiles of fam's factors (batched / graph modes)
  const DevOpSet* ops = nullptr;       // op streams of fam's factors (stage 5; batched / graph modes)
  JobLayout L;
  JobPtrs P;
  Tune t;
  uint32_t* d_out;   // [n_max][I], or [n_max][np][dlen] in the coefficient form
  long out_row_stride = 0;   // elements per output row
};

int tiles_for(int64_t rows, int rows_tile) {
  return static_cast<int>(std::max<int64_t>(1, (rows + rows_tile - 1) / rows_tile));
}

int push(Program& pg, const Step& s, int d0, int d1) {
  PStep ps;
  ps.s = s;
  ps.dep[0] = d0;
  ps.dep[1] = d1;
  pg.steps.push_back(ps);
  return static_cast<int>(pg.steps.size()) - 1;
}

// Output vectors past this size take non-temporal row stores.
constexpr int64_t kNtStoreBytes = int64_t(1) << 30;

Step gather_step(const JobCtx& j, const DevCsr& c, const uint32_t* in, uint32_t* out, long out_cstride, bool fused,
                 bool general) {
  Step s{};
  s.op = kOpGather;
  s.general = general ? 1 : 0;
  s.ntiles = tiles_for(c.n_rows, j.L.rows_tile);
  GatherArgs& a = s.u.g;
  a.csr = c;
  a.in = in;
  a.out = out;
  a.in_cstride = static_cast<long>(j.L.s_max) * j.L.W;
  a.out_cstride = out_cstride;
  a.ic = j.P.ic();
  a.rows_per_wave = j.t.rpw;
  if (fused) {
    a.w = j.P.w;
    a.w_cstride = static_cast<long>(j.L.s_nc) * j.L.W;
    a.partial = j.P.part;
    a.p_cstride = static_cast<long>(j.L.nparts) * j.L.W;
  }
  // rows of an output far larger than the 256 MiB Infinity Cache: written
  // once, read a launch later (a fused read-out reads its rows back at once)
  a.nt_store = (!fused && !j.L.cf && static_cast<int64_t>(c.n_rows) * j.L.W * 4 * j.L.nchunk > kNtStoreBytes) ? 1 : 0;
  return s;
}

ReduceArgs reduce_args(const JobCtx& j, int out_row) {
  return ReduceArgs{j.P.part, static_cast<long>(j.L.nparts) * j.L.W, j.L.nparts, j.P.ic(),
                    j.P.part2, static_cast<long>(j.L.ngroups) * j.L.W, j.L.ngroups,
                    j.d_out ? j.d_out + static_cast<long>(out_row) * (j.out_row_stride ? j.out_row_stride : j.L.I)
                            : nullptr,
                    j.L.I};
}

// The read-out of one row: level-1 then level-2 reduction of the partials.
int push_reduce(Program& pg, const JobCtx& j, int out_row, int dep) {
  Step s{};
  s.op = kOpReduce1;
  s.ntiles = j.L.ngroups;
  s.u.r = reduce_args(j, out_row);
  const int r1 = push(pg, s, dep, -1);
  s.op = kOpReduce2;
  s.ntiles = 1;
  return push(pg, s, r1, -1);
}

// Set-up: w = (T_1^last)^T ... (T_m^last)^T (R e_0) built in x0/x1 and
// written to w, then x = e_0 in x0 and Z_1 = <w, e_0>.  Linear chain.
// Coefficient form: read-out of the state in x by the read-out factors in
// gather form, T_1^last first (x -> L_1 -> ... -> L_m, ping-pong through
// ra / rb), then the single state left (all singletons) emitted as output
// row out_row.  Returns the emit step.
int push_readout_cf(Program& pg, const JobCtx& j, const uint32_t* x, int after, int out_row) {
  const JobLayout& L = j.L;
  const uint32_t* in = x;
  long in_cs = static_cast<long>(L.s_max) * L.W;
  const long r_cs = static_cast<long>(L.l_max) * L.W;
  uint32_t* buf[2] = {j.P.ra, j.P.rb};
  for (int i = 1; i <= L.m; ++i) {
    uint32_t* out = buf[(i - 1) % 2];
    Step g = gather_step(j, j.dm->last_fwd[i - 1], in, out, r_cs, false, j.fam->general);
    g.u.g.in_cstride = in_cs;
    g.cf = L.wide ? 2 : 1;
    g.u.g.deg_step = L.V == 8 ? L.m : 0;
    g.u.g.deg_row0 = out_row;
    after = push(pg, g, after, -1);
    in = out;
    in_cs = r_cs;
  }
  Step e{};
  e.op = kOpEmit;
  e.ntiles = 1;
  e.u.e = EmitArgs{in, r_cs, j.d_out ? j.d_out + static_cast<long>(out_row) * j.out_row_stride : nullptr, L.dlen};
  return push(pg, e, after, -1);
}

// Coefficient form, row 0: x0 = e_0 (coefficient array 1 in every chunk),
// then its read-out.  With 512-slot rows every row of x0, x1, ra and rb is
// cleared first: the gathers leave the slots above their degree bound
// untouched, so those slots must start at zero (the second half of the e0
// area is zeros).  Narrower rows are written whole, and only x0's NCNNN rows
// are filled.
int add_setup_cf(Program& pg, const JobCtx& j) {
  const JobLayout& L = j.L;
  const long cs_x = static_cast<long>(L.s_max) * L.W;
  const long cs_r = static_cast<long>(L.l_max) * L.W;
  const uint32_t* zeros = j.P.e0 + L.ipad;
  struct {
    uint32_t* x;
    long cs;
    int64_t rows;
    const uint32_t* v0;
  } fills[4] = {{j.P.x0, cs_x, L.V == 8 ? L.s_max : L.s_nc, j.P.e0}, {j.P.x1, cs_x, L.s_max, zeros},
                {j.P.ra, cs_r, L.l_max, zeros}, {j.P.rb, cs_r, L.l_max, zeros}};
  const int nfills = L.V == 8 ? 4 : 1;
  int last = -1;
  for (int k = 0; k < nfills; ++k) {
    const auto& f = fills[k];
    Step s{};
    s.op = kOpFill;
    s.ntiles = tiles_for(f.rows, L.rows_tile);
    s.u.f = FillArgs{f.x, f.cs, static_cast<int>(f.rows), f.v0, j.t.rpw};
    last = push(pg, s, last, -1);
  }
  return push_readout_cf(pg, j, j.P.x0, last, 0);
}

int add_setup(Program& pg, const JobCtx& j) {
  if (j.L.cf) return add_setup_cf(pg, j);
  const JobLayout& L = j.L;
  const long cs_x = static_cast<long>(L.s_max) * L.W;
  const long cs_w = static_cast<long>(L.s_nc) * L.W;
  Step s{};
  s.op = kOpFill;
  s.ntiles = 1;
  s.u.f = FillArgs{j.P.x0, cs_x, 1, j.P.r1, j.t.rpw};
  int last = push(pg, s, -1, -1);
  uint32_t* cur = j.P.x0;
  uint32_t* oth = j.P.x1;
  for (int i = L.m; i >= 1; --i) {
    const bool to_w = (i == 1);
    Step g = gather_step(j, j.dm->last[i - 1], cur, to_w ? j.P.w : oth, to_w ? cs_w : cs_x, false, true);
    last = push(pg, g, last, -1);
    std::swap(cur, oth);
  }
  s = Step{};
  s.op = kOpFill;
  s.ntiles = tiles_for(L.s_nc, L.rows_tile);
  s.u.f = FillArgs{j.P.x0, cs_x, static_cast<int>(L.s_nc), nullptr, j.t.rpw};
  last = push(pg, s, last, -1);
  s = Step{};
  s.op = kOpDot;
  s.ntiles = L.nparts;
  s.u.d = DotArgs{j.P.x0, j.P.w, cs_x, cs_w, static_cast<int>(L.s_nc), j.P.ic(), j.P.part,
                  static_cast<long>(L.nparts) * L.W, j.t.rpw};
  last = push(pg, s, last, -1);
  return push_reduce(pg, j, 0, last);
}

// Rows: out rows r = r_first..r_last (0-based; row r holds P of m x (r+1)),
// each x <- F_n ... F_1 x over the family's factors (F = one factor T_i, or
// a product of consecutive ones), the read-out fused into F_n, then a reduce.
// `after` is the step the first factor waits for; `prev_reduce` the last
// reduce issued before (its partials are overwritten by the next T_m).
void add_rows(Program& pg, const JobCtx& j, int r_first, int r_last, int after, int prev_reduce) {
  const JobLayout& L = j.L;
  const long cs_x = static_cast<long>(L.s_max) * L.W;
  const int nf = static_cast<int>(j.fam->fac.size());
  for (int r = r_first; r <= r_last; ++r) {
    const long done_gathers = static_cast<long>(r - 1) * nf;
    uint32_t* cur = (done_gathers % 2 == 0) ? j.P.x0 : j.P.x1;
    uint32_t* oth = (cur == j.P.x0) ? j.P.x1 : j.P.x0;
    int tm = -1;
    if (L.cf) {
      // coefficient form: the factors, then the read-out chain on a copy
      for (int i = 1; i <= nf; ++i) {
        Step g = gather_step(j, j.fam->fac[i - 1], cur, oth, cs_x, false, j.fam->general);
        g.cf = L.wide ? 2 : 1;
        g.u.g.deg_step = L.V == 8 ? L.m : 0;
        g.u.g.deg_row0 = r;
        after = push(pg, g, after, -1);
        std::swap(cur, oth);
      }
      after = push_readout_cf(pg, j, cur, after, r);
      continue;
    }
    for (int i = 1; i <= nf; ++i) {
      const bool fused = (i == nf);
      // direct gathers over a target order (stages 4, 6) also take the last
      // factor, whose fused read-out follows the target list
      const bool ordered = j.t.stage == 4 || j.t.stage == 6;
      const DevStaged* sd = (j.stg && (!fused || ordered)) ? &j.stg->fac[i - 1] : nullptr;
      // LDS slots: the widest tile's sources, at most the staging limit (a
      // tile of one exceptional row reads the rest from memory)
      const int cap = sd ? std::min(sd->max_slots, stage_slots(j.L.V)) : 0;
      const int lds = cap * j.L.W * 4;
      Step g = gather_step(j, j.fam->fac[i - 1], cur, oth, cs_x, fused, j.fam->general);
      if (j.ops) {
        // op-stream gathers: every in-range buffer offset below 2^31
        if (j.ops->fac[i - 1].n_cols * L.W * 4 >= static_cast<int64_t>(kOpRange))
          throw ArgError("op-stream gathers: a chunk's input vector exceeds 2 GiB");
        g.u.g.ops = j.ops->fac[i - 1].ops;
        g.u.g.op_row = j.ops->fac[i - 1].op_row;
      }
      if (sd && (j.t.stage == 4 || j.t.stage == 6)) {
        // direct gathers over the clustered order: positions of targets that
        // share sources are adjacent, so the shared rows come from the caches
        g.u.g.csr.row_ptr = sd->csr.row_ptr;
        g.u.g.csr.ent = sd->ent_src;
        g.u.g.tile_tgt = sd->tgt;
      } else if (sd && sd->max_slots > 0 && lds <= kStageMaxLds) {
        g.ntiles = std::max(1, sd->n_tiles);
        g.lds_bytes = lds;
        g.u.g.csr = sd->csr;
        g.u.g.tile_row0 = sd->tile_row0;
        g.u.g.tile_src0 = sd->tile_src0;
        g.u.g.tile_src = sd->src;
        g.u.g.tile_tgt = sd->tgt;
        g.u.g.stage_cap = cap;
        // stage 3: pipelined ranges of clustered tiles, where the tiles fit its limits
        const int pcap = std::min(cap, kPipeSlotsPerWave * j.t.wpb);
        const size_t plds = pipe_lds_bytes(pcap, j.L.W);
        // (each thread copies two of a tile's entry words and one row pointer:
        // a tile's entries must fit 2 x block and its rows + 1 the block)
        const int block = 64 * j.t.wpb;
        if (j.t.stage == 3 && sd->max_rows <= kPipeMaxRows && sd->max_rows + 1 <= block &&
            sd->max_ent <= std::min(kPipeMaxEnt, 2 * block) && plds <= kPipeMaxLds) {
          const int tpb = pipe_tiles_per_block(sd->n_tiles, j.L.nchunk);
          g.u.g.tile_ent0 = sd->tile_ent0;
          g.u.g.n_tiles = sd->n_tiles;
          g.u.g.tiles_per_block = tpb;
          g.ntiles = (sd->n_tiles + tpb - 1) / tpb;
          g.lds_bytes = static_cast<int>(plds);
          g.u.g.stage_cap = pcap;
        }
      }
      tm = push(pg, g, after, fused ? prev_reduce : -1);
      after = tm;
      std::swap(cur, oth);
    }
    prev_reduce = push_reduce(pg, j, r, tm);
  }
}

Program strip_program(const JobCtx& j, int n_max) {
  Program pg;
  pg.nchunk = j.L.nchunk;
  if (n_max < 1) return pg;
  int red = add_setup(pg, j);
  if (n_max > 1) add_rows(pg, j, 1, n_max - 1, red, red);
  return pg;
}

// ---------------------------------------------------------------------------
// Eager execution of a program: one launch per step, grid (ntiles, nchunk)
// ---------------------------------------------------------------------------
// Launches one step over chunks [c0, c0 + nch).
// Coefficient-form gather arguments of a step: under a graph replay the
// degree bound follows the device row counter.
GatherArgs cf_args(const Step& s, const int* row_ctr) {
  GatherArgs g = s.u.g;
  if (row_ctr && g.deg_step) g.deg_row = row_ctr;
  return g;
}

template <int V, int U>
void launch_step_vu(const Step& s, int c0, int nch, int wpb, int xcd, hipStream_t st, const int* row_ctr,
                    long row_stride) {
  dim3 grid(s.ntiles, nch), block(64 * wpb);
  switch (s.op) {
    case kOpGather:
      if (s.cf == 2) {
        if (s.general)
          hipLaunchKernelGGL((k_gather<V, U, true, true, true>), grid, block, 0, st, cf_args(s, row_ctr), xcd, c0);
        else
          hipLaunchKernelGGL((k_gather<V, U, false, true, true>), grid, block, 0, st, cf_args(s, row_ctr), xcd, c0);
      } else if (s.cf) {
        if (s.general)
          hipLaunchKernelGGL((k_gather<V, U, true, true>), grid, block, 0, st, cf_args(s, row_ctr), xcd, c0);
        else
          hipLaunchKernelGGL((k_gather<V, U, false, true>), grid, block, 0, st, cf_args(s, row_ctr), xcd, c0);
      } else if (s.u.g.tile_row0) {
        if constexpr (V <= 2) {
          if (s.u.g.tile_ent0) {
            if (s.general)
              hipLaunchKernelGGL((k_stage_pipe<V, U, true>), grid, block, s.lds_bytes, st, s.u.g, xcd, c0);
            else
              hipLaunchKernelGGL((k_stage_pipe<V, U, false>), grid, block, s.lds_bytes, st, s.u.g, xcd, c0);
          } else if (s.general)
            hipLaunchKernelGGL((k_stage<V, U, true>), grid, block, s.lds_bytes, st, s.u.g, xcd, c0);
          else
            hipLaunchKernelGGL((k_stage<V, U, false>), grid, block, s.lds_bytes, st, s.u.g, xcd, c0);
        } else {
          throw std::runtime_error("staged tiles need lanes_v 1 or 2");
        }
      } else if (s.u.g.ops) {
        if constexpr (V <= 2)
          hipLaunchKernelGGL(k_gather_ops<V>, grid, block, 0, st, s.u.g, xcd, c0);
        else
          throw std::runtime_error("op-stream gathers need lanes_v 1 or 2");
      } else if (s.general) {
        hipLaunchKernelGGL((k_gather<V, U, true, false>), grid, block, 0, st, s.u.g, xcd, c0);
      } else {
        hipLaunchKernelGGL((k_gather<V, U, false, false>), grid, block, 0, st, s.u.g, xcd, c0);
      }
      break;
    case kOpEmit:
      if (row_ctr)
        hipLaunchKernelGGL(k_emit_counted, dim3(nch), dim3(256), 0, st, s.u.e, c0, row_ctr, row_stride);
      else
        hipLaunchKernelGGL(k_emit, dim3(nch), dim3(256), 0, st, s.u.e, c0);
      break;
    case kOpDot: hipLaunchKernelGGL(k_dot<V>, grid, block, 0, st, s.u.d, xcd, c0); break;
    case kOpFill: hipLaunchKernelGGL(k_fill<V>, grid, block, 0, st, s.u.f, c0); break;
    case kOpReduce1:
      hipLaunchKernelGGL(k_reduce1<V>, dim3(s.ntiles, nch), dim3(256), 0, st, s.u.r, c0);
      break;
    case kOpReduce2:
      if (row_ctr)
        hipLaunchKernelGGL(k_reduce2_counted<V>, dim3(nch), dim3(256), 0, st, s.u.r, c0, row_ctr, row_stride);
      else
        hipLaunchKernelGGL(k_reduce2<V>, dim3(nch), dim3(256), 0, st, s.u.r, c0);
      break;
  }
  HIPX(hipGetLastError());
}

// lanes_v 8: the coefficient form's steps only (gathers, fills, emits).
void launch_step_cf8(const Step& s, int c0, int nch, int wpb, int xcd, hipStream_t st, const int* row_ctr,
                     long row_stride) {
  dim3 grid(s.ntiles, nch), block(64 * wpb);
  switch (s.op) {
    case kOpGather:
      if (!s.cf || s.u.g.w) throw std::runtime_error("lanes_v 8 is for the coefficient form only");
      if (s.cf == 2 && s.general)
        hipLaunchKernelGGL((k_gather_cf8<true, true>), grid, block, 0, st, cf_args(s, row_ctr), xcd, c0);
      else if (s.cf == 2)
        hipLaunchKernelGGL((k_gather_cf8<false, true>), grid, block, 0, st, cf_args(s, row_ctr), xcd, c0);
      else if (s.general)
        hipLaunchKernelGGL((k_gather_cf8<true, false>), grid, block, 0, st, cf_args(s, row_ctr), xcd, c0);
      else
        hipLaunchKernelGGL((k_gather_cf8<false, false>), grid, block, 0, st, cf_args(s, row_ctr), xcd, c0);
      break;
    case kOpEmit:
      if (row_ctr)
        hipLaunchKernelGGL(k_emit_counted, dim3(nch), dim3(256), 0, st, s.u.e, c0, row_ctr, row_stride);
      else
        hipLaunchKernelGGL(k_emit, dim3(nch), dim3(256), 0, st, s.u.e, c0);
      break;
    case kOpFill: hipLaunchKernelGGL(k_fill<8>, grid, block, 0, st, s.u.f, c0); break;
    default: throw std::runtime_error("lanes_v 8 is for the coefficient form only");
  }
  HIPX(hipGetLastError());
}

void launch_step(const Step& s, const Tune& t, int c0, int nch, hipStream_t st, const int* row_ctr = nullptr,
                 long row_stride = 0) {
  const int key = t.V * 10 + t.U;
  switch (key) {
    case 84: launch_step_cf8(s, c0, nch, t.wpb, t.xcd, st, row_ctr, row_stride); break;
    case 14: launch_step_vu<1, 4>(s, c0, nch, t.wpb, t.xcd, st, row_ctr, row_stride); break;
    case 18: launch_step_vu<1, 8>(s, c0, nch, t.wpb, t.xcd, st, row_ctr, row_stride); break;
    case 24: launch_step_vu<2, 4>(s, c0, nch, t.wpb, t.xcd, st, row_ctr, row_stride); break;
    case 28: launch_step_vu<2, 8>(s, c0, nch, t.wpb, t.xcd, st, row_ctr, row_stride); break;
    case 44: launch_step_vu<4, 4>(s, c0, nch, t.wpb, t.xcd, st, row_ctr, row_stride); break;
    default: launch_step_vu<4, 8>(s, c0, nch, t.wpb, t.xcd, st, row_ctr, row_stride); break;
  }
}

// Instance chunks split into up to `streams` groups that run their step
// sequences on parallel streams (fork/join through events), so one group's
// kernel tail overlaps another group's kernels.  Groups never share data.
struct ChunkGroups {
  int n = 1;
  int c0[4], nch[4];
};

ChunkGroups chunk_groups(int nchunk, int streams) {
  ChunkGroups g;
  g.n = std::max(1, std::min(streams, nchunk));
  for (int k = 0; k < g.n; ++k) {
    g.c0[k] = nchunk * k / g.n;
    g.nch[k] = nchunk * (k + 1) / g.n - g.c0[k];
  }
  return g;
}

struct AuxStreams {
  hipStream_t s[3] = {nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
};
std::mutex g_aux_mu;
AuxStreams g_aux[64], g_aux_capture[64];

AuxStreams& aux_streams(bool capture) {
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  AuxStreams& a = capture ? g_aux_capture[dev] : g_aux[dev];
  if (!a.fork) {
    for (int k = 0; k < 3; ++k) {
      HIPX(hipStreamCreateWithFlags(&a.s[k], hipStreamNonBlocking));
      HIPX(hipEventCreateWithFlags(&a.join[k], hipEventDisableTiming));
    }
    HIPX(hipEventCreateWithFlags(&a.fork, hipEventDisableTiming));
  }
  return a;
}

// Runs `body(group, stream)` for every chunk group, group 0 on `st` and the
// others on auxiliary streams forked from and joined back into `st`.
template <class F>
void for_groups(const ChunkGroups& g, hipStream_t st, bool capture, F&& body) {
  if (g.n == 1) {
    body(0, st);
    return;
  }
  std::lock_guard<std::mutex> lk(g_aux_mu);
  AuxStreams& a = aux_streams(capture);
  HIPX(hipEventRecord(a.fork, st));
  for (int k = 1; k < g.n; ++k) HIPX(hipStreamWaitEvent(a.s[k - 1], a.fork, 0));
  body(0, st);
  for (int k = 1; k < g.n; ++k) body(k, a.s[k - 1]);
  for (int k = 1; k < g.n; ++k) {
    HIPX(hipEventRecord(a.join[k - 1], a.s[k - 1]));
    HIPX(hipStreamWaitEvent(st, a.join[k - 1], 0));
  }
}

void run_eager(const Program& pg, const Tune& t, hipStream_t st, bool capture = false,
               const int* row_ctr = nullptr, long row_stride = 0) {
  ChunkGroups g = chunk_groups(pg.nchunk, t.streams);
  for_groups(g, st, capture, [&](int k, hipStream_t s) {
    for (const PStep& ps : pg.steps) launch_step(ps.s, t, g.c0[k], g.nch[k], s, row_ctr, row_stride);
  });
}

// ---------------------------------------------------------------------------
// hipGraph row sweep: a run of rows (rows_per_graph) captured once and
// replayed; every chunk group is a chain of its own from the start of a
// replay to its end
// ---------------------------------------------------------------------------
struct GraphKey {
  void* ws;
  uint32_t* out;
  int lattice, m, I, V, rpw, wpb, xcd, rows_per_graph;
  int cf_len;   // coefficient form: coefficients per row and prime (0: evaluation form)
  int split = 0;  // instances of a lanes_v 4 split's second job (0: one job)
  bool operator<(const GraphKey& o) const {
    return std::tie(ws, out, lattice, m, I, V, rpw, wpb, xcd, rows_per_graph, cf_len, split) <
           std::tie(o.ws, o.out, o.lattice, o.m, o.I, o.V, o.rpw, o.wpb, o.xcd, o.rows_per_graph, o.cf_len, o.split);
  }
};
struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  int dev = -1;
};
std::mutex g_graph_mu;
std::map<GraphKey, GraphEntry> g_graphs;
hipStream_t g_capture_stream[64] = {nullptr};

hipStream_t capture_stream() {
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  if (!g_capture_stream[dev]) HIPX(hipStreamCreateWithFlags(&g_capture_stream[dev], hipStreamNonBlocking));
  return g_capture_stream[dev];
}

// Held across every capture on a capture stream: two host threads capturing
// on one stream at once would record into one graph.  Taken before any other
// lock a capture needs (split stream, auxiliary streams, graph caches).
std::mutex g_capture_mu;

// One chain of a captured row replay: the rows of one chunk group of one
// job, on its own stream, with its own row counter.
struct RowChain {
  const JobCtx* j;
  const Program* rows;   // `per` rows, equal lengths
  int c0, nch;
  int* ctr;
  hipStream_t s;
};

// The row's last read-out kernel for a chain of one chunk (one workgroup):
// writes the row its counter names, then advances the counter itself, so a
// row ends in one launch instead of two.  Every thread reads the counter
// before the barrier; thread 0 writes it after.
template <int V>
__global__ void __launch_bounds__(256) k_reduce2_counted_bump(ReduceArgs a, int chunk, int* row, long row_stride) {
  const int r = *row;
  reduce2_tile<V>(a, chunk, a.out + static_cast<long>(r) * row_stride);
  __syncthreads();
  if (threadIdx.x == 0) *row = r + 1;
}

// Whether a chain's rows end in a read-out that can advance the counter
// itself (evaluation form, one chunk).
bool ends_in_counted_reduce(const RowChain& c, int per) {
  const size_t len = c.rows->steps.size() / per;
  return c.nch == 1 && len > 0 && c.rows->steps[len - 1].s.op == kOpReduce2 && c.j->t.V <= 4;
}

// Records `per` rows of every chain, step by step across the chains, each
// row ending in a bump of that chain's own counter.  Chains never wait for
// one another: a chunk group reads and writes only its own chunks, and the
// counted read-out kernels read its own counter.
void record_chains(const std::vector<RowChain>& ch, int per) {
  for (int r = 0; r < per; ++r) {
    size_t most = 0;
    for (const RowChain& c : ch) most = std::max(most, c.rows->steps.size() / per);
    for (size_t i = 0; i < most; ++i)
      for (const RowChain& c : ch) {
        const size_t len = c.rows->steps.size() / per;
        if (i >= len) continue;
        const Step& s = c.rows->steps[r * len + i].s;
        if (i + 1 == len && ends_in_counted_reduce(c, per)) {
          const long stride = c.j->out_row_stride;
          if (c.j->t.V == 1)
            hipLaunchKernelGGL(k_reduce2_counted_bump<1>, dim3(1), dim3(256), 0, c.s, s.u.r, c.c0, c.ctr, stride);
          else if (c.j->t.V == 2)
            hipLaunchKernelGGL(k_reduce2_counted_bump<2>, dim3(1), dim3(256), 0, c.s, s.u.r, c.c0, c.ctr, stride);
          else
            hipLaunchKernelGGL(k_reduce2_counted_bump<4>, dim3(1), dim3(256), 0, c.s, s.u.r, c.c0, c.ctr, stride);
        } else {
          launch_step(s, c.j->t, c.c0, c.nch, c.s, c.ctr, c.j->out_row_stride);
        }
      }
    for (const RowChain& c : ch)
      if (!ends_in_counted_reduce(c, per)) hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, c.s, c.ctr);
    HIPX(hipGetLastError());
  }
}

// The chains of job `j` (one per chunk group; group g counts rows in
// ctr[g]): group 0 on `s0`, group g > 0 on the capture set's auxiliary
// stream g - 1.
void add_chains(std::vector<RowChain>& ch, const JobCtx& j, const Program& rows, int* ctr, hipStream_t s0,
                const AuxStreams& a, int aux0 = 0) {
  const ChunkGroups g = chunk_groups(j.L.nchunk, j.t.streams);
  if (aux0 + g.n - 1 > 3) throw std::runtime_error("more chunk-group chains than auxiliary streams");
  for (int k = 0; k < g.n; ++k)
    ch.push_back(RowChain{&j, &rows, g.c0[k], g.nch[k], ctr + k, k ? a.s[aux0 + k - 1] : s0});
}

// Sets the row counter of every chunk group of `j` to 1.
void reset_row_counters(const JobCtx& j, int* ctr, hipStream_t st) {
  const ChunkGroups g = chunk_groups(j.L.nchunk, j.t.streams);
  for (int k = 0; k < g.n; ++k) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, ctr + k, 1);
  HIPX(hipGetLastError());
}

// Rows per captured graph: a multiple of the rows after which the ping-pong
// vectors return to their start (two when a row has an odd number of
// launches), up to kGraphRows, so that the chunk groups' chains run
// independently across those rows instead of meeting at every replay's end.
constexpr int kGraphRows = 32;
int rows_per_graph(const JobCtx& j, int rows) {
  const int base = (static_cast<int>(j.fam->fac.size()) % 2 == 1) ? 2 : 1;
  return std::max(base, std::min(rows, kGraphRows) / base * base);
}

void run_graph(const JobCtx& j, int n_max, int* row_ctr, void* ws, hipStream_t st) {
  Program setup;
  setup.nchunk = j.L.nchunk;
  int red = add_setup(setup, j);
  (void)red;
  run_eager(setup, j.t, st);
  if (n_max <= 1) return;
  const int rows = n_max - 1;
  const int per = rows_per_graph(j, rows);
  const int replays = rows / per;
  const int tail = rows - replays * per;
  reset_row_counters(j, row_ctr, st);
  if (replays > 0) {
    GraphKey key{ws, j.d_out, j.L.lattice, j.L.m, j.L.I, j.t.V, j.t.rpw, j.t.wpb,
                 j.t.stage * 10000 + j.t.fuse * 1000 + j.t.xcd * 100 + j.t.U * 10 + j.t.streams, per,
                 j.L.cf ? j.L.dlen : 0};
    hipGraphExec_t exec = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_graph_mu);
      auto it = g_graphs.find(key);
      if (it != g_graphs.end()) exec = it->second.exec;
    }
    if (!exec) {
      Program rows_pg;
      rows_pg.nchunk = j.L.nchunk;
      // rows 1..per starting from the parity of row 1 (x in x0)
      add_rows(rows_pg, j, 1, per, -1, -1);
      // reduce2 and emit write the row given by their chunk group's device
      // counter, which the group's chain advances after each of its rows
      for (PStep& ps : rows_pg.steps) {
        if (ps.s.op == kOpReduce2) ps.s.u.r.out = j.d_out;
        if (ps.s.op == kOpEmit) ps.s.u.e.dst = j.d_out;
      }
      std::lock_guard<std::mutex> lk_cap(g_capture_mu);
      std::lock_guard<std::mutex> lk_aux(g_aux_mu);
      AuxStreams& a = aux_streams(true);
      std::vector<RowChain> ch;
      hipStream_t cs = capture_stream();
      add_chains(ch, j, rows_pg, row_ctr, cs, a);
      HIPX(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      if (ch.size() > 1) HIPX(hipEventRecord(a.fork, cs));
      for (size_t k = 1; k < ch.size(); ++k) HIPX(hipStreamWaitEvent(ch[k].s, a.fork, 0));
      record_chains(ch, per);
      for (size_t k = 1; k < ch.size(); ++k) {
        HIPX(hipEventRecord(a.join[k - 1], ch[k].s));
        HIPX(hipStreamWaitEvent(cs, a.join[k - 1], 0));
      }
      hipGraph_t graph = nullptr;
      HIPX(hipStreamEndCapture(cs, &graph));
      HIPX(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      HIPX(hipGraphDestroy(graph));
      std::lock_guard<std::mutex> lk(g_graph_mu);
      g_graphs[key] = GraphEntry{exec, 0};
    }
    for (int k = 0; k < replays; ++k) HIPX(hipGraphLaunch(exec, st));
  }
  if (tail > 0) {
    Program tail_pg;
    tail_pg.nchunk = j.L.nchunk;
    add_rows(tail_pg, j, n_max - tail, n_max - 1, -1, -1);
    run_eager(tail_pg, j.t, st);
  }
}

// Graph row replay of a lanes_v 4 split (split_plan): both jobs' rows are
// captured into ONE graph as parallel branches (the second forked from the
// capture stream through a library stream and joined back), each chunk
// group of each job a chain with its own row counter.  Two graphs on two caller-visible streams would leave
// their overlap to how the runtime maps streams to hardware queues; branches
// of one graph do not depend on it.
struct SplitStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_split_cap_mu;
SplitStream g_split_cap[64];

void run_graph_split(const JobCtx& ja, const JobCtx& jb, int n_max, int* ctr_a, int* ctr_b, void* ws,
                     hipStream_t st) {
  const JobCtx* js[2] = {&ja, &jb};
  int* ctrs[2] = {ctr_a, ctr_b};
  for (int k = 0; k < 2; ++k) {
    Program setup;
    setup.nchunk = js[k]->L.nchunk;
    (void)add_setup(setup, *js[k]);
    run_eager(setup, js[k]->t, st);
  }
  if (n_max <= 1) return;
  const int rows = n_max - 1;
  const int per = rows_per_graph(ja, rows);
  const int replays = rows / per;
  const int tail = rows - replays * per;
  for (int k = 0; k < 2; ++k) reset_row_counters(*js[k], ctrs[k], st);
  if (replays > 0) {
    GraphKey key{ws, ja.d_out, ja.L.lattice, ja.L.m, ja.L.I, ja.t.V, ja.t.rpw, ja.t.wpb,
                 ja.t.stage * 10000 + ja.t.fuse * 1000 + ja.t.xcd * 100 + ja.t.U * 10 + ja.t.streams, per, 0,
                 jb.L.I};
    hipGraphExec_t exec = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_graph_mu);
      auto it = g_graphs.find(key);
      if (it != g_graphs.end()) exec = it->second.exec;
    }
    if (!exec) {
      Program rows_pg[2];
      for (int k = 0; k < 2; ++k) {
        rows_pg[k].nchunk = js[k]->L.nchunk;
        add_rows(rows_pg[k], *js[k], 1, per, -1, -1);
        for (PStep& ps : rows_pg[k].steps)
          if (ps.s.op == kOpReduce2) ps.s.u.r.out = js[k]->d_out;
      }
      std::lock_guard<std::mutex> lk_cap(g_capture_mu);
      std::lock_guard<std::mutex> lk(g_split_cap_mu);
      std::lock_guard<std::mutex> lk_aux(g_aux_mu);
      int dev = 0;
      HIPX(hipGetDevice(&dev));
      SplitStream& cb = g_split_cap[dev];
      if (!cb.s) {
        HIPX(hipStreamCreateWithFlags(&cb.s, hipStreamNonBlocking));
        HIPX(hipEventCreateWithFlags(&cb.fork, hipEventDisableTiming));
        HIPX(hipEventCreateWithFlags(&cb.join, hipEventDisableTiming));
      }
      AuxStreams& a = aux_streams(true);
      hipStream_t cs = capture_stream();
      // the first job's chunk groups on the capture stream and the auxiliary
      // streams, the second job (one group) on the library stream
      std::vector<RowChain> ch;
      add_chains(ch, ja, rows_pg[0], ctrs[0], cs, a);
      const size_t na = ch.size();
      add_chains(ch, jb, rows_pg[1], ctrs[1], cb.s, a, static_cast<int>(na) - 1);
      HIPX(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      HIPX(hipEventRecord(cb.fork, cs));
      for (size_t k = 1; k < ch.size(); ++k) HIPX(hipStreamWaitEvent(ch[k].s, cb.fork, 0));
      record_chains(ch, per);
      // chains on auxiliary streams (all but the two jobs' first) join
      // through those streams' events, the second job's first through the
      // split stream's
      for (size_t k = 1; k < ch.size(); ++k) {
        if (k == na) continue;
        const size_t ax = k < na ? k - 1 : k - 2;
        HIPX(hipEventRecord(a.join[ax], ch[k].s));
        HIPX(hipStreamWaitEvent(cs, a.join[ax], 0));
      }
      HIPX(hipEventRecord(cb.join, cb.s));
      HIPX(hipStreamWaitEvent(cs, cb.join, 0));
      hipGraph_t graph = nullptr;
      HIPX(hipStreamEndCapture(cs, &graph));
      HIPX(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      HIPX(hipGraphDestroy(graph));
      std::lock_guard<std::mutex> lk2(g_graph_mu);
      g_graphs[key] = GraphEntry{exec, 0};
    }
    for (int k = 0; k < replays; ++k) HIPX(hipGraphLaunch(exec, st));
  }
  if (tail > 0) {
    for (int k = 0; k < 2; ++k) {
      Program tail_pg;
      tail_pg.nchunk = js[k]->L.nchunk;
      add_rows(tail_pg, *js[k], n_max - tail, n_max - 1, -1, -1);
      run_eager(tail_pg, js[k]->t, st);
    }
  }
}

// ---------------------------------------------------------------------------
// Grouped execution: stage k is ONE launch running step k of every
// (program, chunk) item; stages run in stream order.  A whole batch or sweep
// can be captured as one hipGraph.
// ---------------------------------------------------------------------------
struct StageImage {
  std::vector<Step> steps;          // stage-major
  std::vector<int> tile_start;      // per stage: nsteps+1 prefix sums
  std::vector<int> step_off, tile_off, nsteps, ntiles;  // per stage
};

// Stage image of the (program, chunk) items of one chunk group: with
// `groups` > 1, chunk c of program k belongs to group (c + k) mod groups
// (chunks are independent, so the groups can run on parallel streams).
StageImage build_stages(const std::vector<const Program*>& progs, int groups = 1, int group = 0) {
  StageImage im;
  size_t maxlen = 0;
  for (const Program* pg : progs) maxlen = std::max(maxlen, pg->steps.size());
  for (size_t k = 0; k < maxlen; ++k) {
    im.step_off.push_back(static_cast<int>(im.steps.size()));
    im.tile_off.push_back(static_cast<int>(im.tile_start.size()));
    int tiles = 0, n = 0;
    // Items with the most tiles first: workgroups are dispatched in index
    // order, so the largest items start first and the small ones fill the
    // launch's tail instead of forming it.
    std::vector<Step> items;
    for (size_t pi = 0; pi < progs.size(); ++pi) {
      const Program* pg = progs[pi];
      if (k >= pg->steps.size()) continue;
      for (int c = 0; c < pg->nchunk; ++c) {
        if ((c + static_cast<int>(pi)) % groups != group) continue;
        Step s = pg->steps[k].s;
        s.chunk = c;
        items.push_back(s);
      }
    }
    std::stable_sort(items.begin(), items.end(), [](const Step& a, const Step& b) { return a.ntiles > b.ntiles; });
    for (const Step& s : items) {
      im.tile_start.push_back(tiles);
      tiles += s.ntiles;
      im.steps.push_back(s);
      ++n;
    }
    im.tile_start.push_back(tiles);
    im.nsteps.push_back(n);
    im.ntiles.push_back(tiles);
  }
  return im;
}

// Device bytes of the stage tables for `nsteps` items-steps over `nstages` stages.
size_t stage_bytes(long nsteps, long nstages) {
  return align_up(std::max<long>(nsteps, 1) * sizeof(Step)) + align_up((nsteps + nstages + 1) * sizeof(int));
}

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}

void launch_stages(const StageImage& im, const Step* d_steps, const int* d_tiles, const Tune& t, hipStream_t st) {
  for (size_t k = 0; k < im.nsteps.size(); ++k) {
    if (im.nsteps[k] == 0) continue;
    GroupArgs g{d_steps + im.step_off[k], d_tiles + im.tile_off[k], im.nsteps[k], t.xcd};
    dim3 grid(im.ntiles[k]), block(64 * t.wpb);
    bool general = false;
    for (int i = 0; i < im.nsteps[k]; ++i) general = general || im.steps[im.step_off[k] + i].general;
    switch (t.V * 100 + t.U * 10 + (general ? 1 : 0)) {
      case 140: hipLaunchKernelGGL((k_grouped<1, 4, false>), grid, block, 0, st, g); break;
      case 141: hipLaunchKernelGGL((k_grouped<1, 4, true>), grid, block, 0, st, g); break;
      case 180: hipLaunchKernelGGL((k_grouped<1, 8, false>), grid, block, 0, st, g); break;
      case 181: hipLaunchKernelGGL((k_grouped<1, 8, true>), grid, block, 0, st, g); break;
      case 240: hipLaunchKernelGGL((k_grouped<2, 4, false>), grid, block, 0, st, g); break;
      case 241: hipLaunchKernelGGL((k_grouped<2, 4, true>), grid, block, 0, st, g); break;
      case 280: hipLaunchKernelGGL((k_grouped<2, 8, false>), grid, block, 0, st, g); break;
      case 281: hipLaunchKernelGGL((k_grouped<2, 8, true>), grid, block, 0, st, g); break;
      case 440: hipLaunchKernelGGL((k_grouped<4, 4, false>), grid, block, 0, st, g); break;
      case 441: hipLaunchKernelGGL((k_grouped<4, 4, true>), grid, block, 0, st, g); break;
      case 480: hipLaunchKernelGGL((k_grouped<4, 8, false>), grid, block, 0, st, g); break;
      default: hipLaunchKernelGGL((k_grouped<4, 8, true>), grid, block, 0, st, g); break;
    }
    HIPX(hipGetLastError());
  }
}

// One cached graph per stage-table location.  The graph's kernels read the
// stage tables from caller memory at `base`, so the tables are uploaded again
// before every launch (the caller may have reused that memory since); the
// cache only saves the capture and instantiation.  `done` is a library-owned
// event recorded after every launch of the graph: a replaced graph is
// destroyed once that event has completed, without touching the caller's
// stream (which may no longer exist).
struct StageGraph {
  uint64_t hash = 0;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
};
std::mutex g_sgraph_mu;
std::map<void*, StageGraph> g_sgraphs;

void retire_stage_graph(StageGraph& g) {
  if (g.done) {
    (void)hipEventSynchronize(g.done);
    (void)hipEventDestroy(g.done);
  }
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g = StageGraph{};
}

void drop_stage_graphs_in(void* lo, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_sgraph_mu);
  for (auto it = g_sgraphs.begin(); it != g_sgraphs.end();) {
    char* k = static_cast<char*>(it->first);
    if (k >= static_cast<char*>(lo) && k < static_cast<char*>(lo) + bytes) {
      retire_stage_graph(it->second);
      it = g_sgraphs.erase(it);
    } else {
      ++it;
    }
  }
}

// Uploads the stage tables to `base` and runs them on `st`, either as
// separate launches or as one (cached) graph.
// Runs the programs' steps as grouped launches, in `groups` chunk groups on
// parallel streams (forked from and joined into `st`); `base` holds the
// groups' stage tables, at most groups x stage_bytes(steps, stages).  With
// as_graph, the launches are captured once per (base, tables) and replayed.
void run_grouped(const std::vector<const Program*>& progs, const Tune& t, void* base, hipStream_t st, bool as_graph,
                 int groups = 1) {
  groups = std::max(1, std::min(groups, 4));
  std::vector<StageImage> ims;
  for (int g = 0; g < groups; ++g) {
    StageImage im = build_stages(progs, groups, g);
    if (!im.steps.empty()) ims.push_back(std::move(im));
  }
  if (ims.empty()) return;
  char* b = static_cast<char*>(base);
  std::vector<Step*> d_steps;
  std::vector<int*> d_tiles;
  size_t off = 0;
  // The cached graph depends on what its launches capture: the tuning, and
  // per stage the table offsets, step and tile counts and the kernel chosen
  // (general coefficients or not).  The step records themselves are read
  // from the tables, uploaded before every launch, so their bytes (which
  // hold padding and unused union members) are not hashed.
  uint64_t h = fnv1a(&t, sizeof(t));
  for (const StageImage& im : ims) {
    d_steps.push_back(reinterpret_cast<Step*>(b + off));
    off += align_up(im.steps.size() * sizeof(Step));
    d_tiles.push_back(reinterpret_cast<int*>(b + off));
    off += align_up(im.tile_start.size() * sizeof(int));
    const size_t ns = im.steps.size();
    h = fnv1a(&ns, sizeof(ns), h);
    h = fnv1a(im.tile_start.data(), im.tile_start.size() * sizeof(int), h);
    h = fnv1a(im.step_off.data(), im.step_off.size() * sizeof(int), h);
    h = fnv1a(im.tile_off.data(), im.tile_off.size() * sizeof(int), h);
    h = fnv1a(im.nsteps.data(), im.nsteps.size() * sizeof(int), h);
    h = fnv1a(im.ntiles.data(), im.ntiles.size() * sizeof(int), h);
    for (const Step& st_k : im.steps) h = fnv1a(&st_k.general, sizeof(st_k.general), h);
  }
  auto upload_all = [&]() {
    for (size_t g = 0; g < ims.size(); ++g) {
      upload(d_steps[g], ims[g].steps.data(), ims[g].steps.size() * sizeof(Step), st);
      upload(d_tiles[g], ims[g].tile_start.data(), ims[g].tile_start.size() * sizeof(int), st);
    }
  };
  auto launch_all = [&](hipStream_t s0, bool capture) {
    ChunkGroups cg;
    cg.n = static_cast<int>(ims.size());
    for_groups(cg, s0, capture, [&](int g, hipStream_t s) { launch_stages(ims[g], d_steps[g], d_tiles[g], t, s); });
  };
  upload_all();
  if (!as_graph) {
    launch_all(st, false);
    return;
  }
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_sgraph_mu);
    auto it = g_sgraphs.find(base);
    if (it != g_sgraphs.end()) {
      if (it->second.hash == h) {
        exec = it->second.exec;
        done = it->second.done;
      } else {
        retire_stage_graph(it->second);
        g_sgraphs.erase(it);
      }
    }
  }
  if (!exec) {
    std::lock_guard<std::mutex> lk_cap(g_capture_mu);
    hipStream_t cs = capture_stream();
    HIPX(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    launch_all(cs, true);
    hipGraph_t graph = nullptr;
    HIPX(hipStreamEndCapture(cs, &graph));
    HIPX(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    HIPX(hipGraphDestroy(graph));
    HIPX(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    std::lock_guard<std::mutex> lk(g_sgraph_mu);
    g_sgraphs[base] = StageGraph{h, exec, done};
  }
  HIPX(hipGraphLaunch(exec, st));
  HIPX(hipEventRecord(done, st));
}

int n_factors(int m, int fuse) { return (m + fuse - 1) / fuse; }

int strip_program_len(int m, int fuse, int n_max) {
  return n_max < 1 ? 0 : (m + 5) + (n_max - 1) * (n_factors(m, fuse) + 2);
}

// ---------------------------------------------------------------------------
// Plain per-instance path
// ---------------------------------------------------------------------------
struct PlainLayout {
  size_t x0, x1, w, bytes;
  int64_t s_nc, s_max;
};

PlainLayout plain_layout(int lattice, int m) {
  Sizes s = space_sizes(lattice, m);
  PlainLayout L;
  L.s_nc = s.s_nc;
  L.s_max = s.s_max;
  L.x0 = 0;
  L.x1 = align_up(s.s_max * 4);
  L.w = L.x1 + align_up(s.s_max * 4);
  L.bytes = L.w + align_up(s.s_nc * 4);
  return L;
}

void run_plain(const DevMaps& dm, int lattice, int m, int n_max, const std::vector<Inst>& inst, void* ws,
               hipStream_t st, uint32_t* d_out) {
  const PlainLayout L = plain_layout(lattice, m);
  char* b = static_cast<char*>(ws);
  uint32_t* x0 = reinterpret_cast<uint32_t*>(b + L.x0);
  uint32_t* x1 = reinterpret_cast<uint32_t*>(b + L.x1);
  uint32_t* w = reinterpret_cast<uint32_t*>(b + L.w);
  const int I = static_cast<int>(inst.size());
  auto g = [](int64_t n) { return dim3(static_cast<unsigned>((n + 255) / 256)); };
  for (int k = 0; k < I; ++k) {
    PlainConsts c{};
    c.p = inst[k].p;
    c.pinv = neg_inv_2_32(c.p);
    for (size_t code = 0; code < dm.codes.size(); ++code) {
      c.cval[code] = coef_mod(dm.codes[code], inst[k].q, c.p);
      c.cshp[code] = shoup_of(c.cval[code], c.p);
    }
    const uint32_t r1 = static_cast<uint32_t>((uint64_t(1) << 32) % c.p);
    hipLaunchKernelGGL(k_fill_plain, dim3(1), dim3(256), 0, st, x0, 1, r1);
    uint32_t* cur = x0;
    uint32_t* oth = x1;
    for (int i = m; i >= 1; --i) {
      const DevCsr& csr = dm.last[i - 1];
      uint32_t* dst = (i == 1) ? w : oth;
      hipLaunchKernelGGL(k_gather_plain, g(csr.n_rows), dim3(256), 0, st, csr, cur, dst, c);
      std::swap(cur, oth);
    }
    hipLaunchKernelGGL(k_fill_plain, g(L.s_nc), dim3(256), 0, st, x0, static_cast<int>(L.s_nc), 1u);
    hipLaunchKernelGGL(k_dot_plain, dim3(1), dim3(256), 0, st, x0, w, static_cast<int>(L.s_nc), c.p, c.pinv,
                       d_out + k);
    cur = x0;
    oth = x1;
    for (int r = 1; r < n_max; ++r) {
      for (int i = 1; i <= m; ++i) {
        const DevCsr& csr = dm.fwd[i - 1];
        hipLaunchKernelGGL(k_gather_plain, g(csr.n_rows), dim3(256), 0, st, csr, cur, oth, c);
        std::swap(cur, oth);
      }
      hipLaunchKernelGGL(k_dot_plain, dim3(1), dim3(256), 0, st, cur, w, static_cast<int>(L.s_nc), c.p, c.pinv,
                         d_out + static_cast<long>(r) * I + k);
    }
    HIPX(hipGetLastError());
  }
}

// ---------------------------------------------------------------------------
// Resident mode: one launch per strip (or per batch of strips); workgroup g
// holds K instances' state vectors in LDS (resident.hpp)
// ---------------------------------------------------------------------------
constexpr size_t kResMaxLds = 160 * 1024;

// Workspace of one resident job: per-instance code values and quotients,
// the job record, p, -p^{-1}, 2^32 mod p, 1 / p as a double, the code values
// as doubles, and the read-out vector [I][s_nc].  Code tables hold [I][nc]
// (nc codes of the family) in room for kMaxCodes.  One upload carries what
// the job's arithmetic reads, the job record included: [coef, rcp) for the
// modular form, [table, coff + I nc doubles) for the double form.
struct ResLayout {
  int I = 0, K = 1, ngroups = 0;
  int64_t s_nc = 0, s_max = 0;
  size_t coef = 0, coefs = 0, table = 0, p = 0, pinv = 0, r1 = 0, rcp = 0, coff = 0, w = 0, bytes = 0;
};

ResLayout res_layout(int lattice, int m, int I, const Tune& t) {
  ResLayout L;
  L.I = I;
  L.K = t.V;
  L.ngroups = (I + L.K - 1) / L.K;
  Sizes s = space_sizes(lattice, m);
  L.s_nc = s.s_nc;
  L.s_max = s.s_max;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += align_up(b);
    return o;
  };
  L.coef = take(static_cast<size_t>(I) * kMaxCodes * 4);
  L.coefs = take(static_cast<size_t>(I) * kMaxCodes * 4);
  L.table = take(sizeof(ResidentJob));
  L.p = take(static_cast<size_t>(I) * 4);
  L.pinv = take(static_cast<size_t>(I) * 4);
  L.r1 = take(static_cast<size_t>(I) * 4);
  L.rcp = take(static_cast<size_t>(I) * 8);
  L.coff = take(static_cast<size_t>(I) * kMaxCodes * 8);
  L.w = take(static_cast<size_t>(I) * L.s_nc * 4);
  L.bytes = off;
  return L;
}

// The double form's bound (resident.hpp): (longest row) x max |c(q)| <= 2^21.
constexpr int64_t kExactBound = int64_t(1) << 21;
constexpr int64_t kExactCode = kExactBound;

// c(q) as an exact integer (Horner; saturated at +-2^80, far past any bound
// it is compared with: q < 2^32 and the degree is at most 3).
__int128 code_value(const Poly& c, uint32_t q) {
  const __int128 cap = static_cast<__int128>(1) << 80;
  __int128 acc = 0;
  for (int k = kMaxDeg; k >= 0; --k) {
    acc = acc * q + c.c[k];
    if (acc > cap) acc = cap;
    if (acc < -cap) acc = -cap;
  }
  return acc;
}

// Whether every row of the strip's maps stays within the double form's
// bound at every instance.
bool resident_exact(const std::vector<Poly>& codes, const std::vector<Inst>& inst, int max_row) {
  __int128 big = 0;
  for (const Inst& in : inst)
    for (const Poly& c : codes) {
      const __int128 v = code_value(c, in.q);
      big = std::max(big, v < 0 ? -v : v);
    }
  return big <= kExactCode && static_cast<__int128>(std::max(max_row, 1)) * big <= kExactBound;
}

// Host image of the constants region [coef .. w) of a resident job: every
// code's value at each instance's q (the family's codes are polynomials in q
// with the base table first, so the read-out maps' codes are included).
std::vector<uint32_t> res_image(const ResLayout& L, const std::vector<Inst>& inst, const std::vector<Poly>& codes) {
  const int nc = static_cast<int>(codes.size());
  std::vector<uint32_t> img((L.w - L.coef) / 4, 0);
  uint32_t* coef = img.data() + (L.coef - L.coef) / 4;
  uint32_t* coefs = img.data() + (L.coefs - L.coef) / 4;
  uint32_t* p = img.data() + (L.p - L.coef) / 4;
  uint32_t* pinv = img.data() + (L.pinv - L.coef) / 4;
  uint32_t* r1 = img.data() + (L.r1 - L.coef) / 4;
  char* bytes = reinterpret_cast<char*>(img.data()) - L.coef;
  for (int i = 0; i < L.I; ++i) {
    const Inst& in = inst[i];
    for (int c = 0; c < nc; ++c) {
      const uint32_t v = coef_mod(codes[c], in.q, in.p);
      coef[static_cast<size_t>(i) * nc + c] = v;
      coefs[static_cast<size_t>(i) * nc + c] = shoup_of(v, in.p);
      // the integer itself where it is small (the double form runs only
      // when every value is: resident_exact)
      const __int128 e = code_value(codes[c], in.q);
      const double d = (e > kExactCode || e < -kExactCode) ? 0.0 : static_cast<double>(static_cast<int64_t>(e));
      std::memcpy(bytes + L.coff + (static_cast<size_t>(i) * nc + c) * 8, &d, 8);
    }
    const double rc = 1.0 / static_cast<double>(in.p);
    std::memcpy(bytes + L.rcp + static_cast<size_t>(i) * 8, &rc, 8);
    p[i] = in.p;
    pinv[i] = neg_inv_2_32(in.p);
    r1[i] = static_cast<uint32_t>((uint64_t(1) << 32) % in.p);
  }
  return img;
}

// The job record of one strip whose resident workspace starts at `base`;
// checks that the spaces fit the kernel's LDS and chain as the kernel
// assumes: it reads only rows the step before it wrote (the factors map
// NCNNN -> ... -> NCNNN, the read-out maps chain from their first space down
// to the NCNNN space, all within the LDS vectors).
ResidentJob resident_job(const DevMaps& dm, const DevFamily& fam, const ResLayout& L, void* base, int n_max,
                         uint32_t* d_out, int g0, size_t& lds, const std::vector<Inst>& inst, const Tune& t) {
  if (dm.m > kResMaxM) throw std::runtime_error("resident mode: m above the kernel's limit");
  // the double form unless stage 1 asks for the modular one or a row could
  // leave its exact range
  bool exact = false;
  if (t.stage == 0) exact = resident_exact(fam.codes, inst, dev_sell(dm, fam, false).max_row);
  const DevSellSet& sell = dev_sell(dm, fam, !exact);
  const int nf = static_cast<int>(sell.fac.size());
  const int nc = static_cast<int>(fam.codes.size());
  if (nf < 1 || nf > kResMaxM || nc > kMaxCodes) throw std::runtime_error("resident mode: factor family out of range");
  lds = resident_lds_bytes(static_cast<int>(L.s_max), nc, L.K);
  if (lds > kResMaxLds)
    throw std::runtime_error("resident mode: two state vectors of " + std::to_string(L.s_max) + " states x " +
                             std::to_string(L.K) + " instances need " + std::to_string(lds) +
                             " bytes of LDS, more than the 160 KiB a workgroup can hold");
  ResidentJob J{};
  for (int f = 0; f < nf; ++f) {
    const DevSell& c = sell.fac[f];
    const int64_t want_cols = f == 0 ? L.s_nc : sell.fac[f - 1].n_rows;
    if (c.n_rows > L.s_max || c.n_cols != want_cols || (f == nf - 1 && c.n_rows != L.s_nc))
      throw std::runtime_error("resident mode: factor spaces do not chain");
    J.fac[f] = c;
  }
  for (int i = 0; i < dm.m; ++i) {
    const DevSell& c = sell.last[i];
    if (c.n_rows > L.s_max || c.n_cols > L.s_max || (i + 1 < dm.m && c.n_cols != sell.last[i + 1].n_rows))
      throw std::runtime_error("resident mode: read-out spaces do not chain");
    J.last[i] = c;
  }
  if (sell.last[0].n_rows != L.s_nc) throw std::runtime_error("resident mode: read-out vector size mismatch");
  char* b = static_cast<char*>(base);
  J.nf = nf;
  J.m = dm.m;
  J.s_nc = static_cast<int>(L.s_nc);
  J.s_max = static_cast<int>(L.s_max);
  J.n_max = n_max;
  J.I = L.I;
  J.ncodes = nc;
  J.g0 = g0;
  J.ngroups = L.ngroups;
  J.coef = reinterpret_cast<const uint32_t*>(b + L.coef);
  J.coefs = reinterpret_cast<const uint32_t*>(b + L.coefs);
  J.coff = reinterpret_cast<const double*>(b + L.coff);
  J.rcp = reinterpret_cast<const double*>(b + L.rcp);
  J.exact = exact ? 1 : 0;
  J.p = reinterpret_cast<const uint32_t*>(b + L.p);
  J.pinv = reinterpret_cast<const uint32_t*>(b + L.pinv);
  J.r1 = reinterpret_cast<const uint32_t*>(b + L.r1);
  J.w = reinterpret_cast<uint32_t*>(b + L.w);
  J.out = d_out;
  return J;
}

// Lifts the dynamic-LDS limit of k_resident<K> to 160 KiB once per device.
template <int K>
void allow_resident_lds() {
  static bool done[64] = {false};
  static std::mutex mu;
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if (done[dev]) return;
  HIPX(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_resident<K>),
                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kResMaxLds)));
  done[dev] = true;
}

// Launches every job's workgroups at once (one launch: no workgroup waits on
// another); `table` holds the job records, uploaded by the caller on `st`.
void run_resident(const std::vector<ResidentJob>& jobs, size_t lds, const Tune& t, const void* table, hipStream_t st) {
  if (jobs.empty()) return;
  int total = 0;
  for (const ResidentJob& J : jobs) total = std::max(total, J.g0 + J.ngroups);
  if (total < 1) return;
  const ResidentJob* d = static_cast<const ResidentJob*>(table);
  const int nj = static_cast<int>(jobs.size());
  dim3 grid(total), block(64 * t.wpb);
  switch (t.V) {
    case 1:
      allow_resident_lds<1>();
      hipLaunchKernelGGL(k_resident<1>, grid, block, lds, st, d, nj);
      break;
    case 2:
      allow_resident_lds<2>();
      hipLaunchKernelGGL(k_resident<2>, grid, block, lds, st, d, nj);
      break;
    default:
      allow_resident_lds<4>();
      hipLaunchKernelGGL(k_resident<4>, grid, block, lds, st, d, nj);
      break;
  }
  HIPX(hipGetLastError());
}

// Refuses, before any device work, a width whose two state vectors alone
// exceed the LDS a workgroup can hold.
void check_resident_fits(int lattice, int m, const Tune& t) {
  const Sizes s = space_sizes(lattice, m);
  if (resident_lds_bytes(static_cast<int>(s.s_max), 0, t.V) > kResMaxLds)
    throw std::runtime_error("resident mode: two state vectors of " + std::to_string(s.s_max) + " states x " +
                             std::to_string(t.V) + " instances exceed the 160 KiB of LDS a workgroup can hold");
}

size_t resident_workspace_bytes(int lattice, int m, int I, const Tune& t) {
  check_resident_fits(lattice, m, t);
  return res_layout(lattice, m, I, t).bytes;
}

// ---------------------------------------------------------------------------
// Strip front end shared by the sync and async calls
// ---------------------------------------------------------------------------
int rows_tile_of(const Tune& t) { return t.rpw * t.wpb; }

// Staged tiles for the forward factors of a batched or graph-mode job.
// The grouped kernel runs plain gathers, so grouped launches (batches,
// server steps, grouped strips) take the target orders of stages 4
// (clustered) and 6 (interleaved) but not LDS staging or op streams.
void check_batch_stage(const Tune& t) {
  if (t.stage != 0 && t.stage != 4 && t.stage != 6)
    throw ArgError("grouped launches (chromatic_batch, server steps, grouped strips) take stage 0, 4 or 6");
}

// Stages 4 and 6 only reorder a factor's targets, so grouped launches (whose
// kernel gathers directly) take them too; LDS staging (1-3) and op streams
// (5) need their own kernels (batched and graph modes).
void bind_staging(JobCtx& j, int mode) {
  const bool direct = mode == CHROM_MODE_BATCHED || mode == CHROM_MODE_GRAPH;
  if (mode == CHROM_MODE_GROUPED && j.t.stage == 4)
    j.stg = &dev_staged(*j.dm, *j.fam, stage_slots(std::min(j.t.V, 2)), rows_tile_of(j.t), 2);
  else if (j.t.stage == 5 && direct)
    j.ops = &dev_ops(*j.dm, *j.fam);
  else if (j.t.stage == 6 && (direct || mode == CHROM_MODE_GROUPED))
    j.stg = &dev_staged(*j.dm, *j.fam, j.t.wpb, rows_tile_of(j.t), 3);
  else if (j.t.stage && j.t.stage != 5 && j.t.stage != 6 && j.t.V <= 2 &&
           (mode == CHROM_MODE_BATCHED || mode == CHROM_MODE_GRAPH))
    j.stg = &dev_staged(*j.dm, *j.fam, stage_slots(j.t.V), rows_tile_of(j.t), j.t.stage == 1 ? 1 : 2);
  else if (j.t.stage == 4 && (mode == CHROM_MODE_BATCHED || mode == CHROM_MODE_GRAPH))
    j.stg = &dev_staged(*j.dm, *j.fam, stage_slots(std::min(j.t.V, 2)), rows_tile_of(j.t), 2);
}

// One job's region: its layout, the graph row counter, grouped stage tables.
size_t job_workspace_bytes(int lattice, int m, int I, int n_max_hint, int mode, const Tune& t) {
  JobLayout L = job_layout(lattice, m, I, t, kMaxCodes, rows_tile_of(t));
  size_t b = L.bytes + 256;  // + graph row counter
  if (mode == CHROM_MODE_GROUPED) {
    const long len = strip_program_len(m, t.fuse, n_max_hint);
    b += stage_bytes(L.nchunk * len, len);
  }
  return b;
}

// lanes_v 4 runs chunks of 256 instances.  When the instance count is not a
// multiple of 256, the lanes of the last chunk past it would compute padding;
// instead the first floor(I / 256) * 256 instances run at lanes_v 4 and the
// rest as a second job at lanes_v 2 (1 for at most 64 instances), on a
// parallel branch (batched and graph modes).  Instances are
// independent, so the residues are the same.  Each job has its own region
// of the workspace.
struct SplitPlan {
  int n = 1;
  int I[2] = {0, 0};
  Tune t[2];
  size_t off[2] = {0, 0};
  size_t bytes = 0;
};

SplitPlan split_plan(int lattice, int m, int I, int n_max_hint, int mode, const Tune& t) {
  SplitPlan sp;
  sp.I[0] = I;
  sp.t[0] = t;
  if ((mode == CHROM_MODE_BATCHED || mode == CHROM_MODE_GRAPH) && t.V == 4 && I > 256 && I % 256 != 0) {
    sp.n = 2;
    sp.I[0] = I / 256 * 256;
    sp.I[1] = I - sp.I[0];
    sp.t[1] = t;
    // lanes_v 1 for at most 64 left, else 2, one chunk group.  (128 left as
    // two lanes_v 1 chains took the square 14x15 step from 8.32 to 8.25 ms
    // but the 18x19 strip, whose vectors live in HBM, from about 720 to
    // 741 ms: 256-byte rows gather less efficiently there.)
    sp.t[1].V = sp.I[1] <= 64 ? 1 : 2;
    sp.t[1].streams = 1;
  }
  for (int k = 0; k < sp.n; ++k) {
    sp.off[k] = sp.bytes;
    sp.bytes += align_up(job_workspace_bytes(lattice, m, sp.I[k], n_max_hint, mode, sp.t[k]));
  }
  return sp;
}

size_t workspace_bytes(int lattice, int m, int I, int n_max_hint, int mode, const Tune& t) {
  if (mode == CHROM_MODE_PLAIN) return plain_layout(lattice, m).bytes;
  if (mode == CHROM_MODE_RESIDENT) return resident_workspace_bytes(lattice, m, I, t);
  return split_plan(lattice, m, I, n_max_hint, mode, t).bytes;
}

// The second job of a split in batched mode runs on a library stream forked
// from and joined back into the caller's (one per device).
std::mutex g_split_mu;
SplitStream g_split[64];

template <class F>
void fork_join_split(hipStream_t st, F&& body) {
  std::lock_guard<std::mutex> lk(g_split_mu);
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  SplitStream& ss = g_split[dev];
  if (!ss.s) {
    HIPX(hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking));
    HIPX(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming));
    HIPX(hipEventCreateWithFlags(&ss.join, hipEventDisableTiming));
  }
  HIPX(hipEventRecord(ss.fork, st));
  HIPX(hipStreamWaitEvent(ss.s, ss.fork, 0));
  body(0, st);
  body(1, ss.s);
  HIPX(hipEventRecord(ss.join, ss.s));
  HIPX(hipStreamWaitEvent(st, ss.join, 0));
}

int strip_async_impl(int lattice, int m, int n_max, const uint32_t* q, int nq, const uint32_t* p, int np, int mode,
                     const chrom_tuning* tune, void* ws, size_t ws_bytes, hipStream_t st, uint32_t* d_out) {
  check_args(lattice, m, n_max);
  check_mode(mode);
  std::vector<Inst> inst = make_instances(q, nq, p, np);
  Tune t = resolve(tune, false, mode == CHROM_MODE_RESIDENT);
  if (mode == CHROM_MODE_RESIDENT) check_resident_fits(lattice, m, t);
  if (mode == CHROM_MODE_GROUPED) check_batch_stage(t);
  if (n_max == 0) return CHROM_OK;
  if (!ws || !d_out) throw ArgError("null workspace or output");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) throw ArgError("workspace must be 256-byte aligned");
  const int I = static_cast<int>(inst.size());
  const size_t need = (mode == CHROM_MODE_PLAIN) ? plain_layout(lattice, m).bytes
                                                 : workspace_bytes(lattice, m, I, n_max, mode, t);
  if (ws_bytes < need) throw MemError("workspace too small: need " + std::to_string(need) + " bytes");
  const DevMaps& dm = dev_maps(lattice, m);
  if (mode == CHROM_MODE_PLAIN) {
    run_plain(dm, lattice, m, n_max, inst, ws, st, d_out);
    return CHROM_OK;
  }
  if (mode == CHROM_MODE_RESIDENT) {
    const DevFamily& fam = dev_family(dm, t.fuse);
    ResLayout R = res_layout(lattice, m, I, t);
    size_t lds = 0;
    std::vector<ResidentJob> jobs{resident_job(dm, fam, R, ws, n_max, d_out, 0, lds, inst, t)};
    std::vector<uint32_t> img = res_image(R, inst, fam.codes);
    std::memcpy(reinterpret_cast<char*>(img.data()) + (R.table - R.coef), jobs.data(), sizeof(ResidentJob));
    // one upload: the job record and the constants the job's arithmetic reads
    const size_t nc = fam.codes.size();
    const size_t lo = jobs[0].exact ? R.table : R.coef;
    const size_t hi = jobs[0].exact ? R.coff + static_cast<size_t>(I) * nc * 8 : R.rcp;
    upload(static_cast<char*>(ws) + lo, reinterpret_cast<const char*>(img.data()) + (lo - R.coef), hi - lo, st);
    run_resident(jobs, lds, t, static_cast<char*>(ws) + R.table, st);
    return CHROM_OK;
  }
  const SplitPlan sp = split_plan(lattice, m, I, n_max, mode, t);
  // job k: instances [i0, i0 + sp.I[k]) of the list, its own workspace
  // region, output columns i0.. of rows of I; constants uploaded on `s`
  auto make_job = [&](int k, hipStream_t s) {
    const int i0 = k == 0 ? 0 : sp.I[0];
    const std::vector<Inst> sub(inst.begin() + i0, inst.begin() + i0 + sp.I[k]);
    const Tune& tk = sp.t[k];
    char* wk = static_cast<char*>(ws) + sp.off[k];
    JobCtx j;
    j.dm = &dm;
    j.fam = &dev_family(dm, tk.fuse);
    j.t = tk;
    j.L = job_layout(lattice, m, sp.I[k], tk, kMaxCodes, rows_tile_of(tk));
    j.P = job_ptrs(j.L, wk);
    j.d_out = d_out + i0;
    j.out_row_stride = I;
    bind_staging(j, mode);
    std::vector<uint32_t> img = const_image(j.L, sub, j.fam->codes, j.fam->shift);
    upload(wk + j.L.p, img.data(), img.size() * 4, s);
    return j;
  };
  auto row_ctr_of = [&](int k, const JobCtx& j) {
    return reinterpret_cast<int*>(static_cast<char*>(ws) + sp.off[k] + j.L.bytes);
  };
  if (sp.n == 2 && mode == CHROM_MODE_GRAPH) {
    const JobCtx ja = make_job(0, st), jb = make_job(1, st);
    run_graph_split(ja, jb, n_max, row_ctr_of(0, ja), row_ctr_of(1, jb), ws, st);
    return CHROM_OK;
  }
  auto run_job = [&](int k, hipStream_t s) {
    const JobCtx j = make_job(k, s);
    const Tune& tk = j.t;
    char* wk = static_cast<char*>(ws) + sp.off[k];
    int* row_ctr = row_ctr_of(k, j);
    if (mode == CHROM_MODE_BATCHED) {
      Program pg = strip_program(j, n_max);
      run_eager(pg, tk, s);
    } else if (mode == CHROM_MODE_GRAPH) {
      run_graph(j, n_max, row_ctr, wk, s);
    } else {
      Program pg = strip_program(j, n_max);
      run_grouped({&pg}, tk, wk + j.L.bytes + 256, s, true);
    }
  };
  if (sp.n == 1)
    run_job(0, st);
  else
    fork_join_split(st, run_job);
  return CHROM_OK;
}

struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t n) {
    if (n && hipMalloc(&p, n) != hipSuccess) throw MemError("device allocation of " + std::to_string(n) + " bytes failed");
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

int strip_sync_impl(int lattice, int m, int n_max, const uint32_t* q, int nq, const uint32_t* p, int np, int mode,
                    const chrom_tuning* tune, uint32_t* out) {
  check_args(lattice, m, n_max);
  check_mode(mode);
  std::vector<Inst> inst = make_instances(q, nq, p, np);
  if (n_max == 0) return CHROM_OK;
  if (!out) throw ArgError("null output");
  Tune t = resolve(tune, false, mode == CHROM_MODE_RESIDENT);
  if (mode == CHROM_MODE_RESIDENT) check_resident_fits(lattice, m, t);
  if (mode == CHROM_MODE_GROUPED) check_batch_stage(t);
  const int I = static_cast<int>(inst.size());
  const size_t wsb = workspace_bytes(lattice, m, I, n_max, mode, t);
  DevBuf ws(wsb);
  const size_t outb = static_cast<size_t>(n_max) * I * 4;
  DevBuf dout(outb);
  HIPX(hipMemset(dout.p, 0, outb));
  int rc = strip_async_impl(lattice, m, n_max, q, nq, p, np, mode, tune, ws.p, wsb, nullptr,
                            static_cast<uint32_t*>(dout.p));
  if (rc != CHROM_OK) return rc;
  HIPX(hipDeviceSynchronize());
  HIPX(hipMemcpy(out, dout.p, outb, hipMemcpyDeviceToHost));
  if (mode == CHROM_MODE_GROUPED) drop_stage_graphs_in(ws.p, wsb);
  if (mode == CHROM_MODE_GRAPH) {
    // graphs captured on this workspace are invalid once it is freed
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
      if (it->first.ws == ws.p) {
        (void)hipGraphExecDestroy(it->second.exec);
        it = g_graphs.erase(it);
      } else {
        ++it;
      }
    }
  }
  return CHROM_OK;
}

// ---------------------------------------------------------------------------
// Coefficient form (normalised weights as truncated polynomials in x = 1/q)
// ---------------------------------------------------------------------------
// Largest read-out space of the coefficient form: T_i^last leaves the
// points 1..i singletons, N(m - i) states, largest for i = 1.
int64_t readout_l_max(int lattice, int m) {
  (void)lattice;
  return std::max<int64_t>(1, ncnnn_count(m - 1));
}

// lanes_v 0 (or no tuning): the smallest of 1, 2, 4, 8 whose 64 lanes_v
// slots hold x^0 .. x^d_max.
Tune resolve_series(const chrom_tuning* tune, int d_max) {
  chrom_tuning tt{};
  if (tune) tt = *tune;
  if (!tt.lanes_v) tt.lanes_v = d_max < 64 ? 1 : (d_max < 128 ? 2 : (d_max < 256 ? 4 : 8));
  Tune t = resolve(&tt, true);
  if (t.fuse != 1) throw ArgError("the coefficient form runs single factors only (fuse 1)");
  if (t.stage) throw ArgError("the coefficient form does not stage tiles");
  return t;
}

size_t series_workspace_bytes(int lattice, int m, int np, int d_max, const Tune& t) {
  return job_layout_series(lattice, m, np, d_max, t, readout_l_max(lattice, m)).bytes + 256;  // + row counter
}

void check_primes(const uint32_t* p, int np) {
  if (np < 1 || !p) throw ArgError("need at least one prime");
  for (int b = 0; b < np; ++b)
    if (p[b] <= 2u || p[b] >= (1u << 31) || (p[b] & 1u) == 0u)
      throw ArgError("each prime must be odd with 2 < p < 2^31");
}

int series_async_impl(int lattice, int m, int n_max, int d_max, const uint32_t* p, int np, int mode,
                      const chrom_tuning* tune, void* ws, size_t ws_bytes, hipStream_t st, uint32_t* d_out) {
  check_args(lattice, m, n_max);
  if (mode != CHROM_MODE_BATCHED && mode != CHROM_MODE_GRAPH)
    throw ArgError("the coefficient form runs in batched or graph mode");
  check_primes(p, np);
  Tune t = resolve_series(tune, d_max);
  if (n_max == 0) return CHROM_OK;
  if (!ws || !d_out) throw ArgError("null workspace or output");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) throw ArgError("workspace must be 256-byte aligned");
  const DevMaps& dm = dev_maps(lattice, m, true);
  JobCtx j;
  j.dm = &dm;
  j.fam = &dev_family(dm, 1);
  j.t = t;
  j.L = job_layout_series(lattice, m, np, d_max, t, dm.l_max);
  if (ws_bytes < j.L.bytes + 256) throw MemError("workspace too small: need " + std::to_string(j.L.bytes + 256) + " bytes");
  j.P = job_ptrs(j.L, ws);
  j.d_out = d_out;
  j.out_row_stride = static_cast<long>(np) * j.L.dlen;
  std::vector<Inst> inst(j.L.ipad);
  for (int k = 0; k < j.L.ipad; ++k) inst[k] = Inst{0u, p[k / j.L.W]};
  std::vector<uint32_t> img = const_image(j.L, inst, j.fam->codes, 0);
  upload(static_cast<char*>(ws) + j.L.p, img.data(), img.size() * 4, st);
  std::vector<uint32_t> e0(2 * static_cast<size_t>(j.L.ipad), 0u);   // e_0, then zeros
  for (int c = 0; c < np; ++c) e0[static_cast<size_t>(c) * j.L.W] = 1u;
  upload(static_cast<char*>(ws) + j.L.e0, e0.data(), e0.size() * 4, st);
  int* row_ctr = reinterpret_cast<int*>(static_cast<char*>(ws) + j.L.bytes);
  if (mode == CHROM_MODE_BATCHED) {
    Program pg = strip_program(j, n_max);
    run_eager(pg, t, st);
  } else {
    run_graph(j, n_max, row_ctr, ws, st);
  }
  return CHROM_OK;
}

void drop_graphs_on(void* ws) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto it = g_graphs.begin(); it != g_graphs.end();) {
    if (it->first.ws == ws) {
      (void)hipGraphExecDestroy(it->second.exec);
      it = g_graphs.erase(it);
    } else {
      ++it;
    }
  }
}

int series_sync_impl(int lattice, int m, int n_max, int d_max, const uint32_t* p, int np, int mode,
                     const chrom_tuning* tune, uint32_t* out) {
  check_args(lattice, m, n_max);
  check_primes(p, np);
  if (n_max == 0) return CHROM_OK;
  if (!out) throw ArgError("null output");
  const Tune t = resolve_series(tune, d_max);
  const size_t wsb = series_workspace_bytes(lattice, m, np, d_max, t);
  DevBuf ws(wsb);
  const size_t outb = static_cast<size_t>(n_max) * np * (d_max + 1) * 4;
  DevBuf dout(outb);
  HIPX(hipMemset(dout.p, 0, outb));
  int rc = series_async_impl(lattice, m, n_max, d_max, p, np, mode, tune, ws.p, wsb, nullptr,
                             static_cast<uint32_t*>(dout.p));
  if (rc != CHROM_OK) return rc;
  HIPX(hipDeviceSynchronize());
  HIPX(hipMemcpy(out, dout.p, outb, hipMemcpyDeviceToHost));
  if (mode == CHROM_MODE_GRAPH) drop_graphs_on(ws.p);
  return CHROM_OK;
}

// Queues rows x m gather launches (T_1..T_m, read-out fused into T_m) on a
// workspace that chromatic_strip_async (batched mode, same tuning) has set
// up; nothing else.  Lets a caller time the factor kernel alone.
int factor_launches_impl(int lattice, int m, const uint32_t* q, int nq, const uint32_t* p, int np, int rows,
                         const chrom_tuning* tune, void* ws, size_t ws_bytes, hipStream_t st) {
  check_args(lattice, m, 1);
  if (rows < 1) throw ArgError("rows must be >= 1");
  std::vector<Inst> inst = make_instances(q, nq, p, np);
  Tune t = resolve(tune);
  const int I = static_cast<int>(inst.size());
  if (!ws || ws_bytes < workspace_bytes(lattice, m, I, 1, CHROM_MODE_BATCHED, t))
    throw MemError("workspace missing or too small");
  const DevMaps& dm = dev_maps(lattice, m);
  // the jobs of a lanes_v 4 split, one after the other on `st`: step by
  // step, the first job's launch then the second's
  const SplitPlan sp = split_plan(lattice, m, I, 1, CHROM_MODE_BATCHED, t);
  std::vector<JobCtx> jobs(sp.n);
  std::vector<Program> gathers(sp.n);
  for (int k = 0; k < sp.n; ++k) {
    JobCtx& j = jobs[k];
    j.dm = &dm;
    j.fam = &dev_family(dm, sp.t[k].fuse);
    j.t = sp.t[k];
    j.L = job_layout(lattice, m, sp.I[k], sp.t[k], kMaxCodes, rows_tile_of(sp.t[k]));
    j.P = job_ptrs(j.L, static_cast<char*>(ws) + sp.off[k]);
    j.d_out = nullptr;
    bind_staging(j, CHROM_MODE_BATCHED);
    Program pg;
    pg.nchunk = j.L.nchunk;
    add_rows(pg, j, 1, rows, -1, -1);
    gathers[k].nchunk = pg.nchunk;
    for (const PStep& ps : pg.steps)
      if (ps.s.op == kOpGather) gathers[k].steps.push_back(ps);
  }
  const size_t nsteps = gathers[0].steps.size();
  for (size_t i = 0; i < nsteps; ++i)
    for (int k = 0; k < sp.n; ++k) {
      Program one;
      one.nchunk = gathers[k].nchunk;
      one.steps.push_back(gathers[k].steps[i]);
      run_eager(one, jobs[k].t, st);
    }
  return CHROM_OK;
}

// ---------------------------------------------------------------------------
// Many jobs in one graph of grouped launches
// ---------------------------------------------------------------------------
struct BatchPlan {
  std::vector<size_t> job_off;
  std::vector<JobLayout> layouts;
  size_t queue_off = 0, bytes = 0;
  long nsteps = 0, nstages = 0;
  int groups = 1;   // chunk groups on parallel streams (tuning `streams`, 1..4)
};

BatchPlan batch_plan(const chrom_job* jobs, int njobs, const Tune& t) {
  if (njobs < 0 || (njobs > 0 && !jobs)) throw ArgError("bad job list");
  BatchPlan bp;
  size_t off = 0;
  for (int k = 0; k < njobs; ++k) {
    const chrom_job& jb = jobs[k];
    check_args(jb.lattice, jb.m, jb.n_max);
    if (jb.nq < 1 || jb.np < 1) throw ArgError("job needs q points and primes");
    JobLayout L = job_layout(jb.lattice, jb.m, jb.nq * jb.np, t, kMaxCodes, rows_tile_of(t));
    bp.layouts.push_back(L);
    bp.job_off.push_back(off);
    off += align_up(L.bytes);
    bp.nsteps += static_cast<long>(L.nchunk) * strip_program_len(jb.m, t.fuse, jb.n_max);
    bp.nstages = std::max<long>(bp.nstages, strip_program_len(jb.m, t.fuse, jb.n_max));
  }
  bp.queue_off = off;
  // Chunk groups on parallel graph branches are switched off for batches:
  // a tuning run over many batch shapes ended in a host segmentation fault
  // on a three-group candidate whose cause was not found.  `streams` is
  // ignored here, as it was before the groups existed.
  bp.groups = 1;
  bp.bytes = off + bp.groups * stage_bytes(bp.nsteps, bp.nstages);
  return bp;
}

int batch_impl(const chrom_job* jobs, int njobs, const chrom_tuning* tune, void* ws, size_t ws_bytes, hipStream_t st) {
  Tune t = resolve(tune);
  check_batch_stage(t);
  BatchPlan bp = batch_plan(jobs, njobs, t);
  if (njobs == 0) return CHROM_OK;
  if (!ws) throw ArgError("null workspace");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) throw ArgError("workspace must be 256-byte aligned");
  if (ws_bytes < bp.bytes) throw MemError("workspace too small: need " + std::to_string(bp.bytes) + " bytes");
  std::vector<Program> progs(njobs);
  std::vector<const Program*> pp;
  for (int k = 0; k < njobs; ++k) {
    const chrom_job& jb = jobs[k];
    std::vector<Inst> inst = make_instances(jb.q_points, jb.nq, jb.primes, jb.np);
    if (jb.n_max > 0 && !jb.d_out) throw ArgError("null job output");
    const DevMaps& dm = dev_maps(jb.lattice, jb.m);
    JobCtx j;
    j.dm = &dm;
    j.fam = &dev_family(dm, t.fuse);
    j.t = t;
    j.L = bp.layouts[k];
    void* base = static_cast<char*>(ws) + bp.job_off[k];
    j.P = job_ptrs(j.L, base);
    j.d_out = jb.d_out;
    j.out_row_stride = j.L.I;
    bind_staging(j, CHROM_MODE_GROUPED);   // stages 4 and 6: the target orders
    if (jb.n_max > 0) {
      std::vector<uint32_t> img = const_image(j.L, inst, j.fam->codes, j.fam->shift);
      upload(static_cast<char*>(base) + j.L.p, img.data(), img.size() * 4, st);
    }
    progs[k] = strip_program(j, jb.n_max);
    pp.push_back(&progs[k]);
  }
  run_grouped(pp, t, static_cast<char*>(ws) + bp.queue_off, st, true, bp.groups);
  return CHROM_OK;
}

// ---------------------------------------------------------------------------
// Server step
// ---------------------------------------------------------------------------
std::mutex g_srv_mu;
void* g_srv_queue[64] = {nullptr};
size_t g_srv_queue_bytes[64] = {0};

void* server_queue(size_t bytes) {
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_srv_mu);
  if (g_srv_queue_bytes[dev] < bytes) {
    if (g_srv_queue[dev]) {
      HIPX(hipDeviceSynchronize());
      HIPX(hipFree(g_srv_queue[dev]));
    }
    size_t nb = std::max(bytes, size_t(1) << 22);
    if (hipMalloc(&g_srv_queue[dev], nb) != hipSuccess) throw MemError("server queue allocation failed");
    g_srv_queue_bytes[dev] = nb;
  }
  return g_srv_queue[dev];
}

int server_step_impl(chrom_slot* slots, int nslots, int rows, const chrom_tuning* tune, hipStream_t st) {
  if (nslots < 0 || (nslots > 0 && !slots)) throw ArgError("bad slot list");
  if (rows < 1) throw ArgError("rows must be >= 1");
  Tune t = resolve(tune);
  check_batch_stage(t);
  std::vector<Program> progs(nslots);
  std::vector<const Program*> pp;
  std::vector<int> new_done(nslots);
  for (int k = 0; k < nslots; ++k) {
    chrom_slot& sl = slots[k];
    check_args(sl.lattice, sl.m, sl.n_max);
    new_done[k] = sl.rows_done;
    if (sl.rows_done >= sl.n_max) continue;
    if (sl.rows_done < 0) throw ArgError("rows_done must be >= 0");
    const int I = sl.nq * sl.np;
    if (I < 1) throw ArgError("slot needs q points and primes");
    JobLayout L = job_layout(sl.lattice, sl.m, I, t, kMaxCodes, rows_tile_of(t));
    if (!sl.d_state || sl.state_bytes < L.bytes) throw MemError("slot state buffer too small");
    if (reinterpret_cast<uintptr_t>(sl.d_state) % 256 != 0) throw ArgError("slot state must be 256-byte aligned");
    if (!sl.d_out) throw ArgError("null slot output");
    const DevMaps& dm = dev_maps(sl.lattice, sl.m);
    JobCtx j;
    j.dm = &dm;
    j.fam = &dev_family(dm, t.fuse);
    j.t = t;
    j.L = L;
    j.P = job_ptrs(L, sl.d_state);
    j.d_out = sl.d_out;
    j.out_row_stride = j.L.I;
    bind_staging(j, CHROM_MODE_GROUPED);   // stages 4 and 6: the target orders
    progs[k].nchunk = L.nchunk;
    int first = sl.rows_done;
    int last_row = std::min(sl.n_max - 1, first + rows - 1);  // 0-based out rows to produce
    if (first == 0) {
      std::vector<Inst> inst = make_instances(sl.q_points, sl.nq, sl.primes, sl.np);
      std::vector<uint32_t> img = const_image(L, inst, j.fam->codes, j.fam->shift);
      upload(static_cast<char*>(sl.d_state) + L.p, img.data(), img.size() * 4, st);
      int red = add_setup(progs[k], j);
      if (last_row >= 1) add_rows(progs[k], j, 1, last_row, red, red);
    } else {
      add_rows(progs[k], j, first, last_row, -1, -1);
    }
    new_done[k] = last_row + 1;
    pp.push_back(&progs[k]);
  }
  int nsteps = 0;
  for (const Program* pg : pp) nsteps += pg->nchunk * static_cast<int>(pg->steps.size());
  if (nsteps > 0) {
    long nstages = 0;
    for (const Program* pg : pp) nstages = std::max<long>(nstages, static_cast<long>(pg->steps.size()));
    void* q = server_queue(stage_bytes(nsteps, nstages));
    run_grouped(pp, t, q, st, false);
  }
  for (int k = 0; k < nslots; ++k) slots[k].rows_done = new_done[k];
  return CHROM_OK;
}

// ---------------------------------------------------------------------------
// No-allocation strip: the workspace is a file-scope device array
// ---------------------------------------------------------------------------
// For callers that cannot allocate (graph capture, tight serving loops): the
// batched strip with its workspace in `scratch`, a device array of
// kScratchBytes that every GPU the library runs on holds until the process
// ends.  Host code never passes `scratch` itself to a kernel or a copy: it
// uses the address hipGetSymbolAddress returns for the current device
// (scratch_ptr).  The per-instance constants are computed on the device from
// q and p passed as kernel arguments, so the call queues kernels only.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kNoAllocMaxQ = 512, kNoAllocMaxP = 64;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {nullptr};

// Device address of `scratch` on the current device, looked up once per device.
void* scratch_ptr() {
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw std::runtime_error("device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPX(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw HipError("hipGetSymbolAddress returned a null address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

// Kernel-argument image of a job's constants (the host-side const_image,
// computed on the device).
struct ConstSetupArgs {
  int nq, np, I, ipad, shift;
  uint32_t q[kNoAllocMaxQ];
  uint32_t p[kNoAllocMaxP];
  uint32_t poly[2 * kMaxCodes];
  uint32_t *dp, *dpinv, *dr1, *dtv, *dts, *dpoly;
};

__global__ void k_setup_consts(const ConstSetupArgs a) {
  const int i = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < 2 * kMaxCodes) a.dpoly[i] = a.poly[i];
  if (i >= a.ipad) return;
  const int inst = i < a.I ? i : 0;             // padding repeats instance 0
  const uint32_t p = a.p[inst % a.np];
  const uint32_t q = a.q[inst / a.np] % p;
  uint32_t inv = p;                             // -p^{-1} mod 2^32 by Newton's iteration
  for (int k = 0; k < 5; ++k) inv *= 2u - p * inv;
  const uint32_t sm = static_cast<uint32_t>(((a.shift % static_cast<int64_t>(p)) + p) % p);
  const uint32_t tv = static_cast<uint32_t>((static_cast<uint64_t>(q) + p - sm) % p);
  a.dp[i] = p;
  a.dpinv[i] = 0u - inv;
  a.dr1[i] = static_cast<uint32_t>((uint64_t(1) << 32) % p);
  a.dtv[i] = tv;
  a.dts[i] = static_cast<uint32_t>((static_cast<uint64_t>(tv) << 32) / p);
}

int strip_noalloc_impl(int lattice, int m, int n_max, const uint32_t* q, int nq, const uint32_t* p, int np,
                       const chrom_tuning* tune, hipStream_t st, uint32_t* d_out) {
  check_args(lattice, m, n_max);
  std::vector<Inst> inst = make_instances(q, nq, p, np);
  if (nq > kNoAllocMaxQ || np > kNoAllocMaxP)
    throw ArgError("at most " + std::to_string(kNoAllocMaxQ) + " q points and " + std::to_string(kNoAllocMaxP) +
                   " primes");
  Tune t = resolve(tune);
  if (t.streams != 1 || t.stage != 0) throw ArgError("the no-allocation strip runs one stream without staging");
  if (n_max == 0) return CHROM_OK;
  if (!d_out) throw ArgError("null output");
  const int I = static_cast<int>(inst.size());
  JobLayout L = job_layout(lattice, m, I, t, kMaxCodes, rows_tile_of(t));
  if (L.bytes > kScratchBytes)
    throw ArgError("this strip needs " + std::to_string(L.bytes) + " bytes of workspace, more than the " +
                   std::to_string(kScratchBytes) + " the no-allocation strip holds");
  // maps and family must already be on the device (chromatic_prepare; fused
  // families after one call of another entry point with that fuse)
  const DevMaps* dm = nullptr;
  {
    int dev = 0;
    HIPX(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev.find(std::make_tuple(dev, lattice, m, 0));
    if (it != g_dev.end()) dm = it->second.get();
  }
  if (!dm) throw ArgError("the factor maps of this (lattice, m) are not on the device: call chromatic_prepare first");
  const DevFamily* fam = nullptr;
  {
    std::lock_guard<std::mutex> lk(dm->fam_mu);
    auto it = dm->fam.find(t.fuse);
    if (it != dm->fam.end()) fam = it->second.get();
  }
  if (!fam) throw ArgError("the fused maps of this fuse are not on the device: run the strip once with it first");
  void* ws = scratch_ptr();
  JobCtx j;
  j.dm = dm;
  j.fam = fam;
  j.t = t;
  j.L = L;
  j.P = job_ptrs(L, ws);
  j.d_out = d_out;
  j.out_row_stride = L.I;
  ConstSetupArgs a{};
  a.nq = nq;
  a.np = np;
  a.I = I;
  a.ipad = L.ipad;
  a.shift = fam->shift;
  for (int k = 0; k < nq; ++k) a.q[k] = q[k];
  for (int k = 0; k < np; ++k) a.p[k] = p[k];
  if (fam->codes.size() < 2 || !(fam->codes[0].c[0] == 1 && fam->codes[1].c[0] == -1))
    throw std::runtime_error("code table must start with +1 and -1");
  for (size_t c = 0; c < fam->codes.size(); ++c) {
    const Poly d = shift_basis(fam->codes[c], fam->shift);
    a.poly[c] = pack_poly(d);
    a.poly[kMaxCodes + c] = pack_mask(d);
  }
  a.dp = j.P.p;
  a.dpinv = j.P.pinv;
  a.dr1 = j.P.r1;
  a.dtv = j.P.tv;
  a.dts = j.P.ts;
  a.dpoly = j.P.poly;
  const int nthreads = std::max(L.ipad, 2 * kMaxCodes);
  hipLaunchKernelGGL(k_setup_consts, dim3((nthreads + 255) / 256), dim3(256), 0, st, a);
  HIPX(hipGetLastError());
  Program pg = strip_program(j, n_max);
  run_eager(pg, t, st);
  return CHROM_OK;
}

}  // namespace
}  // namespace cs

// ===========================================================================
// C ABI
// ===========================================================================
using namespace cs;

extern "C" {

const char* chromatic_last_error(void) { return g_err.c_str(); }

const char* chromatic_version(void) { return "chromstrip 0.1 (gfx950)"; }

int chromatic_strip(int lattice, int m, int n_max, const uint32_t* q_points, int nq, const uint32_t* primes, int np,
                    uint32_t* out) {
  return guarded([&] { return strip_sync_impl(lattice, m, n_max, q_points, nq, primes, np, CHROM_MODE_PLAIN, nullptr, out); });
}

int chromatic_strip_batched(int lattice, int m, int n_max, const uint32_t* q_points, int nq, const uint32_t* primes,
                            int np, int mode, const chrom_tuning* tune, uint32_t* out) {
  return guarded([&] {
    check_mode(mode);
    if (mode == CHROM_MODE_PLAIN) throw ArgError("use chromatic_strip for the plain path");
    return strip_sync_impl(lattice, m, n_max, q_points, nq, primes, np, mode, tune, out);
  });
}

size_t chromatic_workspace_bytes(int lattice, int m, int n_max, int nq, int np, int mode, const chrom_tuning* tune) {
  size_t r = 0;
  int rc = guarded([&] {
    check_args(lattice, m, n_max);
    if (nq < 1 || np < 1) throw ArgError("need nq, np >= 1");
    check_mode(mode);
    Tune t = resolve(tune, false, mode == CHROM_MODE_RESIDENT);
    if (mode == CHROM_MODE_GROUPED) check_batch_stage(t);
    r = workspace_bytes(lattice, m, nq * np, n_max, mode, t);
    return CHROM_OK;
  });
  return rc == CHROM_OK ? r : 0;
}

int chromatic_strip_noalloc(int lattice, int m, int n_max, const uint32_t* q_points, int nq, const uint32_t* primes,
                            int np, const chrom_tuning* tune, void* stream, uint32_t* d_out) {
  return guarded([&] {
    return strip_noalloc_impl(lattice, m, n_max, q_points, nq, primes, np, tune, static_cast<hipStream_t>(stream),
                              d_out);
  });
}

int chromatic_strip_async(int lattice, int m, int n_max, const uint32_t* q_points, int nq, const uint32_t* primes,
                          int np, int mode, const chrom_tuning* tune, void* d_workspace, size_t ws_bytes, void* stream,
                          uint32_t* d_out) {
  return guarded([&] {
    return strip_async_impl(lattice, m, n_max, q_points, nq, primes, np, mode, tune, d_workspace, ws_bytes,
                            static_cast<hipStream_t>(stream), d_out);
  });
}

size_t chromatic_series_workspace_bytes(int lattice, int m, int n_max, int np, int d_max, int mode,
                                        const chrom_tuning* tune) {
  size_t r = 0;
  int rc = guarded([&] {
    check_args(lattice, m, n_max);
    if (np < 1) throw ArgError("need np >= 1");
    if (mode != CHROM_MODE_BATCHED && mode != CHROM_MODE_GRAPH)
      throw ArgError("the coefficient form runs in batched or graph mode");
    r = series_workspace_bytes(lattice, m, np, d_max, resolve_series(tune, d_max));
    return CHROM_OK;
  });
  return rc == CHROM_OK ? r : 0;
}

int chromatic_series_async(int lattice, int m, int n_max, int d_max, const uint32_t* primes, int np, int mode,
                           const chrom_tuning* tune, void* d_workspace, size_t ws_bytes, void* stream,
                           uint32_t* d_out) {
  return guarded([&] {
    return series_async_impl(lattice, m, n_max, d_max, primes, np, mode, tune, d_workspace, ws_bytes,
                             static_cast<hipStream_t>(stream), d_out);
  });
}

int chromatic_series(int lattice, int m, int n_max, int d_max, const uint32_t* primes, int np, int mode,
                     const chrom_tuning* tune, uint32_t* out) {
  return guarded([&] { return series_sync_impl(lattice, m, n_max, d_max, primes, np, mode, tune, out); });
}

int chromatic_factor_launches(int lattice, int m, const uint32_t* q_points, int nq, const uint32_t* primes, int np,
                              int rows, const chrom_tuning* tune, void* d_workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    return factor_launches_impl(lattice, m, q_points, nq, primes, np, rows, tune, d_workspace, ws_bytes,
                                static_cast<hipStream_t>(stream));
  });
}

int chromatic_prepare(int lattice, int m) {
  return guarded([&] {
    check_args(lattice, m, 0);
    (void)dev_family(dev_maps(lattice, m), 1);
    return CHROM_OK;
  });
}

int chromatic_prepare_series(int lattice, int m) {
  return guarded([&] {
    check_args(lattice, m, 0);
    const DevMaps& dm = dev_maps(lattice, m, true);
    (void)dev_family(dm, 1);
    return CHROM_OK;
  });
}

int chromatic_series_map_export(int lattice, int m, int which, int idx, int64_t* n_rows, int64_t* n_cols,
                                int64_t* nnz, int32_t* row_ptr, uint32_t* entries) {
  return guarded([&] {
    check_args(lattice, m, 0);
    if (which != 4 && which != 5) throw ArgError("which must be 4 (forward) or 5 (read-out)");
    if (idx < 0 || idx >= m) throw ArgError("idx out of range");
    const DevMaps& dm = dev_maps(lattice, m, true);
    const DevCsr& c = which == 4 ? dm.fwd[idx] : dm.last_fwd[idx];
    int32_t total = 0;
    HIPX(hipMemcpy(&total, c.row_ptr + c.n_rows, 4, hipMemcpyDeviceToHost));
    if (n_rows) *n_rows = c.n_rows;
    if (n_cols) *n_cols = c.n_cols;
    if (nnz) *nnz = total;
    if (row_ptr) HIPX(hipMemcpy(row_ptr, c.row_ptr, (static_cast<size_t>(c.n_rows) + 1) * 4, hipMemcpyDeviceToHost));
    if (entries && total > 0) HIPX(hipMemcpy(entries, c.ent, static_cast<size_t>(total) * 4, hipMemcpyDeviceToHost));
    return CHROM_OK;
  });
}

int chromatic_check_expansion(int lattice, int m, int normalised) {
  return guarded([&] {
    check_args(lattice, m, 0);
    if (normalised != 0 && normalised != 1) throw ArgError("normalised must be 0 or 1");
    const std::string diff = check_expansion(lattice, m, normalised == 1);
    if (!diff.empty()) throw std::runtime_error("expansion check: " + diff);
    return CHROM_OK;
  });
}

int chromatic_prepare_host(int lattice, int m, int normalised) {
  return guarded([&] {
    check_args(lattice, m, 0);
    if (normalised != 0 && normalised != 1) throw ArgError("normalised must be 0 or 1");
    (void)get_maps(lattice, m, normalised == 1);
    return CHROM_OK;
  });
}

void chromatic_release_maps(void) {
  (void)guarded([&] {
    {
      std::lock_guard<std::mutex> lk(g_graph_mu);
      for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second.exec);
      g_graphs.clear();
    }
    std::lock_guard<std::mutex> lk(g_dev_mu);
    for (auto& kv : g_dev) {
      int cur = 0;
      (void)hipGetDevice(&cur);
      (void)hipSetDevice(std::get<0>(kv.first));
      (void)hipDeviceSynchronize();
      for (auto& fam : kv.second->fam) {
        for (auto& st : fam.second->staged) (void)hipFree(st.second->base);
        if (fam.second->sell) (void)hipFree(fam.second->sell->base);
        if (fam.second->sell_one) (void)hipFree(fam.second->sell_one->base);
        if (fam.second->ops) (void)hipFree(fam.second->ops->base);
        if (fam.second->base) (void)hipFree(fam.second->base);
      }
      (void)hipFree(kv.second->base);
      for (void* a : kv.second->allocs) (void)hipFree(a);
      (void)hipSetDevice(cur);
    }
    g_dev.clear();
    release_host_maps();
    return CHROM_OK;
  });
}

size_t chromatic_batch_workspace_bytes(const chrom_job* jobs, int njobs, const chrom_tuning* tune) {
  size_t r = 0;
  int rc = guarded([&] {
    Tune t = resolve(tune);
    check_batch_stage(t);
    r = batch_plan(jobs, njobs, t).bytes;
    return CHROM_OK;
  });
  return rc == CHROM_OK ? r : 0;
}

int chromatic_batch(const chrom_job* jobs, int njobs, const chrom_tuning* tune, void* d_workspace, size_t ws_bytes,
                    void* stream) {
  return guarded([&] { return batch_impl(jobs, njobs, tune, d_workspace, ws_bytes, static_cast<hipStream_t>(stream)); });
}

size_t chromatic_slot_state_bytes(int lattice, int m, int nq, int np, const chrom_tuning* tune) {
  size_t r = 0;
  int rc = guarded([&] {
    check_args(lattice, m, 0);
    if (nq < 1 || np < 1) throw ArgError("need nq, np >= 1");
    Tune t = resolve(tune);
    r = job_layout(lattice, m, nq * np, t, kMaxCodes, rows_tile_of(t)).bytes;
    return CHROM_OK;
  });
  return rc == CHROM_OK ? r : 0;
}

int chromatic_server_step(chrom_slot* slots, int nslots, int rows, const chrom_tuning* tune, void* stream) {
  return guarded([&] { return server_step_impl(slots, nslots, rows, tune, static_cast<hipStream_t>(stream)); });
}

int chromatic_device_status(void* stream) {
  return guarded([&] {
    HIPX(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    HIPX(hipGetLastError());
    return CHROM_OK;
  });
}

int64_t chromatic_motzkin(int k) { return motzkin(k); }

int64_t chromatic_space_size(int m, int space, int i) {
  if (m < 1 || m > CHROM_MAX_M) return fail(CHROM_EINVAL, "m out of range");
  if (space == CHROM_SPACE_NCNNN) return Space{kNcnnn, m, 0}.size();
  if (space == CHROM_SPACE_SQ_INTER) {
    if (i < 1 || i >= m) return fail(CHROM_EINVAL, "i must be in 1..m-1");
    return Space{kSqInter, m, i}.size();
  }
  if (space == CHROM_SPACE_LAST) {
    if (i < 0 || i > m) return fail(CHROM_EINVAL, "i must be in 0..m");
    return i == 0 ? Space{kNcnnn, m, 0}.size() : Space{kLast, m, i}.size();
  }
  return fail(CHROM_EINVAL, "unknown space");
}

static bool space_of(int m, int space, int i, Space* sp) {
  if (m < 1 || m > CHROM_MAX_M) return false;
  if (space == CHROM_SPACE_NCNNN) {
    *sp = Space{kNcnnn, m, 0};
    return true;
  }
  if (space == CHROM_SPACE_SQ_INTER && i >= 1 && i < m) {
    *sp = Space{kSqInter, m, i};
    return true;
  }
  if (space == CHROM_SPACE_LAST && i >= 0 && i <= m) {
    *sp = i == 0 ? Space{kNcnnn, m, 0} : Space{kLast, m, i};
    return true;
  }
  return false;
}

int64_t chromatic_rank(int m, int space, int i, const uint8_t* lab) {
  Space sp;
  if (!lab || !space_of(m, space, i, &sp)) return fail(CHROM_EINVAL, "bad space or labels") - 1;
  Part p;
  std::memcpy(p.lab, lab, m);
  canonicalize(p, m);
  if (!is_noncrossing(p, m)) return -1;
  return sp.rank(p);
}

int chromatic_unrank(int m, int space, int i, int64_t r, uint8_t* lab) {
  Space sp;
  if (!lab || !space_of(m, space, i, &sp)) return fail(CHROM_EINVAL, "bad space or labels");
  if (r < 0 || r >= sp.size()) return fail(CHROM_EINVAL, "rank out of range");
  Part p;
  sp.unrank(r, p);
  std::memcpy(lab, p.lab, m);
  return CHROM_OK;
}

int chromatic_maps_info(int lattice, int m, chrom_maps_info* info) {
  return guarded([&] {
    check_args(lattice, m, 0);
    if (!info) throw ArgError("null info");
    const MapSet& ms = get_maps(lattice, m);
    info->n_factors = m;
    info->n_last = m;
    info->n_codes = static_cast<int>(ms.codes.size());
    info->total_nnz = ms.total_nnz();
    info->max_states = ms.max_states();
    return CHROM_OK;
  });
}

int chromatic_family_info(int lattice, int m, int fuse, int* n_factors, int* n_codes, int64_t* coef) {
  return guarded([&] {
    check_args(lattice, m, 0);
    if (fuse < 1 || fuse > kMaxFuse) throw ArgError("fuse must be in 1..3");
    const MapSet& ms = get_maps(lattice, m);
    const std::vector<Poly>& codes = fuse == 1 ? ms.codes : ms.family(fuse).codes;
    if (n_factors) *n_factors = fuse == 1 ? m : static_cast<int>(ms.family(fuse).fac.size());
    if (n_codes) *n_codes = static_cast<int>(codes.size());
    if (coef)
      for (size_t c = 0; c < codes.size(); ++c)
        for (int k = 0; k <= kMaxDeg; ++k) coef[c * (kMaxDeg + 1) + k] = codes[c].c[k];
    return CHROM_OK;
  });
}

int chromatic_map_export(int lattice, int m, int which, int idx, int64_t* n_rows, int64_t* n_cols, int64_t* nnz,
                         int32_t* row_ptr, uint32_t* entries) {
  return guarded([&] {
    check_args(lattice, m, 0);
    if (which < 0 || which > 5) throw ArgError("which must be in 0..5");
    const MapSet& ms = get_maps(lattice, m, which >= 4);
    const Csr* c = nullptr;
    if (which <= 1 || which >= 4) {
      if (idx < 0 || idx >= m) throw ArgError("idx out of range");
      c = (which == 0 || which == 4) ? &ms.fwd[idx] : (which == 1 ? &ms.last[idx] : &ms.last_fwd[idx]);
    } else {
      const Family& f = ms.family(which);
      if (idx < 0 || idx >= static_cast<int>(f.fac.size())) throw ArgError("idx out of range");
      c = &f.fac[idx];
    }
    if (n_rows) *n_rows = c->n_rows;
    if (n_cols) *n_cols = c->n_cols;
    if (nnz) *nnz = c->nnz();
    if (row_ptr) std::memcpy(row_ptr, c->row_ptr.data(), c->row_ptr.size() * 4);
    if (entries && !c->ent.empty()) std::memcpy(entries, c->ent.data(), c->ent.size() * 4);
    return CHROM_OK;
  });
}

int chromatic_code_table(int lattice, int m, int normalised, int* n_codes, int64_t* coef) {
  return guarded([&] {
    check_args(lattice, m, 0);
    const MapSet& ms = get_maps(lattice, m, normalised != 0);
    if (n_codes) *n_codes = static_cast<int>(ms.codes.size());
    if (coef)
      for (size_t c = 0; c < ms.codes.size(); ++c)
        for (int k = 0; k <= kMaxDeg; ++k) coef[c * (kMaxDeg + 1) + k] = ms.codes[c].c[k];
    return CHROM_OK;
  });
}

int chromatic_stage_export(int lattice, int m, int fuse, int idx, int slots, int rows, int32_t* n_tiles,
                           int64_t* n_src, int32_t* max_slots, int32_t* tile_row0, int32_t* tile_src0,
                           int32_t* src, uint32_t* entries) {
  return guarded([&] {
    check_args(lattice, m, 0);
    if (fuse < 1 || fuse > kMaxFuse) throw ArgError("fuse must be in 1..3");
    if (slots < 1 || rows < 1) throw ArgError("slots and rows must be >= 1");
    const MapSet& ms = get_maps(lattice, m);
    const std::vector<Csr>& fac = (fuse == 1) ? ms.fwd : ms.family(fuse).fac;
    if (idx < 0 || idx >= static_cast<int>(fac.size())) throw ArgError("idx out of range");
    const StagedCsr st = build_staged(fac[idx], slots, rows);
    if (n_tiles) *n_tiles = st.n_tiles();
    if (n_src) *n_src = static_cast<int64_t>(st.src.size());
    if (max_slots) *max_slots = st.max_slots;
    if (tile_row0) std::memcpy(tile_row0, st.tile_row0.data(), st.tile_row0.size() * 4);
    if (tile_src0) std::memcpy(tile_src0, st.tile_src0.data(), st.tile_src0.size() * 4);
    if (src && !st.src.empty()) std::memcpy(src, st.src.data(), st.src.size() * 4);
    if (entries && !st.ent.empty()) std::memcpy(entries, st.ent.data(), st.ent.size() * 4);
    return CHROM_OK;
  });
}

int chromatic_op_export(int lattice, int m, int fuse, int idx, int32_t* shift, int64_t* n_words,
                        int32_t* row_first, uint32_t* words) {
  return guarded([&] {
    check_args(lattice, m, 0);
    if (fuse < 1 || fuse > kMaxFuse) throw ArgError("fuse must be in 1..3");
    const MapSet& ms = get_maps(lattice, m);
    const std::vector<Csr>& fac = (fuse == 1) ? ms.fwd : ms.family(fuse).fac;
    const std::vector<Poly>& codes = (fuse == 1) ? ms.codes : ms.family(fuse).codes;
    if (idx < 0 || idx >= static_cast<int>(fac.size())) throw ArgError("idx out of range");
    bool general = false;
    const int s = choose_shift(codes, fac, general);
    std::vector<uint32_t> w;
    std::vector<int32_t> rp;
    build_op_stream(fac[idx], codes, s, w, rp);
    if (shift) *shift = s;
    if (n_words) *n_words = static_cast<int64_t>(w.size());
    if (row_first) std::memcpy(row_first, rp.data(), rp.size() * 4);
    if (words) std::memcpy(words, w.data(), w.size() * 4);
    return CHROM_OK;
  });
}

int chromatic_cluster_export(int lattice, int m, int fuse, int idx, int slots, int rows, int32_t* n_tiles,
                             int64_t* n_src, int32_t* max_slots, int32_t* tile_row0, int32_t* tile_src0,
                             int32_t* src, int32_t* tgt, int32_t* row_ptr, uint32_t* entries) {
  return guarded([&] {
    check_args(lattice, m, 0);
    if (fuse < 1 || fuse > kMaxFuse) throw ArgError("fuse must be in 1..3");
    if (slots < 1 || rows < 1) throw ArgError("slots and rows must be >= 1");
    const MapSet& ms = get_maps(lattice, m);
    const std::vector<Csr>& fac = (fuse == 1) ? ms.fwd : ms.family(fuse).fac;
    if (idx < 0 || idx >= static_cast<int>(fac.size())) throw ArgError("idx out of range");
    const StagedCsr st = build_clustered(fac[idx], slots, rows);
    if (n_tiles) *n_tiles = st.n_tiles();
    if (n_src) *n_src = static_cast<int64_t>(st.src.size());
    if (max_slots) *max_slots = st.max_slots;
    if (tile_row0) std::memcpy(tile_row0, st.tile_row0.data(), st.tile_row0.size() * 4);
    if (tile_src0) std::memcpy(tile_src0, st.tile_src0.data(), st.tile_src0.size() * 4);
    if (src && !st.src.empty()) std::memcpy(src, st.src.data(), st.src.size() * 4);
    if (tgt && !st.tgt.empty()) std::memcpy(tgt, st.tgt.data(), st.tgt.size() * 4);
    if (row_ptr) std::memcpy(row_ptr, st.row_ptr.data(), st.row_ptr.size() * 4);
    if (entries && !st.ent.empty()) std::memcpy(entries, st.ent.data(), st.ent.size() * 4);
    return CHROM_OK;
  });
}

}  // extern "C"
