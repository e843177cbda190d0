// Factor maps: each per-site factor of the sparse transfer matrix as a
// sparse integer matrix over ranked states.
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

#include "states.hpp"

namespace cs {

enum Lattice { kSquare = 0, kTriangular = 1 };

constexpr int kMaxCodes = 16;
constexpr uint32_t kSrcBits = 28;
constexpr uint32_t kSrcMask = (1u << kSrcBits) - 1;

// Compressed sparse rows.  Entry word: column state rank in the low 28 bits,
// coefficient code in the high 4 bits.
struct Csr {
  int64_t n_rows = 0, n_cols = 0;
  std::vector<int32_t> row_ptr;   // n_rows + 1
  std::vector<uint32_t> ent;      // nnz
  int64_t nnz() const { return static_cast<int64_t>(ent.size()); }
};

struct MapSet {
  int lattice = 0, m = 0;
  // fwd[i-1]: factor T_i, rows = states after it, columns = states before it
  // (gather form: out[row] = sum over entries coef * in[col]).
  std::vector<Csr> fwd;
  // last[i-1]: (T_i^last)^T, rows = states before T_i^last (space L_{i-1}),
  // columns = states after it (L_i).  Applied for i = m..1 to e_0 it gives
  // the read-out vector w = T_last^T e_0 over the NCNNN states.
  std::vector<Csr> last;
  int n_codes = 0;
  int code_a[kMaxCodes] = {0}, code_b[kMaxCodes] = {0};  // code k: a + b q
  int64_t total_nnz() const;
  int64_t max_states() const;
  size_t host_bytes() const;
};

// Builds every map of (lattice, m); threads = 0 uses the hardware count.
// Throws std::runtime_error on failure.
std::unique_ptr<MapSet> build_maps(int lattice, int m, int threads = 0);

// Host-side map cache (thread safe): built on first request.
const MapSet& get_maps(int lattice, int m);
void release_host_maps();

}  // namespace cs
