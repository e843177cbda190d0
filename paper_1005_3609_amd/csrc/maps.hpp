// Factor maps: each per-site factor of the sparse transfer matrix as a
// sparse integer matrix over ranked states, and products of consecutive
// factors ("fused" families) for kernels that skip writing the states in
// between.
#pragma once

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "states.hpp"

namespace cs {

enum Lattice { kSquare = 0, kTriangular = 1 };

constexpr int kMaxCodes = 64;
constexpr uint32_t kSrcBits = 26;
constexpr uint32_t kSrcMask = (1u << kSrcBits) - 1;
constexpr int kMaxDeg = 3;  // coefficient polynomials in q up to q^3 (three fused factors)
constexpr int kMaxFuse = 3;

// Compressed sparse rows.  Entry word: column state rank in the low 26 bits,
// coefficient code in the high 6 bits.
struct Csr {
  int64_t n_rows = 0, n_cols = 0;
  std::vector<int32_t> row_ptr;   // n_rows + 1
  std::vector<uint32_t> ent;      // nnz
  int64_t nnz() const { return static_cast<int64_t>(ent.size()); }
};

// Coefficient polynomial c[0] + c[1] q + c[2] q^2 + c[3] q^3.
struct Poly {
  int64_t c[kMaxDeg + 1] = {0, 0, 0, 0};
  bool operator<(const Poly& o) const {
    for (int k = kMaxDeg; k >= 0; --k)
      if (c[k] != o.c[k]) return c[k] < o.c[k];
    return false;
  }
  bool operator==(const Poly& o) const {
    for (int k = 0; k <= kMaxDeg; ++k)
      if (c[k] != o.c[k]) return false;
    return true;
  }
  bool zero() const { return c[0] == 0 && c[1] == 0 && c[2] == 0 && c[3] == 0; }
};

// Products T_hi ... T_lo of consecutive forward factors, covering 1..m.
// Family k = 1 is the single factors themselves.
struct Family {
  int k = 1;
  std::vector<Csr> fac;           // rows: states after T_hi; columns: states before T_lo
  std::vector<int> lo, hi;        // 1-based site ranges
  std::vector<Poly> codes;        // extends the base table (same numbers for shared codes)
};

// Numbering of the spaces between the forward factors of a row (internal to
// the maps; the NCNNN space before the first and after the last factor keeps
// the paper's order): the paper's order, the reader order (each space by the
// first row of the next factor that reads it) or the site order (each space
// by its states' labels read from the point after the last one the factor
// writing it touches, round to that point).
enum StateOrder { kOrderPaper = 0, kOrderReader = 1, kOrderSite = 2 };

struct MapSet {
  int lattice = 0, m = 0;
  int order = kOrderReader;
  // Coefficients in z = q (false) or in z = x = 1/q, the normalised weights
  // of eq. Z_modified (true).
  bool normalised = false;
  // fwd[i-1]: factor T_i, rows = states after it, columns = states before it
  // (gather form: out[row] = sum over entries coef * in[col]).
  std::vector<Csr> fwd;
  // last[i-1]: (T_i^last)^T, rows = states before T_i^last (space L_{i-1}),
  // columns = states after it (L_i).  Applied for i = m..1 to e_0 it gives
  // the read-out vector w = T_last^T e_0 over the NCNNN states.
  std::vector<Csr> last;
  // Normalised sets only: last_fwd[i-1] = T_i^last in gather form (rows =
  // states after it, L_i; columns = states before it, L_{i-1}), for a
  // read-out that applies T_last to the state of every row.
  std::vector<Csr> last_fwd;
  std::vector<Poly> codes;        // base table: codes of fwd, last and last_fwd
  int64_t total_nnz() const;
  int64_t max_states() const;
  size_t host_bytes() const;
  // Fused families, built on first request (thread safe).
  const Family& family(int k) const;

 private:
  mutable std::mutex fam_mu_;
  mutable std::map<int, std::unique_ptr<Family>> fam_;
};

// A factor cut into tiles of consecutive target rows for kernels that stage
// each tile's source rows in on-chip memory: tile t covers rows
// [tile_row0[t], tile_row0[t+1]) and reads the distinct source states
// src[tile_src0[t] .. tile_src0[t+1]) (ascending); the entries keep their
// codes, with the source replaced by its position (slot) in that list.
struct StagedCsr {
  std::vector<int32_t> tile_row0, tile_src0, src;
  std::vector<uint32_t> ent;      // code << kSrcBits | slot, in the order of row_ptr
  int max_slots = 0;              // largest source list of a tile
  // Clustered tiles only: the tiles' target rows in tile order (tile t holds
  // positions tile_row0[t] .. tile_row0[t+1]-1, position k writing row
  // tgt[k]) and the row pointers of that order.  Empty: tile t holds the
  // consecutive rows tile_row0[t] .. and the map's own row pointers apply.
  std::vector<int32_t> tgt, row_ptr;
  std::vector<uint32_t> ent_src;   // clustered: the entry words with their sources, in tile order
  // first entry of each tile (n_tiles + 1), the largest tile's rows and entries
  std::vector<int32_t> tile_ent0;
  int max_rows = 0, max_ent = 0;
  int n_tiles() const { return static_cast<int>(tile_row0.size()) - 1; }
};

// Greedy tiling: a tile grows row by row while it has at most `rows` rows and
// `slots` distinct sources (a single row with more sources forms a tile of
// its own).
StagedCsr build_staged(const Csr& c, int slots, int rows);

// Clustered tiling: a tile grows from the lowest unplaced target through the
// sources it reads -- every unplaced reader of a source already in the tile
// joins while the tile keeps at most `rows` targets and `slots` distinct
// sources (and at most `max_ent` entries) -- and when that search closes,
// the next unplaced target seeds it again if it fits.  Targets that read the same sources share a tile, so a
// tile stages fewer source rows per target than a run of consecutive rows
// (square m = 14 fused pairs: about 1.5 against 2.8 per target at 64 targets
// and 96 slots).
StagedCsr build_clustered(const Csr& c, int slots, int rows, int max_ent = 1 << 30);

// Interleaved order for direct gathers: within every whole tile of
// `rows_tile` = waves x rows-per-wavefront consecutive target rows, the k-th
// row of wavefront w is tile row k * waves + w, so at each step of their row
// loops the tile's wavefronts work on adjacent rows (which share sources);
// a last partial tile keeps its order.  With `order`, the rows are first
// taken in that sequence (order[k] = the k-th row).  Fills tgt, row_ptr and
// ent_src (tile_row0 = {0}, no slots).
StagedCsr build_interleaved(const Csr& c, int rows_tile, int waves, const std::vector<int32_t>* order = nullptr);

// The NCNNN states of m points sorted by their canonical labelling read in
// the natural point order (rank in the paper's order at each position).
std::vector<int32_t> ncnnn_natural_order(int m);

// Builds every single-factor map of (lattice, m); threads = 0 uses the
// hardware count; paper_order keeps the paper's state order between the
// forward factors.  Otherwise the evaluation form takes the site order and
// the normalised form the reader order (the order the device-side builder of
// the normalised maps reproduces); CHROMSTRIP_STATE_ORDER = paper, reader or
// site overrides either.  Fused families keep the numbering of the single
// factors' spaces (site order) or take their own reader order.  Throws
// std::runtime_error on failure.
std::unique_ptr<MapSet> build_maps(int lattice, int m, int threads = 0, bool normalised = false,
                                   bool paper_order = false);

// Host-side map cache (thread safe): built on first request, one map set at
// a time (a global build lock; each build is itself threaded).
// release_host_maps invalidates every reference handed out and must not run
// concurrently with other calls.
const MapSet& get_maps(int lattice, int m, bool normalised = false);
void release_host_maps();

}  // namespace cs
