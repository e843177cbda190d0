// Factor-map builder.
//
// Every per-site factor of arXiv 1005.3609 is expanded on each source state
// with the single-edge operators of Sec. 3.1 at v = -1, either in
// un-normalised form with coefficients in q (a component pays q when it
// leaves the layer):
//   H_{a,b} s = s - J_{a,b} s          (0 if a, b already share a block)
//   V_i s     = -s + D_i s             ((q-1) s if i is alone in s)
//   D_i s     = i made a singleton     (q s if i is alone in s)
// or in the normalised form of eq. Z_modified with coefficients in x = 1/q
// (a join pays x, nothing pays on leaving):
//   H_{a,b} s = s - x J_{a,b} s,  V_i s = -x s + D_i s,  D_i s as above without q
//   P         = drop states whose listed neighbour pairs share a block
// Factors (1-based site i, Sec. 3.2 - 3.3):
//   square      T_i = P_{j != i} V_i H_{i,i+1} (i < m),  T_m = P_all V_m
//   triangular  T_i = P_all V_i H_{i-1,i} H_{i,i+1}  (H's omitted at the ends)
//   read-out    T_i^last = P_{j > i} D_i H_{i,i+1}   (H omitted for i = m)
// Every coefficient is a small-integer polynomial (degree <= 1 in q for a
// single un-normalised factor, <= 3 in x for a normalised one); it is stored
// as a code into a per-map-set table.  Products of consecutive factors (fused
// families) carry polynomial coefficients of degree up to the number of
// factors multiplied.
#include "maps.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <tuple>

namespace cs {

namespace {

// Coefficient key of a polynomial c0 + c1 z + c2 z^2 + c3 z^3 (z = q in the
// un-normalised form, z = x = 1/q in the normalised one), each c_k in
// [-8, 8].
constexpr int kKeyOff = 8, kKeyBase = 17, kKeys = kKeyBase * kKeyBase * kKeyBase * kKeyBase;
inline int coef_key(const int (&c)[kMaxDeg + 1]) {
  int key = 0;
  for (int k = kMaxDeg; k >= 0; --k) {
    if (c[k] < -kKeyOff || c[k] > kKeyOff) throw std::runtime_error("coefficient out of the supported range");
    key = key * kKeyBase + (c[k] + kKeyOff);
  }
  return key;
}
inline Poly key_poly(int key) {
  Poly p;
  for (int k = 0; k <= kMaxDeg; ++k) {
    p.c[k] = key % kKeyBase - kKeyOff;
    key /= kKeyBase;
  }
  return p;
}

struct Term {
  Part p;
  int c[kMaxDeg + 1];  // coefficient polynomial
};

inline bool coef_zero(const Term& t) { return t.c[0] == 0 && t.c[1] == 0 && t.c[2] == 0 && t.c[3] == 0; }

// c -> sign * z * c
inline void times_z(Term& t, int sign) {
  if (t.c[kMaxDeg] != 0) throw std::runtime_error("coefficient degree above 3");
  for (int k = kMaxDeg; k > 0; --k) t.c[k] = sign * t.c[k - 1];
  t.c[0] = 0;
}

// Applies single-edge operators to a short list of terms.  Un-normalised
// (z = q): H = 1 - J, V = -1 + D, D pays q when its point is alone.
// Normalised (z = x = 1/q, eq. Z_modified): J pays x, so H = 1 - x J,
// V = -x + D, and D never pays.
class Expander {
 public:
  Expander(int m, bool normalised) : m_(m), norm_(normalised) {}
  void reset(const Part& p) {
    terms_.clear();
    Term t;
    t.p = p;
    t.c[0] = 1;
    t.c[1] = t.c[2] = t.c[3] = 0;
    terms_.push_back(t);
  }
  // H_{x,y} = 1 - J_{x,y}  (J pays x in the normalised form)
  void H(int x, int y) {
    tmp_.clear();
    for (const Term& t : terms_) {
      if (same_block(t.p, x, y)) continue;
      tmp_.push_back(t);
      Term j = t;
      join(j.p, m_, x, y);
      if (norm_) {
        times_z(j, -1);
      } else {
        for (int k = 0; k <= kMaxDeg; ++k) j.c[k] = -t.c[k];
      }
      tmp_.push_back(j);
    }
    terms_.swap(tmp_);
  }
  // V_i = -1 + D_i (un-normalised) or -x + D_i (normalised)
  void V(int i) {
    tmp_.clear();
    for (const Term& t : terms_) {
      Term present = t;
      if (norm_) {
        times_z(present, -1);
      } else {
        for (int k = 0; k <= kMaxDeg; ++k) present.c[k] = -t.c[k];
      }
      tmp_.push_back(present);
      Term d = t;
      if (is_alone(t.p, m_, i)) {
        if (!norm_) times_z(d, 1);  // the component leaves the layer: q
      } else {
        detach(d.p, m_, i);
      }
      tmp_.push_back(d);
    }
    terms_.swap(tmp_);
  }
  // D_i
  void D(int i) {
    for (Term& t : terms_) {
      if (is_alone(t.p, m_, i)) {
        if (!norm_) times_z(t, 1);
      } else {
        detach(t.p, m_, i);
      }
    }
  }
  // Projectors P_{x,x+1} for every x with bit x set in `forbid`.
  void P(uint32_t forbid) {
    tmp_.clear();
    for (const Term& t : terms_) {
      bool ok = true;
      for (int x = 0; x + 1 < m_; ++x)
        if (((forbid >> x) & 1u) && t.p.lab[x] == t.p.lab[x + 1]) {
          ok = false;
          break;
        }
      if (ok) tmp_.push_back(t);
    }
    terms_.swap(tmp_);
  }
  // Combines equal states and drops zero coefficients.
  void merge() {
    tmp_.clear();
    for (const Term& t : terms_) {
      bool found = false;
      for (Term& u : tmp_)
        if (std::memcmp(u.p.lab, t.p.lab, m_) == 0) {
          for (int k = 0; k <= kMaxDeg; ++k) u.c[k] += t.c[k];
          found = true;
          break;
        }
      if (!found) tmp_.push_back(t);
    }
    terms_.clear();
    for (const Term& t : tmp_)
      if (!coef_zero(t)) terms_.push_back(t);
  }
  const std::vector<Term>& terms() const { return terms_; }

 private:
  int m_;
  bool norm_;
  std::vector<Term> terms_, tmp_;
};

uint32_t all_pairs(int m) { return m >= 2 ? ((1u << (m - 1)) - 1u) : 0u; }

// One factor's definition: spaces and the operator sequence.
struct FactorDef {
  Space in, out;
  int lattice, m, site;  // site: 1-based i
  bool last;

  void expand(Expander& e) const {
    const int s = site - 1;  // 0-based point of site i
    if (last) {
      if (site < m) e.H(s, s + 1);
      e.D(s);
      uint32_t forbid = 0;
      for (int x = s + 1; x + 1 < m; ++x) forbid |= 1u << x;
      e.P(forbid);
    } else if (lattice == kSquare) {
      if (site < m) e.H(s, s + 1);
      e.V(s);
      uint32_t forbid = all_pairs(m);
      if (site < m) forbid &= ~(1u << s);
      e.P(forbid);
    } else {
      if (site < m) e.H(s, s + 1);
      if (site > 1) e.H(s - 1, s);
      e.V(s);
      e.P(all_pairs(m));
    }
    e.merge();
  }
};

FactorDef forward_def(int lattice, int m, int i) {
  FactorDef d;
  d.lattice = lattice;
  d.m = m;
  d.site = i;
  d.last = false;
  if (lattice == kSquare) {
    d.in = (i == 1) ? Space{kNcnnn, m, 0} : Space{kSqInter, m, i - 1};
    d.out = (i == m) ? Space{kNcnnn, m, 0} : Space{kSqInter, m, i};
  } else {
    d.in = Space{kNcnnn, m, 0};
    d.out = Space{kNcnnn, m, 0};
  }
  return d;
}

FactorDef last_def(int lattice, int m, int i) {
  FactorDef d;
  d.lattice = lattice;
  d.m = m;
  d.site = i;
  d.last = true;
  d.in = (i == 1) ? Space{kNcnnn, m, 0} : Space{kLast, m, i - 1};
  d.out = Space{kLast, m, i};
  return d;
}

// Runs f(thread, lo, hi) over contiguous ascending ranges; the first
// exception thrown by any worker is rethrown here.
template <class F>
void parallel_for(int64_t n, int threads, F&& f) {
  if (threads <= 1 || n < 4096) {
    f(0, int64_t(0), n);
    return;
  }
  std::vector<std::thread> pool;
  std::exception_ptr err;
  std::mutex err_mu;
  int64_t chunk = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    pool.emplace_back([&, t, lo, hi] {
      try {
        f(t, lo, hi);
      } catch (...) {
        std::lock_guard<std::mutex> lk(err_mu);
        if (!err) err = std::current_exception();
      }
    });
  }
  for (auto& th : pool) th.join();
  if (err) std::rethrow_exception(err);
}

// Host threads for map builds: CHROMSTRIP_THREADS if set (> 0), else the
// hardware's count.  Results do not depend on it.
int build_threads() {
  const char* v = std::getenv("CHROMSTRIP_THREADS");
  if (v) {
    const int n = std::atoi(v);
    if (n > 0) return n;
  }
  return static_cast<int>(std::max(1u, std::thread::hardware_concurrency()));
}

struct Triple {
  int32_t row, col;
  int32_t key;
};

// Runs f(i) for i = 0..n-1, one thread each (n small: one per buffer).
template <class F>
void each_thread(int n, F&& f) {
  if (n <= 1) {
    if (n == 1) f(0);
    return;
  }
  std::vector<std::thread> pool;
  std::exception_ptr err;
  std::mutex err_mu;
  for (int i = 0; i < n; ++i)
    pool.emplace_back([&, i] {
      try {
        f(i);
      } catch (...) {
        std::lock_guard<std::mutex> lk(err_mu);
        if (!err) err = std::current_exception();
      }
    });
  for (auto& th : pool) th.join();
  if (err) std::rethrow_exception(err);
}

// Exclusive prefix sum of counts into row pointers (n + 1 entries).
void row_pointers(const std::vector<int32_t>& cnt, std::vector<int32_t>& row_ptr) {
  const int64_t n = static_cast<int64_t>(cnt.size());
  row_ptr.assign(n + 1, 0);
  int64_t acc = 0;
  for (int64_t r = 0; r < n; ++r) {
    acc += cnt[r];
    if (acc > INT32_MAX) throw std::runtime_error("too many map entries for 32-bit row pointers");
    row_ptr[r + 1] = static_cast<int32_t>(acc);
  }
}

// Sorts the entries of rows [lo, hi) by column, then by the parallel `keys`
// value (rows hold a handful of entries: insertion sort), so that the CSR
// does not depend on the order its entries were scattered in.
void sort_rows(const std::vector<int32_t>& row_ptr, std::vector<uint32_t>& ent, int32_t* keys, int64_t lo,
               int64_t hi) {
  for (int64_t r = lo; r < hi; ++r) {
    const int64_t a0 = row_ptr[r], a1 = row_ptr[r + 1];
    for (int64_t a = a0 + 1; a < a1; ++a)
      for (int64_t b = a; b > a0; --b) {
        const uint32_t cp = ent[b - 1] & kSrcMask, cb = ent[b] & kSrcMask;
        const bool swap = cp > cb || (cp == cb && (keys ? keys[b - 1] > keys[b] : ent[b - 1] > ent[b]));
        if (!swap) break;
        std::swap(ent[b - 1], ent[b]);
        if (keys) std::swap(keys[b - 1], keys[b]);
      }
  }
}

// Builds one factor with coefficient keys in place of codes (resolved later).
void build_factor(const FactorDef& d, bool gather_form, bool normalised, int threads, Csr& csr,
                  std::vector<int32_t>& keys, std::atomic<uint64_t>* seen) {
  const int64_t nin = d.in.size(), nout = d.out.size();
  if (nin > int64_t(kSrcMask) || nout > int64_t(kSrcMask))
    throw std::runtime_error("state space too large for 26-bit ranks");
  std::vector<std::vector<Triple>> buf(std::max(threads, 1));
  parallel_for(nin, threads, [&](int t, int64_t lo, int64_t hi) {
    Expander e(d.m, normalised);
    auto& out = buf[t];
    out.reserve(static_cast<size_t>((hi - lo) * 4));
    std::vector<uint64_t> local_seen((kKeys + 63) / 64, 0);
    for (int64_t r = lo; r < hi; ++r) {
      Part p;
      d.in.unrank(r, p);
      e.reset(p);
      d.expand(e);
      for (const Term& term : e.terms()) {
        int64_t tr = d.out.rank(term.p);
        if (tr < 0) throw std::runtime_error("target outside its space: " + to_string(term.p, d.m));
        const int key = coef_key(term.c);
        local_seen[key / 64] |= 1ull << (key % 64);
        if (gather_form)
          out.push_back({static_cast<int32_t>(tr), static_cast<int32_t>(r), key});
        else
          out.push_back({static_cast<int32_t>(r), static_cast<int32_t>(tr), key});
      }
    }
    for (int w = 0; w < (kKeys + 63) / 64; ++w)
      if (local_seen[w]) seen[w].fetch_or(local_seen[w]);
  });
  const int64_t nrows = gather_form ? nout : nin;
  csr.n_rows = nrows;
  csr.n_cols = gather_form ? nin : nout;
  // Parallel assembly: row counts by atomic increments, row pointers, then
  // every buffer scatters its triples through atomic row cursors; the rows
  // are sorted afterwards, so the result is the same for any schedule.
  int64_t nnz = 0;
  for (auto& b : buf) nnz += static_cast<int64_t>(b.size());
  if (nnz > INT32_MAX) throw std::runtime_error("too many map entries for 32-bit row pointers");
  const int nb = static_cast<int>(buf.size());
  std::vector<int32_t> cnt(nrows, 0);
  each_thread(nb, [&](int t) {
    for (const Triple& x : buf[t]) __atomic_fetch_add(&cnt[x.row], 1, __ATOMIC_RELAXED);
  });
  row_pointers(cnt, csr.row_ptr);
  csr.ent.assign(nnz, 0);
  keys.assign(nnz, 0);
  std::vector<int32_t>& cur = cnt;  // reused as row cursors
  for (int64_t r = 0; r < nrows; ++r) cur[r] = csr.row_ptr[r];
  each_thread(nb, [&](int t) {
    for (const Triple& x : buf[t]) {
      const int32_t at = __atomic_fetch_add(&cur[x.row], 1, __ATOMIC_RELAXED);
      csr.ent[at] = static_cast<uint32_t>(x.col);
      keys[at] = x.key;
    }
    std::vector<Triple>().swap(buf[t]);
  });
  parallel_for(nrows, threads,
               [&](int, int64_t lo, int64_t hi) { sort_rows(csr.row_ptr, csr.ent, keys.data(), lo, hi); });
}

// Renumbers the rows of `c` by new_row[old] and its columns by new_col[old]
// (either may be empty = identity); entries of a row end up sorted by column.
void renumber(Csr& c, const std::vector<int32_t>& new_row, const std::vector<int32_t>& new_col, int threads) {
  const int64_t nr = c.n_rows;
  std::vector<int32_t> old_of(nr);
  for (int64_t r = 0; r < nr; ++r) old_of[new_row.empty() ? r : new_row[r]] = static_cast<int32_t>(r);
  Csr out;
  out.n_rows = c.n_rows;
  out.n_cols = c.n_cols;
  std::vector<int32_t> len(nr);
  for (int64_t r = 0; r < nr; ++r) len[r] = c.row_ptr[old_of[r] + 1] - c.row_ptr[old_of[r]];
  row_pointers(len, out.row_ptr);
  out.ent.resize(c.ent.size());
  parallel_for(nr, threads, [&](int, int64_t lo, int64_t hi) {
    for (int64_t r = lo; r < hi; ++r) {
      const int32_t o = old_of[r];
      int64_t w = out.row_ptr[r];
      for (int64_t e = c.row_ptr[o]; e < c.row_ptr[o + 1]; ++e) {
        const uint32_t col = c.ent[e] & kSrcMask, code = c.ent[e] >> kSrcBits;
        const uint32_t nc = new_col.empty() ? col : static_cast<uint32_t>(new_col[col]);
        out.ent[w++] = nc | (code << kSrcBits);
      }
    }
    sort_rows(out.row_ptr, out.ent, nullptr, lo, hi);
  });
  c = std::move(out);
}

// Reader order for the spaces between consecutive factors F_1..F_n of one
// transfer row.  The NCNNN space before F_1 and after F_n (the read-out
// vector's space) keeps the paper's order.  Going backwards, the space
// between F_k and F_{k+1} is ordered by the first target row of F_{k+1} --
// in its own output order, already fixed -- that reads it (ties by old rank;
// unread states last).  The rows of F_{k+1} are then visited in an order
// that touches most sources for the first time in increasing address order,
// and re-reads of a source follow its first read closely, so they are served
// by the L2.  The numbering is internal to the maps: every factor is
// renumbered consistently.
void reader_order(std::vector<Csr>& facs, int threads) {
  const int n = static_cast<int>(facs.size());
  if (n < 2) return;
  std::vector<std::vector<int32_t>> perm(n + 1);  // perm[k][old] = new, space after F_k
  for (int k = n - 1; k >= 1; --k) {
    const Csr& t = facs[k];  // F_{k+1}: rows in space k+1, columns in space k
    const int64_t ns = t.n_cols, nrows = t.n_rows;
    // first[s]: the lowest (new) row of F_{k+1} reading s; nrows if none
    std::vector<int32_t> first(ns, static_cast<int32_t>(nrows));
    parallel_for(nrows, threads, [&](int, int64_t lo, int64_t hi) {
      for (int64_t r = lo; r < hi; ++r) {
        const int32_t nr = perm[k + 1].empty() ? static_cast<int32_t>(r) : perm[k + 1][r];
        for (int64_t e = t.row_ptr[r]; e < t.row_ptr[r + 1]; ++e) {
          int32_t* f = &first[t.ent[e] & kSrcMask];
          int32_t seen = __atomic_load_n(f, __ATOMIC_RELAXED);
          while (nr < seen && !__atomic_compare_exchange_n(f, &seen, nr, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
          }
        }
      }
    });
    // stable counting sort of the states by first reader (ties by old rank)
    std::vector<int32_t> start(nrows + 2, 0);
    for (int64_t s = 0; s < ns; ++s) ++start[first[s] + 1];
    for (int64_t b = 0; b <= nrows; ++b) start[b + 1] += start[b];
    perm[k].assign(ns, 0);
    for (int64_t s = 0; s < ns; ++s) perm[k][s] = start[first[s]]++;
  }
  for (int k = 0; k < n; ++k) renumber(facs[k], perm[k + 1], perm[k], threads);
}

// Site order for the spaces between the forward factors T_1..T_n of one row.
// T_k (1-based site k) touches points up to k (0-based: the pair (k-1, k)
// and the vertical edge at k-1, and on the triangular lattice the pair
// (k-2, k-1)), so the sources a target of T_k reads agree with it on the
// other points up to a merge of two blocks.  Numbering the targets of T_k --
// the space after it -- lexicographically by their canonical labelling read
// from point k+1 to m-1 and then from 0 to k, the touched points last, puts
// the readers of a source next to each other: a run of targets re-reads its
// sources while they are still cached.  A fused factor T_hi ... T_lo writes
// the space after T_hi, numbered for T_hi, which touches the highest points
// of the product.  The target rows are then also visited in that order.
void site_order(std::vector<Csr>& fwd, int lattice, int m, int threads) {
  const int n = static_cast<int>(fwd.size());
  if (n < 2) return;
  std::vector<std::vector<int32_t>> perm(n + 1);  // perm[k][old] = new, space after T_k
  std::exception_ptr err;
  std::mutex err_mu;
  // spaces are independent: one thread each, every thread sorts its own
  std::vector<std::thread> pool;
  std::atomic<int> next{1};
  const int nt = std::max(1, std::min(threads, n - 1));
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&] {
      try {
        for (int k = next++; k < n; k = next++) {
          const Space sp = lattice == kSquare ? Space{kSqInter, m, k} : Space{kNcnnn, m, 0};
          const int64_t ns = sp.size();
          if (ns != fwd[k - 1].n_rows || ns != fwd[k].n_cols) throw std::runtime_error("site order: space size");
          std::vector<std::pair<unsigned __int128, int32_t>> key(ns);
          Part p;
          for (int64_t r = 0; r < ns; ++r) {
            sp.unrank(r, p);
            uint8_t relab[kMaxM + 1];
            std::memset(relab, 0xff, sizeof relab);
            uint8_t used = 0;
            unsigned __int128 x = 0;
            for (int j = 0; j < m; ++j) {
              const int pt = (k + 1 + j) % m;
              uint8_t& c = relab[p.lab[pt]];
              if (c == 0xff) c = used++;
              x = (x << 5) | c;
            }
            key[r] = {x, static_cast<int32_t>(r)};
          }
          std::sort(key.begin(), key.end());
          std::vector<int32_t> pk(ns);
          for (int64_t j = 0; j < ns; ++j) pk[key[j].second] = static_cast<int32_t>(j);
          perm[k] = std::move(pk);
        }
      } catch (...) {
        std::lock_guard<std::mutex> lk(err_mu);
        if (!err) err = std::current_exception();
      }
    });
  for (auto& th : pool) th.join();
  if (err) std::rethrow_exception(err);
  for (int k = 0; k < n; ++k) renumber(fwd[k], perm[k + 1], perm[k], threads);
}

// The numbering to use: paper_order or CHROMSTRIP_STATE_ORDER, else the
// site order for the evaluation form and the reader order for the normalised
// form (whose maps are also built on the device, in that order; it never
// takes the site order).
int state_order(bool normalised, bool paper_order) {
  if (paper_order) return kOrderPaper;
  const char* env = std::getenv("CHROMSTRIP_STATE_ORDER");
  if (env && *env) {
    const std::string v(env);
    if (v == "paper") return kOrderPaper;
    if (v == "reader") return kOrderReader;
    if (v == "site") return normalised ? kOrderReader : kOrderSite;
    throw std::runtime_error("CHROMSTRIP_STATE_ORDER must be paper, reader or site");
  }
  return normalised ? kOrderReader : kOrderSite;
}

// Adds two polynomials / multiplies them (degrees stay <= kMaxDeg).
Poly padd(const Poly& a, const Poly& b) {
  Poly r;
  for (int k = 0; k <= kMaxDeg; ++k) r.c[k] = a.c[k] + b.c[k];
  return r;
}
Poly pmul(const Poly& a, const Poly& b) {
  int64_t full[2 * kMaxDeg + 1] = {0};
  for (int i = 0; i <= kMaxDeg; ++i)
    for (int j = 0; j <= kMaxDeg; ++j) full[i + j] += a.c[i] * b.c[j];
  for (int k = kMaxDeg + 1; k <= 2 * kMaxDeg; ++k)
    if (full[k] != 0) throw std::runtime_error("coefficient degree above 3");
  Poly r;
  for (int k = 0; k <= kMaxDeg; ++k) r.c[k] = full[k];
  return r;
}

// F = T_hi ... T_lo from the single factors (any consistent numbering).
// Entries carry polynomials; entries that cancel exactly are dropped.
struct PolyCsr {
  int64_t n_rows = 0, n_cols = 0;
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col;
  std::vector<Poly> coef;
};

PolyCsr to_poly(const Csr& c, const std::vector<Poly>& codes) {
  PolyCsr p;
  p.n_rows = c.n_rows;
  p.n_cols = c.n_cols;
  p.row_ptr.assign(c.row_ptr.begin(), c.row_ptr.end());
  p.col.resize(c.ent.size());
  p.coef.resize(c.ent.size());
  for (size_t e = 0; e < c.ent.size(); ++e) {
    p.col[e] = static_cast<int32_t>(c.ent[e] & kSrcMask);
    p.coef[e] = codes[c.ent[e] >> kSrcBits];
  }
  return p;
}

// (T · P): row r of T combines rows of P.
PolyCsr compose(const PolyCsr& t, const PolyCsr& p, int threads) {
  PolyCsr out;
  out.n_rows = t.n_rows;
  out.n_cols = p.n_cols;
  std::vector<std::vector<std::pair<int32_t, Poly>>> rows(t.n_rows);
  parallel_for(t.n_rows, threads, [&](int, int64_t lo, int64_t hi) {
    std::vector<std::pair<int32_t, Poly>> acc;
    for (int64_t r = lo; r < hi; ++r) {
      acc.clear();
      for (int64_t e = t.row_ptr[r]; e < t.row_ptr[r + 1]; ++e) {
        const int32_t mid = t.col[e];
        for (int64_t f = p.row_ptr[mid]; f < p.row_ptr[mid + 1]; ++f) {
          const Poly term = pmul(t.coef[e], p.coef[f]);
          bool found = false;
          for (auto& kv : acc)
            if (kv.first == p.col[f]) {
              kv.second = padd(kv.second, term);
              found = true;
              break;
            }
          if (!found) acc.emplace_back(p.col[f], term);
        }
      }
      auto& dst = rows[r];
      for (auto& kv : acc)
        if (!kv.second.zero()) dst.push_back(kv);
      std::sort(dst.begin(), dst.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    }
  });
  out.row_ptr.assign(t.n_rows + 1, 0);
  for (int64_t r = 0; r < t.n_rows; ++r) out.row_ptr[r + 1] = out.row_ptr[r] + static_cast<int64_t>(rows[r].size());
  out.col.resize(out.row_ptr.back());
  out.coef.resize(out.row_ptr.back());
  for (int64_t r = 0; r < t.n_rows; ++r) {
    int64_t w = out.row_ptr[r];
    for (auto& kv : rows[r]) {
      out.col[w] = kv.first;
      out.coef[w] = kv.second;
      ++w;
    }
  }
  return out;
}

std::unique_ptr<Family> build_family(const MapSet& ms, int k) {
  const int m = ms.m;
  const int threads = build_threads();
  auto fam = std::make_unique<Family>();
  fam->k = k;
  fam->codes = ms.codes;
  std::map<Poly, int> code_of;
  for (size_t c = 0; c < ms.codes.size(); ++c) code_of[ms.codes[c]] = static_cast<int>(c);
  std::vector<PolyCsr> prods;
  for (int lo = 1; lo <= m; lo += k) {
    const int hi = std::min(m, lo + k - 1);
    PolyCsr p = to_poly(ms.fwd[lo - 1], ms.codes);
    for (int j = lo + 1; j <= hi; ++j) p = compose(to_poly(ms.fwd[j - 1], ms.codes), p, threads);
    fam->lo.push_back(lo);
    fam->hi.push_back(hi);
    prods.push_back(std::move(p));
  }
  // new coefficient polynomials get codes after the base table, in order
  std::map<Poly, int> fresh;
  for (const PolyCsr& p : prods)
    for (const Poly& c : p.coef)
      if (!code_of.count(c)) fresh[c] = 0;
  for (auto& kv : fresh) {
    if (static_cast<int>(fam->codes.size()) >= kMaxCodes)
      throw std::runtime_error("more than 64 distinct coefficients in a fused family");
    code_of[kv.first] = static_cast<int>(fam->codes.size());
    fam->codes.push_back(kv.first);
  }
  for (const PolyCsr& p : prods) {
    Csr c;
    c.n_rows = p.n_rows;
    c.n_cols = p.n_cols;
    if (p.row_ptr.back() > INT32_MAX) throw std::runtime_error("too many entries in a fused factor");
    c.row_ptr.assign(p.row_ptr.begin(), p.row_ptr.end());
    c.ent.resize(p.col.size());
    for (size_t e = 0; e < p.col.size(); ++e)
      c.ent[e] = static_cast<uint32_t>(p.col[e]) | (static_cast<uint32_t>(code_of[p.coef[e]]) << kSrcBits);
    fam->fac.push_back(std::move(c));
  }
  // site order: the spaces keep the single factors' numbering, made for the
  // factor that writes each of them
  if (ms.order == kOrderReader) reader_order(fam->fac, threads);
  return fam;
}

}  // namespace

int64_t MapSet::total_nnz() const {
  int64_t s = 0;
  for (auto& c : fwd) s += c.nnz();
  for (auto& c : last) s += c.nnz();
  return s;
}

int64_t MapSet::max_states() const {
  int64_t s = 0;
  for (auto& c : fwd) s = std::max({s, c.n_rows, c.n_cols});
  for (auto& c : last) s = std::max({s, c.n_rows, c.n_cols});
  return s;
}

const Family& MapSet::family(int k) const {
  if (normalised && k > 1) throw std::runtime_error("fused families are built for the un-normalised form only");
  std::lock_guard<std::mutex> lk(fam_mu_);
  auto it = fam_.find(k);
  if (it != fam_.end()) return *it->second;
  auto f = build_family(*this, k);
  const Family& ref = *f;
  fam_.emplace(k, std::move(f));
  return ref;
}

size_t MapSet::host_bytes() const {
  size_t s = 0;
  for (auto& c : fwd) s += c.row_ptr.size() * 4 + c.ent.size() * 4;
  for (auto& c : last) s += c.row_ptr.size() * 4 + c.ent.size() * 4;
  return s;
}

// One stderr line per built site when CHROMSTRIP_VERBOSE=1 (large widths take
// minutes on the host).
struct BuildLog {
  bool on;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  BuildLog() {
    const char* v = std::getenv("CHROMSTRIP_VERBOSE");
    on = v && std::string(v) == "1";
  }
  void line(int lattice, int m, bool normalised, const char* what, int i) const {
    if (!on) return;
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "[maps %s m=%d%s] %s %d  %.1f s\n", lattice == kSquare ? "square" : "triangular", m,
                 normalised ? " normalised" : "", what, i, s);
    std::fflush(stderr);
  }
};

std::unique_ptr<MapSet> build_maps(int lattice, int m, int threads, bool normalised, bool paper_order) {
  if (lattice != kSquare && lattice != kTriangular) throw std::runtime_error("bad lattice");
  if (m < 1 || m > kMaxM) throw std::runtime_error("m out of range");
  if (threads <= 0) threads = build_threads();
  auto ms = std::make_unique<MapSet>();
  ms->lattice = lattice;
  ms->m = m;
  ms->normalised = normalised;
  ms->fwd.resize(m);
  ms->last.resize(m);
  if (normalised) ms->last_fwd.resize(m);
  std::vector<std::vector<int32_t>> fkeys(m), lkeys(m), gkeys(m);
  std::vector<std::atomic<uint64_t>> seen((kKeys + 63) / 64);
  for (auto& w : seen) w = 0;
  // The coefficient form reads its read-out maps in gather form only, so a
  // normalised set leaves the scatter-form `last` empty.
  const BuildLog log;
  for (int i = 1; i <= m; ++i) {
    build_factor(forward_def(lattice, m, i), true, normalised, threads, ms->fwd[i - 1], fkeys[i - 1], seen.data());
    if (normalised)
      build_factor(last_def(lattice, m, i), true, normalised, threads, ms->last_fwd[i - 1], gkeys[i - 1],
                   seen.data());
    else
      build_factor(last_def(lattice, m, i), false, normalised, threads, ms->last[i - 1], lkeys[i - 1], seen.data());
    log.line(lattice, m, normalised, "site", i);
  }
  // Codes: +1 -> 0, -1 -> 1, then every other coefficient in key order.
  std::vector<int> key_to_code(kKeys, -1);
  auto add = [&](int key) {
    if (key_to_code[key] >= 0) return;
    if (static_cast<int>(ms->codes.size()) >= kMaxCodes) throw std::runtime_error("too many distinct coefficients");
    key_to_code[key] = static_cast<int>(ms->codes.size());
    ms->codes.push_back(key_poly(key));
  };
  const int one[kMaxDeg + 1] = {1, 0, 0, 0}, minus_one[kMaxDeg + 1] = {-1, 0, 0, 0};
  add(coef_key(one));
  add(coef_key(minus_one));
  for (int k = 0; k < kKeys; ++k)
    if ((seen[k / 64].load() >> (k % 64)) & 1ull) add(k);
  auto finish = [&](Csr& c, const std::vector<int32_t>& keys) {
    parallel_for(static_cast<int64_t>(c.ent.size()), threads, [&](int, int64_t lo, int64_t hi) {
      for (int64_t e = lo; e < hi; ++e) c.ent[e] |= static_cast<uint32_t>(key_to_code[keys[e]]) << kSrcBits;
    });
  };
  for (int i = 0; i < m; ++i) {
    finish(ms->fwd[i], fkeys[i]);
    if (normalised)
      finish(ms->last_fwd[i], gkeys[i]);
    else
      finish(ms->last[i], lkeys[i]);
  }
  ms->order = state_order(normalised, paper_order);
  if (ms->order == kOrderReader) reader_order(ms->fwd, threads);
  if (ms->order == kOrderSite) site_order(ms->fwd, lattice, m, threads);
  log.line(lattice, m, normalised, ms->order == kOrderSite ? "site order, sites" : "state order, sites", m);
  return ms;
}

StagedCsr build_staged(const Csr& c, int slots, int rows) {
  if (slots < 1 || rows < 1) throw std::runtime_error("bad staging limits");
  StagedCsr st;
  st.ent.resize(c.ent.size());
  st.tile_row0.push_back(0);
  st.tile_src0.push_back(0);
  std::vector<int32_t> slot_of(static_cast<size_t>(std::max<int64_t>(c.n_cols, 1)), -1);
  std::vector<int32_t> cur;
  const int64_t n = c.n_rows;
  int64_t r = 0;
  while (r < n) {
    const int64_t r0 = r;
    cur.clear();
    while (r < n && r - r0 < rows) {
      // distinct sources this row would add
      int add = 0;
      for (int32_t e = c.row_ptr[r]; e < c.row_ptr[r + 1]; ++e) {
        const int32_t s = static_cast<int32_t>(c.ent[e] & kSrcMask);
        if (slot_of[s] == -1) {
          slot_of[s] = -2;
          ++add;
        }
      }
      const bool fits = static_cast<int>(cur.size()) + add <= slots || r == r0;
      for (int32_t e = c.row_ptr[r]; e < c.row_ptr[r + 1]; ++e) {
        const int32_t s = static_cast<int32_t>(c.ent[e] & kSrcMask);
        if (slot_of[s] == -2) {
          if (fits) {
            slot_of[s] = static_cast<int32_t>(cur.size());
            cur.push_back(s);
          } else {
            slot_of[s] = -1;
          }
        }
      }
      if (!fits) break;
      ++r;
    }
    std::sort(cur.begin(), cur.end());
    for (size_t i = 0; i < cur.size(); ++i) slot_of[cur[i]] = static_cast<int32_t>(i);
    for (int32_t e = c.row_ptr[r0]; e < c.row_ptr[r]; ++e) {
      const uint32_t w = c.ent[e];
      st.ent[e] = (w & ~kSrcMask) | static_cast<uint32_t>(slot_of[w & kSrcMask]);
    }
    st.src.insert(st.src.end(), cur.begin(), cur.end());
    for (int32_t s : cur) slot_of[s] = -1;
    st.max_slots = std::max(st.max_slots, static_cast<int>(cur.size()));
    st.tile_row0.push_back(static_cast<int32_t>(r));
    st.tile_src0.push_back(static_cast<int32_t>(st.src.size()));
  }
  for (int t = 0; t <= st.n_tiles(); ++t) st.tile_ent0.push_back(c.row_ptr[st.tile_row0[t]]);
  for (int t = 0; t < st.n_tiles(); ++t) {
    st.max_rows = std::max(st.max_rows, st.tile_row0[t + 1] - st.tile_row0[t]);
    st.max_ent = std::max(st.max_ent, st.tile_ent0[t + 1] - st.tile_ent0[t]);
  }
  return st;
}

std::vector<int32_t> ncnnn_natural_order(int m) {
  const Space sp{kNcnnn, m, 0};
  const int64_t n = sp.size();
  std::vector<std::pair<unsigned __int128, int32_t>> key(n);
  Part p;
  for (int64_t r = 0; r < n; ++r) {
    sp.unrank(r, p);   // canonical: labels numbered by first appearance
    unsigned __int128 x = 0;
    for (int j = 0; j < m; ++j) x = (x << 5) | p.lab[j];
    key[r] = {x, static_cast<int32_t>(r)};
  }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> order(n);
  for (int64_t k = 0; k < n; ++k) order[k] = key[k].second;
  return order;
}

StagedCsr build_interleaved(const Csr& c, int rows_tile, int waves, const std::vector<int32_t>* order) {
  if (rows_tile < 1 || waves < 1 || rows_tile % waves != 0) throw std::runtime_error("bad interleave shape");
  const int64_t n = c.n_rows;
  if (order && static_cast<int64_t>(order->size()) != n) throw std::runtime_error("row order of the wrong size");
  const int rpw = rows_tile / waves;
  StagedCsr st;
  st.tile_row0.push_back(0);
  st.tile_src0.push_back(0);
  st.tgt.resize(n);
  const int64_t whole = n / rows_tile * rows_tile;
  for (int64_t pos = 0; pos < n; ++pos) {
    int64_t q = pos;
    if (pos < whole) {
      const int64_t b = pos / rows_tile, o = pos % rows_tile;
      const int64_t w = o / rpw, k = o % rpw;
      q = b * rows_tile + k * waves + w;
    }
    st.tgt[pos] = order ? (*order)[q] : static_cast<int32_t>(q);
  }
  st.row_ptr.assign(n + 1, 0);
  for (int64_t pos = 0; pos < n; ++pos) {
    const int32_t r = st.tgt[pos];
    st.row_ptr[pos + 1] = st.row_ptr[pos] + (c.row_ptr[r + 1] - c.row_ptr[r]);
  }
  st.ent_src.resize(c.ent.size());
  for (int64_t pos = 0; pos < n; ++pos) {
    const int32_t r = st.tgt[pos];
    std::copy(c.ent.begin() + c.row_ptr[r], c.ent.begin() + c.row_ptr[r + 1], st.ent_src.begin() + st.row_ptr[pos]);
  }
  return st;
}

StagedCsr build_clustered(const Csr& c, int slots, int rows, int max_ent) {
  if (slots < 1 || rows < 1) throw std::runtime_error("bad staging limits");
  const int64_t n = c.n_rows, nc = std::max<int64_t>(c.n_cols, 1);
  // readers of every source
  std::vector<int64_t> cp(static_cast<size_t>(nc) + 1, 0);
  for (uint32_t w : c.ent) ++cp[(w & kSrcMask) + 1];
  for (int64_t i = 0; i < nc; ++i) cp[i + 1] += cp[i];
  std::vector<int32_t> rd(c.ent.size());
  {
    std::vector<int64_t> cur(cp.begin(), cp.end() - 1);
    for (int64_t r = 0; r < n; ++r)
      for (int32_t e = c.row_ptr[r]; e < c.row_ptr[r + 1]; ++e) rd[cur[c.ent[e] & kSrcMask]++] = static_cast<int32_t>(r);
  }
  StagedCsr st;
  st.tile_row0.push_back(0);
  st.tile_src0.push_back(0);
  st.row_ptr.push_back(0);
  std::vector<char> placed(static_cast<size_t>(n), 0);
  std::vector<int32_t> slot_of(static_cast<size_t>(nc), -1);
  std::vector<int32_t> tsrc, ttgt;
  int64_t next = 0, done = 0, tent = 0;
  auto new_sources_count = [&](int64_t r) {
    int k = 0;
    for (int32_t e = c.row_ptr[r]; e < c.row_ptr[r + 1]; ++e) k += slot_of[c.ent[e] & kSrcMask] == -1;
    return k;   // counts a source twice if the row reads it twice (an upper bound)
  };
  auto fits = [&](int64_t r) {
    return static_cast<int>(tsrc.size()) + new_sources_count(r) <= slots &&
           tent + (c.row_ptr[r + 1] - c.row_ptr[r]) <= max_ent;
  };

  auto add = [&](int64_t r) {
    placed[r] = 1;
    ++done;
    tent += c.row_ptr[r + 1] - c.row_ptr[r];
    ttgt.push_back(static_cast<int32_t>(r));
    for (int32_t e = c.row_ptr[r]; e < c.row_ptr[r + 1]; ++e) {
      const uint32_t s = c.ent[e] & kSrcMask;
      if (slot_of[s] == -1) {
        slot_of[s] = static_cast<int32_t>(tsrc.size());
        tsrc.push_back(static_cast<int32_t>(s));
      }
    }
  };
  while (done < n) {
    while (placed[next]) ++next;
    tsrc.clear();
    ttgt.clear();
    tent = 0;
    add(next);   // a row over the limits forms a tile of its own
    size_t qi = 0;
    for (;;) {
      if (static_cast<int>(ttgt.size()) >= rows) break;
      if (qi >= tsrc.size()) {
        while (next < n && placed[next]) ++next;
        if (next >= n || !fits(next)) break;
        add(next);
        continue;
      }
      const int32_t s = tsrc[qi++];
      for (int64_t k = cp[s]; k < cp[s + 1] && static_cast<int>(ttgt.size()) < rows; ++k) {
        const int32_t t = rd[k];
        if (placed[t] || !fits(t)) continue;
        add(t);
      }
    }
    // slots in ascending source order; entries renumbered
    std::vector<int32_t> sorted(tsrc);
    std::sort(sorted.begin(), sorted.end());
    for (size_t i = 0; i < sorted.size(); ++i) slot_of[sorted[i]] = static_cast<int32_t>(i);
    for (int32_t t : ttgt) {
      for (int32_t e = c.row_ptr[t]; e < c.row_ptr[t + 1]; ++e) {
        const uint32_t w = c.ent[e];
        st.ent.push_back((w & ~kSrcMask) | static_cast<uint32_t>(slot_of[w & kSrcMask]));
        st.ent_src.push_back(w);
      }
      st.row_ptr.push_back(static_cast<int32_t>(st.ent.size()));
      st.tgt.push_back(t);
    }
    st.src.insert(st.src.end(), sorted.begin(), sorted.end());
    for (int32_t sv : sorted) slot_of[sv] = -1;
    st.max_slots = std::max(st.max_slots, static_cast<int>(sorted.size()));
    st.max_rows = std::max(st.max_rows, static_cast<int>(ttgt.size()));
    st.max_ent = std::max<int>(st.max_ent, static_cast<int>(tent));
    st.tile_row0.push_back(static_cast<int32_t>(st.tgt.size()));
    st.tile_src0.push_back(static_cast<int32_t>(st.src.size()));
  }
  for (int t = 0; t <= st.n_tiles(); ++t) st.tile_ent0.push_back(st.row_ptr[st.tile_row0[t]]);
  return st;
}

namespace {
// One slot per (lattice, m, normalised).  Builds take the global build lock
// as well, so map sets build one at a time; a request for a set already
// built only takes its slot's lock.
struct CacheSlot {
  std::mutex mu;
  std::unique_ptr<MapSet> ms;
};
std::mutex g_cache_mu;
std::mutex g_build_mu;
std::map<std::tuple<int, int, bool>, std::shared_ptr<CacheSlot>> g_cache;
}  // namespace

const MapSet& get_maps(int lattice, int m, bool normalised) {
  std::shared_ptr<CacheSlot> slot;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto& s = g_cache[std::make_tuple(lattice, m, normalised)];
    if (!s) s = std::make_shared<CacheSlot>();
    slot = s;
  }
  std::lock_guard<std::mutex> lk(slot->mu);
  if (!slot->ms) {
    std::lock_guard<std::mutex> build(g_build_mu);
    slot->ms = build_maps(lattice, m, 0, normalised);  // a failed build leaves the slot empty
  }
  return *slot->ms;
}

void release_host_maps() {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache.clear();
}

}  // namespace cs
