// Layer states and the ranking bijection of Sec. 3.4 (arXiv 1005.3609).
//
// Ordering (Sec. 3.4): among NCNNN partitions of n points, those where the
// first point is a singleton come first, ordered as the partitions of the
// other n-1 points; then those where it is joined, grouped by k where 3+k is
// the smallest other point of its block (k = 0..n-3, increasing), and inside
// a group ordered with the partition of points 2..2+k as the more
// significant digit and that of 3+k..n as the less significant one.  The
// counts obey eq. M_recurs, so ranks follow from prefix sums of
// N(k+1) N(n-k-2), with N(n) = M_{n-1} the number of NCNNN partitions.
#include "states.hpp"

#include <cstring>
#include <mutex>

namespace cs {

namespace {

struct Tables {
  int64_t M[41];
  // cum[n][k]: first rank of group k among NCNNN partitions of n points
  // (n >= 3); cum[n][n-2] = N(n).
  int64_t cum[kMaxM + 1][kMaxM + 1];
  Tables() {
    M[0] = M[1] = 1;
    for (int p = 2; p <= 40; ++p) {
      int64_t s = M[p - 1];
      for (int k = 0; k <= p - 2; ++k) s += M[k] * M[p - k - 2];
      M[p] = s;
    }
    std::memset(cum, 0, sizeof(cum));
    for (int n = 3; n <= kMaxM; ++n) {
      int64_t c = N(n - 1);
      for (int k = 0; k <= n - 3; ++k) {
        cum[n][k] = c;
        c += N(k + 1) * N(n - k - 2);
      }
      cum[n][n - 2] = c;
    }
  }
  int64_t N(int n) const { return n <= 0 ? 1 : M[n - 1]; }
};

const Tables& tables() {
  static const Tables t;
  return t;
}

// Next point of the same block to the right, or -1.
void next_in_block(const Part& p, int m, int8_t* nxt) {
  int8_t last[256];
  std::memset(last, -1, sizeof(last));
  for (int x = m - 1; x >= 0; --x) {
    nxt[x] = last[p.lab[x]];
    last[p.lab[x]] = static_cast<int8_t>(x);
  }
}

int64_t rank_seg(const int8_t* nxt, int lo, int hi) {
  const Tables& t = tables();
  int64_t acc = 0;
  // Iterative form of: rank(lo,hi) = rank(lo+1,hi) if lo is alone, else
  // cum + rank(lo+1, j-1) * N(right) + rank(j, hi).  The inner segment's
  // rank needs its own recursion; the right segment continues the loop.
  while (true) {
    int n = hi - lo + 1;
    if (n <= 2) return acc;
    int j = nxt[lo];
    if (j < 0 || j > hi) {
      ++lo;
      continue;
    }
    int k = j - lo - 2;
    if (k < 0) return -1;  // neighbours in one block: not NCNNN
    int64_t nright = t.N(n - k - 2);
    int64_t inner = rank_seg(nxt, lo + 1, j - 1);
    if (inner < 0) return -1;
    acc += t.cum[n][k] + inner * nright;
    lo = j;  // + rank(j, hi)
  }
}

void unrank_seg(int64_t r, int lo, int hi, uint8_t* blk, int& next_id) {
  const Tables& t = tables();
  while (true) {
    int n = hi - lo + 1;
    if (n <= 0) return;
    if (n <= 2) {
      for (int x = lo; x <= hi; ++x) blk[x] = static_cast<uint8_t>(next_id++);
      return;
    }
    if (r < t.N(n - 1)) {
      blk[lo] = static_cast<uint8_t>(next_id++);
      ++lo;
      continue;
    }
    int k = 0;
    while (k + 1 <= n - 3 && t.cum[n][k + 1] <= r) ++k;
    int64_t rr = r - t.cum[n][k];
    int64_t nright = t.N(n - k - 2);
    int64_t a = rr / nright, b = rr % nright;
    unrank_seg(a, lo + 1, lo + 1 + k, blk, next_id);
    unrank_seg(b, lo + 2 + k, hi, blk, next_id);
    blk[lo] = blk[lo + 2 + k];
    return;
  }
}

bool adjacent_ok(const Part& p, int m, int allowed_left) {
  for (int x = 0; x + 1 < m; ++x)
    if (p.lab[x] == p.lab[x + 1] && x != allowed_left) return false;
  return true;
}

}  // namespace

int64_t motzkin(int k) { return (k < 0 || k > 40) ? -1 : tables().M[k]; }
int64_t ncnnn_count(int n) { return tables().N(n); }

void canonicalize(Part& p, int m) {
  uint8_t map[256];
  std::memset(map, 0xff, sizeof(map));
  uint8_t next = 0;
  for (int x = 0; x < m; ++x) {
    uint8_t& t = map[p.lab[x]];
    if (t == 0xff) t = next++;
    p.lab[x] = t;
  }
}

bool same_block(const Part& p, int a, int b) { return p.lab[a] == p.lab[b]; }

bool is_alone(const Part& p, int m, int a) {
  for (int x = 0; x < m; ++x)
    if (x != a && p.lab[x] == p.lab[a]) return false;
  return true;
}

void join(Part& p, int m, int a, int b) {
  uint8_t from = p.lab[b], to = p.lab[a];
  if (from == to) return;
  for (int x = 0; x < m; ++x)
    if (p.lab[x] == from) p.lab[x] = to;
  canonicalize(p, m);
}

void detach(Part& p, int m, int a) {
  p.lab[a] = 0xfe;  // a label no canonical partition uses
  canonicalize(p, m);
}

bool is_noncrossing(const Part& p, int m) {
  for (int a = 0; a < m; ++a)
    for (int b = a + 1; b < m; ++b) {
      if (p.lab[b] == p.lab[a]) continue;
      for (int c = b + 1; c < m; ++c) {
        if (p.lab[c] != p.lab[a]) continue;
        for (int d = c + 1; d < m; ++d)
          if (p.lab[d] == p.lab[b]) return false;
      }
    }
  return true;
}

int64_t ncnnn_rank(const Part& p, int m) {
  if (!adjacent_ok(p, m, -1)) return -1;
  int8_t nxt[kMaxM];
  next_in_block(p, m, nxt);
  return rank_seg(nxt, 0, m - 1);
}

void ncnnn_unrank(int64_t r, int n, Part& p) {
  int next_id = 0;
  unrank_seg(r, 0, n - 1, p.lab, next_id);
  canonicalize(p, n);
}

int64_t Space::size() const {
  const Tables& t = tables();
  switch (kind) {
    case kNcnnn: return t.N(m);
    case kSqInter: return t.N(m) + t.N(m - 1);
    case kLast: return t.N(m - i);
  }
  return -1;
}

int64_t Space::rank(const Part& p) const {
  switch (kind) {
    case kNcnnn:
      return ncnnn_rank(p, m);
    case kSqInter: {
      // 0-based pair (i-1, i) is the paper's (i, i+1)
      if (!adjacent_ok(p, m, i - 1)) return -1;
      if (p.lab[i - 1] != p.lab[i]) return ncnnn_rank(p, m);
      Part c;
      int w = 0;
      for (int x = 0; x < m; ++x)
        if (x != i) c.lab[w++] = p.lab[x];
      int64_t r = ncnnn_rank(c, m - 1);
      return r < 0 ? -1 : tables().N(m) + r;
    }
    case kLast: {
      for (int x = 0; x < i; ++x)
        if (!is_alone(p, m, x)) return -1;
      if (i >= m) return 0;
      if (!adjacent_ok(p, m, -1)) return -1;
      int8_t nxt[kMaxM];
      next_in_block(p, m, nxt);
      return rank_seg(nxt, i, m - 1);
    }
  }
  return -1;
}

void Space::unrank(int64_t r, Part& p) const {
  switch (kind) {
    case kNcnnn:
      ncnnn_unrank(r, m, p);
      return;
    case kSqInter: {
      int64_t n0 = tables().N(m);
      if (r < n0) {
        ncnnn_unrank(r, m, p);
        return;
      }
      Part c;
      ncnnn_unrank(r - n0, m - 1, c);
      // expand contracted point i-1 into points i-1 and i
      int w = 0;
      for (int x = 0; x < m; ++x) {
        if (x == i) {
          p.lab[x] = c.lab[i - 1];
        } else {
          p.lab[x] = c.lab[w++];
        }
      }
      canonicalize(p, m);
      return;
    }
    case kLast: {
      int next_id = 0;
      for (int x = 0; x < i && x < m; ++x) p.lab[x] = static_cast<uint8_t>(next_id++);
      if (i < m) unrank_seg(r, i, m - 1, p.lab, next_id);
      canonicalize(p, m);
      return;
    }
  }
}

std::string to_string(const Part& p, int m) {
  std::string s;
  bool done[kMaxM] = {false};
  for (int a = 0; a < m; ++a) {
    if (done[a]) continue;
    s += '(';
    for (int b = a; b < m; ++b)
      if (p.lab[b] == p.lab[a]) {
        done[b] = true;
        if (b + 1 >= 10) s += '{' + std::to_string(b + 1) + '}';
        else s += static_cast<char>('0' + b + 1);
      }
    s += ')';
  }
  return s;
}

}  // namespace cs
