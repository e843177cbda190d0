// Per-state factor expansion for building maps on the device (arXiv
// 1005.3609, Sec. 3.1-3.4).  One thread takes one source state: it unranks
// it (Sec. 3.4), applies the single-edge operators of one factor at v = -1
// (Sec. 3.1-3.3; the normalised bookkeeping of eq. Z_modified or the
// un-normalised one), and ranks every resulting state in the target space.
// Everything here works on fixed-size arrays (no allocation, no recursion)
// so that the same functions run in a kernel and, for checking, on the host.
//
// The state order is the paper's (no reader-order relabelling), and the
// coefficient keys are those of the host builder (base 17, offset 8, c_3
// most significant), so maps built from this expansion match the host
// builder's in the paper's order.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define CS_HD __host__ __device__
#else
#define CS_HD
#endif

namespace cs {
namespace dx {

constexpr int kM = 20;        // widest strip
constexpr int kTerms = 8;     // terms of one expansion: two joins and V, 2^3
constexpr int kKeyOff = 8, kKeyBase = 17, kKeys = kKeyBase * kKeyBase * kKeyBase * kKeyBase;

// Motzkin numbers and the group offsets of the ranking (eq. M_recurs):
// cum[n][k] is the first rank of group k among the NCNNN partitions of n
// points, cum[n][n-2] their number.
struct Tables {
  int64_t M[41];
  int64_t cum[kM + 1][kM + 1];
};

inline void make_tables(Tables& t) {
  t.M[0] = t.M[1] = 1;
  for (int p = 2; p <= 40; ++p) {
    int64_t s = t.M[p - 1];
    for (int k = 0; k <= p - 2; ++k) s += t.M[k] * t.M[p - k - 2];
    t.M[p] = s;
  }
  for (int n = 0; n <= kM; ++n)
    for (int k = 0; k <= kM; ++k) t.cum[n][k] = 0;
  for (int n = 3; n <= kM; ++n) {
    int64_t c = (n - 1 <= 0) ? 1 : t.M[n - 2];
    for (int k = 0; k <= n - 3; ++k) {
      t.cum[n][k] = c;
      const int64_t a = (k + 1 <= 0) ? 1 : t.M[k];
      const int64_t b = (n - k - 2 <= 0) ? 1 : t.M[n - k - 3];
      c += a * b;
    }
    t.cum[n][n - 2] = c;
  }
}

// Number of NCNNN partitions of n points (M_{n-1}; 1 for n <= 0).
CS_HD inline int64_t count(const Tables& t, int n) { return n <= 0 ? 1 : t.M[n - 1]; }

// A partition of points 0..m-1 as block labels.  Canonical labels are
// numbered by first appearance and stay below m; kLoose marks a point just
// detached (before relabelling).
struct Part {
  uint8_t lab[kM];
};
constexpr uint8_t kLoose = kM;

CS_HD inline void canonicalize(Part& p, int m) {
  uint8_t map[kM + 1];
  for (int x = 0; x <= kM; ++x) map[x] = 0xff;
  uint8_t next = 0;
  for (int x = 0; x < m; ++x) {
    const int l = p.lab[x];
    if (map[l] == 0xff) map[l] = next++;
    p.lab[x] = map[l];
  }
}

CS_HD inline bool is_alone(const Part& p, int m, int a) {
  for (int x = 0; x < m; ++x)
    if (x != a && p.lab[x] == p.lab[a]) return false;
  return true;
}

CS_HD inline void join(Part& p, int m, int a, int b) {
  const uint8_t from = p.lab[b], to = p.lab[a];
  if (from == to) return;
  for (int x = 0; x < m; ++x)
    if (p.lab[x] == from) p.lab[x] = to;
  canonicalize(p, m);
}

CS_HD inline void detach(Part& p, int m, int a) {
  p.lab[a] = kLoose;
  canonicalize(p, m);
}

// Neighbours in one block are allowed only for the pair (allowed_left,
// allowed_left + 1).
CS_HD inline bool adjacent_ok(const Part& p, int m, int allowed_left) {
  for (int x = 0; x + 1 < m; ++x)
    if (p.lab[x] == p.lab[x + 1] && x != allowed_left) return false;
  return true;
}

// nxt[x]: the next point of x's block to the right, or -1.
CS_HD inline void next_in_block(const Part& p, int m, int8_t* nxt) {
  int8_t last[kM];
  for (int x = 0; x < kM; ++x) last[x] = -1;
  for (int x = m - 1; x >= 0; --x) {
    nxt[x] = last[p.lab[x]];
    last[p.lab[x]] = static_cast<int8_t>(x);
  }
}

// Rank of the points [lo, hi] (Sec. 3.4), or -1 for a pair of neighbours in
// one block.  The ranking's recursion (an inner segment between a point and
// the next point of its block, then the segment to the right) is linear in
// the inner ranks, so a stack of (segment, multiplier) frames replaces it.
CS_HD inline int64_t rank_seg(const Tables& t, const int8_t* nxt, int lo0, int hi0) {
  int slo[kM + 1], shi[kM + 1];
  int64_t smul[kM + 1];
  int sp = 0;
  slo[sp] = lo0;
  shi[sp] = hi0;
  smul[sp] = 1;
  ++sp;
  int64_t acc = 0;
  while (sp > 0) {
    --sp;
    int lo = slo[sp];
    const int hi = shi[sp];
    const int64_t mul = smul[sp];
    while (true) {
      const int n = hi - lo + 1;
      if (n <= 2) break;
      const int j = nxt[lo];
      if (j < 0 || j > hi) {
        ++lo;
        continue;
      }
      const int k = j - lo - 2;
      if (k < 0) return -1;
      acc += mul * t.cum[n][k];
      if (sp > kM) return -1;  // cannot happen for m <= kM: one frame per open block
      slo[sp] = lo + 1;
      shi[sp] = j - 1;
      smul[sp] = mul * count(t, n - k - 2);
      ++sp;
      lo = j;
    }
  }
  return acc;
}

// Unranks the points [lo0, hi0] into link[]: link[x] = the next point of x's
// block (x joined to it) or -1 (x's block continues no further right).
CS_HD inline void unrank_links(const Tables& t, int64_t r0, int lo0, int hi0, int8_t* link) {
  int64_t sr[kM + 1];
  int slo[kM + 1], shi[kM + 1];
  int sp = 0;
  sr[sp] = r0;
  slo[sp] = lo0;
  shi[sp] = hi0;
  ++sp;
  while (sp > 0) {
    --sp;
    int64_t r = sr[sp];
    int lo = slo[sp];
    const int hi = shi[sp];
    while (true) {
      const int n = hi - lo + 1;
      if (n <= 0) break;
      if (n <= 2) {
        for (int x = lo; x <= hi; ++x) link[x] = -1;
        break;
      }
      if (r < count(t, n - 1)) {
        link[lo] = -1;
        ++lo;
        continue;
      }
      int k = 0;
      while (k + 1 <= n - 3 && t.cum[n][k + 1] <= r) ++k;
      const int64_t rr = r - t.cum[n][k];
      const int64_t nright = count(t, n - k - 2);
      if (sp > kM) return;  // cannot happen for m <= kM
      sr[sp] = rr / nright;
      slo[sp] = lo + 1;
      shi[sp] = lo + 1 + k;
      ++sp;
      link[lo] = static_cast<int8_t>(lo + 2 + k);
      lo = lo + 2 + k;
      r = rr % nright;
    }
  }
}

// Labels from links, right to left, points [lo, hi]; then canonical.
CS_HD inline void labels_from_links(Part& p, int m, int lo, int hi, const int8_t* link, int next_id) {
  for (int x = hi; x >= lo; --x) p.lab[x] = link[x] < 0 ? static_cast<uint8_t>(next_id++) : p.lab[link[x]];
  canonicalize(p, m);
}

enum SpaceKind { kNcnnn = 0, kSqInter = 1, kLast = 2 };

// A state space: NCNNN partitions of m points; the square intermediate space
// after T_i (0-based pair (i-1, i) may share a block); the read-out space
// after T_i^last (points 0..i-1 singletons).
struct Space {
  int kind, m, i;
};

CS_HD inline int64_t space_size(const Tables& t, const Space& s) {
  switch (s.kind) {
    case kNcnnn: return count(t, s.m);
    case kSqInter: return count(t, s.m) + count(t, s.m - 1);
    default: return count(t, s.m - s.i);
  }
}

CS_HD inline int64_t ncnnn_rank(const Tables& t, const Part& p, int m) {
  if (!adjacent_ok(p, m, -1)) return -1;
  int8_t nxt[kM];
  next_in_block(p, m, nxt);
  return rank_seg(t, nxt, 0, m - 1);
}

CS_HD inline int64_t space_rank(const Tables& t, const Space& s, const Part& p) {
  const int m = s.m, i = s.i;
  switch (s.kind) {
    case kNcnnn:
      return ncnnn_rank(t, p, m);
    case kSqInter: {
      if (!adjacent_ok(p, m, i - 1)) return -1;
      if (p.lab[i - 1] != p.lab[i]) return ncnnn_rank(t, p, m);
      Part c;
      int w = 0;
      for (int x = 0; x < m; ++x)
        if (x != i) c.lab[w++] = p.lab[x];
      const int64_t r = ncnnn_rank(t, c, m - 1);
      return r < 0 ? -1 : count(t, m) + r;
    }
    default: {
      for (int x = 0; x < i && x < m; ++x)
        if (!is_alone(p, m, x)) return -1;
      if (i >= m) return 0;
      if (!adjacent_ok(p, m, -1)) return -1;
      int8_t nxt[kM];
      next_in_block(p, m, nxt);
      return rank_seg(t, nxt, i, m - 1);
    }
  }
}

CS_HD inline void space_unrank(const Tables& t, const Space& s, int64_t r, Part& p) {
  const int m = s.m, i = s.i;
  int8_t link[kM];
  switch (s.kind) {
    case kNcnnn:
      unrank_links(t, r, 0, m - 1, link);
      labels_from_links(p, m, 0, m - 1, link, 0);
      return;
    case kSqInter: {
      const int64_t n0 = count(t, m);
      if (r < n0) {
        unrank_links(t, r, 0, m - 1, link);
        labels_from_links(p, m, 0, m - 1, link, 0);
        return;
      }
      Part c;
      unrank_links(t, r - n0, 0, m - 2, link);
      labels_from_links(c, m - 1, 0, m - 2, link, 0);
      int w = 0;
      for (int x = 0; x < m; ++x) p.lab[x] = (x == i) ? c.lab[i - 1] : c.lab[w++];
      canonicalize(p, m);
      return;
    }
    default: {
      for (int x = 0; x < i && x < m; ++x) p.lab[x] = static_cast<uint8_t>(x);
      if (i < m) {
        unrank_links(t, r, i, m - 1, link);
        labels_from_links(p, m, i, m - 1, link, i);
      } else {
        canonicalize(p, m);
      }
      return;
    }
  }
}

// A term: a state and its coefficient polynomial c0 + c1 z + c2 z^2 + c3 z^3
// (z = q un-normalised, z = x = 1/q normalised).
struct Term {
  Part p;
  int8_t c[4];
};

// The terms of one expansion; `bad` is set when a coefficient leaves the
// supported range (degree above 3, |c_k| > 8) or the list would overflow.
struct Expansion {
  Term t[kTerms];
  int n;
  int m;
  bool norm;
  bool bad;
};

CS_HD inline void times_z(Expansion& e, Term& u, int sign) {
  if (u.c[3] != 0) e.bad = true;
  for (int k = 3; k > 0; --k) u.c[k] = static_cast<int8_t>(sign * u.c[k - 1]);
  u.c[0] = 0;
}

CS_HD inline void op_H(Expansion& e, int a, int b) {
  Term out[kTerms];
  int n = 0;
  for (int s = 0; s < e.n; ++s) {
    const Term& u = e.t[s];
    if (u.p.lab[a] == u.p.lab[b]) continue;  // (1 - J) s = 0 when a, b share a block
    if (n + 2 > kTerms) {
      e.bad = true;
      return;
    }
    out[n++] = u;
    Term j = u;
    join(j.p, e.m, a, b);
    if (e.norm) {
      times_z(e, j, -1);
    } else {
      for (int k = 0; k < 4; ++k) j.c[k] = static_cast<int8_t>(-u.c[k]);
    }
    out[n++] = j;
  }
  for (int s = 0; s < n; ++s) e.t[s] = out[s];
  e.n = n;
}

CS_HD inline void op_V(Expansion& e, int i) {
  Term out[kTerms];
  int n = 0;
  for (int s = 0; s < e.n; ++s) {
    const Term& u = e.t[s];
    if (n + 2 > kTerms) {
      e.bad = true;
      return;
    }
    Term present = u;
    if (e.norm) {
      times_z(e, present, -1);
    } else {
      for (int k = 0; k < 4; ++k) present.c[k] = static_cast<int8_t>(-u.c[k]);
    }
    out[n++] = present;
    Term d = u;
    if (is_alone(u.p, e.m, i)) {
      if (!e.norm) times_z(e, d, 1);
    } else {
      detach(d.p, e.m, i);
    }
    out[n++] = d;
  }
  for (int s = 0; s < n; ++s) e.t[s] = out[s];
  e.n = n;
}

CS_HD inline void op_D(Expansion& e, int i) {
  for (int s = 0; s < e.n; ++s) {
    Term& u = e.t[s];
    if (is_alone(u.p, e.m, i)) {
      if (!e.norm) times_z(e, u, 1);
    } else {
      detach(u.p, e.m, i);
    }
  }
}

// Keeps the terms with no pair (x, x+1), bit x of `forbid` set, in one block.
CS_HD inline void op_P(Expansion& e, uint32_t forbid) {
  int n = 0;
  for (int s = 0; s < e.n; ++s) {
    bool ok = true;
    for (int x = 0; x + 1 < e.m; ++x)
      if (((forbid >> x) & 1u) && e.t[s].p.lab[x] == e.t[s].p.lab[x + 1]) {
        ok = false;
        break;
      }
    if (ok) e.t[n++] = e.t[s];
  }
  e.n = n;
}

// Combines equal states (first appearance order) and drops zero terms.
CS_HD inline void merge(Expansion& e) {
  Term out[kTerms];
  int n = 0;
  for (int s = 0; s < e.n; ++s) {
    int f = -1;
    for (int o = 0; o < n && f < 0; ++o) {
      bool same = true;
      for (int x = 0; x < e.m; ++x)
        if (out[o].p.lab[x] != e.t[s].p.lab[x]) {
          same = false;
          break;
        }
      if (same) f = o;
    }
    if (f >= 0) {
      for (int k = 0; k < 4; ++k) {
        const int v = out[f].c[k] + e.t[s].c[k];
        if (v < -kKeyOff || v > kKeyOff) e.bad = true;
        out[f].c[k] = static_cast<int8_t>(v);
      }
    } else {
      out[n++] = e.t[s];
    }
  }
  e.n = 0;
  for (int s = 0; s < n; ++s)
    if (out[s].c[0] || out[s].c[1] || out[s].c[2] || out[s].c[3]) e.t[e.n++] = out[s];
}

CS_HD inline int coef_key(const int8_t* c) {
  int key = 0;
  for (int k = 3; k >= 0; --k) key = key * kKeyBase + (c[k] + kKeyOff);
  return key;
}

// One factor (Sec. 3.2-3.3): site i (1-based) of a strip of width m, its
// spaces, and whether it is the read-out factor T_i^last.
struct Factor {
  Space in, out;
  int lattice;  // 0 square, 1 triangular
  int m, site;
  int last;
  int norm;
};

CS_HD inline uint32_t all_pairs(int m) { return m >= 2 ? ((1u << (m - 1)) - 1u) : 0u; }

CS_HD inline Factor forward_factor(int lattice, int m, int i, bool norm) {
  Factor f;
  f.lattice = lattice;
  f.m = m;
  f.site = i;
  f.last = 0;
  f.norm = norm ? 1 : 0;
  if (lattice == 0) {
    f.in = (i == 1) ? Space{kNcnnn, m, 0} : Space{kSqInter, m, i - 1};
    f.out = (i == m) ? Space{kNcnnn, m, 0} : Space{kSqInter, m, i};
  } else {
    f.in = Space{kNcnnn, m, 0};
    f.out = Space{kNcnnn, m, 0};
  }
  return f;
}

CS_HD inline Factor last_factor(int lattice, int m, int i, bool norm) {
  Factor f;
  f.lattice = lattice;
  f.m = m;
  f.site = i;
  f.last = 1;
  f.norm = norm ? 1 : 0;
  f.in = (i == 1) ? Space{kNcnnn, m, 0} : Space{kLast, m, i - 1};
  f.out = Space{kLast, m, i};
  return f;
}

// Expands source state r of factor f: up to kTerms (target rank, key)
// pairs; returns their number, or -1 when the expansion is outside what the
// maps can hold (coefficient range, a target outside its space).
CS_HD inline int expand_source(const Tables& t, const Factor& f, int64_t r, int32_t* tgt, int32_t* key) {
  Expansion e;
  e.m = f.m;
  e.norm = f.norm != 0;
  e.bad = false;
  e.n = 1;
  space_unrank(t, f.in, r, e.t[0].p);
  for (int k = 0; k < 4; ++k) e.t[0].c[k] = 0;
  e.t[0].c[0] = 1;
  const int s = f.site - 1;
  const int m = f.m;
  if (f.last) {
    if (f.site < m) op_H(e, s, s + 1);
    op_D(e, s);
    uint32_t forbid = 0;
    for (int x = s + 1; x + 1 < m; ++x) forbid |= 1u << x;
    op_P(e, forbid);
  } else if (f.lattice == 0) {
    if (f.site < m) op_H(e, s, s + 1);
    op_V(e, s);
    uint32_t forbid = all_pairs(m);
    if (f.site < m) forbid &= ~(1u << s);
    op_P(e, forbid);
  } else {
    if (f.site < m) op_H(e, s, s + 1);
    if (f.site > 1) op_H(e, s - 1, s);
    op_V(e, s);
    op_P(e, all_pairs(m));
  }
  merge(e);
  if (e.bad) return -1;
  const int64_t nout = space_size(t, f.out);
  for (int k = 0; k < e.n; ++k) {
    const int64_t tr = space_rank(t, f.out, e.t[k].p);
    if (tr < 0 || tr >= nout) return -1;
    tgt[k] = static_cast<int32_t>(tr);
    key[k] = coef_key(e.t[k].c);
  }
  return e.n;
}

}  // namespace dx
}  // namespace cs
