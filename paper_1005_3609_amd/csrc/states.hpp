// Layer states: non-crossing partitions of m <= CHROM_MAX_M points, their
// spaces and the ranking of Sec. 3.4 (eq. M_recurs) of arXiv 1005.3609.
#pragma once

#include <cstdint>
#include <string>

namespace cs {

constexpr int kMaxM = 20;

// A partition of points 0..m-1 (the paper's 1..m) as block labels.
struct Part {
  uint8_t lab[kMaxM];
};

// Motzkin numbers M_k (eq. M_recurs), k <= 40.
int64_t motzkin(int k);
// Number of NCNNN partitions of n points: M_{n-1}, and 1 for n = 0.
int64_t ncnnn_count(int n);

// Canonical relabelling: labels numbered by first appearance.
void canonicalize(Part& p, int m);
bool same_block(const Part& p, int a, int b);
bool is_alone(const Part& p, int m, int a);
// Blocks of a and b merged.
void join(Part& p, int m, int a, int b);
// Point a removed from its block and made a singleton.
void detach(Part& p, int m, int a);
bool is_noncrossing(const Part& p, int m);

// The state spaces.  kind: 0 = NCNNN, 1 = square intermediate after T_i
// (0-based pair (i-1, i) may share a block; i = 1..m-1 in the paper's
// numbering), 2 = read-out space after T_i^last (points 1..i singletons).
enum SpaceKind { kNcnnn = 0, kSqInter = 1, kLast = 2 };

struct Space {
  int kind;
  int m;
  int i;  // paper's site index (1-based) for kSqInter/kLast
  int64_t size() const;
  // Rank of p (0-based, paper order); -1 if p violates the space's
  // adjacency rule.  p must be non-crossing.
  int64_t rank(const Part& p) const;
  // Canonical partition of rank r.
  void unrank(int64_t r, Part& p) const;
};

// NCNNN rank of points [lo, hi] of p (0-based, inclusive), assuming the
// segment is closed under p's blocks except that its first point may share a
// block with points outside on the left only.
int64_t ncnnn_rank(const Part& p, int m);
void ncnnn_unrank(int64_t r, int n, Part& p);

std::string to_string(const Part& p, int m);

}  // namespace cs
