// Host logic of the BICO summary (Sec. 2.1: clustering features in a tree of
// spheres; Sec. 2.3.1: weighted insertion), free of device calls so that it
// also builds as plain C++.  The closest reference among the children of a
// node can come from outside (the device search of kmx_bico.hip) as a hint:
// for a block of points, the closest among the first u children that node had
// when the block started; everything else is decided here in FP64 with sums
// in coordinate order and no fused multiply-adds.
//
// Tree.  A feature holds (W, S, Q) = (weight, weighted sum of its points,
// weighted sum of their squared lengths), a reference point and its children.
// Its cost against its centroid S / W is Q - ||S||^2 / W (Sec. 2.1).  A point
// x with w copies walks down from the root: among the children of the current
// node it takes the one whose reference is closest (ties: the oldest); if no
// reference lies within the level's radius R_i = sqrt(T / 2^(3 + i)) it opens
// a feature (w, w x, w ||x||^2) there; otherwise w' = min(w, floor((sT - sc) /
// (s D - T + c))) copies join that feature (all w when s D - T + c <= 0; s = W,
// c its cost, D = ||x - S / W||^2) and the rest descend to its children.  When
// the tree holds more than m features, T doubles and every feature is
// re-inserted, in breadth-first order of the old tree, into an empty tree:
// it follows its reference point down, merges into the closest feature within
// the radius whose merged cost stays within T, descends when it would not,
// and otherwise keeps its (W, S, Q) as a new feature.  The summary is the
// centroids S / W with weights W in breadth-first order.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include <immintrin.h>

#pragma clang fp contract(off)

namespace kmx {
namespace bico {

struct Feature {
  int32_t level;
  int32_t parent;               // -1: below the root
  std::vector<int32_t> kids;    // creation order
  double W, Q;
};

struct Core {
  int d = 0;
  int64_t m = 0;
  double T = 0.0;
  std::vector<Feature> f;       // creation order
  std::vector<double> S;        // f.size() x d
  std::vector<float> ref;       // f.size() x d
  std::vector<int32_t> roots;   // first-level features, creation order
  int64_t rebuilds = 0, host_scans = 0;
};

// Search hints of a block of points for the child list of one node (-1: the
// root): for point q, the closest among the node's first u children (lab[q],
// an index into that list) with the device's two smallest distances.
struct NodeHints {
  int32_t node = -1;
  size_t u = 0;
  std::vector<int32_t> lab;
  std::vector<float> d1, d2;
};

// Nodes whose child lists a block's search hints cover: the root when it has
// children, then the nodes with the most children (at least kBigKids), at
// most kHintNodes in all.  (A test build may lower kBigKids to reach the
// node hints on small trees.)
#ifndef KMX_BICO_BIG_KIDS
#define KMX_BICO_BIG_KIDS 32
#endif
constexpr size_t kBigKids = KMX_BICO_BIG_KIDS;
constexpr size_t kHintNodes = 16;

inline double sq_dist(const float* a, const float* b, int d) {
  double s = 0.0;
  for (int j = 0; j < d; ++j) {
    const double t = (double)a[j] - (double)b[j];
    s += t * t;
  }
  return s;
}

inline double sq_norm(const double* v, int d) {
  double s = 0.0;
  for (int j = 0; j < d; ++j) s += v[j] * v[j];
  return s;
}

inline double radius2(const Core& b, int level) { return b.T / std::ldexp(1.0, 3 + level); }

// Appends a feature below `parent` (-1: the root) and returns its id.  The
// parent's child list is looked up after the feature array has grown (which
// moves the features and their child lists).
inline int32_t open_feature(Core& b, const float* r, double W, const double* S, double Q,
                            int level, int32_t parent) {
  const int32_t id = (int32_t)b.f.size();
  Feature nf;
  nf.level = level;
  nf.parent = parent;
  nf.W = W;
  nf.Q = Q;
  b.f.push_back(std::move(nf));
  b.S.insert(b.S.end(), S, S + b.d);
  b.ref.insert(b.ref.end(), r, r + b.d);
  if (parent < 0) b.roots.push_back(id);
  else b.f[parent].kids.push_back(id);
  return id;
}

inline const std::vector<int32_t>& kids_of(const Core& b, int32_t parent) {
  return parent < 0 ? b.roots : b.f[parent].kids;
}

// Squared distances of x (as doubles, xd) to eight references, each summed
// in coordinate order exactly as sq_dist sums it: t = x_j - r_j and t * t
// rounded as in the scalar code, the squares of four coordinates of four
// references transposed so that each lane of an accumulator adds its own
// reference's squares one coordinate after another (the same bits; only the
// additions of different references overlap).  Host x86 with AVX2.
__attribute__((target("avx2"))) inline void dist8_avx2(const double* xd, const float* const* r,
                                                       int d, double* out) {
  __m256d acc0 = _mm256_setzero_pd(), acc1 = _mm256_setzero_pd();
  int j = 0;
  for (; j + 4 <= d; j += 4) {
    const __m256d xv = _mm256_loadu_pd(xd + j);
    __m256d q[8];
    for (int i = 0; i < 8; ++i) {
      const __m256d t = _mm256_sub_pd(xv, _mm256_cvtps_pd(_mm_loadu_ps(r[i] + j)));
      q[i] = _mm256_mul_pd(t, t);
    }
    for (int h = 0; h < 2; ++h) {
      // rows q[4h + i] = squares of reference 4h + i at coordinates j .. j + 3
      const __m256d a = q[4 * h], b = q[4 * h + 1], c = q[4 * h + 2], e = q[4 * h + 3];
      const __m256d ab_lo = _mm256_unpacklo_pd(a, b);   // a0 b0 a2 b2
      const __m256d ab_hi = _mm256_unpackhi_pd(a, b);   // a1 b1 a3 b3
      const __m256d ce_lo = _mm256_unpacklo_pd(c, e);   // c0 e0 c2 e2
      const __m256d ce_hi = _mm256_unpackhi_pd(c, e);   // c1 e1 c3 e3
      const __m256d c0 = _mm256_permute2f128_pd(ab_lo, ce_lo, 0x20);   // a0 b0 c0 e0
      const __m256d c1 = _mm256_permute2f128_pd(ab_hi, ce_hi, 0x20);   // a1 b1 c1 e1
      const __m256d c2 = _mm256_permute2f128_pd(ab_lo, ce_lo, 0x31);   // a2 b2 c2 e2
      const __m256d c3 = _mm256_permute2f128_pd(ab_hi, ce_hi, 0x31);   // a3 b3 c3 e3
      __m256d& acc = h ? acc1 : acc0;
      acc = _mm256_add_pd(acc, c0);
      acc = _mm256_add_pd(acc, c1);
      acc = _mm256_add_pd(acc, c2);
      acc = _mm256_add_pd(acc, c3);
    }
  }
  _mm256_storeu_pd(out, acc0);
  _mm256_storeu_pd(out + 4, acc1);
  for (; j < d; ++j)
    for (int i = 0; i < 8; ++i) {
      const double t = xd[j] - (double)r[i][j];
      out[i] += t * t;
    }
}

// Whether the scans take dist8_avx2 (KMX_BICO_SCALAR_SCAN: never, so that a
// test build covers the portable loop, which gives the same bits).
inline bool host_avx2() {
#ifdef KMX_BICO_SCALAR_SCAN
  return false;
#else
  static const bool ok = __builtin_cpu_supports("avx2");
  return ok;
#endif
}

// Closest reference among ids[from, to) (strictly closer replaces: the oldest
// wins ties).  Eight references at a time: eight independent sums, each in
// coordinate order as sq_dist takes it (the same bits), so the additions of
// different references overlap instead of waiting on one chain.
inline void scan(const Core& b, const std::vector<int32_t>& ids, size_t from, size_t to,
                 const float* x, int32_t& best, double& bd) {
  constexpr int L = 8;
  const int d = b.d;
  size_t q = from;
  if (to >= from + L) {
    const bool avx2 = host_avx2();
    std::vector<double> xd(avx2 ? d : 0);
    for (int j = 0; j < (int)xd.size(); ++j) xd[j] = (double)x[j];
    for (; q + L <= to; q += L) {
      const float* r[L];
      double s[L];
      for (int i = 0; i < L; ++i) r[i] = &b.ref[(size_t)ids[q + i] * d];
      if (avx2) {
        dist8_avx2(xd.data(), r, d, s);
      } else {
        for (int i = 0; i < L; ++i) s[i] = 0.0;
        for (int j = 0; j < d; ++j) {
          const double xj = (double)x[j];
          for (int i = 0; i < L; ++i) {
            const double t = xj - (double)r[i][j];
            s[i] += t * t;
          }
        }
      }
      for (int i = 0; i < L; ++i)
        if (best < 0 || s[i] < bd) {
          best = ids[q + i];
          bd = s[i];
        }
    }
  }
  for (; q < to; ++q) {
    const int32_t id = ids[q];
    const double dd = sq_dist(x, &b.ref[(size_t)id * d], d);
    if (best < 0 || dd < bd) {
      best = id;
      bd = dd;
    }
  }
}

inline std::vector<int32_t> bfs(const Core& b) {
  std::vector<int32_t> out(b.roots.begin(), b.roots.end());
  for (size_t q = 0; q < out.size(); ++q)
    for (int32_t c : b.f[out[q]].kids) out.push_back(c);
  return out;
}

inline std::vector<int32_t> hint_nodes(const Core& b) {
  std::vector<int32_t> out;
  if (!b.roots.empty()) out.push_back(-1);
  std::vector<std::pair<size_t, int32_t>> big;
  for (size_t id = 0; id < b.f.size(); ++id)
    if (b.f[id].kids.size() >= kBigKids) big.push_back({b.f[id].kids.size(), (int32_t)id});
  std::sort(big.begin(), big.end(), [](const std::pair<size_t, int32_t>& a,
                                       const std::pair<size_t, int32_t>& c) {
    return a.first != c.first ? a.first > c.first : a.second < c.second;
  });
  for (const auto& e : big) {
    if (out.size() >= kHintNodes) break;
    out.push_back(e.second);
  }
  return out;
}

// Closest reference to x among the children of `parent` (best < 0: none).
// With a hint for this node, the device's choice is re-measured in FP64, the
// children added after the hint are scanned, and all of them are scanned when
// the device's two distances lie within 1e-6 of each other (too near for FP32
// to order them); without one, every child is scanned.
inline void closest(Core& b, int32_t parent, const float* x, const std::vector<NodeHints>* hints,
                    int64_t q, int32_t& best, double& bd) {
  const std::vector<int32_t>& kids = kids_of(b, parent);
  best = -1;
  bd = 0.0;
  const NodeHints* h = nullptr;
  if (hints)
    for (const NodeHints& nh : *hints)
      if (nh.node == parent) {
        h = &nh;
        break;
      }
  if (h && h->u > 0 && h->u <= kids.size() && h->lab[q] >= 0 && (size_t)h->lab[q] < h->u) {
    if (h->u > 1 && !(h->d2[q] - h->d1[q] > 1e-6f * h->d2[q])) {
      scan(b, kids, 0, h->u, x, best, bd);
      b.host_scans++;
    } else {
      best = kids[h->lab[q]];
      bd = sq_dist(x, &b.ref[(size_t)best * b.d], b.d);
    }
    scan(b, kids, h->u, kids.size(), x, best, bd);
  } else {
    scan(b, kids, 0, kids.size(), x, best, bd);
  }
}

// w copies of x; hints (nullable) for point q of the block.
inline void insert_point(Core& b, const float* x, double w, const std::vector<NodeHints>* hints,
                         int64_t q) {
  const int d = b.d;
  std::vector<double> xd(d), tmp(d);
  for (int j = 0; j < d; ++j) xd[j] = (double)x[j];
  const double qn = sq_norm(xd.data(), d);
  int32_t parent = -1;
  int level = 1;
  while (w > 0) {
    int32_t best;
    double bd;
    closest(b, parent, x, hints, q, best, bd);
    if (best < 0 || bd > radius2(b, level)) {
      for (int j = 0; j < d; ++j) tmp[j] = w * xd[j];
      open_feature(b, x, w, tmp.data(), w * qn, level, parent);
      break;
    }
    Feature& F = b.f[best];
    double* S = &b.S[(size_t)best * d];
    const double s = F.W;
    const double c = F.Q - sq_norm(S, d) / s;
    double D = 0.0;
    for (int j = 0; j < d; ++j) {
      const double t = xd[j] - S[j] / s;
      D += t * t;
    }
    const double den = s * D - b.T + c;
    double wp = w;
    if (den > 0) wp = std::min(w, std::floor((s * b.T - s * c) / den));
    if (wp > 0) {
      F.W += wp;
      for (int j = 0; j < d; ++j) S[j] += wp * xd[j];
      F.Q += wp * qn;
      w -= wp;
    }
    parent = best;
    ++level;
  }
}

// Rebuild: T doubles and every feature is re-inserted into an empty tree.
// query(refs, nq, hints) may fill search hints for the nq references of a
// block (for the nodes hint_nodes names at the block's start; return false
// for an error; no hints is always correct).
template <class Query>
bool rebuild(Core& b, int64_t block, Query&& query) {
  const int d = b.d;
  const std::vector<int32_t> order = bfs(b);
  std::vector<Feature> of;
  of.swap(b.f);
  std::vector<double> oS;
  oS.swap(b.S);
  std::vector<float> oref;
  oref.swap(b.ref);
  b.roots.clear();
  b.T *= 2.0;
  b.rebuilds++;
  const int64_t nold = (int64_t)order.size();
  std::vector<float> stage((size_t)block * d);
  std::vector<NodeHints> hints;
  std::vector<double> mS(d);
  for (int64_t q0 = 0; q0 < nold; q0 += block) {
    const int64_t nq = std::min(block, nold - q0);
    for (int64_t q = 0; q < nq; ++q)
      std::memcpy(&stage[(size_t)q * d], &oref[(size_t)order[q0 + q] * d],
                  (size_t)d * sizeof(float));
    hints.clear();
    if (!b.roots.empty() && !query(stage.data(), nq, hints)) return false;
    for (int64_t q = 0; q < nq; ++q) {
      const int32_t o = order[q0 + q];
      const float* r = &oref[(size_t)o * d];
      const double* Sf = &oS[(size_t)o * d];
      int32_t parent = -1;
      int level = 1;
      while (true) {
        int32_t best;
        double bd;
        closest(b, parent, r, &hints, q, best, bd);
        if (best < 0 || bd > radius2(b, level)) {
          open_feature(b, r, of[o].W, Sf, of[o].Q, level, parent);
          break;
        }
        Feature& G = b.f[best];
        double* Sg = &b.S[(size_t)best * d];
        const double W = G.W + of[o].W;
        const double Q = G.Q + of[o].Q;
        for (int j = 0; j < d; ++j) mS[j] = Sg[j] + Sf[j];
        if (Q - sq_norm(mS.data(), d) / W <= b.T) {
          G.W = W;
          G.Q = Q;
          std::memcpy(Sg, mS.data(), (size_t)d * sizeof(double));
          break;
        }
        parent = best;
        ++level;
      }
    }
  }
  return true;
}

}  // namespace bico
}  // namespace kmx
