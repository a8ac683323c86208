// CPU harness of the BICO host logic (paper_1502_04265_amd/csrc/bico_core.h)
// for tests/test_bico_host.py: inserts the rows of an input file block by
// block as the library does, with search hints from a host stand-in for the
// device search (FP64 argmin over the children each hinted node had when the
// block started, distances rounded to FP32), and writes the features in
// breadth-first order.
//   input : int64 n, int32 d, int64 m, double T0, int32 block, int32 has_w,
//           float32 X[n][d], float64 w[n] (when has_w)
//   output: int64 count, double T, int64 rebuilds, int64 host_scans, then per
//           feature int32 level, double W, double Q, float32 ref[d],
//           float64 S[d]
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "bico_core.h"

using namespace kmx::bico;

// Hints for the nodes hint_nodes names: the FP64 argmin over each node's
// children, distances rounded to FP32 (a stand-in for the device search).
static void hints_for(const Core& c, const float* rows, int64_t nq, std::vector<NodeHints>& out) {
  out.clear();
  for (int32_t node : hint_nodes(c)) {
    const std::vector<int32_t>& kids = kids_of(c, node);
    NodeHints h;
    h.node = node;
    h.u = kids.size();
    h.lab.assign(nq, 0);
    h.d1.assign(nq, 0.f);
    h.d2.assign(nq, 0.f);
    for (int64_t q = 0; q < nq; ++q) {
      const float* x = rows + (size_t)q * c.d;
      int32_t best = -1;
      double b1 = 0.0, b2 = 1e300;
      for (size_t r = 0; r < kids.size(); ++r) {
        const double dd = sq_dist(x, &c.ref[(size_t)kids[r] * c.d], c.d);
        if (best < 0 || dd < b1) {
          b2 = best < 0 ? 1e300 : b1;
          b1 = dd;
          best = (int32_t)r;
        } else if (dd < b2) {
          b2 = dd;
        }
      }
      h.lab[q] = best;
      h.d1[q] = (float)b1;
      h.d2[q] = b2 >= 1e300 ? __builtin_inff() : (float)b2;
    }
    out.push_back(std::move(h));
  }
}

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* in = std::fopen(argv[1], "rb");
  if (!in) return 3;
  int64_t n, m;
  int32_t d, block, has_w;
  double T0;
  if (std::fread(&n, 8, 1, in) != 1 || std::fread(&d, 4, 1, in) != 1 ||
      std::fread(&m, 8, 1, in) != 1 || std::fread(&T0, 8, 1, in) != 1 ||
      std::fread(&block, 4, 1, in) != 1 || std::fread(&has_w, 4, 1, in) != 1)
    return 4;
  std::vector<float> X((size_t)n * d);
  std::vector<double> w(n, 1.0);
  if (std::fread(X.data(), 4, X.size(), in) != X.size()) return 5;
  if (has_w && std::fread(w.data(), 8, n, in) != (size_t)n) return 6;
  std::fclose(in);

  Core c;
  c.d = d;
  c.m = m;
  c.T = T0;
  std::vector<NodeHints> hints;
  int64_t i0 = 0;
  while (i0 < n) {
    const int64_t nb = std::min<int64_t>(block, n - i0);
    hints_for(c, &X[(size_t)i0 * d], nb, hints);
    int64_t done = 0;
    for (int64_t q = 0; q < nb; ++q) {
      done = q + 1;
      if (w[i0 + q] == 0.0) continue;
      insert_point(c, &X[(size_t)(i0 + q) * d], w[i0 + q], &hints, q);
      if ((int64_t)c.f.size() > c.m) {
        while ((int64_t)c.f.size() > c.m)
          rebuild(c, 7, [&](const float* refs, int64_t nq, std::vector<NodeHints>& h) {
            hints_for(c, refs, nq, h);
            return true;
          });
        break;
      }
    }
    i0 += done;
  }

  FILE* out = std::fopen(argv[2], "wb");
  if (!out) return 7;
  const int64_t cnt = (int64_t)c.f.size();
  std::fwrite(&cnt, 8, 1, out);
  std::fwrite(&c.T, 8, 1, out);
  std::fwrite(&c.rebuilds, 8, 1, out);
  std::fwrite(&c.host_scans, 8, 1, out);
  for (int32_t id : bfs(c)) {
    std::fwrite(&c.f[id].level, 4, 1, out);
    std::fwrite(&c.f[id].W, 8, 1, out);
    std::fwrite(&c.f[id].Q, 8, 1, out);
    std::fwrite(&c.ref[(size_t)id * d], 4, d, out);
    std::fwrite(&c.S[(size_t)id * d], 8, d, out);
  }
  std::fclose(out);
  return 0;
}
