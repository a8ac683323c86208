// Weighted k-means++ seeding (Sec. 1: first center uniformly at random, each
// further center with probability proportional to the squared distance to the
// closest chosen center; Sec. 2.2: run on the weighted summary, a weight-w
// point standing for w copies as in Sec. 2.3.1).
//
// One launch per round r.  Every block streams its rows of X once: for r >= 1
// it lowers D2_i to ||x_i - c_{r-1}||^2 (FP64 direct differences of the FP32
// inputs, exact up to the final sums) and writes the FP64 block sum of
// w_i * D2_i (r = 0: of w_i).  A row is read by a group of G lanes, lane s
// taking the 16-byte chunks s, s + G, ... of the row; a lane keeps the NV
// loads of its group's next row in flight while it reduces the current row,
// and the previous center's chunks stay in registers as FP64 for the whole
// block (NV = 0: rows wider than 512 chunks, one row at a time, the center
// re-read from the cache).  The last block to finish (atomic
// ticket) draws u_r from SplitMix64, finds the first block whose inclusive
// prefix of block sums strictly exceeds u_r * M, then the first row inside it
// (each search: every thread sums a contiguous slice, one block scan, one
// thread walks the slice that crosses), copies that row into C and marks it
// chosen.  If the mass M is zero it draws by weight among the rows not chosen
// yet.
#include "kmx_device.h"
#include "kmx_internal.h"

namespace kmx {

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t r) {
  // state after r + 1 increments of the golden-ratio constant, then the mix
  uint64_t z = seed + (r + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Inclusive scan of doubles over the 256 threads of a block (fixed order).
// Uses sh[0..3]; contains barriers, so every thread must call it.
__device__ double block_incl_scan_256(double v, double* sh) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double x = v;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const double y = __shfl_up(x, m, 64);
    if (lane >= m) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  double add = 0.0;
  for (int q = 0; q < w; ++q) add += sh[q];
  __syncthreads();
  return add + x;
}

// Sum over the 256 threads of a block in a fixed order.  Uses sh[0..3].
__device__ double block_sum_256(double v, double* sh) {
  v = wave_sum_f64(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  const double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  __syncthreads();
  return r;
}

// First i in [lo, hi) whose inclusive prefix of mass(.) strictly exceeds
// target (prefixes scanned 256 entries at a time).  If rounding leaves no such
// i, the last i with positive mass; if there is none, -1.  *excl receives the
// exclusive prefix at the returned index when it was a strict hit.
// Uses sh[0..7]; every thread must call it.
template <typename F>
__device__ int64_t pick_linear(int64_t lo, int64_t hi, double target, F mass, double* sh,
                               unsigned long long* red, double* excl) {
  double carry = 0.0;
  if (threadIdx.x == 0) {
    red[0] = ~0ull;
    red[1] = 0ull;
  }
  __syncthreads();
  for (int64_t s = lo; s < hi; s += 256) {
    const int64_t i = s + threadIdx.x;
    const double v = (i < hi) ? mass(i) : 0.0;
    const double inc = block_incl_scan_256(v, sh) + carry;
    if (i < hi && inc > target) atomicMin(&red[0], (unsigned long long)i);
    if (i < hi && v > 0.0) atomicMax(&red[1], (unsigned long long)(i + 1));
    if (threadIdx.x == 255) sh[4] = inc;
    __syncthreads();
    const unsigned long long f = red[0];
    if (f != ~0ull && (int64_t)f == i) sh[5] = inc - v;
    carry = sh[4];
    __syncthreads();
    if (f != ~0ull) {
      if (excl) *excl = sh[5];
      __syncthreads();
      return (int64_t)f;
    }
  }
  return (int64_t)red[1] - 1;
}

// The same search in two levels: thread t sums the contiguous slice
// [lo + t per, lo + (t + 1) per) in index order, one block scan gives the
// slices' prefixes, and the first thread whose inclusive prefix exceeds
// target walks its slice again from its exclusive prefix.  If the walk finds
// no crossing (the scan and the walk round differently), the last index with
// positive mass in that slice; with no crossing anywhere, the last index with
// positive mass; if there is none, -1.  Uses sh[0..3]; every thread must
// call it.
template <typename F>
__device__ int64_t pick_sliced(int64_t lo, int64_t hi, double target, F mass, double* sh,
                               unsigned long long* red, double* excl) {
  __shared__ double sinc[256];
  __shared__ long long spick;
  __shared__ double sbefore;
  const int t = threadIdx.x;
  const int64_t per = (hi - lo + 255) / 256;
  const int64_t a = min(hi, lo + (int64_t)t * per), b = min(hi, a + per);
  double loc = 0.0;
  int64_t lastpos = -1;
  for (int64_t i = a; i < b; ++i) {
    const double v = mass(i);
    loc += v;
    if (v > 0.0) lastpos = i;
  }
  if (t == 0) {
    red[0] = ~0ull;
    red[1] = 0ull;
    spick = -1;
  }
  const double inc = block_incl_scan_256(loc, sh);   // barriers order the resets above
  sinc[t] = inc;
  if (b > a && inc > target) atomicMin(&red[0], (unsigned long long)t);
  if (lastpos >= 0) atomicMax(&red[1], (unsigned long long)(lastpos + 1));
  __syncthreads();
  const unsigned long long ts = red[0];
  if (ts != ~0ull && (unsigned long long)t == ts) {
    double run = (t > 0) ? sinc[t - 1] : 0.0;
    int64_t found = -1;
    for (int64_t i = a; i < b; ++i) {
      const double nr = run + mass(i);
      if (nr > target) {
        found = i;
        break;
      }
      run = nr;
    }
    if (found < 0) found = lastpos;
    spick = found;
    sbefore = run;
  }
  __syncthreads();
  int64_t pick = spick;
  const bool hit = ts != ~0ull && pick >= 0;
  if (!hit) pick = (int64_t)red[1] - 1;
  if (excl && hit) *excl = sbefore;
  __syncthreads();
  return pick;
}

typedef __attribute__((ext_vector_type(4))) float sf32x4_t;

// Chunk q (elements 4q .. 4q + 3) of a row of length d; zeros past the row.
template <bool VEC>
__device__ __forceinline__ sf32x4_t load_chunk(const float* p, int q, int d, bool valid) {
  sf32x4_t v = {0.f, 0.f, 0.f, 0.f};
  if (!valid) return v;
  if (VEC) return *(const sf32x4_t*)(p + 4 * q);
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (4 * q + e < d) v[e] = p[4 * q + e];
  return v;
}

// Round r's draw, by the last block of a round (every thread calls it):
// u_r from SplitMix64, the first block whose inclusive prefix of the block
// masses part[0 .. nb) strictly exceeds u_r M, then the first row inside it
// (rpb rows per block); with zero mass a draw by weight among the rows not
// chosen yet, and with no positive weight left the first row not chosen.
// Writes row `pick` into C (row r), idx_out[r] (nullable) and chosen.
__device__ void seed_draw(const float* __restrict__ X, int64_t n, int d, int64_t ldx,
                          const float* __restrict__ w, int r, uint64_t seed,
                          const double* __restrict__ D2, uint8_t* __restrict__ chosen,
                          const double* part, int nb, int64_t rpb, float* __restrict__ C,
                          int64_t* __restrict__ idx_out, double* sh, unsigned long long* red) {
  const volatile double* pv = part;
  const uint64_t z = splitmix64_at(seed, (uint64_t)r);
  const double u = (double)(z >> 11) * 0x1.0p-53;
  double t = 0.0;
  for (int q = threadIdx.x; q < nb; q += 256) t += pv[q];
  const double M = block_sum_256(t, sh);
  int64_t pick = -1;
  if (M > 0.0) {
    const double target = u * M;
    double before = 0.0;
    int64_t qb = pick_sliced(0, nb, target, [&](int64_t q) { return pv[q]; }, sh, red, &before);
    if (qb >= 0) {
      const int64_t b0 = qb * rpb;
      const int64_t b1 = min(n, b0 + rpb);
      const double tin = target - before;
      if (r == 0) {
        pick = pick_sliced(b0, b1, tin, [&](int64_t i) { return w ? (double)w[i] : 1.0; }, sh,
                           red, nullptr);
      } else {
        pick = pick_sliced(b0, b1, tin,
                           [&](int64_t i) { return (w ? (double)w[i] : 1.0) * D2[i]; }, sh,
                           red, nullptr);
      }
    }
  }
  if (pick < 0) {
    // zero mass: draw by weight among the rows not chosen yet
    double tt = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256)
      tt += chosen[i] ? 0.0 : (w ? (double)w[i] : 1.0);
    const double M2 = block_sum_256(tt, sh);
    if (M2 > 0.0) {
      pick = pick_linear(0, n, u * M2,
                         [&](int64_t i) { return chosen[i] ? 0.0 : (w ? (double)w[i] : 1.0); },
                         sh, red, nullptr);
    }
    if (pick < 0) {
      // no positive weight left: the first row not chosen yet (else row 0)
      if (threadIdx.x == 0) red[0] = ~0ull;
      __syncthreads();
      for (int64_t i = threadIdx.x; i < n; i += 256)
        if (!chosen[i]) atomicMin(&red[0], (unsigned long long)i);
      __syncthreads();
      const unsigned long long f = red[0];
      pick = (f == ~0ull) ? 0 : (int64_t)f;
    }
  }
  __syncthreads();
  // ---- 3. write the center (an exact copy of the row) ----
  const float* xs = X + pick * ldx;
  float* cr = C + (int64_t)r * d;
  for (int q = threadIdx.x; q < d; q += 256) cr[q] = xs[q];
  if (threadIdx.x == 0) {
    chosen[pick] = 1;
    if (idx_out) idx_out[r] = pick;
  }
}

template <int G, int NV, bool VEC>
__global__ __launch_bounds__(256) void seed_round_kernel(
    const float* __restrict__ X, int64_t n, int d, int64_t ldx, const float* __restrict__ w,
    int r, uint64_t seed, double* __restrict__ D2, uint8_t* __restrict__ chosen,
    double* __restrict__ part, unsigned int* __restrict__ ctr, float* __restrict__ C,
    int64_t* __restrict__ idx_out, int64_t rpb, int32_t* __restrict__ sa,
    const double* __restrict__ cc2, int* __restrict__ nread,
    unsigned long long* __restrict__ rows_read) {
  __shared__ double sh[8];
  __shared__ unsigned long long red[2];
  __shared__ unsigned int ticket;
  constexpr int NG = 256 / G;          // lane groups (rows in flight) per block
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int sub = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  const int64_t r0 = (int64_t)b * rpb;
  const int64_t r1 = min(n, r0 + rpb);
  const int nch = (d + 3) >> 2;

  // ---- 1. lower D2 against the previous center; block mass ----
  double macc = 0.0;
  if (r == 0) {
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) macc += w ? (double)w[i] : 1.0;
  } else {
    // Rows that need the distance to c = c_{r-1}: all of them in round 1;
    // afterwards a row whose nearest chosen center c_a (index sa) satisfies
    // ||c - c_a||^2 >= 4 D2 (1 + 1e-8) keeps its D2 (triangle inequality:
    // ||x - c|| >= ||c - c_a|| - ||x - c_a|| >= ||x - c_a||, with room for the
    // FP64 rounding of both distances; cc2 is rounded down), so its row is
    // not read.  The rows that need it are listed in row order (ballots), so
    // every sum keeps a fixed order.
    __shared__ int slist[kSeedRows];
    __shared__ int wtot[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int cnt = 0;
    for (int64_t s0 = r0; s0 < r1; s0 += 256) {
      const int64_t i = s0 + threadIdx.x;
      bool need = false;
      if (i < r1) {
        need = true;
        if (r >= 2) {
          const double dv = D2[i];
          if (cc2[sa[i]] >= 4.0 * dv * (1.0 + 1e-8)) {
            need = false;
            macc += w ? (double)w[i] * dv : dv;
          }
        }
      }
      const unsigned long long bal = __ballot(need);
      if (lane == 0) wtot[wv] = __popcll(bal);
      __syncthreads();
      int off = cnt;
      for (int q = 0; q < wv; ++q) off += wtot[q];
      if (need) slist[off + __popcll(bal & ((1ull << lane) - 1ull))] = (int)(i - r0);
      cnt += (wtot[0] + wtot[1]) + (wtot[2] + wtot[3]);
      __syncthreads();
    }
    const float* c = C + (int64_t)(r - 1) * d;
    double cd[NV > 0 ? NV : 1][4];
    if constexpr (NV > 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const sf32x4_t cv = load_chunk<false>(c, sub + G * v, d, sub + G * v < nch);
#pragma unroll
        for (int e = 0; e < 4; ++e) cd[v][e] = (double)cv[e];
      }
    }
    // NV > 0: the chunks of the group's next listed row are loaded while the
    // current one is reduced
    sf32x4_t xn[NV > 0 ? NV : 1];
    if constexpr (NV > 0) {
      const bool ok = grp < cnt;
      const int64_t i0 = ok ? r0 + slist[grp] : 0;
#pragma unroll
      for (int v = 0; v < NV; ++v)
        xn[v] = load_chunk<VEC>(X + i0 * ldx, sub + G * v, d, ok && sub + G * v < nch);
    }
    for (int jl = grp; jl < cnt; jl += NG) {
      const int64_t i = r0 + slist[jl];
      double acc = 0.0;
      if constexpr (NV > 0) {
        sf32x4_t xv[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) xv[v] = xn[v];
        const bool ok = jl + NG < cnt;
        const int64_t inx = ok ? r0 + slist[jl + NG] : 0;
#pragma unroll
        for (int v = 0; v < NV; ++v)
          xn[v] = load_chunk<VEC>(X + inx * ldx, sub + G * v, d, ok && sub + G * v < nch);
        double a4[4] = {0.0, 0.0, 0.0, 0.0};   // four independent FMA chains
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double df = (double)xv[v][e] - cd[v][e];
            a4[e] = fma(df, df, a4[e]);
          }
        acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
      } else {
        const float* x = X + i * ldx;
#pragma unroll 4
        for (int q = sub; q < nch; q += G) {
          const sf32x4_t xv = load_chunk<VEC>(x, q, d, true);
          const sf32x4_t cv = load_chunk<VEC>(c, q, d, true);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double df = (double)xv[e] - (double)cv[e];
            acc = fma(df, df, acc);
          }
        }
      }
      // butterfly over the group: every lane of it ends with the same bits
#pragma unroll
      for (int m = G / 2; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
      if (sub == 0) {
        const double old = (r == 1) ? 0.0 : D2[i];
        const bool closer = (r == 1) || acc < old;
        const double dv = closer ? acc : old;
        if (closer) sa[i] = r - 1;
        D2[i] = dv;
        macc += w ? (double)w[i] * dv : dv;
      }
    }
    if (threadIdx.x == 0) nread[b] = cnt;
  }
  const double bsum = block_sum_256(macc, sh);
  if (threadIdx.x == 0) {
    part[b] = bsum;
    __threadfence();
    ticket = atomicAdd(ctr, 1u);
  }
  __syncthreads();
  if (ticket != (unsigned)(nb - 1)) return;

  // ---- 2. the last block draws the row ----
  __threadfence();
  if (r >= 1 && rows_read) {
    const volatile int* nv = nread;
    long long t_read = 0;
    for (int q = threadIdx.x; q < nb; q += 256) t_read += nv[q];
    const double tr = block_sum_256((double)t_read, sh);
    if (threadIdx.x == 0) *rows_read += (unsigned long long)tr;
  }
  seed_draw(X, n, d, ldx, w, r, seed, D2, chosen, part, nb, rpb, C, idx_out, sh, red);
  if (threadIdx.x == 0) *ctr = 0u;
}

// Squared distances from the newest center c_{r-1} to the earlier centers,
// FP64 sums of the FP32 differences rounded down by 1e-12 relative (a lower
// bound on the exact value); one wave per earlier center.
__global__ __launch_bounds__(256) void center_gap_kernel(const float* __restrict__ C, int r,
                                                         int d, double* __restrict__ cc2) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= r - 1) return;   // uniform per wave
  const float* c = C + (int64_t)(r - 1) * d;
  const float* cj = C + (int64_t)j * d;
  double acc = 0.0;
  for (int q = lane; q < d; q += 64) {
    const double df = (double)c[q] - (double)cj[q];
    acc = fma(df, df, acc);
  }
  acc = wave_sum_f64(acc);
  if (lane == 0) cc2[j] = acc * (1.0 - 1e-12);
}

// ---------------------------------------------------------------------------
// Batched seeding: round r of every instance with k > r in one launch.
// Instances are ordered by decreasing k, so the active ones are a prefix and
// their blocks (kSeedRows rows each) a prefix of the block space; a block
// finds its instance by binary search on the first block indices.  Each
// block lowers D2 of its rows against the instance's center r - 1 (16 lanes
// per row, FP64 sums of the FP32 differences) and writes its block mass; from
// round 2 on a row whose closest chosen center c_a satisfies
// ||c_{r-1} - c_a||^2 >= 4 D2 (1 + 1e-8) keeps its D2 unread (the test of
// seed_round_kernel).  The instance's last block (its own atomic ticket)
// draws as seed_draw does for one instance.
// ---------------------------------------------------------------------------
// Squared gaps of every active instance's newest center c_{r-1} to its
// earlier centers (as center_gap_kernel): one wave per (instance, center).
__global__ __launch_bounds__(256) void seed_batched_gap_kernel(const SeedInst* __restrict__ insts,
                                                               int m, int r) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (g >= (int64_t)m * (r - 1)) return;   // uniform per wave
  const SeedInst& I = insts[g / (r - 1)];
  const int j = (int)(g % (r - 1));
  const float* c = I.C + (int64_t)(r - 1) * I.d;
  const float* cj = I.C + (int64_t)j * I.d;
  double acc = 0.0;
  for (int q = lane; q < I.d; q += 64) {
    const double df = (double)c[q] - (double)cj[q];
    acc = fma(df, df, acc);
  }
  acc = wave_sum_f64(acc);
  if (lane == 0) I.cc2[j] = acc * (1.0 - 1e-12);
}

hipError_t launch_seed_batched_gaps(hipStream_t s, const SeedInst* insts, int m, int r) {
  if (m <= 0 || r < 2) return hipSuccess;
  const int64_t waves = (int64_t)m * (r - 1);
  hipLaunchKernelGGL(seed_batched_gap_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s,
                     insts, m, r);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void seed_batched_round_kernel(const SeedInst* __restrict__ insts,
                                                                 int m, int r) {
  __shared__ double sh[8];
  __shared__ unsigned long long red[2];
  __shared__ unsigned int ticket;
  constexpr int G = 16, NG = 256 / G;
  int lo = 0, hi = m - 1;   // last instance whose first block is <= blockIdx.x
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (insts[mid].blk0 <= (int64_t)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const SeedInst I = insts[lo];
  const int b = (int)((int64_t)blockIdx.x - I.blk0);
  const int64_t rpb = kSeedRows;
  const int64_t r0 = (int64_t)b * rpb;
  const int64_t r1 = min(I.n, r0 + rpb);
  const int sub = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  const float* w = I.w;
  double macc = 0.0;
  if (r == 0) {
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) macc += w ? (double)w[i] : 1.0;
  } else {
    const float* c = I.C + (int64_t)(r - 1) * I.d;
    // whole 16-byte chunks when the rows and the centers are aligned
    const bool vec = (I.d % 4 == 0) && (I.ldx % 4 == 0) && ((((uintptr_t)I.X) & 15) == 0) &&
                     ((((uintptr_t)I.C) & 15) == 0);
    const int nch = (I.d + 3) >> 2;
    for (int64_t i = r0 + grp; i < r1; i += NG) {   // uniform within a lane group
      if (r >= 2) {
        const double dv = I.D2[i];
        if (I.cc2[I.sa[i]] >= 4.0 * dv * (1.0 + 1e-8)) {   // uniform within the group
          if (sub == 0) macc += w ? (double)w[i] * dv : dv;
          continue;
        }
      }
      const float* x = I.X + i * I.ldx;
      double acc = 0.0;
      if (vec) {
        // two chunks in flight per lane, four independent FMA chains
        double a4[4] = {0.0, 0.0, 0.0, 0.0};
        for (int q = sub; q < nch; q += 2 * G) {
          const bool two = q + G < nch;
          const sf32x4_t x0 = *(const sf32x4_t*)(x + 4 * q);
          const sf32x4_t c0 = *(const sf32x4_t*)(c + 4 * q);
          sf32x4_t x1 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
          if (two) {
            x1 = *(const sf32x4_t*)(x + 4 * (q + G));
            c1 = *(const sf32x4_t*)(c + 4 * (q + G));
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double df = (double)x0[e] - (double)c0[e];
            a4[e] = fma(df, df, a4[e]);
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double df = (double)x1[e] - (double)c1[e];
            a4[e] = fma(df, df, a4[e]);
          }
        }
        acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
      } else {
        for (int q = sub; q < I.d; q += G) {
          const double df = (double)x[q] - (double)c[q];
          acc = fma(df, df, acc);
        }
      }
#pragma unroll
      for (int msk = G / 2; msk >= 1; msk >>= 1) acc += __shfl_xor(acc, msk, 64);
      if (sub == 0) {
        const double old = (r == 1) ? 0.0 : I.D2[i];
        const bool closer = (r == 1) || acc < old;
        const double dv = closer ? acc : old;
        if (closer) I.sa[i] = r - 1;
        I.D2[i] = dv;
        macc += w ? (double)w[i] * dv : dv;
      }
    }
  }
  const double bsum = block_sum_256(macc, sh);
  if (threadIdx.x == 0) {
    I.part[b] = bsum;
    __threadfence();
    ticket = atomicAdd(I.ctr, 1u);
  }
  __syncthreads();
  if (ticket != (unsigned)(I.nb - 1)) return;
  __threadfence();
  seed_draw(I.X, I.n, I.d, I.ldx, w, r, I.seed, I.D2, I.chosen, I.part, I.nb, rpb, I.C, I.idx, sh,
            red);
  if (threadIdx.x == 0) *I.ctr = 0u;
}

hipError_t launch_seed_batched_round(hipStream_t s, const SeedInst* insts, int m, int r,
                                     int64_t blocks) {
  if (m <= 0 || blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(seed_batched_round_kernel, dim3((unsigned)blocks), dim3(256), 0, s, insts, m,
                     r);
  return hipGetLastError();
}

hipError_t launch_seed_round(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                             const float* w, int r, uint64_t seed, double* D2, uint8_t* chosen,
                             double* part, unsigned int* ctr, float* C_out, int64_t* idx_out,
                             int32_t* sa, double* cc2, int* nread,
                             unsigned long long* rows_read) {
  if (r >= 2) {
    hipLaunchKernelGGL(center_gap_kernel, dim3((unsigned)((r - 1 + 3) / 4)), dim3(256), 0, s,
                       C_out, r, d, cc2);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t rpb = kSeedRows;
  const int nb = (int)((n + rpb - 1) / rpb);
  const int nch = (d + 3) / 4;
  // whole 16-byte chunks: rows of X and of C start 16-byte aligned
  const bool vec = (d % 4 == 0) && (ldx % 4 == 0) && ((((uintptr_t)X) & 15) == 0) &&
                   ((((uintptr_t)C_out) & 15) == 0);
#define KMX_S(G_, NV_)                                                                           \
  do {                                                                                           \
    if (vec)                                                                                     \
      hipLaunchKernelGGL((seed_round_kernel<G_, NV_, true>), dim3(nb), dim3(256), 0, s, X, n, d, \
                         ldx, w, r, seed, D2, chosen, part, ctr, C_out, idx_out, rpb, sa, cc2,    \
                         nread, rows_read);                                                     \
    else                                                                                         \
      hipLaunchKernelGGL((seed_round_kernel<G_, NV_, false>), dim3(nb), dim3(256), 0, s, X, n,   \
                         d, ldx, w, r, seed, D2, chosen, part, ctr, C_out, idx_out, rpb, sa,     \
                         cc2, nread, rows_read);                                                \
    return hipGetLastError();                                                                    \
  } while (0)
  if (nch <= 16) KMX_S(4, 4);
  if (nch <= 32) KMX_S(8, 4);
  if (nch <= 64) KMX_S(16, 4);
  if (nch <= 128) KMX_S(16, 8);
  if (nch <= 256) KMX_S(32, 8);
  if (nch <= 512) KMX_S(64, 8);
  KMX_S(64, 0);
#undef KMX_S
}

}  // namespace kmx
