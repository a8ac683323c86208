// Candidate router and its certificate (inference side).
//
// The router is a two-layer perceptron  z = W2 relu(W1 x + b1) + b2  with
// H = 256 hidden units and one output per center, trained (k_train.hip) on
// the labels of earlier Lloyd iterations.  It proposes 16 candidate centers
// per point.  A proposal is used only under a triangle-inequality
// certificate (Elkan 2003): with b the proposal's best center and D an upper
// bound of ||x - c_b||, every center c with ||c_b - c|| >= 2 D satisfies
// ||x - c|| >= ||c_b - c|| - ||x - c_b|| >= D >= ||x - c_b||, so it cannot be
// closer than c_b.  The centers inside that radius are read from c_b's sorted
// neighbour list (a k x k table of lower bounds of the center distances,
// rebuilt for every center set).  No neighbour inside: c_b is the exact
// closest center.  One or two, all of them candidates: the exact short
// re-check decides between them and c_b.  Otherwise the row goes through the
// GEMM assignment.  Labels are therefore those of the assignment step
// (Sec. 1) whatever the network proposes; only the amount of GEMM work
// depends on it.
//
// Forward pass layout (gfx950 MFMA 16x16x32 BF16, FP32 accumulate).  As in
// the assignment GEMM, the point fragments stay in registers (B operand) and
// weight tiles stream through LDS (A operand).  Layer 1 turns 16 hidden
// units per tile into BF16 relu activations that remain in registers: lane l
// holds units 4(l/16)..4(l/16)+3 of each 16-unit tile, and two consecutive
// tiles form exactly the eight BF16 values the lane supplies for one 32-wide
// K unit of layer 2.  The layer-2 weight columns are stored in that
// permuted order, so no data moves between lanes.  The biases initialise the
// accumulators.
//
// Proposals.  Each lane keeps the four largest logits of the centers it
// sees, i.e. of one quarter of the centers (quarter q = (j mod 16) div 4).
// The 16 proposals of a point are these four per quarter: they contain the
// exact top four logits and, unless one quarter holds more than four of the
// top 16, the exact top 16.  Logits are ordered through the monotone map of
// float bits to unsigned integers; the low ib bits carry the center index.
#include "kmx_device.h"
#include "kmx_internal.h"

namespace kmx {

typedef __attribute__((ext_vector_type(8))) __bf16 rbf16x8_t;
typedef __attribute__((ext_vector_type(2))) __bf16 rbf16x2_t;
typedef __attribute__((ext_vector_type(4))) float rf32x4_t;
typedef __attribute__((ext_vector_type(4))) unsigned int ru32x4_t;

__device__ __forceinline__ unsigned r_med3(unsigned a, unsigned b, unsigned c) {
  return max(min(a, b), min(max(a, b), c));
}

__device__ __forceinline__ void r_top4(unsigned key, unsigned& v1, unsigned& v2, unsigned& v3,
                                       unsigned& v4) {
  const unsigned n1 = max(v1, key);
  const unsigned n2 = r_med3(v1, v2, key);
  const unsigned n3 = r_med3(v2, v3, key);
  const unsigned n4 = r_med3(v3, v4, key);
  v1 = n1;
  v2 = n2;
  v3 = n3;
  v4 = n4;
}

// Order-preserving map of float bit patterns onto unsigned integers.
__device__ __forceinline__ unsigned ordered_bits(float f) {
  const unsigned u = __float_as_uint(f);
  return u ^ ((unsigned)((int)u >> 31) | 0x80000000u);
}

template <int NKU, int NCG, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void router_fwd_kernel(
    const uint16_t* __restrict__ Xq, int64_t xs, int64_t n, const uint16_t* __restrict__ W1a,
    const float* __restrict__ b1, const uint16_t* __restrict__ W2a,
    const float* __restrict__ b2p, int kpad, int ib, uint32_t* __restrict__ keys,
    const int* __restrict__ rows, const unsigned long long* __restrict__ row_count,
    const int* __restrict__ gate) {
  if (gate && *gate) return;
  // with a row list: points 0 .. *row_count - 1 are the rows rows[p]
  if (rows) n = (int64_t)*row_count;
  constexpr int ROW1 = NKU * 64;                     // bytes of a W1a row
  constexpr int UROW1 = NKU * 4 + 1;                 // 16-byte units of a padded LDS row
  constexpr int PITCH1 = UROW1 * 16;
  constexpr int CH1 = (kRouterBN1 * UROW1 + 63) / 64;
  constexpr int ROW2 = kRouterHU * 64;               // bytes of a W2a row
  constexpr int UROW2 = kRouterHU * 4 + 1;
  constexpr int PITCH2 = UROW2 * 16;
  constexpr int CH2 = (kRouterBN2 * UROW2 + 63) / 64;
  constexpr int CHM = CH1 > CH2 ? CH1 : CH2;
  constexpr int NT1 = kRouterH / kRouterBN1;
  constexpr int RB2 = kRouterBN2 / 16;
  constexpr int PPB = WAVES * 16 * NCG;
  static_assert(NT1 % 2 == 0, "layer 2 starts on buffer 0");
  __shared__ __attribute__((aligned(1024))) unsigned char lds[2][CHM * 1024];
  __shared__ __attribute__((aligned(16))) float sb1[kRouterH];
  __shared__ __attribute__((aligned(16))) float sb2[kRouterMaxK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int prow = lane & 15;
  const int grp = lane >> 4;
  const int64_t nblk = (n + PPB - 1) / PPB;
  const int ntiles2 = kpad / kRouterBN2;
  const unsigned mask = (1u << ib) - 1u;

  for (int i = tid; i < kRouterH; i += WAVES * 64) sb1[i] = b1[i];
  for (int i = tid; i < kpad; i += WAVES * 64) sb2[i] = b2p[i];
  __syncthreads();

  // Direct-to-LDS copy of a tile of `nrows` rows (rowb bytes each) into LDS
  // rows of urow 16-byte units (one pad unit); lane l of chunk c carries the
  // padded unit c*64 + l.  Pad units re-load the tile's first unit.
  auto issue = [&](const unsigned char* base, int rowb, int urow, int nrows, int chunks,
                   int buf) {
    for (int c = wave; c < chunks; c += WAVES) {
      const int q = c * 64 + lane;
      const int row = q / urow;
      const int uc = q - row * urow;
      const unsigned char* src = (row < nrows && uc < urow - 1) ? base + row * rowb + uc * 16 : base;
      __builtin_amdgcn_global_load_lds(
          (const void*)src, (__attribute__((address_space(3))) void*)(&lds[buf][c * 1024]), 16,
          0, 0);
    }
  };

  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t p_base = blk * PPB + (int64_t)wave * (16 * NCG);
    ru32x4_t xf[NCG][NKU];
    int64_t src[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
      const int64_t p = p_base + cg * 16 + prow;
      const bool pv = p < n;
      src[cg] = pv ? (rows ? (int64_t)rows[p] : p) : -1;
#pragma unroll
      for (int ku = 0; ku < NKU; ++ku) {
        ru32x4_t v = {0u, 0u, 0u, 0u};
        if (pv) v = *(const ru32x4_t*)(Xq + src[cg] * xs + ku * 32 + grp * 8);
        xf[cg][ku] = v;
      }
    }

    // ---- layer 1: hidden activations, kept as layer-2 B fragments ----
    ru32x4_t hf[NCG][kRouterHU];
    issue((const unsigned char*)W1a, ROW1, UROW1, kRouterBN1, CH1, 0);
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT1; ++t) {
      const int buf = t & 1;
      if (t + 1 < NT1)
        issue((const unsigned char*)W1a + (t + 1) * kRouterBN1 * ROW1, ROW1, UROW1, kRouterBN1,
              CH1, buf ^ 1);
      else
        issue((const unsigned char*)W2a, ROW2, UROW2, kRouterBN2, CH2, buf ^ 1);
      const rf32x4_t bias = *(const rf32x4_t*)(&sb1[t * kRouterBN1 + grp * 4]);
      rf32x4_t acc[NCG];
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg) acc[cg] = bias;
      const unsigned char* abase = &lds[buf][prow * PITCH1 + grp * 16];
#pragma unroll
      for (int ku = 0; ku < NKU; ++ku) {
        const ru32x4_t a = *(const ru32x4_t*)(abase + ku * 64);
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg)
          acc[cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(rbf16x8_t, a), __builtin_bit_cast(rbf16x8_t, xf[cg][ku]),
              acc[cg], 0, 0, 0);
      }
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg) {
        const rbf16x2_t p0 = {(__bf16)fmaxf(acc[cg][0], 0.0f), (__bf16)fmaxf(acc[cg][1], 0.0f)};
        const rbf16x2_t p1 = {(__bf16)fmaxf(acc[cg][2], 0.0f), (__bf16)fmaxf(acc[cg][3], 0.0f)};
        hf[cg][t >> 1][(t & 1) * 2] = __builtin_bit_cast(unsigned, p0);
        hf[cg][t >> 1][(t & 1) * 2 + 1] = __builtin_bit_cast(unsigned, p1);
      }
      __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }

    // ---- layer 2: logits and the per-quarter top four ----
    unsigned v1[NCG], v2[NCG], v3[NCG], v4[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) v1[cg] = v2[cg] = v3[cg] = v4[cg] = 0u;
    for (int t2 = 0; t2 < ntiles2; ++t2) {
      const int buf = t2 & 1;
      if (t2 + 1 < ntiles2)
        issue((const unsigned char*)W2a + (int64_t)(t2 + 1) * kRouterBN2 * ROW2, ROW2, UROW2,
              kRouterBN2, CH2, buf ^ 1);
      rf32x4_t acc[NCG][RB2];
#pragma unroll
      for (int rb = 0; rb < RB2; ++rb) {
        const rf32x4_t bias = *(const rf32x4_t*)(&sb2[t2 * kRouterBN2 + rb * 16 + grp * 4]);
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) acc[cg][rb] = bias;
      }
      const unsigned char* abase = &lds[buf][prow * PITCH2 + grp * 16];
#pragma unroll
      for (int u = 0; u < kRouterHU; ++u) {
#pragma unroll
        for (int rb = 0; rb < RB2; ++rb) {
          const ru32x4_t a = *(const ru32x4_t*)(abase + rb * 16 * PITCH2 + u * 64);
#pragma unroll
          for (int cg = 0; cg < NCG; ++cg)
            acc[cg][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(rbf16x8_t, a), __builtin_bit_cast(rbf16x8_t, hf[cg][u]),
                acc[cg][rb], 0, 0, 0);
        }
      }
      const unsigned ibase = mask - (unsigned)(t2 * kRouterBN2 + grp * 4);
#pragma unroll
      for (int rb = 0; rb < RB2; ++rb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const unsigned idx = ibase - (unsigned)(rb * 16 + i);
#pragma unroll
          for (int cg = 0; cg < NCG; ++cg) {
            const unsigned key = (ordered_bits(acc[cg][rb][i]) & ~mask) | (idx & mask);
            r_top4(key, v1[cg], v2[cg], v3[cg], v4[cg]);
          }
        }
      }
      __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }

#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
      if (src[cg] >= 0) {
        const ru32x4_t o = {v1[cg], v2[cg], v3[cg], v4[cg]};
        *(ru32x4_t*)(keys + src[cg] * kRouterM + grp * 4) = o;
      }
    }
  }
}

// Rows of the list rows[0 .. *count) whose proposals were not computed yet in
// this run (have[row] == 0): marked and appended to out (positions from one
// atomic per wave; any order).  *out_count must be zero before.
__global__ __launch_bounds__(256) void need_proposals_kernel(const int* __restrict__ rows,
                                                             const unsigned long long* __restrict__ count,
                                                             uint8_t* __restrict__ have,
                                                             int* __restrict__ out,
                                                             unsigned long long* __restrict__ out_count,
                                                             const int* __restrict__ gate) {
  if (gate && *gate) return;
  const int64_t m = (int64_t)*count;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
    const int64_t q = base + threadIdx.x;
    int r = -1;
    bool need = false;
    if (q < m) {
      r = rows[q];
      need = have[r] == 0;
      if (need) have[r] = 1;
    }
    const unsigned long long bal = __ballot(need);
    if (bal == 0ull) continue;
    const int first = __ffsll((long long)bal) - 1;
    unsigned long long pos = 0;
    if (lane == first) pos = atomicAdd(out_count, (unsigned long long)__popcll(bal));
    pos = __shfl(pos, first, 64);
    if (need) out[pos + __popcll(bal & ((1ull << lane) - 1ull))] = r;
  }
}

hipError_t launch_need_proposals(hipStream_t s, const int* rows, const unsigned long long* count,
                                 int64_t max_rows, uint8_t* have, int* out,
                                 unsigned long long* out_count, const int* gate, int num_cus) {
  int64_t blocks = (max_rows + 255) / 256;
  if (blocks > (int64_t)num_cus * 4) blocks = (int64_t)num_cus * 4;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(need_proposals_kernel, dim3((unsigned)blocks), dim3(256), 0, s, rows, count,
                     have, out, out_count, gate);
  return hipGetLastError();
}

// Units of 32 BF16 columns the forward pass reads from each row of the
// quantized X (dp columns): the smallest instantiated count covering d.
static const int kRouterUnits[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};

int router_units(int d, int dp) {
  const int need = (d + 31) / 32;
  for (int u : kRouterUnits)
    if (u >= need && u * 32 <= dp) return u;
  return -1;
}

template <int NKU, int NCG, int WAVES>
static hipError_t run_router_fwd(hipStream_t s, const uint16_t* Xq, int64_t xs, int64_t n,
                                 const uint16_t* W1a, const float* b1, const uint16_t* W2a,
                                 const float* b2p, int kpad, int ib, uint32_t* keys,
                                 const int* rows, const unsigned long long* row_count,
                                 const int* gate, int num_cus) {
  const int64_t ppb = (int64_t)WAVES * 16 * NCG;
  int64_t blocks = (n + ppb - 1) / ppb;
  const int64_t cap = (int64_t)num_cus * 2;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((router_fwd_kernel<NKU, NCG, WAVES>), dim3((unsigned)blocks),
                     dim3(WAVES * 64), 0, s, Xq, xs, n, W1a, b1, W2a, b2p, kpad, ib, keys, rows,
                     row_count, gate);
  return hipGetLastError();
}

hipError_t launch_router_fwd(hipStream_t s, const uint16_t* Xq, int64_t dp, int64_t n, int d,
                             const uint16_t* W1a, const float* b1, const uint16_t* W2a,
                             const float* b2p, int kpad, uint32_t* keys, const int* gate,
                             int num_cus, const int* rows, const unsigned long long* row_count) {
  if (kpad % kRouterBN2 != 0 || kpad > kRouterMaxK) return hipErrorInvalidValue;
  int ib = 1;
  while ((1 << ib) < kpad) ++ib;
  switch (router_units(d, (int)dp)) {
// Two point groups per wave keep both layers' fragments in registers; for 8
// and 16 units that needs more than the 256 registers of two waves per SIMD,
// so those run one wave per SIMD (four waves per workgroup).
#define KMX_R(U, G, W)                                                                     \
  case U:                                                                                  \
    return run_router_fwd<U, G, W>(s, Xq, dp, n, W1a, b1, W2a, b2p, kpad, ib, keys, rows, \
                                   row_count, gate, num_cus)
    KMX_R(1, 2, 8);
    KMX_R(2, 2, 8);
    KMX_R(3, 2, 8);
    KMX_R(4, 2, 8);
    KMX_R(6, 2, 8);
    KMX_R(8, 2, 4);
    KMX_R(12, 2, 8);
    KMX_R(16, 2, 4);
    KMX_R(24, 1, 8);
    KMX_R(32, 1, 8);
#undef KMX_R
    default:
      return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Inference layouts of the network from the FP32 parameters.
//   W1a[h][c] = bf16(W1[h][c]) for c < d, 0 up to the row length r1;
//   W2a[j][p] = bf16(W2[j][pi(p)]), p = 32u + 8g + e, pi(p) = 32u + 4g + e
//               for e < 4 and 32u + 16 + 4g + (e - 4) otherwise; zero rows
//               for padding centers;
//   b2p[j]    = b2[j], -inf for padding centers.
// ---------------------------------------------------------------------------
__global__ void router_layout_kernel(const float* __restrict__ W1, const float* __restrict__ W2,
                                     const float* __restrict__ b2, int d, int k, int kpad, int r1,
                                     uint16_t* __restrict__ W1a, uint16_t* __restrict__ W2a,
                                     float* __restrict__ b2p) {
  const int64_t n1 = (int64_t)kRouterH * r1;
  const int64_t n2 = (int64_t)kpad * kRouterH;
  const int64_t total = n1 + n2 + kpad;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n1) {
      const int h = (int)(i / r1), c = (int)(i % r1);
      W1a[i] = (c < d) ? f32_to_bf16_rne(W1[(int64_t)h * d + c]) : (uint16_t)0;
    } else if (i < n1 + n2) {
      const int64_t e2 = i - n1;
      const int j = (int)(e2 / kRouterH), p = (int)(e2 % kRouterH);
      const int u = p >> 5, g = (p >> 3) & 3, e = p & 7;
      const int h = 32 * u + (e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4));
      W2a[e2] = (j < k) ? f32_to_bf16_rne(W2[(int64_t)j * kRouterH + h]) : (uint16_t)0;
    } else {
      const int j = (int)(i - n1 - n2);
      b2p[j] = (j < k) ? b2[j] : -__builtin_inff();
    }
  }
}

hipError_t launch_router_layout(hipStream_t s, const float* W1, const float* W2, const float* b2,
                                int d, int k, int kpad, int r1, uint16_t* W1a, uint16_t* W2a,
                                float* b2p) {
  const int64_t total = (int64_t)kRouterH * r1 + (int64_t)kpad * kRouterH + kpad;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(router_layout_kernel, dim3((unsigned)blocks), dim3(256), 0, s, W1, W2, b2, d,
                     k, kpad, r1, W1a, W2a, b2p);
  return hipGetLastError();
}

// Proposals as center indices (-1 where a quarter had fewer than four
// centers): cand[i][4q + r] is the r-th best of quarter q.
__global__ void router_decode_kernel(const uint32_t* __restrict__ keys, int64_t count, int k,
                                     int ib, int32_t* __restrict__ cand) {
  const unsigned mask = (1u << ib) - 1u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(mask - (keys[i] & mask));
    cand[i] = (j < k) ? j : -1;
  }
}

hipError_t launch_router_decode(hipStream_t s, const uint32_t* keys, int64_t count, int k,
                                int kpad, int32_t* cand) {
  int ib = 1;
  while ((1 << ib) < kpad) ++ib;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(router_decode_kernel, dim3((unsigned)blocks), dim3(256), 0, s, keys, count, k,
                     ib, cand);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Center-distance table.  Pass 1 on the matrix cores: D[b][c] = a lower bound
// of ||c_b - c_c|| from the Gram form ||c_b||^2 + ||c_c||^2 - 2 g, g = c_b . c_c.
// A workgroup takes a 32 x 32 tile of center pairs (tiles on and above the
// diagonal; an off-diagonal tile also writes its transpose), stages 128
// columns of both center blocks at a time in LDS, and its four waves form g
// for 16 x 16 pairs each with FP32 MFMAs (16x16x4).  The accumulated g is
// within gamma ||c_b|| ||c_c|| of the exact product, gamma = K 2^-23 / (1 -
// K 2^-23) with K = (columns rounded up to 128) + 1 (every accumulation step
// faithfully rounded, as for the assignment's FP32 pass); the squared norms
// are FP64 sums of the staged FP32 values (relative error below 2^-40 for any
// d this path takes).  So sqrt(||c_b||^2 + ||c_c||^2 - 2 g - 2 gamma ||c_b||
// ||c_c||), less a 2^-38 relative slack for the FP64 steps and rounded down,
// is a lower bound.  Pass 2 (a workgroup per center): the kNbrL nearest other
// centers sorted by that bound ((bound, index) keys), and the bound of the
// next one (+inf when none).
// ---------------------------------------------------------------------------
constexpr int kGramT = 32;    // centers per tile side
constexpr int kGramK = 128;   // staged columns
constexpr int kGramP = kGramK + 4;   // padded LDS row (conflict-free column reads)

__global__ __launch_bounds__(256) void center_gram_kernel(const float* __restrict__ C, int k, int d,
                                                          float* __restrict__ D,
                                                          const int* __restrict__ gate) {
  if (gate && *gate) return;
  const int T = (k + kGramT - 1) / kGramT;
  int rem = (int)blockIdx.x, bi = 0;   // block -> tile (bi, ci), bi <= ci
  while (rem >= T - bi) {
    rem -= T - bi;
    ++bi;
  }
  const int ci = bi + rem;
  const int b0 = bi * kGramT, c0 = ci * kGramT;
  __shared__ __attribute__((aligned(16))) float Bs[kGramT * kGramP];
  __shared__ __attribute__((aligned(16))) float Cs[kGramT * kGramP];
  __shared__ double nB[kGramT], nC[kGramT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 16, wc = (wave & 1) * 16;   // the wave's 16 x 16 pairs
  const int lr = lane & 15, lk = lane >> 4;
  // staging: thread t holds row t / 8, columns 16 (t % 8) .. + 15 of the chunk
  const int sr = tid >> 3, sk = (tid & 7) * 16;
  const bool vb_row = b0 + sr < k, vc_row = c0 + sr < k;
  const float* brow = C + (int64_t)(vb_row ? b0 + sr : 0) * d;
  const float* crow = C + (int64_t)(vc_row ? c0 + sr : 0) * d;
  const bool vec = ((((uintptr_t)C) & 15) == 0) && (d % 4 == 0);
  rf32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  double pb[2] = {0.0, 0.0}, pc[2] = {0.0, 0.0};
  for (int k0 = 0; k0 < d; k0 += kGramK) {
    float vb[16], vc[16];
    if (vec && k0 + sk + 16 <= d) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 a = vb_row ? *(const float4*)(brow + k0 + sk + 4 * q) : make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 c = vc_row ? *(const float4*)(crow + k0 + sk + 4 * q) : make_float4(0.f, 0.f, 0.f, 0.f);
        vb[4 * q] = a.x; vb[4 * q + 1] = a.y; vb[4 * q + 2] = a.z; vb[4 * q + 3] = a.w;
        vc[4 * q] = c.x; vc[4 * q + 1] = c.y; vc[4 * q + 2] = c.z; vc[4 * q + 3] = c.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int kc = k0 + sk + e;
        vb[e] = (vb_row && kc < d) ? brow[kc] : 0.0f;
        vc[e] = (vc_row && kc < d) ? crow[kc] : 0.0f;
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      Bs[sr * kGramP + sk + e] = vb[e];
      Cs[sr * kGramP + sk + e] = vc[e];
      pb[e & 1] = fma((double)vb[e], (double)vb[e], pb[e & 1]);
      pc[e & 1] = fma((double)vc[e], (double)vc[e], pc[e & 1]);
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kGramK; kk += 4) {
      const float a = Bs[(wr + lr) * kGramP + kk + lk];
      const float b = Cs[(wc + lr) * kGramP + kk + lk];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // squared norms: the eight threads of a row (fixed order)
  double sb = pb[0] + pb[1], sc = pc[0] + pc[1];
#pragma unroll
  for (int m = 1; m <= 4; m <<= 1) {
    sb += __shfl_xor(sb, m, 64);
    sc += __shfl_xor(sc, m, 64);
  }
  if ((tid & 7) == 0) {
    nB[sr] = sb;
    nC[sr] = sc;
  }
  __syncthreads();
  const int kst = (d + kGramK - 1) / kGramK * kGramK + 1;
  const double gam = (double)kst * 0x1p-23 / (1.0 - (double)kst * 0x1p-23);
  // lane l holds g for rows 4 (l / 16) + q and column l % 16 of the wave's block
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int rb = wr + 4 * lk + q, rc = wc + lr;
    const int b = b0 + rb, c = c0 + rc;
    if (b >= k || c >= k) continue;
    float v = __builtin_inff();
    if (b != c) {
      const double nb = nB[rb], nc = nC[rc];
      const double cross = sqrt(nb * nc) * (1.0 + 0x1p-40);
      const double s2 = (nb + nc) * (1.0 - 0x1p-38) - 2.0 * (double)acc[q] - 2.0 * gam * cross;
      v = dist_down(s2);
    }
    D[(int64_t)b * k + c] = v;
    if (bi != ci) D[(int64_t)c * k + b] = v;
  }
}

// Pass 2: one workgroup per center b, four waves.  Keys (bound bits << 32 |
// index; all ones for no center) are taken 64 at a time, one per lane, wave w
// taking chunks w, w + 4, ...; a chunk is sorted across the wave by a bitonic
// network of shuffles and reversed, and the lane-wise minimum with the wave's
// running ascending list of the 64 smallest so far is a bitonic sequence
// holding the 64 smallest of both, which a bitonic merge sorts again.  The
// four lists are merged the same way through LDS (two rounds).  Lane i of
// wave 0 ends with the i-th smallest key: the (bound, index) order of a full
// sort, without it.
__device__ __forceinline__ unsigned long long wave_sort_asc(unsigned long long key, int lane) {
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const unsigned long long o = __shfl_xor(key, stride, 64);
      const bool up = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      key = (lower == up) ? (key < o ? key : o) : (key > o ? key : o);
    }
  }
  return key;
}

// best (ascending across lanes) <- the 64 smallest of best and other
// (other descending across lanes)
__device__ __forceinline__ unsigned long long wave_merge_asc(unsigned long long best,
                                                            unsigned long long other, int lane) {
  unsigned long long key = best < other ? best : other;
#pragma unroll
  for (int stride = 32; stride > 0; stride >>= 1) {
    const unsigned long long o = __shfl_xor(key, stride, 64);
    const bool lower = (lane & stride) == 0;
    key = lower ? (key < o ? key : o) : (key > o ? key : o);
  }
  return key;
}

__global__ __launch_bounds__(256) void center_select_kernel(const float* __restrict__ D, int k,
                                                            int32_t* __restrict__ nbr,
                                                            float* __restrict__ nbd,
                                                            const int* __restrict__ gate) {
  if (gate && *gate) return;
  __shared__ unsigned long long lst[3][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = (int)blockIdx.x;
  const unsigned long long none = ~0ull;
  unsigned long long best = none;   // ascending across lanes
  for (int c0 = w * 64; c0 < k; c0 += 256) {
    const int j = c0 + lane;
    unsigned long long key = none;
    if (j < k && j != b)
      key = ((unsigned long long)__float_as_uint(D[(int64_t)b * k + j]) << 32) | (unsigned)j;
    key = wave_sort_asc(key, lane);
    best = wave_merge_asc(best, __shfl(key, 63 - lane, 64), lane);
  }
  // waves 1 and 3 hand their lists (reversed) to waves 0 and 2, then wave 2 to wave 0
  if (w & 1) lst[w >> 1][63 - lane] = best;
  __syncthreads();
  if (!(w & 1)) best = wave_merge_asc(best, lst[w >> 1][lane], lane);
  if (w == 2) lst[2][63 - lane] = best;
  __syncthreads();
  if (w != 0) return;
  best = wave_merge_asc(best, lst[2][lane], lane);
  const bool nb = best == none;
  if (lane < kNbrL) nbr[(int64_t)b * kNbrL + lane] = nb ? -1 : (int)(best & 0xFFFFFFFFull);
  if (lane <= kNbrL)
    nbd[(int64_t)b * (kNbrL + 1) + lane] = nb ? __builtin_inff() : __uint_as_float((unsigned)(best >> 32));
}

hipError_t launch_center_table(hipStream_t s, const float* C, int k, int d, float* D, int32_t* nbr,
                               float* nbd, const int* gate) {
  if (k > kRouterMaxK) return hipErrorInvalidValue;
  const unsigned T = (unsigned)((k + kGramT - 1) / kGramT);
  hipLaunchKernelGGL(center_gram_kernel, dim3(T * (T + 1) / 2), dim3(256), 0, s, C, k, d, D, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(center_select_kernel, dim3((unsigned)k), dim3(256), 0, s, D, k, nbr, nbd,
                     gate);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Certificate.  16 lanes per row, 4 rows per wave; a workgroup decides a
// chunk of 1024 rows, then appends its list entries with one atomic per list.
//   D_ub = sqrt(s (1 + (d + 16) u)) (1 + 4 u) + ||x - x~||, s the FP32 sum of
//          (x~_e - c_e)^2 over the BF16 row x~ (triangle inequality for the
//          quantization, relative error of the sum below (d/16 + 8) u);
//   R    = 2 D_ub (1 + 8 u);
//   m    = number of listed neighbours with lower bound < R.
// Decision: m = 0 -> label = b; 1 <= m <= 2 -> label = b plus a short
// re-check entry with b and those neighbours as its candidates (every other
// center is excluded, so the exact comparison of the three is the argmin);
// otherwise (or the list is exhausted, or no proposal) -> GEMM row list.
// ROUTED = false takes the previous label as the only candidate.
// ---------------------------------------------------------------------------
template <bool ROUTED, int NX, bool FULL>
__global__ __launch_bounds__(256) void router_cert_kernel(
    const uint16_t* __restrict__ Xq, int64_t xs, int64_t n, int d, const float* __restrict__ C,
    int k, const RowStats* __restrict__ rs, const uint32_t* __restrict__ keys, int ib,
    const int32_t* __restrict__ nbr, const float* __restrict__ nbd, int32_t* __restrict__ label,
    FlagEntry* __restrict__ flags, int* __restrict__ fb_rows, LoopState* __restrict__ st,
    const int* __restrict__ gate, const int* __restrict__ rows,
    const unsigned long long* __restrict__ row_count, BoundsOut bo) {
  if (gate && *gate) return;
  // rows != nullptr: the points are rows[0 .. *row_count) instead of 0 .. n
  const int64_t npts = rows ? (int64_t)(*row_count) : n;
  constexpr int RPW = 256;
  constexpr int RPB = 4 * RPW;
  __shared__ unsigned char kind[RPB];  // 0 certified, 1 certified + re-check, 2 GEMM, 3 none
  __shared__ int rn0[RPB], rn1[RPB];
  __shared__ int wcnt[2][4];
  __shared__ unsigned long long wbase[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = lane & 15, sub = lane >> 4;
  const unsigned mask = (1u << ib) - 1u;
  const float u = 5.9604645e-8f;
  const float gam = (float)(d + 16) * u;
  const int64_t nchunks = (npts + RPB - 1) / RPB;
  auto row_of = [&](int64_t i) -> int64_t { return rows ? (int64_t)rows[i] : i; };
  const unsigned long long below = (1ull << lane) - 1ull;

  for (int64_t chk = blockIdx.x; chk < nchunks; chk += gridDim.x) {
    const int64_t r0 = chk * RPB + (int64_t)wave * RPW;
    // The selection input of the next pass (proposal keys, or the previous
    // label) is fetched one pass ahead, and everything that depends on the
    // selected center (its row, neighbour bounds and ids) is issued together
    // with the point's own row: one memory round trip per pass.
    auto fetch_sel = [&](int pass) -> unsigned {
      const int64_t ri = r0 + pass * 4 + sub;
      if (ri >= npts) return 0u;
      const int64_t rr = row_of(ri);
      return ROUTED ? keys[rr * kRouterM + q] : (unsigned)label[rr];
    };
    unsigned sel_next = fetch_sel(0);
    for (int pass = 0; pass < RPW / 4; ++pass) {
      const int slot = pass * 4 + sub;
      const bool valid = r0 + slot < npts;
      const int64_t r = valid ? row_of(r0 + slot) : 0;
      const unsigned sel = sel_next;
      if (pass + 1 < RPW / 4) sel_next = fetch_sel(pass + 1);
      int b0 = 0, cand = -1;
      bool ok = valid;
      if (ROUTED) {
        const int ci = (int)(mask - (sel & mask));
        cand = (valid && ci < k) ? ci : -1;
        const unsigned best = row16_max((cand >= 0) ? sel : 0u);
        if (best == 0u) ok = false;
        b0 = ok ? (int)(mask - (best & mask)) : 0;
        if (b0 >= k) {
          ok = false;
          b0 = 0;
        }
      } else {
        b0 = valid ? (int)sel : 0;
        if (b0 < 0 || b0 >= k) {
          ok = false;
          b0 = 0;
        }
      }

      const float* nd = nbd + (int64_t)b0 * (kNbrL + 1);
      const float nd0 = nd[q], nd1 = nd[q + 16], ndl = nd[kNbrL];
      const int nb0 = nbr[(int64_t)b0 * kNbrL], nb1 = nbr[(int64_t)b0 * kNbrL + 1];
      const float rx = valid ? rs[r].rx : 0.0f;

      // upper bound of ||x - c_b0||
      const float* c = C + (int64_t)b0 * d;
      const uint16_t* xr = Xq + (valid ? r : 0) * xs;
      float s = 0.0f;
      if (NX > 0) {
        ru32x4_t xv[NX > 0 ? NX : 1];
        float4 ca[NX > 0 ? NX : 1], cb[NX > 0 ? NX : 1];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
          const int e0 = q * 8 + 128 * i;
          if (FULL || e0 < d) {
            xv[i] = *(const ru32x4_t*)(xr + e0);
            ca[i] = *(const float4*)(c + e0);
            cb[i] = *(const float4*)(c + e0 + 4);
          }
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
          if (FULL || q * 8 + 128 * i < d) {
            const float cc[8] = {ca[i].x, ca[i].y, ca[i].z, ca[i].w,
                                 cb[i].x, cb[i].y, cb[i].z, cb[i].w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const unsigned w2 = xv[i][e >> 1];
              const float xe = __uint_as_float((e & 1) ? (w2 & 0xFFFF0000u) : (w2 << 16));
              const float df = xe - cc[e];
              s = __builtin_fmaf(df, df, s);
            }
          }
        }
      } else {
        for (int e0 = q * 8; e0 < d; e0 += 128) {
          const int e1 = min(e0 + 8, d);
          for (int e = e0; e < e1; ++e) {
            const float df = bf16_to_f32(xr[e]) - c[e];
            s = __builtin_fmaf(df, df, s);
          }
        }
      }
      s = row16_sum(s);
      const float dub = sqrtf(s * (1.0f + gam)) * (1.0f + 4.0f * u) + rx;
      const float R = 2.0f * dub * (1.0f + 8.0f * u);

      // b0's sorted neighbour list: m neighbours have a lower bound below R
      const unsigned long long bal0 = __ballot(nd0 < R);
      const unsigned long long bal1 = __ballot(nd1 < R);
      const int m = __popcll((bal0 >> (16 * sub)) & 0xFFFFull) +
                    __popcll((bal1 >> (16 * sub)) & 0xFFFFull);
      const bool exhausted = (m == kNbrL) && (ndl < R);
      const int n0 = (m >= 1) ? nb0 : -2;
      const int n1 = (m >= 2) ? nb1 : -2;
      int kd;
      if (!valid) kd = 3;
      else if (!ok || exhausted || m > 2) kd = 2;
      else kd = (m == 0) ? 0 : 1;
      // carried bounds: certified rows get ||x - c_b|| <= dub and, for every
      // center outside the first m neighbours, ||x - c|| >= nd[m] - dub (the
      // short re-check completes a listed row's bounds)
      const float ndm = __shfl(nd0, (lane & 48) + (m < 16 ? m : 0), 64);
      if (q == 0) {
        const int rec = wave * RPW + slot;
        kind[rec] = (unsigned char)kd;
        rn0[rec] = n0;
        rn1[rec] = (m == 2) ? n1 : -1;
        if (kd <= 1) label[r] = b0;
        if (bo.ub && kd <= 1) {
          bo.ub[r] = kd == 0 ? dub : __builtin_inff();
          bo.sec[r] = -1;
          bo.lb[r] = f64_to_f32_down((double)ndm - (double)dub);
        }
      }
    }
    __syncthreads();

    int nf = 0, nb = 0;
    for (int i = lane; i < RPW; i += 64) {
      const int kd = kind[wave * RPW + i];
      nf += (kd == 1);
      nb += (kd == 2);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      nf += __shfl_xor(nf, m, 64);
      nb += __shfl_xor(nb, m, 64);
    }
    if (lane == 0) {
      wcnt[0][wave] = nf;
      wcnt[1][wave] = nb;
    }
    __syncthreads();
    if (tid == 0) {
      const int sf = wcnt[0][0] + wcnt[0][1] + wcnt[0][2] + wcnt[0][3];
      const int sb = wcnt[1][0] + wcnt[1][1] + wcnt[1][2] + wcnt[1][3];
      wbase[0] = sf ? atomicAdd(&st->flagged, (unsigned long long)sf) : 0ull;
      wbase[1] = sb ? atomicAdd(&st->routed_fallback, (unsigned long long)sb) : 0ull;
      if (sf) atomicAdd(&st->routed_listed, (unsigned long long)sf);
    }
    __syncthreads();
    unsigned long long of = wbase[0], ob = wbase[1];
    for (int w = 0; w < wave; ++w) {
      of += wcnt[0][w];
      ob += wcnt[1][w];
    }
    for (int i0 = 0; i0 < RPW; i0 += 64) {
      const int rec = wave * RPW + i0 + lane;
      const int kd = kind[rec];
      const unsigned long long bf = __ballot(kd == 1);
      const unsigned long long bb = __ballot(kd == 2);
      const int row = (kd == 1 || kd == 2) ? (int)row_of(r0 + i0 + lane) : 0;
      if (kd == 1) {
        FlagEntry fe;
        fe.row = row;
        fe.cand2 = rn0[rec];
        fe.cand3 = rn1[rec];
        fe.pad = 0;
        flags[of + __popcll(bf & below)] = fe;
      }
      if (kd == 2) fb_rows[ob + __popcll(bb & below)] = row;
      of += __popcll(bf);
      ob += __popcll(bb);
    }
    __syncthreads();
  }
}

hipError_t launch_router_cert(hipStream_t s, const uint16_t* Xq, int64_t dp, int64_t n, int d,
                              const float* C, int k, const RowStats* rs, const uint32_t* keys,
                              int kpad, const int32_t* nbr, const float* nbd, int32_t* label,
                              FlagEntry* flags, int* fb_rows, LoopState* st, const int* gate,
                              int num_cus, const int* rows, const unsigned long long* row_count,
                              BoundsOut bo) {
  int ib = 1;
  while ((1 << ib) < kpad) ++ib;
  // one 1024-row chunk per workgroup up to 32 per CU
  int64_t blocks = (n + 1023) / 1024;
  const int64_t cap = (int64_t)num_cus * 32;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  // the distance pass keeps the row in registers (NX 128-column pieces per
  // 16 lanes) when both rows are 16-byte aligned in whole 8-column pieces
  const bool vec = ((((uintptr_t)C) & 15) == 0) && (((uintptr_t)Xq & 15) == 0) && (d % 8 == 0) &&
                   (dp % 8 == 0);
  const int nx = !vec ? 0 : d <= 128 ? 1 : d <= 256 ? 2 : d <= 512 ? 4 : d <= 1024 ? 8 : 0;
  // FULL: every 128-column piece lies inside the row (d = 128 NX)
  const bool full = nx > 0 && d == 128 * nx;
#define KMX_C(R_, NX_, F_)                                                                    \
  hipLaunchKernelGGL((router_cert_kernel<R_, NX_, F_>), dim3((unsigned)blocks), dim3(256), 0, \
                     s, Xq, dp, n, d, C, k, rs, keys, ib, nbr, nbd, label, flags, fb_rows, st, \
                     gate, rows, row_count, bo)
#define KMX_CN(R_)                                                 \
  switch (nx) {                                                    \
    case 1: if (full) KMX_C(R_, 1, true); else KMX_C(R_, 1, false); break; \
    case 2: if (full) KMX_C(R_, 2, true); else KMX_C(R_, 2, false); break; \
    case 4: if (full) KMX_C(R_, 4, true); else KMX_C(R_, 4, false); break; \
    case 8: if (full) KMX_C(R_, 8, true); else KMX_C(R_, 8, false); break; \
    default: KMX_C(R_, 0, false); break;                           \
  }
  if (keys) {
    KMX_CN(true)
  } else {
    KMX_CN(false)
  }
#undef KMX_CN
#undef KMX_C
  return hipGetLastError();
}

// fbh[slot] = rows sent to the GEMM by the last certificate pass (or `all`
// when all_rows != 0); skipped once the loop has stopped.
__global__ void record_fallback_kernel(const LoopState* __restrict__ st, int64_t* __restrict__ fbh,
                                       int slot, int all_rows, int64_t all,
                                       const int* __restrict__ gate) {
  if (gate && *gate) return;
  if (threadIdx.x == 0) fbh[slot] = all_rows ? all : (int64_t)st->routed_fallback;
}

hipError_t launch_record_fallback(hipStream_t s, const LoopState* st, int64_t* fbh, int slot,
                                  int all_rows, int64_t all, const int* gate) {
  hipLaunchKernelGGL(record_fallback_kernel, dim3(1), dim3(64), 0, s, st, fbh, slot, all_rows, all,
                     gate);
  return hipGetLastError();
}

}  // namespace kmx
