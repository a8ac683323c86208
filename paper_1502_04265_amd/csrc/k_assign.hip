// Assignment step of Lloyd's algorithm (Sec. 1: assign every point to its
// closest center), as a distance GEMM on the gfx950 matrix cores with the
// argmin fused into the epilogue.
//
// Ranking.  ||x - c_j||^2 = ||x||^2 - 2 (x.c_j - ||c_j||^2 / 2), so the
// closest center maximizes tau_j = x.c_j - h_j with h_j = ||c_j||^2 / 2.  The
// GEMM produces x~.c~_j (BF16 or FP32 operands, FP32 accumulation); the
// epilogue forms t_j = x~.c~_j - h_j + o_x with a per-row offset o_x that
// makes every t_j positive, so its float bits order like unsigned integers.
// The low `ib` bits are replaced by (mask - j): one unsigned max then keeps
// the best score and, on equal truncated scores, the lowest index.  Each lane
// keeps the top three keys of the centers it sees; lanes holding the same
// point merge at the end.
//
// Soundness.  For every center |t_j - (tau_j + o_x)| <= E(x), where E bounds
// the FP32 accumulation (gamma_K ||x~|| ||c~||), the quantization of both
// operands (||x - x~|| ||c~|| + ||x|| ||c - c~||), the rounding of h_j and of
// the epilogue, and the key truncation.  If t_1 - t_2 > 2E the GEMM's top-1 is
// the exact argmin.  Otherwise the row is flagged: when t_1 - t_3 > 2E only
// the two listed centers can win and the re-check compares those two;
// otherwise it re-checks every center.  The re-check computes distances as
// FP32 direct differences with error-free transformations (TwoSum/TwoProd
// double-float accumulation), so labels agree with exact arithmetic except
// on ties closer than about 1e-13 relative.
//
// Layout.  MFMA 16x16x32 BF16 (or 16x16x4 FP32): A = 16 centers x K (from
// LDS), B = K x 16 points (held in registers for the whole center loop),
// D[center][point]: lane l holds point l%16 and centers 4(l/16)+i.  Each lane
// reads 16 contiguous bytes of a row per "unit" (8 BF16 or 4 FP32); A and B
// use the same unit-to-k mapping, so the contraction order inside a unit is
// irrelevant to the result's definition.
#include "kmx_device.h"
#include "kmx_internal.h"

namespace kmx {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float f32x4_t;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4_t;

__device__ __forceinline__ void top3_insert(unsigned key, unsigned& v1, unsigned& v2,
                                            unsigned& v3) {
  unsigned a = max(v1, key), b = min(v1, key);
  v1 = a;
  unsigned c = max(v2, b), e = min(v2, b);
  v2 = c;
  v3 = max(v3, e);
}

template <bool BF16, int NKU, int NCG, int BN, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void assign_kernel(
    const void* __restrict__ Xsrc, int64_t xs, int vec_ok, int64_t n, int d, int dp,
    const RowStats* __restrict__ rs, const void* __restrict__ Cq, const float* __restrict__ ch,
    int k, int kpad, int ib, const CenterStats* __restrict__ cs, int32_t* __restrict__ label,
    float* __restrict__ d1o, float* __restrict__ d2o, FlagEntry* __restrict__ flags,
    LoopState* __restrict__ st, const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int NT = WAVES * 64;
  constexpr int RB = BN / 16;
  constexpr int ROWB = NKU * 64;         // bytes of one center row (all units)
  constexpr int PITCH = ROWB + 16;       // padded LDS row pitch
  constexpr int UNITS = BN * NKU * 4;    // 16-byte units per tile
  constexpr int UPT = (UNITS + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][BN * PITCH];
  __shared__ __attribute__((aligned(16))) float hsh[2][BN];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int prow = lane & 15;
  const int grp = lane >> 4;
  const int64_t p_base = ((int64_t)blockIdx.x * WAVES + wave) * (16 * NCG);

  // ---- point fragments (B operand), loaded once ----
  u32x4_t xf[NCG][NKU];
#pragma unroll
  for (int cg = 0; cg < NCG; ++cg) {
    const int64_t p = p_base + cg * 16 + prow;
    const bool pv = p < n;
#pragma unroll
    for (int ku = 0; ku < NKU; ++ku) {
      u32x4_t v = {0u, 0u, 0u, 0u};
      if (BF16) {
        if (pv) {
          const uint16_t* src = (const uint16_t*)Xsrc + p * xs + ku * 32 + grp * 8;
          v = *(const u32x4_t*)src;
        }
      } else {
        const int e0 = ku * 16 + grp * 4;
        const float* src = (const float*)Xsrc + p * xs + e0;
        if (pv) {
          if (vec_ok && e0 + 4 <= d) {
            v = *(const u32x4_t*)src;
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (e0 + q < d) v[q] = __float_as_uint(src[q]);
          }
        }
      }
      xf[cg][ku] = v;
    }
  }

  // ---- per-point offset o_x so that every score is positive ----
  const float cqm = __uint_as_float(cs->cq_max);
  const float rcm = __uint_as_float(cs->rc_max);
  const float cnm = __uint_as_float(cs->cn_max);
  float ox[NCG];
#pragma unroll
  for (int cg = 0; cg < NCG; ++cg) {
    const int64_t p = p_base + cg * 16 + prow;
    float nxq = (p < n) ? rs[p].nxq : 0.0f;
    ox[cg] = (nxq * cqm + 0.5f * cnm * cnm) * 1.001f + 1.0f;
  }

  const unsigned mask = (ib >= 32) ? 0xFFFFFFFFu : ((1u << ib) - 1u);
  unsigned v1[NCG], v2[NCG], v3[NCG];
#pragma unroll
  for (int cg = 0; cg < NCG; ++cg) v1[cg] = v2[cg] = v3[cg] = 0u;

  const int ntiles = kpad / BN;
  u32x4_t stage[UPT];
  float hstage = 0.0f;

  auto gload = [&](int tile) {
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int u = tid + NT * i;
      if (u < UNITS) {
        const int row = u / (NKU * 4);
        const int col = u % (NKU * 4);
        const unsigned char* src = (const unsigned char*)Cq +
                                   ((int64_t)(tile * BN + row)) * ROWB + col * 16;
        stage[i] = *(const u32x4_t*)src;
      }
    }
    if (tid < BN) hstage = ch[tile * BN + tid];
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int u = tid + NT * i;
      if (u < UNITS) {
        const int row = u / (NKU * 4);
        const int col = u % (NKU * 4);
        *(u32x4_t*)(&lds[buf][row * PITCH + col * 16]) = stage[i];
      }
    }
    if (tid < BN) hsh[buf][tid] = hstage;
  };

  gload(0);
  lstore(0);
  __syncthreads();

  for (int t = 0; t < ntiles; ++t) {
    const int buf = t & 1;
    if (t + 1 < ntiles) gload(t + 1);

    f32x4_t acc[NCG][RB];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) acc[cg][rb] = (f32x4_t){0.f, 0.f, 0.f, 0.f};

#pragma unroll
    for (int ku = 0; ku < NKU; ++ku) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const u32x4_t a =
            *(const u32x4_t*)(&lds[buf][(rb * 16 + prow) * PITCH + ku * 64 + grp * 16]);
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) {
          if (BF16) {
            acc[cg][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, xf[cg][ku]),
                acc[cg][rb], 0, 0, 0);
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              acc[cg][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                  __uint_as_float(a[q]), __uint_as_float(xf[cg][ku][q]), acc[cg][rb], 0, 0, 0);
          }
        }
      }
    }

    // ---- epilogue: scores -> keys -> running top-3 ----
    const bool last = (t == ntiles - 1);
    const unsigned ibase = mask - (unsigned)(t * BN + grp * 4);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const f32x4_t hv = *(const f32x4_t*)(&hsh[buf][rb * 16 + grp * 4]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int jl = rb * 16 + grp * 4 + i;  // center within the tile
        const bool valid = !last || (t * BN + jl < k);
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) {
          const float tt = (acc[cg][rb][i] - hv[i]) + ox[cg];
          unsigned key = (__float_as_uint(tt) & ~mask) | (ibase - (unsigned)(rb * 16 + i));
          key = valid ? key : 0u;
          top3_insert(key, v1[cg], v2[cg], v3[cg]);
        }
      }
    }

    if (t + 1 < ntiles) lstore(buf ^ 1);
    __syncthreads();
  }

  // ---- merge the four lanes that hold the same point ----
#pragma unroll
  for (int cg = 0; cg < NCG; ++cg) {
#pragma unroll
    for (int m = 16; m <= 32; m <<= 1) {
      unsigned o1 = __shfl_xor(v1[cg], m, 64);
      unsigned o2 = __shfl_xor(v2[cg], m, 64);
      unsigned o3 = __shfl_xor(v3[cg], m, 64);
      top3_insert(o1, v1[cg], v2[cg], v3[cg]);
      top3_insert(o2, v1[cg], v2[cg], v3[cg]);
      top3_insert(o3, v1[cg], v2[cg], v3[cg]);
    }
  }

  // ---- decision, outputs and the re-check list ----
  const float ua = 1.1920929e-7f;   // 2^-23: covers any faithful accumulation rounding
  const float u = 5.9604645e-8f;    // 2^-24
  const float Kf = (float)(dp + 1);
  const float gam = Kf * ua / (1.0f - Kf * ua);
#pragma unroll
  for (int cg = 0; cg < NCG; ++cg) {
    const int64_t p = p_base + cg * 16 + prow;
    const bool writer = (grp == (cg & 3)) && (p < n);
    bool flagged = false, full = false;
    int cand2 = 0;
    if (writer) {
      const RowStats r = rs[p];
      const float o = ox[cg];
      float E = gam * r.nxq * cqm + r.rx * cqm + r.nx * rcm + u * 0.5f * cnm * cnm +
                4.0f * u * o + ldexpf(2.0f * o, ib - 23);
      E = E * 1.0001f;
      const float t1 = __uint_as_float(v1[cg] & ~mask);
      // keys of real centers are never 0; the clamps only guard non-finite input
      const int i1 = v1[cg] ? min((int)(mask - (v1[cg] & mask)), k - 1) : 0;
      label[p] = i1;
      if (d1o) d1o[p] = fmaxf(r.xn2 - 2.0f * (t1 - o), 0.0f);
      if (v2[cg] != 0u) {
        const float t2 = __uint_as_float(v2[cg] & ~mask);
        cand2 = min((int)(mask - (v2[cg] & mask)), k - 1);
        if (d2o) d2o[p] = fmaxf(r.xn2 - 2.0f * (t2 - o), 0.0f);
        flagged = (t1 - t2) <= 2.0f * E;
        if (flagged && v3[cg] != 0u) {
          const float t3 = __uint_as_float(v3[cg] & ~mask);
          full = (t1 - t3) <= 2.0f * E;
        }
      } else if (d2o) {
        d2o[p] = __builtin_inff();
      }
    }
    const unsigned long long fm = __ballot(flagged);
    if (fm) {
      const unsigned long long ffm = __ballot(full);
      unsigned long long basei = 0;
      if (lane == 0) {
        basei = atomicAdd(&st->flagged, (unsigned long long)__popcll(fm));
        if (ffm) atomicAdd(&st->flagged_full, (unsigned long long)__popcll(ffm));
      }
      basei = __shfl(basei, 0, 64);
      if (flagged) {
        const unsigned long long below = fm & ((1ull << lane) - 1ull);
        FlagEntry fe;
        fe.row = (int)p | (full ? (int)0x80000000 : 0);
        fe.cand2 = cand2;
        flags[basei + __popcll(below)] = fe;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Kernel configurations.  dp is the padded row length: BF16 rows are padded
// to a multiple of 32 elements (one 16x16x32 unit), FP32 rows to 16.
// ---------------------------------------------------------------------------
static int units_for(int prec, int d) {
  const int kpu = (prec == KMX_BF16) ? 32 : 16;
  int u = (d + kpu - 1) / kpu;
  int p = 1;
  while (p < u) p <<= 1;
  return p;
}

int assign_dpad(int prec, int d) {
  const int kpu = (prec == KMX_BF16) ? 32 : 16;
  return units_for(prec, d) * kpu;
}

// Centers per LDS tile: each of the two tile buffers stays within about 66 KB.
int assign_tile_n(int prec, int d) {
  const int nku = units_for(prec, d);
  if (prec == KMX_BF16) return (nku <= 16) ? 64 : 32;
  if (nku <= 4) return 64;
  if (nku <= 32) return 32;
  return 16;
}

template <bool BF16, int NKU, int NCG, int BN, int WAVES>
static hipError_t run_assign(hipStream_t s, const void* Xsrc, int64_t xs, int vec_ok, int64_t n,
                             int d, int dp, const RowStats* rs, const void* Cq, const float* ch,
                             int k, int kpad, int ib, const CenterStats* cs, int32_t* label,
                             float* d1, float* d2, FlagEntry* flags, LoopState* st,
                             const int* gate) {
  const int64_t ppb = (int64_t)WAVES * 16 * NCG;
  const int64_t blocks = (n + ppb - 1) / ppb;
  hipLaunchKernelGGL((assign_kernel<BF16, NKU, NCG, BN, WAVES>), dim3((unsigned)blocks),
                     dim3(WAVES * 64), 0, s, Xsrc, xs, vec_ok, n, d, dp, rs, Cq, ch, k, kpad, ib,
                     cs, label, d1, d2, flags, st, gate);
  return hipGetLastError();
}

hipError_t launch_assign(hipStream_t s, int prec, const float* X, int64_t ldx, const uint16_t* Xq,
                         int64_t n, int d, int dp, const RowStats* rs, const void* Cq,
                         const float* ch, int k, int kpad, const CenterStats* cs, int32_t* label,
                         float* d1, float* d2, FlagEntry* flags, LoopState* st, const int* gate) {
  int ib = 1;
  while ((1 << ib) < kpad) ++ib;
  const int nku = units_for(prec, d);
  if (prec == KMX_BF16) {
    const void* src = Xq;
    const int64_t xs = dp;
#define KMX_A(NKU_, NCG_, BN_, W_)                                                              \
  return run_assign<true, NKU_, NCG_, BN_, W_>(s, src, xs, 1, n, d, dp, rs, Cq, ch, k, kpad, ib, \
                                               cs, label, d1, d2, flags, st, gate)
    switch (nku) {
      case 1: KMX_A(1, 4, 64, 8);
      case 2: KMX_A(2, 4, 64, 8);
      case 4: KMX_A(4, 4, 64, 8);
      case 8: KMX_A(8, 2, 64, 8);
      case 16: KMX_A(16, 2, 64, 8);
      case 32: KMX_A(32, 1, 32, 8);
      default: return hipErrorInvalidValue;
    }
#undef KMX_A
  } else {
    const int vec_ok = ((((uintptr_t)X) & 15) == 0) && (ldx % 4 == 0);
#define KMX_A(NKU_, NCG_, BN_, W_)                                                               \
  return run_assign<false, NKU_, NCG_, BN_, W_>(s, X, ldx, vec_ok, n, d, dp, rs, Cq, ch, k, kpad, \
                                                ib, cs, label, d1, d2, flags, st, gate)
    switch (nku) {
      case 1: KMX_A(1, 4, 64, 8);
      case 2: KMX_A(2, 4, 64, 8);
      case 4: KMX_A(4, 2, 64, 8);
      case 8: KMX_A(8, 2, 32, 8);
      case 16: KMX_A(16, 2, 32, 8);
      case 32: KMX_A(32, 1, 32, 8);
      case 64: KMX_A(64, 1, 16, 4);
      default: return hipErrorInvalidValue;
    }
#undef KMX_A
  }
}

// ---------------------------------------------------------------------------
// Re-check of flagged rows.  One wave per list entry.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void recheck_kernel(const float* __restrict__ X, int64_t n,
                                                      int d, int64_t ldx,
                                                      const float* __restrict__ C, int k,
                                                      int32_t* __restrict__ label,
                                                      float* __restrict__ d1o,
                                                      const FlagEntry* __restrict__ flags,
                                                      const LoopState* __restrict__ st,
                                                      const int* __restrict__ done) {
  if (done && *done) return;
  const unsigned long long cnt = st->flagged;
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t e = gw; e < (int64_t)cnt; e += nw) {
    const FlagEntry fe = flags[e];
    const int row = fe.row & 0x7FFFFFFF;
    const bool full = fe.row < 0;
    if (row >= n) continue;
    const float* x = X + (int64_t)row * ldx;
    int best = label[row];
    float bh, bl;
    if (!full) {
      const int c2 = fe.cand2;
      float s1 = 0.f, e1 = 0.f, s2 = 0.f, e2 = 0.f;
      const float* a = C + (int64_t)best * d;
      const float* b = C + (int64_t)c2 * d;
      for (int c = lane; c < d; c += 64) {
        const float xv = x[c];
        df_acc_sqdiff(xv, a[c], s1, e1);
        df_acc_sqdiff(xv, b[c], s2, e2);
      }
      wave_sum_df(s1, e1);
      wave_sum_df(s2, e2);
      float h1, l1, h2, l2;
      df_norm(s1, e1, h1, l1);
      df_norm(s2, e2, h2, l2);
      const bool take2 = df_less(h2, l2, h1, l1) || (h1 == h2 && l1 == l2 && c2 < best);
      if (take2) { best = c2; bh = h2; bl = l2; } else { bh = h1; bl = l1; }
    } else {
      // Pass 1: plain FP32 distances, one center per lane, to find the minimum.
      const float gam = (float)(d + 3) * 5.9604645e-8f;
      float m = __builtin_inff();
      for (int jb = 0; jb < k; jb += 64) {
        const int j = jb + lane;
        if (j < k) {
          const float* cj = C + (int64_t)j * d;
          float acc = 0.f;
          for (int c = 0; c < d; ++c) {
            const float dd = x[c] - cj[c];
            acc = __builtin_fmaf(dd, dd, acc);
          }
          m = fminf(m, acc);
        }
      }
#pragma unroll
      for (int s = 32; s >= 1; s >>= 1) m = fminf(m, __shfl_xor(m, s, 64));
      const float thr = m * (1.0f + gam) / (1.0f - gam) * 1.0001f + 1e-30f;
      // Pass 2: every center within the plain-FP32 error band gets the exact test.
      bh = __builtin_inff();
      bl = 0.f;
      best = -1;
      for (int jb = 0; jb < k; jb += 64) {
        const int j = jb + lane;
        bool cand = false;
        if (j < k) {
          const float* cj = C + (int64_t)j * d;
          float acc = 0.f;
          for (int c = 0; c < d; ++c) {
            const float dd = x[c] - cj[c];
            acc = __builtin_fmaf(dd, dd, acc);
          }
          cand = acc <= thr;
        }
        unsigned long long cm = __ballot(cand);
        while (cm) {
          const int t = __ffsll((long long)cm) - 1;
          cm &= cm - 1ull;
          const int jj = jb + t;
          const float* cj = C + (int64_t)jj * d;
          float s1 = 0.f, e1 = 0.f;
          for (int c = lane; c < d; c += 64) df_acc_sqdiff(x[c], cj[c], s1, e1);
          wave_sum_df(s1, e1);
          float h1, l1;
          df_norm(s1, e1, h1, l1);
          if (best < 0 || df_less(h1, l1, bh, bl)) { bh = h1; bl = l1; best = jj; }
        }
      }
    }
    if (lane == 0) {
      label[row] = best;
      if (d1o) d1o[row] = bh;
    }
  }
}

hipError_t launch_recheck(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
                          const float* C, int k, int32_t* label, float* d1,
                          const FlagEntry* flags, const LoopState* st, int num_cus,
                          const int* gate) {
  int64_t blocks = (n + 3) / 4;
  const int64_t cap = (int64_t)num_cus * 8;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(recheck_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, n, d, ldx, C, k,
                     label, d1, flags, st, gate);
  return hipGetLastError();
}

}  // namespace kmx
