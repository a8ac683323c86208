// Assignment step of Lloyd's algorithm (Sec. 1: assign every point to its
// closest center), as a distance GEMM on the gfx950 matrix cores with the
// argmin fused into the epilogue.
//
// Ranking.  ||x - c_j||^2 = ||x||^2 - 2 (x.c_j - h_j) with h_j = ||c_j||^2 / 2,
// so the closest center maximizes x.c_j - h_j.  The kernel forms the positive
// score t_j = x~.c~_j - h_j + O (x~, c~ the GEMM operands: BF16 copies, or the
// FP32 values), whose float bits order like unsigned integers.
//   BF16: the accumulator starts at O - h_j (rounded to FP32) and the MFMAs
//     add x~.c~_j, so it ends at t_j; O is one offset per assignment (max row
//     norm times max center norm plus max h).
//   FP32: the score is the float acc - h_j itself (no offset), and the lane
//     keeps the three best scores with the indices of the first two.
//   Split BF16 (the last pass of the BF16 and FP8 cascades): every FP32 value
//     v is split into hi = bf16(v) and lo = bf16(v - hi), and the MFMAs form
//     x_hi.c_hi in one accumulator and x_hi.c_lo + x_lo.c_hi in a second; the
//     score is (acc1 + acc2) - h_j, ranked as for FP32.  The dropped part
//     x_lo.c_lo + (remainders of both splits) is below 3.02 2^-16 sum |x_i c_i|
//     (each split leaves at most 2^-16 |v|), and the BF16 matrix instructions
//     run about five times the FP32 ones' rate.
//   FP8 (E4M3, per-row power-of-two scales 2^e_x, one scale 2^e_c for all
//     centers): the scaled MFMA applies 2^(e_x + e_c) to each product, so the
//     accumulator holds x~.c~_j in the units of x; it starts at O - h_j.
// The low `ib` bits of t_j are replaced by (mask - j): an unsigned max keeps
// the best score and, between equal truncated scores, the lowest index.  A
// lane keeps the four (BF16) or three (FP32) largest keys it has seen (max
// and med3 operations); the four lanes holding one point merge at the end.
//
// Soundness.  For every center |t_j - (x.c_j - h_j + O)| <= E(x), where E
// covers the FP32 accumulation (gamma_K sum |x~_i c~_ji|), the quantization of
// both operands (||x - x~|| ||c~|| + ||x|| ||c - c~||), the rounding of the
// start value O - h_j and of the epilogue, and the key truncation.  If t_1 - t_2 > 2E the top key's
// center is the exact argmin.  Otherwise the row is flagged: the centers whose
// score lies within 2E of the top can win; when they are among the listed two
// (BF16: three) the short re-check compares them.  Otherwise the row needs
// every center: the BF16 pass sends it to the split-BF16 pass (same kernel,
// list of rows), whose much tighter bound leaves it a short re-check in all
// but exceptional cases; rows still open after that pass are re-checked
// against every center.  The re-check decides with plain FP32
// direct differences where their error bound allows and otherwise with
// error-free transformations (double-float accumulation), so labels agree
// with exact arithmetic except on ties closer than about 1e-13 relative.
//
// The FP8 MFMA's internal summation is not IEEE round-to-nearest: its error
// is bounded here per instruction by 2^-10 sum |x~_i c~_ji| (the products'
// own summation; worst case measured on adversarial inputs 2^-12.0 of that
// sum) plus 2^-19 (|acc in| + sum |x~_i c~_ji|) (the alignment of the
// products to a large accumulator: up to 13.5 units in the last place of it
// measured, 16 allowed), on top of the FP32 rounding of each step.  No
// published accumulation rule of the instruction backs these constants;
// kmx_mfma_probe lets a test check them on the device at hand.
//
// Layout.  MFMA 16x16x32 BF16 (also split BF16), 16x16x128 FP8 or 16x16x4 FP32: A = 16 centers
// x K (from LDS), B = K x 16 points (registers, loaded once per block of
// points), D[center][point]: lane l holds point l%16 and centers 4(l/16)+i.
// Each lane reads 16 (FP8: 32) contiguous bytes of a row per "unit" (8 BF16,
// 32 FP8 or 4 FP32 values); A and B use the same unit-to-k mapping, so the
// contraction order inside a unit does not change what is computed.
#include "kmx_device.h"
#include "kmx_internal.h"

namespace kmx {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float f32x4_t;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4_t;
typedef __attribute__((ext_vector_type(8))) int i32x8_t;

// FP8 x FP8 MFMA with E8M0 block scales: sa for A, byte SEL of sb for B.
template <int SEL>
__device__ __forceinline__ f32x4_t mfma_f8_sel(const i32x8_t& a, const i32x8_t& b, f32x4_t c,
                                               int sa, int sb) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, sa, SEL, sb);
}
// sel is a constant after unrolling, so the switch folds away.
__device__ __forceinline__ f32x4_t mfma_f8_scaled(int sel, const i32x8_t& a, const i32x8_t& b,
                                                  f32x4_t c, int sa, int sb) {
  switch (sel & 3) {
    case 0: return mfma_f8_sel<0>(a, b, c, sa, sb);
    case 1: return mfma_f8_sel<1>(a, b, c, sa, sb);
    case 2: return mfma_f8_sel<2>(a, b, c, sa, sb);
    default: return mfma_f8_sel<3>(a, b, c, sa, sb);
  }
}

// Measurement of the matrix instructions exactly as the assignment issues
// them, from start values C (zero when C == nullptr): instance q computes
// D_q = C_q + A_q B_q^T, D_q and C_q 16 x 16 FP32, D[i][j] = row i of A_q with
// row j of B_q, one wave per instance, lane l holding rows l % 16 of both
// operands at the same K positions (the assignment's layout):
//   prec 2: scaled FP8 E4M3 16x16x128, A_q, B_q 16 x 128 bytes, E8M0 scale
//           sa[q] for every row of A_q and sb[16 q + j] for row j of B_q;
//   prec 1: BF16 16x16x32, A_q, B_q 16 x 32 BF16 values;
//   prec 0: FP32 16x16x4, A_q, B_q 16 x 4 floats.
template <int PREC>
__global__ __launch_bounds__(64) void mfma_probe_kernel(const uint8_t* __restrict__ A,
                                                        const uint8_t* __restrict__ B,
                                                        const uint8_t* __restrict__ sa,
                                                        const uint8_t* __restrict__ sb,
                                                        const float* __restrict__ C,
                                                        float* __restrict__ D) {
  constexpr int ROWB = PREC == 2 ? 128 : (PREC == 1 ? 64 : 16);   // bytes per operand row
  const int q = blockIdx.x;
  const int lane = threadIdx.x;
  const int r = lane & 15, g = lane >> 4;
  const uint8_t* a = A + (int64_t)q * 16 * ROWB + r * ROWB;
  const uint8_t* b = B + (int64_t)q * 16 * ROWB + r * ROWB;
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  if (C) {
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = C[(int64_t)q * 256 + (4 * g + i) * 16 + r];
  }
  if constexpr (PREC == 2) {
    i32x8_t av, bv;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      av[i] = ((const int*)(a + g * 32))[i];
      bv[i] = ((const int*)(b + g * 32))[i];
    }
    acc = mfma_f8_sel<0>(av, bv, acc, (int)sa[q], (int)sb[q * 16 + r]);
  } else if constexpr (PREC == 1) {
    const u32x4_t av = *(const u32x4_t*)(a + g * 16);
    const u32x4_t bv = *(const u32x4_t*)(b + g * 16);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, av),
                                                  __builtin_bit_cast(bf16x8_t, bv), acc, 0, 0, 0);
  } else {
    const float av = ((const float*)a)[g];
    const float bv = ((const float*)b)[g];
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
  }
  // lane l holds column (B row) l % 16 and rows (A rows) 4 (l / 16) + i
#pragma unroll
  for (int i = 0; i < 4; ++i) D[(int64_t)q * 256 + (4 * g + i) * 16 + r] = acc[i];
}

hipError_t launch_mfma_probe(hipStream_t s, int prec, const uint8_t* A, const uint8_t* B,
                             const uint8_t* sa, const uint8_t* sb, const float* C, float* D,
                             int count) {
  if (prec == KMX_FP8E4M3)
    hipLaunchKernelGGL(mfma_probe_kernel<2>, dim3((unsigned)count), dim3(64), 0, s, A, B, sa, sb,
                       C, D);
  else if (prec == KMX_BF16)
    hipLaunchKernelGGL(mfma_probe_kernel<1>, dim3((unsigned)count), dim3(64), 0, s, A, B, sa, sb,
                       C, D);
  else
    hipLaunchKernelGGL(mfma_probe_kernel<0>, dim3((unsigned)count), dim3(64), 0, s, A, B, sa, sb,
                       C, D);
  return hipGetLastError();
}

__device__ __forceinline__ unsigned med3u(unsigned a, unsigned b, unsigned c) {
  return max(min(a, b), min(max(a, b), c));
}

// (v1 >= v2 >= v3) <- the three largest of {v1, v2, v3, key}
__device__ __forceinline__ void top3_insert(unsigned key, unsigned& v1, unsigned& v2,
                                            unsigned& v3) {
  const unsigned n1 = max(v1, key);
  const unsigned n2 = med3u(v1, v2, key);
  const unsigned n3 = med3u(v2, v3, key);
  v1 = n1;
  v2 = n2;
  v3 = n3;
}

// (v1 >= v2 >= v3 >= v4) <- the four largest of {v1, v2, v3, v4, key}
__device__ __forceinline__ void top4_insert(unsigned key, unsigned& v1, unsigned& v2,
                                            unsigned& v3, unsigned& v4) {
  const unsigned n1 = max(v1, key);
  const unsigned n2 = med3u(v1, v2, key);
  const unsigned n3 = med3u(v2, v3, key);
  const unsigned n4 = med3u(v3, v4, key);
  v1 = n1;
  v2 = n2;
  v3 = n3;
  v4 = n4;
}

// Arguments of one assignment pass as seen by a block.
struct AssignArgs {
  const void* Xsrc;            // rows of the GEMM operand (FP32 X, BF16 or FP8 copy)
  int64_t xs;                  // row stride (elements of the operand; bytes for FP8)
  int vec_ok;                  // FP32 rows allow 16-byte loads
  const uint8_t* sx8;          // FP8 row scales (E8M0)
  int64_t npts;                // points: rows[0 .. npts) or 0 .. npts
  const int* rows;             // optional row list
  int d, dp;
  const RowStats* rs;
  const void* Cq;              // padded center rows
  const float* ch;             // per-center values (FP32: h_j; FP8: O - h_j)
  int k, kpad, ib;
  const CenterStats* cs;
  int32_t* label;
  float* d1o;
  float* d2o;
  int koff;                    // added to every center index written
  int64_t list_off;            // added to every row index written into a list
  FlagEntry* flags;
  int* full_rows;
  unsigned long long* full_ctr;
  int cascade_all;
  int* brute;
  LoopState* st;
  int count_undecided;
  // carried bounds (nullable), written for the rows this pass decides; for
  // listed rows bo.lb covers the centers not listed and the re-check
  // completes the rest
  BoundsOut bo;
};

template <int MODE, int NKU, int NCG, int BN, int WAVES>
struct AssignShape {
  static constexpr int UB = (MODE == 2) ? 32 : 16;     // bytes per lane and unit
  // bytes of one center row (split BF16: NKU units of high parts, then NKU of low parts)
  static constexpr int ROWB = (MODE == 3) ? 2 * NKU * 64 : NKU * UB * 4;
  static constexpr int UROW = ROWB / 16 + 1;           // 16-byte units per LDS row
  static constexpr int CHUNKS = (BN * UROW + 63) / 64; // 1 KB direct-to-LDS copies per tile
  static constexpr int BUFB = CHUNKS * 1024;           // bytes of one tile buffer
  static constexpr int PPB = WAVES * 16 * NCG;         // points per block
};

// One block of PPB points starting at point blk * PPB: point fragments, the
// loop over every center tile, the merge of the four lanes of a point, the
// decision and the re-check list entries.  lds holds two tile buffers, hsh
// two rows of BN per-center values, wcnt 3 * WAVES counters, wbase 3 bases.
template <int MODE, int NKU, int NCG, int BN, int WAVES, int PF, bool EP, int SUBT>
__device__ __forceinline__ void assign_block(const AssignArgs& A, int64_t blk,
                                             unsigned char* lds, float* hsh, int* wcnt,
                                             unsigned long long* wbase) {
  constexpr bool BF16 = (MODE == 1);
  constexpr bool F8 = (MODE == 2);
  constexpr bool SPLIT = (MODE == 3);
  constexpr bool PK = BF16 || F8;        // packed keys (BF16, FP8)
  // FP8: each lane keeps its three best keys during the tile loop (a vector
  // operation less per key); the decision then treats a row whose lane-wise
  // third best lies inside the bound as having more than three candidates
  constexpr bool T3 = F8;
  // 16-byte fragments per lane and unit (split BF16: the high, then the low parts)
  constexpr int NF = (F8 || SPLIT) ? 2 : 1;
  constexpr int NT = WAVES * 64;
  // SUBT sub-tiles per LDS tile: the keys of each BN / SUBT centers are
  // inserted before the next ones are computed, so the accumulators stay
  // those of one sub-tile while the tile barrier is paid once per BN centers
  static_assert(BN % SUBT == 0 && (BN / SUBT) % 16 == 0, "sub-tiles of whole 16-center blocks");
  static_assert(SUBT == 1 || (MODE == 2 && !EP), "sub-tiles: FP8 without the pipelined epilogue");
  constexpr int BNS = BN / SUBT;
  constexpr int RB = BNS / 16;
  using S = AssignShape<MODE, NKU, NCG, BN, WAVES>;
  constexpr int ROWB = S::ROWB;
  constexpr int PITCH = ROWB + 16;       // padded LDS row pitch
  constexpr int UROW = S::UROW;
  constexpr int CHUNKS = S::CHUNKS;
  constexpr int BUFB = S::BUFB;
  constexpr int PPB = S::PPB;
  (void)NT;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int prow = lane & 15;
  const int grp = lane >> 4;
  const int ntiles = A.kpad / BN;
  const unsigned mask = (A.ib >= 32) ? 0xFFFFFFFFu : ((1u << A.ib) - 1u);
  const float cqm = __uint_as_float(A.cs->cq_max);
  const float rcm = __uint_as_float(A.cs->rc_max);
  const float cnm = __uint_as_float(A.cs->cn_max);
  const float Og = A.cs->O;
  const int cexp = A.cs->c_exp;
  {
    const int64_t p_base = blk * PPB + (int64_t)wave * (16 * NCG);

    // ---- point fragments (B operand) for this block ----
    int src_row[NCG];                  // n <= 2^31 - 2: row ids fit 32 bits
    u32x4_t xf[NCG][NKU * NF];
    // E8M0 scale of point group cg in byte cg (FP8; the MFMA selects the byte)
    static_assert(!F8 || NCG <= 4, "four point-group scales per register");
    unsigned sxp = 0u;
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
      const int64_t p = p_base + cg * 16 + prow;
      const bool pv = p < A.npts;
      const int64_t r = pv ? (A.rows ? (int64_t)A.rows[p] : p) : -1;
      src_row[cg] = (int)r;
      if (F8) sxp |= (pv ? (unsigned)A.sx8[r] : 127u) << (8 * (cg & 3));
      // packed operands: invalid points read row 0 (always present) and are
      // zeroed afterwards, so the loads issue without branches
      const int64_t rl = pv ? r : 0;
#pragma unroll
      for (int ku = 0; ku < NKU * NF; ++ku) {
        if constexpr (SPLIT) {
          // values (ku / 2) * 32 + grp * 8 .. + 7 of the FP32 row, split into
          // the high parts (fragment ku) and the low parts (fragment ku + 1)
          if (ku & 1) continue;
          const int e0 = (ku >> 1) * 32 + grp * 8;
          float xv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) xv[q] = 0.0f;
          if (pv) {
            const float* src = (const float*)A.Xsrc + r * A.xs + e0;
            if (A.vec_ok && e0 + 8 <= A.d) {
              const float4 a = *(const float4*)src;
              const float4 b = *(const float4*)(src + 4);
              xv[0] = a.x; xv[1] = a.y; xv[2] = a.z; xv[3] = a.w;
              xv[4] = b.x; xv[5] = b.y; xv[6] = b.z; xv[7] = b.w;
            } else {
#pragma unroll
              for (int q = 0; q < 8; ++q)
                if (e0 + q < A.d) xv[q] = src[q];
            }
          }
          u32x4_t hv, lv;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const uint16_t h0 = f32_to_bf16_rne(xv[2 * q]);
            const uint16_t h1 = f32_to_bf16_rne(xv[2 * q + 1]);
            const uint16_t l0 = f32_to_bf16_rne(xv[2 * q] - bf16_to_f32(h0));
            const uint16_t l1 = f32_to_bf16_rne(xv[2 * q + 1] - bf16_to_f32(h1));
            hv[q] = (unsigned)h0 | ((unsigned)h1 << 16);
            lv[q] = (unsigned)l0 | ((unsigned)l1 << 16);
          }
          xf[cg][ku] = hv;
          xf[cg][ku + 1] = lv;
          continue;
        }
        u32x4_t v = {0u, 0u, 0u, 0u};
        if (F8) {
          v = *(const u32x4_t*)((const uint8_t*)A.Xsrc + rl * A.xs + (ku >> 1) * 128 + grp * 32 +
                                (ku & 1) * 16);
          if (!pv) v = (u32x4_t){0u, 0u, 0u, 0u};
        } else if (BF16) {
          v = *(const u32x4_t*)((const uint16_t*)A.Xsrc + rl * A.xs + ku * 32 + grp * 8);
          if (!pv) v = (u32x4_t){0u, 0u, 0u, 0u};
        } else {
          const int e0 = ku * 16 + grp * 4;
          const float* src = (const float*)A.Xsrc + r * A.xs + e0;
          if (pv) {
            if (A.vec_ok && e0 + 4 <= A.d) {
              v = *(const u32x4_t*)src;
            } else {
#pragma unroll
              for (int q = 0; q < 4; ++q)
                if (e0 + q < A.d) v[q] = __float_as_uint(src[q]);
            }
          }
        }
        xf[cg][ku] = v;
      }
    }

    // BF16 state: four packed keys per point.  FP32 state: the three best
    // scores and the indices of the first two, kept exactly.
    unsigned v1[NCG], v2[NCG], v3[NCG], v4[NCG];
    float f1[NCG], f2[NCG], f3[NCG];
    int j1[NCG], j2[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
      v1[cg] = v2[cg] = v3[cg] = v4[cg] = 0u;
      f1[cg] = f2[cg] = f3[cg] = -__builtin_inff();
      j1[cg] = j2[cg] = 0x7FFFFFFF;
    }

    // Tile copy: LDS chunk c (1 KB) receives the 16-byte units c*64 .. c*64+63
    // of the padded tile, lane l the unit c*64 + l (the order the direct-to-LDS
    // load writes them).  Pad units re-load the tile's first unit.
    float hstage = 0.0f;
    auto issue_tile = [&](int tile, int buf) {
      const unsigned char* tbase = (const unsigned char*)A.Cq + (int64_t)tile * BN * ROWB;
#pragma unroll
      for (int c = wave; c < CHUNKS; c += WAVES) {
        const int q = c * 64 + lane;
        const int row = q / UROW;
        const int uc = q - row * UROW;
        const unsigned char* src =
            (row < BN && uc < UROW - 1) ? tbase + row * ROWB + uc * 16 : tbase;
        __builtin_amdgcn_global_load_lds(
            (const void*)src, (__attribute__((address_space(3))) void*)(&lds[buf * BUFB + c * 1024]), 16,
            0, 0);
      }
      if (tid < BN) hstage = A.ch[tile * BN + tid];
    };
    auto finish_tile = [&](int buf) {
      if (tid < BN) hsh[buf * BN + tid] = hstage;
      __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    };

    issue_tile(0, 0);
    finish_tile(0);
    __syncthreads();

    // EP (packed keys only): the keys of tile t - 1 are inserted while the
    // MFMAs of tile t run, a slice after each unit, so the matrix core and
    // the vector ALU overlap within a wave.  Inserting key 0 changes nothing
    // (every kept key is >= 0), which disables the slices of the first tile.
    constexpr bool PIPE = EP && PK;
    constexpr int NSC = NCG * RB * 4;    // keys per lane and tile
    f32x4_t accp[NCG][RB];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) accp[cg][rb] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
    auto insert_prev = [&](int sidx, unsigned ibase_p, unsigned pm) {
      const int rb = sidx / (4 * NCG), i = (sidx / NCG) % 4, cg = sidx % NCG;
      const unsigned idx = ibase_p - (unsigned)(rb * 16 + i);
      const unsigned key = ((__float_as_uint(accp[cg][rb][i]) & ~mask) | idx) & pm;
      if constexpr (T3) top3_insert(key, v1[cg], v2[cg], v3[cg]);
      else top4_insert(key, v1[cg], v2[cg], v3[cg], v4[cg]);
    };

    // Packed keys of one tile into the running top-4.  With eight waves the
    // second half inserts its keys after the tile's barrier instead of
    // before it: the two waves sharing a SIMD then run their vector epilogue
    // while the other one issues matrix instructions.  (The keys live in
    // registers only, so the barrier does not order them.)
    const bool late = (WAVES == 8) && (wave >= WAVES / 2);
    auto insert_tile = [&](const f32x4_t (&a)[NCG][RB], int c0) {   // c0: first center
      const unsigned ibase = mask - (unsigned)(c0 + grp * 4);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const unsigned idx = ibase - (unsigned)(rb * 16 + i);
#pragma unroll
          for (int cg = 0; cg < NCG; ++cg) {
            const unsigned key = (__float_as_uint(a[cg][rb][i]) & ~mask) | idx;
            if constexpr (T3) top3_insert(key, v1[cg], v2[cg], v3[cg]);
            else top4_insert(key, v1[cg], v2[cg], v3[cg], v4[cg]);
          }
        }
      }
    };

    for (int t = 0; t < ntiles; ++t) {
      const int buf = t & 1;
      if (t + 1 < ntiles) issue_tile(t + 1, buf ^ 1);
      const unsigned ibase_p = mask - (unsigned)((t - 1) * BN + grp * 4);
      const unsigned pm = (t > 0) ? 0xFFFFFFFFu : 0u;

      f32x4_t acc[NCG][RB];
      f32x4_t accx[NCG][RB];   // split BF16: x_hi.c_lo + x_lo.c_hi
#pragma unroll
      for (int st = 0; st < SUBT; ++st) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        f32x4_t a0 = {0.f, 0.f, 0.f, 0.f};
        if (PK) a0 = *(const f32x4_t*)(&hsh[buf * BN + st * BNS + rb * 16 + grp * 4]);
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) {
          acc[cg][rb] = a0;
          accx[cg][rb] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
        }
      }

      if constexpr (F8) {
        // A fragments one unit ahead, as for BF16 below
        const unsigned char* abase = &lds[buf * BUFB + (st * BNS + prow) * PITCH + grp * 32];
        u32x4_t af8[2][RB][2];
        auto load_a8 = [&](int q, int slot) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            af8[slot][rb][0] = *(const u32x4_t*)(abase + rb * 16 * PITCH + q * 128);
            af8[slot][rb][1] = *(const u32x4_t*)(abase + rb * 16 * PITCH + q * 128 + 16);
          }
        };
        load_a8(0, 0);
#pragma unroll
        for (int ku = 0; ku < NKU; ++ku) {
          if (ku + 1 < NKU) load_a8(ku + 1, (ku + 1) & 1);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            const i32x8_t a = __builtin_bit_cast(
                i32x8_t, __builtin_shufflevector(af8[ku & 1][rb][0], af8[ku & 1][rb][1], 0, 1, 2,
                                                 3, 4, 5, 6, 7));
#pragma unroll
            for (int cg = 0; cg < NCG; ++cg) {
              const i32x8_t b = __builtin_bit_cast(
                  i32x8_t, __builtin_shufflevector(xf[cg][2 * ku], xf[cg][2 * ku + 1], 0, 1, 2, 3,
                                                   4, 5, 6, 7));
              acc[cg][rb] = mfma_f8_scaled(cg, a, b, acc[cg][rb], cexp, (int)sxp);
            }
          }
          if constexpr (PIPE) {
#pragma unroll
            for (int sidx = 0; sidx < NSC; ++sidx)
              if (sidx * NKU / NSC == ku) insert_prev(sidx, ibase_p, pm);
          }
        }
      } else if constexpr (SPLIT) {
        // high and low center parts PF units ahead, as for BF16 below
        constexpr int NB = PF + 1;
        constexpr int LOFF = NKU * 64;   // bytes from a row's high parts to its low parts
        u32x4_t afh[NB][RB], afl[NB][RB];
        const unsigned char* abase = &lds[buf * BUFB + (st * BNS + prow) * PITCH + grp * 16];
#pragma unroll
        for (int q = 0; q < PF; ++q)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            if (q < NKU) {
              afh[q][rb] = *(const u32x4_t*)(abase + rb * 16 * PITCH + q * 64);
              afl[q][rb] = *(const u32x4_t*)(abase + rb * 16 * PITCH + LOFF + q * 64);
            }
#pragma unroll
        for (int ku = 0; ku < NKU; ++ku) {
          if (ku + PF < NKU) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
              afh[(ku + PF) % NB][rb] = *(const u32x4_t*)(abase + rb * 16 * PITCH + (ku + PF) * 64);
              afl[(ku + PF) % NB][rb] =
                  *(const u32x4_t*)(abase + rb * 16 * PITCH + LOFF + (ku + PF) * 64);
            }
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            const bf16x8_t ah = __builtin_bit_cast(bf16x8_t, afh[ku % NB][rb]);
            const bf16x8_t al = __builtin_bit_cast(bf16x8_t, afl[ku % NB][rb]);
#pragma unroll
            for (int cg = 0; cg < NCG; ++cg) {
              const bf16x8_t xh = __builtin_bit_cast(bf16x8_t, xf[cg][2 * ku]);
              const bf16x8_t xl = __builtin_bit_cast(bf16x8_t, xf[cg][2 * ku + 1]);
              acc[cg][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xh, acc[cg][rb], 0, 0, 0);
              accx[cg][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xl, accx[cg][rb], 0, 0, 0);
              accx[cg][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, xh, accx[cg][rb], 0, 0, 0);
            }
          }
        }
      } else {
      // A fragments run PF units ahead of the MFMAs that use them; the
      // scheduling barrier keeps the compiler from sinking the reads next to
      // their use (which would expose the LDS latency at every unit).
      constexpr int NB = PF + 1;
      u32x4_t afr[NB][RB];
      const unsigned char* abase = &lds[buf * BUFB + (st * BNS + prow) * PITCH + grp * 16];
#pragma unroll
      for (int q = 0; q < PF; ++q)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
          if (q < NKU) afr[q][rb] = *(const u32x4_t*)(abase + rb * 16 * PITCH + q * 64);
#pragma unroll
      for (int ku = 0; ku < NKU; ++ku) {
        if (ku + PF < NKU) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            afr[(ku + PF) % NB][rb] =
                *(const u32x4_t*)(abase + rb * 16 * PITCH + (ku + PF) * 64);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const u32x4_t a = afr[ku % NB][rb];
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
                    __uint_as_float(a[q]), __uint_as_float(xf[cg][ku][q]), acc[cg][rb], 0, 0,
                    0);
            }
          }
        }
        if constexpr (PIPE) {
#pragma unroll
          for (int sidx = 0; sidx < NSC; ++sidx)
            if (sidx * NKU / NSC == ku) insert_prev(sidx, ibase_p, pm);
        }
      }
      }

      // ---- epilogue: running top-4 (BF16, FP8) or top-3 ----
      if constexpr (PIPE) {
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) accp[cg][rb] = acc[cg][rb];
      } else if constexpr (PK) {
        if (!late || st + 1 < SUBT) insert_tile(acc, t * BN + st * BNS);
      } else {
        // centers arrive in increasing index order per lane: a strict '>'
        // keeps the lower index on ties
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const f32x4_t hv = *(const f32x4_t*)(&hsh[buf * BN + st * BNS + rb * 16 + grp * 4]);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int j = t * BN + st * BNS + rb * 16 + grp * 4 + i;
#pragma unroll
            for (int cg = 0; cg < NCG; ++cg) {
              const float tt =
                  (SPLIT ? (acc[cg][rb][i] + accx[cg][rb][i]) : acc[cg][rb][i]) - hv[i];
              const bool c1 = tt > f1[cg], c2 = tt > f2[cg], c3 = tt > f3[cg];
              f3[cg] = c2 ? f2[cg] : (c3 ? tt : f3[cg]);
              f2[cg] = c1 ? f1[cg] : (c2 ? tt : f2[cg]);
              j2[cg] = c1 ? j1[cg] : (c2 ? j : j2[cg]);
              f1[cg] = c1 ? tt : f1[cg];
              j1[cg] = c1 ? j : j1[cg];
            }
          }
        }
      }

      }   // sub-tiles

      if (t + 1 < ntiles) finish_tile(buf ^ 1);
      __syncthreads();
      if constexpr (PK && !PIPE) {
        if (late) insert_tile(acc, t * BN + (SUBT - 1) * BNS);
      }
    }
    if constexpr (PIPE) {
      const unsigned ibase_p = mask - (unsigned)((ntiles - 1) * BN + grp * 4);
#pragma unroll
      for (int sidx = 0; sidx < NSC; ++sidx) insert_prev(sidx, ibase_p, 0xFFFFFFFFu);
    }

    // ---- merge the four lanes that hold the same point ----
    // w3: the largest lane-wise third best (T3); a lane whose third best is
    // inside the bound may hold further candidates that no lane kept
    unsigned w3[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
      w3[cg] = 0u;
      if constexpr (T3) {
        w3[cg] = v3[cg];
        w3[cg] = max(w3[cg], (unsigned)__shfl_xor((int)w3[cg], 16, 64));
        w3[cg] = max(w3[cg], (unsigned)__shfl_xor((int)w3[cg], 32, 64));
      }
    }
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
#pragma unroll
      for (int m = 16; m <= 32; m <<= 1) {
        if constexpr (PK) {
          const unsigned o1 = __shfl_xor(v1[cg], m, 64);
          const unsigned o2 = __shfl_xor(v2[cg], m, 64);
          const unsigned o3 = __shfl_xor(v3[cg], m, 64);
          const unsigned o4 = __shfl_xor(v4[cg], m, 64);
          top4_insert(o1, v1[cg], v2[cg], v3[cg], v4[cg]);
          top4_insert(o2, v1[cg], v2[cg], v3[cg], v4[cg]);
          top4_insert(o3, v1[cg], v2[cg], v3[cg], v4[cg]);
          top4_insert(o4, v1[cg], v2[cg], v3[cg], v4[cg]);
        } else {
          const float g1 = __shfl_xor(f1[cg], m, 64), g2 = __shfl_xor(f2[cg], m, 64);
          const float g3 = __shfl_xor(f3[cg], m, 64);
          const int k1 = __shfl_xor(j1[cg], m, 64), k2 = __shfl_xor(j2[cg], m, 64);
          // insert (g1,k1), (g2,k2) with the index tie-break, then g3 as a value
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const float tt = q ? g2 : g1;
            const int jj = q ? k2 : k1;
            const bool c1 = tt > f1[cg] || (tt == f1[cg] && jj < j1[cg]);
            const bool c2 = tt > f2[cg] || (tt == f2[cg] && jj < j2[cg]);
            const bool c3 = tt > f3[cg];
            f3[cg] = c2 ? f2[cg] : (c3 ? tt : f3[cg]);
            f2[cg] = c1 ? f1[cg] : (c2 ? tt : f2[cg]);
            j2[cg] = c1 ? j1[cg] : (c2 ? jj : j2[cg]);
            f1[cg] = c1 ? tt : f1[cg];
            j1[cg] = c1 ? jj : j1[cg];
          }
          f3[cg] = fmaxf(f3[cg], g3);
        }
      }
    }

    // ---- decision, outputs, re-check lists ----
    const float ua = 1.1920929e-7f;  // 2^-23: covers any faithful accumulation rounding
    const float u = 5.9604645e-8f;   // 2^-24
    const float Kf = (float)(A.dp + 1);
    const float gam = Kf * ua / (1.0f - Kf * ua);
    // After the merge every lane of a point holds the point's state, so lane
    // group grp decides point group 4 ps + grp: one pass per four groups,
    // with every lane at work when there are four.
    constexpr int NPS = (NCG + 3) / 4;
    unsigned long long fmask[NPS], gmask[NPS], bmask[NPS];
    int cand2v[NPS], cand3v[NPS];
    int64_t rowv[NPS];
    int nf_w = 0, ng_w = 0, nfull_w = 0;
#pragma unroll
    for (int ps = 0; ps < NPS; ++ps) {
      const int cg = ps * 4 + grp;
      int64_t r = -1;
      unsigned sv1 = 0u, sv2 = 0u, sv3 = 0u, sv4 = 0u, sw3 = 0u;
      float sf1 = 0.f, sf2 = 0.f, sf3 = 0.f;
      int sj1 = 0, sj2 = 0;
#pragma unroll
      for (int c = ps * 4; c < ps * 4 + 4 && c < NCG; ++c) {
        if (cg == c) {
          r = src_row[c];
          sv1 = v1[c]; sv2 = v2[c]; sv3 = v3[c]; sv4 = v4[c]; sw3 = w3[c];
          sf1 = f1[c]; sf2 = f2[c]; sf3 = f3[c]; sj1 = j1[c]; sj2 = j2[c];
        }
      }
      rowv[ps] = r;
      const bool writer = (cg < NCG) && (r >= 0);
      bool flagged = false, full = false;
      int cand2 = 0, cand3 = -1;
      if (writer) {
        const RowStats rw = A.rs[r];
        float t1, t2 = 0.f, t3 = 0.f, t4 = 0.f, E, off;
        int i1, i3 = -1;
        bool has2, has3, has4 = false;
        if constexpr (PK) {
          const unsigned hi = ~mask;
          off = Og;
          if constexpr (BF16) {
            // dp + 1 accumulation steps (the products and the start value),
            // both quantizations, the rounding of O - h_j, the key truncation
            E = gam * (rw.nxq * cqm + Og) + rw.rx * cqm + rw.nx * rcm + u * Og +
                ldexpf(2.0f * Og, A.ib - 23);
          } else {
            // NKU accumulation steps of FP32 rounding, the FP8 instruction's
            // internal summation (2^-10 sum |x~ c~|) and its alignment to the
            // accumulator (2^-19 of |acc in| + sum |x~ c~|, |acc in| <= 2 O), the
            // rounding of O - h_j
            const float gk = (float)NKU * ua;
            const float ga = (float)NKU * 1.9073486e-6f;   // NKU * 2^-19
            E = (9.765625e-4f + gk + ga) * rw.nxq * cqm + (gk + 2.0f * ga) * Og + rw.rx * cqm +
                rw.nx * rcm + u * Og + ldexpf(2.0f * Og, A.ib - 23);
          }
          t1 = __uint_as_float(sv1 & hi);
          i1 = (sv1 & hi) ? min((int)(mask - (sv1 & mask)), A.k - 1) : 0;
          has2 = (sv2 & hi) != 0u;
          has3 = (sv3 & hi) != 0u;
          has4 = (sv4 & hi) != 0u;
          if (has2) {
            t2 = __uint_as_float(sv2 & hi);
            cand2 = min((int)(mask - (sv2 & mask)), A.k - 1);
          }
          if (has3) {
            t3 = __uint_as_float(sv3 & hi);
            i3 = min((int)(mask - (sv3 & mask)), A.k - 1);
          }
          if (has4) t4 = __uint_as_float(sv4 & hi);
        } else {
          off = 0.0f;
          if constexpr (SPLIT) {
            // x_hi.c_hi: dp + 1 accumulation steps over at most (1 + 2^-8)^2
            // sum |x_i c_i|; the cross terms: 2 dp + 1 steps over at most
            // 2^-7 (1 + 2^-8)^2 of it; the dropped part (3.02 2^-16 of it);
            // the sum of the two accumulators and the subtraction of h_j (u
            // each), the rounding of h_j; an absolute term for results and
            // split parts below the smallest normal float (flushed or not)
            const float Kx = (float)(2 * A.dp + 1);
            const float gamx = Kx * ua / (1.0f - Kx * ua);
            E = (1.008f * gam + 0.008f * gamx + 3.1f * 1.52587890625e-5f + 2.04f * u) * rw.nx * cnm +
                1.5f * u * cnm * cnm +
                0x1p-120f * (sqrtf((float)A.dp) * (rw.nx + cnm) + (float)A.dp);
          } else {
            E = (gam + u) * rw.nx * cnm + 1.5f * u * cnm * cnm;
          }
          t1 = sf1;
          i1 = min(max(sj1, 0), A.k - 1);
          has2 = sf2 > -__builtin_inff();
          has3 = sf3 > -__builtin_inff();
          if (has2) {
            t2 = sf2;
            cand2 = min(max(sj2, 0), A.k - 1);
          }
          if (has3) t3 = sf3;
        }
        E *= 1.0001f;
        A.label[r] = A.koff + i1;
        if (A.d1o) A.d1o[r] = fmaxf(rw.xn2 - 2.0f * (t1 - off), 0.0f);
        // squared distance = ||x||^2 - 2 (true score - off); every true score
        // lies within E of its computed (truncated) key; ||x||^2 itself is an
        // FP32 rounding (relative 2^-24)
        const double xhi = (double)rw.xn2 * (1.0 + 0x1p-23), xlo = (double)rw.xn2 * (1.0 - 0x1p-23);
        auto lb_of = [&](float tn) {   // every center whose computed key is <= tn
          return dist_down(xlo - 2.0 * ((double)tn + (double)E - (double)off));
        };
        if (has2) {
          if (A.d2o) A.d2o[r] = fmaxf(rw.xn2 - 2.0f * (t2 - off), 0.0f);
          flagged = (t1 - t2) <= 2.0f * E;
          if (T3 && flagged && (sw3 & ~mask) &&
              (t1 - __uint_as_float(sw3 & ~mask)) <= 2.0f * E) {
            full = true;
          } else if (flagged && has3 && (t1 - t3) <= 2.0f * E) {
            // BF16 keeps a fourth key: three listed candidates suffice unless
            // the fourth is inside the band too
            if (PK) {
              cand3 = i3;
              full = has4 && (t1 - t4) <= 2.0f * E;
            } else {
              full = true;
            }
          }
          if (A.bo.ub && !full) {
            if (!flagged) {
              // decided here: the label's distance, the runner-up's (second
              // key) and every other center's (below the third kept key, or a
              // lane-wise third best that dropped further keys)
              bool hasr = has3;
              float tr = t3;
              if (T3 && (sw3 & ~mask)) {
                const float tw = __uint_as_float(sw3 & ~mask);
                tr = hasr ? fmaxf(tr, tw) : tw;
                hasr = true;
              }
              A.bo.ub[r] = dist_up(xhi - 2.0 * ((double)t1 - (double)E - (double)off));
              A.bo.sec[r] = A.koff + cand2;
              A.bo.l2[r] = lb_of(t2);
              A.bo.lb[r] = hasr ? lb_of(tr) : __builtin_inff();
            } else {
              // listed: the re-check sets the upper bound and completes the
              // lower bound with the listed runner-up; here the centers not
              // listed (below the next kept key, or a lane-wise third best
              // that dropped further keys)
              bool hasn = cand3 >= 0 ? has4 : has3;
              float tn = cand3 >= 0 ? t4 : t3;
              if (T3 && (sw3 & ~mask)) {
                const float tw = __uint_as_float(sw3 & ~mask);
                tn = hasn ? fmaxf(tn, tw) : tw;
                hasn = true;
              }
              A.bo.ub[r] = __builtin_inff();
              A.bo.sec[r] = -1;
              A.bo.lb[r] = hasn ? lb_of(tn) : __builtin_inff();
            }
          }
        } else {
          if (A.d2o) A.d2o[r] = __builtin_inff();
          if (A.bo.ub) {   // a single center
            A.bo.ub[r] = dist_up(xhi - 2.0 * ((double)t1 - (double)E - (double)off));
            A.bo.sec[r] = -1;
            A.bo.l2[r] = __builtin_inff();
            A.bo.lb[r] = __builtin_inff();
          }
        }
      }
      // cascade_all: every undecided row goes to the next GEMM pass
      const bool to_full = (full || (A.cascade_all && flagged)) && (A.full_rows != nullptr);
      const bool to_brute = full && (A.full_rows == nullptr);
      const bool to_flags = flagged && !full && !to_full;
      fmask[ps] = __ballot(to_flags);
      gmask[ps] = __ballot(to_full);
      bmask[ps] = __ballot(to_brute);
      cand2v[ps] = cand2;
      cand3v[ps] = cand3;
      nf_w += __popcll(fmask[ps]);
      ng_w += __popcll(gmask[ps]);
      nfull_w += __popcll(bmask[ps]);
    }
    // one atomic per list and workgroup; waves take consecutive slices
    if (lane == 0) {
      wcnt[0 * WAVES + wave] = nf_w;
      wcnt[1 * WAVES + wave] = ng_w;
      wcnt[2 * WAVES + wave] = nfull_w;
    }
    __syncthreads();
    if (tid == 0) {
      int sf = 0, sg = 0, sx = 0;
      for (int w = 0; w < WAVES; ++w) {
        sf += wcnt[0 * WAVES + w];
        sg += wcnt[1 * WAVES + w];
        sx += wcnt[2 * WAVES + w];
      }
      wbase[0] = sf ? atomicAdd(&A.st->flagged, (unsigned long long)sf) : 0ull;
      wbase[1] = sg ? atomicAdd(A.full_ctr, (unsigned long long)sg) : 0ull;
      wbase[2] = sx ? atomicAdd(&A.st->flagged_full, (unsigned long long)sx) : 0ull;
      if (A.count_undecided && (sf + sg + sx))
        atomicAdd(&A.st->undecided, (unsigned long long)(sf + sg + sx));
    }
    __syncthreads();
    unsigned long long of = wbase[0], og = wbase[1], ob = wbase[2];
    for (int w = 0; w < wave; ++w) {
      of += wcnt[0 * WAVES + w];
      og += wcnt[1 * WAVES + w];
      ob += wcnt[2 * WAVES + w];
    }
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int ps = 0; ps < NPS; ++ps) {
      if ((fmask[ps] >> lane) & 1ull) {
        FlagEntry fe;
        fe.row = (int)(rowv[ps] + A.list_off);
        fe.cand2 = A.koff + cand2v[ps];
        fe.cand3 = cand3v[ps] >= 0 ? A.koff + cand3v[ps] : -1;
        fe.pad = 0;
        A.flags[of + __popcll(fmask[ps] & below)] = fe;
      }
      if ((gmask[ps] >> lane) & 1ull) A.full_rows[og + __popcll(gmask[ps] & below)] =
          (int)(rowv[ps] + A.list_off);
      if ((bmask[ps] >> lane) & 1ull) A.brute[ob + __popcll(bmask[ps] & below)] =
          (int)(rowv[ps] + A.list_off);
      of += __popcll(fmask[ps]);
      og += __popcll(gmask[ps]);
      ob += __popcll(bmask[ps]);
    }
    __syncthreads();
  }
}

// MODE: 0 FP32, 1 BF16, 2 FP8 E4M3, 3 split BF16.  Persistent over the blocks of points.
template <int MODE, int NKU, int NCG, int BN, int WAVES, int PF = 1, bool EP = false,
          int SUBT = 1>
__global__ __launch_bounds__(WAVES * 64) void assign_kernel(AssignArgs A,
                                                            const unsigned long long* row_count,
                                                            const int* __restrict__ gate) {
  if (gate && *gate) return;
  using S = AssignShape<MODE, NKU, NCG, BN, WAVES>;
  __shared__ __attribute__((aligned(1024))) unsigned char lds[2 * S::BUFB];
  __shared__ __attribute__((aligned(16))) float hsh[2 * BN];
  __shared__ int wcnt[3 * WAVES];
  __shared__ unsigned long long wbase[3];
  if (A.rows) A.npts = (int64_t)(*row_count);
  const int64_t nblk = (A.npts + S::PPB - 1) / S::PPB;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x)
    assign_block<MODE, NKU, NCG, BN, WAVES, PF, EP, SUBT>(A, blk, lds, hsh, wcnt, wbase);
}

// ---------------------------------------------------------------------------
// Kernel configurations.
// BF16 rows hold d values and zero padding: dp = 32*NKU with NKU the first
// entry of kBf16Units covering d.  FP8 rows hold d values and zero padding:
// dp = 128*NKU bytes.  FP32 rows are padded to 16*NKU, NKU a power of two.
// Split-BF16 rows are padded like BF16 rows (dp = 32*NKU values per part).
// ---------------------------------------------------------------------------
static const int kBf16Units[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
static const int kF8Units[] = {1, 2, 3, 4, 6, 8};

static int units_for(int prec, int d) {
  if (prec == KMX_BF16 || prec == kSplitBf16) {
    const int need = (d + 31) / 32;
    for (int u : kBf16Units)
      if (u >= need) return u;
    return -1;
  }
  if (prec == KMX_FP8E4M3) {
    const int need = (d + 127) / 128;
    for (int u : kF8Units)
      if (u >= need) return u;
    return -1;
  }
  const int need = (d + 15) / 16;
  int p = 1;
  while (p < need) p <<= 1;
  return p <= 64 ? p : -1;
}

int assign_dpad(int prec, int d) {
  const int u = units_for(prec, d);
  if (u < 0) return -1;
  return u * ((prec == KMX_BF16 || prec == kSplitBf16) ? 32 : (prec == KMX_FP8E4M3) ? 128 : 16);
}

// FP8 rows of 4 units (d <= 512) with many centers: LDS tiles of 64 or 128
// centers taken as sub-tiles of 32 (one tile barrier per tile); with few
// centers, tiles of 32 (less padding).
static int f8_tile4(int k) { return k > 512 ? 128 : (k > 256 ? 64 : 32); }

// Centers per LDS tile: each of the two tile buffers stays within ~72 KB.
int assign_tile_n(int prec, int d, int k) {
  const int nku = units_for(prec, d);
  if (prec == KMX_FP8E4M3)
    return nku <= 3 ? 64 : (nku == 4 ? f8_tile4(k) : (nku <= 6 ? 32 : 16));
  if (prec == KMX_BF16) return (nku <= 3 || nku == 6 || nku == 8) ? 64 : 32;
  if (prec == kSplitBf16) return nku <= 16 ? 32 : 16;
  if (nku <= 4) return 64;
  if (nku <= 32) return 32;
  return 16;
}

template <int MODE, int NKU, int NCG, int BN, int WAVES, int PF = 1, bool EP = false,
          int SUBT = 1>
static hipError_t run_assign(hipStream_t s, const void* Xsrc, int64_t xs, int vec_ok,
                             const uint8_t* sx8, int64_t n, const int* rows,
                             const unsigned long long* row_count, int d, int dp,
                             const RowStats* rs, const void* Cq, const float* ch, int k, int kpad,
                             int ib, const CenterStats* cs, int32_t* label, float* d1, float* d2,
                             FlagEntry* flags, int* full_rows, unsigned long long* full_ctr,
                             int cascade_all, int* brute, LoopState* st, const int* gate,
                             int num_cus, BoundsOut bo) {
  if (kpad % BN != 0) return hipErrorInvalidValue;   // center padding must match the tile
  AssignArgs A;
  A.Xsrc = Xsrc;
  A.xs = xs;
  A.vec_ok = vec_ok;
  A.sx8 = sx8;
  A.npts = n;
  A.rows = rows;
  A.d = d;
  A.dp = dp;
  A.rs = rs;
  A.Cq = Cq;
  A.ch = ch;
  A.k = k;
  A.kpad = kpad;
  A.ib = ib;
  A.cs = cs;
  A.label = label;
  A.d1o = d1;
  A.d2o = d2;
  A.koff = 0;
  A.list_off = 0;
  A.flags = flags;
  A.full_rows = full_rows;
  A.full_ctr = full_ctr;
  A.cascade_all = cascade_all;
  A.brute = brute;
  A.st = st;
  A.count_undecided = rows == nullptr;
  A.bo = bo;
  const int64_t ppb = (int64_t)WAVES * 16 * NCG;
  int64_t blocks = (n + ppb - 1) / ppb;
  if (rows) {
    const int64_t cap = (int64_t)num_cus * 2;
    if (blocks > cap) blocks = cap;
  }
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((assign_kernel<MODE, NKU, NCG, BN, WAVES, PF, EP, SUBT>), dim3((unsigned)blocks),
                     dim3(WAVES * 64), 0, s, A, row_count, gate);
  return hipGetLastError();
}

hipError_t launch_assign(hipStream_t s, int prec, const float* X, int64_t ldx, const void* Xq,
                         const uint8_t* sx8, int64_t n, const int* rows,
                         const unsigned long long* row_count, int d, int dp, const RowStats* rs,
                         const void* Cq, const float* ch, int k, int kpad, const CenterStats* cs,
                         int32_t* label, float* d1, float* d2, FlagEntry* flags, int* full_rows,
                         unsigned long long* full_ctr, int cascade_all, int* brute, LoopState* st,
                         const int* gate, int num_cus, BoundsOut bo) {
  int ib = 1;
  while ((1 << ib) < kpad) ++ib;
  const int nku = units_for(prec, d);
  if (prec == KMX_BF16) {
#define KMX_A(NKU_, NCG_, BN_, W_, EP_)                                                          \
  return run_assign<1, NKU_, NCG_, BN_, W_, 1, EP_>(s, Xq, dp, 1, nullptr, n, rows, row_count, d, dp, rs, \
                                            Cq, ch, k, kpad, ib, cs, label, d1, d2, flags,      \
                                            full_rows, full_ctr, cascade_all, brute, st, gate, num_cus, bo)
    switch (nku) {
      case 1: KMX_A(1, 4, 64, 8, false);
      case 2: KMX_A(2, 4, 64, 8, false);
      case 3: KMX_A(3, 4, 64, 8, false);
      case 4: KMX_A(4, 4, 32, 8, false);
      case 6: KMX_A(6, 2, 64, 8, false);
      case 8: KMX_A(8, 2, 64, 8, false);
      case 12: KMX_A(12, 2, 32, 8, false);
      case 16: KMX_A(16, 2, 32, 8, false);
      case 24: KMX_A(24, 1, 32, 8, false);
      case 32: KMX_A(32, 1, 32, 8, false);
      default: return hipErrorInvalidValue;
    }
#undef KMX_A
  }
  if (prec == KMX_FP8E4M3) {
    if (!sx8) return hipErrorInvalidValue;
#define KMX_A(NKU_, NCG_, BN_, W_, EP_, SUB_)                                                \
  return run_assign<2, NKU_, NCG_, BN_, W_, 1, EP_, SUB_>(s, Xq, dp, 1, sx8, n, rows, row_count, d, dp, rs, \
                                            Cq, ch, k, kpad, ib, cs, label, d1, d2, flags,  \
                                            full_rows, full_ctr, cascade_all, brute, st, gate, num_cus, bo)
    switch (nku) {
      case 1: KMX_A(1, 4, 64, 8, true, 1);
      case 2: KMX_A(2, 4, 64, 8, false, 1);
      case 3: KMX_A(3, 2, 64, 8, false, 1);
      case 4:
        if (f8_tile4(k) == 128) KMX_A(4, 4, 128, 8, false, 4);
        if (f8_tile4(k) == 64) KMX_A(4, 4, 64, 8, false, 2);
        KMX_A(4, 4, 32, 8, false, 1);
      case 6: KMX_A(6, 1, 32, 8, true, 1);
      case 8: KMX_A(8, 1, 16, 8, true, 1);
      default: return hipErrorInvalidValue;
    }
#undef KMX_A
  }
  const int vec_ok = ((((uintptr_t)X) & 15) == 0) && (ldx % 4 == 0);
  if (prec == kSplitBf16) {
    // point fragments (high + low parts) and two accumulators per center
    // block: fewer point groups per wave than BF16 at the same width
#define KMX_A(NKU_, NCG_, BN_, W_)                                                               \
  return run_assign<3, NKU_, NCG_, BN_, W_>(s, X, ldx, vec_ok, nullptr, n, rows, row_count, d, \
                                            dp, rs, Cq, ch, k, kpad, ib, cs, label, d1, d2,     \
                                            flags, full_rows, full_ctr, cascade_all, brute, st, gate, num_cus, bo)
    switch (nku) {
      case 1: KMX_A(1, 4, 32, 8);
      case 2: KMX_A(2, 4, 32, 8);
      case 3: KMX_A(3, 2, 32, 8);
      case 4: KMX_A(4, 2, 32, 8);
      case 6: KMX_A(6, 2, 32, 8);
      case 8: KMX_A(8, 1, 32, 8);
      case 12: KMX_A(12, 1, 32, 8);
      case 16: KMX_A(16, 1, 32, 8);
      case 24: KMX_A(24, 1, 16, 4);
      case 32: KMX_A(32, 1, 16, 4);
      default: return hipErrorInvalidValue;
    }
#undef KMX_A
  }
#define KMX_A(NKU_, NCG_, BN_, W_)                                                               \
  return run_assign<0, NKU_, NCG_, BN_, W_>(s, X, ldx, vec_ok, nullptr, n, rows, row_count, d, \
                                            dp, rs, Cq, ch, k, kpad, ib, cs, label, d1, d2,     \
                                            flags, full_rows, full_ctr, cascade_all, brute, st, gate, num_cus, bo)
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

}  // namespace kmx

namespace kmx {

// ---------------------------------------------------------------------------
// Batched assignment: the instances of a batched Lloyd call, one persistent
// launch per width group.  A work item is one block of points of one
// instance; the instance's variant selects the tile shape (point groups per
// wave, centers per tile), its own centers and statistics.  Items are ordered
// by decreasing cost and taken round-robin by the workgroups.
// ---------------------------------------------------------------------------
constexpr int kBatchWaves = 8;
// (variant id, BF16 units, point groups per wave, centers per tile); three
// shapes per width group (BF16 units 1, 2, 4, 8, 12, 16).
#define KMX_BG0(X) X(0, 1, 4, 64) X(1, 1, 4, 16) X(2, 1, 2, 32)
#define KMX_BG1(X) X(3, 2, 4, 64) X(4, 2, 4, 16) X(5, 2, 2, 32)
#define KMX_BG2(X) X(6, 4, 4, 32) X(7, 4, 4, 16) X(8, 4, 2, 64)
#define KMX_BG3(X) X(9, 8, 2, 64) X(10, 8, 2, 16) X(11, 8, 2, 32)
#define KMX_BG4(X) X(12, 12, 2, 32) X(13, 12, 2, 16) X(14, 12, 1, 32)
#define KMX_BG5(X) X(15, 16, 2, 32) X(16, 16, 2, 16) X(17, 16, 1, 32)
#define KMX_BVARIANTS(X) KMX_BG0(X) KMX_BG1(X) KMX_BG2(X) KMX_BG3(X) KMX_BG4(X) KMX_BG5(X)

constexpr int bmax(int a, int b) { return a > b ? a : b; }
template <int NKU, int NCG, int BN>
constexpr int bbuf() {
  return AssignShape<1, NKU, NCG, BN, kBatchWaves>::BUFB;
}
#define KMX_BUFMAX(ID, NKU, NCG, BN) bmax(bbuf<NKU, NCG, BN>(),
#define KMX_CLOSE(ID, NKU, NCG, BN) )
constexpr int kGroupBuf[6] = {
    KMX_BG0(KMX_BUFMAX) 0 KMX_BG0(KMX_CLOSE), KMX_BG1(KMX_BUFMAX) 0 KMX_BG1(KMX_CLOSE),
    KMX_BG2(KMX_BUFMAX) 0 KMX_BG2(KMX_CLOSE), KMX_BG3(KMX_BUFMAX) 0 KMX_BG3(KMX_CLOSE),
    KMX_BG4(KMX_BUFMAX) 0 KMX_BG4(KMX_CLOSE), KMX_BG5(KMX_BUFMAX) 0 KMX_BG5(KMX_CLOSE)};
#undef KMX_BUFMAX
#undef KMX_CLOSE

struct BVariant {
  int nku, ncg, bn;
};
#define KMX_BV(ID, NKU, NCG, BN) {NKU, NCG, BN},
static const BVariant kBVariants[] = {KMX_BVARIANTS(KMX_BV)};
#undef KMX_BV

static const int kBatchGroupUnits[6] = {1, 2, 4, 8, 12, 16};

static int batch_group(int d) {
  const int need = (d + 31) / 32;
  for (int g = 0; g < 6; ++g)
    if (d >= 1 && kBatchGroupUnits[g] >= need) return g;
  return -1;
}

int batched_dpad(int d) {
  const int g = batch_group(d);
  return g < 0 ? -1 : 32 * kBatchGroupUnits[g];
}

int batched_variants(int d) { return batch_group(d) < 0 ? 0 : 3; }
int batched_variant_id(int d, int v) { return 3 * batch_group(d) + v; }
int batched_variant_tile(int d, int v) { return kBVariants[batched_variant_id(d, v)].bn; }
int batched_variant_ppb(int d, int v) {
  return kBatchWaves * 16 * kBVariants[batched_variant_id(d, v)].ncg;
}

// One item of the batched assignment: the instance's rows and centers as
// assign_block arguments.
template <int NKU, int NCG, int BN>
__device__ __forceinline__ void batched_block(const BatchInst& I, int blk,
                                              FlagEntry* __restrict__ flags,
                                              int* __restrict__ brute, LoopState* __restrict__ st,
                                              int32_t* __restrict__ label, unsigned char* lds,
                                              float* hsh, int* wcnt, unsigned long long* wbase) {
  AssignArgs A;
  A.Xsrc = I.xq + I.row0 * I.dp;
  A.xs = I.dp;
  A.vec_ok = 1;
  A.sx8 = nullptr;
  A.npts = I.n;
  A.rows = nullptr;
  A.d = I.d;
  A.dp = I.dp;
  A.rs = I.rs + I.row0;
  A.Cq = I.cq + (int64_t)I.cpad0 * I.dp;
  A.ch = I.ch + I.hd0;
  A.k = I.k;
  A.kpad = I.kpad;
  A.ib = I.ib;
  A.cs = I.cs;
  A.label = label + I.grow0;
  A.d1o = nullptr;
  A.d2o = nullptr;
  A.koff = I.koff;
  A.list_off = I.grow0;
  A.flags = flags;
  A.full_rows = nullptr;
  A.full_ctr = nullptr;
  A.cascade_all = 0;
  A.brute = brute;
  A.st = st;
  A.count_undecided = 1;
  A.bo = BoundsOut();
  assign_block<1, NKU, NCG, BN, kBatchWaves, 1, false, 1>(A, blk, lds, hsh, wcnt, wbase);
}

// Persistent over the items [begin, end) of one width group; each item's
// instance selects one of the group's three tile shapes.  (Calls to
// out-of-line per-shape functions gave wrong labels on gfx950; every shape
// is inlined here.)
template <int G>
__global__ __launch_bounds__(kBatchWaves * 64) void assign_batched_kernel(
    const BatchItem* __restrict__ items, int begin, int end, const BatchInst* __restrict__ insts,
    FlagEntry* __restrict__ flags, int* __restrict__ brute, LoopState* __restrict__ st,
    int32_t* __restrict__ label) {
  __shared__ __attribute__((aligned(1024))) unsigned char lds[2 * kGroupBuf[G]];
  __shared__ __attribute__((aligned(16))) float hsh[2 * 64];
  __shared__ int wcnt[3 * kBatchWaves];
  __shared__ unsigned long long wbase[3];
  for (int it = begin + (int)blockIdx.x; it < end; it += (int)gridDim.x) {
    const BatchItem item = items[it];
    const BatchInst& I = insts[item.inst];
#define KMX_BCASE(ID, NKU, NCG, BN)                                                           \
  case ID:                                                                                    \
    batched_block<NKU, NCG, BN>(I, item.blk, flags, brute, st, label, lds, hsh, wcnt, wbase); \
    break;
#define KMX_GROUP_CASES(GG, LIST)                         \
  if constexpr (G == GG) {                                \
    switch (I.variant) { LIST(KMX_BCASE) default: break; } \
  }
    KMX_GROUP_CASES(0, KMX_BG0)
    KMX_GROUP_CASES(1, KMX_BG1)
    KMX_GROUP_CASES(2, KMX_BG2)
    KMX_GROUP_CASES(3, KMX_BG3)
    KMX_GROUP_CASES(4, KMX_BG4)
    KMX_GROUP_CASES(5, KMX_BG5)
#undef KMX_GROUP_CASES
#undef KMX_BCASE
  }
}

int batched_group(int d) { return batch_group(d); }

hipError_t launch_assign_batched(hipStream_t s, int group, const BatchItem* items, int begin,
                                 int end, const BatchInst* insts, FlagEntry* flags, int* brute,
                                 LoopState* st, int32_t* label, int grid) {
  const int nitems = end - begin;
  if (nitems <= 0) return hipSuccess;
  if (grid < 1) grid = 1;
  if (grid > nitems) grid = nitems;
  switch (group) {
#define KMX_G(G)                                                                                \
  case G:                                                                                       \
    hipLaunchKernelGGL(assign_batched_kernel<G>, dim3((unsigned)grid), dim3(kBatchWaves * 64), \
                       0, s, items, begin, end, insts, flags, brute, st, label);               \
    return hipGetLastError();
    KMX_G(0)
    KMX_G(1)
    KMX_G(2)
    KMX_G(3)
    KMX_G(4)
    KMX_G(5)
#undef KMX_G
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace kmx
