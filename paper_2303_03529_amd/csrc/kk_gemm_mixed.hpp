// Split-precision (FP16 x 3) MFMA transforms for gfx950.
//
// Each FP64 operand M is held as two FP16 matrices, M_hi = fp16(s M) and
// M_lo = fp16(s M - M_hi), with a power-of-two scale s chosen so that
// max |s M| <= 2^14. Their sum carries ~22 significant bits. A product is
// formed from three FP16 MFMA products, A_hi B_hi + A_hi B_lo + A_lo B_hi,
// accumulated in FP32 by v_mfma_f32_32x32x16_f16; the dropped A_lo B_lo term
// and the FP32 accumulation leave a relative error of a few 1e-7 per entry.
// Everything outside the products stays FP64: the unscaling, the Fermi
// divided differences and their Hadamard product, the diagonal capture for
// the chemical-potential shift and the Mulliken dot products with G.
//
// Layout (NT form): out[m][n] = sum_k At[m][k] * Bt[n][k] with At, Bt stored
// row-major with k contiguous, so each lane's 8 FP16 MFMA operands are one
// 16-byte LDS read. The forward transform is a full-tile product A = C^T U~ G
// (At = (U~ C)^T, Bt = G^T; EPI_STORE: A in FP32) followed by fermi_symmetrize,
// which forms X = (A + A^T) / 2 in FP64 and Y = F o X. The back-transform uses
// At = C (row i, k = l) and Bt = Y (symmetric, so row k of Y is column k).
#pragma once

#include <hip/hip_runtime.h>

#include "kk_gemm.hpp"

namespace kk {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16x __attribute__((ext_vector_type(16)));

// Products of a split pass, as a mask over the operand pairs (At piece, Bt piece) of a stage:
// bit 0 (1, 0), bit 1 (0, 1), bit 2 (0, 0), bit 3 (1, 1), bit 4 (0, 2), bit 5 (2, 0); bits 4
// and 5 stream a third piece of each operand (direct-to-LDS loop only).
constexpr int PROD_F16X3 = 0x7;   // FP16: hi lo, lo hi, hi hi
constexpr int PROD_RES = 0x30;    // hi res and res hi on the third pieces (the BF16 refinement)
constexpr int PROD_ALL6 = 0x3F;   // BF16: hi hi, hi lo, lo hi, lo lo and PROD_RES, in one pass

// One 32 x 32 x 16 MFMA on 16-bit operands held as raw 8-element registers.
template <bool BF16>
__device__ __forceinline__ f16x mfma16(const h8& a, const h8& b, const f16x& c) {
  if constexpr (BF16)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0,
                                                   0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Every 16-bit operand buffer is typed _Float16; on a BF16 handle it holds BF16 bit patterns.
template <bool BF16>
__device__ __forceinline__ _Float16 to16(double v) {
  if constexpr (BF16)
    return __builtin_bit_cast(_Float16, (__bf16)(float)v);
  else
    return (_Float16)(float)v;
}
template <bool BF16>
__device__ __forceinline__ double from16(_Float16 x) {
  if constexpr (BF16)
    return (double)(float)__builtin_bit_cast(__bf16, x);
  else
    return (double)x;
}

struct MixedItem {
  const _Float16 *a0h, *a0l, *b0h, *b0l;  // At, Bt as two 16-bit pieces each, [n][n], k contiguous
  const _Float16 *a0r, *b0r;              // their third pieces (products with PROD_RES bits)
  _Float16 *yh, *yl, *yr;                 // forward: Y split at scale sc[1] (yr: third BF16 piece)
  const double* g;                        // back: G (FP64)
  const double *eps, *f, *fc, *w;         // forward: spectrum
  double* xdiag;                          // forward: diag X
  double* part;                           // back: Mulliken partials [parts][n]
  const double* sc;                       // device scalars: [0] = 1 / product scale, [1] = Y scale
  float* x32;                             // EPI_STORE: the product A in FP32, [n][n]
};

struct MixedArgs {
  int n, k, ntiles, nitems;  // padded size, contraction length (<= n), tiles per item, items
  const int2* tiles;
  const int* stop;
  double beta;
  // Stream-K schedule (gemm_mixed_sk; sk_grid = 0 for one workgroup per tile): the
  // nitems x ntiles x (k / 32) K stages of a launch, in the order (item, tile of the table,
  // stage), are cut into sk_grid equal ranges, one per workgroup. The j-th segment of a tile
  // (along K) stores its partial result in slot j of the item's output, sk_stride elements
  // after slot j - 1; slots past a tile's last segment, up to sk_slots, are cleared
  // (Mulliken partials) or not read (the symmetrizing pass, which finds the segment count of
  // each sk_side x sk_side tile from its table position, tile_table_pos).
  int sk_grid, sk_slots, sk_side;
  size_t sk_stride;
  MixedItem item[MAX_GEMM_BATCH];
};

// Position of tile (tm, tn) of a TM x TN grid in the tile table: groups of TILE_GROUP tile
// rows, each group walked column by column (within a column, row by row).
constexpr int TILE_GROUP = 4;
__host__ __device__ inline int tile_table_pos(int tm, int tn, int TM, int TN) {
  const int g0 = tm - tm % TILE_GROUP, gr = TM - g0 < TILE_GROUP ? TM - g0 : TILE_GROUP;
  return g0 * TN + tn * gr + (tm - g0);
}

// Stream-K: the workgroup whose range [w total / grid, (w + 1) total / grid) holds stage x,
// and the number of segments of launch tile t (nk stages each).
__host__ __device__ inline int sk_owner(long x, int grid, long total) {
  return (int)(((x + 1) * grid - 1) / total);
}
__host__ __device__ inline int sk_segments(int t, int nk, int grid, long total) {
  return sk_owner((long)(t + 1) * nk - 1, grid, total) - sk_owner((long)t * nk, grid, total) + 1;
}

template <int BM_, int BN_, int BK_, int WAVES_M_, int WAVES_N_, int MINB_, int FLUSH_ = 0, bool BF16_ = false,
          int PROD_ = PROD_F16X3>
struct MixedCfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_;
  static constexpr bool BF16 = BF16_;
  static constexpr int PROD = PROD_;
  // FLUSH > 0: accumulate FLUSH stages in a fresh FP32 accumulator, then add it
  // to a running FP32 total (two-level summation, smaller rounding growth).
  static constexpr int FLUSH = FLUSH_;
  static constexpr int WAVES_M = WAVES_M_, WAVES_N = WAVES_N_;
  static constexpr int THREADS = 64 * WAVES_M * WAVES_N;
  static constexpr int WTM = BM / WAVES_M / 32;
  static constexpr int WTN = BN / WAVES_N / 32;
  static constexpr int MIN_BLOCKS = MINB_;
  static constexpr bool DL = false;
  static constexpr int KP = BK + 8;                 // padded LDS row (halves)
  static_assert((KP / 8) % 2 == 1, "LDS row stride must be an odd number of 16-byte slots");
  static constexpr int SMEM_BYTES = 2 * 2 * (BM + BN) * KP * 2;  // [buf][hi/lo] of A and B
  static_assert(64 % (BK / 8) == 0 && 16 % (BK / 8) == 0, "piece mapping");
  static_assert(BM % (32 * WAVES_M) == 0 && BN % (32 * WAVES_N) == 0, "wave tiling");
  static_assert(BK % 16 == 0, "BK");
  static_assert((PROD & PROD_RES) == 0, "third pieces need the direct-to-LDS loop");
};

// Configuration of the direct-to-LDS main loop: BM x BN tile, K stage 32, a ring
// of NS stages in LDS, one workgroup per CU.
template <int BM_, int BN_, int WAVES_M_, int WAVES_N_, int NS_, int FLUSH_, bool BF16_ = false,
          int PROD_ = PROD_F16X3>
struct MixedDlCfg {
  static constexpr bool DL = true;
  static constexpr bool BF16 = BF16_;
  static constexpr int PROD = PROD_;
  static constexpr int BM = BM_, BN = BN_, BK = 32, NS = NS_, FLUSH = FLUSH_;
  static constexpr int WAVES_M = WAVES_M_, WAVES_N = WAVES_N_, WAVES = WAVES_M * WAVES_N;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int WTM = BM / WAVES_M / 32, WTN = BN / WAVES_N / 32;
  static constexpr int MIN_BLOCKS = 1;
  static constexpr int A_BLK = BM / 16, B_BLK = BN / 16;     // 1 KB blocks of 16 rows
  static constexpr int NPC = (PROD & PROD_RES) ? 3 : 2;        // pieces of each operand streamed
  static constexpr int STAGE_BLK = NPC * (A_BLK + B_BLK);      // hi, lo (and the third piece) of A and B
  static constexpr int PER_WAVE = STAGE_BLK / WAVES;
  static constexpr int STAGE_BYTES = STAGE_BLK * 1024;
  static constexpr int SMEM_BYTES = NS * STAGE_BYTES;
  static_assert(STAGE_BLK % WAVES == 0, "DMA blocks per wave");
  static_assert(BM % (32 * WAVES_M) == 0 && BN % (32 * WAVES_N) == 0, "wave tiling");
  static_assert(NS >= 2 && NS <= 5, "ring depth");
  static_assert(NS * STAGE_BYTES <= 160 * 1024, "LDS");
};

// LDS of one split-precision tile's main loop (one static buffer per configuration).
template <class Cfg>
__device__ __forceinline__ unsigned char* mixed_smem() {
  __shared__ __attribute__((aligned(1024))) unsigned char smem[Cfg::SMEM_BYTES];
  return smem;
}

// The NP 16-bit pieces of v: p0 = round(v), p1 = round(v - p0), p2 = round(v - p0 - p1).
template <bool BF16, int NP>
__device__ __forceinline__ void split_pieces(double v, _Float16 (&p)[NP]) {
  double r = v;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    p[q] = to16<BF16>(r);
    if (q + 1 < NP) r -= from16<BF16>(p[q]);
  }
}

// Main loop with register staging: global -> registers -> LDS (double buffer).
// Leaves the FP32 sums in acc; ends with a barrier.
template <class Cfg>
__device__ __forceinline__ void mixed_mainloop_lds(const MixedItem& it, const int n, const int kc, const int m0,
                                                   const int n0, f16x (&acc)[Cfg::WTM][Cfg::WTN]) {
  constexpr int BM = Cfg::BM, BN = Cfg::BN, BK = Cfg::BK, KP = Cfg::KP;
  constexpr int WTM = Cfg::WTM, WTN = Cfg::WTN;
  constexpr int CPR = BK / 8;  // 16-byte chunks per row per matrix

  // [buf][hi/lo][row][k]
  auto As = reinterpret_cast<_Float16 (*)[2][BM][KP]>(mixed_smem<Cfg>());
  auto Bs = reinterpret_cast<_Float16 (*)[2][BN][KP]>(mixed_smem<Cfg>() + 2 * 2 * BM * KP * 2);

  const int tid = threadIdx.x;
  const int nk = kc / BK;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave / Cfg::WAVES_N, wn = wave % Cfg::WAVES_N;
  const int l32 = lane & 31, lh = lane >> 5;

  f16x tot[Cfg::FLUSH > 0 ? WTM : 1][Cfg::FLUSH > 0 ? WTN : 1];
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int j = 0; j < WTN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  if constexpr (Cfg::FLUSH > 0) {
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int j = 0; j < WTN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[i][j][r] = 0.f;
  }

  // Staging: each thread moves APM 16-byte pieces of A_hi and of A_lo, and BPM
  // of B_hi and B_lo, per stage. Offsets are fixed for the whole K loop.
  constexpr int APM = BM * CPR / Cfg::THREADS, BPM = BN * CPR / Cfg::THREADS;
  static_assert(APM * Cfg::THREADS == BM * CPR && BPM * Cfg::THREADS == BN * CPR, "piece split");
  int aoff[APM], boff[BPM], alds[APM], blds[BPM];
  // Piece c -> (row, chunk): CPR consecutive lanes share a row (coalesced loads),
  // and the 16 lanes of one LDS write pass take rows r, r + 16/CPR, ... so that
  // their 16-byte slots (row stride KP = odd multiple of 8 halves) hit distinct banks.
  auto piece = [](int c, int& row, int& ch) __attribute__((always_inline)) {
    constexpr int RPW = 64 / CPR;          // rows per wave-instruction
    constexpr int RPP = 16 / CPR;          // rows per 16-lane pass
    const int l = c % 64, q = l / CPR;
    row = (c / 64) * RPW + (q % RPP) * (RPW / RPP) + q / RPP;
    ch = l % CPR;
  };
#pragma unroll
  for (int p = 0; p < APM; ++p) {
    int row, ch;
    piece(tid + p * Cfg::THREADS, row, ch);
    aoff[p] = (m0 + row) * n + ch * 8;
    alds[p] = row * KP + ch * 8;
  }
#pragma unroll
  for (int p = 0; p < BPM; ++p) {
    int row, ch;
    piece(tid + p * Cfg::THREADS, row, ch);
    boff[p] = (n0 + row) * n + ch * 8;
    blds[p] = row * KP + ch * 8;
  }
  h8 sah[APM], sal[APM], sbh[BPM], sbl[BPM];

#define KK_MLOAD(kt)                                                                         \
  {                                                                                          \
    const int k0 = (kt) * BK;                                                                \
    const _Float16 *ah = it.a0h + k0, *al = it.a0l + k0, *bh = it.b0h + k0, *bl = it.b0l + k0; \
    _Pragma("unroll") for (int p = 0; p < APM; ++p) {                                        \
      sah[p] = *reinterpret_cast<const h8*>(ah + aoff[p]);                                   \
      sal[p] = *reinterpret_cast<const h8*>(al + aoff[p]);                                   \
    }                                                                                        \
    _Pragma("unroll") for (int p = 0; p < BPM; ++p) {                                        \
      sbh[p] = *reinterpret_cast<const h8*>(bh + boff[p]);                                   \
      sbl[p] = *reinterpret_cast<const h8*>(bl + boff[p]);                                   \
    }                                                                                        \
  }
#define KK_MSTORE(buf)                                                                       \
  {                                                                                          \
    _Pragma("unroll") for (int p = 0; p < APM; ++p) {                                        \
      *reinterpret_cast<h8*>(&As[buf][0][0][0] + alds[p]) = sah[p];                          \
      *reinterpret_cast<h8*>(&As[buf][1][0][0] + alds[p]) = sal[p];                          \
    }                                                                                        \
    _Pragma("unroll") for (int p = 0; p < BPM; ++p) {                                        \
      *reinterpret_cast<h8*>(&Bs[buf][0][0][0] + blds[p]) = sbh[p];                          \
      *reinterpret_cast<h8*>(&Bs[buf][1][0][0] + blds[p]) = sbl[p];                          \
    }                                                                                        \
  }

  KK_MLOAD(0);
  KK_MSTORE(0);
  __syncthreads();

  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) KK_MLOAD(kt + 1);
#pragma unroll
    for (int ks = 0; ks < BK / 16; ++ks) {
      h8 ah[WTM], al[WTM], bh[WTN], bl[WTN];
      const int kofs = ks * 16 + lh * 8;
#pragma unroll
      for (int i = 0; i < WTM; ++i) {
        const int r = wm * (BM / Cfg::WAVES_M) + i * 32 + l32;
        ah[i] = *reinterpret_cast<const h8*>(&As[buf][0][r][kofs]);
        al[i] = *reinterpret_cast<const h8*>(&As[buf][1][r][kofs]);
      }
#pragma unroll
      for (int j = 0; j < WTN; ++j) {
        const int r = wn * (BN / Cfg::WAVES_N) + j * 32 + l32;
        bh[j] = *reinterpret_cast<const h8*>(&Bs[buf][0][r][kofs]);
        bl[j] = *reinterpret_cast<const h8*>(&Bs[buf][1][r][kofs]);
      }
      // the products cycle over the accumulators so no MFMA waits on the previous one
      constexpr bool BF = Cfg::BF16;
      if constexpr (Cfg::PROD & 8) {
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
          for (int j = 0; j < WTN; ++j) acc[i][j] = mfma16<BF>(al[i], bl[j], acc[i][j]);
      }
      if constexpr (Cfg::PROD & 1) {
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
          for (int j = 0; j < WTN; ++j) acc[i][j] = mfma16<BF>(al[i], bh[j], acc[i][j]);
      }
      if constexpr (Cfg::PROD & 2) {
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
          for (int j = 0; j < WTN; ++j) acc[i][j] = mfma16<BF>(ah[i], bl[j], acc[i][j]);
      }
      if constexpr (Cfg::PROD & 4) {
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
          for (int j = 0; j < WTN; ++j) acc[i][j] = mfma16<BF>(ah[i], bh[j], acc[i][j]);
      }
    }
    if constexpr (Cfg::FLUSH > 0) {
      if ((kt + 1) % Cfg::FLUSH == 0 || !more) {
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
          for (int j = 0; j < WTN; ++j) {
            tot[i][j] += acc[i][j];
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
          }
      }
    }
    if (more) KK_MSTORE(buf ^ 1);
    __syncthreads();
  }
#undef KK_MLOAD
#undef KK_MSTORE
  if constexpr (Cfg::FLUSH > 0) {
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int j = 0; j < WTN; ++j) acc[i][j] = tot[i][j];
  }
}

// Epilogue of a split-precision tile (both forms of the main loop).
template <int EPI, class Cfg>
__device__ __forceinline__ void mixed_epilogue(const MixedItem& it, const int n, const int2 tile,
                                               const f16x (&acc)[Cfg::WTM][Cfg::WTN]) {
  constexpr int BM = Cfg::BM, BN = Cfg::BN;
  constexpr int WTM = Cfg::WTM, WTN = Cfg::WTN;
  const int m0 = tile.x * BM, n0 = tile.y * BN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave / Cfg::WAVES_N, wn = wave % Cfg::WAVES_N;
  const int l32 = lane & 31, lh = lane >> 5;
  // Accumulator element (i, j, r) of this lane:
  //   m = m0 + wm*(BM/WAVES_M) + i*32 + 8*(r/4) + 4*lh + r%4,  n = n0 + wn*(BN/WAVES_N) + j*32 + l32.
  const double inv = it.sc[0];
  const int mw = m0 + wm * (BM / Cfg::WAVES_M) + 4 * lh;
  const int nw = n0 + wn * (BN / Cfg::WAVES_N) + l32;
  if constexpr (EPI == EPI_STORE) {
    // 32 consecutive columns of one row per instruction and accumulator element
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = mw + i * 32 + 8 * (r / 4) + (r % 4);
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
          float* o = it.x32 + (size_t)m * n + nw + j * 32;
          *o = acc[i][j][r];
        }
      }
  } else if constexpr (!Cfg::DL || Cfg::THREADS > 256) {  // EPI_MULLIKEN
    // Each row sum over the lane's columns, summed over the 32 lanes of its half-wave (the
    // wave's columns) one row at a time.
    const int p = tile.y * Cfg::WAVES_N + wn;
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = mw + i * 32 + 8 * (r / 4) + (r % 4);
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < WTN; ++j) s += (double)acc[i][j][r] * it.g[(size_t)m * n + nw + j * 32];
        s *= inv;
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        s += __shfl_xor(s, 8);
        s += __shfl_xor(s, 16);
        if (l32 == 0) it.part[(size_t)p * n + m] = s;
      }
  } else {  // EPI_MULLIKEN, 4-wave direct-to-LDS tiles (64 x 64)
    // The short contractions of these tiles leave the epilogue a large share of the kernel:
    // the lane's Q = 16 WTM row sums over its columns are summed over the 32 lanes of its
    // half-wave by a transposing butterfly. At the step over lane bit b a lane keeps the half
    // of its sums selected by that bit and adds its partner's copy of them, so the half-wave
    // ends with one complete row sum per lane (or lane pair): Q or Q - 1 exchanges instead
    // of 5 Q, and one store for the wave's rows (16 to 56 atoms: 4-8 % more updates/s in
    // both split forms; on 8-wave tiles level at 128 atoms and 1 % slower with stream-K at
    // 170 atoms).
    constexpr int Q = WTM * 16;
    static_assert(Q == 16 || Q == 32, "one or two row sums per lane pair");
    const int p = tile.y * Cfg::WAVES_N + wn;
    double v[Q];
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = mw + i * 32 + 8 * (r / 4) + (r % 4);
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < WTN; ++j) s += (double)acc[i][j][r] * it.g[(size_t)m * n + nw + j * 32];
        v[i * 16 + r] = s * inv;
      }
#pragma unroll
    for (int b = 4; b >= 0; --b) {
      const int h = Q >> (5 - b);  // sums kept after this step (0: a plain pair sum)
      if (h == 0) {
        v[0] += __shfl_xor(v[0], 1 << b);
      } else {
        const bool upper = (l32 >> b) & 1;
#pragma unroll
        for (int k = 0; k < h; ++k) {
          const double keep = upper ? v[k + h] : v[k];
          const double send = upper ? v[k] : v[k + h];
          v[k] = keep + __shfl_xor(send, 1 << b);
        }
      }
    }
    // lane bits 4..0 (Q = 32) or 4..1 (Q = 16) are the bits of the sum's index q = 16 i + r
    const int q = Q == 32 ? l32 : (l32 >> 1);
    const int m = mw + (q >> 4) * 32 + 8 * ((q & 15) >> 2) + (q & 3);
    if (Q == 32 || (l32 & 1) == 0) it.part[(size_t)p * n + m] = v[0];
  }
}

// Wait until at most N vector-memory operations of this wave are outstanding
// (vmcnt = N; expcnt and lgkmcnt left at their maxima, i.e. not waited on).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Main loop with direct-to-LDS loads (gfx950 LDS DMA). Each wave instruction
// global_load_lds_dwordx4 copies 16 bytes per lane into 1 KB of LDS at lane
// order, i.e. 16 rows x 32 halves of one operand; a stage (K = 32) of A_hi,
// A_lo, B_hi, B_lo is 2 (BM + BN) / 16 such blocks (with third pieces A_r and B_r,
// 3 (BM + BN) / 16, in the order A pieces, B pieces), shared out over the waves.
// Stages go into a ring of NS slots and are issued NS - 1 stages ahead, with no
// staging registers. Within a block, row r (0..15) holds its four 16-byte
// k-chunks c at slot 4 r + (c ^ f(r)), f(r) = (((r >> 1) ^ (r >> 3)) & 1) |
// (((r >> 2) & 1) << 1), so that the 16 (or 8) lanes of one LDS read pass,
// which read 16 consecutive rows at one chunk, fall in distinct banks; each
// lane loads the global chunk that belongs at its slot.
//
// The LDS -> register fragment reads are software pipelined: the fragments of the next 16-wide K step (the second half of this
// stage, or the first half of the next stage after its barrier) are read while
// the MFMAs of the current step run, so a wave no longer stalls on each LDS read
// before its products. Two fragment register sets alternate. The barrier before
// a stage waits for every wave's DMA of that stage and also for
// this wave's reads of the previous stage (lgkmcnt 0), so its slot can be refilled.
// Leaves the FP32 sums in acc; ends with a barrier.
template <class Cfg>
__device__ __forceinline__ void mixed_mainloop_dl(const MixedItem& it, const int n, const int kc, const int m0,
                                                  const int n0, f16x (&acc)[Cfg::WTM][Cfg::WTN]) {
  constexpr int BM = Cfg::BM, BN = Cfg::BN, BK = 32, NS = Cfg::NS, PW = Cfg::PER_WAVE;
  constexpr int WTM = Cfg::WTM, WTN = Cfg::WTN;
  constexpr int A_BLK = Cfg::A_BLK, B_BLK = Cfg::B_BLK, SB = Cfg::STAGE_BYTES, NPC = Cfg::NPC;
  // enter_stage(s) refills the slot of stage s - 1, whose last fragment reads (its second
  // half, read before its first half's products) every wave has finished by then
  static_assert(NS >= 2, "ring depth");
  unsigned char* const ring = mixed_smem<Cfg>();

  const int tid = threadIdx.x;
  const int nk = kc / BK;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;  // wave index in an SGPR
  const int wm = wave / Cfg::WAVES_N, wn = wave % Cfg::WAVES_N;
  const int l32 = lane & 31, lh = lane >> 5;
  const int rr = lane >> 2;
  const int fr = (((rr >> 1) ^ (rr >> 3)) & 1) | (((rr >> 2) & 1) << 1);
  const int gch = (lane & 3) ^ fr;

  // per-lane LDS byte offsets of the fragment rows (chunk swizzle applied per K step)
  int aoff[WTM], boff[WTN], af[WTM], bf[WTN];
#pragma unroll
  for (int i = 0; i < WTM; ++i) {
    const int r = wm * (BM / Cfg::WAVES_M) + i * 32 + l32, rb = r & 15;
    aoff[i] = r * 64;
    af[i] = (((rb >> 1) ^ (rb >> 3)) & 1) | (((rb >> 2) & 1) << 1);
  }
#pragma unroll
  for (int j = 0; j < WTN; ++j) {
    const int r = wn * (BN / Cfg::WAVES_N) + j * 32 + l32, rb = r & 15;
    boff[j] = r * 64;
    bf[j] = (((rb >> 1) ^ (rb >> 3)) & 1) | (((rb >> 2) & 1) << 1);
  }

  f16x tot[Cfg::FLUSH > 0 ? WTM : 1][Cfg::FLUSH > 0 ? WTN : 1];
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int j = 0; j < WTN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  if constexpr (Cfg::FLUSH > 0) {
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int j = 0; j < WTN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[i][j][r] = 0.f;
  }

  // operand pointers read from the kernel arguments once (scalar loads inside the loop
  // would force lgkmcnt(0) waits and serialize the pipelined LDS reads)
  const _Float16 *const pa0[3] = {it.a0h, it.a0l, NPC == 3 ? it.a0r : nullptr};
  const _Float16 *const pb0[3] = {it.b0h, it.b0l, NPC == 3 ? it.b0r : nullptr};
  auto issue = [&](int kt) __attribute__((always_inline)) {
    const int k0 = kt * BK;
    unsigned char* slot = ring + (kt % NS) * SB;
#pragma unroll
    for (int j = 0; j < PW; ++j) {
      // block j WAVES + wave (wave-uniform): for a given j the waves' blocks lie in one or
      // two pieces, so the piece's pointer is a scalar choice rather than an indexed array
      // (interleaved against wave-contiguous blocks: 128 atoms FP16 x 3 1222 -> 1259
      // updates/s, 432 atoms 71.3 -> 74.1, one process)
      const int blk = j * Cfg::WAVES + wave;
      const _Float16* src;
      int row0;
      if (blk < NPC * A_BLK) {
        const int p = blk / A_BLK;
        src = p == 0 ? pa0[0] : (p == 1 ? pa0[1] : pa0[2]);
        row0 = m0 + (blk - p * A_BLK) * 16;
      } else {
        const int b = blk - NPC * A_BLK, p = b / B_BLK;
        src = p == 0 ? pb0[0] : (p == 1 ? pb0[1] : pb0[2]);
        row0 = n0 + (b - p * B_BLK) * 16;
      }
      const _Float16* g = src + (size_t)(row0 + rr) * n + k0 + gch * 8;
      __builtin_amdgcn_global_load_lds((const void*)g,
                                       (void __attribute__((address_space(3)))*)(slot + blk * 1024), 16, 0, 0);
    }
  };
  // stage s landed for every wave; s - 1's slot free; refill it with stage s + NS - 1
  auto enter_stage = [&](int s) __attribute__((always_inline)) {
    const int ahead = min(NS - 2, nk - 1 - s);
    if constexpr (NS >= 5) { if (ahead >= 3) wait_vmcnt<3 * PW>(); }
    if constexpr (NS >= 4) { if (ahead == 2) wait_vmcnt<2 * PW>(); }
    if (ahead == 1) wait_vmcnt<PW>();
    if (ahead <= 0) wait_vmcnt<0>();
    __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (3 << 14));  // lgkmcnt(0): this wave's reads of stage s-1 done
    __builtin_amdgcn_s_barrier();
    if (s + NS - 1 < nk) issue(s + NS - 1);
  };
  auto load = [&](h8 (&xa)[WTM][NPC], h8 (&xb)[WTN][NPC], int s, int ks) __attribute__((always_inline)) {
    const unsigned char* slot = ring + (s % NS) * SB;
    const int c = ks * 2 + lh;
#pragma unroll
    for (int i = 0; i < WTM; ++i) {
      const int off = aoff[i] + ((c ^ af[i]) << 4);
#pragma unroll
      for (int p = 0; p < NPC; ++p) xa[i][p] = *reinterpret_cast<const h8*>(slot + p * A_BLK * 1024 + off);
    }
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
      const int off = boff[j] + ((c ^ bf[j]) << 4);
#pragma unroll
      for (int p = 0; p < NPC; ++p)
        xb[j][p] = *reinterpret_cast<const h8*>(slot + (NPC * A_BLK + p * B_BLK) * 1024 + off);
    }
  };
  auto mfma = [&](const h8 (&xa)[WTM][NPC], const h8 (&xb)[WTN][NPC]) __attribute__((always_inline)) {
    constexpr bool BF = Cfg::BF16;
    // the smallest products first: third-piece products, lo lo, the cross terms, hi hi
    if constexpr (Cfg::PROD & 32) {
#pragma unroll
      for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = mfma16<BF>(xa[i][NPC - 1], xb[j][0], acc[i][j]);
    }
    if constexpr (Cfg::PROD & 16) {
#pragma unroll
      for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = mfma16<BF>(xa[i][0], xb[j][NPC - 1], acc[i][j]);
    }
    if constexpr (Cfg::PROD & 8) {
#pragma unroll
      for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = mfma16<BF>(xa[i][1], xb[j][1], acc[i][j]);
    }
    if constexpr (Cfg::PROD & 1) {
#pragma unroll
      for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = mfma16<BF>(xa[i][1], xb[j][0], acc[i][j]);
    }
    if constexpr (Cfg::PROD & 2) {
#pragma unroll
      for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = mfma16<BF>(xa[i][0], xb[j][1], acc[i][j]);
    }
    if constexpr (Cfg::PROD & 4) {
#pragma unroll
      for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = mfma16<BF>(xa[i][0], xb[j][0], acc[i][j]);
    }
  };

  h8 pa[WTM][NPC], pb[WTN][NPC], qa[WTM][NPC], qb[WTN][NPC];
#pragma unroll
  for (int s = 0; s < NS - 1; ++s)
    if (s < nk) issue(s);
  auto flush = [&]() __attribute__((always_inline)) {
    if constexpr (Cfg::FLUSH > 0) {
#pragma unroll
      for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
          tot[i][j] += acc[i][j];
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
        }
    }
  };
  enter_stage(0);
  load(pa, pb, 0, 0);
  // the last stage is peeled off so that no branch sits between a fragment read and
  // its use (a join would make the LDS wait count conservative, i.e. wait for all)
  for (int kt = 0; kt < nk - 1; ++kt) {
    load(qa, qb, kt, 1);  // second half of this stage, read during the first half's products
    mfma(pa, pb);
    enter_stage(kt + 1);
    load(pa, pb, kt + 1, 0);  // first half of the next stage, read during this stage's second half
    mfma(qa, qb);
    if ((kt + 1) % (Cfg::FLUSH > 0 ? Cfg::FLUSH : 1) == 0) flush();
  }
  load(qa, qb, nk - 1, 1);
  mfma(pa, pb);
  mfma(qa, qb);
  flush();
  __syncthreads();  // all reads of the ring done before a persistent workgroup's next tile
  if constexpr (Cfg::FLUSH > 0) {
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int j = 0; j < WTN; ++j) acc[i][j] = tot[i][j];
  }
}

// One output tile over a contraction of length kc (see f64_tile); ends with a barrier.
template <int EPI, class Cfg>
__device__ __forceinline__ void mixed_tile(const MixedItem& it, const int n, const int kc, const int2 tile) {
  static_assert(EPI == EPI_STORE || EPI == EPI_MULLIKEN, "split-precision epilogues");
  const int m0 = tile.x * Cfg::BM, n0 = tile.y * Cfg::BN;
  f16x acc[Cfg::WTM][Cfg::WTN];
  if constexpr (Cfg::DL)
    mixed_mainloop_dl<Cfg>(it, n, kc, m0, n0, acc);
  else
    mixed_mainloop_lds<Cfg>(it, n, kc, m0, n0, acc);
  mixed_epilogue<EPI, Cfg>(it, n, tile, acc);
}

template <int EPI, class Cfg>
__global__ __launch_bounds__(Cfg::THREADS, Cfg::MIN_BLOCKS) void gemm_mixed(const MixedArgs args) {
  if (args.stop != nullptr && *args.stop != 0) return;
  const int total = args.ntiles * args.nitems;
  const int logical = xcd_remap(blockIdx.x, total);
  const int z = logical / args.ntiles;
  mixed_tile<EPI, Cfg>(args.item[z], args.n, args.k, args.tiles[logical - z * args.ntiles]);
}

// Stream-K form of gemm_mixed for launches with fewer tiles than CUs, or a last round of
// workgroups far from full (MixedArgs): every workgroup takes an equal share of the launch's
// K stages, in one or a few segments of consecutive tiles, and runs each segment as the
// product over that part of the contraction (operands k-contiguous: a column offset) into
// the segment's partial slot. A workgroup holding the first segment of a Mulliken tile also
// clears the tile's slots past its last segment, so that the combine can sum every slot.
template <int EPI, class Cfg>
__global__ __launch_bounds__(Cfg::THREADS, Cfg::MIN_BLOCKS) void gemm_mixed_sk(const MixedArgs args) {
  static_assert(Cfg::DL && Cfg::BK == 32, "stream-K runs the direct-to-LDS main loop");
  static_assert(EPI == EPI_STORE || EPI == EPI_MULLIKEN, "partial slots, no accumulation");
  if (args.stop != nullptr && *args.stop != 0) return;
  const int grid = gridDim.x, nk = args.k / Cfg::BK;
  const long total = (long)args.nitems * args.ntiles * nk;
  const int w = xcd_remap(blockIdx.x, grid);
  long s = (long)w * total / grid;
  const long e = (long)(w + 1) * total / grid;
  while (s < e) {
    const int t = (int)(s / nk);
    const int k0 = (int)(s - (long)t * nk);
    const int k1 = (int)((long)nk < k0 + (e - s) ? (long)nk : k0 + (e - s));
    const int z = t / args.ntiles;
    const int2 tile = args.tiles[t - z * args.ntiles];
    const int j = w - sk_owner((long)t * nk, grid, total);
    MixedItem it = args.item[z];
    const int ko = k0 * Cfg::BK;
    it.a0h += ko; it.a0l += ko; it.b0h += ko; it.b0l += ko;
    if constexpr ((Cfg::PROD & PROD_RES) != 0) { it.a0r += ko; it.b0r += ko; }
    if constexpr (EPI == EPI_STORE)
      it.x32 += j * args.sk_stride;
    else
      it.part += j * args.sk_stride;
    mixed_tile<EPI, Cfg>(it, args.n, (k1 - k0) * Cfg::BK, tile);
    if constexpr (EPI == EPI_MULLIKEN) {
      if (j == 0) {
        const int nseg = sk_segments(t, nk, grid, total);
        double* const base = args.item[z].part;
        for (int q = nseg; q < args.sk_slots; ++q)
          for (int i = threadIdx.x; i < Cfg::BM * Cfg::WAVES_N; i += Cfg::THREADS) {
            const int m = tile.x * Cfg::BM + i % Cfg::BM, p = tile.y * Cfg::WAVES_N + i / Cfg::BM;
            base[q * args.sk_stride + (size_t)p * args.n + m] = 0.0;
          }
      }
    }
    s += k1 - k0;
  }
}

// Block sides of the second pass of the split forward transform in its full-tile form (for
// one block pair (I <= J) of an item: X = (A + A^T) / 2 / s_prod in FP64 from the FP32
// product A, Y = F o X off the diagonal and Y_ii = -w_i X_ii, split at the Y scale into
// block (I, J) and its mirror; fermi_symmetrize_chunks and fermi_symmetrize_v8 in
// kk_fused.hpp). Small handles: 32 x 32 blocks of 256 threads, 4 elements per thread (64 x 64
// blocks: 24 instead of 14 us at Nb = 1152). Large handles and split batches: 64 x 64 blocks
// of 512 threads, 8 elements per thread, whose 256-byte row reads and 128-byte row writes use
// HBM better than the 128- and 64-byte segments of 32 x 32 blocks.
constexpr int SYM_B = 32;
#ifndef KK_SYM_B_LARGE
#define KK_SYM_B_LARGE 64
#endif
constexpr int SYM_B_LARGE = KK_SYM_B_LARGE;
constexpr int SYM_T_LARGE = SYM_B_LARGE >= 64 ? 512 : 256;

using MCfg128x128 = MixedCfg<128, 128, 32, 2, 2, 2>;
using MCfg128x128f8 = MixedCfg<128, 128, 32, 2, 2, 2, 8>;
using MCfg128x128k64 = MixedCfg<128, 128, 64, 2, 2, 1>;
using MCfg256x128 = MixedCfg<256, 128, 32, 4, 2, 1>;
using MCfg256x256 = MixedCfg<256, 256, 32, 2, 4, 1>;
using MCfg256x256f8 = MixedCfg<256, 256, 32, 2, 4, 1, 8>;
using MCfg128x256 = MixedCfg<128, 256, 32, 2, 4, 1>;
using MCfg64x64f8 = MixedCfg<64, 64, 32, 2, 2, 4, 8>;  // small systems of a batch
using MCfg128x128k16f16b2 = MixedCfg<128, 128, 16, 2, 2, 2, 16>;
using MCfg128x256f8 = MixedCfg<128, 256, 32, 2, 2, 1, 8>;
using MCfg256x128w8f8 = MixedCfg<256, 128, 32, 4, 2, 1, 8>;
using MCfg128x128k64f4 = MixedCfg<128, 128, 64, 2, 2, 1, 4>;
using MCfg128x128w8f8 = MixedCfg<128, 128, 32, 4, 2, 2, 8>;
// Direct-to-LDS shapes (one workgroup per CU). At Nb = 9216: 256 x 128 with a
// 3-stage ring 254 / 295 TFLOP/s (forward / back, algorithmic), 128 x 128 with 3
// stages 245 / 267, against 253 / 289 for the register-staged default.
using MDl128x128n3 = MixedDlCfg<128, 128, 4, 2, 3, 8>;
using MDl128x128n4 = MixedDlCfg<128, 128, 4, 2, 4, 8>;
using MDl256x128n3 = MixedDlCfg<256, 128, 4, 2, 3, 8>;
using MDl256x128w16 = MixedDlCfg<256, 128, 8, 2, 3, 8>;  // 16 waves of 32 x 64

// Product configurations (each serves both products of a handle: the forward's
// A = C^T U~ G and the back-transform). Large: the direct-to-LDS 256 x 128 shape with a
// 3-stage ring, one workgroup of 16 waves (32 x 64 each) per CU. With the full-tile forward
// the 8-wave form of this shape ran 5-9 % faster than the register-staged 128 x 128 shape at
// Nb = 3888-9216 on MI355X (1024 atoms: forward step 10.7 vs 11.3 ms, back 9.5 vs 9.9 ms) and
// the 64-cluster batch 4.5 % faster, but 18 % slower at Nb = 1152, where its 256 padding and
// one workgroup per CU leave the chip under-filled; 16 waves of 32 x 64 added 4 % at 1024
// atoms and 2.5 % at 432 (16 waves of 64 x 32: 3 % and 1 %; 128 x 256: 1.5 %; flush every 4
// stages: slower).
// Small (Nb <= 2304): the direct-to-LDS main loop on 128 x 128 tiles of 8 waves (32 x 64
// each), 3-stage ring (96 KB, one workgroup per CU). With the full-tile forward it beat the
// register-staged 128 x 128 shape (K stage 32, two workgroups per CU) by 10 % at 128 atoms and
// 2 % at 16 and 250 atoms; 4- and 5-stage rings were level or 1 % slower, 16 waves of 32 x 32
// and 8 of 64 x 32 slower at 250 atoms, 4 waves of 64 x 64 7-9 % slower, and taking the large
// shape from Nb = 2048 gained nothing at 250 atoms. Counters of the register-staged shapes: no
// LDS bank conflicts, LDS busy ~27 % and MFMA busy ~40 % of cycles, while the chip clock drops
// to ~1.7 GHz during these kernels (2.4 GHz during the FP64 ones). -DKK_MLARGE_CFG=...,
// -DKK_MSMALL_CFG=... and -DKK_SPLIT_LARGE_NB=... select others for re-tuning.
#ifndef KK_MLARGE_CFG
#define KK_MLARGE_CFG MDl256x128w16
#endif
#ifndef KK_MSMALL_CFG
#define KK_MSMALL_CFG MDl128x128n3
#endif
using MLargeCfg = KK_MLARGE_CFG;
using MSmallCfg = KK_MSMALL_CFG;

// The same tile shape with other split arithmetic (the BF16 form's products).
template <class Cfg, bool BF16, int PROD>
struct WithProducts;
template <int BM, int BN, int WM, int WN, int NS, int FL, bool B0, int P0, bool BF16, int PROD>
struct WithProducts<MixedDlCfg<BM, BN, WM, WN, NS, FL, B0, P0>, BF16, PROD> {
  using type = MixedDlCfg<BM, BN, WM, WN, NS, FL, BF16, PROD>;
};
template <int BM, int BN, int BK, int WM, int WN, int MB, int FL, bool B0, int P0, bool BF16, int PROD>
struct WithProducts<MixedCfg<BM, BN, BK, WM, WN, MB, FL, B0, P0>, BF16, PROD> {
  using type = MixedCfg<BM, BN, BK, WM, WN, MB, FL, BF16, PROD>;
};
// BF16 form: the six products (PROD_ALL6) in one pass over three pieces of each operand, so
// that every piece crosses the CU's operand stream once. Small shape: 48 KB stages in a
// 3-stage ring (144 KB). Large: the 72 KB stages of 256 x 128 leave room for a 2-stage ring
// only (144 KB), and their 72 DMA blocks go to 8 waves (64 x 64 each; 16 do not divide them).
// Against the earlier two passes (hi/lo products stored, then hi res + res hi added by a
// second pass over the residual pieces) at 432 and 1024 atoms: 37.3 -> 42.8 and 2.0 -> 2.3
// updates/s (one process), results 3-6e-8 apart (the summation order).
using MSmallBf6 = WithProducts<MSmallCfg, true, PROD_ALL6>::type;
using MLargeBf6 = MixedDlCfg<256, 128, 4, 2, 2, 8, true, PROD_ALL6>;
static_assert(MLargeBf6::BM == MLargeCfg::BM && MLargeBf6::BN == MLargeCfg::BN &&
                  MLargeBf6::WAVES_N == MLargeCfg::WAVES_N,
              "the BF16 large products share the large shape's tile table and partial rows");

// Padded dimension of a split-precision handle: the larger tile side of its product
// configuration, so that the tiles cover the padded matrices exactly.
template <class Cfg>
constexpr int mixed_pad() { return Cfg::BM > Cfg::BN ? Cfg::BM : Cfg::BN; }
constexpr int MIXED_PAD_LARGE = mixed_pad<MLargeCfg>(), MIXED_PAD_SMALL = mixed_pad<MSmallCfg>();
static_assert(MIXED_PAD_LARGE % MLargeCfg::BM == 0 && MIXED_PAD_LARGE % MLargeCfg::BN == 0 &&
                  MIXED_PAD_SMALL % MSmallCfg::BM == 0 && MIXED_PAD_SMALL % MSmallCfg::BN == 0 &&
                  MIXED_PAD_LARGE % SYM_B_LARGE == 0 && MIXED_PAD_SMALL % SYM_B == 0,
              "the product tiles and the symmetrizing blocks must divide the padding");

// ---------------------------------------------------------------------------
// Split helpers

// dst_hi/lo[r][c] = split(scale * src[r][c] (or src[c][r] if transpose)), all np x np;
// NP = 3 also writes the third piece to res (BF16 form).
template <bool BF16 = false, int NP = 2>
__global__ void split_matrix(const double* __restrict__ src, int np, int transpose, const double* __restrict__ scale_p,
                             _Float16* __restrict__ hi, _Float16* __restrict__ lo, _Float16* __restrict__ res) {
  __shared__ double t[32][33];
  const double s = *scale_p;
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  auto put = [&](size_t o, double v) {
    _Float16 pc[NP];
    split_pieces<BF16, NP>(v, pc);
    hi[o] = pc[0];
    lo[o] = pc[1];
    if constexpr (NP == 3) res[o] = pc[2];
  };
  if (transpose) {
    for (int k = ty; k < 32; k += 8) t[k][tx] = src[(size_t)(bx + k) * np + by + tx];
    __syncthreads();
    for (int k = ty; k < 32; k += 8) put((size_t)(by + k) * np + bx + tx, s * t[tx][k]);
  } else {
    for (int k = ty; k < 32; k += 8) {
      const size_t o = (size_t)(by + k) * np + bx + tx;
      put(o, s * src[o]);
    }
  }
}

// Row-scaled split for the forward A operands: dst[r][c] = split(sc * u[c] * src[r][c]),
// src = C^T or G^T in FP64 (row r = eigenstate, column c = orbital).
template <bool BF16 = false, int NP = 2>
__device__ __forceinline__ void split_scaled_columns_dev(const double* __restrict__ src, int np,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ sc_p, _Float16* __restrict__ hi,
                                                         _Float16* __restrict__ lo, const int* __restrict__ stop,
                                                         int bx, int gdx, _Float16* __restrict__ re = nullptr) {
  if (stop != nullptr && *stop != 0) return;
  const double s = *sc_p;
  // 8 consecutive columns of one row per thread and step (np is a multiple of 128 and
  // at most 65536, so the group count fits 32 bits): 16-byte loads and stores only.
  const unsigned per_row = (unsigned)np / 8u, total = per_row * (unsigned)np;
  for (unsigned g = (unsigned)bx * blockDim.x + threadIdx.x; g < total; g += (unsigned)gdx * blockDim.x) {
    const unsigned r = g / per_row, c0 = (g - r * per_row) * 8u;
    const size_t base = (size_t)r * np + c0;
    const d2* sv = reinterpret_cast<const d2*>(src + base);
    const d2* uv = reinterpret_cast<const d2*>(u + c0);
    h8 vp[NP];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const d2 v = sv[q], w = uv[q];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        _Float16 pc[NP];
        split_pieces<BF16, NP>(s * w[e] * v[e], pc);
#pragma unroll
        for (int k = 0; k < NP; ++k) vp[k][2 * q + e] = pc[k];
      }
    }
    *reinterpret_cast<h8*>(hi + base) = vp[0];
    *reinterpret_cast<h8*>(lo + base) = vp[1];
    if constexpr (NP == 3) *reinterpret_cast<h8*>(re + base) = vp[2];
  }
}

// Per-row max |x| and sum x^2 of an np x np FP64 matrix (one block per row).
__global__ void row_stats(const double* __restrict__ m, int np, double* __restrict__ rmax,
                          double* __restrict__ rnorm2) {
  __shared__ double sh[17];
  __shared__ double shm[1024];
  const double* row = m + (size_t)blockIdx.x * np;
  double mx = 0.0, s2 = 0.0;
  for (int c = threadIdx.x; c < np; c += blockDim.x) {
    const double v = row[c];
    mx = fmax(mx, fabs(v));
    s2 += v * v;
  }
  s2 = block_sum(s2, sh);
  shm[threadIdx.x] = mx;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) shm[threadIdx.x] = fmax(shm[threadIdx.x], shm[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    rmax[blockIdx.x] = shm[0];
    rnorm2[blockIdx.x] = s2;
  }
}

__device__ __forceinline__ double pow2_scale(double bound, int top) {
  // largest power of two s with s * bound <= 2^top (1 if bound is 0)
  if (!(bound > 0.0)) return 1.0;
  return ldexp(1.0, top - (int)ceil(log2(bound)));
}

// Reduce row statistics of C^T and G^T (rows = columns of C and G) into the
// per-spin constants: [0] s_C, [1] s_G, [2] max column norm of C, [3] of G.
__global__ void const_scales(const double* __restrict__ cmax, const double* __restrict__ cn2,
                             const double* __restrict__ gmax, const double* __restrict__ gn2, int np,
                             double* __restrict__ out) {
  __shared__ double sm[4][1024];
  double a = 0, b = 0, c = 0, d = 0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    a = fmax(a, cmax[i]); b = fmax(b, gmax[i]); c = fmax(c, cn2[i]); d = fmax(d, gn2[i]);
  }
  sm[0][threadIdx.x] = a; sm[1][threadIdx.x] = b; sm[2][threadIdx.x] = c; sm[3][threadIdx.x] = d;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int q = 0; q < 4; ++q) sm[q][threadIdx.x] = fmax(sm[q][threadIdx.x], sm[q][threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = pow2_scale(sm[0][0], 14);
    out[1] = pow2_scale(sm[1][0], 14);
    out[2] = sqrt(sm[2][0]);
    out[3] = sqrt(sm[3][0]);
  }
}

// Gauge centring of direction b's potentials before they are split: a potential
// shift c common to both spins and all orbitals changes H1 by c S, so X by c I,
// and leaves the response exactly zero (the shared chemical potential moves by c).
// Subtracting c keeps the response and removes what would otherwise cancel only
// after the low-precision products: with c the w-weighted mean of u~ over both
// spins (w = beta f (1 - f), the weights of the chemical-potential shift), the
// large common part of gamma v_q and the part the chemical-potential shift takes
// back are both gone. Falls back to the midrange of u~ when sum w = 0.
// One block of 1024 threads per direction.
__device__ __forceinline__ void center_potentials_dev(double* __restrict__ u, int np, int nb,
                                                      const double* __restrict__ w0, const double* __restrict__ w1,
                                                      const int* __restrict__ stop, int b) {
  if (stop != nullptr && *stop != 0) return;
  __shared__ double sh[17];
  __shared__ double smin[1024], smax[1024];
  double* u0 = u + (size_t)(2 * b) * np;
  double* u1 = u0 + np;
  double lo = 1e300, hi = -1e300, su = 0.0, sw = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    lo = fmin(lo, fmin(u0[i], u1[i]));
    hi = fmax(hi, fmax(u0[i], u1[i]));
    su += w0[i] * u0[i] + w1[i] * u1[i];
    sw += w0[i] + w1[i];
  }
  su = block_sum(su, sh);
  sw = block_sum(sw, sh);
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + st]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + st]);
    }
    __syncthreads();
  }
  const double c = sw > 0.0 ? su / sw : 0.5 * (smin[0] + smax[0]);
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    u0[i] -= c;
    u1[i] -= c;
  }
}

__global__ void center_potentials(double* __restrict__ u, int np, int nb, const double* __restrict__ w0,
                                  const double* __restrict__ w1, const int* __restrict__ stop) {
  center_potentials_dev(u, np, nb, w0, w1, stop, blockIdx.x);
}

// Per response item z = 2 b + s: scales of the split operands. With
// umax = max |u~|, s_u = 2^-ceil(log2 umax); |Y| <= (beta/4) umax ncC ncG bounds
// the Hadamard product (|F| <= beta/4), giving s_Y. Writes
//   msc[z*8 + 0] = 1/(s_C s_G s_u)  forward unscale
//   msc[z*8 + 1] = s_Y              scale of the stored Y split
//   msc[z*8 + 2] = 1/(s_C s_Y)      back-transform unscale
//   msc[z*8 + 3] = s_C s_u, [4] = s_G s_u  scales of the (U~ C)^T, (U~ G)^T splits
__device__ __forceinline__ void mixed_scales_dev(const double* __restrict__ u, int np,
                                                 const double* __restrict__ mconst, double beta,
                                                 double* __restrict__ msc, const int* __restrict__ stop, int z) {
  if (stop != nullptr && *stop != 0) return;
  __shared__ double sm[1024];
  const int s = z & 1;
  const double* uz = u + (size_t)z * np;
  double mx = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) mx = fmax(mx, fabs(uz[i]));
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double umax = sm[0];
    const double sC = mconst[s * 4 + 0], sG = mconst[s * 4 + 1];
    const double su = pow2_scale(umax, 0);
    const double sY = pow2_scale(0.25 * beta * umax * mconst[s * 4 + 2] * mconst[s * 4 + 3], 14);
    msc[z * 8 + 0] = 1.0 / (sC * sG * su);
    msc[z * 8 + 1] = sY;
    msc[z * 8 + 2] = 1.0 / (sC * sY);
    msc[z * 8 + 3] = sC * su;
    msc[z * 8 + 4] = sG * su;
  }
}

__global__ void mixed_scales(const double* __restrict__ u, int np, const double* __restrict__ mconst,
                             double beta, double* __restrict__ msc, const int* __restrict__ stop) {
  mixed_scales_dev(u, np, mconst, beta, msc, stop, blockIdx.x);
}

}  // namespace kk
