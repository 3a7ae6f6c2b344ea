// FP64 MFMA tile GEMM for gfx950 with three fused epilogues.
//
// Every dense contraction of the response runs through one kernel shape:
//   acc[m][n] = sum_k A[k][m] * B[k][n]
// with both operands stored k-major (row k contiguous along m or n), padded to
// a multiple of 128 so no access needs a bounds check. In that layout the
// forward eigenbasis transform X = C^T U~ G (+ its transpose) and the
// back-transform P = C Y (with C^T stored) read both panels along rows, which
// is the coalesced direction.
//
// Tile: BM x BN per workgroup of WAVES_M x WAVES_N waves; each wave owns a
// (BM/WAVES_M) x (BN/WAVES_N) block of v_mfma_f64_16x16x4 accumulators. K
// advances BK per stage through double-buffered LDS with the next stage's
// global loads in flight while the current stage is multiplied.
//
// Epilogues
//   EPI_STORE   out[m][n] = acc                                (setup products)
//   EPI_FERMI   Sec. II.C first-order Fermi response in the eigenbasis:
//               X = 1/2 acc (acc accumulates C^T U~ G + G^T U~ C over a K of
//               2 Nb), Y_mn = F_mn X_mn for m < n written to (m,n) and (n,m),
//               Y_mm = -w_m X_mm and X_mm saved for the chemical-potential
//               shift. Tiles entirely below the diagonal are not launched;
//               elements below it are skipped.
//   EPI_MULLIKEN  Sec. III.A Mulliken rows: part[p][m] = sum over the wave's
//               columns n of acc[m][n] * G[m][n]; the caller sums the parts.
//   EPI_FERMI_XY  EPI_FERMI that also writes X itself (both triangles) to xout,
//               for the reverse pass, which needs X and Y of each direction.
//   EPI_ACCUM   out[m][n] += acc                                (adjoint sums)
//   EPI_XSTORE  out[m][n] = acc with the row scale applied like EPI_FERMI: the
//               product A = C^T U~ G over full tiles (one K half), which
//               fermi_symmetrize_f64 turns into Y in place
#pragma once

#include <hip/hip_runtime.h>

namespace kk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int PAD = 128;    // every padded dimension is a multiple of this
constexpr int MAX_GEMM_BATCH = 16;

enum { EPI_STORE = 0, EPI_FERMI = 1, EPI_MULLIKEN = 2, EPI_FERMI_XY = 3, EPI_ACCUM = 4, EPI_XSTORE = 5 };

struct GemmItem {
  const double* a0;   // first K half: A operand, [K][n] row-major
  const double* b0;   // first K half: B operand
  const double* a1;   // second K half (EPI_FERMI) or unused
  const double* b1;
  const double* scale;  // per-k scale of A rows (EPI_FERMI: u~ per orbital), length n
  double* out;          // EPI_STORE: product; EPI_FERMI: Y
  const double* g;      // EPI_MULLIKEN: G, [n][n]
  const double* eps;    // EPI_FERMI: eigenvalues (padded with 0)
  const double* f;      // occupations f
  const double* fc;     // 1 - f
  const double* w;      // beta f (1 - f)
  double* xdiag;        // EPI_FERMI: diag X
  double* part;         // EPI_MULLIKEN: [parts][n]
  double* xout;         // EPI_FERMI_XY: X
};

struct GemmArgs {
  int n;          // padded dimension; M = N = n, row stride n
  int k_half;     // rows per K half (= n)
  int two_halves; // 1: K runs over both halves (a0,b0) then (a1,b1)
  int ntiles;     // tiles per item
  int nitems;     // batch items
  const int2* tiles;  // tile coordinates (tm, tn), in launch order
  const int* stop;    // if non-null and *stop != 0 the launch does nothing
  double beta;        // 1 / kT (EPI_FERMI)
  GemmItem item[MAX_GEMM_BATCH];
};

// Hardware hands workgroup ids to the 8 XCDs round-robin; give each XCD a
// contiguous range of logical tiles so neighbouring tiles share its L2.
__device__ __forceinline__ int xcd_remap(int bid, int total) {
  const int x = bid & 7, slot = bid >> 3;
  const int q = total >> 3, r = total & 7;
  return (x < r) ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

// (f_lo - f_hi)/(e_lo - e_hi) for the pair, lo = lower eigenvalue, written as
// -beta f_lo (1 - f_hi) phi(beta (e_lo - e_hi)), phi(z) = expm1(z)/z, phi(0) = 1.
__device__ __forceinline__ double fermi_divided_difference(double em, double fm, double fcm,
                                                           double en, double fn, double fcn,
                                                           double beta) {
  double flo, fchi, z;
  if (em <= en) {
    flo = fm; fchi = fcn; z = beta * (em - en);
  } else {
    flo = fn; fchi = fcm; z = beta * (en - em);
  }
  const double phi = (z == 0.0) ? 1.0 : expm1(z) / z;
  return -beta * flo * fchi * phi;
}

template <int BM_, int BN_, int BK_, int WAVES_M_, int WAVES_N_, int MINB_>
struct TileCfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_;
  static constexpr int WAVES_M = WAVES_M_, WAVES_N = WAVES_N_;
  static constexpr int THREADS = 64 * WAVES_M * WAVES_N;
  static constexpr int WTM = BM / WAVES_M / 16;  // MFMA tiles per wave along m
  static constexpr int WTN = BN / WAVES_N / 16;  // along n
  static constexpr int MIN_BLOCKS = MINB_;
  // MIN_BLOCKS co-resident workgroups need this many waves per SIMD, which caps
  // the registers per lane the compiler may use (512 / WAVES_PER_EU).
  static constexpr int WAVES_PER_EU = (MIN_BLOCKS * THREADS / 64 + 3) / 4;
  // global -> LDS staging: each thread moves double2 pieces
  static constexpr int A_PIECES = BK * BM / 2 / THREADS;
  static constexpr int B_PIECES = BK * BN / 2 / THREADS;
  static_assert(BM % (16 * WAVES_M) == 0 && BN % (16 * WAVES_N) == 0, "wave tiling");
  static_assert(BK % 4 == 0, "BK");
  static_assert(A_PIECES >= 1 && B_PIECES >= 1, "staging");
  static_assert((BK * BM / 2) % THREADS == 0 && (BK * BN / 2) % THREADS == 0, "staging split");
  static_assert(PAD % BM == 0 && PAD % BN == 0, "tile must divide the padding");
  static constexpr int LDS_BYTES = 2 * BK * (BM + BN) * 8;
};

// One output tile: both operands n x n (row stride n), K = k_half or 2 k_half.
// Ends with a barrier, so a workgroup may run several tiles in sequence.
template <int EPI, class Cfg>
__device__ __forceinline__ void f64_tile(const GemmItem& it, const int n, const int k_half, const bool two_halves,
                                         const int2 tile, const double beta_arg) {
  constexpr int BM = Cfg::BM, BN = Cfg::BN, BK = Cfg::BK;
  constexpr int WTM = Cfg::WTM, WTN = Cfg::WTN;
  constexpr int AP = Cfg::A_PIECES, BP = Cfg::B_PIECES;
  constexpr int APR = BM / 2;  // double2 pieces per A row
  constexpr int BPR = BN / 2;
  const int m0 = tile.x * BM, n0 = tile.y * BN;

  __shared__ double As[2][BK][BM];
  __shared__ double Bs[2][BK][BN];

  const int tid = threadIdx.x;
  const int nk = (two_halves ? 2 * k_half : k_half) / BK;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave / Cfg::WAVES_N, wn = wave % Cfg::WAVES_N;
  const int lr = lane >> 4, lc = lane & 15;

  d4 acc[WTM][WTN];
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int j = 0; j < WTN; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};

  // Global -> register -> LDS staging, one stage ahead: the loads of stage kt + 1 are
  // issued at the start of step kt and written to LDS at its end, and nothing in
  // between waits for them; the loads are unconditional (the last step reloads the last
  // stage, written to the idle buffer and never read), because a conditional load makes
  // the compiler wait for every load in flight before the write.
  // The forward transform's row scales go through a 3-slot LDS ring: the BK scales of
  // stage s are loaded by the first BK threads at the start of step s - 2, put in slot
  // s % 3 at its end, and multiplied in when stage s is written to LDS (end of step s - 1).
  constexpr bool SCALED = EPI == EPI_FERMI || EPI == EPI_FERMI_XY || EPI == EPI_XSTORE;
  __shared__ double Ss[SCALED ? 3 : 1][BK];
  d2 ra[AP], rb[BP];
  double sreg = 0.0;
  // Byte offsets of this thread's staging pieces within a K stage (loop invariant; BK
  // rows of n <= 65536 doubles span at most 8 MB, so 32 bits hold them); the stage's
  // uniform part goes into the base pointers.
  unsigned aoff[AP], boff[BP];
#pragma unroll
  for (int p = 0; p < AP; ++p) {
    const int idx = tid + p * Cfg::THREADS;
    const int row = idx / APR, col = (idx % APR) * 2;
    aoff[p] = (unsigned)(row * n + col) * 8u;
  }
#pragma unroll
  for (int p = 0; p < BP; ++p) {
    const int idx = tid + p * Cfg::THREADS;
    const int row = idx / BPR, col = (idx % BPR) * 2;
    boff[p] = (unsigned)(row * n + col) * 8u;
  }
  auto gload = [&](const int kt) __attribute__((always_inline)) {
    int k0 = kt * BK;
    const double* A = it.a0;
    const double* B = it.b0;
    if (two_halves && k0 >= k_half) {
      A = it.a1; B = it.b1; k0 -= k_half;
    }
    const char* Ab = reinterpret_cast<const char*>(A + (size_t)k0 * n + m0);
    const char* Bb = reinterpret_cast<const char*>(B + (size_t)k0 * n + n0);
#pragma unroll
    for (int p = 0; p < AP; ++p) ra[p] = *reinterpret_cast<const d2*>(Ab + aoff[p]);
#pragma unroll
    for (int p = 0; p < BP; ++p) rb[p] = *reinterpret_cast<const d2*>(Bb + boff[p]);
  };
  auto sload = [&](const int kt) __attribute__((always_inline)) {
    if constexpr (SCALED) {
      int k0 = kt * BK;
      if (two_halves && k0 >= k_half) k0 -= k_half;
      if (tid < BK) sreg = it.scale[k0 + tid];
    }
  };
  auto sstore = [&](const int kt) __attribute__((always_inline)) {
    if constexpr (SCALED) {
      if (tid < BK) Ss[kt % 3][tid] = sreg;
    }
  };
  auto lstore = [&](const int buf, const int kt) __attribute__((always_inline)) {
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int idx = tid + p * Cfg::THREADS;
      d2 v = ra[p];
      if constexpr (SCALED) v *= Ss[kt % 3][idx / APR];
      *reinterpret_cast<d2*>(&As[buf][idx / APR][(idx % APR) * 2]) = v;
    }
#pragma unroll
    for (int p = 0; p < BP; ++p) {
      const int idx = tid + p * Cfg::THREADS;
      *reinterpret_cast<d2*>(&Bs[buf][idx / BPR][(idx % BPR) * 2]) = rb[p];
    }
  };

  gload(0);
  sload(0);
  sstore(0);
  sload(min(1, nk - 1));
  sstore(1);
  __syncthreads();
  lstore(0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    gload(min(kt + 1, nk - 1));
    sload(min(kt + 2, nk - 1));
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      double a[WTM], b[WTN];
#pragma unroll
      for (int i = 0; i < WTM; ++i) a[i] = As[buf][kk * 4 + lr][wm * (BM / Cfg::WAVES_M) + i * 16 + lc];
#pragma unroll
      for (int j = 0; j < WTN; ++j) b[j] = Bs[buf][kk * 4 + lr][wn * (BN / Cfg::WAVES_N) + j * 16 + lc];
#pragma unroll
      for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    lstore(buf ^ 1, kt + 1);
    sstore(kt + 2);
    __syncthreads();
  }

  // Accumulator element (i, j, r) of this lane sits at
  //   m = m0 + wm*(BM/WAVES_M) + i*16 + lr + 4r,  n = n0 + wn*(BN/WAVES_N) + j*16 + lc.
  const int mw = m0 + wm * (BM / Cfg::WAVES_M) + lr;
  const int nw = n0 + wn * (BN / Cfg::WAVES_N) + lc;
  if constexpr (EPI == EPI_STORE || EPI == EPI_ACCUM || EPI == EPI_XSTORE) {
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int j = 0; j < WTN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double* o = it.out + (size_t)(mw + i * 16 + 4 * r) * n + nw + j * 16;
          if constexpr (EPI == EPI_ACCUM) *o += acc[i][j][r];
          else *o = acc[i][j][r];
        }
  } else if constexpr (EPI == EPI_FERMI || EPI == EPI_FERMI_XY) {
    const double beta = beta_arg;
    // Column spectra are re-read per row (cached) rather than held, which keeps the
    // epilogue inside the main loop's register budget.
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mw + i * 16 + 4 * r;
        const double em = it.eps[m], fm = it.f[m], fcm = it.fc[m];
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
          const int c = nw + j * 16;
          if (m > c) continue;
          const double en = it.eps[c], fn = it.f[c], fcn = it.fc[c];
          const double x = 0.5 * acc[i][j][r];
          if constexpr (EPI == EPI_FERMI_XY) {
            it.xout[(size_t)m * n + c] = x;
            it.xout[(size_t)c * n + m] = x;
          }
          if (m == c) {
            it.xdiag[m] = x;
            it.out[(size_t)m * n + m] = -it.w[m] * x;
          } else {
            const double y = fermi_divided_difference(em, fm, fcm, en, fn, fcn, beta) * x;
            it.out[(size_t)m * n + c] = y;
            it.out[(size_t)c * n + m] = y;
          }
        }
      }
  } else {  // EPI_MULLIKEN
    const int p = tile.y * Cfg::WAVES_N + wn;
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mw + i * 16 + 4 * r;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < WTN; ++j) s += acc[i][j][r] * it.g[(size_t)m * n + nw + j * 16];
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        s += __shfl_xor(s, 8);
        if (lc == 0) it.part[(size_t)p * n + m] = s;
      }
  }
}

template <int EPI, class Cfg>
__global__ __launch_bounds__(Cfg::THREADS, Cfg::MIN_BLOCKS) void gemm_f64(const GemmArgs args) {
  if (args.stop != nullptr && *args.stop != 0) return;
  const int total = args.ntiles * args.nitems;
  const int logical = xcd_remap(blockIdx.x, total);
  const int z = logical / args.ntiles;
  f64_tile<EPI, Cfg>(args.item[z], args.n, args.k_half, args.two_halves != 0,
                     args.tiles[logical - z * args.ntiles], args.beta);
}

// Second pass of the FP64 forward transform when it runs as a full-tile product
// (EPI_XSTORE): out holds A = C^T U~ G; for each B x B block pair (I <= J),
// X = (A + A^T) / 2, Y = F o X off the diagonal and Y_ii = -w_i X_ii (X_ii to
// xdiag), written in place over A: block (I, J) element by element by the
// thread that read it, block (J, I) through LDS after the whole of it was read.
// pair indexes the upper triangle row-major; T threads. Small handles: 32 x 32 blocks of
// 256 threads; large handles and FP64 batches: 64 x 64 blocks of 512 threads (512-byte rows).
constexpr int SYM64_B = 32;
constexpr int SYM64_B_LARGE = 64, SYM64_T_LARGE = 512;
static_assert(PAD % SYM64_B_LARGE == 0, "the symmetrizing blocks must divide the padding");
template <int B = SYM64_B, int T = 256>
__device__ __forceinline__ void fermi_symmetrize_f64_dev(const GemmItem& it, const int n, const double beta,
                                                         const int pair) {
  static_assert(T % B == 0 && B % (T / B) == 0, "thread mapping");
  const int nblk = n / B;
  int I = 0, rem = pair;
  while (rem >= nblk - I) {
    rem -= nblk - I;
    ++I;
  }
  const int J = I + rem;
  __shared__ double At[B][B + 1];  // block (J, I) of A, then the mirror of Y
  const int tx = threadIdx.x % B, ty = threadIdx.x / B;
  constexpr int RS = T / B;
  double* const Y = it.out;
  for (int r = ty; r < B; r += RS) At[r][tx] = Y[(size_t)(J * B + r) * n + I * B + tx];
  __syncthreads();
  const int c = J * B + tx;
  const double en = it.eps[c], fn = it.f[c], fcn = it.fc[c];
  double yv[B / RS];
#pragma unroll
  for (int q = 0; q < B / RS; ++q) {
    const int r = ty + q * RS, m = I * B + r;
    double* const o = Y + (size_t)m * n + c;
    const double x = 0.5 * (*o + At[tx][r]);
    double y;
    if (m == c) {
      it.xdiag[m] = x;
      y = -it.w[m] * x;
    } else {
      y = fermi_divided_difference(it.eps[m], it.f[m], it.fc[m], en, fn, fcn, beta) * x;
    }
    *o = y;
    yv[q] = y;
  }
  if (I == J) return;  // a diagonal block is symmetric by construction
  __syncthreads();     // every read of At is done
#pragma unroll
  for (int q = 0; q < B / RS; ++q) At[tx][ty + q * RS] = yv[q];
  __syncthreads();
  for (int r = ty; r < B; r += RS) Y[(size_t)(J * B + r) * n + I * B + tx] = At[r][tx];
}

// Single system: blockIdx.x = block pair, blockIdx.y = item.
template <int B, int T>
__global__ __launch_bounds__(T) void fermi_symmetrize_f64(const GemmArgs args) {
  if (args.stop != nullptr && *args.stop != 0) return;
  fermi_symmetrize_f64_dev<B, T>(args.item[blockIdx.y], args.n, args.beta, blockIdx.x);
}

// Configurations. The default (128 x 128 tile, 8 waves of 32 x 64, two
// workgroups and 16 waves per CU) was the fastest of the shapes below for
// both transforms at Nb = 9216 and 3888 on MI355X; the others stay available
// for re-tuning (-DKK_FWD_CFG=..., -DKK_BACK_CFG=...).
using Cfg128x128 = TileCfg<128, 128, 16, 2, 2, 2>;
using Cfg128x64 = TileCfg<128, 64, 16, 2, 2, 2>;
using Cfg64x128 = TileCfg<64, 128, 16, 2, 2, 2>;
using Cfg128x128w8 = TileCfg<128, 128, 16, 4, 2, 2>;
using Cfg128x128k32 = TileCfg<128, 128, 32, 2, 2, 1>;
using Cfg128x128k8 = TileCfg<128, 128, 8, 2, 2, 2>;
using Cfg64x64 = TileCfg<64, 64, 16, 2, 2, 3>;

using Cfg128x128w16 = TileCfg<128, 128, 16, 4, 4, 1>;
using Cfg128x128w8n = TileCfg<128, 128, 16, 2, 4, 2>;

#ifndef KK_FWD_CFG
#define KK_FWD_CFG Cfg128x128w8
#endif
#ifndef KK_BACK_CFG
#define KK_BACK_CFG Cfg128x128w8
#endif
#ifndef KK_STORE_CFG
#define KK_STORE_CFG Cfg128x128w8
#endif
using FwdCfg = KK_FWD_CFG;
using BackCfg = KK_BACK_CFG;
using StoreCfg = KK_STORE_CFG;

}  // namespace kk
