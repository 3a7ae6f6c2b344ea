// FP64 MFMA tile GEMM for gfx950 with three fused epilogues.
//
// Every dense contraction of the response runs through one kernel shape:
//   acc[m][n] = sum_k A[k][m] * B[k][n]
// with both operands stored k-major (row k contiguous along m or n), padded to
// a multiple of the 128 x 128 tile so no access needs a bounds check. In that
// layout the forward eigenbasis transform X = C^T U~ G (+ its transpose) and
// the back-transform P = C Y (with C^T stored) read both panels along rows,
// which is the coalesced direction.
//
// Tile: 128 x 128 per 256-thread workgroup, 4 waves in 2 x 2, each wave a
// 64 x 64 block made of 4 x 4 v_mfma_f64_16x16x4 accumulators (64 doubles per
// lane). K advances 16 per stage through double-buffered LDS (64 KiB), with the
// next stage's global loads in flight while the current stage is multiplied.
//
// Epilogues
//   EPI_STORE   out[m][n] = acc                                (setup products)
//   EPI_FERMI   Sec. II.C first-order Fermi response in the eigenbasis:
//               X = 1/2 acc (acc accumulates C^T U~ G + G^T U~ C over a K of
//               2 Nb), Y_mn = F_mn X_mn for m != n written to (m,n) and (n,m),
//               Y_mm = -w_m X_mm and X_mm saved for the chemical-potential
//               shift. Only upper-triangle tiles are launched.
//   EPI_MULLIKEN  Sec. III.A Mulliken rows: part[p][m] = sum_{n in tile half}
//               acc[m][n] * G[m][n]; the caller sums the parts per atom.
#pragma once

#include <hip/hip_runtime.h>

namespace kk {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TILE = 128;   // M and N tile
constexpr int BK = 16;      // K per LDS stage
constexpr int NTHREADS = 256;
constexpr int MAX_GEMM_BATCH = 16;

enum { EPI_STORE = 0, EPI_FERMI = 1, EPI_MULLIKEN = 2 };

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
  double* part;         // EPI_MULLIKEN: [2 * n / TILE][n]
};

struct GemmArgs {
  int n;          // padded dimension (multiple of TILE); M = N = n, row stride n
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

template <int EPI>
__global__ __launch_bounds__(NTHREADS, 2) void gemm_f64(const GemmArgs args) {
  if (args.stop != nullptr && *args.stop != 0) return;
  const int total = args.ntiles * args.nitems;
  const int logical = xcd_remap(blockIdx.x, total);
  const int z = logical / args.ntiles;
  const int2 tile = args.tiles[logical - z * args.ntiles];
  const GemmItem& it = args.item[z];
  const int n = args.n;
  const int m0 = tile.x * TILE, n0 = tile.y * TILE;

  __shared__ double As[2][BK][TILE];
  __shared__ double Bs[2][BK][TILE];

  const int tid = threadIdx.x;
  const int lrow = tid >> 6;         // 0..3, plus 4 * j
  const int lcol = (tid & 63) * 2;   // two doubles per thread per row
  const int nk = (args.two_halves ? 2 * args.k_half : args.k_half) / BK;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane >> 4, lc = lane & 15;

  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};

  double2 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
#define KK_GLOAD(kt)                                                                   \
  {                                                                                    \
    int k0 = (kt) * BK;                                                                \
    const double* A = it.a0;                                                           \
    const double* B = it.b0;                                                           \
    if (args.two_halves && k0 >= args.k_half) {                                        \
      A = it.a1; B = it.b1; k0 -= args.k_half;                                         \
    }                                                                                  \
    const double* pa = A + (size_t)(k0 + lrow) * n + m0 + lcol;                        \
    const double* pb = B + (size_t)(k0 + lrow) * n + n0 + lcol;                        \
    const size_t st4 = (size_t)4 * n;                                                  \
    ra0 = *reinterpret_cast<const double2*>(pa);                                       \
    ra1 = *reinterpret_cast<const double2*>(pa + st4);                                 \
    ra2 = *reinterpret_cast<const double2*>(pa + 2 * st4);                             \
    ra3 = *reinterpret_cast<const double2*>(pa + 3 * st4);                             \
    rb0 = *reinterpret_cast<const double2*>(pb);                                       \
    rb1 = *reinterpret_cast<const double2*>(pb + st4);                                 \
    rb2 = *reinterpret_cast<const double2*>(pb + 2 * st4);                             \
    rb3 = *reinterpret_cast<const double2*>(pb + 3 * st4);                             \
    if constexpr (EPI == EPI_FERMI) {                                                  \
      const double* sc = it.scale + k0 + lrow;                                         \
      const double s0 = sc[0], s1 = sc[4], s2 = sc[8], s3 = sc[12];                    \
      ra0.x *= s0; ra0.y *= s0; ra1.x *= s1; ra1.y *= s1;                              \
      ra2.x *= s2; ra2.y *= s2; ra3.x *= s3; ra3.y *= s3;                              \
    }                                                                                  \
  }
#define KK_LSTORE(buf)                                                                 \
  {                                                                                    \
    *reinterpret_cast<double2*>(&As[buf][lrow][lcol]) = ra0;                           \
    *reinterpret_cast<double2*>(&As[buf][lrow + 4][lcol]) = ra1;                       \
    *reinterpret_cast<double2*>(&As[buf][lrow + 8][lcol]) = ra2;                       \
    *reinterpret_cast<double2*>(&As[buf][lrow + 12][lcol]) = ra3;                      \
    *reinterpret_cast<double2*>(&Bs[buf][lrow][lcol]) = rb0;                           \
    *reinterpret_cast<double2*>(&Bs[buf][lrow + 4][lcol]) = rb1;                       \
    *reinterpret_cast<double2*>(&Bs[buf][lrow + 8][lcol]) = rb2;                       \
    *reinterpret_cast<double2*>(&Bs[buf][lrow + 12][lcol]) = rb3;                      \
  }

  KK_GLOAD(0);
  KK_LSTORE(0);
  __syncthreads();

  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) KK_GLOAD(kt + 1);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[buf][kk * 4 + lr][wm * 64 + i * 16 + lc];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[buf][kk * 4 + lr][wn * 64 + j * 16 + lc];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) KK_LSTORE(buf ^ 1);
    __syncthreads();
  }
#undef KK_GLOAD
#undef KK_LSTORE

  // Accumulator element (i, j, r) of this lane sits at
  //   m = m0 + wm*64 + i*16 + lr + 4r,  n = n0 + wn*64 + j*16 + lc.
  if constexpr (EPI == EPI_STORE) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * 64 + i * 16 + lr + 4 * r;
          const int c = n0 + wn * 64 + j * 16 + lc;
          it.out[(size_t)m * n + c] = acc[i][j][r];
        }
  } else if constexpr (EPI == EPI_FERMI) {
    const bool diag_tile = tile.x == tile.y;
    const double beta = args.beta;
    double en[4], fn[4], fcn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = n0 + wn * 64 + j * 16 + lc;
      en[j] = it.eps[c]; fn[j] = it.f[c]; fcn[j] = it.fc[c];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + i * 16 + lr + 4 * r;
        const double em = it.eps[m], fm = it.f[m], fcm = it.fc[m];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = n0 + wn * 64 + j * 16 + lc;
          if (diag_tile && m > c) continue;
          const double x = 0.5 * acc[i][j][r];
          if (m == c) {
            it.xdiag[m] = x;
            it.out[(size_t)m * n + m] = -it.w[m] * x;
          } else {
            const double y = fermi_divided_difference(em, fm, fcm, en[j], fn[j], fcn[j], beta) * x;
            it.out[(size_t)m * n + c] = y;
            it.out[(size_t)c * n + m] = y;
          }
        }
      }
  } else {  // EPI_MULLIKEN
    const int p = tile.y * 2 + wn;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + i * 16 + lr + 4 * r;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = n0 + wn * 64 + j * 16 + lc;
          s += acc[i][j][r] * it.g[(size_t)m * n + c];
        }
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        s += __shfl_xor(s, 8);
        if (lc == 0) it.part[(size_t)p * n + m] = s;
      }
  }
}

}  // namespace kk
