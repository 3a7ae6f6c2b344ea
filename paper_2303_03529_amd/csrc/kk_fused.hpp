// Fused Krylov-step kernels for small systems. Below a few hundred atoms a
// response is a handful of short launches around the two transforms; here one
// launch orthonormalizes the new direction and builds its spin potentials (for
// the split forms also their gauge centring and each block's largest centred
// potential), and the split forms' operand split reduces those maxima into the
// item scales itself, so that the chain before the forward transform is one
// launch (FP64) or two (split forms) instead of two or five.
//
// Every block repeats the orthonormalization (2 rank dot products over 2N
// numbers, cached reads) so that no grid-wide synchronization is needed; block 0
// alone writes the new direction and the Krylov state. The rank is the loop index
// passed by the host: while the expansion runs (stop == 0) it equals the number
// of accepted directions.
#pragma once

#include <hip/hip_runtime.h>

#include "kk_kernels.hpp"
#include "kk_gemm_mixed.hpp"

namespace kk {

constexpr int FUSED_MAX_N2 = 1024;   // 2N up to this uses the fused step (N <= 512)
constexpr int FUSED_THREADS = 256;
constexpr int FUSED_PER = FUSED_MAX_N2 / FUSED_THREADS;
constexpr int FUSED_ATOMS = 16;      // atoms per block
constexpr int FUSED_MAX_BLOCKS = (FUSED_MAX_N2 / 2 + FUSED_ATOMS - 1) / FUSED_ATOMS;

// Centring vector of a split handle: the w-weighted mean over both spins of the
// potentials u^s = gamma v_q + s W v_m is c(v) = cvec . v with
//   cvec[J]     = sum_I (W^up_I + W^dn_I) gamma_IJ / sum w,
//   cvec[N + I] = W (W^up_I - W^dn_I) / sum w,
// W^s_I = sum_{i in I} w^s_i (gamma symmetric). Zero when sum w = 0 (no centring).
// One block of 256 threads per J in [0, N), block N does the moment part.
__global__ void centre_vector(const double* __restrict__ gamma, int natoms, double W, const int* __restrict__ offsets,
                              const double* __restrict__ w0, const double* __restrict__ w1,
                              const double* __restrict__ wsum_p, double* __restrict__ cvec) {
  __shared__ double sh[17];
  const double wsum = *wsum_p;
  const int J = blockIdx.x;
  double s = 0.0;
  for (int I = threadIdx.x; I < natoms; I += blockDim.x) {
    double wu = 0.0, wd = 0.0;
    for (int i = offsets[I]; i < offsets[I + 1]; ++i) {
      wu += w0[i];
      wd += w1[i];
    }
    if (J < natoms)
      s += (wu + wd) * gamma[(size_t)I * natoms + J];
    else
      cvec[natoms + I] = wsum > 0.0 ? W * (wu - wd) / wsum : 0.0;
  }
  if (J < natoms) {
    s = block_sum(s, sh);
    if (threadIdx.x == 0) cvec[J] = wsum > 0.0 ? s / wsum : 0.0;
  }
}

// One Krylov step's prologue: v_rank = MGS^2(src)/||.|| (two passes against V[0..rank);
// or the end of the expansion on breakdown), then u^s_I = sum_J gamma_IJ v_q[J] + s W v_m[I]
// on every orbital of the block's atoms (Sec. III.A). With cvec given (split forms) the
// potentials are centred by c = cvec . v (the response to a common shift is zero) and
// pmax[2 blockIdx.x + s] receives the block's largest |u^s - c|.
// Grid: ceil(N / FUSED_ATOMS) blocks of FUSED_THREADS; 2N <= FUSED_MAX_N2.
__global__ void __launch_bounds__(FUSED_THREADS)
    orth_potentials(const double* __restrict__ src, double* __restrict__ V, int n2, KrylovState* st, int rank,
                    const double* __restrict__ gamma, int natoms, double W, const int* __restrict__ offsets, int np,
                    double* __restrict__ u, const double* __restrict__ cvec, double* __restrict__ pmax) {
  __shared__ double sv[FUSED_MAX_N2];
  __shared__ double mred[2][FUSED_THREADS / WAVE];
  __shared__ double cshared;
  __shared__ int accepted;
  if (st->stop) return;
  if (threadIdx.x < WAVE) {
    // Orthonormalization in wave 0 (shuffle reductions, no barriers); the next row of V is
    // loaded before each projection's reduction.
    constexpr int PER = FUSED_MAX_N2 / WAVE;
    const int lane0 = threadIdx.x;
    double w[PER], nn = 0.0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int i = lane0 + e * WAVE;
      w[e] = i < n2 ? src[i] : 0.0;
      nn += w[e] * w[e];
    }
    const double start = sqrt(wave_sum(nn));
    auto load_row = [&](int j, double (&dst)[PER]) {
      const double* vj = V + (size_t)j * n2;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int i = lane0 + e * WAVE;
        dst[e] = i < n2 ? vj[i] : 0.0;
      }
    };
    const int steps = 2 * rank;
    double cur[PER], nxt[PER] = {};
    if (steps > 0) load_row(0, cur);
    for (int t = 0; t < steps; ++t) {
      if (t + 1 < steps) load_row((t + 1) % rank, nxt);
      double d = 0.0;
#pragma unroll
      for (int e = 0; e < PER; ++e) d += cur[e] * w[e];
      d = wave_sum(d);
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        w[e] -= d * cur[e];
        cur[e] = nxt[e];
      }
    }
    nn = 0.0;
#pragma unroll
    for (int e = 0; e < PER; ++e) nn += w[e] * w[e];
    const double nrm = sqrt(wave_sum(nn));
    const bool ok = nrm > BREAKDOWN_TOL * start && rank < MAX_RANK;  // every block decides alike
    double cpart = 0.0;
    if (ok) {
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int i = lane0 + e * WAVE;
        if (i < n2) {
          const double vi = w[e] / nrm;
          sv[i] = vi;
          if (blockIdx.x == 0) V[(size_t)rank * n2 + i] = vi;
          if (cvec != nullptr) cpart += cvec[i] * vi;
        }
      }
    }
    cpart = wave_sum(cpart);
    if (lane0 == 0) {
      accepted = ok ? 1 : 0;
      cshared = cpart;
      if (!ok && blockIdx.x == 0) {
        st->stop = 1;
        if (rank > 0) st->status = 1;
      }
    }
  }
  __syncthreads();
  if (!accepted) return;
  const double c = cvec != nullptr ? cshared : 0.0;
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  constexpr int NW = FUSED_THREADS / WAVE;
  const int a0 = blockIdx.x * FUSED_ATOMS, a1 = min(natoms, a0 + FUSED_ATOMS);
  double m0 = 0.0, m1 = 0.0;
  for (int a = a0 + wave; a < a1; a += NW) {
    const double* g = gamma + (size_t)a * natoms;
    double s = 0.0;
    for (int j = lane; j < natoms; j += WAVE) s += g[j] * sv[j];
    s = wave_sum(s);
    const double up = s + W * sv[natoms + a] - c, dn = s - W * sv[natoms + a] - c;
    m0 = fmax(m0, fabs(up));
    m1 = fmax(m1, fabs(dn));
    for (int i = offsets[a] + lane; i < offsets[a + 1]; i += WAVE) {
      u[i] = up;
      u[(size_t)np + i] = dn;
    }
  }
  if (pmax != nullptr) {
    if (lane == 0) {
      mred[0][wave] = m0;
      mred[1][wave] = m1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      double mx = 0.0;
      for (int q = 0; q < NW; ++q) mx = fmax(mx, mred[threadIdx.x][q]);
      pmax[2 * blockIdx.x + threadIdx.x] = mx;
    }
  }
  if (blockIdx.x == 0) {
    __syncthreads();
    if (threadIdx.x == 0) st->rank = rank + 1;
  }
}

// The split forms' operand split after orth_potentials: the item scales from the blocks'
// largest centred potentials (as mixed_scales computes them from the potentials; block
// x = 0 of each item stores them for the products and the symmetrizing pass), then
// (U~ C)^T split at s_C s_u. Grid (blocks, 2 items).
template <bool BF16, int NP>
__global__ void split_operands_fused(const double* __restrict__ CT0, const double* __restrict__ CT1, int np,
                                     const double* __restrict__ u, const double* __restrict__ pmax, int nblk,
                                     const double* __restrict__ mconst, double beta, double* __restrict__ msc,
                                     _Float16* __restrict__ uct_h, _Float16* __restrict__ uct_l,
                                     _Float16* __restrict__ uct_r, const int* __restrict__ stop) {
  __shared__ double scale;
  if (stop != nullptr && *stop != 0) return;
  const int z = blockIdx.y;
  if (threadIdx.x == 0) {
    double umax = 0.0;
    for (int b = 0; b < nblk; ++b) umax = fmax(umax, pmax[2 * b + z]);
    const double sC = mconst[z * 4 + 0], sG = mconst[z * 4 + 1];
    const double s_u = pow2_scale(umax, 0);
    const double sY = pow2_scale(0.25 * beta * umax * mconst[z * 4 + 2] * mconst[z * 4 + 3], 14);
    scale = sC * s_u;
    if (blockIdx.x == 0) {
      msc[z * 8 + 0] = 1.0 / (sC * sG * s_u);
      msc[z * 8 + 1] = sY;
      msc[z * 8 + 2] = 1.0 / (sC * sY);
      msc[z * 8 + 3] = sC * s_u;
      msc[z * 8 + 4] = sG * s_u;
    }
  }
  __syncthreads();
  const size_t off = (size_t)z * np * np;
  split_scaled_columns_dev<BF16, NP>(z ? CT1 : CT0, np, u + (size_t)z * np, &scale, uct_h + off, uct_l + off,
                                     nullptr, blockIdx.x, gridDim.x, NP == 3 ? uct_r + off : nullptr);
}

// ---------------------------------------------------------------------------
// Symmetrizing passes of the small-system forward transforms, also for K-split
// products. With few tiles per launch the product of each item can be split along
// its contraction into NCH chunks, each a separate GEMM item writing its own partial
// product; these passes sum the partials (in chunk order, so results stay bitwise
// reproducible) while they form X = (A + A^T) / 2 and Y = F o X. NCH = 1 is the
// unsplit product. Every global load of a pass (the partials of the thread's
// elements of block (I, J) and of block (J, I), the spectrum of its rows and column)
// is issued before the first is used, so that a block waits for memory once.

// Block pair (I <= J) from the upper-triangle index, row-major.
__device__ __forceinline__ int2 upper_pair(int pair, int nblk) {
  int I = 0, rem = pair;
  while (rem >= nblk - I) {
    rem -= nblk - I;
    ++I;
  }
  return make_int2(I, I + rem);
}

// FP64: A_j at it.out + j cstride; X_ii goes to xdiag, Y_ii = -w_i X_ii, Y = F o X
// elsewhere, written over A_0 (block (I, J) by the thread that read it, block (J, I)
// through LDS after the whole pair was read). B x B blocks, T threads.
template <int B, int T, int NCH>
__global__ __launch_bounds__(T) void fermi_symmetrize_f64_chunks(const GemmArgs args, size_t cstride) {
  static_assert(T % B == 0 && B % (T / B) == 0, "thread mapping");
  if (args.stop != nullptr && *args.stop != 0) return;
  const GemmItem& it = args.item[blockIdx.y];
  const int n = args.n;
  const int2 ij = upper_pair(blockIdx.x, n / B);
  const int I = ij.x, J = ij.y;
  constexpr int RS = T / B, Q = B / RS;
  __shared__ double At[B][B + 1];
  const int tx = threadIdx.x % B, ty = threadIdx.x / B;
  double* const Y = it.out;
  const int c = J * B + tx;
  double own[NCH][Q], mir[NCH][Q], em[Q], fm[Q], fcm[Q], wm[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = ty + q * RS;
    const size_t oo = (size_t)(I * B + r) * n + c, om = (size_t)(J * B + r) * n + I * B + tx;
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      own[j][q] = Y[oo + j * cstride];
      mir[j][q] = Y[om + j * cstride];
    }
    const int m = I * B + r;
    em[q] = it.eps[m]; fm[q] = it.f[m]; fcm[q] = it.fc[m]; wm[q] = it.w[m];
  }
  const double en = it.eps[c], fn = it.f[c], fcn = it.fc[c];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double a = mir[0][q];
#pragma unroll
    for (int j = 1; j < NCH; ++j) a += mir[j][q];
    At[ty + q * RS][tx] = a;
  }
  __syncthreads();
  double yv[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = ty + q * RS, m = I * B + r;
    double a = own[0][q];
#pragma unroll
    for (int j = 1; j < NCH; ++j) a += own[j][q];
    const double x = 0.5 * (a + At[tx][r]);
    double y;
    if (m == c) {
      it.xdiag[m] = x;
      y = -wm[q] * x;
    } else {
      y = fermi_divided_difference(em[q], fm[q], fcm[q], en, fn, fcn, args.beta) * x;
    }
    yv[q] = y;
    Y[(size_t)m * n + c] = y;  // only this thread read this element, and it read all chunks of it
  }
  if (I == J) return;  // a diagonal block is symmetric by construction
  __syncthreads();     // every read of At is done
#pragma unroll
  for (int q = 0; q < Q; ++q) At[tx][ty + q * RS] = yv[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = ty + q * RS;
    Y[(size_t)(J * B + r) * n + I * B + tx] = At[r][tx];
  }
}

// Split forms: the FP32 partial products at it.x32 + j cstride, X scaled by 1 / the
// product scale, Y written as NP 16-bit pieces at the Y scale (as fermi_symmetrize does).
template <int B, int T, bool BF16, int NP, int NCH>
__global__ __launch_bounds__(T) void fermi_symmetrize_chunks(const MixedArgs args, size_t cstride) {
  static_assert(T % B == 0 && B % (T / B) == 0, "thread mapping");
  static_assert(NP == 2 || NP == 3, "two or three pieces");
  if (args.stop != nullptr && *args.stop != 0) return;
  const MixedItem& it = args.item[blockIdx.y];
  const int n = args.n;
  const int2 ij = upper_pair(blockIdx.x, n / B);
  const int I = ij.x, J = ij.y;
  constexpr int RS = T / B, Q = B / RS;
  __shared__ double At[B][B + 1];
  __shared__ _Float16 Tp[NP][B][B + 2];
  const int tx = threadIdx.x % B, ty = threadIdx.x / B;
  const int c = J * B + tx;
  float own[NCH][Q], mir[NCH][Q];
  double em[Q], fm[Q], fcm[Q], wm[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = ty + q * RS;
    const size_t oo = (size_t)(I * B + r) * n + c, om = (size_t)(J * B + r) * n + I * B + tx;
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      own[j][q] = it.x32[oo + j * cstride];
      mir[j][q] = it.x32[om + j * cstride];
    }
    const int m = I * B + r;
    em[q] = it.eps[m]; fm[q] = it.f[m]; fcm[q] = it.fc[m]; wm[q] = it.w[m];
  }
  const double en = it.eps[c], fn = it.f[c], fcn = it.fc[c];
  const double inv = it.sc[0], sy = it.sc[1];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double a = (double)mir[0][q];
#pragma unroll
    for (int j = 1; j < NCH; ++j) a += (double)mir[j][q];
    At[ty + q * RS][tx] = a;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = ty + q * RS, m = I * B + r;
    const size_t o = (size_t)m * n + c;
    double a = (double)own[0][q];
#pragma unroll
    for (int j = 1; j < NCH; ++j) a += (double)own[j][q];
    const double x = 0.5 * inv * (a + At[tx][r]);
    double y;
    if (m == c) {
      it.xdiag[m] = x;
      y = -wm[q] * x * sy;
    } else {
      y = fermi_divided_difference(em[q], fm[q], fcm[q], en, fn, fcn, args.beta) * x * sy;
    }
    _Float16 pc[NP];
    split_pieces<BF16, NP>(y, pc);
    it.yh[o] = pc[0];
    it.yl[o] = pc[1];
    if constexpr (NP == 3) it.yr[o] = pc[2];
#pragma unroll
    for (int p = 0; p < NP; ++p) Tp[p][tx][r] = pc[p];
  }
  if (I == J) return;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = ty + q * RS;
    const size_t o = (size_t)(J * B + r) * n + I * B + tx;
    it.yh[o] = Tp[0][r][tx];
    it.yl[o] = Tp[1][r][tx];
    if constexpr (NP == 3) it.yr[o] = Tp[2][r][tx];
  }
}

}  // namespace kk
