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

// Wave 0 of a block: the direction in sv (2N = n2 entries, LDS) orthonormalized against
// V[0..rank) by two MGS passes, rows below `staged` read from vl (LDS), the rest from V; then
// normalized, with the breakdown test ||w|| <= BREAKDOWN_TOL ||src||. On success sv holds
// v_rank (block 0 also stores it as row `rank` of V), *cs = cvec . v (0 without cvec) and
// *accepted = 1; otherwise *accepted = 0 and block 0 ends the expansion in the Krylov state.
// Every block computes the same bits, so every block decides alike. PER >= n2 / WAVE.
template <int PER>
__device__ __forceinline__ void orth_wave0(double* sv, const double* vl, int staged, double* V, int n2, int rank,
                                           KrylovState* st, const double* __restrict__ cvec, int* accepted,
                                           double* cs) {
  const int lane = threadIdx.x & (WAVE - 1);
  double w[PER], nn = 0.0;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int i = lane + e * WAVE;
    w[e] = i < n2 ? sv[i] : 0.0;
    nn += w[e] * w[e];
  }
  const double start = sqrt(wave_sum_dpp(nn));
  for (int t = 0; t < 2 * rank; ++t) {
    const int j = t < rank ? t : t - rank;
    double r[PER], d = 0.0;
    if (j < staged) {  // the two sources in separate branches keep the LDS reads ds_read
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int i = lane + e * WAVE;
        r[e] = i < n2 ? vl[j * n2 + i] : 0.0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int i = lane + e * WAVE;
        r[e] = i < n2 ? V[(size_t)j * n2 + i] : 0.0;
      }
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) d += r[e] * w[e];
    d = wave_sum_dpp(d);
#pragma unroll
    for (int e = 0; e < PER; ++e) w[e] -= d * r[e];
  }
  nn = 0.0;
#pragma unroll
  for (int e = 0; e < PER; ++e) nn += w[e] * w[e];
  const double nrm = sqrt(wave_sum_dpp(nn));
  const bool ok = nrm > BREAKDOWN_TOL * start && rank < MAX_RANK;
  double cpart = 0.0;
  if (ok) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int i = lane + e * WAVE;
      if (i < n2) {
        const double vi = w[e] / nrm;
        sv[i] = vi;
        if (blockIdx.x == 0) V[(size_t)rank * n2 + i] = vi;
        if (cvec != nullptr) cpart += cvec[i] * vi;
      }
    }
  }
  cpart = wave_sum_dpp(cpart);
  if (lane == 0) {
    *accepted = ok ? 1 : 0;
    *cs = cpart;
    if (!ok && blockIdx.x == 0) {
      st->stop = 1;
      if (rank > 0) st->status = 1;
    }
  }
}

// One Krylov step's prologue: v_rank = MGS^2(src)/||.|| (two passes against V[0..rank);
// or the end of the expansion on breakdown), then u^s_I = sum_J gamma_IJ v_q[J] + s W v_m[I]
// on every orbital of the block's atoms (Sec. III.A). With cvec given (split forms) the
// potentials are centred by c = cvec . v (the response to a common shift is zero) and
// pmax[2 blockIdx.x + s] receives the block's largest |u^s - c|.
// The block first issues all its global loads (the stop flag, src, the centring vector and
// the first rows of V, up to FUSED_LDS_ROWS doubles, for LDS; its atoms' rows of gamma and
// orbital ranges into registers) and tests the flag afterwards. Wave 0 then
// runs the 2 rank projections out of LDS (rows past the staged ones from global memory),
// and every wave forms its atoms' potentials from the new direction in LDS.
// Grid: ceil(N / FUSED_ATOMS) blocks of FUSED_THREADS; 2N <= FUSED_MAX_N2.
constexpr int FUSED_LDS_ROWS = 8192;  // doubles of V staged in LDS (64 KB)
__global__ void __launch_bounds__(FUSED_THREADS)
    orth_potentials(const double* __restrict__ src, double* __restrict__ V, int n2, KrylovState* st, int rank,
                    const double* __restrict__ gamma, int natoms, double W, const int* __restrict__ offsets, int np,
                    double* __restrict__ u, const double* __restrict__ cvec, double* __restrict__ pmax) {
  __shared__ double sv[FUSED_MAX_N2];
  __shared__ double vl[FUSED_LDS_ROWS];
  __shared__ double mred[2][FUSED_THREADS / WAVE];
  __shared__ double cvl[FUSED_MAX_N2];
  __shared__ double cshared;
  __shared__ int accepted;
  // the stop flag is read with the other loads and tested once they are issued (all of
  // them are in bounds either way), so that it costs no round trip of its own
  const int stopped = st->stop;
  constexpr int NW = FUSED_THREADS / WAVE, APW = FUSED_ATOMS / NW, GPER = FUSED_MAX_N2 / 2 / WAVE;
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const int a0 = blockIdx.x * FUSED_ATOMS, a1 = min(natoms, a0 + FUSED_ATOMS);
  const int staged = min(rank, FUSED_LDS_ROWS / n2);
  // every global load of the block first, into registers (a load and its LDS store per
  // loop step would wait for each load in turn)
  constexpr int SPT = FUSED_MAX_N2 / FUSED_THREADS, VPT = FUSED_LDS_ROWS / FUSED_THREADS;
  const int nv = staged * n2;
  double sr[SPT], vr[VPT], cr[SPT];
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    const int i = threadIdx.x + k * FUSED_THREADS;
    sr[k] = i < n2 ? src[i] : 0.0;
    cr[k] = (cvec != nullptr && i < n2) ? cvec[i] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < VPT; ++k) {
    const int i = threadIdx.x + k * FUSED_THREADS;
    vr[k] = i < nv ? V[i] : 0.0;
  }
  double g[APW][GPER];
  int ob[APW], oe[APW];
#pragma unroll
  for (int t = 0; t < APW; ++t) {
    const int a = a0 + wave + t * NW;
#pragma unroll
    for (int e = 0; e < GPER; ++e) {
      const int j = lane + e * WAVE;
      g[t][e] = (a < a1 && j < natoms) ? gamma[(size_t)a * natoms + j] : 0.0;
    }
    ob[t] = a < a1 ? offsets[a] : 0;
    oe[t] = a < a1 ? offsets[a + 1] : 0;
  }
  if (stopped) return;  // the same value in every thread: before the first barrier
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    const int i = threadIdx.x + k * FUSED_THREADS;
    if (i < n2) {
      sv[i] = sr[k];
      cvl[i] = cr[k];
    }
  }
#pragma unroll
  for (int k = 0; k < VPT; ++k) {
    const int i = threadIdx.x + k * FUSED_THREADS;
    if (i < nv) vl[i] = vr[k];
  }
  __syncthreads();
  if (wave == 0) orth_wave0<FUSED_MAX_N2 / WAVE>(sv, vl, staged, V, n2, rank, st, cvl, &accepted, &cshared);
  __syncthreads();
  if (!accepted) return;
  const double c = cvec != nullptr ? cshared : 0.0;
  double m0 = 0.0, m1 = 0.0;
#pragma unroll
  for (int t = 0; t < APW; ++t) {
    const int a = a0 + wave + t * NW;  // wave-uniform
    if (a >= a1) break;
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < GPER; ++e) {
      const int j = lane + e * WAVE;
      if (j < natoms) s += g[t][e] * sv[j];
    }
    s = wave_sum_dpp(s);
    const double up = s + W * sv[natoms + a] - c, dn = s - W * sv[natoms + a] - c;
    m0 = fmax(m0, fabs(up));
    m1 = fmax(m1, fabs(dn));
    for (int i = ob[t] + lane; i < oe[t]; i += WAVE) {
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

// (U~ C)^T at scale s in NP 16-bit pieces for one group of 8 consecutive columns of row r
// (16-byte loads and stores): the arithmetic of split_scaled_columns_dev.
template <bool BF16, int NP>
__device__ __forceinline__ void split_group8(const d2 (&v)[4], const d2 (&w)[4], double s, size_t base,
                                             _Float16* __restrict__ hi, _Float16* __restrict__ lo,
                                             _Float16* __restrict__ re) {
  h8 vp[NP];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      _Float16 pc[NP];
      split_pieces<BF16, NP>(s * w[q][e] * v[q][e], pc);
#pragma unroll
      for (int k = 0; k < NP; ++k) vp[k][2 * q + e] = pc[k];
    }
  *reinterpret_cast<h8*>(hi + base) = vp[0];
  *reinterpret_cast<h8*>(lo + base) = vp[1];
  if constexpr (NP == 3) *reinterpret_cast<h8*>(re + base) = vp[2];
}

// The split forms' operand split after orth_potentials: the item scales from the blocks'
// largest centred potentials (as mixed_scales computes them from the potentials; block
// x = 0 of each item stores them for the products and the symmetrizing pass), then
// (U~ C)^T split at s_C s_u, grid-stride over 8-column groups. Every thread forms the
// scales itself (a few cached loads), and its first group's operand and potentials are
// loaded together with them, so that the block waits for memory once before it computes.
// Grid (blocks, 2 items).
template <bool BF16, int NP>
__global__ void split_operands_fused(const double* __restrict__ CT0, const double* __restrict__ CT1, int np,
                                     const double* __restrict__ u, const double* __restrict__ pmax, int nblk,
                                     const double* __restrict__ mconst, double beta, double* __restrict__ msc,
                                     _Float16* __restrict__ uct_h, _Float16* __restrict__ uct_l,
                                     _Float16* __restrict__ uct_r, const int* __restrict__ stop) {
  const int z = blockIdx.y;
  const double* src = z ? CT1 : CT0;
  const double* uz = u + (size_t)z * np;
  const size_t off = (size_t)z * np * np;
  const unsigned per_row = (unsigned)np / 8u, total = per_row * (unsigned)np;
  const unsigned g0 = (unsigned)blockIdx.x * blockDim.x + threadIdx.x, gs = (unsigned)gridDim.x * blockDim.x;
  d2 v[4], w[4];
  size_t base = 0;
  if (g0 < total) {
    const unsigned r = g0 / per_row, c0 = (g0 - r * per_row) * 8u;
    base = (size_t)r * np + c0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = reinterpret_cast<const d2*>(src + base)[q];
      w[q] = reinterpret_cast<const d2*>(uz + c0)[q];
    }
  }
  const int stopped = stop != nullptr ? *stop : 0;
  double umax = 0.0;
  for (int b = 0; b < nblk; ++b) umax = fmax(umax, pmax[2 * b + z]);
  const double sC = mconst[z * 4 + 0], sG = mconst[z * 4 + 1];
  if (stopped) return;
  const double s_u = pow2_scale(umax, 0);
  const double scale = sC * s_u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double sY = pow2_scale(0.25 * beta * umax * mconst[z * 4 + 2] * mconst[z * 4 + 3], 14);
    msc[z * 8 + 0] = 1.0 / (sC * sG * s_u);
    msc[z * 8 + 1] = sY;
    msc[z * 8 + 2] = 1.0 / (sC * sY);
    msc[z * 8 + 3] = sC * s_u;
    msc[z * 8 + 4] = sG * s_u;
  }
  _Float16* re = NP == 3 ? uct_r + off : nullptr;
  if (g0 < total) split_group8<BF16, NP>(v, w, scale, base, uct_h + off, uct_l + off, re);
  for (unsigned g = g0 + gs; g < total; g += gs) {
    const unsigned r = g / per_row, c0 = (g - r * per_row) * 8u;
    const size_t bg = (size_t)r * np + c0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = reinterpret_cast<const d2*>(src + bg)[q];
      w[q] = reinterpret_cast<const d2*>(uz + c0)[q];
    }
    split_group8<BF16, NP>(v, w, scale, bg, uct_h + off, uct_l + off, re);
  }
}

// The combine of the fused small-system step: the same results as combine (dmu from
// w . diag X of both spins, per-atom sums of the Mulliken partial rows, dmu t_s, the (q, m)
// mix and, with ft, the preconditioned derivative -(q1 - vsub)), with every load of a block
// issued before the first is used: the partial rows of an atom are read as flattened
// (row, orbital) pairs, COMBINE_BATCH per lane and spin at once. One wave per atom,
// COMBINE_THREADS threads; grid (ceil(N / COMBINE_ATOMS), directions).
constexpr int COMBINE_BATCH = 8;
__global__ void __launch_bounds__(COMBINE_THREADS)
    combine_small(const double* __restrict__ xdiag, const double* __restrict__ part, int nparts,
                  const double* __restrict__ w_up, const double* __restrict__ w_dn,
                  const double* __restrict__ wsum_p, const double* __restrict__ t, int nb, int np,
                  const int* __restrict__ offsets, int natoms, double* __restrict__ q1,
                  const int* __restrict__ stop, const double* __restrict__ vsub, double* __restrict__ ft) {
  __shared__ double sh[17];
  const int b = blockIdx.y;
  const int lane = threadIdx.x & (WAVE - 1);
  const int a = blockIdx.x * (COMBINE_THREADS / WAVE) + (int)(threadIdx.x / WAVE);
  const bool have = a < natoms;
  // first round of loads: the stop flag, the atom's orbital range, its t_s, and the w . diag X
  // terms of dmu; the partial rows (which need the range) follow in a second
  const int stopped = stop != nullptr ? *stop : 0;
  const int i0 = have ? offsets[a] : 0, i1 = have ? offsets[a + 1] : 0;
  const double tu = have ? t[a] : 0.0, td = have ? t[natoms + a] : 0.0;
  const double wsum = *wsum_p;
  const double* xu = xdiag + ((size_t)b * 2 + 0) * np;
  const double* xd = xdiag + ((size_t)b * 2 + 1) * np;
  double s = 0.0;
  for (int base = 0; base < nb; base += 4 * COMBINE_THREADS) {
    double wu[4], xuv[4], wd[4], xdv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = base + threadIdx.x + k * COMBINE_THREADS;
      const bool ok = i < nb;
      wu[k] = ok ? w_up[i] : 0.0;
      xuv[k] = ok ? xu[i] : 0.0;
      wd[k] = ok ? w_dn[i] : 0.0;
      xdv[k] = ok ? xd[i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) s += wu[k] * xuv[k] + wd[k] * xdv[k];
  }
  if (stopped) return;  // the same value in every thread: before the first barrier
  const int norb = i1 - i0, tot = nparts * norb;
  const double* p0 = part + ((size_t)b * 2 + 0) * nparts * np + i0;
  const double* p1 = part + ((size_t)b * 2 + 1) * nparts * np + i0;
  double acc0 = 0.0, acc1 = 0.0;
  for (int base = 0; base < tot; base += COMBINE_BATCH * WAVE) {
    double v0[COMBINE_BATCH], v1[COMBINE_BATCH];
#pragma unroll
    for (int k = 0; k < COMBINE_BATCH; ++k) {
      const int e = base + lane + k * WAVE;
      const bool ok = e < tot;
      const int p = ok ? e / norb : 0;
      const size_t o = (size_t)p * np + (e - p * norb);
      v0[k] = ok ? p0[o] : 0.0;
      v1[k] = ok ? p1[o] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < COMBINE_BATCH; ++k) {
      acc0 += v0[k];
      acc1 += v1[k];
    }
  }
  s = block_sum(s, sh);
  acc0 = wave_sum(acc0);
  acc1 = wave_sum(acc1);
  if (!have || lane != 0) return;
  const double dmu = wsum > 0.0 ? s / wsum : 0.0;
  const double d0 = acc0 + dmu * tu, d1 = acc1 + dmu * td;
  const double qa = d0 + d1, ma = d0 - d1;
  q1[(size_t)b * 2 * natoms + a] = qa;
  q1[(size_t)b * 2 * natoms + natoms + a] = ma;
  if (ft != nullptr) {  // the preconditioned directional derivative with K0 = -I: -(q1 - v)
    ft[a] = -(qa - vsub[a]);
    ft[natoms + a] = -(ma - vsub[natoms + a]);
  }
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
// through LDS after the whole pair was read). B x B blocks of T = B * B / 4 threads: thread
// (r, q) takes columns 4q..4q+3 of row r of both blocks (16-byte loads and stores).
template <int B, int T, int NCH>
__global__ __launch_bounds__(T) void fermi_symmetrize_f64_chunks(const GemmArgs args, size_t cstride) {
  static_assert(T * 4 == B * B, "4 elements per thread");
  const int stopped = args.stop != nullptr ? *args.stop : 0;  // tested once the loads are issued
  const GemmItem& it = args.item[blockIdx.y];
  const int n = args.n;
  const int2 ij = upper_pair(blockIdx.x, n / B);
  const int I = ij.x, J = ij.y;
  __shared__ double At[B][B + 1];
  const int r = threadIdx.x / (B / 4), c4 = (threadIdx.x % (B / 4)) * 4;
  double* const Y = it.out;
  const int m = I * B + r, cb = J * B + c4;
  const size_t oo = (size_t)m * n + cb, om = (size_t)(J * B + r) * n + I * B + c4;
  d2 own[NCH][2], mir[NCH][2];
#pragma unroll
  for (int j = 0; j < NCH; ++j)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      own[j][h] = reinterpret_cast<const d2*>(Y + oo + j * cstride)[h];
      mir[j][h] = reinterpret_cast<const d2*>(Y + om + j * cstride)[h];
    }
  const double em = it.eps[m], fm = it.f[m], fcm = it.fc[m], wm = it.w[m];
  d2 en[2], fn[2], fcn[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    en[h] = reinterpret_cast<const d2*>(it.eps + cb)[h];
    fn[h] = reinterpret_cast<const d2*>(it.f + cb)[h];
    fcn[h] = reinterpret_cast<const d2*>(it.fc + cb)[h];
  }
  if (stopped) return;  // the same value in every thread: before the first barrier
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    double a = mir[0][e >> 1][e & 1];
#pragma unroll
    for (int j = 1; j < NCH; ++j) a += mir[j][e >> 1][e & 1];
    At[r][c4 + e] = a;
  }
  __syncthreads();
  double yv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = c4 + e;
    double a = own[0][e >> 1][e & 1];
#pragma unroll
    for (int j = 1; j < NCH; ++j) a += own[j][e >> 1][e & 1];
    const double x = 0.5 * (a + At[c][r]);
    double y;
    if (m == cb + e) {
      it.xdiag[m] = x;
      y = -wm * x;
    } else {
      y = fermi_divided_difference(em, fm, fcm, en[e >> 1][e & 1], fn[e >> 1][e & 1], fcn[e >> 1][e & 1],
                                   args.beta) * x;
    }
    yv[e] = y;
  }
  // only this thread read these elements of block (I, J), all chunks of them
  reinterpret_cast<d2*>(Y + oo)[0] = d2{yv[0], yv[1]};
  reinterpret_cast<d2*>(Y + oo)[1] = d2{yv[2], yv[3]};
  if (I == J) return;  // a diagonal block is symmetric by construction
  __syncthreads();     // every read of At is done
#pragma unroll
  for (int e = 0; e < 4; ++e) At[c4 + e][r] = yv[e];
  __syncthreads();
  reinterpret_cast<d2*>(Y + om)[0] = d2{At[r][c4], At[r][c4 + 1]};
  reinterpret_cast<d2*>(Y + om)[1] = d2{At[r][c4 + 2], At[r][c4 + 3]};
}

// Split forms: the FP32 partial products at it.x32 + j cstride, X scaled by 1 / the
// product scale, Y written as NP 16-bit pieces at the Y scale (as fermi_symmetrize does).
// Same thread layout, 16-byte loads and 8-byte stores. After a stream-K product
// (args.sk_grid > 0) each of the two blocks sums only the slots its product tile filled
// (NCH = the most segments of any tile).
typedef float f4v __attribute__((ext_vector_type(4)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
template <int B, int T, bool BF16, int NP, int NCH>
__global__ __launch_bounds__(T) void fermi_symmetrize_chunks(const MixedArgs args, size_t cstride) {
  static_assert(T * 4 == B * B, "4 elements per thread");
  static_assert(NP == 2 || NP == 3, "two or three pieces");
  const int stopped = args.stop != nullptr ? *args.stop : 0;  // tested once the loads are issued
  const MixedItem& it = args.item[blockIdx.y];
  const int n = args.n;
  const int2 ij = upper_pair(blockIdx.x, n / B);
  const int I = ij.x, J = ij.y;
  __shared__ double At[B][B + 1];
  __shared__ _Float16 Tp[NP][B][B + 4];
  const int r = threadIdx.x / (B / 4), c4 = (threadIdx.x % (B / 4)) * 4;
  const int m = I * B + r, cb = J * B + c4;
  const size_t oo = (size_t)m * n + cb, om = (size_t)(J * B + r) * n + I * B + c4;
  int nown = NCH, nmir = NCH;
  if (args.sk_grid > 0) {
    const int nk = args.k / 32, nt = n / args.sk_side, ti = I * B / args.sk_side, tj = J * B / args.sk_side;
    const long total = (long)args.nitems * args.ntiles * nk;
    const int t0 = blockIdx.y * args.ntiles;
    nown = sk_segments(t0 + tile_table_pos(ti, tj, nt, nt), nk, args.sk_grid, total);
    nmir = sk_segments(t0 + tile_table_pos(tj, ti, nt, nt), nk, args.sk_grid, total);
  }
  f4v own[NCH], mir[NCH];
#pragma unroll
  for (int j = 0; j < NCH; ++j) {
    own[j] = j < nown ? *reinterpret_cast<const f4v*>(it.x32 + oo + j * cstride) : f4v{0.f, 0.f, 0.f, 0.f};
    mir[j] = j < nmir ? *reinterpret_cast<const f4v*>(it.x32 + om + j * cstride) : f4v{0.f, 0.f, 0.f, 0.f};
  }
  const double em = it.eps[m], fm = it.f[m], fcm = it.fc[m], wm = it.w[m];
  d2 en[2], fn[2], fcn[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    en[h] = reinterpret_cast<const d2*>(it.eps + cb)[h];
    fn[h] = reinterpret_cast<const d2*>(it.f + cb)[h];
    fcn[h] = reinterpret_cast<const d2*>(it.fc + cb)[h];
  }
  const double inv = it.sc[0], sy = it.sc[1];
  if (stopped) return;  // the same value in every thread: before the first barrier
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    double a = (double)mir[0][e];
#pragma unroll
    for (int j = 1; j < NCH; ++j) a += (double)mir[j][e];
    At[r][c4 + e] = a;
  }
  __syncthreads();
  h4v pv[NP];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = c4 + e;
    double a = (double)own[0][e];
#pragma unroll
    for (int j = 1; j < NCH; ++j) a += (double)own[j][e];
    const double x = 0.5 * inv * (a + At[c][r]);
    double y;
    if (m == cb + e) {
      it.xdiag[m] = x;
      y = -wm * x * sy;
    } else {
      y = fermi_divided_difference(em, fm, fcm, en[e >> 1][e & 1], fn[e >> 1][e & 1], fcn[e >> 1][e & 1],
                                   args.beta) * x * sy;
    }
    _Float16 pc[NP];
    split_pieces<BF16, NP>(y, pc);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pv[p][e] = pc[p];
      Tp[p][c][r] = pc[p];
    }
  }
  *reinterpret_cast<h4v*>(it.yh + oo) = pv[0];
  *reinterpret_cast<h4v*>(it.yl + oo) = pv[1];
  if constexpr (NP == 3) *reinterpret_cast<h4v*>(it.yr + oo) = pv[2];
  if (I == J) return;
  __syncthreads();
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    h4v t;
#pragma unroll
    for (int e = 0; e < 4; ++e) t[e] = Tp[p][r][c4 + e];
    _Float16* dst = p == 0 ? it.yh : (p == 1 ? it.yl : it.yr);
    *reinterpret_cast<h4v*>(dst + om) = t;
  }
}

// Symmetrizing pass of the split forms for one 64 x 64 block pair (I <= J) of an item (the
// arithmetic of fermi_symmetrize_chunks, element by element), with eight
// consecutive elements per thread: thread (r, q) of 512 takes columns 8q..8q+7 of row r of
// both blocks (32-byte loads of A, 16-byte stores of each Y piece), and every global load of
// the block is issued before the first is used. Used by large split handles and by the split
// batches (b_symmetrize).
template <bool BF16, int NP>
__device__ __forceinline__ void fermi_symmetrize_v8_dev(const MixedItem& it, const int n, const double beta,
                                                        const int pair) {
  static_assert(NP == 2 || NP == 3, "two or three pieces");
  constexpr int B = 64;
  const int2 ij = upper_pair(pair, n / B);
  const int I = ij.x, J = ij.y;
  __shared__ double At[B][B + 1];
  __shared__ _Float16 Tp[NP][B][B + 8];
  const int r = threadIdx.x >> 3, c8 = (threadIdx.x & 7) * 8;
  const int m = I * B + r, cb = J * B + c8;
  const size_t oo = (size_t)m * n + cb, om = (size_t)(J * B + r) * n + I * B + c8;
  const f4v own0 = *reinterpret_cast<const f4v*>(it.x32 + oo);
  const f4v own1 = *reinterpret_cast<const f4v*>(it.x32 + oo + 4);
  const f4v mir0 = *reinterpret_cast<const f4v*>(it.x32 + om);
  const f4v mir1 = *reinterpret_cast<const f4v*>(it.x32 + om + 4);
  const double em = it.eps[m], fm = it.f[m], fcm = it.fc[m], wm = it.w[m];
  d2 en[4], fn[4], fcn[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    en[h] = reinterpret_cast<const d2*>(it.eps + cb)[h];
    fn[h] = reinterpret_cast<const d2*>(it.f + cb)[h];
    fcn[h] = reinterpret_cast<const d2*>(it.fc + cb)[h];
  }
  const double inv = it.sc[0], sy = it.sc[1];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    At[r][c8 + e] = (double)mir0[e];
    At[r][c8 + 4 + e] = (double)mir1[e];
  }
  __syncthreads();
  h8 pv[NP];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int c = c8 + e;
    const double a = (double)(e < 4 ? own0[e & 3] : own1[e & 3]);
    const double x = 0.5 * inv * (a + At[c][r]);
    double y;
    if (m == cb + e) {
      it.xdiag[m] = x;
      y = -wm * x * sy;
    } else {
      y = fermi_divided_difference(em, fm, fcm, en[e >> 1][e & 1], fn[e >> 1][e & 1], fcn[e >> 1][e & 1], beta) *
          x * sy;
    }
    _Float16 pc[NP];
    split_pieces<BF16, NP>(y, pc);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pv[p][e] = pc[p];
      Tp[p][c][r] = pc[p];
    }
  }
  *reinterpret_cast<h8*>(it.yh + oo) = pv[0];
  *reinterpret_cast<h8*>(it.yl + oo) = pv[1];
  if constexpr (NP == 3) *reinterpret_cast<h8*>(it.yr + oo) = pv[2];
  if (I == J) return;  // a diagonal block is symmetric by construction (the same in every thread)
  __syncthreads();
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    h8 t;
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = Tp[p][r][c8 + e];
    *reinterpret_cast<h8*>((p == 0 ? it.yh : p == 1 ? it.yl : it.yr) + om) = t;
  }
}

// Single split handles on the large tiles: blockIdx.x = block pair, blockIdx.y = item.
template <bool BF16, int NP>
__global__ __launch_bounds__(512) void fermi_symmetrize_v8(const MixedArgs args) {
  if (args.stop != nullptr && *args.stop != 0) return;
  fermi_symmetrize_v8_dev<BF16, NP>(args.item[blockIdx.y], args.n, args.beta, blockIdx.x);
}

}  // namespace kk
