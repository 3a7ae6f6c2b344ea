// Reverse pass of the rank-m Krylov kernel: gradients of a scalar L(K delta)
// with respect to delta, gamma, W and the expansion-point spin Hamiltonians.
//
// Krylov part (Sec. II.G). The forward builds v_1 = f~/|f~|, f~_k = A v_k with
// A = K0 (R - I) (R the response, q1 = R v), v_{k+1} = the normalized part of
// f~_k orthogonal to v_1..v_k, and x = V c with c solving (F~^T F~) c = F~^T f~.
// Its reverse, given x_bar:
//   c_bar = V^T x_bar, V_bar = x_bar c^T, z = O^-1 c_bar, f~_bar = F~ z,
//   F~_bar = r z^T - F~ z c^T with r = f~ - F~ c (least-squares adjoint);
//   then for k = rank..1: the adjoint of the orthonormalization that made
//   v_{k+1} from f~_k (w_bar = (I - v v^T) v_bar_{k+1} / rho_k,
//   F~_bar_k += (I - V_k V_k^T) w_bar, V_bar_j -= w_bar h_j + f~_k p_j),
//   lambda_k = F~_bar_k, y_k = K0^T lambda_k and v_bar_k += A^T lambda_k
//   = R^T y_k - y_k.
// The response is self-adjoint in the metric Gamma = diag(gamma, W I):
// R = M chi M Gamma with chi the symmetric potential-space response and
// M = [[I, I], [I, -I]], so R^T y = Gamma g with g = M chi M y, the response
// to the potentials (y_q + y_m, y_q - y_m) with identity coupling.
// Parameter gradients: gamma_bar += g_q v_q^T, W_bar += g_m . v_m, and
// dL/dH^sigma from the change of chi with the expansion point.
//
// Expansion-point part (Sec. II.C). With a = M y_k and b = M Gamma v_k,
// s_k = a^T chi b = sum_sigma sum_ij F_ij Xa_ij Xb_ij + Wsum dmu_a dmu_b,
// Xa = C^T H1[a] C. Under a symmetric change E of H^sigma (E' = C^T E C in the
// eigenbasis) the levels move by E'_ii, the eigenvectors rotate by
// E'_ij / (eps_j - eps_i) and mu follows the electron count. Summed over k:
//   E'_bar_ij = ((K - K^T)_ij + (w_i - w_j) D_ij) / (eps_i - eps_j),  i != j,
//     K = sum_k Y0_b Xa + Y0_a Xb (Y0 = F o X),  D = sum_k dmu_b Xa + dmu_a Xb,
//   E'_bar_ii = g_i - w_i / Wsum sum_sigma,j g_j,
//     g_i = sum_k sum_j 2 f[e_i, e_i, e_j] Xa_ij Xb_ij
//           + w'_i (Xa_ii dmu_b + Xb_ii dmu_a - dmu_a dmu_b),
// with f[.,.,.] the second divided difference of the Fermi function and
// w' = -f''. Pairs closer than tau = 1e-3 kT take the same sum written with
// second divided differences, sum_l f[e_i, e_j, e_l] (Xb_il Xa_lj + Xa_il Xb_lj),
// which has no small denominator. Finally dL/dH^sigma = C E'_bar C^T.
#pragma once

#include <hip/hip_runtime.h>

#include "kk_gemm.hpp"
#include "kk_kernels.hpp"

namespace kk {

// Second and fourth derivatives of f(x) = 1/(1+exp(beta(x - mu))).
__device__ __forceinline__ void fermi_d2_d4(double x, double mu, double beta, double* d2, double* d4) {
  const double f = occ(x, mu, beta), fc = occ(-x, -mu, beta), g = f * fc, b2 = beta * beta;
  *d2 = b2 * g * (fc - f);
  *d4 = b2 * b2 * g * (fc - f) * (1.0 - 12.0 * g);
}

// f[x, y, z] for nodes with known f and 1 - f. Nodes spread less than tau:
// expansion about their mean c, f''(c)/2 + f''''(c) h2 / 24 with h2 = 1/2 sum
// of squared deviations (the first-order term vanishes about the mean); else
// (f[b, c] - f[a, b]) / (c - a) over the widest pair of the sorted nodes.
__device__ __forceinline__ double fermi_dd2(double x, double fx, double fcx, double y, double fy, double fcy,
                                            double z, double fz, double fcz, double mu, double beta,
                                            double tau) {
#define KK_SWAP3(p, q)                              \
  if (p > q) {                                      \
    double t_ = p; p = q; q = t_;                   \
    t_ = f##p; f##p = f##q; f##q = t_;              \
    t_ = fc##p; fc##p = fc##q; fc##q = t_;          \
  }
  KK_SWAP3(x, y)
  KK_SWAP3(y, z)
  KK_SWAP3(x, y)
#undef KK_SWAP3
  if (z - x < tau) {
    const double c = (x + y + z) / 3.0;
    const double dx = x - c, dy = y - c, dz = z - c;
    const double h2 = 0.5 * (dx * dx + dy * dy + dz * dz);
    double d2, d4;
    fermi_d2_d4(c, mu, beta, &d2, &d4);
    return 0.5 * d2 + d4 * h2 / 24.0;
  }
  const double f_yz = fermi_divided_difference(y, fy, fcy, z, fz, fcz, beta);
  const double f_xy = fermi_divided_difference(x, fx, fcx, y, fy, fcy, beta);
  return (f_yz - f_xy) / (z - x);
}

// (w_i - w_j)/(e_i - e_j) with w = -f', for |e_i - e_j| < tau: -(f''(m) + f''''(m) h^2 / 6).
__device__ __forceinline__ double w_dd_close(double ei, double ej, double mu, double beta) {
  const double m = 0.5 * (ei + ej), h = 0.5 * (ei - ej);
  double d2, d4;
  fermi_d2_d4(m, mu, beta, &d2, &d4);
  return -(d2 + d4 * h * h / 6.0);
}

struct AdjSpin {
  const double *Xa, *Xb;          // np x np
  const double *eps, *f, *fc, *w;  // np
  double* D;                       // np x np accumulator
  double* gdiag;                   // np accumulator
};
struct AdjSpins {
  AdjSpin s[2];
};

// Reverse-pass state of the Krylov loop on the device.
//   Vbar, Fbar: MAX_RANK x n2, bbar: n2.
// One block of 1024 threads; n2 <= 8192.
__global__ void __launch_bounds__(1024) adj_init(const double* __restrict__ V, const double* __restrict__ Ft,
                                                 const double* __restrict__ ftilde, int n2,
                                                 const KrylovState* __restrict__ st,
                                                 const double* __restrict__ xbar, double* __restrict__ Vbar,
                                                 double* __restrict__ Fbar, double* __restrict__ bbar) {
  __shared__ double sh[17];
  __shared__ double O[MAX_RANK][MAX_RANK + 1];
  __shared__ double c[MAX_RANK], z[MAX_RANK];
  __shared__ int ok;
  const int r = st->rank;
  for (int a = 0; a < r; ++a) {
    for (int b = 0; b <= a; ++b) {
      double d = 0.0;
      for (int i = threadIdx.x; i < n2; i += blockDim.x) d += Ft[(size_t)a * n2 + i] * Ft[(size_t)b * n2 + i];
      d = block_sum(d, sh);
      if (threadIdx.x == 0) O[a][b] = d;
    }
    double d = 0.0, e = 0.0;
    for (int i = threadIdx.x; i < n2; i += blockDim.x) {
      d += Ft[(size_t)a * n2 + i] * ftilde[i];
      e += V[(size_t)a * n2 + i] * xbar[i];
    }
    d = block_sum(d, sh);
    e = block_sum(e, sh);
    if (threadIdx.x == 0) { c[a] = d; z[a] = e; }
  }
  if (threadIdx.x == 0) {
    ok = 1;
    for (int j = 0; j < r && ok; ++j) {
      double dj = O[j][j];
      for (int k = 0; k < j; ++k) dj -= O[j][k] * O[j][k];
      if (!(dj > 0.0)) { ok = 0; break; }
      const double ljj = sqrt(dj);
      O[j][j] = ljj;
      for (int i = j + 1; i < r; ++i) {
        double s = O[i][j];
        for (int k = 0; k < j; ++k) s -= O[i][k] * O[j][k];
        O[i][j] = s / ljj;
      }
    }
    for (int pass = 0; pass < 2 && ok; ++pass) {  // c = O^-1 F~^T f~, z = O^-1 V^T x_bar
      double* x = pass ? z : c;
      for (int i = 0; i < r; ++i) {
        double s = x[i];
        for (int k = 0; k < i; ++k) s -= O[i][k] * x[k];
        x[i] = s / O[i][i];
      }
      for (int i = r - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k < r; ++k) s -= O[k][i] * x[k];
        x[i] = s / O[i][i];
      }
    }
    if (!ok)
      for (int i = 0; i < r; ++i) { c[i] = 0.0; z[i] = 0.0; }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n2; i += blockDim.x) {
    double res = ftilde[i], fz = 0.0;
    for (int a = 0; a < r; ++a) {
      const double fa = Ft[(size_t)a * n2 + i];
      res -= c[a] * fa;
      fz += z[a] * fa;
    }
    bbar[i] = fz;
    const double xb = xbar[i];
    for (int a = 0; a < r; ++a) {
      Fbar[(size_t)a * n2 + i] = res * z[a] - fz * c[a];
      Vbar[(size_t)a * n2 + i] = xb * c[a];
    }
  }
}

// Reverse of the orthonormalization that produced v_{k+1} from f~_k (skipped
// for the last direction), then y = -lambda_k (K0 = -I) or lambda_k (the host
// applies K0^T). One block.
__global__ void __launch_bounds__(1024) adj_gs(const double* __restrict__ V, const double* __restrict__ Ft, int n2,
                                               int k, int last, double* __restrict__ Vbar,
                                               double* __restrict__ Fbar, double* __restrict__ y, int negate) {
  __shared__ double sh[17];
  __shared__ double hh[MAX_RANK], pp[MAX_RANK];
  constexpr int PER = 8;
  double* fb = Fbar + (size_t)k * n2;
  if (!last) {
    const double* vn = V + (size_t)(k + 1) * n2;
    const double* fk = Ft + (size_t)k * n2;
    const double* vb = Vbar + (size_t)(k + 1) * n2;
    double rho = 0.0, t = 0.0;
    for (int i = threadIdx.x; i < n2; i += blockDim.x) {
      rho += vn[i] * fk[i];
      t += vn[i] * vb[i];
    }
    rho = block_sum(rho, sh);
    t = block_sum(t, sh);
    double wb[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int i = threadIdx.x + e * blockDim.x;
      wb[e] = i < n2 ? (vb[i] - vn[i] * t) / rho : 0.0;
    }
    for (int j = 0; j <= k; ++j) {
      const double* vj = V + (size_t)j * n2;
      double h = 0.0, p = 0.0;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int i = threadIdx.x + e * blockDim.x;
        if (i < n2) {
          h += vj[i] * fk[i];
          p += vj[i] * wb[e];
        }
      }
      h = block_sum(h, sh);
      p = block_sum(p, sh);
      if (threadIdx.x == 0) { hh[j] = h; pp[j] = p; }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int i = threadIdx.x + e * blockDim.x;
      if (i >= n2) continue;
      double proj = 0.0;
      for (int j = 0; j <= k; ++j) {
        const double vji = V[(size_t)j * n2 + i];
        proj += vji * pp[j];
        Vbar[(size_t)j * n2 + i] -= wb[e] * hh[j] + fk[i] * pp[j];
      }
      fb[i] += wb[e] - proj;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n2; i += blockDim.x) y[i] = negate ? -fb[i] : fb[i];
}

// y = A^T x for a row-major n x n A (one thread per output; coalesced over columns).
__global__ void gemv_t(const double* __restrict__ A, const double* __restrict__ x, int n, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += A[(size_t)j * n + i] * x[j];
  y[i] = s;
}

// Chemical-potential shifts of the two directions of a reverse step: items
// 0,1 = (a, up/dn), 2,3 = (b, up/dn) of xdiag. One block per direction.
__global__ void adj_dmu(const double* __restrict__ xdiag, int nb, int np, const double* __restrict__ w0,
                        const double* __restrict__ w1, const double* __restrict__ wsum_p, double* __restrict__ dmu) {
  __shared__ double sh[17];
  const int p = blockIdx.x;
  const double* x0 = xdiag + (size_t)(2 * p) * np;
  const double* x1 = xdiag + (size_t)(2 * p + 1) * np;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += w0[i] * x0[i] + w1[i] * x1[i];
  s = block_sum(s, sh);
  const double wsum = *wsum_p;
  if (threadIdx.x == 0) dmu[p] = wsum > 0.0 ? s / wsum : 0.0;
}

// Row i of spin blockIdx.y: D_ij += dmu_b Xa_ij + dmu_a Xb_ij and
// g_i += sum_j 2 f[e_i, e_i, e_j] Xa_ij Xb_ij + w'_i (Xa_ii dmu_b + Xb_ii dmu_a - dmu_a dmu_b).
__global__ void adj_rows(AdjSpins sp, int nb, int np, const double* __restrict__ dmu, const double* __restrict__ mu_p,
                         double beta, double tau) {
  __shared__ double sh[17];
  const AdjSpin& s = sp.s[blockIdx.y];
  const int i = blockIdx.x;
  const double da = dmu[0], db = dmu[1], mu = *mu_p;
  const double ei = s.eps[i], fi = s.f[i], fci = s.fc[i];
  const double* xa = s.Xa + (size_t)i * np;
  const double* xb = s.Xb + (size_t)i * np;
  double* d = s.D + (size_t)i * np;
  double acc = 0.0;
  for (int j = threadIdx.x; j < nb; j += blockDim.x) {
    const double a = xa[j], b = xb[j];
    d[j] += db * a + da * b;
    acc += 2.0 * fermi_dd2(ei, fi, fci, ei, fi, fci, s.eps[j], s.f[j], s.fc[j], mu, beta, tau) * a * b;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    double d2, d4;
    fermi_d2_d4(ei, mu, beta, &d2, &d4);
    s.gdiag[i] += acc - d2 * (xa[i] * db + xb[i] * da - da * db);
  }
}

// Near-degenerate pairs: pk[p] += sum_l f[e_i, e_j, e_l] (Xb_il Xa_jl + Xa_il Xb_jl)
// (X symmetric). pairs[p] = (i, j) for p < n0 in spin 0, then spin 1. One block per pair.
__global__ void adj_pairs(AdjSpins sp, const int2* __restrict__ pairs, int n0, int nb, int np,
                          const double* __restrict__ mu_p, double beta, double tau, double* __restrict__ pk) {
  __shared__ double sh[17];
  const int p = blockIdx.x;
  const AdjSpin& s = sp.s[p < n0 ? 0 : 1];
  const int i = pairs[p].x, j = pairs[p].y;
  const double mu = *mu_p;
  const double ei = s.eps[i], fi = s.f[i], fci = s.fc[i], ej = s.eps[j], fj = s.f[j], fcj = s.fc[j];
  const double *xai = s.Xa + (size_t)i * np, *xbi = s.Xb + (size_t)i * np;
  const double *xaj = s.Xa + (size_t)j * np, *xbj = s.Xb + (size_t)j * np;
  double acc = 0.0;
  for (int l = threadIdx.x; l < nb; l += blockDim.x)
    acc += fermi_dd2(ei, fi, fci, ej, fj, fcj, s.eps[l], s.f[l], s.fc[l], mu, beta, tau) *
           (xbi[l] * xaj[l] + xai[l] * xbj[l]);
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) pk[p] += acc;
}

// E'_bar of one spin in the eigenbasis (see the header), 32 x 32 tiles; pairs
// closer than tau are left at 0 for adj_pair_final.
__global__ void adj_final(const double* __restrict__ K, const double* __restrict__ D, const double* __restrict__ eps,
                          const double* __restrict__ w, const double* __restrict__ gdiag,
                          const double* __restrict__ gtot_p, const double* __restrict__ wsum_p, int nb, int np,
                          double tau, double* __restrict__ Ep) {
  __shared__ double kt[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int r = ty; r < 32; r += 8) kt[r][tx] = K[(size_t)(bx + r) * np + by + tx];  // K^T tile
  __syncthreads();
  const double wsum = *wsum_p, gtot = *gtot_p;
  for (int r = ty; r < 32; r += 8) {
    const int i = by + r, j = bx + tx;
    double v = 0.0;
    if (i < nb && j < nb) {
      if (i == j) {
        v = gdiag[i] - (wsum > 0.0 ? w[i] / wsum * gtot : 0.0);
      } else {
        const double gap = eps[i] - eps[j];
        if (fabs(gap) >= tau) {
          const size_t ij = (size_t)i * np + j;
          v = ((K[ij] - kt[tx][r]) + (w[i] - w[j]) * D[ij]) / gap;
        }
      }
    }
    Ep[(size_t)i * np + j] = v;
  }
}

__global__ void adj_pair_final(const int2* __restrict__ pairs, int n0, int npairs, const double* __restrict__ pk,
                               const double* __restrict__ D0, const double* __restrict__ D1,
                               const double* __restrict__ e0, const double* __restrict__ e1,
                               const double* __restrict__ mu_p, double beta, int np, double* __restrict__ Ep0,
                               double* __restrict__ Ep1) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const bool s1 = p >= n0;
  const double* D = s1 ? D1 : D0;
  const double* e = s1 ? e1 : e0;
  double* Ep = s1 ? Ep1 : Ep0;
  const int i = pairs[p].x, j = pairs[p].y;
  const double v = pk[p] + w_dd_close(e[i], e[j], *mu_p, beta) * D[(size_t)i * np + j];
  Ep[(size_t)i * np + j] = v;
  Ep[(size_t)j * np + i] = v;
}

// v_bar_k += Gamma g - y and gamma_bar += g_q v_q^T; one wave per atom row.
__global__ void adj_apply(const double* __restrict__ gamma, int N, double W, const double* __restrict__ g,
                          const double* __restrict__ y, const double* __restrict__ vk, double* __restrict__ vbar,
                          double* __restrict__ gamma_bar) {
  const int a = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  if (a >= N) return;
  const double* gr = gamma + (size_t)a * N;
  double* gb = gamma_bar + (size_t)a * N;
  const double ga = g[a];
  double s = 0.0;
  for (int j = lane; j < N; j += WAVE) {
    s += gr[j] * g[j];
    gb[j] += ga * vk[j];
  }
  s = wave_sum(s);
  if (lane == 0) {
    vbar[a] += s - y[a];
    vbar[N + a] += W * g[N + a] - y[N + a];
  }
}

// W_bar += g_m . v_m (one block, fixed order).
__global__ void adj_wbar(const double* __restrict__ g, const double* __restrict__ vk, int N, double* __restrict__ wbar) {
  __shared__ double sh[17];
  double s = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) s += g[N + i] * vk[N + i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *wbar += s;
}

// f~_bar += reverse of v_1 = f~ / |f~|; out = -f~_bar (K0 = -I) or f~_bar. One block.
__global__ void __launch_bounds__(1024) adj_finish(const double* __restrict__ V, const double* __restrict__ Vbar,
                                                   const double* __restrict__ ftilde, int n2,
                                                   const double* __restrict__ bbar, double* __restrict__ out,
                                                   int negate) {
  __shared__ double sh[17];
  double t = 0.0, nn = 0.0;
  for (int i = threadIdx.x; i < n2; i += blockDim.x) {
    t += V[i] * Vbar[i];
    nn += ftilde[i] * ftilde[i];
  }
  t = block_sum(t, sh);
  const double nrm = sqrt(block_sum(nn, sh));
  for (int i = threadIdx.x; i < n2; i += blockDim.x) {
    const double b = bbar[i] + (nrm > 0.0 ? (Vbar[i] - V[i] * t) / nrm : 0.0);
    out[i] = negate ? -b : b;
  }
}

// dst (nb x nb) = src (np x np) without the padding.
__global__ void unpad_copy(const double* __restrict__ src, int np, double* __restrict__ dst, int nb) {
  const size_t n = (size_t)nb * nb;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / nb, j = e - i * nb;
    dst[e] = src[i * np + j];
  }
}

}  // namespace kk
