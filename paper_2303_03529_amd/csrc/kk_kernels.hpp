// Vector, reduction and setup kernels of the spin-charge response and the
// Krylov loop. All reductions use a fixed order, so results are bitwise
// reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>

namespace kk {

constexpr int WAVE = 64;
constexpr double BREAKDOWN_TOL = 1e-13;
constexpr int MAX_RANK = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Wave-wide sum of a double in a fixed order, the same bits in every lane, for serial
// reduction chains (the orthonormalization, the m x m solve): within each row of 16 lanes by DPP moves
// (rotate by 8 and 4, then exchange with lane ^ 2 and lane ^ 1: every step adds two values
// that the partner lane adds in the other order, so all 16 lanes end with the same bits),
// then the four row sums read from lanes 0, 16, 32 and 48 and added as (r0 + r1) + (r2 + r3).
// The cross-lane moves stay in the VALU, where a shuffle through the LDS crossbar costs a
// round trip per step.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_f64(double v, int lane) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0x128>(v);  // row_ror:8
  v += dpp_f64<0x124>(v);  // row_ror:4
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Sum over a block of up to 1024 threads (multiple of 64); every thread gets
// thread 0's total. sh must hold at least 17 doubles.
__device__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const int nw = blockDim.x / WAVE;
  v = wave_sum(v);
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  if (wave == 0) {
    double t = (lane < nw) ? sh[lane] : 0.0;
    t = wave_sum(t);
    if (lane == 0) sh[16] = t;
  }
  __syncthreads();
  const double r = sh[16];
  __syncthreads();
  return r;
}

// dst (np x np, zero padded) = src (nb x nb) or its transpose. 32 x 32 tiles.
__global__ void pad_copy(const double* __restrict__ src, int nb, double* __restrict__ dst, int np,
                         int transpose) {
  __shared__ double t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int k = ty; k < 32; k += 8) {
    // read source rows coalesced: source tile origin is (by, bx) if plain, (bx, by) if transposed
    const int sr = (transpose ? bx : by) + k, sc = (transpose ? by : bx) + tx;
    t[k][tx] = (sr < nb && sc < nb) ? src[(size_t)sr * nb + sc] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int dr = by + k, dc = bx + tx;
    if (dr < np && dc < np) dst[(size_t)dr * np + dc] = transpose ? t[tx][k] : t[k][tx];
  }
}

// dst (np x np) = src^T (both np x np).
__global__ void transpose_sq(const double* __restrict__ src, double* __restrict__ dst, int np) {
  __shared__ double t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) t[k][tx] = src[(size_t)(bx + k) * np + by + tx];
  __syncthreads();
  for (int k = ty; k < 32; k += 8) dst[(size_t)(by + k) * np + bx + tx] = t[tx][k];
}

__device__ __forceinline__ double occ(double e, double mu, double beta) {
  return 1.0 / (1.0 + exp(beta * (e - mu)));
}

// Sec. II.C: one chemical potential for both spins with sum_sigma sum_k
// f(eps_k) = N_e. Bisection on [min eps - 40 kT, max eps + 40 kT], then Newton
// steps with dN/dmu = sum beta f (1 - f). One block of 1024 threads.
__global__ void __launch_bounds__(1024) solve_mu(const double* __restrict__ e_up,
                                                 const double* __restrict__ e_dn, int nb,
                                                 double n_e, double beta, double* mu_out) {
  __shared__ double sh[17];
  const double kT = 1.0 / beta;
  double lo = 1e300, hi = -1e300;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    lo = fmin(lo, fmin(e_up[i], e_dn[i]));
    hi = fmax(hi, fmax(e_up[i], e_dn[i]));
  }
  // min/max via sums of one-hot is awkward; use LDS reductions directly.
  __shared__ double smin[1024], smax[1024];
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  lo = smin[0] - 40.0 * kT;
  hi = smax[0] + 40.0 * kT;
  __syncthreads();
  for (int iter = 0; iter < 400; ++iter) {
    const double mid = 0.5 * (lo + hi);
    double c = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) c += occ(e_up[i], mid, beta) + occ(e_dn[i], mid, beta);
    c = block_sum(c, sh);
    if (c < n_e) lo = mid; else hi = mid;
    if (hi - lo <= 1e-15 * fmax(1.0, fabs(mid))) break;
  }
  double mu = 0.5 * (lo + hi);
  for (int it = 0; it < 3; ++it) {
    double c = 0.0, d = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
      const double fu = occ(e_up[i], mu, beta), fd = occ(e_dn[i], mu, beta);
      c += fu + fd;
      d += fu * occ(-e_up[i], -mu, beta) + fd * occ(-e_dn[i], -mu, beta);
    }
    c = block_sum(c, sh);
    d = block_sum(d, sh) * beta;
    const double resid = c - n_e;
    if (d <= 0.0 || fabs(resid) <= 1e-13 * n_e) break;
    mu -= resid / d;
  }
  if (threadIdx.x == 0) *mu_out = mu;
}

// Occupations of one spin: f = 1/(1+exp(beta(e-mu))), fc = 1 - f (computed as
// f of the mirrored argument), w = beta f fc; padded entries (i >= nb) are 0.
__global__ void occupations(const double* __restrict__ eps_in, int nb, int np,
                            const double* __restrict__ mu_p, double beta, double* __restrict__ eps,
                            double* __restrict__ f, double* __restrict__ fc, double* __restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  if (i < nb) {
    const double mu = *mu_p, e = eps_in[i];
    const double a = occ(e, mu, beta), b = occ(-e, -mu, beta);
    eps[i] = e; f[i] = a; fc[i] = b; w[i] = beta * a * b;
  } else {
    eps[i] = 0.0; f[i] = 0.0; fc[i] = 0.0; w[i] = 0.0;
  }
}

// out[s*natoms + I] = sum_{i in I} sum_k X_s[i][k] * Y_s[i][k] * (wk ? wk_s[k] : 1)
// for s = 0, 1 (two spins). One block per atom.
__global__ void atom_row_dots(const double* __restrict__ x0, const double* __restrict__ x1, int ldx,
                              const double* __restrict__ y0, const double* __restrict__ y1, int ldy,
                              const double* __restrict__ wk0, const double* __restrict__ wk1,
                              int ncols, const int* __restrict__ offsets, int natoms,
                              double* __restrict__ out) {
  __shared__ double sh[17];
  const int a = blockIdx.x;
  const int r0 = offsets[a], r1 = offsets[a + 1];
  for (int s = 0; s < 2; ++s) {
    const double* x = s ? x1 : x0;
    const double* y = s ? y1 : y0;
    const double* wk = s ? wk1 : wk0;
    double acc = 0.0;
    for (int i = r0; i < r1; ++i) {
      const double* xr = x + (size_t)i * ldx;
      const double* yr = y + (size_t)i * ldy;
      for (int k = threadIdx.x; k < ncols; k += blockDim.x) {
        const double p = xr[k] * yr[k];
        acc += wk ? p * wk[k] : p;
      }
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[s * natoms + a] = acc;
  }
}

// Mulliken projection of caller density-matrix changes (Sec. III.A):
// dn^s_I = sum_{i in I} sum_j dD^s_ij S_ji, S symmetric so S_ji = S_ij.
// Output (dq, dm) = (dn_up + dn_dn, dn_up - dn_dn). One block per atom and item.
__global__ void mulliken_rows(const double* __restrict__ dup, const double* __restrict__ ddn, int nb,
                              const double* __restrict__ S, int lds, const int* __restrict__ offsets,
                              int natoms, double* __restrict__ dqm) {
  __shared__ double sh[17];
  const int a = blockIdx.x, b = blockIdx.y;
  const size_t mat = (size_t)nb * nb * b;
  const int r0 = offsets[a], r1 = offsets[a + 1];
  double su = 0.0, sd = 0.0;
  for (int i = r0; i < r1; ++i) {
    const double* pu = dup + mat + (size_t)i * nb;
    const double* pd = ddn + mat + (size_t)i * nb;
    const double* ps = S + (size_t)i * lds;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
      const double s = ps[k];
      su += pu[k] * s;
      sd += pd[k] * s;
    }
  }
  su = block_sum(su, sh);
  sd = block_sum(sd, sh);
  if (threadIdx.x == 0) {
    dqm[(size_t)b * 2 * natoms + a] = su + sd;
    dqm[(size_t)b * 2 * natoms + natoms + a] = su - sd;
  }
}

// Per-orbital spin potentials for a batch of directions (Sec. III.A):
// u^s_I = sum_J gamma_IJ v_q[J] + sign_s W v_m[I], written to every orbital of
// atom I in u[(b*2 + s)*np + i]. One wave per (atom, direction). With gamma
// NULL the coupling is the identity, u^s_I = v_q[I] + sign_s W v_m[I] (the
// reverse pass uses it with W = 1 to apply the transposed response).
__device__ __forceinline__ void potentials_dev(const double* __restrict__ gamma, int natoms, double W,
                                               const double* __restrict__ v, int batch,
                                               const int* __restrict__ offsets, int np, double* __restrict__ u,
                                               const int* __restrict__ stop, int bx) {
  if (stop != nullptr && *stop != 0) return;
  const int wid = (bx * blockDim.x + threadIdx.x) / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  if (wid >= natoms * batch) return;
  const int b = wid / natoms, a = wid - b * natoms;
  const double* vb = v + (size_t)b * 2 * natoms;
  double s = 0.0;
  if (gamma != nullptr) {
    const double* g = gamma + (size_t)a * natoms;
    for (int j = lane; j < natoms; j += WAVE) s += g[j] * vb[j];
    s = wave_sum(s);
  } else {
    s = vb[a];
  }
  const double up = s + W * vb[natoms + a];
  const double dn = s - W * vb[natoms + a];
  for (int i = offsets[a] + lane; i < offsets[a + 1]; i += WAVE) {
    u[((size_t)b * 2 + 0) * np + i] = up;
    u[((size_t)b * 2 + 1) * np + i] = dn;
  }
}

__global__ void potentials(const double* __restrict__ gamma, int natoms, double W,
                           const double* __restrict__ v, int batch, const int* __restrict__ offsets,
                           int np, double* __restrict__ u, const int* __restrict__ stop) {
  potentials_dev(gamma, natoms, W, v, batch, offsets, np, u, stop, blockIdx.x);
}

// Combine the two spins (Sec. II.C, III.A): dmu from the diagonal of X,
// Mulliken sums per atom, and q1 = (dn_up + dn_dn, dn_up - dn_dn).
//   xdiag[(b*2+s)*np + i], part[(b*2+s)][p][np], t[s*natoms + I] = sum_{i in I}
//   sum_k C_ik w_k G_ik (the response to a unit chemical-potential shift),
//   wsum = sum_s sum_i w_i.
// One wave per atom: its lanes split the partial rows, each adds the atom's
// orbitals of its rows, and the wave reduces. Grid: (ceil(natoms / waves per
// block), batch); every block also reduces dmu over all orbitals (cached reads).
__device__ __forceinline__ void combine_dev(const double* __restrict__ xdiag, const double* __restrict__ part,
                                            int nparts, int part_stride, const double* __restrict__ w_up,
                                            const double* __restrict__ w_dn, const double* __restrict__ wsum_p,
                                            const double* __restrict__ t, int nb, int np,
                                            const int* __restrict__ offsets, int natoms, double* __restrict__ q1,
                                            const int* __restrict__ stop, int bx, int by,
                                            const double* __restrict__ vsub = nullptr, double* __restrict__ ft = nullptr) {
  if (stop != nullptr && *stop != 0) return;
  __shared__ double sh[17];
  const int b = by;
  const double* xu = xdiag + ((size_t)b * 2 + 0) * np;
  const double* xd = xdiag + ((size_t)b * 2 + 1) * np;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += w_up[i] * xu[i] + w_dn[i] * xd[i];
  s = block_sum(s, sh);
  const double wsum = *wsum_p;
  const double dmu = wsum > 0.0 ? s / wsum : 0.0;
  const int lane = threadIdx.x & (WAVE - 1);
  const int a = bx * (blockDim.x / WAVE) + (int)(threadIdx.x / WAVE);
  if (a >= natoms) return;
  const int i0 = offsets[a], i1 = offsets[a + 1];
  double dn[2];
  for (int sp = 0; sp < 2; ++sp) {
    const double* pp = part + ((size_t)b * 2 + sp) * part_stride * np;
    double acc = 0.0;
    for (int p = lane; p < nparts; p += WAVE)
      for (int i = i0; i < i1; ++i) acc += pp[(size_t)p * np + i];
    dn[sp] = wave_sum(acc) + dmu * t[sp * natoms + a];
  }
  if (lane == 0) {
    const double qa = dn[0] + dn[1], ma = dn[0] - dn[1];
    q1[(size_t)b * 2 * natoms + a] = qa;
    q1[(size_t)b * 2 * natoms + natoms + a] = ma;
    if (ft != nullptr) {  // the preconditioned directional derivative with K0 = -I: -(q1 - v)
      ft[a] = -(qa - vsub[a]);
      ft[natoms + a] = -(ma - vsub[natoms + a]);
    }
  }
}

// Blocks of the combine kernels: COMBINE_THREADS threads, one wave per atom.
constexpr int COMBINE_THREADS = 256;
constexpr int COMBINE_ATOMS = COMBINE_THREADS / WAVE;

__global__ void combine(const double* __restrict__ xdiag, const double* __restrict__ part, int nparts,
                        const double* __restrict__ w_up, const double* __restrict__ w_dn,
                        const double* __restrict__ wsum_p, const double* __restrict__ t, int nb, int np,
                        const int* __restrict__ offsets, int natoms, double* __restrict__ q1,
                        const int* __restrict__ stop, const double* __restrict__ vsub = nullptr,
                        double* __restrict__ ft = nullptr) {
  combine_dev(xdiag, part, nparts, nparts, w_up, w_dn, wsum_p, t, nb, np, offsets, natoms, q1, stop, blockIdx.x,
              blockIdx.y, vsub, ft);
}

// sum of both spins' w (one block).
__global__ void sum_two(const double* __restrict__ a, const double* __restrict__ b, int n,
                        double* __restrict__ out) {
  __shared__ double sh[17];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += a[i] + b[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------------------
// Krylov loop (Sec. II.G)

struct KrylovState {
  int rank;       // accepted directions
  int stop;       // 1 after a breakdown, a zero starting vector or reaching the residual target
  int status;     // 0 ok, 1 breakdown, -5 singular Gram matrix
  int pad;
  double min_pivot, max_pivot;
  double ls_residual;  // ||F~ c - f~|| / ||f~|| of the last solve
};

// y = K0 (x - sub) (sub may be null), or -(x - sub) when K0 is null.
// One wave per row. Skipped after a breakdown when stop is given. With reset given (the
// first launch of an update, stop null) thread 0 also clears that Krylov state.
__global__ void precondition(const double* __restrict__ K0, const double* __restrict__ x,
                             const double* __restrict__ sub, double* __restrict__ y, int n2,
                             const int* __restrict__ stop, KrylovState* reset = nullptr) {
  if (reset != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
    reset->rank = 0; reset->stop = 0; reset->status = 0; reset->pad = 0;
    reset->min_pivot = 0.0; reset->max_pivot = 0.0; reset->ls_residual = 1.0;
  }
  if (stop != nullptr && *stop != 0) return;
  const int row = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  if (row >= n2) return;
  if (K0 == nullptr) {
    if (lane == 0) y[row] = -(x[row] - (sub ? sub[row] : 0.0));
    return;
  }
  const double* kr = K0 + (size_t)row * n2;
  double s = 0.0;
  for (int j = lane; j < n2; j += WAVE) s += kr[j] * (x[j] - (sub ? sub[j] : 0.0));
  s = wave_sum(s);
  if (lane == 0) y[row] = s;
}

// Orthogonalize src against the accepted directions V[0..rank) with modified
// Gram-Schmidt, two passes; accept it as V[rank] if its norm kept more than
// BREAKDOWN_TOL of its starting norm, else stop the expansion. One block of
// at least n2 / 8 threads.
__device__ __forceinline__ void orth_dev(const double* __restrict__ src, double* __restrict__ V, int n2,
                                         KrylovState* st) {
  __shared__ double sh[17];
  if (st->stop) return;
  const int rank = st->rank;
  constexpr int PER = 8;  // n2 <= 8 * 1024
  double w[PER];
  double nn = 0.0;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int i = threadIdx.x + e * blockDim.x;
    w[e] = i < n2 ? src[i] : 0.0;
    nn += w[e] * w[e];
  }
  const double start = sqrt(block_sum(nn, sh));
  // Two passes of projections against v_0 .. v_{rank-1}, in order; the entries of
  // the next v_j are loaded before the current projection's reduction, so the
  // loop waits on reductions, not on loads. Entries past n2 are zero in w and v.
  auto load_row = [&](int j, double* dst) {
    const double* vj = V + (size_t)j * n2;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int i = threadIdx.x + e * blockDim.x;
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
    d = block_sum(d, sh);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      w[e] -= d * cur[e];
      cur[e] = nxt[e];
    }
  }
  nn = 0.0;
#pragma unroll
  for (int e = 0; e < PER; ++e) nn += w[e] * w[e];
  const double nrm = sqrt(block_sum(nn, sh));
  if (!(nrm > BREAKDOWN_TOL * start) || rank >= MAX_RANK) {
    if (threadIdx.x == 0) {
      st->stop = 1;
      if (rank > 0) st->status = 1;
    }
    return;
  }
  double* vr = V + (size_t)rank * n2;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int i = threadIdx.x + e * blockDim.x;
    if (i < n2) vr[i] = w[e] / nrm;
  }
  __syncthreads();
  if (threadIdx.x == 0) st->rank = rank + 1;
}

__global__ void __launch_bounds__(1024) krylov_orthonormalize(const double* __restrict__ src,
                                                              double* __restrict__ V, int n2,
                                                              KrylovState* st) {
  orth_dev(src, V, n2, st);
}

// O = F~^T F~, rhs = F~^T f~, Cholesky O = L L^T, c = O^-1 rhs, x = V c, and the
// projected residual ||F~ c - f~|| / ||f~|| formed explicitly. On a non-positive
// pivot x = 0 and status = -5. With stop_tol > 0 a residual <= stop_tol ends the
// expansion (used by the adaptive-rank call after each direction). One block.
__device__ __forceinline__ void solve_dev(const double* __restrict__ V, const double* __restrict__ Ft,
                                          const double* __restrict__ ftilde, int n2, KrylovState* st,
                                          double* __restrict__ x, double stop_tol) {
  __shared__ double sr[2][16];
  __shared__ double O[MAX_RANK][MAX_RANK + 1];
  __shared__ double c[MAX_RANK];
  __shared__ int ok;
  const int r = st->rank;
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  // The r (r + 1) / 2 entries of O and the r of the right-hand side, one wave each (fixed
  // lane order and reduction tree, so the result is deterministic); 4 loads per lane in flight.
  {
    const int npairs = r * (r + 1) / 2;
    for (int p = wave; p < npairs + r; p += nw) {
      int a, b = -1;
      if (p < npairs) {
        a = 0;
        while ((a + 1) * (a + 2) / 2 <= p) ++a;
        b = p - a * (a + 1) / 2;
      } else {
        a = p - npairs;
      }
      const double* fa = Ft + (size_t)a * n2;
      const double* y = b >= 0 ? Ft + (size_t)b * n2 : ftilde;
      double d4[4] = {0.0, 0.0, 0.0, 0.0};
      for (int base = 0; base < n2; base += 4 * WAVE) {
        double xa[4], xb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int i = base + lane + k * WAVE;
          xa[k] = i < n2 ? fa[i] : 0.0;
          xb[k] = i < n2 ? y[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) d4[k] += xa[k] * xb[k];
      }
      const double d = wave_sum_dpp((d4[0] + d4[1]) + (d4[2] + d4[3]));
      if (lane == 0) {
        if (b >= 0) { O[a][b] = d; O[b][a] = d; }
        else c[a] = d;
      }
    }
  }
  __syncthreads();
  if (wave == 0) {
    // Cholesky O = L L^T in wave 0, lane i owning row i (r <= MAX_RANK = WAVE): column j's
    // entries l_ij = O_ij / l_jj, then the trailing update O_ik -= l_ij l_kj (k <= i), l_kj
    // taken from lane k. One wave's LDS accesses complete in order.
    int good = 1;
    double pmin = 0.0, pmax = 0.0;
    for (int j = 0; j < r; ++j) {
      const double dj = O[j][j];
      if (!(dj > 0.0)) {  // the same value in every lane
        good = 0;
        break;
      }
      pmin = (j == 0) ? dj : fmin(pmin, dj);
      pmax = (j == 0) ? dj : fmax(pmax, dj);
      const double ljj = sqrt(dj);
      const bool below = lane > j && lane < r;
      const double lij = below ? O[lane][j] / ljj : 0.0;
      if (lane == j) O[j][j] = ljj;
      if (below) O[lane][j] = lij;
      for (int k = j + 1; k < r; ++k) {
        const double lkj = lane_f64(lij, k);
        if (below && k <= lane) O[lane][k] -= lij * lkj;
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (good) {
      double ci = lane < r ? c[lane] : 0.0;
      for (int j = 0; j < r; ++j) {  // L y = rhs
        const double yj = lane_f64(ci / O[j][j], j);
        if (lane == j) ci = yj;
        else if (lane > j && lane < r) ci -= O[lane][j] * yj;
      }
      for (int j = r - 1; j >= 0; --j) {  // L^T c = y
        const double xj = lane_f64(ci / O[j][j], j);
        if (lane == j) ci = xj;
        else if (lane < j) ci -= O[j][lane] * xj;
      }
      if (lane < r) c[lane] = ci;
    }
    if (lane == 0) {
      ok = good;
      if (!good) st->status = -5;
      st->min_pivot = pmin;
      st->max_pivot = pmax;
    }
  }
  __syncthreads();
  const int okv = ok;
  double rr = 0.0, ff = 0.0;
  for (int i = threadIdx.x; i < n2; i += blockDim.x) {
    double s = 0.0, fi = 0.0;
    if (okv) {
      int k = 0;
      for (; k + 4 <= r; k += 4) {
        double vv[4], fv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          vv[q] = V[(size_t)(k + q) * n2 + i];
          fv[q] = Ft[(size_t)(k + q) * n2 + i];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          s += c[k + q] * vv[q];
          fi += c[k + q] * fv[q];
        }
      }
      for (; k < r; ++k) {
        s += c[k] * V[(size_t)k * n2 + i];
        fi += c[k] * Ft[(size_t)k * n2 + i];
      }
    }
    x[i] = s;
    const double fti = ftilde[i];
    const double e = fi - fti;
    rr += e * e;
    ff += fti * fti;
  }
  rr = wave_sum_dpp(rr);
  ff = wave_sum_dpp(ff);
  if (lane == 0) {
    sr[0][wave] = rr;
    sr[1][wave] = ff;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    rr = 0.0;
    ff = 0.0;
    for (int q = 0; q < nw; ++q) {
      rr += sr[0][q];
      ff += sr[1][q];
    }
    const double res = ff > 0.0 ? sqrt(rr / ff) : 0.0;
    st->ls_residual = res;
    if (stop_tol > 0.0 && okv && res <= stop_tol) st->stop = 1;
  }
}

__global__ void __launch_bounds__(1024) krylov_solve(const double* __restrict__ V,
                                                     const double* __restrict__ Ft,
                                                     const double* __restrict__ ftilde, int n2,
                                                     KrylovState* st, double* __restrict__ x,
                                                     double stop_tol) {
  solve_dev(V, Ft, ftilde, n2, st, x, stop_tol);
}

// Host-side copies of the argument lists of precondition and krylov_solve (declaration
// order), read from and written back to a kernel node of a captured graph so that a replay
// can take other input and output pointers.
template <class T>
inline T kernel_arg(void** kp, int i) {
  T v;
  __builtin_memcpy(&v, kp[i], sizeof v);
  return v;
}

struct PreconditionArgs {
  static constexpr int COUNT = 7;
  const double *K0, *x, *sub;
  double* y;
  int n2;
  const int* stop;
  KrylovState* reset;
  static PreconditionArgs from(void** kp) {
    return {kernel_arg<const double*>(kp, 0), kernel_arg<const double*>(kp, 1), kernel_arg<const double*>(kp, 2),
            kernel_arg<double*>(kp, 3),       kernel_arg<int>(kp, 4),           kernel_arg<const int*>(kp, 5),
            kernel_arg<KrylovState*>(kp, 6)};
  }
  void pointers(void** out) {
    out[0] = &K0; out[1] = &x; out[2] = &sub; out[3] = &y; out[4] = &n2; out[5] = &stop; out[6] = &reset;
  }
};

struct SolveArgs {
  static constexpr int COUNT = 7;
  const double *V, *Ft, *ftilde;
  int n2;
  KrylovState* st;
  double* out;
  double tol;
  static SolveArgs from(void** kp) {
    return {kernel_arg<const double*>(kp, 0), kernel_arg<const double*>(kp, 1), kernel_arg<const double*>(kp, 2),
            kernel_arg<int>(kp, 3),           kernel_arg<KrylovState*>(kp, 4),  kernel_arg<double*>(kp, 5),
            kernel_arg<double>(kp, 6)};
  }
  void pointers(void** o) {
    o[0] = &V; o[1] = &Ft; o[2] = &ftilde; o[3] = &n2; o[4] = &st; o[5] = &out; o[6] = &tol;
  }
};

// (q, m) Mulliken vector of per-spin atom populations: out = (p_up + p_dn - ref, p_up - p_dn),
// ref = neutral-atom populations (may be null).
__global__ void mix_spins(const double* __restrict__ p, const double* __restrict__ ref, int natoms,
                          double* __restrict__ out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= natoms) return;
  const double u = p[a], d = p[natoms + a];
  out[a] = u + d - (ref ? ref[a] : 0.0);
  out[natoms + a] = u - d;
}

// Extended-Lagrangian update of the electronic coordinates (Sec. II.F):
//   n(t+dt) = 2 n(t) - n(t-dt) - kappa K f + alpha sum_k c_k n(t - k dt),
// hist[k] = n(t - k dt) for k = 0..kmax (row-major (kmax+1) x n2), Kf the
// kernel applied to the residual f = q[n] - n, c on the device.
__global__ void xlbomd_update(const double* __restrict__ hist, int kmax, int n2, const double* __restrict__ Kf,
                              double kappa, double alpha, const double* __restrict__ c,
                              double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  const double n0 = hist[i];
  const double n1 = kmax >= 1 ? hist[(size_t)n2 + i] : n0;
  double diss = 0.0;
  for (int k = 0; k <= kmax; ++k) diss += c[k] * hist[(size_t)k * n2 + i];
  out[i] = 2.0 * n0 - n1 - kappa * Kf[i] + alpha * diss;
}

}  // namespace kk
