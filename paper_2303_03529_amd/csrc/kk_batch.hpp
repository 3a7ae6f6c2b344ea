// Batched rank-m Krylov kernel over many independent systems of uneven size.
//
// Every system keeps its own prepared state (a full single-system handle);
// the batch adds device descriptor tables so that each step of the Krylov
// loop is ONE launch for all systems: small kernels take the system from
// blockIdx.y, and the two dense transforms are persistent kernels that walk a
// global tile list (system, spin, tile row, tile column) sorted by cost.
// The whole update is captured once into a hipGraph and replayed.
#pragma once

#include <hip/hip_runtime.h>

#include "kk_gemm.hpp"
#include "kk_gemm_mixed.hpp"
#include "kk_kernels.hpp"

namespace kk {

struct SysDesc {
  int natoms, nb, np, nparts;  // nparts: Mulliken partial rows written per spin by the tile class in use
  int part_stride, pad;        // rows reserved per spin in part
  double W, beta;
  const int* offsets;
  const double* gamma;
  double* u;        // 2 x np (spin potentials per orbital)
  double* xdiag;    // 2 x np
  double* part;     // 2 x nparts x np
  const double *w0, *w1, *wsum, *t;
  double *V, *Ft, *ftilde, *q1;
  KrylovState* kst;
  // split-precision path
  double* msc;             // 2 x 8
  const double* mconst;    // 8
  const double *CT0, *CT1;
  _Float16 *uct_h, *uct_l;  // 2 x np^2 each
};

struct BatchItemF64 {
  GemmItem g;
  int n, k;  // padded size; contraction length (rows past the system's nb are zero)
  const int* stop;
  double beta;
};

struct BatchItemMixed {
  MixedItem g;
  int n, k;
  const int* stop;
  double beta;
};

__global__ void b_reset(SysDesc* d) {
  if (threadIdx.x == 0) {
    KrylovState* st = d[blockIdx.x].kst;
    st->rank = 0; st->stop = 0; st->status = 0; st->pad = 0;
    st->min_pivot = 0.0; st->max_pivot = 0.0; st->ls_residual = 1.0;
  }
}

// f~ = K0 delta with K0 = -I; delta from the pointer table.
__global__ void b_init(const SysDesc* __restrict__ d, const double* const* __restrict__ delta) {
  const SysDesc& s = d[blockIdx.y];
  const int n2 = 2 * s.natoms;
  const double* x = delta[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += gridDim.x * blockDim.x) s.ftilde[i] = -x[i];
}

__global__ void __launch_bounds__(1024) b_orth(SysDesc* d, int k) {
  const SysDesc& s = d[blockIdx.x];
  const int n2 = 2 * s.natoms;
  const double* src = (k == 0) ? s.ftilde : s.Ft + (size_t)(k - 1) * n2;
  orth_dev(src, s.V, n2, s.kst);
}

__global__ void b_potentials(const SysDesc* __restrict__ d, int k) {
  const SysDesc& s = d[blockIdx.y];
  const int n2 = 2 * s.natoms;
  if ((int)(blockIdx.x * blockDim.x / WAVE) >= s.natoms) return;
  potentials_dev(s.gamma, s.natoms, s.W, s.V + (size_t)k * n2, 1, s.offsets, s.np, s.u, &s.kst->stop,
                 blockIdx.x);
}

__global__ void b_center(const SysDesc* __restrict__ d) {
  const SysDesc& s = d[blockIdx.x];
  center_potentials_dev(s.u, s.np, s.nb, s.w0, s.w1, &s.kst->stop, 0);
}

__global__ void b_mixed_scales(const SysDesc* __restrict__ d) {
  const SysDesc& s = d[blockIdx.y];
  mixed_scales_dev(s.u, s.np, s.mconst, s.beta, s.msc, &s.kst->stop, blockIdx.x);
}

// blockIdx.z = system, blockIdx.y = spin: the split forward operand (U~ C)^T
__global__ void b_split(const SysDesc* __restrict__ d) {
  const SysDesc& s = d[blockIdx.z];
  const int spin = blockIdx.y;
  const size_t np2 = (size_t)s.np * s.np;
  split_scaled_columns_dev(spin ? s.CT1 : s.CT0, s.np, s.u + (size_t)spin * s.np, s.msc + spin * 8 + 3,
                           s.uct_h + spin * np2, s.uct_l + spin * np2, &s.kst->stop, blockIdx.x, gridDim.x);
}

// The forward's symmetrizing pass over every item of the batch: blockIdx.x runs over
// the block pairs of all items, item z owning [pair_off[z], pair_off[z + 1]).
__device__ __forceinline__ int pair_item(const int* __restrict__ pair_off, int nitems, int g) {
  int lo = 0, hi = nitems;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (pair_off[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}
// Block side of the pair list: split batches pad every system to the large split tile and
// take its 64 x 64 block pairs (512 threads); FP64 batches (padded to 128) 64 x 64 as well.
constexpr int BATCH_SYM_B_MIXED = SYM_B_LARGE, BATCH_SYM_T_MIXED = SYM_T_LARGE;
constexpr int BATCH_SYM_B_F64 = SYM64_B_LARGE, BATCH_SYM_T_F64 = SYM64_T_LARGE;

// (Against the earlier pass with one element per thread and row: the same bits, and
// the 64-cluster split batch 19.59 -> 19.76 batch updates/s, one process.)
__global__ __launch_bounds__(BATCH_SYM_T_MIXED) void b_symmetrize(const BatchItemMixed* __restrict__ items,
                                                                  const int* __restrict__ pair_off, int nitems) {
  static_assert(BATCH_SYM_B_MIXED == 64 && BATCH_SYM_T_MIXED == 512, "64 x 64 pairs, 8 elements per thread");
  const int z = pair_item(pair_off, nitems, blockIdx.x);
  const BatchItemMixed& it = items[z];
  if (*it.stop) return;
  fermi_symmetrize_v8_dev<false, 2>(it.g, it.n, it.beta, blockIdx.x - pair_off[z]);
}

__global__ __launch_bounds__(BATCH_SYM_T_F64) void b_symmetrize_f64(const BatchItemF64* __restrict__ items,
                                                        const int* __restrict__ pair_off, int nitems) {
  const int z = pair_item(pair_off, nitems, blockIdx.x);
  const BatchItemF64& it = items[z];
  if (*it.stop) return;
  fermi_symmetrize_f64_dev<BATCH_SYM_B_F64, BATCH_SYM_T_F64>(it.g, it.n, it.beta, blockIdx.x - pair_off[z]);
}

__global__ void b_combine(const SysDesc* __restrict__ d) {
  const SysDesc& s = d[blockIdx.y];
  if ((int)(blockIdx.x * (blockDim.x / WAVE)) >= s.natoms) return;
  combine_dev(s.xdiag, s.part, s.nparts, s.part_stride, s.w0, s.w1, s.wsum, s.t, s.nb, s.np, s.offsets, s.natoms, s.q1,
              &s.kst->stop, blockIdx.x, 0);
}

// f~_k = -(q1 - v_k) (K0 = -I)
__global__ void b_precond(const SysDesc* __restrict__ d, int k) {
  const SysDesc& s = d[blockIdx.y];
  if (s.kst->stop) return;
  const int n2 = 2 * s.natoms;
  const double* v = s.V + (size_t)k * n2;
  double* out = s.Ft + (size_t)k * n2;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += gridDim.x * blockDim.x)
    out[i] = -(s.q1[i] - v[i]);
}

__global__ void __launch_bounds__(1024) b_solve(SysDesc* d, double* const* out) {
  const SysDesc& s = d[blockIdx.x];
  solve_dev(s.V, s.Ft, s.ftilde, 2 * s.natoms, s.kst, out[blockIdx.x], 0.0);
}

__global__ void b_info(const SysDesc* __restrict__ d, int ns, KrylovState* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) out[i] = *d[i].kst;
}

// Persistent transforms: each workgroup takes tiles t = blockIdx.x, + gridDim.x, ...
// from a list sorted by decreasing cost; a tile of a system whose Krylov
// expansion has stopped is skipped (uniformly for the workgroup).
// Held to MIN_BLOCKS workgroups per CU: the two-half forward form with the Fermi
// epilogue, which this kernel ran before the full-tile forward, took ~164 registers per
// lane and one workgroup per CU when left to itself (13 % slower); the full-tile
// product and the back-transform fit without spilling.
template <int EPI, class Cfg>
__global__ __launch_bounds__(Cfg::THREADS) __attribute__((amdgpu_waves_per_eu(Cfg::WAVES_PER_EU))) void b_gemm_f64(const BatchItemF64* __restrict__ items,
                                                                          const int4* __restrict__ tiles,
                                                                          int ntiles, int two_halves) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int4 tl = tiles[t];
    const BatchItemF64& it = items[tl.x];
    if (*it.stop) continue;
    f64_tile<EPI, Cfg>(it.g, it.n, it.k, two_halves != 0, make_int2(tl.y, tl.z), it.beta);
  }
}

// Held to MIN_BLOCKS workgroups per CU as well (the two-half forward form with a staged
// mirror epilogue, which this kernel ran before the full-tile forward, took ~190 registers
// and one workgroup per CU when left to itself, 4 % slower). The split products have one K
// half, so the last argument (kept for one launcher of both precisions) must be 0.
template <int EPI, class Cfg>
__global__ __launch_bounds__(Cfg::THREADS) __attribute__((amdgpu_waves_per_eu((Cfg::MIN_BLOCKS * Cfg::THREADS / 64 + 3) / 4)))
void b_gemm_mixed(const BatchItemMixed* __restrict__ items, const int4* __restrict__ tiles, int ntiles,
                  int /*two_halves*/) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int4 tl = tiles[t];
    const BatchItemMixed& it = items[tl.x];
    if (*it.stop) continue;
    mixed_tile<EPI, Cfg>(it.g, it.n, it.k, make_int2(tl.y, tl.z));
  }
}

}  // namespace kk
