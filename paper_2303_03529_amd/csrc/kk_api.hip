// C ABI of the spin-charge Krylov kernel library (declared in include/krylov_kernel.h).
//
// Data layout in device memory (np = Nb rounded up to the 128 tile, zero padded):
//   per spin s: C_s = Z Q_s, CT_s = C_s^T, G_s = S C_s    (np x np each, row-major)
//               eps_s, f_s, fc_s = 1 - f_s, w_s = beta f fc   (np each)
//               t_s[I] = sum_{i in I} sum_k C_ik w_k G_ik     (response to a unit mu shift)
//   S (np x np) for mulliken_project, gamma (N x N), atom offsets (N+1).
// Per response item (direction b, spin s): u~ (np), Y (np x np), diag X (np),
// Mulliken partial row sums (one row of np per wave column of each tile column).
//
// One response (Sec. II.G directional derivative) is four launches per batch:
//   potentials -> gemm<FERMI> (X = 1/2(C^T U~ G + G^T U~ C), Y = F o X) ->
//   gemm<MULLIKEN> (P = C Y, rows dotted with G) -> combine (mu shift, per-atom
//   sums, charge/spin mix). The mu shift enters only through t_s, because
//   C diag(w) C^T S has fixed Mulliken populations.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "krylov_kernel.h"
#include "kk_gemm.hpp"
#include "kk_kernels.hpp"
#include "kk_gemm_mixed.hpp"

namespace {

thread_local std::string g_err;

kk_status fail(kk_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_OR_FAIL(expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(KK_EHIP, "%s: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

#define LAUNCH_CHECK(what)                                                                 \
  do {                                                                                     \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess) return fail(KK_EHIP, "launch %s: %s", what, hipGetErrorString(e_)); \
  } while (0)

constexpr int MAX_CHUNK = kk::MAX_GEMM_BATCH / 2;  // directions per GEMM launch
constexpr size_t WORKSPACE_BUDGET = size_t(12) << 30;  // bytes of Y workspace per handle
constexpr int MAX_EVENTS = 8192;

}  // namespace

struct kk_handle_s {
  hipStream_t stream = nullptr;
  bool prepared = false;
  int natoms = 0, nb = 0, np = 0, nparts = 0;
  double W = 0, kT = 0, beta = 0, n_e = 0;
  std::vector<void*> owned;  // every device allocation of the prepared state

  double *S = nullptr, *gamma = nullptr;
  double *C[2] = {nullptr, nullptr}, *CT[2] = {nullptr, nullptr}, *G[2] = {nullptr, nullptr};
  double *eps[2] = {nullptr, nullptr}, *f[2] = {nullptr, nullptr}, *fc[2] = {nullptr, nullptr},
         *w[2] = {nullptr, nullptr};
  double *t = nullptr, *mu = nullptr, *wsum = nullptr;
  int* offsets = nullptr;
  int2 *tiles_upper = nullptr, *tiles_full = nullptr, *tiles_store = nullptr;
  int n_upper = 0, n_full = 0, n_store = 0;

  // split-precision state (precision == KK_MIXED_F16)
  int precision = KK_FP64;
  double* GT[2] = {nullptr, nullptr};
  _Float16 *Ch[2] = {nullptr, nullptr}, *Cl[2] = {nullptr, nullptr};
  _Float16 *CTh[2] = {nullptr, nullptr}, *CTl[2] = {nullptr, nullptr};
  _Float16 *GTh[2] = {nullptr, nullptr}, *GTl[2] = {nullptr, nullptr};
  double* mconst = nullptr;  // per spin: s_C, s_G, max column norms of C and G
  int2 *mtiles_upper = nullptr, *mtiles_full = nullptr;
  int n_mupper = 0, n_mfull = 0;
  _Float16 *uct_h = nullptr, *uct_l = nullptr, *ugt_h = nullptr, *ugt_l = nullptr;
  _Float16 *yh = nullptr, *yl = nullptr;
  double* msc = nullptr;
  double* mscratch = nullptr;  // 4 np doubles: row statistics for the split scales

  // response workspace (grown on demand)
  int chunk_cap = 0;
  double *u = nullptr, *Y = nullptr, *xdiag = nullptr, *part = nullptr;
  // Krylov workspace
  double *V = nullptr, *Ft = nullptr, *ftilde = nullptr, *q1 = nullptr;
  kk::KrylovState* kst = nullptr;

  // kernel timing
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<int, int>>> ev_used;  // (kernel id, (start ev, end ev))
  int ev_next = 0;

  std::vector<void*> ws_owned;  // response workspace, replaced when it grows

  void free_workspace() {
    for (void* p : ws_owned) (void)hipFree(p);
    ws_owned.clear();
    chunk_cap = 0;
    u = Y = xdiag = part = nullptr;
    uct_h = uct_l = ugt_h = ugt_l = yh = yl = nullptr;
    msc = nullptr;
  }

  void release() {
    if (owned.empty() && ws_owned.empty()) {
      prepared = false;
      return;
    }
    (void)hipStreamSynchronize(stream);
    free_workspace();
    for (void* p : owned) (void)hipFree(p);
    owned.clear();
    prepared = false;
    V = Ft = ftilde = q1 = nullptr;
    kst = nullptr;
  }
};

namespace {

kk_status dalloc(std::vector<void*>& owner, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(KK_ENOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  }
  owner.push_back(*p);
  return KK_OK;
}

template <typename T>
kk_status dalloc_t(kk_handle h, T** p, size_t count, bool workspace = false) {
  void* q = nullptr;
  kk_status st = dalloc(workspace ? h->ws_owned : h->owned, &q, count * sizeof(T));
  *p = static_cast<T*>(q);
  return st;
}

// Zero device memory with a plain kernel (no memset nodes if a caller captures).
__global__ void zero_fill(double* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

kk_status zero(kk_handle h, double* p, size_t n) {
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
  zero_fill<<<std::max(blocks, 1), 256, 0, h->stream>>>(p, n);
  LAUNCH_CHECK("zero_fill");
  return KK_OK;
}

// Tile orders. Full grid: groups of 8 tile rows, sweep columns inside a group,
// so the tiles resident on one XCD share A and B panels. Upper: the same
// order restricted to tiles holding at least one element with m <= n.
std::vector<int2> tile_order(int np, int bm, int bn, bool upper) {
  std::vector<int2> v;
  const int TM = np / bm, TN = np / bn;
  const int GROUP = 8;
  for (int g0 = 0; g0 < TM; g0 += GROUP)
    for (int tn = 0; tn < TN; ++tn)
      for (int tm = g0; tm < std::min(TM, g0 + GROUP); ++tm)
        if (!upper || tm * bm <= tn * bn + bn - 1) v.push_back(make_int2(tm, tn));
  return v;
}

struct ProfileScope {
  kk_handle h;
  int id;
  int ev0 = -1;
  ProfileScope(kk_handle hh, int kid) : h(hh), id(kid) {
    if (h->profiling && h->ev_next + 2 <= (int)h->ev_pool.size()) {
      ev0 = h->ev_next;
      h->ev_next += 2;
      (void)hipEventRecord(h->ev_pool[ev0], h->stream);
    }
  }
  ~ProfileScope() {
    if (ev0 >= 0) {
      (void)hipEventRecord(h->ev_pool[ev0 + 1], h->stream);
      h->ev_used.push_back({id, {ev0, ev0 + 1}});
    }
  }
};

kk_status launch_gemm(kk_handle h, int epi, kk::GemmArgs& a) {
  const int grid = a.ntiles * a.nitems;
  if (grid <= 0) return KK_OK;
  if (a.nitems > kk::MAX_GEMM_BATCH) return fail(KK_EINVAL, "internal: too many GEMM items");
  if (epi == kk::EPI_STORE) {
    kk::gemm_f64<kk::EPI_STORE, kk::StoreCfg><<<grid, kk::StoreCfg::THREADS, 0, h->stream>>>(a);
  } else if (epi == kk::EPI_FERMI) {
    ProfileScope ps(h, 0);
    kk::gemm_f64<kk::EPI_FERMI, kk::FwdCfg><<<grid, kk::FwdCfg::THREADS, 0, h->stream>>>(a);
  } else {
    ProfileScope ps(h, 1);
    kk::gemm_f64<kk::EPI_MULLIKEN, kk::BackCfg><<<grid, kk::BackCfg::THREADS, 0, h->stream>>>(a);
  }
  LAUNCH_CHECK("gemm_f64");
  return KK_OK;
}

kk_status ensure_workspace(kk_handle h, int chunk) {
  if (chunk <= h->chunk_cap) return KK_OK;
  const size_t np = h->np, items = (size_t)2 * chunk;
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  h->free_workspace();
  kk_status st;
  if ((st = dalloc_t(h, &h->u, items * np, true))) return st;
  if (h->precision == KK_FP64) {
    if ((st = dalloc_t(h, &h->Y, items * np * np, true))) return st;
  } else {
    for (_Float16** q : {&h->uct_h, &h->uct_l, &h->ugt_h, &h->ugt_l, &h->yh, &h->yl})
      if ((st = dalloc_t(h, q, items * np * np, true))) return st;
    if ((st = dalloc_t(h, &h->msc, items * 8, true))) return st;
  }
  if ((st = dalloc_t(h, &h->xdiag, items * np, true))) return st;
  if ((st = dalloc_t(h, &h->part, items * h->nparts * np, true))) return st;
  if ((st = zero(h, h->u, items * np))) return st;
  h->chunk_cap = chunk;
  return KK_OK;
}

int max_chunk(kk_handle h) {
  // FP64: one Y per spin; split path: six FP16 matrices per spin
  const size_t per_dir = (size_t)2 * h->np * h->np * (h->precision == KK_FP64 ? sizeof(double) : 6 * sizeof(_Float16));
  size_t c = WORKSPACE_BUDGET / std::max<size_t>(per_dir, 1);
  return (int)std::max<size_t>(1, std::min<size_t>(c, MAX_CHUNK));
}

// Responses of `batch` directions v (batch x 2N) into q1 (batch x 2N); batch <= chunk_cap.
kk_status response_chunk(kk_handle h, int batch, const double* v, double* q1, const int* stop) {
  const int N = h->natoms, np = h->np;
  {
    const int waves = N * batch, threads = 256;
    const int blocks = (waves * kk::WAVE + threads - 1) / threads;
    kk::potentials<<<blocks, threads, 0, h->stream>>>(h->gamma, N, h->W, v, batch, h->offsets, np,
                                                       h->u, stop);
    LAUNCH_CHECK("potentials");
  }
  kk::GemmArgs fa{};
  fa.n = np; fa.k_half = np; fa.two_halves = 1; fa.ntiles = h->n_upper; fa.nitems = 2 * batch;
  fa.tiles = h->tiles_upper; fa.stop = stop; fa.beta = h->beta;
  kk::GemmArgs ba{};
  ba.n = np; ba.k_half = np; ba.two_halves = 0; ba.ntiles = h->n_full; ba.nitems = 2 * batch;
  ba.tiles = h->tiles_full; ba.stop = stop; ba.beta = h->beta;
  for (int b = 0; b < batch; ++b)
    for (int s = 0; s < 2; ++s) {
      const int z = 2 * b + s;
      double* Yz = h->Y + (size_t)z * np * np;
      kk::GemmItem& fi = fa.item[z];
      fi.a0 = h->C[s]; fi.b0 = h->G[s]; fi.a1 = h->G[s]; fi.b1 = h->C[s];
      fi.scale = h->u + (size_t)z * np; fi.out = Yz;
      fi.eps = h->eps[s]; fi.f = h->f[s]; fi.fc = h->fc[s]; fi.w = h->w[s];
      fi.xdiag = h->xdiag + (size_t)z * np;
      kk::GemmItem& bi = ba.item[z];
      bi.a0 = h->CT[s]; bi.b0 = Yz; bi.g = h->G[s];
      bi.part = h->part + (size_t)z * h->nparts * np;
    }
  kk_status st;
  if ((st = launch_gemm(h, kk::EPI_FERMI, fa))) return st;
  if ((st = launch_gemm(h, kk::EPI_MULLIKEN, ba))) return st;
  {
    const int threads = 256;
    dim3 grid((N + threads - 1) / threads, batch);
    kk::combine<<<grid, threads, 0, h->stream>>>(h->xdiag, h->part, h->nparts, h->w[0], h->w[1],
                                                  h->wsum, h->t, h->nb, np, h->offsets, N, q1, stop);
    LAUNCH_CHECK("combine");
  }
  return KK_OK;
}

kk_status launch_mixed(kk_handle h, int epi, kk::MixedArgs& a) {
  const int grid = a.ntiles * a.nitems;
  if (grid <= 0) return KK_OK;
  if (a.nitems > kk::MAX_GEMM_BATCH) return fail(KK_EINVAL, "internal: too many GEMM items");
  if (epi == kk::EPI_FERMI) {
    ProfileScope ps(h, 0);
    kk::gemm_mixed<kk::EPI_FERMI, kk::MFwdCfg><<<grid, kk::MFwdCfg::THREADS, 0, h->stream>>>(a);
  } else {
    ProfileScope ps(h, 1);
    kk::gemm_mixed<kk::EPI_MULLIKEN, kk::MBackCfg><<<grid, kk::MBackCfg::THREADS, 0, h->stream>>>(a);
  }
  LAUNCH_CHECK("gemm_mixed");
  return KK_OK;
}

// Split-precision responses: same steps as response_chunk, with the two
// transforms on FP16 x 3 MFMA products (Y kept as an FP16 split).
kk_status response_chunk_mixed(kk_handle h, int batch, const double* v, double* q1, const int* stop) {
  const int N = h->natoms, np = h->np;
  const size_t np2 = (size_t)np * np;
  {
    const int waves = N * batch, threads = 256;
    const int blocks = (waves * kk::WAVE + threads - 1) / threads;
    kk::potentials<<<blocks, threads, 0, h->stream>>>(h->gamma, N, h->W, v, batch, h->offsets, np,
                                                       h->u, stop);
    LAUNCH_CHECK("potentials");
  }
  kk::mixed_scales<<<2 * batch, 1024, 0, h->stream>>>(h->u, np, h->mconst, h->beta, h->msc, stop);
  LAUNCH_CHECK("mixed_scales");
  for (int z = 0; z < 2 * batch; ++z) {
    const int s = z & 1;
    const int blocks = (int)std::min<size_t>((np2 + 255) / 256, 16384);
    kk::split_scaled_columns<<<blocks, 256, 0, h->stream>>>(h->CT[s], np, h->u + (size_t)z * np,
                                                             h->msc + z * 8 + 3, h->uct_h + z * np2,
                                                             h->uct_l + z * np2, stop);
    LAUNCH_CHECK("split_scaled_columns");
    kk::split_scaled_columns<<<blocks, 256, 0, h->stream>>>(h->GT[s], np, h->u + (size_t)z * np,
                                                             h->msc + z * 8 + 4, h->ugt_h + z * np2,
                                                             h->ugt_l + z * np2, stop);
    LAUNCH_CHECK("split_scaled_columns");
  }
  kk::MixedArgs fa{};
  fa.n = np; fa.k_half = np; fa.two_halves = 1; fa.ntiles = h->n_mupper; fa.nitems = 2 * batch;
  fa.tiles = h->mtiles_upper; fa.stop = stop; fa.beta = h->beta;
  kk::MixedArgs ba{};
  ba.n = np; ba.k_half = np; ba.two_halves = 0; ba.ntiles = h->n_mfull; ba.nitems = 2 * batch;
  ba.tiles = h->mtiles_full; ba.stop = stop; ba.beta = h->beta;
  for (int z = 0; z < 2 * batch; ++z) {
    const int s = z & 1;
    kk::MixedItem& fi = fa.item[z];
    fi.a0h = h->uct_h + z * np2; fi.a0l = h->uct_l + z * np2; fi.b0h = h->GTh[s]; fi.b0l = h->GTl[s];
    fi.a1h = h->ugt_h + z * np2; fi.a1l = h->ugt_l + z * np2; fi.b1h = h->CTh[s]; fi.b1l = h->CTl[s];
    fi.yh = h->yh + z * np2; fi.yl = h->yl + z * np2;
    fi.eps = h->eps[s]; fi.f = h->f[s]; fi.fc = h->fc[s]; fi.w = h->w[s];
    fi.xdiag = h->xdiag + (size_t)z * np;
    fi.sc = h->msc + z * 8;
    kk::MixedItem& bi = ba.item[z];
    bi.a0h = h->Ch[s]; bi.a0l = h->Cl[s]; bi.b0h = h->yh + z * np2; bi.b0l = h->yl + z * np2;
    bi.g = h->G[s];
    bi.part = h->part + (size_t)z * h->nparts * np;
    bi.sc = h->msc + z * 8 + 2;
  }
  kk_status st;
  if ((st = launch_mixed(h, kk::EPI_FERMI, fa))) return st;
  if ((st = launch_mixed(h, kk::EPI_MULLIKEN, ba))) return st;
  {
    const int threads = 256;
    dim3 grid((N + threads - 1) / threads, batch);
    kk::combine<<<grid, threads, 0, h->stream>>>(h->xdiag, h->part, h->nparts, h->w[0], h->w[1],
                                                  h->wsum, h->t, h->nb, np, h->offsets, N, q1, stop);
    LAUNCH_CHECK("combine");
  }
  return KK_OK;
}

kk_status response_any(kk_handle h, int batch, const double* v, double* q1, const int* stop) {
  return h->precision == KK_FP64 ? response_chunk(h, batch, v, q1, stop)
                                 : response_chunk_mixed(h, batch, v, q1, stop);
}

kk_status check_handle(kk_handle h) {
  if (!h) return fail(KK_EINVAL, "handle is NULL");
  if (!h->prepared) return fail(KK_ENOTPREPARED, "kk_prepare has not succeeded on this handle");
  return KK_OK;
}

// Every device buffer of a prepared handle for its (natoms, np, precision),
// plus the tile tables (which depend only on np).
kk_status allocate_prepared(kk_handle h) {
  const int np = h->np, n_atoms = h->natoms;
  const size_t np2 = (size_t)np * np;
  kk_status st;
  if ((st = dalloc_t(h, &h->S, np2))) return st;
  for (int s = 0; s < 2; ++s) {
    if ((st = dalloc_t(h, &h->C[s], np2))) return st;
    if ((st = dalloc_t(h, &h->CT[s], np2))) return st;
    if ((st = dalloc_t(h, &h->G[s], np2))) return st;
    if ((st = dalloc_t(h, &h->eps[s], np))) return st;
    if ((st = dalloc_t(h, &h->f[s], np))) return st;
    if ((st = dalloc_t(h, &h->fc[s], np))) return st;
    if ((st = dalloc_t(h, &h->w[s], np))) return st;
  }
  if ((st = dalloc_t(h, &h->gamma, (size_t)n_atoms * n_atoms))) return st;
  if ((st = dalloc_t(h, &h->t, (size_t)2 * n_atoms))) return st;
  if ((st = dalloc_t(h, &h->mu, 1))) return st;
  if ((st = dalloc_t(h, &h->wsum, 1))) return st;
  if ((st = dalloc_t(h, &h->offsets, (size_t)n_atoms + 1))) return st;
  std::vector<int2> up = tile_order(np, kk::FwdCfg::BM, kk::FwdCfg::BN, true);
  std::vector<int2> full = tile_order(np, kk::BackCfg::BM, kk::BackCfg::BN, false);
  std::vector<int2> stt = tile_order(np, kk::StoreCfg::BM, kk::StoreCfg::BN, false);
  h->n_upper = (int)up.size();
  h->n_full = (int)full.size();
  h->n_store = (int)stt.size();
  if ((st = dalloc_t(h, &h->tiles_upper, up.size()))) return st;
  if ((st = dalloc_t(h, &h->tiles_full, full.size()))) return st;
  if ((st = dalloc_t(h, &h->tiles_store, stt.size()))) return st;
  const int n2 = 2 * n_atoms;
  if ((st = dalloc_t(h, &h->V, (size_t)kk::MAX_RANK * n2))) return st;
  if ((st = dalloc_t(h, &h->Ft, (size_t)kk::MAX_RANK * n2))) return st;
  if ((st = dalloc_t(h, &h->ftilde, (size_t)n2))) return st;
  if ((st = dalloc_t(h, &h->q1, (size_t)n2))) return st;
  if ((st = dalloc_t(h, &h->kst, 1))) return st;
  HIP_OR_FAIL(hipMemcpyAsync(h->tiles_upper, up.data(), sizeof(int2) * up.size(), hipMemcpyHostToDevice,
                             h->stream));
  HIP_OR_FAIL(hipMemcpyAsync(h->tiles_full, full.data(), sizeof(int2) * full.size(), hipMemcpyHostToDevice,
                             h->stream));
  HIP_OR_FAIL(hipMemcpyAsync(h->tiles_store, stt.data(), sizeof(int2) * stt.size(), hipMemcpyHostToDevice,
                             h->stream));
  if (h->precision == KK_MIXED_F16) {
    if ((st = dalloc_t(h, &h->mconst, 8))) return st;
    if ((st = dalloc_t(h, &h->mscratch, (size_t)4 * np))) return st;
    for (int s = 0; s < 2; ++s) {
      if ((st = dalloc_t(h, &h->GT[s], np2))) return st;
      for (_Float16** q : {&h->Ch[s], &h->Cl[s], &h->CTh[s], &h->CTl[s], &h->GTh[s], &h->GTl[s]})
        if ((st = dalloc_t(h, q, np2))) return st;
    }
    std::vector<int2> mup = tile_order(np, kk::MFwdCfg::BM, kk::MFwdCfg::BN, true);
    std::vector<int2> mfull = tile_order(np, kk::MBackCfg::BM, kk::MBackCfg::BN, false);
    h->n_mupper = (int)mup.size();
    h->n_mfull = (int)mfull.size();
    if ((st = dalloc_t(h, &h->mtiles_upper, mup.size()))) return st;
    if ((st = dalloc_t(h, &h->mtiles_full, mfull.size()))) return st;
    HIP_OR_FAIL(hipMemcpyAsync(h->mtiles_upper, mup.data(), sizeof(int2) * mup.size(), hipMemcpyHostToDevice,
                               h->stream));
    HIP_OR_FAIL(hipMemcpyAsync(h->mtiles_full, mfull.data(), sizeof(int2) * mfull.size(),
                               hipMemcpyHostToDevice, h->stream));
  }
  // the host tile vectors must outlive the copies
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  return KK_OK;
}

// Split-precision operands, once per prepared expansion point: G^T (FP64) and
// the FP16 splits of C, C^T, G^T with their power-of-two scales.
kk_status prepare_mixed(kk_handle h) {
  const int np = h->np;
  double* rmax = h->mscratch;
  double* rn2 = rmax + 2 * np;
  for (int s = 0; s < 2; ++s) {
    dim3 pg(np / 32, np / 32), pb(256);
    kk::transpose_sq<<<pg, pb, 0, h->stream>>>(h->G[s], h->GT[s], np);
    LAUNCH_CHECK("transpose G");
    // rows of C^T are columns of C; rows of G^T columns of G
    kk::row_stats<<<np, 1024, 0, h->stream>>>(h->CT[s], np, rmax, rn2);
    LAUNCH_CHECK("row_stats");
    kk::row_stats<<<np, 1024, 0, h->stream>>>(h->GT[s], np, rmax + np, rn2 + np);
    LAUNCH_CHECK("row_stats");
    kk::const_scales<<<1, 1024, 0, h->stream>>>(rmax, rn2, rmax + np, rn2 + np, np, h->mconst + 4 * s);
    LAUNCH_CHECK("const_scales");
    kk::split_matrix<<<pg, pb, 0, h->stream>>>(h->C[s], np, 0, h->mconst + 4 * s, h->Ch[s], h->Cl[s]);
    kk::split_matrix<<<pg, pb, 0, h->stream>>>(h->CT[s], np, 0, h->mconst + 4 * s, h->CTh[s], h->CTl[s]);
    kk::split_matrix<<<pg, pb, 0, h->stream>>>(h->GT[s], np, 0, h->mconst + 4 * s + 1, h->GTh[s], h->GTl[s]);
    LAUNCH_CHECK("split_matrix");
  }
  return KK_OK;
}

}  // namespace

extern "C" {

const char* kk_last_error(void) { return g_err.c_str(); }

kk_status kk_create(kk_handle* h, void* hip_stream) {
  if (!h) return fail(KK_EINVAL, "kk_create: output pointer is NULL");
  *h = new (std::nothrow) kk_handle_s();
  if (!*h) return fail(KK_ENOMEM, "kk_create: out of host memory");
  (*h)->stream = static_cast<hipStream_t>(hip_stream);
  g_err.clear();
  return KK_OK;
}

kk_status kk_destroy(kk_handle h) {
  if (!h) return fail(KK_EINVAL, "kk_destroy: handle is NULL");
  h->release();
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  delete h;
  return KK_OK;
}

kk_status kk_prepare(kk_handle h, int n_atoms, const int* atom_offsets, int n_basis, const double* S,
                     const double* Z, const double* Q_up, const double* Q_dn, const double* eps_up,
                     const double* eps_dn, const double* gamma, double W, double kT,
                     double n_electrons, int precision) {
  if (!h) return fail(KK_EINVAL, "kk_prepare: handle is NULL");
  if (n_atoms < 1 || n_basis < 1) return fail(KK_EINVAL, "kk_prepare: n_atoms and n_basis must be >= 1");
  if (2 * n_atoms > 8 * 1024) return fail(KK_EINVAL, "kk_prepare: at most 4096 atoms are supported");
  if (!atom_offsets || !S || !Z || !Q_up || !Q_dn || !eps_up || !eps_dn || !gamma)
    return fail(KK_EINVAL, "kk_prepare: NULL array argument");
  if (!(kT > 0.0)) return fail(KK_EINVAL, "kk_prepare: kT must be > 0");
  if (!(n_electrons > 0.0 && n_electrons < 2.0 * n_basis))
    return fail(KK_EINVAL, "kk_prepare: need 0 < n_electrons < 2 n_basis");
  if (precision != KK_FP64 && precision != KK_MIXED_F16)
    return fail(KK_EINVAL, "kk_prepare: unsupported precision %d", precision);
  if (atom_offsets[0] != 0 || atom_offsets[n_atoms] != n_basis)
    return fail(KK_EINVAL, "kk_prepare: atom_offsets must start at 0 and end at n_basis");
  for (int a = 0; a < n_atoms; ++a)
    if (atom_offsets[a + 1] <= atom_offsets[a])
      return fail(KK_EINVAL, "kk_prepare: atom_offsets must be strictly increasing (atom %d)", a);

  const bool mixed = precision == KK_MIXED_F16;
  const int pad = mixed ? kk::MIXED_PAD : kk::PAD;
  const int nb = n_basis, np = (nb + pad - 1) / pad * pad;
  // Re-preparing the same shape (an SCF or MD loop) reuses every buffer.
  const bool reuse = h->prepared && h->natoms == n_atoms && h->nb == nb && h->precision == precision;
  h->prepared = false;
  kk_status st;
  if (!reuse) {
    h->release();
    h->precision = precision;
    h->natoms = n_atoms; h->nb = nb; h->np = np;
    h->nparts = mixed ? (np / kk::MBackCfg::BN) * kk::MBackCfg::WAVES_N
                      : (np / kk::BackCfg::BN) * kk::BackCfg::WAVES_N;
    if ((st = allocate_prepared(h))) return st;
  }
  h->W = W; h->kT = kT; h->beta = 1.0 / kT; h->n_e = n_electrons;
  HIP_OR_FAIL(hipMemcpyAsync(h->offsets, atom_offsets, sizeof(int) * (n_atoms + 1), hipMemcpyHostToDevice,
                             h->stream));
  HIP_OR_FAIL(hipMemcpyAsync(h->gamma, gamma, sizeof(double) * n_atoms * n_atoms, hipMemcpyDeviceToDevice,
                             h->stream));

  // Padded copies: S, Z^T (into CT[0]) and Q_s (into CT[1] as scratch), then
  // C_s = Z Q_s, G_s = S C_s, CT_s = C_s^T.
  dim3 pg(np / 32, np / 32), pb(256);
  kk::pad_copy<<<pg, pb, 0, h->stream>>>(S, nb, h->S, np, 0);
  LAUNCH_CHECK("pad_copy S");
  kk::pad_copy<<<pg, pb, 0, h->stream>>>(Z, nb, h->G[0], np, 1);  // G[0] holds Z^T for now
  LAUNCH_CHECK("pad_copy Z");
  const double* Qs[2] = {Q_up, Q_dn};
  for (int s = 0; s < 2; ++s) {
    kk::pad_copy<<<pg, pb, 0, h->stream>>>(Qs[s], nb, h->CT[s], np, 0);
    LAUNCH_CHECK("pad_copy Q");
  }
  kk::GemmArgs a{};
  a.n = np; a.k_half = np; a.two_halves = 0; a.ntiles = h->n_store; a.tiles = h->tiles_store;
  a.stop = nullptr; a.nitems = 2;
  for (int s = 0; s < 2; ++s) {  // C_s[m][n] = sum_k Z^T[k][m] Q_s[k][n]
    a.item[s] = kk::GemmItem{};
    a.item[s].a0 = h->G[0]; a.item[s].b0 = h->CT[s]; a.item[s].out = h->C[s];
  }
  if ((st = launch_gemm(h, kk::EPI_STORE, a))) return st;
  for (int s = 0; s < 2; ++s) {  // G_s[m][n] = sum_k S[k][m] C_s[k][n] (S symmetric)
    a.item[s] = kk::GemmItem{};
    a.item[s].a0 = h->S; a.item[s].b0 = h->C[s]; a.item[s].out = h->G[s];
  }
  if ((st = launch_gemm(h, kk::EPI_STORE, a))) return st;
  for (int s = 0; s < 2; ++s) {
    kk::transpose_sq<<<pg, pb, 0, h->stream>>>(h->C[s], h->CT[s], np);
    LAUNCH_CHECK("transpose C");
  }
  // chemical potential and occupations (eps copied into padded arrays)
  kk::solve_mu<<<1, 1024, 0, h->stream>>>(eps_up, eps_dn, nb, n_electrons, h->beta, h->mu);
  LAUNCH_CHECK("solve_mu");
  const double* es[2] = {eps_up, eps_dn};
  for (int s = 0; s < 2; ++s) {
    kk::occupations<<<(np + 255) / 256, 256, 0, h->stream>>>(es[s], nb, np, h->mu, h->beta, h->eps[s],
                                                              h->f[s], h->fc[s], h->w[s]);
    LAUNCH_CHECK("occupations");
  }
  kk::sum_two<<<1, 1024, 0, h->stream>>>(h->w[0], h->w[1], np, h->wsum);
  LAUNCH_CHECK("sum_two");
  kk::atom_row_dots<<<n_atoms, 256, 0, h->stream>>>(h->C[0], h->C[1], np, h->G[0], h->G[1], np, h->w[0],
                                                     h->w[1], np, h->offsets, n_atoms, h->t);
  LAUNCH_CHECK("atom_row_dots");
  if (mixed && (st = prepare_mixed(h))) return st;
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  h->prepared = true;
  g_err.clear();
  return KK_OK;
}

kk_status kk_get_mu(kk_handle h, double* mu) {
  kk_status st = check_handle(h);
  if (st) return st;
  if (!mu) return fail(KK_EINVAL, "kk_get_mu: output is NULL");
  HIP_OR_FAIL(hipMemcpyAsync(mu, h->mu, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  return KK_OK;
}

kk_status density_response_batch(kk_handle h, int batch, const double* v, double* q1) {
  kk_status st = check_handle(h);
  if (st) return st;
  if (batch < 1) return fail(KK_EINVAL, "density_response_batch: batch must be >= 1");
  if (!v || !q1) return fail(KK_EINVAL, "density_response_batch: NULL array argument");
  const int chunk = std::min(batch, max_chunk(h));
  if ((st = ensure_workspace(h, chunk))) return st;
  const size_t n2 = 2 * (size_t)h->natoms;
  for (int b0 = 0; b0 < batch; b0 += chunk) {
    const int nbat = std::min(chunk, batch - b0);
    if ((st = response_any(h, nbat, v + b0 * n2, q1 + b0 * n2, nullptr))) return st;
  }
  g_err.clear();
  return KK_OK;
}

kk_status mulliken_project(kk_handle h, int batch, const double* dD_up, const double* dD_dn, double* dqm) {
  kk_status st = check_handle(h);
  if (st) return st;
  if (batch < 1) return fail(KK_EINVAL, "mulliken_project: batch must be >= 1");
  if (!dD_up || !dD_dn || !dqm) return fail(KK_EINVAL, "mulliken_project: NULL array argument");
  dim3 grid(h->natoms, batch);
  kk::mulliken_rows<<<grid, 256, 0, h->stream>>>(dD_up, dD_dn, h->nb, h->S, h->np, h->offsets, h->natoms,
                                                  dqm);
  LAUNCH_CHECK("mulliken_rows");
  g_err.clear();
  return KK_OK;
}

}  // extern "C"

namespace {

kk_status krylov_run(kk_handle h, const char* who, const double* delta, int m, double tol, const double* K0,
                     double* Kdelta, kk_info* info) {
  kk_status st = check_handle(h);
  if (st) return st;
  const int n2 = 2 * h->natoms;
  if (!delta || !Kdelta) return fail(KK_EINVAL, "%s: NULL array argument", who);
  if (m < 1 || m > std::min(n2, kk::MAX_RANK))
    return fail(KK_EINVAL, "%s: need 1 <= m <= min(2N, %d), got %d", who, kk::MAX_RANK, m);
  if (!(tol >= 0.0)) return fail(KK_EINVAL, "%s: tolerance must be >= 0", who);
  if ((st = ensure_workspace(h, 1))) return st;
  const int* stop = &h->kst->stop;
  const int gv_threads = 256, gv_blocks = (n2 * kk::WAVE + gv_threads - 1) / gv_threads;

  kk::krylov_reset<<<1, 64, 0, h->stream>>>(h->kst);
  LAUNCH_CHECK("krylov_reset");
  kk::precondition<<<gv_blocks, gv_threads, 0, h->stream>>>(K0, delta, nullptr, h->ftilde, n2, nullptr);
  LAUNCH_CHECK("precondition");
  for (int k = 0; k < m; ++k) {
    const double* src = (k == 0) ? h->ftilde : h->Ft + (size_t)(k - 1) * n2;
    kk::krylov_orthonormalize<<<1, 1024, 0, h->stream>>>(src, h->V, n2, h->kst);
    LAUNCH_CHECK("krylov_orthonormalize");
    const double* vk = h->V + (size_t)k * n2;
    if ((st = response_any(h, 1, vk, h->q1, stop))) return st;
    kk::precondition<<<gv_blocks, gv_threads, 0, h->stream>>>(K0, h->q1, vk, h->Ft + (size_t)k * n2, n2,
                                                               stop);
    LAUNCH_CHECK("precondition");
    if (tol > 0.0 && k + 1 < m) {  // residual of the rank-(k+1) solve; may end the expansion
      kk::krylov_solve<<<1, 1024, 0, h->stream>>>(h->V, h->Ft, h->ftilde, n2, h->kst, Kdelta, tol);
      LAUNCH_CHECK("krylov_solve");
    }
  }
  kk::krylov_solve<<<1, 1024, 0, h->stream>>>(h->V, h->Ft, h->ftilde, n2, h->kst, Kdelta, 0.0);
  LAUNCH_CHECK("krylov_solve");
  if (info) {
    kk::KrylovState hs;
    HIP_OR_FAIL(hipMemcpyAsync(&hs, h->kst, sizeof hs, hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    info->rank_used = hs.rank;
    info->status = hs.status;
    info->min_pivot = hs.min_pivot;
    info->max_pivot = hs.max_pivot;
    info->ls_residual = hs.ls_residual;
    g_err.clear();
    if (hs.status == KK_ESINGULAR) return fail(KK_ESINGULAR, "%s: Gram matrix not positive definite", who);
    return hs.status == 1 ? KK_BREAKDOWN : KK_OK;
  }
  g_err.clear();
  return KK_OK;
}

}  // namespace

extern "C" {

kk_status krylov_kernel_apply(kk_handle h, const double* delta, int m, const double* K0, double* Kdelta,
                              kk_info* info) {
  return krylov_run(h, "krylov_kernel_apply", delta, m, 0.0, K0, Kdelta, info);
}

kk_status krylov_kernel_apply_adaptive(kk_handle h, const double* delta, int m_max, double tol,
                                       const double* K0, double* Kdelta, kk_info* info) {
  return krylov_run(h, "krylov_kernel_apply_adaptive", delta, m_max, tol, K0, Kdelta, info);
}

kk_status kk_ground_state_charges(kk_handle h, const double* reference, double* qm) {
  kk_status st = check_handle(h);
  if (st) return st;
  if (!qm) return fail(KK_EINVAL, "kk_ground_state_charges: NULL output");
  if ((st = ensure_workspace(h, 1))) return st;
  const int N = h->natoms;
  // populations per spin into the first 2N doubles of the response scratch
  kk::atom_row_dots<<<N, 256, 0, h->stream>>>(h->C[0], h->C[1], h->np, h->G[0], h->G[1], h->np, h->f[0],
                                               h->f[1], h->np, h->offsets, N, h->q1);
  LAUNCH_CHECK("atom_row_dots");
  kk::mix_spins<<<(N + 255) / 256, 256, 0, h->stream>>>(h->q1, reference, N, qm);
  LAUNCH_CHECK("mix_spins");
  g_err.clear();
  return KK_OK;
}

kk_status kk_xlbomd_update(kk_handle h, const double* n_hist, int k_max, const double* Kf, double kappa,
                           double alpha, const double* c, double* n_new) {
  kk_status st = check_handle(h);
  if (st) return st;
  if (!n_hist || !Kf || !n_new || (k_max >= 0 && !c)) return fail(KK_EINVAL, "kk_xlbomd_update: NULL array argument");
  if (k_max < 0 || k_max > 32) return fail(KK_EINVAL, "kk_xlbomd_update: need 0 <= k_max <= 32");
  const int n2 = 2 * h->natoms;
  kk::xlbomd_update<<<(n2 + 255) / 256, 256, 0, h->stream>>>(n_hist, k_max, n2, Kf, kappa, alpha, c, n_new);
  LAUNCH_CHECK("xlbomd_update");
  g_err.clear();
  return KK_OK;
}

kk_status kk_profile_enable(kk_handle h, int enable) {
  if (!h) return fail(KK_EINVAL, "kk_profile_enable: handle is NULL");
  if (enable && h->ev_pool.empty()) {
    h->ev_pool.resize(2 * MAX_EVENTS);
    for (auto& e : h->ev_pool) HIP_OR_FAIL(hipEventCreate(&e));
  }
  h->profiling = enable != 0;
  return KK_OK;
}

kk_status kk_profile_reset(kk_handle h) {
  if (!h) return fail(KK_EINVAL, "kk_profile_reset: handle is NULL");
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  h->ev_used.clear();
  h->ev_next = 0;
  return KK_OK;
}

kk_status kk_profile_read(kk_handle h, int kernel_id, double* total_ms, int* launches) {
  if (!h) return fail(KK_EINVAL, "kk_profile_read: handle is NULL");
  if (!total_ms || !launches) return fail(KK_EINVAL, "kk_profile_read: NULL output");
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  double tot = 0.0;
  int cnt = 0;
  for (auto& u : h->ev_used) {
    if (u.first != kernel_id) continue;
    float ms = 0.f;
    HIP_OR_FAIL(hipEventElapsedTime(&ms, h->ev_pool[u.second.first], h->ev_pool[u.second.second]));
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  return KK_OK;
}

}  // extern "C"
