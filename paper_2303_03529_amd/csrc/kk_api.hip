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
#include <climits>
#include <type_traits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "krylov_kernel.h"
#include "kk_gemm.hpp"
#include "kk_kernels.hpp"
#include "kk_gemm_mixed.hpp"
#include "kk_adjoint.hpp"
#include "kk_fused.hpp"

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

// A split-precision handle also runs FP64 GEMMs on its padded size (the
// setup products and the FP64 reverse sweep), so its padding is a multiple of
// the tile sides of both kernel families. Handles with Nb above SPLIT_LARGE_NB,
// and every system of a split batch, take the large product configuration.
constexpr int SPLIT_PAD_LARGE = kk::MIXED_PAD_LARGE > kk::PAD ? kk::MIXED_PAD_LARGE : kk::PAD;
constexpr int SPLIT_PAD_SMALL = kk::MIXED_PAD_SMALL > kk::PAD ? kk::MIXED_PAD_SMALL : kk::PAD;
static_assert(SPLIT_PAD_LARGE % kk::MIXED_PAD_LARGE == 0 && SPLIT_PAD_LARGE % kk::PAD == 0 &&
                  SPLIT_PAD_SMALL % kk::MIXED_PAD_SMALL == 0 && SPLIT_PAD_SMALL % kk::PAD == 0,
              "split-precision padding must be a multiple of every tile side");
// The large shape pays for its coarser padding above this size: at 432 atoms (Nb = 3888,
// padded to 4096 against 3968) it ran 48.6 updates/s against 42.4 on the small shape, at 686
// atoms 12.9 against 11.4.
#ifndef KK_SPLIT_LARGE_NB
#define KK_SPLIT_LARGE_NB 2304
#endif
constexpr int SPLIT_LARGE_NB = KK_SPLIT_LARGE_NB;
// Small systems fill the chip better with 64 x 64 tiles (a 128-atom system has
// 45 upper 128 x 128 forward tiles per spin for 256 CUs). Up to this padded
// size the FP64 response transforms (both) use them; the reverse pass and the
// setup products keep the large tiles. On MI355X: FP64 forward 0.22 vs 0.34 ms
// and back 0.144 vs 0.169 ms at Nb = 1152, forward 1.08 vs 1.20 ms and back
// equal at Nb = 2250, 64 x 64 slower from Nb = 3888. The batch uses the same
// shapes for its small-tile class (SmallMx in the split form).
#ifndef KK_SMALL_NP_F64
#define KK_SMALL_NP_F64 2304
#endif
constexpr int SMALL_NP_F64 = KK_SMALL_NP_F64;
// ... unless the 128 x 128 tiles (one workgroup per tile and spin) fit one per CU, or fill
// their rounds of one workgroup per CU to at least LARGE_TILE_FILL. Unsplit handles, one
// process, m = 8, FP64 updates/s on 64 x 64 / 128 x 128 tiles (full-tile forward): 140 atoms (200 workgroups for 256 CUs) 297.6 /
// 324.2, 150 (242) 277.6 / 303.5, 200 (450, two rounds 88 % full) 119.6 / 131.0, 220 (512)
// 108.8 / 120.0, 250 (648, three rounds 84 %) 67.8 / 71.8 (62.5 with the upper-tile form);
// but 160 and 170 (288, 56 %) 204.9 / 165.7 and 194.2 / 156.8, 190 (392, 77 %) 142.0 / 139.0,
// 230 (578, 75 %) 84.1 / 78.5.
// Measured from a padded size of 1280 up; smaller handles are K-split (128 x 128 or, up to
// 512, 64 x 64 tiles) or run the tiny class.
constexpr double LARGE_TILE_FILL = 0.8;
constexpr int LARGE_FILL_MIN_NP = 1280;
bool f64_large_tiles_fill(int np, int cus) {
  if (np < LARGE_FILL_MIN_NP) return false;
  const int w = 2 * (np / kk::BackCfg::BM) * (np / kk::BackCfg::BN);
  const int rounds = (w + cus - 1) / cus;
  return rounds == 1 || w >= LARGE_TILE_FILL * rounds * cus;
}
using SmallF64 = kk::Cfg64x64;
// Tiny systems (padded size up to TINY_NP_F64): the same 64 x 64 tiles with a K stage of 32,
// half the stages of the latency-bound K loop (16 atoms, Nb = 144: 12.2 us per transform on
// K stages of 16).
constexpr int TINY_NP_F64 = 256;
using TinyF64 = kk::TileCfg<64, 64, 32, 2, 2, 2>;
static_assert(TinyF64::BM == SmallF64::BM && TinyF64::BN == SmallF64::BN && TinyF64::WAVES_N == SmallF64::WAVES_N,
              "the tiny class shares the small class's tile tables and partial rows");
using SmallMx = kk::MCfg64x64f8;
// Split forms of small systems (padded size up to MTINY_MAX_NP): the direct-to-LDS loop on
// 64 x 64 tiles of 4 waves (32 x 32 each), whose K-split fills the chip where the 128 x 128
// tiles leave it mostly idle (37 atoms: 216 workgroups instead of 72).
#ifndef KK_MTINY_MAX_NP
#define KK_MTINY_MAX_NP 512
#endif
constexpr int MTINY_MAX_NP = KK_MTINY_MAX_NP;
using MTinyCfg = kk::MixedDlCfg<64, 64, 2, 2, 3, 8>;
using MTinyBf6 = kk::MixedDlCfg<64, 64, 2, 2, 3, 8, true, kk::PROD_ALL6>;
static_assert(SPLIT_PAD_SMALL % MTinyCfg::BM == 0, "tiny split tiles must divide the padding");
static_assert(kk::PAD % SmallF64::BM == 0 && SPLIT_PAD_LARGE % SmallMx::BM == 0, "small tiles must divide the padding");
// Rows nb..np-1 of every operand a response transform or a setup product
// contracts over are zero (the padded copies of S, Z, Q and the potentials are
// zero there, hence C, G and Y too), so those contractions stop at nb rounded up
// to KSTEP, which every K stage divides. The reverse pass keeps the full np.
constexpr int KSTEP = 32;
static_assert(KSTEP % kk::FwdCfg::BK == 0 && KSTEP % kk::BackCfg::BK == 0 && KSTEP % kk::StoreCfg::BK == 0 &&
                  KSTEP % SmallF64::BK == 0 && KSTEP % TinyF64::BK == 0 && KSTEP % kk::MLargeCfg::BK == 0 && KSTEP % kk::MSmallCfg::BK == 0 &&
                  KSTEP % SmallMx::BK == 0 && kk::PAD % KSTEP == 0,
              "KSTEP must be a multiple of every K stage and divide the padding");
constexpr size_t WORKSPACE_BUDGET = size_t(12) << 30;  // bytes of Y workspace per handle
constexpr int MAX_EVENTS = 8192;

}  // namespace

struct kk_handle_s {
  hipStream_t stream = nullptr;
  bool prepared = false;
  int natoms = 0, nb = 0, np = 0, nparts = 0;
  int kc = 0;  // contraction length of the transforms: nb rounded up to KSTEP (<= np)
  // K-split of the response transforms (choose_ksplit): the forward in kch chunks of kck rows,
  // the back-transform in kchb (= kch), nbase Mulliken partial rows per back chunk
  // (nparts = kchb nbase)
  int kch = 1, kchb = 1, kck = 0, nbase = 0;
  // Stream-K products (split forms, small shape; choose_stream_k): kch = kchb = the slots
  // of partial results per item, sk_grid workgroups per product launch
  bool sk = false;
  int sk_grid = 0;
  bool ktiny = false;  // FP64 K-split on 64 x 64 TinyF64 tiles (small_f64 and tiny_f64 then set)
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
  // small systems: 64 x 64 tiles for the FP64 response transforms
  bool small_f64 = false;
  bool tiny_f64 = false;  // small_f64 with np <= TINY_NP_F64: TinyF64 kernels
  bool mx_large = false;  // split products on MLargeCfg (else MSmallCfg)
  bool mx_tiny = false;   // split products on MTinyCfg / MTinyBf6 (64 x 64 tiles)
  bool full_fwd = false;  // FP64 forward as full tiles + fermi_symmetrize_f64 (K-splits, 64 x 64 tiles, full_forward_pairs)
  int2 *stiles_upper = nullptr, *stiles_full = nullptr;
  int n_supper = 0, n_sfull = 0;

  // split-precision state (precision KK_MIXED_F16 or KK_MIXED_BF16; the BF16 form keeps a
  // third piece of every split operand, *r, for its refinement products)
  int precision = KK_FP64;
  bool bf16 = false;
  double* GT[2] = {nullptr, nullptr};
  _Float16 *Ch[2] = {nullptr, nullptr}, *Cl[2] = {nullptr, nullptr}, *Cr[2] = {nullptr, nullptr};
  _Float16 *GTh[2] = {nullptr, nullptr}, *GTl[2] = {nullptr, nullptr}, *GTr[2] = {nullptr, nullptr};
  double* mconst = nullptr;  // per spin: s_C, s_G, max column norms of C and G
  int2* mtiles_full = nullptr;  // both split transforms of a single system: full tiles
  int n_mfull = 0;
  _Float16 *uct_h = nullptr, *uct_l = nullptr, *uct_r = nullptr;  // (U~ C)^T split per direction
  float* x32 = nullptr;  // split forward: the product C^T U~ G per direction, FP32
  _Float16 *yh = nullptr, *yl = nullptr, *yr = nullptr;
  double* msc = nullptr;
  double* mscratch = nullptr;  // 4 np doubles: row statistics for the split scales
  double* cvec = nullptr;      // 2N: centring vector of the fused small-system step (kk_fused.hpp)
  double* pmax = nullptr;      // 2 per block of the fused step: largest centred potentials

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

  // last Krylov expansion left in V / Ft / ftilde (for a reverse pass that reuses it)
  bool fwd_valid = false;
  int fwd_m = 0;
  const double* fwd_K0 = nullptr;
  long prepare_gen = 0;  // bumped by every successful kk_prepare
  long alloc_gen = 0;    // bumped by every device allocation of the handle

  // Captured single-system update (krylov_run without profiling): captured on a private
  // stream (the caller's may be the null stream, which cannot capture) and replayed on the
  // handle's stream while its key (K0, m, tol, allocation generation, W, beta) holds. The
  // caller's delta and K delta are arguments of two kinds of kernel node (the first
  // precondition reads delta, every krylov_solve writes K delta); a call with other
  // pointers rewrites those nodes' arguments in the executable graph.
  hipStream_t gstream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct GraphArgNode {
    hipGraphNode_t node;
    hipKernelNodeParams p;
  };
  GraphArgNode g_pre{};                // precondition(K0, delta, sub, y, n2, stop, reset)
  kk::PreconditionArgs g_pre_args{};
  std::vector<GraphArgNode> g_solve;   // krylov_solve(V, Ft, ftilde, n2, st, Kdelta, tol)
  std::vector<kk::SolveArgs> g_solve_args;
  const double* g_delta = nullptr;
  double* g_kd = nullptr;
  const double* g_K0 = nullptr;
  int g_m = -1;
  double g_tol = -1.0;
  long g_gen = -1;
  double g_W = 0.0, g_beta = 0.0;
  bool no_graph = false;  // set if a capture failed: the eager path from then on

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    g_m = -1;
    g_solve.clear();
    g_solve_args.clear();
  }

  // reverse-pass workspace (krylov_kernel_adjoint), allocated on first use
  std::vector<void*> adj_owned;
  double *aX = nullptr, *aY = nullptr, *aK = nullptr, *aD = nullptr;  // 4, 4, 2, 2 padded matrices
  double *au = nullptr, *axdiag = nullptr, *apart = nullptr, *agdiag = nullptr;
  double *admu = nullptr, *agtot = nullptr, *ag = nullptr, *ay = nullptr, *alam = nullptr;
  double *aVbar = nullptr, *aFbar = nullptr, *abbar = nullptr, *aKd = nullptr;
  std::vector<void*> pair_owned;
  int2* apairs = nullptr;
  double* apk = nullptr;
  int pair_cap = 0, an0 = 0, an1 = 0;
  long pairs_gen = -1;

  void free_adjoint() {
    for (void* p : adj_owned) (void)hipFree(p);
    for (void* p : pair_owned) (void)hipFree(p);
    adj_owned.clear();
    pair_owned.clear();
    aX = aY = aK = aD = au = axdiag = apart = agdiag = nullptr;
    admu = agtot = ag = ay = alam = aVbar = aFbar = abbar = aKd = nullptr;
    apairs = nullptr;
    apk = nullptr;
    pair_cap = an0 = an1 = 0;
    pairs_gen = -1;
  }

  void free_workspace() {
    for (void* p : ws_owned) (void)hipFree(p);
    ws_owned.clear();
    chunk_cap = 0;
    u = Y = xdiag = part = nullptr;
    uct_h = uct_l = uct_r = yh = yl = yr = nullptr;
    x32 = nullptr;
    msc = nullptr;
  }

  void release() {
    if (owned.empty() && ws_owned.empty() && adj_owned.empty()) {
      prepared = false;
      return;
    }
    (void)hipStreamSynchronize(stream);
    if (gstream) (void)hipStreamSynchronize(gstream);
    drop_graph();
    free_workspace();
    free_adjoint();
    fwd_valid = false;
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
  ++h->alloc_gen;
  return st;
}

// Zero device memory with a plain kernel (no memset nodes if a caller captures).
__global__ void zero_fill(double* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// The per-direction split operand (U~ C)^T of every item of a response chunk in
// one launch: blockIdx.y = item z = 2 direction + spin, split from C^T at its scale.
template <bool BF16 = false, int NP = 2>
__global__ void split_operands(const double* __restrict__ CT0, const double* __restrict__ CT1, int np,
                               const double* __restrict__ u, const double* __restrict__ msc,
                               _Float16* __restrict__ uct_h, _Float16* __restrict__ uct_l,
                               const int* __restrict__ stop, _Float16* __restrict__ uct_r) {
  const int z = blockIdx.y;
  const size_t off = (size_t)z * np * np;
  kk::split_scaled_columns_dev<BF16, NP>((z & 1) ? CT1 : CT0, np, u + (size_t)z * np, msc + z * 8 + 3, uct_h + off,
                                         uct_l + off, stop, blockIdx.x, gridDim.x,
                                         NP == 3 ? uct_r + off : nullptr);
}

kk_status zero(kk_handle h, double* p, size_t n) {
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
  zero_fill<<<std::max(blocks, 1), 256, 0, h->stream>>>(p, n);
  LAUNCH_CHECK("zero_fill");
  return KK_OK;
}

int cu_count() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus;
}

// K-split of the response transforms of one small system. When the two items of a
// transform (one per spin) have fewer tiles than the chip has CUs, each item's contraction
// is cut into c chunks of kck rows (a multiple of KSTEP, at least KSPLIT_MIN_K rows for FP64
// and KSPLIT_MIN_K_SPLIT for the split forms, all c chunks inside the padding, whose rows past
// kc are zero); every chunk is a GEMM item of its own
// and the partial results are summed in a fixed order afterwards (forward: by the
// symmetrizing pass; back: by combine, as further Mulliken partial rows).
// FP64 (two workgroups per CU): c minimizes the per-CU work ceil(2 tiles c / CUs) / c and is
// taken when that is at most 3/4 of the unsplit figure (Nb = 1152: c = 3, 486 workgroups).
// Split forms (one workgroup per CU, whose blocks pay a fixed prologue and epilogue and
// whose partial products cost the symmetrizing pass more): the largest c whose 2 tiles c
// workgroups still fit one per CU (Nb = 1152: none; 1017: 2; 504: 4). Measured updates/s,
// split off / on, FP64 | FP16 x 3 | BF16: 128 atoms 417 / 504 | 1138 / 1052 | 700 / 650 (the
// split forms' c = 3 there is what this rule now avoids), 113 atoms 605 / 665 | 1255 / 1333 |
// 778 / 842, 56 atoms 1366 / 1555 | 1794 / 1948 | 1145 / 1289. The split forms' shorter
// chunks reach the smallest systems (16 atoms, kc = 160: four chunks of 64 rows; FP16 x 3 /
// BF16 6135 -> 6407 / 5605 -> 6237 updates/s, 17 atoms 6118 -> 6427 / 5606 -> 6262); FP64
// chunks that short would leave its 64 x 64 tiles for the K-split's 128 x 128 ones and ran
// 14 % slower there.
// -DKK_KSPLIT_MAX=1 turns the K-split off (for re-tuning).
#ifndef KK_KSPLIT_MAX
#define KK_KSPLIT_MAX 4
#endif
constexpr int KSPLIT_MAX = KK_KSPLIT_MAX, KSPLIT_MIN_K = 128, KSPLIT_MIN_K_SPLIT = 64;
int choose_ksplit(int np, int kc, int tiles, int cus, bool one_per_cu, int* chunk_rows, int min_k = 0) {
  *chunk_rows = kc;
  if (2 * tiles > cus) return 1;
  if (min_k == 0) min_k = one_per_cu ? KSPLIT_MIN_K_SPLIT : KSPLIT_MIN_K;
  auto load = [&](int c) { return (double)((2 * tiles * c + cus - 1) / cus) / c; };
  int best = 1, best_ck = kc;
  for (int c = 2; c <= KSPLIT_MAX; ++c) {
    const int ck = ((kc + c - 1) / c + KSTEP - 1) / KSTEP * KSTEP;
    if (ck < min_k || c * ck > np) continue;
    const bool better = one_per_cu ? 2 * tiles * c <= cus : load(c) < load(best);
    if (better) {
      best = c;
      best_ck = ck;
    }
  }
  if (!one_per_cu && load(best) > 0.75 * load(1)) return 1;
  *chunk_rows = best_ck;
  return best;
}

// Stream-K products for the split forms' small shape (gemm_mixed_sk), taken where no
// one-round K-split applies and one workgroup per tile would leave the workgroup rounds
// on the chip's CUs less than SK_FILL full. Returns the most segments of any tile of a
// one-direction launch (the slots per item; launches of more directions need no more), or
// 1 for no stream-K. The products stream their operands at about the same aggregate rate
// whether 162 or 256 CUs run them (the clock drops as more of them run), so stream-K gains
// only where a round is mostly empty: measured in one process, m = 8, FP16 x 3 / BF16
// updates/s without / with it, 170 atoms (Nb = 1530, 288 tiles, 2 rounds 56 % full)
// 608 / 676 and 412 / 460, but 128 atoms (162 tiles, 63 %) 1240 / 1152 and 940 / 911, 250
// atoms (648 tiles, 84 %) 289 / 246 and 189 / 161.
#ifndef KK_STREAM_K
#define KK_STREAM_K 1
#endif
constexpr double SK_FILL = 0.6;
int choose_stream_k(int tiles_per_item, int nk, int cus) {
  if (!KK_STREAM_K) return 1;
  const int tiles = 2 * tiles_per_item, rounds = (tiles + cus - 1) / cus;
  // fewer tiles are the one-round K-split's; the slot of a segment counts the workgroups
  // between it and its tile's first, which needs every range non-empty (stages >= grid)
  if (2 * tiles < cus || (long)tiles * nk < cus) return 1;
  if ((double)tiles / ((double)rounds * cus) >= SK_FILL) return 1;
  const long total = (long)tiles * nk;
  int slots = 1;
  for (int t = 0; t < tiles; ++t) slots = std::max(slots, kk::sk_segments(t, nk, cus, total));
  return slots;
}

// Form of the FP64 forward transform of one direction (both spins): the upper
// tiles over two K halves with the Fermi product in the epilogue, or all tiles
// over one half (half the cost each) followed by fermi_symmetrize_f64. The 64 x 64 tiles
// (unsplit handles of padded size 1536-2176 after f64_large_tiles_fill and the K-splits)
// always take the full form: FP64 updates/s, m = 8, one process, upper / full form, 170
// atoms 193.8 / 210.0, 165 atoms 197.9 / 215.2, 190 atoms 133.6 / 140.9, 230 atoms 84.1 /
// 85.2.
// The 128 x 128 tiles (two co-resident workgroups per CU) compare modelled launch times
// instead: w workgroups of `len` K-loop units on `cus` CUs run as whole rounds of two per CU,
// then the rest one per CU (at most cus of them) or two; two co-resident workgroups take
// PAIR_TIME of one alone, and the full form's symmetrizing pass SYM_TIME. Counting both slots
// as whole rounds chose badly where a round of pairs meets a round of singles; FP64 updates/s
// (m = 8, one process) with this choice against that one: 200 atoms (full form) 128.9 ->
// 132.0, 250 atoms 67.5 -> 71.8, 270 atoms 58.4 -> 66.6, 398 atoms 18.6 -> 19.9, 512 atoms
// 9.5 -> 9.9; 432 and 1024 atoms choose as before (upper form 3.89 against 3.95 ms, full form
// 46.4 against 47.2 ms).
constexpr double PAIR_TIME = 1.7, SYM_TIME = 0.1;
double launch_time(int w, int cus, double len) {
  const int p = w / (2 * cus), r = w - 2 * cus * p;
  return len * (PAIR_TIME * p + (r == 0 ? 0.0 : r <= cus ? 1.0 : PAIR_TIME));
}
bool full_forward_pairs(int n_upper, int n_full, int cus) {
  return launch_time(2 * n_full, cus, 1.0) + SYM_TIME < launch_time(2 * n_upper, cus, 2.0);
}

// Tile table order: groups of GROUP tile rows, each group walked column by column, so that
// the workgroups of one XCD (a contiguous range of the table, see xcd_remap) share a few A
// panels and sweep the B panels together. At Nb = 9216 on MI355X groups of 2-6 rows ran the
// split transforms 2-3 % faster than 8 (16 and 32: 2-9 % slower; 1: slower); the FP64 ones
// were indifferent between 2 and 8. upper: the same order restricted to the tiles holding at
// least one element with m <= n.
std::vector<int2> tile_order(int np, int bm, int bn, bool upper) {
  std::vector<int2> v;
  const int TM = np / bm, TN = np / bn;
  const int GROUP = kk::TILE_GROUP;  // the order kk::tile_table_pos computes
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

// Symmetrizing passes of the small-system forward transforms over nch partial products
// (kk_fused.hpp; nch = 1: the unsplit product), 32 x 32 block pairs of 256 threads.
template <int NCH>
void sym_f64_launch(kk_handle h, const kk::GemmArgs& sa, size_t cstride) {
  const int nblk = sa.n / kk::SYM64_B;
  kk::fermi_symmetrize_f64_chunks<kk::SYM64_B, 256, NCH>
      <<<dim3(nblk * (nblk + 1) / 2, sa.nitems), 256, 0, h->stream>>>(sa, cstride);
}
kk_status launch_sym_f64(kk_handle h, const kk::GemmArgs& sa, int nch, size_t cstride) {
  switch (nch) {
    case 1: sym_f64_launch<1>(h, sa, cstride); break;
    case 2: sym_f64_launch<2>(h, sa, cstride); break;
    case 3: sym_f64_launch<3>(h, sa, cstride); break;
    case 4: sym_f64_launch<4>(h, sa, cstride); break;
    default: return fail(KK_EINVAL, "internal: K-split into %d chunks", nch);
  }
  LAUNCH_CHECK("fermi_symmetrize_f64_chunks");
  return KK_OK;
}
template <bool BF16, int NP, int NCH>
void sym_mixed_launch(kk_handle h, const kk::MixedArgs& sa, size_t cstride) {
  const int nblk = sa.n / kk::SYM_B;
  kk::fermi_symmetrize_chunks<kk::SYM_B, 256, BF16, NP, NCH>
      <<<dim3(nblk * (nblk + 1) / 2, sa.nitems), 256, 0, h->stream>>>(sa, cstride);
}
template <bool BF16, int NP>
kk_status launch_sym_mixed_t(kk_handle h, const kk::MixedArgs& sa, int nch, size_t cstride) {
  switch (nch) {
    case 1: sym_mixed_launch<BF16, NP, 1>(h, sa, cstride); break;
    case 2: sym_mixed_launch<BF16, NP, 2>(h, sa, cstride); break;
    case 3: sym_mixed_launch<BF16, NP, 3>(h, sa, cstride); break;
    case 4: sym_mixed_launch<BF16, NP, 4>(h, sa, cstride); break;
    default: return fail(KK_EINVAL, "internal: K-split into %d chunks", nch);
  }
  LAUNCH_CHECK("fermi_symmetrize_chunks");
  return KK_OK;
}
kk_status launch_sym_mixed(kk_handle h, const kk::MixedArgs& sa, int nch, size_t cstride) {
  return h->bf16 ? launch_sym_mixed_t<true, 3>(h, sa, nch, cstride)
                 : launch_sym_mixed_t<false, 2>(h, sa, nch, cstride);
}

// cls: 0 the large tiles (FwdCfg / BackCfg), 1 SmallF64, 2 TinyF64.
kk_status launch_gemm(kk_handle h, int epi, kk::GemmArgs& a, int cls = 0) {
  const int grid = a.ntiles * a.nitems;
  if (grid <= 0) return KK_OK;
  if (a.nitems > kk::MAX_GEMM_BATCH) return fail(KK_EINVAL, "internal: too many GEMM items");
  const bool small = cls != 0;
  if (epi == kk::EPI_STORE) {
    kk::gemm_f64<kk::EPI_STORE, kk::StoreCfg><<<grid, kk::StoreCfg::THREADS, 0, h->stream>>>(a);
  } else if (epi == kk::EPI_FERMI) {
    ProfileScope ps(h, 0);
    if (cls == 2)
      kk::gemm_f64<kk::EPI_FERMI, TinyF64><<<grid, TinyF64::THREADS, 0, h->stream>>>(a);
    else if (cls == 1)
      kk::gemm_f64<kk::EPI_FERMI, SmallF64><<<grid, SmallF64::THREADS, 0, h->stream>>>(a);
    else
      kk::gemm_f64<kk::EPI_FERMI, kk::FwdCfg><<<grid, kk::FwdCfg::THREADS, 0, h->stream>>>(a);
  } else if (epi == kk::EPI_XSTORE) {  // forward: full-tile product into Y, then Y = F o X in place
    ProfileScope ps(h, 0);
    if (cls == 2)
      kk::gemm_f64<kk::EPI_XSTORE, TinyF64><<<grid, TinyF64::THREADS, 0, h->stream>>>(a);
    else if (cls == 1)
      kk::gemm_f64<kk::EPI_XSTORE, SmallF64><<<grid, SmallF64::THREADS, 0, h->stream>>>(a);
    else
      kk::gemm_f64<kk::EPI_XSTORE, kk::BackCfg><<<grid, kk::BackCfg::THREADS, 0, h->stream>>>(a);
    LAUNCH_CHECK("gemm_f64");
    if (small) {
      kk_status st = launch_sym_f64(h, a, 1, 0);
      if (st) return st;
    } else {
      const int nblk = a.n / kk::SYM64_B_LARGE;
      kk::fermi_symmetrize_f64<kk::SYM64_B_LARGE, kk::SYM64_T_LARGE>
          <<<dim3(nblk * (nblk + 1) / 2, a.nitems), kk::SYM64_T_LARGE, 0, h->stream>>>(a);
    }
  } else if (epi == kk::EPI_FERMI_XY) {
    ProfileScope ps(h, 2);
    kk::gemm_f64<kk::EPI_FERMI_XY, kk::FwdCfg><<<grid, kk::FwdCfg::THREADS, 0, h->stream>>>(a);
  } else if (epi == kk::EPI_ACCUM) {
    ProfileScope ps(h, 3);
    kk::gemm_f64<kk::EPI_ACCUM, kk::BackCfg><<<grid, kk::BackCfg::THREADS, 0, h->stream>>>(a);
  } else {
    ProfileScope ps(h, 1);
    if (cls == 2)
      kk::gemm_f64<kk::EPI_MULLIKEN, TinyF64><<<grid, TinyF64::THREADS, 0, h->stream>>>(a);
    else if (cls == 1)
      kk::gemm_f64<kk::EPI_MULLIKEN, SmallF64><<<grid, SmallF64::THREADS, 0, h->stream>>>(a);
    else
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
  const size_t kch = h->kch;  // K-split: one partial product per chunk
  if (h->precision == KK_FP64) {
    if ((st = dalloc_t(h, &h->Y, items * kch * np * np, true))) return st;
  } else {
    for (_Float16** q : {&h->uct_h, &h->uct_l, &h->yh, &h->yl})
      if ((st = dalloc_t(h, q, items * np * np, true))) return st;
    if (h->bf16)
      for (_Float16** q : {&h->uct_r, &h->yr})
        if ((st = dalloc_t(h, q, items * np * np, true))) return st;
    if ((st = dalloc_t(h, &h->x32, items * kch * np * np, true))) return st;
    if ((st = dalloc_t(h, &h->msc, items * 8, true))) return st;
  }
  if ((st = dalloc_t(h, &h->xdiag, items * np, true))) return st;
  if ((st = dalloc_t(h, &h->part, items * h->nparts * np, true))) return st;
  if ((st = zero(h, h->u, items * np))) return st;
  h->chunk_cap = chunk;
  return KK_OK;
}

int max_chunk(kk_handle h) {
  // FP64: one Y per spin and chunk; split path: four (BF16: six) 16-bit matrices per spin and
  // one FP32 per spin and chunk
  const size_t kch = h->kch;
  const size_t per_dir = (size_t)2 * h->np * h->np *
                         (h->precision == KK_FP64 ? kch * sizeof(double)
                                                  : (h->bf16 ? 6 : 4) * sizeof(_Float16) + kch * sizeof(float));
  size_t c = WORKSPACE_BUDGET / std::max<size_t>(per_dir, 1);
  return (int)std::max<size_t>(1, std::min<size_t>(c, kk::MAX_GEMM_BATCH / (2 * kch)));
}

// The last step of a response: q1 (and with K0 = -I the preconditioned derivative ft) from
// the Mulliken partial rows and diag X (combine; combine_small for the fused small step).
kk_status launch_combine(kk_handle h, int batch, double* q1, const int* stop, const double* vsub, double* ft) {
  const int N = h->natoms;
  dim3 grid((N + kk::COMBINE_ATOMS - 1) / kk::COMBINE_ATOMS, batch);
  if (2 * N <= kk::FUSED_MAX_N2)
    kk::combine_small<<<grid, kk::COMBINE_THREADS, 0, h->stream>>>(h->xdiag, h->part, h->nparts, h->w[0], h->w[1],
                                                                  h->wsum, h->t, h->nb, h->np, h->offsets, N, q1,
                                                                  stop, vsub, ft);
  else
    kk::combine<<<grid, kk::COMBINE_THREADS, 0, h->stream>>>(h->xdiag, h->part, h->nparts, h->w[0], h->w[1],
                                                             h->wsum, h->t, h->nb, h->np, h->offsets, N, q1, stop,
                                                             vsub, ft);
  LAUNCH_CHECK("combine");
  return KK_OK;
}

// K-split FP64 transforms (choose_ksplit) of `batch` directions whose potentials are in h->u:
// the forward as kch full-tile partial products per item into Y (chunk j of item z at
// Y + (z kch + j) np^2), summed and symmetrized into the first; the back-transform as kch
// partial Mulliken products per item, rows j nbase .. (j + 1) nbase - 1 of the item's partials.
kk_status ksplit_transforms_f64(kk_handle h, int batch, const int* stop) {
  const int np = h->np, kch = h->kch, ck = h->kck;
  const size_t np2 = (size_t)np * np;
  const bool tiny = h->ktiny;  // chunks of 64 x 64 TinyF64 tiles, else of the 128 x 128 ones
  kk::GemmArgs fa{}, sa{}, ba{};
  fa.n = np; fa.k_half = ck; fa.two_halves = 0; fa.ntiles = tiny ? h->n_sfull : h->n_full;
  fa.nitems = 2 * batch * kch;
  fa.tiles = tiny ? h->stiles_full : h->tiles_full; fa.stop = stop; fa.beta = h->beta;
  sa = fa;
  sa.nitems = 2 * batch;
  ba = fa;
  for (int z = 0; z < 2 * batch; ++z) {
    const int s = z & 1;
    double* Y0 = h->Y + (size_t)z * kch * np2;
    kk::GemmItem& si = sa.item[z];
    si = kk::GemmItem{};
    si.out = Y0; si.eps = h->eps[s]; si.f = h->f[s]; si.fc = h->fc[s]; si.w = h->w[s];
    si.xdiag = h->xdiag + (size_t)z * np;
    for (int j = 0; j < kch; ++j) {
      const size_t k0 = (size_t)j * ck;
      kk::GemmItem& fi = fa.item[z * kch + j];
      fi = kk::GemmItem{};
      fi.a0 = h->C[s] + k0 * np; fi.b0 = h->G[s] + k0 * np; fi.scale = h->u + (size_t)z * np + k0;
      fi.out = Y0 + j * np2;
      kk::GemmItem& bi = ba.item[z * kch + j];
      bi = kk::GemmItem{};
      bi.a0 = h->CT[s] + k0 * np; bi.b0 = Y0 + k0 * np; bi.g = h->G[s];
      bi.part = h->part + ((size_t)z * h->nparts + (size_t)j * h->nbase) * np;
    }
  }
  if (fa.nitems > kk::MAX_GEMM_BATCH) return fail(KK_EINVAL, "internal: too many GEMM items");
  {
    ProfileScope ps(h, 0);
    if (tiny)
      kk::gemm_f64<kk::EPI_XSTORE, TinyF64><<<fa.ntiles * fa.nitems, TinyF64::THREADS, 0, h->stream>>>(fa);
    else
      kk::gemm_f64<kk::EPI_XSTORE, kk::BackCfg><<<fa.ntiles * fa.nitems, kk::BackCfg::THREADS, 0, h->stream>>>(fa);
    LAUNCH_CHECK("gemm_f64 k-split");
    kk_status st = launch_sym_f64(h, sa, kch, np2);
    if (st) return st;
  }
  {
    ProfileScope ps(h, 1);
    if (tiny)
      kk::gemm_f64<kk::EPI_MULLIKEN, TinyF64><<<ba.ntiles * ba.nitems, TinyF64::THREADS, 0, h->stream>>>(ba);
    else
      kk::gemm_f64<kk::EPI_MULLIKEN, kk::BackCfg><<<ba.ntiles * ba.nitems, kk::BackCfg::THREADS, 0, h->stream>>>(ba);
    LAUNCH_CHECK("gemm_f64 k-split");
  }
  return KK_OK;
}

// The two FP64 response transforms of `batch` directions whose potentials are in h->u.
kk_status transforms_f64(kk_handle h, int batch, const int* stop) {
  if (h->kch > 1) return ksplit_transforms_f64(h, batch, stop);
  const int np = h->np;
  const bool small = h->small_f64;
  kk::GemmArgs fa{};
  // forward (full_fwd): A = C^T U~ G over full tiles into Y, then X = (A + A^T) / 2 and
  // Y = F o X in place; otherwise upper tiles over both K halves with the Fermi epilogue
  const bool full = h->full_fwd;
  fa.n = np; fa.k_half = h->kc; fa.two_halves = full ? 0 : 1;
  fa.ntiles = small ? (full ? h->n_sfull : h->n_supper) : (full ? h->n_full : h->n_upper);
  fa.nitems = 2 * batch; fa.tiles = small ? (full ? h->stiles_full : h->stiles_upper) : (full ? h->tiles_full : h->tiles_upper);
  fa.stop = stop; fa.beta = h->beta;
  kk::GemmArgs ba{};
  ba.n = np; ba.k_half = h->kc; ba.two_halves = 0; ba.ntiles = small ? h->n_sfull : h->n_full;
  ba.nitems = 2 * batch; ba.tiles = small ? h->stiles_full : h->tiles_full; ba.stop = stop; ba.beta = h->beta;
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
  const int cls = h->tiny_f64 ? 2 : small ? 1 : 0;
  if ((st = launch_gemm(h, full ? kk::EPI_XSTORE : kk::EPI_FERMI, fa, cls))) return st;
  if ((st = launch_gemm(h, kk::EPI_MULLIKEN, ba, cls))) return st;
  return KK_OK;
}

// Responses of `batch` directions v (batch x 2N) into q1 (batch x 2N); batch <= chunk_cap.
// identity = true: potentials v_q +/- v_m per atom (gamma = I, W = 1), the transposed-response
// form the reverse pass needs.
// prologue_done: the potentials of the single direction are already in h->u (the fused
// Krylov step wrote them); vsub, ft (K0 = -I only): combine also writes ft = -(q1 - vsub).
kk_status response_chunk(kk_handle h, int batch, const double* v, double* q1, const int* stop,
                         bool identity = false, bool prologue_done = false, const double* vsub = nullptr,
                         double* ft = nullptr) {
  const int N = h->natoms, np = h->np;
  if (!prologue_done) {
    const int waves = N * batch, threads = 256;
    const int blocks = (waves * kk::WAVE + threads - 1) / threads;
    kk::potentials<<<blocks, threads, 0, h->stream>>>(identity ? nullptr : h->gamma, N, identity ? 1.0 : h->W, v,
                                                       batch, h->offsets, np,
                                                       h->u, stop);
    LAUNCH_CHECK("potentials");
  }
  kk_status st;
  if ((st = transforms_f64(h, batch, stop))) return st;
  return launch_combine(h, batch, q1, stop, vsub, ft);
}

// Split-precision transform step: the forward (full-tile product into the FP32
// workspace, then the symmetrizing pass that writes the split Y) or the back-transform.
// a2, b2 (BF16 form only): per item the third pieces of At and Bt, whose products with the
// hi pieces (the refinement) run in the same pass as the four hi/lo products (PROD_ALL6).
// K-split (sym != nullptr): a's items are the kch chunks of each of sym's items, whose
// symmetrizing pass sums their partial products.
// Large split handles symmetrize on 64 x 64 block pairs with eight elements per thread
// (fermi_symmetrize_v8): against the earlier pass with one element per thread and row,
// the same bits and, one process, FP16 x 3 / BF16 updates/s 1024 atoms 4.348 -> 4.357 /
// 2.392 -> 2.406, 432 atoms 77.03 -> 77.40 / 44.27 -> 44.87.
static_assert(kk::SYM_B_LARGE == 64, "the large handles' symmetrizing pass runs 64 x 64 block pairs");
template <class Cfg>
kk_status launch_bf16_single(kk_handle h, bool forward, kk::MixedArgs& a, const _Float16* const* a2,
                             const _Float16* const* b2, const kk::MixedArgs* sym, int kch) {
  const int grid = a.ntiles * a.nitems;
  for (int z = 0; z < a.nitems; ++z) { a.item[z].a0r = a2[z]; a.item[z].b0r = b2[z]; }
  if (forward) {
    if (a.sk_grid > 0)
      kk::gemm_mixed_sk<kk::EPI_STORE, Cfg><<<a.sk_grid, Cfg::THREADS, 0, h->stream>>>(a);
    else
      kk::gemm_mixed<kk::EPI_STORE, Cfg><<<grid, Cfg::THREADS, 0, h->stream>>>(a);
    LAUNCH_CHECK("gemm_mixed bf16 one pass");
    if (h->mx_large) {
      const int nblk = a.n / kk::SYM_B_LARGE;
      kk::fermi_symmetrize_v8<true, 3><<<dim3(nblk * (nblk + 1) / 2, a.nitems), 512, 0, h->stream>>>(a);
      LAUNCH_CHECK("fermi_symmetrize bf16");
      return KK_OK;
    }
    return launch_sym_mixed(h, sym != nullptr ? *sym : a, kch, (size_t)a.n * a.n);
  }
  if (a.sk_grid > 0)
    kk::gemm_mixed_sk<kk::EPI_MULLIKEN, Cfg><<<a.sk_grid, Cfg::THREADS, 0, h->stream>>>(a);
  else
    kk::gemm_mixed<kk::EPI_MULLIKEN, Cfg><<<grid, Cfg::THREADS, 0, h->stream>>>(a);
  LAUNCH_CHECK("gemm_mixed bf16 one pass");
  return KK_OK;
}

// sym, kch: the K-split form, as for launch_bf16_single (small product configuration only).
kk_status launch_mixed(kk_handle h, bool forward, kk::MixedArgs& a, const _Float16* const* a2 = nullptr,
                       const _Float16* const* b2 = nullptr, const kk::MixedArgs* sym = nullptr, int kch = 1) {
  const int grid = a.ntiles * a.nitems;
  if (grid <= 0) return KK_OK;
  if (a.nitems > kk::MAX_GEMM_BATCH) return fail(KK_EINVAL, "internal: too many GEMM items");
  if ((kch > 1 || a.sk_grid > 0) && h->mx_large) return fail(KK_EINVAL, "internal: K-split on the large split tiles");
  if (h->bf16) {
    ProfileScope ps(h, forward ? 0 : 1);
    return h->mx_large  ? launch_bf16_single<kk::MLargeBf6>(h, forward, a, a2, b2, sym, kch)
           : h->mx_tiny ? launch_bf16_single<MTinyBf6>(h, forward, a, a2, b2, sym, kch)
                        : launch_bf16_single<kk::MSmallBf6>(h, forward, a, a2, b2, sym, kch);
  }
  if (forward) {
    ProfileScope ps(h, 0);
    if (h->mx_large)
      kk::gemm_mixed<kk::EPI_STORE, kk::MLargeCfg><<<grid, kk::MLargeCfg::THREADS, 0, h->stream>>>(a);
    else if (h->mx_tiny)
      kk::gemm_mixed<kk::EPI_STORE, MTinyCfg><<<grid, MTinyCfg::THREADS, 0, h->stream>>>(a);
    else if (a.sk_grid > 0)
      kk::gemm_mixed_sk<kk::EPI_STORE, kk::MSmallCfg><<<a.sk_grid, kk::MSmallCfg::THREADS, 0, h->stream>>>(a);
    else
      kk::gemm_mixed<kk::EPI_STORE, kk::MSmallCfg><<<grid, kk::MSmallCfg::THREADS, 0, h->stream>>>(a);
    LAUNCH_CHECK("gemm_mixed");
    if (!h->mx_large) {
      kk_status st = launch_sym_mixed(h, sym != nullptr ? *sym : a, kch, (size_t)a.n * a.n);
      if (st) return st;
    } else {
      const int nblk = a.n / kk::SYM_B_LARGE;
      kk::fermi_symmetrize_v8<false, 2><<<dim3(nblk * (nblk + 1) / 2, a.nitems), 512, 0, h->stream>>>(a);
    }
    LAUNCH_CHECK("fermi_symmetrize");
  } else {
    ProfileScope ps(h, 1);
    if (h->mx_large)
      kk::gemm_mixed<kk::EPI_MULLIKEN, kk::MLargeCfg><<<grid, kk::MLargeCfg::THREADS, 0, h->stream>>>(a);
    else if (h->mx_tiny)
      kk::gemm_mixed<kk::EPI_MULLIKEN, MTinyCfg><<<grid, MTinyCfg::THREADS, 0, h->stream>>>(a);
    else if (a.sk_grid > 0)
      kk::gemm_mixed_sk<kk::EPI_MULLIKEN, kk::MSmallCfg><<<a.sk_grid, kk::MSmallCfg::THREADS, 0, h->stream>>>(a);
    else
      kk::gemm_mixed<kk::EPI_MULLIKEN, kk::MSmallCfg><<<grid, kk::MSmallCfg::THREADS, 0, h->stream>>>(a);
  }
  LAUNCH_CHECK("gemm_mixed");
  return KK_OK;
}

// Split-precision responses: same steps as response_chunk, with the two
// transforms on FP16 x 3 MFMA products (Y kept as an FP16 split).
kk_status response_chunk_mixed(kk_handle h, int batch, const double* v, double* q1, const int* stop,
                               bool identity = false, bool prologue_done = false, const double* vsub = nullptr,
                               double* ft = nullptr) {
  const int N = h->natoms, np = h->np;
  const size_t np2 = (size_t)np * np;
  const int blocks = (int)std::max<size_t>(1, std::min<size_t>((np2 / 8 + 255) / 256, 16384 / (2 * batch)));
  if (prologue_done) {  // one direction after orth_potentials: scales from its block maxima, then the split
    const int nblk = (N + kk::FUSED_ATOMS - 1) / kk::FUSED_ATOMS;
    if (h->bf16)
      kk::split_operands_fused<true, 3><<<dim3(blocks, 2), 256, 0, h->stream>>>(
          h->CT[0], h->CT[1], np, h->u, h->pmax, nblk, h->mconst, h->beta, h->msc, h->uct_h, h->uct_l, h->uct_r,
          stop);
    else
      kk::split_operands_fused<false, 2><<<dim3(blocks, 2), 256, 0, h->stream>>>(
          h->CT[0], h->CT[1], np, h->u, h->pmax, nblk, h->mconst, h->beta, h->msc, h->uct_h, h->uct_l, nullptr,
          stop);
    LAUNCH_CHECK("split_operands_fused");
  } else {
    {
      const int waves = N * batch, threads = 256;
      const int wblocks = (waves * kk::WAVE + threads - 1) / threads;
      kk::potentials<<<wblocks, threads, 0, h->stream>>>(identity ? nullptr : h->gamma, N, identity ? 1.0 : h->W, v,
                                                          batch, h->offsets, np, h->u, stop);
      LAUNCH_CHECK("potentials");
    }
    kk::center_potentials<<<batch, 1024, 0, h->stream>>>(h->u, np, h->nb, h->w[0], h->w[1], stop);
    LAUNCH_CHECK("center_potentials");
    kk::mixed_scales<<<2 * batch, 1024, 0, h->stream>>>(h->u, np, h->mconst, h->beta, h->msc, stop);
    LAUNCH_CHECK("mixed_scales");
    if (h->bf16)
      split_operands<true, 3><<<dim3(blocks, 2 * batch), 256, 0, h->stream>>>(h->CT[0], h->CT[1], np, h->u, h->msc,
                                                                               h->uct_h, h->uct_l, stop, h->uct_r);
    else
      split_operands<<<dim3(blocks, 2 * batch), 256, 0, h->stream>>>(h->CT[0], h->CT[1], np, h->u, h->msc, h->uct_h,
                                                                      h->uct_l, stop, nullptr);
    LAUNCH_CHECK("split_operands");
  }
  // forward: A = C^T U~ G over full tiles (At = (U~ C)^T, Bt = G^T), X = (A + A^T) / 2.
  // K-split (kch > 1): item z's forward chunk j is GEMM item z kch + j over contraction rows
  // [j kck, (j + 1) kck) (operands k-contiguous: a column offset) with its FP32 partial
  // product at x32 + (z kch + j) np^2; sa holds the unsplit items for the symmetrizing pass,
  // which sums the partials. Back chunk j (kchb = kch) writes its Mulliken partials at rows
  // j nbase.. of the item's partials, which the combine sums with the rest.
  // Stream-K (h->sk): one GEMM item per spin and direction over the whole contraction; the
  // kch = kchb partial slots of each are filled by the segments of gemm_mixed_sk.
  const int kch = h->sk ? 1 : h->kch, kchb = h->sk ? 1 : h->kchb;
  const size_t ck = kch > 1 ? h->kck : 0, ckb = kchb > 1 ? h->kck : 0;
  kk::MixedArgs fa{};
  fa.n = np; fa.k = kch > 1 ? h->kck : h->kc; fa.ntiles = h->n_mfull; fa.nitems = 2 * batch * kch;
  fa.tiles = h->mtiles_full; fa.stop = stop; fa.beta = h->beta;
  if (h->sk) {
    fa.sk_grid = h->sk_grid;
    fa.sk_slots = h->kch;
    fa.sk_side = kk::MSmallCfg::BM;
    fa.sk_stride = np2;
    // the item's partial slots (sized for one direction) must hold every tile's segments of
    // this launch; longer launches cut fewer segments per tile, checked here all the same
    const int nk = h->kc / kk::MSmallCfg::BK, tiles = 2 * batch * h->n_mfull;
    const long total = (long)tiles * nk;
    for (int t = 0; t < tiles; ++t)
      if (kk::sk_segments(t, nk, h->sk_grid, total) > h->kch)
        return fail(KK_EINVAL, "internal: stream-K tile %d needs more than %d slots", t, h->kch);
  }
  kk::MixedArgs ba = fa;
  ba.k = kchb > 1 ? h->kck : h->kc;
  ba.nitems = 2 * batch * kchb;
  if (h->sk) {
    ba.sk_slots = h->kchb;
    ba.sk_stride = (size_t)h->nbase * np;
  }
  kk::MixedArgs sa = fa;
  sa.nitems = 2 * batch;
  if (fa.nitems > kk::MAX_GEMM_BATCH || ba.nitems > kk::MAX_GEMM_BATCH)
    return fail(KK_EINVAL, "internal: too many GEMM items");
  // BF16 refinement operands: residual pieces of (U~ C)^T and G^T (forward), C and Y (back)
  const _Float16 *fa2[kk::MAX_GEMM_BATCH], *fb2[kk::MAX_GEMM_BATCH], *ba2[kk::MAX_GEMM_BATCH],
      *bb2[kk::MAX_GEMM_BATCH];
  for (int z = 0; z < 2 * batch; ++z) {
    const int s = z & 1;
    kk::MixedItem& si = sa.item[z];
    si = kk::MixedItem{};
    si.x32 = h->x32 + (size_t)z * h->kch * np2;
    si.yh = h->yh + z * np2; si.yl = h->yl + z * np2; si.yr = h->bf16 ? h->yr + z * np2 : nullptr;
    si.eps = h->eps[s]; si.f = h->f[s]; si.fc = h->fc[s]; si.w = h->w[s];
    si.xdiag = h->xdiag + (size_t)z * np;
    si.sc = h->msc + z * 8;
    for (int j = 0; j < kch; ++j) {
      const size_t k0 = j * ck;
      const int q = z * kch + j;
      kk::MixedItem& fi = fa.item[q];
      fi = si;
      fi.a0h = h->uct_h + z * np2 + k0; fi.a0l = h->uct_l + z * np2 + k0;
      fi.b0h = h->GTh[s] + k0; fi.b0l = h->GTl[s] + k0;
      fi.x32 = si.x32 + j * np2;
      if (h->bf16) { fa2[q] = h->uct_r + z * np2 + k0; fb2[q] = h->GTr[s] + k0; }
    }
    for (int j = 0; j < kchb; ++j) {
      const size_t k0 = j * ckb;
      const int q = z * kchb + j;
      kk::MixedItem& bi = ba.item[q];
      bi = kk::MixedItem{};
      bi.a0h = h->Ch[s] + k0; bi.a0l = h->Cl[s] + k0; bi.b0h = h->yh + z * np2 + k0; bi.b0l = h->yl + z * np2 + k0;
      bi.g = h->G[s];
      bi.part = h->part + ((size_t)z * h->nparts + (size_t)j * h->nbase) * np;
      bi.sc = h->msc + z * 8 + 2;
      if (h->bf16) { ba2[q] = h->Cr[s] + k0; bb2[q] = h->yr + z * np2 + k0; }
    }
  }
  kk_status st;
  if ((st = launch_mixed(h, true, fa, fa2, fb2, kch > 1 ? &sa : nullptr, h->kch))) return st;
  if ((st = launch_mixed(h, false, ba, ba2, bb2))) return st;
  return launch_combine(h, batch, q1, stop, vsub, ft);
}

kk_status response_any(kk_handle h, int batch, const double* v, double* q1, const int* stop,
                       bool identity = false, bool prologue_done = false, const double* vsub = nullptr,
                       double* ft = nullptr) {
  return h->precision == KK_FP64 ? response_chunk(h, batch, v, q1, stop, identity, prologue_done, vsub, ft)
                                 : response_chunk_mixed(h, batch, v, q1, stop, identity, prologue_done, vsub, ft);
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
  std::vector<int2> sup, sfull, mfull;
  if (h->small_f64) {
    sup = tile_order(np, SmallF64::BM, SmallF64::BN, true);
    sfull = tile_order(np, SmallF64::BM, SmallF64::BN, false);
    h->n_supper = (int)sup.size();
    h->n_sfull = (int)sfull.size();
    if ((st = dalloc_t(h, &h->stiles_upper, sup.size()))) return st;
    if ((st = dalloc_t(h, &h->stiles_full, sfull.size()))) return st;
    HIP_OR_FAIL(hipMemcpyAsync(h->stiles_upper, sup.data(), sizeof(int2) * sup.size(), hipMemcpyHostToDevice,
                               h->stream));
    HIP_OR_FAIL(hipMemcpyAsync(h->stiles_full, sfull.data(), sizeof(int2) * sfull.size(), hipMemcpyHostToDevice,
                               h->stream));
  }
  h->n_upper = (int)up.size();
  h->n_full = (int)full.size();
  h->n_store = (int)stt.size();
  static_assert(kk::FwdCfg::MIN_BLOCKS == kk::BackCfg::MIN_BLOCKS, "one slot count for both forward forms");
  h->full_fwd = h->kch > 1 || h->small_f64 || full_forward_pairs(h->n_upper, h->n_full, cu_count());
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
  if (h->precision != KK_FP64) {
    if ((st = dalloc_t(h, &h->mconst, 8))) return st;
    if ((st = dalloc_t(h, &h->mscratch, (size_t)4 * np))) return st;
    if ((st = dalloc_t(h, &h->cvec, (size_t)2 * n_atoms))) return st;
    if ((st = dalloc_t(h, &h->pmax, (size_t)2 * kk::FUSED_MAX_BLOCKS))) return st;
    for (int s = 0; s < 2; ++s) {
      if ((st = dalloc_t(h, &h->GT[s], np2))) return st;
      for (_Float16** q : {&h->Ch[s], &h->Cl[s], &h->GTh[s], &h->GTl[s]})
        if ((st = dalloc_t(h, q, np2))) return st;
      if (h->bf16)
        for (_Float16** q : {&h->Cr[s], &h->GTr[s]})
          if ((st = dalloc_t(h, q, np2))) return st;
    }
    mfull = h->mx_large  ? tile_order(np, kk::MLargeCfg::BM, kk::MLargeCfg::BN, false)
            : h->mx_tiny ? tile_order(np, MTinyCfg::BM, MTinyCfg::BN, false)
                         : tile_order(np, kk::MSmallCfg::BM, kk::MSmallCfg::BN, false);
    h->n_mfull = (int)mfull.size();
    if (h->sk) {  // the symmetrizing pass of a stream-K product finds tiles by kk::tile_table_pos
      const int T = np / kk::MSmallCfg::BM;
      for (int i = 0; i < h->n_mfull; ++i)
        if (kk::tile_table_pos(mfull[i].x, mfull[i].y, T, T) != i)
          return fail(KK_EINVAL, "internal: tile table order differs from tile_table_pos");
    }
    if ((st = dalloc_t(h, &h->mtiles_full, mfull.size()))) return st;
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
    if (s == 0 && 2 * h->natoms <= kk::FUSED_MAX_N2) {
      kk::centre_vector<<<h->natoms + 1, 256, 0, h->stream>>>(h->gamma, h->natoms, h->W, h->offsets, h->w[0], h->w[1],
                                                               h->wsum, h->cvec);
      LAUNCH_CHECK("centre_vector");
    }
    if (h->bf16) {
      kk::split_matrix<true, 3><<<pg, pb, 0, h->stream>>>(h->C[s], np, 0, h->mconst + 4 * s, h->Ch[s], h->Cl[s],
                                                          h->Cr[s]);
      kk::split_matrix<true, 3><<<pg, pb, 0, h->stream>>>(h->GT[s], np, 0, h->mconst + 4 * s + 1, h->GTh[s],
                                                          h->GTl[s], h->GTr[s]);
    } else {
      kk::split_matrix<<<pg, pb, 0, h->stream>>>(h->C[s], np, 0, h->mconst + 4 * s, h->Ch[s], h->Cl[s], nullptr);
      kk::split_matrix<<<pg, pb, 0, h->stream>>>(h->GT[s], np, 0, h->mconst + 4 * s + 1, h->GTh[s], h->GTl[s],
                                                 nullptr);
    }
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
  (void)hipStreamSynchronize(h->stream);
  if (h->gstream) (void)hipStreamSynchronize(h->gstream);
  h->drop_graph();
  if (h->gstream) (void)hipStreamDestroy(h->gstream);
  delete h;
  return KK_OK;
}

}  // extern "C"

namespace {

// kk_prepare; split_large selects the large split product configuration whatever the size
// (a batch's systems).
kk_status prepare_impl(kk_handle h, int n_atoms, const int* atom_offsets, int n_basis, const double* S,
                       const double* Z, const double* Q_up, const double* Q_dn, const double* eps_up,
                       const double* eps_dn, const double* gamma, double W, double kT, double n_electrons,
                       int precision, bool split_large) {
  if (!h) return fail(KK_EINVAL, "kk_prepare: handle is NULL");
  if (n_atoms < 1 || n_basis < 1) return fail(KK_EINVAL, "kk_prepare: n_atoms and n_basis must be >= 1");
  if (2 * n_atoms > 8 * 1024) return fail(KK_EINVAL, "kk_prepare: at most 4096 atoms are supported");
  if (n_basis > 65536) return fail(KK_EINVAL, "kk_prepare: at most 65536 basis functions are supported");
  if (!atom_offsets || !S || !Z || !Q_up || !Q_dn || !eps_up || !eps_dn || !gamma)
    return fail(KK_EINVAL, "kk_prepare: NULL array argument");
  if (!(kT > 0.0)) return fail(KK_EINVAL, "kk_prepare: kT must be > 0");
  if (!(n_electrons > 0.0 && n_electrons < 2.0 * n_basis))
    return fail(KK_EINVAL, "kk_prepare: need 0 < n_electrons < 2 n_basis");
  if (precision != KK_FP64 && precision != KK_MIXED_F16 && precision != KK_MIXED_BF16)
    return fail(KK_EINVAL, "kk_prepare: unsupported precision %d", precision);
  if (atom_offsets[0] != 0 || atom_offsets[n_atoms] != n_basis)
    return fail(KK_EINVAL, "kk_prepare: atom_offsets must start at 0 and end at n_basis");
  for (int a = 0; a < n_atoms; ++a)
    if (atom_offsets[a + 1] <= atom_offsets[a])
      return fail(KK_EINVAL, "kk_prepare: atom_offsets must be strictly increasing (atom %d)", a);

  const bool mixed = precision != KK_FP64;
  const bool mx_large = mixed && (split_large || n_basis > SPLIT_LARGE_NB);
  const int pad = mixed ? (mx_large ? SPLIT_PAD_LARGE : SPLIT_PAD_SMALL) : kk::PAD;
  const int nb = n_basis, np = (nb + pad - 1) / pad * pad;
  // Re-preparing the same shape (an SCF or MD loop) reuses every buffer.
  const bool reuse = h->prepared && h->natoms == n_atoms && h->nb == nb && h->np == np &&
                     h->precision == precision && h->mx_large == mx_large;
  h->prepared = false;
  h->fwd_valid = false;
  kk_status st;
  if (!reuse) {
    h->release();
    h->precision = precision;
    h->bf16 = precision == KK_MIXED_BF16;
    h->natoms = n_atoms; h->nb = nb; h->np = np;
    h->kc = (nb + KSTEP - 1) / KSTEP * KSTEP;
    // the K-split runs on the 128 x 128 tiles of either form, for FP64 systems up to a padded
    // size of 512 on 64 x 64 tiles (a batch's systems never split)
    h->kch = 1;
    h->kck = h->kc;
    h->sk = false;
    h->sk_grid = 0;
    h->ktiny = false;
    h->mx_tiny = mixed && !mx_large && !split_large && np <= MTINY_MAX_NP;
    if (!split_large && !mx_large) {
      const int tiles = h->mx_tiny ? (np / MTinyCfg::BM) * (np / MTinyCfg::BN)
                        : mixed    ? (np / kk::MSmallCfg::BM) * (np / kk::MSmallCfg::BN)
                                   : (np / kk::BackCfg::BM) * (np / kk::BackCfg::BN);
      h->kch = choose_ksplit(np, h->kc, tiles, cu_count(), mixed, &h->kck);
      if (mixed && !h->mx_tiny && h->kch == 1) {
        const int slots = choose_stream_k(tiles, h->kc / kk::MSmallCfg::BK, cu_count());
        if (slots > 1) {
          h->sk = true;
          h->sk_grid = cu_count();
          h->kch = slots;
        }
      }
    }
    // Both transforms split alike. (The split back-transform repeats its epilogue, the
    // Mulliken product with G, per chunk; split into two rounds of workgroups, as the FP64
    // rule would have it at Nb = 1152, it ran slower, 37.4 against 35.1 us, but in the one
    // round the split forms' rule allows it is faster: 113 atoms, m = 8, FP16 x 3 1480 ->
    // 1627 updates/s, BF16 1169 -> 1320; 56 atoms 2241 -> 2575 and 1916 -> 2370.)
    h->kchb = h->kch;
    h->small_f64 = !mixed && np <= SMALL_NP_F64 && h->kch == 1 && !f64_large_tiles_fill(np, cu_count());
    h->tiny_f64 = h->small_f64 && np <= TINY_NP_F64;
#ifndef KK_TINY_KSPLIT
#define KK_TINY_KSPLIT 1
#endif
#ifndef KK_KTINY_MAX_NP
#define KK_KTINY_MAX_NP 512
#endif
    if (KK_TINY_KSPLIT && !mixed && np <= KK_KTINY_MAX_NP && !split_large) {
      // FP64 systems up to a padded size of 512 split the contraction of 64 x 64 tiles
      // (TinyF64, K stage 32) instead, in chunks down to two K stages, whenever the FP64 rule
      // splits them at all (16 atoms, kc = 160: four chunks of 64 rows, 128 workgroups
      // instead of 32; 37 atoms: three chunks of 128 rows, 216 workgroups instead of the
      // 128 x 128 split's 54). Updates/s against the 128 x 128 split or the unsplit 64 x 64
      // tiles, one process: 16 atoms m = 4 6048 -> 7082, 8 atoms 7187 -> 7795, 29 atoms m = 8
      // 1680 -> 2977, 37 atoms 1816 -> 2747, 56 atoms 1734 -> 2100; from a padded size of 640
      // the rule stops splitting these tiles (70 and 85 atoms: level).
      const int t64 = (np / TinyF64::BM) * (np / TinyF64::BN);
      int ck = h->kc;
      const int c = choose_ksplit(np, h->kc, t64, cu_count(), false, &ck, 2 * TinyF64::BK);
      if (c > 1) {
        h->kch = h->kchb = c;
        h->kck = ck;
        h->ktiny = true;
        h->small_f64 = h->tiny_f64 = true;
      }
    }
    h->mx_large = mx_large;
    h->nbase = mixed ? (mx_large    ? (np / kk::MLargeCfg::BN) * kk::MLargeCfg::WAVES_N
                        : h->mx_tiny ? (np / MTinyCfg::BN) * MTinyCfg::WAVES_N
                                     : (np / kk::MSmallCfg::BN) * kk::MSmallCfg::WAVES_N)
                     : h->small_f64 ? (np / SmallF64::BN) * SmallF64::WAVES_N
                                    : (np / kk::BackCfg::BN) * kk::BackCfg::WAVES_N;
    h->nparts = h->kchb * h->nbase;
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
  a.n = np; a.k_half = h->kc; a.two_halves = 0; a.ntiles = h->n_store; a.tiles = h->tiles_store;
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
  ++h->prepare_gen;
  g_err.clear();
  return KK_OK;
}

}  // namespace

extern "C" {

kk_status kk_prepare(kk_handle h, int n_atoms, const int* atom_offsets, int n_basis, const double* S,
                     const double* Z, const double* Q_up, const double* Q_dn, const double* eps_up,
                     const double* eps_dn, const double* gamma, double W, double kT,
                     double n_electrons, int precision) {
  return prepare_impl(h, n_atoms, atom_offsets, n_basis, S, Z, Q_up, Q_dn, eps_up, eps_dn, gamma, W, kT,
                      n_electrons, precision, false);
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

kk_status enqueue_krylov(kk_handle h, const double* delta, int m, double tol, const double* K0, double* Kdelta);
kk_status krylov_graph(kk_handle h, const double* delta, int m, double tol, const double* K0, double* Kdelta);

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
  if (!h->profiling && !h->no_graph) {
    st = krylov_graph(h, delta, m, tol, K0, Kdelta);
    if (st == KK_EHIP && h->no_graph) st = enqueue_krylov(h, delta, m, tol, K0, Kdelta);  // capture refused
  } else {
    st = enqueue_krylov(h, delta, m, tol, K0, Kdelta);
  }
  if (st) return st;
  h->fwd_valid = true;
  h->fwd_m = m;
  h->fwd_K0 = K0;
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

// The launches of one update (Algorithm of Sec. II.E: precondition, m Krylov steps of
// orthonormalize / response / precondition, least-squares solve) on h->stream.
kk_status enqueue_krylov(kk_handle h, const double* delta, int m, double tol, const double* K0, double* Kdelta) {
  kk_status st;
  const int n2 = 2 * h->natoms;
  const int* stop = &h->kst->stop;
  const int gv_threads = 256, gv_blocks = (n2 * kk::WAVE + gv_threads - 1) / gv_threads;
  // orthonormalization: one block just large enough for 8 entries per thread
  const int orth_threads = std::max(64, std::min(1024, ((n2 + 7) / 8 + 63) / 64 * 64));

  // f~ = K0 delta (or -delta), and the Krylov state cleared, in one launch
  kk::precondition<<<gv_blocks, gv_threads, 0, h->stream>>>(K0, delta, nullptr, h->ftilde, n2, nullptr, h->kst);
  LAUNCH_CHECK("precondition");
  // Small systems: one launch orthonormalizes and builds the potentials (kk_fused.hpp), and
  // with K0 = -I the combine also preconditions.
  const bool fused = n2 <= kk::FUSED_MAX_N2;
  for (int k = 0; k < m; ++k) {
    const double* src = (k == 0) ? h->ftilde : h->Ft + (size_t)(k - 1) * n2;
    const double* vk = h->V + (size_t)k * n2;
    double* ftk = h->Ft + (size_t)k * n2;
    if (fused) {
      const bool split = h->precision != KK_FP64;
      kk::orth_potentials<<<(h->natoms + kk::FUSED_ATOMS - 1) / kk::FUSED_ATOMS, kk::FUSED_THREADS, 0,
                            h->stream>>>(src, h->V, n2, h->kst, k, h->gamma, h->natoms, h->W, h->offsets, h->np,
                                         h->u, split ? h->cvec : nullptr, split ? h->pmax : nullptr);
      LAUNCH_CHECK("orth_potentials");
      if ((st = response_any(h, 1, vk, h->q1, stop, false, true, K0 ? nullptr : vk, K0 ? nullptr : ftk)))
        return st;
    } else {
      kk::krylov_orthonormalize<<<1, orth_threads, 0, h->stream>>>(src, h->V, n2, h->kst);
      LAUNCH_CHECK("krylov_orthonormalize");
      if ((st = response_any(h, 1, vk, h->q1, stop))) return st;
    }
    if (!fused || K0 != nullptr) {
      kk::precondition<<<gv_blocks, gv_threads, 0, h->stream>>>(K0, h->q1, vk, ftk, n2, stop);
      LAUNCH_CHECK("precondition");
    }
    if (tol > 0.0 && k + 1 < m) {  // residual of the rank-(k+1) solve; may end the expansion
      kk::krylov_solve<<<1, 1024, 0, h->stream>>>(h->V, h->Ft, h->ftilde, n2, h->kst, Kdelta, tol);
      LAUNCH_CHECK("krylov_solve");
    }
  }
  kk::krylov_solve<<<1, 1024, 0, h->stream>>>(h->V, h->Ft, h->ftilde, n2, h->kst, Kdelta, 0.0);
  LAUNCH_CHECK("krylov_solve");
  return KK_OK;
}

// One update as a graph launch: capture on first use and whenever the key changes.
kk_status find_graph_args(kk_handle h, const double* delta, double* Kdelta);
kk_status set_graph_args(kk_handle h, const double* delta, double* Kdelta);

kk_status krylov_graph(kk_handle h, const double* delta, int m, double tol, const double* K0, double* Kdelta) {
  if (!h->gstream) HIP_OR_FAIL(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
  hipStream_t user = h->stream;
  // The graph bakes in buffer pointers and two prepared scalars (W and beta = 1/kT); a
  // prepare of the same shape rewrites the buffers in place, so it keeps the graph unless
  // one of those scalars changed.
  if (!h->gexec || h->g_K0 != K0 || h->g_m != m || h->g_tol != tol || h->g_gen != h->alloc_gen ||
      h->g_W != h->W || h->g_beta != h->beta) {
    // the last replay may still be running on the handle's stream: let it finish before its
    // exec goes
    HIP_OR_FAIL(hipStreamSynchronize(user));
    h->drop_graph();
    h->stream = h->gstream;
    hipError_t e = hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal);
    kk_status st = KK_OK;
    hipGraph_t g = nullptr;
    if (e == hipSuccess) {
      st = enqueue_krylov(h, delta, m, tol, K0, Kdelta);
      e = hipStreamEndCapture(h->gstream, &g);
    }
    h->stream = user;
    if (st || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      if (st) return st;
      h->no_graph = true;
      return fail(KK_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      h->no_graph = true;
      return fail(KK_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    h->graph = g;
    if ((st = find_graph_args(h, delta, Kdelta))) {
      h->drop_graph();
      h->no_graph = true;
      return st;
    }
    h->g_K0 = K0;
    h->g_m = m;
    h->g_tol = tol;
    h->g_gen = h->alloc_gen;
    h->g_W = h->W;
    h->g_beta = h->beta;
  }
  if (delta != h->g_delta || Kdelta != h->g_kd) {
    // an executable graph's node is not rewritten under a replay that may still run
    HIP_OR_FAIL(hipStreamSynchronize(user));
    kk_status st = set_graph_args(h, delta, Kdelta);
    if (st) return st;
  }
  HIP_OR_FAIL(hipGraphLaunch(h->gexec, user));
  return KK_OK;
}

// The kernel nodes of a freshly captured update that take the caller's pointers: the
// precondition whose input is delta (the first launch) and every krylov_solve, which
// writes K delta. Their arguments are kept so that set_graph_args can rebuild them.
kk_status find_graph_args(kk_handle h, const double* delta, double* Kdelta) {
  size_t n = 0;
  HIP_OR_FAIL(hipGraphGetNodes(h->graph, nullptr, &n));
  std::vector<hipGraphNode_t> nodes(n);
  HIP_OR_FAIL(hipGraphGetNodes(h->graph, nodes.data(), &n));
  int npre = 0;
  for (hipGraphNode_t nd : nodes) {
    hipGraphNodeType type;
    HIP_OR_FAIL(hipGraphNodeGetType(nd, &type));
    if (type != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams p{};
    HIP_OR_FAIL(hipGraphKernelNodeGetParams(nd, &p));
    if (p.kernelParams == nullptr) continue;
    if (p.func == reinterpret_cast<void*>(&kk::precondition)) {
      const kk::PreconditionArgs a = kk::PreconditionArgs::from(p.kernelParams);
      if (a.x != delta || a.reset == nullptr) continue;
      h->g_pre = {nd, p};
      h->g_pre_args = a;
      ++npre;
    } else if (p.func == reinterpret_cast<void*>(&kk::krylov_solve)) {
      const kk::SolveArgs a = kk::SolveArgs::from(p.kernelParams);
      if (a.out != Kdelta) continue;
      h->g_solve.push_back({nd, p});
      h->g_solve_args.push_back(a);
    }
  }
  if (npre != 1 || h->g_solve.empty())
    return fail(KK_EHIP, "graph: found %d input and %zu output nodes in the captured update", npre,
                h->g_solve.size());
  h->g_delta = delta;
  h->g_kd = Kdelta;
  return KK_OK;
}

kk_status set_graph_args(kk_handle h, const double* delta, double* Kdelta) {
  if (delta != h->g_delta) {
    kk::PreconditionArgs a = h->g_pre_args;
    a.x = delta;
    void* args[kk::PreconditionArgs::COUNT];
    a.pointers(args);
    hipKernelNodeParams p = h->g_pre.p;
    p.kernelParams = args;
    p.extra = nullptr;
    HIP_OR_FAIL(hipGraphExecKernelNodeSetParams(h->gexec, h->g_pre.node, &p));
    h->g_pre_args = a;
    h->g_delta = delta;
  }
  if (Kdelta != h->g_kd) {
    for (size_t i = 0; i < h->g_solve.size(); ++i) {
      kk::SolveArgs a = h->g_solve_args[i];
      a.out = Kdelta;
      void* args[kk::SolveArgs::COUNT];
      a.pointers(args);
      hipKernelNodeParams p = h->g_solve[i].p;
      p.kernelParams = args;
      p.extra = nullptr;
      HIP_OR_FAIL(hipGraphExecKernelNodeSetParams(h->gexec, h->g_solve[i].node, &p));
      h->g_solve_args[i] = a;
    }
    h->g_kd = Kdelta;
  }
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

// ===========================================================================
// Allocation-free update (krylov_kernel_apply_noalloc).
//
// The response workspace of one direction (potentials, Y or its split-precision
// operands, diag X, Mulliken partial rows) lives in a fixed device array instead of
// handle memory the library allocates on first use. Every GPU that loads the library
// holds its own copy of the array until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(96) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of this device's scratch array (looked up once per device).
kk_status scratch_for_current_device(void** out) {
  int dev = 0;
  HIP_OR_FAIL(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(KK_EINVAL, "device %d beyond the supported %d", dev, NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return fail(KK_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KK_OK;
}

// Carves the one-direction response workspace of h out of a scratch region of `cap`
// bytes (sub-buffers 256-byte aligned). With base = nullptr only the size is computed.
struct ScratchLayout {
  size_t bytes = 0;
  double *u = nullptr, *Y = nullptr, *xdiag = nullptr, *part = nullptr, *msc = nullptr;
  _Float16 *uct_h = nullptr, *uct_l = nullptr, *uct_r = nullptr, *yh = nullptr, *yl = nullptr, *yr = nullptr;
  float* x32 = nullptr;
};

ScratchLayout scratch_layout(kk_handle h, unsigned char* base) {
  ScratchLayout L;
  const size_t np = h->np, items = 2, np2 = np * np, kch = h->kch;
  auto take = [&](size_t nbytes) -> void* {
    void* p = base ? base + L.bytes : nullptr;
    L.bytes += (nbytes + 255) / 256 * 256;
    return p;
  };
  L.u = static_cast<double*>(take(items * np * sizeof(double)));
  if (h->precision == KK_FP64) {
    L.Y = static_cast<double*>(take(items * kch * np2 * sizeof(double)));
  } else {
    L.uct_h = static_cast<_Float16*>(take(items * np2 * sizeof(_Float16)));
    L.uct_l = static_cast<_Float16*>(take(items * np2 * sizeof(_Float16)));
    L.yh = static_cast<_Float16*>(take(items * np2 * sizeof(_Float16)));
    L.yl = static_cast<_Float16*>(take(items * np2 * sizeof(_Float16)));
    if (h->bf16) {
      L.uct_r = static_cast<_Float16*>(take(items * np2 * sizeof(_Float16)));
      L.yr = static_cast<_Float16*>(take(items * np2 * sizeof(_Float16)));
    }
    L.x32 = static_cast<float*>(take(items * kch * np2 * sizeof(float)));
    L.msc = static_cast<double*>(take(items * 8 * sizeof(double)));
  }
  L.xdiag = static_cast<double*>(take(items * np * sizeof(double)));
  L.part = static_cast<double*>(take(items * (size_t)h->nparts * np * sizeof(double)));
  return L;
}

}  // namespace

extern "C" {

kk_status krylov_kernel_apply_noalloc(kk_handle h, const double* delta, int m, const double* K0, double* Kdelta,
                                      kk_info* info) {
  const char* who = "krylov_kernel_apply_noalloc";
  kk_status st = check_handle(h);
  if (st) return st;
  const int n2 = 2 * h->natoms;
  if (!delta || !Kdelta) return fail(KK_EINVAL, "%s: NULL array argument", who);
  if (m < 1 || m > std::min(n2, kk::MAX_RANK))
    return fail(KK_EINVAL, "%s: need 1 <= m <= min(2N, %d), got %d", who, kk::MAX_RANK, m);
  const size_t need = scratch_layout(h, nullptr).bytes;
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(KK_EINVAL, "%s: this handle needs %zu bytes of scratch, above the fixed %zu (padded size %d)", who,
                need, NOALLOC_SCRATCH_BYTES, h->np);
  void* base = nullptr;
  if ((st = scratch_for_current_device(&base))) return st;
  const ScratchLayout L = scratch_layout(h, static_cast<unsigned char*>(base));

  // Point the handle's one-direction workspace at the scratch for this call only.
  struct Saved {
    int chunk_cap;
    double *u, *Y, *xdiag, *part, *msc;
    _Float16 *uct_h, *uct_l, *uct_r, *yh, *yl, *yr;
    float* x32;
  } sv{h->chunk_cap, h->u, h->Y, h->xdiag, h->part, h->msc, h->uct_h, h->uct_l, h->uct_r, h->yh, h->yl, h->yr,
       h->x32};
  h->chunk_cap = 1;
  h->u = L.u; h->Y = L.Y; h->xdiag = L.xdiag; h->part = L.part; h->msc = L.msc;
  h->uct_h = L.uct_h; h->uct_l = L.uct_l; h->uct_r = L.uct_r; h->yh = L.yh; h->yl = L.yl; h->yr = L.yr;
  h->x32 = L.x32;
  // the padded tail of the potentials must read zero; the scratch holds the last call's data
  st = zero(h, h->u, (size_t)2 * h->np);
  if (!st) st = enqueue_krylov(h, delta, m, 0.0, K0, Kdelta);
  h->chunk_cap = sv.chunk_cap;
  h->u = sv.u; h->Y = sv.Y; h->xdiag = sv.xdiag; h->part = sv.part; h->msc = sv.msc;
  h->uct_h = sv.uct_h; h->uct_l = sv.uct_l; h->uct_r = sv.uct_r; h->yh = sv.yh; h->yl = sv.yl; h->yr = sv.yr;
  h->x32 = sv.x32;
  if (st) return st;
  h->fwd_valid = true;
  h->fwd_m = m;
  h->fwd_K0 = K0;
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

}  // extern "C"

// ===========================================================================
// Reverse pass (differentiation form): kernels in kk_adjoint.hpp.

namespace {

// Mulliken partial rows per spin written by the FP64 back-transform of the reverse pass.
int adj_nparts(kk_handle h) { return (h->np / kk::BackCfg::BN) * kk::BackCfg::WAVES_N; }

// Reverse-pass workspace: the Krylov vectors always; the 12 padded matrices of the
// expansion-point part only once a call asks for dL/dH.
kk_status ensure_adjoint(kk_handle h, bool want_H) {
  const size_t np = h->np, np2 = np * np, n2 = 2 * (size_t)h->natoms;
  kk_status st;
  auto get = [&](double** p, size_t count) -> kk_status {
    void* q = nullptr;
    kk_status e = dalloc(h->adj_owned, &q, count * sizeof(double));
    *p = static_cast<double*>(q);
    return e;
  };
  if (want_H && !h->aX) {
    if ((st = get(&h->aX, 4 * np2))) return st;
    if ((st = get(&h->aY, 4 * np2))) return st;
    if ((st = get(&h->aK, 2 * np2))) return st;
    if ((st = get(&h->aD, 2 * np2))) return st;
  }
  if (h->ag) return KK_OK;
  if ((st = get(&h->au, 4 * np))) return st;
  if ((st = get(&h->axdiag, 4 * np))) return st;
  if ((st = get(&h->apart, 2 * (size_t)adj_nparts(h) * np))) return st;
  if ((st = get(&h->agdiag, 2 * np))) return st;
  if ((st = get(&h->admu, 2))) return st;
  if ((st = get(&h->agtot, 1))) return st;
  if ((st = get(&h->ag, n2))) return st;
  if ((st = get(&h->ay, n2))) return st;
  if ((st = get(&h->alam, n2))) return st;
  if ((st = get(&h->abbar, n2))) return st;
  if ((st = get(&h->aKd, n2))) return st;
  if ((st = get(&h->aVbar, kk::MAX_RANK * n2))) return st;
  if ((st = get(&h->aFbar, kk::MAX_RANK * n2))) return st;
  return KK_OK;
}

// Level pairs (i < j) of each spin closer than tau, from the prepared levels.
kk_status ensure_pairs(kk_handle h, double tau) {
  if (h->pairs_gen == h->prepare_gen) return KK_OK;
  const int nb = h->nb;
  std::vector<double> e(2 * (size_t)nb);
  HIP_OR_FAIL(hipMemcpyAsync(e.data(), h->eps[0], sizeof(double) * nb, hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(hipMemcpyAsync(e.data() + nb, h->eps[1], sizeof(double) * nb, hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  std::vector<int2> pairs;
  int counts[2] = {0, 0};
  constexpr size_t MAX_PAIRS = size_t(1) << 24;
  for (int s = 0; s < 2; ++s) {
    const double* es = e.data() + (size_t)s * nb;
    std::vector<int> idx(nb);
    for (int i = 0; i < nb; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return es[a] < es[b] || (es[a] == es[b] && a < b); });
    for (int p = 0; p < nb; ++p)
      for (int q = p + 1; q < nb && es[idx[q]] - es[idx[p]] < tau; ++q) {
        const int i = std::min(idx[p], idx[q]), j = std::max(idx[p], idx[q]);
        pairs.push_back(make_int2(i, j));
        ++counts[s];
        if (pairs.size() > MAX_PAIRS)
          return fail(KK_EINVAL, "krylov_kernel_adjoint: more than %zu near-degenerate level pairs", MAX_PAIRS);
      }
  }
  const int np_ = (int)pairs.size();
  if (np_ > h->pair_cap) {
    for (void* p : h->pair_owned) (void)hipFree(p);
    h->pair_owned.clear();
    h->apairs = nullptr;
    h->apk = nullptr;
    h->pair_cap = 0;
    void* q = nullptr;
    kk_status st;
    if ((st = dalloc(h->pair_owned, &q, sizeof(int2) * (size_t)np_))) return st;
    h->apairs = static_cast<int2*>(q);
    if ((st = dalloc(h->pair_owned, &q, sizeof(double) * (size_t)np_))) return st;
    h->apk = static_cast<double*>(q);
    h->pair_cap = np_;
  }
  if (np_ > 0) {
    HIP_OR_FAIL(hipMemcpyAsync(h->apairs, pairs.data(), sizeof(int2) * pairs.size(), hipMemcpyHostToDevice,
                               h->stream));
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));  // the host vector must outlive the copy
  }
  h->an0 = counts[0];
  h->an1 = counts[1];
  h->pairs_gen = h->prepare_gen;
  return KK_OK;
}

}  // namespace

extern "C" {

kk_status krylov_kernel_adjoint(kk_handle h, const double* delta, int m, const double* K0, const double* Kdelta_bar,
                                int reuse_forward, double* Kdelta, double* delta_bar, double* gamma_bar,
                                double* W_bar, double* H_bar_up, double* H_bar_dn, kk_info* info) {
  static const char* who = "krylov_kernel_adjoint";
  kk_status st = check_handle(h);
  if (st) return st;
  if (!delta || !Kdelta_bar || !delta_bar || !gamma_bar || !W_bar)
    return fail(KK_EINVAL, "%s: NULL array argument", who);
  if ((H_bar_up == nullptr) != (H_bar_dn == nullptr))
    return fail(KK_EINVAL, "%s: give both H_bar_up and H_bar_dn, or neither", who);
  const bool want_H = H_bar_up != nullptr;
  const int N = h->natoms, n2 = 2 * N, np = h->np, nb = h->nb;
  const size_t np2 = (size_t)np * np;
  if (m < 1 || m > std::min(n2, kk::MAX_RANK))
    return fail(KK_EINVAL, "%s: need 1 <= m <= min(2N, %d), got %d", who, kk::MAX_RANK, m);
  const double tau = 1e-3 * h->kT;

  if ((st = ensure_adjoint(h, want_H))) return st;
  if ((st = ensure_workspace(h, 1))) return st;
  // forward expansion: recomputed, or the one the last kernel call left
  if (reuse_forward) {
    if (!h->fwd_valid || h->fwd_m != m || h->fwd_K0 != K0)
      return fail(KK_EINVAL, "%s: reuse_forward needs the last kernel call on this handle to have used the same "
                             "m and K0", who);
  } else {
    kk_info fi;
    if ((st = krylov_run(h, who, delta, m, 0.0, K0, Kdelta ? Kdelta : h->aKd, &fi)) < 0) return st;
  }
  kk::KrylovState hs;
  HIP_OR_FAIL(hipMemcpyAsync(&hs, h->kst, sizeof hs, hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  if (hs.status == KK_ESINGULAR) return fail(KK_ESINGULAR, "%s: Gram matrix not positive definite", who);
  if (want_H && (st = ensure_pairs(h, tau))) return st;
  const int r = hs.rank;
  const int npairs = want_H ? h->an0 + h->an1 : 0;

  if (want_H) {
    if ((st = zero(h, h->aK, 2 * np2))) return st;
    if ((st = zero(h, h->aD, 2 * np2))) return st;
    if ((st = zero(h, h->agdiag, 2 * (size_t)np))) return st;
    if (npairs > 0 && (st = zero(h, h->apk, npairs))) return st;
  }
  if ((st = zero(h, gamma_bar, (size_t)N * N))) return st;
  if ((st = zero(h, W_bar, 1))) return st;

  kk::adj_init<<<1, 1024, 0, h->stream>>>(h->V, h->Ft, h->ftilde, n2, h->kst, Kdelta_bar, h->aVbar, h->aFbar,
                                          h->abbar);
  LAUNCH_CHECK("adj_init");

  kk::AdjSpins sp{};
  for (int s = 0; s < 2; ++s) {
    sp.s[s].Xa = h->aX + (size_t)s * np2;
    sp.s[s].Xb = h->aX + (size_t)(2 + s) * np2;
    sp.s[s].eps = h->eps[s]; sp.s[s].f = h->f[s]; sp.s[s].fc = h->fc[s]; sp.s[s].w = h->w[s];
    sp.s[s].D = h->aD + (size_t)s * np2;
    sp.s[s].gdiag = h->agdiag + (size_t)s * np;
  }
  const int wave_blocks = (N * kk::WAVE + 255) / 256;
  for (int k = r - 1; k >= 0; --k) {
    const double* vk = h->V + (size_t)k * n2;
    // lambda_k and y_k = K0^T lambda_k
    kk::adj_gs<<<1, 1024, 0, h->stream>>>(h->V, h->Ft, n2, k, k == r - 1, h->aVbar, h->aFbar,
                                          K0 ? h->alam : h->ay, K0 ? 0 : 1);
    LAUNCH_CHECK("adj_gs");
    if (K0) {
      kk::gemv_t<<<(n2 + 255) / 256, 256, 0, h->stream>>>(K0, h->alam, n2, h->ay);
      LAUNCH_CHECK("gemv_t");
    }
    if (!want_H) {
      // only g = M chi M y is needed: one response with identity coupling, in the handle's precision
      if ((st = response_any(h, 1, h->ay, h->ag, nullptr, true))) return st;
      kk::adj_apply<<<wave_blocks, 256, 0, h->stream>>>(h->gamma, N, h->W, h->ag, h->ay, vk,
                                                         h->aVbar + (size_t)k * n2, gamma_bar);
      LAUNCH_CHECK("adj_apply");
      kk::adj_wbar<<<1, 256, 0, h->stream>>>(h->ag, vk, N, W_bar);
      LAUNCH_CHECK("adj_wbar");
      continue;
    }
    // potentials: a = M y (identity coupling), b = M Gamma v_k
    kk::potentials<<<wave_blocks, 256, 0, h->stream>>>(nullptr, N, 1.0, h->ay, 1, h->offsets, np, h->au, nullptr);
    kk::potentials<<<wave_blocks, 256, 0, h->stream>>>(h->gamma, N, h->W, vk, 1, h->offsets, np, h->au + 2 * np,
                                                        nullptr);
    LAUNCH_CHECK("potentials");
    // X and Y0 of the four items (a up, a dn, b up, b dn)
    kk::GemmArgs fa{};
    fa.n = np; fa.k_half = np; fa.two_halves = 1; fa.ntiles = h->n_upper; fa.nitems = 4;
    fa.tiles = h->tiles_upper; fa.beta = h->beta;
    for (int z = 0; z < 4; ++z) {
      const int s = z & 1;
      kk::GemmItem& it = fa.item[z];
      it.a0 = h->C[s]; it.b0 = h->G[s]; it.a1 = h->G[s]; it.b1 = h->C[s];
      it.scale = h->au + (size_t)z * np; it.out = h->aY + (size_t)z * np2; it.xout = h->aX + (size_t)z * np2;
      it.eps = h->eps[s]; it.f = h->f[s]; it.fc = h->fc[s]; it.w = h->w[s];
      it.xdiag = h->axdiag + (size_t)z * np;
    }
    if ((st = launch_gemm(h, kk::EPI_FERMI_XY, fa))) return st;
    // g = M chi M y: back-transform and Mulliken sums of the a items
    kk::GemmArgs ba{};
    ba.n = np; ba.k_half = np; ba.two_halves = 0; ba.ntiles = h->n_full; ba.nitems = 2;
    ba.tiles = h->tiles_full; ba.beta = h->beta;
    for (int s = 0; s < 2; ++s) {
      kk::GemmItem& it = ba.item[s];
      it.a0 = h->CT[s]; it.b0 = h->aY + (size_t)s * np2; it.g = h->G[s];
      it.part = h->apart + (size_t)s * adj_nparts(h) * np;
    }
    if ((st = launch_gemm(h, kk::EPI_MULLIKEN, ba))) return st;
    {
      dim3 grid((N + kk::COMBINE_ATOMS - 1) / kk::COMBINE_ATOMS, 1);
      kk::combine<<<grid, kk::COMBINE_THREADS, 0, h->stream>>>(h->axdiag, h->apart, adj_nparts(h), h->w[0], h->w[1],
                                                              h->wsum, h->t,
                                                nb, np, h->offsets, N, h->ag, nullptr);
      LAUNCH_CHECK("combine");
    }
    kk::adj_dmu<<<2, 1024, 0, h->stream>>>(h->axdiag, nb, np, h->w[0], h->w[1], h->wsum, h->admu);
    LAUNCH_CHECK("adj_dmu");
    // K += Y0_b Xa + Y0_a Xb per spin
    kk::GemmArgs ka{};
    ka.n = np; ka.k_half = np; ka.two_halves = 1; ka.ntiles = h->n_full; ka.nitems = 2;
    ka.tiles = h->tiles_full; ka.beta = h->beta;
    for (int s = 0; s < 2; ++s) {
      kk::GemmItem& it = ka.item[s];
      it.a0 = h->aY + (size_t)(2 + s) * np2; it.b0 = h->aX + (size_t)s * np2;
      it.a1 = h->aY + (size_t)s * np2; it.b1 = h->aX + (size_t)(2 + s) * np2;
      it.out = h->aK + (size_t)s * np2;
    }
    if ((st = launch_gemm(h, kk::EPI_ACCUM, ka))) return st;
    {
      dim3 grid(nb, 2);
      kk::adj_rows<<<grid, 256, 0, h->stream>>>(sp, nb, np, h->admu, h->mu, h->beta, tau);
      LAUNCH_CHECK("adj_rows");
    }
    if (npairs > 0) {
      kk::adj_pairs<<<npairs, 256, 0, h->stream>>>(sp, h->apairs, h->an0, nb, np, h->mu, h->beta, tau, h->apk);
      LAUNCH_CHECK("adj_pairs");
    }
    kk::adj_apply<<<wave_blocks, 256, 0, h->stream>>>(h->gamma, N, h->W, h->ag, h->ay, vk,
                                                       h->aVbar + (size_t)k * n2, gamma_bar);
    LAUNCH_CHECK("adj_apply");
    kk::adj_wbar<<<1, 256, 0, h->stream>>>(h->ag, vk, N, W_bar);
    LAUNCH_CHECK("adj_wbar");
  }
  // dL/d delta
  if (r > 0) {
    kk::adj_finish<<<1, 1024, 0, h->stream>>>(h->V, h->aVbar, h->ftilde, n2, h->abbar, K0 ? h->alam : delta_bar,
                                              K0 ? 0 : 1);
    LAUNCH_CHECK("adj_finish");
    if (K0) {
      kk::gemv_t<<<(n2 + 255) / 256, 256, 0, h->stream>>>(K0, h->alam, n2, delta_bar);
      LAUNCH_CHECK("gemv_t");
    }
  } else if ((st = zero(h, delta_bar, n2))) {
    return st;
  }
  if (!want_H) {
    if (info) {
      HIP_OR_FAIL(hipStreamSynchronize(h->stream));
      info->rank_used = hs.rank;
      info->status = hs.status;
      info->min_pivot = hs.min_pivot;
      info->max_pivot = hs.max_pivot;
      info->ls_residual = hs.ls_residual;
    }
    g_err.clear();
    return hs.status == 1 ? KK_BREAKDOWN : KK_OK;
  }
  // dL/dH^sigma = C E'_bar C^T
  kk::sum_two<<<1, 1024, 0, h->stream>>>(h->agdiag, h->agdiag + np, np, h->agtot);
  LAUNCH_CHECK("sum_two");
  double* Ep[2] = {h->aX, h->aX + np2};
  for (int s = 0; s < 2; ++s) {
    dim3 grid(np / 32, np / 32);
    kk::adj_final<<<grid, 256, 0, h->stream>>>(h->aK + (size_t)s * np2, h->aD + (size_t)s * np2, h->eps[s],
                                                h->w[s], h->agdiag + (size_t)s * np, h->agtot, h->wsum, nb, np, tau,
                                                Ep[s]);
    LAUNCH_CHECK("adj_final");
  }
  if (npairs > 0) {
    kk::adj_pair_final<<<(npairs + 255) / 256, 256, 0, h->stream>>>(h->apairs, h->an0, npairs, h->apk, h->aD,
                                                                     h->aD + np2, h->eps[0], h->eps[1], h->mu,
                                                                     h->beta, np, Ep[0], Ep[1]);
    LAUNCH_CHECK("adj_pair_final");
  }
  kk::GemmArgs a{};
  a.n = np; a.k_half = np; a.two_halves = 0; a.ntiles = h->n_store; a.tiles = h->tiles_store; a.nitems = 2;
  for (int s = 0; s < 2; ++s) {  // U1 = E'_bar C^T
    a.item[s] = kk::GemmItem{};
    a.item[s].a0 = Ep[s]; a.item[s].b0 = h->CT[s]; a.item[s].out = h->aY + (size_t)s * np2;
  }
  if ((st = launch_gemm(h, kk::EPI_STORE, a))) return st;
  for (int s = 0; s < 2; ++s) {  // C U1
    a.item[s] = kk::GemmItem{};
    a.item[s].a0 = h->CT[s]; a.item[s].b0 = h->aY + (size_t)s * np2; a.item[s].out = h->aY + (size_t)(2 + s) * np2;
  }
  if ((st = launch_gemm(h, kk::EPI_STORE, a))) return st;
  double* Hb[2] = {H_bar_up, H_bar_dn};
  for (int s = 0; s < 2; ++s) {
    const int blocks = (int)std::min<size_t>(((size_t)nb * nb + 255) / 256, 65536);
    kk::unpad_copy<<<blocks, 256, 0, h->stream>>>(h->aY + (size_t)(2 + s) * np2, np, Hb[s], nb);
    LAUNCH_CHECK("unpad_copy");
  }
  if (info) {
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    info->rank_used = hs.rank;
    info->status = hs.status;
    info->min_pivot = hs.min_pivot;
    info->max_pivot = hs.max_pivot;
    info->ls_residual = hs.ls_residual;
  }
  g_err.clear();
  return hs.status == 1 ? KK_BREAKDOWN : KK_OK;
}

}  // extern "C"

// ===========================================================================
// Batched form: many independent systems, one graph launch per update.

#include "kk_batch.hpp"

namespace {

// Tile configurations a batch chooses between: large systems use the default
// transforms, systems with np <= small_np_max use 64 x 64 tiles.

struct TileClass {  // full-tile list of one tile class, shared by both transforms
  int4* tiles = nullptr;
  int n = 0;
};

}  // namespace

struct kk_batch_s {
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;  // private stream (a capturable, non-null stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int ns = 0, precision = KK_FP64, maxN = 0, max_np = 0;
  bool prepared = false;
  std::vector<kk_handle> sys;
  std::vector<void*> owned;
  kk::SysDesc* d_sys = nullptr;
  void* d_items_fwd = nullptr;   // BatchItemF64 or BatchItemMixed, 2 per system
  void* d_items_back = nullptr;
  int* d_pair_off = nullptr;     // first symmetrizing block pair of each forward item
  int sym_pairs = 0;             // block pairs over all forward items
  TileClass cls[2];              // 0: large tiles, 1: small tiles
  const double** d_delta = nullptr;
  double** d_out = nullptr;
  kk::KrylovState* d_info = nullptr;
  std::vector<const double*> h_delta;
  std::vector<double*> h_out;
  std::vector<int> np_of;
  std::vector<kk::SysDesc> h_sys;   // host copy of the descriptors (nparts depends on the tile class)
  std::vector<int> parts_large, parts_small;
  // tuning state
  int small_np_max = 0, grid_mult = 2;
  bool tuned = false;
  double tuned_ms = 0.0;
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_m = -1;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    graph_m = -1;
  }
  void release() {
    if (stream) (void)hipStreamSynchronize(stream);
    drop_graph();
    for (kk_handle h : sys) kk_destroy(h);
    sys.clear();
    for (void* p : owned) (void)hipFree(p);
    owned.clear();
    for (auto& c : cls) c = TileClass{};
    d_sys = nullptr; d_items_fwd = d_items_back = nullptr; d_delta = nullptr; d_out = nullptr; d_info = nullptr;
    d_pair_off = nullptr;
    sym_pairs = 0;
    prepared = false;
    tuned = false;
  }
};

namespace {

template <typename T>
kk_status balloc(kk_batch b, T** p, size_t count) {
  void* q = nullptr;
  kk_status st = dalloc(b->owned, &q, count * sizeof(T));
  *p = static_cast<T*>(q);
  return st;
}

// Build the tile lists of both classes for a threshold: items (2 per system)
// sorted by decreasing np so the persistent workgroups start with the costly tiles.
// Both transforms walk the full tiles (the forward as the product A = C^T U~ G).
kk_status build_tile_lists(kk_batch b, int small_np_max) {
  const bool mixed = b->precision == KK_MIXED_F16;
  std::vector<int> order(b->ns);
  for (int i = 0; i < b->ns; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->np_of[x] > b->np_of[y]; });
  std::vector<int4> lists[2];
  for (int i : order) {
    const int np = b->np_of[i];
    const int c = np <= small_np_max ? 1 : 0;
    int bm, bn, sbm, sbn;
    if (mixed) { bm = kk::MLargeCfg::BM; bn = kk::MLargeCfg::BN; sbm = SmallMx::BM; sbn = SmallMx::BN; }
    else { bm = kk::BackCfg::BM; bn = kk::BackCfg::BN; sbm = SmallF64::BM; sbn = SmallF64::BN; }
    const int tbm = c ? sbm : bm, tbn = c ? sbn : bn;
    for (int s = 0; s < 2; ++s) {
      const int item = 2 * i + s;
      for (const int2& t : tile_order(np, tbm, tbn, false)) lists[c].push_back(make_int4(item, t.x, t.y, 0));
    }
  }
  for (int i = 0; i < b->ns; ++i)
    b->h_sys[i].nparts = b->np_of[i] <= small_np_max ? b->parts_small[i] : b->parts_large[i];
  HIP_OR_FAIL(hipMemcpyAsync(b->d_sys, b->h_sys.data(), sizeof(kk::SysDesc) * b->ns, hipMemcpyHostToDevice,
                             b->stream));
  for (int c = 0; c < 2; ++c) {
    TileClass& tc = b->cls[c];
    tc.n = (int)lists[c].size();
    if (!tc.tiles) {  // capacity for every system in either class: the larger per-system count (small tiles)
      size_t cap = 0;
      for (int i = 0; i < b->ns; ++i) {
        const int np = b->np_of[i];
        const int sb = mixed ? SmallMx::BM : SmallF64::BM;
        cap += 2 * (size_t)(np / sb) * (np / sb);
      }
      kk_status st;
      if ((st = balloc(b, &tc.tiles, cap + 1))) return st;
    }
    if (tc.n)
      HIP_OR_FAIL(hipMemcpyAsync(tc.tiles, lists[c].data(), sizeof(int4) * tc.n, hipMemcpyHostToDevice, b->stream));
  }
  HIP_OR_FAIL(hipStreamSynchronize(b->stream));
  return KK_OK;
}

template <int EPI, class Cfg, class Item>
kk_status launch_persistent(kk_batch b, const Item* items, const int4* tiles, int ntiles, int two_halves) {
  if (ntiles == 0) return KK_OK;
  const int grid = std::min(ntiles, cu_count() * b->grid_mult);
  if constexpr (std::is_same<Item, kk::BatchItemF64>::value)
    kk::b_gemm_f64<EPI, Cfg><<<grid, Cfg::THREADS, 0, b->stream>>>(items, tiles, ntiles, two_halves);
  else
    kk::b_gemm_mixed<EPI, Cfg><<<grid, Cfg::THREADS, 0, b->stream>>>(items, tiles, ntiles, two_halves);
  LAUNCH_CHECK("b_gemm");
  return KK_OK;
}

// Every kernel of one batched rank-m update, in order, on the private stream.
kk_status enqueue_update(kk_batch b, int m) {
  const int ns = b->ns;
  const int bx_vec = (2 * b->maxN + 255) / 256;
  kk::b_reset<<<ns, 64, 0, b->stream>>>(b->d_sys);
  LAUNCH_CHECK("b_reset");
  kk::b_init<<<dim3(bx_vec, ns), 256, 0, b->stream>>>(b->d_sys, b->d_delta);
  LAUNCH_CHECK("b_init");
  const bool mixed = b->precision == KK_MIXED_F16;
  kk_status st;
  for (int k = 0; k < m; ++k) {
    kk::b_orth<<<ns, 1024, 0, b->stream>>>(b->d_sys, k);
    LAUNCH_CHECK("b_orth");
    kk::b_potentials<<<dim3((b->maxN * kk::WAVE + 255) / 256, ns), 256, 0, b->stream>>>(b->d_sys, k);
    LAUNCH_CHECK("b_potentials");
    if (mixed) {
      kk::b_center<<<ns, 1024, 0, b->stream>>>(b->d_sys);
      LAUNCH_CHECK("b_center");
      kk::b_mixed_scales<<<dim3(2, ns), 1024, 0, b->stream>>>(b->d_sys);
      LAUNCH_CHECK("b_mixed_scales");
      const size_t np2 = (size_t)b->max_np * b->max_np;
// Workgroups per (system, spin), sized for the largest system; they stride over their
// system's rows. Most systems of a batch are smaller, and their surplus workgroups exit at
// once: a cap of 128 ran the 64-cluster batch 1.5 % faster than 2048 (512: level with 128,
// 32: slower).
#ifndef KK_BSPLIT_CAP
#define KK_BSPLIT_CAP 128
#endif
      const int blocks = (int)std::min<size_t>((np2 / 8 + 255) / 256, KK_BSPLIT_CAP);
      kk::b_split<<<dim3(blocks, 2, ns), 256, 0, b->stream>>>(b->d_sys);
      LAUNCH_CHECK("b_split");
      auto* fi = static_cast<const kk::BatchItemMixed*>(b->d_items_fwd);
      auto* bi = static_cast<const kk::BatchItemMixed*>(b->d_items_back);
      // forward: full-tile products A = C^T U~ G (the back-transform's tile lists), then
      // one symmetrizing pass over all items
      if ((st = launch_persistent<kk::EPI_STORE, kk::MLargeCfg>(b, fi, b->cls[0].tiles, b->cls[0].n, 0)))
        return st;
      if ((st = launch_persistent<kk::EPI_STORE, SmallMx>(b, fi, b->cls[1].tiles, b->cls[1].n, 0))) return st;
      kk::b_symmetrize<<<b->sym_pairs, kk::BATCH_SYM_T_MIXED, 0, b->stream>>>(fi, b->d_pair_off, 2 * ns);
      LAUNCH_CHECK("b_symmetrize");
      if ((st = launch_persistent<kk::EPI_MULLIKEN, kk::MLargeCfg>(b, bi, b->cls[0].tiles, b->cls[0].n, 0)))
        return st;
      if ((st = launch_persistent<kk::EPI_MULLIKEN, SmallMx>(b, bi, b->cls[1].tiles, b->cls[1].n, 0)))
        return st;
    } else {
      auto* fi = static_cast<const kk::BatchItemF64*>(b->d_items_fwd);
      auto* bi = static_cast<const kk::BatchItemF64*>(b->d_items_back);
      // forward: full-tile products A = C^T U~ G into Y, then one in-place symmetrizing pass
      if ((st = launch_persistent<kk::EPI_XSTORE, kk::BackCfg>(b, fi, b->cls[0].tiles, b->cls[0].n, 0)))
        return st;
      if ((st = launch_persistent<kk::EPI_XSTORE, SmallF64>(b, fi, b->cls[1].tiles, b->cls[1].n, 0))) return st;
      kk::b_symmetrize_f64<<<b->sym_pairs, kk::BATCH_SYM_T_F64, 0, b->stream>>>(fi, b->d_pair_off, 2 * ns);
      LAUNCH_CHECK("b_symmetrize_f64");
      if ((st = launch_persistent<kk::EPI_MULLIKEN, kk::BackCfg>(b, bi, b->cls[0].tiles, b->cls[0].n, 0)))
        return st;
      if ((st = launch_persistent<kk::EPI_MULLIKEN, SmallF64>(b, bi, b->cls[1].tiles, b->cls[1].n, 0)))
        return st;
    }
    kk::b_combine<<<dim3((b->maxN + kk::COMBINE_ATOMS - 1) / kk::COMBINE_ATOMS, ns), kk::COMBINE_THREADS, 0,
                    b->stream>>>(b->d_sys);
    LAUNCH_CHECK("b_combine");
    kk::b_precond<<<dim3(bx_vec, ns), 256, 0, b->stream>>>(b->d_sys, k);
    LAUNCH_CHECK("b_precond");
  }
  kk::b_solve<<<ns, 1024, 0, b->stream>>>(b->d_sys, b->d_out);
  LAUNCH_CHECK("b_solve");
  kk::b_info<<<(ns + 255) / 256, 256, 0, b->stream>>>(b->d_sys, ns, b->d_info);
  LAUNCH_CHECK("b_info");
  return KK_OK;
}

kk_status upload_pointer_tables(kk_batch b, const double* const* delta, double* const* out) {
  for (int i = 0; i < b->ns; ++i) {
    b->h_delta[i] = delta[i];
    b->h_out[i] = out[i];
  }
  HIP_OR_FAIL(hipMemcpyAsync(b->d_delta, b->h_delta.data(), sizeof(double*) * b->ns, hipMemcpyHostToDevice,
                             b->stream));
  HIP_OR_FAIL(hipMemcpyAsync(b->d_out, b->h_out.data(), sizeof(double*) * b->ns, hipMemcpyHostToDevice,
                             b->stream));
  return KK_OK;
}

// Autotuner: time one update for every (small-tile threshold, workgroups per CU)
// candidate on the batch's own systems and keep the fastest.
kk_status autotune(kk_batch b, int m) {
  const int thresholds[] = {0, 512, 1024, 1 << 30};
  const int mults[] = {1, 2, 4};
  hipEvent_t e0, e1;
  HIP_OR_FAIL(hipEventCreate(&e0));
  HIP_OR_FAIL(hipEventCreate(&e1));
  double best = 1e300;
  int best_t = 0, best_m = 2;
  kk_status st = KK_OK;
  for (int th : thresholds) {
    if ((st = build_tile_lists(b, th))) break;
    for (int gm : mults) {
      b->grid_mult = gm;
      if ((st = enqueue_update(b, m))) break;  // warm-up
      (void)hipEventRecord(e0, b->stream);
      if ((st = enqueue_update(b, m))) break;
      (void)hipEventRecord(e1, b->stream);
      if (hipEventSynchronize(e1) != hipSuccess) { st = fail(KK_EHIP, "autotune: event sync failed"); break; }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) { best = ms; best_t = th; best_m = gm; }
    }
    if (st) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  b->small_np_max = best_t;
  b->grid_mult = best_m;
  b->tuned_ms = best;
  b->tuned = true;
  return build_tile_lists(b, best_t);
}

}  // namespace

extern "C" {

kk_status kk_batch_create(kk_batch* b, void* hip_stream) {
  if (!b) return fail(KK_EINVAL, "kk_batch_create: output pointer is NULL");
  *b = new (std::nothrow) kk_batch_s();
  if (!*b) return fail(KK_ENOMEM, "kk_batch_create: out of host memory");
  (*b)->user_stream = static_cast<hipStream_t>(hip_stream);
  g_err.clear();
  return KK_OK;
}

kk_status kk_batch_destroy(kk_batch b) {
  if (!b) return fail(KK_EINVAL, "kk_batch_destroy: batch is NULL");
  b->release();
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return KK_OK;
}

kk_status kk_batch_prepare(kk_batch b, int n_systems, const int* n_atoms, const int* const* atom_offsets,
                           const double* const* S, const double* const* Z, const double* const* Q_up,
                           const double* const* Q_dn, const double* const* eps_up, const double* const* eps_dn,
                           const double* const* gamma, const double* W, const double* kT,
                           const double* n_electrons, int precision) {
  if (!b) return fail(KK_EINVAL, "kk_batch_prepare: batch is NULL");
  if (n_systems < 1 || n_systems > 4096) return fail(KK_EINVAL, "kk_batch_prepare: need 1 <= n_systems <= 4096");
  if (precision != KK_FP64 && precision != KK_MIXED_F16)
    return fail(KK_EINVAL, "kk_batch_prepare: precision %d is not supported in batches (KK_FP64, KK_MIXED_F16)",
                precision);
  if (!n_atoms || !atom_offsets || !S || !Z || !Q_up || !Q_dn || !eps_up || !eps_dn || !gamma || !W || !kT ||
      !n_electrons)
    return fail(KK_EINVAL, "kk_batch_prepare: NULL array argument");
  b->release();
  if (!b->stream) {
    HIP_OR_FAIL(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    HIP_OR_FAIL(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    HIP_OR_FAIL(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
  }
  // inputs are the caller's: wait for its stream before reading them
  HIP_OR_FAIL(hipEventRecord(b->ev_in, b->user_stream));
  HIP_OR_FAIL(hipStreamWaitEvent(b->stream, b->ev_in, 0));
  b->ns = n_systems;
  b->precision = precision;
  b->maxN = 0;
  b->max_np = 0;
  b->np_of.assign(n_systems, 0);
  kk_status st;
  for (int i = 0; i < n_systems; ++i) {
    kk_handle h = nullptr;
    if ((st = kk_create(&h, b->stream))) return st;
    b->sys.push_back(h);
    const int nb = n_atoms[i] >= 1 && atom_offsets[i] ? atom_offsets[i][n_atoms[i]] : 0;
    if ((st = prepare_impl(h, n_atoms[i], atom_offsets[i], nb, S[i], Z[i], Q_up[i], Q_dn[i], eps_up[i],
                           eps_dn[i], gamma[i], W[i], kT[i], n_electrons[i], precision, true))) {
      char buf[600];
      snprintf(buf, sizeof buf, "system %d: %s", i, g_err.c_str());
      return fail(st, "kk_batch_prepare: %s", buf);
    }
    if ((st = ensure_workspace(h, 1))) return st;
    b->maxN = std::max(b->maxN, h->natoms);
    b->max_np = std::max(b->max_np, h->np);
    b->np_of[i] = h->np;
  }
  // device descriptors
  const bool mixed = precision == KK_MIXED_F16;
  std::vector<kk::SysDesc>& sd = b->h_sys;
  sd.assign(n_systems, kk::SysDesc{});
  b->parts_large.assign(n_systems, 0);
  b->parts_small.assign(n_systems, 0);
  std::vector<kk::BatchItemF64> f64f, f64b;
  std::vector<kk::BatchItemMixed> mxf, mxb;
  for (int i = 0; i < n_systems; ++i) {
    kk_handle h = b->sys[i];
    const size_t np = h->np, np2 = np * np;
    // Mulliken partial rows: one per wave column of a tile column, for either tile class
    b->parts_large[i] = mixed ? (h->np / kk::MLargeCfg::BN) * kk::MLargeCfg::WAVES_N
                              : (h->np / kk::BackCfg::BN) * kk::BackCfg::WAVES_N;
    b->parts_small[i] = mixed ? (h->np / SmallMx::BN) * SmallMx::WAVES_N
                              : (h->np / SmallF64::BN) * SmallF64::WAVES_N;
    const int part_rows = std::max(b->parts_large[i], b->parts_small[i]);
    double* part = nullptr;
    if ((st = balloc(b, &part, (size_t)2 * part_rows * np))) return st;
    kk::SysDesc& d = sd[i];
    d.natoms = h->natoms; d.nb = h->nb; d.np = h->np; d.nparts = b->parts_large[i]; d.part_stride = part_rows;
    d.W = h->W; d.beta = h->beta; d.offsets = h->offsets; d.gamma = h->gamma;
    d.u = h->u; d.xdiag = h->xdiag; d.part = part;
    d.w0 = h->w[0]; d.w1 = h->w[1]; d.wsum = h->wsum; d.t = h->t;
    d.V = h->V; d.Ft = h->Ft; d.ftilde = h->ftilde; d.q1 = h->q1; d.kst = h->kst;
    d.msc = h->msc; d.mconst = h->mconst;
    d.CT0 = h->CT[0]; d.CT1 = h->CT[1];
    d.uct_h = h->uct_h; d.uct_l = h->uct_l;
    for (int s = 0; s < 2; ++s) {
      if (mixed) {
        kk::BatchItemMixed fi{}, bi{};
        fi.n = bi.n = h->np; fi.k = bi.k = h->kc; fi.beta = bi.beta = h->beta; fi.stop = bi.stop = &h->kst->stop;
        kk::MixedItem& F = fi.g;
        F.a0h = h->uct_h + s * np2; F.a0l = h->uct_l + s * np2; F.b0h = h->GTh[s]; F.b0l = h->GTl[s];
        F.yh = h->yh + s * np2; F.yl = h->yl + s * np2; F.x32 = h->x32 + s * np2;
        F.eps = h->eps[s]; F.f = h->f[s]; F.fc = h->fc[s]; F.w = h->w[s];
        F.xdiag = h->xdiag + s * np; F.sc = h->msc + s * 8;
        kk::MixedItem& B = bi.g;
        B.a0h = h->Ch[s]; B.a0l = h->Cl[s]; B.b0h = h->yh + s * np2; B.b0l = h->yl + s * np2;
        B.g = h->G[s]; B.part = part + (size_t)s * part_rows * np; B.sc = h->msc + s * 8 + 2;
        mxf.push_back(fi);
        mxb.push_back(bi);
      } else {
        kk::BatchItemF64 fi{}, bi{};
        fi.n = bi.n = h->np; fi.k = bi.k = h->kc; fi.beta = bi.beta = h->beta; fi.stop = bi.stop = &h->kst->stop;
        kk::GemmItem& F = fi.g;
        F.a0 = h->C[s]; F.b0 = h->G[s]; F.a1 = h->G[s]; F.b1 = h->C[s];
        F.scale = h->u + s * np; F.out = h->Y + s * np2;
        F.eps = h->eps[s]; F.f = h->f[s]; F.fc = h->fc[s]; F.w = h->w[s]; F.xdiag = h->xdiag + s * np;
        kk::GemmItem& B = bi.g;
        B.a0 = h->CT[s]; B.b0 = h->Y + s * np2; B.g = h->G[s]; B.part = part + (size_t)s * part_rows * np;
        f64f.push_back(fi);
        f64b.push_back(bi);
      }
    }
  }
  if ((st = balloc(b, &b->d_sys, n_systems))) return st;
  HIP_OR_FAIL(hipMemcpyAsync(b->d_sys, sd.data(), sizeof(kk::SysDesc) * n_systems, hipMemcpyHostToDevice, b->stream));
  // symmetrizing block pairs of the forward items (2 per system, spin fastest); the
  // offsets index one launch's blocks, so their total must fit an int
  std::vector<int> pair_off(1, 0);
  long long total_pairs = 0;
  const int bsym = mixed ? kk::BATCH_SYM_B_MIXED : kk::BATCH_SYM_B_F64;
  for (int i = 0; i < n_systems; ++i)
    for (int s = 0; s < 2; ++s) {
      if (b->sys[i]->np % bsym != 0) return fail(KK_EINVAL, "internal: padded size not a multiple of the block pairs");
      const long long nblk = b->sys[i]->np / bsym;
      total_pairs += nblk * (nblk + 1) / 2;
      if (total_pairs > INT_MAX) return fail(KK_EINVAL, "kk_batch_prepare: too many block pairs in one batch");
      pair_off.push_back((int)total_pairs);
    }
  b->sym_pairs = pair_off.back();
  if ((st = balloc(b, &b->d_pair_off, pair_off.size()))) return st;
  HIP_OR_FAIL(hipMemcpyAsync(b->d_pair_off, pair_off.data(), sizeof(int) * pair_off.size(), hipMemcpyHostToDevice,
                             b->stream));
  if (mixed) {
    kk::BatchItemMixed *f, *bk;
    if ((st = balloc(b, &f, mxf.size()))) return st;
    if ((st = balloc(b, &bk, mxb.size()))) return st;
    HIP_OR_FAIL(hipMemcpyAsync(f, mxf.data(), sizeof(kk::BatchItemMixed) * mxf.size(), hipMemcpyHostToDevice, b->stream));
    HIP_OR_FAIL(hipMemcpyAsync(bk, mxb.data(), sizeof(kk::BatchItemMixed) * mxb.size(), hipMemcpyHostToDevice, b->stream));
    b->d_items_fwd = f;
    b->d_items_back = bk;
  } else {
    kk::BatchItemF64 *f, *bk;
    if ((st = balloc(b, &f, f64f.size()))) return st;
    if ((st = balloc(b, &bk, f64b.size()))) return st;
    HIP_OR_FAIL(hipMemcpyAsync(f, f64f.data(), sizeof(kk::BatchItemF64) * f64f.size(), hipMemcpyHostToDevice, b->stream));
    HIP_OR_FAIL(hipMemcpyAsync(bk, f64b.data(), sizeof(kk::BatchItemF64) * f64b.size(), hipMemcpyHostToDevice, b->stream));
    b->d_items_fwd = f;
    b->d_items_back = bk;
  }
  if ((st = balloc(b, &b->d_delta, n_systems))) return st;
  if ((st = balloc(b, &b->d_out, n_systems))) return st;
  if ((st = balloc(b, &b->d_info, n_systems))) return st;
  b->h_delta.assign(n_systems, nullptr);
  b->h_out.assign(n_systems, nullptr);
  if ((st = build_tile_lists(b, 0))) return st;
  HIP_OR_FAIL(hipStreamSynchronize(b->stream));
  b->prepared = true;
  g_err.clear();
  return KK_OK;
}

kk_status krylov_kernel_apply_batch(kk_batch b, const double* const* delta, int m, double* const* Kdelta,
                                    kk_info* info) {
  if (!b) return fail(KK_EINVAL, "krylov_kernel_apply_batch: batch is NULL");
  if (!b->prepared) return fail(KK_ENOTPREPARED, "kk_batch_prepare has not succeeded on this batch");
  if (!delta || !Kdelta) return fail(KK_EINVAL, "krylov_kernel_apply_batch: NULL array argument");
  int min_n2 = 1 << 30;
  for (int i = 0; i < b->ns; ++i) {
    if (!delta[i] || !Kdelta[i]) return fail(KK_EINVAL, "krylov_kernel_apply_batch: NULL pointer for system %d", i);
    min_n2 = std::min(min_n2, 2 * b->sys[i]->natoms);
  }
  if (m < 1 || m > std::min(min_n2, kk::MAX_RANK))
    return fail(KK_EINVAL, "krylov_kernel_apply_batch: need 1 <= m <= min(2N_i, %d), got %d", kk::MAX_RANK, m);
  HIP_OR_FAIL(hipEventRecord(b->ev_in, b->user_stream));
  HIP_OR_FAIL(hipStreamWaitEvent(b->stream, b->ev_in, 0));
  kk_status st;
  if ((st = upload_pointer_tables(b, delta, Kdelta))) return st;
  if (!b->tuned) {
    if ((st = autotune(b, m))) return st;
    HIP_OR_FAIL(hipStreamSynchronize(b->stream));
    b->drop_graph();
  }
  if (b->graph_m != m) {
    HIP_OR_FAIL(hipStreamSynchronize(b->stream));  // the last replay may still run
    b->drop_graph();
    HIP_OR_FAIL(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    st = enqueue_update(b, m);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(KK_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    b->graph = g;
    HIP_OR_FAIL(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_m = m;
  }
  HIP_OR_FAIL(hipGraphLaunch(b->exec, b->stream));
  HIP_OR_FAIL(hipEventRecord(b->ev_out, b->stream));
  HIP_OR_FAIL(hipStreamWaitEvent(b->user_stream, b->ev_out, 0));
  if (info) {
    std::vector<kk::KrylovState> hs(b->ns);
    HIP_OR_FAIL(hipMemcpyAsync(hs.data(), b->d_info, sizeof(kk::KrylovState) * b->ns, hipMemcpyDeviceToHost,
                               b->stream));
    HIP_OR_FAIL(hipStreamSynchronize(b->stream));
    bool breakdown = false, singular = false;
    for (int i = 0; i < b->ns; ++i) {
      info[i].rank_used = hs[i].rank;
      info[i].status = hs[i].status;
      info[i].min_pivot = hs[i].min_pivot;
      info[i].max_pivot = hs[i].max_pivot;
      info[i].ls_residual = hs[i].ls_residual;
      breakdown |= hs[i].status == 1;
      singular |= hs[i].status == KK_ESINGULAR;
    }
    g_err.clear();
    if (singular) return fail(KK_ESINGULAR, "krylov_kernel_apply_batch: a Gram matrix is not positive definite");
    return breakdown ? KK_BREAKDOWN : KK_OK;
  }
  g_err.clear();
  return KK_OK;
}

kk_status kk_batch_set_tuning(kk_batch b, int small_np_max, int workgroups_per_cu) {
  if (!b) return fail(KK_EINVAL, "kk_batch_set_tuning: batch is NULL");
  if (!b->prepared) return fail(KK_ENOTPREPARED, "kk_batch_prepare has not succeeded on this batch");
  if (small_np_max < 0) return fail(KK_EINVAL, "kk_batch_set_tuning: small_np_max must be >= 0");
  if (workgroups_per_cu < 1 || workgroups_per_cu > 8)
    return fail(KK_EINVAL, "kk_batch_set_tuning: need 1 <= workgroups_per_cu <= 8, got %d", workgroups_per_cu);
  HIP_OR_FAIL(hipStreamSynchronize(b->stream));  // a replay may still read the tile lists
  b->drop_graph();
  kk_status st;
  if ((st = build_tile_lists(b, small_np_max))) return st;
  b->small_np_max = small_np_max;
  b->grid_mult = workgroups_per_cu;
  b->tuned_ms = 0.0;
  b->tuned = true;
  g_err.clear();
  return KK_OK;
}

kk_status kk_batch_tuning(kk_batch b, int* small_np_max, int* workgroups_per_cu, double* update_ms) {
  if (!b) return fail(KK_EINVAL, "kk_batch_tuning: batch is NULL");
  if (!b->tuned) return fail(KK_ENOTPREPARED, "kk_batch_tuning: no update has run yet");
  if (small_np_max) *small_np_max = b->small_np_max;
  if (workgroups_per_cu) *workgroups_per_cu = b->grid_mult;
  if (update_ms) *update_ms = b->tuned_ms;
  return KK_OK;
}

}  // extern "C"
