// C-ABI of the reflector library (include/refl.h): argument checks,
// workspace layout, and the host-side sequencing of the kernels.
//
// refl_sign, all precisions:
//   set-up  H upper triangle -> padded symmetric FP64 copy Hf; alpha =
//           ||H - sI||_inf (section 4.3) unless given; X_0 = (H - sI)/alpha
//           in the bulk storage (FP64, FP32 or BF16 words).
//   bulk    Newton-Schulz steps X <- X (3I - X^2)/2 (eq. NS), each two
//           symmetric MFMA products with fused epilogues; after the first
//           product of every step the host reads ||X^2 - I||_F and trace X
//           (one 16-byte copy) and applies the stopping rule.
//   output  FP64/FP32: R = the last iterate.  MIXED: an FP64 correction of
//           the target eigenspace that uses H itself (subspace extraction
//           from (I - X)/2, Rayleigh-Ritz, projected CG correction sweeps),
//           then R = I - 2 V V^T and the Davis-Kahan certificate.
//
// Index certificate (used by every path): for symmetric X with
// b = sqrt(d) ||X^2 - I||_F < 1, the number j of negative eigenvalues of X
// satisfies |trace X - (d - 2j)| <= b, so j is the integer nearest to
// (d - trace X)/2 whenever that distance is below 1/2 ... more precisely j
// is the unique integer with |trace X - (d - 2j)| < 1.  Sign preservation
// of the Newton-Schulz polynomials (Lemma 3.4) makes j the inertia of
// H - sI when the iterate is accurate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/refl.h"
#include "common.h"
#include "dbg.h"
#include "hostla.h"
#include "launch.h"

using namespace refl;

struct refl_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  void* ws_user = nullptr;
  size_t ws_user_bytes = 0;
  void* ws_own = nullptr;
  size_t ws_own_bytes = 0;
  double* pinned = nullptr;  // host pinned scalars (SC_COUNT doubles + CG state)
  std::vector<hipEvent_t> ev;  // params.timing: start/stop pairs of the bulk products
  std::vector<hipEvent_t> bulk_ev;  // completion of the pipelined bulk steps
  double* lz_pin = nullptr;    // host pinned copies of the Lanczos blocks and flags
  size_t lz_pin_bytes = 0;
  void* batch_pin = nullptr;   // host pinned staging of the batched solve
  size_t batch_pin_bytes = 0;
  hipEvent_t lz_ev[2] = {nullptr, nullptr};
  hipStream_t cap = nullptr;   // stream the batched step graph is captured on
  // The batched step graph of the last call, kept for the next call with the
  // same workspace, precision, orders, tile edges and list of tiled problems.
  hipGraphExec_t bgraph = nullptr;
  std::vector<int64_t> bgraph_key;
  hipStream_t side = nullptr;  // batched solve: small problems run beside the grouped steps
  hipEvent_t side_ev[2] = {nullptr, nullptr};  // fork and join of the side stream
  int ncu = 256;               // compute units of the device
  // Allocation-free calls (refl_sign_noalloc): the device address of this
  // device's fixed scratch array (resolved at refl_create), and the flag
  // that turns every allocation site on the refl_sign path into an error
  // or a pre-created resource for the duration of such a call.
  void* scratch = nullptr;
  hipError_t scratch_err = hipSuccess;
  bool no_alloc = false;
  char err[512] = {0};
};

// State of a shift policy over a sequence of Hessians (refl_policy_*).
struct refl_policy_s {
  refl_policy_params_t pp;
  int device = 0;
  bool have = false;            // a certified shift from an earlier call is in force
  double s = 0.0;               // last shift returned
  double lam_k = 0.0, lam_k1 = 0.0, eps = 0.0;  // estimates of the last refresh
  int64_t dref = 0;             // order of H_ref
  double* Href = nullptr;       // REUSE: upper triangle of the Hessian of the last refresh (ld dref)
  double* dscr = nullptr;       // device partials + one result slot
  size_t dscr_n = 0;
  double* Vwarm = nullptr;      // warm_start: Ritz block of the last refresh (d x b, ld dwarm)
  int64_t dwarm = 0;            // its order (0: none yet)
  int calls = 0, refreshes = 0;
};

namespace {

constexpr double NaN = std::numeric_limits<double>::quiet_NaN();

refl_status_t fail(refl_handle_t h, refl_status_t st, const char* fmt, ...) {
  if (h) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(h->err, sizeof(h->err), fmt, ap);
    va_end(ap);
  }
  return st;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(h, REFL_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Bump allocator over one device allocation (256-byte aligned pieces).
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = (size_t)round_up((int64_t)off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

constexpr int MAXB = 32;  // widest block of vectors
constexpr int BULK_RING = 16;  // MIXED bulk: completion events of the steps in flight
// Pinned host staging of the Lanczos blocks created with every handle:
// 2 J b^2 doubles with J b <= d and b <= 32, so orders up to 2048, which
// covers every order whose workspace fits the allocation-free scratch.
constexpr size_t LZ_PIN_INITIAL = sizeof(double) * 2 * 2048 * 32 + 4096;

// Block-Lanczos buffers (carved only when the shift is estimated).
struct LzWork {
  int b = 0, J = 0, nmax = 0;
  double *V = nullptr, *W = nullptr, *C = nullptr;
  double *ppart = nullptr, *gp[2] = {nullptr, nullptr};  // Gram partials, by round parity
  double *Bacc = nullptr, *TA = nullptr, *TB = nullptr;
  double* gsum = nullptr;  // summed Gram matrix of the first Cholesky QR round of a step
  int* flag = nullptr;
};

struct Work {
  int d, dp, ntiles, words;
  int ts, dk;  // bulk tile edge and K extent of the bulk products
  int64_t ps;  // plane stride (elements) of word storage
  double* Hf;
  float* H32;  // MIXED with cg_f32: FP32 copy of H for the inner solves
  double* scal;
  double* rowsum;
  double* partials;
  double* partials_t;  // update products' trace partials (single-problem device loops)
  double *qr_gp[2], *qr_B;  // device Cholesky QR of the correction's blocks: Gram partials, R
  int* qr_flag;
  bool h32_ready = false;  // H32 already holds the FP32 copy of H (written with X_0)
  int2* tiles;
  // bulk (only the ones of the precision are non-null)
  double *X64[2], *N64;
  float *X32[2], *N32;
  uint16_t *Xw[3], *Nw;
  // block vectors (ld = dp), polish and apply
  double *V, *W, *Z, *Rr, *P[2], *AP, *T1, *T2, *G, *thin, *gwork, *cgpart;
  void* cgstate;
  LzWork lz;
};

// Bulk tile edge for the word products: the edge whose upper-triangle tile
// count, spread over the device's compute units, finishes first (a 192 tile
// does 2.25x the work of a 128 tile at about 1.4x its per-CU throughput).
int choose_tile(int64_t d, int words, int ncu) {
  if (words > 2) return 128;
  // REFL_BULK_TILE=128|192 overrides the choice (tests, tuning).
  if (const char* e = std::getenv("REFL_BULK_TILE")) {
    const int v = std::atoi(e);
    if (v == 128 || v == 192) return v;
  }
  double best = 1e300;
  int bt = 128;
  for (int ts : {128, 192}) {
    const int64_t nt = (d + ts - 1) / ts, tiles = nt * (nt + 1) / 2;
    const int64_t rounds = (tiles + ncu - 1) / ncu;
    const double cost = (double)rounds * ts * ts / (ts == 192 ? 1.4 : 1.0);
    if (cost < best) {
      best = cost;
      bt = ts;
    }
  }
  return bt;
}

void carve_lanczos(Carve& c, LzWork& z, int64_t d, int dp, int k, int steps);

void build_tiles_nt(int nt, std::vector<int2>& host);

// Padding unit of the FP64 / FP32 matrices for tile edge ts: a multiple of
// ts and of 64 (the set-up kernels work in 64 x 64 tiles).
int pad_unit_f(int ts) { return ts % 64 == 0 ? ts : ts * 2; }

// Tile edge of the FP64 / FP32 products for order d, from a cost model:
// the edge whose upper-tile list finishes first on the device's compute
// units.  A unit holds several blocks of a small edge at once (LDS-limited)
// and they share its matrix cores; a tile of edge ts costs ts^2 dp / eff(ts)
// with eff fitted to measured launches (d = 1024..4096).  Used when the
// measurement below is switched off.
int model_tile_f(int64_t d, bool fp64, int ncu) {
  double best = 1e300;
  int bt = TILE;
  for (int ts : {128, 96, 64}) {
    const int64_t dp = round_up(d, pad_unit_f(ts));
    const int64_t nt = dp / ts;
    const int64_t tiles = nt * (nt + 1) / 2;
    const int64_t occ = sym_gemm_f_blocks_per_cu(fp64 ? 1 : 0, ts);
    const int64_t rounds = (tiles + ncu * occ - 1) / (ncu * occ);
    const int64_t conc = std::min<int64_t>(occ, (tiles + ncu - 1) / ncu);
    const double eff = ts == 128 ? 1.0 : ts == 96 ? 0.9 : 1.3;
    const double cost = (double)rounds * conc * ts * ts * (double)dp / eff;
    if (cost < best) {
      best = cost;
      bt = ts;
    }
  }
  return bt;
}

// Measured choice (the tile autotuner): on the first FP64 / FP32 solve of
// order d on a device, one symmetric product of each candidate edge is timed
// (HIP events, after a warm-up launch) on a pseudo-random dp x dp operand in
// scratch memory the tuner allocates and frees, and the fastest edge is
// cached for the process.  REFL_F_TILE=32|64|96|128 forces an edge (32 only so);
// REFL_F_TUNE=0 uses the cost model instead.  The edge changes only how the
// products are tiled: each output entry is the same sum in the same order.
std::mutex g_tile_mu;
std::map<std::tuple<int, int, int64_t>, int> g_tile_cache;

int select_tile_f(refl_handle_t h, int64_t d, bool fp64) {
  if (const char* e = std::getenv("REFL_F_TILE")) {
    const int v = std::atoi(e);
    if (v == 32 || v == 64 || v == 96 || v == 128) return v;
  }
  if (const char* e = std::getenv("REFL_F_TUNE"))
    if (std::atoi(e) == 0) return model_tile_f(d, fp64, h->ncu);
  const auto key = std::make_tuple(h->device, fp64 ? 1 : 0, d);
  std::lock_guard<std::mutex> lock(g_tile_mu);
  auto it = g_tile_cache.find(key);
  if (it != g_tile_cache.end()) return it->second;
  const int fallback = model_tile_f(d, fp64, h->ncu);
  // Timing needs a buffer of its own: an allocation-free call takes the
  // cost model's edge (not cached, so a later refl_sign still measures).
  if (h->no_alloc) return fallback;
  // The 32 edge is not a candidate: alone on the device it is the fastest
  // product up to d = 1536 (it spreads the tiles over every compute unit),
  // but batched calls, which must use refl_sign's edge to return the same
  // results bit for bit, run a third slower with it on a full device.
  const int cands[3] = {128, 96, 64};
  int64_t dpmax = 0;
  for (int ts : cands) dpmax = std::max<int64_t>(dpmax, round_up(d, pad_unit_f(ts)));
  const size_t es = fp64 ? sizeof(double) : sizeof(float);
  const int64_t ntmax = dpmax / 32;
  const size_t tmax = (size_t)(ntmax * (ntmax + 1) / 2);
  char* buf = nullptr;
  const size_t bytes = (size_t)dpmax * dpmax * (sizeof(double) + 2 * es) + tmax * (sizeof(int2) + sizeof(double)) + 4096;
  if (hipSetDevice(h->device) != hipSuccess || hipMalloc(&buf, bytes) != hipSuccess) return fallback;
  hipStream_t st = h->stream;
  Carve c(buf);
  double* R = c.take<double>((size_t)dpmax * dpmax);
  void* X = c.take<char>(es * dpmax * dpmax);
  void* N = c.take<char>(es * dpmax * dpmax);
  int2* tiles = c.take<int2>(tmax);
  double* parts = c.take<double>(tmax);
  double* one = c.take<double>(1);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = fallback;
  float best_ms = 1e30f;
  bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  const double h_one = 1.0;
  ok = ok && hipMemcpyAsync(one, &h_one, sizeof(double), hipMemcpyHostToDevice, st) == hipSuccess;
  for (int ts : cands) {
    if (!ok) break;
    const int dp = (int)round_up(d, pad_unit_f(ts));
    std::vector<int2> tl;
    build_tiles_nt(dp / ts, tl);
    const int nt = (int)tl.size();
    ok = hipMemcpyAsync(tiles, tl.data(), sizeof(int2) * nt, hipMemcpyHostToDevice, st) == hipSuccess &&
         random_block(R, dp, dp, dp, 0x7115ull + ts, st) == hipSuccess &&
         (fp64 ? launch_init_x0_f64(R, dp, (int)d, 0.0, one, (double*)X, st)
               : launch_init_x0_f32(R, dp, (int)d, 0.0, one, (float*)X, st)) == hipSuccess;
    auto product = [&]() {
      return fp64 ? launch_sym_gemm_f64(ts, GEMM_RESIDUAL, (double*)X, (double*)X, nullptr,
                                        (double*)N, dp, (int)d, dp, tiles, nt, parts, st)
                  : launch_sym_gemm_f32(ts, GEMM_RESIDUAL, (float*)X, (float*)X, nullptr,
                                        (float*)N, dp, (int)d, dp, tiles, nt, parts, st);
    };
    ok = ok && product() == hipSuccess && hipEventRecord(e0, st) == hipSuccess &&
         product() == hipSuccess && product() == hipSuccess &&
         hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (ok && ms < best_ms) {
      best_ms = ms;
      best = ts;
    }
  }
  (void)hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  if (!ok) {
    (void)hipGetLastError();
    return fallback;
  }
  g_tile_cache[key] = best;
  return best;
}

// Workspace of refl_sign / refl_sign_apply (kind SIGN), refl_apply (APPLY)
// or refl_estimate_shift (ESTIMATE: the FP64 copy of H and the Lanczos
// buffers only).
enum LayoutKind { LAYOUT_SIGN, LAYOUT_APPLY, LAYOUT_ESTIMATE };

size_t layout(Work& w, void* base, int64_t d, const refl_params_t& p, LayoutKind kind,
              refl_handle_t h) {
  const int ncu = h->ncu;
  Carve c(base);
  const bool for_apply = kind == LAYOUT_APPLY;
  w.d = (int)d;
  if (!for_apply && p.precision == REFL_PREC_MIXED) {
    w.ts = choose_tile(d, p.words, ncu);
    w.dp = (int)round_up(d, w.ts);
  } else if (kind == LAYOUT_SIGN) {
    w.ts = select_tile_f(h, d, p.precision == REFL_PREC_FP64);
    w.dp = (int)round_up(d, pad_unit_f(w.ts));
  } else if (kind == LAYOUT_ESTIMATE) {
    w.ts = TILE;
    w.dp = (int)round_up(d, w.ts);
  } else {
    w.ts = TILE;
    w.dp = (int)round_up(d, w.ts);
  }
  w.dk = (p.precision == REFL_PREC_MIXED) ? (int)round_up(d, 32) : w.dp;
  const int64_t dp = w.dp, n2 = dp * dp;
  const int nt = w.dp / w.ts;
  w.ntiles = nt * (nt + 1) / 2;
  w.words = p.words;
  w.ps = n2;
  w.scal = c.take<double>(SC_COUNT);
  w.tiles = c.take<int2>(w.ntiles);
  w.partials = c.take<double>(w.ntiles);
  w.partials_t = c.take<double>(w.ntiles);
  w.rowsum = c.take<double>(2 * dp);
  w.X64[0] = w.X64[1] = w.N64 = nullptr;
  w.X32[0] = w.X32[1] = w.N32 = nullptr;
  w.Xw[0] = w.Xw[1] = w.Xw[2] = w.Nw = nullptr;
  w.lz = LzWork();
  if (kind == LAYOUT_ESTIMATE) {
    w.Hf = c.take<double>(n2);
    w.thin = c.take<double>(thin_work_doubles((int)dp));
    carve_lanczos(c, w.lz, d, w.dp, p.k, p.lanczos_steps);
    return c.off + 256;
  }
  w.H32 = nullptr;
  if (!for_apply) {
    w.Hf = c.take<double>(n2);
    if (p.precision == REFL_PREC_MIXED && p.cg_f32 != REFL_CG_FP64) w.H32 = c.take<float>(n2);
    if (p.precision == REFL_PREC_FP64) {
      w.X64[0] = c.take<double>(n2);
      w.X64[1] = c.take<double>(n2);
      w.N64 = c.take<double>(n2);
    } else if (p.precision == REFL_PREC_FP32) {
      w.X32[0] = c.take<float>(n2);
      w.X32[1] = c.take<float>(n2);
      w.N32 = c.take<float>(n2);
    } else {
      const int W = p.words;
      w.Xw[0] = c.take<uint16_t>(W * n2);
      w.Xw[1] = c.take<uint16_t>(W * n2);
      w.Xw[2] = c.take<uint16_t>(W * n2);
      w.Nw = c.take<uint16_t>(W * n2);
    }
  } else {
    w.Hf = nullptr;
  }
  w.V = c.take<double>(dp * MAXB);
  w.W = c.take<double>(dp * MAXB);
  w.Z = c.take<double>(dp * MAXB);
  w.Rr = c.take<double>(dp * MAXB);
  w.P[0] = c.take<double>(dp * MAXB);
  w.P[1] = c.take<double>(dp * MAXB);
  w.AP = c.take<double>(dp * MAXB);
  w.T1 = c.take<double>(dp * MAXB);
  w.T2 = c.take<double>(dp * MAXB);
  w.G = c.take<double>(MAXB * MAXB * 2);
  w.thin = c.take<double>(thin_work_doubles((int)dp));
  w.gwork = c.take<double>(gram_work_doubles((int)dp));
  w.cgpart = c.take<double>(cg_part_doubles((int)dp));
  w.cgstate = c.take<char>(cg_state_bytes());
  w.qr_gp[0] = c.take<double>(lz_gram_part_doubles((int)dp, MAXB));
  w.qr_gp[1] = c.take<double>(lz_gram_part_doubles((int)dp, MAXB));
  w.qr_B = c.take<double>(MAXB * MAXB);
  w.qr_flag = c.take<int>(4);
  if (!for_apply && p.shift_mode == REFL_SHIFT_LANCZOS) carve_lanczos(c, w.lz, d, w.dp, p.k, p.lanczos_steps);
  return c.off + 256;
}

refl_status_t ensure_workspace(refl_handle_t h, size_t need, void** out) {
  if (h->no_alloc) {
    if (!h->scratch)
      return fail(h, REFL_ERR_DEVICE, "scratch address of device %d unavailable: %s", h->device,
                  hipGetErrorString(h->scratch_err));
    if (need > NOALLOC_SCRATCH_BYTES)
      return fail(h, REFL_ERR_INVALID_ARG,
                  "this order and these parameters need %zu bytes of workspace; the "
                  "allocation-free entry point has %zu",
                  need, NOALLOC_SCRATCH_BYTES);
    *out = h->scratch;
    return REFL_OK;
  }
  if (h->ws_user && h->ws_user_bytes >= need) {
    *out = h->ws_user;
    return REFL_OK;
  }
  if (h->ws_own && h->ws_own_bytes >= need) {
    *out = h->ws_own;
    return REFL_OK;
  }
  if (h->ws_own) {
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipFree(h->ws_own));
    h->ws_own = nullptr;
    h->ws_own_bytes = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess || !p)
    return fail(h, REFL_ERR_NO_MEMORY, "workspace allocation of %zu bytes failed", need);
  h->ws_own = p;
  h->ws_own_bytes = need;
  *out = p;
  return REFL_OK;
}

refl_status_t check_params(refl_handle_t h, int64_t d, const refl_params_t* p) {
  if (!p) return fail(h, REFL_ERR_INVALID_ARG, "params is NULL");
  if (d < 2 || d > (int64_t)1 << 16) return fail(h, REFL_ERR_INVALID_ARG, "d=%lld outside 2..65536", (long long)d);
  if (p->k < 0 || p->k > d - 1) return fail(h, REFL_ERR_INVALID_ARG, "k=%d outside 0..d-1", p->k);
  if (p->k == 0 && p->shift_mode != REFL_SHIFT_GIVEN)
    return fail(h, REFL_ERR_INVALID_ARG, "k=0 (report the index) needs a given shift");
  if (p->precision < 0 || p->precision > 2) return fail(h, REFL_ERR_INVALID_ARG, "bad precision");
  if (p->shift_mode != REFL_SHIFT_GIVEN && p->shift_mode != REFL_SHIFT_LANCZOS)
    return fail(h, REFL_ERR_INVALID_ARG, "bad shift_mode");
  if (p->scale_mode != REFL_SCALE_INF && p->scale_mode != REFL_SCALE_GIVEN &&
      p->scale_mode != REFL_SCALE_LANCZOS && p->scale_mode != REFL_SCALE_FRO)
    return fail(h, REFL_ERR_INVALID_ARG, "bad scale_mode");
  if (p->scale_mode == REFL_SCALE_LANCZOS && p->shift_mode != REFL_SHIFT_LANCZOS)
    return fail(h, REFL_ERR_INVALID_ARG, "scale_mode LANCZOS needs shift_mode LANCZOS");
  if (p->lanczos_steps < 0) return fail(h, REFL_ERR_INVALID_ARG, "lanczos_steps must be >= 0");
  if (p->scale_mode == REFL_SCALE_GIVEN && !(p->alpha > 0.0 && std::isfinite(p->alpha)))
    return fail(h, REFL_ERR_INVALID_ARG, "alpha must be finite and > 0");
  if (p->shift_mode == REFL_SHIFT_GIVEN && !std::isfinite(p->s))
    return fail(h, REFL_ERR_NOT_FINITE, "shift is not finite");
  if (p->max_iter < 1) return fail(h, REFL_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (p->timing < 0) return fail(h, REFL_ERR_INVALID_ARG, "timing must be >= 0");
  if (p->fixed_steps < 0) return fail(h, REFL_ERR_INVALID_ARG, "fixed_steps must be >= 0");
  if (p->precision == REFL_PREC_MIXED) {
    if (p->words < 1 || p->words > 3) return fail(h, REFL_ERR_INVALID_ARG, "words must be 1..3");
    if (p->words_max != 0 && (p->words_max < p->words || p->words_max > 3))
      return fail(h, REFL_ERR_INVALID_ARG, "words_max must be 0 or words..3");
    if (p->cg_f32 < REFL_CG_FP64 || p->cg_f32 > REFL_CG_AUTO)
      return fail(h, REFL_ERR_INVALID_ARG, "bad cg_f32");
    if (p->fixed_steps == 0 && p->k > MAXB)
      return fail(h, REFL_ERR_UNSUPPORTED, "MIXED correction supports k <= %d", MAXB);
    if (p->polish_sweeps < 0 || p->cg_max_iter < 1 || !(p->cg_tol > 0.0))
      return fail(h, REFL_ERR_INVALID_ARG, "bad polish parameters");
  }
  if (!(p->tol >= 0.0)) return fail(h, REFL_ERR_INVALID_ARG, "tol must be >= 0");
  if (p->check_symmetric != 0 && p->check_symmetric != 1)
    return fail(h, REFL_ERR_INVALID_ARG, "check_symmetric must be 0 or 1");
  if (p->check_symmetric && !(p->sym_tol >= 0.0 && std::isfinite(p->sym_tol)))
    return fail(h, REFL_ERR_INVALID_ARG, "sym_tol must be finite and >= 0");
  return REFL_OK;
}

// Opt-in symmetry check of H (params.check_symmetric): max_{i<j} |H_ij - H_ji|
// against sym_tol max |H_ij|, both as maxima (no summation order), a NaN
// anywhere failing.  slot and slot + 1 of scal receive the two maxima.
refl_status_t check_symmetry(refl_handle_t h, int64_t d, const double* dH, int64_t ldh,
                             double sym_tol, double* scal, int slot) {
  hipStream_t st = h->stream;
  HIPCHK(launch_asym_max(dH, ldh, (int)d, scal, slot, st));
  double* hsc = h->pinned;
  HIPCHK(hipMemcpyAsync(hsc + slot, scal + slot, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double asym = hsc[slot], amax = hsc[slot + 1];
  if (!(asym <= sym_tol * amax) || !std::isfinite(amax))
    return fail(h, REFL_ERR_NOT_SYMMETRIC, "max |H_ij - H_ji| = %.3e exceeds %.3e max |H_ij| (%.3e)",
                asym, sym_tol, amax);
  return REFL_OK;
}

// Upper tiles (I <= J) ordered so that the work-groups that share an XCD
// (block b runs on XCD b % 8) take a compact patch of the triangle: tiles
// are listed by bands of 4 tile rows, column by column, the list is cut into
// 8 consecutive pieces, and block b takes element b / 8 of piece b % 8.
void build_tiles_nt(int nt, std::vector<int2>& host) {
  std::vector<int2> order;
  for (int b0 = 0; b0 < nt; b0 += 4)
    for (int J = b0; J < nt; ++J)
      for (int I = b0; I < std::min(b0 + 4, nt); ++I)
        if (I <= J) order.push_back(make_int2(I, J));
  const int T = (int)order.size();
  int start[8], s0 = 0;
  for (int x = 0; x < 8; ++x) {
    start[x] = s0;
    s0 += (T - x + 7) / 8;
  }
  host.resize(T);
  for (int b = 0; b < T; ++b) host[b] = order[start[b % 8] + b / 8];
}
void build_tiles(const Work& w, std::vector<int2>& host) { build_tiles_nt(w.dp / w.ts, host); }

// Index certificate: returns j, or -1 if b = sqrt(d)||X^2-I||_F >= 1 or no
// integer j has |trace - (d - 2j)| < 1.
int index_certificate(int64_t d, double resid, double trace) {
  const double b = std::sqrt((double)d) * resid;
  if (!(b < 1.0)) return -1;
  const double jr = std::nearbyint(((double)d - trace) / 2.0);
  if (std::fabs(trace - ((double)d - 2.0 * jr)) < 1.0) return (int)jr;
  return -1;
}

struct Bulk {
  int steps = 0;
  double resid = NaN, trace = NaN;
  int cur = 0;  // which X buffer holds the last iterate
  bool converged = false;
};

// FP32 / FP64 problems of order d <= SMALL_MAX_* run the whole iteration in
// one LDS-resident launch (launch_ns_small); REFL_SMALL=0 sends them through
// the tiled products instead (tests compare the two).
bool small_order(int64_t d, bool fp64) {
  const char* e = std::getenv("REFL_SMALL");
  const bool off = e && e[0] == '0';
  return !off && d >= 1 && d <= (fp64 ? SMALL_MAX_F64 : SMALL_MAX_F32);
}
static_assert(sizeof(SmallProb) == 32 && sizeof(BatchRule) == 16 && sizeof(BatchStep) == 48,
              "staging layout of the small-order launch");

// Orthonormalise the d x nb block V (ld dp) by two rounds of Cholesky QR,
// on the device with the block-Lanczos kernels (slab Gram partials, then
// two k_lz_cholqr rounds; no host round trip).  A pivot that is not
// positive sets bit 1 of w.qr_flag, which the caller clears before its
// first call; the flag is copied to the pinned slot qr_flag_host() behind
// the kernels and tested at the caller's next synchronisation
// (qr_lost_rank).
int* qr_flag_host(refl_handle_t h) {
  return reinterpret_cast<int*>(reinterpret_cast<char*>(h->pinned + SC_COUNT) + sizeof(CgHost) + 128);
}
// Pinned staging of the Rayleigh-Ritz exchanges (behind the 256-byte tail):
// slot 0 and 1 hold MAXB x MAXB doubles (a Gram matrix read back, the Ritz
// rotation sent), slot 2 MAXB doubles.  A copy from pinned memory is queued
// without the runtime's pageable staging; a slot is rewritten only after
// the next synchronisation of the stream, when its copy has completed.
double* rr_pin(refl_handle_t h, int slot) {
  return reinterpret_cast<double*>(reinterpret_cast<char*>(h->pinned + SC_COUNT) + sizeof(CgHost) + 256) +
         (size_t)slot * MAXB * MAXB;
}
refl_status_t orthonormalise(refl_handle_t h, Work& w, double*& V, double*& spare, int nb) {
  hipStream_t st = h->stream;
  HIPCHK(lz_gram(V, w.dp, nb, w.d, w.qr_gp[0], st));
  HIPCHK(lz_cholqr(w.qr_gp[0], LZ_GRAM_ROWS, w.d, nb, 0.0, w.qr_B, 0, nullptr, nullptr, w.qr_flag, 1, V,
                   w.dp, spare, w.dp, w.qr_gp[1], LZ_QR_PLAIN, nullptr, st));
  HIPCHK(lz_cholqr(w.qr_gp[1], 256, w.d, nb, 0.0, w.qr_B, 1, nullptr, nullptr, w.qr_flag, 2, spare,
                   w.dp, spare, w.dp, nullptr, LZ_QR_PLAIN, nullptr, st));
  HIPCHK(hipMemcpyAsync(qr_flag_host(h), w.qr_flag, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  std::swap(V, spare);
  return REFL_OK;
}
bool qr_lost_rank(refl_handle_t h) { return (qr_flag_host(h)[0] & 1) != 0; }

// Block CG on (I - V V^T)(H - theta_c)(I - V V^T) z_c = r_c, c < k (V: d x k,
// ld dp), from the state *hs (theta, rho0, tol2, k, nb set by the caller;
// r in cb.R[0], cb.Z zeroed), over H in FP64 or its FP32 copy.  On return
// *hs holds the final state (iters, done).
refl_status_t cg_solve(refl_handle_t h, Work& w, bool use32, const double* V, int k, const CgBufs& cb,
                       int max_iter, CgHost* hs, bool pipe = false) {
  hipStream_t st = h->stream;
  const int64_t ld = w.dp;
  HIPCHK(hipMemcpyAsync(w.cgstate, hs, sizeof(CgHost), hipMemcpyHostToDevice, st));
  // The first batch is 32 iterations (every correction solve here needs
  // more); each later one runs to where the residuals, extrapolated
  // geometrically from the last two checks, reach the tolerance (plus two),
  // within 8..64: a host check drains the queue, so fewer checks save more
  // than the few iterations queued past convergence cost (they return at
  // once).  Iteration max_iter + 1 only runs the convergence test.
  const int nb = hs->nb;
  const double tol2 = hs->tol2;
  std::vector<double> rho0(hs->rho0, hs->rho0 + nb), gprev(rho0);
  int itprev = 0;
  int issued = 0, batch = 32;
  while (true) {
    for (int b = 0; b < batch && issued <= max_iter + 1; ++b, ++issued) {
      if (pipe)
        HIPCHK(cg_pipe_iteration(w.Hf, use32 ? w.H32 : nullptr, ld, w.d, k, k, V, ld, cb, w.cgstate,
                                 w.thin, w.cgpart, issued, max_iter, st));
      else
        HIPCHK(cg_iteration(w.Hf, use32 ? w.H32 : nullptr, ld, w.d, k, V, ld, cb, w.cgstate, w.thin,
                            w.cgpart, issued, max_iter, st));
    }
    HIPCHK(hipMemcpyAsync(hs, w.cgstate, sizeof(CgHost), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hs->done || issued > max_iter + 1) break;
    // The newest residual norms (the two state slots hold the last two
    // iterations'; the smaller of each pair is taken).
    const int itnow = hs->iters;
    double need = 0.0;
    bool known = itnow > itprev;
    for (int c = 0; c < nb && known; ++c) {
      const double g = std::min(hs->gam[0][c], hs->gam[1][c]);
      if (!(g > tol2 * rho0[c])) continue;
      if (!(g < gprev[c]) || !(gprev[c] > 0.0)) {
        known = false;
        break;
      }
      const double rate = std::log(g / gprev[c]) / (itnow - itprev);  // < 0
      need = std::max(need, std::log(tol2 * rho0[c] / g) / rate);
    }
    if (known) {
      for (int c = 0; c < nb; ++c) gprev[c] = std::min(hs->gam[0][c], hs->gam[1][c]);
      itprev = itnow;
      batch = std::min(64, std::max(8, (int)std::ceil(need) + 2));
    } else {
      batch = 16;
    }
  }
  return REFL_OK;
}

// FP64 correction of the target eigenspace for the MIXED path.  On entry
// X (words) is the bulk iterate.  On exit V (ld dp, k columns) is an
// orthonormal basis, and *E_fro, *theta_max describe the last Rayleigh-Ritz.
refl_status_t polish(refl_handle_t h, Work& w, const refl_params_t& p, double s,
                     const uint16_t* X, double** Vout, refl_info_t* info,
                     std::vector<double>* theta_out = nullptr) {
  const int d = w.d, k = p.k;
  const int64_t ld = w.dp;
  hipStream_t st = h->stream;
  double* V = w.V;
  double* spare = w.T1;
  HIPCHK(hipMemsetAsync(w.qr_flag, 0, 4 * sizeof(int), st));
  qr_flag_host(h)[0] = 0;
  HIPCHK(random_block(V, ld, d, k, p.seed ^ 0x5EEDull, st));
  // Subspace extraction with the approximate projector (I - X)/2.
  for (int it = 0; it < 2; ++it) {
    HIPCHK(symthin_words(w.words, X, w.dp, w.ps, d, V, ld, k, w.T2, ld, w.thin, st));
    HIPCHK(lincomb(d, k, -0.5, w.T2, ld, 0.5, V, ld, st));  // V = (V - X V)/2
    refl_status_t r = orthonormalise(h, w, V, spare, k);
    if (r != REFL_OK) return r;
  }
  std::vector<double> Q(k * k), th(k);
  double* G = rr_pin(h, 0);    // Gram matrices read back
  double* Cc = rr_pin(h, 1);   // Ritz rotation sent
  double* nrm = rr_pin(h, 2);  // -theta sent
  double* Wm = w.W;
  double* Wspare = w.T2;
  double E_fro = NaN, theta_max = NaN, dk = NaN;
  int sweeps = 0, cg_total = 0;
  bool use32 = false;
  CgHost* hs = reinterpret_cast<CgHost*>(h->pinned + SC_COUNT);
  while (true) {
    // Rayleigh-Ritz on span(V) with H (FP64).
    HIPCHK(symthin_f64(w.Hf, ld, d, V, ld, k, Wm, ld, w.thin, st));
    HIPCHK(gram(V, ld, k, Wm, ld, k, d, w.G, w.gwork, st));
    HIPCHK(hipMemcpyAsync(G, w.G, sizeof(double) * k * k, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (qr_lost_rank(h)) return fail(h, REFL_ERR_NOT_CONVERGED, "Cholesky QR: block lost rank");
    if (sym_eig_small(k, G, th.data(), Q.data()) != 0)
      return fail(h, REFL_ERR_NOT_CONVERGED, "Rayleigh-Ritz eigensolver failed");
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) Cc[i + k * j] = Q[(size_t)i * k + j];  // column-major
    HIPCHK(hipMemcpyAsync(w.G, Cc, sizeof(double) * k * k, hipMemcpyHostToDevice, st));
    HIPCHK(block_axpy(d, k, k, 0.0, spare, ld, 1.0, V, ld, w.G, st));
    std::swap(V, spare);
    HIPCHK(block_axpy(d, k, k, 0.0, Wspare, ld, 1.0, Wm, ld, w.G, st));
    std::swap(Wm, Wspare);
    // Residual E = W - V Theta, projected onto the complement of V.
    for (int c = 0; c < k; ++c) nrm[c] = -th[c];
    HIPCHK(hipMemcpyAsync(w.G + MAXB * MAXB, nrm, sizeof(double) * k, hipMemcpyHostToDevice, st));
    HIPCHK(lincomb(d, k, 1.0, Wm, ld, 0.0, w.Rr, ld, st));
    HIPCHK(col_axpy(d, k, w.Rr, ld, w.G + MAXB * MAXB, V, ld, st));
    HIPCHK(gram(V, ld, k, w.Rr, ld, k, d, w.G, w.gwork, st));
    HIPCHK(block_axpy(d, k, k, 1.0, w.Rr, ld, -1.0, V, ld, w.G, st));
    HIPCHK(gram(w.Rr, ld, k, w.Rr, ld, k, d, w.G, w.gwork, st));
    HIPCHK(hipMemcpyAsync(G, w.G, sizeof(double) * k * k, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double e2 = 0.0;
    for (int c = 0; c < k; ++c) e2 += G[c + k * c];
    E_fro = std::sqrt(e2);
    theta_max = th[k - 1];
    dk = (theta_max < s) ? 2.0 * std::sqrt(2.0) * E_fro / (s - theta_max) : INFINITY;
    if (dk <= p.tol || sweeps >= p.polish_sweeps) break;
    // The inner solves may read an FP32 copy of H: each solve then corrects
    // to about u32 alpha / (s - theta_max) relative (alpha >= ||H - sI||_2,
    // s - theta_max the distance of the Ritz values to the shift), while
    // this Rayleigh-Ritz step and the certificate stay in FP64.
    if (!use32 && w.H32 &&
        (p.cg_f32 == REFL_CG_FP32 ||
         (p.cg_f32 == REFL_CG_AUTO && theta_max < s && info &&
          0x1.0p-24 * info->alpha / (s - theta_max) < 1e-3))) {
      if (!w.h32_ready) HIPCHK(launch_shifted_f32(w.Hf, w.dp, d, 0.0, w.H32, st));
      use32 = true;
    }
    // Correction: (I - VV^T)(H - theta_c)(I - VV^T) z_c = -E_c by block CG.
    // Besides its own buffers the solve uses the blocks that are free until
    // the next Rayleigh-Ritz step: spare (not V), Wm and Wspare.
    HIPCHK(lincomb(d, k, -1.0, w.Rr, ld, 0.0, w.Rr, ld, st));
    HIPCHK(lincomb(d, k, 0.0, w.Rr, ld, 0.0, w.Z, ld, st));
    const CgBufs cb = {{w.Rr, spare}, {w.P[0], w.P[1]}, {Wm, Wspare}, w.AP, w.Z, Wspare};
    std::memset(hs, 0, sizeof(CgHost));
    for (int c = 0; c < k; ++c) {
      hs->theta[c] = th[c];
      hs->rho0[c] = G[c + k * c];
    }
    hs->tol2 = p.cg_tol * p.cg_tol;
    hs->k = k;
    hs->nb = k;
    refl_status_t cr = cg_solve(h, w, use32, V, k, cb, p.cg_max_iter, hs, true);
    if (cr != REFL_OK) return cr;
    cg_total += hs->iters;
    // V <- orth(V + Z)
    HIPCHK(lincomb(d, k, 1.0, w.Z, ld, 1.0, V, ld, st));
    refl_status_t r = orthonormalise(h, w, V, spare, k);
    if (r != REFL_OK) return r;
    ++sweeps;
  }
  *Vout = V;
  if (theta_out) *theta_out = th;
  if (info) {
    info->polish_sweeps = sweeps;
    info->cg_iters = cg_total;
    info->commutator_fro = 2.0 * std::sqrt(2.0) * E_fro;
    info->dk_bound = dk;
  }
  if (!(dk <= p.tol) && p.tol > 0.0)
    return fail(h, REFL_ERR_NOT_CONVERGED, "certified bound %.3e above tol %.3e after %d sweeps",
                dk, p.tol, sweeps);
  return REFL_OK;
}

// ------------------------------------------------------------ block Lanczos
// Shift estimation (section 4.3: a partial eigensolver near the target gap,
// then the midpoint of Prop. 4.1 and the margin test of Prop. 4.2).  Block
// width b = min(k + 4, 32, d); at most floor(d / b) steps; the convergence
// test runs after step ceil((k + 1) / b) and then every ceil(64 / b) steps,
// and always at the last step.


int lz_block(int64_t d, int k) { return (int)std::min<int64_t>(std::min(k + 4, 32), d); }
int lz_cap(int64_t d, int b, int steps) {
  const int cap = (int)(d / b);
  return steps > 0 ? std::min(steps, cap) : cap;
}

void carve_lanczos(Carve& c, LzWork& z, int64_t d, int dp, int k, int steps) {
  z.b = lz_block(d, k);
  z.J = lz_cap(d, z.b, steps);
  z.nmax = (z.J + 1) * z.b;
  const int64_t ld = dp;
  z.V = c.take<double>(ld * z.nmax);
  z.W = c.take<double>(ld * z.b);
  z.C = c.take<double>((size_t)z.nmax * z.b);
  z.ppart = c.take<double>(lz_proj_part_doubles((int)d, z.nmax, z.b));
  z.gp[0] = c.take<double>(lz_gram_part_doubles((int)d, z.b));
  z.gp[1] = c.take<double>(lz_gram_part_doubles((int)d, z.b));
  z.Bacc = c.take<double>((size_t)z.b * z.b);
  z.TA = c.take<double>((size_t)z.J * z.b * z.b);
  z.TB = c.take<double>((size_t)z.J * z.b * z.b);
  z.gsum = c.take<double>((size_t)lz_nb_pad(z.b) * lz_nb_pad(z.b));
  z.flag = c.take<int>(4);
}

struct LzResult {
  double lam_k = NaN, lam_k1 = NaN, eps = NaN, s = NaN, rho = NaN;
  int steps = 0;
  bool converged = false;
};

// Runs the estimate on the padded symmetric copy Hf (ld dp).  Returns
// REFL_OK with r filled (converged or at the step cap), or a device error.
// With `start` (d x b, ld lds) the run starts from that block instead of
// the seeded one; with `ritz_out` (d x b, ld ldr) it also returns the Ritz
// vectors of its b smallest Ritz values (the warm start of a later run on a
// nearby matrix).
refl_status_t lanczos_run(refl_handle_t h, const double* Hf, int dp, int64_t d, int k, uint64_t seed,
                          LzWork& z, double* thin, LzResult& r, const double* start = nullptr,
                          int64_t lds = 0, double* ritz_out = nullptr, int64_t ldr = 0) {
  hipStream_t st = h->stream;
  const int b = z.b, J = z.J;
  const int64_t ld = dp;
  const double shift_rel = 11.0 * ((double)d * b + (double)b * (b + 1)) * 2.220446049250313e-16;
  HIPCHK(hipMemsetAsync(z.flag, 0, 4 * sizeof(int), st));
  // Q_1: the start block, orthonormalised by shifted CholQR3.
  // Rounds first..2 of CholQR3 on z.W, whose Gram partials (LZ_GRAM_ROWS-row
  // slabs) are in gp[0]; the last round writes Q to dst.  The second round
  // finishes the QR itself when its Gram matrix is already close to I, and
  // the third then does nothing.  A Lanczos step runs round 0 inside its
  // second projection pass (lz_project_qr) and starts here at round 1.
  auto cholqr3_rounds = [&](int first, double* dst, double* Arec, double* Brec,
                            int tag) -> refl_status_t {
    for (int round = first; round < 3; ++round) {
      const bool last = round == 2;
      const int mode = round == 0 ? LZ_QR_PLAIN : round == 1 ? LZ_QR_MAYBE_LAST : LZ_QR_SKIPPABLE;
      double* gin = z.gp[(round - first) & 1];
      double* gout = last ? nullptr : z.gp[(round - first + 1) & 1];
      HIPCHK(lz_cholqr(gin, round == first ? LZ_GRAM_ROWS : 256, (int)d, b, round == 0 ? shift_rel : 0.0,
                       z.Bacc, round, round >= 1 ? Arec : nullptr, round >= 1 ? Brec : nullptr, z.flag,
                       tag, z.W, ld, last ? dst : z.W, ld, gout, mode, round == 1 ? dst : nullptr, st));
    }
    return REFL_OK;
  };
  auto cholqr3 = [&](double* dst, double* Arec, double* Brec, int tag) -> refl_status_t {
    HIPCHK(lz_gram(z.W, ld, b, (int)d, z.gp[0], st));
    return cholqr3_rounds(0, dst, Arec, Brec, tag);
  };
  if (start)
    HIPCHK(hipMemcpy2DAsync(z.W, sizeof(double) * ld, start, sizeof(double) * lds,
                            sizeof(double) * d, b, hipMemcpyDeviceToDevice, st));
  else
    HIPCHK(random_block(z.W, ld, (int)d, b, seed, st));
  refl_status_t rs = cholqr3(z.V, nullptr, nullptr, 0);
  if (rs != REFL_OK) return rs;
  const int j0 = std::max(1, (k + 1 + b - 1) / b);
  // A test every ceil(64 / b) steps: testing every 2 or 4 steps (b = 9,
  // d = 4096) was slower, the host tests then falling behind the device.
  const int ci = std::max(1, (64 + b - 1) / b);
  // Pinned host copies: TA blocks, TB blocks, then two flag slots.
  const size_t blk = (size_t)b * b;
  const size_t pin_need = sizeof(double) * 2 * J * blk + 4 * sizeof(int) + 64;
  if (h->lz_pin_bytes < pin_need) {
    if (h->no_alloc)
      return fail(h, REFL_ERR_INVALID_ARG, "Lanczos staging of %zu bytes exceeds the %zu created with the handle",
                  pin_need, h->lz_pin_bytes);
    if (h->lz_pin) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipHostFree(h->lz_pin));
      h->lz_pin = nullptr;
      h->lz_pin_bytes = 0;
    }
    if (hipHostMalloc((void**)&h->lz_pin, pin_need, hipHostMallocDefault) != hipSuccess)
      return fail(h, REFL_ERR_NO_MEMORY, "pinned host buffer of %zu bytes", pin_need);
    h->lz_pin_bytes = pin_need;
  }
  for (int e = 0; e < 2; ++e)
    if (!h->lz_ev[e]) {
      if (h->no_alloc) return fail(h, REFL_ERR_DEVICE, "Lanczos events missing");
      HIPCHK(hipEventCreateWithFlags(&h->lz_ev[e], hipEventDisableTiming));
    }
  double* hTA = h->lz_pin;
  double* hTB = h->lz_pin + J * blk;
  int* hflag = reinterpret_cast<int*>(h->lz_pin + 2 * J * blk);
  // Evaluates the test made after step j (its copies in slot `slot`); sets
  // done when the run is finished (r filled).  Each test starts its
  // bisections from the previous test's Ritz values.
  RitzCheck prev_rc;
  bool have_prev = false;
  // Residual bounds of the last two evaluated tests, for the schedule below.
  int hist_j[2] = {0, 0}, nhist = 0;
  double hist_eps[2] = {NaN, NaN}, hist_gap = NaN;
  // True when the test after step jt is expected to pass: its residual
  // bound, extrapolated geometrically from the last two tests, is below
  // twice the threshold.  Such a test is evaluated two steps after it is
  // enqueued instead of one interval later, so that fewer steps run past
  // convergence.
  auto expect_pass = [&](int jt) {
    if (nhist < 2 || !(hist_eps[1] > 0.0) || !(hist_eps[0] > hist_eps[1]) || hist_j[1] <= hist_j[0])
      return false;
    const double rate = std::log(hist_eps[1] / hist_eps[0]) / (hist_j[1] - hist_j[0]);
    const double pred = hist_eps[1] * std::exp(rate * (jt - hist_j[1]));
    return pred < 0.5 * hist_gap;
  };
  auto evaluate = [&](int j, int slot, int& done) -> refl_status_t {
    done = 0;
    HIPCHK(hipEventSynchronize(h->lz_ev[slot]));
    const int* fl = hflag + 2 * slot;
    // A QR that lost rank at step jb: with only a near-invariant space (bit
    // 2) B_jb is still valid, so T_jb and its residual are used; after a
    // failed Cholesky (bit 1) the last valid state is step jb - 1.
    int jj = j;
    bool stop = (j == J);
    if (fl[1] > 0 && fl[1] <= j) {
      jj = (fl[0] & 1) ? fl[1] - 1 : fl[1];
      stop = true;
      if (jj < 1) return fail(h, REFL_ERR_NOT_CONVERGED, "Lanczos: start block lost rank");
    }
    if (jj * b < k + 1) {
      if (stop) return fail(h, REFL_ERR_NOT_CONVERGED, "Lanczos: basis too small for k=%d", k);
      return REFL_OK;
    }
    RitzCheck rc;
    ritz_check(jj, b, k, hTA, hTB, false, rc, have_prev ? &prev_rc : nullptr);
    const double eps = std::max(rc.res_k, rc.res_k1);
    const bool conv = eps < 0.25 * (rc.th_k1 - rc.th_k);
    hist_j[0] = hist_j[1];
    hist_eps[0] = hist_eps[1];
    hist_j[1] = jj;
    hist_eps[1] = eps;
    hist_gap = rc.th_k1 - rc.th_k;
    ++nhist;
    // The extreme Ritz values are needed by the last test only.  They are
    // first found (from the Gershgorin bounds) by the test before the one
    // expected to pass, while the device still runs a full interval of
    // steps, and then followed from test to test (a few inertia counts).
    const bool had_ext = have_prev && std::isfinite(prev_rc.th_min);
    if (conv || stop || had_ext || expect_pass(jj + ci))
      ritz_extremes(jj, b, hTA, hTB, rc, had_ext ? &prev_rc : nullptr);
    prev_rc = rc;
    have_prev = true;
    if (conv || stop) {
      r.lam_k = rc.th_k;
      r.lam_k1 = rc.th_k1;
      r.eps = eps;
      r.s = 0.5 * (rc.th_k + rc.th_k1);
      r.rho = std::max(rc.th_max - r.s, r.s - rc.th_min);
      r.steps = jj;
      r.converged = conv;
      done = 1;
    }
    return REFL_OK;
  };
  // Ritz block of the finished run (r.steps steps): Y from the band matrix on
  // the host, then ritz_out = V Y on the device.  The copy of -Y is
  // enqueued behind the steps still in flight, which read z.C; the stream is
  // synchronised before Y goes out of scope.
  auto ritz_block = [&]() -> refl_status_t {
    if (!ritz_out) return REFL_OK;
    const int n = r.steps * b;
    std::vector<double> Y((size_t)n * b);
    if (n < b || ritz_vectors(r.steps, b, hTA, hTB, b, Y.data()) != 0)
      return fail(h, REFL_ERR_NOT_CONVERGED, "Lanczos: no Ritz block for the warm start");
    for (double& v : Y) v = -v;
    HIPCHK(hipMemcpyAsync(z.C, Y.data(), sizeof(double) * Y.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemset2DAsync(z.W, sizeof(double) * ld, 0, sizeof(double) * d, b, st));
    HIPCHK(lz_combine(z.V, ld, n, z.C, b, (int)d, z.W, z.W, ld, st));
    HIPCHK(hipMemcpy2DAsync(ritz_out, sizeof(double) * ldr, z.W, sizeof(double) * ld,
                            sizeof(double) * d, b, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return REFL_OK;
  };
  // The test after step j is evaluated on the host while the device runs
  // the steps up to the next test, or only the next two steps when the test
  // is expected to pass (steps enqueued past convergence are discarded).
  int pending = -1, pending_slot = 0, pending_lead = 0, ntest = 0, copied = 0;
  for (int j = 1; j <= J; ++j) {
    const int n = j * b;
    const double* Qj = z.V + (int64_t)(n - b) * ld;
    double* Aj = z.TA + (size_t)(j - 1) * blk;
    double* Bj = z.TB + (size_t)(j - 1) * blk;
    HIPCHK(symthin_f64(Hf, ld, (int)d, Qj, ld, b, z.W, ld, thin, st));
    if ((int64_t)n >= d) {
      HIPCHK(lz_project(z.V, ld, n, z.W, ld, b, (int)d, z.C, Aj, b, 0, z.ppart, nullptr, st));
      HIPCHK(lz_project(z.V, ld, n, z.W, ld, b, (int)d, z.C, Aj, b, 1, z.ppart, nullptr, st));
      HIPCHK(hipMemsetAsync(Bj, 0, sizeof(double) * blk, st));  // the basis spans R^d
    } else {
      // The first pass leaves the Gram partials of its output in gp[1]; the
      // second runs CholQR3's round 0 on them and leaves those of its
      // output in gp[0] for rounds 1 and 2.
      HIPCHK(lz_project(z.V, ld, n, z.W, ld, b, (int)d, z.C, Aj, b, 0, z.ppart, z.gp[1], st));
      HIPCHK(lz_project_qr(z.V, ld, n, z.W, ld, b, (int)d, z.C, Aj, b, 1, z.ppart, z.gp[1], z.gsum,
                           shift_rel, z.Bacc, z.flag, j, z.gp[0], st));
      refl_status_t rq = cholqr3_rounds(1, z.V + (int64_t)n * ld, Aj, Bj, j);
      if (rq != REFL_OK) return rq;
    }
    // A warm start may converge within a few steps: those are all tested.
    const bool test = (j >= j0 && ((j - j0) % ci == 0 || (start && j - j0 < 4))) || j == J;
    if (!test) {
      if (pending > 0 && j - pending >= pending_lead) {
        int done = 0;
        refl_status_t e = evaluate(pending, pending_slot, done);
        if (e == REFL_OK && done) e = ritz_block();
        if (e != REFL_OK || done) {
          HIPCHK(hipStreamSynchronize(st));
          return e;
        }
        pending = -1;
      }
      continue;
    }
    const int slot = ntest++ & 1;
    const size_t nb_new = (size_t)(j - copied) * blk;
    HIPCHK(hipMemcpyAsync(hTA + copied * blk, z.TA + copied * blk, sizeof(double) * nb_new,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hTB + copied * blk, z.TB + copied * blk, sizeof(double) * nb_new,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hflag + 2 * slot, z.flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(h->lz_ev[slot], st));
    copied = j;
    if (pending > 0) {
      int done = 0;
      refl_status_t e = evaluate(pending, pending_slot, done);
      if (e == REFL_OK && done) e = ritz_block();
      if (e != REFL_OK || done) {
        HIPCHK(hipStreamSynchronize(st));
        return e;
      }
    }
    pending = j;
    pending_slot = slot;
    pending_lead = expect_pass(j) ? 2 : J;
  }
  if (pending > 0) {
    int done = 0;
    refl_status_t e = evaluate(pending, pending_slot, done);
    if (e == REFL_OK && done) e = ritz_block();
    HIPCHK(hipStreamSynchronize(st));
    if (e != REFL_OK || done) return e;
  }
  return fail(h, REFL_ERR_NOT_CONVERGED, "Lanczos: no test at the step cap");
}

// Status of an estimate by Prop. 4.2: the margin m_hat must exceed eps.
refl_status_t lanczos_status(refl_handle_t h, const LzResult& r) {
  const double gap = r.lam_k1 - r.lam_k;
  if (!(gap > 1e-14 * std::max(std::fabs(r.lam_k), std::fabs(r.lam_k1))))
    return fail(h, REFL_ERR_NO_GAP, "Lanczos estimates of lambda_k and lambda_k+1 coincide (%.6e, %.6e)",
                r.lam_k, r.lam_k1);
  const double m_hat = std::min(r.s - r.lam_k, r.lam_k1 - r.s);
  if (!(m_hat > r.eps))
    return fail(h, REFL_ERR_NOT_ADMISSIBLE,
                "Lanczos margin %.3e does not exceed the residual bound %.3e after %d steps", m_hat,
                r.eps, r.steps);
  return REFL_OK;
}

// Shared body of refl_sign and refl_sign_apply.  If dR is non-null, R is
// written; otherwise dY = R dV.
// What a MIXED solve leaves for a later step in the same workspace (the
// gradient of the limit, refl_sign_grad): the layout, the final Ritz basis V
// (d x k, ld dp) and its Ritz values, ascending.  V spans the certified
// eigenspace, so R = I - 2 V V^T.
struct MixedKeep {
  Work w;
  double* V = nullptr;
  int k = 0;
  std::vector<double> theta;
};

// MIXED: the largest word count the call may escalate to.
int words_cap(const refl_params_t& p) { return p.words_max > 0 ? p.words_max : p.words; }

// Estimated scaled margin below which the MIXED bulk starts with three words
// (measured on planted spectra at d = 1024: at gamma = 3e-6 and below the
// two-word bulk needs a second correction sweep and the three-word one does
// not; at 9e-6 both need one and two words are faster).
constexpr double GAMMA_BF16X6 = 5e-6;

refl_status_t sign_impl(refl_handle_t h, int64_t d, const double* dH, int64_t ldh,
                        const refl_params_t* pin, double* dR, int64_t ldr, int64_t nrhs,
                        const double* dV, int64_t ldv, double* dY, int64_t ldy,
                        refl_info_t* info, MixedKeep* keep = nullptr);

// The MIXED call again with `words` words per operand, the shift s and the
// scale of the first attempt (given), the Lanczos estimates of the first
// attempt carried into info, and the first attempt's time added to the
// set-up time.
refl_status_t restart_words(refl_handle_t h, int64_t d, const double* dH, int64_t ldh,
                            const refl_params_t& p, int words, double s, const refl_info_t& first,
                            double t_start, double* dR, int64_t ldr, int64_t nrhs,
                            const double* dV, int64_t ldv, double* dY, int64_t ldy,
                            refl_info_t* info, MixedKeep* keep) {
  refl_params_t q = p;
  q.words = words;
  q.shift_mode = REFL_SHIFT_GIVEN;
  q.s = s;
  q.scale_mode = REFL_SCALE_GIVEN;
  q.alpha = first.alpha;
  q.check_symmetric = 0;
  refl_info_t inf2;
  const double t_restart = now_ms();
  const refl_status_t r = sign_impl(h, d, dH, ldh, &q, dR, ldr, nrhs, dV, ldv, dY, ldy, &inf2, keep);
  if (info) {
    inf2.lanczos_steps = first.lanczos_steps;
    inf2.lam_k = first.lam_k;
    inf2.lam_k1 = first.lam_k1;
    inf2.eps = first.eps;
    inf2.margin = first.margin;
    inf2.rho = first.rho;
    inf2.gamma = first.gamma;
    inf2.ms_setup += t_restart - t_start;
    inf2.ms_total += t_restart - t_start;
    *info = inf2;
  }
  return r;
}

refl_status_t sign_impl(refl_handle_t h, int64_t d, const double* dH, int64_t ldh,
                        const refl_params_t* pin, double* dR, int64_t ldr, int64_t nrhs,
                        const double* dV, int64_t ldv, double* dY, int64_t ldy,
                        refl_info_t* info, MixedKeep* keep) {
  const double t_start = now_ms();
  refl_status_t rs = check_params(h, d, pin);
  if (rs != REFL_OK) return rs;
  if (!dH || ldh < d) return fail(h, REFL_ERR_INVALID_ARG, "H is NULL or ldh < d");
  refl_params_t p = *pin;
  refl_info_t inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.lam_k = inf.lam_k1 = inf.eps = inf.margin = NaN;
  inf.commutator_fro = inf.dk_bound = NaN;
  inf.rho = inf.gamma = NaN;
  inf.index_j = -1;
  HIPCHK(hipSetDevice(h->device));
  Work w;
  const size_t need = layout(w, nullptr, d, p, LAYOUT_SIGN, h);
  void* base = nullptr;
  rs = ensure_workspace(h, need, &base);
  if (rs != REFL_OK) return rs;
  layout(w, base, d, p, LAYOUT_SIGN, h);
  inf.bulk_tile = w.ts;
  inf.bulk_words = p.precision == REFL_PREC_MIXED ? p.words : 0;
  hipStream_t st = h->stream;
  double* hsc = h->pinned;
  if (p.check_symmetric) {
    rs = check_symmetry(h, d, dH, ldh, p.sym_tol, w.scal, SC_SYM);
    if (rs != REFL_OK) return rs;
  }

  // ---- set-up ----
  std::vector<int2> tl;
  build_tiles(w, tl);
  HIPCHK(hipMemcpyAsync(w.tiles, tl.data(), sizeof(int2) * tl.size(), hipMemcpyHostToDevice, st));
  HIPCHK(launch_mirror_upper(dH, ldh, (int)d, w.Hf, w.dp, st));
  double alpha_given = p.alpha;
  if (p.shift_mode == REFL_SHIFT_LANCZOS) {
    LzResult lr;
    rs = lanczos_run(h, w.Hf, w.dp, d, p.k, p.seed, w.lz, w.thin, lr);
    if (rs != REFL_OK) return rs;
    inf.lanczos_steps = lr.steps;
    inf.lam_k = lr.lam_k;
    inf.lam_k1 = lr.lam_k1;
    inf.eps = lr.eps;
    inf.margin = std::min(lr.s - lr.lam_k, lr.lam_k1 - lr.s) - lr.eps;
    inf.s = lr.s;
    rs = lanczos_status(h, lr);
    if (rs != REFL_OK) {
      if (info) *info = inf;
      return rs;
    }
    p.s = lr.s;
    inf.rho = lr.rho;
    if (p.scale_mode == REFL_SCALE_LANCZOS) alpha_given = 1.05 * lr.rho;
  }
  const double s = p.s;
  inf.s = s;
  HIPCHK(launch_scale_inf(w.Hf, w.dp, (int)d, s, p.scale_mode == REFL_SCALE_FRO,
                          p.scale_mode == REFL_SCALE_GIVEN || p.scale_mode == REFL_SCALE_LANCZOS,
                          alpha_given,
                          w.rowsum, w.scal, st));
  const int W = p.words;
  if (p.precision == REFL_PREC_FP64) {
    HIPCHK(launch_init_x0_f64(w.Hf, w.dp, (int)d, s, w.scal, w.X64[0], st));
    HIPCHK(launch_trace_f64(w.X64[0], w.dp, (int)d, w.scal, SC_TRACE, st));
  } else if (p.precision == REFL_PREC_FP32) {
    HIPCHK(launch_init_x0_f32(w.Hf, w.dp, (int)d, s, w.scal, w.X32[0], st));
    HIPCHK(launch_trace_f32(w.X32[0], w.dp, (int)d, w.scal, SC_TRACE, st));
  } else {
    HIPCHK(launch_init_x0_words(W, w.Hf, w.dp, (int)d, s, w.scal, w.Xw[0], w.ps, w.H32, st));
    w.h32_ready = w.H32 != nullptr;
    HIPCHK(launch_trace_words(W, w.Xw[0], w.ps, w.dp, (int)d, w.scal, SC_TRACE, st));
  }
  HIPCHK(hipMemcpyAsync(hsc, w.scal, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hsc[SC_NONFINITE] > 0.0) return fail(h, REFL_ERR_NOT_FINITE, "H holds non-finite entries");
  inf.alpha = hsc[SC_ALPHA];
  if (!(inf.alpha > 0.0) || !std::isfinite(inf.alpha))
    return fail(h, REFL_ERR_NOT_FINITE, "scale alpha=%g is not a positive finite number", inf.alpha);
  if (p.shift_mode == REFL_SHIFT_LANCZOS)
    inf.gamma = std::min(s - inf.lam_k, inf.lam_k1 - s) / inf.alpha;
  // Bulk precision from the estimated scaled margin: below GAMMA_BF16X6 the
  // three-word bulk certifies the index with one correction sweep where two
  // words need two, so the call restarts with three words (same shift and
  // scale, the Lanczos results carried over).
  if (p.precision == REFL_PREC_MIXED && p.fixed_steps == 0 && p.shift_mode == REFL_SHIFT_LANCZOS &&
      p.words < 3 && words_cap(p) >= 3 && inf.gamma < GAMMA_BF16X6)
    return restart_words(h, d, dH, ldh, p, 3, s, inf, t_start, dR, ldr, nrhs, dV, ldv, dY, ldy, info,
                         keep);
  const double t_setup = now_ms();

  // ---- bulk ----
  Bulk b;
  double trace_cur = hsc[SC_TRACE];
  const bool fixed = p.fixed_steps > 0;
  const int cap = fixed ? p.fixed_steps : p.max_iter;
  // Optional event pairs around each bulk product (2 per step).
  size_t nev = 0;
  const size_t max_ev = 2 * (size_t)(cap + 2);
  if (p.timing) {
    if (h->no_alloc && h->ev.size() < 2 * max_ev)
      return fail(h, REFL_ERR_INVALID_ARG, "params.timing creates events: not available without allocation");
    // Timing only: no system-scope fence at each record (the cache
    // writeback and invalidation it implies cost about 10 us per step).
    while (h->ev.size() < 2 * max_ev) {
      hipEvent_t e;
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      h->ev.push_back(e);
    }
  }
  auto ev_start = [&]() -> hipError_t {
    return p.timing ? hipEventRecord(h->ev[2 * nev], st) : hipSuccess;
  };
  auto ev_stop = [&]() -> hipError_t {
    if (!p.timing) return hipSuccess;
    hipError_t e = hipEventRecord(h->ev[2 * nev + 1], st);
    ++nev;
    return e;
  };
  int bulk_extra = 0;
  if (const char* e = std::getenv("REFL_BULK_EXTRA")) bulk_extra = std::max(0, std::atoi(e));
  refl_status_t bulk_status = REFL_OK;
  if (p.precision == REFL_PREC_MIXED && !fixed) {
    // MIXED bulk: the stopping rule (index certificate, then the words'
    // floor; MixedRule in launch.h) runs on the device after each residual
    // product (k_reduce_decide), so the host enqueues steps four at a time
    // and keeps one group queued beyond the one whose step record it reads;
    // the products of steps past the stop read the device flag and return at
    // once.  X_m lives in buffer m % 3.  Rule, record, flag and step counter
    // are staged like the FP32 / FP64 path's; the record is copied back after
    // each group into one of two host slots.
    constexpr int STEPS_AHEAD = 4;
    char* hs = reinterpret_cast<char*>(h->pinned + SC_COUNT) + sizeof(CgHost);
    char* ds = reinterpret_cast<char*>(w.scal + SC_SCRATCH + 4);
    MixedRule* ru = reinterpret_cast<MixedRule*>(hs);
    BatchStep* sq = reinterpret_cast<BatchStep*>(hs + 16);
    int* hlive = reinterpret_cast<int*>(hs + 64);
    int* hctl = reinterpret_cast<int*>(hs + 72);
    char* rec[2] = {hs + 96, hs + 160};  // BatchStep, live, ctl of ds + 16 .. ds + 80
    const MixedRule* d_ru = reinterpret_cast<const MixedRule*>(ds);
    BatchStep* d_sq = reinterpret_cast<BatchStep*>(ds + 16);
    int* d_live = reinterpret_cast<int*>(ds + 64);
    int* d_ctl = reinterpret_cast<int*>(ds + 72);
    ru->d = (int)d;
    ru->extra = bulk_extra;
    ru->cap = cap;
    ru->pad = 0;
    std::memset(sq, 0, sizeof(BatchStep));
    sq->trace = trace_cur;
    sq->resid = NaN;
    sq->state = BATCH_LIVE;
    *hlive = 1;
    hctl[0] = 0;
    hctl[1] = 1;
    HIPCHK(hipMemcpyAsync(ds, hs, 80, hipMemcpyHostToDevice, st));
    std::vector<hipEvent_t>& lev = h->bulk_ev;
    while ((int)lev.size() < 2) {
      if (h->no_alloc) return fail(h, REFL_ERR_DEVICE, "bulk events missing");
      hipEvent_t e;
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      lev.push_back(e);
    }
    // With params.timing = N > 1 only the products of every N-th step are
    // timed (each event pair costs the device some microseconds).
    const int tstride = p.timing > 1 ? p.timing : 1;
    auto enqueue_step = [&](int m) -> hipError_t {
      uint16_t* Xm = w.Xw[m % 3];
      uint16_t* Xn = w.Xw[(m + 1) % 3];
      const bool tm = m % tstride == 0;
      hipError_t e;
      if (tm && (e = ev_start()) != hipSuccess) return e;
      if ((e = launch_sym_gemm_words(W, w.ts, GEMM_RESIDUAL, Xm, Xm, nullptr, w.Nw, w.dp, w.ps, (int)d,
                                     w.dk, w.tiles, w.ntiles, w.partials, st, d_live)) != hipSuccess)
        return e;
      if (tm && (e = ev_stop()) != hipSuccess) return e;
      if ((e = launch_reduce_decide(w.partials, w.partials_t, w.ntiles, w.scal, d_ru, d_sq, d_live,
                                    d_ctl, m % 3, st)) != hipSuccess)
        return e;
      if (tm && (e = ev_start()) != hipSuccess) return e;
      if ((e = launch_sym_gemm_words(W, w.ts, GEMM_UPDATE, Xm, w.Nw, Xm, Xn, w.dp, w.ps, (int)d, w.dk,
                                     w.tiles, w.ntiles, w.partials_t, st, d_live)) != hipSuccess)
        return e;
      return tm ? ev_stop() : hipSuccess;
    };
    int enq = 0;  // steps enqueued
    int group = STEPS_AHEAD;
    auto enqueue_group = [&](int slot) -> hipError_t {
      hipError_t e = hipSuccess;
      for (int i = 0; i < group && enq <= cap && e == hipSuccess; ++i, ++enq) e = enqueue_step(enq);
      if (e == hipSuccess) e = hipMemcpyAsync(rec[slot], ds + 16, 64, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipEventRecord(lev[slot], st);
      return e;
    };
    HIPCHK(enqueue_group(0));
    int last = 0;  // last group enqueued
    bool stopped = false;
    for (int g = 0;; ++g) {
      if (last == g && enq <= cap) {
        HIPCHK(enqueue_group((g + 1) & 1));
        last = g + 1;
      }
      HIPCHK(hipEventSynchronize(lev[g & 1]));
      const int* rctl = reinterpret_cast<const int*>(rec[g & 1] + 56);
      if (rctl[1] == 0) {
        std::memcpy(sq, rec[g & 1], sizeof(BatchStep));
        stopped = true;
        break;
      }
      if (last == g) break;
      // Near the hand-over (the certificate needs sqrt(d) r < 1, and a step
      // roughly squares a small residual) the groups shrink to one step, so
      // that few steps past the stop are queued.
      const double r_last = reinterpret_cast<const BatchStep*>(rec[g & 1])->resid;
      if (std::isfinite(r_last) && std::sqrt((double)d) * r_last < 64.0) group = 1;
    }
    if (!stopped) {
      if (info) *info = inf;
      return fail(h, REFL_ERR_DEVICE, "bulk iteration still running after the step limit");
    }
    b.steps = sq->m;
    b.cur = sq->par;
    b.resid = sq->resid;
    b.trace = sq->trace;
    b.converged = sq->state == BATCH_CONVERGED;
    if (sq->state == BATCH_NONFINITE)
      bulk_status = fail(h, REFL_ERR_NOT_FINITE, "iterate diverged at step %d", b.steps);
    // Timed launches: those of the steps taken (residual products of steps
    // 0..m, update products of steps 0..m-1), in enqueue order.
    size_t taken = 0;
    for (int m = 0; m <= b.steps; m += tstride) taken += m < b.steps ? 2 : 1;
    nev = std::min(nev, taken);
  } else if (p.precision != REFL_PREC_MIXED && small_order(d, p.precision == REFL_PREC_FP64)) {
    // Every step in one launch, X and N held in LDS, the stopping rule on
    // the device.  Problem, rule and step record are staged through the
    // pinned tail of the scalar block and free scalar slots on the device.
    const bool f64 = p.precision == REFL_PREC_FP64;
    char* hs = reinterpret_cast<char*>(h->pinned + SC_COUNT) + sizeof(CgHost);
    char* ds = reinterpret_cast<char*>(w.scal + SC_SCRATCH + 4);
    SmallProb* sp = reinterpret_cast<SmallProb*>(hs);
    BatchRule* ru = reinterpret_cast<BatchRule*>(hs + 32);
    BatchStep* sq = reinterpret_cast<BatchStep*>(hs + 48);
    sp->X[0] = f64 ? (void*)w.X64[0] : (void*)w.X32[0];
    sp->X[1] = f64 ? (void*)w.X64[1] : (void*)w.X32[1];
    sp->d = (int)d;
    sp->dp = w.dp;
    sp->slot = 0;
    sp->pad = 0;
    ru->tol = p.tol;
    ru->fixed_steps = p.fixed_steps;
    ru->max_iter = p.max_iter;
    std::memset(sq, 0, sizeof(BatchStep));
    sq->trace = trace_cur;
    sq->resid = NaN;
    sq->state = BATCH_LIVE;
    HIPCHK(hipMemcpyAsync(ds, hs, 96, hipMemcpyHostToDevice, st));
    HIPCHK(ev_start());
    HIPCHK(launch_ns_small(f64, reinterpret_cast<const SmallProb*>(ds), 1,
                           reinterpret_cast<const BatchRule*>(ds + 32),
                           reinterpret_cast<BatchStep*>(ds + 48), st));
    HIPCHK(ev_stop());
    HIPCHK(hipMemcpyAsync(sq, ds + 48, sizeof(BatchStep), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    b.steps = sq->m;
    b.cur = sq->par;
    b.resid = sq->resid;
    b.trace = sq->trace;
    b.converged = sq->state == BATCH_CONVERGED;
    if (sq->state == BATCH_NONFINITE)
      bulk_status = fail(h, REFL_ERR_NOT_FINITE, "iterate diverged at step %d", b.steps);
  } else if (p.precision != REFL_PREC_MIXED) {
    // FP32 / FP64: the stopping rule runs on the device after each residual
    // product (k_batch_decide on this one problem: the rule of the host loop
    // below, step for step), so the host enqueues STEPS_AHEAD steps at a time
    // and reads the step record once per group; the products of steps past
    // the stop find *live == 0 and do nothing.  Rule, record, live flag and
    // step counter are staged like the small-order launch's.
    constexpr int STEPS_AHEAD = 4;
    const bool f64 = p.precision == REFL_PREC_FP64;
    char* hs = reinterpret_cast<char*>(h->pinned + SC_COUNT) + sizeof(CgHost);
    char* ds = reinterpret_cast<char*>(w.scal + SC_SCRATCH + 4);
    BatchRule* ru = reinterpret_cast<BatchRule*>(hs);
    BatchStep* sq = reinterpret_cast<BatchStep*>(hs + 16);
    int* hlive = reinterpret_cast<int*>(hs + 64);
    int* hctl = reinterpret_cast<int*>(hs + 72);
    BatchRule* d_ru = reinterpret_cast<BatchRule*>(ds);
    BatchStep* d_sq = reinterpret_cast<BatchStep*>(ds + 16);
    int* d_live = reinterpret_cast<int*>(ds + 64);
    int* d_ctl = reinterpret_cast<int*>(ds + 72);
    ru->tol = p.tol;
    ru->fixed_steps = p.fixed_steps;
    ru->max_iter = p.max_iter;
    std::memset(sq, 0, sizeof(BatchStep));
    sq->trace = trace_cur;
    sq->resid = NaN;
    sq->state = BATCH_LIVE;
    *hlive = 1;
    hctl[0] = 0;
    hctl[1] = 1;
    HIPCHK(hipMemcpyAsync(ds, hs, 80, hipMemcpyHostToDevice, st));
    auto product = [&](int mode, int c, hipStream_t ss) -> hipError_t {
      if (f64)
        return mode == GEMM_RESIDUAL
                   ? launch_sym_gemm_f64(w.ts, mode, w.X64[c], w.X64[c], nullptr, w.N64, w.dp, (int)d,
                                         w.dp, w.tiles, w.ntiles, w.partials, ss, d_live)
                   : launch_sym_gemm_f64(w.ts, mode, w.X64[c], w.N64, w.X64[c], w.X64[c ^ 1], w.dp,
                                         (int)d, w.dp, w.tiles, w.ntiles, w.partials_t, ss, d_live);
      return mode == GEMM_RESIDUAL
                 ? launch_sym_gemm_f32(w.ts, mode, w.X32[c], w.X32[c], nullptr, w.N32, w.dp, (int)d,
                                       w.dp, w.tiles, w.ntiles, w.partials, ss, d_live)
                 : launch_sym_gemm_f32(w.ts, mode, w.X32[c], w.N32, w.X32[c], w.X32[c ^ 1], w.dp,
                                       (int)d, w.dp, w.tiles, w.ntiles, w.partials_t, ss, d_live);
    };
    // One step on stream ss (timing events on the handle's stream).
    auto enqueue_step = [&](int c, hipStream_t ss) -> hipError_t {
      const bool ev = ss == st;
      hipError_t e;
      if (ev && (e = ev_start()) != hipSuccess) return e;
      if ((e = product(GEMM_RESIDUAL, c, ss)) != hipSuccess) return e;
      if (ev && (e = ev_stop()) != hipSuccess) return e;
      if ((e = launch_reduce_decide(w.partials, w.partials_t, w.ntiles, w.scal, d_ru, d_sq, d_live,
                                    d_ctl, c, ss)) != hipSuccess)
        return e;
      if (ev && (e = ev_start()) != hipSuccess) return e;
      if ((e = product(GEMM_UPDATE, c, ss)) != hipSuccess) return e;
      if (ev && (e = ev_stop()) != hipSuccess) return e;
      return hipSuccess;
    };
    // (Capturing a group of steps as a HIP graph was measured as well: no
    // faster at d = 64 .. 2048, the step time being the device's, and each
    // call pays the instantiation.)
    int enq = 0;  // steps enqueued (step m uses X[m & 1])
    hipError_t le = hipSuccess;
    for (;;) {
      for (int i = 0; i < STEPS_AHEAD && enq <= cap && le == hipSuccess; ++i, ++enq)
        le = enqueue_step(enq & 1, st);
      if (le == hipSuccess) le = hipMemcpyAsync(hs + 16, ds + 16, 64, hipMemcpyDeviceToHost, st);
      if (le == hipSuccess) le = hipStreamSynchronize(st);
      if (le != hipSuccess || hctl[1] == 0 || enq > cap) break;
    }
    if (le != hipSuccess) return fail(h, REFL_ERR_DEVICE, "steps: %s", hipGetErrorString(le));
    if (hctl[1] != 0) {
      if (info) *info = inf;
      return fail(h, REFL_ERR_DEVICE, "iteration still running after the step limit");
    }
    b.steps = sq->m;
    b.cur = sq->par;
    b.resid = sq->resid;
    b.trace = sq->trace;
    b.converged = sq->state == BATCH_CONVERGED;
    if (sq->state == BATCH_NONFINITE)
      bulk_status = fail(h, REFL_ERR_NOT_FINITE, "iterate diverged at step %d", b.steps);
    // Timed launches: only those of the steps taken (residual products of
    // steps 0..m, update products of steps 0..m-1), not the skipped ones.
    nev = std::min(nev, (size_t)(2 * b.steps + 1));
  } else {
    // MIXED with a fixed depth (the finite-step filter p_m in BF16 words):
    // m steps, each residual product read back for the reported residual.
    while (true) {
      const int c = b.cur;
      HIPCHK(ev_start());
      HIPCHK(launch_sym_gemm_words(W, w.ts, GEMM_RESIDUAL, w.Xw[c], w.Xw[c], nullptr, w.Nw, w.dp,
                                   w.ps, (int)d, w.dk, w.tiles, w.ntiles, w.partials, st));
      HIPCHK(ev_stop());
      HIPCHK(launch_reduce_sum(w.partials, w.ntiles, w.scal, SC_RESID2, st));
      HIPCHK(hipMemcpyAsync(hsc + SC_RESID2, w.scal + SC_RESID2, sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      const double resid = std::sqrt(std::fmax(hsc[SC_RESID2], 0.0));
      b.resid = resid;
      b.trace = trace_cur;
      if (!std::isfinite(resid)) {
        bulk_status = fail(h, REFL_ERR_NOT_FINITE, "iterate diverged at step %d", b.steps);
        break;
      }
      if (b.steps >= cap) {
        b.converged = true;
        break;
      }
      HIPCHK(ev_start());
      HIPCHK(launch_sym_gemm_words(W, w.ts, GEMM_UPDATE, w.Xw[c], w.Nw, w.Xw[c], w.Xw[c ^ 1], w.dp,
                                   w.ps, (int)d, w.dk, w.tiles, w.ntiles, w.partials, st));
      HIPCHK(ev_stop());
      HIPCHK(launch_reduce_sum(w.partials, w.ntiles, w.scal, SC_TRACE, st));
      HIPCHK(hipMemcpyAsync(hsc + SC_TRACE, w.scal + SC_TRACE, sizeof(double), hipMemcpyDeviceToHost, st));
      b.cur ^= 1;
      b.steps += 1;
      HIPCHK(hipStreamSynchronize(st));
      trace_cur = hsc[SC_TRACE];
    }
  }
  if (p.timing) {
    HIPCHK(hipStreamSynchronize(st));
    double tot = 0.0;
    for (size_t i = 0; i < nev; ++i) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]));
      tot += ms;
    }
    inf.ms_gemm = tot;
    inf.gemm_launches = (int)nev;
  }
  inf.ns_steps = b.steps;
  inf.resid_fro = b.resid;
  inf.trace = b.trace;
  inf.index_j = index_certificate(d, b.resid, b.trace);
  const double t_bulk = now_ms();
  if (bulk_status != REFL_OK) {
    if (info) *info = inf;
    return bulk_status;
  }

  // ---- output ----
  refl_status_t out_status = REFL_OK;
  if (!b.converged) out_status = fail(h, REFL_ERR_NOT_CONVERGED, "no convergence after %d steps (resid %.3e)", b.steps, b.resid);
  if (!fixed && p.k > 0 && inf.index_j >= 0 && inf.index_j != p.k)
    out_status = fail(h, REFL_ERR_NOT_ADMISSIBLE,
                      "index certificate found %d negative eigenvalues of H - sI, not k=%d",
                      inf.index_j, p.k);
  const int c = b.cur;
  // Precision escalation: a bulk that ended without the index certificate,
  // or (target k given) with another index, is run again with one more word
  // per operand while words_max allows.
  if (p.precision == REFL_PREC_MIXED && !fixed && p.words < words_cap(p) &&
      (!b.converged || inf.index_j < 0 || (p.k > 0 && inf.index_j != p.k)))
    return restart_words(h, d, dH, ldh, p, p.words + 1, s, inf, t_start, dR, ldr, nrhs, dV, ldv, dY, ldy,
                         info, keep);
  if (p.precision == REFL_PREC_MIXED && !fixed) {
    if (inf.index_j < 0 || (p.k > 0 && inf.index_j != p.k)) {
      if (out_status == REFL_OK)
        out_status = fail(h, REFL_ERR_NOT_ADMISSIBLE, "index certificate did not hold for k=%d", p.k);
      if (info) *info = inf;
      return out_status;
    }
    if (p.k == 0) {
      // No target index: the certified one.  With j = 0 or d, H - sI is
      // definite and R = sgn(H - sI) = +I or -I exactly.
      const int j = inf.index_j;
      if (j == 0 || j == d) {
        const double sg = j == 0 ? 1.0 : -1.0;
        if (keep) {
          keep->w = w;
          keep->V = nullptr;
          keep->k = j;
        }
        if (dR) {
          HIPCHK(form_reflector(w.V, w.dp, 0, (int)d, dR, ldr, st));
          if (sg < 0.0) HIPCHK(lincomb((int)d, (int)d, 0.0, dR, ldr, -1.0, dR, ldr, st));
        } else {
          for (int64_t c0 = 0; c0 < nrhs; c0 += MAXB) {
            const int nb = (int)std::min<int64_t>(MAXB, nrhs - c0);
            HIPCHK(lincomb((int)d, nb, sg, dV + c0 * ldv, ldv, 0.0, dY + c0 * ldy, ldy, st));
          }
        }
        HIPCHK(hipStreamSynchronize(st));
        if (info) *info = inf;
        return out_status;
      }
      if (j > MAXB) {
        if (info) *info = inf;
        return fail(h, REFL_ERR_UNSUPPORTED, "certified index %d: MIXED correction supports up to %d", j, MAXB);
      }
      p.k = j;
    }
    double* V = nullptr;
    refl_status_t pr = polish(h, w, p, s, w.Xw[c], &V, &inf, keep ? &keep->theta : nullptr);
    if (keep) {
      keep->w = w;
      keep->V = V;
      keep->k = p.k;
    }
    if (pr != REFL_OK && pr != REFL_ERR_NOT_CONVERGED) {
      if (info) *info = inf;
      return pr;
    }
    if (out_status == REFL_OK) out_status = pr;
    if (dR) {
      HIPCHK(form_reflector(V, w.dp, p.k, (int)d, dR, ldr, st));
    } else {
      // Y = V_in - 2 V (V^T V_in), in blocks of MAXB columns.
      for (int64_t c0 = 0; c0 < nrhs; c0 += MAXB) {
        const int nb = (int)std::min<int64_t>(MAXB, nrhs - c0);
        HIPCHK(gram(V, w.dp, p.k, dV + c0 * ldv, ldv, nb, (int)d, w.G, w.gwork, st));
        HIPCHK(lincomb((int)d, nb, 1.0, dV + c0 * ldv, ldv, 0.0, dY + c0 * ldy, ldy, st));
        HIPCHK(block_axpy((int)d, p.k, nb, 1.0, dY + c0 * ldy, ldy, -2.0, V, w.dp, w.G, st));
      }
    }
  } else {
    if (dR) {
      if (p.precision == REFL_PREC_FP64)
        HIPCHK(launch_copy_out_f64(w.X64[c], w.dp, (int)d, dR, ldr, st));
      else if (p.precision == REFL_PREC_FP32)
        HIPCHK(launch_copy_out_f32(w.X32[c], w.dp, (int)d, dR, ldr, st));
      else
        HIPCHK(launch_copy_out_words(W, w.Xw[c], w.ps, w.dp, (int)d, dR, ldr, st));
    } else {
      for (int64_t c0 = 0; c0 < nrhs; c0 += MAXB) {
        const int nb = (int)std::min<int64_t>(MAXB, nrhs - c0);
        if (p.precision == REFL_PREC_FP64)
          HIPCHK(thin_gemm_f64(w.X64[c], w.dp, (int)d, dV + c0 * ldv, ldv, nb, dY + c0 * ldy, ldy, w.thin, st));
        else if (p.precision == REFL_PREC_FP32)
          HIPCHK(thin_gemm_f32(w.X32[c], w.dp, (int)d, dV + c0 * ldv, ldv, nb, dY + c0 * ldy, ldy, w.thin, st));
        else
          HIPCHK(thin_gemm_words(W, w.Xw[c], w.dp, w.ps, (int)d, dV + c0 * ldv, ldv, nb, dY + c0 * ldy, ldy, w.thin, st));
      }
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  const double t_end = now_ms();
  inf.ms_setup = t_setup - t_start;
  inf.ms_bulk = t_bulk - t_setup;
  inf.ms_polish = t_end - t_bulk;
  inf.ms_total = t_end - t_start;
  if (info) *info = inf;
  return out_status;
}


// ---------------------------------------------------------------- batched
// Many independent problems (refl_sign_batched).  Each problem keeps its own
// FP64 copy of H, iterate pair and N.  Set-up and output run as grouped
// launches over all problems; the Newton-Schulz products of every problem
// still iterating run as ONE grouped launch per product, over the
// concatenated upper-tile lists.  Tile partials land in per-problem ranges
// laid out exactly as refl_sign's, and each range is reduced in refl_sign's
// order, so every problem takes the same steps and returns the same R, bit
// for bit, as a refl_sign call with its parameters.
//
// Host/device overlap: after the first product of step m the host reads the
// residuals while the device already runs the second product of step m for
// every problem of the step (for a problem that stops at m that product is
// discarded: it writes the other iterate of the pair), so the device does not
// wait for the host's stopping decisions.
struct BatchProb {
  int d = 0, dp = 0, ts = TILE, ntiles = 0;
  double* Hf = nullptr;   // FP64 copy of H; FP32 after the bulk: FP64 copy of the iterate
  void* X[2] = {nullptr, nullptr};
  void* N = nullptr;
  double* N64 = nullptr;  // FP32: N of the FP64 certificate product
  double* rowsum = nullptr;
  double* scal = nullptr; // SC_ALPHA, SC_NONFINITE of this problem
};

constexpr int BSC = 2;  // scalar slots per problem (SC_ALPHA, SC_NONFINITE)

struct BatchWork {
  std::vector<BatchProb> pr;
  int ttot = 0, maxdp = 0;
  double *scal = nullptr, *partials = nullptr;
  GemmProblem *probs = nullptr, *probs64 = nullptr;
  BatchDesc* desc = nullptr;
  int4* tiles[3] = {nullptr, nullptr, nullptr};  // two step lists, the final list
  int* begin[3] = {nullptr, nullptr, nullptr};
  int* slot[3] = {nullptr, nullptr, nullptr};
  int* sbeg = nullptr;  // set-up prefix arrays: mirror, rows, init (3 (n + 1))
  int* cbeg = nullptr;  // output prefix arrays: R rows, Hf rows (2 (n + 1))
  double *res = nullptr, *trace = nullptr, *cert = nullptr;
  BatchRule* rules = nullptr;  // device-driven stopping rule
  BatchStep* stp = nullptr;
  int* live = nullptr;
  int* ctl = nullptr;          // step counter, live count
  SmallProb* small = nullptr;  // problems of the LDS-resident launch
};

// Tile edges of the batched FP32 / FP64 products, in the order their tile
// lists are laid out and launched.
constexpr int NEDGE = 4;
constexpr int BATCH_EDGES[NEDGE] = {128, 96, 64, 32};
int edge_class(int ts) { return ts == 128 ? 0 : ts == 96 ? 1 : ts == 64 ? 2 : 3; }

size_t batch_layout(BatchWork& bw, void* base, int nprob, const int64_t* d, const int* ts,
                    bool fp64) {
  Carve c(base);
  bw.pr.assign(nprob, BatchProb());
  bw.ttot = 0;
  bw.maxdp = 0;
  const size_t es = fp64 ? sizeof(double) : sizeof(float);
  bw.scal = c.take<double>((size_t)BSC * nprob);
  for (int p = 0; p < nprob; ++p) {
    BatchProb& q = bw.pr[p];
    q.d = (int)d[p];
    q.ts = ts[p];
    q.dp = (int)round_up(d[p], pad_unit_f(q.ts));
    const int nt = q.dp / q.ts;
    q.ntiles = nt * (nt + 1) / 2;
    bw.ttot += q.ntiles;
    bw.maxdp = std::max(bw.maxdp, q.dp);
    const size_t n2 = (size_t)q.dp * q.dp;
    q.Hf = c.take<double>(n2);
    q.X[0] = c.take<char>(es * n2);
    q.X[1] = c.take<char>(es * n2);
    q.N = c.take<char>(es * n2);
    q.N64 = fp64 ? nullptr : c.take<double>(n2);
    q.rowsum = c.take<double>(2 * (size_t)q.dp);
    q.scal = bw.scal ? bw.scal + (size_t)BSC * p : nullptr;
  }
  bw.probs = c.take<GemmProblem>(nprob);
  bw.probs64 = c.take<GemmProblem>(nprob);
  bw.desc = c.take<BatchDesc>(nprob);
  for (int b = 0; b < 3; ++b) {
    bw.tiles[b] = c.take<int4>(bw.ttot);
    bw.begin[b] = c.take<int>(nprob + 1);
    bw.slot[b] = c.take<int>(nprob);
  }
  bw.partials = c.take<double>(bw.ttot);
  bw.sbeg = c.take<int>(3 * ((size_t)nprob + 1));
  bw.cbeg = c.take<int>(2 * ((size_t)nprob + 1));
  bw.res = c.take<double>(nprob);
  bw.trace = c.take<double>(nprob);
  bw.cert = c.take<double>(nprob);
  bw.rules = c.take<BatchRule>(nprob);
  bw.stp = c.take<BatchStep>(nprob);
  bw.live = c.take<int>(nprob);
  bw.ctl = c.take<int>(2);
  bw.small = c.take<SmallProb>(nprob);
  return c.off + 256;
}

// Host staging of the batched solve: one pinned block, carved like the
// device workspace (each buffer is the source or target of one copy).
struct BatchPin {
  GemmProblem *probs, *probs64;
  BatchDesc* desc;
  double *scal, *res, *trace, *cert;
  BatchRule* rules;
  BatchStep* stp;
  int *live, *ctl;
  SmallProb* small;
  int4* tiles[3];
  int *begin[3], *slot[3];
  int *sbeg, *cbeg;
};

size_t batch_pin_layout(BatchPin& bp, void* base, int nprob, int ttot) {
  Carve c(base);
  bp.probs = c.take<GemmProblem>(nprob);
  bp.probs64 = c.take<GemmProblem>(nprob);
  bp.desc = c.take<BatchDesc>(nprob);
  bp.scal = c.take<double>((size_t)BSC * nprob);
  bp.res = c.take<double>(nprob);
  bp.trace = c.take<double>(nprob);
  bp.cert = c.take<double>(nprob);
  bp.rules = c.take<BatchRule>(nprob);
  bp.stp = c.take<BatchStep>(nprob);
  bp.live = c.take<int>(nprob);
  bp.ctl = c.take<int>(2);
  bp.small = c.take<SmallProb>(nprob);
  for (int b = 0; b < 3; ++b) {
    bp.tiles[b] = c.take<int4>(ttot);
    bp.begin[b] = c.take<int>(nprob + 1);
    bp.slot[b] = c.take<int>(nprob);
  }
  bp.sbeg = c.take<int>(3 * ((size_t)nprob + 1));
  bp.cbeg = c.take<int>(2 * ((size_t)nprob + 1));
  return c.off + 256;
}

// Grouped tile list over the problems ids[0..n): range q of the partials is
// begin[q] .. begin[q + 1) and holds problem ids[q]'s tiles in the order of
// build_tiles_nt; slot[q] = ids[q].  The tiles of each edge class (one
// grouped launch each, BATCH_EDGES order) are contiguous, cnt[c] of them;
// within a class the largest problems come first (their tiles take
// longest).  Returns the number of tiles.
int batch_tiles(const BatchWork& bw, const std::vector<int>& ids, int4* tiles, int* begin,
                int* slot, int* cnt) {
  const int n = (int)ids.size();
  begin[0] = 0;
  for (int q = 0; q < n; ++q) {
    begin[q + 1] = begin[q] + bw.pr[ids[q]].ntiles;
    slot[q] = ids[q];
  }
  std::vector<int> ord(n);
  for (int q = 0; q < n; ++q) ord[q] = q;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    const BatchProb &pa = bw.pr[ids[a]], &pb = bw.pr[ids[b]];
    const int ca = edge_class(pa.ts), cb = edge_class(pb.ts);
    return ca != cb ? ca < cb : pa.dp > pb.dp;
  });
  std::vector<int2> tl;
  int t = 0;
  for (int c = 0; c < NEDGE; ++c) cnt[c] = 0;
  for (int q : ord) {
    const BatchProb& pq = bw.pr[ids[q]];
    build_tiles_nt(pq.dp / pq.ts, tl);
    for (size_t i = 0; i < tl.size(); ++i)
      tiles[t++] = make_int4(ids[q], tl[i].x, tl[i].y, begin[q] + (int)i);
    cnt[edge_class(pq.ts)] += (int)tl.size();
  }
  return t;
}

refl_status_t batch_check(refl_handle_t h, int nprob, const int64_t* d, const double* const* dH,
                          const int64_t* ldh, const refl_params_t* params, double* const* dR,
                          const int64_t* ldr) {
  if (nprob < 1) return fail(h, REFL_ERR_INVALID_ARG, "nprob must be >= 1");
  if (!d || !params) return fail(h, REFL_ERR_INVALID_ARG, "d or params is NULL");
  for (int p = 0; p < nprob; ++p) {
    refl_status_t rs = check_params(h, d[p], &params[p]);
    if (rs != REFL_OK) {
      char msg[sizeof(h->err)];
      std::snprintf(msg, sizeof(msg), "%s", h->err);
      return fail(h, rs, "problem %d: %s", p, msg);
    }
    const refl_params_t& q = params[p];
    if (q.precision != params[0].precision)
      return fail(h, REFL_ERR_INVALID_ARG, "problem %d: every problem needs the same precision", p);
    if (q.precision == REFL_PREC_MIXED)
      return fail(h, REFL_ERR_UNSUPPORTED, "problem %d: batched solves run FP64 or FP32", p);
    if (q.shift_mode != REFL_SHIFT_GIVEN)
      return fail(h, REFL_ERR_UNSUPPORTED, "problem %d: batched solves need a given shift", p);
  }
  if (!dH || !ldh || !dR || !ldr) return fail(h, REFL_ERR_INVALID_ARG, "NULL pointer array");
  for (int p = 0; p < nprob; ++p) {
    if (!dH[p] || ldh[p] < d[p]) return fail(h, REFL_ERR_INVALID_ARG, "problem %d: H is NULL or ldh < d", p);
    if (!dR[p] || ldr[p] < d[p]) return fail(h, REFL_ERR_INVALID_ARG, "problem %d: R is NULL or ldr < d", p);
  }
  return REFL_OK;
}

refl_status_t batched_impl(refl_handle_t h, int nprob, const int64_t* d, const double* const* dH,
                           const int64_t* ldh, const refl_params_t* params, double* const* dR,
                           const int64_t* ldr, refl_info_t* info, refl_status_t* status) {
  const double t_start = now_ms();
  refl_status_t rs = batch_check(h, nprob, d, dH, ldh, params, dR, ldr);
  if (rs != REFL_OK) {
    if (status && nprob > 0)
      for (int p = 0; p < nprob; ++p) status[p] = rs;
    return rs;
  }
  const bool fp64 = params[0].precision == REFL_PREC_FP64;
  HIPCHK(hipSetDevice(h->device));
  // Each problem's tile edge is the one refl_sign would use for it.
  std::vector<int> tsv(nprob);
  for (int p = 0; p < nprob; ++p) tsv[p] = select_tile_f(h, d[p], fp64);
  BatchWork bw;
  const size_t need = batch_layout(bw, nullptr, nprob, d, tsv.data(), fp64);
  void* base = nullptr;
  rs = ensure_workspace(h, need, &base);
  if (rs != REFL_OK) return rs;
  batch_layout(bw, base, nprob, d, tsv.data(), fp64);
  hipStream_t st = h->stream;
  BatchPin bp;
  const size_t pin_need = batch_pin_layout(bp, nullptr, nprob, bw.ttot);
  if (h->batch_pin_bytes < pin_need) {
    HIPCHK(hipStreamSynchronize(st));
    if (h->batch_pin) (void)hipHostFree(h->batch_pin);
    h->batch_pin = nullptr;
    h->batch_pin_bytes = 0;
    if (hipHostMalloc(&h->batch_pin, pin_need, hipHostMallocDefault) != hipSuccess || !h->batch_pin)
      return fail(h, REFL_ERR_NO_MEMORY, "pinned staging of %zu bytes failed", pin_need);
    h->batch_pin_bytes = pin_need;
  }
  batch_pin_layout(bp, h->batch_pin, nprob, bw.ttot);

  std::vector<refl_info_t> inf(nprob);
  std::vector<refl_status_t> pst(nprob, REFL_OK);
  for (int p = 0; p < nprob; ++p) {
    std::memset(&inf[p], 0, sizeof(refl_info_t));
    refl_info_t& f = inf[p];
    f.lam_k = f.lam_k1 = f.eps = f.margin = NaN;
    f.commutator_fro = f.dk_bound = NaN;
    f.resid_fro = f.trace = f.rho = f.gamma = NaN;
    f.index_j = -1;
    f.s = params[p].s;
    f.bulk_tile = tsv[p];
  }

  // Opt-in symmetry checks (the problems' scalar slots are free until the
  // set-up writes them).
  bool any_sym = false;
  for (int p = 0; p < nprob; ++p) {
    if (!params[p].check_symmetric) continue;
    any_sym = true;
    HIPCHK(launch_asym_max(dH[p], ldh[p], (int)d[p], bw.scal + BSC * p, 0, st));
  }
  if (any_sym) {
    HIPCHK(hipMemcpyAsync(bp.scal, bw.scal, sizeof(double) * BSC * nprob, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int p = 0; p < nprob; ++p) {
      if (!params[p].check_symmetric) continue;
      const double asym = bp.scal[BSC * p], amax = bp.scal[BSC * p + 1];
      if (!(asym <= params[p].sym_tol * amax) || !std::isfinite(amax)) pst[p] = REFL_ERR_NOT_SYMMETRIC;
    }
  }

  // ---- set-up: descriptors, then five grouped launches ----
  int* mb = bp.sbeg;
  int* rb = mb + (nprob + 1);
  int* ib = rb + (nprob + 1);
  mb[0] = rb[0] = ib[0] = 0;
  for (int p = 0; p < nprob; ++p) {
    const BatchProb& q = bw.pr[p];
    GemmProblem& g = bp.probs[p];
    GemmProblem& g64 = bp.probs64[p];
    g.X[0] = q.X[0];
    g.X[1] = q.X[1];
    g.N = q.N;
    g64.X[0] = g64.X[1] = q.Hf;
    g64.N = q.N64;
    g.ld = g64.ld = q.dp;
    g.d = g64.d = q.d;
    g.dp = g64.dp = q.dp;
    g.pad = g64.pad = 0;
    BatchDesc& e = bp.desc[p];
    e.H = dH[p];
    e.ldh = ldh[p];
    e.Hf = q.Hf;
    e.X[0] = q.X[0];
    e.X[1] = q.X[1];
    e.rowsum = q.rowsum;
    e.scal = q.scal;
    e.R = dR[p];
    e.ldr = ldr[p];
    e.s = params[p].s;
    e.alpha_given = params[p].alpha;
    e.d = q.d;
    e.dp = q.dp;
    e.scale_given = params[p].scale_mode == REFL_SCALE_GIVEN;
    e.norm = params[p].scale_mode == REFL_SCALE_FRO;
    e.par = 0;
    e.pad = 0;
    mb[p + 1] = mb[p] + (q.dp / 64) * (q.dp / 64);
    rb[p + 1] = rb[p] + (q.d + 3) / 4;
    ib[p + 1] = ib[p] + batch_init_blocks(q.dp);
  }
  HIPCHK(hipMemcpyAsync(bw.probs, bp.probs, sizeof(GemmProblem) * nprob, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bw.probs64, bp.probs64, sizeof(GemmProblem) * nprob, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bw.desc, bp.desc, sizeof(BatchDesc) * nprob, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bw.sbeg, bp.sbeg, sizeof(int) * 3 * (nprob + 1), hipMemcpyHostToDevice, st));
  HIPCHK(launch_batch_setup(fp64, bw.desc, nprob, bw.sbeg, mb[nprob], bw.sbeg + (nprob + 1),
                            rb[nprob], bw.sbeg + 2 * (nprob + 1), ib[nprob], bw.trace, st));
  HIPCHK(hipMemcpyAsync(bp.scal, bw.scal, sizeof(double) * BSC * nprob, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(bp.trace, bw.trace, sizeof(double) * nprob, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<int> cur;
  std::vector<double> trace_cur(nprob, NaN);
  for (int p = 0; p < nprob; ++p) {
    inf[p].alpha = bp.scal[BSC * p + SC_ALPHA];
    trace_cur[p] = bp.trace[p];
    if (pst[p] != REFL_OK)
      continue;
    if (bp.scal[BSC * p + SC_NONFINITE] > 0.0 || !(inf[p].alpha > 0.0) ||
        !std::isfinite(inf[p].alpha))
      pst[p] = REFL_ERR_NOT_FINITE;
    else
      cur.push_back(p);
  }
  const double t_setup = now_ms();

  // ---- bulk ----
  const int fprec = fp64 ? 1 : 0;
  const bool timing = params[0].timing != 0;
  size_t nev = 0;
  auto ev_pair = [&]() -> hipError_t {
    while (h->ev.size() < 2 * (nev + 1)) {
      hipEvent_t e;
      hipError_t er = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);  // timing only
      if (er != hipSuccess) return er;
      h->ev.push_back(e);
    }
    return hipSuccess;
  };
  int cls[3][NEDGE] = {};  // tiles per edge class of each list
  // One grouped launch per edge class present in list lb.
  auto grouped_list = [&](int fp, int mode, const GemmProblem* probs, int lb, int par,
                          const int* live, hipStream_t s) -> hipError_t {
    int off = 0;
    for (int c = 0; c < NEDGE; ++c) {
      if (cls[lb][c] > 0) {
        hipError_t e = launch_sym_gemm_grouped(fp, mode, BATCH_EDGES[c], probs, bw.tiles[lb] + off,
                                               cls[lb][c], par, bw.partials, live, s);
        if (e != hipSuccess) return e;
      }
      off += cls[lb][c];
    }
    return hipSuccess;
  };
  // Step list in buffer lb: build and upload.
  auto upload_list = [&](int lb, const std::vector<int>& ids) -> int {
    const int nt = batch_tiles(bw, ids, bp.tiles[lb], bp.begin[lb], bp.slot[lb], cls[lb]);
    const int nq = (int)ids.size();
    if (hipMemcpyAsync(bw.tiles[lb], bp.tiles[lb], sizeof(int4) * nt, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(bw.begin[lb], bp.begin[lb], sizeof(int) * (nq + 1), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(bw.slot[lb], bp.slot[lb], sizeof(int) * nq, hipMemcpyHostToDevice, st) != hipSuccess)
      return -1;
    return nt;
  };
  // The stopping rule runs on the device (k_batch_decide, the rule of
  // refl_sign), so a step needs no host decision: the residual product, its
  // per-problem sums, the decision, the update product (tiles of stopped
  // problems do nothing) and the trace sums.  All problems iterate in step:
  // step m uses parity m & 1, and the host only reads the live count every
  // BATCH_GRAPH_STEPS steps.  Those steps are captured once per call in a
  // HIP graph and the graph is launched until no problem is live (eager
  // launches instead with params.timing, for the per-launch events, or with
  // REFL_BATCH_GRAPH=0).
  //
  // Problems of small order (small_order) take no part in the grouped steps:
  // each runs its whole iteration in one work-group of the LDS-resident
  // launch, on a side stream beside the steps (the same kernel as refl_sign
  // uses for them, so their results match single calls too).
  constexpr int BATCH_GRAPH_STEPS = 4;
  std::vector<int> tiled, smallp;
  for (int p : cur) (small_order(d[p], fp64) ? smallp : tiled).push_back(p);
  const int nq0 = (int)tiled.size();
  const int nsm = (int)smallp.size();
  int maxsteps = 0;
  std::vector<char> live0(nprob, 0);
  for (int p : cur) live0[p] = 1;
  for (int p = 0; p < nprob; ++p) {
    bp.rules[p].tol = params[p].tol;
    bp.rules[p].fixed_steps = params[p].fixed_steps;
    bp.rules[p].max_iter = params[p].max_iter;
    std::memset(&bp.stp[p], 0, sizeof(BatchStep));
    bp.stp[p].trace = trace_cur[p];
    bp.stp[p].resid = NaN;
    bp.stp[p].state = live0[p] ? BATCH_LIVE : BATCH_NONFINITE;
    bp.live[p] = 0;
  }
  for (int p : tiled) {
    bp.live[p] = 1;
    maxsteps = std::max(maxsteps, params[p].fixed_steps > 0 ? params[p].fixed_steps : params[p].max_iter);
  }
  for (int q = 0; q < nsm; ++q) {
    const BatchProb& pq = bw.pr[smallp[q]];
    SmallProb& e = bp.small[q];
    e.X[0] = pq.X[0];
    e.X[1] = pq.X[1];
    e.d = pq.d;
    e.dp = pq.dp;
    e.slot = smallp[q];
    e.pad = 0;
  }
  bp.ctl[0] = 0;
  bp.ctl[1] = nq0;
  HIPCHK(hipMemcpyAsync(bw.rules, bp.rules, sizeof(BatchRule) * nprob, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bw.stp, bp.stp, sizeof(BatchStep) * nprob, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bw.live, bp.live, sizeof(int) * nprob, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bw.ctl, bp.ctl, sizeof(int) * 2, hipMemcpyHostToDevice, st));
  if (nsm > 0) HIPCHK(hipMemcpyAsync(bw.small, bp.small, sizeof(SmallProb) * nsm, hipMemcpyHostToDevice, st));
  // Fork: the small problems' launch goes to the side stream after the
  // uploads above; the join below comes before the step records are read.
  const bool fork = nsm > 0 && nq0 > 0;
  if (fork) {
    if (!h->side) HIPCHK(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
    for (hipEvent_t& e : h->side_ev)
      if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(hipEventRecord(h->side_ev[0], st));
    HIPCHK(hipStreamWaitEvent(h->side, h->side_ev[0], 0));
  }
  if (nsm > 0) {
    hipStream_t ss = fork ? h->side : st;
    HIPCHK(launch_ns_small(fp64, bw.small, nsm, bw.rules, bw.stp, ss));
    if (fork) HIPCHK(hipEventRecord(h->side_ev[1], ss));
  }
  const int lb = 0;
  const int nt_all = nq0 == 0 ? 0 : upload_list(lb, tiled);
  // Error returns between fork and join first drain the side stream.
  auto drain_side = [&]() {
    if (fork) (void)hipStreamSynchronize(h->side);
  };
  if (nt_all < 0) {
    drain_side();
    return fail(h, REFL_ERR_DEVICE, "tile list upload failed");
  }
  auto step = [&](int par, hipStream_t s) -> hipError_t {
    hipError_t e;
    const bool ev = timing && s == st;
    if (ev) {
      if ((e = ev_pair()) != hipSuccess) return e;
      if ((e = hipEventRecord(h->ev[2 * nev], s)) != hipSuccess) return e;
    }
    if ((e = grouped_list(fprec, GEMM_RESIDUAL, bw.probs, lb, par, bw.live, s)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(h->ev[2 * nev++ + 1], s)) != hipSuccess) return e;
    if ((e = launch_reduce_ranges(bw.partials, bw.begin[lb], bw.slot[lb], nq0, bw.res, s)) != hipSuccess)
      return e;
    if ((e = launch_batch_decide(nprob, bw.res, bw.trace, bw.rules, bw.stp, bw.live, bw.ctl, par, s)) !=
        hipSuccess)
      return e;
    if (ev) {
      if ((e = ev_pair()) != hipSuccess) return e;
      if ((e = hipEventRecord(h->ev[2 * nev], s)) != hipSuccess) return e;
    }
    if ((e = grouped_list(fprec, GEMM_UPDATE, bw.probs, lb, par, bw.live, s)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(h->ev[2 * nev++ + 1], s)) != hipSuccess) return e;
    return launch_reduce_ranges(bw.partials, bw.begin[lb], bw.slot[lb], nq0, bw.trace, s);
  };
  const char* genv = std::getenv("REFL_BATCH_GRAPH");
  const bool use_graph = nq0 > 0 && !timing && !(genv && genv[0] == '0');
  hipGraphExec_t gexec = nullptr;
  // The graph holds only workspace addresses and host-side counts, all fixed
  // by this key; a call with the same key (the same problem set solved
  // again, e.g. by an outer iteration) launches the instantiated graph of
  // the previous call.
  std::vector<int64_t> key = {reinterpret_cast<int64_t>(base), (int64_t)need, fprec, nprob, nq0};
  for (int p = 0; p < nprob; ++p) {
    key.push_back(d[p]);
    key.push_back(tsv[p]);
  }
  key.insert(key.end(), tiled.begin(), tiled.end());
  for (int c = 0; c < NEDGE; ++c) key.push_back(cls[lb][c]);
  if (use_graph && h->bgraph && h->bgraph_key == key) gexec = h->bgraph;
  if (use_graph && !gexec) {
    if (h->bgraph) {
      (void)hipGraphExecDestroy(h->bgraph);
      h->bgraph = nullptr;
      h->bgraph_key.clear();
    }
    hipError_t ce = h->cap ? hipSuccess : hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
    if (ce == hipSuccess) ce = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
    if (ce != hipSuccess) {
      drain_side();
      return fail(h, REFL_ERR_DEVICE, "batched step graph: %s", hipGetErrorString(ce));
    }
    for (int i = 0; i < BATCH_GRAPH_STEPS && ce == hipSuccess; ++i) ce = step(i & 1, h->cap);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(h->cap, &graph);
    if (ce == hipSuccess) ce = ee;
    if (ce == hipSuccess) ce = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (ce != hipSuccess) {
      if (gexec) (void)hipGraphExecDestroy(gexec);
      drain_side();
      return fail(h, REFL_ERR_DEVICE, "batched step graph: %s", hipGetErrorString(ce));
    }
    h->bgraph = gexec;
    h->bgraph_key = key;
  }
  // Each round runs BATCH_GRAPH_STEPS steps; every problem stops by its
  // step limit, so the rounds are bounded.
  const int rounds = nq0 == 0 ? 0 : maxsteps / BATCH_GRAPH_STEPS + 2;
  hipError_t le = hipSuccess;
  for (int round = 0; round < rounds && le == hipSuccess; ++round) {
    if (gexec) {
      le = hipGraphLaunch(gexec, st);
    } else {
      for (int i = 0; i < BATCH_GRAPH_STEPS && le == hipSuccess; ++i) le = step(i & 1, st);
    }
    if (le == hipSuccess) le = hipMemcpyAsync(bp.ctl, bw.ctl, sizeof(int) * 2, hipMemcpyDeviceToHost, st);
    if (le == hipSuccess) le = hipStreamSynchronize(st);
    if (le == hipSuccess && bp.ctl[1] == 0) break;
  }
  if (fork) {
    const hipError_t je = hipStreamWaitEvent(st, h->side_ev[1], 0);
    if (le == hipSuccess) le = je;
  }
  if (le != hipSuccess) return fail(h, REFL_ERR_DEVICE, "batched steps: %s", hipGetErrorString(le));
  if (nq0 > 0 && bp.ctl[1] != 0)
    return fail(h, REFL_ERR_DEVICE, "batched steps: %d problems still iterating after the step limit",
                bp.ctl[1]);
  HIPCHK(hipMemcpyAsync(bp.stp, bw.stp, sizeof(BatchStep) * nprob, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<char> converged(nprob, 0);
  std::vector<int> done;  // problems that stopped with an iterate to return
  for (int p : cur) {
    const BatchStep& q = bp.stp[p];
    inf[p].ns_steps = q.m;
    inf[p].resid_fro = q.resid;
    inf[p].trace = q.trace;
    if (q.state == BATCH_NONFINITE) {
      pst[p] = REFL_ERR_NOT_FINITE;
      continue;
    }
    converged[p] = q.state == BATCH_CONVERGED;
    bp.desc[p].par = q.par;
    done.push_back(p);
  }

  // ---- output: FP32 certificate in FP64, then R, for every problem in done ----
  std::sort(done.begin(), done.end());
  const int nd = (int)done.size();
  if (nd > 0) {
    int* rbeg = bp.cbeg;
    int* hbeg = rbeg + (nprob + 1);
    rbeg[0] = hbeg[0] = 0;
    constexpr int CR = BATCH_COPY_ROWS;
    for (int q = 0; q < nd; ++q) {
      rbeg[q + 1] = rbeg[q] + (bw.pr[done[q]].d + CR - 1) / CR;
      hbeg[q + 1] = hbeg[q] + (bw.pr[done[q]].dp + CR - 1) / CR;
    }
    HIPCHK(hipMemcpyAsync(bw.desc, bp.desc, sizeof(BatchDesc) * nprob, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bw.cbeg, bp.cbeg, sizeof(int) * 2 * (nprob + 1), hipMemcpyHostToDevice, st));
    const int nt_fin = batch_tiles(bw, done, bp.tiles[2], bp.begin[2], bp.slot[2], cls[2]);
    HIPCHK(hipMemcpyAsync(bw.tiles[2], bp.tiles[2], sizeof(int4) * nt_fin, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bw.begin[2], bp.begin[2], sizeof(int) * (nd + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bw.slot[2], bp.slot[2], sizeof(int) * nd, hipMemcpyHostToDevice, st));
    if (!fp64) {
      HIPCHK(launch_batch_copy(0, bw.desc, bw.cbeg + (nprob + 1), bw.slot[2], nd, hbeg[nd], 1, st));
      HIPCHK(grouped_list(1, GEMM_RESIDUAL, bw.probs64, 2, 0, nullptr, st));
      HIPCHK(launch_reduce_ranges(bw.partials, bw.begin[2], bw.slot[2], nd, bw.cert, st));
      HIPCHK(hipMemcpyAsync(bp.cert, bw.cert, sizeof(double) * nprob, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(launch_batch_copy(fprec, bw.desc, bw.cbeg, bw.slot[2], nd, rbeg[nd], 0, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  double ms_gemm = 0.0;
  if (timing) {
    for (size_t i = 0; i < nev; ++i) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]));
      ms_gemm += ms;
    }
  }
  const double t_end = now_ms();

  // ---- certificates and statuses ----
  refl_status_t first = REFL_OK;
  for (int p = 0; p < nprob; ++p) {
    refl_info_t& f = inf[p];
    const refl_params_t& pp = params[p];
    f.ms_setup = t_setup - t_start;
    f.ms_bulk = t_end - t_setup;
    f.ms_total = t_end - t_start;
    if (timing) {
      f.ms_gemm = ms_gemm;
      f.gemm_launches = (int)nev;
    }
    if (pst[p] == REFL_OK) {
      if (!fp64) f.resid_fro = std::sqrt(std::fmax(bp.cert[p], 0.0));
      f.index_j = index_certificate(d[p], f.resid_fro, f.trace);
      if (!converged[p]) pst[p] = REFL_ERR_NOT_CONVERGED;
      if (pp.fixed_steps == 0 && pp.k > 0 && f.index_j >= 0 && f.index_j != pp.k)
        pst[p] = REFL_ERR_NOT_ADMISSIBLE;
    }
    if (pst[p] != REFL_OK && first == REFL_OK) {
      first = pst[p];
      if (pst[p] == REFL_ERR_NOT_FINITE)
        fail(h, first, "problem %d: H or the iterate is not finite", p);
      else if (pst[p] == REFL_ERR_NOT_SYMMETRIC)
        fail(h, first, "problem %d: H is not symmetric to sym_tol", p);
      else if (pst[p] == REFL_ERR_NOT_CONVERGED)
        fail(h, first, "problem %d: no convergence after %d steps (resid %.3e)", p, f.ns_steps,
             f.resid_fro);
      else
        fail(h, first, "problem %d: index certificate found %d negative eigenvalues, not k=%d", p,
             f.index_j, pp.k);
    }
  }
  if (info)
    for (int p = 0; p < nprob; ++p) info[p] = inf[p];
  if (status)
    for (int p = 0; p < nprob; ++p) status[p] = pst[p];
  return first;
}

// ---------------------------------------------------------------- gradient
// refl_sign_grad: the forward iteration of refl_sign (FP64 / FP32) with the
// derivative of its m steps, by a checkpointed reverse sweep or by forward
// tangents (see include/refl.h for the recurrences).
struct GradWork {
  int d = 0, dp = 0, ts = TILE, ntiles = 0, nfull = 0, c = 1, nck = 0;
  bool fp64 = true;
  double *Hf = nullptr, *scal = nullptr, *rowsum = nullptr, *partials = nullptr;
  int2 *tiles = nullptr, *full = nullptr;
  void *Gs = nullptr, *Gb[2] = {nullptr, nullptr}, *Pn = nullptr, *ring[2] = {nullptr, nullptr};
  std::vector<void*> ck, xs, ns;  // checkpoints, segment iterates, segment N
  bool keep_all = false;  // every X_j and N_j of the forward kept: no recomputation
};

int grad_cap(const refl_params_t& p) { return p.fixed_steps > 0 ? p.fixed_steps : p.max_iter; }

size_t grad_layout(GradWork& g, void* base, int64_t d, const refl_params_t& p, refl_handle_t h) {
  Carve c(base);
  g.fp64 = p.precision == REFL_PREC_FP64;
  const size_t es = g.fp64 ? sizeof(double) : sizeof(float);
  g.d = (int)d;
  g.ts = select_tile_f(h, d, g.fp64);
  g.dp = (int)round_up(d, pad_unit_f(g.ts));
  const int nt = g.dp / g.ts;
  g.ntiles = nt * (nt + 1) / 2;
  g.nfull = nt * nt;
  const int cap = grad_cap(p);
  const bool reverse = p.grad_mode == REFL_GRAD_REVERSE;
  const size_t n2 = (size_t)g.dp * g.dp;
  // Reverse mode keeps every X_j and N_j of the forward (no recomputation in
  // the reverse sweep) when they fit in KEEP_ALL_BYTES and no interval is
  // requested; otherwise X_j every c steps, with each segment's iterates
  // recomputed before its reverse sweep.  The gradient is the same bit for
  // bit either way (the same products on the same iterates).
  constexpr double KEEP_ALL_BYTES = 16.0 * (1 << 30);
  g.keep_all = reverse && p.ckpt_every == 0 && 2.0 * (cap + 1) * (double)(es * n2) <= KEEP_ALL_BYTES;
  g.c = 1;
  if (reverse && !g.keep_all)
    g.c = p.ckpt_every > 0 ? std::min(p.ckpt_every, cap)
                           : std::max(1, (int)std::ceil(std::sqrt((double)cap)));
  g.nck = reverse ? cap / g.c + 1 : 0;
  g.scal = c.take<double>(SC_COUNT);
  g.tiles = c.take<int2>(g.ntiles);
  g.full = c.take<int2>(g.nfull);
  g.partials = c.take<double>(std::max(g.nfull, dot_partials()));
  g.rowsum = c.take<double>(2 * (size_t)g.dp);
  g.Hf = c.take<double>(n2);
  g.Gs = c.take<char>(es * n2);
  g.Gb[0] = c.take<char>(es * n2);
  g.Gb[1] = c.take<char>(es * n2);
  g.Pn = c.take<char>(es * n2);
  g.ring[0] = c.take<char>(es * n2);
  g.ring[1] = c.take<char>(es * n2);
  g.ck.assign(g.nck, nullptr);
  for (auto& q : g.ck) q = c.take<char>(es * n2);
  g.xs.assign(reverse && !g.keep_all ? g.c : 0, nullptr);
  for (auto& q : g.xs) q = c.take<char>(es * n2);
  g.ns.assign(g.keep_all ? cap + 1 : (reverse ? g.c : 1), nullptr);
  for (auto& q : g.ns) q = c.take<char>(es * n2);
  return c.off + 256;
}

// Every (I, J) of the nt x nt tile grid, row bands of 4 as build_tiles_nt,
// cut into 8 consecutive pieces for the 8 XCDs.
void build_tiles_full(int nt, std::vector<int2>& host) {
  std::vector<int2> order;
  for (int b0 = 0; b0 < nt; b0 += 4)
    for (int J = 0; J < nt; ++J)
      for (int I = b0; I < std::min(b0 + 4, nt); ++I) order.push_back(make_int2(I, J));
  const int T = (int)order.size();
  int start[8], s0 = 0;
  for (int x = 0; x < 8; ++x) {
    start[x] = s0;
    s0 += (T - x + 7) / 8;
  }
  host.resize(T);
  for (int b = 0; b < T; ++b) host[b] = order[start[b % 8] + b / 8];
}

// Gradient of the limit L(H) = <G, R_k(H)> = <G, sgn(H - sI)> after a MIXED
// solve.  With A = H - sI = sum_i lambda_i q_i q_i^T, the derivative of sgn
// at A applied to a symmetric E is sum over i < k < j of
//   2 (q_j q_j^T E q_i q_i^T + q_i q_i^T E q_j q_j^T) / (lambda_j - lambda_i),
// the Daleckii-Krein divided differences of sgn across the gap.  It is
// self-adjoint, so the gradient is that map applied to sym(G):
//   grad = 2 (Z V^T + V Z^T),  z_c = sum_{j > k} q_j q_j^T sym(G) v_c / (lambda_j - theta_c),
// where z_c solves (I - V V^T)(H - theta_c)(I - V V^T) z_c = (I - V V^T) sym(G) v_c,
// with V the certified basis of the target eigenspace and theta_c its Ritz
// values: positive definite on the complement of V, the operator of the
// correction's inner solves, here in FP64 to a relative residual of
// GRAD_CG_TOL.  loss = tr G - 2 tr(V^T sym(G) V).
constexpr double GRAD_CG_TOL = 1e-10;

refl_status_t grad_mixed(refl_handle_t h, int64_t d, const double* dH, int64_t ldh,
                         const refl_params_t& p, const double* dG, int64_t ldg, double* dGrad,
                         int64_t ldgr, double* loss, double* dR, int64_t ldr, refl_info_t* info) {
  MixedKeep kp;
  refl_info_t inf;
  refl_status_t rs = sign_impl(h, d, dH, ldh, &p, dR, ldr, 0, nullptr, 0, nullptr, 0, &inf, &kp);
  if (rs != REFL_OK) {
    if (info) *info = inf;
    return rs;
  }
  const double t0 = now_ms();
  Work& w = kp.w;
  hipStream_t st = h->stream;
  const int dd = (int)d, k = kp.k;
  const int64_t ld = w.dp, n2 = (int64_t)w.dp * w.dp;
  double* hsc = h->pinned;
  // sym(G), dp x dp FP64, in the word planes (free once the forward is done).
  double* Gs = reinterpret_cast<double*>(w.Xw[0]);
  const size_t room = (size_t)(reinterpret_cast<char*>(w.Nw) - reinterpret_cast<char*>(w.Xw[0])) +
                      (size_t)w.words * n2 * sizeof(uint16_t);
  if (room < sizeof(double) * (size_t)n2) return fail(h, REFL_ERR_DEVICE, "gradient: word planes too small");
  HIPCHK(launch_sym_in_f64(dG, ldg, dd, nullptr, Gs, w.dp, st));
  HIPCHK(launch_trace_f64(Gs, w.dp, dd, w.scal, SC_SCRATCH, st));
  int iters = 0;
  double trGVV = 0.0;
  refl_status_t out = REFL_OK;
  if (!kp.V || k == 0 || k == dd) {
    // R = +I or -I: locally constant, zero gradient.
    HIPCHK(hipMemset2DAsync(dGrad, sizeof(double) * ldgr, 0, sizeof(double) * d, d, st));
  } else {
    double* V = kp.V;
    double* spare = V == w.V ? w.T1 : w.V;
    std::vector<double> C((size_t)k * k), Bn((size_t)k * k);
    // B = (I - V V^T) sym(G) V into Rr; C = V^T sym(G) V.
    HIPCHK(symthin_f64(Gs, ld, dd, V, ld, k, w.W, ld, w.thin, st));
    HIPCHK(gram(V, ld, k, w.W, ld, k, dd, w.G, w.gwork, st));
    HIPCHK(hipMemcpyAsync(C.data(), w.G, sizeof(double) * k * k, hipMemcpyDeviceToHost, st));
    HIPCHK(lincomb(dd, k, 1.0, w.W, ld, 0.0, w.Rr, ld, st));
    HIPCHK(block_axpy(dd, k, k, 1.0, w.Rr, ld, -1.0, V, ld, w.G, st));
    HIPCHK(gram(w.Rr, ld, k, w.Rr, ld, k, dd, w.G, w.gwork, st));
    HIPCHK(hipMemcpyAsync(Bn.data(), w.G, sizeof(double) * k * k, hipMemcpyDeviceToHost, st));
    HIPCHK(lincomb(dd, k, 0.0, w.Rr, ld, 0.0, w.Z, ld, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int c = 0; c < k; ++c) trGVV += C[c + (size_t)k * c];
    CgHost* hs = reinterpret_cast<CgHost*>(h->pinned + SC_COUNT);
    std::memset(hs, 0, sizeof(CgHost));
    for (int c = 0; c < k; ++c) {
      hs->theta[c] = kp.theta[c];
      hs->rho0[c] = Bn[c + (size_t)k * c];
    }
    hs->tol2 = GRAD_CG_TOL * GRAD_CG_TOL;
    hs->k = k;
    hs->nb = k;
    const CgBufs cb = {{w.Rr, spare}, {w.P[0], w.P[1]}, {w.W, w.T2}, w.AP, w.Z, nullptr};
    const int cap = 4 * p.cg_max_iter;
    rs = cg_solve(h, w, false, V, k, cb, cap, hs);
    if (rs != REFL_OK) return rs;
    iters = hs->iters;
    HIPCHK(form_sym_pair(w.Z, V, ld, k, dd, 2.0, dGrad, ldgr, st));
    if (iters >= cap)
      out = fail(h, REFL_ERR_NOT_CONVERGED, "gradient solve: %d iterations without reaching %.0e", iters,
                 GRAD_CG_TOL);
  }
  HIPCHK(hipMemcpyAsync(hsc + SC_SCRATCH, w.scal + SC_SCRATCH, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double trG = hsc[SC_SCRATCH];
  if (loss) {
    if (!kp.V || k == 0 || k == dd)
      *loss = (k == dd ? -1.0 : 1.0) * trG;
    else
      *loss = trG - 2.0 * trGVV;
  }
  const double t1 = now_ms();
  inf.cg_iters += iters;
  inf.ms_polish += t1 - t0;
  inf.ms_total += t1 - t0;
  if (info) *info = inf;
  return out;
}

refl_status_t grad_impl(refl_handle_t h, int64_t d, const double* dH, int64_t ldh,
                        const refl_params_t* pin, const double* dG, int64_t ldg, double* dGrad,
                        int64_t ldgr, double* loss, double* dR, int64_t ldr, refl_info_t* info) {
  const double t_start = now_ms();
  refl_status_t rs = check_params(h, d, pin);
  if (rs != REFL_OK) return rs;
  if (!dH || ldh < d) return fail(h, REFL_ERR_INVALID_ARG, "H is NULL or ldh < d");
  if (!dG || ldg < d) return fail(h, REFL_ERR_INVALID_ARG, "G is NULL or ldg < d");
  if (!dGrad || ldgr < d) return fail(h, REFL_ERR_INVALID_ARG, "gradient output is NULL or ld < d");
  if (dR && ldr < d) return fail(h, REFL_ERR_INVALID_ARG, "ldr < d");
  const refl_params_t p = *pin;
  if (p.precision == REFL_PREC_MIXED) {
    if (p.fixed_steps > 0)
      return fail(h, REFL_ERR_UNSUPPORTED, "MIXED gradient: the limit only (fixed_steps must be 0)");
    return grad_mixed(h, d, dH, ldh, p, dG, ldg, dGrad, ldgr, loss, dR, ldr, info);
  }
  if (p.shift_mode != REFL_SHIFT_GIVEN)
    return fail(h, REFL_ERR_UNSUPPORTED, "refl_sign_grad needs a given shift");
  if (p.grad_mode != REFL_GRAD_REVERSE && p.grad_mode != REFL_GRAD_TANGENT)
    return fail(h, REFL_ERR_INVALID_ARG, "bad grad_mode");
  if (p.ckpt_every < 0) return fail(h, REFL_ERR_INVALID_ARG, "ckpt_every must be >= 0");
  refl_info_t inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.lam_k = inf.lam_k1 = inf.eps = inf.margin = NaN;
  inf.commutator_fro = inf.dk_bound = inf.rho = inf.gamma = NaN;
  inf.index_j = -1;
  inf.s = p.s;
  HIPCHK(hipSetDevice(h->device));
  GradWork g;
  const size_t need = grad_layout(g, nullptr, d, p, h);
  void* base = nullptr;
  rs = ensure_workspace(h, need, &base);
  if (rs != REFL_OK) return rs;
  grad_layout(g, base, d, p, h);
  hipStream_t st = h->stream;
  double* hsc = h->pinned;
  const bool fp64 = g.fp64, reverse = p.grad_mode == REFL_GRAD_REVERSE;
  const int dd = (int)d, dp = g.dp;
  inf.bulk_tile = g.ts;
  if (p.check_symmetric) {
    rs = check_symmetry(h, d, dH, ldh, p.sym_tol, g.scal, SC_SYM);
    if (rs != REFL_OK) return rs;
  }

  // ---- set-up ----
  {
    std::vector<int2> tl;
    build_tiles_nt(dp / g.ts, tl);
    HIPCHK(hipMemcpyAsync(g.tiles, tl.data(), sizeof(int2) * tl.size(), hipMemcpyHostToDevice, st));
    std::vector<int2> tf;
    build_tiles_full(dp / g.ts, tf);
    HIPCHK(hipMemcpyAsync(g.full, tf.data(), sizeof(int2) * tf.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));  // the host vectors go out of scope
  }
  HIPCHK(launch_mirror_upper(dH, ldh, dd, g.Hf, dp, st));
  HIPCHK(launch_scale_inf(g.Hf, dp, dd, p.s, p.scale_mode == REFL_SCALE_FRO,
                          p.scale_mode == REFL_SCALE_GIVEN, p.alpha, g.rowsum, g.scal, st));
  void* X0 = reverse ? g.ck[0] : g.ring[0];
  if (fp64) {
    HIPCHK(launch_init_x0_f64(g.Hf, dp, dd, p.s, g.scal, (double*)X0, st));
    HIPCHK(launch_trace_f64((const double*)X0, dp, dd, g.scal, SC_TRACE, st));
    HIPCHK(launch_sym_in_f64(dG, ldg, dd, nullptr, (double*)g.Gs, dp, st));
    if (!reverse) HIPCHK(launch_sym_in_f64(dG, ldg, dd, g.scal, (double*)g.Gb[0], dp, st));
  } else {
    HIPCHK(launch_init_x0_f32(g.Hf, dp, dd, p.s, g.scal, (float*)X0, st));
    HIPCHK(launch_trace_f32((const float*)X0, dp, dd, g.scal, SC_TRACE, st));
    HIPCHK(launch_sym_in_f32(dG, ldg, dd, nullptr, (float*)g.Gs, dp, st));
    if (!reverse) HIPCHK(launch_sym_in_f32(dG, ldg, dd, g.scal, (float*)g.Gb[0], dp, st));
  }
  HIPCHK(hipMemcpyAsync(hsc, g.scal, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hsc[SC_NONFINITE] > 0.0) return fail(h, REFL_ERR_NOT_FINITE, "H holds non-finite entries");
  inf.alpha = hsc[SC_ALPHA];
  if (!(inf.alpha > 0.0) || !std::isfinite(inf.alpha))
    return fail(h, REFL_ERR_NOT_FINITE, "scale alpha=%g is not a positive finite number", inf.alpha);
  const double t_setup = now_ms();

  // ---- products ----
  size_t nev = 0;
  auto timed = [&](bool on) -> hipError_t {
    if (!p.timing) return hipSuccess;
    if (on) {
      while (h->ev.size() < 2 * (nev + 1)) {
        hipEvent_t e;
        hipError_t er = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);  // timing only
        if (er != hipSuccess) return er;
        h->ev.push_back(e);
      }
      return hipEventRecord(h->ev[2 * nev], st);
    }
    hipError_t er = hipEventRecord(h->ev[2 * nev + 1], st);
    ++nev;
    return er;
  };
  auto residual = [&](void* X, void* N) -> hipError_t {
    return fp64 ? launch_sym_gemm_f64(g.ts, GEMM_RESIDUAL, (double*)X, (double*)X, nullptr, (double*)N,
                                      dp, dd, dp, g.tiles, g.ntiles, g.partials, st)
                : launch_sym_gemm_f32(g.ts, GEMM_RESIDUAL, (float*)X, (float*)X, nullptr, (float*)N, dp,
                                      dd, dp, g.tiles, g.ntiles, g.partials, st);
  };
  auto update = [&](void* X, void* N, void* out) -> hipError_t {
    return fp64 ? launch_sym_gemm_f64(g.ts, GEMM_UPDATE, (double*)X, (double*)N, (double*)X,
                                      (double*)out, dp, dd, dp, g.tiles, g.ntiles, g.partials, st)
                : launch_sym_gemm_f32(g.ts, GEMM_UPDATE, (float*)X, (float*)N, (float*)X, (float*)out, dp,
                                      dd, dp, g.tiles, g.ntiles, g.partials, st);
  };
  // Gout = derivative map at X (with N = I - X^2) applied to Gin.
  auto dstep = [&](void* X, void* N, void* Gin, void* Gout) -> refl_status_t {
    HIPCHK(timed(true));
    if (fp64) {
      HIPCHK(launch_sym_gemm_f64(g.ts, GEMM_PLAIN_NEG, (double*)X, (double*)Gin, nullptr, (double*)g.Pn,
                                 dp, dd, dp, g.full, g.nfull, g.partials, st));
      HIPCHK(launch_adjoint_step_f64(g.ts, (double*)Gin, (double*)N, (double*)g.Pn, (double*)X,
                                     (double*)Gout, dp, dd, dp, g.tiles, g.ntiles, g.partials, st));
    } else {
      HIPCHK(launch_sym_gemm_f32(g.ts, GEMM_PLAIN_NEG, (float*)X, (float*)Gin, nullptr, (float*)g.Pn, dp,
                                 dd, dp, g.full, g.nfull, g.partials, st));
      HIPCHK(launch_adjoint_step_f32(g.ts, (float*)Gin, (float*)N, (float*)g.Pn, (float*)X,
                                     (float*)Gout, dp, dd, dp, g.tiles, g.ntiles, g.partials, st));
    }
    HIPCHK(timed(false));
    return REFL_OK;
  };

  // ---- forward, with the tangent beside it in tangent mode ----
  const bool fixed = p.fixed_steps > 0;
  const int cap = grad_cap(p);
  std::vector<double> hist;
  double trace_cur = hsc[SC_TRACE];
  bool converged = false;
  int m = 0;
  void* cur = X0;
  void* Tcur = g.Gb[0];  // tangent mode: Xdot_j (Xdot_0 = sym(G)/alpha)
  int tg = 1;
  for (;; ++m) {
    void* N = g.keep_all ? g.ns[m] : g.ns[0];
    HIPCHK(residual(cur, N));
    HIPCHK(launch_reduce_sum(g.partials, g.ntiles, g.scal, SC_RESID2, st));
    HIPCHK(hipMemcpyAsync(hsc + SC_RESID2, g.scal + SC_RESID2, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double resid = std::sqrt(std::fmax(hsc[SC_RESID2], 0.0));
    inf.resid_fro = resid;
    inf.trace = trace_cur;
    hist.push_back(resid);
    if (!std::isfinite(resid)) {
      inf.ns_steps = m;
      if (info) *info = inf;
      return fail(h, REFL_ERR_NOT_FINITE, "iterate diverged at step %d", m);
    }
    bool stop = false;
    if (fixed) {
      if (m >= cap) stop = converged = true;
    } else {
      const size_t n = hist.size();
      if (resid < p.tol) stop = converged = true;
      else if (n >= 3 && resid < STAG_R && resid > 0.5 * hist[n - 3]) stop = true;
      else if (m >= cap) stop = true;
    }
    if (stop) break;
    if (!reverse) {
      rs = dstep(cur, N, Tcur, g.Gb[tg]);
      if (rs != REFL_OK) return rs;
      Tcur = g.Gb[tg];
      tg ^= 1;
    }
    void* dst = (reverse && (m + 1) % g.c == 0) ? g.ck[(m + 1) / g.c] : g.ring[(m + 1) & 1];
    HIPCHK(update(cur, N, dst));
    HIPCHK(launch_reduce_sum(g.partials, g.ntiles, g.scal, SC_TRACE, st));
    HIPCHK(hipMemcpyAsync(hsc + SC_TRACE, g.scal + SC_TRACE, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    trace_cur = hsc[SC_TRACE];
    cur = dst;
  }
  inf.ns_steps = m;
  inf.index_j = index_certificate(d, inf.resid_fro, inf.trace);
  if (dR) {
    if (fp64) HIPCHK(launch_copy_out_f64((const double*)cur, dp, dd, dR, ldr, st));
    else HIPCHK(launch_copy_out_f32((const float*)cur, dp, dd, dR, ldr, st));
  }
  const int64_t n2 = (int64_t)dp * dp;
  if (fp64) HIPCHK(launch_dot_f64((const double*)g.Gs, (const double*)cur, n2, g.partials, g.scal, SC_SCRATCH, st));
  else HIPCHK(launch_dot_f32((const float*)g.Gs, (const float*)cur, n2, g.partials, g.scal, SC_SCRATCH, st));
  HIPCHK(hipMemcpyAsync(hsc + SC_SCRATCH, g.scal + SC_SCRATCH, sizeof(double), hipMemcpyDeviceToHost, st));
  const double t_fwd = now_ms();

  // ---- reverse sweep over segments of c steps ----
  if (reverse && g.keep_all) {
    void* Gcur = g.Gs;
    int gi = 0;
    for (int j = m - 1; j >= 0; --j) {
      rs = dstep(g.ck[j], g.ns[j], Gcur, g.Gb[gi]);
      if (rs != REFL_OK) return rs;
      Gcur = g.Gb[gi];
      gi ^= 1;
    }
    if (fp64) HIPCHK(launch_copy_out_scaled_f64((const double*)Gcur, dp, dd, g.scal, dGrad, ldgr, st));
    else HIPCHK(launch_copy_out_scaled_f32((const float*)Gcur, dp, dd, g.scal, dGrad, ldgr, st));
  } else if (reverse) {
    void* Gcur = g.Gs;
    int gi = 0;
    const int nseg = (m + g.c - 1) / g.c;
    std::vector<void*> xj(g.c);
    for (int sgm = nseg - 1; sgm >= 0; --sgm) {
      const int a = sgm * g.c, b = std::min(a + g.c, m);
      xj[0] = g.ck[sgm];
      for (int j = a; j < b; ++j) {
        HIPCHK(residual(xj[j - a], g.ns[j - a]));
        if (j + 1 < b) {
          HIPCHK(update(xj[j - a], g.ns[j - a], g.xs[j + 1 - a]));
          xj[j + 1 - a] = g.xs[j + 1 - a];
        }
      }
      for (int j = b - 1; j >= a; --j) {
        rs = dstep(xj[j - a], g.ns[j - a], Gcur, g.Gb[gi]);
        if (rs != REFL_OK) return rs;
        Gcur = g.Gb[gi];
        gi ^= 1;
      }
    }
    if (fp64) HIPCHK(launch_copy_out_scaled_f64((const double*)Gcur, dp, dd, g.scal, dGrad, ldgr, st));
    else HIPCHK(launch_copy_out_scaled_f32((const float*)Gcur, dp, dd, g.scal, dGrad, ldgr, st));
  } else {
    if (fp64) HIPCHK(launch_copy_out_f64((const double*)Tcur, dp, dd, dGrad, ldgr, st));
    else HIPCHK(launch_copy_out_f32((const float*)Tcur, dp, dd, dGrad, ldgr, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  if (loss) *loss = hsc[SC_SCRATCH];
  if (p.timing) {
    double tot = 0.0;
    for (size_t i = 0; i < nev; ++i) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]));
      tot += ms;
    }
    inf.ms_gemm = tot;
    inf.gemm_launches = (int)nev;
  }
  const double t_end = now_ms();
  inf.ms_setup = t_setup - t_start;
  inf.ms_bulk = t_fwd - t_setup;
  inf.ms_polish = t_end - t_fwd;
  inf.ms_total = t_end - t_start;
  if (info) *info = inf;
  if (!converged)
    return fail(h, REFL_ERR_NOT_CONVERGED, "no convergence after %d steps (resid %.3e)", m, inf.resid_fro);
  if (!fixed && p.k > 0 && inf.index_j >= 0 && inf.index_j != p.k)
    return fail(h, REFL_ERR_NOT_ADMISSIBLE,
                "index certificate found %d negative eigenvalues of H - sI, not k=%d", inf.index_j, p.k);
  return REFL_OK;
}

// ------------------------------------------------------------ estimation
// Block Lanczos on H (refl_estimate_shift and the policy refreshes).
refl_status_t estimate_impl(refl_handle_t h, int64_t d, const double* dH, int64_t ldh, int k,
                            int steps, uint64_t seed, LzResult& lr, const double* start = nullptr,
                            double* ritz_out = nullptr) {
  if (!dH || ldh < d) return fail(h, REFL_ERR_INVALID_ARG, "H is NULL or ldh < d");
  refl_params_t p;
  refl_params_default(&p);
  p.k = k;
  p.shift_mode = REFL_SHIFT_LANCZOS;
  p.lanczos_steps = steps;
  p.seed = seed;
  refl_status_t rs = check_params(h, d, &p);
  if (rs != REFL_OK) return rs;
  HIPCHK(hipSetDevice(h->device));
  Work w;
  const size_t need = layout(w, nullptr, d, p, LAYOUT_ESTIMATE, h);
  void* base = nullptr;
  rs = ensure_workspace(h, need, &base);
  if (rs != REFL_OK) return rs;
  layout(w, base, d, p, LAYOUT_ESTIMATE, h);
  HIPCHK(launch_mirror_upper(dH, ldh, (int)d, w.Hf, w.dp, h->stream));
  return lanczos_run(h, w.Hf, w.dp, d, k, seed, w.lz, w.thin, lr, start, d, ritz_out, d);
}

#ifdef REFL_DEBUG
}  // namespace
namespace refl {
int refl_dbg_take_gemm_w();
int refl_dbg_take_gemm_f();
int refl_dbg_take_misc();
int refl_dbg_take_lanczos();
}  // namespace refl
namespace {
// Reads and clears every unit's guard record after the stream's work; a
// tripped guard takes precedence over the call's own status.
refl_status_t dbg_finish(refl_handle_t h, refl_status_t rs) {
  if (!h) return rs;
  if (hipSetDevice(h->device) != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
    return rs == REFL_OK ? fail(h, REFL_ERR_DEVICE, "stream synchronisation failed") : rs;
  int (*const take[])() = {refl_dbg_take_gemm_w, refl_dbg_take_gemm_f, refl_dbg_take_misc,
                           refl_dbg_take_lanczos};
  int site = 0;
  for (auto f : take) {
    const int v = f();
    if (v != 0 && site <= 0) site = v;
  }
  if (site < 0) return fail(h, REFL_ERR_DEVICE, "debug guard records unreadable");
  if (site > 0) return fail(h, REFL_ERR_BOUNDS, "launch-extent guard tripped: %s", dbg_site_name(site));
  return rs;
}
#else
inline refl_status_t dbg_finish(refl_handle_t, refl_status_t rs) { return rs; }
#endif

// REFL_LOG (environment, read once): when set and not "0", every entry point
// that runs device work writes one line to stderr as it returns: its name,
// the order, the status and, where the caller passed a refl_info_t, the
// solve's figures (steps, sweeps, inner iterations, certified index, the
// last residual, the Davis-Kahan bound, wall-clock per phase); on an error
// also the handle's message.
bool log_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("REFL_LOG");
    return e && *e && std::strcmp(e, "0") != 0;
  }();
  return on;
}

refl_status_t log_call(refl_handle_t h, const char* name, int64_t d, refl_status_t rs,
                       const refl_info_t* info) {
  if (!log_enabled()) return rs;
  if (info)
    std::fprintf(stderr,
                 "refl: %s d=%lld status=%s steps=%d sweeps=%d cg=%d j=%d tile=%d words=%d "
                 "resid=%.3e dk=%.3e ms=%.3f (setup %.3f bulk %.3f polish %.3f)\n",
                 name, (long long)d, refl_status_string(rs), info->ns_steps, info->polish_sweeps,
                 info->cg_iters, info->index_j, info->bulk_tile, info->bulk_words, info->resid_fro,
                 info->dk_bound, info->ms_total, info->ms_setup, info->ms_bulk, info->ms_polish);
  else
    std::fprintf(stderr, "refl: %s d=%lld status=%s\n", name, (long long)d, refl_status_string(rs));
  if (rs != REFL_OK && h) std::fprintf(stderr, "refl:   %s\n", h->err);
  return rs;
}

}  // namespace

extern "C" {

refl_status_t refl_params_default(refl_params_t* p) {
  if (!p) return REFL_ERR_INVALID_ARG;
  std::memset(p, 0, sizeof(*p));
  p->k = 1;
  p->s = 0.0;
  p->shift_mode = REFL_SHIFT_GIVEN;
  p->scale_mode = REFL_SCALE_INF;
  p->precision = REFL_PREC_FP64;
  p->alpha = 0.0;
  p->tol = 1e-12;
  p->max_iter = 100;
  p->fixed_steps = 0;
  p->words = 2;
  p->polish_sweeps = 2;
  p->cg_tol = 1e-6;
  p->cg_max_iter = 400;
  p->lanczos_steps = 0;
  p->seed = 0;
  p->timing = 0;
  p->grad_mode = REFL_GRAD_REVERSE;
  p->ckpt_every = 0;
  p->cg_f32 = REFL_CG_AUTO;
  p->check_symmetric = 0;
  p->sym_tol = 0.0;
  p->words_max = 3;
  return REFL_OK;
}

refl_status_t refl_create(refl_handle_t* out, int device, void* hip_stream) {
  if (!out) return REFL_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return REFL_ERR_DEVICE;
  refl_handle_s* h = new (std::nothrow) refl_handle_s();
  if (!h) return REFL_ERR_NO_MEMORY;
  h->device = device;
  h->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete h;
    return REFL_ERR_DEVICE;
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      ncu > 0)
    h->ncu = ncu;
  const size_t pin_bytes = sizeof(double) * SC_COUNT + sizeof(CgHost) + 256 +
                           sizeof(double) * (2 * MAXB * MAXB + MAXB);
  if (hipHostMalloc((void**)&h->pinned, pin_bytes, hipHostMallocDefault) != hipSuccess) {
    delete h;
    return REFL_ERR_NO_MEMORY;
  }
  std::memset(h->pinned, 0, pin_bytes);
  // Resources the refl_sign path would otherwise create on first use, made
  // here so that refl_sign_noalloc never has to.
  bool ok = hipHostMalloc((void**)&h->lz_pin, LZ_PIN_INITIAL, hipHostMallocDefault) == hipSuccess;
  if (ok) h->lz_pin_bytes = LZ_PIN_INITIAL;
  for (int e = 0; ok && e < 2; ++e)
    ok = hipEventCreateWithFlags(&h->lz_ev[e], hipEventDisableTiming) == hipSuccess;
  while (ok && (int)h->bulk_ev.size() < BULK_RING) {
    hipEvent_t e;
    ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    if (ok) h->bulk_ev.push_back(e);
  }
  if (!ok) {
    refl_destroy(h);
    return REFL_ERR_NO_MEMORY;
  }
  // The fixed scratch of the allocation-free entry point on this device
  // (current here).  A failure is kept and reported by that entry point
  // only; every other call works without it.
  h->scratch_err = noalloc_scratch(device, &h->scratch);
  if (h->scratch_err != hipSuccess) {
    h->scratch = nullptr;
    (void)hipGetLastError();
  }
  *out = h;
  return REFL_OK;
}

refl_status_t refl_destroy(refl_handle_t h) {
  if (!h) return REFL_ERR_INVALID_ARG;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  if (h->ws_own) (void)hipFree(h->ws_own);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->bulk_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->lz_ev)
    if (e) (void)hipEventDestroy(e);
  if (h->lz_pin) (void)hipHostFree(h->lz_pin);
  if (h->batch_pin) (void)hipHostFree(h->batch_pin);
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->bgraph) (void)hipGraphExecDestroy(h->bgraph);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->side) (void)hipStreamDestroy(h->side);
  for (hipEvent_t e : h->side_ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
  return REFL_OK;
}

refl_status_t refl_set_stream(refl_handle_t h, void* hip_stream) {
  if (!h) return REFL_ERR_INVALID_ARG;
  h->stream = (hipStream_t)hip_stream;
  return REFL_OK;
}

refl_status_t refl_workspace_size(refl_handle_t h, int64_t d, const refl_params_t* p,
                                  size_t* bytes) {
  if (!h || !bytes) return REFL_ERR_INVALID_ARG;
  refl_status_t rs = check_params(h, d, p);
  if (rs != REFL_OK) return rs;
  Work w;
  *bytes = layout(w, nullptr, d, *p, LAYOUT_SIGN, h);
  return REFL_OK;
}

refl_status_t refl_set_workspace(refl_handle_t h, void* dptr, size_t bytes) {
  if (!h) return REFL_ERR_INVALID_ARG;
  if (dptr && ((uintptr_t)dptr % 256) != 0)
    return fail(h, REFL_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  h->ws_user = dptr;
  h->ws_user_bytes = dptr ? bytes : 0;
  return REFL_OK;
}

refl_status_t refl_sign(refl_handle_t h, int64_t d, const double* dH, int64_t ldh,
                        const refl_params_t* p, double* dR, int64_t ldr, refl_info_t* info) {
  if (!h) return REFL_ERR_INVALID_ARG;
  if (!dR || ldr < d) return fail(h, REFL_ERR_INVALID_ARG, "R is NULL or ldr < d");
  return log_call(h, "refl_sign", d,
                  dbg_finish(h, sign_impl(h, d, dH, ldh, p, dR, ldr, 0, nullptr, 0, nullptr, 0, info)),
                  info);
}

refl_status_t refl_sign_noalloc(refl_handle_t h, int64_t d, const double* dH, int64_t ldh,
                                const refl_params_t* p, double* dR, int64_t ldr, refl_info_t* info) {
  if (!h) return REFL_ERR_INVALID_ARG;
  if (!dR || ldr < d) return fail(h, REFL_ERR_INVALID_ARG, "R is NULL or ldr < d");
  if (p && p->timing)
    return fail(h, REFL_ERR_INVALID_ARG, "params.timing creates events: not available without allocation");
  struct Scope {
    refl_handle_t h;
    explicit Scope(refl_handle_t hh) : h(hh) { h->no_alloc = true; }
    ~Scope() { h->no_alloc = false; }
  } scope(h);
  return log_call(h, "refl_sign_noalloc", d,
                  dbg_finish(h, sign_impl(h, d, dH, ldh, p, dR, ldr, 0, nullptr, 0, nullptr, 0, info)),
                  info);
}

refl_status_t refl_sign_apply(refl_handle_t h, int64_t d, const double* dH, int64_t ldh,
                              const refl_params_t* p, int64_t nrhs, const double* dV,
                              int64_t ldv, double* dY, int64_t ldy, refl_info_t* info) {
  if (!h) return REFL_ERR_INVALID_ARG;
  if (nrhs < 1 || !dV || !dY || ldv < d || ldy < d)
    return fail(h, REFL_ERR_INVALID_ARG, "bad V/Y block (nrhs >= 1, ld >= d)");
  return log_call(h, "refl_sign_apply", d,
                  dbg_finish(h, sign_impl(h, d, dH, ldh, p, nullptr, 0, nrhs, dV, ldv, dY, ldy, info)),
                  info);
}

refl_status_t refl_apply(refl_handle_t h, int64_t d, const double* dR, int64_t ldr, int64_t nrhs,
                         const double* dV, int64_t ldv, double* dY, int64_t ldy) {
  if (!h) return REFL_ERR_INVALID_ARG;
  if (d < 1 || !dR || ldr < d || nrhs < 1 || !dV || !dY || ldv < d || ldy < d)
    return fail(h, REFL_ERR_INVALID_ARG, "bad arguments to refl_apply");
  HIPCHK(hipSetDevice(h->device));
  refl_params_t p;
  refl_params_default(&p);
  Work w;
  const size_t need = layout(w, nullptr, d, p, LAYOUT_APPLY, h);
  void* base = nullptr;
  refl_status_t rs = ensure_workspace(h, need, &base);
  if (rs != REFL_OK) return rs;
  layout(w, base, d, p, LAYOUT_APPLY, h);
  for (int64_t c0 = 0; c0 < nrhs; c0 += MAXB) {
    const int nb = (int)std::min<int64_t>(MAXB, nrhs - c0);
    HIPCHK(thin_gemm_f64(dR, ldr, (int)d, dV + c0 * ldv, ldv, nb, dY + c0 * ldy, ldy, w.thin, h->stream));
  }
  return log_call(h, "refl_apply", d, dbg_finish(h, REFL_OK), nullptr);
}

refl_status_t refl_estimate_shift(refl_handle_t h, int64_t d, const double* dH, int64_t ldh,
                                  int32_t k, int32_t steps, uint64_t seed, double* s,
                                  double* lam_k, double* lam_k1, double* eps, double* rho) {
  if (!h) return REFL_ERR_INVALID_ARG;
  if (!s || !lam_k || !lam_k1 || !eps || !rho) return fail(h, REFL_ERR_INVALID_ARG, "NULL output");
  LzResult lr;
  refl_status_t rs = dbg_finish(h, estimate_impl(h, d, dH, ldh, k, steps, seed, lr));
  if (rs != REFL_OK) return log_call(h, "refl_estimate_shift", d, rs, nullptr);
  *s = lr.s;
  *lam_k = lr.lam_k;
  *lam_k1 = lr.lam_k1;
  *eps = lr.eps;
  *rho = lr.rho;
  return log_call(h, "refl_estimate_shift", d, lanczos_status(h, lr), nullptr);
}

refl_status_t refl_sign_batched_workspace_size(refl_handle_t h, int32_t nprob, const int64_t* d,
                                               const refl_params_t* params, size_t* bytes) {
  if (!h || !bytes) return REFL_ERR_INVALID_ARG;
  if (nprob < 1 || !d || !params) return fail(h, REFL_ERR_INVALID_ARG, "nprob, d or params");
  for (int p = 0; p < nprob; ++p) {
    refl_status_t rs = check_params(h, d[p], &params[p]);
    if (rs != REFL_OK) return rs;
  }
  const bool fp64 = params[0].precision == REFL_PREC_FP64;
  std::vector<int> tsv(nprob);
  for (int p = 0; p < nprob; ++p) tsv[p] = select_tile_f(h, d[p], fp64);
  BatchWork bw;
  *bytes = batch_layout(bw, nullptr, nprob, d, tsv.data(), fp64);
  return REFL_OK;
}

refl_status_t refl_sign_batched(refl_handle_t h, int32_t nprob, const int64_t* d,
                                const double* const* dH, const int64_t* ldh,
                                const refl_params_t* params, double* const* dR,
                                const int64_t* ldr, refl_info_t* info, refl_status_t* status) {
  if (!h) return REFL_ERR_INVALID_ARG;
  return log_call(h, "refl_sign_batched (order of problem 0)", nprob > 0 && d ? d[0] : 0,
                  dbg_finish(h, batched_impl(h, nprob, d, dH, ldh, params, dR, ldr, info, status)),
                  nullptr);
}

refl_status_t refl_sign_grad(refl_handle_t h, int64_t d, const double* dH, int64_t ldh,
                             const refl_params_t* p, const double* dG, int64_t ldg, double* dGrad,
                             int64_t ldgr, double* loss, double* dR, int64_t ldr,
                             refl_info_t* info) {
  if (!h) return REFL_ERR_INVALID_ARG;
  return log_call(h, "refl_sign_grad", d,
                  dbg_finish(h, grad_impl(h, d, dH, ldh, p, dG, ldg, dGrad, ldgr, loss, dR, ldr, info)),
                  info);
}

refl_status_t refl_policy_create(refl_handle_t h, const refl_policy_params_t* pp,
                                 refl_policy_t* out) {
  if (!h || !pp || !out) return REFL_ERR_INVALID_ARG;
  *out = nullptr;
  if (pp->mode < REFL_POLICY_MIDPOINT || pp->mode > REFL_POLICY_REUSE)
    return fail(h, REFL_ERR_INVALID_ARG, "bad policy mode");
  if (pp->k < 1) return fail(h, REFL_ERR_INVALID_ARG, "policy k must be >= 1");
  if (pp->mode == REFL_POLICY_DAMPED &&
      !(pp->beta > 0.0 && pp->beta <= 1.0 && pp->clip > 0.0 && pp->clip <= 1.0))
    return fail(h, REFL_ERR_INVALID_ARG, "DAMPED needs 0 < beta <= 1 and 0 < clip <= 1");
  if (pp->mode == REFL_POLICY_REUSE && !(pp->tau >= 0.0 && pp->tau < 1.0))
    return fail(h, REFL_ERR_INVALID_ARG, "REUSE needs 0 <= tau < 1");
  if (pp->lanczos_steps < 0) return fail(h, REFL_ERR_INVALID_ARG, "lanczos_steps must be >= 0");
  refl_policy_s* pol = new (std::nothrow) refl_policy_s();
  if (!pol) return fail(h, REFL_ERR_NO_MEMORY, "policy allocation failed");
  pol->pp = *pp;
  pol->device = h->device;
  *out = pol;
  return REFL_OK;
}

refl_status_t refl_policy_destroy(refl_policy_t pol) {
  if (!pol) return REFL_ERR_INVALID_ARG;
  (void)hipSetDevice(pol->device);
  (void)hipDeviceSynchronize();
  if (pol->Href) (void)hipFree(pol->Href);
  if (pol->dscr) (void)hipFree(pol->dscr);
  if (pol->Vwarm) (void)hipFree(pol->Vwarm);
  delete pol;
  return REFL_OK;
}

static refl_status_t policy_shift_impl(refl_handle_t h, refl_policy_t pol, int64_t d, const double* dH,
                                       int64_t ldh, double* s_out, refl_policy_info_t* info) {
  if (!h || !pol || !s_out) return REFL_ERR_INVALID_ARG;
  if (pol->device != h->device) return fail(h, REFL_ERR_INVALID_ARG, "policy and handle devices differ");
  if (!dH || ldh < d || d < 2 || pol->pp.k > d - 1)
    return fail(h, REFL_ERR_INVALID_ARG, "H is NULL, ldh < d, or k outside 1..d-1");
  HIPCHK(hipSetDevice(h->device));
  hipStream_t st = h->stream;
  const refl_policy_params_t& pp = pol->pp;
  refl_policy_info_t inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.drift = NaN;
  pol->calls += 1;
  // Reuse: certified margin of the kept shift at this H.
  if (pp.mode == REFL_POLICY_REUSE && pol->have && pol->dref == d) {
    const size_t need = (size_t)diff_fro_partials((int)d) + 1;
    if (pol->dscr_n < need) {
      if (pol->dscr) HIPCHK(hipFree(pol->dscr));
      pol->dscr = nullptr;
      pol->dscr_n = 0;
      if (hipMalloc(&pol->dscr, need * sizeof(double)) != hipSuccess)
        return fail(h, REFL_ERR_NO_MEMORY, "policy scratch allocation failed");
      pol->dscr_n = need;
    }
    double* slot = pol->dscr + (need - 1);
    HIPCHK(launch_diff_fro_upper(dH, ldh, pol->Href, pol->dref, (int)d, pol->dscr, slot, 0, st));
    HIPCHK(hipMemcpyAsync(h->pinned + SC_SCRATCH, slot, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double drift = std::sqrt(std::fmax(h->pinned[SC_SCRATCH], 0.0));
    const double margin =
        std::min(pol->s - pol->lam_k, pol->lam_k1 - pol->s) - pol->eps - drift;
    if (margin > pp.tau * 0.5 * (pol->lam_k1 - pol->lam_k)) {
      inf.s = pol->s;
      inf.lam_k = pol->lam_k;
      inf.lam_k1 = pol->lam_k1;
      inf.eps = pol->eps;
      inf.margin = margin;
      inf.drift = drift;
      inf.calls = pol->calls;
      inf.refreshes = pol->refreshes;
      *s_out = pol->s;
      if (info) *info = inf;
      return REFL_OK;
    }
  }
  // Refresh: estimate the gap endpoints on this H.  With warm_start the
  // run starts from the Ritz block of the previous refresh on a matrix of
  // the same order (and falls back to the seeded start if that run fails),
  // and leaves its own Ritz block for the next refresh.
  LzResult lr;
  refl_status_t rs = REFL_ERR_NOT_CONVERGED;
  bool ran = false;
  if (pp.warm_start) {
    const int b = lz_block(d, pp.k);
    if (pol->dwarm != d) {
      if (pol->Vwarm) HIPCHK(hipFree(pol->Vwarm));
      pol->Vwarm = nullptr;
      pol->dwarm = 0;
      if (hipMalloc(&pol->Vwarm, sizeof(double) * (size_t)d * b) != hipSuccess)
        return fail(h, REFL_ERR_NO_MEMORY, "policy warm-start block (%lld x %d) failed", (long long)d, b);
    } else {
      rs = estimate_impl(h, d, dH, ldh, pp.k, pp.lanczos_steps, pp.seed, lr, pol->Vwarm, pol->Vwarm);
      ran = rs == REFL_OK;
    }
    if (!ran) {
      lr = LzResult();
      rs = estimate_impl(h, d, dH, ldh, pp.k, pp.lanczos_steps, pp.seed, lr, nullptr, pol->Vwarm);
      ran = true;
    }
    pol->dwarm = rs == REFL_OK ? d : 0;
  }
  if (!ran) rs = estimate_impl(h, d, dH, ldh, pp.k, pp.lanczos_steps, pp.seed, lr);
  pol->refreshes += 1;
  inf.refreshed = 1;
  inf.lanczos_steps = lr.steps;
  inf.calls = pol->calls;
  inf.refreshes = pol->refreshes;
  inf.lam_k = lr.lam_k;
  inf.lam_k1 = lr.lam_k1;
  inf.eps = lr.eps;
  if (rs != REFL_OK && rs != REFL_ERR_NOT_ADMISSIBLE && rs != REFL_ERR_NO_GAP) {
    pol->have = false;
    return rs;
  }
  if (rs == REFL_ERR_NO_GAP) {
    pol->have = false;
    inf.s = lr.s;
    inf.margin = NaN;
    *s_out = lr.s;
    if (info) *info = inf;
    return rs;
  }
  double s = lr.s;  // the midpoint (Prop. 4.1)
  const double w = 0.5 * (lr.lam_k1 - lr.lam_k) - lr.eps;  // certified half-width
  if (pp.mode == REFL_POLICY_DAMPED && pol->have && w > 0.0) {
    const double raw = (1.0 - pp.beta) * pol->s + pp.beta * s;
    const double lo = lr.lam_k + lr.eps + pp.clip * w, hi = lr.lam_k1 - lr.eps - pp.clip * w;
    s = std::min(std::max(raw, lo), hi);
  }
  const double margin = std::min(s - lr.lam_k, lr.lam_k1 - s) - lr.eps;
  inf.s = s;
  inf.margin = margin;
  *s_out = s;
  const bool ok = margin > 0.0;
  pol->have = ok;
  if (ok) {
    pol->s = s;
    pol->lam_k = lr.lam_k;
    pol->lam_k1 = lr.lam_k1;
    pol->eps = lr.eps;
    if (pp.mode == REFL_POLICY_REUSE) {
      if (pol->dref != d || !pol->Href) {
        if (pol->Href) HIPCHK(hipFree(pol->Href));
        pol->Href = nullptr;
        pol->dref = 0;
        if (hipMalloc(&pol->Href, (size_t)d * d * sizeof(double)) != hipSuccess) {
          pol->have = false;
          return fail(h, REFL_ERR_NO_MEMORY, "policy copy of H (%lld^2 doubles) failed", (long long)d);
        }
        pol->dref = d;
      }
      HIPCHK(launch_copy_upper(dH, ldh, pol->Href, d, (int)d, st));
      HIPCHK(hipStreamSynchronize(st));
    }
  }
  if (info) *info = inf;
  if (!ok)
    return fail(h, REFL_ERR_NOT_ADMISSIBLE, "policy shift margin %.3e is not positive", margin);
  return REFL_OK;
}

refl_status_t refl_policy_shift(refl_handle_t h, refl_policy_t pol, int64_t d, const double* dH,
                                int64_t ldh, double* s_out, refl_policy_info_t* info) {
  return log_call(h, "refl_policy_shift", d,
                  dbg_finish(h, policy_shift_impl(h, pol, d, dH, ldh, s_out, info)), nullptr);
}

int refl_debug_build(void) {
#ifdef REFL_DEBUG
  return 1;
#else
  return 0;
#endif
}

const char* refl_status_string(refl_status_t s) {
  // A C caller may pass any int: read the code as an int rather than load
  // an out-of-range value of the enum type.
  int code;
  static_assert(sizeof(code) == sizeof(s), "status codes are ints");
  std::memcpy(&code, &s, sizeof(code));
  switch (code) {
    case REFL_OK: return "REFL_OK";
    case REFL_ERR_INVALID_ARG: return "REFL_ERR_INVALID_ARG";
    case REFL_ERR_DEVICE: return "REFL_ERR_DEVICE";
    case REFL_ERR_NO_MEMORY: return "REFL_ERR_NO_MEMORY";
    case REFL_ERR_NOT_CONVERGED: return "REFL_ERR_NOT_CONVERGED";
    case REFL_ERR_NOT_ADMISSIBLE: return "REFL_ERR_NOT_ADMISSIBLE";
    case REFL_ERR_NO_GAP: return "REFL_ERR_NO_GAP";
    case REFL_ERR_NOT_SYMMETRIC: return "REFL_ERR_NOT_SYMMETRIC";
    case REFL_ERR_NOT_FINITE: return "REFL_ERR_NOT_FINITE";
    case REFL_ERR_UNSUPPORTED: return "REFL_ERR_UNSUPPORTED";
    case REFL_ERR_BOUNDS: return "REFL_ERR_BOUNDS";
  }
  return "REFL_ERR_UNKNOWN";
}

const char* refl_last_error(refl_handle_t h) { return h ? h->err : "NULL handle"; }

}  // extern "C"
