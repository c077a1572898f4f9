// C ABI of the tensor B-spline library: argument validation, taps, workspace layout and the
// host-side orchestration of the HIP kernels (apply, RHS, fused CG, refinement, time step).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tbs.h"
#include "common.h"
#include "net.h"
#include "stencil.h"
#include "transfer.h"
#include "varcoef.h"
#include "refine.h"

using namespace tbs;

// ------------------------------------------------------------------------------------------
// error text

static thread_local std::string g_last_error;

static int set_err(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIPCHK(expr)                                                                             \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return set_err(TBS_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

extern "C" const char* tbs_strerror(int code) {
  switch (code) {
    case TBS_OK: return "ok";
    case TBS_E_INVAL: return "invalid argument";
    case TBS_E_NOMEM: return "workspace missing or too small";
    case TBS_E_HIP: return "HIP runtime error";
    case TBS_E_BREAKDOWN: return "CG breakdown (p^T A p <= 0 or non-finite value)";
    case TBS_E_STATE: return "call out of order";
    case TBS_W_NOT_CONVERGED: return "not converged within the iteration limit";
  }
  return "unknown code";
}

extern "C" const char* tbs_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------------------------------
// B-spline taps (FP64, host): m_k = b^{2n+1}(k), s_k = -(b^{2n+1})''(k)

// centred B-spline of degree p at x by the truncated-power form of the (p+1)-fold box convolution
static double bspline_val(int p, double x) {
  const double half = 0.5 * (p + 1);
  if (!(x > -half && x < half)) return 0.0;
  double acc = 0.0, binom = 1.0, fact = 1.0;
  for (int i = 2; i <= p; ++i) fact *= i;
  for (int j = 0; j <= p + 1; ++j) {
    const double t = x + half - j;
    if (t > 0) acc += ((j & 1) ? -binom : binom) * std::pow(t, p);
    binom = binom * (p + 1 - j) / (j + 1);
  }
  return acc / fact;
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on P_q from the three-term recurrence
static void gauss_legendre(int q, double* x, double* w) {
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;  // P_0(z), P_1(z)
      for (int k = 2; k <= q; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);  // P_q'(z)
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// derivative of the degree-p B-spline: difference of two shifted degree p-1 splines (p >= 1)
static double bspline_der(int p, double x) { return bspline_val(p - 1, x + 0.5) - bspline_val(p - 1, x - 0.5); }

// Corner blocks of the box-domain (Robin / penalty) operator, unit spacing (Sec. 2.2 Robin form,
// Sec. 2.3 boundary branch): the box mass and stiffness integrals over [0, Nc] differ from the
// Toeplitz taps only where both B-splines reach past an end, by minus their integral over
// (-inf, 0]; the boundary matrix is E[r][c] = b(-k_r) b(-k_c).  Rows and columns r, c < z, offsets
// k = index - floor(n/2); exact up to rounding (n+1 Gauss points on every half-unit piece).
static void robin_corners(int n, const double h[3], double tau, double gamma, RobinCorner* rb) {
  const int z = 2 * (n / 2) + 1;
  double gx[8], gw[8];
  gauss_legendre(n + 1, gx, gw);
  std::memset(rb, 0, sizeof(*rb));
  rb->z = z;
  const double a[3] = {tau / (h[0] * h[0]), tau / (h[1] * h[1]), tau / (h[2] * h[2])};
  const double e[3] = {tau / (2.0 * gamma * h[0]), tau / (2.0 * gamma * h[1]), tau / (2.0 * gamma * h[2])};
  for (int r = 0; r < z; ++r) {
    for (int c = 0; c < z; ++c) {
      const double kr = r - n / 2, kc = c - n / 2;
      double im = 0.0, ik = 0.0;
      for (int piece = 0; piece < 2 * (n + 3); ++piece) {  // [-(n+3), 0] in half-unit pieces
        const double lo = -(n + 3) + 0.5 * piece, mid = lo + 0.25;
        for (int g = 0; g < n + 1; ++g) {
          const double x = mid + 0.25 * gx[g], w = 0.25 * gw[g];
          im += w * bspline_val(n, x - kr) * bspline_val(n, x - kc);
          ik += w * bspline_der(n, x - kr) * bspline_der(n, x - kc);
        }
      }
      const double E = bspline_val(n, -kr) * bspline_val(n, -kc);
      const int i = r * kRobinMaxZ + c;
      rb->cm[i] = -im;
      rb->cvx[i] = -im - a[0] * ik + e[0] * E;
      rb->cwy[i] = -a[1] * ik + e[1] * E;
      rb->cwz[i] = -a[2] * ik + e[2] * E;
    }
  }
}

static void make_taps(int n, double* m, double* s) {
  const int p = 2 * n + 1;
  for (int k = 0; k <= n; ++k) {
    m[k] = bspline_val(p, (double)k);
    // second derivative = second difference of the degree p-2 spline (derivative rule twice)
    s[k] = -(bspline_val(p - 2, k + 1.0) - 2.0 * bspline_val(p - 2, (double)k) + bspline_val(p - 2, k - 1.0));
  }
}

// ------------------------------------------------------------------------------------------
// context

struct tbs_ctx {
  int64_t nx, ny, nz, N;
  int n, bc;
  double h[3], tau;
  double gamma;      // Robin / penalty parameter (TBS_BC_ROBIN)
  RobinCorner rb;    // its corner blocks
  hipStream_t st;
  Taps taps;
  int tiles_x, tiles_y, nchunks, zc, nblocks, nparts;
  char* ws;
  size_t ws_bytes;
  tbs_opts opts;
  Scalars* host_scal;  // pinned mirror, allocated on first solver call
  int transform_degree;  // > 0: transform context (operator = sampled-B-spline evaluation filter)
  tbs_ctx* coarse;       // coarse-grid guess: context of the halved grid (opts.coarse_guess)
  int64_t cgrid[3];
  // learned-guess backoff (opts.guess_backoff): consecutive rejections, steps left to skip
  int guess_rejects, guess_wait;
  hipEvent_t cost_ev[4];  // guess_backoff 2: network + test start / end, CG loop start / end
  bool cost_ev_made;
  int cgf_pend;  // host copy of the pending x-update count of the one-kernel CG (for its byte count)
  bool cgf_xzero;  // host copy of Scalars::xzero for the refinement's inner solve (same use)
  // CG session state (tbs_cg_begin / tbs_cg_step)
  int cg_active, cg_dt, cg_enq;
  void* cg_x;
  // kernel timing (tbs_prof_enable)
  struct ProfRec { int kind; int k; double bytes; hipEvent_t e0, e1; };
  int prof_on;
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  double prof_ms[TBS_PROF_KINDS], prof_bytes[TBS_PROF_KINDS];
  int64_t prof_count[TBS_PROF_KINDS];
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static bool aligned_ptr(const void* p) { return p && ((uintptr_t)p & 255u) == 0; }

static void plan_geometry(tbs_ctx* c, int zchunk) {
  c->tiles_x = (int)((c->nx + kTileX - 1) / kTileX);
  c->tiles_y = (int)((c->ny + kTileY - 1) / kTileY);  // finest tiling: bounds the partial-sum count
  const int64_t tiles = (int64_t)c->tiles_x * c->tiles_y;
  const int64_t plan_tiles = (int64_t)c->tiles_x * ((c->ny + kTileYPlan - 1) / kTileYPlan);
  // about 8192 workgroups (many times what 256 CUs hold at once: the z-marching waves finish at
  // different times and short chunks even out the tail), but chunks of at least 4(2n+1) planes;
  // at 928^3 this gives 93-plane chunks, 1 % faster for the CG iteration than 186
  int64_t want = (8192 + plan_tiles - 1) / plan_tiles;
  const int64_t minzc = std::max<int64_t>(16, 4 * (2 * c->n + 1));
  int64_t maxchunks = std::max<int64_t>(1, c->nz / minzc);
  int64_t chunks = std::min(want, maxchunks);
  if (chunks < 1) chunks = 1;
  c->zc = (int)((c->nz + chunks - 1) / chunks);
  if (zchunk > 0) c->zc = (int)std::min<int64_t>(zchunk, c->nz);
  c->nchunks = (int)((c->nz + c->zc - 1) / c->zc);
  c->nblocks = (int)(tiles * c->nchunks);
  c->nparts = std::max(c->nblocks, kVecBlocks);
}

// workspace layout: [scalars x4][part0][part1][part2][part3][arrays...]
enum { SC_CG = 0, SC_AUX = 1 };
static size_t ws_head(const tbs_ctx* c) { return 1024 + 4 * align256((size_t)c->nparts * 8); }

struct Layout {
  size_t bytes;
  size_t off[8];
  size_t coff[6];  // coarse-grid guess: FP64 r0, transfer temporaries T1, T2, coarse b, coarse x, coarse workspace
};

extern "C" size_t tbs_workspace_bytes(const tbs_ctx* c, int prec);

static Layout layout(const tbs_ctx* c, int prec) {
  Layout L{};
  size_t o = ws_head(c);
  const size_t N = (size_t)c->N;
  auto put = [&](int i, size_t esz) { L.off[i] = o; o += align256(N * esz); };
  switch (prec) {
    case -1: break;
    case TBS_PREC_FP64:  // b, r, pA, pB, q, rB, qB (rB, qB: second r, q of the one-kernel iteration)
      put(0, 8); put(1, 8); put(2, 8); put(3, 8); put(4, 8); put(5, 8); put(6, 8); break;
    case TBS_PREC_FP32:  // b, x, r, pA, pB, q, rB, qB (f32; rB, qB: second r, q of the one-kernel iteration)
      put(0, 4); put(1, 4); put(2, 4); put(3, 4); put(4, 4); put(5, 4); put(6, 4); put(7, 4); break;
    case TBS_PREC_MIXED:  // b64, r32, d, pA, pB, q, rB, qB
      put(0, 8); put(1, 4); put(2, 4); put(3, 4); put(4, 4); put(5, 4); put(6, 4); put(7, 4); break;
    case TBS_PREC_MIXED_BF16:  // b64, r32, d, pA(bf16), pB(bf16), q, rB, qB
      put(0, 8); put(1, 4); put(2, 4); put(3, 2); put(4, 2); put(5, 4); put(6, 4); put(7, 4); break;
  }
  if (prec >= 0 && c->coarse) {
    const size_t Nc = (size_t)(c->cgrid[0] * c->cgrid[1] * c->cgrid[2]);
    const size_t t1 = (size_t)(c->cgrid[0] * c->ny * c->nz), t2 = (size_t)(c->cgrid[0] * c->cgrid[1] * c->nz);
    const size_t sz[6] = {N * 8, t1 * 8, t2 * 8, Nc * 8, Nc * 8, tbs_workspace_bytes(c->coarse, TBS_PREC_FP64)};
    for (int i = 0; i < 6; ++i) { L.coff[i] = o; o += align256(sz[i]); }
  }
  L.bytes = o;
  return L;
}

static Scalars* scal(const tbs_ctx* c, int slot) { return (Scalars*)(c->ws + slot * 256); }
static double* part0(const tbs_ctx* c) { return (double*)(c->ws + 1024); }
static double* part1(const tbs_ctx* c) { return (double*)(c->ws + 1024 + align256((size_t)c->nparts * 8)); }
static double* part2(const tbs_ctx* c) { return (double*)(c->ws + 1024 + 2 * align256((size_t)c->nparts * 8)); }
static double* part3(const tbs_ctx* c) { return (double*)(c->ws + 1024 + 3 * align256((size_t)c->nparts * 8)); }

static StencilArgs base_args(const tbs_ctx* c) {
  StencilArgs a{};
  a.rscale = 1.0;
  a.nx = (int)c->nx; a.ny = (int)c->ny; a.nz = (int)c->nz; a.zc = c->zc;
  a.tiles_x = c->tiles_x; a.tiles_y = c->tiles_y; a.nchunks = c->nchunks; a.nblocks = c->nblocks;
  a.t = c->taps;
  if (c->ws) {
    a.part0 = part0(c);
    a.part1 = part1(c);
    a.part2 = part2(c);
    a.part3 = part3(c);
  }
  a.order = c->opts.tile_order;
  a.nt_store = c->opts.nt_store;
  if (c->bc == TBS_BC_ROBIN) a.rb = c->rb;
  return a;
}

extern "C" int tbs_setup(tbs_ctx** out, const int64_t grid[3], int degree, const double h[3], double tau, int bc,
                         void* hip_stream) {
  if (!out || !grid || !h) return set_err(TBS_E_INVAL, "null argument");
  *out = nullptr;
  if (degree < 1 || degree > 5) return set_err(TBS_E_INVAL, "degree %d not in 1..5", degree);
  if (bc != TBS_BC_PERIODIC && bc != TBS_BC_DIRICHLET) return set_err(TBS_E_INVAL, "bad boundary condition %d", bc);
  if (!(tau > 0.0) || !std::isfinite(tau)) return set_err(TBS_E_INVAL, "tau must be positive and finite");
  for (int d = 0; d < 3; ++d) {
    if (!(h[d] > 0.0) || !std::isfinite(h[d])) return set_err(TBS_E_INVAL, "h[%d] must be positive", d);
    if (grid[d] < 2 * degree + 1) return set_err(TBS_E_INVAL, "grid[%d]=%lld < 2n+1", d, (long long)grid[d]);
  }
  if (grid[0] * grid[1] > (int64_t)1 << 30 || grid[2] > (int64_t)1 << 30 ||
      grid[0] > (int64_t)1 << 24 || grid[1] > (int64_t)1 << 24)
    return set_err(TBS_E_INVAL, "grid too large");
  tbs_ctx* c = new (std::nothrow) tbs_ctx();
  if (!c) return set_err(TBS_E_INVAL, "out of host memory");
  c->nx = grid[0]; c->ny = grid[1]; c->nz = grid[2];
  c->N = grid[0] * grid[1] * grid[2];
  c->n = degree; c->bc = bc;
  for (int d = 0; d < 3; ++d) c->h[d] = h[d];
  c->tau = tau;
  c->st = (hipStream_t)hip_stream;
  make_taps(degree, c->taps.m, c->taps.s);
  for (int k = degree + 1; k < 6; ++k) c->taps.m[k] = c->taps.s[k] = 0.0;
  c->taps.ax = tau / (h[0] * h[0]);
  c->taps.ay = tau / (h[1] * h[1]);
  c->taps.az = tau / (h[2] * h[2]);
  c->taps.tau = tau;
  plan_geometry(c, 0);
  c->opts.inner_rtol = 1e-6;
  c->opts.inner_max_iter = 500;
  c->opts.max_sweeps = 12;
  c->opts.poll_every = 4;
  c->opts.zchunk = 0;
  c->opts.tile_order = 0;
  c->opts.nt_store = 0;
  c->opts.fused_cg = 1;
  c->opts.coarse_guess = 0;
  c->opts.coarse_rtol = 1e-2;
  c->opts.fused_rhs = 1;
  *out = c;
  return TBS_OK;
}

// Box domain with the Robin / penalty boundary branch (Sec. 2.2, Sec. 2.3): N_d = Nc_d + 1 + 2 floor(n/2)
// coefficients per axis; the stencil kernels run with truncated bands plus the corner blocks.
extern "C" int tbs_setup_robin(tbs_ctx** out, const int64_t grid[3], int degree, const double h[3], double tau,
                               double gamma, void* hip_stream) {
  if (!out || !grid || !h) return set_err(TBS_E_INVAL, "null argument");
  *out = nullptr;
  if (!(gamma > 0.0) || !std::isfinite(gamma)) return set_err(TBS_E_INVAL, "gamma must be positive and finite");
  if (degree < 1 || degree > 5) return set_err(TBS_E_INVAL, "degree %d not in 1..5", degree);
  const int z = 2 * (degree / 2) + 1;
  // the two corner zones and a band apart (the z-pass reuses its corner accumulators from the low end
  // to the high end), so no spline spans the box either
  const int64_t nmin = 2 * z + degree;
  for (int d = 0; d < 3; ++d)
    if (grid[d] < nmin) return set_err(TBS_E_INVAL, "grid[%d]=%lld < %lld for a Robin box of degree %d", d,
                                       (long long)grid[d], (long long)nmin, degree);
  int rc = tbs_setup(out, grid, degree, h, tau, TBS_BC_DIRICHLET, hip_stream);
  if (rc) return rc;
  tbs_ctx* c = *out;
  c->bc = TBS_BC_ROBIN;
  c->gamma = gamma;
  robin_corners(degree, h, tau, gamma, &c->rb);
  return TBS_OK;
}

// Transform context: the stencil kernels with half-width W = floor(degree / 2), mass taps replaced by
// the sampled B-spline b^degree(k) and no stiffness, so the operator is the evaluation filter
// E = Bx By Bz (Table 1 interpolation row; Sec. 2.3, Fig. figBspnSignProc).
extern "C" int tbs_transform_setup(tbs_ctx** out, const int64_t grid[3], int degree, int bc, void* hip_stream) {
  if (!out || !grid) return set_err(TBS_E_INVAL, "null argument");
  *out = nullptr;
  if (degree < 2 || degree > 5) return set_err(TBS_E_INVAL, "transform degree %d not in 2..5", degree);
  const int W = degree / 2;
  const double h1[3] = {1.0, 1.0, 1.0};
  int rc = tbs_setup(out, grid, W, h1, 1.0, bc, hip_stream);
  if (rc) return rc;
  tbs_ctx* c = *out;
  c->transform_degree = degree;
  for (int k = 0; k < 6; ++k) {
    c->taps.m[k] = k <= W ? bspline_val(degree, (double)k) : 0.0;
    c->taps.s[k] = 0.0;
  }
  c->taps.ax = c->taps.ay = c->taps.az = 0.0;
  c->taps.tau = 0.0;
  c->tau = 0.0;
  return TBS_OK;
}

extern "C" void tbs_destroy(tbs_ctx* c) {
  if (!c) return;
  if (c->coarse) tbs_destroy(c->coarse);
  if (c->host_scal) (void)hipHostFree(c->host_scal);
  for (auto& r : c->prof_pending) { (void)hipEventDestroy(r.e0); (void)hipEventDestroy(r.e1); }
  for (auto e : c->prof_pool) (void)hipEventDestroy(e);
  if (c->cost_ev_made)
    for (auto e : c->cost_ev) (void)hipEventDestroy(e);
  delete c;
}

// ------------------------------------------------------------------------------------------
// kernel timing: events around launches on the context stream

static hipEvent_t prof_event(tbs_ctx* c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Opens a record (kind, CG iteration index k or -1, algorithmic bytes); returns its slot or -1.
static int prof_begin(tbs_ctx* c, int kind, int k, double bytes) {
  if (!c->prof_on) return -1;
  tbs_ctx::ProfRec r{kind, k, bytes, prof_event(c), prof_event(c)};
  if (!r.e0 || !r.e1) return -1;
  (void)hipEventRecord(r.e0, c->st);
  c->prof_pending.push_back(r);
  return (int)c->prof_pending.size() - 1;
}

static void prof_end(tbs_ctx* c, int slot) {
  if (slot >= 0) (void)hipEventRecord(c->prof_pending[slot].e1, c->st);
}

// Accumulates finished records (the stream must have been synchronised).  CG records with an
// iteration index >= nit_limit belong to launches that found the solve converged: dropped.
static void prof_collect(tbs_ctx* c, int nit_limit) {
  for (auto& r : c->prof_pending) {
    if (!(r.k >= 0 && r.k >= nit_limit)) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
        c->prof_ms[r.kind] += ms;
        c->prof_bytes[r.kind] += r.bytes;
        c->prof_count[r.kind] += 1;
      }
    }
    c->prof_pool.push_back(r.e0);
    c->prof_pool.push_back(r.e1);
  }
  c->prof_pending.clear();
}

extern "C" int tbs_prof_enable(tbs_ctx* c, int on) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!c->prof_pending.empty()) {
    if (hipStreamSynchronize(c->st) != hipSuccess) return set_err(TBS_E_HIP, "stream sync failed");
    prof_collect(c, 1 << 30);
  }
  c->prof_on = on ? 1 : 0;
  for (int i = 0; i < TBS_PROF_KINDS; ++i) { c->prof_ms[i] = 0; c->prof_bytes[i] = 0; c->prof_count[i] = 0; }
  return TBS_OK;
}

extern "C" int tbs_prof_read(tbs_ctx* c, int kind, double* ms, double* bytes, int64_t* launches) {
  if (!c || kind < 0 || kind >= TBS_PROF_KINDS) return set_err(TBS_E_INVAL, "bad profiling kind");
  if (!c->prof_pending.empty()) {
    if (hipStreamSynchronize(c->st) != hipSuccess) return set_err(TBS_E_HIP, "stream sync failed");
    prof_collect(c, 1 << 30);
  }
  if (ms) *ms = c->prof_ms[kind];
  if (bytes) *bytes = c->prof_bytes[kind];
  if (launches) *launches = c->prof_count[kind];
  return TBS_OK;
}

extern "C" size_t tbs_workspace_bytes(const tbs_ctx* c, int prec) {
  if (!c || prec < -1 || prec > TBS_PREC_MIXED_BF16) return 0;
  return layout(c, prec).bytes;
}

extern "C" int tbs_bind_workspace(tbs_ctx* c, void* p, size_t bytes) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!aligned_ptr(p)) return set_err(TBS_E_INVAL, "workspace must be a 256-byte aligned device pointer");
  if (bytes < ws_head(c)) return set_err(TBS_E_NOMEM, "workspace smaller than the minimum %zu", ws_head(c));
  c->ws = (char*)p;
  c->ws_bytes = bytes;
  c->cg_active = 0;
  return TBS_OK;
}

extern "C" int tbs_taps(const tbs_ctx* c, double* m, double* s) {
  if (!c || !m || !s) return set_err(TBS_E_INVAL, "null argument");
  for (int k = 0; k <= c->n; ++k) { m[k] = c->taps.m[k]; s[k] = c->taps.s[k]; }
  return TBS_OK;
}

extern "C" int tbs_set_opts(tbs_ctx* c, const tbs_opts* o) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!o) {
    c->opts.inner_rtol = 1e-6; c->opts.inner_max_iter = 500; c->opts.max_sweeps = 12; c->opts.poll_every = 4;
    c->opts.zchunk = 0; c->opts.tile_order = 0; c->opts.nt_store = 0; c->opts.fused_cg = 1;
    c->opts.coarse_guess = 0; c->opts.coarse_rtol = 1e-2; c->opts.guess_backoff = 0; c->opts.guess_test = 0;
    c->opts.fused_rhs = 1;
  } else {
    if (!(o->inner_rtol > 0 && o->inner_rtol < 1) || o->inner_max_iter < 1 || o->max_sweeps < 1 ||
        o->poll_every < 0 || o->zchunk < 0 || o->tile_order < 0 || o->tile_order > 1 || o->nt_store < 0 ||
        o->nt_store > 1 || o->fused_cg < 0 || o->fused_cg > 1 || o->coarse_guess < 0 || o->coarse_guess > 1 ||
        !(o->coarse_rtol > 0 && o->coarse_rtol < 1) || o->guess_backoff < 0 || o->guess_backoff > 2 ||
        o->guess_test < 0 || o->guess_test > 1 || o->fused_rhs < 0 || o->fused_rhs > 1)
      return set_err(TBS_E_INVAL, "bad options");
    if (o->coarse_guess) {
      if (c->transform_degree) return set_err(TBS_E_INVAL, "coarse guess on a transform context");
      if (c->bc == TBS_BC_ROBIN) return set_err(TBS_E_INVAL, "coarse guess on a Robin box");
      if (c->n % 2 == 0) return set_err(TBS_E_INVAL, "coarse guess needs an odd degree (nested dyadic spaces)");
      const int64_t g[3] = {c->nx, c->ny, c->nz};
      for (int d = 0; d < 3; ++d) {
        if (c->bc == TBS_BC_PERIODIC && (g[d] & 1)) return set_err(TBS_E_INVAL, "periodic coarse guess needs even sizes");
        if (g[d] / 2 < 2 * c->n + 1) return set_err(TBS_E_INVAL, "coarse grid[%d] = %lld < 2n+1", d, (long long)(g[d] / 2));
      }
    }
    c->opts = *o;
  }
  c->guess_rejects = c->guess_wait = 0;
  if (c->opts.coarse_guess && !c->coarse) {
    const int64_t gc[3] = {c->nx / 2, c->ny / 2, c->nz / 2};
    const double hc[3] = {2.0 * c->h[0], 2.0 * c->h[1], 2.0 * c->h[2]};
    int rc = tbs_setup(&c->coarse, gc, c->n, hc, c->tau, c->bc, (void*)c->st);
    if (rc) return rc;
    for (int d = 0; d < 3; ++d) c->cgrid[d] = gc[d];
    c->ws = nullptr;  // the workspace grows by the coarse region: rebind
  } else if (!c->opts.coarse_guess && c->coarse) {
    tbs_destroy(c->coarse);
    c->coarse = nullptr;
  }
  // the partial-sum buffers are sized for the automatic geometry; a smaller chunk means more blocks
  const size_t old_head = ws_head(c);
  plan_geometry(c, c->opts.zchunk);
  if (c->ws && ws_head(c) > old_head) c->ws = nullptr;  // bound workspace no longer fits: rebind
  return TBS_OK;
}

static int need_ws(const tbs_ctx* c, int prec) {
  if (!c->ws) return set_err(TBS_E_NOMEM, "no workspace bound");
  const size_t need = layout(c, prec).bytes;
  if (c->ws_bytes < need) return set_err(TBS_E_NOMEM, "workspace %zu bytes < %zu needed", c->ws_bytes, need);
  return TBS_OK;
}

static int ensure_host_scal(tbs_ctx* c) {
  if (!c->host_scal) HIPCHK(hipHostMalloc((void**)&c->host_scal, sizeof(Scalars) * 2, hipHostMallocDefault));
  return TBS_OK;
}

static int read_scal(tbs_ctx* c, int slot, Scalars* outv) {
  int rc = ensure_host_scal(c);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(c->host_scal, scal(c, slot), sizeof(Scalars), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  *outv = *c->host_scal;
  return TBS_OK;
}

// ------------------------------------------------------------------------------------------
// operator entry points

extern "C" int tbs_apply(tbs_ctx* c, const void* u, int in_dt, void* y, int out_dt) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!aligned_ptr(u) || !aligned_ptr(y)) return set_err(TBS_E_INVAL, "u and y must be 256-byte aligned device pointers");
  if (u == y) return set_err(TBS_E_INVAL, "u and y must not alias");
  const bool ok = (in_dt == TBS_F64 && out_dt == TBS_F64) || (in_dt == TBS_F32 && out_dt == TBS_F32) ||
                  (in_dt == TBS_BF16 && out_dt == TBS_F32) || (in_dt == TBS_F32 && out_dt == TBS_F64) ||
                  (in_dt == TBS_BF16 && out_dt == TBS_F64);
  if (!ok) return set_err(TBS_E_INVAL, "unsupported dtype combination (%d -> %d)", in_dt, out_dt);
  StencilArgs a = base_args(c);
  a.in0 = u;
  a.out0 = y;
  const double esz[3] = {8, 4, 2};
  const int kind = (out_dt == TBS_F64 && in_dt == TBS_F64) ? 0 : (in_dt == TBS_F32 && out_dt == TBS_F32) ? 1
                 : (in_dt == TBS_BF16 && out_dt == TBS_F32) ? 2 : -1;
  const int ps = kind >= 0 ? prof_begin(c, kind, -1, (double)c->N * (esz[in_dt] + esz[out_dt])) : -1;
  HIPCHK(launch_apply(a, c->n, c->bc, in_dt, out_dt, c->st));
  prof_end(c, ps);
  return TBS_OK;
}

extern "C" int tbs_rhs(tbs_ctx* c, const void* u_prev, const void* q, void* b, int dt) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!aligned_ptr(u_prev) || !aligned_ptr(b) || (q && !aligned_ptr(q)))
    return set_err(TBS_E_INVAL, "arrays must be 256-byte aligned device pointers");
  if (b == u_prev || b == q) return set_err(TBS_E_INVAL, "b must not alias the inputs");
  if (dt != TBS_F64 && dt != TBS_F32) return set_err(TBS_E_INVAL, "rhs dtype must be F64 or F32");
  StencilArgs a = base_args(c);
  a.in0 = u_prev;
  a.in1 = q;
  a.out0 = b;
  const double e = dt == TBS_F64 ? 8 : 4;
  const int ps = prof_begin(c, dt == TBS_F64 ? 3 : 4, -1, (double)c->N * e * (q ? 3 : 2));
  HIPCHK(launch_rhs(a, c->n, c->bc, dt, c->st));
  prof_end(c, ps);
  return TBS_OK;
}

// Variable-coefficient operator (Sec. 2.3 coefficient expansion, Sec. 2.4 three-index kernels):
// cell-wise Gauss quadrature tables and the strip geometry of the sum-factorised kernel.
extern "C" int tbs_apply_varcoef(tbs_ctx* c, const void* u, const void* d, const void* m, void* y, int dt) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (c->transform_degree || c->bc == TBS_BC_ROBIN)
    return set_err(TBS_E_STATE, "the variable-coefficient operator needs a periodic or Dirichlet solver context");
  if (!aligned_ptr(u) || !aligned_ptr(d) || !aligned_ptr(m) || !aligned_ptr(y))
    return set_err(TBS_E_INVAL, "arrays must be 256-byte aligned device pointers");
  if (y == u || y == d || y == m) return set_err(TBS_E_INVAL, "y must not alias the inputs");
  if (dt != TBS_F64 && dt != TBS_F32) return set_err(TBS_E_INVAL, "varcoef dtype must be F64 or F32");
  const int n = c->n, Q = (3 * n + 2) / 2;
  VarcoefArgs a{};
  a.nx = (int)c->nx; a.ny = (int)c->ny; a.nz = (int)c->nz;
  a.tiles_x = (int)((c->nx + vc_tile_x(n) - 1) / vc_tile_x(n));
  a.tiles_y = (int)((c->ny + kVcTileY - 1) / kVcTileY);
  // about 16384 single-wave workgroups, z-chunks of at least 16 planes
  const int64_t strips = (int64_t)a.tiles_x * a.tiles_y;
  int64_t chunks = std::min<int64_t>((16384 + strips - 1) / strips, std::max<int64_t>(1, c->nz / 16));
  a.zc = (int)((c->nz + chunks - 1) / chunks);
  a.nchunks = (int)((c->nz + a.zc - 1) / a.zc);
  a.nblocks = a.tiles_x * a.tiles_y * a.nchunks;
  a.c = u; a.d = d; a.m = m; a.y = y;
  double gx[kVcMaxQ], gw[kVcMaxQ];
  gauss_legendre(Q, gx, gw);
  for (int q = 0; q < Q; ++q) {
    const double sq = 0.5 * (1.0 + gx[q]);  // Gauss point in the unit cell
    a.w[q] = 0.5 * gw[q];
    for (int t = 0; t <= n; ++t) {
      const double x = sq + 0.5 * (n - 1) - t;  // distance from the t-th B-spline's centre
      a.bv[q * kVcMaxB + t] = bspline_val(n, x);
      a.bd[q * kVcMaxB + t] = bspline_der(n, x);
    }
  }
  a.ihx2 = 1.0 / (c->h[0] * c->h[0]);
  a.ihy2 = 1.0 / (c->h[1] * c->h[1]);
  a.ihz2 = 1.0 / (c->h[2] * c->h[2]);
  const double esz = dt == TBS_F64 ? 8 : 4;
  const int ps = prof_begin(c, dt == TBS_F64 ? 13 : 14, -1, (double)c->N * 4 * esz);
  HIPCHK(launch_varcoef(a, n, c->bc, dt == TBS_F64 ? 0 : 1, c->st));
  prof_end(c, ps);
  return TBS_OK;
}

// b = M u (FP64) and r = b - A u (FP32) in one pass (source-free step, no Robin), norms to scal slot
static int rhs_resid_async(tbs_ctx* c, const double* u, double* b, void* r, int slot) {
  StencilArgs a = base_args(c);
  a.in0 = u;
  a.out1 = b;
  a.out0 = r;
  const int ps = prof_begin(c, 16, -1, (double)c->N * (8 + 8 + 4));
  HIPCHK(launch_rhs_resid(a, c->n, c->bc, c->st));
  prof_end(c, ps);
  HIPCHK(launch_finalize(FIN_NORMS, part0(c), part1(c), stencil_blocks(a, M_RHSRES, 8, c->n, c->bc), scal(c, slot), 0.0,
                         c->st));
  return TBS_OK;
}

// r = (b - A x) rscale (FP64), its norms to scal slot; r written if r != NULL (r_dt F64/F32)
static int resid_async(tbs_ctx* c, const double* x, const double* b, void* r, int r_dt, int slot, int fin_op,
                       double rtol, double rscale = 1.0) {
  StencilArgs a = base_args(c);
  a.rscale = rscale;
  a.in0 = x;
  a.bvec = b;
  a.out0 = r;
  const int ps = prof_begin(c, 8, -1, (double)c->N * (16 + (r ? (r_dt == TBS_F32 ? 4 : 8) : 0)));
  HIPCHK(launch_resid(a, c->n, c->bc, r_dt == TBS_F32 ? 1 : 0, c->st));
  prof_end(c, ps);
  HIPCHK(launch_finalize(fin_op, part0(c), part1(c), stencil_blocks(a, M_RESID, 8, c->n, c->bc), scal(c, slot), rtol, c->st));
  return TBS_OK;
}

extern "C" int tbs_residual(tbs_ctx* c, const double* x, const double* b, void* r, int r_dt, double* rnorm,
                            double* bnorm) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!aligned_ptr(x) || !aligned_ptr(b) || (r && !aligned_ptr(r)))
    return set_err(TBS_E_INVAL, "arrays must be 256-byte aligned device pointers");
  if (r && (r == (void*)x || r == (void*)b)) return set_err(TBS_E_INVAL, "r must not alias x or b");
  if (r && r_dt != TBS_F64 && r_dt != TBS_F32) return set_err(TBS_E_INVAL, "r dtype must be F64 or F32");
  int rc = need_ws(c, -1);
  if (rc) return rc;
  rc = resid_async(c, x, b, r, r_dt, SC_AUX, FIN_NORMS, 0.0);
  if (rc) return rc;
  Scalars s;
  rc = read_scal(c, SC_AUX, &s);
  if (rc) return rc;
  if (rnorm) *rnorm = std::sqrt(s.out);
  if (bnorm) *bnorm = std::sqrt(s.out2);
  return TBS_OK;
}

// ------------------------------------------------------------------------------------------
// allocation-free residual: the per-workgroup partial sums and the reduction scalars live in a
// library-owned static device array instead of the bound workspace

constexpr int kNoAllocMaxBlocks = TBS_NOALLOC_MAX_BLOCKS;
constexpr size_t kScratchBytes = 256 + 2 * (size_t)kNoAllocMaxBlocks * sizeof(double);  // Scalars, part0, part1
constexpr int kMaxDevices = 64;

// Host code never passes this name to a kernel: it is a host-side stand-in; the device address
// of each GPU's copy comes from hipGetSymbolAddress (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
static int scratch_ptr(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_err(TBS_E_INVAL, "device index %d not below %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_err(TBS_E_HIP, "hipGetSymbolAddress returned a null address");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return TBS_OK;
}

extern "C" int tbs_residual_noalloc(tbs_ctx* c, const double* x, const double* b, void* r, int r_dt, double* norms) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!aligned_ptr(x) || !aligned_ptr(b) || (r && !aligned_ptr(r)))
    return set_err(TBS_E_INVAL, "arrays must be 256-byte aligned device pointers");
  if (!norms || ((uintptr_t)norms & 7u)) return set_err(TBS_E_INVAL, "norms must be an 8-byte aligned device pointer");
  if (r && (r == (void*)x || r == (void*)b)) return set_err(TBS_E_INVAL, "r must not alias x or b");
  if ((void*)norms == (void*)x || (void*)norms == (void*)b || (r && (void*)norms == r))
    return set_err(TBS_E_INVAL, "norms must not alias the arrays");
  if (r && r_dt != TBS_F64 && r_dt != TBS_F32) return set_err(TBS_E_INVAL, "r dtype must be F64 or F32");
  StencilArgs a = base_args(c);
  const int nb = stencil_blocks(a, M_RESID, 8, c->n, c->bc);
  if (nb > kNoAllocMaxBlocks)
    return set_err(TBS_E_INVAL, "residual launch needs %d workgroups, the static buffer holds %d", nb, kNoAllocMaxBlocks);
  if (c->st) {
    int sdev = -1, cur = -1;
    HIPCHK(hipStreamGetDevice(c->st, &sdev));
    HIPCHK(hipGetDevice(&cur));
    if (sdev != cur) return set_err(TBS_E_INVAL, "the context's stream is on device %d, device %d is current", sdev, cur);
  }
  void* sp = nullptr;
  int rc = scratch_ptr(&sp);
  if (rc) return rc;
  Scalars* sc = (Scalars*)sp;
  double* p0 = (double*)((char*)sp + 256);
  double* p1 = p0 + kNoAllocMaxBlocks;
  a.in0 = x;
  a.bvec = b;
  a.out0 = r;
  a.part0 = p0;
  a.part1 = p1;
  a.part2 = a.part3 = nullptr;
  HIPCHK(launch_resid(a, c->n, c->bc, r_dt == TBS_F32 ? 1 : 0, c->st));
  HIPCHK(launch_finalize(FIN_NORMS, p0, p1, nb, sc, 0.0, c->st));
  HIPCHK(launch_norms_out(sc, norms, c->st));
  return TBS_OK;
}

extern "C" int tbs_dot(tbs_ctx* c, const void* a, const void* b, int dt, double* out) {
  if (!c || !out) return set_err(TBS_E_INVAL, "null argument");
  if (!aligned_ptr(a) || !aligned_ptr(b)) return set_err(TBS_E_INVAL, "arrays must be 256-byte aligned device pointers");
  if (dt != TBS_F64 && dt != TBS_F32) return set_err(TBS_E_INVAL, "dot dtype must be F64 or F32");
  int rc = need_ws(c, -1);
  if (rc) return rc;
  HIPCHK(launch_dot(a, b, c->N, dt, part0(c), c->st));
  HIPCHK(launch_finalize(FIN_DOT, part0(c), nullptr, kVecBlocks, scal(c, SC_AUX), 0.0, c->st));
  Scalars s;
  rc = read_scal(c, SC_AUX, &s);
  if (rc) return rc;
  *out = s.out;
  return TBS_OK;
}

extern "C" int tbs_stream_copy(tbs_ctx* c, const void* src, void* dst, size_t bytes) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!aligned_ptr(src) || !aligned_ptr(dst)) return set_err(TBS_E_INVAL, "arrays must be 256-byte aligned device pointers");
  if (src == dst) return set_err(TBS_E_INVAL, "src and dst must differ");
  const char* s = (const char*)src;
  const char* d = (const char*)dst;
  if (s < d + bytes && d < s + bytes) return set_err(TBS_E_INVAL, "src and dst overlap");
  HIPCHK(launch_stream_copy(src, dst, (int64_t)bytes, c->st));
  return TBS_OK;
}

extern "C" int tbs_convert(tbs_ctx* c, const void* src, int sdt, void* dst, int ddt) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!aligned_ptr(src) || !aligned_ptr(dst)) return set_err(TBS_E_INVAL, "arrays must be 256-byte aligned device pointers");
  if (sdt < 0 || sdt > 2 || ddt < 0 || ddt > 2 || sdt == ddt) return set_err(TBS_E_INVAL, "bad conversion");
  HIPCHK(launch_convert(src, sdt, dst, ddt, c->N, c->st));
  return TBS_OK;
}

// ------------------------------------------------------------------------------------------
// CG core.  dt: 0 f64, 1 f32, 2 f32 with p in bf16.  Arrays: x (iterate), r, pA, pB, q.

struct CgArrays {
  void* x;
  void* r;
  void* p[2];
  void* q;
  void* r2;  // one-kernel iteration: r and q alternate between (r, r2) and (q, q2)
  void* q2;
};

static int cg1_async(tbs_ctx* c, const CgArrays& A, int dt, int k) {
  StencilArgs a = base_args(c);
  a.in0 = A.r;
  a.in1 = A.p[k & 1];
  a.out1 = A.p[(k + 1) & 1];
  a.out0 = A.q;
  a.io0 = A.x;
  a.scal = scal(c, SC_CG);
  a.first = (k == 0);
  const double tc = dt == 0 ? 8 : 4, tp = dt == 0 ? 8 : (dt == 1 ? 4 : 2);
  // first iteration: read r, write p and q; later: read r, p_old, x, write p, q, x
  const double b1 = (double)c->N * (k == 0 ? (2 * tc + tp) : (4 * tc + 2 * tp));
  int ps = prof_begin(c, 5 + dt, k, b1);
  HIPCHK(launch_cg1(a, c->n, c->bc, dt, c->st));
  prof_end(c, ps);
  HIPCHK(launch_finalize(FIN_ALPHA, part0(c), nullptr, stencil_blocks(a, M_CG1, dt == 0 ? 8 : 4, c->n, c->bc), scal(c, SC_CG),
                         0.0, c->st));
  ps = prof_begin(c, dt == 0 ? 9 : 10, k, (double)c->N * 3 * tc);
  HIPCHK(launch_cg2(A.r, A.q, c->N, dt == 0 ? 0 : 1, part0(c), scal(c, SC_CG), c->st));
  prof_end(c, ps);
  HIPCHK(launch_finalize(FIN_BETA, part0(c), nullptr, kVecBlocks, scal(c, SC_CG), 0.0, c->st));
  return TBS_OK;
}

// One-kernel CG iteration k (dt 0: FP64, 1: FP32, 2: FP32 with bf16 p): r_k = r_{k-1} - alpha q_{k-1}, p_k = r_k + beta p_{k-1},
// q_k = A p_k and the FP64 partial sums of p.q, r.q, q.q and r.r in one stencil launch, then one
// reduction; every second iteration also x += alpha2 p_{k-2} + alpha p_{k-1} (the two pending
// updates).  r, p and q alternate between two arrays (halo reads of the old values and writes of
// the new ones overlap in one launch).
static int cgf_async(tbs_ctx* c, const CgArrays& A, int dt, int k) {
  StencilArgs a = base_args(c);
  void* R[2] = {A.r, A.r2};
  void* Q[2] = {A.q, A.q2};
  a.in0 = R[k & 1];
  a.in1 = A.p[k & 1];
  a.in2 = Q[k & 1];
  a.out0 = Q[(k + 1) & 1];
  a.out1 = A.p[(k + 1) & 1];
  a.out2 = R[(k + 1) & 1];
  a.io0 = A.x;
  a.scal = scal(c, SC_CG);
  a.first = (k == 0);
  const double tc = dt == 0 ? 8 : 4, tp = dt == 0 ? 8 : (dt == 1 ? 4 : 2);
  // first iteration: read r, write r, p, q; later: read r, q, p_old, write r, p, q, and on the
  // iterations that advance x also read x, p_{k-2} and write x
  const int pend = k == 0 ? 0 : c->cgf_pend;
  // (the first x update of the refinement's inner solve does not read x = 0)
  const double xr = (pend == 2 && c->cgf_xzero) ? 0 : tc;
  const double b1 = (double)c->N * (k == 0 ? 3 * tc + tp : (pend == 2 ? 5 * tc + xr + 3 * tp : 2 * (2 * tc + tp)));
  c->cgf_pend = (pend == 2 ? 0 : pend) + 1;
  if (pend == 2) c->cgf_xzero = false;
  int ps = prof_begin(c, dt == 0 ? 15 : (dt == 1 ? 11 : 12), k, b1);
  HIPCHK(launch_cgf(a, c->n, c->bc, dt, c->st));
  prof_end(c, ps);
  HIPCHK(launch_finalize(FIN_FUSED, part0(c), part1(c), stencil_blocks(a, M_CGF, (int)tc, c->n, c->bc), scal(c, SC_CG),
                         0.0, c->st, part2(c), part3(c)));
  return TBS_OK;
}

// Runs CG iterations k = k0 .. until done / max_iter, then flushes the pending x update (unless
// keep_pending: the caller then applies it, e.g. with launch_refine_add, and clears the flag).
// Returns TBS_OK, TBS_W_NOT_CONVERGED or TBS_E_BREAKDOWN; *nit receives the completed count.
// nopoll: every iteration up to max_iter is enqueued without a host poll (the kernels of a solve
// that has converged return at once), nothing waits on the host, and *nit receives max_iter.
static int cg_loop(tbs_ctx* c, const CgArrays& A, int dt, int k0, int max_iter, int* nit, bool keep_pending = false,
                   bool nopoll = false) {
  int k = k0, rc;
  if (nopoll) {
    for (; k < max_iter; ++k) {
      rc = c->opts.fused_cg ? cgf_async(c, A, dt, k) : cg1_async(c, A, dt, k);
      if (rc) return rc;
    }
    if (!keep_pending) {
      HIPCHK(launch_flush(A.x, A.p[0], A.p[1], c->N, dt, scal(c, SC_CG), c->st));
      HIPCHK(launch_finalize(FIN_CLEAR_PENDING, nullptr, nullptr, 0, scal(c, SC_CG), 0.0, c->st));
      c->cgf_pend = 0;
    }
    *nit = k;
    return TBS_OK;
  }
  Scalars s;
  rc = read_scal(c, SC_CG, &s);
  if (rc) return rc;
  const int poll = c->opts.poll_every > 0 ? c->opts.poll_every : 4;
  while (!s.done && k < max_iter) {
    const int batch = std::min(poll, max_iter - k);
    for (int i = 0; i < batch; ++i) {
      rc = c->opts.fused_cg ? cgf_async(c, A, dt, k++) : cg1_async(c, A, dt, k++);
      if (rc) return rc;
    }
    rc = read_scal(c, SC_CG, &s);
    if (rc) return rc;
    k = s.nit;
    prof_collect(c, s.nit);
  }
  if (!keep_pending) {
    HIPCHK(launch_flush(A.x, A.p[0], A.p[1], c->N, dt, scal(c, SC_CG), c->st));
    HIPCHK(launch_finalize(FIN_CLEAR_PENDING, nullptr, nullptr, 0, scal(c, SC_CG), 0.0, c->st));
    c->cgf_pend = 0;
  }
  *nit = s.nit;
  if (s.status == TBS_E_BREAKDOWN) return set_err(TBS_E_BREAKDOWN, "CG breakdown after %d iterations", s.nit);
  return s.done ? TBS_OK : TBS_W_NOT_CONVERGED;
}

// r = b - A x and CG scalars for dt 0 (FP64, via the residual kernel) or 1/2 (FP32 apply + sub)
static int cg_init_async(tbs_ctx* c, const void* b, const CgArrays& A, int dt, double rtol) {
  if (dt == 0) return resid_async(c, (const double*)A.x, (const double*)b, A.r, TBS_F64, SC_CG, FIN_INIT, rtol);
  // FP32: q = A x, then r = b - q with the partial sums of r.r and b.b
  StencilArgs a = base_args(c);
  a.in0 = A.x;
  a.out0 = A.q;
  HIPCHK(launch_apply(a, c->n, c->bc, 1, 1, c->st));
  HIPCHK(launch_sub_norm(A.r, b, A.q, c->N, 1, part0(c), part1(c), c->st));
  HIPCHK(launch_finalize(FIN_INIT, part0(c), part1(c), kVecBlocks, scal(c, SC_CG), rtol, c->st));
  return TBS_OK;
}

extern "C" int tbs_cg_begin(tbs_ctx* c, const void* b, void* x, int dt, double rtol) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!aligned_ptr(b) || !aligned_ptr(x)) return set_err(TBS_E_INVAL, "arrays must be 256-byte aligned device pointers");
  if (b == x) return set_err(TBS_E_INVAL, "b and x must not alias");
  if (dt != TBS_F64 && dt != TBS_F32) return set_err(TBS_E_INVAL, "CG dtype must be F64 or F32");
  if (!(rtol >= 0.0)) return set_err(TBS_E_INVAL, "rtol must be >= 0");
  const int prec = dt == TBS_F64 ? TBS_PREC_FP64 : TBS_PREC_FP32;
  int rc = need_ws(c, prec);
  if (rc) return rc;
  const Layout L = layout(c, prec);
  CgArrays A;
  A.x = x;
  A.r2 = A.q2 = nullptr;
  if (dt == TBS_F64) {
    A.r = c->ws + L.off[1]; A.p[0] = c->ws + L.off[2]; A.p[1] = c->ws + L.off[3]; A.q = c->ws + L.off[4];
    A.r2 = c->ws + L.off[5]; A.q2 = c->ws + L.off[6];
  } else {
    A.r = c->ws + L.off[2]; A.p[0] = c->ws + L.off[3]; A.p[1] = c->ws + L.off[4]; A.q = c->ws + L.off[5];
    A.r2 = c->ws + L.off[6]; A.q2 = c->ws + L.off[7];
  }
  rc = cg_init_async(c, b, A, dt == TBS_F64 ? 0 : 1, rtol);
  if (rc) return rc;
  c->cg_active = 1;
  c->cg_dt = dt;
  c->cg_enq = 0;
  c->cg_x = x;
  return TBS_OK;
}

extern "C" int tbs_cg_step(tbs_ctx* c, int n_iters, double* rel_res_out, int* iters_out) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!c->cg_active) return set_err(TBS_E_STATE, "tbs_cg_step before tbs_cg_begin");
  if (n_iters < 0) return set_err(TBS_E_INVAL, "n_iters must be >= 0");
  const int prec = c->cg_dt == TBS_F64 ? TBS_PREC_FP64 : TBS_PREC_FP32;
  int rc = need_ws(c, prec);
  if (rc) return rc;
  const Layout L = layout(c, prec);
  CgArrays A;
  A.x = c->cg_x;
  A.r2 = A.q2 = nullptr;
  if (c->cg_dt == TBS_F64) {
    A.r = c->ws + L.off[1]; A.p[0] = c->ws + L.off[2]; A.p[1] = c->ws + L.off[3]; A.q = c->ws + L.off[4];
    A.r2 = c->ws + L.off[5]; A.q2 = c->ws + L.off[6];
  } else {
    A.r = c->ws + L.off[2]; A.p[0] = c->ws + L.off[3]; A.p[1] = c->ws + L.off[4]; A.q = c->ws + L.off[5];
    A.r2 = c->ws + L.off[6]; A.q2 = c->ws + L.off[7];
  }
  int nit = 0;
  rc = cg_loop(c, A, c->cg_dt == TBS_F64 ? 0 : 1, c->cg_enq, c->cg_enq + n_iters, &nit, false,
               c->opts.poll_every == 0);
  c->cg_enq = nit;
  if (rc < 0) return rc;
  if (rel_res_out || iters_out) {
    Scalars s;
    int rc2 = read_scal(c, SC_CG, &s);
    if (rc2) return rc2;
    if (rel_res_out) *rel_res_out = s.bb > 0 ? std::sqrt(s.rr / s.bb) : 0.0;
    if (iters_out) *iters_out = s.nit;
  }
  return rc == TBS_W_NOT_CONVERGED ? TBS_OK : rc;
}

// ------------------------------------------------------------------------------------------
// B-spline transforms on a transform context

extern "C" int tbs_transform_eval(tbs_ctx* c, const void* coef, void* samples, int dt) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!c->transform_degree) return set_err(TBS_E_STATE, "not a transform context");
  if (!coef) return set_err(TBS_E_INVAL, "null coefficients");
  return tbs_rhs(c, coef, nullptr, samples, dt);  // E coef: the mass-only stencil with the evaluation taps
}

static int fp64_relres(tbs_ctx* c, const double* x, const double* b, double* rel);

extern "C" int tbs_transform_interp(tbs_ctx* c, const double* samples, double* coef, double rtol, int max_iter,
                                    int* iters, double* rel_res) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!c->transform_degree) return set_err(TBS_E_STATE, "not a transform context");
  if (!aligned_ptr(samples) || !aligned_ptr(coef)) return set_err(TBS_E_INVAL, "arrays must be 256-byte aligned device pointers");
  if (samples == coef) return set_err(TBS_E_INVAL, "samples and coef must not alias");
  if (!(rtol >= 0.0) || max_iter < 0) return set_err(TBS_E_INVAL, "bad rtol / max_iter");
  int rc = need_ws(c, TBS_PREC_FP64);
  if (rc) return rc;
  c->cg_active = 0;
  const Layout L = layout(c, TBS_PREC_FP64);
  CgArrays A{coef, c->ws + L.off[1], {c->ws + L.off[2], c->ws + L.off[3]}, c->ws + L.off[4], c->ws + L.off[5],
             c->ws + L.off[6]};
  rc = cg_init_async(c, samples, A, 0, rtol);
  if (rc) return rc;
  int nit = 0;
  const int result = cg_loop(c, A, 0, 0, max_iter, &nit);
  if (result < 0 && result != TBS_E_BREAKDOWN) return result;
  double rel = 0.0;
  rc = fp64_relres(c, coef, samples, &rel);
  if (rc) return rc;
  if (iters) *iters = nit;
  if (rel_res) *rel_res = rel;
  return result;
}

// ------------------------------------------------------------------------------------------
// implicit time step

static int copy_async(tbs_ctx* c, void* dst, const void* src, size_t bytes) {
  HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->st));
  return TBS_OK;
}

static int fp64_relres(tbs_ctx* c, const double* x, const double* b, double* rel) {
  int rc = resid_async(c, x, b, nullptr, TBS_F64, SC_AUX, FIN_NORMS, 0.0);
  if (rc) return rc;
  Scalars s;
  rc = read_scal(c, SC_AUX, &s);
  if (rc) return rc;
  *rel = s.out2 > 0 ? std::sqrt(s.out / s.out2) : std::sqrt(s.out);
  return TBS_OK;
}

// guess_backoff 2: adds the time since cost_ev[2] (recorded before a CG loop) to *ms
static int cost_lap(tbs_ctx* c, double* ms) {
  HIPCHK(hipEventRecord(c->cost_ev[3], c->st));
  HIPCHK(hipEventSynchronize(c->cost_ev[3]));
  float t = 0.f;
  HIPCHK(hipEventElapsedTime(&t, c->cost_ev[2], c->cost_ev[3]));
  *ms += t;
  return TBS_OK;
}

extern "C" int tbs_timestep(tbs_ctx* c, const double* u_prev, const double* q, double* u_next, int prec, double rtol,
                            int max_iter, tbs_net* net, tbs_stats* stats) {
  if (!c) return set_err(TBS_E_INVAL, "null context");
  if (!aligned_ptr(u_prev) || !aligned_ptr(u_next) || (q && !aligned_ptr(q)))
    return set_err(TBS_E_INVAL, "arrays must be 256-byte aligned device pointers");
  if (u_next == u_prev || u_next == q) return set_err(TBS_E_INVAL, "u_next must not alias the inputs");
  if (prec < TBS_PREC_FP64 || prec > TBS_PREC_MIXED_BF16) return set_err(TBS_E_INVAL, "bad precision mode");
  if (c->transform_degree) return set_err(TBS_E_STATE, "tbs_timestep on a transform context");
  if (!(rtol >= 0.0) || max_iter < 0) return set_err(TBS_E_INVAL, "bad rtol / max_iter");
  int rc = need_ws(c, prec);
  if (rc) return rc;
  c->cg_active = 0;
  const Layout L = layout(c, prec);
  const size_t N = (size_t)c->N;
  tbs_stats st{};
  st.rel_res_learned = NAN;
  st.rel_res_coarse = NAN;

  // the network is run unless the backoff policy is waiting out an earlier rejection
  tbs_net* g = (prec != TBS_PREC_FP32) ? net : nullptr;
  if (g && c->opts.guess_backoff && c->guess_wait > 0) {
    --c->guess_wait;
    g = nullptr;
    st.skipped_learned_guess = 1;
  }

  // refined path: the plain guess's residual (FP32 copy, norms and partial sums) is the first
  // refinement sweep's residual whenever the plain guess is kept, so it is computed last and reused
  bool have_res0 = false;
  Scalars res0{};
  // right-hand side, FP64 except for the raw FP32 path (which builds its FP64 b after the solve).
  // A source-free refined step that starts from the plain guess forms b = M u and the first
  // sweep's residual b - A u in one pass over u (the same b, bit for bit, as the rhs kernel's)
  double* b64 = (prec == TBS_PREC_FP32) ? nullptr : (double*)(c->ws + L.off[0]);
  if (prec != TBS_PREC_FP32) {
    const bool refined_path = (prec == TBS_PREC_MIXED || prec == TBS_PREC_MIXED_BF16);
    const bool fused_rhs = refined_path && !q && !g && c->bc != TBS_BC_ROBIN && c->opts.fused_rhs &&
                           !(c->coarse && c->opts.coarse_guess);
    if (fused_rhs) {
      rc = rhs_resid_async(c, u_prev, b64, c->ws + L.off[1], SC_AUX);
      if (rc) return rc;
      rc = read_scal(c, SC_AUX, &res0);
      if (rc) return rc;
      have_res0 = true;
    } else {
      rc = tbs_rhs(c, u_prev, q, b64, TBS_F64);
      if (rc) return rc;
    }
  }
  // cost-aware backoff: events around the network and its test, and around the rest of the step
  const bool costed = g && c->opts.guess_backoff == 2;
  if (costed) {
    if (!c->cost_ev_made) {
      int made = 0;
      while (made < 4 && hipEventCreate(&c->cost_ev[made]) == hipSuccess) ++made;
      if (made < 4) {
        while (made > 0) (void)hipEventDestroy(c->cost_ev[--made]);
        return set_err(TBS_E_HIP, "hipEventCreate failed");
      }
      c->cost_ev_made = true;
    }
    HIPCHK(hipEventRecord(c->cost_ev[0], c->st));
  }
  double t_cg = 0.0;  // guess_backoff 2: time of this step's CG loops (ms)

  // initial guess: plain u^k, or the network guess if its FP64 residual is smaller.  The current
  // iterate is u_next once have_x is set, else u_prev itself: u_next is only written when a guess
  // is formed there, when a path needs it in place, or by the first refinement correction
  // (u_next = u_prev + d), which saves a full FP64 copy per step.
  bool have_x = false;
  auto ensure_x = [&]() -> int {
    if (have_x) return TBS_OK;
    have_x = true;
    return copy_async(c, u_next, u_prev, N * 8);
  };
  if (g) {
    const float* du = nullptr;
    const int64_t grid[3] = {c->nx, c->ny, c->nz};
    rc = tbs_net_guess_internal(g, grid, c->bc == TBS_BC_PERIODIC, c->tau, c->st, u_prev, q, &du);
    if (rc) return rc;
    const bool refined = (prec == TBS_PREC_MIXED || prec == TBS_PREC_MIXED_BF16);
    if (c->opts.guess_test == 1) {
      // energy test: r0 = b - A u^k (FP64 kernel, kept as FP32 in the first sweep's residual array),
      // A du in FP32, gamma = r0.du / du.A du minimises ||x* - (u^k + gamma du)||_A, and the A-norm of
      // the error drops by 2 gamma r0.du - gamma^2 du.A du (= (r0.du)^2 / du.A du)
      float* r0 = (float*)(c->ws + L.off[1]);
      float* adu = (float*)(c->ws + L.off[refined ? 5 : 4]);
      rc = resid_async(c, u_prev, b64, r0, TBS_F32, SC_AUX, FIN_NORMS, 0.0);
      if (rc) return rc;
      StencilArgs a = base_args(c);
      a.in0 = du;
      a.out0 = adu;
      HIPCHK(launch_apply(a, c->n, c->bc, 1, 1, c->st));
      HIPCHK(launch_dot(r0, du, c->N, 1, part0(c), c->st));
      HIPCHK(launch_finalize(FIN_DOT, part0(c), nullptr, kVecBlocks, scal(c, 2), 0.0, c->st));
      HIPCHK(launch_dot(du, adu, c->N, 1, part0(c), c->st));
      HIPCHK(launch_finalize(FIN_DOT, part0(c), nullptr, kVecBlocks, scal(c, 3), 0.0, c->st));
      Scalars d1, d2;
      rc = read_scal(c, SC_AUX, &res0);
      if (!rc) rc = read_scal(c, 2, &d1);
      if (!rc) rc = read_scal(c, 3, &d2);
      if (rc) return rc;
      st.rel_res_plain = res0.out2 > 0 ? std::sqrt(res0.out / res0.out2) : std::sqrt(res0.out);
      const double gam = (d2.out > 0.0 && std::isfinite(d1.out / d2.out)) ? d1.out / d2.out : 0.0;
      const double drop = 2.0 * gam * d1.out - gam * gam * d2.out;
      st.learned_gamma = gam;
      if (drop > 0.0 && std::isfinite(drop)) {
        HIPCHK(launch_guess_combine(u_next, u_prev, du, c->N, gam, c->st));
        have_x = true;
        st.used_learned_guess = 1;
      } else {
        have_res0 = refined;  // r0 and its norms are the first sweep's residual
      }
    } else {
      // residual test: u^k + du is kept if its FP64 residual is smaller than that of u^k
      HIPCHK(launch_guess_combine(u_next, u_prev, du, c->N, 1.0, c->st));
      have_x = true;
      st.learned_gamma = 1.0;
      rc = fp64_relres(c, u_next, b64, &st.rel_res_learned);
      if (rc) return rc;
      if (refined) {
        rc = resid_async(c, u_prev, b64, c->ws + L.off[1], TBS_F32, SC_AUX, FIN_NORMS, 0.0);
        if (rc) return rc;
        rc = read_scal(c, SC_AUX, &res0);
        if (rc) return rc;
        st.rel_res_plain = res0.out2 > 0 ? std::sqrt(res0.out / res0.out2) : std::sqrt(res0.out);
      } else {
        rc = fp64_relres(c, u_prev, b64, &st.rel_res_plain);
        if (rc) return rc;
      }
      if (st.rel_res_learned < st.rel_res_plain) {
        st.used_learned_guess = 1;
      } else {
        have_x = false;  // back to the plain guess u_prev
        have_res0 = refined;
      }
    }
  }
  if (costed) HIPCHK(hipEventRecord(c->cost_ev[1], c->st));

  if (!g && c->coarse && c->opts.coarse_guess && prec != TBS_PREC_FP32) {
    // coarse-grid guess: u_next = u_prev + P d, A_c d = P^T (b - A u_prev) / 8
    double* r0 = (double*)(c->ws + L.coff[0]);
    double* t1 = (double*)(c->ws + L.coff[1]);
    double* t2 = (double*)(c->ws + L.coff[2]);
    double* bcv = (double*)(c->ws + L.coff[3]);
    double* xc = (double*)(c->ws + L.coff[4]);
    tbs_ctx* cc = c->coarse;
    const int per = c->bc == TBS_BC_PERIODIC;
    rc = resid_async(c, u_prev, b64, r0, TBS_F64, SC_AUX, FIN_NORMS, 0.0);
    if (rc) return rc;
    Scalars sp;
    rc = read_scal(c, SC_AUX, &sp);
    if (rc) return rc;
    st.rel_res_plain = sp.out2 > 0 ? std::sqrt(sp.out / sp.out2) : std::sqrt(sp.out);
    const int nx = (int)c->nx, ny = (int)c->ny, nz = (int)c->nz;
    const int cx = (int)c->cgrid[0], cy = (int)c->cgrid[1], cz = (int)c->cgrid[2];
    {  // restriction, 1/2 per axis (the Galerkin 1/8)
      const int d1[3] = {cx, ny, nz}, d2[3] = {cx, cy, nz}, d3[3] = {cx, cy, cz};
      HIPCHK(launch_transfer(r0, t1, d1, nx, 0, 0, per, c->n, 0.5, 0, c->st));
      HIPCHK(launch_transfer(t1, t2, d2, ny, 1, 0, per, c->n, 0.5, 0, c->st));
      HIPCHK(launch_transfer(t2, bcv, d3, nz, 2, 0, per, c->n, 0.5, 0, c->st));
    }
    rc = tbs_bind_workspace(cc, c->ws + L.coff[5], tbs_workspace_bytes(cc, TBS_PREC_FP64));
    if (rc) return rc;
    HIPCHK(launch_fill(xc, 0, cc->N, c->st));
    const Layout Lc = layout(cc, TBS_PREC_FP64);
    CgArrays Ac{xc, cc->ws + Lc.off[1], {cc->ws + Lc.off[2], cc->ws + Lc.off[3]}, cc->ws + Lc.off[4], cc->ws + Lc.off[5],
                cc->ws + Lc.off[6]};
    rc = cg_init_async(cc, bcv, Ac, 0, c->opts.coarse_rtol);
    if (rc) return rc;
    int cit = 0;
    rc = cg_loop(cc, Ac, 0, 0, c->opts.inner_max_iter, &cit);
    if (rc < 0 && rc != TBS_E_BREAKDOWN) return rc;
    st.coarse_iters = cit;
    rc = ensure_x();  // the last prolongation pass adds into u_next = u_prev
    if (rc) return rc;
    {  // prolongation, added to u_next = u_prev
      const int d1[3] = {cx, cy, nz}, d2[3] = {cx, ny, nz}, d3[3] = {nx, ny, nz};
      HIPCHK(launch_transfer(xc, t2, d1, cz, 2, 1, per, c->n, 1.0, 0, c->st));
      HIPCHK(launch_transfer(t2, t1, d2, cy, 1, 1, per, c->n, 1.0, 0, c->st));
      HIPCHK(launch_transfer(t1, u_next, d3, cx, 0, 1, per, c->n, 1.0, 1, c->st));
    }
    if (prec == TBS_PREC_MIXED || prec == TBS_PREC_MIXED_BF16) {
      // the guess's residual (FP32 copy and norms) is the first refinement sweep's when it is kept
      rc = resid_async(c, u_next, b64, c->ws + L.off[1], TBS_F32, SC_AUX, FIN_NORMS, 0.0);
      if (rc) return rc;
      Scalars sg;
      rc = read_scal(c, SC_AUX, &sg);
      if (rc) return rc;
      st.rel_res_coarse = sg.out2 > 0 ? std::sqrt(sg.out / sg.out2) : std::sqrt(sg.out);
      if (st.rel_res_coarse < st.rel_res_plain) {
        res0 = sg;
        have_res0 = true;
      }
    } else {
      rc = fp64_relres(c, u_next, b64, &st.rel_res_coarse);
      if (rc) return rc;
    }
    if (st.rel_res_coarse < st.rel_res_plain) {
      st.used_coarse_guess = 1;
    } else {
      have_x = false;  // back to the plain guess u_prev
      have_res0 = false;
    }
  }

  int result = TBS_OK;
  if (prec == TBS_PREC_FP64) {
    rc = ensure_x();  // CG iterates in place on u_next
    if (rc) return rc;
    CgArrays A{u_next, c->ws + L.off[1], {c->ws + L.off[2], c->ws + L.off[3]}, c->ws + L.off[4], c->ws + L.off[5],
               c->ws + L.off[6]};
    rc = cg_init_async(c, b64, A, 0, rtol);
    if (rc) return rc;
    Scalars s;
    rc = read_scal(c, SC_CG, &s);
    if (rc) return rc;
    st.rel_res0 = s.bb > 0 ? std::sqrt(s.rr0 / s.bb) : 0.0;
    if (!g && !st.used_coarse_guess && std::isnan(st.rel_res_coarse)) st.rel_res_plain = st.rel_res0;
    if (st.used_learned_guess) st.rel_res_learned = st.rel_res0;
    int nit = 0;
    if (costed) HIPCHK(hipEventRecord(c->cost_ev[2], c->st));
    result = cg_loop(c, A, 0, 0, max_iter, &nit);
    if (costed && (rc = cost_lap(c, &t_cg))) return rc;
    st.iters = nit;
    if (result < 0 && result != TBS_E_BREAKDOWN) return result;
    rc = fp64_relres(c, u_next, b64, &st.rel_res_fp64);
    if (rc) return rc;
  } else if (prec == TBS_PREC_FP32) {
    float* b32 = (float*)(c->ws + L.off[0]);
    float* x32 = (float*)(c->ws + L.off[1]);
    float* r32 = (float*)(c->ws + L.off[2]);
    // b32 = M(u + tau q) in FP32 arithmetic on FP32-rounded inputs
    HIPCHK(launch_convert(u_prev, 0, x32, 1, c->N, c->st));
    if (q) HIPCHK(launch_convert(q, 0, r32, 1, c->N, c->st));
    rc = tbs_rhs(c, x32, q ? r32 : nullptr, b32, TBS_F32);
    if (rc) return rc;
    CgArrays A{x32, r32, {c->ws + L.off[3], c->ws + L.off[4]}, c->ws + L.off[5], c->ws + L.off[6], c->ws + L.off[7]};
    rc = cg_init_async(c, b32, A, 1, rtol);
    if (rc) return rc;
    Scalars s;
    rc = read_scal(c, SC_CG, &s);
    if (rc) return rc;
    st.rel_res0 = s.bb > 0 ? std::sqrt(s.rr0 / s.bb) : 0.0;
    st.rel_res_plain = st.rel_res0;
    int nit = 0;
    result = cg_loop(c, A, 1, 0, max_iter, &nit);
    st.iters = nit;
    if (result < 0 && result != TBS_E_BREAKDOWN) return result;
    HIPCHK(launch_convert(x32, 1, u_next, 0, c->N, c->st));
    // FP64 residual of the FP32 answer against the FP64 right-hand side (b64 built in r-space)
    double* b64w = (double*)(c->ws + L.off[2]);  // r32 + pA span >= 8N bytes: reuse as FP64 b
    rc = tbs_rhs(c, u_prev, q, b64w, TBS_F64);
    if (rc) return rc;
    rc = fp64_relres(c, u_next, b64w, &st.rel_res_fp64);
    if (rc) return rc;
  } else {
    // iterative refinement: FP64 outer residual, FP32 inner CG (p in bf16 for MIXED_BF16)
    const int dt = (prec == TBS_PREC_MIXED_BF16) ? 2 : 1;
    float* r32 = (float*)(c->ws + L.off[1]);
    float* d32 = (float*)(c->ws + L.off[2]);
    CgArrays A{d32, r32, {c->ws + L.off[3], c->ws + L.off[4]}, c->ws + L.off[5], c->ws + L.off[6], c->ws + L.off[7]};
    int total = 0, sweeps = 0;
    // a check expected to pass (the last sweep met its inner tolerance eta and rel eta <= rtol, rel
    // the residual it started from) first forms only the norms; the FP32 residual is stored only if
    // it fails after all
    bool expect_pass = false;
    for (;;) {
      Scalars s;
      double rscale = 1.0;  // the stored FP32 residual is r * rscale; the correction is scaled back
      if (sweeps == 0 && have_res0) {
        s = res0;  // r32 and the residual partial sums of u_next = u_prev are already in place
      } else {
        bool need_r = true;
        if (expect_pass && have_x) {
          rc = resid_async(c, u_next, b64, nullptr, TBS_F32, SC_AUX, FIN_NORMS, 0.0);
          if (rc) return rc;
          rc = read_scal(c, SC_AUX, &s);
          if (rc) return rc;
          const double relc = s.out2 > 0 ? std::sqrt(s.out / s.out2) : std::sqrt(s.out);
          need_r = !(relc <= rtol || s.out2 == 0.0);
        }
        if (need_r) {
          rc = resid_async(c, have_x ? u_next : u_prev, b64, r32, TBS_F32, SC_AUX, FIN_NORMS, 0.0);
          if (rc) return rc;
          rc = read_scal(c, SC_AUX, &s);
          if (rc) return rc;
        }
      }
      {
        // the inner FP32 solve sees r / s (the refinement's scaling, a power of two near the RMS of
        // r) whenever r's elements would leave the normal FP32 range: redo the residual scaled
        const double rms = std::sqrt(s.out / (double)c->N);
        if (rms > 0.0 && std::isfinite(rms) && (rms < 0x1p-96 || rms > 0x1p96)) {
          rscale = std::ldexp(1.0, -std::ilogb(rms));
          rc = resid_async(c, have_x ? u_next : u_prev, b64, r32, TBS_F32, SC_AUX, FIN_NORMS, 0.0, rscale);
          if (rc) return rc;
          rc = read_scal(c, SC_AUX, &s);
          if (rc) return rc;
        }
      }
      const double rel = s.out2 > 0 ? std::sqrt(s.out / s.out2) : std::sqrt(s.out);
      if (sweeps == 0) {
        st.rel_res0 = rel;
        if (!g && std::isnan(st.rel_res_coarse)) st.rel_res_plain = rel;
        if (st.used_learned_guess) st.rel_res_learned = rel;
      }
      st.rel_res_fp64 = rel;
      if (!std::isfinite(rel)) { result = set_err(TBS_E_BREAKDOWN, "non-finite residual"); break; }
      if (rel <= rtol || s.out2 == 0.0) { result = TBS_OK; break; }
      if (sweeps >= c->opts.max_sweeps || total >= max_iter) { result = TBS_W_NOT_CONVERGED; break; }
      // inner solve A d = r32 from d = 0 to relative tolerance eta (no tighter than needed)
      // a bf16-stored direction limits the attainable inner accuracy: never ask it for less than 1e-4
      const double eta = std::max(std::max(c->opts.inner_rtol, dt == 2 ? 1e-4 : 0.0), 0.5 * rtol / rel);
      expect_pass = (rel * eta <= rtol);
      // the one-kernel iteration takes d = 0 as given (not read until its first x update writes d,
      // nor by the refinement update if no update came), so d needs no zero fill
      const bool dzero = c->opts.fused_cg != 0;
      if (!dzero) HIPCHK(launch_fill(d32, 1, c->N, c->st));
      HIPCHK(launch_finalize(dzero ? FIN_INIT_XZERO : FIN_INIT, part0(c), part0(c),
                             stencil_blocks(base_args(c), M_RESID, 8, c->n, c->bc), scal(c, SC_CG), eta, c->st));
      c->cgf_xzero = dzero;
      int nit = 0;
      const int cap = std::min(c->opts.inner_max_iter, std::max(1, max_iter - total));
      // the inner solve's last x update is left pending and applied by the refinement update:
      // u_next = (u_next or u_prev) + (d + alpha p) in one pass over the arrays
      if (costed) HIPCHK(hipEventRecord(c->cost_ev[2], c->st));
      int irc = cg_loop(c, A, dt, 0, cap, &nit, true);
      c->cgf_xzero = false;
      if (costed && (rc = cost_lap(c, &t_cg))) return rc;
      total += nit;
      expect_pass = expect_pass && irc == TBS_OK;
      if (irc == TBS_E_BREAKDOWN && nit == 0) { result = irc; break; }
      if (irc < 0 && irc != TBS_E_BREAKDOWN) return irc;
      HIPCHK(launch_refine_add(u_next, have_x ? u_next : u_prev, d32, A.p[0], A.p[1], c->N, dt, scal(c, SC_CG),
                               1.0 / rscale, c->st));
      HIPCHK(launch_finalize(FIN_CLEAR_PENDING, nullptr, nullptr, 0, scal(c, SC_CG), 0.0, c->st));
      have_x = true;
      ++sweeps;
    }
    rc = ensure_x();  // no correction was added: the answer is the guess u_prev
    if (rc) return rc;
    st.iters = total;
    st.sweeps = sweeps;
  }
  if (g) {
    // backoff bookkeeping: a rejected guess counts, and so (energy test) does a kept one that did not
    // halve the plain guess's residual: it cannot save the iterations its network costs
    bool paid = st.used_learned_guess &&
                (c->opts.guess_test == 0 || st.rel_res_learned <= 0.5 * st.rel_res_plain);
    int wait = 0;
    if (costed) {
      // cost-aware: the kept guess saved ln(learned / plain) / ln(rho) iterations, rho the solve's mean
      // residual reduction per iteration; it paid if they took longer than the network and its test.
      // An iteration's time is the CG loops' time over their iterations (the step's fixed work, its
      // right-hand side and residual checks, is not saved by a better guess)
      HIPCHK(hipEventSynchronize(c->cost_ev[1]));
      float t_guess = 0.f;
      HIPCHK(hipEventElapsedTime(&t_guess, c->cost_ev[0], c->cost_ev[1]));
      const double t_iter = st.iters > 0 ? t_cg / st.iters : 0.0;
      st.learned_cost_iters = t_iter > 0.0 ? t_guess / t_iter : 0.0;
      double saved = 0.0;
      if (st.used_learned_guess && st.iters > 0 && st.rel_res0 > 0.0 && st.rel_res_fp64 > 0.0 &&
          st.rel_res_fp64 < st.rel_res0 && st.rel_res_learned > 0.0 && st.rel_res_plain > 0.0) {
        const double log_rho = std::log(st.rel_res_fp64 / st.rel_res0) / st.iters;
        saved = std::max(0.0, std::log(st.rel_res_learned / st.rel_res_plain) / log_rho);
      }
      st.learned_saved_iters = saved;
      // a kept guess that left nothing to iterate paid in full
      const bool solved = st.used_learned_guess && st.iters == 0 && result == TBS_OK;
      paid = paid && (solved || (t_iter > 0.0 && saved >= st.learned_cost_iters));
      if (!paid) {
        // at least as many steps as such a guess would need to pay once
        const double steps = saved > 0.0 ? std::ceil(st.learned_cost_iters / saved) : 64.0;
        wait = (int)std::min(64.0, std::max(1.0, steps));
      }
    }
    if (paid) {
      c->guess_rejects = 0;
    } else {
      ++c->guess_rejects;
      if (c->opts.guess_backoff) c->guess_wait = std::max(wait, 1 << std::min(c->guess_rejects - 1, 6));
    }
  }
  st.status = result;
  if (stats) *stats = st;
  return result;
}
