// C ABI of the SSFM march (include/shg.h): plans, validation, schedules, the
// forward launch sequence and its cached HIP graph.
#include "shg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "kernels.hpp"
#include "plan.hpp"

namespace shg {

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int ok() {
  g_last_error.clear();
  return SHG_OK;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? SHG_ENOMEM : SHG_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

// ---------------------------------------------------------------- timing
// Optional per-kernel timing: launches go through hipExtLaunchKernelGGL with a
// start/stop event pair that brackets the dispatch itself.
struct LaunchTimer {
  Plan* pl;
  // returns false if no event pair could be obtained (then launch untimed)
  bool next(int kind, hipEvent_t* a, hipEvent_t* b) {
    if (!pl || !pl->timing) return false;
    const size_t need = 2 * (pl->ev_used + 1);
    while (pl->ev_pool.size() < need) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return false;
      pl->ev_pool.push_back(e);
    }
    *a = pl->ev_pool[2 * pl->ev_used];
    *b = pl->ev_pool[2 * pl->ev_used + 1];
    if (pl->ev_kind.size() <= pl->ev_used) pl->ev_kind.resize(pl->ev_used + 1);
    pl->ev_kind[pl->ev_used] = kind;
    pl->ev_used++;
    return true;
  }
};

template <typename K, typename A>
static void launch(K kernel, dim3 grid, dim3 block, hipStream_t st, LaunchTimer* tm, int kind,
                   const A& args) {
  hipEvent_t e0, e1;
  if (tm && tm->next(kind, &e0, &e1)) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0, e1, 0, args);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, st, args);
  }
}

// ---------------------------------------------------------------- schedules
template <typename R, int N, int E, int WG>
constexpr bool row_valid() {
  if constexpr (E > N) return false;
  constexpr int G = N / E;
  constexpr int rows = RowShape<G, WG>::rows;
  constexpr size_t lds = (size_t)rows * 4 * padded_len<N>() * sizeof(cx<R>);
  if (G * rows > 1024 || lds > 64 * 1024) return false;
  if constexpr (sizeof(R) == 8) return (E == 4 || E == 8) && WG == 64;
  return true;
}

template <typename R, int N, int E, int TC>
constexpr bool col_valid() {
  if constexpr (E > N) return false;
  constexpr int G = N / E;
  constexpr size_t lds = (size_t)2 * padded_len<N>() * TC * sizeof(cx<R>);
  if (G * TC < 32 || G * TC > 512 || lds > 64 * 1024) return false;
  if constexpr (sizeof(R) == 8) return (E == 4 || E == 8) && G * TC <= 128;
  return true;
}

template <typename R, int N, int E, int WG>
bool row_try(int e, int wg, const RowArgs<R>* a, hipStream_t st, int* rows_out, LaunchTimer* tm) {
  if constexpr (row_valid<R, N, E, WG>()) {
    if (e != E || wg != WG) return false;
    constexpr int G = N / E;
    using S = RowShape<G, WG>;
    if (rows_out) *rows_out = S::rows;
    if (a) {
      if (a->temp)
        launch(row_pass<R, N, G, S::rows, true>, dim3(a->ny / S::rows), dim3(S::threads), st, tm,
               0, *a);
      else
        launch(row_pass<R, N, G, S::rows, false>, dim3(a->ny / S::rows), dim3(S::threads), st, tm,
               0, *a);
    }
    return true;
  } else {
    (void)e; (void)wg; (void)a; (void)st; (void)rows_out; (void)tm;
    return false;
  }
}

template <typename R, int N, int E, int TC>
bool col_try(int e, int tc, const ColArgs<R>* a, hipStream_t st, LaunchTimer* tm) {
  if constexpr (col_valid<R, N, E, TC>()) {
    if (e != E || tc != TC) return false;
    if (a) {
      launch(col_pass<R, N, N / E, TC>, dim3(2 * a->tiles), dim3((N / E) * TC), st, tm, 1, *a);
    }
    return true;
  } else {
    (void)e; (void)tc; (void)a; (void)st; (void)tm;
    return false;
  }
}

// Wide schedule: e = 1 (one cell per thread), wg = WideShape<N>::threads.
template <typename R, int N>
bool row_wide_try(int e, int wg, const RowArgs<R>* a, hipStream_t st, int* rows_out,
                  LaunchTimer* tm) {
  using S = WideShape<N>;
  constexpr size_t lds = (size_t)(2 * S::rows + 4 * S::rows) * padded_len<N>() * sizeof(cx<R>);
  if constexpr (lds > 64 * 1024) {
    (void)e; (void)wg; (void)a; (void)st; (void)rows_out; (void)tm;
    return false;
  } else {
    if (e != 1 || wg != S::threads) return false;
    if (rows_out) *rows_out = S::rows;
    if (a) {
      if (a->temp)
        launch(row_pass_wide<R, N, true>, dim3(a->ny / S::rows), dim3(S::threads), st, tm, 0, *a);
      else
        launch(row_pass_wide<R, N, false>, dim3(a->ny / S::rows), dim3(S::threads), st, tm, 0,
               *a);
    }
    return true;
  }
}

template <typename R, int N>
bool row_dispatch_n(int e, int wg, const RowArgs<R>* a, hipStream_t st, int* rows,
                    LaunchTimer* tm) {
  return row_wide_try<R, N>(e, wg, a, st, rows, tm) || row_try<R, N, 4, 64>(e, wg, a, st, rows, tm) ||
         row_try<R, N, 4, 256>(e, wg, a, st, rows, tm) ||
         row_try<R, N, 8, 64>(e, wg, a, st, rows, tm) ||
         row_try<R, N, 8, 256>(e, wg, a, st, rows, tm) ||
         row_try<R, N, 16, 64>(e, wg, a, st, rows, tm) ||
         row_try<R, N, 16, 256>(e, wg, a, st, rows, tm);
}

template <typename R, int N>
bool col_dispatch_n(int e, int tc, const ColArgs<R>* a, hipStream_t st, LaunchTimer* tm) {
  return col_try<R, N, 4, 1>(e, tc, a, st, tm) || col_try<R, N, 4, 2>(e, tc, a, st, tm) ||
         col_try<R, N, 4, 4>(e, tc, a, st, tm) || col_try<R, N, 4, 8>(e, tc, a, st, tm) ||
         col_try<R, N, 4, 16>(e, tc, a, st, tm) || col_try<R, N, 8, 1>(e, tc, a, st, tm) ||
         col_try<R, N, 8, 2>(e, tc, a, st, tm) || col_try<R, N, 8, 4>(e, tc, a, st, tm) ||
         col_try<R, N, 8, 8>(e, tc, a, st, tm) || col_try<R, N, 8, 16>(e, tc, a, st, tm) ||
         col_try<R, N, 16, 1>(e, tc, a, st, tm) || col_try<R, N, 16, 2>(e, tc, a, st, tm) ||
         col_try<R, N, 16, 4>(e, tc, a, st, tm) || col_try<R, N, 16, 8>(e, tc, a, st, tm) ||
         col_try<R, N, 16, 16>(e, tc, a, st, tm);
}

template <typename R>
bool row_dispatch(int n, int e, int wg, const RowArgs<R>* a, hipStream_t st, int* rows,
                  LaunchTimer* tm = nullptr) {
  switch (n) {
    case 16: return row_dispatch_n<R, 16>(e, wg, a, st, rows, tm);
    case 32: return row_dispatch_n<R, 32>(e, wg, a, st, rows, tm);
    case 64: return row_dispatch_n<R, 64>(e, wg, a, st, rows, tm);
    case 128: return row_dispatch_n<R, 128>(e, wg, a, st, rows, tm);
    case 256: return row_dispatch_n<R, 256>(e, wg, a, st, rows, tm);
    case 512: return row_dispatch_n<R, 512>(e, wg, a, st, rows, tm);
    default: return false;
  }
}

template <typename R>
bool col_dispatch(int n, int e, int tc, const ColArgs<R>* a, hipStream_t st,
                  LaunchTimer* tm = nullptr) {
  switch (n) {
    case 16: return col_dispatch_n<R, 16>(e, tc, a, st, tm);
    case 32: return col_dispatch_n<R, 32>(e, tc, a, st, tm);
    case 64: return col_dispatch_n<R, 64>(e, tc, a, st, tm);
    case 128: return col_dispatch_n<R, 128>(e, tc, a, st, tm);
    case 256: return col_dispatch_n<R, 256>(e, tc, a, st, tm);
    case 512: return col_dispatch_n<R, 512>(e, tc, a, st, tm);
    default: return false;
  }
}

// Is (e, wg) a built row schedule for this grid?  rows_out gets rows per block.
bool row_supported(const Plan& pl, int e, int wg, int* rows) {
  int r = 0;
  bool okk = pl.dtype == SHG_C64 ? row_dispatch<float>(pl.p.nx, e, wg, nullptr, nullptr, &r)
                                 : row_dispatch<double>(pl.p.nx, e, wg, nullptr, nullptr, &r);
  if (!okk || pl.p.ny % r != 0) return false;
  if (rows) *rows = r;
  return true;
}

bool col_supported(const Plan& pl, int e, int tc) {
  bool okk = pl.dtype == SHG_C64 ? col_dispatch<float>(pl.p.ny, e, tc, nullptr, nullptr)
                                 : col_dispatch<double>(pl.p.ny, e, tc, nullptr, nullptr);
  return okk && pl.p.nx % tc == 0;
}

// Default schedules, from on-device sweeps of every built schedule.
// Single instance (latency bound): the wide row pass (one cell per thread) and
// a column pass with few elements per thread.  Batches (throughput bound):
// more elements per thread, fewer LDS round trips.  The autotuner may override
// both.
struct SchedRow {
  int n;
  int re, rw, ce, ct;
};
static const SchedRow kSingle[] = {{16, 1, 256, 4, 16}, {32, 1, 256, 4, 8}, {64, 1, 256, 4, 4},
                                   {128, 1, 256, 4, 2}, {256, 1, 256, 4, 2}, {512, 1, 512, 8, 4}};
static const SchedRow kBatch[] = {{16, 4, 64, 4, 16}, {32, 4, 64, 4, 8}, {64, 4, 64, 4, 4},
                                  {128, 4, 64, 16, 8}, {256, 4, 64, 16, 8}, {512, 4, 64, 8, 4}};

static bool apply_row(Plan& pl, int re, int rw, int* rows) { return row_supported(pl, re, rw, rows); }

static void pick(Plan& pl, const SchedRow* table, int* re, int* rw, int* ce, int* ct) {
  *re = *rw = *ce = *ct = 0;
  for (int i = 0; i < 6; ++i) {
    if (table[i].n == pl.p.nx) {
      int rows;
      if (apply_row(pl, table[i].re, table[i].rw, &rows)) {
        *re = table[i].re;
        *rw = table[i].rw;
      }
    }
    if (table[i].n == pl.p.ny) {
      int tc = table[i].ct;
      while (tc > 1 && !col_supported(pl, table[i].ce, tc)) tc >>= 1;
      if (col_supported(pl, table[i].ce, tc)) {
        *ce = table[i].ce;
        *ct = tc;
      }
    }
  }
  // fall back to any built schedule
  const int es[] = {4, 8, 16};
  const int wgs[] = {64, 256};
  for (int e : es)
    for (int w : wgs) {
      int rows;
      if (!*re && row_supported(pl, e, w, &rows)) {
        *re = e;
        *rw = w;
      }
    }
  for (int e : es)
    for (int tc = 16; tc >= 1 && !*ce; tc >>= 1)
      if (col_supported(pl, e, tc)) {
        *ce = e;
        *ct = tc;
      }
}

// The adjoint row pass follows the single-instance row schedule (it has a wide
// variant too); row_supported covers both since they share shapes.
static void pick_adjoint(Plan& pl) {
  pl.adj_e = pl.row_e;
  pl.adj_wg = pl.row_wg;
}

void default_schedule(Plan& pl) {
  pick(pl, kSingle, &pl.row_e, &pl.row_wg, &pl.col_e, &pl.col_tc);
  row_supported(pl, pl.row_e, pl.row_wg, &pl.row_rows);
  pick(pl, kBatch, &pl.b_row_e, &pl.b_row_wg, &pl.b_col_e, &pl.b_col_tc);
  pick_adjoint(pl);
}

// ---------------------------------------------------------------- tables
// W_n^k = exp(-2 pi i k / n) as R hi + lo (evaluated in long double); the lo
// part is only used in single precision.
template <typename R>
static std::vector<Tw<R>> twiddles(int n) {
  std::vector<Tw<R>> w(n);
  for (int k = 0; k < n; ++k) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * k / n;
    const long double cl = std::cos(a), sl = std::sin(a);
    const R c = (R)cl, s = (R)sl;
    const bool split = sizeof(R) == 4;
    w[k] = {c, s, split ? (R)(cl - (long double)c) : (R)0, split ? (R)(sl - (long double)s) : (R)0};
  }
  return w;
}

static double fftfreq(int i, int n, double d) {
  const int m = (i < (n + 1) / 2) ? i : i - n;
  return (double)m / ((double)n * d);
}

// exp(2 i pi^2 q^2 dz / k) for q = fftfreq(n, d); optional extra real factor.
static std::vector<double> prop_factor(int n, double d, double dz, double k, double extra,
                                       double tan_walkoff = 0.0) {
  std::vector<double> out(2 * n);
  for (int i = 0; i < n; ++i) {
    const double q = fftfreq(i, n, d);
    // diffraction, plus the walk-off translation by tan(rho) dz (x axis only)
    const double th = 2.0 * M_PI * M_PI * q * q * dz / k - 2.0 * M_PI * q * tan_walkoff * dz;
    out[2 * i] = extra * std::cos(th);
    out[2 * i + 1] = extra * std::sin(th);
  }
  return out;
}

static int upload(void** dst, const void* src, size_t bytes) {
  hipError_t e = hipMalloc(dst, bytes);
  if (e != hipSuccess) {
    *dst = nullptr;
    return hip_fail(e, "hipMalloc(plan table)");
  }
  e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(plan table)");
  return SHG_OK;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }
static bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }
static bool pow2_in_range(int v) { return v >= 16 && v <= 512 && (v & (v - 1)) == 0; }

int validate_params(const shg_params* p) {
  if (!pow2_in_range(p->nx) || !pow2_in_range(p->ny))
    return fail(SHG_EINVAL, "nx=%d ny=%d: each must be a power of two in [16, 512]", p->nx, p->ny);
  if (p->nz < 1) return fail(SHG_EINVAL, "nz=%d must be >= 1", p->nz);
  if (!finite_pos(p->lx) || !finite_pos(p->ly) || !finite_pos(p->lcr))
    return fail(SHG_EINVAL, "lx, ly, lcr must be finite and positive");
  if (!finite_pos(p->lambda_f) || !finite_pos(p->n_f) || !finite_pos(p->n_sh))
    return fail(SHG_EINVAL, "lambda_f, n_f, n_sh must be finite and positive");
  if (!std::isfinite(p->d_eff)) return fail(SHG_EINVAL, "d_eff must be finite");
  if (!finite_nonneg(p->alpha_f) || !finite_nonneg(p->alpha_sh) || !finite_nonneg(p->beta_f) ||
      !finite_nonneg(p->beta_sh))
    return fail(SHG_EINVAL, "absorption coefficients must be finite and >= 0");
  if (!std::isfinite(p->dk0) || !std::isfinite(p->ddk_dT) || !std::isfinite(p->ddk_dT2) ||
      !std::isfinite(p->ddk_dT3) || !std::isfinite(p->dn_dT) || !std::isfinite(p->t_ref))
    return fail(SHG_EINVAL, "dk0, ddk_dT, ddk_dT2, ddk_dT3, dn_dT, t_ref must be finite");
  if (!finite_nonneg(p->grating_period) || !std::isfinite(p->grating_a) ||
      !std::isfinite(p->grating_b))
    return fail(SHG_EINVAL, "grating_period must be finite and >= 0, grating_a/b finite");
  if (p->grating_period > 0.0) {
    const double x = p->t_ref - 298.15;
    if (!(1.0 + x * (p->grating_a + x * p->grating_b) > 0.0))
      return fail(SHG_EINVAL, "grating period must be positive at t_ref");
  }
  if (p->checkpoint_every < 0) return fail(SHG_EINVAL, "checkpoint_every must be >= 0");
  if (!(std::fabs(p->walkoff_f) < M_PI / 2) || !(std::fabs(p->walkoff_sh) < M_PI / 2))
    return fail(SHG_EINVAL, "walk-off angles must be finite with |rho| < pi/2");
  if (p->flags & ~(uint32_t)(SHG_UNDEPLETED | SHG_NO_GRAPH | SHG_SPLIT_LNL | SHG_CHECK_FINITE))
    return fail(SHG_EINVAL, "unknown flag bits 0x%x", p->flags);
  return SHG_OK;
}

static constexpr double kEps0 = 8.8541878128e-12;
static constexpr double kC = 299792458.0;

// Default adjoint checkpoint interval K.  The adjoint keeps ceil(nz/K) + 1
// checkpoints and stages K steps (both fields plus the temperature phase Psi,
// 5 reals per cell); the last segment is staged by the forward sweep itself, so
// only the first nz - K steps are recomputed, and with recomputed segments the
// staging is double-buffered (2K steps).  K = nz (nothing recomputed) when that
// fits in kAdjointStateBudget, else the largest K whose checkpoints and staging
// fit, but at least ceil(sqrt(nz)).
static constexpr size_t kAdjointStateBudget = size_t(16) << 30;

static int auto_checkpoint(int nz, size_t cells, int real_bytes) {
  const size_t per_step = cells * 5 * (size_t)real_bytes;
  const size_t slots = std::max<size_t>(1, kAdjointStateBudget / per_step);
  if ((size_t)nz + 2 <= slots) return nz;
  int k_min = 1;
  while ((size_t)k_min * k_min < (size_t)nz) ++k_min;
  for (int k = nz; k > k_min; --k) {
    const size_t segs = ((size_t)nz + k - 1) / k;
    if (2 * (size_t)k + segs + 1 <= slots) return k;
  }
  return k_min;
}

int build_plan(Plan& pl) {
  const shg_params& p = pl.p;
  const double lam_f = p.lambda_f, lam_sh = lam_f / 2.0;
  pl.dx = p.lx / p.nx;
  pl.dy = p.ly / p.ny;
  pl.dz = p.lcr / p.nz;
  pl.k_f = 2.0 * M_PI * p.n_f / lam_f;
  pl.k_sh = 2.0 * M_PI * p.n_sh / lam_sh;
  pl.kappa_f = 2.0 * M_PI * p.d_eff / (p.n_f * lam_f);
  pl.kappa_sh = 2.0 * M_PI * p.d_eff / (p.n_sh * lam_f);
  pl.tpa_f = p.beta_f * kEps0 * kC * p.n_f / 2.0;
  pl.tpa_sh = p.beta_sh * kEps0 * kC * p.n_sh / 2.0;
  pl.lens_f = 2.0 * M_PI * p.dn_dT / lam_f;
  pl.lens_sh = 2.0 * M_PI * p.dn_dT / lam_sh;
  pl.pscale_f = kEps0 * kC * p.n_f / 2.0 * pl.dx * pl.dy;
  pl.pscale_sh = kEps0 * kC * p.n_sh / 2.0 * pl.dx * pl.dy;
  pl.real_bytes = pl.dtype == SHG_C64 ? 4 : 8;
  pl.ckpt = p.checkpoint_every > 0 ? std::min(p.checkpoint_every, p.nz)
                                   : auto_checkpoint(p.nz, (size_t)p.nx * p.ny, pl.real_bytes);
  int rc;
  if (pl.dtype == SHG_C64) {
    auto tx = twiddles<float>(p.nx), ty = twiddles<float>(p.ny);
    if ((rc = upload(&pl.tw_x, tx.data(), tx.size() * sizeof(tx[0])))) return rc;
    if ((rc = upload(&pl.tw_y, ty.data(), ty.size() * sizeof(ty[0])))) return rc;
  } else {
    auto tx = twiddles<double>(p.nx), ty = twiddles<double>(p.ny);
    if ((rc = upload(&pl.tw_x, tx.data(), tx.size() * sizeof(tx[0])))) return rc;
    if ((rc = upload(&pl.tw_y, ty.data(), ty.size() * sizeof(ty[0])))) return rc;
  }
  const double norm = 1.0 / ((double)p.nx * (double)p.ny);
  const double ks[2] = {pl.k_f, pl.k_sh};
  const double al[2] = {p.alpha_f, p.alpha_sh};
  const double rho[2] = {p.walkoff_f, p.walkoff_sh};
  for (int w = 0; w < 2; ++w) {
    auto mx = prop_factor(p.nx, pl.dx, pl.dz, ks[w], 1.0, std::tan(rho[w]));
    auto my = prop_factor(p.ny, pl.dy, pl.dz, ks[w], std::exp(-al[w] * pl.dz / 2.0) * norm);
    if ((rc = upload((void**)&pl.mx[w], mx.data(), mx.size() * sizeof(double)))) return rc;
    if ((rc = upload((void**)&pl.my[w], my.data(), my.size() * sizeof(double)))) return rc;
    if (p.flags & SHG_SPLIT_LNL) {
      const double hz = pl.dz / 2.0;
      auto mxh = prop_factor(p.nx, pl.dx, hz, ks[w], 1.0, std::tan(rho[w]));
      auto myh = prop_factor(p.ny, pl.dy, hz, ks[w], std::exp(-al[w] * hz / 2.0) * norm);
      if ((rc = upload((void**)&pl.mxh[w], mxh.data(), mxh.size() * sizeof(double)))) return rc;
      if ((rc = upload((void**)&pl.myh[w], myh.data(), myh.size() * sizeof(double)))) return rc;
    }
  }
  default_schedule(pl);
  if (pl.row_e == 0 || pl.col_e == 0)
    return fail(SHG_EUNSUPPORTED, "no built schedule for nx=%d ny=%d", p.nx, p.ny);
  // the forward workspace and the finiteness flag are allocated here, so the
  // march itself never allocates (and can be recorded under stream capture)
  pl.own_ws_bytes = forward_ws_bytes(pl);
  hipError_t e = hipMalloc(&pl.own_ws, pl.own_ws_bytes);
  if (e != hipSuccess) {
    pl.own_ws = nullptr;
    return hip_fail(e, "hipMalloc(forward workspace)");
  }
  if (p.flags & SHG_CHECK_FINITE) {
    e = hipMalloc((void**)&pl.finite_flag, sizeof(int));
    if (e != hipSuccess) {
      pl.finite_flag = nullptr;
      return hip_fail(e, "hipMalloc(finite flag)");
    }
  }
  return SHG_OK;
}

void free_timing(Plan& pl) {
  for (hipEvent_t e : pl.ev_pool) (void)hipEventDestroy(e);
  pl.ev_pool.clear();
  pl.ev_kind.clear();
  pl.ev_used = 0;
}

void free_plan_tables(Plan& pl) {
  free_timing(pl);
  for (auto& g : pl.graphs) (void)hipGraphExecDestroy(g.exec);
  pl.graphs.clear();
  if (pl.cap_stream) (void)hipStreamDestroy(pl.cap_stream);
  pl.cap_stream = nullptr;
  void* ptrs[] = {pl.tw_x, pl.tw_y, pl.mx[0], pl.mx[1], pl.my[0], pl.my[1], pl.mxh[0], pl.mxh[1],
                  pl.myh[0], pl.myh[1], pl.own_ws,
                  pl.batch_ws, pl.finite_flag};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  pl.tw_x = pl.tw_y = nullptr;
  pl.mx[0] = pl.mx[1] = pl.my[0] = pl.my[1] = nullptr;
  pl.mxh[0] = pl.mxh[1] = pl.myh[0] = pl.myh[1] = nullptr;
  pl.own_ws = nullptr;
  pl.batch_ws = nullptr;
  pl.finite_flag = nullptr;
  free_adjoint(pl);
  free_batch(pl);
}

// ---------------------------------------------------------------- forward
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t forward_ws_bytes(const Plan& pl) {
  const size_t phase = (size_t)pl.p.nz * 5 * 4 * pl.real_bytes;   // [nz][5] StageCoef
  const size_t parts = (size_t)pl.p.ny * 2 * sizeof(double);
  const size_t psi = (size_t)pl.p.nx * pl.p.ny * pl.real_bytes;
  return align256(phase) + align256(parts) + align256(psi);
}

template <typename R>
static int enqueue_forward_t(Plan& pl, const FwdIO& io, const double* dk_z, int s0, int s1,
                             char* ws, double* powers, hipStream_t st, bool make_phase,
                             bool timed) {
  const shg_params& p = pl.p;
  StageCoef<R>* phase = (StageCoef<R>*)ws;
  double* partials = (double*)(ws + align256((size_t)p.nz * 5 * sizeof(StageCoef<R>)));
  R* psi = (R*)(ws + align256((size_t)p.nz * 5 * sizeof(StageCoef<R>)) +
                align256((size_t)p.ny * 2 * sizeof(double)));
  if (make_phase) {
    // kappa as the kernels' real type, like the batch's table
    hipLaunchKernelGGL((phase_table<R>), dim3(1), dim3(256), 0, st, dk_z, p.dk0, p.nz, pl.dz,
                       (double)(R)pl.kappa_f, (double)(R)pl.kappa_sh, phase);
  }
  const size_t n2 = (size_t)p.nx * p.ny;
  cx<R>* wa = (cx<R>*)io.a_work;
  cx<R>* wb = (cx<R>*)io.b_work;
  cx<R>* tap = (cx<R>*)io.tap;
  RowArgs<R> ra{};
  ra.tw = (const Tw<R>*)pl.tw_x;
  ra.phase = phase;
  ra.ny = p.ny;
  ra.kf = (R)pl.kappa_f;
  ra.ks = (R)pl.kappa_sh;
  ra.tf = (R)(pl.tpa_f / 2.0);
  ra.ts = (R)(pl.tpa_sh / 2.0);
  ra.h = (R)(pl.dz / 2.0);
  ra.undepleted = (p.flags & SHG_UNDEPLETED) ? 1 : 0;
  R* heat = (R*)io.heat;
  ra.hi_f = (R)(kEps0 * kC * p.n_f / 2.0);
  ra.hi_sh = (R)(kEps0 * kC * p.n_sh / 2.0);
  ra.ha_f = (R)p.alpha_f;
  ra.hb_f = (R)p.beta_f;
  ra.ha_sh = (R)p.alpha_sh;
  ra.hb_sh = (R)p.beta_sh;
  if (io.temp) {
    ra.temp = (const R*)io.temp;
    ra.psi = io.psi ? (R*)io.psi : psi;
    ra.t_ref = (R)p.t_ref;
    ra.dk = make_dk_shift<R>(p.ddk_dT, p.ddk_dT2, p.ddk_dT3, p.grating_period, p.grating_a,
                             p.grating_b, p.t_ref);
    ra.lens_f = (R)pl.lens_f;
    ra.lens_sh = (R)pl.lens_sh;
    ra.dz = (R)pl.dz;
    if (!io.psi) {
      hipLaunchKernelGGL((psi_init<R>), dim3((n2 + 255) / 256), dim3(256), 0, st, ra.temp, s0,
                         p.t_ref,
                         make_dk_shift<double>(p.ddk_dT, p.ddk_dT2, p.ddk_dT3, p.grating_period,
                                               p.grating_a, p.grating_b, p.t_ref),
                         pl.dz, ra.psi, n2);
    }
  }
  R* tap_psi = (R*)io.tap_psi;
  ColArgs<R> ca{};
  ca.f[0] = wa;
  ca.f[1] = wb;
  ca.tw = (const Tw<R>*)pl.tw_y;
  for (int w = 0; w < 2; ++w) {
    ca.mx[w] = pl.mx[w];
    ca.my[w] = pl.my[w];
  }
  ca.nx = p.nx;
  ca.tiles = p.nx / pl.col_tc;
  ca.conj_prop = 0;
  int rows = 1;
  LaunchTimer tm{timed ? &pl : nullptr};
  if (p.flags & SHG_SPLIT_LNL) {
    // L/2 - N - L/2: FFT_x, half-step column pass, then per step the whole
    // nonlinear step between IFFT_x and FFT_x and a column pass (half-step for
    // the last), and a closing IFFT_x
    ColArgs<R> ch = ca;
    for (int w = 0; w < 2; ++w) {
      ch.mx[w] = pl.mxh[w];
      ch.my[w] = pl.myh[w];
    }
    ra.ain = (const cx<R>*)io.a_in;
    ra.bin = (const cx<R>*)io.b_in;
    ra.aout = wa;
    ra.bout = wb;
    ra.tap_a = ra.tap_b = nullptr;
    ra.s_second = ra.s_first = -1;
    ra.full = 1;
    ra.inv_in = 0;
    ra.fwd_out = 1;
    ra.partials = nullptr;
    ra.heat = nullptr;
    if (!row_dispatch<R>(p.nx, pl.row_e, pl.row_wg, &ra, st, &rows, &tm))
      return fail(SHG_EUNSUPPORTED, "row schedule e=%d wg=%d not built", pl.row_e, pl.row_wg);
    if (!col_dispatch<R>(p.ny, pl.col_e, pl.col_tc, &ch, st, &tm))
      return fail(SHG_EUNSUPPORTED, "column schedule e=%d tc=%d not built", pl.col_e, pl.col_tc);
    ra.ain = wa;
    ra.bin = wb;
    ra.inv_in = 1;
    for (int s = s0; s < s1; ++s) {
      ra.s_first = s;
      // staging for the adjoint: the real-space state entering step s's RK4
      ra.tap_a = tap ? tap + (size_t)(s - s0) * 2 * n2 : nullptr;
      ra.tap_b = tap ? tap + (size_t)(s - s0) * 2 * n2 + n2 : nullptr;
      ra.tap_psi = tap_psi ? tap_psi + (size_t)(s - s0) * n2 : nullptr;
      row_dispatch<R>(p.nx, pl.row_e, pl.row_wg, &ra, st, &rows, &tm);
      col_dispatch<R>(p.ny, pl.col_e, pl.col_tc, s == s1 - 1 ? &ch : &ca, st, &tm);
    }
    ra.tap_a = ra.tap_b = nullptr;
    ra.tap_psi = nullptr;
    ra.s_first = -1;
    ra.fwd_out = 0;
    ra.aout = (cx<R>*)io.a_out;
    ra.bout = (cx<R>*)io.b_out;
    ra.partials = powers ? partials : nullptr;
    row_dispatch<R>(p.nx, pl.row_e, pl.row_wg, &ra, st, &rows, &tm);
    if (powers) {
      hipLaunchKernelGGL(power_finalize, dim3(1), dim3(256), 0, st, (const double*)partials,
                         p.ny / rows, pl.pscale_f, pl.pscale_sh, powers);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return SHG_OK;
  }
  // first row pass: N(dz/2) of step s0, then FFT_x
  ra.ain = (const cx<R>*)io.a_in;
  ra.bin = (const cx<R>*)io.b_in;
  ra.aout = wa;
  ra.bout = wb;
  ra.tap_a = ra.tap_b = nullptr;
  ra.s_second = -1;
  ra.s_first = s0;
  ra.inv_in = 0;
  ra.fwd_out = 1;
  ra.partials = nullptr;
  ra.heat = heat ? heat + (size_t)s0 * n2 : nullptr;
  if (!row_dispatch<R>(p.nx, pl.row_e, pl.row_wg, &ra, st, &rows, &tm))
    return fail(SHG_EUNSUPPORTED, "row schedule e=%d wg=%d not built", pl.row_e, pl.row_wg);
  for (int s = s0; s < s1; ++s) {
    if (!col_dispatch<R>(p.ny, pl.col_e, pl.col_tc, &ca, st, &tm))
      return fail(SHG_EUNSUPPORTED, "column schedule e=%d tc=%d not built", pl.col_e, pl.col_tc);
    const bool last = (s == s1 - 1);
    ra.ain = wa;
    ra.bin = wb;
    ra.aout = last ? (cx<R>*)io.a_out : wa;
    ra.bout = last ? (cx<R>*)io.b_out : wb;
    ra.tap_a = tap ? tap + (size_t)(s - s0) * 2 * n2 : nullptr;
    ra.tap_b = tap ? tap + (size_t)(s - s0) * 2 * n2 + n2 : nullptr;
    ra.tap_psi = tap_psi ? tap_psi + (size_t)(s - s0) * n2 : nullptr;
    ra.s_second = s;
    ra.s_first = last ? -1 : s + 1;
    ra.inv_in = 1;
    ra.fwd_out = last ? 0 : 1;
    ra.partials = (last && powers) ? partials : nullptr;
    ra.heat = heat ? heat + (size_t)(s + 1) * n2 : nullptr;
    row_dispatch<R>(p.nx, pl.row_e, pl.row_wg, &ra, st, &rows, &tm);
  }
  if (powers) {
    hipLaunchKernelGGL(power_finalize, dim3(1), dim3(256), 0, st, (const double*)partials,
                       p.ny / rows, pl.pscale_f, pl.pscale_sh, powers);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return SHG_OK;
}

int enqueue_forward_io(Plan& pl, const FwdIO& io, const double* dk_z, int s0, int s1, void* ws,
                       double* powers, hipStream_t st, bool make_phase, bool timed) {
  if (pl.dtype == SHG_C64)
    return enqueue_forward_t<float>(pl, io, dk_z, s0, s1, (char*)ws, powers, st, make_phase,
                                    timed);
  return enqueue_forward_t<double>(pl, io, dk_z, s0, s1, (char*)ws, powers, st, make_phase, timed);
}

int launch_col(Plan& pl, void* a, void* b, int conj, hipStream_t st, bool half) {
  if (half && !pl.mxh[0]) return fail(SHG_ESTATE, "no half-step propagator tables");
  const double* const* mx = half ? pl.mxh : pl.mx;
  const double* const* my = half ? pl.myh : pl.my;
  bool okk;
  if (pl.dtype == SHG_C64) {
    ColArgs<float> ca{};
    ca.f[0] = (cx<float>*)a;
    ca.f[1] = (cx<float>*)b;
    ca.tw = (const Tw<float>*)pl.tw_y;
    for (int w = 0; w < 2; ++w) {
      ca.mx[w] = mx[w];
      ca.my[w] = my[w];
    }
    ca.nx = pl.p.nx;
    ca.tiles = pl.p.nx / pl.col_tc;
    ca.conj_prop = conj;
    okk = col_dispatch<float>(pl.p.ny, pl.col_e, pl.col_tc, &ca, st);
  } else {
    ColArgs<double> ca{};
    ca.f[0] = (cx<double>*)a;
    ca.f[1] = (cx<double>*)b;
    ca.tw = (const Tw<double>*)pl.tw_y;
    for (int w = 0; w < 2; ++w) {
      ca.mx[w] = mx[w];
      ca.my[w] = my[w];
    }
    ca.nx = pl.p.nx;
    ca.tiles = pl.p.nx / pl.col_tc;
    ca.conj_prop = conj;
    okk = col_dispatch<double>(pl.p.ny, pl.col_e, pl.col_tc, &ca, st);
  }
  if (!okk) return fail(SHG_EUNSUPPORTED, "column schedule e=%d tc=%d not built", pl.col_e, pl.col_tc);
  return SHG_OK;
}

int enqueue_forward(Plan& pl, void* a, void* b, const double* dk_z, int s0, int s1, void* ws,
                    double* powers, hipStream_t st) {
  FwdIO io{a, b, a, b, a, b, nullptr};
  return enqueue_forward_io(pl, io, dk_z, s0, s1, ws, powers, st, true);
}

int enqueue_forward_temp(Plan& pl, void* a, void* b, const double* dk_z, const void* temp, int s0,
                         int s1, void* ws, double* powers, hipStream_t st, void* heat) {
  FwdIO io{a, b, a, b, a, b, nullptr};
  io.temp = temp;
  io.heat = heat;
  return enqueue_forward_io(pl, io, dk_z, s0, s1, ws, powers, st, true);
}

// Replays a cached graph of the whole launch sequence when the arguments are
// the same as last time; otherwise captures a new one on a private stream.
static int run_forward(Plan& pl, void* a, void* b, const double* dk_z, const void* temp, int s0,
                       int s1, void* ws, double* powers, hipStream_t st, void* heat) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  const bool use_graph = !(pl.p.flags & SHG_NO_GRAPH) && !pl.timing &&
                         cs == hipStreamCaptureStatusNone && (s1 - s0) >= 2;
  if (!use_graph) return enqueue_forward_temp(pl, a, b, dk_z, temp, s0, s1, ws, powers, st, heat);
  GraphKey key{a,  b,  dk_z, temp, heat, ws, powers, s0, s1, pl.row_e, pl.row_wg, pl.col_e,
               pl.col_tc};
  size_t hit = 0;
  while (hit < pl.graphs.size() && !(pl.graphs[hit].key == key)) ++hit;
  if (hit == pl.graphs.size()) {
    if (!pl.cap_stream) {
      e = hipStreamCreateWithFlags(&pl.cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    }
    e = hipStreamBeginCapture(pl.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    int rc = enqueue_forward_temp(pl, a, b, dk_z, temp, s0, s1, ws, powers, pl.cap_stream, heat);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(pl.cap_stream, &g);
    if (rc != SHG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    if ((int)pl.graphs.size() == Plan::kGraphCache) {
      (void)hipGraphExecDestroy(pl.graphs.back().exec);
      pl.graphs.pop_back();
    }
    pl.graphs.insert(pl.graphs.begin(), Plan::CachedGraph{key, exec});
  } else if (hit > 0) {
    std::rotate(pl.graphs.begin(), pl.graphs.begin() + hit, pl.graphs.begin() + hit + 1);
  }
  e = hipGraphLaunch(pl.graphs.front().exec, st);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return SHG_OK;
}

int check_plan(const shg_plan* plan) {
  if (!plan) return fail(SHG_ESTATE, "plan is NULL");
  const Plan* pl = reinterpret_cast<const Plan*>(plan);
  if (pl->magic != Plan::kMagic) return fail(SHG_ESTATE, "plan is not live (destroyed or invalid)");
  return SHG_OK;
}

int sticky_device_error() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "earlier HIP error");
  return SHG_OK;
}

int check_finite(Plan& pl, const void* data, size_t count, bool dbl, const char* what,
                 hipStream_t st) {
  if (!data || count == 0) return SHG_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone)
    return fail(SHG_EINVAL, "SHG_CHECK_FINITE scans synchronise the stream: not under capture");
  if (!pl.finite_flag) return fail(SHG_ESTATE, "plan has no finiteness flag");
  const dim3 grid((unsigned)std::min<size_t>(4096, (count + 255) / 256));
  hipLaunchKernelGGL(flag_clear, dim3(1), dim3(64), 0, st, pl.finite_flag);
  if (dbl || pl.dtype == SHG_C128)
    hipLaunchKernelGGL((finite_scan<double>), grid, dim3(256), 0, st, (const double*)data, count,
                       pl.finite_flag);
  else
    hipLaunchKernelGGL((finite_scan<float>), grid, dim3(256), 0, st, (const float*)data, count,
                       pl.finite_flag);
  int found = 0;
  e = hipMemcpyAsync(&found, pl.finite_flag, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "finiteness scan");
  if (found) return fail(SHG_ENONFINITE, "%s holds NaN or Inf", what);
  return SHG_OK;
}

int propagate(Plan& pl, void* a_f, void* a_sh, const double* dk_z, const void* temp, int s0,
              int s1, void* ws, double* powers, hipStream_t st, void* heat) {
  if (!a_f || !a_sh) return fail(SHG_EINVAL, "a_f and a_sh must be non-NULL device pointers");
  if (!(0 <= s0 && s0 < s1 && s1 <= pl.p.nz))
    return fail(SHG_EINVAL, "step range [%d, %d) not within [0, nz=%d]", s0, s1, pl.p.nz);
  int rc = sticky_device_error();
  if (rc) return rc;
  const size_t field = 2 * (size_t)pl.p.nx * pl.p.ny;
  if (checks_finite(pl)) {
    if ((rc = check_finite(pl, a_f, field, false, "input a_f", st)) ||
        (rc = check_finite(pl, a_sh, field, false, "input a_sh", st)) ||
        (rc = check_finite(pl, dk_z, (size_t)pl.p.nz, true, "dk_z", st)) ||
        (rc = check_finite(pl, temp, (size_t)pl.p.nz * field / 2, false, "temp", st)))
      return rc;
  }
  if (!ws) ws = pl.own_ws;
  rc = run_forward(pl, a_f, a_sh, dk_z, temp, s0, s1, ws, powers, st, heat);
  if (rc || !checks_finite(pl)) return rc;
  if ((rc = check_finite(pl, a_f, field, false, "the march's output a_f", st)) ||
      (rc = check_finite(pl, a_sh, field, false, "the march's output a_sh", st)))
    return rc;
  return SHG_OK;
}

// ---------------------------------------------------------------- static workspace
// Workspace of shg_propagate_noalloc: a device array of fixed size, one copy
// per GPU, held until the process ends.  Its name is only a host-side handle;
// the device address comes from hipGetSymbolAddress, taken once per device
// (with that device current) when the first plan is created there, and is the
// only form passed to kernels.  Every call on a GPU shares that GPU's copy.
constexpr size_t kStaticWsBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;   // device address per device id
static std::vector<int> g_scratch_state;   // 0 = not set up, 1 = ready, 2 = failed

static void static_ws_setup(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) {
    g_scratch_ptr.resize(device + 1, nullptr);
    g_scratch_state.resize(device + 1, 0);
  }
  if (g_scratch_state[device]) return;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
  g_scratch_state[device] = e == hipSuccess ? 1 : 2;
}

static void* static_ws(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= (int)g_scratch_ptr.size() || g_scratch_state[device] != 1)
    return nullptr;
  return g_scratch_ptr[device];
}

static int propagate_noalloc(Plan& pl, void* a_f, void* a_sh, const double* dk_z,
                             const void* temp, int s0, int s1, double* powers, hipStream_t st) {
  if (!a_f || !a_sh) return fail(SHG_EINVAL, "a_f and a_sh must be non-NULL device pointers");
  if (!(0 <= s0 && s0 < s1 && s1 <= pl.p.nz))
    return fail(SHG_EINVAL, "step range [%d, %d) not within [0, nz=%d]", s0, s1, pl.p.nz);
  if (checks_finite(pl))
    return fail(SHG_EINVAL, "SHG_CHECK_FINITE is not available without allocation");
  const size_t need = forward_ws_bytes(pl);
  if (need > kStaticWsBytes)
    return fail(SHG_EINVAL,
                "plan needs %zu bytes of workspace (nz=%d, %dx%d); the static workspace holds "
                "%zu bytes: use shg_propagate",
                need, pl.p.nz, pl.p.nx, pl.p.ny, kStaticWsBytes);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != pl.device)
    return fail(SHG_EINVAL, "plan was created on device %d, current device is %d", pl.device, dev);
  void* ws = static_ws(dev);
  if (!ws) return fail(SHG_EDEVICE, "static workspace address unavailable on device %d", dev);
  int rc = sticky_device_error();
  if (rc) return rc;
  FwdIO io{a_f, a_sh, a_f, a_sh, a_f, a_sh, nullptr};
  io.temp = temp;
  return enqueue_forward_io(pl, io, dk_z, s0, s1, ws, powers, st, true, false);
}

}  // namespace shg

using namespace shg;

extern "C" {

int shg_plan_create(shg_plan** out, const shg_params* p, shg_dtype dtype) {
  if (!out) return fail(SHG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return fail(SHG_EINVAL, "params is NULL");
  if (dtype != SHG_C64 && dtype != SHG_C128) return fail(SHG_EINVAL, "unknown dtype %d", (int)dtype);
  int rc = validate_params(p);
  if (rc) return rc;
  Plan* pl = new (std::nothrow) Plan();
  if (!pl) return fail(SHG_ENOMEM, "host allocation failed");
  static std::atomic<uint64_t> next_serial{1};
  pl->serial = next_serial.fetch_add(1);
  pl->p = *p;
  pl->dtype = dtype;
  (void)hipGetDevice(&pl->device);
  rc = build_plan(*pl);
  if (rc) {
    std::string msg = g_last_error;
    free_plan_tables(*pl);
    delete pl;
    g_last_error = msg;
    return rc;
  }
  static_ws_setup(pl->device);
  pl->magic = Plan::kMagic;
  *out = reinterpret_cast<shg_plan*>(pl);
  return ok();
}

int shg_plan_destroy(shg_plan* plan) {
  if (!plan) return ok();
  int rc = check_plan(plan);
  if (rc) return rc;
  Plan* pl = reinterpret_cast<Plan*>(plan);
  free_plan_tables(*pl);
  pl->magic = 0;
  delete pl;
  return ok();
}

size_t shg_workspace_bytes(const shg_plan* plan, int for_adjoint) {
  if (check_plan(plan)) return 0;
  const Plan* pl = reinterpret_cast<const Plan*>(plan);
  return for_adjoint ? adjoint_ws_bytes(*pl) : forward_ws_bytes(*pl);
}

int shg_propagate(shg_plan* plan, void* a_f, void* a_sh, const double* dk_z, const void* temp,
                  int32_t s_begin, int32_t s_end, void* workspace, double* powers, void* stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  Plan* pl = reinterpret_cast<Plan*>(plan);
  rc = propagate(*pl, a_f, a_sh, dk_z, temp, s_begin, s_end, workspace, powers,
                 (hipStream_t)stream, nullptr);
  return rc ? rc : ok();
}

int shg_propagate_noalloc(shg_plan* plan, void* a_f, void* a_sh, const double* dk_z,
                          const void* temp, int32_t s_begin, int32_t s_end, double* powers,
                          void* stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  Plan* pl = reinterpret_cast<Plan*>(plan);
  rc = propagate_noalloc(*pl, a_f, a_sh, dk_z, temp, s_begin, s_end, powers, (hipStream_t)stream);
  return rc ? rc : ok();
}

int shg_propagate_heat(shg_plan* plan, void* a_f, void* a_sh, const double* dk_z,
                       const void* temp, void* heat, void* workspace, double* powers,
                       void* stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!heat) return fail(SHG_EINVAL, "heat must be a non-NULL device pointer");
  Plan* pl = reinterpret_cast<Plan*>(plan);
  if (pl->p.flags & SHG_SPLIT_LNL)
    return fail(SHG_EUNSUPPORTED, "the heat source output needs the N/2 - L - N/2 split");
  rc = propagate(*pl, a_f, a_sh, dk_z, temp, 0, pl->p.nz, workspace, powers,
                 (hipStream_t)stream, heat);
  return rc ? rc : ok();
}

int shg_plan_set_schedule(shg_plan* plan, int32_t row_e, int32_t row_wg, int32_t col_e,
                          int32_t col_tc) {
  int rc = check_plan(plan);
  if (rc) return rc;
  Plan* pl = reinterpret_cast<Plan*>(plan);
  const int re = row_e ? row_e : pl->row_e, rw = row_wg ? row_wg : pl->row_wg;
  const int ce = col_e ? col_e : pl->col_e, ct = col_tc ? col_tc : pl->col_tc;
  int rows = 0;
  if (!row_supported(*pl, re, rw, &rows))
    return fail(SHG_EUNSUPPORTED, "row schedule e=%d wg=%d not built for nx=%d ny=%d", re, rw,
                pl->p.nx, pl->p.ny);
  if (!col_supported(*pl, ce, ct))
    return fail(SHG_EUNSUPPORTED, "column schedule e=%d tc=%d not built for nx=%d ny=%d", ce, ct,
                pl->p.nx, pl->p.ny);
  pl->row_e = re;
  pl->row_wg = rw;
  pl->row_rows = rows;
  pl->adj_e = re;
  pl->adj_wg = rw;
  pl->col_e = ce;
  pl->col_tc = ct;
  return ok();
}

int shg_plan_set_batch_schedule(shg_plan* plan, int32_t row_e, int32_t row_wg, int32_t col_e,
                                int32_t col_tc) {
  int rc = check_plan(plan);
  if (rc) return rc;
  Plan* pl = reinterpret_cast<Plan*>(plan);
  const int re = row_e ? row_e : pl->b_row_e, rw = row_wg ? row_wg : pl->b_row_wg;
  const int ce = col_e ? col_e : pl->b_col_e, ct = col_tc ? col_tc : pl->b_col_tc;
  int rows = 0;
  if (!row_supported(*pl, re, rw, &rows))
    return fail(SHG_EUNSUPPORTED, "row schedule e=%d wg=%d not built for nx=%d ny=%d", re, rw,
                pl->p.nx, pl->p.ny);
  if (!col_supported(*pl, ce, ct))
    return fail(SHG_EUNSUPPORTED, "column schedule e=%d tc=%d not built for nx=%d ny=%d", ce, ct,
                pl->p.nx, pl->p.ny);
  pl->b_row_e = re;
  pl->b_row_wg = rw;
  pl->b_col_e = ce;
  pl->b_col_tc = ct;
  return ok();
}

int shg_plan_describe(const shg_plan* plan, char* buf, size_t len) {
  int rc = check_plan(plan);
  if (rc) return rc;
  const Plan* pl = reinterpret_cast<const Plan*>(plan);
  if (buf && len) {
    snprintf(buf, len,
             "dtype=%s nx=%d ny=%d nz=%d row(e=%d wg=%d rows=%d) adj(e=%d wg=%d K=%d) "
             "col(e=%d tc=%d) batch(row e=%d wg=%d col e=%d tc=%d) graph=%d",
             pl->dtype == SHG_C64 ? "c64" : "c128", pl->p.nx, pl->p.ny, pl->p.nz, pl->row_e,
             pl->row_wg, pl->row_rows, pl->adj_e, pl->adj_wg, pl->ckpt, pl->col_e, pl->col_tc,
             pl->b_row_e,
             pl->b_row_wg, pl->b_col_e, pl->b_col_tc,
             (pl->p.flags & SHG_NO_GRAPH) ? 0 : 1);
  }
  return ok();
}

int shg_plan_set_timing(shg_plan* plan, int32_t enable) {
  int rc = check_plan(plan);
  if (rc) return rc;
  Plan* pl = reinterpret_cast<Plan*>(plan);
  pl->timing = enable ? 1 : 0;
  pl->ev_used = 0;
  return ok();
}

int shg_plan_kernel_times(shg_plan* plan, double* out) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!out) return fail(SHG_EINVAL, "out is NULL");
  Plan* pl = reinterpret_cast<Plan*>(plan);
  double sum[2] = {0.0, 0.0}, cnt[2] = {0.0, 0.0};
  for (size_t i = 0; i < pl->ev_used; ++i) {
    hipError_t e = hipEventSynchronize(pl->ev_pool[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, pl->ev_pool[2 * i], pl->ev_pool[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    const int k = pl->ev_kind[i] ? 1 : 0;
    sum[k] += ms;
    cnt[k] += 1.0;
  }
  out[0] = sum[0];
  out[1] = cnt[0];
  out[2] = sum[1];
  out[3] = cnt[1];
  pl->ev_used = 0;
  return ok();
}

const char* shg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
