// Heat equation and the self-consistent field <-> temperature loop: thermal
// plans, the two solvers (diagonalisation in x and y with FP64 GEMMs and
// tridiagonal solves along z, the default;
// Jacobi-preconditioned conjugate gradients) and the loop of the flowchart in
// Sec. 4 (q = 0 -> T -> march with dk(T) -> q -> T -> ...).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "plan.hpp"
#include "thermal_kernels.hpp"

namespace shg {

// Device state of the direct solver, built on its first use.
struct Fdm {
  bool ready = false;
  rocblas_handle h = nullptr;
  FdmBox box{};
  double* pm[3] = {};       // forward factors P_d (column-major m_d x m_d)
  double* qm[3] = {};       // backward factors Q_d
  double* lam[3] = {};      // eigenvalues
  double* tz_diag = nullptr;   // z: diagonal and off-diagonal of A_z = W^-1 S (tridiagonal solve)
  double* tz_off = nullptr;
};

struct Therm {
  static constexpr uint64_t kMagic = 0x5348475f54484552ull;  // "SHG_THER"
  uint64_t magic = 0;
  shg_thermal_params p{};
  shg_dtype dtype = SHG_C64;
  int device = 0;
  ThermGeom g{};
  int nblk = 0;             // blocks of the grid-stride kernels
  dim3 dgrid, dblock;       // launch of the tiled direction/apply kernel
  int nblk_dir = 0;         // its block count
  size_t real_bytes = 4;
  Fdm fdm;
};

// Workspace: theta, r, p0, p1, Ap, t_prev, heat (one node vector each), block
// partials, device scalars.
struct ThermLayout {
  size_t theta, r, p0, p1, ap, t_prev, heat, part, sc, f0, f1, total;
};

static ThermLayout therm_layout(const Therm& th) {
  ThermLayout L{};
  const size_t vec = align256(th.g.n * th.real_bytes);
  size_t off = 0;
  for (size_t* f : {&L.theta, &L.r, &L.p0, &L.p1, &L.ap, &L.t_prev, &L.heat}) {
    *f = off;
    off += vec;
  }
  L.part = off;
  off += align256((size_t)std::max(2 * th.nblk, th.nblk_dir) * sizeof(double));
  L.sc = off;
  off += align256(16 * sizeof(double));
  L.f0 = L.f1 = off;
  if (th.p.method == SHG_THERMAL_DIRECT) {
    const size_t fb = align256(th.g.n * sizeof(double));
    L.f1 = off + fb;
    off += 2 * fb;
  }
  L.total = off;
  return L;
}

static bool is_pow2_grid(int v) { return v >= 16 && v <= 512 && (v & (v - 1)) == 0; }

static int validate_thermal(const shg_thermal_params* p) {
  if (!is_pow2_grid(p->nx) || !is_pow2_grid(p->ny))
    return fail(SHG_EINVAL, "nx=%d ny=%d: each must be a power of two in [16, 512]", p->nx, p->ny);
  if (p->nz < 1) return fail(SHG_EINVAL, "nz=%d must be >= 1", p->nz);
  if (!(p->lx > 0 && p->ly > 0 && p->lcr > 0) || !std::isfinite(p->lx) || !std::isfinite(p->ly) ||
      !std::isfinite(p->lcr))
    return fail(SHG_EINVAL, "lx, ly, lcr must be finite and positive");
  if (!(p->k_th > 0) || !std::isfinite(p->k_th))
    return fail(SHG_EINVAL, "k_th must be finite and positive");
  if (!(p->h_conv >= 0) || !std::isfinite(p->h_conv))
    return fail(SHG_EINVAL, "h_conv must be finite and >= 0");
  if (!std::isfinite(p->t_inf) || !std::isfinite(p->t_oven))
    return fail(SHG_EINVAL, "t_inf and t_oven must be finite");
  bool oven = false, cooled = false;
  for (int f = 0; f < 6; ++f) {
    if (p->faces[f] != SHG_FACE_AIR && p->faces[f] != SHG_FACE_OVEN &&
        p->faces[f] != SHG_FACE_INSULATED)
      return fail(SHG_EINVAL, "faces[%d]=%d is not SHG_FACE_AIR/OVEN/INSULATED", f, p->faces[f]);
    oven |= p->faces[f] == SHG_FACE_OVEN;
    cooled |= p->faces[f] == SHG_FACE_AIR && p->h_conv > 0;
  }
  if (!oven && !cooled)
    return fail(SHG_EINVAL, "no oven face and no convective face: the temperature is not fixed");
  if (p->method != SHG_THERMAL_DIRECT && p->method != SHG_THERMAL_CG)
    return fail(SHG_EINVAL, "method=%d is not SHG_THERMAL_DIRECT or SHG_THERMAL_CG", p->method);
  return SHG_OK;
}

static int ilog2(size_t v) {
  int k = 0;
  while (((size_t)1 << k) < v) ++k;
  return k;
}

static void build_geom(Therm& th) {
  const shg_thermal_params& p = th.p;
  ThermGeom& g = th.g;
  g.nx = p.nx;
  g.ny = p.ny;
  g.nzn = p.nz + 1;
  g.log2_nx = ilog2((size_t)p.nx);
  g.log2_plane = ilog2((size_t)p.nx * p.ny);
  const double h[3] = {p.lx / p.nx, p.ly / p.ny, p.lcr / p.nz};
  const double beta = p.h_conv / p.k_th;
  for (int d = 0; d < 3; ++d) {
    g.ih2[d] = 1.0 / (h[d] * h[d]);
    g.conv_lo[d] = p.faces[2 * d] == SHG_FACE_AIR ? 2.0 * beta / h[d] : 0.0;
    g.conv_hi[d] = p.faces[2 * d + 1] == SHG_FACE_AIR ? 2.0 * beta / h[d] : 0.0;
  }
  // per node class: role_d = 0 interior, 1 on the low face, 2 on the high face
  for (int cls = 0; cls < 27; ++cls) {
    const int role[3] = {cls % 3, (cls / 3) % 3, cls / 9};
    bool oven = false;
    double w = 1.0, dsum = 0.0, src = 0.0;
    for (int d = 0; d < 3; ++d) {
      dsum += 2.0 * g.ih2[d];
      if (role[d] == 0) continue;
      const int f = 2 * d + (role[d] - 1);
      w *= 0.5;
      oven |= p.faces[f] == SHG_FACE_OVEN;
      if (p.faces[f] == SHG_FACE_AIR) {
        dsum += 2.0 * beta / h[d];
        src -= 2.0 * beta * (p.t_oven - p.t_inf) / h[d];
      }
    }
    g.oven[cls] = oven ? 1 : 0;
    g.w[cls] = oven ? 0.0 : w;
    g.inv_diag[cls] = oven ? 0.0 : 1.0 / (w * dsum);
    g.src[cls] = oven ? 0.0 : w * src;
  }
  g.inv_k = 1.0 / p.k_th;
  g.n = (size_t)p.nx * p.ny * (p.nz + 1);
  th.nblk = (int)std::min<size_t>(2048, (g.n + 255) / 256);
  const int tx = std::min(64, p.nx), ty = 256 / tx;
  th.dblock = dim3(tx, ty);
  th.dgrid = dim3(p.nx / tx, p.ny / ty, (g.nzn + kThermZ - 1) / kThermZ);
  th.nblk_dir = (int)(th.dgrid.x * th.dgrid.y * th.dgrid.z);
  th.real_bytes = th.dtype == SHG_C64 ? 4 : 8;
}

static int check_therm(const shg_thermal* t) {
  if (!t) return fail(SHG_ESTATE, "thermal plan is NULL");
  const Therm* th = reinterpret_cast<const Therm*>(t);
  if (th->magic != Therm::kMagic) return fail(SHG_ESTATE, "not a live thermal plan");
  return SHG_OK;
}

// Conjugate gradients on theta = T - T_oven, warm-started from t_nodes.
template <typename R>
static int solve_t(Therm& th, const R* heat, R* t_nodes, R* t_mid, double tol, int max_iter,
                   char* ws, int* iters_out, double* resid_out, hipStream_t st) {
  const ThermLayout L = therm_layout(th);
  const ThermGeom& g = th.g;
  R* theta = (R*)(ws + L.theta);
  R* r = (R*)(ws + L.r);
  R* pc = (R*)(ws + L.p0);
  R* pn = (R*)(ws + L.p1);
  R* ap = (R*)(ws + L.ap);
  double* part = (double*)(ws + L.part);
  double* sc = (double*)(ws + L.sc);
  const dim3 grid(th.nblk), blk(256);
  hipLaunchKernelGGL((th_init<R>), grid, blk, 0, st, g, (const R*)t_nodes, th.p.t_oven, theta, pc);
  hipLaunchKernelGGL((th_residual<R>), grid, blk, 0, st, g, heat, (const R*)theta, r, part);
  hipLaunchKernelGGL(th_scalars, dim3(1), blk, 0, st, (const double*)part, th.nblk, 0, sc);
  double hs[kCount];
  hipError_t e = hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "thermal residual");
  const double bnorm = std::sqrt(hs[kBb]);
  int it = 0;
  double res = hs[kRz] > 0.0 ? 1.0 : 0.0;
  constexpr int kCheck = 16;
  while (it < max_iter && hs[kRz] > 0.0 && bnorm > 0.0) {
    const int chunk = std::min(kCheck, max_iter - it);
    for (int k = 0; k < chunk; ++k) {
      hipLaunchKernelGGL((th_direction_apply<R>), th.dgrid, th.dblock, 0, st, g, (const R*)r,
                         (const R*)pc, pn, ap, (const double*)sc, part);
      hipLaunchKernelGGL(th_scalars, dim3(1), blk, 0, st, (const double*)part, th.nblk_dir, 1, sc);
      hipLaunchKernelGGL((th_update<R>), grid, blk, 0, st, g, theta, r, (const R*)pn,
                         (const R*)ap, (const double*)sc, part);
      hipLaunchKernelGGL(th_scalars, dim3(1), blk, 0, st, (const double*)part, th.nblk, 2, sc);
      std::swap(pc, pn);
    }
    it += chunk;
    e = hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "thermal iteration");
    res = std::sqrt(std::max(hs[kRr], 0.0)) / bnorm;
    if (!std::isfinite(res)) return fail(SHG_EDEVICE, "thermal solve diverged (residual %g)", res);
    if (res <= tol) break;
  }
  if (bnorm == 0.0) {
    // no source and no convective drive: theta = 0 everywhere
    e = hipMemsetAsync(theta, 0, g.n * sizeof(R), st);
    if (e != hipSuccess) return hip_fail(e, "clearing theta");
    res = 0.0;
  }
  hipLaunchKernelGGL((th_finish<R>), grid, blk, 0, st, g, (const R*)theta, th.p.t_oven, t_nodes);
  if (t_mid) {
    const size_t plane = (size_t)g.nx * g.ny;
    hipLaunchKernelGGL((th_midplanes<R>), grid, blk, 0, st, (const R*)t_nodes, plane,
                       plane * (size_t)(g.nzn - 1), t_mid);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "thermal kernel launch");
  if (iters_out) *iters_out = it;
  if (resid_out) *resid_out = res;
  return SHG_OK;
}

static void free_fdm(Fdm& f) {
  for (int d = 0; d < 3; ++d) {
    if (f.pm[d]) (void)hipFree(f.pm[d]);
    if (f.qm[d]) (void)hipFree(f.qm[d]);
    if (f.lam[d]) (void)hipFree(f.lam[d]);
    f.pm[d] = f.qm[d] = f.lam[d] = nullptr;
  }
  if (f.tz_diag) (void)hipFree(f.tz_diag);
  if (f.tz_off) (void)hipFree(f.tz_off);
  f.tz_diag = f.tz_off = nullptr;
  if (f.h) (void)rocblas_destroy_handle(f.h);
  f.h = nullptr;
  f.ready = false;
}

static int blas_fail(rocblas_status s, const char* what) {
  return fail(SHG_EDEVICE, "%s: %s", what, rocblas_status_to_string(s));
}

// The 1-D operators; for x and y their eigendecompositions (rocSOLVER,
// tridiagonal divide and conquer, FP64) and the factors P_d, Q_d; for z the
// tridiagonal A_z itself, solved per mode pair.
static int fdm_setup(Therm& th, hipStream_t st) {
  Fdm& f = th.fdm;
  if (f.ready) return SHG_OK;
  free_fdm(f);
  rocblas_status bs = rocblas_create_handle(&f.h);
  if (bs != rocblas_status_success) return blas_fail(bs, "rocblas_create_handle");
  bs = rocblas_set_stream(f.h, st);
  if (bs != rocblas_status_success) return blas_fail(bs, "rocblas_set_stream");
  const shg_thermal_params& p = th.p;
  const int nd[3] = {p.nx, p.ny, p.nz + 1};
  const double h[3] = {p.lx / p.nx, p.ly / p.ny, p.lcr / p.nz};
  const double beta = p.h_conv / p.k_th;
  double *dd = nullptr, *ee = nullptr, *uu = nullptr, *ww = nullptr;
  rocblas_int* info = nullptr;
  int rc = SHG_OK;
  hipError_t e = hipSuccess;
  for (int d = 0; d < 3 && rc == SHG_OK; ++d) {
    const int lo = p.faces[2 * d], hi = p.faces[2 * d + 1];
    const int a = lo == SHG_FACE_OVEN ? 1 : 0;
    const int b = nd[d] - 1 - (hi == SHG_FACE_OVEN ? 1 : 0);
    const int m = b - a + 1;
    f.box.a[d] = a;
    f.box.m[d] = m;
    const double ih2 = 1.0 / (h[d] * h[d]);
    const double clo = lo == SHG_FACE_AIR ? 2.0 * beta / h[d] : 0.0;
    const double chi = hi == SHG_FACE_AIR ? 2.0 * beta / h[d] : 0.0;
    // weighted symmetric operator S and weights on the free nodes a..b
    std::vector<double> w(m), sd(m), D(m), E(std::max(m - 1, 1));
    for (int k = 0; k < m; ++k) {
      const int i = a + k;
      if (i == 0) {
        w[k] = 0.5;
        sd[k] = ih2 + 0.5 * clo;
      } else if (i == nd[d] - 1) {
        w[k] = 0.5;
        sd[k] = ih2 + 0.5 * chi;
      } else {
        w[k] = 1.0;
        sd[k] = 2.0 * ih2;
      }
    }
    for (int k = 0; k < m; ++k) D[k] = sd[k] / w[k];
    if (d == 2) {
      // A_z = W^-1 S: diagonal sd/w, off-diagonal -ih2/w in each row
      std::vector<double> od(m);
      for (int k = 0; k < m; ++k) od[k] = -ih2 / w[k];
      e = hipMalloc(&f.tz_diag, m * sizeof(double));
      if (e == hipSuccess) e = hipMalloc(&f.tz_off, m * sizeof(double));
      if (e == hipSuccess)
        e = hipMemcpyAsync(f.tz_diag, D.data(), m * sizeof(double), hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(f.tz_off, od.data(), m * sizeof(double), hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) rc = hip_fail(e, "direct solver set-up");
      continue;
    }
    for (int k = 0; k + 1 < m; ++k) E[k] = -ih2 / std::sqrt(w[k] * w[k + 1]);
    const size_t mm = (size_t)m * m;
    e = hipMalloc(&dd, m * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&ee, E.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&uu, mm * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&ww, m * sizeof(double));
    if (e == hipSuccess && !info) e = hipMalloc(&info, sizeof(rocblas_int));
    if (e == hipSuccess) e = hipMalloc(&f.pm[d], mm * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&f.qm[d], mm * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&f.lam[d], m * sizeof(double));
    if (e == hipSuccess) e = hipMemcpyAsync(dd, D.data(), m * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ee, E.data(), E.size() * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ww, w.data(), m * sizeof(double), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
      rc = hip_fail(e, "direct solver set-up");
    } else {
      bs = rocsolver_dstedc(f.h, rocblas_evect_tridiagonal, m, dd, ee, uu, m, info);
      rocblas_int hinfo = 0;
      if (bs == rocblas_status_success)
        e = hipMemcpyAsync(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (bs != rocblas_status_success) {
        rc = blas_fail(bs, "rocsolver_dstedc");
      } else if (e != hipSuccess) {
        rc = hip_fail(e, "rocsolver_dstedc");
      } else if (hinfo != 0) {
        rc = fail(SHG_EDEVICE, "tridiagonal eigensolver failed (info %d)", (int)hinfo);
      } else {
        hipLaunchKernelGGL(fdm_factors, dim3((unsigned)std::min<size_t>(4096, (mm + 255) / 256)),
                           dim3(256), 0, st, m, (const double*)uu, (const double*)ww, f.pm[d],
                           f.qm[d]);
        e = hipMemcpyAsync(f.lam[d], dd, m * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "direct solver factors");
      }
    }
    for (double** q : {&dd, &ee, &uu, &ww}) {
      if (*q) (void)hipFree(*q);
      *q = nullptr;
    }
  }
  if (info) (void)hipFree(info);
  if (rc) {
    free_fdm(f);
    return rc;
  }
  f.ready = true;
  return SHG_OK;
}

// y = M along one axis of the packed m0 x m1 x m2 array x (x fastest).
static int fdm_mode(Fdm& f, int axis, const double* mat, const double* x, double* y) {
  const int m0 = f.box.m[0], m1 = f.box.m[1], m2 = f.box.m[2];
  const double one = 1.0, zero = 0.0;
  rocblas_status bs;
  if (axis == 0) {
    bs = rocblas_dgemm(f.h, rocblas_operation_none, rocblas_operation_none, m0, m1 * m2, m0, &one,
                       mat, m0, x, m0, &zero, y, m0);
  } else if (axis == 1) {
    bs = rocblas_dgemm_strided_batched(f.h, rocblas_operation_none, rocblas_operation_transpose, m0,
                                       m1, m1, &one, x, m0, (rocblas_stride)m0 * m1, mat, m1, 0,
                                       &zero, y, m0, (rocblas_stride)m0 * m1, m2);
  } else {
    bs = rocblas_dgemm(f.h, rocblas_operation_none, rocblas_operation_transpose, m0 * m1, m2, m2,
                       &one, x, m0 * m1, mat, m2, &zero, y, m0 * m1);
  }
  return bs == rocblas_status_success ? SHG_OK : blas_fail(bs, "rocblas_dgemm");
}

template <typename R>
static int solve_direct(Therm& th, const R* heat, R* t_nodes, R* t_mid, char* ws, double* resid_out,
                        hipStream_t st) {
  {
    // ovens on both ends of a two-node direction leave no free node: T = T_oven
    const shg_thermal_params& p = th.p;
    const int nd[3] = {p.nx, p.ny, p.nz + 1};
    for (int d = 0; d < 3; ++d) {
      const int free_nodes = nd[d] - (p.faces[2 * d] == SHG_FACE_OVEN) -
                             (p.faces[2 * d + 1] == SHG_FACE_OVEN);
      if (free_nodes <= 0) {
        const ThermLayout L = therm_layout(th);
        R* theta = (R*)(ws + L.theta);
        hipError_t e = hipMemsetAsync(theta, 0, th.g.n * sizeof(R), st);
        if (e != hipSuccess) return hip_fail(e, "clearing theta");
        hipLaunchKernelGGL((th_finish<R>), dim3(th.nblk), dim3(256), 0, st, th.g,
                           (const R*)theta, p.t_oven, t_nodes);
        if (t_mid) {
          const size_t plane = (size_t)p.nx * p.ny;
          hipLaunchKernelGGL((th_midplanes<R>), dim3(th.nblk), dim3(256), 0, st,
                             (const R*)t_nodes, plane, plane * (size_t)p.nz, t_mid);
        }
        if (resid_out) *resid_out = 0.0;
        e = hipGetLastError();
        return e == hipSuccess ? SHG_OK : hip_fail(e, "thermal kernel launch");
      }
    }
  }
  int rc = fdm_setup(th, st);
  if (rc) return rc;
  Fdm& f = th.fdm;
  rocblas_status bs = rocblas_set_stream(f.h, st);
  if (bs != rocblas_status_success) return blas_fail(bs, "rocblas_set_stream");
  const ThermLayout L = therm_layout(th);
  const ThermGeom& g = th.g;
  double* f0 = (double*)(ws + L.f0);
  double* f1 = (double*)(ws + L.f1);
  double* part = (double*)(ws + L.part);
  double* sc = (double*)(ws + L.sc);
  const size_t np = (size_t)f.box.m[0] * f.box.m[1] * f.box.m[2];
  const dim3 grid((unsigned)std::min<size_t>(4096, (np + 255) / 256)), blk(256);
  hipLaunchKernelGGL((fdm_gather<R>), grid, blk, 0, st, g, f.box, heat, f0);
  // forward transforms x, y; tridiagonal solves along z; backward transforms
  if ((rc = fdm_mode(f, 0, f.pm[0], f0, f1)) || (rc = fdm_mode(f, 1, f.pm[1], f1, f0))) return rc;
  const size_t nxy = (size_t)f.box.m[0] * f.box.m[1];
  hipLaunchKernelGGL(fdm_tri_z, dim3((unsigned)std::min<size_t>(4096, (nxy + 255) / 256)), blk, 0, st,
                     f.box, (const double*)f.lam[0], (const double*)f.lam[1],
                     (const double*)f.tz_diag, (const double*)f.tz_off, f0, f1);
  if ((rc = fdm_mode(f, 0, f.qm[0], f0, f1)) || (rc = fdm_mode(f, 1, f.qm[1], f1, f0))) return rc;
  // f1 <- theta in FP64 on all nodes (the packed solution in f0 is then free)
  hipLaunchKernelGGL((fdm_scatter<R>), dim3(th.nblk), blk, 0, st, g, f.box, (const double*)f0,
                     th.p.t_oven, f1, t_nodes);
  if (t_mid) {
    const size_t plane = (size_t)g.nx * g.ny;
    hipLaunchKernelGGL((th_midplanes<R>), dim3(th.nblk), blk, 0, st, (const R*)t_nodes, plane,
                       plane * (size_t)(g.nzn - 1), t_mid);
  }
  if (!resid_out) {
    // no residual requested (the self-consistent loop): no check, no wait
    const hipError_t le = hipGetLastError();
    return le == hipSuccess ? SHG_OK : hip_fail(le, "direct solve");
  }
  // residual of the node equations for the FP64 solution: |b - A theta| / |b|
  hipLaunchKernelGGL((th_residual<double, true, R>), dim3(th.nblk), blk, 0, st, g, heat,
                     (const double*)f1, f0, part);
  hipLaunchKernelGGL(th_scalars, dim3(1), blk, 0, st, (const double*)part, th.nblk, 0, sc);
  double hs[kCount];
  hipError_t e = hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "direct solve");
  *resid_out = hs[kBb] > 0.0 ? std::sqrt(hs[kRz] / hs[kBb]) : std::sqrt(hs[kRz]);
  return SHG_OK;
}

static int solve_any(Therm& th, const void* heat, void* t_nodes, void* t_mid, double tol,
                     int max_iter, void* ws, int* iters, double* resid, hipStream_t st) {
  if (th.p.method == SHG_THERMAL_DIRECT) {
    if (iters) *iters = 0;
    if (th.dtype == SHG_C64)
      return solve_direct<float>(th, (const float*)heat, (float*)t_nodes, (float*)t_mid,
                                 (char*)ws, resid, st);
    return solve_direct<double>(th, (const double*)heat, (double*)t_nodes, (double*)t_mid,
                                (char*)ws, resid, st);
  }
  if (th.dtype == SHG_C64)
    return solve_t<float>(th, (const float*)heat, (float*)t_nodes, (float*)t_mid, tol, max_iter,
                          (char*)ws, iters, resid, st);
  return solve_t<double>(th, (const double*)heat, (double*)t_nodes, (double*)t_mid, tol, max_iter,
                         (char*)ws, iters, resid, st);
}

template <typename R>
static int max_change(Therm& th, const void* a, const void* b, char* ws, double* out,
                      hipStream_t st) {
  const ThermLayout L = therm_layout(th);
  double* part = (double*)(ws + L.part);
  double* sc = (double*)(ws + L.sc);
  hipLaunchKernelGGL((th_max_change<R>), dim3(th.nblk), dim3(256), 0, st, (const R*)a,
                     (const R*)b, th.g.n, part);
  hipLaunchKernelGGL(th_max_final, dim3(1), dim3(256), 0, st, (const double*)part, th.nblk,
                     sc + kCount);
  hipError_t e = hipMemcpyAsync(out, sc + kCount, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? SHG_OK : hip_fail(e, "temperature change");
}

static int self_consistent(Plan& pl, Therm& th, const void* a_f0, const void* a_sh0,
                           const double* dk_z, void* a_f, void* a_sh, void* t_nodes, void* t_mid,
                           double tol_t, int max_outer, double solve_tol, int max_iter, char* ws,
                           int* outer_out, double* change_out, hipStream_t st) {
  const ThermLayout L = therm_layout(th);
  void* heat = ws + L.heat;
  void* t_prev = ws + L.t_prev;
  const size_t vec = th.g.n * th.real_bytes;
  const size_t field = (size_t)pl.p.nx * pl.p.ny * 2 * th.real_bytes;
  // q = 0 -> T
  hipError_t e = hipMemsetAsync(heat, 0, vec, st);
  if (e != hipSuccess) return hip_fail(e, "clearing the heat source");
  int rc = solve_any(th, heat, t_nodes, t_mid, solve_tol, max_iter, ws, nullptr, nullptr, st);
  if (rc) return rc;
  double change = 0.0;
  int k = 0;
  while (k < max_outer) {
    e = hipMemcpyAsync(a_f, a_f0, field, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(a_sh, a_sh0, field, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(t_prev, t_nodes, vec, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "copies of the loop");
    if ((rc = propagate(pl, a_f, a_sh, dk_z, t_mid, 0, pl.p.nz, nullptr, nullptr, st, heat)))
      return rc;
    if ((rc = solve_any(th, heat, t_nodes, t_mid, solve_tol, max_iter, ws, nullptr, nullptr, st)))
      return rc;
    rc = th.dtype == SHG_C64 ? max_change<float>(th, t_nodes, t_prev, ws, &change, st)
                             : max_change<double>(th, t_nodes, t_prev, ws, &change, st);
    if (rc) return rc;
    ++k;
    if (change <= tol_t) break;
  }
  if (outer_out) *outer_out = k;
  if (change_out) *change_out = change;
  return SHG_OK;
}

}  // namespace shg

using namespace shg;

extern "C" {

int shg_thermal_create(shg_thermal** out, const shg_thermal_params* p, shg_dtype dtype) {
  if (!out) return fail(SHG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return fail(SHG_EINVAL, "params is NULL");
  if (dtype != SHG_C64 && dtype != SHG_C128) return fail(SHG_EINVAL, "unknown dtype %d", (int)dtype);
  int rc = validate_thermal(p);
  if (rc) return rc;
  Therm* th = new (std::nothrow) Therm();
  if (!th) return fail(SHG_ENOMEM, "host allocation failed");
  th->p = *p;
  th->dtype = dtype;
  (void)hipGetDevice(&th->device);
  build_geom(*th);
  th->magic = Therm::kMagic;
  *out = reinterpret_cast<shg_thermal*>(th);
  return ok();
}

int shg_thermal_destroy(shg_thermal* t) {
  if (!t) return ok();
  int rc = check_therm(t);
  if (rc) return rc;
  Therm* th = reinterpret_cast<Therm*>(t);
  free_fdm(th->fdm);
  th->magic = 0;
  delete th;
  return ok();
}

size_t shg_thermal_workspace_bytes(const shg_thermal* t) {
  if (check_therm(t)) return 0;
  return therm_layout(*reinterpret_cast<const Therm*>(t)).total;
}

int shg_thermal_solve(shg_thermal* t, const void* heat, void* t_nodes, void* t_mid, double tol,
                      int32_t max_iter, void* workspace, int32_t* iterations, double* residual,
                      void* stream) {
  int rc = check_therm(t);
  if (rc) return rc;
  if (!heat || !t_nodes || !workspace)
    return fail(SHG_EINVAL, "heat, t_nodes and workspace must be non-NULL device pointers");
  if (!(tol > 0) || max_iter < 1) return fail(SHG_EINVAL, "tol must be > 0 and max_iter >= 1");
  if ((rc = sticky_device_error())) return rc;
  Therm* th = reinterpret_cast<Therm*>(t);
  int it = 0;
  double res = 0.0;
  rc = solve_any(*th, heat, t_nodes, t_mid, tol, max_iter, workspace, &it, &res,
                 (hipStream_t)stream);
  if (iterations) *iterations = it;
  if (residual) *residual = res;
  return rc ? rc : ok();
}

int shg_self_consistent(shg_plan* plan, shg_thermal* t, const void* a_f0, const void* a_sh0,
                        const double* dk_z, void* a_f, void* a_sh, void* t_nodes, void* t_mid,
                        double tol_t, int32_t max_outer, double solve_tol, int32_t max_iter,
                        void* workspace, int32_t* outer, double* change, void* stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if ((rc = check_therm(t))) return rc;
  Plan* pl = reinterpret_cast<Plan*>(plan);
  Therm* th = reinterpret_cast<Therm*>(t);
  if (!a_f0 || !a_sh0 || !a_f || !a_sh || !t_nodes || !t_mid || !workspace)
    return fail(SHG_EINVAL, "fields, t_nodes, t_mid and workspace must be non-NULL");
  if (pl->dtype != th->dtype) return fail(SHG_EINVAL, "plan and thermal plan dtypes differ");
  const shg_thermal_params& q = th->p;
  if (q.nx != pl->p.nx || q.ny != pl->p.ny || q.nz != pl->p.nz || q.lx != pl->p.lx ||
      q.ly != pl->p.ly || q.lcr != pl->p.lcr)
    return fail(SHG_EINVAL, "the thermal grid (nx, ny, nz, lx, ly, lcr) must match the plan's");
  if (!(tol_t > 0) || max_outer < 1 || !(solve_tol > 0) || max_iter < 1)
    return fail(SHG_EINVAL, "tolerances must be > 0 and iteration limits >= 1");
  if ((rc = sticky_device_error())) return rc;
  int k = 0;
  double ch = 0.0;
  rc = self_consistent(*pl, *th, a_f0, a_sh0, dk_z, a_f, a_sh, t_nodes, t_mid, tol_t, max_outer,
                       solve_tol, max_iter, (char*)workspace, &k, &ch, (hipStream_t)stream);
  if (outer) *outer = k;
  if (change) *change = ch;
  return rc ? rc : ok();
}

}  // extern "C"
