// Forward SSFM kernels for gfx950: the row pass, the column pass, the
// per-call mismatch-phase table and the exit power reduction.
//
// One z-step of Eq. 14 (N/2 - L - N/2) is executed as two passes over both
// fields, each reading and writing the state once:
//   row pass    IFFT_x -> N(dz/2) second half of step s-1 -> N(dz/2) first
//               half of step s -> FFT_x        (one block owns whole rows)
//   column pass FFT_y -> multiply by the propagator of Eq. A.4 -> IFFT_y
//                                               (one block owns whole columns)
// so between passes the state is held in the (q_x, y) mixed domain.  The first
// row pass of a march skips the IFFT and the second half-step, and the last one
// skips the first half-step and the FFT.
#pragma once
#include <hip/hip_runtime.h>

#include "fft.hpp"

namespace shg {

// ---------------------------------------------------------------- nonlinear step
// Right-hand side of the nonlinear operator N (Eq. 11 with the coupling and TPA
// readings documented in shg.h):
//   fa = cf * b * conj(a) - tf |a|^2 a,   cf = i kappa_F exp(-i phi)
//   fb = cs * a^2         - ts |b|^2 b,   cs = i kappa_SH exp(+i phi)
// tf = beta~_F / 2, ts = beta~_SH / 2.
template <typename R>
__device__ __forceinline__ void nl_rhs(cx<R> a, cx<R> b, cx<R> cf, cx<R> cs, R tf, R ts,
                                       bool undepleted, cx<R>& fa, cx<R>& fb) {
  const cx<R> a2 = {a.re * a.re - a.im * a.im, (a.re + a.re) * a.im};
  fb = cs * a2 - scale(b, ts * norm2(b));
  if (undepleted) {
    fa = {(R)0, (R)0};
  } else {
    fa = cf * mul_conj(b, a) - scale(a, tf * norm2(a));
  }
}

// Coupling factors at the three distinct stage points of one RK4 half-step.
template <typename R>
struct HalfStep {
  cx<R> cf[3], cs[3];
};

// Coupling factors at one stage point of the per-step table: with
// e = exp(-i phi), cf = i kappa_F e and cs = i kappa_SH conj(e), formed in FP64
// when the table is built and rounded once.  A step has 5 points (z_s + k dz/4,
// k = 0..4); a half-step uses points 0, 1, 2 or 2, 3, 4 (stride 1), a full step
// of the L/2 - N - L/2 order points 0, 2, 4 (stride 2).
template <typename R>
struct StageCoef {
  cx<R> cf, cs;
};

template <typename R, typename P>
__device__ __forceinline__ HalfStep<R> half_step_coefs(P __restrict__ e, int stride = 1) {
  HalfStep<R> h;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const StageCoef<R> c = gload(e + k * stride);
    h.cf[k] = c.cf;
    h.cs[k] = c.cs;
  }
  return h;
}

// Classical RK4 over one half-step of length h with stage points t0, t0 + h/2,
// t0 + h/2, t0 + h (Sec. 3; the RK4 of the paper's nonlinear step).
template <bool UND, typename R>
__device__ __forceinline__ void rk4_cell_u(cx<R>& a, cx<R>& b, const HalfStep<R>& c, R tf, R ts,
                                           R h) {
  const R h2 = h * (R)0.5;
  cx<R> k1a, k1b, k2a, k2b, k3a, k3b, k4a, k4b;
  nl_rhs(a, b, c.cf[0], c.cs[0], tf, ts, UND, k1a, k1b);
  nl_rhs(a + scale(k1a, h2), b + scale(k1b, h2), c.cf[1], c.cs[1], tf, ts, UND, k2a, k2b);
  nl_rhs(a + scale(k2a, h2), b + scale(k2b, h2), c.cf[1], c.cs[1], tf, ts, UND, k3a, k3b);
  nl_rhs(a + scale(k3a, h), b + scale(k3b, h), c.cf[2], c.cs[2], tf, ts, UND, k4a, k4b);
  const R h6 = h * (R)(1.0 / 6.0);   // a product: a division is ten instructions
  a = a + scale(k1a + scale(k2a + k3a, (R)2) + k4a, h6);
  b = b + scale(k1b + scale(k2b + k3b, (R)2) + k4b, h6);
}
// The undepleted flag is uniform over a launch: one branch per half-step
// chooses a body specialised for it, instead of a branch in every stage.
template <typename R>
__device__ __forceinline__ void rk4_cell(cx<R>& a, cx<R>& b, const HalfStep<R>& c, R tf, R ts,
                                         R h, bool und) {
  if (und) rk4_cell_u<true>(a, b, c, tf, ts, h);
  else rk4_cell_u<false>(a, b, c, tf, ts, h);
}
// The same for the E cells of a thread.
template <int E, typename R>
__device__ __forceinline__ void rk4_cells(cx<R> (&a)[E], cx<R> (&b)[E], const HalfStep<R>& c, R tf,
                                          R ts, R h, bool und) {
  if (und) {
#pragma unroll
    for (int m = 0; m < E; ++m) rk4_cell_u<true>(a[m], b[m], c, tf, ts, h);
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) rk4_cell_u<false>(a[m], b[m], c, tf, ts, h);
  }
}

// ---------------------------------------------------------------- temperature
// With a temperature field the mismatch and the index are per cell.  On step s
// the phase is phi = Phi_s + dk_s tau + Psi_s + d_s tau, tau = z - z_s, where
// Phi_s + dk_s tau comes from the uniform table, dT_s = T_s - T_ref is the
// mid-plane sample, d_s = c1 dT_s + c2 dT_s^2 + c3 dT_s^3 is the cell's
// thermal mismatch shift and Psi_s = sum_{s' < s} d_s' dz is carried per cell.
// The thermal lens adds -i g_j dT_s A_j, g_j = (2 pi / lambda_j) dn/dT.
template <typename R>
struct HalfStepT {
  cx<R> cf[3], cs[3];
  R gf, gs;               // lens rates g_F dT, g_SH dT
};

__device__ __forceinline__ void sincos_r(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_r(double x, double* s, double* c) { sincos(x, s, c); }

// Thermal mismatch shift d(dT) = dk(T) - dk(T_ref) of Eq. 4, dT = T - T_ref:
// the dispersion part is the cubic dT (c1 + dT (c2 + dT c3)); the grating part
// 2 pi/Lambda(T_ref) - 2 pi/Lambda(T), Lambda = Lambda25 u, u = 1 + a x + b x^2,
// x = T - 25 C, is evaluated as g dT (a + b (2 xr + dT)) / u(T) with
// g = 2 pi / (Lambda25 u(T_ref)) and xr = T_ref - 25 C, which has no
// cancellation (g = 0 without a grating term).
template <typename R>
struct DkT {
  R c1, c2, c3;           // dispersion cubic
  R g, g25, a, b, xr;     // grating: 2 pi/(Lambda25 u_ref), 2 pi/Lambda25, a, b, T_ref - 25 C
};

// Built in FP64 on the host from the plan parameters (lam25 = 0: no grating term).
template <typename R>
inline DkT<R> make_dk_shift(double c1, double c2, double c3, double lam25, double a, double b,
                            double t_ref) {
  const double xr = t_ref - 298.15;
  const double g25 = lam25 > 0.0 ? 2.0 * M_PI / lam25 : 0.0;
  const double uref = 1.0 + xr * (a + xr * b);
  DkT<R> k;
  k.c1 = (R)c1;
  k.c2 = (R)c2;
  k.c3 = (R)c3;
  k.g = (R)(g25 / uref);
  k.g25 = (R)g25;
  k.a = (R)(lam25 > 0.0 ? a : 0.0);
  k.b = (R)(lam25 > 0.0 ? b : 0.0);
  k.xr = (R)xr;
  return k;
}

template <typename R>
__device__ __forceinline__ R thermal_dk(R dT, const DkT<R>& k) {
  R d = dT * (k.c1 + dT * (k.c2 + dT * k.c3));
  if (k.g != (R)0) {
    const R x = k.xr + dT;
    const R u = (R)1 + x * (k.a + x * k.b);
    d += k.g * dT * (k.a + k.b * (k.xr + x)) / u;
  }
  return d;
}
template <typename R>
__device__ __forceinline__ R thermal_dk_slope(R dT, const DkT<R>& k) {
  R d = k.c1 + dT * ((R)2 * k.c2 + (R)3 * k.c3 * dT);
  if (k.g25 != (R)0) {
    const R x = k.xr + dT;
    const R u = (R)1 + x * (k.a + x * k.b);
    d += k.g25 * (k.a + (R)2 * k.b * x) / (u * u);
  }
  return d;
}

// exp(-i x)
template <typename R>
__device__ __forceinline__ cx<R> expi_neg(R x) {
  R sn, c;
  sincos_r(x, &sn, &c);
  return {c, -sn};
}

// exp(-i x) for the phase advance of a quarter step, dkc dz/4, a small angle:
// Taylor series of cos and sin when |x| <= 1/8 in float (first omitted term
// below 6e-9) or 1/16 in double (below 3e-19), else sincos.
template <typename R>
__device__ __forceinline__ cx<R> expi_neg_small(R x) {
  const R x2 = x * x;
  if constexpr (sizeof(R) == 4) {
    if (fabsf(x) <= 0.125f) {
      const float c = 1.0f + x2 * (-0.5f + x2 * (1.0f / 24.0f));
      const float sn = x * (1.0f + x2 * (-1.0f / 6.0f + x2 * (1.0f / 120.0f)));
      return {c, -sn};
    }
  } else {
    if (fabs(x) <= 0.0625) {
      const double c = 1.0 + x2 * (-1.0 / 2 + x2 * (1.0 / 24 + x2 * (-1.0 / 720 + x2 * (1.0 / 40320))));
      const double sn =
          x * (1.0 + x2 * (-1.0 / 6 + x2 * (1.0 / 120 + x2 * (-1.0 / 5040 + x2 * (1.0 / 362880)))));
      return {c, -sn};
    }
  }
  return expi_neg(x);
}

// Stage coefficients of one cell's half-step or full step with a temperature
// field: u the uniform coupling factors at the three stage points, rho =
// exp(-i phase) of the cell's own phase at the first stage, step = exp(-i dkc
// qdz) the advance from stage to stage (qdz = dz/4 for a half-step, dz/2 for a
// full step) and dT the lens sample: cf = u.cf rho, cs = u.cs conj(rho).  The
// phase at the start of a step is the carried Psi of the cell, exp(-i Psi) is
// formed once per pass, and the later stages and the next step's start follow
// by products of step: the second half of a step starts at step^2, the next
// step at step^4 of the start of this one.
template <typename R>
__device__ __forceinline__ HalfStepT<R> thermal_coefs(const HalfStep<R>& u, cx<R> rho, cx<R> step,
                                                      R dT, R lens_f, R lens_sh) {
  HalfStepT<R> h;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    h.cf[k] = u.cf[k] * rho;
    h.cs[k] = u.cs[k] * conjg(rho);
    rho = rho * step;
  }
  h.gf = lens_f * dT;
  h.gs = lens_sh * dT;
  return h;
}

// nl_rhs plus the thermal-lens terms -i g A.
template <typename R>
__device__ __forceinline__ void nl_rhs_t(cx<R> a, cx<R> b, cx<R> cf, cx<R> cs, R tf, R ts, R gf,
                                         R gs, bool und, cx<R>& fa, cx<R>& fb) {
  nl_rhs(a, b, cf, cs, tf, ts, und, fa, fb);
  fb = fb + cx<R>{gs * b.im, -gs * b.re};
  if (!und) fa = fa + cx<R>{gf * a.im, -gf * a.re};
}

template <bool UND, typename R>
__device__ __forceinline__ void rk4_cell_t_u(cx<R>& a, cx<R>& b, const HalfStepT<R>& c, R tf, R ts,
                                             R h) {
  const R h2 = h * (R)0.5;
  cx<R> k1a, k1b, k2a, k2b, k3a, k3b, k4a, k4b;
  nl_rhs_t(a, b, c.cf[0], c.cs[0], tf, ts, c.gf, c.gs, UND, k1a, k1b);
  nl_rhs_t(a + scale(k1a, h2), b + scale(k1b, h2), c.cf[1], c.cs[1], tf, ts, c.gf, c.gs, UND, k2a,
           k2b);
  nl_rhs_t(a + scale(k2a, h2), b + scale(k2b, h2), c.cf[1], c.cs[1], tf, ts, c.gf, c.gs, UND, k3a,
           k3b);
  nl_rhs_t(a + scale(k3a, h), b + scale(k3b, h), c.cf[2], c.cs[2], tf, ts, c.gf, c.gs, UND, k4a,
           k4b);
  const R h6 = h * (R)(1.0 / 6.0);   // a product: a division is ten instructions
  a = a + scale(k1a + scale(k2a + k3a, (R)2) + k4a, h6);
  b = b + scale(k1b + scale(k2b + k3b, (R)2) + k4b, h6);
}
template <typename R>
__device__ __forceinline__ void rk4_cell_t(cx<R>& a, cx<R>& b, const HalfStepT<R>& c, R tf, R ts,
                                           R h, bool und) {
  if (und) rk4_cell_t_u<true>(a, b, c, tf, ts, h);
  else rk4_cell_t_u<false>(a, b, c, tf, ts, h);
}

// ---------------------------------------------------------------- row pass
template <typename R>
struct RowArgs {
  const cx<R>* ain;       // fundamental [ny][nx], read
  const cx<R>* bin;       // second harmonic [ny][nx], read
  cx<R>* aout;            // written (may equal ain: in place)
  cx<R>* bout;
  cx<R>* tap_a;           // optional: real-space state before the second half-step
  cx<R>* tap_b;
  const Tw<R>* tw;        // W_nx^k, k = 0..nx-1
  const StageCoef<R>* phase;  // [nz][5] coupling factors at z_s + {0, 1/4, 1/2, 3/4, 1} dz
  double* partials;       // [gridDim.x][2] sums of |A|^2 (last pass), or null
  int ny;
  int s_second;           // step whose second half-step runs here, or -1
  int s_first;            // step whose first half-step runs here, or -1
  int inv_in;             // apply IFFT_x after loading
  int fwd_out;            // apply FFT_x before storing
  int full;               // s_first runs a whole step over dz (L/2 - N - L/2 order)
  R kf, ks;               // kappa_F, kappa_SH
  R tf, ts;               // beta~_F / 2, beta~_SH / 2
  R h;                    // dz / 2
  int undepleted;
  // temperature field (THERMAL row passes only)
  const R* temp;          // [nz][ny][nx] mid-plane samples
  R* psi;                 // [ny][nx] in: Psi at the oldest step touched; out: at the newest
  R* tap_psi;             // optional: Psi_{s_second} (adjoint recompute)
  R t_ref, lens_f, lens_sh, dz;
  DkT<R> dk;              // mismatch shift of each cell's temperature
  // optional heat source (Sec. 2.2) of the state at this pass's step boundary
  // (after the second half-step of s_second, before the first of s_first)
  R* heat;                // [ny][nx] plane, or null
  R hi_f, hi_sh;          // eps0 c n_j / 2: intensity per |A_j|^2
  R ha_f, hb_f, ha_sh, hb_sh;   // alpha_j, beta_j
};

// q = sum_j alpha_j I_j + beta_j I_j^2, I_j = (eps0 c n_j / 2) |A_j|^2
template <typename R>
__device__ __forceinline__ R heat_density(cx<R> a, cx<R> b, const RowArgs<R>& p) {
  const R i_f = p.hi_f * norm2(a), i_s = p.hi_sh * norm2(b);
  return i_f * (p.ha_f + p.hb_f * i_f) + i_s * (p.ha_sh + p.hb_sh * i_s);
}

template <int G, int WG>
struct RowShape {
  static constexpr int rows = WG > G ? WG / G : 1;
  static constexpr int threads = G * rows;
};

// Fixed-order block reduction of two doubles; result valid in thread 0.
template <int T>
__device__ __forceinline__ void block_sum2(double& x, double& y, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    x += __shfl_down(x, off, 64);
    y += __shfl_down(y, off, 64);
  }
  constexpr int W = (T + 63) / 64;
  if constexpr (W > 1) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
      red[2 * w] = x;
      red[2 * w + 1] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      x = 0.0;
      y = 0.0;
      for (int i = 0; i < W; ++i) {
        x += red[2 * i];
        y += red[2 * i + 1];
      }
    }
  }
}

template <typename R, int N, int G, int ROWS, bool TH = false>
__device__ __forceinline__ void row_body(const RowArgs<R>& p, int blk) {
  constexpr int E = N / G;
  constexpr int P = padded_len<N>();
  // transforms within one wavefront with one butterfly per thread and pass
  // work in place: one LDS buffer per field instead of two
  constexpr int LB = (G <= 64 && stockham_one_butterfly<E, N>()) ? 1 : 2;
  __shared__ cx<R> lds[ROWS][2][LB][P];
  __shared__ double red[2 * ((G * ROWS + 63) / 64)];
  const int t = threadIdx.x % G;
  const int rr = threadIdx.x / G;
  const int y = blk * ROWS + rr;
  const size_t row = (size_t)y * N;
  const auto ain = gp(p.ain), bin = gp(p.bin);
  const auto aout = gp(p.aout), bout = gp(p.bout);
  cx<R> va[E], vb[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    va[m] = gload(ain + (row + t + G * m));
    vb[m] = gload(bin + (row + t + G * m));
  }
  const LdsView<R, 1> a0{&lds[rr][0][0][0]}, a1{&lds[rr][0][LB - 1][0]};
  const LdsView<R, 1> b0{&lds[rr][1][0][0]}, b1{&lds[rr][1][LB - 1][0]};
  TwRegs<R, N, G> twr;
  tw_load(twr, t, p.tw);
  // stage coefficients of the uniform-mismatch half-steps, loaded before the
  // transform so that the phase-table reads overlap it
  const int stf = p.full ? 2 : 1;
  HalfStep<R> c2{}, c1{};
  if constexpr (!TH) {
    if (p.s_second >= 0) c2 = half_step_coefs<R>(gp(p.phase) + 5 * p.s_second + 2);
    if (p.s_first >= 0) c1 = half_step_coefs<R>(gp(p.phase) + 5 * p.s_first, stf);
  }
  if (p.inv_in) {
    fft_pre<R, N, G, true, 1, (G <= 64)>(va, a0, a1, t, twr);
    fft_pre<R, N, G, true, 1, (G <= 64)>(vb, b0, b1, t, twr);
  }
  const bool und = p.undepleted != 0;
  if (p.tap_a) {
    const auto ta = gp(p.tap_a), tb = gp(p.tap_b);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      gstore(ta + (row + t + G * m), va[m]);
      gstore(tb + (row + t + G * m), vb[m]);
    }
  }
  if constexpr (TH) {
    const size_t n2 = (size_t)p.ny * N;
    const R qdz = p.dz * (R)0.25;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const size_t idx = row + t + G * m;
      R psi = p.psi[idx];
      if (p.tap_psi) p.tap_psi[idx] = psi;
      cx<R> rho = expi_neg(psi);
      if (p.s_second >= 0) {
        const R dT = p.temp[(size_t)p.s_second * n2 + idx] - p.t_ref;
        const R dkc = thermal_dk(dT, p.dk);
        const cx<R> step = expi_neg_small(dkc * qdz), st2 = step * step;
        const HalfStepT<R> c =
            thermal_coefs(half_step_coefs<R>(gp(p.phase) + 5 * p.s_second + 2), rho * st2,
                          step, dT, p.lens_f, p.lens_sh);
        rk4_cell_t(va[m], vb[m], c, p.tf, p.ts, p.h, und);
        psi += dkc * p.dz;
        rho = rho * (st2 * st2);
      }
      if (p.heat) p.heat[idx] = heat_density(va[m], vb[m], p);
      if (p.s_first >= 0) {
        const R dT = p.temp[(size_t)p.s_first * n2 + idx] - p.t_ref;
        const R dkc = thermal_dk(dT, p.dk);
        const int st = p.full ? 2 : 1;
        const HalfStepT<R> c =
            thermal_coefs(half_step_coefs<R>(gp(p.phase) + 5 * p.s_first, st), rho,
                          expi_neg_small(dkc * (qdz * st)), dT, p.lens_f, p.lens_sh);
        rk4_cell_t(va[m], vb[m], c, p.tf, p.ts, p.h * st, und);
        if (p.full) psi += dkc * p.dz;
      }
      // psi now holds Psi at the start of the newest step touched (s_first, or
      // s_second + 1 after a last pass, or s_first + 1 after a full step), so a
      // march [s0, s1) leaves Psi_{s1}
      if (p.s_second >= 0 || (p.full && p.s_first >= 0)) p.psi[idx] = psi;
    }
  } else {
    if (p.s_second >= 0) rk4_cells(va, vb, c2, p.tf, p.ts, p.h, und);
    if (p.heat) {
      const auto ht = gp(p.heat);
#pragma unroll
      for (int m = 0; m < E; ++m) ht[row + t + G * m] = heat_density(va[m], vb[m], p);
    }
    if (p.s_first >= 0) rk4_cells(va, vb, c1, p.tf, p.ts, p.h * stf, und);
  }
  if (p.fwd_out) {
    fft_pre<R, N, G, false, 1, (G <= 64)>(va, a0, a1, t, twr);
    fft_pre<R, N, G, false, 1, (G <= 64)>(vb, b0, b1, t, twr);
  }
#pragma unroll
  for (int m = 0; m < E; ++m) {
    gstore(aout + (row + t + G * m), va[m]);
    gstore(bout + (row + t + G * m), vb[m]);
  }
  if (p.partials) {
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      sa += (double)va[m].re * (double)va[m].re + (double)va[m].im * (double)va[m].im;
      sb += (double)vb[m].re * (double)vb[m].re + (double)vb[m].im * (double)vb[m].im;
    }
    block_sum2<G * ROWS>(sa, sb, red);
    if (threadIdx.x == 0) {
      const auto pt = gp(p.partials);
      pt[2 * blk] = sa;
      pt[2 * blk + 1] = sb;
    }
  }
}

template <typename R, int N, int G, int ROWS, bool TH>
__global__ void __launch_bounds__(G * ROWS) row_pass(RowArgs<R> p) {
  row_body<R, N, G, ROWS, TH>(p, blockIdx.x);
}

// Psi at the start of step s_begin: sum_{s < s_begin} d(T_s - T_ref) dz per
// cell, d the mismatch shift (FP64 accumulation); zero for s_begin = 0.
template <typename R>
__global__ void __launch_bounds__(256) psi_init(const R* __restrict__ temp, int s_begin, double t_ref,
                                                DkT<double> dk, double dz, R* __restrict__ psi,
                                                size_t n2) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n2) return;
  double acc = 0.0;
  for (int s = 0; s < s_begin; ++s) {
    const double dT = (double)temp[(size_t)s * n2 + i] - t_ref;
    acc += thermal_dk(dT, dk) * dz;
  }
  psi[i] = (R)acc;
}

// ---------------------------------------------------------------- finiteness scan
// Debugging aid: flag[0] = 1 when any of the n values is NaN or infinite.  Only
// lanes that find one store, all the same value; the flag is cleared first by
// flag_clear on the same stream.
template <typename T>
__global__ void __launch_bounds__(256) finite_scan(const T* __restrict__ x, size_t n,
                                                   int* __restrict__ flag) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    if (!isfinite(x[i])) flag[0] = 1;
}

static __global__ void __launch_bounds__(64) flag_clear(int* __restrict__ flag) {
  if (threadIdx.x == 0) flag[0] = 0;
}

// ---------------------------------------------------------------- wide row pass
// Latency-oriented row pass for marches that are too small to fill the chip:
// every thread owns one cell (both fields) for the two RK4 half-steps, and the
// first half of the block runs the row transforms at 4 elements per thread
// (2 * ROWS transforms of length N).  Cells move between the transform layout
// and the one-cell-per-thread layout through LDS.  Same arithmetic, in the same
// order per cell, as row_body.
template <int N>
struct WideShape {
  static constexpr int threads = N >= 256 ? N : 256;
  static constexpr int rows = threads / N;
  static constexpr int ef = 4;
  static constexpr int g = N / ef;
  static constexpr int fft_threads = 2 * rows * g;
};

template <typename R, int N, bool TH>
__device__ __forceinline__ void row_wide_body(const RowArgs<R>& p, int blk) {
  using S = WideShape<N>;
  constexpr int ROWS = S::rows, G = S::g, EF = S::ef;
  constexpr int P = padded_len<N>();
  __shared__ cx<R> cell[2][ROWS][P];
  __shared__ cx<R> pp[2 * ROWS][2][P];
  __shared__ double red[2 * ((S::threads + 63) / 64)];
  const int tid = threadIdx.x;
  // transform role: transform tr = 2 * row + field, element t + G*m
  const bool fth = tid < S::fft_threads;
  const int tr = transform_index<G>(fth, tid);
  const int t = tid % G;
  const int ff = tr & 1, fr = tr >> 1;
  const size_t frow = (size_t)(blk * ROWS + fr) * N;
  const LdsView<R, 1> q0{&pp[tr][0][0]}, q1{&pp[tr][1][0]};
  // cell role
  const int cr = tid / N, cxi = tid % N;
  const size_t idx = (size_t)(blk * ROWS + cr) * N + cxi;
  cx<R> v[EF];
  cx<R> a, b;
  TwRegs<R, N, G> twr;
  if (fth) tw_load(twr, t, p.tw);
  // the coupling factors of both half-steps are loaded here, unconditionally
  // (a step index < 0 reads step 0, unused), so that no wait on them stands
  // before the field loads
  const int stf = p.full ? 2 : 1;
  const HalfStep<R> c2 = half_step_coefs<R>(gp(p.phase) + 5 * max(p.s_second, 0) + 2);
  const HalfStep<R> c1 = half_step_coefs<R>(gp(p.phase) + 5 * max(p.s_first, 0), stf);
  // with a temperature field: the cell's Psi and its two samples, raw, loaded
  // after the field loads (unconditionally, like the table values), so that
  // the transform waits only for the fields
  R th_psi = (R)0, th_t2 = (R)0, th_t1 = (R)0;
  const auto th_loads = [&]() {
    if constexpr (TH) {
      const size_t n2 = (size_t)p.ny * N;
      th_psi = p.psi[idx];
      th_t2 = p.temp[(size_t)max(p.s_second, 0) * n2 + idx];
      th_t1 = p.temp[(size_t)max(p.s_first, 0) * n2 + idx];
    }
  };
  if (p.inv_in) {
    if (fth) {
      const auto src = gp(pick_ptr(ff, p.ain, p.bin));
#pragma unroll
      for (int m = 0; m < EF; ++m) v[m] = gload(src + (frow + t + G * m));
    }
    th_loads();
    fft_pre<R, N, G, true, 1, (G <= 64)>(v, q0, q1, t, twr, fth);
    if (fth) {
#pragma unroll
      for (int m = 0; m < EF; ++m) cell[ff][fr][pad16(t + G * m)] = v[m];
    }
    __syncthreads();
    a = cell[0][cr][pad16(cxi)];
    b = cell[1][cr][pad16(cxi)];
  } else {
    a = gload(gp(p.ain) + idx);
    b = gload(gp(p.bin) + idx);
    th_loads();
  }
  if (p.tap_a) {
    gstore(gp(p.tap_a) + idx, a);
    gstore(gp(p.tap_b) + idx, b);
  }
  const bool und = p.undepleted != 0;
  if constexpr (TH) {
    // Psi of this cell, the phase rho = exp(-i Psi) and the stage
    // coefficients of each half-step, formed just before its RK4
    if (p.tap_psi) p.tap_psi[idx] = th_psi;
    const R qdz = p.dz * (R)0.25;
    R psi = th_psi;
    cx<R> rho = expi_neg(psi);
    if (p.s_second >= 0) {
      const R dT = th_t2 - p.t_ref;
      const R dkc = thermal_dk(dT, p.dk);
      const cx<R> step = expi_neg_small(dkc * qdz), st2 = step * step;
      const HalfStepT<R> c2t =
          thermal_coefs(c2, rho * st2, step, dT, p.lens_f, p.lens_sh);
      rk4_cell_t(a, b, c2t, p.tf, p.ts, p.h, und);
      psi += dkc * p.dz;
      rho = rho * (st2 * st2);
    }
    if (p.heat) p.heat[idx] = heat_density(a, b, p);
    if (p.s_first >= 0) {
      const R dT = th_t1 - p.t_ref;
      const R dkc = thermal_dk(dT, p.dk);
      const HalfStepT<R> c1t = thermal_coefs(c1, rho,
                                             expi_neg_small(dkc * (qdz * stf)), dT, p.lens_f,
                                             p.lens_sh);
      rk4_cell_t(a, b, c1t, p.tf, p.ts, p.h * stf, und);
      if (p.full) psi += dkc * p.dz;
    }
    // Psi at the start of the newest step touched
    if (p.s_second >= 0 || (p.full && p.s_first >= 0)) p.psi[idx] = psi;
  } else {
    if (p.s_second >= 0) rk4_cell(a, b, c2, p.tf, p.ts, p.h, und);
    if (p.heat) gp(p.heat)[idx] = heat_density(a, b, p);
    if (p.s_first >= 0) rk4_cell(a, b, c1, p.tf, p.ts, p.h * stf, und);
  }
  if (p.fwd_out) {
    // each thread rewrites only the cell it read, so no barrier is needed
    // before the write; the transform wavefronts read after the barrier
    cell[0][cr][pad16(cxi)] = a;
    cell[1][cr][pad16(cxi)] = b;
    __syncthreads();
    if (fth) {
#pragma unroll
      for (int m = 0; m < EF; ++m) v[m] = cell[ff][fr][pad16(t + G * m)];
    }
    fft_pre<R, N, G, false, 1, (G <= 64)>(v, q0, q1, t, twr, fth);
    if (fth) {
      const auto dst = gp(pick_ptr(ff, p.aout, p.bout));
#pragma unroll
      for (int m = 0; m < EF; ++m) gstore(dst + (frow + t + G * m), v[m]);
    }
  } else {
    gstore(gp(p.aout) + idx, a);
    gstore(gp(p.bout) + idx, b);
  }
  if (p.partials) {
    double sa = (double)a.re * (double)a.re + (double)a.im * (double)a.im;
    double sb = (double)b.re * (double)b.re + (double)b.im * (double)b.im;
    block_sum2<S::threads>(sa, sb, red);
    if (threadIdx.x == 0) {
      const auto pt = gp(p.partials);
      pt[2 * blk] = sa;
      pt[2 * blk + 1] = sb;
    }
  }
}

template <typename R, int N, bool TH>
__global__ void __launch_bounds__(WideShape<N>::threads) row_pass_wide(RowArgs<R> p) {
  row_wide_body<R, N, TH>(p, blockIdx.x);
}

// ---------------------------------------------------------------- column pass
template <typename R>
struct ColArgs {
  cx<R>* f[2];            // fields (0 = F, 1 = SH)
  const Tw<R>* tw;        // W_ny^k
  const double* mx[2];    // per wave: exp(2 i pi^2 qx^2 dz / k), interleaved (re, im) [nx]
  const double* my[2];    // per wave: exp(2 i pi^2 qy^2 dz / k) exp(-alpha dz/2) / (nx ny) [ny]
  int nx;                 // row pitch in elements
  int tiles;              // column tiles per field (nx / TC)
  int conj_prop;          // multiply by conj(M) (adjoint of the linear step)
};

// Block b -> (field, tile).  Blocks are dealt to the 8 XCDs round-robin
// (b mod 8); consecutive tiles share L2 lines when TC < 16, so consecutive
// tiles are given to blocks on the same XCD.
__device__ __forceinline__ int xcd_linear_block(int b, int nblk) {
  return (nblk % 8 == 0) ? (b % 8) * (nblk / 8) + b / 8 : b;
}

// Thread t * TC + c works on element rows t + G m of column c, so that the TC
// columns of a row are read by adjacent lanes.  A block of at most 64 threads
// is one wavefront, and its transforms then synchronise at wavefront level.
template <typename R, int N, int G, int TC, bool LATE_MY = false>
__device__ __forceinline__ void col_body(const ColArgs<R>& p) {
  constexpr bool WAVE = G * TC <= 64;
  constexpr int E = N / G;
  constexpr int P = padded_len<N>();
  // a transform of at most two Stockham passes writes and reads only b1, so
  // b0 can share its buffer
  constexpr int LB = stockham_passes<N / G, N>() > 2 ? 2 : 1;
  __shared__ cx<R> lds[LB][P * TC];
  const int c = threadIdx.x % TC;
  const int t = threadIdx.x / TC;
  const int lin = xcd_linear_block(blockIdx.x, gridDim.x);
  // two fields: the block's field by a comparison (no integer division) and
  // its pointers chosen arithmetically among the kernel arguments (no
  // dependent load ahead of the field loads); element offsets fit in 32 bits
  // (a field holds at most 512 x 512 elements)
  const int field = lin >= p.tiles ? 1 : 0;
  const int tile = lin - field * p.tiles;
  const int x = tile * TC + c;
  const auto fld = gp(pick_ptr_uniform(field, p.f[0], p.f[1]));
  const unsigned o0 = (unsigned)x + (unsigned)t * (unsigned)p.nx;
  const unsigned og = (unsigned)(G * p.nx);
  cx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = gload(fld + (o0 + (unsigned)m * og));
  // diffraction + linear loss (Eq. A.4): the FP64 product m_x m_y of this
  // thread's bins, formed before the transforms so that its loads overlap FFT_y
  const auto mxp = gp(pick_ptr_uniform(field, p.mx[0], p.mx[1]));
  const auto myp = gp(pick_ptr_uniform(field, p.my[0], p.my[1]));
  const double sgn = p.conj_prop ? -1.0 : 1.0;
  const double mxr = mxp[2 * x], mxi = sgn * mxp[2 * x + 1];
  const LdsView<R, TC> b0{&lds[0][c]}, b1{&lds[LB - 1][c]};
  TwRegs<R, N, G> twr;
  tw_load(twr, t, p.tw);
  // LATE_MY (the batch passes, bound by throughput): m_y is read after FFT_y,
  // which keeps the 4 E registers of the product free for more resident
  // wavefronts; the arithmetic is the same
  if constexpr (!LATE_MY) {
    double mr[E], mi[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int qy = t + G * m;
      const double myr = myp[2 * qy], myi = sgn * myp[2 * qy + 1];
      mr[m] = mxr * myr - mxi * myi;
      mi[m] = mxr * myi + mxi * myr;
    }
    fft_pre<R, N, G, false, TC, WAVE>(v, b0, b1, t, twr);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const double vr = (double)v[m].re, vi = (double)v[m].im;
      v[m] = {(R)(vr * mr[m] - vi * mi[m]), (R)(vr * mi[m] + vi * mr[m])};
    }
  } else {
    fft_pre<R, N, G, false, TC, WAVE>(v, b0, b1, t, twr);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int qy = t + G * m;
      const double myr = myp[2 * qy], myi = sgn * myp[2 * qy + 1];
      const double mr = mxr * myr - mxi * myi, mi = mxr * myi + mxi * myr;
      const double vr = (double)v[m].re, vi = (double)v[m].im;
      v[m] = {(R)(vr * mr - vi * mi), (R)(vr * mi + vi * mr)};
    }
  }
  fft_pre<R, N, G, true, TC, WAVE>(v, b0, b1, t, twr);
#pragma unroll
  for (int m = 0; m < E; ++m) gstore(fld + (o0 + (unsigned)m * og), v[m]);
}

template <typename R, int N, int G, int TC>
__global__ void __launch_bounds__(G * TC) col_pass(ColArgs<R> p) {
  col_body<R, N, G, TC>(p);
}

// ---------------------------------------------------------------- phase table
// Accumulated mismatch phase (Eq. 3) for a mismatch constant within each step:
// Phi_s = sum_{s' < s} dk_s' dz (FP64 chunked scan in one block), and the
// coupling factors at phi = Phi_s + dk_s k dz / 4, k = 0..4: out[5 s + k] =
// {i kf exp(-i phi), i ks exp(+i phi)}, formed in FP64 and rounded once.
template <typename R>
__device__ __forceinline__ void phase_table_body(const double* __restrict__ dk_z, double dk0,
                                                 int nz, double dz, double kf, double ks,
                                                 StageCoef<R>* __restrict__ out) {
  __shared__ double part[256];
  const auto dkg = gp(dk_z);
  const auto og = gp(out);
  const int tid = threadIdx.x;
  const int chunk = (nz + 255) / 256;
  const int s0 = min(nz, tid * chunk), s1 = min(nz, s0 + chunk);
  double sum = 0.0;
  for (int s = s0; s < s1; ++s) sum += (dk_z ? dkg[s] : dk0) * dz;
  part[tid] = sum;
  __syncthreads();
  if (tid == 0) {
    double acc = 0.0;
    for (int i = 0; i < 256; ++i) {
      const double v = part[i];
      part[i] = acc;
      acc += v;
    }
  }
  __syncthreads();
  double phi = part[tid];
  for (int s = s0; s < s1; ++s) {
    const double dk = dk_z ? dkg[s] : dk0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double sn, cs;
      sincos(phi + dk * (0.25 * k * dz), &sn, &cs);
      // e = cs - i sn: i kf e = kf (sn + i cs), i ks conj(e) = ks (-sn + i cs)
      gstore(og + (5 * s + k),
             StageCoef<R>{{(R)(kf * sn), (R)(kf * cs)}, {(R)(-ks * sn), (R)(ks * cs)}});
    }
    phi += dk * dz;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) phase_table(const double* __restrict__ dk_z, double dk0,
                                                   int nz, double dz, double kf, double ks,
                                                   StageCoef<R>* __restrict__ out) {
  phase_table_body<R>(dk_z, dk0, nz, dz, kf, ks, out);
}

// ---------------------------------------------------------------- powers
// Fixed-order sum of the per-block partials; P_j = scale_j * sum |A_j|^2.
static __global__ void __launch_bounds__(256) power_finalize(const double* __restrict__ partials, int n,
                                                      double scale_f, double scale_sh,
                                                      double* __restrict__ powers) {
  __shared__ double red[8];
  double x = 0.0, y = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    x += partials[2 * i];
    y += partials[2 * i + 1];
  }
  block_sum2<256>(x, y, red);
  if (threadIdx.x == 0) {
    powers[0] = x * scale_f;
    powers[1] = y * scale_sh;
  }
}

}  // namespace shg

namespace shg {

// ---------------------------------------------------------------- batches
// One instance of a batched march.  Instances of one launch share the grid
// size and the schedule; blockIdx.y selects the instance.  The host orders a
// size group by decreasing nz, so the instances still marching at boundary s
// are a prefix and a launch simply covers gridDim.y of them.
template <typename R>
struct BatchInst {
  RowArgs<R> row;         // pointers and coefficients (mode fields set per launch)
  ColArgs<R> col;
  const double* dk_z;     // per-step mismatch or null
  double dk0, dz;
  double pscale_f, pscale_sh;
  double* partials;       // [row blocks][2]
  double* powers;         // [2] or null
  int nz;
  int row_blocks;
  int lnl;                // L/2 - N - L/2 order
  const double* mxh[2];   // half-step propagator factors (lnl)
  const double* myh[2];
};

// Roles of the row pass at boundary s of one instance.
//   N/2 - L - N/2 (0 <= s <= nz): second half-step of s-1 when s >= 1, first
//     half-step of s when s < nz; the last boundary leaves real space and
//     writes the power partials.
//   L/2 - N - L/2: s = -1 is the opening FFT_x; 0 <= s < nz runs the whole
//     step s between IFFT_x and FFT_x; s = nz is the closing IFFT_x.
template <typename R>
__device__ __forceinline__ void batch_row_roles(const BatchInst<R>& I, int s, RowArgs<R>& p) {
  const int nz = I.nz;
  if (I.lnl) {
    p.full = 1;
    p.s_second = -1;
    p.s_first = (s >= 0 && s < nz) ? s : -1;
    p.inv_in = s >= 0 ? 1 : 0;
    p.fwd_out = s < nz ? 1 : 0;
  } else {
    p.full = 0;
    p.s_second = s >= 1 ? s - 1 : -1;
    p.s_first = s < nz ? s : -1;
    p.inv_in = s >= 1 ? 1 : 0;
    p.fwd_out = s < nz ? 1 : 0;
  }
  p.partials = (s == nz && I.powers) ? I.partials : nullptr;
}

template <typename R, int N, int G, int ROWS>
__global__ void __launch_bounds__(G * ROWS) row_pass_batch(const BatchInst<R>* __restrict__ inst,
                                                           int s) {
  const BatchInst<R>& I = inst[blockIdx.y];
  RowArgs<R> p = I.row;
  batch_row_roles(I, s, p);
  row_body<R, N, G, ROWS>(p, blockIdx.x);
}

template <typename R, int N>
__global__ void __launch_bounds__(WideShape<N>::threads) row_pass_batch_wide(
    const BatchInst<R>* __restrict__ inst, int s) {
  const BatchInst<R>& I = inst[blockIdx.y];
  RowArgs<R> p = I.row;
  batch_row_roles(I, s, p);
  row_wide_body<R, N, false>(p, blockIdx.x);
}

// Batch column passes of 16 elements per thread on 256-point columns need
// about 170 VGPRs; a bound of three wavefronts per SIMD keeps them at 168
// (three resident wavefronts instead of two).
template <int N, int G>
struct ColBatchWaves {
  static constexpr int value = (N == 256 && N / G == 16) ? 3 : 1;
};

// Column pass after row boundary s: the full-step propagator, or in the
// L/2 - N - L/2 order the half-step one for the opening (s = -1) and the
// instance's last step (s = nz - 1).
template <typename R, int N, int G, int TC>
__global__ void __launch_bounds__(G * TC, (ColBatchWaves<N, G>::value))
    col_pass_batch(const BatchInst<R>* __restrict__ inst, int s) {
  const BatchInst<R>& I = inst[blockIdx.y];
  if (I.lnl && (s < 0 || s == I.nz - 1)) {
    ColArgs<R> c = I.col;
    for (int w = 0; w < 2; ++w) {
      c.mx[w] = I.mxh[w];
      c.my[w] = I.myh[w];
    }
    col_body<R, N, G, TC, true>(c);
  } else {
    col_body<R, N, G, TC, true>(I.col);
  }
}

template <typename R>
__global__ void __launch_bounds__(256) phase_table_batch(const BatchInst<R>* __restrict__ inst) {
  const BatchInst<R>& I = inst[blockIdx.x];
  phase_table_body<R>(I.dk_z, I.dk0, I.nz, I.dz, (double)I.row.kf, (double)I.row.ks,
                      const_cast<StageCoef<R>*>(I.row.phase));
}

template <typename R>
__global__ void __launch_bounds__(256) power_finalize_batch(const BatchInst<R>* __restrict__ inst) {
  __shared__ double red[8];
  const BatchInst<R>& I = inst[blockIdx.x];
  if (!I.powers) return;
  const auto part = gp(I.partials);
  double x = 0.0, y = 0.0;
  for (int i = threadIdx.x; i < I.row_blocks; i += 256) {
    x += part[2 * i];
    y += part[2 * i + 1];
  }
  block_sum2<256>(x, y, red);
  if (threadIdx.x == 0) {
    const auto pw = gp(I.powers);
    pw[0] = x * I.pscale_f;
    pw[1] = y * I.pscale_sh;
  }
}

}  // namespace shg
