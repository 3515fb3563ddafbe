// Kernels of the reverse (adjoint) march.
//
// The forward step y_s -> N1 -> v_s -> L -> u_s -> N2 -> y_{s+1} (N1, N2 the RK4
// half-steps, L the Fourier-space linear step) is pulled back as
//   lambda_u = N2^T(lambda_y),  lambda_v = L^H(lambda_u),  lambda_y = N1^T(lambda_v).
// L^H = IFFT2(conj(M) FFT2(.)), so the adjoint column pass is the forward column
// pass with conj(M).  The adjoint row pass mirrors the forward row pass: load
// lambda, IFFT_x, pull back through the first half-step of step s and the second
// half-step of step s-1 (recomputing their stage states from the staged forward
// state u_{s-1}), FFT_x, store.  Complex gradients use the convention
// g = dL/dRe + i dL/dIm, for which a complex-linear map pulls back by its
// Hermitian adjoint and a pointwise map f(a, conj a) by
//   g_a = g_f conj(df/da) + conj(g_f) df/d(conj a).
#pragma once
#include "kernels.hpp"

namespace shg {

// Pull the cotangent (ka, kb) of f = N(a, b) back to (a, b).
//   fa = cf b conj(a) - tf |a|^2 a:  dfa/da = -2 tf |a|^2, dfa/dconj(a) = cf b - tf a^2,
//                                    dfa/db = cf conj(a)
//   fb = cs a^2 - ts |b|^2 b:        dfb/da = 2 cs a, dfb/db = -2 ts |b|^2,
//                                    dfb/dconj(b) = -ts b^2
// Also returns the derivative of L along the mismatch phase phi
// (dfa/dphi = -i cf b conj(a), dfb/dphi = +i cs a^2): Re(conj(k) . df/dphi).
template <typename R>
__device__ __forceinline__ void nl_vjp(cx<R> a, cx<R> b, cx<R> cf, cx<R> cs, R tf, R ts, bool und,
                                       cx<R> ka, cx<R> kb, cx<R>& ga, cx<R>& gb, R& dphi) {
  const cx<R> a2 = {a.re * a.re - a.im * a.im, (a.re + a.re) * a.im};
  const cx<R> b2 = {b.re * b.re - b.im * b.im, (b.re + b.re) * b.im};
  const cx<R> cs_a2 = cs * a2;
  // from fb
  ga = scale(mul_conj(kb, cs) * conjg(a), (R)2);                       // kb 2 conj(cs) conj(a)
  gb = scale(kb, (R)-2 * ts * norm2(b)) + conjg(kb) * scale(b2, -ts);
  dphi = -(kb.re * cs_a2.im - kb.im * cs_a2.re);                       // -Im(conj(kb) cs a^2)
  if (!und) {
    const cx<R> cf_bca = cf * mul_conj(b, a);                           // cf b conj(a)
    ga = ga + scale(ka, (R)-2 * tf * norm2(a)) + conjg(ka) * (cf * b - scale(a2, tf));
    gb = gb + mul_conj(ka, cf) * a;                                     // ka conj(cf) a
    dphi += ka.re * cf_bca.im - ka.im * cf_bca.re;                      // Im(conj(ka) cf b conj(a))
  }
}

// Stage inputs u2, u3, u4 of one RK4 half-step (u1 is its input).
template <typename R>
struct Rk4Stages {
  cx<R> u2a, u2b, u3a, u3b, u4a, u4b;
};

// The forward half-step of rk4_cell that also keeps its stage inputs, for a
// later pull-back through the same half-step.
template <bool UND, typename R>
__device__ __forceinline__ void rk4_cell_keep_u(cx<R>& a, cx<R>& b, const HalfStep<R>& c, R tf,
                                                R ts, R h, Rk4Stages<R>& st) {
  const R h2 = h * (R)0.5;
  cx<R> k1a, k1b, k2a, k2b, k3a, k3b, k4a, k4b;
  nl_rhs(a, b, c.cf[0], c.cs[0], tf, ts, UND, k1a, k1b);
  st.u2a = a + scale(k1a, h2);
  st.u2b = b + scale(k1b, h2);
  nl_rhs(st.u2a, st.u2b, c.cf[1], c.cs[1], tf, ts, UND, k2a, k2b);
  st.u3a = a + scale(k2a, h2);
  st.u3b = b + scale(k2b, h2);
  nl_rhs(st.u3a, st.u3b, c.cf[1], c.cs[1], tf, ts, UND, k3a, k3b);
  st.u4a = a + scale(k3a, h);
  st.u4b = b + scale(k3b, h);
  nl_rhs(st.u4a, st.u4b, c.cf[2], c.cs[2], tf, ts, UND, k4a, k4b);
  const R h6 = h * (R)(1.0 / 6.0);
  a = a + scale(k1a + scale(k2a + k3a, (R)2) + k4a, h6);
  b = b + scale(k1b + scale(k2b + k3b, (R)2) + k4b, h6);
}

// Reverse of one RK4 half-step whose stage inputs are known.
// (a, b)    in: input state y of the half-step; st its stage inputs
// (la, lb)  in: cotangent of the output; out: cotangent of the input
// gphi, gphit accumulate dL/dphi and dL/dphi * t over the four stages, where
// the stage points are t0, t0 + h/2, t0 + h/2, t0 + h.
template <bool UND, typename R>
__device__ __forceinline__ void rk4_vjp_from_u(cx<R> a, cx<R> b, const Rk4Stages<R>& st,
                                               cx<R>& la, cx<R>& lb, const HalfStep<R>& c, R tf,
                                               R ts, R h, R t0, R& gphi, R& gphit) {
  const R h2 = h * (R)0.5;
  const cx<R> u2a = st.u2a, u2b = st.u2b, u3a = st.u3a, u3b = st.u3b, u4a = st.u4a,
              u4b = st.u4b;
  const R h6 = h * (R)(1.0 / 6.0), h3 = h * (R)(1.0 / 3.0);
  cx<R> ga, gb;
  R dp;
  // stage 4
  cx<R> kba = scale(la, h6), kbb = scale(lb, h6);
  nl_vjp(u4a, u4b, c.cf[2], c.cs[2], tf, ts, UND, kba, kbb, ga, gb, dp);
  cx<R> sa = ga, sb = gb;
  gphi += dp;
  gphit += dp * (t0 + h);
  // stage 3
  kba = scale(la, h3) + scale(ga, h);
  kbb = scale(lb, h3) + scale(gb, h);
  nl_vjp(u3a, u3b, c.cf[1], c.cs[1], tf, ts, UND, kba, kbb, ga, gb, dp);
  sa = sa + ga;
  sb = sb + gb;
  gphi += dp;
  gphit += dp * (t0 + h2);
  // stage 2
  kba = scale(la, h3) + scale(ga, h2);
  kbb = scale(lb, h3) + scale(gb, h2);
  nl_vjp(u2a, u2b, c.cf[1], c.cs[1], tf, ts, UND, kba, kbb, ga, gb, dp);
  sa = sa + ga;
  sb = sb + gb;
  gphi += dp;
  gphit += dp * (t0 + h2);
  // stage 1
  kba = scale(la, h6) + scale(ga, h2);
  kbb = scale(lb, h6) + scale(gb, h2);
  nl_vjp(a, b, c.cf[0], c.cs[0], tf, ts, UND, kba, kbb, ga, gb, dp);
  sa = sa + ga;
  sb = sb + gb;
  gphi += dp;
  gphit += dp * t0;
  la = la + sa;
  lb = lb + sb;
}
// Reverse of one RK4 half-step with its stage inputs recomputed from y.
template <bool UND, typename R>
__device__ __forceinline__ void rk4_vjp_u(cx<R> a, cx<R> b, cx<R>& la, cx<R>& lb,
                                        const HalfStep<R>& c, R tf, R ts, R h, R t0,
                                        R& gphi, R& gphit) {
  const R h2 = h * (R)0.5;
  cx<R> k1a, k1b, k2a, k2b, k3a, k3b;
  Rk4Stages<R> st;
  nl_rhs(a, b, c.cf[0], c.cs[0], tf, ts, UND, k1a, k1b);
  st.u2a = a + scale(k1a, h2);
  st.u2b = b + scale(k1b, h2);
  nl_rhs(st.u2a, st.u2b, c.cf[1], c.cs[1], tf, ts, UND, k2a, k2b);
  st.u3a = a + scale(k2a, h2);
  st.u3b = b + scale(k2b, h2);
  nl_rhs(st.u3a, st.u3b, c.cf[1], c.cs[1], tf, ts, UND, k3a, k3b);
  st.u4a = a + scale(k3a, h);
  st.u4b = b + scale(k3b, h);
  rk4_vjp_from_u<UND>(a, b, st, la, lb, c, tf, ts, h, t0, gphi, gphit);
}
template <typename R>
__device__ __forceinline__ void rk4_vjp(cx<R> a, cx<R> b, cx<R>& la, cx<R>& lb,
                                        const HalfStep<R>& c, R tf, R ts, R h, bool und, R t0,
                                        R& gphi, R& gphit) {
  if (und) rk4_vjp_u<true>(a, b, la, lb, c, tf, ts, h, t0, gphi, gphit);
  else rk4_vjp_u<false>(a, b, la, lb, c, tf, ts, h, t0, gphi, gphit);
}
template <typename R>
__device__ __forceinline__ void rk4_cell_keep(cx<R>& a, cx<R>& b, const HalfStep<R>& c, R tf,
                                              R ts, R h, bool und, Rk4Stages<R>& st) {
  if (und) rk4_cell_keep_u<true>(a, b, c, tf, ts, h, st);
  else rk4_cell_keep_u<false>(a, b, c, tf, ts, h, st);
}
template <typename R>
__device__ __forceinline__ void rk4_vjp_from(cx<R> a, cx<R> b, const Rk4Stages<R>& st, cx<R>& la,
                                             cx<R>& lb, const HalfStep<R>& c, R tf, R ts, R h,
                                             bool und, R t0, R& gphi, R& gphit) {
  if (und) rk4_vjp_from_u<true>(a, b, st, la, lb, c, tf, ts, h, t0, gphi, gphit);
  else rk4_vjp_from_u<false>(a, b, st, la, lb, c, tf, ts, h, t0, gphi, gphit);
}

template <typename R>
struct RowAdjArgs {
  cx<R>* la;              // cotangent, F (in place)
  cx<R>* lb;              // cotangent, SH
  const cx<R>* ua;        // forward state: u_{s_second} if s_second >= 0, else y_{s_first}
  const cx<R>* ub;
  const Tw<R>* tw;
  const StageCoef<R>* phase;  // [nz][5] coupling factors at the stage points
  double* gp_first;       // [gridDim.x][2] {dL/dphi, dL/dphi * t} of the first half-step, or null
  double* gp_second;      // same for the second half-step, or null
  int ny;
  int s_second;           // step whose second half-step is pulled back, or -1
  int s_first;            // step whose first half-step is pulled back, or -1
  int inv_in;             // lambda arrives in the (q_x, y) domain: apply IFFT_x on load
  int fwd_out;            // apply FFT_x before storing (lambda leaves in the (q_x, y) domain)
  int full;               // s_first is a whole step over 2h (L/2 - N - L/2 order)
  R kf, ks, tf, ts, h;
  int undepleted;
};

// Fixed-order block reduction of four doubles; result valid in thread 0.
template <int T>
__device__ __forceinline__ void block_sum4(double (&v)[4], double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] += __shfl_down(v[i], off, 64);
  }
  constexpr int W = (T + 63) / 64;
  if constexpr (W > 1) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) red[4 * w + i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = 0.0;
      for (int j = 0; j < W; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] += red[4 * j + i];
      }
    }
  }
}

// lambda = g_out + 2 w_j c_j A_j(L): cotangent of the exit fields for the loss
// Re<g_out, A(L)> + w_F P_F + w_SH P_SH, P_j = c_j sum |A_j|^2.
template <typename R>
__global__ void __launch_bounds__(256) adjoint_seed(const cx<R>* __restrict__ gf,
                                                    const cx<R>* __restrict__ gs,
                                                    const cx<R>* __restrict__ af,
                                                    const cx<R>* __restrict__ as,
                                                    const double* __restrict__ w, double cf,
                                                    double cs, cx<R>* __restrict__ lf,
                                                    cx<R>* __restrict__ ls, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const R wf = w ? (R)(2.0 * w[0] * cf) : (R)0;
  const R ws = w ? (R)(2.0 * w[1] * cs) : (R)0;
  cx<R> x = scale(af[i], wf), y = scale(as[i], ws);
  if (gf) x = x + gf[i];
  if (gs) y = y + gs[i];
  lf[i] = x;
  ls[i] = y;
}

// Per-step totals: gh[s] = {sum dL/dphi, sum dL/dphi * t} over both half-steps
// of step s and all blocks (fixed order).  One block per step.
static __global__ void __launch_bounds__(256) grad_step_sums(const double* __restrict__ first,
                                                      const double* __restrict__ second,
                                                      int nblk, double* __restrict__ gh) {
  __shared__ double red[8];
  const int s = blockIdx.x;
  const double* f = first + (size_t)s * nblk * 2;
  const double* q = second ? second + (size_t)s * nblk * 2 : nullptr;   // null: one pass per step
  double x = 0.0, y = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) {
    x += f[2 * i] + (q ? q[2 * i] : 0.0);
    y += f[2 * i + 1] + (q ? q[2 * i + 1] : 0.0);
  }
  block_sum2<256>(x, y, red);
  if (threadIdx.x == 0) {
    gh[2 * s] = x;
    gh[2 * s + 1] = y;
  }
}

// dL/d dk_s = H_s + dz * sum_{s' > s} G_s'   (phi on step s is Phi_s + dk_s t,
// Phi_s = sum_{s' < s} dk_s' dz).  Chunked suffix scan in one block.
static __global__ void __launch_bounds__(256) grad_dk_finalize(const double* __restrict__ gh, int nz,
                                                        double dz, double* __restrict__ g_dk) {
  __shared__ double part[256];
  const int tid = threadIdx.x;
  const int chunk = (nz + 255) / 256;
  const int s0 = min(nz, tid * chunk), s1 = min(nz, s0 + chunk);
  double sum = 0.0;
  for (int s = s0; s < s1; ++s) sum += gh[2 * s];
  part[tid] = sum;
  __syncthreads();
  if (tid == 0) {
    double acc = 0.0;
    for (int i = 255; i >= 0; --i) {
      const double v = part[i];
      part[i] = acc;       // sum over later chunks
      acc += v;
    }
  }
  __syncthreads();
  double later = part[tid];
  for (int s = s1 - 1; s >= s0; --s) {
    g_dk[s] = gh[2 * s + 1] + dz * later;
    later += gh[2 * s];
  }
}

}  // namespace shg

namespace shg {

// ---------------------------------------------------------------- temperature
// nl_vjp with the thermal-lens terms -i g A (dfa/da += -i gF, dfb/db += -i gS)
// and the derivative along the lens strength dT:
// dlens = Re(conj(ka)(-i gF/dT a) + conj(kb)(-i gS/dT b)), returned per unit dT
// through lf, ls (the lens coefficients g_j of the plan).
template <typename R>
__device__ __forceinline__ void nl_vjp_t(cx<R> a, cx<R> b, cx<R> cf, cx<R> cs, R tf, R ts, R gf,
                                         R gs, R lf, R ls, bool und, cx<R> ka, cx<R> kb,
                                         cx<R>& ga, cx<R>& gb, R& dphi, R& dlens) {
  nl_vjp(a, b, cf, cs, tf, ts, und, ka, kb, ga, gb, dphi);
  // k * conj(-i g) = k * (i g)
  gb = gb + cx<R>{-gs * kb.im, gs * kb.re};
  dlens = ls * (kb.re * b.im - kb.im * b.re);          // Im(conj(kb) b) * g_SH
  if (!und) {
    ga = ga + cx<R>{-gf * ka.im, gf * ka.re};
    dlens += lf * (ka.re * a.im - ka.im * a.re);
  }
}

// rk4_cell_t keeping its stage inputs (see rk4_cell_keep_u).
template <bool UND, typename R>
__device__ __forceinline__ void rk4_cell_t_keep_u(cx<R>& a, cx<R>& b, const HalfStepT<R>& c, R tf,
                                                  R ts, R h, Rk4Stages<R>& st) {
  const R h2 = h * (R)0.5;
  cx<R> k1a, k1b, k2a, k2b, k3a, k3b, k4a, k4b;
  nl_rhs_t(a, b, c.cf[0], c.cs[0], tf, ts, c.gf, c.gs, UND, k1a, k1b);
  st.u2a = a + scale(k1a, h2);
  st.u2b = b + scale(k1b, h2);
  nl_rhs_t(st.u2a, st.u2b, c.cf[1], c.cs[1], tf, ts, c.gf, c.gs, UND, k2a, k2b);
  st.u3a = a + scale(k2a, h2);
  st.u3b = b + scale(k2b, h2);
  nl_rhs_t(st.u3a, st.u3b, c.cf[1], c.cs[1], tf, ts, c.gf, c.gs, UND, k3a, k3b);
  st.u4a = a + scale(k3a, h);
  st.u4b = b + scale(k3b, h);
  nl_rhs_t(st.u4a, st.u4b, c.cf[2], c.cs[2], tf, ts, c.gf, c.gs, UND, k4a, k4b);
  const R h6 = h * (R)(1.0 / 6.0);
  a = a + scale(k1a + scale(k2a + k3a, (R)2) + k4a, h6);
  b = b + scale(k1b + scale(k2b + k3b, (R)2) + k4b, h6);
}

// rk4_vjp_from_u with the temperature-field terms (lens rates and their
// derivative glens).
template <bool UND, typename R>
__device__ __forceinline__ void rk4_vjp_t_from_u(cx<R> a, cx<R> b, const Rk4Stages<R>& st,
                                                 cx<R>& la, cx<R>& lb, const HalfStepT<R>& c,
                                                 R tf, R ts, R lf, R ls, R h, R t0, R& gphi,
                                                 R& gphit, R& glens) {
  const R h2 = h * (R)0.5;
  const cx<R> u2a = st.u2a, u2b = st.u2b, u3a = st.u3a, u3b = st.u3b, u4a = st.u4a,
              u4b = st.u4b;
  const R h6 = h * (R)(1.0 / 6.0), h3 = h * (R)(1.0 / 3.0);
  cx<R> ga, gb;
  R dp, dl;
  cx<R> kba = scale(la, h6), kbb = scale(lb, h6);
  nl_vjp_t(u4a, u4b, c.cf[2], c.cs[2], tf, ts, c.gf, c.gs, lf, ls, UND, kba, kbb, ga, gb, dp, dl);
  cx<R> sa = ga, sb = gb;
  gphi += dp;
  gphit += dp * (t0 + h);
  glens += dl;
  kba = scale(la, h3) + scale(ga, h);
  kbb = scale(lb, h3) + scale(gb, h);
  nl_vjp_t(u3a, u3b, c.cf[1], c.cs[1], tf, ts, c.gf, c.gs, lf, ls, UND, kba, kbb, ga, gb, dp, dl);
  sa = sa + ga;
  sb = sb + gb;
  gphi += dp;
  gphit += dp * (t0 + h2);
  glens += dl;
  kba = scale(la, h3) + scale(ga, h2);
  kbb = scale(lb, h3) + scale(gb, h2);
  nl_vjp_t(u2a, u2b, c.cf[1], c.cs[1], tf, ts, c.gf, c.gs, lf, ls, UND, kba, kbb, ga, gb, dp, dl);
  sa = sa + ga;
  sb = sb + gb;
  gphi += dp;
  gphit += dp * (t0 + h2);
  glens += dl;
  kba = scale(la, h6) + scale(ga, h2);
  kbb = scale(lb, h6) + scale(gb, h2);
  nl_vjp_t(a, b, c.cf[0], c.cs[0], tf, ts, c.gf, c.gs, lf, ls, UND, kba, kbb, ga, gb, dp, dl);
  sa = sa + ga;
  sb = sb + gb;
  gphi += dp;
  gphit += dp * t0;
  glens += dl;
  la = la + sa;
  lb = lb + sb;
}
// Reverse of one temperature-field RK4 half-step, stage inputs recomputed.
template <bool UND, typename R>
__device__ __forceinline__ void rk4_vjp_t_u(cx<R> a, cx<R> b, cx<R>& la, cx<R>& lb,
                                            const HalfStepT<R>& c, R tf, R ts, R lf, R ls, R h,
                                            R t0, R& gphi, R& gphit, R& glens) {
  const R h2 = h * (R)0.5;
  cx<R> k1a, k1b, k2a, k2b, k3a, k3b;
  Rk4Stages<R> st;
  nl_rhs_t(a, b, c.cf[0], c.cs[0], tf, ts, c.gf, c.gs, UND, k1a, k1b);
  st.u2a = a + scale(k1a, h2);
  st.u2b = b + scale(k1b, h2);
  nl_rhs_t(st.u2a, st.u2b, c.cf[1], c.cs[1], tf, ts, c.gf, c.gs, UND, k2a, k2b);
  st.u3a = a + scale(k2a, h2);
  st.u3b = b + scale(k2b, h2);
  nl_rhs_t(st.u3a, st.u3b, c.cf[1], c.cs[1], tf, ts, c.gf, c.gs, UND, k3a, k3b);
  st.u4a = a + scale(k3a, h);
  st.u4b = b + scale(k3b, h);
  rk4_vjp_t_from_u<UND>(a, b, st, la, lb, c, tf, ts, lf, ls, h, t0, gphi, gphit, glens);
}
template <typename R>
__device__ __forceinline__ void rk4_vjp_t(cx<R> a, cx<R> b, cx<R>& la, cx<R>& lb,
                                          const HalfStepT<R>& c, R tf, R ts, R lf, R ls, R h,
                                          bool und, R t0, R& gphi, R& gphit, R& glens) {
  if (und) rk4_vjp_t_u<true>(a, b, la, lb, c, tf, ts, lf, ls, h, t0, gphi, gphit, glens);
  else rk4_vjp_t_u<false>(a, b, la, lb, c, tf, ts, lf, ls, h, t0, gphi, gphit, glens);
}
template <typename R>
__device__ __forceinline__ void rk4_cell_t_keep(cx<R>& a, cx<R>& b, const HalfStepT<R>& c, R tf,
                                                R ts, R h, bool und, Rk4Stages<R>& st) {
  if (und) rk4_cell_t_keep_u<true>(a, b, c, tf, ts, h, st);
  else rk4_cell_t_keep_u<false>(a, b, c, tf, ts, h, st);
}
template <typename R>
__device__ __forceinline__ void rk4_vjp_t_from(cx<R> a, cx<R> b, const Rk4Stages<R>& st,
                                               cx<R>& la, cx<R>& lb, const HalfStepT<R>& c, R tf,
                                               R ts, R lf, R ls, R h, bool und, R t0, R& gphi,
                                               R& gphit, R& glens) {
  if (und) rk4_vjp_t_from_u<true>(a, b, st, la, lb, c, tf, ts, lf, ls, h, t0, gphi, gphit, glens);
  else rk4_vjp_t_from_u<false>(a, b, st, la, lb, c, tf, ts, lf, ls, h, t0, gphi, gphit, glens);
}

// Per-cell carry of the thermal reverse sweep:
//   x = sum over later steps of dL/dphi (the Psi dependence),
//   y, z, w = dL/dphi, dL/dphi * tau and dL/d(dT) through the lens of the
//             second half-step of the step whose first half comes next.
template <typename R>
struct Carry {
  R x, y, z, w;
};

template <typename R>
struct RowAdjTArgs {
  const R* temp;          // [nz][ny][nx]
  const R* psi;           // Psi at the start of step s_second (or s_first when s_second < 0)
  Carry<R>* carry;        // [ny][nx]
  double* moments;        // [ny][nx][2] running sum of dL/dT (T - T_ref) and dL/dT
  R t_ref, lens_f, lens_sh, dz;
  DkT<R> dk;              // mismatch shift of each cell's temperature
};

// Per-cell inputs of the adjoint row pass that do not depend on the
// cotangent: the staged forward state, the stage coefficients and, with a
// temperature field, Psi, the carry and the two samples.  Loading them before
// the cotangent's transform lets their latency overlap it.
template <typename R, bool TH>
struct AdjPre {
  cx<R> ua, ub;
  HalfStep<R> c1, c2;        // coupling factors of both half-steps
  R psi, t2, t1;             // Psi and the raw samples T of both steps
  Carry<R> cr;
};

// The table values (scalar loads), then the per-cell values (vector loads).
// All unconditional (a step index < 0 reads step 0, unused) and raw, so that
// no wait on them stands before the loads that follow them.
template <typename R, bool TH>
__device__ __forceinline__ void adj_load_table(const RowAdjArgs<R>& p, AdjPre<R, TH>& a) {
  a.c1 = half_step_coefs<R>(gp(p.phase) + 5 * max(p.s_first, 0), p.full ? 2 : 1);
  a.c2 = half_step_coefs<R>(gp(p.phase) + 5 * max(p.s_second, 0) + 2);
}
template <typename R, bool TH>
__device__ __forceinline__ void adj_load_cell(const RowAdjArgs<R>& p, const RowAdjTArgs<R>& q,
                                              size_t idx, size_t n2, AdjPre<R, TH>& a) {
  a.ua = p.ua[idx];
  a.ub = p.ub[idx];
  if constexpr (TH) {
    a.psi = q.psi[idx];
    a.cr = q.carry[idx];
    a.t2 = q.temp[(size_t)max(p.s_second, 0) * n2 + idx];
    a.t1 = q.temp[(size_t)max(p.s_first, 0) * n2 + idx];
  }
}
template <typename R, bool TH>
__device__ __forceinline__ AdjPre<R, TH> adj_load(const RowAdjArgs<R>& p, const RowAdjTArgs<R>& q,
                                                  size_t idx, size_t n2) {
  AdjPre<R, TH> a{};
  adj_load_table<R, TH>(p, a);
  adj_load_cell<R, TH>(p, q, idx, n2, a);
  return a;
}

// Pull-back of one cell through the first half-step of s_first and the second
// half-step of s_second (either may be absent), from the staged forward state.
template <typename R, bool TH>
__device__ __forceinline__ void adj_cell(const RowAdjArgs<R>& p, const RowAdjTArgs<R>& q,
                                         const AdjPre<R, TH>& pre, size_t idx, cx<R>& la,
                                         cx<R>& lb, double (&acc)[4]) {
  const bool und = p.undepleted != 0;
  const R h = p.h;
  const cx<R> ua = pre.ua;
  const cx<R> ub = pre.ub;
  cx<R> ya = ua, yb = ub;
  if constexpr (!TH) {
    const HalfStep<R>& c1 = pre.c1;
    const HalfStep<R>& c2 = pre.c2;
    // the forward second half-step from u, keeping its stage inputs for its
    // own pull-back below
    Rk4Stages<R> stg2{};
    if (p.s_second >= 0) rk4_cell_keep(ya, yb, c2, p.tf, p.ts, h, und, stg2);
    R g = 0, gt = 0;
    if (p.s_first >= 0) {
      rk4_vjp(ya, yb, la, lb, c1, p.tf, p.ts, p.full ? h + h : h, und, (R)0, g, gt);
      acc[0] += (double)g;
      acc[1] += (double)gt;
    }
    if (p.s_second >= 0) {
      g = 0;
      gt = 0;
      rk4_vjp_from(ua, ub, stg2, la, lb, c2, p.tf, p.ts, h, und, h, g, gt);
      acc[2] += (double)g;
      acc[3] += (double)gt;
    }
  } else {
    const R qdz = q.dz * (R)0.25;
    // the forward pass's stage coefficients, formed the same way
    cx<R> rho = expi_neg(pre.psi);
    Carry<R> cr = pre.cr;
    HalfStepT<R> c2{};
    Rk4Stages<R> stg2{};
    if (p.s_second >= 0) {
      const R dT = pre.t2 - q.t_ref;
      const cx<R> step = expi_neg_small(thermal_dk(dT, q.dk) * qdz), st2 = step * step;
      c2 = thermal_coefs(pre.c2, rho * st2, step, dT, q.lens_f, q.lens_sh);
      rk4_cell_t_keep(ya, yb, c2, p.tf, p.ts, h, und, stg2);
      rho = rho * (st2 * st2);
    }
    if (p.s_first >= 0) {
      const R dT = pre.t1 - q.t_ref;
      const int st = p.full ? 2 : 1;
      const HalfStepT<R> c1 =
          thermal_coefs(pre.c1, rho, expi_neg_small(thermal_dk(dT, q.dk) * (qdz * st)),
                        dT, q.lens_f, q.lens_sh);
      R g = 0, gt = 0, gl = 0;
      rk4_vjp_t(ya, yb, la, lb, c1, p.tf, p.ts, q.lens_f, q.lens_sh, h * (R)st, und, (R)0, g, gt,
                gl);
      acc[0] += (double)g;
      acc[1] += (double)gt;
      // step s_first is complete: its second half-step was pulled back earlier
      const R g_dk = gt + cr.z + q.dz * cr.x;              // dL/d dk_s for this cell
      const R g_t = thermal_dk_slope(dT, q.dk) * g_dk + gl + cr.w;   // dL/dT_s
      cr.x += g + cr.y;
      double* mo = q.moments + 2 * idx;
      mo[0] += (double)g_t * (double)dT;
      mo[1] += (double)g_t;
    }
    if (p.s_second >= 0) {
      R g = 0, gt = 0, gl = 0;
      rk4_vjp_t_from(ua, ub, stg2, la, lb, c2, p.tf, p.ts, q.lens_f, q.lens_sh, h, und, h, g, gt,
                     gl);
      acc[2] += (double)g;
      acc[3] += (double)gt;
      cr.y = g;
      cr.z = gt;
      cr.w = gl;
    } else {
      cr.y = cr.z = cr.w = (R)0;
    }
    q.carry[idx] = cr;
  }
}

template <typename R, bool TH>
__device__ __forceinline__ void adj_cell(const RowAdjArgs<R>& p, const RowAdjTArgs<R>& q,
                                         size_t idx, size_t n2, cx<R>& la, cx<R>& lb,
                                         double (&acc)[4]) {
  adj_cell<R, TH>(p, q, adj_load<R, TH>(p, q, idx, n2), idx, la, lb, acc);
}

template <typename R, int T>
__device__ __forceinline__ void adj_partials(const RowAdjArgs<R>& p, double (&acc)[4], double* red,
                                             int blk) {
  if (p.gp_first || p.gp_second) {
    block_sum4<T>(acc, red);
    if (threadIdx.x == 0) {
      if (p.gp_first) {
        p.gp_first[2 * blk] = acc[0];
        p.gp_first[2 * blk + 1] = acc[1];
      }
      if (p.gp_second) {
        p.gp_second[2 * blk] = acc[2];
        p.gp_second[2 * blk + 1] = acc[3];
      }
    }
  }
}

// The forward row pass is out = FFT_x(N(IFFT_x(in))).  Both transforms are
// unnormalised and the DFT matrix is symmetric, so FFT_x^H = IFFT_x and
// IFFT_x^H = FFT_x: the pull-back applies IFFT_x to the incoming cotangent,
// pulls it through the two half-steps in reverse order, and applies FFT_x before
// storing, the same transform sequence as the forward pass.
template <typename R, int N, int G, int ROWS, bool TH>
__global__ void __launch_bounds__(G * ROWS) row_adj_pass(RowAdjArgs<R> p, RowAdjTArgs<R> q) {
  constexpr int E = N / G;
  constexpr int P = padded_len<N>();
  __shared__ cx<R> lds[ROWS][2][2][P];
  __shared__ double red[4 * ((G * ROWS + 63) / 64)];
  const int t = threadIdx.x % G;
  const int rr = threadIdx.x / G;
  const int y = blockIdx.x * ROWS + rr;
  const size_t row = (size_t)y * N;
  const size_t n2 = (size_t)p.ny * N;
  cx<R> va[E], vb[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    va[m] = p.la[row + t + G * m];
    vb[m] = p.lb[row + t + G * m];
  }
  const LdsView<R, 1> a0{&lds[rr][0][0][0]}, a1{&lds[rr][0][1][0]};
  const LdsView<R, 1> b0{&lds[rr][1][0][0]}, b1{&lds[rr][1][1][0]};
  TwRegs<R, N, G> twr;
  tw_load(twr, t, p.tw);
  if (p.inv_in) {
    fft_pre<R, N, G, true, 1, (G <= 64)>(va, a0, a1, t, twr);
    fft_pre<R, N, G, true, 1, (G <= 64)>(vb, b0, b1, t, twr);
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int m = 0; m < E; ++m) adj_cell<R, TH>(p, q, row + t + G * m, n2, va[m], vb[m], acc);
  if (p.fwd_out) {
    fft_pre<R, N, G, false, 1, (G <= 64)>(va, a0, a1, t, twr);
    fft_pre<R, N, G, false, 1, (G <= 64)>(vb, b0, b1, t, twr);
  }
#pragma unroll
  for (int m = 0; m < E; ++m) {
    p.la[row + t + G * m] = va[m];
    p.lb[row + t + G * m] = vb[m];
  }
  adj_partials<R, G * ROWS>(p, acc, red, blockIdx.x);
}

// Wide variant (one cell per thread for the pull-back; see row_wide_body).
template <typename R, int N, bool TH>
__global__ void __launch_bounds__(WideShape<N>::threads) row_adj_pass_wide(RowAdjArgs<R> p,
                                                                            RowAdjTArgs<R> q) {
  using S = WideShape<N>;
  constexpr int ROWS = S::rows, G = S::g, EF = S::ef;
  constexpr int P = padded_len<N>();
  __shared__ cx<R> cell[2][ROWS][P];
  __shared__ cx<R> pp[2 * ROWS][2][P];
  __shared__ double red[4 * ((S::threads + 63) / 64)];
  const int blk = blockIdx.x;
  const int tid = threadIdx.x;
  const bool fth = tid < S::fft_threads;
  const int tr = transform_index<G>(fth, tid);
  const int t = tid % G;
  const int ff = tr & 1, fr = tr >> 1;
  const size_t frow = (size_t)(blk * ROWS + fr) * N;
  const LdsView<R, 1> q0{&pp[tr][0][0]}, q1{&pp[tr][1][0]};
  const int cr = tid / N, cxi = tid % N;
  const size_t idx = (size_t)(blk * ROWS + cr) * N + cxi;
  const size_t n2 = (size_t)p.ny * N;
  cx<R> v[EF];
  cx<R> la, lb;
  TwRegs<R, N, G> twr;
  if (fth) tw_load(twr, t, p.tw);
  // the table values first; the per-cell inputs after the cotangent loads, so
  // that the transform waits only for the cotangent and they arrive during it
  AdjPre<R, TH> pre{};
  adj_load_table<R, TH>(p, pre);
  if (p.inv_in) {
    if (fth) {
      const auto src = gp(pick_ptr(ff, p.la, p.lb));
#pragma unroll
      for (int m = 0; m < EF; ++m) v[m] = gload(src + (frow + t + G * m));
    }
    adj_load_cell<R, TH>(p, q, idx, n2, pre);
    fft_pre<R, N, G, true, 1, (G <= 64)>(v, q0, q1, t, twr, fth);
    if (fth) {
#pragma unroll
      for (int m = 0; m < EF; ++m) cell[ff][fr][pad16(t + G * m)] = v[m];
    }
    __syncthreads();
    la = cell[0][cr][pad16(cxi)];
    lb = cell[1][cr][pad16(cxi)];
  } else {
    la = gload(gp(p.la) + idx);
    lb = gload(gp(p.lb) + idx);
    adj_load_cell<R, TH>(p, q, idx, n2, pre);
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  adj_cell<R, TH>(p, q, pre, idx, la, lb, acc);
  if (p.fwd_out) {
    // each thread rewrites only the cell it read (no barrier before the write)
    cell[0][cr][pad16(cxi)] = la;
    cell[1][cr][pad16(cxi)] = lb;
    __syncthreads();
    if (fth) {
#pragma unroll
      for (int m = 0; m < EF; ++m) v[m] = cell[ff][fr][pad16(t + G * m)];
    }
    fft_pre<R, N, G, false, 1, (G <= 64)>(v, q0, q1, t, twr, fth);
    if (fth) {
      const auto dst = gp(pick_ptr(ff, p.la, p.lb));
#pragma unroll
      for (int m = 0; m < EF; ++m) gstore(dst + (frow + t + G * m), v[m]);
    }
  } else {
    p.la[idx] = la;
    p.lb[idx] = lb;
  }
  adj_partials<R, S::threads>(p, acc, red, blk);
}

template <typename R>
__global__ void __launch_bounds__(256) zero_carry(Carry<R>* __restrict__ c,
                                                  double* __restrict__ mo, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  c[i] = {(R)0, (R)0, (R)0, (R)0};
  mo[2 * i] = 0.0;
  mo[2 * i + 1] = 0.0;
}

template <typename R>
__global__ void __launch_bounds__(256) copy_real(const R* __restrict__ src, R* __restrict__ dst,
                                                 size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Fixed-order sum of the per-cell moments into out[2] (one block).
static __global__ void __launch_bounds__(256) moments_finalize(const double* __restrict__ mo,
                                                               size_t n, double* __restrict__ out) {
  __shared__ double red[8];
  double x = 0.0, y = 0.0;
  for (size_t i = threadIdx.x; i < n; i += 256) {
    x += mo[2 * i];
    y += mo[2 * i + 1];
  }
  block_sum2<256>(x, y, red);
  if (threadIdx.x == 0) {
    out[0] = x;
    out[1] = y;
  }
}

}  // namespace shg
