// Register + LDS Stockham FFT building blocks for gfx950.
//
// A length-N transform is shared by G threads; thread t holds the E = N/G
// elements x[t + G*m], m = 0..E-1, in registers.  Each radix-R pass takes the
// R inputs of butterfly j from indices j + r*N/R, applies the twiddles
// W_{Ns R}^{(j mod Ns) r}, does an in-register DFT_R and writes the outputs to
// (j div Ns)*Ns*R + (j mod Ns) + r*Ns (Stockham auto-sort).  With this thread
// mapping the first pass reads its inputs straight from registers and the last
// pass writes its outputs straight back into the same stride-G register layout,
// so a transform costs (passes - 1) LDS round trips and forward and inverse
// transforms chain with pointwise work in between without any data movement.
//
// The transforms are unnormalised: forward uses exp(-2 pi i nk/N), inverse
// exp(+2 pi i nk/N).  This is the discrete counterpart of the transform pair of
// Appendix A (Eq. A.2); the 1/N normalisation lives in the propagator tables.
#pragma once
#include <hip/hip_runtime.h>

namespace shg {

template <typename R>
struct __align__(2 * sizeof(R)) cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> scale(cx<R> a, R s) { return {a.re * s, a.im * s}; }
template <typename R>
__device__ __forceinline__ cx<R> conjg(cx<R> a) { return {a.re, -a.im}; }
// a * (+i) and a * (-i)
template <typename R>
__device__ __forceinline__ cx<R> mul_pi(cx<R> a) { return {-a.im, a.re}; }
template <typename R>
__device__ __forceinline__ cx<R> mul_mi(cx<R> a) { return {a.im, -a.re}; }
// a * conj(b)
template <typename R>
__device__ __forceinline__ cx<R> mul_conj(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename R>
__device__ __forceinline__ R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }

// Split constants.  A constant rounded to float is off by up to half an ulp
// and, for the values used here (sqrt(1/2), cos and sin of pi/8, most
// twiddles), its modulus is systematically below or above one.  The same
// rounded constants are applied at every step, so over thousands of
// transforms that bias becomes a drift of the power (a few 1e-8 per
// transform).  A correction of that size cannot be applied after rounding (it
// is below half an ulp), so every float constant is carried as hi + lo
// (lo = the rounding residual) and products are formed as
//   x*w = fma(x, w_hi, x*w_lo)
// which rounds once from a nearly exact product; what remains is ordinary
// unbiased rounding.  In double precision the residual is negligible and the
// lo parts are zero.
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R>
struct Tw {
  R c, s;     // exp(-2 pi i k / N), rounded
  R cl, sl;   // rounding residuals (zero in double precision)
};

template <typename R>
struct K16;
template <>
struct K16<float> {   // cos(pi/8), sin(pi/8), sqrt(1/2) as float hi + lo
  static constexpr bool split = true;
  static constexpr float c1 = 0x1.d906bcp-1f, c1l = 0x1.e651a8p-26f;
  static constexpr float s1 = 0x1.87de2ap-2f, s1l = 0x1.abaa58p-28f;
  static constexpr float h = 0x1.6a09e6p-1f, hl = 0x1.9fcef4p-27f;
};
template <>
struct K16<double> {
  static constexpr bool split = false;
  static constexpr double c1 = 0x1.d906bcf328d46p-1, c1l = 0.0;
  static constexpr double s1 = 0x1.87de2a6aea963p-2, s1l = 0.0;
  static constexpr double h = 0x1.6a09e667f3bcdp-1, hl = 0.0;
};

// x * (wr + i wi) where w = (wr + wrl) + i (wi + wil)
template <bool SPLIT, typename R>
__device__ __forceinline__ cx<R> cmul_split(cx<R> x, R wr, R wi, R wrl, R wil) {
  if constexpr (!SPLIT) {
    return {x.re * wr - x.im * wi, x.re * wi + x.im * wr};
  } else {
    const R tr = fmar(-x.im, wil, x.re * wrl);
    const R ti = fmar(x.im, wrl, x.re * wil);
    return {fmar(x.re, wr, fmar(-x.im, wi, tr)), fmar(x.re, wi, fmar(x.im, wr, ti))};
  }
}

// u * (h + hl)
template <typename R>
__device__ __forceinline__ R mul_h(R u) {
  if constexpr (K16<R>::split) return fmar(u, K16<R>::h, u * K16<R>::hl);
  else return u * K16<R>::h;
}

// a * W16^m with W16 = exp(-2 pi i / 16) (forward) or its conjugate (inverse).
template <int M, bool INV, typename R>
__device__ __forceinline__ cx<R> tw16(cx<R> a) {
  constexpr int m = M & 15;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 4) {
    return INV ? mul_pi(a) : mul_mi(a);
  } else if constexpr (m == 8) {
    return {-a.re, -a.im};
  } else if constexpr (m == 12) {
    return INV ? mul_mi(a) : mul_pi(a);
  } else if constexpr ((m & 1) == 0) {
    // exp(-i m pi/8): m=2 -> (1-i)h, m=6 -> (-1-i)h, m=10 -> (-1+i)h, m=14 -> (1+i)h
    constexpr int sr = (m == 2 || m == 14) ? 1 : -1;           // sign of the real part
    constexpr int si0 = (m == 2 || m == 6) ? -1 : 1;           // sign of the imag part (forward)
    constexpr int si = INV ? -si0 : si0;
    // (a.re + i a.im)(sr + i si) h
    if constexpr (sr == 1 && si == 1) return {mul_h(a.re - a.im), mul_h(a.re + a.im)};
    if constexpr (sr == 1 && si == -1) return {mul_h(a.re + a.im), mul_h(a.im - a.re)};
    if constexpr (sr == -1 && si == 1) return {mul_h(-a.re - a.im), mul_h(a.re - a.im)};
    if constexpr (sr == -1 && si == -1) return {mul_h(a.im - a.re), mul_h(-a.re - a.im)};
  } else {
    // odd m: W16^m = (re, im) built from (c1, s1) = (cos pi/8, sin pi/8)
    //  m:   1    3    5    7    9   11   13   15
    //  re: c1   s1  -s1  -c1  -c1  -s1   s1   c1
    //  im:-s1  -c1  -c1  -s1   s1   c1   c1   s1
    constexpr int k = m >> 1;                                   // 0..7
    constexpr bool re_c = (k == 0 || k == 3 || k == 4 || k == 7);
    constexpr int re_sg = (k == 0 || k == 1 || k == 6 || k == 7) ? 1 : -1;
    constexpr int im_sg0 = (k <= 3) ? -1 : 1;
    constexpr int im_sg = INV ? -im_sg0 : im_sg0;
    using K = K16<R>;
    const R wr = (R)re_sg * (re_c ? K::c1 : K::s1), wrl = (R)re_sg * (re_c ? K::c1l : K::s1l);
    const R wi = (R)im_sg * (re_c ? K::s1 : K::c1), wil = (R)im_sg * (re_c ? K::s1l : K::c1l);
    return cmul_split<K::split>(a, wr, wi, wrl, wil);
  }
}

template <bool INV, typename R>
__device__ __forceinline__ void dft2(cx<R>* x) {
  cx<R> a = x[0];
  x[0] = a + x[1];
  x[1] = a - x[1];
}

template <bool INV, typename R>
__device__ __forceinline__ void dft4v(cx<R>& x0, cx<R>& x1, cx<R>& x2, cx<R>& x3) {
  cx<R> a0 = x0 + x2, a1 = x0 - x2, a2 = x1 + x3, a3 = x1 - x3;
  a3 = INV ? mul_pi(a3) : mul_mi(a3);
  x0 = a0 + a2;
  x2 = a0 - a2;
  x1 = a1 + a3;
  x3 = a1 - a3;
}

template <bool INV, typename R>
__device__ __forceinline__ void dft4(cx<R>* x) { dft4v<INV>(x[0], x[1], x[2], x[3]); }

// DFT_8 by decimation in time: two DFT_4 of the even and odd samples.
template <bool INV, typename R>
__device__ __forceinline__ void dft8(cx<R>* x) {
  cx<R> e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  cx<R> o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4v<INV>(e0, e1, e2, e3);
  dft4v<INV>(o0, o1, o2, o3);
  o1 = tw16<2, INV>(o1);
  o2 = tw16<4, INV>(o2);
  o3 = tw16<6, INV>(o3);
  x[0] = e0 + o0; x[4] = e0 - o0;
  x[1] = e1 + o1; x[5] = e1 - o1;
  x[2] = e2 + o2; x[6] = e2 - o2;
  x[3] = e3 + o3; x[7] = e3 - o3;
}

// DFT_16 as 4 x 4: inner DFT_4 over n1 of x[4 n1 + n2], twiddle W16^{n2 k1},
// outer DFT_4 over n2; output X[k1 + 4 k2].
template <bool INV, typename R>
__device__ __forceinline__ void dft16(cx<R>* x) {
  cx<R> y[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cx<R> a = x[n2], b = x[4 + n2], c = x[8 + n2], d = x[12 + n2];
    dft4v<INV>(a, b, c, d);
    y[4 * n2 + 0] = a;
    y[4 * n2 + 1] = b;
    y[4 * n2 + 2] = c;
    y[4 * n2 + 3] = d;
  }
  y[5] = tw16<1, INV>(y[5]);
  y[6] = tw16<2, INV>(y[6]);
  y[7] = tw16<3, INV>(y[7]);
  y[9] = tw16<2, INV>(y[9]);
  y[10] = tw16<4, INV>(y[10]);
  y[11] = tw16<6, INV>(y[11]);
  y[13] = tw16<3, INV>(y[13]);
  y[14] = tw16<6, INV>(y[14]);
  y[15] = tw16<9, INV>(y[15]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<R> a = y[k1], b = y[4 + k1], c = y[8 + k1], d = y[12 + k1];
    dft4v<INV>(a, b, c, d);
    x[k1] = a;
    x[k1 + 4] = b;
    x[k1 + 8] = c;
    x[k1 + 12] = d;
  }
}

template <int RP, bool INV, typename R>
__device__ __forceinline__ void dft(cx<R>* x) {
  if constexpr (RP == 2) dft2<INV>(x);
  else if constexpr (RP == 4) dft4<INV>(x);
  else if constexpr (RP == 8) dft8<INV>(x);
  else dft16<INV>(x);
}

// Largest radix in {16, 8, 4, 2} dividing both the per-thread element count
// and the remaining length.
template <int E, int REM>
struct pick_radix {
  static constexpr int value = (E % 16 == 0 && REM % 16 == 0) ? 16
                               : (E % 8 == 0 && REM % 8 == 0) ? 8
                               : (E % 4 == 0 && REM % 4 == 0) ? 4
                                                               : 2;
};

// Number of Stockham passes of an N-point transform at E elements per thread.
template <int E, int REM>
constexpr int stockham_passes() {
  if constexpr (REM == 1) return 0;
  else return 1 + stockham_passes<E, REM / pick_radix<E, REM>::value>();
}

// True when every Stockham pass but the last has one butterfly per thread
// (radix = elements per thread; the last pass only reads into registers).  A
// wavefront issues all LDS reads of such a pass before its writes and its LDS
// operations complete in order, so a transform held by one wavefront can then
// run its passes in place in a single buffer.
template <int E, int REM>
constexpr bool stockham_one_butterfly() {
  constexpr int RP = pick_radix<E, REM>::value;
  if constexpr (REM == RP) return true;
  else return RP == E && stockham_one_butterfly<E, REM / RP>();
}

// LDS index with one complex of padding per 16 (breaks power-of-two strides).
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }
template <int N>
constexpr int padded_len() { return N + N / 16; }

// LDS view of one transform: element i lives at base[pad16(i) * STRIDE].
template <typename R, int STRIDE>
struct LdsView {
  cx<R>* base;
  __device__ __forceinline__ cx<R>& operator[](int i) const { return base[pad16(i) * STRIDE]; }
};

// One Stockham pass and, recursively, the ones after it.
//   v      registers of this thread (stride-G layout)
//   buf0/1 ping-pong LDS views of this transform
//   tw     twiddle table W_N^k, k = 0..N-1 (forward sign, hi + lo), global memory
template <typename R, int N, int G, bool INV, int NS, int REM, bool FIRST, int STRIDE>
__device__ __forceinline__ void stockham(cx<R> (&v)[N / G], LdsView<R, STRIDE> in,
                                         LdsView<R, STRIDE> out, int t,
                                         const Tw<R>* __restrict__ tw, bool active) {
  constexpr int E = N / G;
  constexpr int RP = pick_radix<E, REM>::value;
  constexpr int NB = E / RP;
  constexpr bool LAST = (REM == RP);
#pragma unroll
  for (int u = 0; u < NB && active; ++u) {
    const int j = t + G * u;
    cx<R> x[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) x[r] = FIRST ? v[u + r * NB] : in[j + r * (N / RP)];
    if constexpr (NS > 1) {
      const int jm = j % NS;
#pragma unroll
      for (int r = 1; r < RP; ++r) {
        const Tw<R> w = tw[jm * r * (N / (NS * RP))];
        x[r] = cmul_split<K16<R>::split>(x[r], w.c, INV ? -w.s : w.s, w.cl, INV ? -w.sl : w.sl);
      }
    }
    dft<RP, INV>(x);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < RP; ++r) v[u + r * NB] = x[r];
    } else {
      const int d = (j / NS) * NS * RP + (j % NS);
#pragma unroll
      for (int r = 0; r < RP; ++r) out[d + r * NS] = x[r];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
    stockham<R, N, G, INV, NS * RP, REM / RP, false, STRIDE>(v, out, in, t, tw, active);
  }
}

// ---------------------------------------------------------------- twiddle prefetch
// The twiddles a thread needs depend only on its index, so they are loaded
// into registers once, before the first barrier, and reused for the forward
// and the inverse transform of a pass (conjugated).  Otherwise each Stockham
// pass would issue its twiddle loads after a barrier and wait on them.
template <int N, int G, int NS, int REM>
struct TwCount {
  static constexpr int E = N / G;
  static constexpr int RP = pick_radix<E, REM>::value;
  static constexpr int NB = E / RP;
  static constexpr int here = NS > 1 ? NB * (RP - 1) : 0;
  static constexpr int value = here + TwCount<N, G, NS * RP, REM / RP>::value;
};
template <int N, int G, int NS>
struct TwCount<N, G, NS, 1> {
  static constexpr int value = 0;
};

template <typename R, int N, int G>
struct TwRegs {
  static constexpr int count = TwCount<N, G, 1, N>::value;
  Tw<R> w[count > 0 ? count : 1];
};

// Global-memory view of a device pointer.  Pointers that kernels read from a
// table in memory (the instances of a batch) are generic to the compiler,
// which then issues flat memory instructions; those count against the LDS
// counter as well, so every LDS wait of a transform would also wait for the
// loads issued ahead of it.  An explicit conversion to the global address
// space gives global instructions (a no-op for pointers that are kernel
// arguments, which the compiler already knows to be global).
template <typename T>
using gmem = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ gmem<T>* gp(T* q) {
  return (gmem<T>*)q;
}

// Loads and stores of the complex and twiddle types through a global view:
// class types cannot be assigned to or from address-space-qualified objects,
// so they move as builtin vectors of 32-bit words.
template <typename T>
__device__ __forceinline__ T gload(const gmem<T>* q) {
  static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
  typedef unsigned V __attribute__((ext_vector_type(sizeof(T) / 4), aligned(alignof(T))));
  return __builtin_bit_cast(T, *reinterpret_cast<const gmem<V>*>(q));
}

template <typename T>
__device__ __forceinline__ T gload(const T* q) {
  return *q;
}

template <typename T>
__device__ __forceinline__ void gstore(gmem<T>* q, T x) {
  static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
  typedef unsigned V __attribute__((ext_vector_type(sizeof(T) / 4), aligned(alignof(T))));
  *reinterpret_cast<gmem<V>*>(q) = __builtin_bit_cast(V, x);
}

// One of two pointers by a per-lane flag f (0 or 1), formed arithmetically
// from their (uniform) values.  Written as a select of two adjacent kernel
// arguments, the choice becomes a per-lane load from the argument segment: a
// dependent memory round trip ahead of the loads that use the pointer.  The
// empty asm hides f's range so that the arithmetic is not turned back into a
// select.
template <typename T>
__device__ __forceinline__ T* pick_ptr(int f, T* p0, T* p1) {
  asm volatile("" : "+v"(f));
  const uintptr_t a = (uintptr_t)p0, b = (uintptr_t)p1;
  return (T*)(a + (uintptr_t)(unsigned)f * (b - a));
}

// The same choice for a flag that is uniform over the wavefront (held in a
// scalar register): a select of two indexed kernel arguments would become a
// scalar load from the argument segment at a computed offset, a dependent
// memory round trip ahead of every load that uses the pointer.
template <typename T>
__device__ __forceinline__ T* pick_ptr_uniform(int f, T* p0, T* p1) {
  f = __builtin_amdgcn_readfirstlane(f);
  asm volatile("" : "+s"(f));
  const uintptr_t a = (uintptr_t)p0, b = (uintptr_t)p1;
  return (T*)(a + (uintptr_t)(unsigned)f * (b - a));
}

// Index of the transform a thread works on: G threads per transform, so with
// G >= 64 the index is uniform over each wavefront and is read as a scalar.
template <int G>
__device__ __forceinline__ int transform_index(bool active, int tid) {
  const int tr = active ? tid / G : 0;
  if constexpr (G >= 64) return __builtin_amdgcn_readfirstlane(tr);
  return tr;
}

template <typename R, int N, int G, int NS, int REM>
__device__ __forceinline__ void tw_gather(Tw<R>* out, int t, const gmem<Tw<R>>* __restrict__ tw) {
  if constexpr (REM > 1) {
    constexpr int E = N / G;
    constexpr int RP = pick_radix<E, REM>::value;
    constexpr int NB = E / RP;
    if constexpr (NS > 1) {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int jm = (t + G * u) % NS;
#pragma unroll
        for (int r = 1; r < RP; ++r) out[u * (RP - 1) + (r - 1)] = gload(tw + jm * r * (N / (NS * RP)));
      }
      tw_gather<R, N, G, NS * RP, REM / RP>(out + NB * (RP - 1), t, tw);
    } else {
      tw_gather<R, N, G, NS * RP, REM / RP>(out, t, tw);
    }
  }
}

template <typename R, int N, int G>
__device__ __forceinline__ void tw_load(TwRegs<R, N, G>& T, int t, const Tw<R>* __restrict__ tw) {
  tw_gather<R, N, G, 1, N>(T.w, t, gp(tw));
}

// Barrier between Stockham passes.  WAVE: every transform belongs to the
// threads of one wavefront, whose LDS buffers no other wavefront touches; a
// wavefront's LDS operations complete in issue order, so a wavefront-level
// barrier that keeps the compiler from moving LDS accesses across it is
// enough (no s_barrier, no wait for the writes to land).  Otherwise a block
// barrier.
template <bool WAVE>
__device__ __forceinline__ void pass_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Stockham pass reading its twiddles from the prefetched registers.
template <typename R, int N, int G, bool INV, int NS, int REM, bool FIRST, int STRIDE,
          bool WAVE = false>
__device__ __forceinline__ void stockham_pre(cx<R> (&v)[N / G], LdsView<R, STRIDE> in,
                                             LdsView<R, STRIDE> out, int t, const Tw<R>* twr,
                                             bool active) {
  constexpr int E = N / G;
  constexpr int RP = pick_radix<E, REM>::value;
  constexpr int NB = E / RP;
  constexpr bool LAST = (REM == RP);
#pragma unroll
  for (int u = 0; u < NB && active; ++u) {
    const int j = t + G * u;
    cx<R> x[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) x[r] = FIRST ? v[u + r * NB] : in[j + r * (N / RP)];
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < RP; ++r) {
        const Tw<R> w = twr[u * (RP - 1) + (r - 1)];
        x[r] = cmul_split<K16<R>::split>(x[r], w.c, INV ? -w.s : w.s, w.cl, INV ? -w.sl : w.sl);
      }
    }
    dft<RP, INV>(x);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < RP; ++r) v[u + r * NB] = x[r];
    } else {
      const int d = (j / NS) * NS * RP + (j % NS);
#pragma unroll
      for (int r = 0; r < RP; ++r) out[d + r * NS] = x[r];
    }
  }
  if constexpr (!LAST) {
    if constexpr (WAVE) {
      if (!active) return;
    }
    pass_sync<WAVE>();
    constexpr int used = NS > 1 ? NB * (RP - 1) : 0;
    stockham_pre<R, N, G, INV, NS * RP, REM / RP, false, STRIDE, WAVE>(v, out, in, t, twr + used,
                                                                      active);
  }
}

// Whole transform of the registers v with prefetched twiddles; one leading
// barrier protects LDS reuse.  Without WAVE all threads of the block must call
// it (threads with active = false only take part in the barriers).  WAVE (see
// pass_sync) needs each transform's threads, and the buffers b0, b1, to
// belong to one wavefront; inactive wavefronts then skip it.
template <typename R, int N, int G, bool INV, int STRIDE, bool WAVE = false>
__device__ __forceinline__ void fft_pre(cx<R> (&v)[N / G], LdsView<R, STRIDE> b0,
                                        LdsView<R, STRIDE> b1, int t, const TwRegs<R, N, G>& T,
                                        bool active = true) {
  static_assert(!WAVE || G * STRIDE <= 64,
                "a wavefront-synchronised transform must fit one wavefront");
  if constexpr (WAVE) {
    if (!active) return;
  }
  if constexpr (pick_radix<N / G, N>::value < N) pass_sync<WAVE>();
  stockham_pre<R, N, G, INV, 1, N, true, STRIDE, WAVE>(v, b0, b1, t, T.w, active);
}

// Whole transform of the registers v.  All threads of the block must call it
// (it contains block barriers); one leading barrier protects LDS reuse.
// Threads with active = false only take part in the barriers.
template <typename R, int N, int G, bool INV, int STRIDE>
__device__ __forceinline__ void fft_regs(cx<R> (&v)[N / G], LdsView<R, STRIDE> b0,
                                         LdsView<R, STRIDE> b1, int t,
                                         const Tw<R>* __restrict__ tw, bool active = true) {
  if constexpr (pick_radix<N / G, N>::value < N) __syncthreads();
  stockham<R, N, G, INV, 1, N, true, STRIDE>(v, b0, b1, t, tw, active);
}

}  // namespace shg
