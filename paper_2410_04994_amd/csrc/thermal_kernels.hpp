// Steady-state heat equation (Sec. 2.2) on the SSFM grid, finite differences
// of Sec. 3.2, solved by Jacobi-preconditioned conjugate gradients.
//
// Nodes: nx x ny transverse samples (the field grid; the x and y faces sit at
// the first and last samples) times nz + 1 planes z_l = l dz.  Unknown:
// theta = T - T_oven.  Nodes on an oven face are theta = 0.  Every other node
// obeys the 7-point equation sum_d (T_{+d} - 2T + T_{-d}) / h_d^2 = -q / k,
// where on an air (or insulated) face the missing outside neighbour is removed
// with the central difference of -k dT/dn = h (T - T_inf).  Multiplying each
// node equation by its control-volume weight w = prod_d (1/2 on a face in
// direction d) makes the operator symmetric positive definite:
//   (A theta)_i = w_i [ sum_d interior: (2 theta - theta_+ - theta_-) / h^2
//                      face:     (2 theta - 2 theta_in) / h^2 + 2 beta_f theta / h ]
//   b_i         = w_i [ q_i / k - sum_{air faces} 2 beta (T_oven - T_inf) / h ]
// with beta = h_conv / k (0 on insulated faces).
#pragma once
#include <hip/hip_runtime.h>

namespace shg {

enum : int { kFaceAir = 0, kFaceOven = 1, kFaceInsulated = 2 };

struct ThermGeom {
  int nx, ny, nzn;          // nodes per axis (nzn = nz + 1); nx, ny powers of two
  int log2_nx, log2_plane;  // log2(nx), log2(nx ny)
  int face[6];              // x-, x+, y-, y+, z-, z+
  double ih2[3];            // 1 / h_d^2
  double conv[6];           // 2 beta / h_d on each face (0 unless air)
  double inv_k;             // 1 / k
  double src_conv[6];       // 2 beta (T_oven - T_inf) / h_d on air faces, else 0
  size_t n;                 // total nodes
};

// Position of node i and its boundary role in each direction.
struct NodePos {
  int c[3];                 // x, y, z index
  bool oven;
};

__device__ __forceinline__ bool is_oven(const ThermGeom& g, const int c[3]) {
  return (c[0] == 0 && g.face[0] == kFaceOven) || (c[0] == g.nx - 1 && g.face[1] == kFaceOven) ||
         (c[1] == 0 && g.face[2] == kFaceOven) || (c[1] == g.ny - 1 && g.face[3] == kFaceOven) ||
         (c[2] == 0 && g.face[4] == kFaceOven) || (c[2] == g.nzn - 1 && g.face[5] == kFaceOven);
}

__device__ __forceinline__ NodePos node_pos(const ThermGeom& g, size_t i) {
  NodePos q;
  q.c[2] = (int)(i >> g.log2_plane);
  const int r = (int)(i & (((size_t)1 << g.log2_plane) - 1));
  q.c[1] = r >> g.log2_nx;
  q.c[0] = r & (g.nx - 1);
  q.oven = is_oven(g, q.c);
  return q;
}

// The neighbour of q one node along direction d (s = +1 or -1).
__device__ __forceinline__ NodePos neighbour(const ThermGeom& g, const NodePos& q, int d, int s) {
  NodePos n = q;
  n.c[d] += s;
  n.oven = is_oven(g, n.c);
  return n;
}

// Control-volume weight and diagonal of A at a free node.
__device__ __forceinline__ void node_weight_diag(const ThermGeom& g, const NodePos& q, double* w,
                                                 double* diag) {
  const int nd[3] = {g.nx, g.ny, g.nzn};
  double ww = 1.0, dg = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    dg += 2.0 * g.ih2[d];
    if (q.c[d] == 0) {
      ww *= 0.5;
      dg += g.conv[2 * d];
    } else if (q.c[d] == nd[d] - 1) {
      ww *= 0.5;
      dg += g.conv[2 * d + 1];
    }
  }
  *w = ww;
  *diag = ww * dg;
}

// (A v)_i at a free node; v(j, qj) gives the value at node j with position qj.
template <typename V>
__device__ __forceinline__ double apply_node(const ThermGeom& g, const NodePos& q, size_t i, V v,
                                             double w) {
  const int nd[3] = {g.nx, g.ny, g.nzn};
  const size_t st[3] = {1, (size_t)g.nx, (size_t)g.nx * g.ny};
  const double c = v(i, q);
  double acc = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (q.c[d] == 0) {
      acc += (2.0 * c - 2.0 * v(i + st[d], neighbour(g, q, d, 1))) * g.ih2[d] + g.conv[2 * d] * c;
    } else if (q.c[d] == nd[d] - 1) {
      acc += (2.0 * c - 2.0 * v(i - st[d], neighbour(g, q, d, -1))) * g.ih2[d] +
             g.conv[2 * d + 1] * c;
    } else {
      acc += (2.0 * c - v(i + st[d], neighbour(g, q, d, 1)) - v(i - st[d], neighbour(g, q, d, -1))) *
             g.ih2[d];
    }
  }
  return w * acc;
}

// Fixed-order sum of one double per thread over a 256-thread block; the result
// is valid in thread 0.
__device__ __forceinline__ double block_sum256(double x, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) x = red[0] + red[1] + red[2] + red[3];
  return x;
}

__device__ __forceinline__ double block_max256(double x, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) x = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  return x;
}

// Device scalars of the iteration.
enum : int { kRz = 0, kPAp, kAlpha, kBeta, kRr, kBb, kCount };

// theta = T - T_oven (0 on oven nodes); p = 0.
template <typename R>
__global__ void __launch_bounds__(256) th_init(ThermGeom g, const R* __restrict__ t_in, double t_oven,
                                               R* __restrict__ theta, R* __restrict__ p0) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < g.n; i += (size_t)gridDim.x * 256) {
    const NodePos q = node_pos(g, i);
    theta[i] = q.oven ? (R)0 : (R)((double)t_in[i] - t_oven);
    p0[i] = (R)0;
  }
}

// r = b - A theta, per-block partials of r.z (z = r / diag) and b.b.
template <typename R>
__global__ void __launch_bounds__(256) th_residual(ThermGeom g, const R* __restrict__ heat,
                                                   const R* __restrict__ theta, R* __restrict__ r,
                                                   double* __restrict__ part) {
  __shared__ double red[4];
  double rz = 0.0, bb = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < g.n; i += (size_t)gridDim.x * 256) {
    const NodePos q = node_pos(g, i);
    if (q.oven) {
      r[i] = (R)0;
      continue;
    }
    double w, dg;
    node_weight_diag(g, q, &w, &dg);
    double src = (double)heat[i] * g.inv_k;
    const int nd[3] = {g.nx, g.ny, g.nzn};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (q.c[d] == 0) src -= g.src_conv[2 * d];
      else if (q.c[d] == nd[d] - 1) src -= g.src_conv[2 * d + 1];
    }
    const double b = w * src;
    const double ax = apply_node(g, q, i, [&](size_t j, const NodePos&) { return (double)theta[j]; }, w);
    const double rr = b - ax;
    r[i] = (R)rr;
    rz += (double)(R)rr * ((double)(R)rr / dg);
    bb += b * b;
  }
  rz = block_sum256(rz, red);
  bb = block_sum256(bb, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rz;
    part[2 * blockIdx.x + 1] = bb;
  }
}

// p_new = r / diag + beta p_old at the node and its neighbours; Ap = A p_new;
// per-block partials of p_new . Ap.
template <typename R>
__global__ void __launch_bounds__(256) th_direction_apply(ThermGeom g, const R* __restrict__ r,
                                                          const R* __restrict__ p_old,
                                                          R* __restrict__ p_new, R* __restrict__ ap,
                                                          const double* __restrict__ sc,
                                                          double* __restrict__ part) {
  __shared__ double red[4];
  const double beta = sc[kBeta];
  double pap = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < g.n; i += (size_t)gridDim.x * 256) {
    const NodePos q = node_pos(g, i);
    if (q.oven) {
      p_new[i] = (R)0;
      ap[i] = (R)0;
      continue;
    }
    // direction at node j, rounded to R as it is stored
    auto pdir = [&](size_t j, const NodePos& qj) {
      if (qj.oven) return 0.0;
      double wj, dj;
      node_weight_diag(g, qj, &wj, &dj);
      return (double)(R)((double)r[j] / dj + beta * (double)p_old[j]);
    };
    double w, dg;
    node_weight_diag(g, q, &w, &dg);
    const double pc = pdir(i, q);
    const double a = apply_node(g, q, i, pdir, w);
    p_new[i] = (R)pc;
    ap[i] = (R)a;
    pap += pc * (double)(R)a;
  }
  pap = block_sum256(pap, red);
  if (threadIdx.x == 0) part[blockIdx.x] = pap;
}

// theta += alpha p; r -= alpha Ap; partials of r.z and r.r.
template <typename R>
__global__ void __launch_bounds__(256) th_update(ThermGeom g, R* __restrict__ theta, R* __restrict__ r,
                                                 const R* __restrict__ p, const R* __restrict__ ap,
                                                 const double* __restrict__ sc,
                                                 double* __restrict__ part) {
  __shared__ double red[4];
  const double alpha = sc[kAlpha];
  double rz = 0.0, rr = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < g.n; i += (size_t)gridDim.x * 256) {
    const NodePos q = node_pos(g, i);
    if (q.oven) continue;
    double w, dg;
    node_weight_diag(g, q, &w, &dg);
    theta[i] = (R)((double)theta[i] + alpha * (double)p[i]);
    const R rn = (R)((double)r[i] - alpha * (double)ap[i]);
    r[i] = rn;
    rz += (double)rn * ((double)rn / dg);
    rr += (double)rn * (double)rn;
  }
  rz = block_sum256(rz, red);
  rr = block_sum256(rr, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rz;
    part[2 * blockIdx.x + 1] = rr;
  }
}

// Scalar steps of the iteration, one block, fixed order.
//   mode 0: after th_residual: rz, bb (and beta = 0 for the first direction)
//   mode 1: after th_direction_apply: alpha = rz / pAp
//   mode 2: after th_update: beta = rz_new / rz, rz = rz_new, rr
__global__ void __launch_bounds__(256) th_scalars(const double* __restrict__ part, int nblk, int mode,
                                                  double* __restrict__ sc) {
  __shared__ double red[4];
  double a = 0.0, b = 0.0;
  const int stride = (mode == 1) ? 1 : 2;
  for (int k = threadIdx.x; k < nblk; k += 256) {
    a += part[stride * k];
    if (stride == 2) b += part[stride * k + 1];
  }
  a = block_sum256(a, red);
  b = block_sum256(b, red);
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    sc[kRz] = a;
    sc[kBb] = b;
    sc[kBeta] = 0.0;
    sc[kRr] = -1.0;
  } else if (mode == 1) {
    sc[kPAp] = a;
    sc[kAlpha] = (a > 0.0) ? sc[kRz] / a : 0.0;
  } else {
    sc[kBeta] = (sc[kRz] > 0.0) ? a / sc[kRz] : 0.0;
    sc[kRz] = a;
    sc[kRr] = b;
  }
}

// T = theta + T_oven; optional mid-planes (T_l + T_{l+1}) / 2 and largest
// change from t_prev (per-block partial maxima).
template <typename R>
__global__ void __launch_bounds__(256) th_finish(ThermGeom g, const R* __restrict__ theta, double t_oven,
                                                 R* __restrict__ t_out) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < g.n; i += (size_t)gridDim.x * 256)
    t_out[i] = (R)((double)theta[i] + t_oven);
}

template <typename R>
__global__ void __launch_bounds__(256) th_midplanes(const R* __restrict__ t, size_t plane, size_t n_mid,
                                                    R* __restrict__ t_mid) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n_mid; i += (size_t)gridDim.x * 256)
    t_mid[i] = (R)(0.5 * ((double)t[i] + (double)t[i + plane]));
}

template <typename R>
__global__ void __launch_bounds__(256) th_max_change(const R* __restrict__ a, const R* __restrict__ b,
                                                     size_t n, double* __restrict__ part) {
  __shared__ double red[4];
  double m = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    m = fmax(m, fabs((double)a[i] - (double)b[i]));
  m = block_max256(m, red);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ void __launch_bounds__(256) th_max_final(const double* __restrict__ part, int nblk,
                                                    double* __restrict__ out) {
  __shared__ double red[4];
  double m = 0.0;
  for (int k = threadIdx.x; k < nblk; k += 256) m = fmax(m, part[k]);
  m = block_max256(m, red);
  if (threadIdx.x == 0) *out = m;
}

}  // namespace shg
