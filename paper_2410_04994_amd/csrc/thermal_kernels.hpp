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
  size_t n;                 // total nodes
  double inv_k;             // 1 / k
  // per node class (27 = 3 x 3 x 3: interior / low face / high face per
  // direction): oven flag, control-volume weight w, 1 / (w diag), and the
  // boundary source term -w sum_{air faces} 2 beta (T_oven - T_inf) / h
  double ih2[3];            // 1 / h_d^2
  double conv_lo[3], conv_hi[3];   // 2 beta / h_d on the low / high face (0 unless air)
  int oven[27];
  double w[27], inv_diag[27], src[27];
};

// Position of node i: coordinates and class.
struct NodePos {
  int c[3];                 // x, y, z index
  int cls;                  // sum_d role_d 3^d, role 0 interior, 1 low face, 2 high face
};

__device__ __forceinline__ int role(int c, int n) { return c == 0 ? 1 : (c == n - 1 ? 2 : 0); }

__device__ __forceinline__ NodePos node_pos(const ThermGeom& g, size_t i) {
  NodePos q;
  q.c[2] = (int)(i >> g.log2_plane);
  const int r = (int)(i & (((size_t)1 << g.log2_plane) - 1));
  q.c[1] = r >> g.log2_nx;
  q.c[0] = r & (g.nx - 1);
  q.cls = role(q.c[0], g.nx) + 3 * role(q.c[1], g.ny) + 9 * role(q.c[2], g.nzn);
  return q;
}

// Class of the neighbour one node along direction d (s = +1 or -1).
__device__ __forceinline__ int neighbour_cls(const ThermGeom& g, const NodePos& q, int d, int s) {
  const int nd[3] = {g.nx, g.ny, g.nzn};
  const int p3[3] = {1, 3, 9};
  const int before = role(q.c[d], nd[d]);
  const int after = role(q.c[d] + s, nd[d]);
  return q.cls + (after - before) * p3[d];
}

// (A v)_i at a free node; v(j, cls_j) gives the value at node j of class cls_j.
// Arithmetic in R (the solver's storage precision).
template <typename R, typename V>
__device__ __forceinline__ R apply_node(const ThermGeom& g, const NodePos& q, size_t i, V v) {
  const int nd[3] = {g.nx, g.ny, g.nzn};
  const size_t st[3] = {1, (size_t)g.nx, (size_t)g.nx * g.ny};
  const R c = v(i, q.cls);
  R acc = (R)0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const R ih2 = (R)g.ih2[d];
    if (q.c[d] == 0) {
      acc += (c - v(i + st[d], neighbour_cls(g, q, d, 1))) * ((R)2 * ih2) + (R)g.conv_lo[d] * c;
    } else if (q.c[d] == nd[d] - 1) {
      acc += (c - v(i - st[d], neighbour_cls(g, q, d, -1))) * ((R)2 * ih2) + (R)g.conv_hi[d] * c;
    } else {
      acc += ((R)2 * c - v(i + st[d], neighbour_cls(g, q, d, 1)) -
              v(i - st[d], neighbour_cls(g, q, d, -1))) * ih2;
    }
  }
  return (R)g.w[q.cls] * acc;
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
    theta[i] = g.oven[q.cls] ? (R)0 : (R)((double)t_in[i] - t_oven);
    p0[i] = (R)0;
  }
}

// r = b - A theta, per-block partials of r.z (z = r / diag), or of r.r when
// RR, and of b.b.
template <typename R, bool RR = false, typename H = R>
__global__ void __launch_bounds__(256) th_residual(ThermGeom g, const H* __restrict__ heat,
                                                   const R* __restrict__ theta, R* __restrict__ r,
                                                   double* __restrict__ part) {
  __shared__ double red[4];
  double rz = 0.0, bb = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < g.n; i += (size_t)gridDim.x * 256) {
    const NodePos q = node_pos(g, i);
    if (g.oven[q.cls]) {
      r[i] = (R)0;
      continue;
    }
    const double b = g.w[q.cls] * ((double)heat[i] * g.inv_k) + g.src[q.cls];
    const double ax = (double)apply_node<R>(g, q, i, [&](size_t j, int) { return theta[j]; });
    const R rr = (R)(b - ax);
    r[i] = rr;
    rz += (double)rr * (double)rr * (RR ? 1.0 : g.inv_diag[q.cls]);
    bb += b * b;
  }
  rz = block_sum256(rz, red);
  bb = block_sum256(bb, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rz;
    part[2 * blockIdx.x + 1] = bb;
  }
}

// Class of the node at (x, y, z).
__device__ __forceinline__ int node_cls(const ThermGeom& g, int x, int y, int z) {
  return role(x, g.nx) + 3 * role(y, g.ny) + 9 * role(z, g.nzn);
}

// p_new = r / diag + beta p_old; Ap = A p_new; per-block partials of p_new . Ap.
// 2.5-D tiling: a block of TX x TY threads owns an x-y tile and marches through
// kThermZ planes.  The direction of the planes below and above stays in
// registers; x and y neighbours come from an LDS copy of the current plane with
// a one-node halo.  Two copies alternate, so one barrier per plane suffices: a
// copy is rewritten two planes later, after every thread has passed the barrier
// of the plane in between.  The raw r and p_old of a thread's node (and of its
// halo node, for threads on a tile edge) are loaded kThermPf planes ahead of
// their use, so that several planes' loads are in flight per wavefront.  r and
// p_old are read about once per node (plus the halo).  A node's class changes
// along z only through its z role, so the per-class values are taken once.
// p_new vanishes on oven nodes because r and p_old do and 1/diag is 0 there.
constexpr int kThermZ = 16;
constexpr int kThermPf = 4;

template <typename R>
__global__ void __launch_bounds__(256) th_direction_apply(ThermGeom g, const R* __restrict__ r,
                                                          const R* __restrict__ p_old,
                                                          R* __restrict__ p_new, R* __restrict__ ap,
                                                          const double* __restrict__ sc,
                                                          double* __restrict__ part) {
  __shared__ R tile[2][420];     // (TY + 2) x (TX + 2) <= 420 for TX TY = 256, TX in [16, 64]
  __shared__ double red[4];
  const int TX = blockDim.x, TY = blockDim.y;
  const int LW = TX + 2;
  const int tx = threadIdx.x, ty = threadIdx.y;
  // Blocks are dealt to the 8 XCDs round-robin (dispatch index mod 8).  Tile
  // lin = (b mod 8) (nb / 8) + b / 8 gives each XCD a contiguous run of tiles,
  // x fastest, then y, then z, so the tiles whose halo rows a block reads run
  // on the same XCD and share its L2.
  const int nb = gridDim.x * gridDim.y * gridDim.z;
  const int b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const int lin = nb % 8 == 0 ? (b % 8) * (nb / 8) + b / 8 : b;
  const int tile_x = lin % gridDim.x, tile_y = (lin / gridDim.x) % gridDim.y;
  const int tile_z = lin / (gridDim.x * gridDim.y);
  const int x = tile_x * TX + tx, y = tile_y * TY + ty;
  const int z0 = tile_z * kThermZ, z1 = min(z0 + kThermZ, g.nzn);
  const size_t plane = (size_t)g.nx * g.ny;
  const R beta = (R)sc[kBeta];
  // halo node of a thread on a tile edge (TX, TY >= 4, so at most one x edge
  // and one y edge): its column index, whether it lies inside the grid, and
  // its LDS slot; a thread off the edges has no halo node (slot -1)
  const int hx = tx == 0 ? x - 1 : x + 1;
  const int sx = tx == 0 ? (ty + 1) * LW : (tx == TX - 1 ? (ty + 1) * LW + TX + 1 : -1);
  const bool inx = sx >= 0 && hx >= 0 && hx < g.nx;
  const int hy = ty == 0 ? y - 1 : y + 1;
  const int sy = ty == 0 ? tx + 1 : (ty == TY - 1 ? (TY + 1) * LW + tx + 1 : -1);
  const bool iny = sy >= 0 && hy >= 0 && hy < g.ny;
  // per z role (0 interior, 1 first plane, 2 last plane): 1 / diag of the node
  // and of its halo nodes, and w and the oven flag of the node
  const int bc = role(x, g.nx) + 3 * role(y, g.ny);
  const int bx = inx ? role(hx, g.nx) + 3 * role(y, g.ny) : 0;
  const int by = iny ? role(x, g.nx) + 3 * role(hy, g.ny) : 0;
  R dc[3], dx[3], dy[3], wc[3];
  int oc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dc[k] = (R)g.inv_diag[bc + 9 * k];
    dx[k] = (R)g.inv_diag[bx + 9 * k];
    dy[k] = (R)g.inv_diag[by + 9 * k];
    wc[k] = (R)g.w[bc + 9 * k];
    oc[k] = g.oven[bc + 9 * k];
  }
  const size_t col = (size_t)y * g.nx + x;
  const size_t colx = (size_t)y * g.nx + hx, coly = (size_t)hy * g.nx + x;
  // raw values: node of plane z0 - 1 + j (j = 0 .. kThermZ + 1), halo nodes of
  // plane z0 + j (j = 0 .. kThermZ - 1); zero outside the grid
  R cr[kThermZ + 2], cp[kThermZ + 2], xr[kThermZ], xp[kThermZ], yr[kThermZ], yp[kThermZ];
  auto load_c = [&](int j) {
    const int zz = z0 - 1 + j;
    cr[j] = (R)0;
    cp[j] = (R)0;
    if (zz >= 0 && zz < g.nzn) {
      const size_t i = (size_t)zz * plane + col;
      cr[j] = r[i];
      cp[j] = p_old[i];
    }
  };
  auto load_h = [&](int j) {
    const int zz = z0 + j;
    xr[j] = xp[j] = yr[j] = yp[j] = (R)0;
    if (zz < g.nzn) {
      if (inx) {
        const size_t i = (size_t)zz * plane + colx;
        xr[j] = r[i];
        xp[j] = p_old[i];
      }
      if (iny) {
        const size_t i = (size_t)zz * plane + coly;
        yr[j] = r[i];
        yp[j] = p_old[i];
      }
    }
  };
  auto zrole = [&](int zz) { return zz == 0 ? 1 : (zz == g.nzn - 1 ? 2 : 0); };
#pragma unroll
  for (int j = 0; j < kThermPf + 2; ++j) load_c(j);
#pragma unroll
  for (int j = 0; j < kThermPf; ++j) load_h(j);
  const R ih2x = (R)g.ih2[0], ih2y = (R)g.ih2[1], ih2z = (R)g.ih2[2];
  R pm = cr[0] * dc[z0 > 0 ? zrole(z0 - 1) : 0] + beta * cp[0];
  R pc = cr[1] * dc[zrole(z0)] + beta * cp[1];
  double pap = 0.0;
#pragma unroll
  for (int k = 0; k < kThermZ; ++k) {
    const int z = z0 + k;
    if (z >= z1) break;
    if (k + kThermPf + 2 < kThermZ + 2) load_c(k + kThermPf + 2);
    if (k + kThermPf < kThermZ) load_h(k + kThermPf);
    const int zr = zrole(z);
    const R pn = cr[k + 2] * dc[z + 1 < g.nzn ? zrole(z + 1) : 0] + beta * cp[k + 2];
    R* t = tile[k & 1];
    t[(ty + 1) * LW + tx + 1] = pc;
    if (sx >= 0) t[sx] = xr[k] * dx[zr] + beta * xp[k];
    if (sy >= 0) t[sy] = yr[k] * dy[zr] + beta * yp[k];
    __syncthreads();
    const size_t i = (size_t)z * plane + col;
    R a = (R)0;
    if (!oc[zr]) {
      const R xm = t[(ty + 1) * LW + tx], xq = t[(ty + 1) * LW + tx + 2];
      const R ym = t[ty * LW + tx + 1], yq = t[(ty + 2) * LW + tx + 1];
      R acc;
      if (x == 0) acc = (pc - xq) * ((R)2 * ih2x) + (R)g.conv_lo[0] * pc;
      else if (x == g.nx - 1) acc = (pc - xm) * ((R)2 * ih2x) + (R)g.conv_hi[0] * pc;
      else acc = ((R)2 * pc - xq - xm) * ih2x;
      if (y == 0) acc += (pc - yq) * ((R)2 * ih2y) + (R)g.conv_lo[1] * pc;
      else if (y == g.ny - 1) acc += (pc - ym) * ((R)2 * ih2y) + (R)g.conv_hi[1] * pc;
      else acc += ((R)2 * pc - yq - ym) * ih2y;
      if (z == 0) acc += (pc - pn) * ((R)2 * ih2z) + (R)g.conv_lo[2] * pc;
      else if (z == g.nzn - 1) acc += (pc - pm) * ((R)2 * ih2z) + (R)g.conv_hi[2] * pc;
      else acc += ((R)2 * pc - pn - pm) * ih2z;
      a = wc[zr] * acc;
      pap += (double)pc * (double)a;
    }
    p_new[i] = pc;
    ap[i] = a;
    pm = pc;
    pc = pn;
  }
  const int flat = ty * TX + tx;
  // block_sum256 indexes threads by threadIdx.x; use the flat index instead
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) pap += __shfl_down(pap, off, 64);
  if ((flat & 63) == 0) red[flat >> 6] = pap;
  __syncthreads();
  if (flat == 0) part[lin] = red[0] + red[1] + red[2] + red[3];
}

// theta += alpha p; r -= alpha Ap; partials of r.z and r.r.
template <typename R>
__global__ void __launch_bounds__(256) th_update(ThermGeom g, R* __restrict__ theta, R* __restrict__ r,
                                                 const R* __restrict__ p, const R* __restrict__ ap,
                                                 const double* __restrict__ sc,
                                                 double* __restrict__ part) {
  __shared__ double red[4];
  const R alpha = (R)sc[kAlpha];
  double rz = 0.0, rr = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < g.n; i += (size_t)gridDim.x * 256) {
    const NodePos q = node_pos(g, i);
    if (g.oven[q.cls]) continue;
    theta[i] = theta[i] + alpha * p[i];
    const R rn = r[i] - alpha * ap[i];
    r[i] = rn;
    rz += (double)rn * (double)rn * g.inv_diag[q.cls];
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
  // each thread sums its partials k = tid, tid + 256, ... in that order; the
  // loads of eight of them are issued before the first is added
  constexpr int U = 8;
  for (int k0 = threadIdx.x; k0 < nblk; k0 += 256 * U) {
    double va[U], vb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + 256 * u;
      va[u] = k < nblk ? part[stride * k] : 0.0;
      vb[u] = (stride == 2 && k < nblk) ? part[stride * k + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (k0 + 256 * u < nblk) {
        a += va[u];
        b += vb[u];
      }
    }
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

// ---------------------------------------------------------------- direct solve
// The operator divided by the control-volume weights is the Kronecker sum
// L_x + L_y + L_z of 1-D operators on the free nodes (the oven faces are whole
// planes), each L_d = W_d^-1 S_d with S_d symmetric tridiagonal.  With
// W_d^-1/2 S_d W_d^-1/2 = U_d Lambda_d U_d^T for d = x, y:
//   theta = (I x Q_y x Q_x) [ (L_z + lx + ly)^-1 (I x P_y x P_x) f ],
//   P_d = U_d^T W_d^1/2,  Q_d = W_d^-1/2 U_d,  f = b / w = q / k + boundary terms,
// where the middle factor is one tridiagonal solve along z per mode pair.
// The mode products are FP64 GEMMs; these kernels gather f, solve along z and
// scatter theta back.
struct FdmBox {
  int a[3];                 // first free node per direction
  int m[3];                 // free nodes per direction
};

template <typename R>
__global__ void __launch_bounds__(256) fdm_gather(ThermGeom g, FdmBox bx, const R* __restrict__ heat,
                                                  double* __restrict__ f) {
  const size_t n = (size_t)bx.m[0] * bx.m[1] * bx.m[2];
  for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) {
    const int i = (int)(k % bx.m[0]);
    const int j = (int)((k / bx.m[0]) % bx.m[1]);
    const int l = (int)(k / ((size_t)bx.m[0] * bx.m[1]));
    const int x = bx.a[0] + i, y = bx.a[1] + j, z = bx.a[2] + l;
    const size_t idx = ((size_t)z * g.ny + y) * g.nx + x;
    const int cls = node_cls(g, x, y, z);
    f[k] = (double)heat[idx] * g.inv_k + g.src[cls] / g.w[cls];
  }
}

// The z direction is not diagonalised: after the x and y transforms every
// mode pair (i, j) leaves the tridiagonal system (A_z + (lx_i + ly_j) I) u = f
// along z, A_z = W^-1 S the weighted 1-D operator (diagonal dg, off-diagonal
// od[k] in row k).  It is diagonally dominant, so the Thomas algorithm solves
// it without pivoting, in FP64.  f is overwritten by u; cp holds the
// eliminated super-diagonal.  One thread per mode pair walks z (adjacent
// threads touch adjacent addresses), loading kTriU planes at a time so that
// several loads are in flight.
constexpr int kTriU = 16;

__global__ void __launch_bounds__(256) fdm_tri_z(FdmBox bx, const double* __restrict__ lx,
                                                 const double* __restrict__ ly,
                                                 const double* __restrict__ dg,
                                                 const double* __restrict__ od,
                                                 double* __restrict__ f, double* __restrict__ cp) {
  const int m0 = bx.m[0], m2 = bx.m[2];
  const size_t plane = (size_t)m0 * bx.m[1];
  for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < plane; q += (size_t)gridDim.x * 256) {
    const double s = lx[q % m0] + ly[q / m0];
    double c = 0.0, d = 0.0;   // c'_{k-1}, d'_{k-1}
    for (int k0 = 0; k0 < m2; k0 += kTriU) {
      double fv[kTriU];
#pragma unroll
      for (int u = 0; u < kTriU; ++u)
        fv[u] = k0 + u < m2 ? f[(size_t)(k0 + u) * plane + q] : 0.0;
#pragma unroll
      for (int u = 0; u < kTriU; ++u) {
        const int k = k0 + u;
        if (k < m2) {
          const double lk = k > 0 ? od[k] : 0.0;
          const double uk = k + 1 < m2 ? od[k] : 0.0;
          const double r = 1.0 / (dg[k] + s - lk * c);
          c = uk * r;
          d = (fv[u] - lk * d) * r;
          f[(size_t)k * plane + q] = d;
          cp[(size_t)k * plane + q] = c;
        }
      }
    }
    double x = 0.0;
    for (int k1 = m2; k1 > 0; k1 -= kTriU) {   // planes k1 - 1 down to k1 - kTriU
      double dv[kTriU], cv[kTriU];
#pragma unroll
      for (int u = 0; u < kTriU; ++u) {
        const int k = k1 - 1 - u;
        dv[u] = k >= 0 ? f[(size_t)k * plane + q] : 0.0;
        cv[u] = k >= 0 ? cp[(size_t)k * plane + q] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kTriU; ++u) {
        const int k = k1 - 1 - u;
        if (k >= 0) {
          x = dv[u] - cv[u] * x;
          f[(size_t)k * plane + q] = x;
        }
      }
    }
  }
}

// theta (0 on oven nodes) in FP64 and in the solver's precision, and
// T = theta + T_oven.
template <typename R>
__global__ void __launch_bounds__(256) fdm_scatter(ThermGeom g, FdmBox bx, const double* __restrict__ u,
                                                   double t_oven, double* __restrict__ theta64,
                                                   R* __restrict__ t_out) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < g.n; i += (size_t)gridDim.x * 256) {
    const NodePos q = node_pos(g, i);
    double th = 0.0;
    if (!g.oven[q.cls]) {
      const size_t k = ((size_t)(q.c[2] - bx.a[2]) * bx.m[1] + (q.c[1] - bx.a[1])) * bx.m[0] +
                       (q.c[0] - bx.a[0]);
      th = u[k];
    }
    theta64[i] = th;
    t_out[i] = (R)(th + t_oven);
  }
}

// P = U^T W^1/2 and Q = W^-1/2 U (column-major, m x m) from the eigenvectors U
// (column-major, column j = mode j) and the weights w.
__global__ void __launch_bounds__(256) fdm_factors(int m, const double* __restrict__ u,
                                                   const double* __restrict__ w, double* __restrict__ pm,
                                                   double* __restrict__ qm) {
  const size_t n = (size_t)m * m;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    const int row = (int)(e % m), col = (int)(e / m);   // element (row, col) at row + col m
    const double uk = u[e];                              // U(row, col): node row, mode col
    qm[e] = uk / sqrt(w[row]);                           // Q(row, col)
    pm[(size_t)row * m + col] = uk * sqrt(w[row]);       // P(col, row) = U(row, col) sqrt(w_row)
  }
}

}  // namespace shg
