// shg_propagate_adjoint: checkpointed reverse march.
//
// (The L/2 - N - L/2 order stages the state entering each step's RK4 and runs
// the mirrored sequence; see the backward sweep.)
//
// Forward sweep: the march runs in segments of K steps; the real-space state at
// the start of every segment is kept (checkpoints).  Backward sweep, segment by
// segment from the exit: the segment is recomputed from its checkpoint with the
// row passes staging, for every step s, the real-space state u_s that enters the
// second half-step; then the adjoint passes run in reverse order
//   row_adj(top: second half of e-1), [col_adj(s), row_adj(first half of s,
//   second half of s-1)] for s = e-1 .. b+1, col_adj(b), row_adj(first half of b)
// and leave the cotangent of the segment's start state in real space.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "adjoint_kernels.hpp"
#include "plan.hpp"

namespace shg {

template <typename R, int N, int E, int WG>
constexpr bool adj_valid() {
  if constexpr (E > N) return false;
  constexpr int G = N / E;
  constexpr int rows = RowShape<G, WG>::rows;
  constexpr size_t lds = (size_t)rows * 4 * padded_len<N>() * sizeof(cx<R>);
  if (G * rows > 1024 || lds > 64 * 1024) return false;
  if constexpr (sizeof(R) == 8) return (E == 4 || E == 8) && WG == 64;
  return true;
}

template <typename R, int N, int E, int WG>
bool adj_try(int e, int wg, const RowAdjArgs<R>* a, const RowAdjTArgs<R>* q, hipStream_t st,
             int* rows_out) {
  if constexpr (adj_valid<R, N, E, WG>()) {
    if (e != E || wg != WG) return false;
    constexpr int G = N / E;
    using S = RowShape<G, WG>;
    if (rows_out) *rows_out = S::rows;
    if (a && q) {
      hipLaunchKernelGGL((row_adj_pass<R, N, G, S::rows, true>), dim3(a->ny / S::rows),
                         dim3(S::threads), 0, st, *a, *q);
    } else if (a) {
      hipLaunchKernelGGL((row_adj_pass<R, N, G, S::rows, false>), dim3(a->ny / S::rows),
                         dim3(S::threads), 0, st, *a, RowAdjTArgs<R>{});
    }
    return true;
  } else {
    (void)e; (void)wg; (void)a; (void)q; (void)st; (void)rows_out;
    return false;
  }
}

template <typename R, int N>
bool adj_wide_try(int e, int wg, const RowAdjArgs<R>* a, const RowAdjTArgs<R>* q, hipStream_t st,
                  int* rows_out) {
  using S = WideShape<N>;
  constexpr size_t lds = (size_t)(6 * S::rows) * padded_len<N>() * sizeof(cx<R>);
  if constexpr (lds > 64 * 1024) {
    (void)e; (void)wg; (void)a; (void)q; (void)st; (void)rows_out;
    return false;
  } else {
    if (e != 1 || wg != S::threads) return false;
    if (rows_out) *rows_out = S::rows;
    if (a && q) {
      hipLaunchKernelGGL((row_adj_pass_wide<R, N, true>), dim3(a->ny / S::rows), dim3(S::threads),
                         0, st, *a, *q);
    } else if (a) {
      hipLaunchKernelGGL((row_adj_pass_wide<R, N, false>), dim3(a->ny / S::rows),
                         dim3(S::threads), 0, st, *a, RowAdjTArgs<R>{});
    }
    return true;
  }
}

template <typename R, int N>
bool adj_dispatch_n(int e, int wg, const RowAdjArgs<R>* a, const RowAdjTArgs<R>* q,
                    hipStream_t st, int* rows) {
  return adj_wide_try<R, N>(e, wg, a, q, st, rows) || adj_try<R, N, 4, 64>(e, wg, a, q, st, rows) ||
         adj_try<R, N, 4, 256>(e, wg, a, q, st, rows) ||
         adj_try<R, N, 8, 64>(e, wg, a, q, st, rows) ||
         adj_try<R, N, 8, 256>(e, wg, a, q, st, rows) ||
         adj_try<R, N, 16, 64>(e, wg, a, q, st, rows) ||
         adj_try<R, N, 16, 256>(e, wg, a, q, st, rows);
}

template <typename R>
bool adj_dispatch(int n, int e, int wg, const RowAdjArgs<R>* a, const RowAdjTArgs<R>* q,
                  hipStream_t st, int* rows) {
  switch (n) {
    case 16: return adj_dispatch_n<R, 16>(e, wg, a, q, st, rows);
    case 32: return adj_dispatch_n<R, 32>(e, wg, a, q, st, rows);
    case 64: return adj_dispatch_n<R, 64>(e, wg, a, q, st, rows);
    case 128: return adj_dispatch_n<R, 128>(e, wg, a, q, st, rows);
    case 256: return adj_dispatch_n<R, 256>(e, wg, a, q, st, rows);
    case 512: return adj_dispatch_n<R, 512>(e, wg, a, q, st, rows);
    default: return false;
  }
}

// Workspace layout of the adjoint (all offsets 256-byte aligned).
struct AdjLayout {
  size_t fwd, ckpt, work, stage, gp1, gp2, gh;
  size_t psi_work, psi_ckpt, psi_stage, carry, moments;   // temperature field only
  size_t total;
  int segs, k, nblk, nbuf;
};

static AdjLayout adj_layout(const Plan& pl) {
  AdjLayout L{};
  const size_t n2 = (size_t)pl.p.nx * pl.p.ny;
  const size_t state = align256(2 * n2 * 2 * pl.real_bytes);   // both fields
  L.k = pl.ckpt;
  L.segs = (pl.p.nz + L.k - 1) / L.k;
  // with recomputed segments the staging (and the recompute's work fields)
  // are double-buffered: segment k uses buffer k mod 2, so the recompute of
  // segment k - 1 can run while the reverse sweep of segment k reads its own
  L.nbuf = L.segs > 1 ? 2 : 1;
  int rows = 1;
  L.nblk = pl.p.ny;   // upper bound on row-pass blocks
  if (row_supported(pl, pl.adj_e, pl.adj_wg, &rows)) L.nblk = pl.p.ny / rows;
  size_t off = 0;
  L.fwd = off;
  off += align256(forward_ws_bytes(pl));
  L.ckpt = off;
  off += state * (L.segs + 1);
  L.work = off;
  off += state * L.nbuf;
  L.stage = off;
  off += state * L.k * L.nbuf;
  L.gp1 = off;
  off += align256((size_t)pl.p.nz * L.nblk * 2 * sizeof(double));
  L.gp2 = off;
  off += align256((size_t)pl.p.nz * L.nblk * 2 * sizeof(double));
  L.gh = off;
  off += align256((size_t)pl.p.nz * 2 * sizeof(double));
  const size_t rplane = align256(n2 * pl.real_bytes);
  L.psi_work = off;
  off += rplane * L.nbuf;
  L.psi_ckpt = off;
  off += rplane * L.segs;
  L.psi_stage = off;
  off += rplane * L.k * L.nbuf;
  L.carry = off;
  off += align256(n2 * 4 * pl.real_bytes);
  L.moments = off;
  off += align256(n2 * 2 * sizeof(double));
  L.total = off;
  return L;
}

size_t adjoint_ws_bytes(const Plan& pl) { return adj_layout(pl).total; }

// Streams, events and the cached graph of a plan's adjoint.  The recompute of
// segment k - 1 runs on `side` while the reverse sweep of segment k runs on the
// caller's stream: rec[b] marks a recompute into buffer b done, used[b] the
// reverse sweep that read buffer b.
struct AdjCache {
  hipStream_t side = nullptr, cap = nullptr;
  hipEvent_t fork = nullptr, join = nullptr, rec[2] = {}, used[2] = {};
  // cached graphs, most recently used first (a few, for callers that cycle
  // through a few output buffers)
  static constexpr int kGraphs = 4;
  struct Entry {
    std::vector<const void*> key;
    hipGraphExec_t exec;
  };
  std::vector<Entry> graphs;
};

void free_adjoint(Plan& pl) {
  AdjCache* c = (AdjCache*)pl.adj;
  if (!c) return;
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  hipEvent_t evs[] = {c->fork, c->join, c->rec[0], c->rec[1], c->used[0], c->used[1]};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  delete c;
  pl.adj = nullptr;
}

static int adj_cache(Plan& pl, AdjCache** out) {
  if (!pl.adj) {
    AdjCache* c = new (std::nothrow) AdjCache();
    if (!c) return fail(SHG_ENOMEM, "host allocation failed");
    hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    hipEvent_t* evs[] = {&c->fork, &c->join, &c->rec[0], &c->rec[1], &c->used[0], &c->used[1]};
    for (hipEvent_t* ev : evs)
      if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    pl.adj = c;
    if (e != hipSuccess) {
      free_adjoint(pl);
      return hip_fail(e, "adjoint streams and events");
    }
  }
  *out = (AdjCache*)pl.adj;
  return SHG_OK;
}

// side: the stream for the segment recomputes (nullptr: everything on st, in
// the same order).
template <typename R>
static int adjoint_t(Plan& pl, const void* a_f_in, const void* a_sh_in, const double* dk_z,
                     const void* temp, const void* g_f_out, const void* g_sh_out,
                     const double* pw, void* g_f_in, void* g_sh_in, double* g_dk, double* g_t,
                     void* a_f_out, void* a_sh_out, double* powers, char* ws, hipStream_t st,
                     AdjCache* ac) {
  const shg_params& p = pl.p;
  const AdjLayout L = adj_layout(pl);
  const size_t n2 = (size_t)p.nx * p.ny;
  const size_t state = align256(2 * n2 * sizeof(cx<R>));
  auto ck = [&](int k) { return (cx<R>*)(ws + L.ckpt + state * k); };
  // per-segment buffers: segment k uses buffer k mod nbuf
  auto work_of = [&](int k) { return (cx<R>*)(ws + L.work + state * (k % L.nbuf)); };
  auto stage_of = [&](int k) { return (cx<R>*)(ws + L.stage + state * L.k * (k % L.nbuf)); };
  double* gp1 = (double*)(ws + L.gp1);
  double* gp2 = (double*)(ws + L.gp2);
  double* gh = (double*)(ws + L.gh);
  char* fws = ws + L.fwd;
  cx<R>* fin_a = a_f_out ? (cx<R>*)a_f_out : ck(L.segs);
  cx<R>* fin_b = a_sh_out ? (cx<R>*)a_sh_out : ck(L.segs) + n2;
  auto seg_in = [&](int k, const void** a, const void** b) {
    if (k == 0) {
      *a = a_f_in;
      *b = a_sh_in;
    } else {
      *a = ck(k);
      *b = ck(k) + n2;
    }
  };
  int rc;
  const bool th = temp != nullptr;
  const size_t rplane = align256(n2 * sizeof(R));
  auto psi_work_of = [&](int k) { return (R*)(ws + L.psi_work + rplane * (k % L.nbuf)); };
  auto psi_ck = [&](int k) { return (R*)(ws + L.psi_ckpt + rplane * k); };
  auto psi_stage_of = [&](int k) {
    return (R*)(ws + L.psi_stage + rplane * L.k * (k % L.nbuf));
  };
  Carry<R>* carry = (Carry<R>*)(ws + L.carry);
  double* moments = (double*)(ws + L.moments);
  const unsigned nb = (unsigned)((n2 + 255) / 256);
  if (th) {
    hipLaunchKernelGGL((psi_init<R>), dim3(nb), dim3(256), 0, st, (const R*)temp, 0, p.t_ref,
                       make_dk_shift<double>(p.ddk_dT, p.ddk_dT2, p.ddk_dT3, p.grating_period,
                                             p.grating_a, p.grating_b, p.t_ref),
                       pl.dz, psi_work_of(0), n2);
  }
  // ---- forward sweep with checkpoints
  for (int k = 0; k < L.segs; ++k) {
    const int b = k * L.k, e = std::min(p.nz, b + L.k);
    const void *ia, *ib;
    seg_in(k, &ia, &ib);
    const bool last = (k == L.segs - 1);
    // the last segment stages its states now, so the backward sweep starts
    // without recomputing it
    cx<R>* w = work_of(0);
    FwdIO io{ia, ib, w, w + n2, last ? (void*)fin_a : (void*)ck(k + 1),
             last ? (void*)fin_b : (void*)(ck(k + 1) + n2), last ? stage_of(k) : nullptr};
    if (th) {
      hipLaunchKernelGGL((copy_real<R>), dim3(nb), dim3(256), 0, st, (const R*)psi_work_of(0),
                         psi_ck(k), n2);
      io.temp = temp;
      io.psi = psi_work_of(0);
      io.tap_psi = last ? psi_stage_of(k) : nullptr;
    }
    rc = enqueue_forward_io(pl, io, dk_z, b, e, fws, last ? powers : nullptr, st, k == 0);
    if (rc) return rc;
  }
  // ---- cotangent of the exit fields
  cx<R>* la = (cx<R>*)g_f_in;
  cx<R>* lb = (cx<R>*)g_sh_in;
  hipLaunchKernelGGL((adjoint_seed<R>), dim3((n2 + 255) / 256), dim3(256), 0, st,
                     (const cx<R>*)g_f_out, (const cx<R>*)g_sh_out, (const cx<R>*)fin_a,
                     (const cx<R>*)fin_b, pw, pl.pscale_f, pl.pscale_sh, la, lb, n2);
  // ---- backward sweep
  RowAdjArgs<R> ra{};
  ra.la = la;
  ra.lb = lb;
  ra.tw = (const Tw<R>*)pl.tw_x;
  ra.phase = (const StageCoef<R>*)fws;
  ra.ny = p.ny;
  ra.kf = (R)pl.kappa_f;
  ra.ks = (R)pl.kappa_sh;
  ra.tf = (R)(pl.tpa_f / 2.0);
  ra.ts = (R)(pl.tpa_sh / 2.0);
  ra.h = (R)(pl.dz / 2.0);
  ra.undepleted = (p.flags & SHG_UNDEPLETED) ? 1 : 0;
  const size_t gstride = (size_t)L.nblk * 2;
  auto g1 = [&](int s) { return g_dk ? gp1 + gstride * s : nullptr; };
  auto g2 = [&](int s) { return g_dk ? gp2 + gstride * s : nullptr; };
  RowAdjTArgs<R> q{};
  RowAdjTArgs<R>* qp = nullptr;
  if (th) {
    q.temp = (const R*)temp;
    q.carry = carry;
    q.moments = moments;
    q.t_ref = (R)p.t_ref;
    q.dk = make_dk_shift<R>(p.ddk_dT, p.ddk_dT2, p.ddk_dT3, p.grating_period, p.grating_a,
                            p.grating_b, p.t_ref);
    q.lens_f = (R)pl.lens_f;
    q.lens_sh = (R)pl.lens_sh;
    q.dz = (R)pl.dz;
    qp = &q;
    hipLaunchKernelGGL((zero_carry<R>), dim3(nb), dim3(256), 0, st, carry, moments, n2);
  }
  auto adj = [&](RowAdjArgs<R>& a, const R* psi, int* rows) {
    q.psi = psi;
    return adj_dispatch<R>(p.nx, pl.adj_e, pl.adj_wg, &a, qp, st, rows);
  };
  int rows = 1;
  const bool lnl = (p.flags & SHG_SPLIT_LNL) != 0;
  ra.full = lnl ? 1 : 0;
  // recompute segment k from its checkpoint on stream rs, staging every step
  auto recompute = [&](int k, hipStream_t rs) {
    const int b = k * L.k, e = std::min(p.nz, b + L.k);
    const void *ia, *ib;
    seg_in(k, &ia, &ib);
    cx<R>* w = work_of(k);
    FwdIO io{ia, ib, w, w + n2, w, w + n2, stage_of(k)};
    if (th) {
      hipLaunchKernelGGL((copy_real<R>), dim3(nb), dim3(256), 0, rs, (const R*)psi_ck(k),
                         psi_work_of(k), n2);
      io.temp = temp;
      io.psi = psi_work_of(k);
      io.tap_psi = psi_stage_of(k);
    }
    return enqueue_forward_io(pl, io, dk_z, b, e, fws, nullptr, rs, false);
  };
  // pull the cotangent back through segment k, whose staged states are in
  // buffer k mod nbuf
  auto reverse_lnl = [&](int k) -> int {
    // L/2 - N - L/2: a segment [b, e) runs FFT_x, a half-step column pass, per
    // step s the row pass IFFT_x . RK4 over dz . FFT_x and a column pass (the
    // half-step one after the last step), and IFFT_x.  Its pull-back, in
    // reverse: FFT_x; conj(M_half); per step s = e-1 .. b the adjoint row pass
    // of s (from the staged RK4 input) and conj(M) of the column pass before s
    // (the half-step one for s = b); IFFT_x.
    const int b = k * L.k, e = std::min(p.nz, b + L.k);
    const void *ia, *ib;
    seg_in(k, &ia, &ib);
    cx<R>* stg = stage_of(k);
    R* spsi = psi_stage_of(k);
    auto staged = [&](int s) { return stg + (size_t)(s - b) * 2 * n2; };
    auto sp = [&](int s) { return spsi + (size_t)(s - b) * n2; };
    ra.ua = staged(e - 1);
    ra.ub = staged(e - 1) + n2;
    ra.s_second = ra.s_first = -1;
    ra.inv_in = 0;
    ra.fwd_out = 1;
    ra.gp_first = ra.gp_second = nullptr;
    if (!adj(ra, sp(e - 1), &rows))
      return fail(SHG_EUNSUPPORTED, "adjoint row schedule e=%d wg=%d not built", pl.adj_e,
                  pl.adj_wg);
    int r;
    if ((r = launch_col(pl, la, lb, 1, st, true))) return r;
    for (int s = e - 1; s >= b; --s) {
      ra.ua = staged(s);
      ra.ub = staged(s) + n2;
      ra.s_first = s;
      ra.inv_in = 1;
      ra.fwd_out = 1;
      ra.gp_first = g1(s);
      adj(ra, sp(s), &rows);
      if ((r = launch_col(pl, la, lb, 1, st, s == b))) return r;
    }
    ra.ua = (const cx<R>*)ia;
    ra.ub = (const cx<R>*)ib;
    ra.s_first = -1;
    ra.inv_in = 1;
    ra.fwd_out = 0;
    ra.gp_first = nullptr;
    adj(ra, th ? psi_ck(k) : nullptr, &rows);
    return (int)SHG_OK;
  };
  auto reverse_nln = [&](int k) -> int {
    const int b = k * L.k, e = std::min(p.nz, b + L.k);
    const void *ia, *ib;
    seg_in(k, &ia, &ib);
    cx<R>* stg = stage_of(k);
    R* spsi = psi_stage_of(k);
    auto staged = [&](int s) { return stg + (size_t)(s - b) * 2 * n2; };
    auto sp = [&](int s) { return spsi + (size_t)(s - b) * n2; };
    // top: second half-step of step e-1, lambda in real space
    ra.ua = staged(e - 1);
    ra.ub = staged(e - 1) + n2;
    ra.s_second = e - 1;
    ra.s_first = -1;
    ra.inv_in = 0;
    ra.fwd_out = 1;
    ra.gp_first = nullptr;
    ra.gp_second = g2(e - 1);
    if (!adj(ra, sp(e - 1), &rows))
      return fail(SHG_EUNSUPPORTED, "adjoint row schedule e=%d wg=%d not built", pl.adj_e,
                  pl.adj_wg);
    int r;
    for (int s = e - 1; s > b; --s) {
      if ((r = launch_col(pl, la, lb, 1, st))) return r;
      ra.ua = staged(s - 1);
      ra.ub = staged(s - 1) + n2;
      ra.s_second = s - 1;
      ra.s_first = s;
      ra.inv_in = 1;
      ra.fwd_out = 1;
      ra.gp_first = g1(s);
      ra.gp_second = g2(s - 1);
      adj(ra, sp(s - 1), &rows);
    }
    if ((r = launch_col(pl, la, lb, 1, st))) return r;
    ra.ua = (const cx<R>*)ia;
    ra.ub = (const cx<R>*)ib;
    ra.s_second = -1;
    ra.s_first = b;
    ra.inv_in = 1;
    ra.fwd_out = 0;
    ra.gp_first = g1(b);
    ra.gp_second = nullptr;
    adj(ra, th ? psi_ck(k) : nullptr, &rows);
    return (int)SHG_OK;
  };
  // Segments from the exit down: the recompute of segment k - 1 is enqueued
  // before the reverse sweep of segment k.  With a side stream it runs there,
  // concurrently, after the reverse sweep of segment k + 1 (the last reader of
  // its buffer); the reverse sweep of k waits for the recompute of k.  Without
  // one the same order on st is already correct (different buffers).
  hipStream_t side = (ac && L.segs > 1) ? ac->side : nullptr;
  hipError_t e = hipSuccess;
  if (side) {
    e = hipEventRecord(ac->fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, ac->fork, 0);
    if (e != hipSuccess) return hip_fail(e, "fork of the recompute stream");
  }
  for (int k = L.segs - 1; k >= 0; --k) {
    if (k >= 1) {
      if (side) {
        if (k + 1 <= L.segs - 1) e = hipStreamWaitEvent(side, ac->used[(k - 1) % 2], 0);
        if (e != hipSuccess) return hip_fail(e, "recompute stream wait");
        if ((rc = recompute(k - 1, side))) return rc;
        e = hipEventRecord(ac->rec[(k - 1) % 2], side);
        if (e != hipSuccess) return hip_fail(e, "recompute stream record");
      } else if ((rc = recompute(k - 1, st))) {
        return rc;
      }
    }
    if (side && k < L.segs - 1) {
      e = hipStreamWaitEvent(st, ac->rec[k % 2], 0);
      if (e != hipSuccess) return hip_fail(e, "wait for a recomputed segment");
    }
    if ((rc = lnl ? reverse_lnl(k) : reverse_nln(k))) return rc;
    if (side) {
      e = hipEventRecord(ac->used[k % 2], st);
      if (e != hipSuccess) return hip_fail(e, "reverse sweep record");
    }
  }
  if (side) {
    e = hipEventRecord(ac->join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ac->join, 0);
    if (e != hipSuccess) return hip_fail(e, "join of the recompute stream");
  }
  if (th && g_t) {
    hipLaunchKernelGGL(moments_finalize, dim3(1), dim3(256), 0, st, (const double*)moments, n2,
                       g_t);
  }
  if (g_dk) {
    hipLaunchKernelGGL(grad_step_sums, dim3(p.nz), dim3(256), 0, st, (const double*)gp1,
                       lnl ? nullptr : (const double*)gp2, p.ny / rows, gh);
    hipLaunchKernelGGL(grad_dk_finalize, dim3(1), dim3(256), 0, st, (const double*)gh, p.nz,
                       pl.dz, g_dk);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return SHG_OK;
}

int propagate_adjoint(Plan& pl, const void* a_f_in, const void* a_sh_in, const double* dk_z,
                      const void* temp, const void* g_f_out, const void* g_sh_out,
                      const double* pw, void* g_f_in, void* g_sh_in, double* g_dk,
                      double* g_t, void* a_f_out, void* a_sh_out, double* powers, void* ws,
                      hipStream_t st) {
  if (!a_f_in || !a_sh_in) return fail(SHG_EINVAL, "a_f_in and a_sh_in must be non-NULL");
  if (!g_f_in || !g_sh_in) return fail(SHG_EINVAL, "g_f_in and g_sh_in must be non-NULL");
  if (!ws) return fail(SHG_EINVAL, "workspace must be non-NULL (shg_workspace_bytes(plan, 1))");
  if (g_t && !temp) return fail(SHG_EINVAL, "g_t_moments requires a temperature field");
  int rc = sticky_device_error();
  if (rc) return rc;
  const size_t field = 2 * (size_t)pl.p.nx * pl.p.ny;
  if (checks_finite(pl)) {
    if ((rc = check_finite(pl, a_f_in, field, false, "input a_f_in", st)) ||
        (rc = check_finite(pl, a_sh_in, field, false, "input a_sh_in", st)) ||
        (rc = check_finite(pl, dk_z, (size_t)pl.p.nz, true, "dk_z", st)) ||
        (rc = check_finite(pl, temp, (size_t)pl.p.nz * field / 2, false, "temp", st)) ||
        (rc = check_finite(pl, g_f_out, field, false, "g_f_out", st)) ||
        (rc = check_finite(pl, g_sh_out, field, false, "g_sh_out", st)) ||
        (rc = check_finite(pl, pw, 2, true, "power_weights", st)))
      return rc;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  const bool capturing = cs != hipStreamCaptureStatusNone;
  // the side stream and events are created on the first call outside capture;
  // a call under the caller's capture before that runs on its stream alone
  AdjCache* ac = (AdjCache*)pl.adj;
  if (!capturing && (rc = adj_cache(pl, &ac))) return rc;
  auto run = [&](hipStream_t s) {
    return pl.dtype == SHG_C64
               ? adjoint_t<float>(pl, a_f_in, a_sh_in, dk_z, temp, g_f_out, g_sh_out, pw, g_f_in,
                                  g_sh_in, g_dk, g_t, a_f_out, a_sh_out, powers, (char*)ws, s, ac)
               : adjoint_t<double>(pl, a_f_in, a_sh_in, dk_z, temp, g_f_out, g_sh_out, pw,
                                   g_f_in, g_sh_in, g_dk, g_t, a_f_out, a_sh_out, powers,
                                   (char*)ws, s, ac);
  };
  if (capturing || (pl.p.flags & SHG_NO_GRAPH) || pl.timing) {
    rc = run(st);
  } else {
    // replay a cached graph of the whole forward + reverse sequence (its two
    // streams become parallel branches) while the arguments stay the same
    const std::vector<const void*> key = {
        a_f_in, a_sh_in, dk_z, temp, g_f_out, g_sh_out, pw, g_f_in, g_sh_in, g_dk, g_t,
        a_f_out, a_sh_out, powers, ws,
        reinterpret_cast<const void*>((uintptr_t)(pl.row_e * 1000 + pl.row_wg)),
        reinterpret_cast<const void*>((uintptr_t)(pl.adj_e * 1000 + pl.adj_wg)),
        reinterpret_cast<const void*>((uintptr_t)(pl.col_e * 1000 + pl.col_tc))};
    size_t hit = 0;
    while (hit < ac->graphs.size() && ac->graphs[hit].key != key) ++hit;
    if (hit == ac->graphs.size()) {
      if (!ac->cap) {
        e = hipStreamCreateWithFlags(&ac->cap, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
      }
      e = hipStreamBeginCapture(ac->cap, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
      rc = run(ac->cap);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(ac->cap, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
      hipGraphExec_t exec = nullptr;
      e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
      if ((int)ac->graphs.size() == AdjCache::kGraphs) {
        (void)hipGraphExecDestroy(ac->graphs.back().exec);
        ac->graphs.pop_back();
      }
      ac->graphs.insert(ac->graphs.begin(), AdjCache::Entry{key, exec});
    } else if (hit > 0) {
      std::rotate(ac->graphs.begin(), ac->graphs.begin() + hit, ac->graphs.begin() + hit + 1);
    }
    e = hipGraphLaunch(ac->graphs.front().exec, st);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  if (rc || !checks_finite(pl)) return rc;
  if ((rc = check_finite(pl, g_f_in, field, false, "the adjoint's output g_f_in", st)) ||
      (rc = check_finite(pl, g_sh_in, field, false, "the adjoint's output g_sh_in", st)))
    return rc;
  return SHG_OK;
}

}  // namespace shg

using namespace shg;

extern "C" int shg_propagate_adjoint(shg_plan* plan, const void* a_f_in, const void* a_sh_in,
                                     const double* dk_z, const void* temp, const void* g_f_out,
                                     const void* g_sh_out, const double* power_weights,
                                     void* g_f_in, void* g_sh_in, double* g_dk_z,
                                     double* g_t_moments, void* a_f_out, void* a_sh_out,
                                     double* powers, void* workspace, void* stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  Plan* pl = reinterpret_cast<Plan*>(plan);
  rc = propagate_adjoint(*pl, a_f_in, a_sh_in, dk_z, temp, g_f_out, g_sh_out, power_weights,
                         g_f_in, g_sh_in, g_dk_z, g_t_moments, a_f_out, a_sh_out, powers,
                         workspace, (hipStream_t)stream);
  return rc ? rc : ok();
}
