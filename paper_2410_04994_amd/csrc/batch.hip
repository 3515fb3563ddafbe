// shg_propagate_batch: many independent instances marched in lock-step passes.
//
// Instances are grouped by (grid, schedule); inside a group they are ordered by
// decreasing nz so that at every boundary the instances still marching form a
// prefix.  Per boundary s there is one row-pass launch per group (gridDim.y =
// instances with nz >= s) and per step one column-pass launch per group
// (gridDim.y = instances with nz > s).  Groups are spread over up to four
// streams forked from the caller's stream and joined back before the exit
// powers, so groups run concurrently.  The whole sequence is captured once into
// a HIP graph (the streams become parallel branches) and replayed while the
// arguments stay the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

namespace shg {

template <typename R, int N, int E, int WG>
constexpr bool brow_valid() {
  if constexpr (E > N) return false;
  constexpr int G = N / E;
  constexpr int rows = RowShape<G, WG>::rows;
  constexpr size_t lds = (size_t)rows * 4 * padded_len<N>() * sizeof(cx<R>);
  if (G * rows > 1024 || lds > 64 * 1024) return false;
  if constexpr (sizeof(R) == 8) return (E == 4 || E == 8) && WG == 64;
  return true;
}

template <typename R, int N, int E, int TC>
constexpr bool bcol_valid() {
  if constexpr (E > N) return false;
  constexpr int G = N / E;
  constexpr size_t lds = (size_t)2 * padded_len<N>() * TC * sizeof(cx<R>);
  if (G * TC < 32 || G * TC > 512 || lds > 64 * 1024) return false;
  if constexpr (sizeof(R) == 8) return (E == 4 || E == 8) && G * TC <= 128;
  return true;
}

template <typename R, int N, int E, int WG>
bool brow_try(int e, int wg, const BatchInst<R>* d, int count, int s, int blocks,
              hipStream_t st) {
  if constexpr (brow_valid<R, N, E, WG>()) {
    if (e != E || wg != WG) return false;
    constexpr int G = N / E;
    using S = RowShape<G, WG>;
    hipLaunchKernelGGL((row_pass_batch<R, N, G, S::rows>), dim3(blocks, count), dim3(S::threads),
                       0, st, d, s);
    return true;
  } else {
    (void)e; (void)wg; (void)d; (void)count; (void)s; (void)blocks; (void)st;
    return false;
  }
}

template <typename R, int N, int E, int TC>
bool bcol_try(int e, int tc, const BatchInst<R>* d, int count, int s, int blocks, hipStream_t st) {
  if constexpr (bcol_valid<R, N, E, TC>()) {
    if (e != E || tc != TC) return false;
    hipLaunchKernelGGL((col_pass_batch<R, N, N / E, TC>), dim3(blocks, count),
                       dim3((N / E) * TC), 0, st, d, s);
    return true;
  } else {
    (void)e; (void)tc; (void)d; (void)count; (void)s; (void)blocks; (void)st;
    return false;
  }
}

template <typename R, int N>
bool brow_wide_try(int e, int wg, const BatchInst<R>* d, int count, int s, int blocks,
                   hipStream_t st) {
  using S = WideShape<N>;
  constexpr size_t lds = (size_t)(6 * S::rows) * padded_len<N>() * sizeof(cx<R>);
  if constexpr (lds > 64 * 1024) {
    (void)e; (void)wg; (void)d; (void)count; (void)s; (void)blocks; (void)st;
    return false;
  } else {
    if (e != 1 || wg != S::threads) return false;
    hipLaunchKernelGGL((row_pass_batch_wide<R, N>), dim3(blocks, count), dim3(S::threads), 0, st,
                       d, s);
    return true;
  }
}

template <typename R, int N>
bool brow_n(int e, int wg, const BatchInst<R>* d, int c, int s, int b, hipStream_t st) {
  return brow_wide_try<R, N>(e, wg, d, c, s, b, st) || brow_try<R, N, 4, 64>(e, wg, d, c, s, b, st) ||
         brow_try<R, N, 4, 256>(e, wg, d, c, s, b, st) ||
         brow_try<R, N, 8, 64>(e, wg, d, c, s, b, st) ||
         brow_try<R, N, 8, 256>(e, wg, d, c, s, b, st) ||
         brow_try<R, N, 16, 64>(e, wg, d, c, s, b, st) ||
         brow_try<R, N, 16, 256>(e, wg, d, c, s, b, st);
}

template <typename R, int N>
bool bcol_n(int e, int tc, const BatchInst<R>* d, int c, int s, int b, hipStream_t st) {
  return bcol_try<R, N, 4, 1>(e, tc, d, c, s, b, st) || bcol_try<R, N, 4, 2>(e, tc, d, c, s, b, st) ||
         bcol_try<R, N, 4, 4>(e, tc, d, c, s, b, st) || bcol_try<R, N, 4, 8>(e, tc, d, c, s, b, st) ||
         bcol_try<R, N, 4, 16>(e, tc, d, c, s, b, st) || bcol_try<R, N, 8, 1>(e, tc, d, c, s, b, st) ||
         bcol_try<R, N, 8, 2>(e, tc, d, c, s, b, st) || bcol_try<R, N, 8, 4>(e, tc, d, c, s, b, st) ||
         bcol_try<R, N, 8, 8>(e, tc, d, c, s, b, st) || bcol_try<R, N, 8, 16>(e, tc, d, c, s, b, st) ||
         bcol_try<R, N, 16, 1>(e, tc, d, c, s, b, st) || bcol_try<R, N, 16, 2>(e, tc, d, c, s, b, st) ||
         bcol_try<R, N, 16, 4>(e, tc, d, c, s, b, st) || bcol_try<R, N, 16, 8>(e, tc, d, c, s, b, st) ||
         bcol_try<R, N, 16, 16>(e, tc, d, c, s, b, st);
}

template <typename R>
bool brow(int n, int e, int wg, const BatchInst<R>* d, int c, int s, int b, hipStream_t st) {
  switch (n) {
    case 16: return brow_n<R, 16>(e, wg, d, c, s, b, st);
    case 32: return brow_n<R, 32>(e, wg, d, c, s, b, st);
    case 64: return brow_n<R, 64>(e, wg, d, c, s, b, st);
    case 128: return brow_n<R, 128>(e, wg, d, c, s, b, st);
    case 256: return brow_n<R, 256>(e, wg, d, c, s, b, st);
    case 512: return brow_n<R, 512>(e, wg, d, c, s, b, st);
    default: return false;
  }
}

template <typename R>
bool bcol(int n, int e, int tc, const BatchInst<R>* d, int c, int s, int b, hipStream_t st) {
  switch (n) {
    case 16: return bcol_n<R, 16>(e, tc, d, c, s, b, st);
    case 32: return bcol_n<R, 32>(e, tc, d, c, s, b, st);
    case 64: return bcol_n<R, 64>(e, tc, d, c, s, b, st);
    case 128: return bcol_n<R, 128>(e, tc, d, c, s, b, st);
    case 256: return bcol_n<R, 256>(e, tc, d, c, s, b, st);
    case 512: return bcol_n<R, 512>(e, tc, d, c, s, b, st);
    default: return false;
  }
}

// Size groups are marched on up to this many concurrent streams, so that the
// small launches of one group (late z-steps, few active instances) overlap
// with the work of the others.
constexpr int kMaxBranches = 4;

struct Group {
  int nx, ny, re, rw, ce, ct, rows;
  int offset;                 // first descriptor of the group
  std::vector<int> nzs;       // nz of the group's instances, decreasing
};

struct BatchPlanInfo {
  bool lnl = false;                          // every plan uses the L/2 - N - L/2 order
  std::vector<Group> groups;
  std::vector<std::vector<int>> branches;   // group indices per stream
  std::vector<int> order;     // descriptor slot -> caller index
  size_t total = 0;   // workspace bytes: per-instance phase tables and power partials
  std::vector<size_t> phase_at, part_at;   // per caller index
};

// Batch state cached on the first plan of the batch.
struct BatchCache {
  std::vector<const void*> key;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  // descriptor table in device memory owned by the cache (not the caller's
  // workspace, which another batch may fill between two replays)
  void* desc = nullptr;
  size_t desc_cap = 0;
  // side streams for the size groups (parallel branches of the captured graph)
  hipStream_t side[kMaxBranches] = {};
  hipEvent_t fork = nullptr, join[kMaxBranches] = {};
};

static int build_info(int n, shg_plan* const* plans, BatchPlanInfo& bi) {
  std::map<std::tuple<int, int, int, int, int, int>, std::vector<int>> by;
  for (int i = 0; i < n; ++i) {
    const Plan& pl = *reinterpret_cast<const Plan*>(plans[i]);
    by[std::make_tuple(pl.p.nx, pl.p.ny, pl.b_row_e, pl.b_row_wg, pl.b_col_e, pl.b_col_tc)]
        .push_back(i);
  }
  const Plan& p0 = *reinterpret_cast<const Plan*>(plans[0]);
  bi.lnl = (p0.p.flags & SHG_SPLIT_LNL) != 0;
  const size_t csize = 2 * (size_t)p0.real_bytes;
  bi.groups.clear();
  bi.order.clear();
  for (auto& kv : by) {
    std::vector<int>& idx = kv.second;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
      return reinterpret_cast<const Plan*>(plans[a])->p.nz > reinterpret_cast<const Plan*>(plans[b])->p.nz;
    });
    Group g{};
    std::tie(g.nx, g.ny, g.re, g.rw, g.ce, g.ct) = kv.first;
    const Plan& pf = *reinterpret_cast<const Plan*>(plans[idx[0]]);
    if (!row_supported(pf, g.re, g.rw, &g.rows))
      return fail(SHG_EUNSUPPORTED, "row schedule e=%d wg=%d not built", g.re, g.rw);
    g.offset = (int)bi.order.size();
    for (int i : idx) {
      bi.order.push_back(i);
      g.nzs.push_back(reinterpret_cast<const Plan*>(plans[i])->p.nz);
    }
    bi.groups.push_back(g);
  }
  size_t off = 0;
  bi.phase_at.assign(n, 0);
  bi.part_at.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    const Plan& pl = *reinterpret_cast<const Plan*>(plans[i]);
    bi.phase_at[i] = off;
    off += align256((size_t)pl.p.nz * 5 * 2 * csize);   // [nz][5] StageCoef
    bi.part_at[i] = off;
    off += align256((size_t)pl.p.ny * 2 * sizeof(double));
  }
  bi.total = off;
  // longest-first assignment of the groups to the branches by cell-steps
  std::vector<std::pair<double, int>> work;
  for (int gi = 0; gi < (int)bi.groups.size(); ++gi) {
    double w = 0.0;
    for (int nz : bi.groups[gi].nzs) w += (double)nz;
    work.push_back({w * bi.groups[gi].nx * bi.groups[gi].ny, gi});
  }
  std::sort(work.begin(), work.end(), [](auto a, auto b) { return a.first > b.first; });
  const int nb = std::min<int>(kMaxBranches, (int)bi.groups.size());
  bi.branches.assign(nb, {});
  std::vector<double> load(nb, 0.0);
  for (auto& w : work) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    bi.branches[b].push_back(w.second);
    load[b] += w.first;
  }
  for (auto& br : bi.branches) std::sort(br.begin(), br.end());
  return SHG_OK;
}

static int validate_batch(int n, shg_plan* const* plans, void* const* a_f, void* const* a_sh) {
  if (n < 1) return fail(SHG_EINVAL, "n=%d must be >= 1", n);
  if (n > 65535) return fail(SHG_EINVAL, "n=%d exceeds 65535 instances", n);
  if (!plans || !a_f || !a_sh) return fail(SHG_EINVAL, "plans, a_f and a_sh must be non-NULL");
  int rc;
  for (int i = 0; i < n; ++i) {
    if ((rc = check_plan(plans[i]))) return fail(rc, "plans[%d]: %s", i, shg_last_error());
    if (!a_f[i] || !a_sh[i]) return fail(SHG_EINVAL, "a_f[%d] / a_sh[%d] is NULL", i, i);
    const Plan& pl = *reinterpret_cast<const Plan*>(plans[i]);
    const Plan& p0 = *reinterpret_cast<const Plan*>(plans[0]);
    if (pl.dtype != p0.dtype) return fail(SHG_EINVAL, "plans[%d] dtype differs from plans[0]", i);
    if ((pl.p.flags & SHG_SPLIT_LNL) != (p0.p.flags & SHG_SPLIT_LNL))
      return fail(SHG_EINVAL, "plans[%d] uses another split order than plans[0]", i);
  }
  return SHG_OK;
}

template <typename R>
static int enqueue_batch(int n, shg_plan* const* plans, void* const* a_f, void* const* a_sh,
                         const double* const* dk_z, char* ws, double* powers,
                         const BatchPlanInfo& bi, hipStream_t st, bool upload,
                         const BatchCache* side, void* desc) {
  BatchInst<R>* dev = (BatchInst<R>*)desc;
  if (upload) {
    std::vector<BatchInst<R>> host(n);
    for (int slot = 0; slot < n; ++slot) {
      const int i = bi.order[slot];
      const Plan& pl = *reinterpret_cast<const Plan*>(plans[i]);
      BatchInst<R>& I = host[slot];
      std::memset(&I, 0, sizeof(I));
      RowArgs<R>& r = I.row;
      r.ain = r.aout = (cx<R>*)a_f[i];
      r.bin = r.bout = (cx<R>*)a_sh[i];
      r.tw = (const Tw<R>*)pl.tw_x;
      r.phase = (const StageCoef<R>*)(ws + bi.phase_at[i]);
      r.ny = pl.p.ny;
      r.kf = (R)pl.kappa_f;
      r.ks = (R)pl.kappa_sh;
      r.tf = (R)(pl.tpa_f / 2.0);
      r.ts = (R)(pl.tpa_sh / 2.0);
      r.h = (R)(pl.dz / 2.0);
      r.undepleted = (pl.p.flags & SHG_UNDEPLETED) ? 1 : 0;
      ColArgs<R>& c = I.col;
      c.f[0] = (cx<R>*)a_f[i];
      c.f[1] = (cx<R>*)a_sh[i];
      c.tw = (const Tw<R>*)pl.tw_y;
      for (int w = 0; w < 2; ++w) {
        c.mx[w] = pl.mx[w];
        c.my[w] = pl.my[w];
      }
      c.nx = pl.p.nx;
      c.tiles = pl.p.nx / pl.b_col_tc;
      c.conj_prop = 0;
      I.lnl = (pl.p.flags & SHG_SPLIT_LNL) ? 1 : 0;
      for (int w = 0; w < 2; ++w) {
        I.mxh[w] = pl.mxh[w];
        I.myh[w] = pl.myh[w];
      }
      I.dk_z = dk_z ? dk_z[i] : nullptr;
      I.dk0 = pl.p.dk0;
      I.dz = pl.dz;
      I.pscale_f = pl.pscale_f;
      I.pscale_sh = pl.pscale_sh;
      I.partials = (double*)(ws + bi.part_at[i]);
      I.powers = powers ? powers + 2 * i : nullptr;
      I.nz = pl.p.nz;
      int brows = 1;
      row_supported(pl, pl.b_row_e, pl.b_row_wg, &brows);
      I.row_blocks = pl.p.ny / brows;
    }
    hipError_t e = hipMemcpyAsync(dev, host.data(), sizeof(BatchInst<R>) * n,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "upload of batch descriptors");
  }
  hipLaunchKernelGGL((phase_table_batch<R>), dim3(n), dim3(256), 0, st, (const BatchInst<R>*)dev);
  hipError_t e = hipSuccess;
  const int nb = (int)bi.branches.size();
  const bool fork = nb > 1 && side;
  if (fork) {
    e = hipEventRecord(side->fork, st);
    for (int b = 0; b < nb && e == hipSuccess; ++b) e = hipStreamWaitEvent(side->side[b], side->fork, 0);
    if (e != hipSuccess) return hip_fail(e, "fork of the batch streams");
  }
  for (int b = 0; b < nb; ++b) {
    hipStream_t bs = fork ? side->side[b] : st;
    int max_nz = 0;
    for (int gi : bi.branches[b]) max_nz = std::max(max_nz, bi.groups[gi].nzs[0]);
    if (bi.lnl) {
      // L/2 - N - L/2: opening FFT_x and half-step column pass of every instance
      for (int gi : bi.branches[b]) {
        const Group& g = bi.groups[gi];
        const int cnt = (int)g.nzs.size();
        if (!brow<R>(g.nx, g.re, g.rw, dev + g.offset, cnt, -1, g.ny / g.rows, bs))
          return fail(SHG_EUNSUPPORTED, "batched row schedule not built");
        if (!bcol<R>(g.ny, g.ce, g.ct, dev + g.offset, cnt, -1, 2 * (g.nx / g.ct), bs))
          return fail(SHG_EUNSUPPORTED, "batched column schedule not built");
      }
    }
    for (int s = 0; s <= max_nz; ++s) {
      for (int gi : bi.branches[b]) {
        const Group& g = bi.groups[gi];
        // instances with nz >= s still have boundary s
        const int cnt = (int)(std::upper_bound(g.nzs.begin(), g.nzs.end(), s, std::greater<int>()) -
                              g.nzs.begin());
        if (cnt == 0) continue;
        if (!brow<R>(g.nx, g.re, g.rw, dev + g.offset, cnt, s, g.ny / g.rows, bs))
          return fail(SHG_EUNSUPPORTED, "batched row schedule not built");
      }
      if (s == max_nz) break;
      for (int gi : bi.branches[b]) {
        const Group& g = bi.groups[gi];
        // instances with nz > s run step s
        const int cnt = (int)(std::lower_bound(g.nzs.begin(), g.nzs.end(), s, std::greater<int>()) -
                              g.nzs.begin());
        if (cnt == 0) continue;
        if (!bcol<R>(g.ny, g.ce, g.ct, dev + g.offset, cnt, s, 2 * (g.nx / g.ct), bs))
          return fail(SHG_EUNSUPPORTED, "batched column schedule not built");
      }
    }
    if (fork) {
      e = hipEventRecord(side->join[b], bs);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, side->join[b], 0);
      if (e != hipSuccess) return hip_fail(e, "join of the batch streams");
    }
  }
  if (powers) {
    hipLaunchKernelGGL((power_finalize_batch<R>), dim3(n), dim3(256), 0, st,
                       (const BatchInst<R>*)dev);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return SHG_OK;
}

void free_batch(Plan& pl) {
  BatchCache* bc = (BatchCache*)pl.batch;
  if (!bc) return;
  if (bc->exec) (void)hipGraphExecDestroy(bc->exec);
  if (bc->cap) (void)hipStreamDestroy(bc->cap);
  for (int b = 0; b < kMaxBranches; ++b) {
    if (bc->side[b]) (void)hipStreamDestroy(bc->side[b]);
    if (bc->join[b]) (void)hipEventDestroy(bc->join[b]);
  }
  if (bc->fork) (void)hipEventDestroy(bc->fork);
  if (bc->desc) (void)hipFree(bc->desc);
  delete bc;
  pl.batch = nullptr;
}

static int run_batch(int n, shg_plan* const* plans, void* const* a_f, void* const* a_sh,
                     const double* const* dk_z, void* ws, double* powers, hipStream_t st) {
  int rc = validate_batch(n, plans, a_f, a_sh);
  if (rc) return rc;
  if ((rc = sticky_device_error())) return rc;
  BatchPlanInfo bi;
  if ((rc = build_info(n, plans, bi))) return rc;
  Plan& p0 = *reinterpret_cast<Plan*>(plans[0]);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  const bool capturing = cs != hipStreamCaptureStatusNone;
  if (!ws) {
    if (!p0.batch_ws || p0.batch_ws_bytes < bi.total) {
      if (capturing)
        return fail(SHG_EINVAL, "no workspace under stream capture: pass one, or run the batch "
                                "once outside capture first");
      if (p0.batch_ws) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        (void)hipFree(p0.batch_ws);
        p0.batch_ws = nullptr;
      }
      e = hipMalloc(&p0.batch_ws, bi.total);
      if (e != hipSuccess) {
        p0.batch_ws = nullptr;
        return hip_fail(e, "hipMalloc(batch workspace)");
      }
      p0.batch_ws_bytes = bi.total;
    }
    ws = p0.batch_ws;
  }
  // cache key: every argument that is baked into the descriptors or the graph;
  // plans enter by serial number (a destroyed plan's address can be reused)
  std::vector<const void*> key;
  key.reserve(5 * n + 2);
  for (int i = 0; i < n; ++i) {
    const Plan* pl = reinterpret_cast<const Plan*>(plans[i]);
    key.push_back(reinterpret_cast<const void*>((uintptr_t)pl->serial));
    key.push_back(a_f[i]);
    key.push_back(a_sh[i]);
    key.push_back(dk_z ? dk_z[i] : nullptr);
    key.push_back(reinterpret_cast<const void*>(
        (uintptr_t)(pl->b_row_e * 1000000 + pl->b_row_wg * 1000 + pl->b_col_e * 100 + pl->b_col_tc)));
  }
  key.push_back(ws);
  key.push_back(powers);
  if (!p0.batch) p0.batch = new BatchCache();
  BatchCache* bc = (BatchCache*)p0.batch;
  const bool same = bc->exec && bc->key == key;
  if (capturing && !same)
    // the caller records this call into its own graph: the descriptors must
    // already be on the device (uploading needs a host synchronisation)
    return fail(SHG_EINVAL, "batch arguments changed while the stream is being captured; "
                            "run the batch once outside capture first");
  if (bi.branches.size() > 1 && !bc->fork) {
    for (int b = 0; b < kMaxBranches && e == hipSuccess; ++b) {
      e = hipStreamCreateWithFlags(&bc->side[b], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&bc->join[b], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bc->fork, hipEventDisableTiming);
    if (e != hipSuccess) {
      for (int b = 0; b < kMaxBranches; ++b) {
        if (bc->side[b]) (void)hipStreamDestroy(bc->side[b]);
        if (bc->join[b]) (void)hipEventDestroy(bc->join[b]);
        bc->side[b] = nullptr;
        bc->join[b] = nullptr;
      }
      if (bc->fork) (void)hipEventDestroy(bc->fork);
      bc->fork = nullptr;
      return hip_fail(e, "creating the batch side streams");
    }
  }
  const BatchCache* side = bc->fork ? bc : nullptr;
  auto enqueue = [&](hipStream_t s, bool upload) {
    return p0.dtype == SHG_C64
               ? enqueue_batch<float>(n, plans, a_f, a_sh, dk_z, (char*)ws, powers, bi, s, upload,
                                      side, bc->desc)
               : enqueue_batch<double>(n, plans, a_f, a_sh, dk_z, (char*)ws, powers, bi, s,
                                       upload, side, bc->desc);
  };
  if (capturing) return enqueue(st, false);
  if (same && !(p0.p.flags & SHG_NO_GRAPH)) {
    e = hipGraphLaunch(bc->exec, st);
    return e == hipSuccess ? SHG_OK : hip_fail(e, "hipGraphLaunch");
  }
  // new arguments (or no graph): drop the old graph and key, then upload the
  // descriptors into the cache's own table
  if (bc->exec) {
    (void)hipGraphExecDestroy(bc->exec);
    bc->exec = nullptr;
  }
  bc->key.clear();
  const size_t desc_bytes =
      (size_t)n * (p0.dtype == SHG_C64 ? sizeof(BatchInst<float>) : sizeof(BatchInst<double>));
  if (bc->desc_cap < desc_bytes) {
    if (bc->desc) {
      e = hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      (void)hipFree(bc->desc);
      bc->desc = nullptr;
      bc->desc_cap = 0;
    }
    e = hipMalloc(&bc->desc, desc_bytes);
    if (e != hipSuccess) {
      bc->desc = nullptr;
      return hip_fail(e, "hipMalloc(batch descriptors)");
    }
    bc->desc_cap = desc_bytes;
  }
  if (p0.p.flags & SHG_NO_GRAPH) return enqueue(st, true);
  if (!bc->cap) {
    e = hipStreamCreateWithFlags(&bc->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  }
  // this call runs directly (uploading the descriptors first); the same
  // sequence is then captured for later calls with the same arguments
  rc = enqueue(st, true);
  if (rc) return rc;
  e = hipStreamBeginCapture(bc->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  rc = enqueue(bc->cap, false);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(bc->cap, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
  e = hipGraphInstantiate(&bc->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    bc->exec = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  bc->key = key;
  return SHG_OK;
}

// run_batch with the SHG_CHECK_FINITE scans of the instances whose plans ask
// for them: inputs before, output fields after.
static int propagate_batch(int n, shg_plan* const* plans, void* const* a_f, void* const* a_sh,
                           const double* const* dk_z, void* ws, double* powers, hipStream_t st) {
  int rc = validate_batch(n, plans, a_f, a_sh);
  if (rc) return rc;
  auto scan = [&](bool inputs) {
    char what[64];
    for (int i = 0; i < n; ++i) {
      Plan& pl = *reinterpret_cast<Plan*>(plans[i]);
      if (!checks_finite(pl)) continue;
      const size_t field = 2 * (size_t)pl.p.nx * pl.p.ny;
      int r;
      snprintf(what, sizeof what, "%s a_f[%d]", inputs ? "input" : "the march's output", i);
      if ((r = check_finite(pl, a_f[i], field, false, what, st))) return r;
      snprintf(what, sizeof what, "%s a_sh[%d]", inputs ? "input" : "the march's output", i);
      if ((r = check_finite(pl, a_sh[i], field, false, what, st))) return r;
      if (inputs && dk_z) {
        snprintf(what, sizeof what, "dk_z[%d]", i);
        if ((r = check_finite(pl, dk_z[i], (size_t)pl.p.nz, true, what, st))) return r;
      }
    }
    return (int)SHG_OK;
  };
  if ((rc = scan(true))) return rc;
  if ((rc = run_batch(n, plans, a_f, a_sh, dk_z, ws, powers, st))) return rc;
  return scan(false);
}

}  // namespace shg

using namespace shg;

extern "C" {

int shg_propagate_batch(int32_t n, shg_plan* const* plans, void* const* a_f, void* const* a_sh,
                        const double* const* dk_z, void* workspace, double* powers,
                        void* stream) {
  int rc = propagate_batch(n, plans, a_f, a_sh, dk_z, workspace, powers, (hipStream_t)stream);
  return rc ? rc : ok();
}

size_t shg_batch_workspace_bytes(int32_t n, shg_plan* const* plans) {
  if (n < 1 || n > 65535 || !plans) return 0;
  for (int i = 0; i < n; ++i)
    if (check_plan(plans[i])) return 0;
  BatchPlanInfo bi;
  if (build_info(n, plans, bi)) return 0;
  return bi.total;
}

}  // extern "C"
