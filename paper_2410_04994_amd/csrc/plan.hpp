// Internal plan object behind the opaque shg_plan handle.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "shg.h"

namespace shg {

struct GraphKey {
  const void* a;
  const void* b;
  const void* dk;
  const void* temp;
  const void* heat;
  const void* ws;
  const void* powers;
  int s0, s1;
  int re, rw, ce, ct;
  bool operator==(const GraphKey& o) const {
    return a == o.a && b == o.b && dk == o.dk && temp == o.temp && heat == o.heat && ws == o.ws &&
           powers == o.powers && s0 == o.s0 &&
           s1 == o.s1 && re == o.re && rw == o.rw && ce == o.ce && ct == o.ct;
  }
};

struct Plan {
  static constexpr uint64_t kMagic = 0x5348475f504c414eull;  // "SHG_PLAN"
  uint64_t magic = 0;
  uint64_t serial = 0;           // unique per plan created in this process
  shg_params p{};
  shg_dtype dtype = SHG_C64;
  int device = 0;
  int real_bytes = 4;
  // derived constants (FP64)
  double dx = 0, dy = 0, dz = 0;
  double k_f = 0, k_sh = 0, kappa_f = 0, kappa_sh = 0;
  double tpa_f = 0, tpa_sh = 0, lens_f = 0, lens_sh = 0;
  double pscale_f = 0, pscale_sh = 0;
  int ckpt = 32;
  // device tables
  void* tw_x = nullptr;          // W_nx^k in the plan's precision
  void* tw_y = nullptr;          // W_ny^k
  double* mx[2] = {nullptr, nullptr};
  double* my[2] = {nullptr, nullptr};
  double* mxh[2] = {nullptr, nullptr};   // half-step factors (L/2 - N - L/2 order)
  double* myh[2] = {nullptr, nullptr};
  // schedule
  int row_e = 0, row_wg = 0, row_rows = 1;
  int adj_e = 0, adj_wg = 0;     // adjoint row pass
  int b_row_e = 0, b_row_wg = 0, b_col_e = 0, b_col_tc = 1;   // schedule inside batches
  int col_e = 0, col_tc = 1;
  // library-owned workspaces: the forward one is allocated with the plan (so
  // shg_propagate without a workspace allocates nothing), the batch one by the
  // first batch that needs it
  void* own_ws = nullptr;
  size_t own_ws_bytes = 0;
  void* batch_ws = nullptr;
  size_t batch_ws_bytes = 0;
  // cached forward graph
  hipStream_t cap_stream = nullptr;
  int* finite_flag = nullptr;  // device int of the SHG_CHECK_FINITE scans (plans with the flag)
  // cached graphs of the march, most recently used first; a few entries, so
  // that callers cycling through a few buffers (e.g. fresh output tensors from
  // an allocator) replay instead of capturing again
  static constexpr int kGraphCache = 4;
  struct CachedGraph {
    GraphKey key;
    hipGraphExec_t exec;
  };
  std::vector<CachedGraph> graphs;
  // optional per-kernel timing (kind 0 = row pass, 1 = column pass)
  int timing = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
  // adjoint state (owned by adjoint.hip)
  void* adj = nullptr;
  // batch cache (owned by batch.hip) when this plan is the first of a batch
  void* batch = nullptr;
};

// Pointers of one forward march: the first row pass reads (a_in, b_in), the
// passes work in place on (a_work, b_work), the last row pass writes
// (a_out, b_out).  tap (optional) receives, for every step s of the range, the
// real-space state before its second half-step at tap + (s - s0) * 2 * nx * ny
// (F then SH).
// temp (optional) is the [nz][ny][nx] temperature field; psi (optional) is
// the per-cell accumulated (T - T_ref) dz buffer holding Psi at s0 (when NULL
// the workspace buffer is used and initialised from temp); tap_psi receives
// Psi at the start of each step s at tap_psi + (s - s0) * nx * ny.
// heat (optional) receives the heat source of the state at every step
// boundary l = s0..s1 at heat + l * nx * ny (the plan's real type).
struct FwdIO {
  const void* a_in;
  const void* b_in;
  void* a_work;
  void* b_work;
  void* a_out;
  void* b_out;
  void* tap;
  const void* temp = nullptr;
  void* psi = nullptr;
  void* tap_psi = nullptr;
  void* heat = nullptr;
};

// shg.hip
int fail(int code, const char* fmt, ...);
int ok();
int hip_fail(hipError_t e, const char* what);
int check_plan(const shg_plan* plan);
int sticky_device_error();
size_t forward_ws_bytes(const Plan& pl);
int enqueue_forward(Plan& pl, void* a, void* b, const double* dk_z, int s0, int s1, void* ws,
                    double* powers, hipStream_t st);
// timed = false launches without the per-kernel events of timing mode.
int enqueue_forward_io(Plan& pl, const FwdIO& io, const double* dk_z, int s0, int s1, void* ws,
                       double* powers, hipStream_t st, bool make_phase, bool timed = true);
int propagate(Plan& pl, void* a_f, void* a_sh, const double* dk_z, const void* temp, int s0,
              int s1, void* ws, double* powers, hipStream_t st, void* heat);
size_t align256(size_t v);
// SHG_CHECK_FINITE: scan `count` reals of the plan's type (or doubles when dbl)
// at `data` (NULL: nothing to scan); SHG_ENONFINITE names `what`.
int check_finite(Plan& pl, const void* data, size_t count, bool dbl, const char* what,
                 hipStream_t st);
inline bool checks_finite(const Plan& pl) { return (pl.p.flags & SHG_CHECK_FINITE) != 0; }
// Column pass over the fields a, b with the plan's propagator (conj: conj(M);
// half: the half-step tables of the L/2 - N - L/2 order).
int launch_col(Plan& pl, void* a, void* b, int conj, hipStream_t st, bool half = false);
bool row_supported(const Plan& pl, int e, int wg, int* rows);
bool col_supported(const Plan& pl, int e, int tc);

// adjoint.hip / thermal.hip / batch.hip
size_t adjoint_ws_bytes(const Plan& pl);
void free_adjoint(Plan& pl);
void free_batch(Plan& pl);


}  // namespace shg
