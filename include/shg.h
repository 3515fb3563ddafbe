/* shg.h - C ABI of the MI355X split-step Fourier (SSFM) march of the coupled
 * second-harmonic-generation equations.
 *
 * What is computed.  The fundamental A_F and second-harmonic A_SH envelopes
 * obey the coupled-wave equations of Sec. 2.1 (Eqs. 1-2) with the accumulated
 * mismatch phase of Eq. 3; the march is the split-step Fourier method of
 * Sec. 3 (Eqs. 11-15): each z-step applies the nonlinear operator N over dz/2
 * by classical RK4, the linear operator L (paraxial diffraction and linear
 * absorption) over dz in Fourier space (Appendix A, Eqs. A.3-A.5), and N over
 * dz/2 again (Eq. 14, order N/2 - L - N/2).  Readings of the printed
 * equations used here:
 *   - coupling kappa_F = 2 pi d / (n_F lambda_F), kappa_SH = 2 pi d / (n_SH lambda_F)
 *     (the printed lambda_SH in the SH coefficient breaks Manley-Rowe energy
 *     conservation with I = eps0 c n |A|^2 / 2 of Sec. 2.2);
 *   - two-photon absorption acts on intensity, beta~_j = beta_j eps0 c n_j / 2;
 *   - the linear loss alpha_j is exact inside the Fourier-space propagator;
 *   - with a temperature field, dk = dk_s + dk(T) - dk(T_ref) per cell, dk(T)
 *     of Eq. 4: its dispersion part (4 pi/lambda_F)(n_SH - n_F) as the cubic
 *     c1 dT + c2 dT^2 + c3 dT^3, dT = T - t_ref, (c1, c2, c3) = (ddk_dT,
 *     ddk_dT2, ddk_dT3), a stand-in for the Sellmeier indices the paper only
 *     cites; its grating part -2 pi / Lambda(T) as printed, Lambda(T) =
 *     grating_period [1 + grating_a (T - 25 C) + grating_b (T - 25 C)^2]; and
 *     a thermal-lens term -i (2 pi / lambda_j) dn_dT dT A_j, with T given at
 *     each step's mid-plane;
 *   - SHG_UNDEPLETED zeroes the whole nonlinear part of dA_F/dz (Sec. 5.1);
 *   - spatial walk-off (the tan(rho) dA/dx term of the package's propagators,
 *     Sec. 4): dA_j/dz gains -tan(rho_j) dA_j/dx, which moves wave j towards +x
 *     by tan(rho_j) per metre; it is linear and applied exactly in L as
 *     exp(-2 i pi q_x tan(rho_j) dz).
 *
 * Conventions.
 *   - SI units throughout: m, W, rad/m, 1/m (intensity absorption), m/W, K.
 *   - Fields are row-major [ny][nx] interleaved complex (re, im), x fastest:
 *     complex64 (float pairs) for SHG_C64 plans, complex128 for SHG_C128.
 *     Sample (m, n) sits at x = (m - nx/2) dx, y = (n - ny/2) dy, dx = lx/nx:
 *     the window is periodic.
 *   - All array arguments are DEVICE pointers owned by the caller.  The
 *     library never frees or retains them beyond the call.
 *   - Calls are asynchronous on the caller's HIP stream (passed as void*,
 *     NULL = default stream).  A plan must not be used on two streams at once.
 *   - Every entry point returns a status code; arguments are validated before
 *     anything is launched, and on error nothing has been enqueued.  A device
 *     fault of an earlier launch surfaces as SHG_EDEVICE.  shg_last_error()
 *     gives a message for the calling thread.
 */
#ifndef SHG_H
#define SHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct shg_plan shg_plan;

/* (the last enumerator widens the type's range to every int32 value, so an
 * invalid value passed by a caller is rejected, not undefined) */
typedef enum { SHG_C64 = 0, SHG_C128 = 1, SHG_DTYPE_RANGE_ = 0x7fffffff } shg_dtype;

enum {
  SHG_OK = 0,
  SHG_EINVAL = 1,       /* invalid argument (message says which)            */
  SHG_EUNSUPPORTED = 2, /* valid but not built here (e.g. grid size)        */
  SHG_ENOMEM = 3,       /* device allocation failed                          */
  SHG_EDEVICE = 4,      /* HIP runtime error, including earlier device faults */
  SHG_ENONFINITE = 5,   /* SHG_CHECK_FINITE found NaN or Inf (message says
                           which array, input or output)                     */
  SHG_ESTATE = 6        /* NULL or destroyed plan                            */
};

/* flags */
enum {
  SHG_UNDEPLETED = 1u << 0, /* undepleted pump: dA_F/dz has no nonlinear part */
  SHG_NO_GRAPH = 1u << 1,   /* launch passes one by one instead of replaying a
                               cached HIP graph of the whole march              */
  SHG_SPLIT_LNL = 1u << 2,  /* the other Strang order of Sec. 3, L/2 - N - L/2:
                               one RK4 over dz per step (stages at 0, dz/2, dz)
                               between two half-step propagators; interior
                               half-steps merge into one column pass.  Not with
                               shg_propagate_heat (SHG_EUNSUPPORTED); all plans
                               of a batch share the order                       */
  SHG_CHECK_FINITE = 1u << 3 /* debugging aid: before a march, scan its input
                               arrays (fields, dk_z, temperature, adjoint
                               cotangents and weights) and after it the output
                               fields for NaN or Inf; SHG_ENONFINITE names the
                               array.  Each scan synchronises the stream (the
                               scan kernels run before the march is enqueued)  */
};

typedef struct {
  int32_t nx, ny, nz;     /* nx, ny powers of two in [16, 512]; nz >= 1        */
  double lx, ly;          /* transverse window widths [m]                      */
  double lcr;             /* crystal length [m]; dz = lcr / nz                 */
  double lambda_f;        /* fundamental vacuum wavelength [m]; SH at half     */
  double n_f, n_sh;       /* refractive indices                                */
  double d_eff;           /* effective nonlinear coefficient [m/V]            */
  double alpha_f, alpha_sh; /* linear intensity absorption [1/m]               */
  double beta_f, beta_sh; /* two-photon absorption [m/W]                       */
  double dk0;             /* phase mismatch [rad/m] when no per-step profile   */
  double ddk_dT;          /* d(dk)/dT [rad/(m K)], temperature field only      */
  double dn_dT;           /* thermo-optic coefficient [1/K], both waves        */
  double t_ref;           /* reference temperature [K]                         */
  uint32_t flags;         /* SHG_UNDEPLETED | SHG_NO_GRAPH                      */
  int32_t checkpoint_every; /* adjoint checkpoint interval K (0 -> automatic:  */
                            /* K = nz when nz staged steps fit in 16 GiB)      */
  double walkoff_f, walkoff_sh; /* spatial walk-off angles rho_F, rho_SH [rad], */
                            /* |rho| < pi/2; 0 for quasi-phase matching        */
  double ddk_dT2, ddk_dT3;  /* quadratic and cubic terms of dk(T) [rad/(m K^2)],*/
                            /* [rad/(m K^3)]; temperature field only, 0 = linear */
  double grating_period;    /* poling period Lambda at 25 C [m], temperature    */
                            /* field only; 0 = no grating term in dk(T)         */
  double grating_a, grating_b; /* thermal expansion of Lambda [1/K], [1/K^2]    */
                            /* about 25 C (2.2e-6, -5.9e-9 for MgO:sPPLT); the  */
                            /* period must stay positive over the field's T     */
} shg_params;

/* Create a plan: validates the parameters, builds the FP64 propagator and
 * twiddle tables (rounded once to the plan's precision where the kernels use
 * that precision), chooses launch schedules, and allocates the plan's small
 * device tables on the current HIP device.
 * Errors: SHG_EINVAL (NULL pointer, nx/ny not a power of two in [16, 512],
 * nz < 1, non-positive or non-finite lengths/indices/wavelength, negative
 * absorption, non-finite dk coefficients, negative grating period or one
 * that is not positive at t_ref, |walk-off| >= pi/2), SHG_ENOMEM, SHG_EDEVICE.  *out is NULL on
 * error. */
int shg_plan_create(shg_plan **out, const shg_params *p, shg_dtype dtype);

/* Release the plan and its device tables.  NULL is accepted (returns SHG_OK).
 * The caller must have synchronised the stream of the plan's last call. */
int shg_plan_destroy(shg_plan *plan);

/* Bytes of device workspace needed by shg_propagate (for_adjoint = 0) or by
 * shg_propagate_adjoint (for_adjoint = 1).  Returns 0 for a NULL plan. */
size_t shg_workspace_bytes(const shg_plan *plan, int for_adjoint);

/* March steps [s_begin, s_end) of the crystal in place (Eq. 14 per step).
 *   a_f, a_sh  in: fields at z = s_begin dz; out: fields at z = s_end dz
 *   dk_z       [nz] double per-step mismatch, or NULL for params.dk0
 *   temp       [nz][ny][nx] mid-plane temperature samples in the plan's real
 *              type (float for C64, double for C128), or NULL for none
 *   workspace  shg_workspace_bytes(plan, 0) bytes, or NULL to use the
 *              plan's own buffer (allocated by shg_plan_create)
 *   powers     double[2] {P_F, P_SH} at z = s_end dz (P = int eps0 c n |A|^2/2
 *              dA, Sec. 2.2), or NULL
 *   stream     hipStream_t as void*
 * The call allocates no device memory.  Outside stream capture it replays a
 * HIP graph of the march that it captures (on a private stream) the first
 * time it sees a set of arguments; under the caller's capture it enqueues the
 * passes themselves, so it can be recorded into the caller's graph.
 * Errors: SHG_ESTATE, SHG_EINVAL (NULL field, 0 <= s_begin < s_end <= nz
 * violated), SHG_EDEVICE, SHG_ENONFINITE (SHG_CHECK_FINITE). */
int shg_propagate(shg_plan *plan, void *a_f, void *a_sh, const double *dk_z,
                  const void *temp, int32_t s_begin, int32_t s_end,
                  void *workspace, double *powers, void *stream);

/* shg_propagate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, hosts that forbid hipMalloc).  Same
 * arguments and results as shg_propagate without `workspace`: the march's
 * workspace (stage-coefficient table, power partials, temperature phase) is a static
 * device array of 4 MiB per GPU, held until the process ends.  The call
 * allocates nothing and creates no graph: the passes are enqueued one by one
 * on `stream` (so it can be recorded into a caller's graph).  Every call on a
 * GPU shares that GPU's array, so calls that overlap on one GPU (concurrent
 * streams or threads) race and must be serialised by the caller; nothing in
 * the array needs to survive between calls.  The current device must be the
 * plan's.  Timing mode (shg_plan_set_timing) does not apply.
 * Errors: as shg_propagate; SHG_EINVAL also when shg_workspace_bytes(plan, 0)
 * exceeds 4 MiB (nz above about 13000 for 512x512 complex128, about 39000
 * for 512x512 complex64), when the current device is not the plan's,
 * or for a plan with SHG_CHECK_FINITE; SHG_EDEVICE when the array's device
 * address could not be obtained. */
int shg_propagate_noalloc(shg_plan *plan, void *a_f, void *a_sh, const double *dk_z,
                          const void *temp, int32_t s_begin, int32_t s_end, double *powers,
                          void *stream);

/* The whole march (steps [0, nz)) as shg_propagate, also writing the heat
 * source of Sec. 2.2, q = sum_j alpha_j I_j + beta_j I_j^2 with
 * I_j = eps0 c n_j |A_j|^2 / 2 [W/m^3], of the fields at every step boundary
 * z_l = l dz, l = 0..nz (the input, the state between the two half-steps of
 * consecutive steps, and the output).  This is the source the heat equation
 * needs for the self-consistent loop.
 *   heat  [nz + 1][ny][nx] in the plan's real type (required)
 * Other arguments and errors as shg_propagate. */
int shg_propagate_heat(shg_plan *plan, void *a_f, void *a_sh, const double *dk_z,
                       const void *temp, void *heat, void *workspace, double *powers,
                       void *stream);

/* Gradient of a real loss L through the whole march (steps [0, nz)), by the
 * reverse of the Eq. 14 step sequence in the plan's split order.
 * The loss is L = Re<g_f_out, A_F(L)> + Re<g_sh_out, A_SH(L)>
 *               + w[0] P_F(L) + w[1] P_SH(L)  (to first order),
 * with complex gradients in the convention g = dL/dRe + i dL/dIm.
 *   a_f_in, a_sh_in    fields at z = 0 (not modified)
 *   dk_z, temp         as for shg_propagate
 *   g_f_out, g_sh_out  seeds dL/dA(L), or NULL for zero
 *   power_weights      device double[2] {w_F, w_SH}, or NULL for zero
 *   g_f_in, g_sh_in    out: dL/dA(0) (same layout as the fields)
 *   g_dk_z             out: [nz] double dL/d dk_s, or NULL
 *   g_t_moments        out: double[2] {sum dL/dT (T - t_ref), sum dL/dT}
 *                      (temp given), or NULL
 *   a_f_out, a_sh_out  out: forward fields at z = L, or NULL
 *   powers             out: double[2] forward exit powers, or NULL
 *   workspace          shg_workspace_bytes(plan, 1) bytes (required)
 * Fields are checkpointed every K = params.checkpoint_every steps; the
 * backward sweep recomputes every segment except the last one, which the
 * forward sweep stages directly (K = nz recomputes nothing).
 * Errors: as shg_propagate; SHG_EINVAL also for a NULL workspace. */
int shg_propagate_adjoint(shg_plan *plan, const void *a_f_in, const void *a_sh_in,
                          const double *dk_z, const void *temp,
                          const void *g_f_out, const void *g_sh_out,
                          const double *power_weights, void *g_f_in, void *g_sh_in,
                          double *g_dk_z, double *g_t_moments, void *a_f_out,
                          void *a_sh_out, double *powers, void *workspace,
                          void *stream);

/* March n independent instances (each over its whole crystal) in one
 * replayable launch sequence.  Plans may differ in every parameter (grid size,
 * nz, coupling, mismatch) but must share the dtype and must not use a
 * temperature field.  Instances advance in lock-step passes grouped by grid
 * size; an instance stops after its own nz steps.
 *   plans[i], a_f[i], a_sh[i]  as for shg_propagate (fields updated in place)
 *   dk_z[i]                    per-instance [nz_i] profile, or NULL entries /
 *                              NULL array for the plans' dk0
 *   workspace                  shg_batch_workspace_bytes(...) bytes (stage-
 *                              coefficient tables and power partials, rewritten by every
 *                              call), or NULL for a buffer kept by plans[0]
 *   powers                     [n][2] double exit powers, or NULL
 * The first call with a set of arguments (plans, fields, profiles, workspace,
 * powers) uploads the instance descriptors into a table owned by plans[0]
 * (allocated or grown then, as is the NULL-workspace buffer), runs the batch
 * and captures it into a graph that later calls with the same arguments
 * replay.  Such a first call synchronises the stream and cannot be recorded
 * into a caller's graph: under stream capture only an already-seen set of
 * arguments is accepted (it enqueues the launches, allocating nothing).
 * Errors: SHG_EINVAL (n < 1, NULL arrays/entries, mixed dtypes, temperature
 * flags, new arguments or a missing NULL-workspace buffer under stream
 * capture), SHG_ENOMEM, SHG_EDEVICE. */
int shg_propagate_batch(int32_t n, shg_plan *const *plans, void *const *a_f,
                        void *const *a_sh, const double *const *dk_z,
                        void *workspace, double *powers, void *stream);

/* Workspace bytes for shg_propagate_batch over these plans (0 on error). */
size_t shg_batch_workspace_bytes(int32_t n, shg_plan *const *plans);

/* Force launch schedules (used by the autotuner and tests).  row_e / col_e:
 * elements per thread of the row / column transforms (4, 8, 16); row_e = 1
 * selects the wide row pass (one cell per thread for the half-steps, row_wg =
 * max(256, nx) threads); row_wg: threads per row-pass block; col_tc: columns
 * per column-pass block.  Zero keeps the current choice.  Errors:
 * SHG_EUNSUPPORTED for a schedule that is not built or does not fit the grid. */
int shg_plan_set_schedule(shg_plan *plan, int32_t row_e, int32_t row_wg,
                          int32_t col_e, int32_t col_tc);

/* Same for the schedule a plan uses inside shg_propagate_batch (batches are
 * throughput bound and default to more elements per thread). */
int shg_plan_set_batch_schedule(shg_plan *plan, int32_t row_e, int32_t row_wg,
                                int32_t col_e, int32_t col_tc);

/* Per-kernel timing for measurement.  While enabled, shg_propagate launches
 * every pass individually (no cached graph) with a HIP start/stop event pair
 * bracketing each kernel.  Enabling or disabling clears the record. */
int shg_plan_set_timing(shg_plan *plan, int32_t enable);

/* Totals of the timed launches since the last query, then clears them:
 * out[0] = row-pass milliseconds, out[1] = row-pass launches,
 * out[2] = column-pass milliseconds, out[3] = column-pass launches.
 * Synchronises with the recorded events.  Errors: SHG_ESTATE, SHG_EINVAL,
 * SHG_EDEVICE. */
int shg_plan_kernel_times(shg_plan *plan, double *out);

/* Write a one-line description of the plan's schedule into buf (NUL
 * terminated, truncated to len).  Returns SHG_OK or SHG_ESTATE. */
int shg_plan_describe(const shg_plan *plan, char *buf, size_t len);

/* Message of the last failed call on this thread ("" if none).  Valid until
 * the next call on this thread. */
const char *shg_last_error(void);

/* ------------------------------------------------------------------------
 * Steady-state heat equation and the self-consistent loop (Sec. 2.2, the
 * finite differences of Sec. 3.2 and the flowchart of Sec. 4).
 *
 * k lap T + q = 0 with q the heat source of shg_propagate_heat, on the nodes
 * of the field grid: nx x ny transverse samples (the x and y faces of the
 * crystal are the first and last samples) times nz + 1 planes z_l = l dz.
 * Nodes on an oven face are held at t_oven (edges and corners included); air
 * faces obey -k dT/dn = h_conv (T - t_inf); insulated faces have no flux.
 * Every other node obeys the second-order 7-point equation, with the outside
 * neighbour of a face node removed through the central difference of its
 * boundary condition.  Both solvers (below) work on the control-volume
 * (symmetric) form of those equations and synchronise the stream (set-up,
 * convergence tests, the residual report), so they cannot be captured into a
 * graph.
 * Temperatures are arrays in the plan's real type: t_nodes [nz + 1][ny][nx]
 * and the mid-planes t_mid [nz][ny][nx] = (T_l + T_{l+1}) / 2 that
 * shg_propagate takes as its temperature field. */
typedef struct shg_thermal shg_thermal;

enum { SHG_FACE_AIR = 0, SHG_FACE_OVEN = 1, SHG_FACE_INSULATED = 2 };

/* Solvers.  SHG_THERMAL_DIRECT: exact.  Divided by the control-volume
 * weights, the operator is the Kronecker sum of three 1-D operators (constant
 * k, oven faces are whole planes).  The x and y operators are diagonalised
 * (rocSOLVER eigendecompositions, once per plan, FP64; four FP64 GEMM mode
 * products per solve), which leaves one tridiagonal system along z per (x, y)
 * mode, solved by elimination in FP64; tol and max_iter are ignored and
 * iterations is 0.  SHG_THERMAL_CG: Jacobi-preconditioned conjugate gradients
 * in the plan's real type with FP64 reductions, stopped at |r| <= tol |b|. */
enum { SHG_THERMAL_DIRECT = 0, SHG_THERMAL_CG = 1 };

typedef struct {
  int32_t nx, ny, nz;     /* the field grid; nodes nx x ny x (nz + 1)          */
  int32_t faces[6];       /* x-, x+, y-, y+, z-, z+: SHG_FACE_*                 */
  int32_t method;         /* SHG_THERMAL_DIRECT (default) or SHG_THERMAL_CG    */
  double lx, ly, lcr;     /* as in shg_params [m]                               */
  double k_th;            /* thermal conductivity [W/(m K)]                     */
  double h_conv;          /* convection coefficient of air faces [W/(m^2 K)]    */
  double t_inf;           /* air temperature [K]                                */
  double t_oven;          /* oven temperature [K]                               */
} shg_thermal_params;

/* Errors: SHG_EINVAL (grid as for shg_plan_create, k_th <= 0, h_conv < 0,
 * non-finite temperatures, unknown face kind, or no oven face and no cooled
 * air face, which leaves T undetermined), SHG_ENOMEM.  Allocates no device
 * memory. */
int shg_thermal_create(shg_thermal **out, const shg_thermal_params *p, shg_dtype dtype);
int shg_thermal_destroy(shg_thermal *th);

/* Device workspace of shg_thermal_solve and shg_self_consistent: seven node
 * vectors (nx ny (nz + 1) reals each), two FP64 node vectors for the direct
 * solver, and a few KB.  The direct solver also keeps its factors (3 m^2 + 3 m
 * doubles per axis, m <= nz + 1) in device memory owned by the plan, built on
 * its first solve. */
size_t shg_thermal_workspace_bytes(const shg_thermal *th);

/* Solve for T with source heat [nz + 1][ny][nx] [W/m^3].
 *   t_nodes    in: initial guess (warm start); out: solution
 *   t_mid      out: mid-plane temperatures, or NULL
 *   tol        stop when |r| <= tol |b| (2-norms of the weighted system)
 *   iterations, residual  out (host pointers, may be NULL)
 * residual: the direct solver reports |b - A theta| / |b| of its FP64
 * solution (before T is rounded to the plan's precision); CG reports the
 * relative norm of its recursively updated residual.
 * Returns after the solve (the host waits on the stream).  Errors:
 * SHG_ESTATE, SHG_EINVAL (NULL arrays or workspace, tol <= 0, max_iter < 1),
 * SHG_ENOMEM, SHG_EDEVICE (including a diverged iteration or a failed
 * eigensolver). */
int shg_thermal_solve(shg_thermal *th, const void *heat, void *t_nodes, void *t_mid, double tol,
                      int32_t max_iter, void *workspace, int32_t *iterations, double *residual,
                      void *stream);

/* The self-consistent loop: T from q = 0, then repeatedly march the input
 * (a_f0, a_sh0) with the mid-plane field of T (per-cell dk(T) and thermal
 * lens), take its heat source and solve for T again, until the largest change
 * of T between two solves is <= tol_t or max_outer marches have run.
 *   a_f, a_sh   out: the fields of the last march
 *   t_nodes     in: initial guess of the first solve; out: final T
 *   t_mid       out: mid-planes of the final T
 *   solve_tol, max_iter  passed to each solve
 *   workspace   shg_thermal_workspace_bytes(th) bytes (the march uses the
 *               plan's own forward workspace)
 *   outer, change  out (host): marches run and the last largest change [K]
 * The thermal grid (nx, ny, nz, lx, ly, lcr) and dtype must match the plan's.
 * Errors: as shg_thermal_solve and shg_propagate. */
int shg_self_consistent(shg_plan *plan, shg_thermal *th, const void *a_f0, const void *a_sh0,
                        const double *dk_z, void *a_f, void *a_sh, void *t_nodes, void *t_mid,
                        double tol_t, int32_t max_outer, double solve_tol, int32_t max_iter,
                        void *workspace, int32_t *outer, double *change, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SHG_H */
