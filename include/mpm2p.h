/*
 * mpm2p.h -- C ABI of the MI355X hot path of the Multiscale Perturbation Method for
 * two-phase flow (MPM-2P) on top of the Multiscale Robin Coupled Method (MRCM),
 * arXiv 2103.11050.
 *
 * The library solves the operator-splitting problem of Section 2 (eq. Darcy for the
 * pressure, eq. BL2D for the saturation) with the modified splitting of Section 4.2
 * (Algorithm 1): explicit upwind transport sub-steps, then a velocity update that is
 * either an MRCM solve with a new set of multiscale basis functions (Section 3) or an
 * MPM-2P solve that reuses the stored ones (Section 4.1, eq:mpm_tf_3 followed by the
 * downscaling problems mpm_upd).
 *
 * Conventions shared by every call
 *  - Every call returns mpm_status (int32): 0 on success, a negative code on error. No C++
 *    exception crosses the boundary.
 *  - Cell arrays are row-major [ny][nx] doubles. x-face fluxes ux are [ny][nx+1], y-face
 *    fluxes uy are [ny+1][nx]: normal flux per unit face length, positive along +x / +y.
 *  - Pointers named dev_* are device (HBM) pointers on the device that is current when
 *    mpm_create is called; every other pointer is host memory.
 *  - The caller owns all device memory: it allocates the workspace (size from
 *    mpm_workspace_size) and keeps it alive until mpm_destroy. The library allocates no
 *    device memory; it allocates a few bytes of pinned host memory per run.
 *  - Work is enqueued on the HIP stream given to mpm_create; calls that return data to the
 *    host (mpm_get_stats) synchronise with that stream.
 *  - Argument errors return MPM_EINVAL before any device work. Errors found by kernels
 *    (a non-positive pivot, a singular interface pivot, a non-finite value) set a device
 *    error word that the next mpm_get_stats or mpm_destroy returns; the run is then
 *    unusable (MPM_ESTATE).
 *  - One run per host thread at a time.
 */
#ifndef MPM2P_H
#define MPM2P_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mpm_status;

enum {
  MPM_OK = 0,
  MPM_EINVAL = -1,     /* invalid argument or descriptor */
  MPM_ENOMEM = -2,     /* workspace smaller than mpm_workspace_size, or host allocation failed */
  MPM_ENOTSPD = -3,    /* a local matrix had a non-positive pivot */
  MPM_ESINGULAR = -4,  /* the interface system had a zero pivot */
  MPM_ENONFINITE = -5, /* a non-finite value appeared in the state */
  MPM_EHIP = -6,       /* a HIP runtime call failed */
  MPM_ESTATE = -7,     /* call not valid in the run's current state */
  MPM_ENOCONV = -8     /* an FP64 refinement of the precision form did not reach refine_rtol */
};

/* Physical boundary kinds, one per side in the order W, E, S, N (eq. Darcy: p = g on the
 * pressure boundary, u.n = z on the flux boundary). */
enum { MPM_BC_NOFLOW = 0, MPM_BC_PRESSURE = 1, MPM_BC_FLUX = 2 };

/* Norm of the switch criterion epsilon = ||kappa^n - kappa^m|| (Section 4.1; Algorithm 1).
 * REL: L2 over cells divided by ||kappa^m||; ABS: L2(Omega). */
enum { MPM_EPS_REL_L2 = 0, MPM_EPS_ABS_L2 = 1 };

/* When epsilon is evaluated (Section 4.2). ALG1: the decision at step n uses epsilon of step
 * n-1, as Algorithm 1 is written. TEXT: the decision uses epsilon of the current saturation,
 * as the description before the algorithm reads. */
enum { MPM_SWITCH_ALG1 = 0, MPM_SWITCH_TEXT = 1 };

/* Arithmetic of the local problems. FP64 everywhere, or FP32 local factors with FP64
 * iterative refinement of every local solve (interface system, residuals, epsilon in FP64). */
enum { MPM_PREC_FP64 = 0, MPM_PREC_FP32_REFINE = 1 };

/* Branch of a velocity update. */
enum { MPM_AUTO = -1, MPM_FORCE_MPM = 0, MPM_FORCE_MRCM = 1 };

#define MPM_ABI_VERSION 3

typedef struct mpm_desc {
  int32_t abi_version;        /* MPM_ABI_VERSION */
  int32_t nx, ny;             /* fine grid (cells) */
  double lx, ly;              /* domain [0,lx] x [0,ly] */
  int32_t sub_x, sub_y;       /* cells per subdomain; nx % sub_x == 0, ny % sub_y == 0. Shorter
                                 side up to 16 cells: at most 256 cells and 64 boundary faces;
                                 17 to 32 cells: at most 1024 cells (FP64, mpm_order 0) */
  int32_t ne_x, ne_y;         /* interface elements per subdomain side along x and along y;
                                 sub_x % ne_x == 0, sub_y % ne_y == 0 (H-bar = H / n_e) */
  double alpha;               /* Robin parameter > 0; beta = alpha H / kappa (eq:beta) */
  double eta;                 /* switch threshold; +inf never updates the basis */
  int32_t eps_norm;           /* MPM_EPS_* */
  int32_t switch_rule;        /* MPM_SWITCH_* */
  int32_t precision;          /* MPM_PREC_* */
  int32_t cn;                 /* transport sub-steps per velocity update (C_n >= 1) */
  double mu_w, mu_o;          /* viscosities; M = mu_o / mu_w (Corey curves of Section 5) */
  int32_t bc_kind[4];         /* MPM_BC_* for W, E, S, N */
  double bc_value[4];         /* g for PRESSURE, outward normal flux z for FLUX (inflow < 0) */
  double s_inj;               /* injected saturation s-bar on inflow boundary faces */
  double cfl;                 /* fraction of the monotone upwind time-step bound, (0, 1] */
  double breakthrough_cut;    /* water cut at the outflow boundary that marks breakthrough */
  int32_t mpm_order;          /* MPM-2P perturbation terms kept: 0 (eq:mpm_tf_3 only, as in the
                                 paper's runs) or 1 (also eq:mpm_tf_4 with l = 1: one more local
                                 solve per subdomain, interface solve and reconstruction per
                                 step; FP64 only) */
  int32_t iface_degree;       /* interface spaces (Section 3.1; -POL of Section 5.2): 0 piecewise
                                 constant U_H, P_H per element (k_U = k_P = 1), 1 piecewise linear
                                 (k_U = k_P = 2: the functions 1 and xi, xi in [-1, 1] along the
                                 element in the global direction, taken at the fine face
                                 midpoints; needs at least two fine faces per element) */
  double refine_rtol;         /* precision form only: the FP64 iterative refinement of a local
                                 solve stops once its largest correction is at most refine_rtol
                                 times the largest entry of the solution, in (0, 1e-2]; a solve
                                 that needs more than 8 corrections sets MPM_ENOCONV. Ignored
                                 for MPM_PREC_FP64 */
} mpm_desc;

typedef struct mpm_stats {
  int64_t te;                 /* elliptic solves so far (T_e) */
  int64_t tm;                 /* basis-set computations so far, the initial one included (T_m) */
  int64_t n_transport;        /* transport sub-steps so far */
  double eps;                 /* last epsilon */
  double t;                   /* simulated time */
  double pvi;                 /* pore volumes injected */
  double water_cut;           /* water cut after the last transport sub-step */
  double dt;                  /* current transport sub-step */
  int32_t breakthrough;       /* 1 once water_cut >= breakthrough_cut */
  int32_t last_branch;        /* MPM_FORCE_MPM or MPM_FORCE_MRCM of the last update */
  int32_t error_word;         /* device error bits (0 if none) */
  int32_t reserved;
} mpm_stats;

typedef struct mpm_run mpm_run;

/* Exact device workspace of a run in bytes (for admission by footprint). */
mpm_status mpm_workspace_size(const mpm_desc* desc, size_t* bytes);

/* Creates a run on the current device. dev_workspace: caller-owned device buffer of at least
 * mpm_workspace_size bytes, 256-byte aligned. hip_stream: a hipStream_t (NULL = default). */
mpm_status mpm_create(const mpm_desc* desc, void* dev_workspace, size_t bytes, void* hip_stream,
                      mpm_run** out);

/* Size of the device array behind mpm_create_static (64 MiB: grids up to 256^2 cells with 16^2-cell
 * subdomains and 4 elements per side). */
#define MPM_STATIC_WORKSPACE_BYTES (64u << 20)

/* mpm_create for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the run's workspace is a file-scope device
 * array of MPM_STATIC_WORKSPACE_BYTES held by the library on every device it runs on until the
 * process ends, instead of a caller buffer. The call allocates nothing: no hipMalloc, hipFree,
 * hipHostMalloc, stream or event; all of the run's work goes on hip_stream (the epsilon and
 * water-cut readback is a copy to host memory on that stream). Every later call on the run is as
 * for mpm_create, except that the run cannot join a batch (mpm_batch_attach returns MPM_ESTATE).
 * The array keeps the contents of the last run that used it; the library clears what its
 * kernels expect at zero. One such run per device at a time: while one is alive (until its
 * mpm_destroy) another mpm_create_static on the same device returns MPM_ESTATE; two threads
 * using one run race, as for any run.
 * Errors: MPM_EINVAL for a bad descriptor; MPM_ENOMEM (mpm_last_error(NULL) gives the sizes) if
 * the run needs more than MPM_STATIC_WORKSPACE_BYTES (mpm_workspace_size plus 256 bytes, rounded
 * to 256); MPM_EHIP if the array's device address cannot be obtained. */
mpm_status mpm_create_static(const mpm_desc* desc, void* hip_stream, mpm_run** out);

/* The data of the problem of Section 2: the absolute permeability K of kappa = lambda(s) K
 * (eq. Darcy; K > 0), the source q (may be NULL: q = 0) and the initial saturation s^0 of eq.
 * BL2D (in [0,1]), copied into the workspace on the run's stream. Device pointers, row-major
 * [ny][nx]; the caller may free them once the copy has run. A non-positive or non-finite K or an
 * s^0 outside [0,1] is found by the first conductivity kernel (mpm_start): MPM_ENOTSPD or
 * MPM_ENONFINITE from the next mpm_get_stats. MPM_EINVAL for a NULL K or s0. */
mpm_status mpm_set_fields(mpm_run* run, const double* dev_K, const double* dev_q, const double* dev_s0);

/* Algorithm 1, first four lines: kappa^0 = lambda(s^0) K, the MRCM velocity, the stored
 * basis functions, n = 1, epsilon = eta. */
mpm_status mpm_start(mpm_run* run);

/* Transport sub-steps with the current velocity (Algorithm 1, the inner for loop). */
mpm_status mpm_transport(mpm_run* run, int32_t nsteps);

/* One velocity update for the current saturation (Algorithm 1, the if/else and the epsilon
 * update). force: MPM_AUTO, MPM_FORCE_MPM or MPM_FORCE_MRCM. */
mpm_status mpm_velocity_update(mpm_run* run, int32_t force);

/* One pass of the while loop of Algorithm 1: C_n transport sub-steps, then a velocity update. */
mpm_status mpm_step(mpm_run* run, int32_t force);

/* Up to max_updates passes of Algorithm 1's while loop (automatic switch), stopping after the
 * first one whose water cut reaches breakthrough_cut when stop_at_breakthrough is nonzero
 * (Section 4.2; the stopping rule of the workloads). *done (host, may be NULL) receives the
 * number of passes made. Errors as mpm_step. */
mpm_status mpm_advance(mpm_run* run, int32_t max_updates, int32_t stop_at_breakthrough, int32_t* done);

/* Text of the last HIP error the run met (host buffer of len bytes, NUL-terminated); with run
 * NULL, why the last mpm_create of the calling thread failed. */
mpm_status mpm_last_error(const mpm_run* run, char* buf, size_t len);

/* Batch of runs stepped together: the batched and serving forms of the workloads (many
 * independent runs of Algorithm 1, Section 4.2, of any sizes). A batch holds `capacity` slots;
 * a slot takes a run (started, or with its fields set and started later by mpm_batch_start)
 * and can be emptied and refilled at any time (continuous batching).
 * Runs with equal descriptors form groups (at most 128 runs per launch): each phase of a step
 * (transport, conductivity and epsilon, local solves, interface solve, reconstruction,
 * downscaling) is one kernel launch for the whole group, on streams the batch owns; the runs of
 * a group whose switch takes the MRCM branch in the same step share that update's launches
 * (one run alone: its own). Other runs
 * step alone on their own streams. The batch owns no device memory; the runs keep their
 * workspaces. While a run is attached, its work is ordered by the batch: work on its stream is
 * ordered before the batch's at attach time and after it at detach time (and around every
 * call on the run itself). A run can be in one batch at a time; mpm_destroy detaches it.
 * Host-side object; one host thread at a time. */
typedef struct mpm_batch mpm_batch;
mpm_status mpm_batch_create(int32_t capacity, mpm_batch** out);
/* MPM_ESTATE if the slot is taken, the run is already in a batch, has no fields set or is
 * poisoned; MPM_EINVAL on a bad slot or NULL. A run attached before mpm_start is started by
 * mpm_batch_start. */
mpm_status mpm_batch_attach(mpm_batch* batch, int32_t slot, mpm_run* run);
/* Algorithm 1, initialisation (conductivity, the first MRCM basis, interface factorisation and
 * velocity; Sections 3 and 4.2), for every attached run not yet started, the runs with equal
 * descriptors together: one launch per phase over a group (at most 128 runs), as in
 * mpm_batch_step. Each run ends as after mpm_start. Returns the first error met; the runs of a
 * group that failed are poisoned. */
mpm_status mpm_batch_start(mpm_batch* batch);
mpm_status mpm_batch_detach(mpm_batch* batch, int32_t slot);
/* One pass of Algorithm 1's while loop (automatic switch) for every filled slot with
 * active[slot] != 0 (active NULL: all filled slots); MPM_ESTATE if one of them is not started.
 * Every run's work is issued before any wait; the runs of a group that take the MRCM branch in
 * the same pass share its launches. breakthrough (host, capacity entries, may be NULL)
 * receives 1 for the stepped runs whose water cut reached breakthrough_cut. Returns the first error met; a run that failed is
 * poisoned, the others are stepped. */
mpm_status mpm_batch_step(mpm_batch* batch, const uint8_t* active, uint8_t* breakthrough);
/* Detaches every run and frees the batch and its streams (the runs stay the caller's). */
mpm_status mpm_batch_destroy(mpm_batch* batch);

/* The current fine velocity u: after an MRCM update the downscaled MRCM velocity (Section 3),
 * after an MPM-2P update the conservative velocity of the downscaling problems (eq. mpm_upd,
 * Section 4.1). Copied on the run's stream into caller-owned device buffers ux [ny][nx+1] and
 * uy [ny+1][nx] (normal flux per unit face length along +x / +y). MPM_ESTATE before mpm_start. */
mpm_status mpm_get_velocity(mpm_run* run, double* dev_ux, double* dev_uy);

/* The current water saturation s of eq. BL2D (after the last transport sub-step), copied on the
 * run's stream into a caller-owned device buffer [ny][nx]. MPM_ESTATE before mpm_set_fields. */
mpm_status mpm_get_saturation(mpm_run* run, double* dev_s);

/* The counters of Algorithm 1 (T_e, T_m as counted in the cost ratio of Section 4.3), the last
 * switch criterion epsilon (Section 4.1), simulated time, pore volumes injected and the outflow
 * water cut that decides breakthrough (Section 5), written into a host struct. Synchronises with
 * the run's stream. Returns the device error word's status, if any bit is set (the run is then
 * poisoned). */
mpm_status mpm_get_stats(mpm_run* run, mpm_stats* out);

/* Waits for the run's work and frees the host-side run (and, for mpm_create_static, releases the
 * device's static array). The workspace stays the caller's. Returns the device error's status. */
mpm_status mpm_destroy(mpm_run* run);

/* Static description of a status code. */
const char* mpm_status_str(mpm_status status);

/* Sizes of the run's plan: subdomains of the decomposition and interface unknowns of eq:mrc2
 * (Section 3; the N-hat of Section 4.3 is twice the unknowns per element), nested-dissection
 * nodes and levels (host memory; any pointer may be NULL). */
mpm_status mpm_plan_info(const mpm_run* run, int64_t* n_sub, int64_t* n_iface, int64_t* n_nodes,
                         int64_t* n_levels);

/* Bytes of the factorisation of the interface system (eq:mrc2, Section 3) that one solve reads: the forward
 * sweep's BI blocks and the backward sweep's [II IB] rows, summed over the nested-dissection
 * nodes, and the size of all fronts (host memory; any pointer may be NULL). */
mpm_status mpm_plan_solve_bytes(const mpm_run* run, int64_t* fwd_bytes, int64_t* bwd_bytes,
                                int64_t* front_bytes);

/* The part of those bytes (eq:mrc2, Section 3) that belongs to the bottom levels of the
 * nested-dissection tree swept by one launch per direction (one workgroup per subtree): *levels =
 * how many (0: the plan has none), *fwd_bytes and *bwd_bytes = the forward sweep's IB (the
 * transpose of BI) and the backward sweep's [II IB] rows of their nodes (host memory; any pointer
 * may be NULL). */
mpm_status mpm_plan_fused_bytes(const mpm_run* run, int32_t* levels, int64_t* fwd_bytes, int64_t* bwd_bytes);

/* Autotuner of the launch shapes of the interface solve (the forward and backward sweeps over the
 * nested-dissection levels of eq:mrc2's factorisation): every admissible shape of each level
 * (lanes per row, column pairs per lane, rows per lane group) is timed over complete solves on the
 * run's stream (best of reps, reps >= 1) and the fastest kept for the run; the result is also
 * cached for the process, so that runs created later with the same decomposition (grid,
 * subdomains, interface elements and degree) start with it (a batch group launches with its
 * first run's shapes). Another shape changes the summation order of the solve: results move at
 * rounding level, so runs compared bitwise must share their shapes. The run must be started and
 * not in a batch (MPM_ESTATE). The bottom levels of the tree can also be swept by one launch per
 * direction (one workgroup per subtree, the default where the fronts fit it); the tuner times that
 * against one launch per level first. Host outputs (any may be NULL when cap is 0): shapes[3 k ..
 * 3 k + 2] = (lanes per row, column pairs per lane, rows per group) of launch k, or (0, number of
 * levels, 0) for the fused bottom levels, forward launches upwards then backward launches
 * downwards, for the first cap / 3 launches; *n = the number of launches; *ms_rule
 * and *ms_tuned = the solve time with the fixed rule and with the chosen shapes (ms). Synchronises
 * with the run's stream. */
mpm_status mpm_tune(mpm_run* run, int32_t reps, int32_t cap, int32_t* shapes, int32_t* n, double* ms_rule,
                    double* ms_tuned);

/* Average duration in milliseconds of each kernel class over the calls since the last reset,
 * measured with HIP events on the run's stream when profiling is enabled (enable = 1; enable = 2
 * also times the launches of the fused bottom sweep levels, inside their phases, whose times
 * then include those events). names/ms/count are host arrays of length cap; returns the number
 * of classes written in *n. */
mpm_status mpm_profile(mpm_run* run, int32_t enable, int32_t reset, int32_t cap, const char** names,
                       double* ms, int64_t* count, int32_t* n);

#ifdef __cplusplus
}
#endif

#endif /* MPM2P_H */
