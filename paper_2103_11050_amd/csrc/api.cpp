// C ABI and host runtime: workspace carving, the velocity updates (MRCM and MPM-2P), the
// transport sub-steps and the modified operator splitting (Section 4.2, Algorithm 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "mpm2p.h"
#include "plan.hpp"

using namespace mpm;

namespace {

// Why the last mpm_create of this thread failed (for mpm_last_error with no run).
thread_local std::string g_create_error;

// max over [0,1] of f'(s) = 2 M s (1-s) / (M s^2 + (1-s)^2)^2 for the Corey curves: the
// interior zero of f'' is the root of the cubic
//   (1 - 2s)(M s^2 + (1-s)^2) - 4 s (1-s)(M s - (1-s)) = 0,
// bracketed by a coarse scan of f' and then bisected to machine precision.
double fprime(double s, double M) {
  const double den = M * s * s + (1.0 - s) * (1.0 - s);
  return 2.0 * M * s * (1.0 - s) / (den * den);
}
double fpp_sign_poly(double s, double M) {
  return (1.0 - 2.0 * s) * (M * s * s + (1.0 - s) * (1.0 - s)) - 4.0 * s * (1.0 - s) * (M * s - (1.0 - s));
}
double max_fprime(double M) {
  const int n = 4096;
  int best = 1;
  double bv = -1.0;
  for (int i = 1; i < n; ++i) {
    const double v = fprime(double(i) / n, M);
    if (v > bv) { bv = v; best = i; }
  }
  double a = double(best - 1) / n, b = double(best + 1) / n;
  double fa = fpp_sign_poly(a, M);
  for (int it = 0; it < 200 && b - a > 0; ++it) {
    const double m = 0.5 * (a + b);
    if (m <= a || m >= b) break;
    const double fm = fpp_sign_poly(m, M);
    if ((fm > 0) == (fa > 0)) { a = m; fa = fm; } else { b = m; }
  }
  double v = std::max(fprime(a, M), fprime(b, M));
  return std::max(v, bv);
}

struct ProfEntry {
  const char* name = nullptr;   // string literal of the kernel class
  double ms = 0.0;
  int64_t count = 0;
};

}  // namespace

struct mpm_run {
  Plan P;
  Geo g;
  hipStream_t st = nullptr;            // the library's stream (all work)
  hipStream_t ust = nullptr;           // the caller's stream (ordering only)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // the MPM-2P step replayed as two graphs: transport sub-steps + kappa/epsilon (one per
  // parity of the saturation double buffer), and the MPM-2P velocity update
  bool use_graphs = true;
  hipGraphExec_t g_trans[2] = {nullptr, nullptr};
  hipGraphExec_t g_mpm = nullptr;
  double* s_base = nullptr;
  int device = 0;
  char* ws = nullptr;
  double *K, *q, *s, *s2, *kn, *km, *ux, *uy, *uxm, *uym, *fac, *S, *h, *vbnd, *ubnd, *leafK;
  double *front, *fI, *slots, *panel, *y, *red, *scal, *dsE, *nfac;
  double* wbnd = nullptr;              // first-order term only
  int32_t* err;
  int32_t* wc_ticket;          // completion counter of the water-cut workgroups (zero between launches)
  float *fac32 = nullptr, *nfac32 = nullptr, *dsE32 = nullptr;   // precision form
  bool f32 = false;
  const LeafUp* leafup = nullptr;
  int32_t* dsflag = nullptr;
  int32_t* dslist = nullptr;
  int32_t* dscount = nullptr;          // number of entries of dslist (device)
  NdArgs nd{};
  hipStream_t st2 = nullptr;           // second stream: factorisations overlapped with the solves
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  const int32_t* subdofs_d = nullptr;
  double fmax_deriv = 0.0;
  double params[SC_FMAX - SC_MUW + 1] = {};   // the run's physics for the scalar block
  double M = 1.0;
  double area = 1.0;
  // Algorithm 1 state
  bool fields = false, started = false, poisoned = false;
  int64_t te = 0, tm = 0, ntr = 0;
  double eps_prev = 0.0;       // epsilon after the last update (known on the host)
  bool eps_pending = false;    // epsilon of the last update still in flight
  int last_branch = MPM_FORCE_MRCM;
  double* pinned = nullptr;    // [eps_num, eps_den, sequence, water cut], written by kernels
  double* pinned_dev = nullptr;  // the same memory as the device sees it
  // a run on the static workspace (mpm_create_static): no stream, event or pinned memory of its
  // own; the kernels write the block above into the workspace and it is copied to pin_host
  bool is_static = false;
  double pin_host[4] = {};
  int64_t eps_seq = 0;           // sequence number of the latest kappa launch
  hipEvent_t ev_eps = nullptr;
  // profiling with HIP events on the run's stream
  bool prof = false;
  bool prof_fine = false;   // also the fused sweep launches, inside their phases
  std::vector<std::pair<const char*, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, ProfEntry> prof_acc;
  std::string last_error;
  // batch membership: while the run steps in a group of a batch, st is the group's stream and
  // home the stream it had before
  mpm_batch* owner = nullptr;
  int32_t owner_slot = -1;
  hipStream_t home = nullptr;
  // the run tables last written to this run's workspace (when it leads a batch group): all
  // runs of the group, and those of them taking the MPM-2P branch
  RunTab tab_host[2] = {};
  unsigned tab_n[2] = {0, 0};
  // launch shape of each interface-sweep level (nd_shape_code; 0 = the fixed rule), by level
  std::vector<int> tune_fwd, tune_bwd;
  // the plan's bottom levels (P.fuse_h of them) swept by one launch per direction
  bool fuse = false;
  const int32_t* fleaves = nullptr;   // per subtree, its subdomains (device)

  hipEvent_t take_event() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    hipEventCreate(&e);
    return e;
  }
  void prof_begin(const char* name, hipEvent_t* b) {
    if (!prof) return;
    *b = take_event();
    hipEventRecord(*b, st);
    (void)name;
  }
  void prof_end(const char* name, hipEvent_t b) {
    if (!prof) return;
    hipEvent_t e = take_event();
    hipEventRecord(e, st);
    pending.push_back({name, {b, e}});
  }
  void prof_collect() {
    for (auto& p : pending) {
      float ms = 0.f;
      hipEventSynchronize(p.second.second);
      hipEventElapsedTime(&ms, p.second.first, p.second.second);
      auto& a = prof_acc[p.first];
      a.name = p.first;
      a.ms += ms;
      a.count += 1;
      pool.push_back(p.second.first);
      pool.push_back(p.second.second);
    }
    pending.clear();
  }
};

namespace {

struct Scope {
  mpm_run* r;
  const char* name;
  hipEvent_t b = nullptr;
  bool on;
  Scope(mpm_run* r_, const char* n, bool fine = false) : r(r_), name(n), on(!fine || r_->prof_fine) {
    if (on) r->prof_begin(n, &b);
  }
  ~Scope() {
    if (on) r->prof_end(name, b);
  }
};

Geo make_geo(const Plan& P) {
  Geo g{};
  g.nx = P.nx; g.ny = P.ny; g.mx = P.mx; g.my = P.my; g.Sx = P.Sx; g.Sy = P.Sy; g.nsub = P.nsub;
  g.nc = P.nc; g.band = P.band; g.xfast = P.xfast; g.nb = P.nb; g.ne_x = P.ne_x; g.ne_y = P.ne_y;
  g.n_vert = P.n_vert; g.ndmax = P.ndmax; g.npol = P.npol;
  g.hx = P.hx; g.hy = P.hy; g.alpha = P.d.alpha;
  g.bc_pack = 0;
  for (int k = 0; k < 4; ++k) g.bc_pack |= (P.d.bc_kind[k] & 3) << (2 * k);
  g.bc_v0 = P.d.bc_value[0]; g.bc_v1 = P.d.bc_value[1]; g.bc_v2 = P.d.bc_value[2]; g.bc_v3 = P.d.bc_value[3];
  g.s_inj = P.d.s_inj;
  g.refine_rtol = P.d.refine_rtol;
  return g;
}

mpm_status hip_check(mpm_run* r, hipError_t e, const char* what) {
  if (e == hipSuccess) return MPM_OK;
  if (r) r->last_error = std::string(what) + ": " + hipGetErrorString(e);
  return MPM_EHIP;
}

#define HIPCHK(r, call)                                   \
  do {                                                    \
    mpm_status s_ = hip_check((r), (call), #call);        \
    if (s_ != MPM_OK) return s_;                          \
  } while (0)

// Status of a nonzero device error word. A non-finite value comes first: it is usually the
// cause of the failed pivots that follow it in the same pass.
mpm_status err_status(int32_t errw) {
  if (errw & ERR_NONFINITE) return MPM_ENONFINITE;
  if (errw & ERR_NOTSPD) return MPM_ENOTSPD;
  if (errw & ERR_SINGULAR) return MPM_ESINGULAR;
  return MPM_ENOCONV;
}

double eps_from(const mpm_run* r, double num, double den) {
  if (r->P.d.eps_norm == MPM_EPS_ABS_L2) return std::sqrt(r->P.hx * r->P.hy * num);
  return std::sqrt(num) / std::sqrt(den);
}

// kappa^n = lambda(s) K and the sums of epsilon against kappa^m, also written by the reduction
// kernel into pinned host memory (the caller records ev_eps after it). With sat the same
// kernel first takes the last transport sub-step (s -> s2, then the buffers swap) and the
// reduction computes the water cut of the new saturation under the current velocity.
// With fork the reduction runs on the second stream, off the path of the velocity update that
// follows (nothing there needs it until the downscaling rewrites the partials, which joins
// the second stream first); the caller records ev_eps on that stream.
mpm_status kappa_and_eps_nodes(mpm_run* r, bool sat = false, bool fork = false) {
  {
    Scope sc(r, sat ? "sat_kappa" : "kappa_eps");
    launch_kappa(r->st, r->g, r->s, r->K, r->kn, r->km, r->red, r->scal, r->dsflag, r->dslist, r->dscount,
                 r->dscount + 1, r->pinned_dev, sat ? r->ux : nullptr, sat ? r->uy : nullptr, one_run(),
                 sat ? r->s2 : nullptr, r->area, fork ? r->st2 : nullptr, r->ev_fork);
  }
  if (sat) std::swap(r->s, r->s2);
  r->eps_seq += 1;
  return MPM_OK;
}

// Host copy of the epsilon sums of the latest kappa launch. The reduction kernel writes them
// to pinned host memory with its sequence number; after the event, a number other than the
// expected one means the data has not reached the host yet: drain the stream and look again.
mpm_status wait_eps(mpm_run* r) {
  volatile double* p = r->pinned;
  if (r->is_static) {   // the copy to pageable host memory has returned, or is drained here
    if (p[2] != double(r->eps_seq)) HIPCHK(r, hipStreamSynchronize(r->st));
    if (p[2] != double(r->eps_seq)) {
      r->last_error = "epsilon sums did not reach host memory";
      return MPM_EHIP;
    }
    return MPM_OK;
  }
  HIPCHK(r, hipEventSynchronize(r->ev_eps));
  if (p[2] != double(r->eps_seq)) {
    HIPCHK(r, hipStreamSynchronize(r->st));
    HIPCHK(r, hipStreamSynchronize(r->st2));
    if (p[2] != double(r->eps_seq)) {
      r->last_error = "epsilon sums did not reach host memory";
      return MPM_EHIP;
    }
  }
  return MPM_OK;
}

// Eager: the reduction forks to the second stream unless graphs are in use (a captured update
// would not join it).
mpm_status kappa_and_eps(mpm_run* r, bool sat = false) {
  const bool fork = !r->use_graphs && r->st2 != r->st;
  mpm_status st = kappa_and_eps_nodes(r, sat, fork);
  if (st) return st;
  if (r->is_static) {
    HIPCHK(r, hipMemcpyAsync(r->pin_host, r->pinned_dev, sizeof(r->pin_host), hipMemcpyDeviceToHost, r->st));
    return MPM_OK;
  }
  HIPCHK(r, hipEventRecord(r->ev_eps, fork ? r->st2 : r->st));
  return MPM_OK;
}

// Work of the caller's stream before a call is ordered before the library's, and the library's
// before the caller's later work.
mpm_status enter(mpm_run* r) {
  if (r->st == r->ust) return MPM_OK;
  HIPCHK(r, hipEventRecord(r->ev_in, r->ust));
  HIPCHK(r, hipStreamWaitEvent(r->st, r->ev_in, 0));
  return MPM_OK;
}
mpm_status leave(mpm_run* r, mpm_status st) {
  if (r->st == r->ust) return st;
  if (hipEventRecord(r->ev_out, r->st) != hipSuccess || hipStreamWaitEvent(r->ust, r->ev_out, 0) != hipSuccess)
    return st ? st : MPM_EHIP;
  return st;
}

// Captures what body() enqueues on the library's stream into an executable graph, then
// launches it once. Returns nullptr (and enqueues nothing) if capture is not available.
template <class F>
hipGraphExec_t capture_and_launch(mpm_run* r, F&& body) {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (hipStreamBeginCapture(r->st, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  const mpm_status st = body();
  const hipError_t e = hipStreamEndCapture(r->st, &graph);
  if (st != MPM_OK || e != hipSuccess || !graph) {
    if (graph) hipGraphDestroy(graph);
    return nullptr;
  }
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
  hipGraphDestroy(graph);
  if (exec && hipGraphLaunch(exec, r->st) != hipSuccess) {
    hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  return exec;
}

// The fused bottom levels of the interface sweeps are on by default; MPM2P_FUSE=0 keeps one
// launch per level (for measurements against them).
bool fuse_default() {
  const char* e = std::getenv("MPM2P_FUSE");
  return !(e && e[0] == '0');
}

LeafOut leaf_dest(const mpm_run* r) { return LeafOut{r->slots, r->leafup, r->nd.map_pool}; }

// With with_v >= 0 the fused backward sweep also reconstructs the boundary fluxes (flux_sub with
// that with_v) where the plan allows it; returns whether it did.
bool nd_solve(mpm_run* r, Runs rt = one_run(), int with_v = -1) {
  const Plan& P = r->P;
  const int L = int(P.level_nodes.size()) - 1;
  const int H = r->fuse ? P.fuse_h : 0;   // levels 1..H: one launch per direction
  const bool flux = H && with_v >= 0 && P.fuse_flux;
  {
    Scope sc(r, "iface_fwd");
    if (H) {
      Scope sf(r, "iface_sub_fwd", true);
      launch_nd_sub_fwd(r->st, r->nd, P.fuse_roots, rt);
    }
    for (int l = H + 1; l < L; ++l) {
      const int nn = int(P.level_nodes[l].size());
      if (!nn) continue;
      const int sh = l < int(r->tune_fwd.size()) ? r->tune_fwd[l] : 0;
      launch_nd_level_fwd(r->st, r->nd, P.level_off[l], nn, P.level_nImax[l], P.level_nBmax[l], rt, sh);
    }
  }
  {
    Scope sc(r, "iface_bwd");
    for (int l = L; l > H; --l) {
      const int nn = int(P.level_nodes[l].size());
      if (!nn) continue;
      const int sh = l < int(r->tune_bwd.size()) ? r->tune_bwd[l] : 0;
      launch_nd_level_bwd(r->st, r->nd, P.level_off[l], nn, P.level_nImax[l], P.level_nmax[l], l == L ? 1 : 0, rt,
                          sh);
    }
    if (H && flux) {
      Scope sb(r, "iface_sub_bwd_flux", true);
      const FluxArgs fa{r->g, r->km, r->S, r->h, r->vbnd, r->subdofs_d, r->ubnd, r->fleaves, with_v};
      launch_nd_sub_bwd(r->st, r->nd, P.fuse_roots, rt, &fa);
    } else if (H) {
      Scope sb(r, "iface_sub_bwd", true);
      launch_nd_sub_bwd(r->st, r->nd, P.fuse_roots, rt);
    }
  }
  return flux;
}

void nd_factor(mpm_run* r, Runs rt = one_run()) {
  const Plan& P = r->P;
  const int L = int(P.level_nodes.size()) - 1;
  Scope sc(r, "iface_factor");
  for (int l = 1; l <= L; ++l) {
    const int nn = int(P.level_nodes[l].size());
    if (!nn) continue;
    launch_nd_level_factor(r->st, r->nd, P.level_off[l], nn, P.level_nmax[l], P.level_nImax[l], P.level_nBmax[l],
                           rt);
  }
}

// flux_done: the interface solve reconstructed the fluxes already; join (if any): waited for
// before the downscaling, the first step that needs the work on the second stream.
mpm_status finish_velocity(mpm_run* r, const double* kap_s, int with_v, int store, Runs rt = one_run(),
                           bool flux_done = false, hipEvent_t join = nullptr) {
  if (!flux_done) {
    Scope sc(r, "flux");
    launch_flux(r->st, r->g, r->km, r->S, r->h, r->vbnd, r->y, r->subdofs_d, r->ubnd, with_v, rt);
  }
  if (with_v && r->P.d.mpm_order == 1) {
    // first-order term (eq:mpm_tf_4): local problems, a second interface solve, u-hat_1 + w
    {
      Scope sc(r, "first_order");
      launch_mpm_first(r->st, r->g, r->kn, r->km, r->uxm, r->uym, r->q, r->fac, r->y, r->subdofs_d, r->ubnd,
                       r->vbnd, r->h, r->wbnd, leaf_dest(r), rt);
    }
    nd_solve(r, rt);
    Scope sc(r, "flux");
    launch_flux(r->st, r->g, r->km, r->S, r->h, r->wbnd, r->y, r->subdofs_d, r->ubnd, 2, rt);
  }
  if (join) HIPCHK(r, hipStreamWaitEvent(r->st, join, 0));
  {
    Scope sc(r, "downscale");
    if (r->f32 && !store)
      launch_downscale_f32(r->st, r->g, kap_s, r->q, r->ubnd, r->ux, r->uy, r->red, r->red + r->P.nsub, r->dsE32,
                           r->nfac32, r->dsflag, r->err, rt);
    else
      launch_downscale(r->st, r->g, kap_s, r->q, r->ubnd, r->ux, r->uy, r->red, r->red + r->P.nsub, r->dsE,
                       r->nfac, r->dsflag, store, r->err, rt);
  }
  if (r->f32 && store) {
    Scope sc(r, "to_f32");
    launch_to_f32(r->st, r->P.n_blocks, r->nfac, r->nfac32, rt);
  }
  {
    Scope sc(r, "dt");
    launch_dt(r->st, r->P.nsub, r->red, r->red + r->P.nsub, r->scal, r->dscount, rt);
  }
  return MPM_OK;
}

// MRCM with a new basis for kappa^n (stored as kappa^m), downscaled with the same kappa.
mpm_status mrcm_update(mpm_run* r) {
  if (r->ev_eps) HIPCHK(r, hipStreamWaitEvent(r->st, r->ev_eps, 0));   // the epsilon reduction may be on st2
  HIPCHK(r, hipMemcpyAsync(r->km, r->kn, size_t(r->P.nx) * r->P.ny * 8, hipMemcpyDeviceToDevice, r->st));
  bool have_fac;
  {
    Scope sc(r, "basis");
    have_fac = launch_basis(r->st, r->g, r->km, r->q, r->S, r->h, r->leafK, leaf_dest(r), r->fac, r->err);
  }
  if (!have_fac) {
    Scope sc(r, "line_factor");
    launch_line_factor(r->st, r->g, r->km, r->fac, r->err);
  }
  if (r->f32) {
    Scope sc(r, "to_f32");
    launch_to_f32(r->st, r->P.n_blocks, r->fac, r->fac32);
  }
  nd_factor(r);
  const bool fd = nd_solve(r, one_run(), 0);
  mpm_status fs = finish_velocity(r, r->km, 0, 1, one_run(), fd);
  if (fs) return fs;
  const size_t fx = size_t(r->P.ny) * (r->P.nx + 1) * 8, fy = size_t(r->P.ny + 1) * r->P.nx * 8;
  HIPCHK(r, hipMemcpyAsync(r->uxm, r->ux, fx, hipMemcpyDeviceToDevice, r->st));
  HIPCHK(r, hipMemcpyAsync(r->uym, r->uy, fy, hipMemcpyDeviceToDevice, r->st));
  r->tm += 1;
  return MPM_OK;
}

// The same update for the runs g (equal descriptors, led by g[0], run table rt): one launch per
// phase over all of them, on the leader's stream.
mpm_status mrcm_update_group(const std::vector<mpm_run*>& g, Runs rt) {
  mpm_run* r = g[0];
  const size_t nc = size_t(r->P.nx) * r->P.ny * 8;
  for (mpm_run* x : g) HIPCHK(r, hipMemcpyAsync(x->km, x->kn, nc, hipMemcpyDeviceToDevice, r->st));
  const bool have_fac = launch_basis(r->st, r->g, r->km, r->q, r->S, r->h, r->leafK, leaf_dest(r), r->fac, r->err, rt);
  if (!have_fac) launch_line_factor(r->st, r->g, r->km, r->fac, r->err, rt);
  if (r->f32) launch_to_f32(r->st, r->P.n_blocks, r->fac, r->fac32, rt);
  nd_factor(r, rt);
  const bool fd = nd_solve(r, rt, 0);
  mpm_status fs = finish_velocity(r, r->km, 0, 1, rt, fd);
  if (fs) return fs;
  const size_t fx = size_t(r->P.ny) * (r->P.nx + 1) * 8, fy = size_t(r->P.ny + 1) * r->P.nx * 8;
  for (mpm_run* x : g) {
    HIPCHK(r, hipMemcpyAsync(x->uxm, x->ux, fx, hipMemcpyDeviceToDevice, r->st));
    HIPCHK(r, hipMemcpyAsync(x->uym, x->uy, fy, hipMemcpyDeviceToDevice, r->st));
    x->tm += 1;
  }
  HIPCHK(r, hipGetLastError());
  return MPM_OK;
}

// MPM-2P: trivial-Robin solve with the stored kappa^m factors, interface solve with the stored
// factorisation, reconstruction, downscaling with kappa^n.
mpm_status mpm_update_body(mpm_run* r, bool capturing, Runs rt = one_run()) {
  // kappa^n Neumann factors of the changed subdomains on the second stream, overlapped with
  // the local and interface solves. It forks at the epsilon event, recorded right after the
  // conductivity and its changed-subdomain list (one marker on the main stream, not two).
  // (Under graph capture the fork must be recorded inside the capture: a marker of its own.)
  // (A run with one stream, the static workspace's, takes them in stream order.)
  const bool two = r->st2 != r->st;
  if (two && capturing) {
    HIPCHK(r, hipEventRecord(r->ev_fork, r->st));
    HIPCHK(r, hipStreamWaitEvent(r->st2, r->ev_fork, 0));
  } else if (two) {
    HIPCHK(r, hipStreamWaitEvent(r->st2, r->ev_eps, 0));
  }
  if (r->f32) launch_ds_factor_f32(r->st2, r->g, r->kn, r->dsE32, r->dslist, r->dscount, r->err, rt);
  else launch_ds_factor(r->st2, r->g, r->kn, r->dsE, r->dslist, r->dscount, r->err, rt);
  if (two) HIPCHK(r, hipEventRecord(r->ev_join, r->st2));
  {
    Scope sc(r, "mpm_local");
    if (r->f32)
      launch_mpm_local_f32(r->st, r->g, r->kn, r->km, r->uxm, r->uym, r->q, r->fac32, r->h, r->vbnd, leaf_dest(r),
                           r->err, rt);
    else
      launch_mpm_local(r->st, r->g, r->kn, r->km, r->uxm, r->uym, r->q, r->fac, r->h, r->vbnd, leaf_dest(r), r->err,
                       rt);
  }
  const bool fd = nd_solve(r, rt, 1);
  return finish_velocity(r, r->kn, 1, 0, rt, fd, two ? r->ev_join : nullptr);
}

mpm_status mpm_update(mpm_run* r) {
  if (r->use_graphs && !r->prof) {
    if (r->g_mpm) {
      HIPCHK(r, hipGraphLaunch(r->g_mpm, r->st));
      return MPM_OK;
    }
    r->g_mpm = capture_and_launch(r, [&] { return mpm_update_body(r, true); });
    if (r->g_mpm) return MPM_OK;
    r->use_graphs = false;   // capture unavailable: stay eager
  }
  return mpm_update_body(r, false);
}

// The update for a decision value (Algorithm 1: "if epsilon > eta"; force overrides it).
mpm_status vu_update(mpm_run* r, int32_t force, double decide) {
  int branch = decide > r->P.d.eta ? MPM_FORCE_MRCM : MPM_FORCE_MPM;
  if (force == MPM_FORCE_MPM || force == MPM_FORCE_MRCM) branch = force;
  mpm_status st;
  if (branch == MPM_FORCE_MRCM) {
    st = mrcm_update(r);
    r->eps_prev = 0.0;
    r->eps_pending = false;
  } else {
    st = mpm_update(r);
    r->eps_pending = true;
  }
  if (st) return st;
  r->last_branch = branch;
  r->te += 1;
  return MPM_OK;
}

// After the update is enqueued: epsilon of this update for the next decision. With the lagged
// rule it was reduced before the solve, so waiting for it does not drain the stream.
mpm_status vu_finish(mpm_run* r) {
  if (r->eps_pending) {
    if (r->P.d.switch_rule == MPM_SWITCH_ALG1) {
      mpm_status st = wait_eps(r);
      if (st) return st;
    }
    r->eps_prev = eps_from(r, r->pinned[0], r->pinned[1]);
    r->eps_pending = false;
  }
  return MPM_OK;
}

// The decision value: epsilon of the current saturation (text rule; waits for it) or of the
// previous update (Algorithm 1 as written).
mpm_status vu_decision(mpm_run* r, double* decide) {
  if (r->P.d.switch_rule == MPM_SWITCH_TEXT) {
    mpm_status st = wait_eps(r);
    if (st) return st;
    *decide = eps_from(r, r->pinned[0], r->pinned[1]);
  } else {
    *decide = r->eps_prev;
  }
  return MPM_OK;
}

mpm_status velocity_update(mpm_run* r, int32_t force, bool kappa_done = false) {
  mpm_status st = MPM_OK;
  if (!kappa_done) st = kappa_and_eps(r);
  if (st) return st;
  double decide;
  st = vu_decision(r, &decide);
  if (st) return st;
  st = vu_update(r, force, decide);
  if (st) return st;
  return vu_finish(r);
}

// Transport sub-steps; the water cut here unless the conductivity reduction that follows
// computes it (wc = false).
mpm_status transport_body(mpm_run* r, int32_t nsteps, bool wc = true) {
  for (int k = 0; k < nsteps; ++k) {
    Scope sc(r, "sat_step");
    launch_sat_step(r->st, r->g, r->s, r->s2, r->ux, r->uy, r->scal, r->area);
    std::swap(r->s, r->s2);
  }
  if (wc) {
    Scope sc(r, "water_cut");
    launch_water_cut(r->st, r->g, r->s, r->ux, r->uy, r->scal, r->red + 2 * r->P.nsub, r->wc_ticket);
  }
  return MPM_OK;
}

mpm_status transport(mpm_run* r, int32_t nsteps, bool wc = true) {
  mpm_status st = transport_body(r, nsteps, wc);
  r->ntr += nsteps;
  return st;
}

// C_n transport sub-steps and kappa^n with its epsilon sums and the water cut (event ev_eps
// recorded after them); the last sub-step is taken by the conductivity kernel. With graphs
// they are one graph per parity of the saturation buffers.
mpm_status transport_and_kappa(mpm_run* r) {
  const int cn = r->P.d.cn;
  if (r->use_graphs && !r->prof) {
    const int par = r->s == r->s_base ? 0 : 1;
    if (r->g_trans[par]) {
      HIPCHK(r, hipGraphLaunch(r->g_trans[par], r->st));
      r->eps_seq += 1;
      for (int k = 0; k < cn; ++k) std::swap(r->s, r->s2);
      r->ntr += cn;
      HIPCHK(r, hipEventRecord(r->ev_eps, r->st));
      return MPM_OK;
    }
    double* s0 = r->s;
    double* s1 = r->s2;
    r->g_trans[par] = capture_and_launch(r, [&] {
      mpm_status st = transport_body(r, cn - 1, false);
      if (st) return st;
      return kappa_and_eps_nodes(r, true);
    });
    if (r->g_trans[par]) {
      r->ntr += cn;
      HIPCHK(r, hipEventRecord(r->ev_eps, r->st));
      return MPM_OK;
    }
    // capture unavailable: stay eager
    r->s = s0;
    r->s2 = s1;
    r->use_graphs = false;
  }
  mpm_status st = transport(r, cn - 1, false);
  if (st) return st;
  r->ntr += 1;
  return kappa_and_eps(r, true);
}

// One pass of Algorithm 1's while loop.
mpm_status step(mpm_run* r, int32_t force) {
  mpm_status st = transport_and_kappa(r);
  if (st) return st;
  return velocity_update(r, force, true);
}

// Points the run's buffers into the workspace ws (the plan's layout) and checks that every
// device pointer the kernels take lies inside it.
bool bind_workspace(mpm_run* r, char* ws) {
  const Plan& P = r->P;
  r->g = make_geo(P);
  r->ws = ws;
  auto D = [&](size_t off) { return reinterpret_cast<double*>(r->ws + off); };
  r->K = D(P.off_K); r->q = D(P.off_q); r->s = D(P.off_s); r->s2 = D(P.off_s2);
  r->kn = D(P.off_kn); r->km = D(P.off_km); r->ux = D(P.off_ux); r->uy = D(P.off_uy);
  r->uxm = D(P.off_uxm); r->uym = D(P.off_uym); r->fac = D(P.off_fac); r->S = D(P.off_S);
  r->h = D(P.off_h); r->vbnd = D(P.off_vbnd); r->ubnd = D(P.off_ubnd); r->leafK = D(P.off_leafK);
  r->front = D(P.off_front); r->fI = D(P.off_fI); r->slots = D(P.off_slot);
  r->panel = D(P.off_panel); r->y = D(P.off_y); r->red = D(P.off_red); r->scal = D(P.off_scal);
  r->dsE = D(P.off_dsE); r->nfac = D(P.off_nfac);
  if (P.d.mpm_order == 1) r->wbnd = D(P.off_wbnd);
  r->f32 = P.d.precision == MPM_PREC_FP32_REFINE;
  if (r->f32) {
    r->fac32 = reinterpret_cast<float*>(r->ws + P.off_fac32);
    r->nfac32 = reinterpret_cast<float*>(r->ws + P.off_nfac32);
    r->dsE32 = reinterpret_cast<float*>(r->ws + P.off_dsE32);
  }
  r->s_base = r->s;
  r->dsflag = reinterpret_cast<int32_t*>(r->ws + P.off_dsflag);
  r->dslist = reinterpret_cast<int32_t*>(r->ws + P.off_dslist);
  r->err = reinterpret_cast<int32_t*>(r->scal + SC_COUNT);
  r->wc_ticket = r->err + 8;   // in the zeroed tail of the scalar block
  r->dscount = r->err + 1;
  r->subdofs_d = reinterpret_cast<const int32_t*>(r->ws + P.off_subdofs);
  r->nd.nodes = reinterpret_cast<const NodeDev*>(r->ws + P.off_nodes);
  r->nd.levels = reinterpret_cast<const int32_t*>(r->ws + P.off_levels);
  r->nd.dof_pool = reinterpret_cast<const int32_t*>(r->ws + P.off_dofpool);
  r->nd.map_pool = reinterpret_cast<const int32_t*>(r->ws + P.off_mappool);
  r->nd.inv_pool = reinterpret_cast<const int32_t*>(r->ws + P.off_invpool);
  r->nd.front = r->front; r->nd.fI = r->fI; r->nd.slots = r->slots; r->nd.panel = r->panel;
  r->nd.leafK = r->leafK; r->nd.y = r->y; r->nd.ndmax = P.ndmax;
  r->nd.piv_b = P.piv_b; r->nd.err = r->err;
  r->nd.lnodes = reinterpret_cast<const NodeDev*>(r->ws + P.off_lnodes);
  r->nd.fnodes = reinterpret_cast<const FuseNode*>(r->ws + P.off_fnodes);
  r->nd.flevels = reinterpret_cast<const FuseLevel*>(r->ws + P.off_flevels);
  r->nd.fxsrc = reinterpret_cast<const int32_t*>(r->ws + P.off_fxsrc);
  r->fleaves = reinterpret_cast<const int32_t*>(r->ws + P.off_fleaves);
  r->nd.fuse_h = P.fuse_h;
  r->fuse = P.fuse_h > 0 && fuse_default();
  r->leafup = reinterpret_cast<const LeafUp*>(r->ws + P.off_leafup);
  r->M = P.d.mu_o / P.d.mu_w;
  r->fmax_deriv = max_fprime(r->M);
  r->params[SC_MUW - SC_MUW] = P.d.mu_w;
  r->params[SC_MUO - SC_MUW] = P.d.mu_o;
  r->params[SC_MRATIO - SC_MUW] = r->M;
  r->params[SC_CFL - SC_MUW] = P.d.cfl;
  r->params[SC_FMAX - SC_MUW] = r->fmax_deriv;
  r->area = P.d.lx * P.d.ly;
  const char* lo = r->ws;
  const char* hi = r->ws + P.total_bytes;
  auto in = [&](const void* p, size_t n) {
    const char* c = static_cast<const char*>(p);
    return c != nullptr && c >= lo && c + n <= hi;
  };
  const size_t cb = size_t(P.nx) * P.ny * 8, ns = size_t(P.nsub);
  const size_t fx = size_t(P.ny) * (P.nx + 1) * 8, fy = size_t(P.ny + 1) * P.nx * 8;
  return in(r->K, cb) && in(r->q, cb) && in(r->s, cb) && in(r->s2, cb) && in(r->kn, cb) && in(r->km, cb) &&
         in(r->ux, fx) && in(r->uy, fy) && in(r->uxm, fx) && in(r->uym, fy) &&
         in(r->S, ns * ((P.nb / 2 + 1) * P.nb) * 8) && in(r->h, ns * P.nb * 8) && in(r->vbnd, ns * P.nb * 8) &&
         in(r->ubnd, ns * P.nb * 8) && in(r->leafK, ns * P.ndmax * P.ndmax * 8) && in(r->red, P.n_red * 8) &&
         in(r->scal, SC_COUNT * 8) && in(r->err, 12) && in(r->dscount, 8) && in(r->dsflag, ns * 4) &&
         in(r->dslist, ns * 4) && in(r->y, size_t(std::max(P.n_iface, 1)) * 8) &&
         in(r->subdofs_d, ns * P.ndmax * 4) && in(r->slots, size_t(std::max<int64_t>(P.slot_doubles, 1)) * 8) &&
         in(r->leafup, ns * sizeof(LeafUp)) &&
         (!r->f32 || (in(r->fac32, P.n_blocks * 4) && in(r->nfac32, P.n_blocks * 4) && in(r->dsE32, P.n_blocks * 4))) &&
         in(r->nd.lnodes, std::max<size_t>(P.lnodes.size(), 1) * sizeof(NodeDev)) &&
         in(r->nd.fnodes, std::max<size_t>(P.fnodes.size(), 1) * sizeof(FuseNode)) &&
         in(r->nd.flevels, std::max<size_t>(P.flevels.size(), 1) * sizeof(FuseLevel)) &&
         in(r->nd.fxsrc, std::max<size_t>(P.fxsrc.size(), 1) * 4) &&
         in(r->fleaves, std::max<size_t>(P.fleaves.size(), 1) * 4) &&
         (P.d.mpm_order != 1 || in(r->wbnd, ns * P.nb * 8));
}

// Uploads the plan's index tables into the workspace and clears what the kernels expect at
// zero (the forward-solve slots, the scalar block with its integer words, the interface
// solution), on the run's stream.
hipError_t upload_plan(mpm_run* r) {
  const Plan& P = r->P;
  auto up = [&](size_t off, const void* src, size_t n) {
    return n ? hipMemcpyAsync(r->ws + off, src, n, hipMemcpyHostToDevice, r->st) : hipSuccess;
  };
  hipError_t e = hipSuccess;
  auto chain = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  chain(up(P.off_nodes, P.nodes.data(), P.nodes.size() * sizeof(NodeDev)));
  chain(up(P.off_levels, P.level_flat.data(), P.level_flat.size() * 4));
  chain(up(P.off_lnodes, P.lnodes.data(), P.lnodes.size() * sizeof(NodeDev)));
  chain(up(P.off_fnodes, P.fnodes.data(), P.fnodes.size() * sizeof(FuseNode)));
  chain(up(P.off_flevels, P.flevels.data(), P.flevels.size() * sizeof(FuseLevel)));
  chain(up(P.off_fxsrc, P.fxsrc.data(), P.fxsrc.size() * 4));
  chain(up(P.off_fleaves, P.fleaves.data(), P.fleaves.size() * 4));
  chain(up(P.off_leafup, P.leafup.data(), P.leafup.size() * sizeof(LeafUp)));
  chain(hipMemsetAsync(r->slots, 0, size_t(std::max<int64_t>(P.slot_doubles, 1)) * 8, r->st));
  chain(up(P.off_dofpool, P.dof_pool.data(), P.dof_pool.size() * 4));
  chain(up(P.off_mappool, P.map_pool.data(), P.map_pool.size() * 4));
  chain(up(P.off_invpool, P.inv_pool.data(), P.inv_pool.size() * 4));
  chain(up(P.off_subdofs, P.sub_dofs.data(), P.sub_dofs.size() * 4));
  chain(up(P.off_subndof, P.sub_ndof.data(), P.sub_ndof.size() * 4));
  chain(hipMemsetAsync(r->scal, 0, SC_COUNT * 8 + 64, r->st));
  chain(hipMemsetAsync(r->y, 0, size_t(std::max(P.n_iface, 1)) * 8, r->st));
  return e;
}

// Workspace of the runs made by mpm_create_static: a file-scope device array, one copy on every
// device the library runs on, held until the process ends. Its name in host code is a host-side
// stand-in; the device address comes from hipGetSymbolAddress, once per device, with that
// device current, and only that address is handed to kernels and copies.
static __device__ __align__(256) char scratch[MPM_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char* g_static_ptr[kMaxDevices] = {};   // device address of scratch on each device
bool g_static_busy[kMaxDevices] = {};   // a live run holds the device's array

// Bytes a run takes from the static array: the plan's workspace, then 256 bytes for the
// epsilon and water-cut block that the reduction kernel writes.
size_t static_bytes(const Plan& P) { return ((P.total_bytes + 255) & ~size_t(255)) + 256; }

// Sweep launch shapes found by mpm_tune, by decomposition (the nested-dissection plan depends on
// the grid, the subdomains, the interface elements and their degree): runs created later with the
// same decomposition start from them.
std::mutex g_tune_mu;
struct TuneChoice {
  std::vector<int> fwd, bwd;
  bool fuse;
};
std::map<std::string, TuneChoice> g_tune_cache;

std::string tune_key(const mpm_desc& d) {
  const int32_t v[7] = {d.nx, d.ny, d.sub_x, d.sub_y, d.ne_x, d.ne_y, d.iface_degree};
  return std::string(reinterpret_cast<const char*>(v), sizeof(v));
}

void tune_from_cache(mpm_run* r) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune_cache.find(tune_key(r->P.d));
  if (it != g_tune_cache.end()) {
    r->tune_fwd = it->second.fwd;
    r->tune_bwd = it->second.bwd;
    r->fuse = it->second.fuse && r->P.fuse_h > 0;
  }
}

void release_static(int device) {
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (device >= 0 && device < kMaxDevices) g_static_busy[device] = false;
}

}  // namespace

extern "C" {

const char* mpm_status_str(mpm_status s) {
  switch (s) {
    case MPM_OK: return "ok";
    case MPM_EINVAL: return "invalid argument";
    case MPM_ENOMEM: return "workspace too small or host allocation failed";
    case MPM_ENOTSPD: return "local matrix not positive definite";
    case MPM_ESINGULAR: return "interface system singular";
    case MPM_ENONFINITE: return "non-finite value";
    case MPM_EHIP: return "HIP runtime error";
    case MPM_ESTATE: return "call not valid in the current state";
    case MPM_ENOCONV: return "refinement of a local solve did not converge";
    default: return "unknown status";
  }
}

mpm_status mpm_workspace_size(const mpm_desc* desc, size_t* bytes) {
  if (!desc || !bytes) return MPM_EINVAL;
  if (validate(*desc, nullptr) != MPM_OK) return MPM_EINVAL;
  Plan P;
  build_plan(*desc, &P);
  *bytes = P.total_bytes;
  return MPM_OK;
}

mpm_status mpm_create(const mpm_desc* desc, void* dev_workspace, size_t bytes, void* hip_stream, mpm_run** out) {
  if (!desc || !out) return MPM_EINVAL;
  *out = nullptr;
  if (validate(*desc, nullptr) != MPM_OK) return MPM_EINVAL;
  if (!dev_workspace || (reinterpret_cast<uintptr_t>(dev_workspace) & 255)) return MPM_EINVAL;
  mpm_run* r = new (std::nothrow) mpm_run();
  if (!r) return MPM_ENOMEM;
  build_plan(*desc, &r->P);
  if (bytes < r->P.total_bytes) { delete r; return MPM_ENOMEM; }
  r->ust = static_cast<hipStream_t>(hip_stream);
  hipGetDevice(&r->device);
#define CREATE_CHK(call)                                                           \
  do {                                                                             \
    const hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                        \
      g_create_error = std::string(#call) + ": " + hipGetErrorString(e_);          \
      return fail(MPM_EHIP);                                                       \
    }                                                                              \
  } while (0)
  auto fail = [&](mpm_status s) {
    if (r->pinned) hipHostFree(r->pinned);
    if (r->ev_eps) hipEventDestroy(r->ev_eps);
    if (r->ev_fork) hipEventDestroy(r->ev_fork);
    if (r->ev_join) hipEventDestroy(r->ev_join);
    if (r->ev_in) hipEventDestroy(r->ev_in);
    if (r->ev_out) hipEventDestroy(r->ev_out);
    if (r->st2) hipStreamDestroy(r->st2);
    if (r->st && r->st != r->ust) hipStreamDestroy(r->st);
    delete r;
    return s;
  };
  if (!bind_workspace(r, static_cast<char*>(dev_workspace))) return fail(MPM_EINVAL);
  CREATE_CHK(hipHostMalloc(reinterpret_cast<void**>(&r->pinned), 64, hipHostMallocDefault));
  CREATE_CHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&r->pinned_dev), r->pinned, 0));
  if (!r->pinned_dev) return fail(MPM_EHIP);
  r->pinned[0] = r->pinned[1] = r->pinned[2] = r->pinned[3] = 0.0;
  // events that only order work on the device (and the epsilon event, whose host-side data
  // is checked by sequence number): device-scope release, no cache writeback to system scope
  const unsigned ev_flags = hipEventDisableTiming | hipEventReleaseToDevice;
  CREATE_CHK(hipEventCreateWithFlags(&r->ev_eps, ev_flags));
  CREATE_CHK(hipEventCreateWithFlags(&r->ev_fork, ev_flags));
  CREATE_CHK(hipEventCreateWithFlags(&r->ev_join, ev_flags));
  CREATE_CHK(hipEventCreateWithFlags(&r->ev_in, hipEventDisableTiming));
  CREATE_CHK(hipEventCreateWithFlags(&r->ev_out, hipEventDisableTiming));
  // Graph replay is opt-in: on gfx950 it measured slower than eager launches for this step.
  // With graphs the work runs on a stream of the library's own (capture needs one), ordered
  // against the caller's stream by events; without, it runs on the caller's stream.
  {
    const char* e = std::getenv("MPM2P_GRAPHS");
    r->use_graphs = e && e[0] && e[0] != '0';
  }
  // the library's streams, default priority
  if (r->use_graphs) {
    CREATE_CHK(hipStreamCreateWithFlags(&r->st, hipStreamNonBlocking));
  } else {
    r->st = r->ust;
  }
  CREATE_CHK(hipStreamCreateWithFlags(&r->st2, hipStreamNonBlocking));
  CREATE_CHK(hipStreamSynchronize(r->ust));
  if (upload_plan(r) != hipSuccess || hipStreamSynchronize(r->st) != hipSuccess) return fail(MPM_EHIP);
  tune_from_cache(r);
  *out = r;
  return MPM_OK;
}

mpm_status mpm_create_static(const mpm_desc* desc, void* hip_stream, mpm_run** out) {
  if (!desc || !out) return MPM_EINVAL;
  *out = nullptr;
  if (validate(*desc, nullptr) != MPM_OK) return MPM_EINVAL;
  mpm_run* r = new (std::nothrow) mpm_run();
  if (!r) return MPM_ENOMEM;
  build_plan(*desc, &r->P);
  const size_t need = static_bytes(r->P);
  if (need > size_t(MPM_STATIC_WORKSPACE_BYTES)) {
    g_create_error = "the run needs " + std::to_string(need) + " bytes of workspace; the static array holds " +
                     std::to_string(size_t(MPM_STATIC_WORKSPACE_BYTES));
    delete r;
    return MPM_ENOMEM;
  }
  if (hipGetDevice(&r->device) != hipSuccess || r->device < 0 || r->device >= kMaxDevices) {
    g_create_error = "no current device";
    delete r;
    return MPM_EHIP;
  }
  char* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_busy[r->device]) {
      g_create_error = "the static workspace of this device is held by another run";
      delete r;
      return MPM_ESTATE;
    }
    if (!g_static_ptr[r->device]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        g_create_error = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
        delete r;
        return MPM_EHIP;
      }
      g_static_ptr[r->device] = static_cast<char*>(p);
    }
    ws = g_static_ptr[r->device];
    g_static_busy[r->device] = true;
  }
  const int device = r->device;
  auto fail = [&](mpm_status s, const char* what, hipError_t e) {
    g_create_error = std::string(what) + ": " + hipGetErrorString(e);
    delete r;
    release_static(device);
    return s;
  };
  r->is_static = true;
  r->use_graphs = false;
  r->ust = static_cast<hipStream_t>(hip_stream);
  r->st = r->st2 = r->ust;   // one stream: the caller's
  if (!bind_workspace(r, ws)) return fail(MPM_EINVAL, "workspace layout does not fit", hipErrorInvalidValue);
  r->pinned = r->pin_host;
  r->pinned_dev = reinterpret_cast<double*>(ws + static_bytes(r->P) - 256);
  hipError_t e = hipMemsetAsync(r->pinned_dev, 0, 256, r->st);
  if (e != hipSuccess) return fail(MPM_EHIP, "hipMemsetAsync", e);
  e = upload_plan(r);
  if (e == hipSuccess) e = hipStreamSynchronize(r->st);
  if (e != hipSuccess) return fail(MPM_EHIP, "plan upload", e);
  tune_from_cache(r);
  *out = r;
  return MPM_OK;
}

mpm_status mpm_set_fields(mpm_run* r, const double* K, const double* q, const double* s0) {
  if (!r || !K || !s0) return MPM_EINVAL;
  mpm_status st = enter(r);
  if (st) return st;
  const size_t nb = size_t(r->P.nx) * r->P.ny * 8;
  auto body = [&]() -> mpm_status {
    HIPCHK(r, hipMemcpyAsync(r->K, K, nb, hipMemcpyDeviceToDevice, r->st));
    if (q) HIPCHK(r, hipMemcpyAsync(r->q, q, nb, hipMemcpyDeviceToDevice, r->st));
    else HIPCHK(r, hipMemsetAsync(r->q, 0, nb, r->st));
    HIPCHK(r, hipMemcpyAsync(r->s, s0, nb, hipMemcpyDeviceToDevice, r->st));
    HIPCHK(r, hipMemsetAsync(r->km, 0, nb, r->st));
    return MPM_OK;
  };
  st = leave(r, body());
  if (st) return st;
  r->fields = true;
  r->started = false;
  return MPM_OK;
}

mpm_status mpm_start(mpm_run* r) {
  if (!r) return MPM_EINVAL;
  if (!r->fields || r->poisoned) return MPM_ESTATE;
  mpm_status st = enter(r);
  if (st) return st;
  // Algorithm 1, initialisation
  auto body = [&]() -> mpm_status {
    HIPCHK(r, hipMemsetAsync(r->scal, 0, SC_COUNT * 8, r->st));
    HIPCHK(r, hipMemcpyAsync(r->scal + SC_MUW, r->params, sizeof(r->params), hipMemcpyHostToDevice, r->st));
    mpm_status s2 = kappa_and_eps(r);
    if (s2) return s2;
    r->te = 0; r->tm = 0; r->ntr = 0;
    return mrcm_update(r);
  };
  st = leave(r, body());
  if (st) return st;
  r->te = 1;
  r->eps_prev = r->P.d.eta;
  r->eps_pending = false;
  r->last_branch = MPM_FORCE_MRCM;
  r->started = true;
  return MPM_OK;
}

mpm_status mpm_transport(mpm_run* r, int32_t nsteps) {
  if (!r || nsteps < 0) return MPM_EINVAL;
  if (!r->started || r->poisoned) return MPM_ESTATE;
  mpm_status st = enter(r);
  if (st) return st;
  return leave(r, transport(r, nsteps));
}

mpm_status mpm_velocity_update(mpm_run* r, int32_t force) {
  if (!r || force < -1 || force > 1) return MPM_EINVAL;
  if (!r->started || r->poisoned) return MPM_ESTATE;
  mpm_status st = enter(r);
  if (st) return st;
  return leave(r, velocity_update(r, force));
}

mpm_status mpm_step(mpm_run* r, int32_t force) {
  if (!r || force < -1 || force > 1) return MPM_EINVAL;
  if (!r->started || r->poisoned) return MPM_ESTATE;
  mpm_status st = enter(r);
  if (st) return st;
  return leave(r, step(r, force));
}

mpm_status mpm_advance(mpm_run* r, int32_t max_updates, int32_t stop_at_breakthrough, int32_t* done) {
  if (!r || max_updates < 0) return MPM_EINVAL;
  if (!r->started || r->poisoned) return MPM_ESTATE;
  mpm_status st = enter(r);
  if (st) return st;
  int32_t n = 0;
  while (n < max_updates) {
    st = step(r, MPM_AUTO);
    if (st) break;
    ++n;
    // the water cut reaches host memory with the epsilon sums of the same step; a pass that
    // took the MRCM branch has not waited for them yet (the wait ends at the conductivity
    // kernel's reduction, ahead of the basis update)
    if (stop_at_breakthrough) {
      st = wait_eps(r);
      if (st) break;
      if (r->pinned[3] >= r->P.d.breakthrough_cut) break;
    }
  }
  if (done) *done = n;
  return leave(r, st);
}

mpm_status mpm_last_error(const mpm_run* r, char* buf, size_t len) {
  if (!buf || !len) return MPM_EINVAL;
  const std::string& e = r ? r->last_error : g_create_error;
  const size_t n = std::min(len - 1, e.size());
  std::memcpy(buf, e.data(), n);
  buf[n] = 0;
  return MPM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batch of runs
// Runs whose descriptors are equal (and whose saturation buffers have the same parity) form a
// group: each phase of a step is one launch for the whole group (grid z over the runs, a table
// of workspace offsets as a kernel argument), on streams the batch owns. Other runs step alone
// on their own streams. Every run's work is issued before any wait.
struct GroupStreams {
  hipStream_t st = nullptr, st2 = nullptr;
  hipEvent_t ev_eps = nullptr, ev_move = nullptr;
};

struct mpm_batch {
  std::vector<mpm_run*> slot;
  std::vector<GroupStreams> gs;
  std::map<std::string, int> gs_of;   // group key -> index into gs
};

namespace {

// The descriptor fields that shape the launches, one by one (no padding bytes), and the
// saturation parity. The viscosities and cfl (read by the kernels from each run's scalar
// block) and eta, the epsilon norm and the breakthrough cut (host-side, per run) may differ
// inside a group.
std::string group_key(const mpm_run* r) {
  const mpm_desc& d = r->P.d;
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
  put(&d.abi_version, 4); put(&d.nx, 4); put(&d.ny, 4); put(&d.lx, 8); put(&d.ly, 8);
  put(&d.sub_x, 4); put(&d.sub_y, 4); put(&d.ne_x, 4); put(&d.ne_y, 4); put(&d.alpha, 8);
  put(&d.switch_rule, 4); put(&d.precision, 4); put(&d.cn, 4); put(d.bc_kind, 16); put(d.bc_value, 32);
  put(&d.s_inj, 8); put(&d.mpm_order, 4); put(&d.iface_degree, 4);
  k.push_back(r->s == r->s_base ? 0 : 1);
  return k;
}

// Index into b->gs of the streams of a group (created on first use; the vector may grow, so
// callers keep the index, not a pointer).
mpm_status group_streams(mpm_batch* b, const std::string& key, int* out) {
  auto it = b->gs_of.find(key);
  if (it != b->gs_of.end()) { *out = it->second; return MPM_OK; }
  constexpr size_t kMaxPairs = 16;   // further groups share stream pairs (serialised, still correct)
  if (b->gs.size() >= kMaxPairs) {
    const int i = int(b->gs_of.size() % kMaxPairs);
    b->gs_of[key] = i;
    *out = i;
    return MPM_OK;
  }
  GroupStreams g;
  const unsigned ev_flags = hipEventDisableTiming | hipEventReleaseToDevice;
  if (hipStreamCreateWithFlags(&g.st, hipStreamNonBlocking) != hipSuccess) return MPM_EHIP;
  if (hipStreamCreateWithFlags(&g.st2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&g.ev_eps, ev_flags) != hipSuccess ||
      hipEventCreateWithFlags(&g.ev_move, hipEventDisableTiming) != hipSuccess) {
    if (g.st2) hipStreamDestroy(g.st2);
    if (g.ev_eps) hipEventDestroy(g.ev_eps);
    hipStreamDestroy(g.st);
    return MPM_EHIP;
  }
  b->gs.push_back(g);
  b->gs_of[key] = int(b->gs.size()) - 1;
  *out = int(b->gs.size()) - 1;
  return MPM_OK;
}

// The run's work moves to stream st (ordered after everything issued for it so far, including
// the caller's stream), or back home with st = nullptr.
mpm_status move_run(mpm_run* r, hipStream_t st) {
  hipStream_t to = st ? st : r->home;
  if (!to || r->st == to) return MPM_OK;
  if (!r->home) {
    mpm_status e = enter(r);
    if (e) return e;
  }
  HIPCHK(r, hipEventRecord(r->ev_out, r->st));
  HIPCHK(r, hipStreamWaitEvent(to, r->ev_out, 0));
  if (!r->home) r->home = r->st;
  r->st = to;
  if (to == r->home) r->home = nullptr;
  return MPM_OK;
}

// Table `which` of the group g led by g[0], written into the leader's workspace on stream st
// when it differs from the one already there.
mpm_status group_tab(const std::vector<mpm_run*>& g, int which, hipStream_t st, Runs* out) {
  mpm_run* L = g[0];
  RunTab& t = L->tab_host[which];
  const unsigned n = unsigned(g.size());
  bool same = L->tab_n[which] == n;
  for (unsigned i = 0; i < n; ++i) {
    const int64_t w = int64_t(g[i]->ws - L->ws);
    const int64_t h = int64_t(reinterpret_cast<char*>(g[i]->pinned_dev) - reinterpret_cast<char*>(L->pinned_dev));
    same = same && t.ws[i] == w && t.host[i] == h;
    t.ws[i] = w;
    t.host[i] = h;
  }
  RunTab* dev = reinterpret_cast<RunTab*>(L->ws + L->P.off_rtab) + which;
  if (!same) {
    HIPCHK(L, hipMemcpyAsync(dev, &t, sizeof(RunTab), hipMemcpyHostToDevice, st));
    L->tab_n[which] = n;
  }
  *out = Runs{dev, n};
  return MPM_OK;
}

// Epsilon sums of the group's latest conductivity launch on the host (one event for the group,
// then each run's sequence number).
mpm_status group_wait_eps(const std::vector<mpm_run*>& g, GroupStreams& gs) {
  if (hipEventSynchronize(gs.ev_eps) != hipSuccess) return MPM_EHIP;
  for (mpm_run* r : g) {
    volatile double* p = r->pinned;
    if (p[2] != double(r->eps_seq)) {
      HIPCHK(r, hipStreamSynchronize(r->st));
      if (p[2] != double(r->eps_seq)) {
        r->last_error = "epsilon sums did not reach host memory";
        return MPM_EHIP;
      }
    }
  }
  return MPM_OK;
}

// One pass of Algorithm 1's while loop for a group of at least two runs on its streams, up to
// the wait for the epsilon of the updated runs (group_finish).
mpm_status group_issue(std::vector<mpm_run*>& g, GroupStreams& gs, std::vector<mpm_run*>* updated) {
  for (mpm_run* r : g) {
    mpm_status e = move_run(r, gs.st);
    if (e) return e;
  }
  mpm_run* L = g[0];
  Runs rt;
  {
    mpm_status e = group_tab(g, 0, gs.st, &rt);
    if (e) return e;
  }
  const int cn = L->P.d.cn;
  // transport sub-steps, conductivity, epsilon sums and water cut of every run (the last
  // sub-step taken by the conductivity kernel)
  for (int k = 0; k + 1 < cn; ++k) {
    launch_sat_step(gs.st, L->g, L->s, L->s2, L->ux, L->uy, L->scal, L->area, rt);
    for (mpm_run* r : g) std::swap(r->s, r->s2);
  }
  launch_kappa(gs.st, L->g, L->s, L->K, L->kn, L->km, L->red, L->scal, L->dsflag, L->dslist, L->dscount,
               L->dscount + 1, L->pinned_dev, L->ux, L->uy, rt, L->s2, L->area);
  for (mpm_run* r : g) std::swap(r->s, r->s2);
  for (mpm_run* r : g) {
    r->eps_seq += 1;
    r->ntr += cn;
  }
  HIPCHK(L, hipGetLastError());
  HIPCHK(L, hipEventRecord(gs.ev_eps, gs.st));
  // decisions (Algorithm 1: epsilon of the previous update; text rule: of this saturation)
  const bool waited = L->P.d.switch_rule == MPM_SWITCH_TEXT;
  if (waited) {
    mpm_status e = group_wait_eps(g, gs);
    if (e) return e;
  }
  std::vector<mpm_run*> mpm, mrcm;
  for (mpm_run* r : g) {
    const double decide = waited ? eps_from(r, r->pinned[0], r->pinned[1]) : r->eps_prev;
    (decide > r->P.d.eta ? mrcm : mpm).push_back(r);
  }
  if (!mpm.empty()) {
    mpm_run* M = mpm[0];
    Runs rm;
    mpm_status et = group_tab(mpm, 1, gs.st, &rm);
    if (et) return et;
    // the ds_factor fork of the first run's update waits for the group's conductivity
    HIPCHK(M, hipEventRecord(M->ev_eps, gs.st));
    mpm_status e = mpm_update_body(M, false, rm);
    if (e) return e;
    HIPCHK(M, hipGetLastError());
    for (mpm_run* r : mpm) {
      r->eps_pending = true;
      r->last_branch = MPM_FORCE_MPM;
      r->te += 1;
    }
  }
  if (mrcm.size() > 1) {
    // the leader's second table: its own run is not in the MPM-2P subset
    Runs rr;
    mpm_status e = group_tab(mrcm, 1, gs.st, &rr);
    if (!e) e = mrcm_update_group(mrcm, rr);
    if (e) return e;
  } else if (!mrcm.empty()) {
    mpm_status e = mrcm_update(mrcm[0]);
    if (e) return e;
  }
  for (mpm_run* r : mrcm) {
    r->eps_prev = 0.0;
    r->eps_pending = false;
    r->last_branch = MPM_FORCE_MRCM;
    r->te += 1;
  }
  *updated = std::move(mpm);
  return MPM_OK;
}

// Epsilon of this step for the runs that took the MPM-2P branch (the next decision's value).
mpm_status group_finish(const std::vector<mpm_run*>& mpm, GroupStreams& gs) {
  if (mpm.empty()) return MPM_OK;
  mpm_status e = group_wait_eps(mpm, gs);
  if (e) return e;
  for (mpm_run* r : mpm) {
    r->eps_prev = eps_from(r, r->pinned[0], r->pinned[1]);
    r->eps_pending = false;
  }
  return MPM_OK;
}

}  // namespace

extern "C" {

mpm_status mpm_batch_create(int32_t capacity, mpm_batch** out) {
  if (capacity <= 0 || !out) return MPM_EINVAL;
  mpm_batch* b = new (std::nothrow) mpm_batch();
  if (!b) return MPM_ENOMEM;
  b->slot.assign(size_t(capacity), nullptr);
  *out = b;
  return MPM_OK;
}

mpm_status mpm_batch_attach(mpm_batch* b, int32_t slot, mpm_run* r) {
  if (!b || !r || slot < 0 || slot >= int32_t(b->slot.size())) return MPM_EINVAL;
  if (b->slot[slot] || r->owner) return MPM_ESTATE;
  if (!r->fields || r->poisoned || r->is_static) return MPM_ESTATE;
  b->slot[slot] = r;
  r->owner = b;
  r->owner_slot = slot;
  return MPM_OK;
}

mpm_status mpm_batch_detach(mpm_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= int32_t(b->slot.size())) return MPM_EINVAL;
  mpm_run* r = b->slot[slot];
  b->slot[slot] = nullptr;
  if (!r) return MPM_OK;
  r->owner = nullptr;
  r->owner_slot = -1;
  mpm_status e = move_run(r, nullptr);
  return e ? e : leave(r, MPM_OK);
}

mpm_status mpm_batch_step(mpm_batch* b, const uint8_t* active, uint8_t* breakthrough) {
  if (!b) return MPM_EINVAL;
  const size_t n = b->slot.size();
  std::vector<mpm_run*> run;
  for (size_t i = 0; i < n; ++i) {
    mpm_run* r = b->slot[i];
    if (!r || (active && !active[i])) continue;
    if (r->poisoned || !r->started) return MPM_ESTATE;
    run.push_back(r);
  }
  mpm_status first = MPM_OK;
  auto note = [&](mpm_run* r, mpm_status st) {
    if (st && !first) first = st;
    if (st) r->poisoned = true;
  };
  // groups in slot order, split into launches of at most MPM_GROUP_MAX runs
  std::vector<std::string> order;
  std::map<std::string, std::vector<mpm_run*>> groups;
  for (mpm_run* r : run) {
    std::string k = group_key(r);
    auto& v = groups[k];
    if (v.empty()) order.push_back(k);
    v.push_back(r);
  }
  struct Issued {
    std::vector<mpm_run*> runs, updated;
    int gs;
  };
  std::vector<Issued> issued;
  std::vector<mpm_run*> alone;
  for (const std::string& k : order) {
    std::vector<mpm_run*>& v = groups[k];
    if (v.size() < 2) {
      alone.push_back(v[0]);
      continue;
    }
    int gs = -1;
    mpm_status st = group_streams(b, k, &gs);
    if (st) {
      for (mpm_run* r : v) note(r, st);
      continue;
    }
    for (size_t a = 0; a < v.size(); a += MPM_GROUP_MAX) {
      std::vector<mpm_run*> chunk(v.begin() + a, v.begin() + std::min(v.size(), a + MPM_GROUP_MAX));
      if (chunk.size() == 1) {
        alone.push_back(chunk[0]);
        continue;
      }
      Issued is{chunk, {}, gs};
      mpm_status e = group_issue(chunk, b->gs[gs], &is.updated);
      if (e) for (mpm_run* r : chunk) note(r, e);
      else issued.push_back(std::move(is));
    }
  }
  // runs stepping alone: every run's transport and conductivity first, then (lagged rule) its
  // update, before any wait; each on its own stream
  for (mpm_run* r : alone) {
    mpm_status st = move_run(r, nullptr);
    if (!st) st = enter(r);
    if (!st) st = transport_and_kappa(r);
    if (!st && r->P.d.switch_rule == MPM_SWITCH_ALG1) st = vu_update(r, MPM_AUTO, r->eps_prev);
    note(r, st);
  }
  for (mpm_run* r : alone) {
    if (r->poisoned || r->P.d.switch_rule != MPM_SWITCH_TEXT) continue;
    double decide;
    mpm_status st = vu_decision(r, &decide);
    if (!st) st = vu_update(r, MPM_AUTO, decide);
    note(r, st);
  }
  for (Issued& is : issued) {
    mpm_status e = group_finish(is.updated, b->gs[is.gs]);
    // the water cut of runs that took the MRCM branch: wait for the group's reduction too
    if (!e && breakthrough && is.updated.size() != is.runs.size()) e = group_wait_eps(is.runs, b->gs[is.gs]);
    if (e) for (mpm_run* r : is.runs) note(r, e);
  }
  for (mpm_run* r : alone) {
    if (r->poisoned) continue;
    mpm_status e = vu_finish(r);
    if (!e && breakthrough) e = wait_eps(r);
    note(r, leave(r, e));
  }
  if (breakthrough)
    for (size_t i = 0; i < n; ++i) {
      mpm_run* r = b->slot[i];
      breakthrough[i] = (r && (!active || active[i]) && r->pinned[3] >= r->P.d.breakthrough_cut) ? 1 : 0;
    }
  return first;
}

mpm_status mpm_batch_start(mpm_batch* b) {
  if (!b) return MPM_EINVAL;
  std::vector<std::string> order;
  std::map<std::string, std::vector<mpm_run*>> groups;
  for (mpm_run* r : b->slot) {
    if (!r || r->started) continue;
    if (r->poisoned) return MPM_ESTATE;
    std::string k = group_key(r);
    auto& v = groups[k];
    if (v.empty()) order.push_back(k);
    v.push_back(r);
  }
  mpm_status first = MPM_OK;
  for (const std::string& k : order) {
    std::vector<mpm_run*>& v = groups[k];
    int gi = -1;
    mpm_status st = group_streams(b, k, &gi);
    for (size_t a = 0; !st && a < v.size(); a += MPM_GROUP_MAX) {
      std::vector<mpm_run*> g(v.begin() + a, v.begin() + std::min(v.size(), a + MPM_GROUP_MAX));
      hipStream_t s = b->gs[gi].st;
      for (mpm_run* r : g)
        if (!st) st = move_run(r, s);
      mpm_run* L = g[0];
      // Algorithm 1, initialisation, for every run of the group at once
      for (mpm_run* r : g) {
        if (st) break;
        if (hipMemsetAsync(r->scal, 0, SC_COUNT * 8, s) != hipSuccess ||
            hipMemcpyAsync(r->scal + SC_MUW, r->params, sizeof(r->params), hipMemcpyHostToDevice, s) != hipSuccess)
          st = MPM_EHIP;
      }
      Runs rt;
      if (!st) st = group_tab(g, 0, s, &rt);
      if (!st) {
        launch_kappa(s, L->g, L->s, L->K, L->kn, L->km, L->red, L->scal, L->dsflag, L->dslist, L->dscount,
                     L->dscount + 1, L->pinned_dev, nullptr, nullptr, rt);
        for (mpm_run* r : g) {
          r->eps_seq += 1;
          r->te = 0; r->tm = 0; r->ntr = 0;
        }
        st = g.size() > 1 ? mrcm_update_group(g, rt) : mrcm_update(L);
      }
      if (st) break;
      for (mpm_run* r : g) {
        r->te = 1;
        r->eps_prev = r->P.d.eta;
        r->eps_pending = false;
        r->last_branch = MPM_FORCE_MRCM;
        r->started = true;
      }
    }
    if (st) {
      if (!first) first = st;
      for (mpm_run* r : v)
        if (!r->started) r->poisoned = true;
    }
  }
  return first;
}

mpm_status mpm_batch_destroy(mpm_batch* b) {
  if (!b) return MPM_EINVAL;
  for (size_t i = 0; i < b->slot.size(); ++i)
    if (b->slot[i]) mpm_batch_detach(b, int32_t(i));
  for (GroupStreams& g : b->gs) {
    hipStreamSynchronize(g.st);
    hipStreamSynchronize(g.st2);
    hipEventDestroy(g.ev_eps);
    hipEventDestroy(g.ev_move);
    hipStreamDestroy(g.st2);
    hipStreamDestroy(g.st);
  }
  delete b;
  return MPM_OK;
}

mpm_status mpm_get_velocity(mpm_run* r, double* ux, double* uy) {
  if (!r || !ux || !uy) return MPM_EINVAL;
  if (!r->started) return MPM_ESTATE;
  mpm_status st = enter(r);
  if (st) return st;
  auto body = [&]() -> mpm_status {
    HIPCHK(r, hipMemcpyAsync(ux, r->ux, size_t(r->P.ny) * (r->P.nx + 1) * 8, hipMemcpyDeviceToDevice, r->st));
    HIPCHK(r, hipMemcpyAsync(uy, r->uy, size_t(r->P.ny + 1) * r->P.nx * 8, hipMemcpyDeviceToDevice, r->st));
    return MPM_OK;
  };
  return leave(r, body());
}

mpm_status mpm_get_saturation(mpm_run* r, double* s) {
  if (!r || !s) return MPM_EINVAL;
  if (!r->fields) return MPM_ESTATE;
  mpm_status st = enter(r);
  if (st) return st;
  auto body = [&]() -> mpm_status {
    HIPCHK(r, hipMemcpyAsync(s, r->s, size_t(r->P.ny) * r->P.nx * 8, hipMemcpyDeviceToDevice, r->st));
    return MPM_OK;
  };
  return leave(r, body());
}

mpm_status mpm_get_stats(mpm_run* r, mpm_stats* out) {
  if (!r || !out) return MPM_EINVAL;
  double sc[SC_COUNT];
  int32_t errw = 0;
  HIPCHK(r, hipMemcpyAsync(sc, r->scal, sizeof(sc), hipMemcpyDeviceToHost, r->st));
  HIPCHK(r, hipMemcpyAsync(&errw, r->err, 4, hipMemcpyDeviceToHost, r->st));
  HIPCHK(r, hipStreamSynchronize(r->st));
  if (r->prof) r->prof_collect();
  std::memset(out, 0, sizeof(*out));
  out->te = r->te;
  out->tm = r->tm;
  out->n_transport = r->ntr;
  out->eps = r->eps_prev;
  out->t = sc[SC_T];
  out->pvi = sc[SC_PVI];
  out->water_cut = sc[SC_WCUT];
  out->dt = sc[SC_DT];
  out->breakthrough = sc[SC_WCUT] >= r->P.d.breakthrough_cut ? 1 : 0;
  out->last_branch = r->last_branch;
  out->error_word = errw;
  if (errw) {
    r->poisoned = true;
    return err_status(errw);
  }
  return MPM_OK;
}

mpm_status mpm_destroy(mpm_run* r) {
  if (!r) return MPM_EINVAL;
  if (r->owner) mpm_batch_detach(r->owner, r->owner_slot);
  int32_t errw = 0;
  hipMemcpyAsync(&errw, r->err, 4, hipMemcpyDeviceToHost, r->st);
  hipStreamSynchronize(r->st);
  for (auto& p : r->pending) { hipEventDestroy(p.second.first); hipEventDestroy(p.second.second); }
  for (auto e : r->pool) hipEventDestroy(e);
  for (auto& gx : r->g_trans)
    if (gx) hipGraphExecDestroy(gx);
  if (r->g_mpm) hipGraphExecDestroy(r->g_mpm);
  if (r->ev_in) hipEventDestroy(r->ev_in);
  if (r->ev_out) hipEventDestroy(r->ev_out);
  if (r->ev_eps) hipEventDestroy(r->ev_eps);
  if (r->ev_fork) hipEventDestroy(r->ev_fork);
  if (r->ev_join) hipEventDestroy(r->ev_join);
  if (r->st2 && r->st2 != r->ust) { hipStreamSynchronize(r->st2); hipStreamDestroy(r->st2); }
  if (r->st && r->st != r->ust) hipStreamDestroy(r->st);
  if (r->pinned && !r->is_static) hipHostFree(r->pinned);
  const bool was_static = r->is_static;
  const int device = r->device;
  delete r;
  if (was_static) release_static(device);
  return errw ? err_status(errw) : MPM_OK;
}

mpm_status mpm_plan_solve_bytes(const mpm_run* r, int64_t* fwd, int64_t* bwd, int64_t* front) {
  if (!r) return MPM_EINVAL;
  int64_t f = 0, b = 0;
  for (const NodeDev& n : r->P.nodes) {
    f += int64_t(n.nB) * n.nI * 8;
    b += int64_t(n.nI) * n.n * 8;
  }
  if (fwd) *fwd = f;
  if (bwd) *bwd = b;
  if (front) *front = r->P.front_doubles * 8;
  return MPM_OK;
}

mpm_status mpm_plan_fused_bytes(const mpm_run* r, int32_t* levels, int64_t* fwd, int64_t* bwd) {
  if (!r) return MPM_EINVAL;
  int64_t f = 0, b = 0;
  for (const FuseNode& x : r->P.fnodes) {
    f += int64_t(x.nd.nB) * x.nd.nI * 8;
    b += int64_t(x.nd.nI) * x.nd.n * 8;
  }
  if (levels) *levels = r->P.fuse_h;
  if (fwd) *fwd = f;
  if (bwd) *bwd = b;
  return MPM_OK;
}

mpm_status mpm_plan_info(const mpm_run* r, int64_t* n_sub, int64_t* n_iface, int64_t* n_nodes, int64_t* n_levels) {
  if (!r) return MPM_EINVAL;
  if (n_sub) *n_sub = r->P.nsub;
  if (n_iface) *n_iface = r->P.n_iface;
  if (n_nodes) *n_nodes = int64_t(r->P.nodes.size());
  if (n_levels) *n_levels = int64_t(r->P.level_nodes.size()) - 1;
  return MPM_OK;
}

// Autotuner of the interface sweeps: for each level of the forward, then of the backward sweep,
// every admissible launch shape is timed over complete interface solves (the other levels at
// their current choice; best of `reps`), and the fastest kept. The solves repeat the last one
// (idempotent: each level writes what only the levels after it read).
mpm_status mpm_tune(mpm_run* r, int32_t reps, int32_t cap, int32_t* shapes, int32_t* n, double* ms_rule,
                    double* ms_tuned) {
  if (!r || reps < 1 || cap < 0 || (cap > 0 && !shapes)) return MPM_EINVAL;
  if (!r->started || r->poisoned || r->owner) return MPM_ESTATE;
  mpm_status st = enter(r);
  if (st) return st;
  const Plan& P = r->P;
  const int L = int(P.level_nodes.size()) - 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool prof = r->prof;   // the trial solves stay out of the kernel profile
  r->prof = false;
  auto body = [&]() -> mpm_status {
    HIPCHK(r, hipEventCreate(&e0));
    HIPCHK(r, hipEventCreate(&e1));
    auto time_solve = [&](double* best) -> mpm_status {
      *best = 1e300;
      for (int k = 0; k < reps + 1; ++k) {   // the first solve warms up
        HIPCHK(r, hipEventRecord(e0, r->st));
        nd_solve(r);
        HIPCHK(r, hipEventRecord(e1, r->st));
        HIPCHK(r, hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(r, hipEventElapsedTime(&ms, e0, e1));
        if (k > 0) *best = std::min(*best, double(ms));
      }
      return MPM_OK;
    };
    r->tune_fwd.assign(std::max(L + 1, 1), 0);
    r->tune_bwd.assign(std::max(L + 1, 1), 0);
    const bool fuse_rule = P.fuse_h > 0 && fuse_default();
    r->fuse = fuse_rule;
    double t_rule = 0.0, t = 0.0;
    mpm_status s2 = time_solve(&t_rule);
    if (s2) return s2;
    double cur = t_rule;
    if (P.fuse_h > 0) {   // the fused bottom levels against one launch per level
      r->fuse = !fuse_rule;
      s2 = time_solve(&t);
      if (s2) return s2;
      if (t < 0.99 * cur) {   // confirmed as the shapes below
        double tc = 0.0, tb = 0.0;
        s2 = time_solve(&tc);
        if (s2) return s2;
        r->fuse = fuse_rule;
        s2 = time_solve(&tb);
        if (s2) return s2;
        if (std::min(t, tc) < 0.99 * std::min(cur, tb)) {
          cur = std::min(t, tc);
          r->fuse = !fuse_rule;
        } else {
          cur = std::min(cur, tb);
        }
      } else {
        r->fuse = fuse_rule;
      }
    }
    const int H = r->fuse ? P.fuse_h : 0;
    for (int dir = 0; dir < 2; ++dir) {
      std::vector<int>& tab = dir == 0 ? r->tune_fwd : r->tune_bwd;
      for (int l = H + 1; l <= L; ++l) {
        if (P.level_nodes[l].empty() || (dir == 0 && l == L)) continue;   // the root has no forward step
        const int len = dir == 0 ? P.level_nImax[l] : P.level_nmax[l];
        const int rows = dir == 0 ? P.level_nBmax[l] : P.level_nImax[l];
        int codes[32];
        const int nc = nd_shape_candidates(len, rows, dir == 1, codes, 32);
        int best = tab[l];
        for (int c = 1; c < nc; ++c) {   // codes[0] is the rule
          tab[l] = codes[c];
          s2 = time_solve(&t);
          if (s2) return s2;
          if (t < 0.99 * cur) {
            // confirmed against the current choice timed again (a single timing of a solve
            // moves by about a percent)
            double tc = 0.0, tb = 0.0;
            s2 = time_solve(&tc);
            if (s2) return s2;
            tab[l] = best;
            s2 = time_solve(&tb);
            if (s2) return s2;
            if (std::min(t, tc) < 0.99 * std::min(cur, tb)) {
              cur = std::min(t, tc);
              best = codes[c];
            } else {
              cur = std::min(cur, tb);
            }
          }
        }
        tab[l] = best;
      }
    }
    s2 = time_solve(&t);
    if (s2) return s2;
    if (t > t_rule) {   // keep the rule if the choice does not hold up
      std::fill(r->tune_fwd.begin(), r->tune_fwd.end(), 0);
      std::fill(r->tune_bwd.begin(), r->tune_bwd.end(), 0);
      r->fuse = fuse_rule;
      t = t_rule;
    }
    if (ms_rule) *ms_rule = t_rule;
    if (ms_tuned) *ms_tuned = t;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[tune_key(P.d)] = TuneChoice{r->tune_fwd, r->tune_bwd, r->fuse};
    }
    // the chosen shape of every launch, forward levels upwards then backward levels downwards
    int32_t k = 0;
    auto put = [&](int code, int len, int rows, bool bwd) {
      int G, U, RP;
      if (code == 0) {
        int c0[1];
        nd_shape_candidates(len, rows, bwd, c0, 1);
        code = c0[0];
      }
      nd_shape_unpack(code, &G, &U, &RP);
      if (3 * k + 2 < cap) {
        shapes[3 * k] = G;
        shapes[3 * k + 1] = U;
        shapes[3 * k + 2] = RP;
      }
      ++k;
    };
    auto put_fused = [&]() {   // the fused bottom levels: (0, their number, 0)
      if (3 * k + 2 < cap) {
        shapes[3 * k] = 0;
        shapes[3 * k + 1] = P.fuse_h;
        shapes[3 * k + 2] = 0;
      }
      ++k;
    };
    const int Hf = r->fuse ? P.fuse_h : 0;
    if (Hf) put_fused();
    for (int l = Hf + 1; l < L; ++l)
      if (!P.level_nodes[l].empty()) put(r->tune_fwd[l], P.level_nImax[l], P.level_nBmax[l], false);
    for (int l = L; l > Hf; --l)
      if (!P.level_nodes[l].empty()) put(r->tune_bwd[l], P.level_nmax[l], P.level_nImax[l], true);
    if (Hf) put_fused();
    if (n) *n = k;
    return MPM_OK;
  };
  st = body();
  r->prof = prof;
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  return leave(r, st);
}

mpm_status mpm_profile(mpm_run* r, int32_t enable, int32_t reset, int32_t cap, const char** names, double* ms,
                       int64_t* count, int32_t* n) {
  if (!r) return MPM_EINVAL;
  HIPCHK(r, hipStreamSynchronize(r->st));
  r->prof_collect();
  int k = 0;
  for (auto& e : r->prof_acc) {
    if (k >= cap) break;
    if (names) names[k] = e.second.name;
    if (ms) ms[k] = e.second.count ? e.second.ms / e.second.count : 0.0;
    if (count) count[k] = e.second.count;
    ++k;
  }
  if (n) *n = k;
  if (reset) r->prof_acc.clear();
  r->prof = enable != 0;
  r->prof_fine = enable == 2;
  return MPM_OK;
}

}  // extern "C"
