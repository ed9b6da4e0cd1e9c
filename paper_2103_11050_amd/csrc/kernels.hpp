// Launchers of the HIP kernels (host side), grouped by file.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace mpm {

// The runs of a launch: n runs (grid z) with the table of their offsets in device memory, or
// one run and no table.
struct Runs {
  const RunTab* tab;
  unsigned n;
};
inline Runs one_run() { return Runs{nullptr, 1u}; }
inline unsigned runs_of(const Runs& rs) { return rs.n; }

// Byte offsets of the workspace and of the pinned block of the run of this workgroup (grid z)
// from the first run's.
__device__ __forceinline__ int64_t ws_off(const RunTab* rt) { return rt ? rt->ws[blockIdx.z] : 0; }
__device__ __forceinline__ int64_t host_off(const RunTab* rt) { return rt ? rt->host[blockIdx.z] : 0; }

// Destination of a subdomain's interface right-hand side B^T h: the slot of its parent in the
// nested-dissection tree (entry map_pool[up.map_off + a] for local unknown a).
struct LeafOut {
  double* slots;
  const LeafUp* up;
  const int32_t* map_pool;
};
__device__ __forceinline__ LeafOut leaf_at(const LeafOut& lo, int64_t o) {
  return LeafOut{at_off(lo.slots, o), at_off(lo.up, o), at_off(lo.map_pool, o)};
}
__device__ __forceinline__ void leaf_out(const LeafOut& lo, int sub, int a, double v) {
  const LeafUp u = lo.up[sub];
  if (u.slot_off >= 0) lo.slots[u.slot_off + lo.map_pool[u.map_off + a]] = v;
}

// Every launcher that takes Runs runs the kernel for rt.n runs at once (grid z), with the
// pointers of the first run; by default for one run.

// local.hip
// With wc_ux non-null the reduction also computes the water cut under (wc_ux, wc_uy); with
// s_new non-null (which needs wc_ux) the kernel first takes a transport sub-step from s into
// s_new under that velocity and works on the new saturation. With st_red the reduction kernel
// goes to that stream, ordered after the tile kernel through ev_red.
void launch_kappa(hipStream_t st, const Geo& g, const double* s, const double* K, double* kn, const double* km,
                  double* red, double* scal, int32_t* flag, int32_t* list, int32_t* count, int32_t* seq,
                  double* host, const double* wc_ux, const double* wc_uy, Runs rt = one_run(),
                  double* s_new = nullptr, double area = 0.0, hipStream_t st_red = nullptr,
                  hipEvent_t ev_red = nullptr);
// the sub-step bound uses the run's cfl and fractional-flow derivative bound from scal
void launch_dt(hipStream_t st, int nsub, const double* red_rate, const double* red_qin, double* scal,
               int32_t* count, Runs rt = one_run());

// basis.hip: returns whether the kappa^m line-block inverses were written as well
bool launch_basis(hipStream_t st, const Geo& g, const double* kap, const double* q, double* S, double* h,
                  double* leafK, LeafOut lo, double* fac, int32_t* err, Runs rt = one_run());
// lines.hip
// The same basis for subdomains of more than 16 lines, by one line-block solve per boundary
// face; always writes the inverse blocks.
void launch_basis_lines(hipStream_t st, const Geo& g, const double* kap, const double* q, double* S, double* h,
                        double* leafK, LeafOut lo, double* fac, int32_t* err, Runs rt = one_run());
void launch_line_factor(hipStream_t st, const Geo& g, const double* kap, double* fac, int32_t* err,
                        Runs rt = one_run());
size_t line_factor_doubles(int nsub, int nc, int band);
void launch_mpm_local(hipStream_t st, const Geo& g, const double* kn, const double* km, const double* uxm,
                      const double* uym, const double* q, const double* fac, double* h, double* vbnd,
                      LeafOut lo, int32_t* err, Runs rt = one_run());
// with_v: 0 u-hat only, 1 u-hat + v, 2 ubnd += u-hat + v (first-order term)
void launch_flux(hipStream_t st, const Geo& g, const double* km, const double* S, const double* h,
                 const double* vbnd, const double* y, const int32_t* sub_dofs, double* ubnd, int with_v,
                 Runs rt = one_run());
// first-order term of MPM-2P after the zeroth-order interface solve and reconstruction: boundary
// fluxes h and interface right-hand side of its trivial-Robin problem, w on the boundary faces
void launch_mpm_first(hipStream_t st, const Geo& g, const double* kn, const double* km, const double* uxm,
                      const double* uym, const double* q, const double* fac, const double* y,
                      const int32_t* sub_dofs, const double* ubnd, const double* vbnd, double* h, double* wbnd,
                      LeafOut lo, Runs rt = one_run());
// Neumann inverse blocks of kappa^n for the subdomains whose conductivity tile differs from
// kappa^m (into Escr, flag[sub] = 1), flag[sub] = 0 elsewhere.
void launch_ds_factor(hipStream_t st, const Geo& g, const double* kap_n, double* Escr, const int32_t* list,
                      const int32_t* count, int32_t* err, Runs rt = one_run());
// store = 1: kap_s is kappa^m, its inverse blocks are formed here and kept (Ekeep).
// store = 0: the blocks come from Escr where flag[sub] is set, else from Ekeep.
// precision form: FP32 inverse blocks, FP64 refinement (MPM-2P steps), and the conversion of
// FP64 blocks kept by an MRCM update
void launch_ds_factor_f32(hipStream_t st, const Geo& g, const double* kap_n, float* Escr, const int32_t* list,
                          const int32_t* count, int32_t* err, Runs rt = one_run());
void launch_mpm_local_f32(hipStream_t st, const Geo& g, const double* kn, const double* km, const double* uxm,
                          const double* uym, const double* q, const float* fac, double* h, double* vbnd,
                          LeafOut lo, int32_t* err, Runs rt = one_run());
void launch_downscale_f32(hipStream_t st, const Geo& g, const double* kap_s, const double* q, const double* ubnd,
                          double* ux, double* uy, double* red_rate, double* red_qin, float* Escr, float* Ekeep,
                          const int32_t* flag, int32_t* err, Runs rt = one_run());
void launch_to_f32(hipStream_t st, size_t n, const double* src, float* dst, Runs rt = one_run());
void launch_downscale(hipStream_t st, const Geo& g, const double* kap_s, const double* q, const double* ubnd,
                      double* ux, double* uy, double* red_rate, double* red_qin, double* Escr, double* Ekeep,
                      const int32_t* flag, int store, int32_t* err, Runs rt = one_run());

// nd.hip: nested-dissection factorisation and solve of the interface system
struct NdArgs {
  const NodeDev* nodes;
  const NodeDev* lnodes;      // the nodes level by level (indexed by level offset + node)
  const int32_t* levels;      // concatenated node lists per level
  const int32_t* dof_pool;
  const int32_t* map_pool;
  const int32_t* inv_pool;
  double* front;
  double* fI;
  double* slots;
  double* panel;
  double* leafK;
  double* y;
  int ndmax;
  int piv_b;
  int32_t* err;
  const FuseNode* fnodes;     // fused bottom levels: the nodes subtree by subtree, level by level
  const FuseLevel* flevels;   // subtree t, level h (1..H): flevels[t H + h - 1]
  const int32_t* fxsrc;       // where the backward sweep finds each fused node's x_B entries
  int fuse_h;                 // H (0: no fused levels)
};
// The same arguments for a workspace at byte offset o.
__device__ __forceinline__ NdArgs nd_at(const NdArgs& a, int64_t o) {
  NdArgs b = a;
  b.nodes = at_off(a.nodes, o);
  b.lnodes = at_off(a.lnodes, o);
  b.levels = at_off(a.levels, o);
  b.dof_pool = at_off(a.dof_pool, o);
  b.map_pool = at_off(a.map_pool, o);
  b.inv_pool = at_off(a.inv_pool, o);
  b.front = at_off(a.front, o);
  b.fI = at_off(a.fI, o);
  b.slots = at_off(a.slots, o);
  b.panel = at_off(a.panel, o);
  b.leafK = at_off(a.leafK, o);
  b.y = at_off(a.y, o);
  b.err = at_off(a.err, o);
  b.fnodes = at_off(a.fnodes, o);
  b.flevels = at_off(a.flevels, o);
  b.fxsrc = at_off(a.fxsrc, o);
  return b;
}
void launch_nd_level_factor(hipStream_t st, const NdArgs& a, int level_off, int nnodes, int nmax, int nImax,
                            int nBmax, Runs rt = one_run());
// Launch shape of a sweep level: lanes per row G, column pairs per lane U, rows per lane group RP,
// packed as G | U << 8 | RP << 16; 0 selects the fixed rule (rows of 1536 or more are taken in
// chunks whatever the code).
int nd_shape_code(int G, int U, int RP);
void nd_shape_unpack(int code, int* G, int* U, int* RP);
// The shapes a level whose rows hold len entries can be launched with (the rule's first), and
// the rule's shape; returns how many were written (at most cap).
int nd_shape_candidates(int len, int rows, bool bwd, int* codes, int cap);
void launch_nd_level_fwd(hipStream_t st, const NdArgs& a, int level_off, int nnodes, int nImax, int nBmax,
                         Runs rt = one_run(), int shape = 0);
void launch_nd_level_bwd(hipStream_t st, const NdArgs& a, int level_off, int nnodes, int nImax, int nmax, int root,
                         Runs rt = one_run(), int shape = 0);
// The reconstruction (flux_sub) done by the fused backward sweep for its subtrees' subdomains,
// leaves[t FUSE_LEAVES + w] for wavefront w of subtree t (-1: none).
struct FluxArgs {
  Geo g;
  const double* km;
  const double* S;
  const double* h;
  const double* vbnd;
  const int32_t* sub_dofs;
  double* ubnd;
  const int32_t* leaves;
  int with_v;
};
// The fused bottom levels (a.fuse_h of them) of the forward and of the backward sweep: one
// workgroup per subtree; with fa, the backward sweep then reconstructs the fluxes.
void launch_nd_sub_fwd(hipStream_t st, const NdArgs& a, int nsubtrees, Runs rt = one_run());
void launch_nd_sub_bwd(hipStream_t st, const NdArgs& a, int nsubtrees, Runs rt = one_run(),
                       const FluxArgs* fa = nullptr);

// transport.hip
// (the viscosity ratio M is the run's, from scal)
void launch_sat_step(hipStream_t st, const Geo& g, const double* s, double* s2, const double* ux,
                     const double* uy, double* scal, double area, Runs rt = one_run());
// part: 2 x 64 doubles of scratch; ticket: a zeroed counter (left at zero)
void launch_water_cut(hipStream_t st, const Geo& g, const double* s, const double* ux, const double* uy,
                      double* scal, double* part, int32_t* ticket, Runs rt = one_run());

}  // namespace mpm
