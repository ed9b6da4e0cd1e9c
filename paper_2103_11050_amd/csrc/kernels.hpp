// Launchers of the HIP kernels (host side), grouped by file.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace mpm {

// local.hip
void launch_kappa(hipStream_t st, const Geo& g, const double* s, const double* K, double* kn, const double* km,
                  double* red, double* scal, int32_t* flag, int32_t* list, int32_t* count);
void launch_dt(hipStream_t st, int nsub, const double* red_rate, const double* red_qin, double cfl,
               double fmax_deriv, double* scal, int32_t* count);

// basis.hip: returns whether the kappa^m line-block inverses were written as well
bool launch_basis(hipStream_t st, const Geo& g, const double* kap, const double* q, double* S, double* h,
                  double* leafK, double* leafr, double* fac, int32_t* err);
// lines.hip
void launch_line_factor(hipStream_t st, const Geo& g, const double* kap, double* fac, int32_t* err);
size_t line_factor_doubles(int nsub, int nc, int band);
void launch_mpm_local(hipStream_t st, const Geo& g, const double* kn, const double* km, const double* uxm,
                      const double* uym, const double* q, const double* fac, double* h, double* vbnd,
                      double* leafr);
void launch_flux(hipStream_t st, const Geo& g, const double* km, const double* S, const double* h,
                 const double* vbnd, const double* y, const int32_t* sub_dofs, double* ubnd, int with_v);
// Neumann inverse blocks of kappa^n for the subdomains whose conductivity tile differs from
// kappa^m (into Escr, flag[sub] = 1), flag[sub] = 0 elsewhere.
void launch_ds_factor(hipStream_t st, const Geo& g, const double* kap_n, double* Escr, const int32_t* list,
                      const int32_t* count, int32_t* err);
// store = 1: kap_s is kappa^m, its inverse blocks are formed here and kept (Ekeep).
// store = 0: the blocks come from Escr where flag[sub] is set, else from Ekeep.
void launch_downscale(hipStream_t st, const Geo& g, const double* kap_s, const double* q, const double* ubnd,
                      double* ux, double* uy, double* red_rate, double* red_qin, double* Escr, double* Ekeep,
                      const int32_t* flag, int store, int32_t* err);

// nd.hip: nested-dissection factorisation and solve of the interface system
struct NdArgs {
  const NodeDev* nodes;
  const int32_t* levels;      // concatenated node lists per level
  const int32_t* dof_pool;
  const int32_t* map_pool;
  const int32_t* inv_pool;
  double* front;
  double* fI;
  double* cB;
  double* panel;
  double* leafK;
  double* leafr;
  double* y;
  int ndmax;
  int piv_b;
  int32_t* err;
  const int32_t* fuse_off;    // subtree offsets into fuse_nodes (bottom levels)
  const int32_t* fuse_nodes;  // subtree nodes, children before parents
};
void launch_nd_level_factor(hipStream_t st, const NdArgs& a, int level_off, int nnodes, int nmax, int nImax);
void launch_nd_level_fwd(hipStream_t st, const NdArgs& a, int level_off, int nnodes, int nmax, int nImax, int nBmax);
void launch_nd_level_bwd(hipStream_t st, const NdArgs& a, int level_off, int nnodes, int nImax, int nmax);
void launch_nd_fused_fwd(hipStream_t st, const NdArgs& a, int nroots, int nmax);
void launch_nd_fused_bwd(hipStream_t st, const NdArgs& a, int nroots, int nmax);

// transport.hip
void launch_sat_step(hipStream_t st, const Geo& g, const double* s, double* s2, const double* ux,
                     const double* uy, double* scal, double M, double area);
void launch_water_cut(hipStream_t st, const Geo& g, const double* s, const double* ux, const double* uy,
                      double* scal, double M);

}  // namespace mpm
