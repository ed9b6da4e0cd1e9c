// Host-side plan of a run: decomposition, interface unknowns, nested-dissection tree of the
// interface system and the layout of every buffer inside the caller's workspace.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "mpm2p.h"

namespace mpm {

// Boundary-face kinds of a subdomain's faces (all faces of the subdomain boundary).
enum FaceKind : int32_t { FACE_NEU = 0, FACE_DIR = 1, FACE_ROB = 2 };

// Device view of one nested-dissection node.
//
// The forward solve passes vectors between levels through slots rather than by gathering: a
// node writes its condensed right-hand side into its parent's slot for it (front order, two
// slots per node, one per child; entries the child does not reach stay zero).
struct NodeDev {
  int32_t n, nI, nB;          // front size, eliminated (separator) and boundary unknowns
  int32_t level;
  int32_t child[2];           // node ids, or -1-sub for a leaf child (subdomain id)
  int32_t map_off[2];         // offsets of the children's extend-add maps into map_pool
  int32_t nB_child[2];        // boundary sizes of the children
  int32_t dof_off;            // offset of the node's front unknowns (I then B) in dof_pool
  int32_t inv_off;            // offset of the inverse extend-add maps in inv_pool: for child c and
                              // front index k, inv_pool[inv_off + c*n + k] = the child's index, or -1
  int32_t up_map_off;         // offset in map_pool of this node's B entries in its parent's front
  int32_t pad;
  int64_t front_off;          // offset (doubles) of the n x n front
  int64_t fI_off;             // offset (doubles) of the eliminated part of the condensed rhs
  int64_t panel_off;          // offset (doubles) of the pivot-block scratch (b*b + 2*b*n), then
                              // of T = F_II^-1 F_IB (nI*nB)
  int64_t slot_off;           // offset (doubles) of the node's two child slots (2 x n)
  int64_t up_slot_off;        // offset of the parent's slot this node writes into (-1: root)
};

// Where a subdomain's interface right-hand side goes: the slot of its parent node and the map
// of its unknowns into the parent's front (slot -1: no tree).
struct LeafUp {
  int64_t slot_off;
  int32_t map_off;
  int32_t pad;
};

// The bottom levels of both sweeps can run as one launch per direction, one workgroup per
// subtree (a node of level <= H whose parent lies above H, with its descendants), the vectors
// that pass between the subtree's levels kept in LDS. Per subtree and level at most FUSE_MAXN
// nodes, forward rows (nI entries) at most FUSE_FWD_NI long, backward rows (n entries) at most
// FUSE_BWD_N long, the front vectors of a level at most FUSE_VEC entries together, its rows at
// most FUSE_ROWS in either direction and its forward work items (a column pair of IB over eight
// of its rows) at most FUSE_ITEMS; over the subtree's levels at most FUSE_SUBVEC front vector
// entries, FUSE_XB boundary entries and FUSE_XRES separator unknowns.
constexpr int FUSE_HMAX = 4, FUSE_MAXN = 8;
constexpr int FUSE_FWD_NI = 64, FUSE_BWD_N = 512, FUSE_VEC = 1024, FUSE_ROWS = 1024;
constexpr int FUSE_XB = 2048, FUSE_XRES = 1024, FUSE_SUBVEC = 4096, FUSE_ITEMS = 1024;
// The fused backward sweep also reconstructs the boundary fluxes of its subtree's subdomains,
// one wavefront each, where every subdomain is a leaf of a fused subtree (at most FUSE_LEAVES per
// subtree) and has at most 64 boundary faces.
constexpr int FUSE_LEAVES = 16;

// A node of a fused subtree with its place in its level's lists: the rows and vector entries of
// the level's nodes before it, forward (nB rows, nI entries) and backward (nI rows, n entries:
// also its place among the level's front vectors); pv = the place of its parent's front vector in
// the subtree's list of them (-1: the parent lies outside the subtree); fc = the forward work
// items of the level's nodes before it (nB / 2 column pairs times ceil(nI / 8) row chunks each).
struct FuseNode {
  NodeDev nd;
  int32_t fr, fv, br, bv, pv, fc;
};
// One level of a fused subtree: nodes fnodes[b .. e), their totals (fC: forward work items), the
// column chunks of the longest backward row (chunks of 64 entries); xc = offset of the level's x_B
// sources in fxsrc, xo = their place in the subtree's list, xr = the place of the level's
// separator unknowns in the subtree's list of them, vb = the place of the level's front vectors
// in the subtree's list of them.
struct FuseLevel {
  int32_t b, e;
  int32_t fR, fV, bR, bV;
  int32_t fC, bch;
  int32_t xc, xo, xr, vb;
};

// Runs of one batch that share their decomposition step through one launch per phase:
// blockIdx.z selects the run, whose workspace (and pinned host block) sits at a byte offset
// from the first run's; the launch carries the first run's pointers and this table, which
// lives in the first run's workspace.
constexpr int MPM_GROUP_MAX = 128;
struct RunTab {
  int64_t ws[MPM_GROUP_MAX];
  int64_t host[MPM_GROUP_MAX];
};

struct Plan {
  mpm_desc d;
  int nx, ny, mx, my, Sx, Sy, nsub;
  double hx, hy;
  int ne_x, ne_y;
  int n_vert, n_horiz, n_elem, n_iface;
  int npol;                   // interface functions per element and field (iface_degree + 1)
  int nc;                     // cells per subdomain
  int band;                   // half bandwidth of the local matrices = min(mx, my)
  int xfast;                  // 1: local cell order has x fastest (band = mx)
  int nb;                     // boundary faces per subdomain = 2 (mx + my)
  int ndmax;                  // max interface unknowns of a subdomain
  // per subdomain
  std::vector<int32_t> sub_ndof;      // interface unknowns
  std::vector<int32_t> sub_dofs;      // nsub * ndmax global unknown ids (local order), -1 pad
  // nested dissection
  std::vector<NodeDev> nodes;         // bottom-up; leaves are not nodes
  std::vector<std::vector<int32_t>> level_nodes;  // level 1.. -> node ids
  std::vector<int32_t> dof_pool;
  std::vector<int32_t> map_pool;
  std::vector<int32_t> inv_pool;
  int root = -1;
  int piv_b = 32;                     // pivot block of the blocked sweep
  std::vector<int32_t> level_nmax, level_nImax, level_nBmax;
  // workspace layout (byte offsets)
  size_t off_K, off_q, off_s, off_s2, off_kn, off_km, off_ux, off_uy, off_uxm, off_uym;
  size_t off_fac, off_dinv, off_S, off_h, off_vbnd, off_ubnd, off_leafK;
  size_t off_front, off_fI, off_panel, off_y;
  size_t off_invpool = 0;
  size_t off_nodes, off_dofpool, off_mappool, off_subdofs, off_subndof, off_levels;
  std::vector<int32_t> level_off;     // offsets of each level's node list in the uploaded level array
  std::vector<int32_t> level_flat;
  std::vector<NodeDev> lnodes;        // the nodes again, level by level (level_flat order)
  std::vector<LeafUp> leafup;         // per subdomain
  // fused bottom levels (fuse_h = 0: none): level h (1..fuse_h) of subtree t is
  // flevels[t fuse_h + h - 1]; a subtree's nodes are contiguous in fnodes, level by level
  int fuse_h = 0, fuse_roots = 0;
  std::vector<FuseLevel> flevels;
  std::vector<FuseNode> fnodes;
  // per fused node and boundary entry, in row order: where the backward sweep finds x_B: >= 0,
  // the subtree's separator unknown of that place; < 0, -1 - its unknown id (outside the subtree)
  std::vector<int32_t> fxsrc;
  bool fuse_flux = false;             // the fused backward sweep reconstructs the fluxes too
  std::vector<int32_t> fleaves;       // per subtree FUSE_LEAVES subdomain ids (-1 past its leaves)
  size_t off_fnodes = 0, off_flevels = 0, off_fxsrc = 0, off_fleaves = 0;
  size_t off_lnodes = 0, off_leafup = 0, off_slot = 0;
  size_t off_dsE = 0, off_nfac = 0;   // downscale inverse blocks: scratch and the kept kappa^m ones
  size_t n_blocks = 0;                // entries of one block set (kept kappa^m Robin, Neumann, scratch)
  size_t off_fac32 = 0, off_nfac32 = 0, off_dsE32 = 0;   // their FP32 copies (precision form only)
  size_t off_dsflag = 0;              // per subdomain: conductivity changed since the last update
  size_t off_dslist = 0;              // the changed subdomains (count in the integer word after the error word)
  size_t off_red, off_scal;
  size_t off_rtab = 0;                // two run tables (batch groups led by this run)
  size_t off_wbnd = 0;                // first-order term: w on the subdomains' boundary faces
  size_t n_red;               // doubles in the reduction scratch
  size_t total_bytes;
  int64_t front_doubles = 0, panel_doubles = 0, fI_doubles = 0, slot_doubles = 0;
};

// Validates the descriptor; returns MPM_OK or MPM_EINVAL with a message.
mpm_status validate(const mpm_desc& d, std::string* why);
// Builds the plan (decomposition, tree, layout). Assumes validate() passed.
void build_plan(const mpm_desc& d, Plan* p);

// Scalars kept on the device (indices into the scalar block of the workspace).
enum Scalar : int {
  SC_EPS_NUM = 0,   // sum (kappa^n - kappa^m)^2
  SC_EPS_DEN,       // sum (kappa^m)^2
  SC_DT,            // transport sub-step
  SC_QIN,           // boundary inflow
  SC_T,             // simulated time
  SC_PVI,
  SC_WCUT,
  SC_MAXRATE,
  // per-run physics read by the kernels (set by mpm_start), so that runs of one batch group
  // may differ in them
  SC_MUW,           // water viscosity
  SC_MUO,           // oil viscosity
  SC_MRATIO,        // M = mu_o / mu_w
  SC_CFL,           // fraction of the monotone time-step bound
  SC_FMAX,          // max over [0, 1] of the fractional-flow derivative
  SC_COUNT = 16
};

}  // namespace mpm
