// Register-resident line-block factorisation of a subdomain's two-point flux matrix.
//
// With cells numbered line by line (a line runs along the shorter side of the subdomain), the
// 5-point matrix is block tridiagonal: diagonal blocks T_j are tridiagonal (couplings inside
// line j) and the off-diagonal blocks are -Y_j with Y_j diagonal (couplings between lines j
// and j+1). Block elimination gives
//   D_0 = T_0,   D_j = T_j - Y_{j-1} D_{j-1}^-1 Y_{j-1},
// and the solve
//   z_0 = r_0,  w_j = D_j^-1 z_j,  z_{j+1} = r_{j+1} + Y_j w_j,
//   x_last = w_last,  x_j = w_j + D_j^-1 (Y_j x_{j+1}).
// One wavefront owns one subdomain. Each D_j^-1 (MF x MF, lines padded with identity rows to
// MF in {8, 16}) is spread over the 64 lanes, EPL entries per lane: lane -> (row, column
// group). Inversion is a Gauss-Jordan sweep with the pivot row and column broadcast by lane
// shuffles; the SPD pivots need no pivoting.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace mpm {

// A block spread over NT lanes (one wavefront, or NT / 64 wavefronts of one workgroup):
// IL = false: lane (row, cg) holds columns cg*EPL + t (contiguous groups);
// IL = true : lane (row, cg) holds columns cg + LPR*t (interleaved), the layout whose entry t
//             is the matrix-core operand of the t-th K-chunk.
template <int MF, bool IL = false, int NT = 64>
struct LB {
  static constexpr int EPL = MF * MF / NT;   // entries per lane
  static constexpr int LPR = MF / EPL;       // lanes per row
  static_assert(EPL >= 1 && LPR * EPL == MF, "block layout");
  int lane, row, cg;
  __device__ LB() {
    lane = threadIdx.x & (NT - 1);
    row = lane / LPR;
    cg = lane % LPR;
  }
  __device__ int col(int t) const { return IL ? cg + LPR * t : cg * EPL + t; }
};

// Capacity of the per-subdomain LDS tiles and per-lane cell arrays of a kernel whose lines are
// padded to MF cells: subdomains of at most S x S cells (16 for MF <= 16, 32 for MF = 32), one
// wavefront of 64 lanes, CPL cells per lane, NB boundary faces, NF faces of one direction and a
// one-cell halo tile of HALO cells.
template <int MF>
struct Cap {
  static constexpr int S = MF == 32 ? 32 : 16;
  static constexpr int NC = S * S;
  static constexpr int CPL = NC / 64;
  static constexpr int NB = 4 * S;
  static constexpr int NF = S * (S + 1);
  static constexpr int HALO = (S + 2) * (S + 2);
};

// Kept line-block inverses are symmetric: each MF x MF block is stored as its upper triangle,
// row by row (MF (MF + 1) / 2 entries); entry (row, col) of the block sits at lb_pk(min, max).
template <int MF>
struct LBP {
  static constexpr int P = MF * (MF + 1) / 2;
};
template <int MF>
__device__ __forceinline__ int lb_pk(int row, int col) {
  const int r = row < col ? row : col, c = row < col ? col : row;
  return r * MF - (r * (r - 1)) / 2 + (c - r);
}

// In-place inverse of the SPD block held as a[t] = D[row][col(t)]. Clears ok on a
// non-positive pivot. The pivot loop runs in groups of EPL so that the register holding
// column k is known at compile time. At each pivot the lanes of row k write that row, and the
// lanes holding column k write that column, into LDS, from which every lane reads the entries
// it needs; the same values, and the same arithmetic, as fetching them from the owning lanes by
// shuffles. piv holds 4 MF doubles: row and column of even pivots, then of odd pivots (two
// buffers, so one synchronisation per pivot: a wavefront-scope fence for one wavefront, whose
// lanes see each other's LDS writes in program order, a workgroup barrier for several).
template <int MF, int NT = 64>
__device__ __forceinline__ void lb_inverse(const LB<MF, false, NT>& L, double (&a)[LB<MF, false, NT>::EPL], bool& ok,
                                           double* piv) {
  constexpr int EPL = LB<MF, false, NT>::EPL;
#pragma unroll 1
  for (int k0 = 0; k0 < MF; k0 += EPL) {
#pragma unroll
    for (int kk = 0; kk < EPL; ++kk) {
      const int k = k0 + kk;
      double* prow = piv + 2 * MF * (k & 1);
      double* pcol = prow + MF;
      if (L.row == k) {
#pragma unroll
        for (int t = 0; t < EPL; ++t) prow[L.col(t)] = a[t];
      }
      if (L.cg == k0 / EPL) pcol[L.row] = a[kk];
      if constexpr (NT == 64) wave_lds_fence();
      else __syncthreads();
      double rk[EPL];
#pragma unroll
      for (int t = 0; t < EPL; ++t) rk[t] = prow[L.col(t)];
      const double ck = pcol[L.row];
      const double d = prow[k];
      ok = ok && (d > 0.0);
      // 1/d: hardware reciprocal refined by two Newton steps (full double precision)
      double rd = __builtin_amdgcn_rcp(d);
      rd = fma(rd, fma(-d, rd, 1.0), rd);
      rd = fma(rd, fma(-d, rd, 1.0), rd);
#pragma unroll
      for (int t = 0; t < EPL; ++t) {
        const int j = L.col(t);
        double v;
        if (L.row == k) v = (j == k) ? -rd : rk[t] * rd;
        else if (j == k) v = ck * rd;
        else v = a[t] - ck * rk[t] * rd;
        a[t] = v;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < EPL; ++t) a[t] = -a[t];
}

// The same inverse for the interleaved layout: pivot k = ck + LPR*tk lives in entry tk.
template <int MF>
__device__ __forceinline__ void lb_inverse_il(const LB<MF, true>& L, double (&a)[LB<MF>::EPL], bool& ok) {
  constexpr int EPL = LB<MF>::EPL, LPR = LB<MF>::LPR;
#pragma unroll
  for (int tk = 0; tk < EPL; ++tk) {
#pragma unroll 1
    for (int ck = 0; ck < LPR; ++ck) {
      const int k = ck + LPR * tk;
      double rk[EPL];
#pragma unroll
      for (int t = 0; t < EPL; ++t) rk[t] = __shfl(a[t], k * LPR + L.cg);
      const double cv = __shfl(a[tk], L.row * LPR + ck);
      const double d = __shfl(a[tk], k * LPR + ck);
      ok = ok && (d > 0.0);
      double rd = __builtin_amdgcn_rcp(d);
      rd = fma(rd, fma(-d, rd, 1.0), rd);
      rd = fma(rd, fma(-d, rd, 1.0), rd);
#pragma unroll
      for (int t = 0; t < EPL; ++t) {
        const int j = L.col(t);
        double v;
        if (L.row == k) v = (j == k) ? -rd : rk[t] * rd;
        else if (j == k) v = cv * rd;
        else v = a[t] - cv * rk[t] * rd;
        a[t] = v;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < EPL; ++t) a[t] = -a[t];
}

// Sum over the LPR consecutive lanes of a row, left in every lane of the row: the same
// additions as a butterfly over lane ^ 1, lane ^ 2 (quad permutations) and, for 8 lanes, the
// other quad of the row (half-row mirror, whose partner is in the other quad like lane ^ 4).
template <int LPR>
__device__ __forceinline__ double row_sum(double v) {
  static_assert(LPR == 1 || LPR == 2 || LPR == 4 || LPR == 8, "row of 1, 2, 4 or 8 lanes");
  if constexpr (LPR >= 2) v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  if constexpr (LPR >= 4) v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  if constexpr (LPR >= 8) v += dpp_f64<0x141>(v);   // row_half_mirror
  return v;
}

// y = D v for vectors replicated over a row's lanes (lane holds v[row]); result replicated.
template <int MF, bool IL>
__device__ __forceinline__ double lb_matvec(const LB<MF, IL>& L, const double (&a)[LB<MF>::EPL], double v) {
  constexpr int EPL = LB<MF>::EPL, LPR = LB<MF>::LPR;
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < EPL; ++t) acc += a[t] * __shfl(v, L.col(t) * LPR);
  return row_sum<LPR>(acc);
}

// Geometry of the line decomposition of a subdomain.
struct LineGeo {
  int len;      // cells per line (band of the banded ordering)
  int nlines;   // number of lines
};

__device__ __forceinline__ LineGeo line_geo(const Geo& g) {
  LineGeo lg;
  lg.len = g.band;
  lg.nlines = g.nc / g.band;
  return lg;
}

// (i, j) of the cell at position pos of line ln (matches loc_index: c = ln * len + pos).
__device__ __forceinline__ void line_cell(const Geo& g, int ln, int pos, int* i, int* j) {
  *i = g.xfast ? pos : ln;
  *j = g.xfast ? ln : pos;
}

// Face weights of a subdomain's matrix, computed once per cell into LDS (local order):
// tE[c] = |f| t of the face to the +x neighbour inside the subdomain (0 on its E edge),
// tN[c] likewise to the +y neighbour, dg[c] = diagonal entry. kf(i, j) gives the cell's
// conductivity.
// mode 0: boundary faces with their Dirichlet/Robin transmissibility (eq:mrc1);
// mode 1: all boundary faces are flux faces and cell 0 is pinned (p = 0): its couplings are
// dropped from the matrix and its diagonal is 1.
template <class KF>
__device__ __forceinline__ void fill_trans_k(const Geo& g, int I, int J, KF kf, int mode, double* tE, double* tN,
                                             double* dg) {
  for (int c = threadIdx.x; c < g.nc; c += blockDim.x) {
    int i, j;
    loc_ij(g, c, &i, &j);
    const double kc = kf(i, j);
    tE[c] = i < g.mx - 1 ? g.hy * harm_trans(kc, kf(i + 1, j), g.hx) : 0.0;
    tN[c] = j < g.my - 1 ? g.hx * harm_trans(kc, kf(i, j + 1), g.hy) : 0.0;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < g.nc; c += blockDim.x) {
    int i, j;
    loc_ij(g, c, &i, &j);
    const double kc = kf(i, j);
    double d = tE[c] + tN[c];
    if (i > 0) d += tE[loc_index(g, i - 1, j)];
    if (j > 0) d += tN[loc_index(g, i, j - 1)];
    if (mode == 0) {
      if (i == 0) { BFace f = bface(g, I, J, j); d += f.flen * bface_trans(g, f, kc); }
      if (i == g.mx - 1) { BFace f = bface(g, I, J, g.my + j); d += f.flen * bface_trans(g, f, kc); }
      if (j == 0) { BFace f = bface(g, I, J, 2 * g.my + i); d += f.flen * bface_trans(g, f, kc); }
      if (j == g.my - 1) { BFace f = bface(g, I, J, 2 * g.my + g.mx + i); d += f.flen * bface_trans(g, f, kc); }
    }
    dg[c] = (mode == 1 && c == 0) ? 1.0 : d;
  }
  __syncthreads();
}

__device__ __forceinline__ void fill_trans(const Geo& g, int I, int J, const double* kl, int mode, double* tE,
                                           double* tN, double* dg) {
  fill_trans_k(g, I, J, [&](int i, int j) { return kl[loc_index(g, i, j)]; }, mode, tE, tN, dg);
}

// Only the couplings between neighbouring lines (what a solve with kept inverse blocks needs):
// ty[c] = |f| t of the face from cell c to its neighbour on the next line (0 on the last line).
// No barrier.
template <class KF>
__device__ __forceinline__ void fill_ycoup_k(const Geo& g, KF kf, double* ty) {
  for (int c = threadIdx.x; c < g.nc; c += blockDim.x) {
    int i, j;
    loc_ij(g, c, &i, &j);
    const double kc = kf(i, j);
    double t;
    if (g.xfast) t = j < g.my - 1 ? g.hx * harm_trans(kc, kf(i, j + 1), g.hy) : 0.0;
    else t = i < g.mx - 1 ? g.hy * harm_trans(kc, kf(i + 1, j), g.hx) : 0.0;
    ty[c] = t;
  }
}

// Couplings in line form. The matrix entries with the pinned cell are zero.
struct LineW {
  const double* tE;
  const double* tN;
  const double* dg;
  int xfast, band, mode;
  // weight between position pos and pos+1 of line ln
  __device__ __forceinline__ double off(int ln, int pos) const {
    const int c = ln * band + pos;
    if (mode == 1 && c == 0) return 0.0;
    return xfast ? tE[c] : tN[c];
  }
  // weight between (ln, pos) and (ln+1, pos)
  __device__ __forceinline__ double y(int ln, int pos) const {
    const int c = ln * band + pos;
    if (mode == 1 && c == 0) return 0.0;
    return xfast ? tN[c] : tE[c];
  }
  __device__ __forceinline__ double diag(int ln, int pos) const { return dg[ln * band + pos]; }
};

// Builds D_ln for line ln in registers: T_ln - Y_{ln-1} Eprev Y_{ln-1}.
template <int MF, bool IL, int NT>
__device__ __forceinline__ void lb_block(const LineW& W, int ln, const LB<MF, IL, NT>& L,
                                         const double (&Eprev)[LB<MF, IL, NT>::EPL],
                                         double (&a)[LB<MF, IL, NT>::EPL]) {
  constexpr int EPL = LB<MF, IL, NT>::EPL;
  const int len = W.band;
  const int r = L.row;
  const bool rin = r < len;
  const double drow = rin ? W.diag(ln, r) : 1.0;
  const double offR = (rin && r + 1 < len) ? W.off(ln, r) : 0.0;
  const double offL = (rin && r > 0) ? W.off(ln, r - 1) : 0.0;
  const double yr = (ln > 0 && rin) ? W.y(ln - 1, r) : 0.0;
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    const int c = L.col(t);
    double v;
    if (c == r) v = drow;
    else if (c == r + 1) v = -offR;
    else if (c == r - 1) v = -offL;
    else v = 0.0;
    if (ln > 0 && rin && c < len) v -= yr * Eprev[t] * W.y(ln - 1, c);
    if (!rin || c >= len) v = (c == r) ? 1.0 : 0.0;
    a[t] = v;
  }
}

// From the Robin-to-flux map S (nb x nb, global) and the boundary fluxes h (LDS) of a
// subdomain: its interface block K_i = B^T S B - D_i (eq:mrc2 with the Robin rows negated;
// D_i couples the U unknowns of one element: sum_f |f| beta_f phi_k phi_k') and the right-hand
// side B^T h, written into the parent's slot. kl: kappa in local order.
// One wavefront; S must be visible to all lanes (barrier before the call).
__device__ __forceinline__ void basis_iface_block(const Geo& g, int I, int J, int sub, const double* kl,
                                                  const double* Ss, const double* hsh, double* leafK,
                                                  const LeafOut& lo) {
  const int nb = g.nb;
  const int nd = sub_ndof(g, I, J);
  double* Ks = leafK + size_t(sub) * g.ndmax * g.ndmax;
  for (int p = threadIdx.x; p < nd * nd; p += 64) {
    const int a = p / nd, c2 = p % nd;
    int fa, na, fb, nbb;
    dof_faces(g, I, J, a, &fa, &na);
    dof_faces(g, I, J, c2, &fb, &nbb);
    double v = 0.0;
    for (int x = fa; x < fa + na; ++x) {
      const BFace ff = bface(g, I, J, x);
      const double wa = bweight(g, ff, a, kl[loc_index(g, ff.i, ff.j)]);
      double sacc = 0.0;
      for (int y = fb; y < fb + nbb; ++y) {
        const BFace fgb = bface(g, I, J, y);
        sacc += Ss[smap_at(nb, x, y)] * bweight(g, fgb, c2, kl[loc_index(g, fgb.i, fgb.j)]);
      }
      v += wa * sacc;
    }
    bool pa, pb;
    int ka, kb;
    dof_kind(g, a, &pa, &ka);
    dof_kind(g, c2, &pb, &kb);
    if (fa == fb && !pa && !pb) {   // U unknowns of the same element
      double dsum = 0.0;
      for (int x = fa; x < fa + na; ++x) {
        const BFace ff = bface(g, I, J, x);
        dsum += ff.flen * robin_beta(g, ff, kl[loc_index(g, ff.i, ff.j)]) * iface_phi(g, ff, ka) *
                iface_phi(g, ff, kb);
      }
      v -= dsum;
    }
    Ks[a * nd + c2] = v;
  }
  for (int a = threadIdx.x; a < nd; a += 64) {
    int fa, na;
    dof_faces(g, I, J, a, &fa, &na);
    double v = 0.0;
    for (int x = fa; x < fa + na; ++x) {
      const BFace ff = bface(g, I, J, x);
      v += bweight(g, ff, a, kl[loc_index(g, ff.i, ff.j)]) * hsh[x];
    }
    leaf_out(lo, sub, a, v);
  }
}

// Right-hand side of the non-homogeneous local problem (eq:mrc_non_homogeneous, Robin datum 0)
// at local cell c: |c| q + sum_DIR |f| t g - sum_NEU |f| z.
__device__ __forceinline__ double basis_rhs0(const Geo& g, int I, int J, int c, const double* kl, double qc) {
  int i, j;
  loc_ij(g, c, &i, &j);
  const double kc = kl[c];
  double r = g.hx * g.hy * qc;
  for (int t = 0; t < 4; ++t) {
    const bool on = (t == 0 && i == 0) || (t == 1 && i == g.mx - 1) || (t == 2 && j == 0) ||
                    (t == 3 && j == g.my - 1);
    if (!on) continue;
    const int fi = t == 0 ? j : t == 1 ? g.my + j : t == 2 ? 2 * g.my + i : 2 * g.my + g.mx + i;
    const BFace f = bface(g, I, J, fi);
    if (f.kind == FACE_DIR) r += f.flen * bface_trans(g, f, kc) * f.value;
    if (f.kind == FACE_NEU) r -= f.flen * f.value;
  }
  return r;
}

}  // namespace mpm
