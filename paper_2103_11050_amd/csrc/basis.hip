// MRCM basis of every subdomain on the matrix cores (A2 + A3).
//
// For subdomain i with local Robin matrix A (eq:mrc1 with zero Robin datum), the homogeneous
// basis functions of eq:mrc_homogeneous enter the interface system and the flux reconstruction
// only through the Robin-to-flux map on the boundary faces,
//   S = W T - W T (E^T A^-1 E) W T,
// where E holds one unit column per boundary face (the adjacent cell) and W T = diag(|f| t_f);
// the non-homogeneous basis function of eq:mrc_non_homogeneous enters through its boundary
// fluxes h = W T (E^T A^-1 r0 - r_D).
//
// With the line-block factorisation A = L diag(D_j) L^T (block bidiagonal L, lines.hpp),
//   E^T A^-1 E = sum_j Z_j^T D_j^-1 Z_j,   Z_0 = E_0,  Z_{j+1} = E_{j+1} + Y_j D_j^-1 Z_j,
// a chain of 16 x 16 by 16 x 64 products per line, each a few FP64 MFMA instructions.
//
// Matrix-core layout. v_mfma_f64_16x16x4 takes A[i][k] from lane k*16 + i, B[k][j] from lane
// k*16 + j and returns C[k' + 4v][j] in lane k'*16 + j, register v. A 16 x 16 matrix X is held
// as x[v] = X[g + 4v][c] in lane 16 g + c; chaining four instructions with K index g + 4 kc
// (chunk kc, lane group g) then consumes and produces X in the same layout, so the line
// recursion and the Gram sums need no data movement. D_j^-1 is computed in the interleaved
// line-block layout, whose entry kc is exactly the A operand of chunk kc after one shuffle.
//
// Columns (boundary faces) are grouped by where they sit in the line ordering:
//   block 0: position 0 of each line,   block 1: last position of each line,
//   block 2: every position of line 0,  block 3: every position of the last line.
// Block 3 is zero until the last line, so it joins the products only there.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"
#include "lines.hpp"

namespace mpm {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma_f64(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// C = A X over the four K-chunks (A operand per chunk in a[kc], X in the matrix-core layout).
__device__ __forceinline__ dbl4 mfma_chain(const double (&a)[4], const dbl4& x) {
  dbl4 c = {0.0, 0.0, 0.0, 0.0};
  c = mfma_f64(a[0], x[0], c);
  c = mfma_f64(a[1], x[1], c);
  c = mfma_f64(a[2], x[2], c);
  c = mfma_f64(a[3], x[3], c);
  return c;
}

// acc += X^T Y for X, Y in the matrix-core layout.
__device__ __forceinline__ void mfma_gram(dbl4& acc, const dbl4& x, const dbl4& y) {
  acc = mfma_f64(x[0], y[0], acc);
  acc = mfma_f64(x[1], y[1], acc);
  acc = mfma_f64(x[2], y[2], acc);
  acc = mfma_f64(x[3], y[3], acc);
}

// Boundary face (index into the bface numbering) of column c of block b, with its line and
// position; -1 past the end of the block.
__device__ __forceinline__ int block_face(const Geo& g, int b, int c, int nl, int len, int* ln, int* pos) {
  int f = -1, l = -1, p = -1;
  if (b == 0 && c < nl) { l = c; p = 0; f = g.xfast ? c : 2 * g.my + c; }
  if (b == 1 && c < nl) { l = c; p = len - 1; f = g.xfast ? g.my + c : 2 * g.my + g.mx + c; }
  if (b == 2 && c < len) { l = 0; p = c; f = g.xfast ? 2 * g.my + c : c; }
  if (b == 3 && c < len) { l = nl - 1; p = c; f = g.xfast ? 2 * g.my + g.mx + c : g.my + c; }
  *ln = l;
  *pos = p;
  return f;
}

__device__ __forceinline__ int gcell3(const Geo& g, int I, int J, int i, int j) {
  return (J * g.my + j) * g.nx + I * g.mx + i;
}

// One wavefront per subdomain. Writes S (nb x nb, row-major per subdomain), h, the interface
// block K_i = B^T S B - D_i with its right-hand side B^T h (eq:mrc2 with the Robin rows
// negated; the right-hand side goes into the parent's slot of the interface solve), and, with
// store_fac, the line-block inverses D_j^-1 in the layout the MPM-2P solve reads
// (E[sub][line][t][lane], contiguous line-block layout, lines padded to 16).
__global__ void __launch_bounds__(64)
k_basis_mfma(Geo g, const double* __restrict__ kap, const double* __restrict__ q, double* __restrict__ Sg,
             double* __restrict__ hg, double* __restrict__ leafK, LeafOut lo, double* __restrict__ fac,
             int store_fac, int32_t* err, const RunTab* __restrict__ rt) {
  {
    const int64_t wo = ws_off(rt);
    kap = at_off(kap, wo);
    q = at_off(q, wo);
    Sg = at_off(Sg, wo);
    hg = at_off(hg, wo);
    leafK = at_off(leafK, wo);
    lo = leaf_at(lo, wo);
    fac = at_off(fac, wo);
    err = at_off(err, wo);
  }
  __shared__ double kl[256], tE[256], tN[256], dg[256], rhs0[256], wsh[64], hsh[64];
  const int sub = xcd_sub(g.nsub);
  const int I = sub % g.Sx, J = sub / g.Sx;
  const int lane = threadIdx.x;
  const int gq = lane >> 4, cc = lane & 15;
  const int len = g.band, nl = g.nc / g.band, nb = g.nb;
  LB<16, true> L;

  for (int c = lane; c < g.nc; c += 64) {
    int i, j;
    loc_ij(g, c, &i, &j);
    kl[c] = kap[gcell3(g, I, J, i, j)];
  }
  __syncthreads();
  fill_trans(g, I, J, kl, 0, tE, tN, dg);
  const LineW W{tE, tN, dg, g.xfast, g.band, 0};

  // non-homogeneous right-hand side: |c| q + sum_DIR |f| t g - sum_NEU |f| z (Robin datum 0)
  for (int c = lane; c < g.nc; c += 64) {
    int i, j;
    loc_ij(g, c, &i, &j);
    rhs0[c] = basis_rhs0(g, I, J, c, kl, q[gcell3(g, I, J, i, j)]);
  }
  if (lane < nb) {
    const BFace f = bface(g, I, J, lane);
    wsh[lane] = f.flen * bface_trans(g, f, kl[loc_index(g, f.i, f.j)]);
  }
  __syncthreads();

  // this lane's column in each block
  int fl[4], fp[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) block_face(g, b, cc, nl, len, &fl[b], &fp[b]);

  dbl4 z[4], w[4];
  dbl4 G[10];   // tiles (0,0) (0,1) (0,2) (1,1) (1,2) (2,2) (0,3) (1,3) (2,3) (3,3)
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    z[b] = dbl4{0.0, 0.0, 0.0, 0.0};
    w[b] = z[b];
  }
#pragma unroll
  for (int t = 0; t < 10; ++t) G[t] = dbl4{0.0, 0.0, 0.0, 0.0};
  double gr[4] = {0.0, 0.0, 0.0, 0.0};   // E^T A^-1 r0, partial over this lane's positions
  double z4 = 0.0;                       // r0 forward-substituted, replicated over a row's lanes
  double prev[4] = {0.0, 0.0, 0.0, 0.0}, cur[4];
  bool ok = true;

#pragma unroll 1
  for (int ln = 0; ln < nl; ++ln) {
    lb_block<16>(W, ln, L, prev, cur);
    lb_inverse_il<16>(L, cur, ok);
#pragma unroll
    for (int t = 0; t < 4; ++t) prev[t] = cur[t];
    if (store_fac) {
      // entry t of lane (row, cg) is D^-1[row][cg + 4t]; the upper triangle, packed
      double* E = fac + (size_t(sub) * nl + ln) * LBP<16>::P;
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (L.row <= L.col(t)) E[lb_pk<16>(L.row, L.col(t))] = cur[t];
    }
    // A operand of D^-1 for chunk kc: D^-1[cc][gq + 4 kc], entry kc of lane (row cc, cg gq)
    double Da[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) Da[kc] = __shfl(cur[kc], cc * 4 + gq);
    // unit columns of the faces on this line
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (fl[b] == ln && fp[b] == gq + 4 * v) z[b][v] += 1.0;
    }
    z4 += L.row < len ? rhs0[ln * len + L.row] : 0.0;
    const bool last = ln == nl - 1;
#pragma unroll
    for (int b = 0; b < 3; ++b) w[b] = mfma_chain(Da, z[b]);
    if (last) w[3] = mfma_chain(Da, z[3]);
    const double w4 = lb_matvec<16>(L, cur, z4);
    mfma_gram(G[0], z[0], w[0]);
    mfma_gram(G[1], z[0], w[1]);
    mfma_gram(G[2], z[0], w[2]);
    mfma_gram(G[3], z[1], w[1]);
    mfma_gram(G[4], z[1], w[2]);
    mfma_gram(G[5], z[2], w[2]);
    if (last) {
      mfma_gram(G[6], z[0], w[3]);
      mfma_gram(G[7], z[1], w[3]);
      mfma_gram(G[8], z[2], w[3]);
      mfma_gram(G[9], z[3], w[3]);
    }
    // r0 column: sum over positions of Z[p][c] (D^-1 z4)[p]
    double w4q[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) w4q[v] = __shfl(w4, (gq + 4 * v) * 4);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
      for (int v = 0; v < 4; ++v) gr[b] += z[b][v] * w4q[v];
    }
    if (!last) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = gq + 4 * v;
        const double yv = p < len ? W.y(ln, p) : 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) z[b][v] = yv * w[b][v];
      }
      z4 = (L.row < len ? W.y(ln, L.row) : 0.0) * w4;
    }
  }
  if (!ok && lane == 0) set_error(err, ERR_NOTSPD);

  // S = W T - W T G W T, each stored entry once (wrapped diagonals)
  double* Ss = Sg + size_t(sub) * smap_doubles(nb);
  auto put = [&](const dbl4& t, int a, int b) {
    int lb_, pb_;
    const int fc = block_face(g, b, cc, nl, len, &lb_, &pb_);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int la, pa;
      const int fr = block_face(g, a, gq + 4 * v, nl, len, &la, &pa);
      if (fr >= 0 && fc >= 0) {
        const double val = (fr == fc ? wsh[fr] : 0.0) - wsh[fr] * t[v] * wsh[fc];
        if (smap_owner(nb, fr, fc)) Ss[smap_at(nb, fr, fc)] = val;
        if (a != b && smap_owner(nb, fc, fr)) Ss[smap_at(nb, fc, fr)] = val;
      }
    }
  };
  put(G[0], 0, 0); put(G[1], 0, 1); put(G[2], 0, 2); put(G[3], 1, 1); put(G[4], 1, 2);
  put(G[5], 2, 2); put(G[6], 0, 3); put(G[7], 1, 3); put(G[8], 2, 3); put(G[9], 3, 3);
  // h = W T (E^T p0 - r_D) on Dirichlet and Robin faces, 0 on Neumann faces
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    gr[b] += __shfl_xor(gr[b], 16);
    gr[b] += __shfl_xor(gr[b], 32);
    if (gq == 0 && fl[b] >= 0) {
      int lx, px;
      const int f = block_face(g, b, cc, nl, len, &lx, &px);
      const BFace bf = bface(g, I, J, f);
      const double rD = bf.kind == FACE_DIR ? bf.value : 0.0;
      const double h = bf.kind == FACE_NEU ? 0.0 : wsh[f] * (gr[b] - rD);
      hsh[f] = h;
      hg[size_t(sub) * nb + f] = h;
    }
  }
  __syncthreads();

  // interface block K_i = B^T S B - D_i and right-hand side B^T h (Gamma faces only)
  basis_iface_block(g, I, J, sub, kl, Ss, hsh, leafK, lo);
}

}  // namespace

// Returns whether the kappa^m line-block inverses were written (lines of 9..16 cells).
bool launch_basis(hipStream_t st, const Geo& g, const double* kap, const double* q, double* S, double* h,
                  double* leafK, LeafOut lo, double* fac, int32_t* err, Runs rt) {
  if (g.band > 16 || g.nc / g.band > 16) {   // longer lines or more lines than the matrix-core blocks take
    launch_basis_lines(st, g, kap, q, S, h, leafK, lo, fac, err, rt);
    return true;
  }
  const int store = g.band > 8 ? 1 : 0;
  hipLaunchKernelGGL(k_basis_mfma, dim3(g.nsub, 1, runs_of(rt)), dim3(64), 0, st, g, kap, q, S, h, leafK, lo, fac,
                     store, err, rt.tab);
  return store != 0;
}

}  // namespace mpm
