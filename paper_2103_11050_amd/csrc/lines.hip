// Line-block kernels: factorisation of the kappa^m local Robin matrices (kept for MPM-2P),
// the MPM-2P trivial-Robin solve and the all-Neumann downscaling, each one wavefront per
// subdomain with the block inverses in registers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "kernels.hpp"
#include "lines.hpp"

namespace mpm {

namespace {


__device__ __forceinline__ int gcell2(const Geo& g, int I, int J, int i, int j) { return (J * g.my + j) * g.nx + I * g.mx + i; }

// A subdomain's tile of a cell field into LDS (local order), four cells per thread in flight at a
// time (their loads issued before the first store; addresses past the tile clamped to its first
// cell, and not stored).
__device__ __forceinline__ void load_tile2(const Geo& g, int I, int J, const double* src, double* dst) {
  constexpr int U = 4;
  for (int c0 = threadIdx.x; c0 < g.nc; c0 += U * blockDim.x) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * blockDim.x;
      int i, j;
      loc_ij(g, c < g.nc ? c : 0, &i, &j);
      v[u] = src[gcell2(g, I, J, i, j)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * blockDim.x;
      if (c < g.nc) dst[c] = v[u];
    }
  }
}

// factor offsets: E[sub][line][packed upper triangle]
template <int MF>
__device__ __forceinline__ size_t efac_off(const Geo& g, int sub) {
  const int nl = g.nc / g.band;
  return size_t(sub) * nl * LBP<MF>::P;
}

// Packed position of entry t of this lane's row (the same for every line).
template <int MF, int NT = 64>
__device__ __forceinline__ void lb_pk_lane(const LB<MF, false, NT>& L, int (&pk)[LB<MF, false, NT>::EPL]) {
#pragma unroll
  for (int t = 0; t < LB<MF, false, NT>::EPL; ++t) pk[t] = lb_pk<MF>(L.row, L.col(t));
}

// Block elimination over all lines; the upper triangles of the inverses D_ln^-1 go to
// Es[ln * P + packed position] (global; a reader in the same kernel needs a barrier first, as
// the entries of a row below the diagonal were written by other lanes).
template <int MF, typename T, int NT = 64>
__device__ __forceinline__ void lb_factor(const Geo& g, const LineW& W, const LB<MF, false, NT>& L, T* Es, bool& ok) {
  constexpr int EPL = LB<MF, false, NT>::EPL;
  const int nl = g.nc / g.band;
  constexpr int P = LBP<MF>::P;
  int pk[EPL];
  lb_pk_lane<MF, NT>(L, pk);
  __shared__ double piv[4 * MF];   // pivot rows and columns of the Gauss-Jordan sweep
  double prev[EPL], cur[EPL];
#pragma unroll
  for (int t = 0; t < EPL; ++t) prev[t] = 0.0;
#pragma unroll 1
  for (int ln = 0; ln < nl; ++ln) {
    lb_block<MF>(W, ln, L, prev, cur);
    lb_inverse<MF, NT>(L, cur, ok, piv);
#pragma unroll
    for (int t = 0; t < EPL; ++t) {
      if (L.row <= L.col(t)) Es[size_t(ln) * P + pk[t]] = T(cur[t]);
      prev[t] = cur[t];
    }
  }
}

// Column steps (COLS = true in the ring solve): each lane reads the EPL entries of its own
// columns of the line's vector from x in LDS, applies its EPL entries of the block to them and
// the LPR lanes of the row sum their parts; the row's first lane writes the result over x, and
// the next step reads those entries back from LDS (the lanes of one wavefront see each other's
// LDS writes in program order). No shuffle per block entry, but three vector reads per lane and
// step; same arithmetic, in the same order, as the row steps.

// Forward step on line ln: z = r_ln + Y_{ln-1} w_{ln-1} on this lane's columns (x holds r_ln
// and, in line ln - 1, w_{ln-1}), w_ln = D_ln^-1 z written over r_ln.
template <int MF>
__device__ __forceinline__ void lb_fwd_step(const LineW& W, const LB<MF>& L, const double (&a)[LB<MF>::EPL], int ln,
                                            double* x) {
  constexpr int EPL = LB<MF>::EPL, LPR = LB<MF>::LPR;
  const int len = W.band;
  wave_lds_fence();   // the previous step's results, written by other lanes
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    const int c = L.col(t);
    double z = 0.0;
    if (c < len) {
      z = x[ln * len + c];
      if (ln > 0) z = fma(W.y(ln - 1, c), x[(ln - 1) * len + c], z);
    }
    acc = fma(a[t], z, acc);
  }
  const double w = row_sum<LPR>(acc);
  if (L.row < len && L.cg == 0) x[ln * len + L.row] = w;
}

// Backward step on line ln < nl - 1: x_ln = w_ln + D_ln^-1 (Y_ln x_{ln+1}), with x_{ln+1}
// final in x and w_ln in line ln of x.
template <int MF>
__device__ __forceinline__ void lb_bwd_step(const LineW& W, const LB<MF>& L, const double (&a)[LB<MF>::EPL], int ln,
                                            double* x) {
  constexpr int EPL = LB<MF>::EPL, LPR = LB<MF>::LPR;
  const int len = W.band;
  wave_lds_fence();   // the previous step's results, written by other lanes
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    const int c = L.col(t);
    const double v = c < len ? W.y(ln, c) * x[(ln + 1) * len + c] : 0.0;
    acc = fma(a[t], v, acc);
  }
  const bool rin = L.row < len;
  const double wl = rin ? x[ln * len + L.row] : 0.0;
  const double xn = wl + row_sum<LPR>(acc);
  if (rin && L.cg == 0) x[ln * len + L.row] = xn;
}

// x (LDS, local order) holds the right-hand side on entry and the solution on exit (the forward
// result w_ln overwrites line ln of the right-hand side, which the row's lanes read before they
// write it); Es holds the block inverses as written by lb_factor. Any line count.
template <int MF>
__device__ __forceinline__ void lb_solve(const Geo& g, const LineW& W, const LB<MF>& L, const double* Es, double* x) {
  constexpr int EPL = LB<MF>::EPL;
  const int nl = g.nc / g.band;
  const int len = g.band;
  const bool rin = L.row < len;
  const bool wr = rin && L.cg == 0;
  const int xr = rin ? L.row : 0;
  constexpr int P = LBP<MF>::P;
  int pk[EPL];
  lb_pk_lane<MF>(L, pk);
  // the next line's block is loaded while the current one is applied
  double e[EPL], en[EPL];
#pragma unroll
  for (int t = 0; t < EPL; ++t) e[t] = Es[pk[t]];
  double wprev = 0.0;
#pragma unroll 1
  for (int ln = 0; ln < nl; ++ln) {
    const int lnn = ln + 1 < nl ? ln + 1 : ln;
#pragma unroll
    for (int t = 0; t < EPL; ++t) en[t] = Es[size_t(lnn) * P + pk[t]];
    double z = rin ? x[ln * len + xr] : 0.0;
    if (ln > 0 && rin) z += W.y(ln - 1, xr) * wprev;
    wprev = lb_matvec<MF>(L, e, z);
    if (wr) x[ln * len + xr] = wprev;
#pragma unroll
    for (int t = 0; t < EPL; ++t) e[t] = en[t];
  }
  double xnext = wprev;   // line nl - 1 holds its solution already
  if (nl >= 2) {
#pragma unroll
    for (int t = 0; t < EPL; ++t) e[t] = Es[size_t(nl - 2) * P + pk[t]];
  }
#pragma unroll 1
  for (int ln = nl - 2; ln >= 0; --ln) {
    const int lnn = ln > 0 ? ln - 1 : 0;
#pragma unroll
    for (int t = 0; t < EPL; ++t) en[t] = Es[size_t(lnn) * P + pk[t]];
    wave_lds_fence();   // w_ln was written by the row's first lane
    const double v = rin ? W.y(ln, xr) * xnext : 0.0;
    xnext = (rin ? x[ln * len + xr] : 0.0) + lb_matvec<MF>(L, e, v);
    if (wr) x[ln * len + xr] = xnext;
#pragma unroll
    for (int t = 0; t < EPL; ++t) e[t] = en[t];
  }
  __syncthreads();
}

// Same solve with a compile-time line count: all inverse blocks are loaded into registers at
// once (every load in flight together) and serve both sweeps, so they are read from memory
// once.
template <int MF, int NL>
__device__ __forceinline__ void lb_load_reg(const LB<MF>& L, const double* Es, double (&E)[NL][LB<MF>::EPL]) {
  constexpr int EPL = LB<MF>::EPL, P = LBP<MF>::P;
  int pk[EPL];
  lb_pk_lane<MF>(L, pk);
#pragma unroll
  for (int ln = 0; ln < NL; ++ln)
#pragma unroll
    for (int t = 0; t < EPL; ++t) E[ln][t] = Es[size_t(ln) * P + pk[t]];
}

// The two sweeps with the blocks already in registers.
template <int MF, int NL>
__device__ __forceinline__ void lb_solve_regs(const LineW& W, const LB<MF>& L, const double (&E)[NL][LB<MF>::EPL],
                                              double* x) {
  const int len = W.band;
  const bool rin = L.row < len;
  double w[NL];
#pragma unroll
  for (int ln = 0; ln < NL; ++ln) {
    double z = rin ? x[ln * len + L.row] : 0.0;
    if (ln > 0 && rin) z += W.y(ln - 1, L.row) * w[ln - 1];
    w[ln] = lb_matvec<MF>(L, E[ln], z);
  }
  double xnext = w[NL - 1];
  if (rin && L.cg == 0) x[(NL - 1) * len + L.row] = xnext;
#pragma unroll
  for (int ln = NL - 2; ln >= 0; --ln) {
    const double v = rin ? W.y(ln, L.row) * xnext : 0.0;
    xnext = w[ln] + lb_matvec<MF>(L, E[ln], v);
    if (rin && L.cg == 0) x[ln * len + L.row] = xnext;
  }
  __syncthreads();
}

// The same two sweeps with the blocks streamed through a ring of D register blocks instead of
// all NL held at once: the uses run forward over lines 0 .. NL-1, then backward over NL-2 .. 0,
// and the load for use k + D is issued right after use k, so D blocks are in flight while one is
// applied. The backward uses re-read blocks that the forward sweep read shortly before (served
// by the caches). Holding D blocks instead of NL frees the registers that bound the resident
// wavefronts per SIMD.
template <int NL>
__device__ __forceinline__ constexpr int ring_line(int k) { return k < NL ? k : 2 * NL - 2 - k; }

template <int MF, int NL, int D>
__device__ __forceinline__ void lb_ring_load(const LB<MF>& L, const double* Es, double (&e)[D][LB<MF>::EPL]) {
  constexpr int EPL = LB<MF>::EPL, P = LBP<MF>::P;
  int pk[EPL];
  lb_pk_lane<MF>(L, pk);
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int t = 0; t < EPL; ++t) e[d][t] = Es[size_t(ring_line<NL>(d)) * P + pk[t]];
}

template <int MF, int NL, int D, bool COLS>
__device__ __forceinline__ void lb_solve_ring(const LineW& W, const LB<MF>& L, const double* Es,
                                              double (&e)[D][LB<MF>::EPL], double* x) {
  constexpr int EPL = LB<MF>::EPL, P = LBP<MF>::P, NU = 2 * NL - 1;
  static_assert(D >= 1 && D < NU, "ring depth");
  int pk[EPL];
  lb_pk_lane<MF>(L, pk);
  const int len = W.band;
  const bool rin = L.row < len;
  const bool wr = rin && L.cg == 0;
  const int xr = rin ? L.row : 0;
  // row steps: the forward result w_ln overwrites line ln of the right-hand side in x (read by
  // the row's lanes before one of them writes it); the backward sweep reads it back
  double xnext = 0.0;
#pragma unroll
  for (int k = 0; k < NU; ++k) {
    const int ln = ring_line<NL>(k);
    if constexpr (COLS) {
      if (k < NL) lb_fwd_step<MF>(W, L, e[k % D], ln, x);
      else lb_bwd_step<MF>(W, L, e[k % D], ln, x);
    } else if (k < NL) {
      double z = rin ? x[ln * len + xr] : 0.0;
      if (ln > 0 && rin) z += W.y(ln - 1, xr) * xnext;
      xnext = lb_matvec<MF>(L, e[k % D], z);
      if (wr) x[ln * len + xr] = xnext;
    } else {
      wave_lds_fence();   // w_ln was written by the row's first lane
      const double v = rin ? W.y(ln, xr) * xnext : 0.0;
      const double wl = rin ? x[ln * len + xr] : 0.0;
      xnext = wl + lb_matvec<MF>(L, e[k % D], v);
      if (wr) x[ln * len + xr] = xnext;
    }
    if (k + D < NU) {
#pragma unroll
      for (int t = 0; t < EPL; ++t) e[k % D][t] = Es[size_t(ring_line<NL>(k + D)) * P + pk[t]];
    }
    // one step at a time: the scheduler would otherwise hoist later steps' loads and LDS reads
    // and hold their results in registers, which is what the ring is there to avoid
    __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();
}

// ------------------------------------------------------------------ FP32 blocks, FP64 refinement
// Precision form: the inverse blocks are stored in FP32 and applied in FP32; each solve is
// recovered by FP64 iterative refinement against the FP64 line form of the same matrix.

template <int MF>
__device__ __forceinline__ float lb_matvec_f(const LB<MF>& L, const float (&a)[LB<MF>::EPL], float v) {
  constexpr int EPL = LB<MF>::EPL, LPR = LB<MF>::LPR;
  float acc = 0.0f;
#pragma unroll
  for (int t = 0; t < EPL; ++t) acc += a[t] * __shfl(v, L.col(t) * LPR);
#pragma unroll
  for (int o = 1; o < LPR; o <<= 1) acc += __shfl_xor(acc, o);
  return acc;
}

// Up to 16 lines of FP32 blocks into registers (nl lines at run time).
template <int MF>
__device__ __forceinline__ void lb_load_f32(const LB<MF>& L, const float* Es, int nl, float (&E)[16][LB<MF>::EPL]) {
  constexpr int EPL = LB<MF>::EPL, P = LBP<MF>::P;
  int pk[EPL];
  lb_pk_lane<MF>(L, pk);
#pragma unroll
  for (int ln = 0; ln < 16; ++ln)
#pragma unroll
    for (int t = 0; t < EPL; ++t) E[ln][t] = ln < nl ? Es[size_t(ln) * P + pk[t]] : 0.0f;
}

// d = M^-1 r with the FP32 blocks (both sweeps in FP32); r and d in LDS, local order, FP64.
template <int MF>
__device__ __forceinline__ void lb_apply_f32(const LineW& W, const LB<MF>& L, int nl,
                                             const float (&E)[16][LB<MF>::EPL], const double* r, double* d) {
  const int len = W.band;
  const bool rin = L.row < len;
  float w[16];
#pragma unroll
  for (int ln = 0; ln < 16; ++ln) {
    w[ln] = 0.0f;
    if (ln < nl) {
      float z = rin ? float(r[ln * len + L.row]) : 0.0f;
      if (ln > 0 && rin) z += float(W.y(ln - 1, L.row)) * w[ln - 1];
      w[ln] = lb_matvec_f<MF>(L, E[ln], z);
    }
  }
  float xn = 0.0f;
#pragma unroll
  for (int ln = 15; ln >= 0; --ln) {
    if (ln < nl) {
      float xv = w[ln];
      if (ln < nl - 1) {
        const float v = rin ? float(W.y(ln, L.row)) * xn : 0.0f;
        xv += lb_matvec_f<MF>(L, E[ln], v);
      }
      xn = xv;
      if (rin && L.cg == 0) d[ln * len + L.row] = double(xv);
    }
  }
  __syncthreads();
}

// r = b - A x in FP64 with A the line form of the matrix (the one the blocks invert).
__device__ __forceinline__ void line_residual(const Geo& g, const LineW& W, int nl, const double* b,
                                              const double* x, double* r) {
  const int len = W.band;
  for (int c = threadIdx.x; c < g.nc; c += blockDim.x) {
    const int ln = c / len, pos = c % len;
    double ax = W.diag(ln, pos) * x[c];
    if (pos + 1 < len) ax -= W.off(ln, pos) * x[c + 1];
    if (pos > 0) ax -= W.off(ln, pos - 1) * x[c - 1];
    if (ln + 1 < nl) ax -= W.y(ln, pos) * x[c + len];
    if (ln > 0) ax -= W.y(ln - 1, pos) * x[c - len];
    r[c] = b[c] - ax;
  }
  __syncthreads();
}

// Refinement budget of the precision form: corrections stop once the largest one is at most
// g.refine_rtol times the largest solution entry, at most REFINE_MAXIT of them.
constexpr int REFINE_MAXIT = 8;

// x holds the right-hand side on entry and the solution on exit (LDS, local order); ws is LDS
// scratch of 3 * nc doubles. One wavefront. Returns whether the tolerance was reached (the
// same value in every lane).
template <int MF>
__device__ __forceinline__ bool lb_solve_refined(const Geo& g, const LineW& W, const LB<MF>& L,
                                                 const float (&E)[16][LB<MF>::EPL], double* x, double* ws) {
  const int nl = g.nc / g.band;
  double* b = ws;
  double* r = ws + g.nc;
  double* d = ws + 2 * g.nc;
  for (int c = threadIdx.x; c < g.nc; c += blockDim.x) b[c] = x[c];
  __syncthreads();
  lb_apply_f32<MF>(W, L, nl, E, b, x);
  bool conv = false;
#pragma unroll 1
  for (int it = 0; it < REFINE_MAXIT; ++it) {
    line_residual(g, W, nl, b, x, r);
    lb_apply_f32<MF>(W, L, nl, E, r, d);
    double dm = 0.0, xm = 0.0;
    for (int c = threadIdx.x; c < g.nc; c += blockDim.x) {
      const double xv = x[c] + d[c];
      x[c] = xv;
      dm = fmax(dm, fabs(d[c]));
      xm = fmax(xm, fabs(xv));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      dm = fmax(dm, __shfl_xor(dm, o));
      xm = fmax(xm, __shfl_xor(xm, o));
    }
    __syncthreads();
    if (dm <= g.refine_rtol * xm) {
      conv = true;
      break;
    }
  }
  return conv;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Factor of the local Robin matrix of kappa^m (eq:mrc1 with zero data), stored for MPM-2P.
template <int MF>
__global__ void __launch_bounds__(64) k_line_factor(Geo g, const double* __restrict__ kap, double* __restrict__ fac,
                                                    int32_t* err, const RunTab* __restrict__ rt) {
  {
    const int64_t wo = ws_off(rt);
    kap = at_off(kap, wo);
    fac = at_off(fac, wo);
    err = at_off(err, wo);
  }
  constexpr int NC = Cap<MF>::NC;
  __shared__ double kl[NC], tE[NC], tN[NC], dg[NC];
  const int sub = xcd_sub(g.nsub);
  const int I = sub % g.Sx, J = sub / g.Sx;
  LB<MF> L;
  load_tile2(g, I, J, kap, kl);
  __syncthreads();
  fill_trans(g, I, J, kl, 0, tE, tN, dg);
  const LineW W{tE, tN, dg, g.xfast, g.band, 0};
  bool ok = true;
  lb_factor<MF>(g, W, L, fac + efac_off<MF>(g, sub), ok);
  if (!ok && L.lane == 0) set_error(err, ERR_NOTSPD);
}

// ---------------------------------------------------------------------------------------------
// MRCM basis (eq:mrc_homogeneous, eq:mrc_non_homogeneous) of a subdomain with more lines than
// the matrix-core kernel takes: the line-block inverses of the local Robin matrix A of
// kappa^m (kept for MPM-2P), then A^-1 applied to the unit vector of each boundary face's
// cell, which gives column f of the Robin-to-flux map S = W T - W T (E^T A^-1 E) W T, and to the
// non-homogeneous right-hand side r0, which gives the boundary fluxes h = W T (E^T A^-1 r0 - r_D);
// then the interface block and its right-hand side. One wavefront per subdomain.
template <int MF>
__global__ void __launch_bounds__(64) k_basis_lines(Geo g, const double* __restrict__ kap,
                                                    const double* __restrict__ q, double* __restrict__ Sg,
                                                    double* __restrict__ hg, double* __restrict__ leafK, LeafOut lo,
                                                    double* __restrict__ fac, int32_t* err,
                                                    const RunTab* __restrict__ rt) {
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
  constexpr int NC = Cap<MF>::NC, NB = Cap<MF>::NB;
  __shared__ double kl[NC], tE[NC], tN[NC], dg[NC], x[NC], wsh[NB], hsh[NB];
  const int sub = xcd_sub(g.nsub);
  const int I = sub % g.Sx, J = sub / g.Sx;
  const int n = g.nc, nb = g.nb;
  load_tile2(g, I, J, kap, kl);
  __syncthreads();
  fill_trans(g, I, J, kl, 0, tE, tN, dg);
  const LineW W{tE, tN, dg, g.xfast, g.band, 0};
  LB<MF> L;
  double* Es = fac + efac_off<MF>(g, sub);
  bool ok = true;
  lb_factor<MF>(g, W, L, Es, ok);   // read back by lb_solve after the barrier below
  if (!ok && L.lane == 0) set_error(err, ERR_NOTSPD);
  for (int fi = threadIdx.x; fi < nb; fi += 64) {
    const BFace f = bface(g, I, J, fi);
    wsh[fi] = f.flen * bface_trans(g, f, kl[loc_index(g, f.i, f.j)]);
  }
  for (int c = threadIdx.x; c < n; c += 64) {
    int i, j;
    loc_ij(g, c, &i, &j);
    x[c] = basis_rhs0(g, I, J, c, kl, q[gcell2(g, I, J, i, j)]);
  }
  __syncthreads();
  lb_solve<MF>(g, W, L, Es, x);
  for (int f = threadIdx.x; f < nb; f += 64) {
    const BFace bf = bface(g, I, J, f);
    const double rD = bf.kind == FACE_DIR ? bf.value : 0.0;
    const double h = bf.kind == FACE_NEU ? 0.0 : wsh[f] * (x[loc_index(g, bf.i, bf.j)] - rD);
    hsh[f] = h;
    hg[size_t(sub) * nb + f] = h;
  }
  double* Ss = Sg + size_t(sub) * smap_doubles(nb);
#pragma unroll 1
  for (int f = 0; f < nb; ++f) {
    __syncthreads();
    const BFace bf = bface(g, I, J, f);
    const int cf = loc_index(g, bf.i, bf.j);
    for (int c = threadIdx.x; c < n; c += 64) x[c] = c == cf ? 1.0 : 0.0;
    __syncthreads();
    lb_solve<MF>(g, W, L, Es, x);
    for (int fr = threadIdx.x; fr < nb; fr += 64) {
      const BFace br = bface(g, I, J, fr);
      if (smap_owner(nb, fr, f))
        Ss[smap_at(nb, fr, f)] = (fr == f ? wsh[f] : 0.0) - wsh[fr] * x[loc_index(g, br.i, br.j)] * wsh[f];
    }
  }
  __syncthreads();
  basis_iface_block(g, I, J, sub, kl, Ss, hsh, leafK, lo);
}

// ---------------------------------------------------------------------------------------------
// Tiles of one subdomain with a one-cell halo (corners excluded), loaded with every global
// read issued before the first use: conductivities kappa^n and kappa^m at
// T[(j + 1) * (mx + 2) + i + 1] and the previous velocity on the subdomain's faces go to LDS
// (ux [my][mx + 1], uy [my + 1][mx]); q stays in registers, qc[s] for local cell
// threadIdx.x + 64 s. Tiles of up to 16^2 cells have every read in flight at once; 32^2 tiles
// (four times the values) are copied through LDS in a plain loop instead, which keeps the
// values in flight within the register budget.
template <int MF>
__device__ __forceinline__ void load_halo_tiles(const Geo& g, int I, int J, const double* __restrict__ kap_n,
                                                const double* __restrict__ kap_m, const double* __restrict__ uxm,
                                                const double* __restrict__ uym, const double* __restrict__ q,
                                                double* kn, double* km, double* ux, double* uy,
                                                double (&qc)[Cap<MF>::CPL]) {
  constexpr int NH = (Cap<MF>::HALO + 63) / 64, NF = (Cap<MF>::NF + 63) / 64, CPL = Cap<MF>::CPL;
  const int TW = g.mx + 2, nh = TW * (g.my + 2);
  const int nfx = g.my * (g.mx + 1), nfy = (g.my + 1) * g.mx;
  if constexpr (MF == 32) {
    constexpr int U = 4;   // entries per thread in flight at a time
    for (int e0 = threadIdx.x; e0 < nh; e0 += 64 * U) {
      double a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 64 * u;
        const int ti = e % TW - 1, tj = e / TW - 1;
        const int gi = I * g.mx + ti, gj = J * g.my + tj;
        const bool edge_i = ti < 0 || ti >= g.mx, edge_j = tj < 0 || tj >= g.my;
        const bool ok = e < nh && !(edge_i && edge_j) && gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny;
        const int gc = ok ? gj * g.nx + gi : 0;
        a[u] = kap_n[gc];
        b[u] = kap_m[gc];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 64 * u;
        if (e < nh) {
          kn[e] = a[u];
          km[e] = b[u];
        }
      }
    }
    for (int e0 = threadIdx.x; e0 < nfx || e0 < nfy; e0 += 64 * U) {
      double fx[U], fy[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 64 * u;
        const int ex = e < nfx ? e : 0, ey = e < nfy ? e : 0;
        fx[u] = uxm[(J * g.my + ex / (g.mx + 1)) * (g.nx + 1) + I * g.mx + ex % (g.mx + 1)];
        fy[u] = uym[(J * g.my + ey / g.mx) * g.nx + I * g.mx + ey % g.mx];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 64 * u;
        if (e < nfx) ux[e] = fx[u];
        if (e < nfy) uy[e] = fy[u];
      }
    }
#pragma unroll
    for (int s = 0; s < CPL; ++s) {
      const int c = threadIdx.x + 64 * s;
      int i, j;
      loc_ij(g, c < g.nc ? c : 0, &i, &j);
      qc[s] = q[(J * g.my + j) * g.nx + I * g.mx + i];
    }
  } else {
    double a[NH], b[NH], fx[NF], fy[NF];
#pragma unroll
    for (int s = 0; s < NH; ++s) {
      const int e = threadIdx.x + 64 * s;
      const int ti = e % TW - 1, tj = e / TW - 1;
      const int gi = I * g.mx + ti, gj = J * g.my + tj;
      const bool edge_i = ti < 0 || ti >= g.mx, edge_j = tj < 0 || tj >= g.my;
      const bool ok = e < nh && !(edge_i && edge_j) && gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny;
      const int gc = ok ? gj * g.nx + gi : 0;
      a[s] = kap_n[gc];
      b[s] = kap_m[gc];
    }
#pragma unroll
    for (int s = 0; s < NF; ++s) {
      const int e = threadIdx.x + 64 * s;
      const int ex = e < nfx ? e : 0, ey = e < nfy ? e : 0;
      fx[s] = uxm[(J * g.my + ex / (g.mx + 1)) * (g.nx + 1) + I * g.mx + ex % (g.mx + 1)];
      fy[s] = uym[(J * g.my + ey / g.mx) * g.nx + I * g.mx + ey % g.mx];
    }
#pragma unroll
    for (int s = 0; s < CPL; ++s) {
      const int c = threadIdx.x + 64 * s;
      int i, j;
      loc_ij(g, c < g.nc ? c : 0, &i, &j);
      qc[s] = q[(J * g.my + j) * g.nx + I * g.mx + i];
    }
#pragma unroll
    for (int s = 0; s < NH; ++s) {
      const int e = threadIdx.x + 64 * s;
      if (e < nh) {
        kn[e] = a[s];
        km[e] = b[s];
      }
    }
#pragma unroll
    for (int s = 0; s < NF; ++s) {
      const int e = threadIdx.x + 64 * s;
      if (e < nfx) ux[e] = fx[s];
      if (e < nfy) uy[e] = fy[s];
    }
  }
  __syncthreads();
}

// v = (t^n / t^m) u~^m on every face of the tile, in place of u~^m (halo tiles as above): the
// harmonic-transmissibility ratio with the neighbour cell (across Gamma too), kappa^n / kappa^m
// of the cell on the physical boundary. One ratio per face, kept in rx, ry when given. No
// barrier.
__device__ __forceinline__ void mpm_face_v(const Geo& g, int I, int J, const double* knt, const double* kmt,
                                           double* uxs, double* uys, double* rx = nullptr, double* ry = nullptr) {
  const int TW = g.mx + 2;
  const int nfx = g.my * (g.mx + 1), nfy = (g.my + 1) * g.mx;
  for (int e = threadIdx.x; e < nfx; e += 64) {
    const int j = e / (g.mx + 1), i = e - j * (g.mx + 1);   // face between local cells i-1 and i
    const int gi = I * g.mx + i;
    const int cl = (j + 1) * TW + i, cr = cl + 1;          // halo indices of the two cells
    double ratio;
    if (gi > 0 && gi < g.nx) ratio = harm_ratio(knt[cr], knt[cl], kmt[cr], kmt[cl]);
    else if (gi == 0) ratio = knt[cr] / kmt[cr];
    else ratio = knt[cl] / kmt[cl];
    uxs[e] = ratio * uxs[e];
    if (rx) rx[e] = ratio;
  }
  for (int e = threadIdx.x; e < nfy; e += 64) {
    const int j = e / g.mx, i = e - j * g.mx;                 // face between local cells j-1 and j
    const int gj = J * g.my + j;
    const int cb = j * TW + i + 1, ct = cb + TW;
    double ratio;
    if (gj > 0 && gj < g.ny) ratio = harm_ratio(knt[ct], knt[cb], kmt[ct], kmt[cb]);
    else if (gj == 0) ratio = knt[ct] / kmt[ct];
    else ratio = knt[cb] / kmt[cb];
    uys[e] = ratio * uys[e];
    if (ry) ry[e] = ratio;
  }
}

// Right-hand side of the trivial-Robin problem at local cell (i, j): |c| q minus the outflow
// of v through the cell's faces (v on the face tiles), z on Neumann faces.
__device__ __forceinline__ double mpm_rhs_cell(const Geo& g, int I, int J, int i, int j, double qv,
                                               const double* vx, const double* vy) {
  const int gi = I * g.mx + i, gj = J * g.my + j;
  double r = g.hx * g.hy * qv;
  {
    const double v = vx[j * (g.mx + 1) + i];
    if (gi > 0) {
      r -= g.hy * (-v);
    } else {
      BFace f = bface(g, I, J, j);
      r -= f.kind == FACE_NEU ? f.flen * f.value : g.hy * (-v);
    }
  }
  {
    const double v = vx[j * (g.mx + 1) + i + 1];
    if (gi < g.nx - 1) {
      r -= g.hy * v;
    } else {
      BFace f = bface(g, I, J, g.my + j);
      r -= f.kind == FACE_NEU ? f.flen * f.value : g.hy * v;
    }
  }
  {
    const double v = vy[j * g.mx + i];
    if (gj > 0) {
      r -= g.hx * (-v);
    } else {
      BFace f = bface(g, I, J, 2 * g.my + i);
      r -= f.kind == FACE_NEU ? f.flen * f.value : g.hx * (-v);
    }
  }
  {
    const double v = vy[(j + 1) * g.mx + i];
    if (gj < g.ny - 1) {
      r -= g.hx * v;
    } else {
      BFace f = bface(g, I, J, 2 * g.my + g.mx + i);
      r -= f.kind == FACE_NEU ? f.flen * f.value : g.hx * v;
    }
  }
  return r;
}

// Outward v on boundary face bf of the subdomain (0 on Neumann faces).
__device__ __forceinline__ double mpm_vbnd_face(const Geo& g, const BFace& bf, const double* vx, const double* vy) {
  if (bf.kind == FACE_NEU) return 0.0;
  if (bf.side == 0) return -vx[bf.j * (g.mx + 1) + bf.i];
  if (bf.side == 1) return vx[bf.j * (g.mx + 1) + bf.i + 1];
  if (bf.side == 2) return -vy[bf.j * g.mx + bf.i];
  return vy[(bf.j + 1) * g.mx + bf.i];
}

// The geometry with the subdomain shape as compile-time constants for FX x FX subdomains (FX =
// 0: as given), so that the index arithmetic of the local kernels folds.
// Blocks in flight in the ring solve of the fixed-shape local kernels.
#ifndef MPM_RING_D
#define MPM_RING_D 4
#endif
constexpr int RING_D = MPM_RING_D;

template <int FX>
__device__ __forceinline__ Geo fix_geo(Geo g) {
  if constexpr (FX > 0) {
    g.mx = FX;
    g.my = FX;
    g.nc = FX * FX;
    g.band = FX;
    g.xfast = 1;
    g.nb = 4 * FX;
  }
  return g;
}

// ---------------------------------------------------------------------------------------------
// Wavefronts per SIMD the fixed-shape FP64 local solve of 16^2 subdomains is compiled for: four
// (at most 128 registers), so that a 1024^2 grid's 4096 subdomains are resident at once.
template <int MF, typename T, int FX>
constexpr int LOCAL_WAVES = (MF == 16 && FX == 16 && sizeof(T) == 8) ? 4 : 1;

// MPM-2P trivial-Robin local solve (eq:mpm_tf_3 with the kappa^m basis): right-hand side
// |c| q - sum_{non-Neumann faces} |f| v_f - sum_{Neumann faces} |f| z with
// v_f = (t^n_f / t^m_f) u~^m_f; zero Dirichlet and Robin data. Outputs the boundary fluxes
// h = W T delta p on Robin/Dirichlet faces, the boundary values of v and the interface
// right-hand side B^T h. The kept inverse blocks and all tiles are requested at entry.
// LDS is reused as the steps retire (kappa^n halo -> line couplings, x-faces -> solution,
// y-faces -> h), about 9.5 KB per subdomain: registers, not LDS, bound the subdomains per CU.
// With T = float the kept blocks are FP32 (all lines in registers, up to 16) and the solve is
// refined in FP64 against the full line form of the matrix.
template <int MF, int NL, typename T, int FX>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(LOCAL_WAVES<MF, T, FX>)))
k_mpm_local_lb(Geo g0, const double* __restrict__ kap_n, const double* __restrict__ kap_m,
               const double* __restrict__ uxm, const double* __restrict__ uym, const double* __restrict__ q,
               const T* __restrict__ fac, double* __restrict__ hg, double* __restrict__ vbnd, LeafOut lo,
               int32_t* err, const RunTab* __restrict__ rt) {
  constexpr bool F32 = sizeof(T) == 4;
  const Geo g = fix_geo<FX>(g0);
  {
    const int64_t wo = ws_off(rt);
    err = at_off(err, wo);
    kap_n = at_off(kap_n, wo);
    kap_m = at_off(kap_m, wo);
    uxm = at_off(uxm, wo);
    uym = at_off(uym, wo);
    q = at_off(q, wo);
    fac = at_off(fac, wo);
    hg = at_off(hg, wo);
    vbnd = at_off(vbnd, wo);
    lo = leaf_at(lo, wo);
  }
  static_assert(!F32 || MF <= 16, "the precision form takes lines of at most 16 cells");
  constexpr int CPL = Cap<MF>::CPL;
  // halo tiles of the two conductivities, the x- and y-face tiles (later: line couplings,
  // solution, boundary fluxes)
  __shared__ double knt[Cap<MF>::HALO], kmt[Cap<MF>::HALO], uxs[Cap<MF>::NF], uys[Cap<MF>::NF];
  __shared__ double xtra[F32 ? 3 * 256 + 768 : 1];   // precision form: tE, tN, dg, refinement scratch
  const int sub = xcd_sub(g.nsub);
  const int I = sub % g.Sx, J = sub / g.Sx;
  const int n = g.nc, nb = g.nb;
  const int TW = g.mx + 2;
  LB<MF> L;
  constexpr int NLR = NL > 0 ? NL : 1;
  constexpr bool RING = !F32 && FX > 0 && NL > 0;   // fixed shape: blocks streamed through a ring
  double E[(F32 || RING) ? 1 : NLR][LB<MF>::EPL];
  double Er[RING ? RING_D : 1][LB<MF>::EPL];
  float Ef[F32 ? 16 : 1][LB<MF>::EPL];
  const T* Es = fac + efac_off<MF>(g, sub);
  if constexpr (F32) lb_load_f32<MF>(L, Es, g.nc / g.band, Ef);
  else if constexpr (RING) lb_ring_load<MF, NL, RING_D>(L, Es, Er);
  else if constexpr (NL > 0) lb_load_reg<MF, NL>(L, Es, E);
  double qc[CPL];
  load_halo_tiles<MF>(g, I, J, kap_n, kap_m, uxm, uym, q, knt, kmt, uxs, uys, qc);
  mpm_face_v(g, I, J, knt, kmt, uxs, uys);
  __syncthreads();
  double rhs[CPL];
#pragma unroll
  for (int s = 0; s < CPL; ++s) {
    const int c = threadIdx.x + 64 * s;
    rhs[s] = 0.0;
    if (c < n) {
      int i, j;
      loc_ij(g, c, &i, &j);
      rhs[s] = mpm_rhs_cell(g, I, J, i, j, qc[s], uxs, uys);
    }
  }
  for (int f = threadIdx.x; f < nb; f += 64)
    vbnd[size_t(sub) * nb + f] = mpm_vbnd_face(g, bface(g, I, J, f), uxs, uys);
  __syncthreads();   // the kappa^n halo and the face tiles are dead from here on
  double* x = uxs;
  double* ty = knt;
#pragma unroll
  for (int s = 0; s < CPL; ++s) {
    const int c = threadIdx.x + 64 * s;
    if (c < n) x[c] = rhs[s];
  }
  auto kmf = [&](int i, int j) { return kmt[(j + 1) * TW + i + 1]; };
  double* tE = xtra;
  double* tN = xtra + 256;
  double* dg = xtra + 512;
  if constexpr (F32) fill_trans_k(g, I, J, kmf, 0, tE, tN, dg);
  else {
    fill_ycoup_k(g, kmf, ty);
    __syncthreads();
  }
  if constexpr (F32) {
    const LineW W{tE, tN, dg, g.xfast, g.band, 0};
    if (!lb_solve_refined<MF>(g, W, L, Ef, x, xtra + 768) && L.lane == 0) set_error(err, ERR_NOCONV);
  } else {
    const LineW W{ty, ty, nullptr, g.xfast, g.band, 0};
    if constexpr (RING) lb_solve_ring<MF, NL, RING_D, true>(W, L, Es, Er, x);
    else if constexpr (NL > 0) lb_solve_regs<MF, NL>(W, L, E, x);
    else lb_solve<MF>(g, W, L, Es, x);
  }
  double* hsh = uys;
  for (int f = threadIdx.x; f < nb; f += 64) {
    BFace bf = bface(g, I, J, f);
    const double km = kmt[(bf.j + 1) * TW + bf.i + 1];
    const double h = bf.kind == FACE_NEU ? 0.0 : bf.flen * bface_trans(g, bf, km) * x[loc_index(g, bf.i, bf.j)];
    hsh[f] = h;
    hg[size_t(sub) * nb + f] = h;
  }
  __syncthreads();
  // interface right-hand side B^T h
  const int nd = sub_ndof(g, I, J);
  for (int a = threadIdx.x; a < nd; a += 64) {
    int f0, cnt;
    dof_faces(g, I, J, a, &f0, &cnt);
    double v = 0.0;
    for (int xx = f0; xx < f0 + cnt; ++xx) {
      BFace ff = bface(g, I, J, xx);
      v += bweight(g, ff, a, kmt[(ff.j + 1) * TW + ff.i + 1]) * hsh[xx];
    }
    leaf_out(lo, sub, a, v);
  }
}

// ---------------------------------------------------------------------------------------------
// First-order term of MPM-2P (eq:mpm_tf_4 with l = 1), after the zeroth-order interface solve
// y and its reconstruction (ubnd = u-hat_0 + v and vbnd = v on the subdomain's boundary
// faces). Per subdomain: delta p_0 from the kept kappa^m blocks with the zeroth-order right-hand
// side and the Robin data r_f = -sgn beta_f U + P of y; the flux u-hat_0 on every face (the mean
// of both sides' reconstructions on Gamma); w = (t^n / t^m - 1) u-hat_0 (0 on Neumann faces);
// then the trivial-Robin problem with source -div w and zero data, whose boundary fluxes h and
// interface right-hand side B^T h go out as for the zeroth order, and w on the boundary faces.
// The reconstruction of the second interface solve adds u-hat_1 + w to ubnd.
template <int MF, int NL, typename T, int FX>   // T: double (the term is FP64 only)
__global__ void __launch_bounds__(64)
k_mpm_first(Geo g0, const double* __restrict__ kap_n, const double* __restrict__ kap_m,
            const double* __restrict__ uxm, const double* __restrict__ uym, const double* __restrict__ q,
            const double* __restrict__ fac, const double* __restrict__ y, const int32_t* __restrict__ sub_dofs,
            const double* __restrict__ ubnd, const double* __restrict__ vbnd, double* __restrict__ hg,
            double* __restrict__ wbnd, LeafOut lo, const RunTab* __restrict__ rt) {
  static_assert(sizeof(T) == 8, "FP64 only");
  static_assert(MF <= 16, "lines of at most 16 cells");
  const Geo g = fix_geo<FX>(g0);
  {
    const int64_t wo = ws_off(rt);
    kap_n = at_off(kap_n, wo);
    kap_m = at_off(kap_m, wo);
    uxm = at_off(uxm, wo);
    uym = at_off(uym, wo);
    q = at_off(q, wo);
    fac = at_off(fac, wo);
    y = at_off(y, wo);
    sub_dofs = at_off(sub_dofs, wo);
    ubnd = at_off(ubnd, wo);
    vbnd = at_off(vbnd, wo);
    hg = at_off(hg, wo);
    wbnd = at_off(wbnd, wo);
    lo = leaf_at(lo, wo);
  }
  __shared__ double knt[18 * 18], kmt[18 * 18], uxs[16 * 17], uys[17 * 16], rx[16 * 17], ry[17 * 16];
  __shared__ double wx[16 * 17], wy[17 * 16], x[256], ty[256], rr[64], hsh[64];
  const int sub = xcd_sub(g.nsub);
  const int I = sub % g.Sx, J = sub / g.Sx;
  const int n = g.nc, nb = g.nb, TW = g.mx + 2;
  LB<MF> L;
  constexpr int NLR = NL > 0 ? NL : 1;
  double E[NLR][LB<MF>::EPL];
  const double* Es = fac + efac_off<MF>(g, sub);
  if constexpr (NL > 0) lb_load_reg<MF, NL>(L, Es, E);
  double qc[4];
  load_halo_tiles<MF>(g, I, J, kap_n, kap_m, uxm, uym, q, knt, kmt, uxs, uys, qc);
  mpm_face_v(g, I, J, knt, kmt, uxs, uys, rx, ry);
  auto kmf = [&](int i, int j) { return kmt[(j + 1) * TW + i + 1]; };
  fill_ycoup_k(g, kmf, ty);
  // Robin data of the zeroth-order interface solution on Gamma faces
  for (int f = threadIdx.x; f < nb; f += 64) {
    const BFace bf = bface(g, I, J, f);
    double r = 0.0;
    if (bf.kind == FACE_ROB) r = robin_datum(g, I, J, bf, kmf(bf.i, bf.j), sub_dofs + size_t(sub) * g.ndmax, y);
    rr[f] = r;
  }
  __syncthreads();
  const LineW W{ty, ty, nullptr, g.xfast, g.band, 0};
  // delta p_0: the zeroth-order right-hand side plus |f| t_f r_f on the Robin faces
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int c = threadIdx.x + 64 * s;
    if (c >= n) continue;
    int i, j;
    loc_ij(g, c, &i, &j);
    double rhs = mpm_rhs_cell(g, I, J, i, j, qc[s], uxs, uys);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bool on = (t == 0 && i == 0) || (t == 1 && i == g.mx - 1) || (t == 2 && j == 0) ||
                      (t == 3 && j == g.my - 1);
      if (!on) continue;
      const int f = t == 0 ? j : t == 1 ? g.my + j : t == 2 ? 2 * g.my + i : 2 * g.my + g.mx + i;
      const BFace bf = bface(g, I, J, f);
      if (bf.kind == FACE_ROB) rhs += bf.flen * bface_trans(g, bf, kmf(i, j)) * rr[f];
    }
    x[c] = rhs;
  }
  __syncthreads();
  if constexpr (NL > 0) lb_solve_regs<MF, NL>(W, L, E, x);
  else lb_solve<MF>(g, W, L, Es, x);
  // u-hat_0 on every face of the tile and w = (ratio - 1) u-hat_0 (+x / +y orientation)
  auto u0_bnd = [&](int f) -> double {   // outward u-hat_0 on boundary face f (mean on Gamma)
    const BFace bf = bface(g, I, J, f);
    const double own = ubnd[size_t(sub) * nb + f] - vbnd[size_t(sub) * nb + f];
    if (bf.kind != FACE_ROB) return own;
    int ns, nf;
    if (bf.side == 0) { ns = sub - 1; nf = g.my + bf.k; }
    else if (bf.side == 1) { ns = sub + 1; nf = bf.k; }
    else if (bf.side == 2) { ns = sub - g.Sx; nf = 2 * g.my + g.mx + bf.k; }
    else { ns = sub + g.Sx; nf = 2 * g.my + bf.k; }
    const double other = ubnd[size_t(ns) * nb + nf] - vbnd[size_t(ns) * nb + nf];
    return 0.5 * (own - other);
  };
  const int nfx = g.my * (g.mx + 1), nfy = (g.my + 1) * g.mx;
  for (int e = threadIdx.x; e < nfx; e += 64) {
    const int j = e / (g.mx + 1), i = e - j * (g.mx + 1);
    double w;
    if (i > 0 && i < g.mx) {
      const int cl = loc_index(g, i - 1, j), cr = loc_index(g, i, j);
      const double u0 = harm_trans(kmf(i - 1, j), kmf(i, j), g.hx) * (x[cl] - x[cr]);
      w = (rx[e] - 1.0) * u0;
    } else {
      const int f = i == 0 ? j : g.my + j;
      const BFace bf = bface(g, I, J, f);
      const double u0 = i == 0 ? -u0_bnd(f) : u0_bnd(f);
      w = bf.kind == FACE_NEU ? 0.0 : (rx[e] - 1.0) * u0;
    }
    wx[e] = w;
  }
  for (int e = threadIdx.x; e < nfy; e += 64) {
    const int j = e / g.mx, i = e - j * g.mx;
    double w;
    if (j > 0 && j < g.my) {
      const int cb = loc_index(g, i, j - 1), ct = loc_index(g, i, j);
      const double u0 = harm_trans(kmf(i, j - 1), kmf(i, j), g.hy) * (x[cb] - x[ct]);
      w = (ry[e] - 1.0) * u0;
    } else {
      const int f = j == 0 ? 2 * g.my + i : 2 * g.my + g.mx + i;
      const BFace bf = bface(g, I, J, f);
      const double u0 = j == 0 ? -u0_bnd(f) : u0_bnd(f);
      w = bf.kind == FACE_NEU ? 0.0 : (ry[e] - 1.0) * u0;
    }
    wy[e] = w;
  }
  __syncthreads();
  // first-order problem: source -div w, zero data
  for (int c = threadIdx.x; c < n; c += 64) {
    int i, j;
    loc_ij(g, c, &i, &j);
    const double out = g.hy * (wx[j * (g.mx + 1) + i + 1] - wx[j * (g.mx + 1) + i]) +
                       g.hx * (wy[(j + 1) * g.mx + i] - wy[j * g.mx + i]);
    x[c] = -out;
  }
  __syncthreads();
  if constexpr (NL > 0) lb_solve_regs<MF, NL>(W, L, E, x);
  else lb_solve<MF>(g, W, L, Es, x);
  for (int f = threadIdx.x; f < nb; f += 64) {
    const BFace bf = bface(g, I, J, f);
    const double h = bf.kind == FACE_NEU ? 0.0 : bf.flen * bface_trans(g, bf, kmf(bf.i, bf.j)) *
                                                     x[loc_index(g, bf.i, bf.j)];
    hsh[f] = h;
    hg[size_t(sub) * nb + f] = h;
    double wo;
    if (bf.side == 0) wo = -wx[bf.j * (g.mx + 1) + bf.i];
    else if (bf.side == 1) wo = wx[bf.j * (g.mx + 1) + bf.i + 1];
    else if (bf.side == 2) wo = -wy[bf.j * g.mx + bf.i];
    else wo = wy[(bf.j + 1) * g.mx + bf.i];
    wbnd[size_t(sub) * nb + f] = wo;
  }
  __syncthreads();
  const int nd = sub_ndof(g, I, J);
  for (int a = threadIdx.x; a < nd; a += 64) {
    int f0, cnt;
    dof_faces(g, I, J, a, &f0, &cnt);
    double v = 0.0;
    for (int xx = f0; xx < f0 + cnt; ++xx) {
      const BFace ff = bface(g, I, J, xx);
      v += bweight(g, ff, a, kmf(ff.i, ff.j)) * hsh[xx];
    }
    leaf_out(lo, sub, a, v);
  }
}

// ---------------------------------------------------------------------------------------------
// Downscaling (eq. mpm_upd): all-Neumann problem with conductivity kap_s per subdomain, the
// mean of both sides' boundary fluxes on Gamma, the own flux on the physical boundary, the
// first cell pinned. The data are made compatible first: the rounding-level defect (net
// outflow minus source, zero for the exact fluxes) is spread over the cells' sources, so that it
// does not leave through the pinned cell's faces alone. Writes the velocity on the faces the
// subdomain owns, the largest outflow rate per cell volume and the inflow through the physical
// boundary.
// With T = float (MPM-2P steps of the precision form; store = 0) the blocks are FP32 and the
// solve is refined in FP64. The blocks are requested at entry.
template <int MF, int NL, typename T, int FX>
__global__ void __launch_bounds__(64)
k_downscale_lb(Geo g0, const double* __restrict__ kap_s, const double* __restrict__ q,
               const double* __restrict__ ubnd, double* __restrict__ ux, double* __restrict__ uy,
               double* __restrict__ red_rate, double* __restrict__ red_qin, T* __restrict__ Escr,
               T* __restrict__ Ekeep, const int32_t* __restrict__ flag, int store, int32_t* err, const RunTab* __restrict__ rt) {
  constexpr bool F32 = sizeof(T) == 4;
  const Geo g = fix_geo<FX>(g0);
  if constexpr (FX > 0) store = 0;   // fixed-shape instances serve the MPM-2P steps only
  {
    const int64_t wo = ws_off(rt);
    kap_s = at_off(kap_s, wo);
    q = at_off(q, wo);
    ubnd = at_off(ubnd, wo);
    ux = at_off(ux, wo);
    uy = at_off(uy, wo);
    red_rate = at_off(red_rate, wo);
    red_qin = at_off(red_qin, wo);
    Escr = at_off(Escr, wo);
    Ekeep = at_off(Ekeep, wo);
    flag = at_off(flag, wo);
    err = at_off(err, wo);
  }
  static_assert(!F32 || MF <= 16, "the precision form takes lines of at most 16 cells");
  constexpr int NC = Cap<MF>::NC, CPL = Cap<MF>::CPL;
  // the conductivity tile is dead once the weights are built and then holds the solution
  __shared__ double kl[NC], w[Cap<MF>::NB], tE[NC], tN[NC], dg[NC];
  __shared__ double wsh[F32 ? 768 : 1];
  double* x = kl;
  const int sub = xcd_sub(g.nsub);
  const int I = sub % g.Sx, J = sub / g.Sx;
  const int n = g.nc, nb = g.nb;
  LB<MF> L;
  const size_t eoff = efac_off<MF>(g, sub);
  T* Es = (!store && flag[sub]) ? Escr + eoff : Ekeep + eoff;
  constexpr int NLR = NL > 0 ? NL : 1;
  constexpr bool RING = !F32 && FX > 0 && NL > 0;   // fixed shape (store = 0): ring of blocks
  double E[(F32 || RING) ? 1 : NLR][LB<MF>::EPL];
  double Er[RING ? RING_D : 1][LB<MF>::EPL];
  float Ef[F32 ? 16 : 1][LB<MF>::EPL];
  if constexpr (F32) lb_load_f32<MF>(L, Es, g.nc / g.band, Ef);
  else if constexpr (RING) lb_ring_load<MF, NL, RING_D>(L, Es, Er);
  else if constexpr (NL > 0) {
    if (!store) lb_load_reg<MF, NL>(L, Es, E);
  }
  load_tile2(g, I, J, kap_s, kl);
  double defect = 0.0;   // net outflow minus source
  for (int f = threadIdx.x; f < nb; f += blockDim.x) {
    BFace bf = bface(g, I, J, f);
    double u = ubnd[size_t(sub) * nb + f];
    if (bf.kind == FACE_ROB) {
      int ns, nf;
      if (bf.side == 0) { ns = sub - 1; nf = g.my + bf.k; }
      else if (bf.side == 1) { ns = sub + 1; nf = bf.k; }
      else if (bf.side == 2) { ns = sub - g.Sx; nf = 2 * g.my + g.mx + bf.k; }
      else { ns = sub + g.Sx; nf = 2 * g.my + bf.k; }
      u = 0.5 * (u - ubnd[size_t(ns) * nb + nf]);
    }
    w[f] = u;
    defect += (f < 2 * g.my ? g.hy : g.hx) * u;
  }
  double qc[CPL];
#pragma unroll
  for (int s = 0; s < CPL; ++s) {
    const int c = threadIdx.x + 64 * s;
    int i, j;
    loc_ij(g, c < n ? c : 0, &i, &j);
    qc[s] = q[gcell2(g, I, J, i, j)];
    if (c < n) defect -= g.hx * g.hy * qc[s];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) defect += __shfl_xor(defect, o);
  const double shift = defect / n;   // added to every cell's |c| q
  __syncthreads();
  fill_trans(g, I, J, kl, 1, tE, tN, dg);
#pragma unroll
  for (int s = 0; s < CPL; ++s) {
    const int c = threadIdx.x + 64 * s;
    if (c >= n) continue;
    int i, j;
    loc_ij(g, c, &i, &j);
    double r = g.hx * g.hy * qc[s] + shift;
    if (i == 0) r -= g.hy * w[j];
    if (i == g.mx - 1) r -= g.hy * w[g.my + j];
    if (j == 0) r -= g.hx * w[2 * g.my + i];
    if (j == g.my - 1) r -= g.hx * w[2 * g.my + g.mx + i];
    x[c] = c == 0 ? 0.0 : r;
  }
  __syncthreads();
  const LineW W{tE, tN, dg, g.xfast, g.band, 1};
  if constexpr (F32) {
    if (!lb_solve_refined<MF>(g, W, L, Ef, x, wsh) && L.lane == 0) set_error(err, ERR_NOCONV);
  } else {
    if constexpr (!RING) {
      if (store) {
        bool ok = true;
        lb_factor<MF>(g, W, L, Es, ok);
        if (!ok && L.lane == 0) set_error(err, ERR_NOTSPD);
        __syncthreads();   // the lower-triangle entries come from other lanes' stores
        if constexpr (NL > 0) lb_load_reg<MF, NL>(L, Es, E);
      }
    }
    if constexpr (RING) {
      // nothing of the flux phase is computed ahead of the solve (it would stay live across it)
      __builtin_amdgcn_sched_barrier(0);
      lb_solve_ring<MF, NL, RING_D, false>(W, L, Es, Er, x);
      __builtin_amdgcn_sched_barrier(0);
    } else if constexpr (NL > 0) lb_solve_regs<MF, NL>(W, L, E, x);
    else lb_solve<MF>(g, W, L, Es, x);
  }
  double rate = 0.0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    int i, j;
    loc_ij(g, c, &i, &j);
    const int gi = I * g.mx + i, gj = J * g.my + j;
    const double pc = x[c];
    double uW, uE, uS, uN;
    // interior faces: the pinned cell's couplings are part of the flux field (tE, tN hold them)
    if (i > 0) { const int d = loc_index(g, i - 1, j); uW = tE[d] / g.hy * (x[d] - pc); }
    else uW = -w[j];
    if (i < g.mx - 1) uE = tE[c] / g.hy * (pc - x[loc_index(g, i + 1, j)]);
    else uE = w[g.my + j];
    if (j > 0) { const int d = loc_index(g, i, j - 1); uS = tN[d] / g.hx * (x[d] - pc); }
    else uS = -w[2 * g.my + i];
    if (j < g.my - 1) uN = tN[c] / g.hx * (pc - x[loc_index(g, i, j + 1)]);
    else uN = w[2 * g.my + g.mx + i];
    ux[gj * (g.nx + 1) + gi] = uW;
    uy[gj * g.nx + gi] = uS;
    if (gi == g.nx - 1) ux[gj * (g.nx + 1) + gi + 1] = uE;
    if (gj == g.ny - 1) uy[(gj + 1) * g.nx + gi] = uN;
    const double out = g.hy * (fmax(uE, 0.0) + fmax(-uW, 0.0)) + g.hx * (fmax(uN, 0.0) + fmax(-uS, 0.0));
    // a non-finite velocity makes the rate infinite (fmax alone would drop a NaN), which the
    // time-step reduction reports
    rate = finite_d(uW + uE + uS + uN) ? fmax(rate, out / (g.hx * g.hy)) : __builtin_inf();
  }
  double qin = 0.0;
  for (int f = threadIdx.x; f < nb; f += blockDim.x) {
    BFace bf = bface(g, I, J, f);
    if (bf.kind != FACE_ROB) qin += bf.flen * fmax(-w[f], 0.0);
  }
  // one wavefront: butterfly reductions
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    rate = fmax(rate, __shfl_xor(rate, o));
    qin += __shfl_xor(qin, o);
  }
  if (threadIdx.x == 0) {
    red_rate[sub] = rate;
    red_qin[sub] = qin;
  }
}

// ---------------------------------------------------------------------------------------------
// Neumann inverse blocks of kappa^n for the subdomains whose conductivity tile changed since the
// last MRCM update (listed by the conductivity kernel; elsewhere the kept kappa^m blocks are
// exact). A fixed grid walks the list. Runs on a second stream, overlapped with the interface
// solve. Blocks of lines of 32 cells are spread over the four wavefronts of a workgroup (NT =
// 256 lanes: four entries each instead of sixteen), the others over one wavefront.
template <int MF, typename T, int NT>
__global__ void __launch_bounds__(NT)
k_ds_factor(Geo g, const double* __restrict__ kap_n, T* __restrict__ Escr, const int32_t* __restrict__ list,
            const int32_t* __restrict__ count, int32_t* err, const RunTab* __restrict__ rt) {
  constexpr int NC = Cap<MF>::NC;
  __shared__ double kl[NC], tE[NC], tN[NC], dg[NC];
  {
    const int64_t wo = ws_off(rt);
    kap_n = at_off(kap_n, wo);
    Escr = at_off(Escr, wo);
    list = at_off(list, wo);
    count = at_off(count, wo);
    err = at_off(err, wo);
  }
  LB<MF, false, NT> L;
  const int n = min(*count, g.nsub);
#pragma unroll 1
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int sub = list[it];
    if (sub < 0 || sub >= g.nsub) continue;
    const int I = sub % g.Sx, J = sub / g.Sx;
    load_tile2(g, I, J, kap_n, kl);
    __syncthreads();
    fill_trans(g, I, J, kl, 1, tE, tN, dg);
    const LineW W{tE, tN, dg, g.xfast, g.band, 1};
    bool ok = true;
    lb_factor<MF>(g, W, L, Escr + efac_off<MF>(g, sub), ok);
    if (!ok && L.lane == 0) set_error(err, ERR_NOTSPD);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------

// Lines padded to MF cells: 8 for lines of up to 8, 16 up to 16, 32 up to 32 (the plan refuses
// longer lines).
static int line_mf(const Geo& g) { return g.band <= 8 ? 8 : g.band <= 16 ? 16 : 32; }

void launch_basis_lines(hipStream_t st, const Geo& g, const double* kap, const double* q, double* S, double* h,
                        double* leafK, LeafOut lo, double* fac, int32_t* err, Runs rt) {
  const dim3 grid(g.nsub, 1, runs_of(rt));
  if (line_mf(g) == 8)
    hipLaunchKernelGGL(k_basis_lines<8>, grid, dim3(64), 0, st, g, kap, q, S, h, leafK, lo, fac, err, rt.tab);
  else if (line_mf(g) == 16)
    hipLaunchKernelGGL(k_basis_lines<16>, grid, dim3(64), 0, st, g, kap, q, S, h, leafK, lo, fac, err, rt.tab);
  else hipLaunchKernelGGL(k_basis_lines<32>, grid, dim3(64), 0, st, g, kap, q, S, h, leafK, lo, fac, err, rt.tab);
}

void launch_line_factor(hipStream_t st, const Geo& g, const double* kap, double* fac, int32_t* err, Runs rt) {
  const dim3 grid(g.nsub, 1, runs_of(rt));
  if (line_mf(g) == 8) hipLaunchKernelGGL(k_line_factor<8>, grid, dim3(64), 0, st, g, kap, fac, err, rt.tab);
  else if (line_mf(g) == 16) hipLaunchKernelGGL(k_line_factor<16>, grid, dim3(64), 0, st, g, kap, fac, err, rt.tab);
  else hipLaunchKernelGGL(k_line_factor<32>, grid, dim3(64), 0, st, g, kap, fac, err, rt.tab);
}

// line length padded to MF in {8, 16, 32}; the solve keeps the blocks in registers for the
// common line counts 8 and 16, and square 8^2 / 16^2 subdomains get compile-time shapes; lines
// of 17 to 32 cells (WIDE kernels only) stream their blocks from memory
#define MPM_LB_LAUNCH(KERNEL, ...) \
  hipLaunchKernelGGL((KERNEL), dim3(g.nsub, 1, runs_of(rt)), dim3(64), 0, st, __VA_ARGS__)
#define MPM_LB_DISPATCH16(KERNEL, FIXOK, ...)                                                      \
  do {                                                                                             \
    const int nl_ = g.nc / g.band;                                                                 \
    const bool sq8_ = (FIXOK) && g.mx == 8 && g.my == 8, sq16_ = (FIXOK) && g.mx == 16 && g.my == 16; \
    if (line_mf(g) == 8) {                                                                         \
      if (sq8_) MPM_LB_LAUNCH((KERNEL<8, 8, double, 8>), __VA_ARGS__);                             \
      else if (nl_ == 8) MPM_LB_LAUNCH((KERNEL<8, 8, double, 0>), __VA_ARGS__);                    \
      else MPM_LB_LAUNCH((KERNEL<8, 0, double, 0>), __VA_ARGS__);                                  \
    } else if (line_mf(g) == 16) {                                                                 \
      if (sq16_) MPM_LB_LAUNCH((KERNEL<16, 16, double, 16>), __VA_ARGS__);                         \
      else if (nl_ == 16) MPM_LB_LAUNCH((KERNEL<16, 16, double, 0>), __VA_ARGS__);                 \
      else MPM_LB_LAUNCH((KERNEL<16, 0, double, 0>), __VA_ARGS__);                                 \
    }                                                                                              \
  } while (0)
#define MPM_LB_DISPATCH(KERNEL, FIXOK, ...)                                                        \
  do {                                                                                             \
    if (line_mf(g) == 32) MPM_LB_LAUNCH((KERNEL<32, 0, double, 0>), __VA_ARGS__);                  \
    else MPM_LB_DISPATCH16(KERNEL, FIXOK, __VA_ARGS__);                                            \
  } while (0)

// precision form: FP32 blocks, lines of up to 16 cells and any line count up to 16 (the plan
// refuses the rest); square 8^2 / 16^2 subdomains get compile-time shapes
#define MPM_LB_DISPATCH_F32(KERNEL, ...)                                                           \
  do {                                                                                             \
    const bool sq8_ = g.mx == 8 && g.my == 8, sq16_ = g.mx == 16 && g.my == 16;                    \
    if (line_mf(g) == 8) {                                                                         \
      if (sq8_) MPM_LB_LAUNCH((KERNEL<8, 16, float, 8>), __VA_ARGS__);                             \
      else MPM_LB_LAUNCH((KERNEL<8, 16, float, 0>), __VA_ARGS__);                                  \
    } else if (line_mf(g) == 16) {                                                                 \
      if (sq16_) MPM_LB_LAUNCH((KERNEL<16, 16, float, 16>), __VA_ARGS__);                          \
      else MPM_LB_LAUNCH((KERNEL<16, 16, float, 0>), __VA_ARGS__);                                 \
    }                                                                                              \
  } while (0)

void launch_mpm_local(hipStream_t st, const Geo& g, const double* kn, const double* km, const double* uxm,
                      const double* uym, const double* q, const double* fac, double* h, double* vbnd,
                      LeafOut lo, int32_t* err, Runs rt) {
  MPM_LB_DISPATCH(k_mpm_local_lb, true, g, kn, km, uxm, uym, q, fac, h, vbnd, lo, err, rt.tab);
}

void launch_mpm_first(hipStream_t st, const Geo& g, const double* kn, const double* km, const double* uxm,
                      const double* uym, const double* q, const double* fac, const double* y,
                      const int32_t* sub_dofs, const double* ubnd, const double* vbnd, double* h, double* wbnd,
                      LeafOut lo, Runs rt) {
  // lines of at most 16 cells (the plan refuses the first-order term for longer ones)
  MPM_LB_DISPATCH16(k_mpm_first, true, g, kn, km, uxm, uym, q, fac, y, sub_dofs, ubnd, vbnd, h, wbnd, lo, rt.tab);
}

template <typename T>
static void ds_factor_any(hipStream_t st, const Geo& g, const double* kap_n, T* Escr, const int32_t* list,
                          const int32_t* count, int32_t* err, Runs rt) {
  const dim3 grid(std::min(g.nsub, 1024), 1, runs_of(rt));
  if (line_mf(g) == 8)
    hipLaunchKernelGGL((k_ds_factor<8, T, 64>), grid, dim3(64), 0, st, g, kap_n, Escr, list, count, err, rt.tab);
  else if (line_mf(g) == 16)
    hipLaunchKernelGGL((k_ds_factor<16, T, 64>), grid, dim3(64), 0, st, g, kap_n, Escr, list, count, err, rt.tab);
  else if constexpr (sizeof(T) == 8)   // FP32 blocks: lines of at most 16 cells
    hipLaunchKernelGGL((k_ds_factor<32, T, 256>), grid, dim3(256), 0, st, g, kap_n, Escr, list, count, err, rt.tab);
}

void launch_ds_factor(hipStream_t st, const Geo& g, const double* kap_n, double* Escr, const int32_t* list,
                      const int32_t* count, int32_t* err, Runs rt) {
  ds_factor_any<double>(st, g, kap_n, Escr, list, count, err, rt);
}

void launch_ds_factor_f32(hipStream_t st, const Geo& g, const double* kap_n, float* Escr, const int32_t* list,
                          const int32_t* count, int32_t* err, Runs rt) {
  ds_factor_any<float>(st, g, kap_n, Escr, list, count, err, rt);
}

void launch_mpm_local_f32(hipStream_t st, const Geo& g, const double* kn, const double* km, const double* uxm,
                          const double* uym, const double* q, const float* fac, double* h, double* vbnd,
                          LeafOut lo, int32_t* err, Runs rt) {
  MPM_LB_DISPATCH_F32(k_mpm_local_lb, g, kn, km, uxm, uym, q, fac, h, vbnd, lo, err, rt.tab);
}

void launch_downscale_f32(hipStream_t st, const Geo& g, const double* kap_s, const double* q, const double* ubnd,
                          double* ux, double* uy, double* red_rate, double* red_qin, float* Escr, float* Ekeep,
                          const int32_t* flag, int32_t* err, Runs rt) {
  MPM_LB_DISPATCH_F32(k_downscale_lb, g, kap_s, q, ubnd, ux, uy, red_rate, red_qin, Escr, Ekeep, flag, 0, err, rt.tab);
}

__global__ void __launch_bounds__(256) k_to_f32(size_t n, const double* __restrict__ src, float* __restrict__ dst,
                                               const RunTab* __restrict__ rt) {
  src = at_off(src, ws_off(rt));
  dst = at_off(dst, ws_off(rt));
  const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) dst[i] = float(src[i]);
}

void launch_to_f32(hipStream_t st, size_t n, const double* src, float* dst, Runs rt) {
  if (!n) return;
  hipLaunchKernelGGL(k_to_f32, dim3(unsigned((n + 255) / 256), 1, runs_of(rt)), dim3(256), 0, st, n, src, dst,
                     rt.tab);
}

void launch_downscale(hipStream_t st, const Geo& g, const double* kap_s, const double* q, const double* ubnd,
                      double* ux, double* uy, double* red_rate, double* red_qin, double* Escr, double* Ekeep,
                      const int32_t* flag, int store, int32_t* err, Runs rt) {
  MPM_LB_DISPATCH(k_downscale_lb, !store, g, kap_s, q, ubnd, ux, uy, red_rate, red_qin, Escr, Ekeep, flag, store, err,
                  rt.tab);
}

size_t line_factor_doubles(int nsub, int nc, int band) {
  const int mf = band <= 8 ? 8 : band <= 16 ? 16 : 32;
  return size_t(nsub) * (nc / band) * (mf * (mf + 1) / 2);
}

}  // namespace mpm
