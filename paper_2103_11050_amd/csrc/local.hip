// Per-subdomain kernels: conductivity and switch criterion, MRCM basis (local Robin
// problems, Robin-to-flux map, interface block), MPM-2P trivial-Robin solve, flux
// reconstruction on subdomain boundaries, and the all-Neumann downscaling.
//
// Local matrices are the two-point flux systems of the lowest-order mixed method with
// trapezoidal velocity quadrature (eq:mrc1 on each subdomain). They are SPD and banded with
// half bandwidth b = min(mx, my); one workgroup factors one subdomain as L D L^T in LDS.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace mpm {

namespace {

constexpr int LOCAL_THREADS = 128;

// ------------------------------------------------------------------ band helpers
// Band storage: A(i, j), i-b <= j <= i, at A[i*(b+1) + (j - i + b)]; diagonal at offset b.

__device__ __forceinline__ double& bandref(double* A, int b, int i, int j) { return A[i * (b + 1) + (j - i + b)]; }

// Two-point flux matrix of a subdomain with conductivity kap (LDS, local order).
// neumann = false: boundary faces carry their Dirichlet/Robin transmissibility (eq:mrc1).
// neumann = true : all boundary faces are flux faces and cell 0 is pinned (p = 0).
__device__ __forceinline__ void assemble_band(const Geo& g, int I, int J, const double* kap, double* A, bool neumann) {
  const int b = g.band, n = g.nc;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    for (int o = 0; o <= b; ++o) A[c * (b + 1) + o] = 0.0;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    int i, j;
    loc_ij(g, c, &i, &j);
    const double kc = kap[c];
    double diag = 0.0;
    // W neighbour / face
    if (i > 0) {
      const int d = loc_index(g, i - 1, j);
      const double w = g.hy * harm_trans(kc, kap[d], g.hx);
      diag += w;
      if (!(neumann && d == 0)) bandref(A, b, c, d) = -w;
    }
    if (i < g.mx - 1) diag += g.hy * harm_trans(kc, kap[loc_index(g, i + 1, j)], g.hx);
    if (j > 0) {
      const int d = loc_index(g, i, j - 1);
      const double w = g.hx * harm_trans(kc, kap[d], g.hy);
      diag += w;
      if (!(neumann && d == 0)) bandref(A, b, c, d) = -w;
    }
    if (j < g.my - 1) diag += g.hx * harm_trans(kc, kap[loc_index(g, i, j + 1)], g.hy);
    if (!neumann) {
      if (i == 0) { BFace f = bface(g, I, J, j); diag += f.flen * bface_trans(g, f, kc); }
      if (i == g.mx - 1) { BFace f = bface(g, I, J, g.my + j); diag += f.flen * bface_trans(g, f, kc); }
      if (j == 0) { BFace f = bface(g, I, J, 2 * g.my + i); diag += f.flen * bface_trans(g, f, kc); }
      if (j == g.my - 1) { BFace f = bface(g, I, J, 2 * g.my + g.mx + i); diag += f.flen * bface_trans(g, f, kc); }
    }
    if (neumann && c == 0) diag = 1.0;
    bandref(A, b, c, c) = diag;
  }
  __syncthreads();
}

// In-place L D L^T of the band. On exit the strict lower band holds L and the diagonal slot
// holds 1/d. Returns false (and sets the error word) on a non-positive pivot.
__device__ __forceinline__ void band_ldlt(const Geo& g, double* A, int32_t* err) {
  const int b = g.band, n = g.nc;
  const int P = b * (b + 1) / 2;
  bool ok = true;
  for (int k = 0; k < n; ++k) {
    const double dk = bandref(A, b, k, k);
    if (!(dk > 0.0)) ok = false;
    const double rk = 1.0 / dk;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
      // pair p -> (di, dj), 1 <= dj <= di <= b
      int di = int((1.0 + sqrt(1.0 + 8.0 * p)) * 0.5);
      while (di * (di - 1) / 2 > p) --di;
      while ((di + 1) * di / 2 <= p) ++di;
      const int dj = p - di * (di - 1) / 2 + 1;
      const int i = k + di, j = k + dj;
      if (i < n) bandref(A, b, i, j) -= bandref(A, b, i, k) * bandref(A, b, j, k) * rk;
    }
    __syncthreads();
  }
  // scale the columns: L(i,k) = A(i,k)/d_k; diagonal slot <- 1/d_k
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    for (int o = 0; o < b; ++o) {
      const int k = i - b + o;
      if (k >= 0) A[i * (b + 1) + o] /= A[k * (b + 1) + b];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) A[i * (b + 1) + b] = 1.0 / A[i * (b + 1) + b];
  __syncthreads();
  if (!ok && threadIdx.x == 0) set_error(err, ERR_NOTSPD);
}

__device__ __forceinline__ int gcell(const Geo& g, int I, int J, int i, int j) {
  return (J * g.my + j) * g.nx + I * g.mx + i;
}

__device__ __forceinline__ void load_tile(const Geo& g, int I, int J, const double* src, double* dst) {
  for (int c = threadIdx.x; c < g.nc; c += blockDim.x) {
    int i, j;
    loc_ij(g, c, &i, &j);
    dst[c] = src[gcell(g, I, J, i, j)];
  }
}

// Restriction B^T of boundary-face quantities to local interface unknowns:
// U unknown: -sgn beta_f on the element's faces; P unknown: 1.
__device__ __forceinline__ double bweight(const Geo& g, const BFace& f, bool is_p, double kc) {
  return is_p ? 1.0 : -f.sgn * robin_beta(g, f, kc);
}

}  // namespace

// ====================================================================== A1: kappa, epsilon

__global__ void __launch_bounds__(256)
k_kappa(int ncell, const double* __restrict__ s, const double* __restrict__ K, double* __restrict__ kap_n,
        const double* __restrict__ kap_m, double mu_w, double mu_o, double* __restrict__ red) {
  __shared__ double sa[256], sb[256];
  const int c = blockIdx.x * 256 + threadIdx.x;
  double a = 0.0, bb = 0.0;
  if (c < ncell) {
    const double sv = s[c];
    const double lam = sv * sv / mu_w + (1.0 - sv) * (1.0 - sv) / mu_o;
    const double kn = lam * K[c];
    kap_n[c] = kn;
    const double km = kap_m[c];
    const double dd = kn - km;
    a = dd * dd;
    bb = km * km;
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = bb;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red[2 * blockIdx.x] = sa[0];
    red[2 * blockIdx.x + 1] = sb[0];
  }
}

// Fixed-order reduction of the epsilon partial sums into the scalar block.
__global__ void __launch_bounds__(256) k_reduce_eps(int nblocks, const double* __restrict__ red,
                                                    double* __restrict__ scal) {
  __shared__ double sa[256], sb[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += 256) {
    a += red[2 * i];
    b += red[2 * i + 1];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scal[SC_EPS_NUM] = sa[0];
    scal[SC_EPS_DEN] = sb[0];
  }
}

// Transport sub-step from the maximum outflow rate and the boundary inflow (fixed order).
__global__ void __launch_bounds__(256) k_dt(int nsub, const double* __restrict__ red_rate,
                                            const double* __restrict__ red_qin, double cfl, double fmax_deriv,
                                            double* __restrict__ scal) {
  __shared__ double sm[256], ss[256];
  reduce_dt(nsub, red_rate, red_qin, cfl, fmax_deriv, scal, sm, ss);
}

// ====================================================================== A2+A3: MRCM basis
// One workgroup per subdomain:
//  * factor the local Robin matrix A_i (eq:mrc1 with zero Robin datum);
//  * the Robin-to-flux map on the boundary faces, S = W T - W T E^T A^-1 E W T, through the
//    Gram form (E^T A^-1 E)_{fg} = sum_k (L^-1 E)_{kf} (L^-1 E)_{kg} / d_k: one forward
//    substitution per boundary face (the homogeneous basis functions of eq:mrc_homogeneous,
//    restricted to what the interface system and the reconstruction need);
//  * the boundary fluxes h of the non-homogeneous basis function (eq:mrc_non_homogeneous);
//  * the subdomain's block of the interface system (eq:mrc2 with the Robin rows negated):
//    K_i = B^T S B - D_i and its right-hand side B^T h.
__global__ void __launch_bounds__(LOCAL_THREADS)
k_basis(Geo g, const double* __restrict__ kap, const double* __restrict__ q, double* __restrict__ Sg, double* __restrict__ hg, double* __restrict__ leafK,
        double* __restrict__ leafr, int32_t* err) {
  extern __shared__ double smem[];
  const int sub = blockIdx.x;
  const int I = sub % g.Sx, J = sub / g.Sx;
  const int b = g.band, n = g.nc, nb = g.nb;
  const int bandsz = n * (b + 1);
  double* A = smem;                                            // band, later S
  double* kl = A + max(bandsz, nb * nb);                       // conductivity tile
  double* rhs0 = kl + n;                                       // non-homogeneous rhs
  double* win = rhs0 + n;                                      // (b+1) x (nb+1) circular window
  double* hsh = win + (b + 1) * (nb + 1);                      // h per face
  double* wsh = hsh + nb;                                      // |f| t_f per face

  load_tile(g, I, J, kap, kl);
  __syncthreads();
  assemble_band(g, I, J, kl, A, false);
  band_ldlt(g, A, err);

  // non-homogeneous right-hand side: |c| q + sum_DIR |f| t g - sum_NEU |f| z (Robin datum 0)
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    int i, j;
    loc_ij(g, c, &i, &j);
    double r = g.hx * g.hy * q[gcell(g, I, J, i, j)];
    int fs[4] = {-1, -1, -1, -1};
    if (i == 0) fs[0] = j;
    if (i == g.mx - 1) fs[1] = g.my + j;
    if (j == 0) fs[2] = 2 * g.my + i;
    if (j == g.my - 1) fs[3] = 2 * g.my + g.mx + i;
    for (int t = 0; t < 4; ++t) {
      if (fs[t] < 0) continue;
      BFace f = bface(g, I, J, fs[t]);
      if (f.kind == FACE_DIR) r += f.flen * bface_trans(g, f, kl[c]) * f.value;
      if (f.kind == FACE_NEU) r -= f.flen * f.value;
    }
    rhs0[c] = r;
  }
  const int col = threadIdx.x;             // column of this thread: boundary face, or nb = rhs0
  int ccol = -1;
  double wcol = 0.0;
  if (col < nb) {
    BFace f = bface(g, I, J, col);
    ccol = loc_index(g, f.i, f.j);
    wcol = f.flen * bface_trans(g, f, kl[ccol]);
    wsh[col] = wcol;
  }
  __syncthreads();
  // window rows 0..b
  if (col <= nb) {
    for (int r = 0; r <= b && r < n; ++r) win[r * (nb + 1) + col] = (col == nb) ? rhs0[r] : (r == ccol ? 1.0 : 0.0);
  }
  double acc[64];
#pragma unroll
  for (int t = 0; t < 64; ++t) acc[t] = 0.0;
  double hacc = 0.0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const int slot = k % (b + 1);
    const double dinv = A[k * (b + 1) + b];
    if (col < nb) {
      const double yk = win[slot * (nb + 1) + col] * dinv;
#pragma unroll
      for (int t = 0; t < 64; ++t)
        if (t < nb) acc[t] += yk * win[slot * (nb + 1) + t];
      hacc += yk * win[slot * (nb + 1) + nb];
    }
    __syncthreads();
    if (col <= nb) {
      const double yk = win[slot * (nb + 1) + col];
      for (int o = 1; o <= b; ++o) {
        if (k + o < n) win[((k + o) % (b + 1)) * (nb + 1) + col] -= A[(k + o) * (b + 1) + (b - o)] * yk;
      }
      const int r = k + b + 1;
      if (r < n) win[slot * (nb + 1) + col] = (col == nb) ? rhs0[r] : (r == ccol ? 1.0 : 0.0);
    }
    __syncthreads();
  }
  // S = W T - W T (E^T A^-1 E) W T ;  h = W T (E^T p0 - r_D)
  double* S = A;
  if (col < nb) {
    BFace f = bface(g, I, J, col);
    double* Srow = Sg + (size_t(sub) * nb + col) * nb;
#pragma unroll
    for (int t = 0; t < 64; ++t) {
      if (t < nb) {
        const double v = (t == col ? wcol : 0.0) - wcol * acc[t] * wsh[t];
        S[col * nb + t] = v;
        Srow[t] = v;
      }
    }
    const double rD = f.kind == FACE_DIR ? f.value : 0.0;
    const double h = f.kind == FACE_NEU ? 0.0 : wcol * (hacc - rD);
    hsh[col] = h;
    hg[size_t(sub) * nb + col] = h;
  }
  __syncthreads();
  // interface block K_i = B^T S B - D_i and rhs B^T h (Gamma faces only)
  const int nd = sub_ndof(g, I, J);
  double* Ks = leafK + size_t(sub) * g.ndmax * g.ndmax;
  for (int p = threadIdx.x; p < nd * nd; p += blockDim.x) {
    const int a = p / nd, c2 = p % nd;
    int fa, na, fb, nbb;
    dof_faces(g, I, J, a, &fa, &na);
    dof_faces(g, I, J, c2, &fb, &nbb);
    const bool pa = a & 1, pb = c2 & 1;
    double v = 0.0;
    for (int x = fa; x < fa + na; ++x) {
      BFace ff = bface(g, I, J, x);
      const double wa = bweight(g, ff, pa, kl[loc_index(g, ff.i, ff.j)]);
      double sacc = 0.0;
      for (int y = fb; y < fb + nbb; ++y) {
        BFace fg = bface(g, I, J, y);
        sacc += S[x * nb + y] * bweight(g, fg, pb, kl[loc_index(g, fg.i, fg.j)]);
      }
      v += wa * sacc;
    }
    if (a == c2 && !pa) {
      double dsum = 0.0;
      for (int x = fa; x < fa + na; ++x) {
        BFace ff = bface(g, I, J, x);
        dsum += ff.flen * robin_beta(g, ff, kl[loc_index(g, ff.i, ff.j)]);
      }
      v -= dsum;
    }
    Ks[a * nd + c2] = v;
  }
  for (int a = threadIdx.x; a < nd; a += blockDim.x) {
    int fa, na;
    dof_faces(g, I, J, a, &fa, &na);
    double v = 0.0;
    for (int x = fa; x < fa + na; ++x) {
      BFace ff = bface(g, I, J, x);
      v += bweight(g, ff, a & 1, kl[loc_index(g, ff.i, ff.j)]) * hsh[x];
    }
    leafr[size_t(sub) * g.ndmax + a] = v;
  }
}

// ====================================================================== A7: boundary fluxes
// Reconstruction on every boundary face of every subdomain from the interface solution:
// W u = h - S r with the Robin data r_f = -sgn beta_f U_l + P_l on Gamma faces (zero on
// Dirichlet faces, whose data are in h); Neumann faces keep z. With with_v the MPM-2P flux
// u-bar = u-hat_0 + v is returned.
__global__ void __launch_bounds__(64)
k_flux(Geo g, const double* __restrict__ kap_m, const double* __restrict__ Sg, const double* __restrict__ hg,
       const double* __restrict__ vbnd, const double* __restrict__ y, const int32_t* __restrict__ sub_dofs,
       double* __restrict__ ubnd, int with_v) {
  __shared__ double r[64];
  const int sub = blockIdx.x;
  const int I = sub % g.Sx, J = sub / g.Sx;
  const int nb = g.nb;
  const int f = threadIdx.x;
  BFace bf;
  if (f < nb) {
    bf = bface(g, I, J, f);
    double rv = 0.0;
    if (bf.kind == FACE_ROB) {
      const int a = bface_dof(g, I, J, bf);
      const int32_t* dofs = sub_dofs + size_t(sub) * g.ndmax;
      const double U = y[dofs[a]], Pv = y[dofs[a + 1]];
      const int gc = (J * g.my + bf.j) * g.nx + I * g.mx + bf.i;
      rv = -bf.sgn * robin_beta(g, bf, kap_m[gc]) * U + Pv;
    }
    r[f] = rv;
  }
  __syncthreads();
  if (f < nb) {
    double u;
    if (bf.kind == FACE_NEU) {
      u = bf.value;
    } else {
      const double* Srow = Sg + (size_t(sub) * nb + f) * nb;
      double acc = hg[size_t(sub) * nb + f];
      for (int t = 0; t < nb; ++t) acc -= Srow[t] * r[t];
      u = acc / bf.flen;
      if (with_v) u += vbnd[size_t(sub) * nb + f];
    }
    ubnd[size_t(sub) * nb + f] = u;
  }
}

// ---------------------------------------------------------------------- launchers

static size_t basis_smem(const Geo& g) {
  const int b = g.band, n = g.nc, nb = g.nb;
  return size_t(max(n * (b + 1), nb * nb) + 2 * n + (b + 1) * (nb + 1) + 2 * nb) * 8;
}
size_t local_smem_max(const Geo& g) { return basis_smem(g); }

void launch_kappa(hipStream_t st, int ncell, const double* s, const double* K, double* kn, const double* km,
                  double mu_w, double mu_o, double* red, double* scal) {
  const int nblk = (ncell + 255) / 256;
  hipLaunchKernelGGL(k_kappa, dim3(nblk), dim3(256), 0, st, ncell, s, K, kn, km, mu_w, mu_o, red);
  hipLaunchKernelGGL(k_reduce_eps, dim3(1), dim3(256), 0, st, nblk, red, scal);
}

void launch_dt(hipStream_t st, int nsub, const double* red_rate, const double* red_qin, double cfl,
               double fmax_deriv, double* scal) {
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(256), 0, st, nsub, red_rate, red_qin, cfl, fmax_deriv, scal);
}

void launch_basis(hipStream_t st, const Geo& g, const double* kap, const double* q, double* S, double* h,
                  double* leafK, double* leafr, int32_t* err) {
  hipLaunchKernelGGL(k_basis, dim3(g.nsub), dim3(LOCAL_THREADS), basis_smem(g), st, g, kap, q, S, h, leafK, leafr,
                     err);
}

void launch_flux(hipStream_t st, const Geo& g, const double* km, const double* S, const double* h,
                 const double* vbnd, const double* y, const int32_t* sub_dofs, double* ubnd, int with_v) {
  hipLaunchKernelGGL(k_flux, dim3(g.nsub), dim3(64), 0, st, g, km, S, h, vbnd, y, sub_dofs, ubnd, with_v);
}

}  // namespace mpm
