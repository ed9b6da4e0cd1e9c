// Device-side geometry and helpers shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "plan.hpp"

namespace mpm {

// Everything a kernel needs to know about the grid and the decomposition, passed by value.
struct Geo {
  int nx, ny, mx, my, Sx, Sy, nsub;
  int nc, band, xfast, nb, ne_x, ne_y, n_vert, ndmax;
  int npol;             // interface functions per element and field: 1 constant, 2 linear
  double hx, hy, alpha;
  int bc_pack;          // MPM_BC_* of side s in bits 2s..2s+1 (sides W, E, S, N)
  double bc_v0, bc_v1, bc_v2, bc_v3;
  double s_inj;
  double refine_rtol;   // precision form: refinement stops at this correction / solution ratio
};

// p moved by o bytes (pointer arithmetic on bytes, so that the compiler keeps the address
// space of p: an integer round trip would turn global loads into flat ones).
template <class T>
__host__ __device__ __forceinline__ T* at_off(T* p, int64_t o) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return reinterpret_cast<T*>(reinterpret_cast<B*>(p) + o);
}

// Physical boundary data of a side without a run-time index into the struct (which would
// force the by-value kernel argument into scratch memory).
__host__ __device__ __forceinline__ int bc_kind_of(const Geo& g, int side) { return (g.bc_pack >> (2 * side)) & 3; }
__host__ __device__ __forceinline__ double bc_value_of(const Geo& g, int side) {
  const double a = (side & 1) ? g.bc_v1 : g.bc_v0;
  const double b = (side & 1) ? g.bc_v3 : g.bc_v2;
  return (side & 2) ? b : a;
}

// Error bits of the device error word. ERR_NOTSPD: a non-positive pivot of a local matrix,
// or a permeability that is not positive; ERR_NONFINITE: a non-finite value in the state, a
// saturation outside [0, 1] beyond rounding, or no flow through any cell (the time step of
// the upwind scheme is then unbounded); ERR_NOCONV: an FP64 refinement of the precision form
// did not reach its tolerance within its iteration limit.
enum : int32_t { ERR_NOTSPD = 1, ERR_SINGULAR = 2, ERR_NONFINITE = 4, ERR_NOCONV = 8 };

// Bounds of the saturation checked on the device: [0, 1] up to the rounding of the monotone
// upwind update.
constexpr double SAT_TOL = 1e-12;

// A double moved between lanes by a DPP pattern (both halves with the same pattern; every lane
// of the wavefront active and every pattern used here reads a lane of the wavefront).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_mov_dpp(int(unsigned(b)), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(int(unsigned(b >> 32)), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (unsigned long long)unsigned(lo) | ((unsigned long long)unsigned(hi) << 32));
}

// Sum over the 64 lanes of a wavefront, the same value in every lane: a butterfly whose partner
// is always in the other half of the group reached so far (quad permutations, half-row and row
// mirrors by DPP, then lane ^ 16 and lane ^ 32 by shuffles); each step adds two equal-order
// pairs, so every lane ends with the same bits.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);   // row_half_mirror: the other quad of the 8
  v += dpp_f64<0x140>(v);   // row_mirror: the other 8 of the 16
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}
// The largest value over the 64 lanes, in every lane (same pattern; fmax is exact).
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  v = fmax(v, __shfl_xor(v, 16));
  v = fmax(v, __shfl_xor(v, 32));
  return v;
}

// Makes the LDS writes of this wavefront's lanes visible to the LDS reads that follow in other
// lanes of the same wavefront: a fence at wavefront scope (the lanes of a wavefront perform their
// LDS accesses in program order; the fence keeps the compiler from reusing values it loaded
// earlier, or moving those reads above the writes).
__device__ __forceinline__ void wave_lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// ---------------------------------------------------------------- subdomain of a workgroup
// The chip dispatches workgroups to its 8 XCDs in turn (linear workgroup id mod 8), and each
// XCD has its own L2. A kernel with one workgroup per subdomain (grid x = nsub) takes the
// subdomain of its workgroup from here: with nsub a multiple of 8, XCD x receives the
// contiguous range [x nsub / 8, (x + 1) nsub / 8), i.e. whole rows of subdomains, so that the
// cache lines neighbouring subdomains share (halo cells, the faces between them) are fetched
// into one L2 instead of two. A bijection of [0, nsub); identity when nsub is not a multiple of 8.
__device__ __forceinline__ int xcd_sub(int nsub) {
  const int b = blockIdx.x;
  if (nsub & 7) return b;
  return (b & 7) * (nsub >> 3) + (b >> 3);
}

// ---------------------------------------------------------------- local cell ordering
// Cells of a subdomain are numbered along the shorter side first so that the 5-point
// matrix has half bandwidth min(mx, my).
__host__ __device__ __forceinline__ int loc_index(const Geo& g, int i, int j) {
  return g.xfast ? j * g.mx + i : i * g.my + j;
}
__host__ __device__ __forceinline__ void loc_ij(const Geo& g, int c, int* i, int* j) {
  // values first, then unconditional stores (a conditional store target would be turned into
  // an address select and force the locals into scratch)
  const int len = g.xfast ? g.mx : g.my;
  const int a = c % len, b = c / len;
  *i = g.xfast ? a : b;
  *j = g.xfast ? b : a;
}

// ---------------------------------------------------------------- Robin-to-flux maps
// The nb x nb map S_i of a subdomain is symmetric and is kept by wrapped diagonals: entry
// (i, j) with d = (j - i) mod nb <= nb / 2 sits at [d][i]; every other entry is read from its
// mirror (j, i). nb / 2 + 1 rows of nb doubles; each row is read coalesced by the lanes.
__host__ __device__ __forceinline__ int smap_doubles(int nb) { return (nb / 2 + 1) * nb; }
// Whether (i, j) is the stored orientation (for d = nb / 2 both orientations are stored).
__device__ __forceinline__ bool smap_owner(int nb, int i, int j) {
  const int d = j >= i ? j - i : j - i + nb;
  return 2 * d <= nb;
}
__device__ __forceinline__ int smap_at(int nb, int i, int j) {
  const int d = j >= i ? j - i : j - i + nb;
  return 2 * d <= nb ? d * nb + i : (nb - d) * nb + j;
}

// ---------------------------------------------------------------- fractional flow, water cut
// Water fractional flow f_w(s) = M s^2 / (M s^2 + (1 - s)^2), M = mu_o / mu_w (eq. BL2D).
__device__ __forceinline__ double frac_w(double s, double M) {
  const double a = M * s * s;
  const double o = 1.0 - s;
  return a / (a + o * o);
}
// Explicit upwind update of cell (gi, gj) over one sub-step dt (eq. BL2D): s - dt/|c| sum_f
// |f| u_f f_w(s_upwind), the injected saturation behind inflow boundary faces.
__device__ __forceinline__ double sat_cell(const Geo& g, const double* __restrict__ s,
                                           const double* __restrict__ ux, const double* __restrict__ uy, int gi,
                                           int gj, double dt, double M) {
  const int c = gj * g.nx + gi;
  const double sc = s[c];
  const double uW = ux[gj * (g.nx + 1) + gi];
  const double uE = ux[gj * (g.nx + 1) + gi + 1];
  const double uS = uy[gj * g.nx + gi];
  const double uN = uy[(gj + 1) * g.nx + gi];
  const double sW = gi > 0 ? s[c - 1] : g.s_inj;
  const double sE = gi < g.nx - 1 ? s[c + 1] : g.s_inj;
  const double sS = gj > 0 ? s[c - g.nx] : g.s_inj;
  const double sN = gj < g.ny - 1 ? s[c + g.nx] : g.s_inj;
  const double FW = g.hy * uW * frac_w(uW > 0.0 ? sW : sc, M);
  const double FE = g.hy * uE * frac_w(uE > 0.0 ? sc : sE, M);
  const double FS = g.hx * uS * frac_w(uS > 0.0 ? sS : sc, M);
  const double FN = g.hx * uN * frac_w(uN > 0.0 ? sc : sN, M);
  return sc - dt / (g.hx * g.hy) * ((FE - FW) + (FN - FS));
}
// Boundary face e of the domain for the water cut, 0 <= e < 2 (nx + ny): W faces j = 0..ny-1,
// then E faces, S faces i = 0..nx-1, N faces. Its normal velocity index in ux or uy, the cell
// behind it, whether it is an x-face and whether the outward normal is +x / +y.
struct DomFace {
  int ui, si;
  bool vert, hi;
};
__device__ __forceinline__ DomFace dom_face(const Geo& g, int e) {
  const int nW = g.ny, nS = g.nx;
  DomFace d;
  d.vert = e < 2 * nW;
  const int k = d.vert ? (e < nW ? e : e - nW) : (e < 2 * nW + nS ? e - 2 * nW : e - 2 * nW - nS);
  d.hi = d.vert ? e >= nW : e >= 2 * nW + nS;
  d.ui = d.vert ? k * (g.nx + 1) + (d.hi ? g.nx : 0) : (d.hi ? g.ny * g.nx : 0) + k;
  d.si = d.vert ? k * g.nx + (d.hi ? g.nx - 1 : 0) : (d.hi ? (g.ny - 1) * g.nx : 0) + k;
  return d;
}

// ---------------------------------------------------------------- boundary faces
// Boundary faces of a subdomain: W faces j=0..my-1, E faces, S faces i=0..mx-1, N faces.
struct BFace {
  int side;     // 0 W, 1 E, 2 S, 3 N
  int i, j;     // local cell adjacent to the face
  int k;        // index along the side
  int kind;     // FACE_NEU / FACE_DIR / FACE_ROB
  double flen;  // face length
  double d;     // cell width normal to the face
  double H;     // subdomain length normal to the face (Robin coefficient)
  double sgn;   // n-check . n^i on Gamma: +1 on E and N sides, -1 on W and S sides
  double value; // physical datum: g (DIR) or outward flux z (NEU)
};

__host__ __device__ __forceinline__ BFace bface(const Geo& g, int I, int J, int f) {
  BFace b;
  if (f < g.my) { b.side = 0; b.k = f; b.i = 0; b.j = f; }
  else if (f < 2 * g.my) { b.side = 1; b.k = f - g.my; b.i = g.mx - 1; b.j = b.k; }
  else if (f < 2 * g.my + g.mx) { b.side = 2; b.k = f - 2 * g.my; b.i = b.k; b.j = 0; }
  else { b.side = 3; b.k = f - 2 * g.my - g.mx; b.i = b.k; b.j = g.my - 1; }
  const bool vert = b.side < 2;
  b.flen = vert ? g.hy : g.hx;
  b.d = vert ? g.hx : g.hy;
  b.H = vert ? g.mx * g.hx : g.my * g.hy;
  b.sgn = (b.side == 1 || b.side == 3) ? 1.0 : -1.0;
  bool phys = (b.side == 0 && I == 0) || (b.side == 1 && I == g.Sx - 1) ||
              (b.side == 2 && J == 0) || (b.side == 3 && J == g.Sy - 1);
  b.value = 0.0;
  if (!phys) {
    b.kind = FACE_ROB;
  } else {
    const int kind = bc_kind_of(g, b.side);
    const double val = bc_value_of(g, b.side);
    if (kind == MPM_BC_PRESSURE) { b.kind = FACE_DIR; b.value = val; }
    else { b.kind = FACE_NEU; b.value = kind == MPM_BC_FLUX ? val : 0.0; }
  }
  return b;
}

// Local interface unknowns of a subdomain: sides W, E, S, N present on Gamma, the elements
// along each side in order, per element U_0 .. U_{npol-1} then P_0 .. P_{npol-1}.
__host__ __device__ __forceinline__ int faces_per_elem(const Geo& g, int side) {
  return side < 2 ? g.my / g.ne_y : g.mx / g.ne_x;
}

// Local position of the U_0 unknown of the element of a Gamma face (U_k at +k, P_k at +npol+k).
__host__ __device__ __forceinline__ int bface_dof(const Geo& g, int I, int J, const BFace& b) {
  const bool hasW = I > 0, hasE = I < g.Sx - 1, hasS = J > 0;
  const int pe = 2 * g.npol;
  const int offW = 0;
  const int offE = offW + (hasW ? pe * g.ne_y : 0);
  const int offS = offE + (hasE ? pe * g.ne_y : 0);
  const int offN = offS + (hasS ? pe * g.ne_x : 0);
  const int off = b.side == 0 ? offW : b.side == 1 ? offE : b.side == 2 ? offS : offN;
  return off + pe * (b.k / faces_per_elem(g, b.side));
}

// First boundary face and face count of the element carrying local interface unknown a.
__host__ __device__ __forceinline__ void dof_faces(const Geo& g, int I, int J, int a, int* f0, int* cnt) {
  const bool hasW = I > 0, hasE = I < g.Sx - 1, hasS = J > 0, hasN = J < g.Sy - 1;
  const int pe = 2 * g.npol;
  const int nW = hasW ? pe * g.ne_y : 0, nE = hasE ? pe * g.ne_y : 0, nS = hasS ? pe * g.ne_x : 0;
  const int nN = hasN ? pe * g.ne_x : 0;
  const int perY = g.my / g.ne_y, perX = g.mx / g.ne_x;
  if (a < nW) { *f0 = (a / pe) * perY; *cnt = perY; return; }
  a -= nW;
  if (a < nE) { *f0 = g.my + (a / pe) * perY; *cnt = perY; return; }
  a -= nE;
  if (a < nS) { *f0 = 2 * g.my + (a / pe) * perX; *cnt = perX; return; }
  a -= nS;
  if (a < nN) { *f0 = 2 * g.my + g.mx + (a / pe) * perX; *cnt = perX; return; }
  *f0 = 0;
  *cnt = 0;
}

// Field (P or U) and function index k of local interface unknown a.
__host__ __device__ __forceinline__ void dof_kind(const Geo& g, int a, bool* is_p, int* k) {
  if (g.npol == 1) {
    *is_p = a & 1;
    *k = 0;
    return;
  }
  const int r = a % (2 * g.npol);
  *is_p = r >= g.npol;
  *k = r >= g.npol ? r - g.npol : r;
}

// Interface function k of a Gamma face's element at the face: 1 for k = 0; for k = 1 the
// midpoint xi in [-1, 1] of the face along the element (the face mean of the linear function;
// the global direction of the interface, so both subdomains see the same value).
__host__ __device__ __forceinline__ double iface_phi(const Geo& g, const BFace& b, int k) {
  if (k == 0) return 1.0;
  const int per = faces_per_elem(g, b.side);
  return double(2 * (b.k % per) + 1) / per - 1.0;
}

__host__ __device__ __forceinline__ int sub_ndof(const Geo& g, int I, int J) {
  return 2 * g.npol * (((I > 0) + (I < g.Sx - 1)) * g.ne_y + ((J > 0) + (J < g.Sy - 1)) * g.ne_x);
}

// Transmissibility per unit length of a boundary face for conductivity kc of its cell.
__host__ __device__ __forceinline__ double bface_trans(const Geo& g, const BFace& b, double kc) {
  if (b.kind == FACE_DIR) return 2.0 * kc / b.d;
  if (b.kind == FACE_ROB) return 1.0 / (b.d / (2.0 * kc) + g.alpha * b.H / kc);
  return 0.0;
}
__host__ __device__ __forceinline__ double robin_beta(const Geo& g, const BFace& b, double kc) {
  return g.alpha * b.H / kc;
}
// Restriction B^T of boundary-face quantities to local interface unknown a (eq:mrc2, Robin
// rows negated), which is also the Robin datum of a's homogeneous basis function: the U_k
// unknown -sgn beta_f phi_k(f), the P_k unknown phi_k(f), on the faces of its element.
__host__ __device__ __forceinline__ double bweight(const Geo& g, const BFace& f, int a, double kc) {
  bool is_p;
  int k;
  dof_kind(g, a, &is_p, &k);
  const double w = is_p ? 1.0 : -f.sgn * robin_beta(g, f, kc);
  return k ? w * iface_phi(g, f, k) : w;
}
// Robin datum -sgn beta_f U_H(f) + P_H(f) of a Gamma face from the interface solution y
// (dofs: the subdomain's global unknown ids in local order).
__device__ __forceinline__ double robin_datum(const Geo& g, int I, int J, const BFace& bf, double kc,
                                              const int32_t* dofs, const double* y) {
  const int a = bface_dof(g, I, J, bf);
  double U = y[dofs[a]], Pv = y[dofs[a + g.npol]];
  if (g.npol == 2) {
    const double xi = iface_phi(g, bf, 1);
    U += xi * y[dofs[a + 1]];
    Pv += xi * y[dofs[a + 3]];
  }
  return -bf.sgn * robin_beta(g, bf, kc) * U + Pv;
}
// Reconstruction on the boundary faces of subdomain sub (at most 64) by one wavefront, lane f
// taking face f (A7): W u = h - S r with the Robin data r_f = -sgn beta_f U_H(f) + P_H(f) on
// Gamma faces (zero on Dirichlet faces, whose data are in h); Neumann faces keep z. With
// with_v the MPM-2P flux u-bar = u-hat_0 + v is returned; with with_v = 2 the first-order
// u-hat_1 + w is added to ubnd (Neumann faces unchanged). r: 64 doubles of LDS for this
// wavefront.
__device__ __forceinline__ void flux_sub(const Geo& g, int sub, const double* __restrict__ kap_m,
                                         const double* __restrict__ Sg, const double* __restrict__ hg,
                                         const double* __restrict__ vbnd, const double* __restrict__ y,
                                         const int32_t* __restrict__ sub_dofs, double* __restrict__ ubnd, int with_v,
                                         int f, double* r) {
  const int I = sub % g.Sx, J = sub / g.Sx;
  const int nb = g.nb;
  // the rows of S do not depend on the interface solution: their loads go out first
  const bool act = f < nb;
  const int D = nb / 2;
  const double* Ss = Sg + size_t(sub) * smap_doubles(nb);
  double sv[33];
#pragma unroll
  for (int d = 0; d < 33; ++d) sv[d] = act && d <= D ? __builtin_nontemporal_load(&Ss[d * nb + f]) : 0.0;
  double acc = act ? hg[size_t(sub) * nb + f] : 0.0;
  const double vb = act && with_v ? vbnd[size_t(sub) * nb + f] : 0.0;
  BFace bf;
  if (act) {
    bf = bface(g, I, J, f);
    double rv = 0.0;
    if (bf.kind == FACE_ROB) {
      const int gc = (J * g.my + bf.j) * g.nx + I * g.mx + bf.i;
      rv = robin_datum(g, I, J, bf, kap_m[gc], sub_dofs + size_t(sub) * g.ndmax, y);
    }
    r[f] = rv;
  }
  wave_lds_fence();   // the lanes read each other's Robin data
  // S_i r, row f of S from its wrapped diagonals: S(f, f + d) = D[d][f] for d <= nb / 2, and
  // S(f, f - e) = D[e][f - e] for the other columns (indices mod nb). Each lane loads its
  // entry of every diagonal row (coalesced, all loads issued together, above); D[e][f - e]
  // come from lane f - e through a cross-lane read. Every lane takes part in those reads, so
  // they are made before the lanes branch on the face kind.
#pragma unroll
  for (int d = 0; d < 33; ++d) {
    if (d <= D) {
      const int t = f + d < nb ? f + d : f + d - nb;
      acc -= sv[d] * r[act ? t : 0];
    }
  }
#pragma unroll
  for (int e = 1; e < 32; ++e) {
    if (e < nb - D) {
      const int t = f >= e ? f - e : f - e + nb;
      const double v = __shfl(sv[e], act ? t : 0);
      acc -= v * r[act ? t : 0];
    }
  }
  if (act) {
    double u;
    if (bf.kind == FACE_NEU) {
      u = bf.value;
    } else {
      u = acc / bf.flen + vb;
    }
    if (with_v == 2) {
      if (bf.kind != FACE_NEU) ubnd[size_t(sub) * nb + f] += u;
    } else {
      ubnd[size_t(sub) * nb + f] = u;
    }
  }
}

// Harmonic transmissibility per unit length between two cells at distance d:
// (d/(2 kc) + d/(2 kd))^-1 = 2 kc kd / (d (kc + kd)), one division.
__host__ __device__ __forceinline__ double harm_trans(double kc, double kd, double d) {
  return 2.0 * kc * kd / (d * (kc + kd));
}
// t^n / t^m of a face between cells c and d (the distance cancels), one division.
__host__ __device__ __forceinline__ double harm_ratio(double knc, double knd, double kmc, double kmd) {
  return (knc * knd * (kmc + kmd)) / (kmc * kmd * (knc + knd));
}

__device__ __forceinline__ void set_error(int32_t* err, int32_t bits) { atomicOr(err, bits); }
// The device error word of a run sits right after its scalar block (the plan lays out the
// scalars, then the integer words: error, changed-subdomain count, sequence number).
__device__ __forceinline__ int32_t* err_word(double* scal) { return reinterpret_cast<int32_t*>(scal + SC_COUNT); }
// Finite (false for NaN and for infinities).
__device__ __forceinline__ bool finite_d(double v) { return fabs(v) <= 1.7976931348623157e308; }

// Transport sub-step from the maximum outflow rate and the boundary inflow, reduced in a fixed
// order from per-subdomain partials (run by one workgroup of 256 threads, sm and ss LDS arrays of
// 4 doubles; each thread issues its loads in batches of 16 before adding them, then each
// wavefront reduces its lanes and thread 0 its wavefronts).
__device__ __forceinline__ void reduce_dt(int nsub, const double* red_rate, const double* red_qin, double* scal,
                                          double* sm, double* ss) {
  constexpr int B = 16;
  const double cfl = scal[SC_CFL], fmax_deriv = scal[SC_FMAX];   // requested first
  double m = 0.0, s = 0.0;
  int bad = 0;   // a non-finite partial (fmax would drop a NaN)
  for (int base = 0; base < nsub; base += 256 * B) {
    double vr[B], vq[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int i = base + threadIdx.x + 256 * u;
      const int ic = i < nsub ? i : 0;
      vr[u] = red_rate[ic];
      vq[u] = red_qin[ic];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (base + int(threadIdx.x) + 256 * u < nsub) {
        m = fmax(m, vr[u]);
        s += vq[u];
        bad |= !finite_d(vr[u]);
      }
    }
  }
  m = wave_max(m);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) {
    sm[threadIdx.x >> 6] = m;
    ss[threadIdx.x >> 6] = s;
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      sm[0] = fmax(sm[0], sm[k]);
      ss[0] += ss[k];
    }
  }
  if (threadIdx.x == 0) {
    // no flow anywhere (rate 0) leaves the step unbounded: flagged, and the step set to 0 so
    // that the saturation is left as it is rather than turned into NaN
    const bool ok = !bad && sm[0] > 0.0 && finite_d(ss[0]);
    scal[SC_MAXRATE] = sm[0];
    scal[SC_QIN] = ss[0];
    scal[SC_DT] = ok ? cfl / (fmax_deriv * sm[0]) : 0.0;
    if (!ok) set_error(err_word(scal), ERR_NONFINITE);
  }
}

}  // namespace mpm
