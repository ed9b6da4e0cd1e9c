// Per-subdomain and per-cell kernels: conductivity and switch criterion (A1) and the flux
// reconstruction on subdomain boundaries from the interface solution (A7).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace mpm {

// ====================================================================== A1: kappa, epsilon

// One workgroup per subdomain tile: kappa^n = lambda(s) K, the tile's partial sums of
// (kappa^n - kappa^m)^2 and (kappa^m)^2, and whether any conductivity of the tile changed
// since the last MRCM update (flag, and the subdomain appended to the list of changed ones).
// With ux non-null, also the tile's partial sums of the water cut (outflow |f| u.n and
// |f| u.n f_w(s) over the domain's boundary faces in the tile) at red[2 nsub + 2 sub].
// With SAT the kernel first takes the transport sub-step of its cells (the saturation update
// is local to the tile, reading the neighbours' old values): s is the old saturation, the new
// one goes to s_new and is the one the conductivity and the water cut use.
template <bool SAT>
__global__ void __launch_bounds__(256)
k_kappa(Geo g, const double* __restrict__ s, double* __restrict__ s_new, const double* __restrict__ K,
        double* __restrict__ kap_n, const double* __restrict__ kap_m, double* __restrict__ red,
        int32_t* __restrict__ flag, int32_t* __restrict__ list, int32_t* __restrict__ count,
        double* __restrict__ scal, const double* __restrict__ ux, const double* __restrict__ uy, double area,
        const RunTab* __restrict__ rt) {
  __shared__ double sa[4], sb[4], sq[4], sw[4];   // per-wavefront partials
  const int64_t wo = ws_off(rt);
  const bool wc = ux != nullptr;
  if (wc) {
    ux = at_off(ux, wo);
    uy = at_off(uy, wo);
  }
  s = at_off(s, wo);
  if constexpr (SAT) s_new = at_off(s_new, wo);
  K = at_off(K, wo);
  kap_n = at_off(kap_n, wo);
  kap_m = at_off(kap_m, wo);
  red = at_off(red, wo);
  flag = at_off(flag, wo);
  list = at_off(list, wo);
  count = at_off(count, wo);
  scal = at_off(scal, wo);
  const double mu_w = scal[SC_MUW], mu_o = scal[SC_MUO];
  const int sub = xcd_sub(g.nsub);
  const int I = sub % g.Sx, J = sub / g.Sx;
  double a = 0.0, bb = 0.0;
  int diff = 0;
  // block-uniform: the tile touches the domain boundary
  const bool edge = wc && (I == 0 || J == 0 || I == g.Sx - 1 || J == g.Sy - 1);
  double wq = 0.0, ww = 0.0;
  // one cell per thread up to 256 cells per tile; larger tiles take several per thread
  for (int c = threadIdx.x; c < g.nc; c += blockDim.x) {
    const int gc = (J * g.my + c / g.mx) * g.nx + I * g.mx + c % g.mx;
    double sv;
    if constexpr (SAT) {
      sv = sat_cell(g, s, ux, uy, I * g.mx + c % g.mx, J * g.my + c / g.mx, scal[SC_DT], scal[SC_MRATIO]);
      s_new[gc] = sv;
    } else {
      sv = s[gc];
    }
    if (edge) {
      const int gi = I * g.mx + c % g.mx, gj = J * g.my + c / g.mx;
      double out = 0.0;
      if (gi == 0) out += g.hy * fmax(-ux[size_t(gj) * (g.nx + 1)], 0.0);
      if (gi == g.nx - 1) out += g.hy * fmax(ux[size_t(gj) * (g.nx + 1) + g.nx], 0.0);
      if (gj == 0) out += g.hx * fmax(-uy[gi], 0.0);
      if (gj == g.ny - 1) out += g.hx * fmax(uy[size_t(g.ny) * g.nx + gi], 0.0);
      wq += out;
      ww += out * frac_w(sv, scal[SC_MRATIO]);
    }
    const double Kc = K[gc];
    // the state the method needs: s in [0, 1] up to rounding, K finite and positive (NaN
    // fails every comparison)
    if (!(sv >= -SAT_TOL && sv <= 1.0 + SAT_TOL) || !finite_d(Kc)) set_error(err_word(scal), ERR_NONFINITE);
    else if (!(Kc > 0.0)) set_error(err_word(scal), ERR_NOTSPD);
    const double lam = sv * sv / mu_w + (1.0 - sv) * (1.0 - sv) / mu_o;
    const double kn = lam * Kc;
    kap_n[gc] = kn;
    const double km = kap_m[gc];
    const double dd = kn - km;
    a += dd * dd;
    bb += km * km;
    diff |= kn != km;
  }
  // the tile's sums: over each wavefront by cross-lane moves, then the wavefronts' partials in
  // order
  a = wave_sum(a);
  bb = wave_sum(bb);
  if (edge) {
    wq = wave_sum(wq);
    ww = wave_sum(ww);
  }
  const int wv = threadIdx.x >> 6, nw = int(blockDim.x) >> 6;
  if ((threadIdx.x & 63) == 0) {
    sa[wv] = a;
    sb[wv] = bb;
    sq[wv] = wq;
    sw[wv] = ww;
  }
  const int changed = __syncthreads_or(diff);
  if (threadIdx.x == 0) {
    double ta = sa[0], tb = sb[0], tq = sq[0], tw = sw[0];
    for (int k = 1; k < nw; ++k) {
      ta += sa[k];
      tb += sb[k];
      tq += sq[k];
      tw += sw[k];
    }
    red[2 * sub] = ta;
    red[2 * sub + 1] = tb;
    if (wc) {
      red[2 * size_t(g.nsub) + 2 * sub] = tq;
      red[2 * size_t(g.nsub) + 2 * sub + 1] = tw;
    }
    flag[sub] = changed;
    if (changed) {
      const int at = atomicAdd(count, 1);
      if (at < g.nsub) list[at] = sub;
    }
    if (SAT && sub == 0) {
      const double dt = scal[SC_DT];
      scal[SC_T] += dt;
      scal[SC_PVI] += dt * scal[SC_QIN] / area;
    }
  }
}

// Fixed-order reduction of the epsilon partial sums into the scalar block; the two sums (and
// the water cut) are also written to host memory, with a sequence number, for the switch
// decision and breakthrough checks. With wc the per-tile water-cut partials of k_kappa are
// reduced as well (fixed order) into the water cut: the transport that precedes the
// conductivity then needs no launch of its own for it.
__global__ void __launch_bounds__(256) k_reduce_eps(int nblocks, int wc, const double* __restrict__ red,
                                                    double* __restrict__ scal, int32_t* __restrict__ seq,
                                                    double* __restrict__ host, const RunTab* __restrict__ rt) {
  constexpr int B = 16;
  __shared__ double sa[4], sb[4], sq[4], sw[4];   // per-wavefront sums
  const int64_t wo = ws_off(rt);
  red = at_off(red, wo);
  scal = at_off(scal, wo);
  seq = at_off(seq, wo);
  host = at_off(host, host_off(rt));
  double q = 0.0, w = 0.0;
  double a = 0.0, b = 0.0;
  for (int base = 0; base < nblocks; base += 256 * B) {
    double va[B], vb[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int i = base + threadIdx.x + 256 * u;
      const int ic = i < nblocks ? i : 0;
      va[u] = red[2 * ic];
      vb[u] = red[2 * ic + 1];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (base + int(threadIdx.x) + 256 * u < nblocks) {
        a += va[u];
        b += vb[u];
      }
    }
    if (wc) {
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int i = base + threadIdx.x + 256 * u;
        const int ic = i < nblocks ? i : 0;
        va[u] = red[2 * nblocks + 2 * ic];
        vb[u] = red[2 * nblocks + 2 * ic + 1];
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (base + int(threadIdx.x) + 256 * u < nblocks) {
          q += va[u];
          w += vb[u];
        }
      }
    }
  }
  a = wave_sum(a);
  b = wave_sum(b);
  q = wave_sum(q);
  w = wave_sum(w);
  if ((threadIdx.x & 63) == 0) {
    const int wv = threadIdx.x >> 6;
    sa[wv] = a;
    sb[wv] = b;
    sq[wv] = q;
    sw[wv] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      sa[0] += sa[k];
      sb[0] += sb[k];
      sq[0] += sq[k];
      sw[0] += sw[k];
    }
    scal[SC_EPS_NUM] = sa[0];
    scal[SC_EPS_DEN] = sb[0];
    if (wc) scal[SC_WCUT] = sq[0] > 0.0 ? sw[0] / sq[0] : 0.0;
    if (!finite_d(sa[0]) || !finite_d(sb[0]) || (wc && !(finite_d(sq[0]) && finite_d(sw[0]))))
      set_error(err_word(scal), ERR_NONFINITE);
    const int32_t n = *seq + 1;
    *seq = n;
    host[0] = sa[0];
    host[1] = sb[0];
    host[3] = scal[SC_WCUT];
    host[2] = double(n);
  }
}

// Transport sub-step from the maximum outflow rate and the boundary inflow (fixed order).
// Also empties the list of changed subdomains for the next velocity update.
__global__ void __launch_bounds__(256) k_dt(int nsub, const double* __restrict__ red_rate,
                                            const double* __restrict__ red_qin,
                                            double* __restrict__ scal, int32_t* __restrict__ count, const RunTab* __restrict__ rt) {
  __shared__ double sm[4], ss[4];
  const int64_t wo = ws_off(rt);
  red_rate = at_off(red_rate, wo);
  red_qin = at_off(red_qin, wo);
  scal = at_off(scal, wo);
  count = at_off(count, wo);
  reduce_dt(nsub, red_rate, red_qin, scal, sm, ss);
  if (threadIdx.x == 0) *count = 0;
}

// ====================================================================== A7: boundary fluxes
// Reconstruction on every boundary face of every subdomain from the interface solution
// (flux_sub), one wavefront per subdomain.
__global__ void __launch_bounds__(64)
k_flux(Geo g, const double* __restrict__ kap_m, const double* __restrict__ Sg, const double* __restrict__ hg,
       const double* __restrict__ vbnd, const double* __restrict__ y, const int32_t* __restrict__ sub_dofs,
       double* __restrict__ ubnd, int with_v, const RunTab* __restrict__ rt) {
  __shared__ double r[64];
  const int64_t wo = ws_off(rt);
  flux_sub(g, xcd_sub(g.nsub), at_off(kap_m, wo), at_off(Sg, wo), at_off(hg, wo), at_off(vbnd, wo), at_off(y, wo),
           at_off(sub_dofs, wo), at_off(ubnd, wo), with_v, threadIdx.x, r);
}

// The same reconstruction for subdomains with 65 to 128 boundary faces: one thread per face
// over two wavefronts; the mirrored entries S(f, f - e) are read from memory, not from another
// lane.
__global__ void __launch_bounds__(128)
k_flux_wide(Geo g, const double* __restrict__ kap_m, const double* __restrict__ Sg, const double* __restrict__ hg,
            const double* __restrict__ vbnd, const double* __restrict__ y, const int32_t* __restrict__ sub_dofs,
            double* __restrict__ ubnd, int with_v, const RunTab* __restrict__ rt) {
  __shared__ double r[128];
  const int64_t wo = ws_off(rt);
  kap_m = at_off(kap_m, wo);
  Sg = at_off(Sg, wo);
  hg = at_off(hg, wo);
  vbnd = at_off(vbnd, wo);
  y = at_off(y, wo);
  sub_dofs = at_off(sub_dofs, wo);
  ubnd = at_off(ubnd, wo);
  const int sub = xcd_sub(g.nsub);
  const int I = sub % g.Sx, J = sub / g.Sx;
  const int nb = g.nb;
  const int f = threadIdx.x;
  const bool act = f < nb;
  const double* Ss = Sg + size_t(sub) * smap_doubles(nb);
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
  __syncthreads();
  if (!act) return;
  // S_i r over the wrapped diagonals in the order of k_flux: S(f, f + d) for d <= nb / 2, then
  // S(f, f - e) for the other columns
  const int D = nb / 2;
  double acc = hg[size_t(sub) * nb + f];
  for (int d = 0; d <= D; ++d) {
    const int t = f + d < nb ? f + d : f + d - nb;
    acc -= Ss[d * nb + f] * r[t];
  }
  for (int e = 1; e < nb - D; ++e) {
    const int t = f >= e ? f - e : f - e + nb;
    acc -= Ss[e * nb + t] * r[t];
  }
  double u;
  if (bf.kind == FACE_NEU) u = bf.value;
  else u = acc / bf.flen + (with_v ? vbnd[size_t(sub) * nb + f] : 0.0);
  if (with_v == 2) {
    if (bf.kind != FACE_NEU) ubnd[size_t(sub) * nb + f] += u;
  } else {
    ubnd[size_t(sub) * nb + f] = u;
  }
}

// ---------------------------------------------------------------------- launchers

void launch_kappa(hipStream_t st, const Geo& g, const double* s, const double* K, double* kn, const double* km,
                  double* red, double* scal, int32_t* flag, int32_t* list, int32_t* count, int32_t* seq,
                  double* host, const double* wc_ux, const double* wc_uy, Runs rt, double* s_new, double area,
                  hipStream_t st_red, hipEvent_t ev_red) {
  const unsigned nr = runs_of(rt);
  // one thread per cell of the tile: the power of two from 64 to 256 that covers it (256 for
  // larger tiles)
  const unsigned bs = g.nc <= 64 ? 64 : g.nc <= 128 ? 128 : 256;
  if (s_new)
    hipLaunchKernelGGL(k_kappa<true>, dim3(g.nsub, 1, nr), dim3(bs), 0, st, g, s, s_new, K, kn, km, red, flag, list,
                       count, scal, wc_ux, wc_uy, area, rt.tab);
  else
    hipLaunchKernelGGL(k_kappa<false>, dim3(g.nsub, 1, nr), dim3(bs), 0, st, g, s, s_new, K, kn, km, red, flag,
                       list, count, scal, wc_ux, wc_uy, area, rt.tab);
  if (st_red) {
    hipEventRecord(ev_red, st);
    hipStreamWaitEvent(st_red, ev_red, 0);
  }
  hipLaunchKernelGGL(k_reduce_eps, dim3(1, 1, nr), dim3(256), 0, st_red ? st_red : st, g.nsub,
                     wc_ux != nullptr ? 1 : 0, red, scal, seq, host, rt.tab);
}

void launch_dt(hipStream_t st, int nsub, const double* red_rate, const double* red_qin, double* scal,
               int32_t* count, Runs rt) {
  hipLaunchKernelGGL(k_dt, dim3(1, 1, runs_of(rt)), dim3(256), 0, st, nsub, red_rate, red_qin, scal, count, rt.tab);
}

void launch_flux(hipStream_t st, const Geo& g, const double* km, const double* S, const double* h,
                 const double* vbnd, const double* y, const int32_t* sub_dofs, double* ubnd, int with_v,
                 Runs rt) {
  if (g.nb > 64)
    hipLaunchKernelGGL(k_flux_wide, dim3(g.nsub, 1, runs_of(rt)), dim3(128), 0, st, g, km, S, h, vbnd, y, sub_dofs,
                       ubnd, with_v, rt.tab);
  else
    hipLaunchKernelGGL(k_flux, dim3(g.nsub, 1, runs_of(rt)), dim3(64), 0, st, g, km, S, h, vbnd, y, sub_dofs, ubnd,
                       with_v, rt.tab);
}

}  // namespace mpm
