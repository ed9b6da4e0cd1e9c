// Saturation transport (eq. BL2D): explicit Euler in time with first-order upwind fluxes and
// the velocity frozen over the sub-steps (Section 4). HBM-bound stencil: each thread updates
// one cell from its four face fluxes and the upwind saturations.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "kernels.hpp"

namespace mpm {

// s2 = s - dt/|c| sum_f |f| u_f f(s_upwind); the injected saturation on inflow boundary faces.
__global__ void __launch_bounds__(256)
k_sat_step(Geo g, const double* __restrict__ s, double* __restrict__ s2, const double* __restrict__ ux,
           const double* __restrict__ uy, double* __restrict__ scal, double area, const RunTab* __restrict__ rt) {
  {
    const int64_t wo = ws_off(rt);
    s = at_off(s, wo);
    s2 = at_off(s2, wo);
    ux = at_off(ux, wo);
    uy = at_off(uy, wo);
    scal = at_off(scal, wo);
  }
  const int gi = blockIdx.x * 64 + (threadIdx.x & 63);
  const int gj = blockIdx.y * 4 + (threadIdx.x >> 6);
  const double dt = scal[SC_DT];
  const double M = scal[SC_MRATIO];
  if (gi < g.nx && gj < g.ny) s2[gj * g.nx + gi] = sat_cell(g, s, ux, uy, gi, gj, dt, M);
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    scal[SC_T] += dt;
    scal[SC_PVI] += dt * scal[SC_QIN] / area;
  }
}

// Water cut over boundary faces with outflow: sum |f| u f(s_c) / sum |f| u. Each workgroup
// takes a contiguous range of the boundary faces and writes its two partial sums; the last one
// to finish (ticket) adds the partials in workgroup order and resets the ticket, so the result
// does not depend on the order in which the workgroups ran.
constexpr int WC_MAX_BLOCKS = 64;
__global__ void __launch_bounds__(256)
k_water_cut(Geo g, const double* __restrict__ s, const double* __restrict__ ux, const double* __restrict__ uy,
            double* __restrict__ scal, double* __restrict__ part, int32_t* __restrict__ ticket, int per,
            const RunTab* __restrict__ rt) {
  {
    const int64_t wo = ws_off(rt);
    s = at_off(s, wo);
    ux = at_off(ux, wo);
    uy = at_off(uy, wo);
    scal = at_off(scal, wo);
    part = at_off(part, wo);
    ticket = at_off(ticket, wo);
  }
  const double M = scal[SC_MRATIO];
  __shared__ double sq[256], sw[256];
  __shared__ int last;
  double q = 0.0, w = 0.0;
  const int nW = g.ny, nS = g.nx;
  const int tot = 2 * nW + 2 * nS;
  const int lo = blockIdx.x * per, hi = min(tot, lo + per);
  for (int base = lo; base < hi; base += 256 * 4) {
    double vu[4], vs[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e0 = base + threadIdx.x + 256 * u;
      const DomFace d = dom_face(g, e0 < hi ? e0 : lo);
      const double uv = (d.vert ? ux : uy)[d.ui];
      vu[u] = d.hi ? uv : -uv;
      vs[u] = s[d.si];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + threadIdx.x + 256 * u;
      if (e < hi) {
        const double fl = e < 2 * nW ? g.hy : g.hx;
        const double out = fl * fmax(vu[u], 0.0);
        q += out;
        w += out * frac_w(vs[u], M);
      }
    }
  }
  auto tree = [&]() {
    sq[threadIdx.x] = q;
    sw[threadIdx.x] = w;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) {
        sq[threadIdx.x] += sq[threadIdx.x + o];
        sw[threadIdx.x] += sw[threadIdx.x + o];
      }
      __syncthreads();
    }
  };
  tree();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sq[0];
    part[2 * blockIdx.x + 1] = sw[0];
    __threadfence();
    last = atomicAdd(ticket, 1) == int(gridDim.x) - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  q = threadIdx.x < gridDim.x ? part[2 * threadIdx.x] : 0.0;
  w = threadIdx.x < gridDim.x ? part[2 * threadIdx.x + 1] : 0.0;
  __syncthreads();
  tree();
  if (threadIdx.x == 0) {
    scal[SC_WCUT] = sq[0] > 0.0 ? sw[0] / sq[0] : 0.0;
    *ticket = 0;
  }
}

void launch_sat_step(hipStream_t st, const Geo& g, const double* s, double* s2, const double* ux,
                     const double* uy, double* scal, double area, Runs rt) {
  dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4, runs_of(rt));
  hipLaunchKernelGGL(k_sat_step, grid, dim3(256), 0, st, g, s, s2, ux, uy, scal, area, rt.tab);
}

void launch_water_cut(hipStream_t st, const Geo& g, const double* s, const double* ux, const double* uy,
                      double* scal, double* part, int32_t* ticket, Runs rt) {
  const int tot = 2 * g.nx + 2 * g.ny;
  const int nblk = std::min(WC_MAX_BLOCKS, (tot + 255) / 256);
  const int per = (tot + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_water_cut, dim3((tot + per - 1) / per, 1, runs_of(rt)), dim3(256), 0, st, g, s, ux, uy,
                     scal, part, ticket, per, rt.tab);
}

}  // namespace mpm
