// Interface system (eq:mrc2) by nested dissection of the skeleton.
//
// The global matrix is the sum over subdomains of K_i = B_i^T S_i B_i - D_i (the Robin rows
// negated, which makes it symmetric; it is quasi-definite: negative definite on the flux
// unknowns, positive definite on the pressure unknowns, so every principal submatrix of every
// Schur complement is non-singular and no pivoting is needed).
//
// Recursive bisection of the subdomain grid gives a tree; a node's front holds the unknowns
// of its separator (I) and of its outer boundary (B). Factorisation, level by level from the
// leaves: extend-add the children's Schur complements into the front, then sweep the I
// unknowns in blocks of piv_b. After the sweep the front holds
//   II = -F_II^-1,  IB = F_II^-1 F_IB,  BI = F_BI F_II^-1,  BB = F_BB - F_BI F_II^-1 F_IB.
// Solve: forward (leaves to root) c_B = f_B - BI f_I; backward (root to leaves)
//   x_I = -II f_I - IB x_B.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace mpm {

namespace {

constexpr int TILE = 64;

__device__ __forceinline__ const double* child_S(const NdArgs& a, const NodeDev& nd, int c, int* stride, int* off) {
  const int ch = nd.child[c];
  if (ch < 0) {
    const int sub = -1 - ch;
    *stride = nd.nB_child[c];
    *off = 0;
    return a.leafK + size_t(sub) * a.ndmax * a.ndmax;
  }
  const NodeDev& cn = a.nodes[ch];
  *stride = cn.n;
  *off = cn.nI;
  return a.front + cn.front_off;
}

__device__ __forceinline__ const double* child_c(const NdArgs& a, const NodeDev& nd, int c) {
  const int ch = nd.child[c];
  if (ch < 0) return a.leafr + size_t(-1 - ch) * a.ndmax;
  return a.cB + a.nodes[ch].cB_off;
}

}  // namespace

__global__ void k_nd_zero(NdArgs a, int loff) {
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int64_t n2 = int64_t(nd.n) * nd.n;
  double* F = a.front + nd.front_off;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n2; e += int64_t(gridDim.x) * blockDim.x) F[e] = 0.0;
}

// Adds child c's Schur complement into the parent front (one child per launch: deterministic).
__global__ void k_nd_extend(NdArgs a, int loff, int c) {
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int nBc = nd.nB_child[c];
  int stride, off;
  const double* S = child_S(a, nd, c, &stride, &off);
  const int32_t* map = a.map_pool + nd.map_off[c];
  double* F = a.front + nd.front_off;
  const int64_t tot = int64_t(nBc) * nBc;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(e / nBc), j = int(e % nBc);
    F[int64_t(map[i]) * nd.n + map[j]] += S[int64_t(off + i) * stride + off + j];
  }
}

// Pivot block kb of every node of the level: P = A_KK, Pinv = P^-1 (Gauss-Jordan sweep in LDS,
// no pivoting). One workgroup per node.
__global__ void __launch_bounds__(256) k_nd_pivot(NdArgs a, int loff, int kb) {
  __shared__ double P[32 * 33];
  __shared__ double colk[32], rowk[32];
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.x]];
  const int pb = a.piv_b;
  const int K0 = kb * pb;
  if (K0 >= nd.nI) return;
  const int bs = min(pb, nd.nI - K0);
  const int n = nd.n;
  const double* F = a.front + nd.front_off;
  double* Pinv = a.panel + nd.panel_off;
  for (int e = threadIdx.x; e < bs * bs; e += blockDim.x) {
    const int i = e / bs, j = e % bs;
    P[i * 33 + j] = F[int64_t(K0 + i) * n + K0 + j];
  }
  __syncthreads();
  // sweep operator on every index of P: afterwards P = -P_orig^-1
  bool ok = true;
  for (int k = 0; k < bs; ++k) {
    const double d = P[k * 33 + k];
    if (!(d != 0.0) || !isfinite(d)) ok = false;
    const double rd = 1.0 / d;
    if (threadIdx.x < bs) {
      colk[threadIdx.x] = P[threadIdx.x * 33 + k];
      rowk[threadIdx.x] = P[k * 33 + threadIdx.x];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < bs * bs; e += blockDim.x) {
      const int i = e / bs, j = e % bs;
      double v;
      if (i == k && j == k) v = -rd;
      else if (i == k) v = rowk[j] * rd;
      else if (j == k) v = colk[i] * rd;
      else v = P[i * 33 + j] - colk[i] * rowk[j] * rd;
      P[i * 33 + j] = v;
    }
    __syncthreads();
  }
  if (!ok && threadIdx.x == 0) set_error(a.err, ERR_SINGULAR);
  for (int e = threadIdx.x; e < bs * bs; e += blockDim.x) {
    const int i = e / bs, j = e % bs;
    Pinv[i * pb + j] = -P[i * 33 + j];
  }
}

// Row panel of pivot block kb: C = old rows A_K* (copied, the update overwrites them) and
// R = Pinv C, 64 columns per workgroup.
__global__ void __launch_bounds__(256) k_nd_rpanel(NdArgs a, int loff, int kb) {
  __shared__ double Pi[32][33];
  __shared__ double Cs[32][65];
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int pb = a.piv_b;
  const int K0 = kb * pb;
  if (K0 >= nd.nI) return;
  const int bs = min(pb, nd.nI - K0);
  const int n = nd.n;
  const int j0 = blockIdx.x * 64;
  if (j0 >= n) return;
  const double* F = a.front + nd.front_off;
  const double* Pinv = a.panel + nd.panel_off;
  double* C = a.panel + nd.panel_off + pb * pb;
  double* R = C + int64_t(pb) * n;
  for (int e = threadIdx.x; e < bs * bs; e += blockDim.x) Pi[e / bs][e % bs] = Pinv[(e / bs) * pb + e % bs];
  for (int e = threadIdx.x; e < bs * 64; e += blockDim.x) {
    const int k = e / 64, t = e % 64;
    const int j = j0 + t;
    double v = 0.0;
    if (j < n) {
      v = F[int64_t(K0 + k) * n + j];
      C[int64_t(k) * n + j] = v;
    }
    Cs[k][t] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < bs * 64; e += blockDim.x) {
    const int k = e / 64, t = e % 64;
    const int j = j0 + t;
    if (j >= n) continue;
    double v = 0.0;
    for (int u = 0; u < bs; ++u) v += Pi[k][u] * Cs[u][t];
    R[int64_t(k) * n + j] = v;
  }
}

// Block sweep update of every front entry (64x64 tiles):
//   i,j not in K : A_ij -= sum_k C_ki R_kj
//   i not in K, j in K : A_ij = R_(j-K0) i
//   i in K, j not in K : A_ij = R_(i-K0) j
//   i,j in K : A_ij = -Pinv
__global__ void __launch_bounds__(256) k_nd_update(NdArgs a, int loff, int kb) {
  __shared__ double Cs[32][TILE + 1];
  __shared__ double Rs[32][TILE + 1];
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int pb = a.piv_b;
  const int K0 = kb * pb;
  if (K0 >= nd.nI) return;
  const int bs = min(pb, nd.nI - K0);
  const int n = nd.n;
  const int tpd = (n + TILE - 1) / TILE;
  const int ti = blockIdx.x / tpd, tj = blockIdx.x % tpd;
  if (ti >= tpd) return;
  const double* Pinv = a.panel + nd.panel_off;
  const double* C = Pinv + pb * pb;
  const double* R = C + int64_t(pb) * n;
  double* F = a.front + nd.front_off;
  const int i0 = ti * TILE, j0 = tj * TILE;
  for (int e = threadIdx.x; e < bs * TILE; e += blockDim.x) {
    const int k = e / TILE, t = e % TILE;
    Cs[k][t] = (i0 + t < n) ? C[int64_t(k) * n + i0 + t] : 0.0;
    Rs[k][t] = (j0 + t < n) ? R[int64_t(k) * n + j0 + t] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  for (int ii = 0; ii < 4; ++ii) {
    const int li = ty + 16 * ii;
    const int i = i0 + li;
    if (i >= n) continue;
    const bool inKi = i >= K0 && i < K0 + bs;
    for (int jj = 0; jj < 4; ++jj) {
      const int lj = tx + 16 * jj;
      const int j = j0 + lj;
      if (j >= n) continue;
      const bool inKj = j >= K0 && j < K0 + bs;
      double* dst = F + int64_t(i) * n + j;
      if (!inKi && !inKj) {
        double acc = 0.0;
        for (int k = 0; k < bs; ++k) acc += Cs[k][li] * Rs[k][lj];
        *dst -= acc;
      } else if (!inKi && inKj) {
        *dst = R[int64_t(j - K0) * n + i];
      } else if (inKi && !inKj) {
        *dst = Rs[i - K0][lj];
      } else {
        *dst = -Pinv[(i - K0) * pb + (j - K0)];
      }
    }
  }
}

// Forward, one level. Every workgroup gathers its node's front right-hand side f (children's
// condensed vectors, child 0 then child 1) into LDS; workgroup 0 stores f_I for the backward
// pass; then groups of G lanes form c_B[j] = f_B[j] - (BI f_I)[j] for rows j of the stored BI
// block (row-major, so each group reads one contiguous row).
__global__ void __launch_bounds__(256) k_nd_fwd(NdArgs a, int loff, int G, int rows_per_block) {
  extern __shared__ double f[];
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int r0 = blockIdx.x * rows_per_block;
  if (r0 >= max(nd.nB, 1)) return;
  for (int i = threadIdx.x; i < nd.n; i += blockDim.x) f[i] = 0.0;
  __syncthreads();
  for (int c = 0; c < 2; ++c) {
    const double* src = child_c(a, nd, c);
    const int32_t* map = a.map_pool + nd.map_off[c];
    for (int i = threadIdx.x; i < nd.nB_child[c]; i += blockDim.x) f[map[i]] += src[i];
    __syncthreads();
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < nd.nI; i += blockDim.x) a.fI[nd.fI_off + i] = f[i];
  const int gl = threadIdx.x % G, grp = threadIdx.x / G;
  const int r1 = min(nd.nB, r0 + rows_per_block);
  for (int j = r0 + grp; j < r1; j += 256 / G) {
    const double* row = a.front + nd.front_off + int64_t(nd.nI + j) * nd.n;
    double acc4[4] = {0, 0, 0, 0};
    int k = gl;
    for (; k + 3 * G < nd.nI; k += 4 * G) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc4[u] += row[k + u * G] * f[k + u * G];
    }
    for (; k < nd.nI; k += G) acc4[0] += row[k] * f[k];
    double acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (gl == 0) a.cB[nd.cB_off + j] = f[nd.nI + j] - acc;
  }
}

// Backward, one level: v = [f_I; x_B] in LDS (x_B gathered from the solution by the node's
// unknown list), then x_I = -[II IB] v, one group of G lanes per row.
__global__ void __launch_bounds__(256) k_nd_bwd(NdArgs a, int loff, int G, int rows_per_block) {
  extern __shared__ double v[];
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int r0 = blockIdx.x * rows_per_block;
  if (r0 >= nd.nI) return;
  const int32_t* dofs = a.dof_pool + nd.dof_off;
  for (int i = threadIdx.x; i < nd.nI; i += blockDim.x) v[i] = a.fI[nd.fI_off + i];
  for (int i = threadIdx.x; i < nd.nB; i += blockDim.x) v[nd.nI + i] = a.y[dofs[nd.nI + i]];
  __syncthreads();
  const int gl = threadIdx.x % G, grp = threadIdx.x / G;
  const int r1 = min(nd.nI, r0 + rows_per_block);
  for (int r = r0 + grp; r < r1; r += 256 / G) {
    const double* row = a.front + nd.front_off + int64_t(r) * nd.n;
    double acc4[4] = {0, 0, 0, 0};
    int k = gl;
    for (; k + 3 * G < nd.n; k += 4 * G) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc4[u] += row[k + u * G] * v[k + u * G];
    }
    for (; k < nd.n; k += G) acc4[0] += row[k] * v[k];
    double acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (gl == 0) a.y[dofs[r]] = -acc;
  }
}

// Register-batched forms of the two sweeps. A workgroup takes RP x (256/G) rows of one node,
// G lanes per row, U columns per lane, and issues every load of its block (and of the vector
// it multiplies) before the first use, so that one level costs about two memory round trips
// (indices, then everything else) rather than one per row. Loads are unconditional at clamped
// (valid) addresses and masked afterwards, so the compiler keeps them all in flight. No LDS and
// no barriers: the forward right-hand side is gathered per lane through the inverse
// extend-add maps.
template <int G, int U, int RP>
__global__ void __launch_bounds__(256) k_nd_fwd_rb(NdArgs a, int loff) {
  constexpr int RPP = 256 / G, RPB = RP * RPP;
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int r0 = blockIdx.x * RPB;
  if (r0 >= max(nd.nB, 1)) return;
  const int gl = threadIdx.x % G, grp = threadIdx.x / G;
  const double* __restrict__ F = a.front + nd.front_off;
  const int32_t* __restrict__ inv0 = a.inv_pool + nd.inv_off;
  const int32_t* __restrict__ inv1 = inv0 + nd.n;
  const double* __restrict__ src0 = child_c(a, nd, 0);
  const double* __restrict__ src1 = child_c(a, nd, 1);
  const int nI1 = max(nd.nI, 1) - 1, nB1 = max(nd.nB, 1) - 1;
  // indices of f at this lane's columns (k < nI) and rows (nI + j)
  int ik0[U], ik1[U], ib0[RP], ib1[RP];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = min(gl + u * G, nI1);
    ik0[u] = inv0[k];
    ik1[u] = inv1[k];
  }
  double m[RP][U];
  if (nd.nB > 0) {
#pragma unroll
    for (int p = 0; p < RP; ++p) {
      const int j = min(r0 + p * RPP + grp, nB1);
      ib0[p] = inv0[nd.nI + j];
      ib1[p] = inv1[nd.nI + j];
    }
#pragma unroll
    for (int p = 0; p < RP; ++p) {
      const int j = min(r0 + p * RPP + grp, nB1);
#pragma unroll
      for (int u = 0; u < U; ++u) m[p][u] = F[int64_t(nd.nI + j) * nd.n + min(gl + u * G, nI1)];
    }
  } else {
    // the root: no boundary rows, only f_I is stored
#pragma unroll
    for (int p = 0; p < RP; ++p) {
      ib0[p] = -1;
      ib1[p] = -1;
#pragma unroll
      for (int u = 0; u < U; ++u) m[p][u] = 0.0;
    }
  }
  double fk[U], fb[RP];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const double x0 = src0[max(ik0[u], 0)], x1 = src1[max(ik1[u], 0)];
    fk[u] = (ik0[u] >= 0 ? x0 : 0.0) + (ik1[u] >= 0 ? x1 : 0.0);
  }
#pragma unroll
  for (int p = 0; p < RP; ++p) {
    const double x0 = src0[max(ib0[p], 0)], x1 = src1[max(ib1[p], 0)];
    fb[p] = (ib0[p] >= 0 ? x0 : 0.0) + (ib1[p] >= 0 ? x1 : 0.0);
  }
  if (blockIdx.x == 0 && grp == 0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = gl + u * G;
      if (k < nd.nI) a.fI[nd.fI_off + k] = fk[u];
    }
  }
#pragma unroll
  for (int p = 0; p < RP; ++p) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) acc += (gl + u * G < nd.nI) ? m[p][u] * fk[u] : 0.0;
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    const int j = r0 + p * RPP + grp;
    if (gl == 0 && j < nd.nB) a.cB[nd.cB_off + j] = fb[p] - acc;
  }
}

template <int G, int U, int RP>
__global__ void __launch_bounds__(256) k_nd_bwd_rb(NdArgs a, int loff) {
  constexpr int RPP = 256 / G, RPB = RP * RPP;
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int r0 = blockIdx.x * RPB;
  if (r0 >= nd.nI) return;
  const int gl = threadIdx.x % G, grp = threadIdx.x / G;
  const double* __restrict__ F = a.front + nd.front_off;
  const int32_t* __restrict__ dofs = a.dof_pool + nd.dof_off;
  const int n1 = nd.n - 1, nI1 = nd.nI - 1;
  // v = [f_I; x_B]: unknown ids of this lane's columns first
  int dk[U];
#pragma unroll
  for (int u = 0; u < U; ++u) dk[u] = dofs[min(gl + u * G, n1)];
  int dr[RP];
#pragma unroll
  for (int p = 0; p < RP; ++p) dr[p] = dofs[min(r0 + p * RPP + grp, nI1)];
  double m[RP][U];
#pragma unroll
  for (int p = 0; p < RP; ++p) {
    const int r = min(r0 + p * RPP + grp, nI1);
#pragma unroll
    for (int u = 0; u < U; ++u) m[p][u] = F[int64_t(r) * nd.n + min(gl + u * G, n1)];
  }
  double v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = gl + u * G;
    const double xi = a.fI[nd.fI_off + min(k, nI1)];
    const double xb = a.y[dk[u]];
    v[u] = k < nd.nI ? xi : (k < nd.n ? xb : 0.0);
  }
#pragma unroll
  for (int p = 0; p < RP; ++p) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) acc += m[p][u] * v[u];
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    const int r = r0 + p * RPP + grp;
    if (gl == 0 && r < nd.nI) a.y[dr[p]] = -acc;
  }
}

// Bottom levels fused: one workgroup walks one subtree, children before parents (forward)
// or parents before children (backward); the per-node work is that of k_nd_fwd / k_nd_bwd.
__global__ void __launch_bounds__(256) k_nd_fwd_fused(NdArgs a) {
  extern __shared__ double f[];
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int idx = a.fuse_off[blockIdx.x]; idx < a.fuse_off[blockIdx.x + 1]; ++idx) {
    const NodeDev nd = a.nodes[a.fuse_nodes[idx]];
    for (int i = threadIdx.x; i < nd.n; i += blockDim.x) f[i] = 0.0;
    __syncthreads();
    for (int c = 0; c < 2; ++c) {
      const double* src = child_c(a, nd, c);
      const int32_t* map = a.map_pool + nd.map_off[c];
      for (int i = threadIdx.x; i < nd.nB_child[c]; i += blockDim.x) f[map[i]] += src[i];
      __syncthreads();
    }
    for (int i = threadIdx.x; i < nd.nI; i += blockDim.x) a.fI[nd.fI_off + i] = f[i];
    for (int j0 = 0; j0 < nd.nB; j0 += 64) {
      const int j = j0 + lane;
      double acc = 0.0;
      if (j < nd.nB) {
        const double* col = a.front + nd.front_off + nd.nI + j;
        for (int i = wv; i < nd.nI; i += 4) acc += col[int64_t(i) * nd.n] * f[i];
      }
      part[wv][lane] = acc;
      __syncthreads();
      if (wv == 0 && j < nd.nB)
        a.cB[nd.cB_off + j] = f[nd.nI + j] - (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(256) k_nd_bwd_fused(NdArgs a) {
  extern __shared__ double v[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int idx = a.fuse_off[blockIdx.x + 1] - 1; idx >= a.fuse_off[blockIdx.x]; --idx) {
    const NodeDev nd = a.nodes[a.fuse_nodes[idx]];
    const int32_t* dofs = a.dof_pool + nd.dof_off;
    for (int i = threadIdx.x; i < nd.nI; i += blockDim.x) v[i] = a.fI[nd.fI_off + i];
    for (int i = threadIdx.x; i < nd.nB; i += blockDim.x) v[nd.nI + i] = a.y[dofs[nd.nI + i]];
    __syncthreads();
    for (int r = wv; r < nd.nI; r += 4) {
      const double* row = a.front + nd.front_off + int64_t(r) * nd.n;
      double acc = 0.0;
      for (int k = lane; k < nd.n; k += 64) acc += row[k] * v[k];
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
      if (lane == 0) a.y[dofs[r]] = -acc;
    }
    __syncthreads();
  }
}

void launch_nd_fused_fwd(hipStream_t st, const NdArgs& a, int nroots, int nmax) {
  hipLaunchKernelGGL(k_nd_fwd_fused, dim3(nroots), dim3(256), size_t(nmax) * 8, st, a);
}

void launch_nd_fused_bwd(hipStream_t st, const NdArgs& a, int nroots, int nmax) {
  hipLaunchKernelGGL(k_nd_bwd_fused, dim3(nroots), dim3(256), size_t(nmax) * 8, st, a);
}

void launch_nd_level_factor(hipStream_t st, const NdArgs& a, int loff, int nnodes, int nmax, int nImax) {
  const int zb = std::min<int64_t>((int64_t(nmax) * nmax + 255) / 256, 1024);
  hipLaunchKernelGGL(k_nd_zero, dim3(zb, nnodes), dim3(256), 0, st, a, loff);
  for (int c = 0; c < 2; ++c) hipLaunchKernelGGL(k_nd_extend, dim3(zb, nnodes), dim3(256), 0, st, a, loff, c);
  const int nblk = (nImax + a.piv_b - 1) / a.piv_b;
  const int tpd = (nmax + TILE - 1) / TILE;
  for (int kb = 0; kb < nblk; ++kb) {
    hipLaunchKernelGGL(k_nd_pivot, dim3(nnodes), dim3(256), 0, st, a, loff, kb);
    hipLaunchKernelGGL(k_nd_rpanel, dim3(tpd, nnodes), dim3(256), 0, st, a, loff, kb);
    hipLaunchKernelGGL(k_nd_update, dim3(tpd * tpd, nnodes), dim3(256), 0, st, a, loff, kb);
  }
}

static int group_for(int len) { return len <= 48 ? 16 : (len <= 96 ? 32 : 64); }

// Rows per workgroup: a multiple of the rows one pass covers, sized for ~2048 workgroups.
static int rows_per_block(int nrows, int nnodes, int G) {
  const int per_pass = 256 / G;
  const int wg_per_node = std::max(1, std::min((nrows + per_pass - 1) / per_pass, (2048 + nnodes - 1) / nnodes));
  const int rpb = (nrows + wg_per_node - 1) / wg_per_node;
  return std::max(per_pass, (rpb + per_pass - 1) / per_pass * per_pass);
}

// Register-batched shape for a row length: lanes per row, columns per lane, rows per lane
// group (about eight loads of the block per lane). Returns false past the largest shape.
struct RbShape {
  int G, U, RP;
};
static bool rb_shape(int len, RbShape* sh) {
  if (len <= 16) *sh = {16, 1, 8};
  else if (len <= 32) *sh = {32, 1, 8};
  else if (len <= 64) *sh = {64, 1, 8};
  else if (len <= 128) *sh = {64, 2, 4};
  else if (len <= 256) *sh = {64, 4, 2};
  else if (len <= 512) *sh = {64, 8, 1};
  else if (len <= 1024) *sh = {64, 16, 1};
  else if (len <= 1536) *sh = {64, 24, 1};
  else if (len <= 2048) *sh = {64, 32, 1};
  else return false;
  return true;
}

#define ND_RB_LAUNCH(KER, sh, rows, nnodes, st, a, loff)                                              \
  do {                                                                                              \
    const int rpb_ = (sh).RP * (256 / (sh).G);                                                      \
    const dim3 grid_(std::max(1, ((rows) + rpb_ - 1) / rpb_), (nnodes));                          \
    if ((sh).G == 16) hipLaunchKernelGGL((KER<16, 1, 8>), grid_, dim3(256), 0, st, a, loff);        \
    else if ((sh).G == 32) hipLaunchKernelGGL((KER<32, 1, 8>), grid_, dim3(256), 0, st, a, loff);   \
    else if ((sh).U == 1) hipLaunchKernelGGL((KER<64, 1, 8>), grid_, dim3(256), 0, st, a, loff);    \
    else if ((sh).U == 2) hipLaunchKernelGGL((KER<64, 2, 4>), grid_, dim3(256), 0, st, a, loff);    \
    else if ((sh).U == 4) hipLaunchKernelGGL((KER<64, 4, 2>), grid_, dim3(256), 0, st, a, loff);    \
    else if ((sh).U == 8) hipLaunchKernelGGL((KER<64, 8, 1>), grid_, dim3(256), 0, st, a, loff);    \
    else if ((sh).U == 16) hipLaunchKernelGGL((KER<64, 16, 1>), grid_, dim3(256), 0, st, a, loff);  \
    else if ((sh).U == 24) hipLaunchKernelGGL((KER<64, 24, 1>), grid_, dim3(256), 0, st, a, loff);  \
    else hipLaunchKernelGGL((KER<64, 32, 1>), grid_, dim3(256), 0, st, a, loff);                    \
  } while (0)

void launch_nd_level_fwd(hipStream_t st, const NdArgs& a, int loff, int nnodes, int nmax, int nImax, int nBmax) {
  RbShape sh;
  if (rb_shape(nImax, &sh)) {
    ND_RB_LAUNCH(k_nd_fwd_rb, sh, std::max(nBmax, 1), nnodes, st, a, loff);
    return;
  }
  const int G = group_for(nImax);
  const int rpb = rows_per_block(std::max(nBmax, 1), nnodes, G);
  const int gx = std::max(1, (nBmax + rpb - 1) / rpb);
  hipLaunchKernelGGL(k_nd_fwd, dim3(gx, nnodes), dim3(256), size_t(nmax) * 8, st, a, loff, G, rpb);
}

void launch_nd_level_bwd(hipStream_t st, const NdArgs& a, int loff, int nnodes, int nImax, int nmax) {
  RbShape sh;
  if (rb_shape(nmax, &sh)) {
    ND_RB_LAUNCH(k_nd_bwd_rb, sh, nImax, nnodes, st, a, loff);
    return;
  }
  const int G = group_for(nmax);
  const int rpb = rows_per_block(nImax, nnodes, G);
  hipLaunchKernelGGL(k_nd_bwd, dim3((nImax + rpb - 1) / rpb, nnodes), dim3(256), size_t(nmax) * 8, st, a, loff, G, rpb);
}

}  // namespace mpm
