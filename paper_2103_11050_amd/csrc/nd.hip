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
// no pivoting), C = old row panel A_K*, R = Pinv C. One workgroup per node.
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
  double* C = Pinv + pb * pb;
  double* R = C + int64_t(pb) * n;
  for (int e = threadIdx.x; e < bs * bs; e += blockDim.x) {
    const int i = e / bs, j = e % bs;
    P[i * 33 + j] = F[int64_t(K0 + i) * n + K0 + j];
  }
  for (int64_t e = threadIdx.x; e < int64_t(bs) * n; e += blockDim.x) {
    const int k = int(e / n), j = int(e % n);
    C[int64_t(k) * n + j] = F[int64_t(K0 + k) * n + j];
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
  __syncthreads();
  // R = Pinv C (bs x n)
  for (int64_t e = threadIdx.x; e < int64_t(bs) * n; e += blockDim.x) {
    const int k = int(e / n), j = int(e % n);
    double v = 0.0;
    for (int t = 0; t < bs; ++t) v += -P[k * 33 + t] * C[int64_t(t) * n + j];
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

// Forward: gather the children's condensed right-hand sides into the node's front vector.
__global__ void __launch_bounds__(256) k_nd_fwd_gather(NdArgs a, int loff) {
  extern __shared__ double f[];
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.x]];
  for (int i = threadIdx.x; i < nd.n; i += blockDim.x) f[i] = 0.0;
  __syncthreads();
  for (int c = 0; c < 2; ++c) {
    const double* src = child_c(a, nd, c);
    const int32_t* map = a.map_pool + nd.map_off[c];
    for (int i = threadIdx.x; i < nd.nB_child[c]; i += blockDim.x) f[map[i]] += src[i];
    __syncthreads();
  }
  for (int i = threadIdx.x; i < nd.nI; i += blockDim.x) a.fI[nd.fI_off + i] = f[i];
  for (int i = threadIdx.x; i < nd.nB; i += blockDim.x) a.cB[nd.cB_off + i] = f[nd.nI + i];
}

// Forward: c_B = f_B - BI f_I, one wavefront per row.
__global__ void __launch_bounds__(256) k_nd_fwd_gemv(NdArgs a, int loff) {
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= nd.nB) return;
  const double* row = a.front + nd.front_off + int64_t(nd.nI + r) * nd.n;
  const double* fI = a.fI + nd.fI_off;
  double acc = 0.0;
  for (int i = lane; i < nd.nI; i += 64) acc += row[i] * fI[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) a.cB[nd.cB_off + r] -= acc;
}

// Backward: x_I = -II f_I - IB x_B, one wavefront per row; scatters x_I into y.
__global__ void __launch_bounds__(256) k_nd_bwd(NdArgs a, int loff) {
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= nd.nI) return;
  const double* row = a.front + nd.front_off + int64_t(r) * nd.n;
  const double* fI = a.fI + nd.fI_off;
  const int32_t* dofs = a.dof_pool + nd.dof_off;
  double acc = 0.0;
  for (int i = lane; i < nd.nI; i += 64) acc += row[i] * fI[i];
  for (int j = lane; j < nd.nB; j += 64) acc += row[nd.nI + j] * a.y[dofs[nd.nI + j]];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) a.y[dofs[r]] = -acc;
}

void launch_nd_level_factor(hipStream_t st, const NdArgs& a, int loff, int nnodes, int nmax, int nImax) {
  const int zb = std::min<int64_t>((int64_t(nmax) * nmax + 255) / 256, 1024);
  hipLaunchKernelGGL(k_nd_zero, dim3(zb, nnodes), dim3(256), 0, st, a, loff);
  for (int c = 0; c < 2; ++c) hipLaunchKernelGGL(k_nd_extend, dim3(zb, nnodes), dim3(256), 0, st, a, loff, c);
  const int nblk = (nImax + a.piv_b - 1) / a.piv_b;
  const int tpd = (nmax + TILE - 1) / TILE;
  for (int kb = 0; kb < nblk; ++kb) {
    hipLaunchKernelGGL(k_nd_pivot, dim3(nnodes), dim3(256), 0, st, a, loff, kb);
    hipLaunchKernelGGL(k_nd_update, dim3(tpd * tpd, nnodes), dim3(256), 0, st, a, loff, kb);
  }
}

void launch_nd_level_fwd(hipStream_t st, const NdArgs& a, int loff, int nnodes, int nmax, int nBmax) {
  hipLaunchKernelGGL(k_nd_fwd_gather, dim3(nnodes), dim3(256), size_t(nmax) * 8, st, a, loff);
  if (nBmax > 0) hipLaunchKernelGGL(k_nd_fwd_gemv, dim3((nBmax + 3) / 4, nnodes), dim3(256), 0, st, a, loff);
}

void launch_nd_level_bwd(hipStream_t st, const NdArgs& a, int loff, int nnodes, int nImax) {
  hipLaunchKernelGGL(k_nd_bwd, dim3((nImax + 3) / 4, nnodes), dim3(256), 0, st, a, loff);
}

}  // namespace mpm
