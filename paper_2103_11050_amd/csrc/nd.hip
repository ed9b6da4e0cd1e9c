// Interface system (eq:mrc2) by nested dissection of the skeleton.
//
// The global matrix is the sum over subdomains of K_i = B_i^T S_i B_i - D_i (the Robin rows
// negated, which makes it symmetric; it is quasi-definite: negative definite on the flux
// unknowns, positive definite on the pressure unknowns, so every principal submatrix of every
// Schur complement is non-singular and no pivoting is needed).
//
// Recursive bisection of the subdomain grid gives a tree; a node's front holds the unknowns
// of its separator (I) and of its outer boundary (B). Factorisation, level by level from the
// leaves: assemble the front from the children's Schur complements; sweep the I unknowns of
// the II block in blocks of piv_b (Gauss-Jordan, II := -F_II^-1); then on the matrix cores
// T = F_II^-1 F_IB and BB := F_BB - F_BI T, and IB := T, BI := T^T (F is symmetric). The front
// then holds
//   II = -F_II^-1,  IB = F_II^-1 F_IB,  BI = F_BI F_II^-1,  BB = F_BB - F_BI F_II^-1 F_IB.
// Solve: forward (leaves to root) c_B = f_B - BI f_I; backward (root to leaves)
//   x_I = -II f_I - IB x_B.
// In the forward sweep vectors travel between levels through slots (see NodeDev): a node's f
// is the sum of its two child slots, so every load of a forward level kernel is independent of
// the others. The backward sweep gathers x_B from the solution vector. The bottom levels of both
// sweeps can instead run as one launch per direction, one workgroup per subtree (end of file).
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

}  // namespace

// Front assembly (extend-add of both children's Schur complements, zero elsewhere), written
// row by row and gathered through the inverse maps: entry (k, l) is
// S0[inv0 k][inv0 l] + S1[inv1 k][inv1 l] with absent terms left out (child 0 first, the same
// sum as adding the children one after the other into a zeroed front).
constexpr int ASM_ROWS = 8;
__global__ void __launch_bounds__(256) k_nd_assemble(NdArgs a0, int loff, const RunTab* __restrict__ rt) {
  const NdArgs a = nd_at(a0, ws_off(rt));
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int n = nd.n;
  const int k0 = blockIdx.x * ASM_ROWS;
  if (k0 >= n) return;
  int st0, of0, st1, of1;
  const double* S0 = child_S(a, nd, 0, &st0, &of0);
  const double* S1 = child_S(a, nd, 1, &st1, &of1);
  const int32_t* inv0 = a.inv_pool + nd.inv_off;
  const int32_t* inv1 = inv0 + n;
  double* F = a.front + nd.front_off;
  const int k1 = min(n, k0 + ASM_ROWS);
  for (int l = threadIdx.x; l < n; l += 256) {
    const int b0 = inv0[l], b1 = inv1[l];
    for (int k = k0; k < k1; ++k) {
      const int a0 = inv0[k], a1 = inv1[k];
      double v = 0.0;
      if (a0 >= 0 && b0 >= 0) v = S0[int64_t(of0 + a0) * st0 + of0 + b0];
      if (a1 >= 0 && b1 >= 0) v += S1[int64_t(of1 + a1) * st1 + of1 + b1];
      F[int64_t(k) * n + l] = v;
    }
  }
}

// Pivot block kb of every node of the level: Pinv = A_KK^-1 by the sweep operator on the block
// held in registers (blocks of 32; one wavefront per node, lane l holds column l % 32 of rows
// 16 (l / 32) .. 16 (l / 32) + 15; a block smaller than 32 is padded with the identity, which
// the sweep leaves decoupled). No pivoting (the front is quasi-definite).
constexpr int PIV = 32;
__global__ void __launch_bounds__(64) k_nd_pivot(NdArgs a0, int loff, int kb, const RunTab* __restrict__ rt) {
  const NdArgs a = nd_at(a0, ws_off(rt));
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.x]];
  const int K0 = kb * PIV;
  if (K0 >= nd.nI) return;
  const int bs = min(PIV, nd.nI - K0);
  const int n = nd.n;
  const double* F = a.front + nd.front_off;
  double* Pinv = a.panel + nd.panel_off;
  const int lane = threadIdx.x, j = lane & 31, h = lane >> 5;
  double p[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 16 * h + r;
    p[r] = (i < bs && j < bs) ? F[int64_t(K0 + i) * n + K0 + j] : (i == j ? 1.0 : 0.0);
  }
  bool ok = true;
#pragma unroll
  for (int k = 0; k < PIV; ++k) {
    const double rowk = __shfl(p[k % 16], j + 32 * (k / 16));    // P[k][j]
    const double d = __shfl(p[k % 16], k + 32 * (k / 16));       // P[k][k]
    double colk[16];                                             // P[16 h + r][k]
#pragma unroll
    for (int r = 0; r < 16; ++r) colk[r] = __shfl(p[r], k + 32 * h);
    ok = ok && d != 0.0 && isfinite(d);
    const double rd = 1.0 / d;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 16 * h + r;
      double v;
      if (i == k && j == k) v = -rd;
      else if (i == k) v = rowk * rd;
      else if (j == k) v = colk[r] * rd;
      else v = p[r] - colk[r] * rowk * rd;
      p[r] = v;
    }
  }
  // afterwards p = -P^-1
  if (!ok && lane == 0) set_error(a.err, ERR_SINGULAR);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 16 * h + r;
    if (i < bs && j < bs) Pinv[i * PIV + j] = -p[r];
  }
}

// Row panel of pivot block kb over the II block: C = old rows A_K* (copied, the update
// overwrites them) and R = Pinv C, 64 columns per workgroup.
__global__ void __launch_bounds__(256) k_nd_rpanel(NdArgs a0, int loff, int kb, const RunTab* __restrict__ rt) {
  const NdArgs a = nd_at(a0, ws_off(rt));
  __shared__ double Pi[32][33];
  __shared__ double Cs[32][65];
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int pb = a.piv_b;
  const int K0 = kb * pb;
  if (K0 >= nd.nI) return;
  const int bs = min(pb, nd.nI - K0);
  const int n = nd.n, ext = nd.nI;
  const int j0 = blockIdx.x * 64;
  if (j0 >= ext) return;
  const double* F = a.front + nd.front_off;
  const double* Pinv = a.panel + nd.panel_off;
  double* C = a.panel + nd.panel_off + pb * pb;
  double* R = C + int64_t(pb) * n;
  for (int e = threadIdx.x; e < bs * bs; e += blockDim.x) Pi[e / bs][e % bs] = Pinv[(e / bs) * pb + e % bs];
  for (int e = threadIdx.x; e < bs * 64; e += blockDim.x) {
    const int k = e / 64, t = e % 64;
    const int j = j0 + t;
    double v = 0.0;
    if (j < ext) {
      v = F[int64_t(K0 + k) * n + j];
      C[int64_t(k) * n + j] = v;
    }
    Cs[k][t] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < bs * 64; e += blockDim.x) {
    const int k = e / 64, t = e % 64;
    const int j = j0 + t;
    if (j >= ext) continue;
    double v = 0.0;
    for (int u = 0; u < bs; ++u) v += Pi[k][u] * Cs[u][t];
    R[int64_t(k) * n + j] = v;
  }
}

// Block sweep update of every entry of the II block (64x64 tiles):
//   i,j not in K : A_ij -= sum_k C_ki R_kj
//   i not in K, j in K : A_ij = R_(j-K0) i
//   i in K, j not in K : A_ij = R_(i-K0) j
//   i,j in K : A_ij = -Pinv
__global__ void __launch_bounds__(256) k_nd_update(NdArgs a0, int loff, int kb, const RunTab* __restrict__ rt) {
  const NdArgs a = nd_at(a0, ws_off(rt));
  __shared__ double Cs[32][TILE + 1];
  __shared__ double Rs[32][TILE + 1];
  const NodeDev nd = a.nodes[a.levels[loff + blockIdx.y]];
  const int pb = a.piv_b;
  const int K0 = kb * pb;
  if (K0 >= nd.nI) return;
  const int bs = min(pb, nd.nI - K0);
  const int n = nd.n, ext = nd.nI;
  const int tpd = (ext + TILE - 1) / TILE;
  const int ti = blockIdx.x / tpd, tj = blockIdx.x % tpd;
  if (ti >= tpd) return;
  const double* Pinv = a.panel + nd.panel_off;
  const double* C = Pinv + pb * pb;
  const double* R = C + int64_t(pb) * n;
  double* F = a.front + nd.front_off;
  const int i0 = ti * TILE, j0 = tj * TILE;
  for (int e = threadIdx.x; e < bs * TILE; e += blockDim.x) {
    const int k = e / TILE, t = e % TILE;
    Cs[k][t] = (i0 + t < ext) ? C[int64_t(k) * n + i0 + t] : 0.0;
    Rs[k][t] = (j0 + t < ext) ? R[int64_t(k) * n + j0 + t] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  for (int ii = 0; ii < 4; ++ii) {
    const int li = ty + 16 * ii;
    const int i = i0 + li;
    if (i >= ext) continue;
    const bool inKi = i >= K0 && i < K0 + bs;
    for (int jj = 0; jj < 4; ++jj) {
      const int lj = tx + 16 * jj;
      const int j = j0 + lj;
      if (j >= ext) continue;
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

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Off the II block, on the FP64 matrix cores, 64 x 64 output tiles of every node of a level:
//   mode 0: T = -II F_IB = F_II^-1 F_IB  (nI x nB, into the node's panel, row stride nB)
//   mode 1: F_BB -= F_BI T               (nB x nB, in place)
// K (= nI) in chunks of 32 staged in LDS, the next chunk's loads issued before the current
// chunk's products. Four wavefronts, each a 32 x 32 quarter as 2 x 2 blocks of 16 x 16;
// v_mfma_f64_16x16x4 takes A[i][k] from lane 16 k + i and B[k][j] from lane 16 k + j and
// returns C[k' + 4 v][j] in lane 16 k' + j, register v.
constexpr int GK = 32;
__global__ void __launch_bounds__(256) k_nd_gemm(NdArgs a0, int loff, int mode, int tiles_n, const RunTab* __restrict__ rt) {
  const NdArgs a = nd_at(a0, ws_off(rt));
  const NodeDev nd = a.lnodes[loff + blockIdx.y];
  const int n = nd.n, nI = nd.nI, nB = nd.nB;
  const int M = mode ? nB : nI, N = nB, K = nI;
  const int i0 = int(blockIdx.x / tiles_n) * 64, j0 = int(blockIdx.x % tiles_n) * 64;
  if (i0 >= M || j0 >= N || K <= 0) return;
  double* F = a.front + nd.front_off;
  double* T = a.panel + nd.panel_off;
  const double* A = mode ? F + int64_t(nI) * n : F;
  const double* B = mode ? T : F + nI;
  double* C = mode ? F + int64_t(nI) * n + nI : T;
  const int lda = n, ldb = mode ? nB : n, ldc = mode ? n : nB;
  __shared__ double As[64][GK + 1];
  __shared__ double Bs[GK][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  // this thread's share of a chunk: A rows ra + 8 q at k column ca, B k rows rb + 4 q at column cb
  const int ra = tid / GK, ca = tid % GK;
  const int rb = tid / 64, cb = tid % 64;
  double pa[8], pb[8];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int gi = i0 + ra + 8 * q, gk = k0 + ca;
      pa[q] = (gi < M && gk < K) ? A[int64_t(gi) * lda + gk] : 0.0;
      const int gk2 = k0 + rb + 4 * q, gj = j0 + cb;
      pb[q] = (gk2 < K && gj < N) ? B[int64_t(gk2) * ldb + gj] : 0.0;
    }
  };
  dbl4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = dbl4{0.0, 0.0, 0.0, 0.0};
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      As[ra + 8 * q][ca] = pa[q];
      Bs[rb + 4 * q][cb] = pb[q];
    }
    __syncthreads();
    if (k0 + GK < K) fetch(k0 + GK);
#pragma unroll
    for (int ks = 0; ks < GK / 4; ++ks) {
      double ao[2], bo[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) ao[bi] = As[wr + 16 * bi + li][4 * ks + lk];
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) bo[bj] = Bs[4 * ks + lk][wc + 16 * bj + li];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ao[bi], bo[bj], acc[bi][bj], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wr + 16 * bi + lk + 4 * v, gj = j0 + wc + 16 * bj + li;
        if (gi < M && gj < N) {
          double* p = C + int64_t(gi) * ldc + gj;
          *p = mode ? *p - acc[bi][bj][v] : -acc[bi][bj][v];
        }
      }
}

// IB := T and BI := T^T, 32 x 32 tiles through LDS (both writes coalesced).
__global__ void __launch_bounds__(256) k_nd_tcopy(NdArgs a0, int loff, int tiles_n, const RunTab* __restrict__ rt) {
  const NdArgs a = nd_at(a0, ws_off(rt));
  const NodeDev nd = a.lnodes[loff + blockIdx.y];
  const int n = nd.n, nI = nd.nI, nB = nd.nB;
  const int r0 = int(blockIdx.x / tiles_n) * 32, c0 = int(blockIdx.x % tiles_n) * 32;
  if (r0 >= nI || c0 >= nB) return;
  double* F = a.front + nd.front_off;
  const double* T = a.panel + nd.panel_off;
  __shared__ double t[32][33];
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + ty + 8 * q, c = c0 + tx;
    if (r < nI && c < nB) {
      const double v = T[int64_t(r) * nB + c];
      t[ty + 8 * q][tx] = v;
      F[int64_t(r) * n + nI + c] = v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = c0 + ty + 8 * q, r = r0 + tx;
    if (r < nI && c < nB) F[int64_t(nI + c) * n + r] = t[tx][ty + 8 * q];
  }
}

// Load at a 32-bit element offset from a base that is uniform over the wavefront (the byte
// offset stays 32-bit, so the base can live in scalar registers).
__device__ __forceinline__ double ld32(const double* base, uint32_t elem) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + (elem << 3));
}

// Sixteen bytes (two consecutive entries) at an even 32-bit element offset from a 16-byte
// aligned base that is uniform over the wavefront.
__device__ __forceinline__ double2 ld32x2(const double* base, uint32_t elem) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  const v2d* q = reinterpret_cast<const v2d*>(reinterpret_cast<const char*>(base) + (elem << 3));
  const v2d v = __builtin_nontemporal_load(q);
  return make_double2(v.x, v.y);
}

// Forward and backward sweeps, one launch per level (above the fused bottom levels, or all of
// them). A workgroup takes RP x (256/G) rows of one node, G lanes per row, U column pairs per
// lane (lane gl holds columns 2 (gl + u G) and
// 2 (gl + u G) + 1: one 16-byte load each; longer rows in chunks of 2 G U), and issues every
// load of its block and of the vector it multiplies before the first use: one memory round trip
// per level. Loads are unconditional at clamped (valid) addresses and masked afterwards so that
// the compiler keeps them all in flight. The vector is loaded once per workgroup (a few entries
// per thread) and shared through LDS, so that the loads of the waves are those of their rows;
// rows longer than 2 G U (CH) load it per wave, chunk by chunk. Front rows start at even
// offsets (every front size n, separator size nI and front offset is even: the unknowns come in
// (U, P) pairs), so the pairs are 16-byte aligned.

// c_B = f_B - BI f_I with f = slot0 + slot1, written into the parent's slot for this node;
// workgroup 0 of the node also stores f_I for the backward sweep. The root is not launched.
// Rows longer than 2 G U (only with CH) are taken in chunks.
template <int G, int U, int RP, bool CH>
__global__ void __launch_bounds__(256) k_nd_fwd_rb(NdArgs a0, int loff, const RunTab* __restrict__ rt) {
  static_assert(RP <= G, "lane p of a row group holds row p's operands");
  const NdArgs a = nd_at(a0, ws_off(rt));
  constexpr int RPP = 256 / G, RPB = RP * RPP, W = 2 * G * U;
  const NodeDev nd = a.lnodes[loff + blockIdx.y];
  // a workgroup past the node's rows (nodes smaller than the level's largest) runs with clamped
  // rows and stores nothing (j >= nB below): no early exit, so that the node record is read in
  // one go rather than field by field around a branch
  const int r0 = blockIdx.x * RPB;
  const int gl = threadIdx.x % G, grp = threadIdx.x / G;
  const double* __restrict__ F = a.front + nd.front_off;
  const double* __restrict__ s0 = a.slots + nd.slot_off;
  const int32_t* __restrict__ up = a.map_pool + nd.up_map_off;
  const int n = nd.n, nI = nd.nI, nI1 = nd.nI - 1, nI2 = nd.nI - 2, nB1 = nd.nB - 1;
  // the per-row operands f_B and the target slot of row p are loaded by lane p of the group only
  const int jm = min(r0 + min(gl, RP - 1) * RPP + grp, nB1);
  const double fbm = s0[nI + jm] + s0[n + nI + jm];
  const int32_t tom = up[jm];
  uint32_t rowoff[RP];
  double acc[RP];
#pragma unroll
  for (int p = 0; p < RP; ++p) {
    const int j = min(r0 + p * RPP + grp, nB1);
    rowoff[p] = uint32_t(nI + j) * uint32_t(n);
    acc[p] = 0.0;
  }
  if constexpr (!CH) {
    constexpr int VPT = (W + 255) / 256;
    __shared__ double fsh[W];
    double2 m[RP][U];
    double fv[VPT];
#pragma unroll
    for (int p = 0; p < RP; ++p)
#pragma unroll
      for (int u = 0; u < U; ++u) m[p][u] = ld32x2(F, rowoff[p] + uint32_t(min(2 * (gl + u * G), nI2)));
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int k = min(int(threadIdx.x) + 256 * i, nI1);
      fv[i] = ld32(s0, k) + ld32(s0, n + k);
    }
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int k = threadIdx.x + 256 * i;
      if (k < nI) {
        fsh[k] = fv[i];
        if (blockIdx.x == 0) a.fI[nd.fI_off + k] = fv[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < RP; ++p)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = 2 * (gl + u * G);
        if (c < nI) {
          acc[p] += m[p][u].x * fsh[c];
          acc[p] += m[p][u].y * fsh[c + 1];
        }
      }
  }
  for (int k0 = 0; k0 < (CH ? nI : 0); k0 += W) {
    double2 m[RP][U], fk[U];
#pragma unroll
    for (int p = 0; p < RP; ++p)
#pragma unroll
      for (int u = 0; u < U; ++u) m[p][u] = ld32x2(F, rowoff[p] + uint32_t(min(k0 + 2 * (gl + u * G), nI2)));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = min(k0 + 2 * (gl + u * G), nI2);
      const double2 sa = ld32x2(s0, k), sb = ld32x2(s0, n + k);
      fk[u] = make_double2(sa.x + sb.x, sa.y + sb.y);
    }
    if (blockIdx.x == 0 && grp == 0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + 2 * (gl + u * G);
        if (k < nI) {
          a.fI[nd.fI_off + k] = fk[u].x;
          a.fI[nd.fI_off + k + 1] = fk[u].y;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < RP; ++p)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k0 + 2 * (gl + u * G) < nI) {
          acc[p] += m[p][u].x * fk[u].x;
          acc[p] += m[p][u].y * fk[u].y;
        }
      }
  }
  double mine = 0.0;
#pragma unroll
  for (int p = 0; p < RP; ++p) {
    double v = acc[p];
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    mine = gl == p ? v : mine;
  }
  const int j = r0 + gl * RPP + grp;
  if (gl < RP && j < nd.nB) a.slots[nd.up_slot_off + tom] = fbm - mine;
}

// x_I = -II f_I - IB x_B, with f_I stored by the forward sweep (at the root: the sum of its two
// slots) and x_B gathered from the solution vector through the node's unknown ids (issued
// first, the block loads behind them); x_I goes to the solution vector.
template <int G, int U, int RP, bool CH, bool ROOT>
__device__ __forceinline__ void k_nd_bwd_body(const NdArgs& a, int loff) {
  static_assert(RP <= G, "lane p of a row group holds row p's unknown id");
  constexpr int RPP = 256 / G, RPB = RP * RPP, W = 2 * G * U;
  const NodeDev nd = a.lnodes[loff + blockIdx.y];
  const int r0 = blockIdx.x * RPB;   // rows past the node's stay clamped and unstored (r >= nI)
  const int gl = threadIdx.x % G, grp = threadIdx.x / G;
  const double* __restrict__ F = a.front + nd.front_off;
  const double* __restrict__ s0 = a.slots + nd.slot_off;
  const double* __restrict__ fI = a.fI + nd.fI_off;
  const int32_t* __restrict__ dofs = a.dof_pool + nd.dof_off;
  const int n = nd.n, nI = nd.nI, n1 = nd.n - 1, n2 = nd.n - 2, nI1 = nd.nI - 1;
  // the unknown id of row p is loaded by lane p of the group only
  const int32_t drm = dofs[min(r0 + min(gl, RP - 1) * RPP + grp, nI1)];
  uint32_t rowoff[RP];
  double acc[RP];
#pragma unroll
  for (int p = 0; p < RP; ++p) {
    const int r = min(r0 + p * RPP + grp, nI1);
    rowoff[p] = uint32_t(r) * uint32_t(n);
    acc[p] = 0.0;
  }
  if constexpr (!CH) {
    constexpr int VPT = (W + 255) / 256;
    __shared__ double vsh[W];
    double2 m[RP][U];
    double vv[VPT];
    // unknown ids of x_B first, so that their gather waits for them only, not for the block
    uint32_t dk[VPT];   // unsigned: no sign extension next to the load, before the block loads
    if constexpr (!ROOT) {
#pragma unroll
      for (int i = 0; i < VPT; ++i) dk[i] = uint32_t(dofs[min(max(int(threadIdx.x) + 256 * i, nI), n1)]);
    }
    // the block loads go out before the gather waits for the ids (the scheduler would hoist the
    // gather above them and start the block stream one round trip late)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int p = 0; p < RP; ++p)
#pragma unroll
      for (int u = 0; u < U; ++u) m[p][u] = ld32x2(F, rowoff[p] + uint32_t(min(2 * (gl + u * G), n2)));
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (ROOT) {
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int k = min(int(threadIdx.x) + 256 * i, n1);
        vv[i] = ld32(s0, k) + ld32(s0, n + k);
      }
    } else {
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int k = threadIdx.x + 256 * i;
        const double xi = ld32(fI, min(k, nI1));
        const double xb = ld32(a.y, dk[i]);
        vv[i] = k < nI ? xi : xb;
      }
    }
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int k = threadIdx.x + 256 * i;
      if (k < n) vsh[k] = vv[i];
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < RP; ++p)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = 2 * (gl + u * G);
        if (c < n) {
          acc[p] += m[p][u].x * vsh[c];
          acc[p] += m[p][u].y * vsh[c + 1];
        }
      }
  }
  for (int k0 = 0; k0 < (CH ? n : 0); k0 += W) {
    int32_t dk[2 * U];
    if constexpr (!ROOT) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + 2 * (gl + u * G);
        dk[2 * u] = dofs[min(max(k, nI), n1)];
        dk[2 * u + 1] = dofs[min(max(k + 1, nI), n1)];
      }
    }
    double2 m[RP][U];
    double v[2 * U];
#pragma unroll
    for (int p = 0; p < RP; ++p)
#pragma unroll
      for (int u = 0; u < U; ++u) m[p][u] = ld32x2(F, rowoff[p] + uint32_t(min(k0 + 2 * (gl + u * G), n2)));
#pragma unroll
    for (int h = 0; h < 2 * U; ++h) {
      const int k = k0 + 2 * (gl + (h / 2) * G) + (h & 1);
      const int ki = min(k, nI1);
      if constexpr (ROOT) {
        v[h] = k < nI ? ld32(s0, ki) + ld32(s0, n + ki) : 0.0;
      } else {
        const double xi = ld32(fI, ki);
        const double xb = a.y[dk[h]];
        v[h] = k < nI ? xi : (k < n ? xb : 0.0);
      }
    }
#pragma unroll
    for (int p = 0; p < RP; ++p)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        acc[p] += m[p][u].x * v[2 * u];
        acc[p] += m[p][u].y * v[2 * u + 1];
      }
  }
  double mine = 0.0;
#pragma unroll
  for (int p = 0; p < RP; ++p) {
    double x = acc[p];
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
    mine = gl == p ? x : mine;
  }
  const int r = r0 + gl * RPP + grp;
  if (gl < RP && r < nI) a.y[drm] = -mine;
}

__global__ void k_nd_flag(int32_t* err, int32_t bits) {
  if (threadIdx.x == 0) set_error(err, bits);
}

void launch_nd_level_factor(hipStream_t st, const NdArgs& a, int loff, int nnodes, int nmax, int nImax,
                            int nBmax, Runs rt) {
  const unsigned nr = runs_of(rt);
  if (a.piv_b != PIV) {   // the pivot kernel holds blocks of PIV in registers
    hipLaunchKernelGGL(k_nd_flag, dim3(1), dim3(64), 0, st, a.err, int32_t(ERR_SINGULAR));
    return;
  }
  hipLaunchKernelGGL(k_nd_assemble, dim3((nmax + ASM_ROWS - 1) / ASM_ROWS, nnodes, nr), dim3(256), 0, st, a, loff,
                     rt.tab);
  const int nblk = (nImax + a.piv_b - 1) / a.piv_b;
  const int tpd = (nImax + TILE - 1) / TILE;
  for (int kb = 0; kb < nblk; ++kb) {
    hipLaunchKernelGGL(k_nd_pivot, dim3(nnodes, 1, nr), dim3(64), 0, st, a, loff, kb, rt.tab);
    hipLaunchKernelGGL(k_nd_rpanel, dim3(tpd, nnodes, nr), dim3(256), 0, st, a, loff, kb, rt.tab);
    hipLaunchKernelGGL(k_nd_update, dim3(tpd * tpd, nnodes, nr), dim3(256), 0, st, a, loff, kb, rt.tab);
  }
  if (nBmax <= 0) return;
  const int tI = (nImax + 63) / 64, tB = (nBmax + 63) / 64;
  hipLaunchKernelGGL(k_nd_gemm, dim3(tI * tB, nnodes, nr), dim3(256), 0, st, a, loff, 0, tB, rt.tab);
  hipLaunchKernelGGL(k_nd_gemm, dim3(tB * tB, nnodes, nr), dim3(256), 0, st, a, loff, 1, tB, rt.tab);
  const int cI = (nImax + 31) / 32, cB = (nBmax + 31) / 32;
  hipLaunchKernelGGL(k_nd_tcopy, dim3(cI * cB, nnodes, nr), dim3(256), 0, st, a, loff, cB, rt.tab);
}

// Shape for a row length: lanes per row, column pairs per lane, rows per lane group (about
// 64 bytes of the block per lane); rows longer than 1536 are taken in chunks of 1024.
struct RbShape {
  int G, U, RP;
};
static RbShape rb_shape(int len) {
  if (len <= 16) return {8, 1, 4};
  if (len <= 32) return {16, 1, 4};
  if (len <= 64) return {32, 1, 4};
  if (len <= 128) return {32, 2, 4};   // half-wave rows (measured ahead of {64, 1, 4})
  if (len <= 256) return {64, 2, 2};
  if (len <= 512) return {64, 4, 1};
  if (len <= 1024) return {64, 8, 1};
  if (len <= 1536) return {64, 12, 1};
  return {64, 0, 1};   // longer rows: chunks of 1024
}

// Rows per lane group available for each row shape (template instances below).
static int rb_rp_options(int G, int U, int* opt) {
  if (G == 8) { opt[0] = 2; opt[1] = 3; opt[2] = 4; return 3; }
  if (G == 16 || G == 32) { opt[0] = 2; opt[1] = 4; return 2; }
  if (U == 1) { opt[0] = 2; opt[1] = 4; opt[2] = 8; return 3; }
  if (U == 2) { opt[0] = 1; opt[1] = 2; opt[2] = 4; return 3; }
  if (U == 4) { opt[0] = 1; opt[1] = 2; return 2; }
  opt[0] = 1;
  return 1;
}

// Where the shape's block holds more rows than a node has, the smallest block that still takes
// all of them (no idle lane groups on small fronts).
static RbShape rb_fit_rows(RbShape sh, int rows) {
  int opt[3];
  const int no = rb_rp_options(sh.G, sh.U, opt);
  const int rpp = 256 / sh.G;
  if (sh.RP * rpp <= rows) return sh;
  for (int i = 0; i < no; ++i)
    if (opt[i] <= sh.RP && opt[i] * rpp >= rows) {
      sh.RP = opt[i];
      break;
    }
  return sh;
}

#define ND_RB_CASE(KER, g, u, rp, ch, ...)                                                           \
  if ((sh).G == g && (sh).U == u && (sh).RP == rp) {                                                \
    hipLaunchKernelGGL((KER<g, u, rp, ch>), grid_, dim3(256), 0, st, __VA_ARGS__);                  \
    break;                                                                                          \
  }
#define ND_RB_LAUNCH(KER, sh, rows, nnodes, nruns, st, ...)                                           \
  do {                                                                                              \
    const int rpb_ = (sh).RP * (256 / (sh).G);                                                      \
    const dim3 grid_(std::max(1, ((rows) + rpb_ - 1) / rpb_), (nnodes), (nruns));                 \
    if ((sh).U == 0) {                                                                              \
      hipLaunchKernelGGL((KER<64, 8, 1, true>), grid_, dim3(256), 0, st, __VA_ARGS__);              \
      break;                                                                                        \
    }                                                                                               \
    ND_RB_CASE(KER, 8, 1, 4, false, __VA_ARGS__) ND_RB_CASE(KER, 8, 1, 3, false, __VA_ARGS__)       \
    ND_RB_CASE(KER, 8, 1, 2, false, __VA_ARGS__) ND_RB_CASE(KER, 16, 1, 4, false, __VA_ARGS__)      \
    ND_RB_CASE(KER, 16, 1, 2, false, __VA_ARGS__) ND_RB_CASE(KER, 32, 1, 4, false, __VA_ARGS__)     \
    ND_RB_CASE(KER, 32, 1, 2, false, __VA_ARGS__) ND_RB_CASE(KER, 32, 2, 4, false, __VA_ARGS__)     \
    ND_RB_CASE(KER, 32, 2, 2, false, __VA_ARGS__) ND_RB_CASE(KER, 32, 4, 2, false, __VA_ARGS__)     \
    ND_RB_CASE(KER, 32, 4, 1, false, __VA_ARGS__) ND_RB_CASE(KER, 64, 1, 8, false, __VA_ARGS__)     \
    ND_RB_CASE(KER, 64, 1, 4, false, __VA_ARGS__) ND_RB_CASE(KER, 64, 1, 2, false, __VA_ARGS__)     \
    ND_RB_CASE(KER, 64, 2, 4, false, __VA_ARGS__) ND_RB_CASE(KER, 64, 2, 2, false, __VA_ARGS__)     \
    ND_RB_CASE(KER, 64, 2, 1, false, __VA_ARGS__) ND_RB_CASE(KER, 64, 4, 2, false, __VA_ARGS__)     \
    ND_RB_CASE(KER, 64, 4, 1, false, __VA_ARGS__) ND_RB_CASE(KER, 64, 8, 1, false, __VA_ARGS__)     \
    ND_RB_CASE(KER, 64, 12, 1, false, __VA_ARGS__)                                                  \
  } while (0)

int nd_shape_code(int G, int U, int RP) { return G | (U << 8) | (RP << 16); }
void nd_shape_unpack(int code, int* G, int* U, int* RP) {
  *G = code & 255;
  *U = (code >> 8) & 255;
  *RP = (code >> 16) & 255;
}

// The instantiated shapes (ND_RB_LAUNCH) whose 2 G U columns cover a row of len entries at most
// four times over, the rule's shape first.
static RbShape rb_shape_bwd(int len);
int nd_shape_candidates(int len, int rows, bool bwd, int* codes, int cap) {
  const RbShape rule = rb_fit_rows(bwd ? rb_shape_bwd(len) : rb_shape(len), rows);
  int n = 0;
  if (n < cap) codes[n++] = nd_shape_code(rule.G, rule.U, rule.RP);
  if (rule.U == 0) return n;   // chunked rows: one shape
  static const RbShape all[] = {{8, 1, 4},  {8, 1, 3},  {8, 1, 2},  {16, 1, 4}, {16, 1, 2}, {32, 1, 4},
                                {32, 1, 2}, {32, 2, 4}, {32, 2, 2}, {32, 4, 2}, {32, 4, 1}, {64, 1, 8},
                                {64, 1, 4}, {64, 1, 2}, {64, 2, 4}, {64, 2, 2}, {64, 2, 1}, {64, 4, 2},
                                {64, 4, 1}, {64, 8, 1}, {64, 12, 1}};
  for (const RbShape& sh : all) {
    const int cols = 2 * sh.G * sh.U;
    if (cols < len || cols > 4 * len) continue;
    if (sh.G == rule.G && sh.U == rule.U && sh.RP == rule.RP) continue;
    if (n < cap) codes[n++] = nd_shape_code(sh.G, sh.U, sh.RP);
  }
  return n;
}

static RbShape rb_pick(int code, RbShape rule) {
  if (code == 0 || rule.U == 0) return rule;
  RbShape sh;
  nd_shape_unpack(code, &sh.G, &sh.U, &sh.RP);
  return sh;
}

void launch_nd_level_fwd(hipStream_t st, const NdArgs& a, int loff, int nnodes, int nImax, int nBmax,
                         Runs rt, int shape) {
  const RbShape sh = rb_pick(shape, rb_fit_rows(rb_shape(nImax), nBmax));
  ND_RB_LAUNCH(k_nd_fwd_rb, sh, nBmax, nnodes, runs_of(rt), st, a, loff, rt.tab);
}

template <int G, int U, int RP, bool CH>
__global__ void __launch_bounds__(256) k_nd_bwd_inner(NdArgs a, int loff, const RunTab* __restrict__ rt) {
  k_nd_bwd_body<G, U, RP, CH, false>(nd_at(a, ws_off(rt)), loff);
}
template <int G, int U, int RP, bool CH>
__global__ void __launch_bounds__(256) k_nd_bwd_root(NdArgs a, int loff, const RunTab* __restrict__ rt) {
  k_nd_bwd_body<G, U, RP, CH, true>(nd_at(a, ws_off(rt)), loff);
}

// The backward sweep takes twice the rows per lane group for rows of 65..512 entries (fewer,
// longer-lived workgroups per level; measured slightly faster).
static RbShape rb_shape_bwd(int len) {
  // (full-wave rows at 65..128 entries here: the half-wave shape was measured on forward rows)
  RbShape sh = len > 64 && len <= 128 ? RbShape{64, 1, 4} : rb_shape(len);
  if (sh.G == 64 && sh.U >= 1 && sh.U <= 4) sh.RP *= 2;
  return sh;
}

void launch_nd_level_bwd(hipStream_t st, const NdArgs& a, int loff, int nnodes, int nImax, int nmax, int root,
                         Runs rt, int shape) {
  const RbShape sh = rb_pick(shape, rb_fit_rows(rb_shape_bwd(nmax), nImax));
  if (root) ND_RB_LAUNCH(k_nd_bwd_root, sh, nImax, nnodes, runs_of(rt), st, a, loff, rt.tab);
  else ND_RB_LAUNCH(k_nd_bwd_inner, sh, nImax, nnodes, runs_of(rt), st, a, loff, rt.tab);
}

// ---------------------------------------------------------------------------------------------
// The bottom levels of both sweeps in one launch per direction. One workgroup takes one subtree
// (a node of level <= H whose parent lies above H, and its descendants) and its levels in order,
// upwards in the forward sweep and downwards in the backward one, with a barrier between levels.
// What passes between the subtree's levels stays in LDS: forward, the front vectors of all its
// nodes (the leaves' slots loaded at the start, each row's result added into its parent's vector,
// two terms per entry at most, so that the order of the additions does not change the sum);
// backward, its separator unknowns (x_B entries from outside the subtree gathered at the start).
// Only the subtree root's forward results, f_I and x_I go out to global memory. The work of all a
// level's nodes is dealt to the workgroup at once, so that a level costs one round trip for its
// block: forward, column pairs of IB over row chunks (sub_fwd_level); backward, the rows of
// [II IB], the products of a row summed over its lane group by halving exchanges. After its
// levels the backward workgroup can also reconstruct the boundary fluxes of the subtree's
// subdomains (flux_sub), one wavefront each.
namespace {

constexpr int SUB_NT = 1024;   // 16 wavefronts: one per subdomain of a four-level subtree

// A level's prefix sums (one of the FuseNode counts) in registers, a bound past every entry
// beyond the level's nodes, and the node of entry i with its first entry by selection: no branch
// or memory access between the loads of a batch. cnt >= 1.
struct SubSel {
  int c[FUSE_MAXN];
  __device__ __forceinline__ SubSel(const FuseNode* f, int cnt, int which) {
#pragma unroll
    for (int q = 0; q < FUSE_MAXN; ++q) {
      const FuseNode& x = f[q < cnt ? q : 0];
      const int v = which == 0 ? x.fr : which == 1 ? x.fv : which == 2 ? x.br : which == 3 ? x.bv : x.fc;
      c[q] = q < cnt ? v : 0x7fffffff;
    }
  }
  __device__ __forceinline__ int node(int i, int* start) const {
    int k = 0, s0 = 0;
#pragma unroll
    for (int q = 1; q < FUSE_MAXN; ++q)
      if (i >= c[q]) {
        k = q;
        s0 = c[q];
      }
    *start = s0;
    return k;
  }
};

// Sums of RQ rows over a group of G lanes, every lane holding partials of all RQ rows: each
// halving exchange (lane bit S) keeps the rows whose bit S matches the lane's and sends the
// others, so that after log2 RQ of them a lane holds row (lane mod RQ) only; the remaining lane
// bits are summed. Lane p < RQ returns row p's sum.
template <int K, int S>
__device__ __forceinline__ void bfly_halve(double* w, int gl) {
  if constexpr (K > 1) {
    const bool bit = (gl >> S) & 1;
#pragma unroll
    for (int j = 0; j < K / 2; ++j) {
      const double lo = w[2 * j], hi = w[2 * j + 1];
      const double keep = bit ? hi : lo, send = bit ? lo : hi;
      w[j] = keep + __shfl_xor(send, 1 << S);
    }
    bfly_halve<K / 2, S + 1>(w, gl);
  }
}
template <int G, int RQ>
__device__ __forceinline__ double bfly_sum(double* w, int gl) {
  bfly_halve<RQ, 0>(w, gl);
  double v = w[0];
#pragma unroll
  for (int o = RQ; o < G; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// One forward level: c_B = f_B - BI f_I = f_B - IB^T f_I (IB is stored as the exact transpose
// of BI), read as IB's rows, which lie in memory one after the other (BI's rows are short pieces
// of the front's long rows). The node's front vector f (I then B part) is in LDS at sv + vb + bv.
// A work item is a column pair of IB over a chunk of eight of its rows; the chunk sums go through
// LDS (part) and are added in chunk order per column, so that the sum does not depend on the
// scheduling. A column's result goes into its parent's vector (LDS) or, at the subtree root, to
// the parent's slot (res, dst; dst -1 for the other rows).
__device__ __forceinline__ void sub_fwd_level(const NdArgs& a, const FuseNode* f, const FuseLevel& lv, double* sv,
                                              double2* part, double* res, int32_t* dst) {
  constexpr int RC = 8;
  const int cnt = lv.e - lv.b;
  const SubSel cs(f, cnt, 4), ps(f, cnt, 0);
  const double* cur = sv + lv.vb;
  const int npair = lv.fR / 2;
  // the targets of this thread's first column pair (fetched with the block loads)
  int32_t t0 = 0, t1 = 0;
  {
    int st;
    const int P = min(int(threadIdx.x), npair - 1);
    const int k = ps.node(2 * P, &st);
    const int j = 2 * P - st;
    const int32_t* mp = a.map_pool + f[k].nd.up_map_off + j;
    t0 = mp[0];
    t1 = mp[1];
  }
  for (int it0 = 0; it0 < lv.fC; it0 += SUB_NT) {
    int st;
    const int it = min(it0 + int(threadIdx.x), lv.fC - 1);
    const int k = cs.node(it, &st);
    const int n = f[k].nd.n, nI = f[k].nd.nI, pairs = f[k].nd.nB / 2;
    const int loc = it - st, q = loc / pairs, p = loc - q * pairs;
    const double* F = a.front + f[k].nd.front_off;
    double2 m[RC];
#pragma unroll
    for (int u = 0; u < RC; ++u)
      m[u] = ld32x2(F, uint32_t(min(RC * q + u, nI - 1)) * uint32_t(n) + uint32_t(nI + 2 * p));
    const double* fI = cur + f[k].bv;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int u = 0; u < RC; ++u)
      if (RC * q + u < nI) {
        sx += m[u].x * fI[RC * q + u];
        sy += m[u].y * fI[RC * q + u];
      }
    if (it0 + int(threadIdx.x) < lv.fC) part[it0 + threadIdx.x] = make_double2(sx, sy);
  }
  __syncthreads();
  for (int P = threadIdx.x; P < npair; P += SUB_NT) {
    int st;
    const int k = ps.node(2 * P, &st);
    const int j = 2 * P - st;   // even column of the node's B part
    const int nI = f[k].nd.nI, pairs = f[k].nd.nB / 2, nch = (nI + RC - 1) / RC;
    const double2* pp = part + f[k].fc + j / 2;
    double2 s = pp[0];
    for (int q = 1; q < nch; ++q) {
      s.x += pp[q * pairs].x;
      s.y += pp[q * pairs].y;
    }
    if (P >= int(SUB_NT)) {   // beyond the first pair of this thread: targets fetched here
      const int32_t* mp = a.map_pool + f[k].nd.up_map_off + j;
      t0 = mp[0];
      t1 = mp[1];
    }
    const double v0 = cur[f[k].bv + nI + j] - s.x, v1 = cur[f[k].bv + nI + j + 1] - s.y;
    const int r = 2 * P;   // the level's row index of column j
    if (f[k].pv >= 0) {
      atomicAdd(sv + f[k].pv + t0, v0);
      atomicAdd(sv + f[k].pv + t1, v1);
      dst[r] = -1;
      dst[r + 1] = -1;
    } else {
      res[r] = v0;
      res[r + 1] = v1;
      dst[r] = int32_t(f[k].nd.up_slot_off) + t0;
      dst[r + 1] = int32_t(f[k].nd.up_slot_off) + t1;
    }
  }
}

// One backward level: x_I = -II f_I - IB x_B, f_I from the forward sweep, x_B from the subtree's
// separator unknowns (xres) or the gathered outside values (xb), by source (xsrc). G = 32 lanes
// per row, CH chunks of 64 columns, 8 / CH rows per lane group and batch; results to xres, their
// unknown ids to xid.
template <int CH>
__device__ __forceinline__ void sub_bwd_level(const NdArgs& a, const FuseNode* f, const FuseLevel& lv,
                                              const int32_t* xsrc, const double* xb, double* xres, int32_t* xid,
                                              double* vsh) {
  constexpr int G = 32, RQ = 8 / CH, NG = SUB_NT / G, STEP = NG * RQ, VPT = FUSE_VEC / SUB_NT;
  const int cnt = lv.e - lv.b, R = lv.bR, V = lv.bV;
  const int gl = threadIdx.x % G, grp = threadIdx.x / G;
  const SubSel rs(f, cnt, 2), vs(f, cnt, 3);
  double xi[VPT];
#pragma unroll
  for (int q = 0; q < VPT; ++q) {
    int st;
    const int i = min(int(threadIdx.x) + SUB_NT * q, V - 1);
    const int k = vs.node(i, &st);
    xi[q] = a.fI[f[k].nd.fI_off + min(i - st, f[k].nd.nI - 1)];
  }
  double2 m[RQ][CH];
  int kq[RQ];
  int32_t drm = 0;
  auto load = [&](int base) {
    const int r0 = base + grp * RQ;
#pragma unroll
    for (int p = 0; p < RQ; ++p) {
      int st;
      const int k = rs.node(min(r0 + p, R - 1), &st);
      const int i = min(r0 + p, R - 1) - st;
      kq[p] = k;
      const int n = f[k].nd.n;
      const double* F = a.front + f[k].nd.front_off;
      const uint32_t ro = uint32_t(i) * uint32_t(n);
#pragma unroll
      for (int c = 0; c < CH; ++c) m[p][c] = ld32x2(F, ro + uint32_t(min(64 * c + 2 * gl, n - 2)));
    }
    int st;
    const int rm = min(r0 + min(gl, RQ - 1), R - 1);
    const int km = rs.node(rm, &st);
    drm = a.dof_pool[f[km].nd.dof_off + rm - st];
  };
  load(0);
#pragma unroll
  for (int q = 0; q < VPT; ++q) {
    const int i = threadIdx.x + SUB_NT * q;
    if (i < V) {
      int st;
      const int k = vs.node(i, &st);
      const int c = i - st, nI = f[k].nd.nI;
      double v = xi[q];
      if (c >= nI) {
        const int e = lv.xo + f[k].fr + c - nI;
        const int32_t src = xsrc[e];
        v = src >= 0 ? xres[src] : xb[e];
      }
      vsh[i] = v;
    }
  }
  __syncthreads();
  for (int base = 0;;) {
    const int r0 = base + grp * RQ;
    double w[RQ];
#pragma unroll
    for (int p = 0; p < RQ; ++p) {
      const int n = f[kq[p]].nd.n;
      const double* fv = vsh + f[kq[p]].bv;
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int col = 64 * c + 2 * gl;
        if (col < n) {
          const double2 x = *reinterpret_cast<const double2*>(fv + col);
          v += m[p][c].x * x.x;
          v += m[p][c].y * x.y;
        }
      }
      w[p] = v;
    }
    const double s = bfly_sum<G, RQ>(w, gl);
    if (gl < RQ && r0 + gl < R) {
      xres[lv.xr + r0 + gl] = -s;
      xid[lv.xr + r0 + gl] = drm;
    }
    base += STEP;
    if (base >= R) break;
    load(base);
  }
  __syncthreads();   // the levels below read these x_I; vsh is reused
}

// The subtree's node records into LDS; returns the index of its first node.
__device__ __forceinline__ int sub_nodes(const NdArgs& a, int t, int H, FuseNode* fn) {
  const FuseLevel* L = a.flevels + size_t(t) * H;
  const int n0 = L[0].b, ntot = L[H - 1].e - n0;
  for (int i = threadIdx.x; i < ntot; i += SUB_NT) fn[i] = a.fnodes[n0 + i];
  return n0;
}

}  // namespace

__global__ void __launch_bounds__(SUB_NT) __attribute__((amdgpu_waves_per_eu(4)))
k_nd_sub_fwd(NdArgs a0, const RunTab* __restrict__ rt) {
  const NdArgs a = nd_at(a0, ws_off(rt));
  __shared__ FuseNode fn[FUSE_HMAX * FUSE_MAXN];
  __shared__ __align__(16) double sv[FUSE_SUBVEC];   // front vectors of the subtree's nodes
  __shared__ double2 part[FUSE_ITEMS];                // chunk sums of the level's column pairs
  __shared__ double res[FUSE_ROWS];
  __shared__ int32_t dst[FUSE_ROWS];
  const int H = a.fuse_h, t = blockIdx.x;
  const int n0 = sub_nodes(a, t, H, fn);
  __syncthreads();
  // the front vectors from the slots the leaf children wrote (both leaves: slot 0 + slot 1, as
  // the level kernels add them), zero where the children are nodes of the subtree
  constexpr int VPT = FUSE_VEC / SUB_NT;
#pragma unroll
  for (int h = 0; h < FUSE_HMAX; ++h) {
    const FuseLevel lv = a.flevels[size_t(t) * H + min(h, H - 1)];
    const int cnt = lv.e - lv.b;
    if (h < H && cnt > 0) {   // uniform
      const FuseNode* f = fn + (lv.b - n0);
      const SubSel vs(f, cnt, 3);
      double u0[VPT], u1[VPT];
#pragma unroll
      for (int q = 0; q < VPT; ++q) {
        int st;
        const int i = min(int(threadIdx.x) + SUB_NT * q, lv.bV - 1);
        const int k = vs.node(i, &st);
        const double* s0 = a.slots + f[k].nd.slot_off;
        u0[q] = s0[i - st];
        u1[q] = s0[f[k].nd.n + i - st];
      }
#pragma unroll
      for (int q = 0; q < VPT; ++q) {
        const int i = threadIdx.x + SUB_NT * q;
        if (i < lv.bV) {
          int st;
          const int k = vs.node(i, &st);
          const bool l0 = f[k].nd.child[0] < 0, l1 = f[k].nd.child[1] < 0;
          sv[lv.vb + i] = l0 && l1 ? u0[q] + u1[q] : l0 ? u0[q] : l1 ? u1[q] : 0.0;
        }
      }
    }
  }
  __syncthreads();
  for (int h = 0; h < H; ++h) {
    const FuseLevel lv = a.flevels[size_t(t) * H + h];
    if (lv.e == lv.b) continue;   // uniform over the workgroup
    const FuseNode* f = fn + (lv.b - n0);
    // f_I of the level's nodes, complete now, kept for the backward sweep
    {
      const SubSel vs(f, lv.e - lv.b, 1);
      for (int i = threadIdx.x; i < lv.fV; i += SUB_NT) {
        int st;
        const int k = vs.node(i, &st);
        a.fI[f[k].nd.fI_off + i - st] = sv[lv.vb + f[k].bv + i - st];
      }
    }
    if (lv.fR > 0) sub_fwd_level(a, f, lv, sv, part, res, dst);
    __syncthreads();   // the levels above read the vectors completed here
    for (int r = threadIdx.x; r < lv.fR; r += SUB_NT)
      if (dst[r] >= 0) a.slots[dst[r]] = res[r];
    __syncthreads();   // res and dst are reused
  }
}

static_assert(SUB_NT / 64 == FUSE_LEAVES && FUSE_VEC >= 64 * FUSE_LEAVES,
              "one wavefront per subdomain of a subtree, its Robin data in the vector buffer");

template <bool FLUX>
__global__ void __launch_bounds__(SUB_NT) __attribute__((amdgpu_waves_per_eu(4)))
k_nd_sub_bwd(NdArgs a0, FluxArgs fa, const RunTab* __restrict__ rt) {
  const NdArgs a = nd_at(a0, ws_off(rt));
  __shared__ FuseNode fn[FUSE_HMAX * FUSE_MAXN];
  __shared__ int32_t xsrc[FUSE_XB];   // x_B sources of the subtree's nodes, level by level
  __shared__ double xb[FUSE_XB];      // x_B values from outside the subtree
  __shared__ double xres[FUSE_XRES];  // the subtree's separator unknowns
  __shared__ int32_t xid[FUSE_XRES];  // and their ids
  __shared__ __align__(16) double vsh[FUSE_VEC];
  const int H = a.fuse_h, t = blockIdx.x;
  const int n0 = sub_nodes(a, t, H, fn);
  // the x_B sources of every level, and the values from outside the subtree
  constexpr int XPT = FUSE_ROWS / SUB_NT;
  int32_t sc[FUSE_HMAX][XPT];
  double sx[FUSE_HMAX][XPT];
#pragma unroll
  for (int h = 0; h < FUSE_HMAX; ++h) {
    const FuseLevel lv = a.flevels[size_t(t) * H + min(h, H - 1)];
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int i = min(int(threadIdx.x) + SUB_NT * q, max(lv.fR - 1, 0));
      sc[h][q] = h < H && lv.fR > 0 ? a.fxsrc[lv.xc + i] : 0;
    }
  }
#pragma unroll
  for (int h = 0; h < FUSE_HMAX; ++h)
#pragma unroll
    for (int q = 0; q < XPT; ++q) sx[h][q] = a.y[sc[h][q] < 0 ? -1 - sc[h][q] : 0];
#pragma unroll
  for (int h = 0; h < FUSE_HMAX; ++h) {
    const FuseLevel lv = a.flevels[size_t(t) * H + min(h, H - 1)];
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int i = threadIdx.x + SUB_NT * q;
      if (h < H && i < lv.fR) {
        xsrc[lv.xo + i] = sc[h][q];
        xb[lv.xo + i] = sx[h][q];
      }
    }
  }
  __syncthreads();
  for (int h = H - 1; h >= 0; --h) {
    const FuseLevel lv = a.flevels[size_t(t) * H + h];
    if (lv.e == lv.b) continue;
    const FuseNode* f = fn + (lv.b - n0);
    if (lv.bch <= 1) sub_bwd_level<1>(a, f, lv, xsrc, xb, xres, xid, vsh);
    else if (lv.bch == 2) sub_bwd_level<2>(a, f, lv, xsrc, xb, xres, xid, vsh);
    else if (lv.bch == 3) sub_bwd_level<3>(a, f, lv, xsrc, xb, xres, xid, vsh);
    else if (lv.bch == 4) sub_bwd_level<4>(a, f, lv, xsrc, xb, xres, xid, vsh);
    else if (lv.bch <= 6) sub_bwd_level<6>(a, f, lv, xsrc, xb, xres, xid, vsh);
    else sub_bwd_level<8>(a, f, lv, xsrc, xb, xres, xid, vsh);
  }
  const FuseLevel top = a.flevels[size_t(t) * H + H - 1];
  for (int r = threadIdx.x; r < top.xr + top.bR; r += SUB_NT) a.y[xid[r]] = xres[r];
  if constexpr (FLUX) {
    // every unknown of the subtree's subdomains is final now (this workgroup's x_I above, the
    // others from the launches before): one wavefront per subdomain
    __syncthreads();
    const int64_t wo = ws_off(rt);
    const int w = threadIdx.x >> 6;
    const int sub = at_off(fa.leaves, wo)[size_t(t) * FUSE_LEAVES + w];
    if (sub >= 0)   // uniform over the wavefront
      flux_sub(fa.g, sub, at_off(fa.km, wo), at_off(fa.S, wo), at_off(fa.h, wo), at_off(fa.vbnd, wo), a.y,
               at_off(fa.sub_dofs, wo), at_off(fa.ubnd, wo), fa.with_v, threadIdx.x & 63, vsh + 64 * w);
  }
}

void launch_nd_sub_fwd(hipStream_t st, const NdArgs& a, int nsubtrees, Runs rt) {
  if (a.fuse_h <= 0 || nsubtrees <= 0) return;
  hipLaunchKernelGGL(k_nd_sub_fwd, dim3(nsubtrees, 1, runs_of(rt)), dim3(SUB_NT), 0, st, a, rt.tab);
}

void launch_nd_sub_bwd(hipStream_t st, const NdArgs& a, int nsubtrees, Runs rt, const FluxArgs* fa) {
  if (a.fuse_h <= 0 || nsubtrees <= 0) return;
  if (fa)
    hipLaunchKernelGGL(k_nd_sub_bwd<true>, dim3(nsubtrees, 1, runs_of(rt)), dim3(SUB_NT), 0, st, a, *fa, rt.tab);
  else
    hipLaunchKernelGGL(k_nd_sub_bwd<false>, dim3(nsubtrees, 1, runs_of(rt)), dim3(SUB_NT), 0, st, a, FluxArgs{},
                       rt.tab);
}

}  // namespace mpm
