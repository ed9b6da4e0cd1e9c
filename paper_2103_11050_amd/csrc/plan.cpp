// Host plan: validation, decomposition, nested dissection of the interface system, layout.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <unordered_map>

namespace mpm {

namespace {

bool finite(double v) { return std::isfinite(v); }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Rect {
  int I0, I1, J0, J1;
};

}  // namespace

mpm_status validate(const mpm_desc& d, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return MPM_EINVAL;
  };
  if (d.abi_version != MPM_ABI_VERSION) return bad("abi_version mismatch");
  if (d.nx <= 0 || d.ny <= 0) return bad("nx, ny must be positive");
  if (d.sub_x <= 0 || d.sub_y <= 0) return bad("sub_x, sub_y must be positive");
  if (d.nx % d.sub_x || d.ny % d.sub_y) return bad("sub_x, sub_y must divide nx, ny");
  if (d.ne_x <= 0 || d.ne_y <= 0) return bad("ne_x, ne_y must be positive");
  if (d.sub_x % d.ne_x || d.sub_y % d.ne_y) return bad("ne_x, ne_y must divide sub_x, sub_y");
  if (!(d.lx > 0) || !(d.ly > 0) || !finite(d.lx) || !finite(d.ly)) return bad("lx, ly must be positive and finite");
  if (!(d.alpha > 0) || !finite(d.alpha)) return bad("alpha must be positive and finite");
  if (std::isnan(d.eta)) return bad("eta must not be NaN");
  if (d.eps_norm != MPM_EPS_REL_L2 && d.eps_norm != MPM_EPS_ABS_L2) return bad("unknown eps_norm");
  if (d.switch_rule != MPM_SWITCH_ALG1 && d.switch_rule != MPM_SWITCH_TEXT) return bad("unknown switch_rule");
  if (d.precision != MPM_PREC_FP64 && d.precision != MPM_PREC_FP32_REFINE) return bad("unknown precision");
  if (d.cn < 1) return bad("cn must be >= 1");
  if (!(d.mu_w > 0) || !(d.mu_o > 0) || !finite(d.mu_w) || !finite(d.mu_o)) return bad("viscosities must be positive");
  bool has_pressure = false;
  for (int k = 0; k < 4; ++k) {
    if (d.bc_kind[k] < 0 || d.bc_kind[k] > 2) return bad("unknown bc_kind");
    if (!finite(d.bc_value[k])) return bad("bc_value must be finite");
    has_pressure |= d.bc_kind[k] == MPM_BC_PRESSURE;
  }
  if (!has_pressure) return bad("at least one side must carry a pressure condition");
  if (!(d.s_inj >= 0 && d.s_inj <= 1)) return bad("s_inj must lie in [0,1]");
  if (!(d.cfl > 0 && d.cfl <= 1)) return bad("cfl must lie in (0,1]");
  if (!(d.breakthrough_cut > 0 && d.breakthrough_cut <= 1)) return bad("breakthrough_cut must lie in (0,1]");
  const int band = std::min(d.sub_x, d.sub_y);
  const long nc = long(d.sub_x) * d.sub_y;
  // local kernels (one wavefront per subdomain, fixed LDS tiles): lines of at most 16 cells
  // with at most 256 cells, 64 boundary faces and 272 faces of each direction per subdomain,
  // or lines of 17 to 32 cells with at most 1024 cells, 128 boundary faces and 1056 faces of
  // each direction
  if (band > 32) return bad("subdomains whose shorter side exceeds 32 cells are not supported");
  const bool wide = band > 16;
  const long cap_nc = wide ? 1024 : 256, cap_nb = wide ? 128 : 64, cap_nf = wide ? 1056 : 272;
  if (nc > cap_nc) return bad(wide ? "more than 1024 cells per subdomain" : "more than 256 cells per subdomain with lines of at most 16 cells");
  if (2 * (long(d.sub_x) + d.sub_y) > cap_nb)
    return bad(wide ? "more than 128 boundary faces per subdomain" : "more than 64 boundary faces per subdomain");
  if (long(d.sub_y) * (d.sub_x + 1) > cap_nf || long(d.sub_y + 1) * d.sub_x > cap_nf)
    return bad("too many faces of one direction per subdomain");
  if (d.mpm_order != 0 && d.mpm_order != 1) return bad("mpm_order must be 0 or 1");
  if (d.mpm_order == 1 && d.precision != MPM_PREC_FP64) return bad("the first-order term is FP64 only");
  if (d.mpm_order == 1 && wide) return bad("the first-order term takes lines of at most 16 cells");
  if (d.precision == MPM_PREC_FP32_REFINE && wide) return bad("the precision form takes lines of at most 16 cells");
  if (d.iface_degree != 0 && d.iface_degree != 1) return bad("iface_degree must be 0 or 1");
  if (d.iface_degree == 1 && (d.sub_x / d.ne_x < 2 || d.sub_y / d.ne_y < 2))
    return bad("linear interface spaces need at least two fine faces per interface element");
  if (d.precision == MPM_PREC_FP32_REFINE && !(d.refine_rtol > 0 && d.refine_rtol <= 1e-2))
    return bad("refine_rtol must lie in (0, 1e-2] for the precision form");
  if (d.precision == MPM_PREC_FP32_REFINE && nc / band > 16)
    return bad("the precision form takes at most 16 lines per subdomain");
  if (2 * (d.iface_degree + 1) * (2 * d.ne_x + 2 * d.ne_y) > 128)
    return bad("more than 128 interface unknowns per subdomain");
  return MPM_OK;
}

void build_plan(const mpm_desc& d, Plan* p) {
  Plan& P = *p;
  P.d = d;
  P.nx = d.nx; P.ny = d.ny; P.mx = d.sub_x; P.my = d.sub_y;
  P.Sx = d.nx / d.sub_x; P.Sy = d.ny / d.sub_y; P.nsub = P.Sx * P.Sy;
  P.hx = d.lx / d.nx; P.hy = d.ly / d.ny;
  P.ne_x = d.ne_x; P.ne_y = d.ne_y;
  P.n_vert = (P.Sx - 1) * P.Sy * P.ne_y;
  P.n_horiz = P.Sx * (P.Sy - 1) * P.ne_x;
  P.n_elem = P.n_vert + P.n_horiz;
  P.npol = d.iface_degree + 1;
  P.n_iface = 2 * P.npol * P.n_elem;
  P.nc = P.mx * P.my;
  P.band = std::min(P.mx, P.my);
  P.xfast = P.mx <= P.my ? 1 : 0;
  P.nb = 2 * (P.mx + P.my);
  P.ndmax = 4 * P.npol * (P.ne_x + P.ne_y);

  auto vert = [&](int I, int J, int k) { return (J * (P.Sx - 1) + I) * P.ne_y + k; };
  auto horiz = [&](int I, int J, int k) { return P.n_vert + (J * P.Sx + I) * P.ne_x + k; };
  // unknowns of element e: U_0 .. U_{npol-1}, P_0 .. P_{npol-1}
  const int pe = 2 * P.npol;
  auto push_e = [pe](std::vector<int32_t>& v, int e) {
    for (int t = 0; t < pe; ++t) v.push_back(pe * e + t);
  };

  // boundary unknowns of a rectangle of subdomains, order: left, right, bottom, top
  auto rect_boundary = [&](const Rect& r) {
    std::vector<int32_t> v;
    if (r.I0 > 0)
      for (int J = r.J0; J < r.J1; ++J)
        for (int k = 0; k < P.ne_y; ++k) push_e(v, vert(r.I0 - 1, J, k));
    if (r.I1 < P.Sx)
      for (int J = r.J0; J < r.J1; ++J)
        for (int k = 0; k < P.ne_y; ++k) push_e(v, vert(r.I1 - 1, J, k));
    if (r.J0 > 0)
      for (int I = r.I0; I < r.I1; ++I)
        for (int k = 0; k < P.ne_x; ++k) push_e(v, horiz(I, r.J0 - 1, k));
    if (r.J1 < P.Sy)
      for (int I = r.I0; I < r.I1; ++I)
        for (int k = 0; k < P.ne_x; ++k) push_e(v, horiz(I, r.J1 - 1, k));
    return v;
  };

  P.sub_ndof.assign(P.nsub, 0);
  P.sub_dofs.assign(size_t(P.nsub) * P.ndmax, -1);
  for (int J = 0; J < P.Sy; ++J)
    for (int I = 0; I < P.Sx; ++I) {
      auto v = rect_boundary(Rect{I, I + 1, J, J + 1});
      const int s = J * P.Sx + I;
      P.sub_ndof[s] = int32_t(v.size());
      std::copy(v.begin(), v.end(), P.sub_dofs.begin() + size_t(s) * P.ndmax);
    }

  // nested dissection: recursive bisection of the subdomain grid, post-order node ids
  P.nodes.clear();
  P.dof_pool.clear();
  P.map_pool.clear();
  P.inv_pool.clear();
  std::vector<int> node_level;
  std::function<std::pair<int, int>(Rect)> build = [&](Rect r) -> std::pair<int, int> {
    if (r.I1 - r.I0 == 1 && r.J1 - r.J0 == 1) return {-1 - (r.J0 * P.Sx + r.I0), 0};
    Rect a = r, b = r;
    std::vector<int32_t> sep;
    if (r.I1 - r.I0 >= r.J1 - r.J0) {
      const int Im = (r.I0 + r.I1) / 2;
      a.I1 = Im; b.I0 = Im;
      for (int J = r.J0; J < r.J1; ++J)
        for (int k = 0; k < P.ne_y; ++k) push_e(sep, vert(Im - 1, J, k));
    } else {
      const int Jm = (r.J0 + r.J1) / 2;
      a.J1 = Jm; b.J0 = Jm;
      for (int I = r.I0; I < r.I1; ++I)
        for (int k = 0; k < P.ne_x; ++k) push_e(sep, horiz(I, Jm - 1, k));
    }
    auto ca = build(a);
    auto cb = build(b);
    auto bnd = rect_boundary(r);
    NodeDev nd{};
    nd.nI = int32_t(sep.size());
    nd.nB = int32_t(bnd.size());
    nd.n = nd.nI + nd.nB;
    nd.level = 1 + std::max(ca.second, cb.second);
    nd.child[0] = ca.first;
    nd.child[1] = cb.first;
    nd.dof_off = int32_t(P.dof_pool.size());
    std::unordered_map<int32_t, int32_t> pos;
    for (size_t i = 0; i < sep.size(); ++i) pos[sep[i]] = int32_t(i);
    for (size_t i = 0; i < bnd.size(); ++i) pos[bnd[i]] = int32_t(sep.size() + i);
    P.dof_pool.insert(P.dof_pool.end(), sep.begin(), sep.end());
    P.dof_pool.insert(P.dof_pool.end(), bnd.begin(), bnd.end());
    const Rect rc[2] = {a, b};
    for (int c = 0; c < 2; ++c) {
      auto cbnd = rect_boundary(rc[c]);
      nd.map_off[c] = int32_t(P.map_pool.size());
      nd.nB_child[c] = int32_t(cbnd.size());
      for (int32_t g : cbnd) P.map_pool.push_back(pos.at(g));
    }
    nd.inv_off = int32_t(P.inv_pool.size());
    P.inv_pool.resize(P.inv_pool.size() + 2 * size_t(nd.n), -1);
    for (int c = 0; c < 2; ++c)
      for (int i = 0; i < nd.nB_child[c]; ++i)
        P.inv_pool[nd.inv_off + size_t(c) * nd.n + P.map_pool[nd.map_off[c] + i]] = i;
    P.nodes.push_back(nd);
    return {int(P.nodes.size()) - 1, nd.level};
  };
  if (P.nsub > 1) {
    auto r = build(Rect{0, P.Sx, 0, P.Sy});
    P.root = r.first;
  } else {
    P.root = -1;
  }
  int maxL = 0;
  for (auto& n : P.nodes) maxL = std::max(maxL, int(n.level));
  P.level_nodes.assign(maxL + 1, {});
  P.level_nmax.assign(maxL + 1, 0);
  P.level_nImax.assign(maxL + 1, 0);
  P.level_nBmax.assign(maxL + 1, 0);
  for (size_t i = 0; i < P.nodes.size(); ++i) {
    auto& n = P.nodes[i];
    P.level_nodes[n.level].push_back(int32_t(i));
    P.level_nmax[n.level] = std::max(P.level_nmax[n.level], n.n);
    P.level_nImax[n.level] = std::max(P.level_nImax[n.level], n.nI);
    P.level_nBmax[n.level] = std::max(P.level_nBmax[n.level], n.nB);
  }
  // per-node storage and the forward-solve slots, level by level, so that the fronts a level
  // kernel reads lie in one contiguous range
  int64_t fo = 0, io = 0, po = 0, so = 0;
  for (const auto& lv : P.level_nodes) {
    for (int32_t id : lv) {
      NodeDev& n = P.nodes[id];
      n.front_off = fo; fo += int64_t(n.n) * n.n;
      n.fI_off = io; io += n.nI;
      // the sweep's pivot block and row panels, later T = F_II^-1 F_IB (nI x nB)
      n.panel_off = po;
      po += std::max(int64_t(P.piv_b) * P.piv_b + 2 * int64_t(P.piv_b) * n.n, int64_t(n.nI) * n.nB);
      n.slot_off = so; so += 2 * int64_t(n.n);
      n.up_slot_off = -1;
      n.up_map_off = -1;
      n.pad = 0;
    }
  }
  P.leafup.assign(P.nsub, LeafUp{-1, -1, 0});
  for (auto& n : P.nodes) {
    for (int c = 0; c < 2; ++c) {
      const int ch = n.child[c];
      const int64_t slot = n.slot_off + int64_t(c) * n.n;
      if (ch < 0) {
        P.leafup[-1 - ch] = LeafUp{slot, n.map_off[c], 0};
      } else {
        P.nodes[ch].up_slot_off = slot;
        P.nodes[ch].up_map_off = n.map_off[c];
      }
    }
  }
  P.front_doubles = fo; P.fI_doubles = io; P.panel_doubles = po; P.slot_doubles = so;

  // workspace layout
  const size_t ncell = size_t(P.nx) * P.ny;
  const size_t nfx = size_t(P.ny) * (P.nx + 1), nfy = size_t(P.ny + 1) * P.nx;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  P.off_K = take(ncell * 8);
  P.off_q = take(ncell * 8);
  P.off_s = take(ncell * 8);
  P.off_s2 = take(ncell * 8);
  P.off_kn = take(ncell * 8);
  P.off_km = take(ncell * 8);
  P.off_ux = take(nfx * 8);
  P.off_uy = take(nfy * 8);
  P.off_uxm = take(nfx * 8);
  P.off_uym = take(nfy * 8);
  {
    const int mf = P.band <= 8 ? 8 : P.band <= 16 ? 16 : 32;
    P.off_fac = take(size_t(P.nsub) * (P.nc / P.band) * (mf * (mf + 1) / 2) * 8);
  }
  P.off_dinv = take(size_t(P.nsub) * P.nc * 8);
  P.off_S = take(size_t(P.nsub) * ((P.nb / 2 + 1) * P.nb) * 8);   // wrapped diagonals of the symmetric maps
  P.off_h = take(size_t(P.nsub) * P.nb * 8);
  P.off_vbnd = take(size_t(P.nsub) * P.nb * 8);
  {
    const int mf = P.band <= 8 ? 8 : P.band <= 16 ? 16 : 32;
    P.off_dsE = take(size_t(P.nsub) * (P.nc / P.band) * (mf * (mf + 1) / 2) * 8);
    P.off_nfac = take(size_t(P.nsub) * (P.nc / P.band) * (mf * (mf + 1) / 2) * 8);
    // precision form: FP32 copies of the three block sets
    P.n_blocks = size_t(P.nsub) * (P.nc / P.band) * (mf * (mf + 1) / 2);   // packed upper triangles
    const bool f32 = d.precision == MPM_PREC_FP32_REFINE;
    P.off_fac32 = take(f32 ? P.n_blocks * 4 : 0);
    P.off_nfac32 = take(f32 ? P.n_blocks * 4 : 0);
    P.off_dsE32 = take(f32 ? P.n_blocks * 4 : 0);
    P.off_dsflag = take(size_t(P.nsub) * 4);
    P.off_dslist = take(size_t(P.nsub) * 4);
  }
  P.off_ubnd = take(size_t(P.nsub) * P.nb * 8);
  P.off_leafK = take(size_t(P.nsub) * P.ndmax * P.ndmax * 8);
  P.off_front = take(size_t(std::max<int64_t>(fo, 1)) * 8);
  P.off_fI = take(size_t(std::max<int64_t>(io, 1)) * 8);
  P.off_slot = take(size_t(std::max<int64_t>(so, 1)) * 8);
  P.off_panel = take(size_t(std::max<int64_t>(po, 1)) * 8);
  P.off_y = take(size_t(std::max(P.n_iface, 1)) * 8);
  P.off_nodes = take(std::max<size_t>(P.nodes.size(), 1) * sizeof(NodeDev));
  P.off_dofpool = take(std::max<size_t>(P.dof_pool.size(), 1) * 4);
  P.off_mappool = take(std::max<size_t>(P.map_pool.size(), 1) * 4);
  P.off_invpool = take(std::max<size_t>(P.inv_pool.size(), 1) * 4);
  P.off_subdofs = take(P.sub_dofs.size() * 4);
  P.off_subndof = take(P.sub_ndof.size() * 4);
  P.level_off.assign(P.level_nodes.size() + 1, 0);
  P.level_flat.clear();
  for (size_t L = 0; L < P.level_nodes.size(); ++L) {
    P.level_off[L] = int32_t(P.level_flat.size());
    P.level_flat.insert(P.level_flat.end(), P.level_nodes[L].begin(), P.level_nodes[L].end());
  }
  P.level_off[P.level_nodes.size()] = int32_t(P.level_flat.size());
  P.off_levels = take(std::max<size_t>(P.level_flat.size(), 1) * 4);
  P.lnodes.clear();
  for (int32_t id : P.level_flat) P.lnodes.push_back(P.nodes[id]);
  P.off_lnodes = take(std::max<size_t>(P.lnodes.size(), 1) * sizeof(NodeDev));
  P.off_leafup = take(std::max<size_t>(P.leafup.size(), 1) * sizeof(LeafUp));
  // subtrees of the fused bottom levels: the deepest H <= FUSE_HMAX below the root level whose
  // subtrees all fit the limits of the fused kernels
  P.fuse_h = 0;
  P.fuse_roots = 0;
  P.flevels.clear();
  P.fnodes.clear();
  P.fxsrc.clear();
  {
    const int top = int(P.level_nodes.size()) - 1;
    std::vector<int32_t> parent(P.nodes.size(), -1);
    for (size_t i = 0; i < P.nodes.size(); ++i)
      for (int c = 0; c < 2; ++c)
        if (P.nodes[i].child[c] >= 0) parent[P.nodes[i].child[c]] = int32_t(i);
    // (the fused kernels keep slot indices in 32 bits)
    const int hmax = P.slot_doubles < (int64_t(1) << 31) ? std::min(FUSE_HMAX, top - 1) : 0;
    for (int H = hmax; H >= 2 && !P.fuse_h; --H) {
      std::vector<FuseLevel> lv;
      std::vector<FuseNode> fn;
      std::vector<int32_t> xs;
      bool ok = true;
      for (int32_t v : P.level_flat) {
        const NodeDev& nv = P.nodes[v];
        if (nv.level > H || (parent[v] >= 0 && P.nodes[parent[v]].level <= H)) continue;
        std::vector<std::vector<int32_t>> byl(H + 1);
        std::vector<int32_t> stack{v};
        while (!stack.empty()) {
          const int32_t u = stack.back();
          stack.pop_back();
          byl[P.nodes[u].level].push_back(u);
          for (int c = 0; c < 2; ++c)
            if (P.nodes[u].child[c] >= 0) stack.push_back(P.nodes[u].child[c]);
        }
        // places within the subtree: each node's front vector in its level (bv), each level's
        // separator unknowns (xr) and boundary entries (xo)
        std::unordered_map<int32_t, int32_t> bv_of, br_of;
        std::vector<int32_t> xr(H + 2, 0), xo(H + 2, 0), vb(H + 2, 0);
        for (int l = 1; l <= H; ++l) {
          int32_t sv = 0, sr = 0, sb = 0;
          for (int32_t u : byl[l]) {
            bv_of[u] = vb[l] + sv;
            br_of[u] = sr;
            sv += P.nodes[u].n;
            sr += P.nodes[u].nI;
            sb += P.nodes[u].nB;
          }
          xr[l + 1] = xr[l] + sr;
          xo[l + 1] = xo[l] + sb;
          vb[l + 1] = vb[l] + sv;
        }
        ok = ok && xr[H + 1] <= FUSE_XRES && xo[H + 1] <= FUSE_XB && vb[H + 1] <= FUSE_SUBVEC;
        for (int l = 1; l <= H; ++l) {
          FuseLevel L{int32_t(fn.size()), 0, 0, 0, 0, 0, 0, 0, int32_t(xs.size()), xo[l], xr[l], vb[l]};
          int nImax = 0, nmax = 0;
          for (int32_t u : byl[l]) {
            const NodeDev& x = P.nodes[u];
            const int32_t p = parent[u];
            const bool inside = p >= 0 && P.nodes[p].level <= H;
            fn.push_back(FuseNode{x, L.fR, L.fV, L.bR, L.bV, inside ? bv_of[p] : -1, L.fC});
            // x_B sources: a separator unknown of an ancestor inside the subtree, else the id
            for (int c = 0; c < x.nB; ++c) {
              const int32_t d = P.dof_pool[x.dof_off + x.nI + c];
              int32_t src = -1 - d;
              for (int32_t an = p; an >= 0 && P.nodes[an].level <= H && src < 0; an = parent[an]) {
                const NodeDev& A = P.nodes[an];
                for (int i = 0; i < A.nI; ++i)
                  if (P.dof_pool[A.dof_off + i] == d) {
                    src = xr[A.level] + br_of[an] + i;
                    break;
                  }
              }
              xs.push_back(src);
            }
            L.fR += x.nB;
            L.fV += x.nI;
            L.bR += x.nI;
            L.bV += x.n;
            L.fC += (x.nB / 2) * ((x.nI + 7) / 8);
            ok = ok && x.nB % 2 == 0;
            nImax = std::max(nImax, int(x.nI));
            nmax = std::max(nmax, int(x.n));
          }
          L.e = int32_t(fn.size());
          L.bch = (nmax + 63) / 64;
          ok = ok && int(byl[l].size()) <= FUSE_MAXN && nImax <= FUSE_FWD_NI && nmax <= FUSE_BWD_N &&
               L.bV <= FUSE_VEC && L.fR <= FUSE_ROWS && L.bR <= FUSE_ROWS && L.fC <= FUSE_ITEMS;
          lv.push_back(L);
        }
      }
      if (!ok) continue;
      P.fuse_h = H;
      P.fuse_roots = int(lv.size()) / H;
      P.flevels = std::move(lv);
      P.fnodes = std::move(fn);
      P.fxsrc = std::move(xs);
    }
  }
  // the subdomains of each subtree, for the reconstruction in the fused backward sweep
  P.fuse_flux = false;
  P.fleaves.clear();
  if (P.fuse_h > 0 && P.nb <= 64) {
    std::vector<int32_t> leaves(size_t(P.fuse_roots) * FUSE_LEAVES, -1);
    std::vector<int> cover(P.nsub, 0);
    bool ok = true;
    for (int t = 0; t < P.fuse_roots && ok; ++t) {
      int cnt = 0;
      for (int i = P.flevels[size_t(t) * P.fuse_h].b; i < P.flevels[size_t(t) * P.fuse_h + P.fuse_h - 1].e; ++i)
        for (int c = 0; c < 2; ++c) {
          const int ch = P.fnodes[i].nd.child[c];
          if (ch >= 0) continue;
          if (cnt == FUSE_LEAVES) {
            ok = false;
            break;
          }
          leaves[size_t(t) * FUSE_LEAVES + cnt++] = -1 - ch;
          cover[-1 - ch] += 1;
        }
    }
    for (int s = 0; s < P.nsub && ok; ++s) ok = cover[s] == 1;
    if (ok) {
      P.fuse_flux = true;
      P.fleaves = std::move(leaves);
    }
  }
  P.off_fnodes = take(std::max<size_t>(P.fnodes.size(), 1) * sizeof(FuseNode));
  P.off_flevels = take(std::max<size_t>(P.flevels.size(), 1) * sizeof(FuseLevel));
  P.off_fxsrc = take(std::max<size_t>(P.fxsrc.size(), 1) * 4);
  P.off_fleaves = take(std::max<size_t>(P.fleaves.size(), 1) * 4);
  const size_t blocks = (ncell + 255) / 256 + size_t(P.nsub) + 64;
  P.n_red = 4 * blocks;
  P.off_red = take(P.n_red * 8);
  P.off_scal = take(SC_COUNT * 8 + 64);
  P.off_rtab = take(2 * sizeof(RunTab));
  if (d.mpm_order == 1) P.off_wbnd = take(size_t(P.nsub) * P.nb * 8);
  P.total_bytes = off;
}

}  // namespace mpm
