// Host-side consistency of the plan (the nested-dissection tree of the interface system, the
// extend-add maps, the records of the fused bottom levels and the workspace layout) for a set of
// decompositions; built and run by
// tests/test_plan.py. Prints one line per decomposition: "ok ..." or the first failed check.
#include <algorithm>
#include <cstddef>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "plan.hpp"

using namespace mpm;

namespace {

// The fused bottom levels: every node of level <= H in exactly one subtree, its records' places
// (prefix sums over the level's nodes, the parent's place in the subtree's vector list), the
// level totals within the kernels' limits, and each x_B source naming the right unknown.
std::string check_fused(const Plan& P) {
  const int H = P.fuse_h, top = int(P.level_nodes.size()) - 1;
  if (H == 0) return P.fnodes.empty() && P.flevels.empty() ? "" : "records without fused levels";
  if (H < 2 || H > FUSE_HMAX || H >= top) return "fused depth";
  if (int(P.flevels.size()) != P.fuse_roots * H) return "level records";
  std::vector<int> seen(P.nodes.size(), 0);
  std::vector<int> parent(P.nodes.size(), -1);
  for (size_t i = 0; i < P.nodes.size(); ++i)
    for (int c = 0; c < 2; ++c)
      if (P.nodes[i].child[c] >= 0) parent[P.nodes[i].child[c]] = int(i);
  auto id_of = [&](const NodeDev& x) {
    for (size_t i = 0; i < P.nodes.size(); ++i)
      if (P.nodes[i].front_off == x.front_off) return int(i);
    return -1;
  };
  int next = 0;
  for (int t = 0; t < P.fuse_roots; ++t) {
    const FuseLevel* L = &P.flevels[size_t(t) * H];
    std::vector<int> ids;   // the subtree's nodes, fnodes order
    int vb = 0, xr = 0, xo = 0;
    for (int h = 1; h <= H; ++h) {
      const FuseLevel& l = L[h - 1];
      if (l.b != next || l.e < l.b || l.e - l.b > FUSE_MAXN) return "node range";
      if (l.vb != vb || l.xr != xr || l.xo != xo) return "level places";
      int fr = 0, fv = 0, br = 0, bv = 0, fc = 0, nmax = 0;
      for (int i = l.b; i < l.e; ++i) {
        const FuseNode& x = P.fnodes[i];
        const int id = id_of(x.nd);
        if (id < 0 || x.nd.level != h) return "fused node";
        ++seen[id];
        ids.push_back(id);
        if (x.fr != fr || x.fv != fv || x.br != br || x.bv != bv || x.fc != fc) return "places in the level";
        fr += x.nd.nB;
        fv += x.nd.nI;
        br += x.nd.nI;
        bv += x.nd.n;
        fc += (x.nd.nB / 2) * ((x.nd.nI + 7) / 8);
        nmax = std::max(nmax, int(x.nd.n));
        if (x.nd.nI > FUSE_FWD_NI || x.nd.n > FUSE_BWD_N || x.nd.nB % 2) return "row limits";
      }
      if (l.fR != fr || l.fV != fv || l.bR != br || l.bV != bv || l.fC != fc || l.bch != (nmax + 63) / 64)
        return "level totals";
      if (bv > FUSE_VEC || fr > FUSE_ROWS || br > FUSE_ROWS || fc > FUSE_ITEMS) return "level limits";
      next = l.e;
      vb += bv;
      xr += br;
      xo += fr;
    }
    if (vb > FUSE_SUBVEC || xr > FUSE_XRES || xo > FUSE_XB) return "subtree limits";
    // parents and x_B sources
    for (int h = 1; h <= H; ++h) {
      const FuseLevel& l = L[h - 1];
      for (int i = l.b; i < l.e; ++i) {
        const FuseNode& x = P.fnodes[i];
        const int id = id_of(x.nd), p = parent[id];
        int pv = -1;
        for (int h2 = h + 1; h2 <= H; ++h2)
          for (int i2 = L[h2 - 1].b; i2 < L[h2 - 1].e; ++i2)
            if (id_of(P.fnodes[i2].nd) == p) pv = L[h2 - 1].vb + P.fnodes[i2].bv;
        if (x.pv != pv) return "parent place";
        if (pv < 0 && (p < 0 || P.nodes[p].level <= H || x.nd.up_slot_off < 0)) return "subtree root";
        for (int c = 0; c < x.nd.nB; ++c) {
          const int d = P.dof_pool[x.nd.dof_off + x.nd.nI + c];
          const int src = P.fxsrc[l.xc + x.fr + c];
          if (src < 0) {
            if (-1 - src != d) return "outside x_B id";
            // no ancestor inside the subtree holds it
            for (int a = p; a >= 0 && P.nodes[a].level <= H; a = parent[a])
              for (int k = 0; k < P.nodes[a].nI; ++k)
                if (P.dof_pool[P.nodes[a].dof_off + k] == d) return "x_B from outside held inside";
            continue;
          }
          bool found = false;
          for (int h2 = h + 1; h2 <= H && !found; ++h2)
            for (int i2 = L[h2 - 1].b; i2 < L[h2 - 1].e; ++i2) {
              const FuseNode& y = P.fnodes[i2];
              const int k = src - L[h2 - 1].xr - y.br;
              if (k >= 0 && k < y.nd.nI && P.dof_pool[y.nd.dof_off + k] == d) found = true;
            }
          if (!found) return "x_B source";
        }
      }
    }
  }
  if (next != int(P.fnodes.size())) return "node records";
  for (size_t i = 0; i < P.nodes.size(); ++i)
    if (seen[i] != (P.nodes[i].level <= H ? 1 : 0)) return "node not in exactly one subtree";
  // the subdomains of each subtree, for the reconstruction in the fused backward sweep: each
  // one a leaf of its subtree, every subdomain in exactly one list
  if (P.fuse_flux) {
    if (P.nb > 64 || int(P.fleaves.size()) != P.fuse_roots * FUSE_LEAVES) return "leaf lists";
    std::vector<int> cov(P.nsub, 0);
    for (int t = 0; t < P.fuse_roots; ++t)
      for (int w = 0; w < FUSE_LEAVES; ++w) {
        const int s = P.fleaves[size_t(t) * FUSE_LEAVES + w];
        if (s < 0) continue;
        if (s >= P.nsub) return "leaf id";
        ++cov[s];
        bool child = false;
        for (int i = P.flevels[size_t(t) * H].b; i < P.flevels[size_t(t) * H + H - 1].e; ++i)
          child = child || P.fnodes[i].nd.child[0] == -1 - s || P.fnodes[i].nd.child[1] == -1 - s;
        if (!child) return "leaf outside its subtree";
      }
    for (int s = 0; s < P.nsub; ++s)
      if (cov[s] != 1) return "subdomain not in exactly one leaf list";
  } else if (!P.fleaves.empty()) {
    return "leaf lists without the fused reconstruction";
  }
  return "";
}

std::string check(const mpm_desc& d) {
  Plan P;
  build_plan(d, &P);
  const int nd = P.n_iface;
  // every interface unknown is eliminated at exactly one node
  std::vector<int> elim(nd, 0);
  for (const NodeDev& n : P.nodes)
    for (int i = 0; i < n.nI; ++i) {
      const int id = P.dof_pool[n.dof_off + i];
      if (id < 0 || id >= nd) return "unknown id out of range";
      elim[id] += 1;
    }
  if (P.nsub > 1)
    for (int id = 0; id < nd; ++id)
      if (elim[id] != 1) return "unknown " + std::to_string(id) + " eliminated " + std::to_string(elim[id]) + " times";
  // children's boundary unknowns sit at the mapped positions of the parent's front, and the
  // inverse maps point back
  for (const NodeDev& n : P.nodes) {
    if (n.n != n.nI + n.nB) return "front size";
    for (int c = 0; c < 2; ++c) {
      const int ch = n.child[c];
      std::vector<int32_t> cb;
      if (ch < 0) {
        const int sub = -1 - ch;
        for (int a = 0; a < P.sub_ndof[sub]; ++a) cb.push_back(P.sub_dofs[size_t(sub) * P.ndmax + a]);
      } else {
        const NodeDev& cn = P.nodes[ch];
        if (cn.level >= n.level) return "child level";
        for (int i = 0; i < cn.nB; ++i) cb.push_back(P.dof_pool[cn.dof_off + cn.nI + i]);
        if (cn.up_map_off != n.map_off[c]) return "up map of a child";
        if (cn.up_slot_off != n.slot_off + int64_t(c) * n.n) return "up slot of a child";
      }
      if (int(cb.size()) != n.nB_child[c]) return "child boundary size";
      for (size_t i = 0; i < cb.size(); ++i) {
        const int pos = P.map_pool[n.map_off[c] + i];
        if (pos < 0 || pos >= n.n) return "map out of range";
        if (P.dof_pool[n.dof_off + pos] != cb[i]) return "map does not match the parent's unknown";
        if (P.inv_pool[n.inv_off + size_t(c) * n.n + pos] != int(i)) return "inverse map";
      }
    }
  }
  // the leaves' right-hand sides go to their parent's slot through the same maps
  for (int s = 0; s < P.nsub && P.nsub > 1; ++s) {
    const LeafUp& u = P.leafup[s];
    if (u.slot_off < 0) return "leaf without parent";
  }
  // storage: disjoint ranges in bounds, each level's fronts one contiguous range
  std::vector<std::pair<int64_t, int64_t>> fr, pa, sl, fi;
  for (const NodeDev& n : P.nodes) {
    fr.push_back({n.front_off, int64_t(n.n) * n.n});
    pa.push_back({n.panel_off, std::max<int64_t>(int64_t(P.piv_b) * P.piv_b + 2 * int64_t(P.piv_b) * n.n,
                                                 int64_t(n.nI) * n.nB)});
    sl.push_back({n.slot_off, 2 * int64_t(n.n)});
    fi.push_back({n.fI_off, n.nI});
  }
  auto disjoint = [](std::vector<std::pair<int64_t, int64_t>> v, int64_t total) {
    std::sort(v.begin(), v.end());
    int64_t end = 0;
    for (auto& r : v) {
      if (r.first < end) return false;
      end = r.first + r.second;
    }
    return end <= total;
  };
  if (!disjoint(fr, P.front_doubles)) return "fronts overlap";
  if (!disjoint(pa, P.panel_doubles)) return "panels overlap";
  if (!disjoint(sl, P.slot_doubles)) return "slots overlap";
  if (!disjoint(fi, P.fI_doubles)) return "f_I ranges overlap";
  for (size_t L = 1; L < P.level_nodes.size(); ++L) {
    int64_t lo = -1, hi = -1, sum = 0;
    for (int32_t id : P.level_nodes[L]) {
      const NodeDev& n = P.nodes[id];
      if (n.level != int(L)) return "level list";
      lo = lo < 0 ? n.front_off : std::min(lo, n.front_off);
      hi = std::max(hi, n.front_off + int64_t(n.n) * n.n);
      sum += int64_t(n.n) * n.n;
    }
    if (hi - lo != sum) return "fronts of level " + std::to_string(L) + " not contiguous";
    for (int k = P.level_off[L]; k < P.level_off[L + 1]; ++k)
      if (P.lnodes[k].level != int(L) || P.lnodes[k].front_off != P.nodes[P.level_flat[k]].front_off)
        return "level-ordered copy";
  }
  // workspace regions: aligned, in bounds
  const size_t offs[] = {P.off_K, P.off_q, P.off_s, P.off_s2, P.off_kn, P.off_km, P.off_ux, P.off_uy, P.off_fac,
                         P.off_S, P.off_h, P.off_ubnd, P.off_leafK, P.off_front, P.off_panel, P.off_y, P.off_red,
                         P.off_scal, P.off_rtab};
  for (size_t o : offs)
    if (o % 256 || o >= P.total_bytes) return "workspace offset";
  if (P.off_front + size_t(std::max<int64_t>(P.front_doubles, 1)) * 8 > P.off_fI) return "front region size";
  for (size_t o : {P.off_fnodes, P.off_flevels, P.off_fxsrc, P.off_fleaves})
    if (o % 256 || o >= P.total_bytes) return "workspace offset";
  const std::string fe = check_fused(P);
  if (!fe.empty()) return "fused levels: " + fe;
  char buf[200];
  std::snprintf(buf, sizeof(buf), "ok nsub %d unknowns %d nodes %zu levels %zu fused %d subtrees %d%s bytes %zu",
                P.nsub, P.n_iface, P.nodes.size(), P.level_nodes.size() - 1, P.fuse_h, P.fuse_roots,
                P.fuse_flux ? " +flux" : "", P.total_bytes);
  return buf;
}

}  // namespace

int main() {
  // the descriptor's layout as the C compiler sees it (the Python binding mirrors it)
  std::printf("desc %zu %zu %zu %zu\n", sizeof(mpm_desc), offsetof(mpm_desc, bc_value), offsetof(mpm_desc, iface_degree),
              offsetof(mpm_desc, refine_rtol));
  // nx, ny, sub_x, sub_y, ne_x, ne_y, iface_degree
  const int shapes[][7] = {{32, 32, 8, 8, 2, 2, 0},    {32, 32, 8, 8, 2, 2, 1},   {12, 8, 4, 4, 2, 1, 0},
                           {30, 20, 10, 10, 5, 2, 0},  {30, 20, 10, 10, 1, 5, 1}, {48, 8, 8, 8, 1, 4, 0},
                           {60, 30, 20, 10, 4, 2, 1},  {16, 10, 16, 10, 1, 1, 0}, {40, 24, 8, 8, 2, 2, 0},
                           {256, 256, 16, 16, 4, 4, 0}, {1024, 1024, 16, 16, 8, 8, 0}, {300, 50, 20, 10, 20, 10, 0},
                           {144, 208, 16, 16, 4, 4, 0}, {200, 120, 8, 8, 2, 2, 1}, {1024, 1024, 16, 16, 8, 8, 1},
                           {512, 128, 32, 32, 8, 8, 1}};
  int bad = 0;
  for (const auto& s : shapes) {
    mpm_desc d{};
    d.abi_version = MPM_ABI_VERSION;
    d.nx = s[0]; d.ny = s[1]; d.lx = 1.0; d.ly = 1.0; d.sub_x = s[2]; d.sub_y = s[3]; d.ne_x = s[4]; d.ne_y = s[5];
    d.iface_degree = s[6];
    d.alpha = 1.0; d.eta = 0.1; d.cn = 1; d.mu_w = 1.0; d.mu_o = 10.0; d.cfl = 0.5; d.breakthrough_cut = 0.5;
    d.bc_kind[0] = MPM_BC_FLUX; d.bc_value[0] = -1.0; d.bc_kind[1] = MPM_BC_PRESSURE; d.s_inj = 1.0;
    std::string why;
    if (validate(d, &why) != MPM_OK) {
      std::printf("%dx%d invalid: %s\n", s[0], s[1], why.c_str());
      bad = 1;
      continue;
    }
    const std::string r = check(d);
    std::printf("%dx%d sub %dx%d ne %d,%d deg %d: %s\n", s[0], s[1], s[2], s[3], s[4], s[5], s[6], r.c_str());
    if (r.compare(0, 2, "ok") != 0) bad = 1;
  }
  return bad;
}
