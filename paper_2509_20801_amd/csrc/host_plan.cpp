// Host-side planning: PML stretch arrays (Sec. 2.2, Eqs. (10)-(13)), the
// overlapping partition (Sec. 2.3, Fig. 3) and the nested-dissection symbolic
// analysis of each local grid (Sec. 2.4: fill-reducing order and the
// elimination tree of dense fronts behind Eq. (22)).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

#include "stf_internal.h"

namespace stf {

namespace {

// Normalised loss at the PML edge: Eq. (13) divided by w*eps0, using
// eta*eps0*w = k0; negative for R < 1.
double sigma_hat_max(int L, int m, double R, double k0, double d) {
  return (m + 1) * std::log(R) / (2.0 * k0 * L * d);
}

// Eq. (10) with the grading of Eqs. (11)-(12): s = 1 + j sigma/(w eps0) at a
// depth `rho` into a PML of L cells of size d.
cd stretch_at(double rho, int L, int m, double R, double k0, double d) {
  double sh = sigma_hat_max(L, m, R, k0, d) * std::pow(rho / (L * d), (double)m);
  return cd(1.0, sh);
}

// Fill s (n nodes) and sh (n+1 half points, sh[i] at i - 1/2) for a PML of L
// cells whose interface half point is `iface` (index into sh) on the low side
// (nodes iface-1, iface-2, ... are PML nodes 1, 2, ...) or the high side.
void pml_low(std::vector<cd>& s, std::vector<cd>& sh, int iface, int L, int m, double R,
             double k0, double d) {
  for (int u = 1; u <= L; ++u) s[iface - u] = stretch_at((u - 0.5) * d, L, m, R, k0, d);
  for (int u = 0; u <= L; ++u) sh[iface - u] = stretch_at(u * d, L, m, R, k0, d);
}
void pml_high(std::vector<cd>& s, std::vector<cd>& sh, int iface, int L, int m, double R,
              double k0, double d) {
  // iface: index of the interface half point; PML node u sits at node iface-1+u.
  for (int u = 1; u <= L; ++u) s[iface - 1 + u] = stretch_at((u - 0.5) * d, L, m, R, k0, d);
  for (int u = 0; u <= L; ++u) sh[iface + u] = stretch_at(u * d, L, m, R, k0, d);
}

AxisCoef coef_from(const std::vector<cd>& s, const std::vector<cd>& sh, double d) {
  AxisCoef c;
  size_t n = s.size();
  c.w.resize(n);
  c.e.resize(n);
  double d2 = d * d;
  for (size_t t = 0; t < n; ++t) {
    c.w[t] = 1.0 / (d2 * s[t] * sh[t]);
    c.e[t] = 1.0 / (d2 * s[t] * sh[t + 1]);
  }
  return c;
}

std::vector<std::pair<int, int>> split_axis(int n, int lo, int hi, int parts) {
  int w = n - lo - hi;
  int base = w / parts, rem = w % parts;
  std::vector<int> cuts{lo};
  for (int k = 0; k < parts; ++k) cuts.push_back(cuts.back() + base + (k < rem ? 1 : 0));
  cuts.front() = 0;
  cuts.back() = n;
  std::vector<std::pair<int, int>> r;
  for (int k = 0; k < parts; ++k) r.push_back({cuts[k], cuts[k + 1]});
  return r;
}

bool finite(double v) { return std::isfinite(v); }

}  // namespace

stf_params normalized(const stf_params& p) {
  stf_params q = p;
  if (q.leaf_size == 0) q.leaf_size = 32;
  return q;
}

void validate_params(const stf_params& p) {
  STF_REQUIRE(p.nx >= 3 && p.ny >= 3, "nx and ny must be >= 3");
  STF_REQUIRE((int64_t)p.nx * p.ny < (int64_t)1 << 31, "nx*ny too large");
  STF_REQUIRE(finite(p.dx) && finite(p.dy) && p.dx > 0 && p.dy > 0, "dx, dy must be > 0");
  STF_REQUIRE(finite(p.k0) && p.k0 > 0, "k0 must be > 0");
  for (int s = 0; s < 4; ++s) STF_REQUIRE(p.pml[s] >= 0, "pml widths must be >= 0");
  STF_REQUIRE(p.pml[0] + p.pml[1] < p.nx && p.pml[2] + p.pml[3] < p.ny,
              "global PML leaves no interior");
  STF_REQUIRE(p.pml_order >= 0 && p.pml_order <= 16, "pml_order out of range");
  STF_REQUIRE(finite(p.pml_R) && p.pml_R > 0 && p.pml_R < 1, "pml_R must be in (0, 1)");
  STF_REQUIRE(p.px >= 1 && p.py >= 1 && p.px <= 1024 && p.py <= 1024, "px, py out of range");
  STF_REQUIRE(p.front_prec == STF_C128 || p.front_prec == STF_C64, "front_prec invalid");
  STF_REQUIRE(p.leaf_size >= 0 && p.leaf_size <= 4096, "leaf_size out of range");
  if (p.px * p.py > 1) {
    STF_REQUIRE(p.overlap >= 0, "overlap must be >= 0");
    STF_REQUIRE(p.local_pml >= 1, "local_pml must be >= 1 with more than one subdomain");
    STF_REQUIRE(p.local_pml_order >= 0 && p.local_pml_order <= 16, "local_pml_order out of range");
    STF_REQUIRE(finite(p.local_pml_R) && p.local_pml_R > 0 && p.local_pml_R < 1,
                "local_pml_R must be in (0, 1)");
    int e = p.overlap + p.local_pml;
    int wx = p.nx - p.pml[0] - p.pml[1], wy = p.ny - p.pml[2] - p.pml[3];
    STF_REQUIRE(p.px == 1 || wx / p.px >= e + 1,
                "x blocks narrower than overlap + local_pml + 1 (partition too fine)");
    STF_REQUIRE(p.py == 1 || wy / p.py >= e + 1,
                "y blocks narrower than overlap + local_pml + 1 (partition too fine)");
    // A middle block narrower than 2e would lie in the extensions of both of
    // its neighbours as well as its own domain.
    STF_REQUIRE(p.px <= 2 || wx / p.px >= 2 * e,
                "x blocks narrower than 2 (overlap + local_pml) with three or more blocks");
    STF_REQUIRE(p.py <= 2 || wy / p.py >= 2 * e,
                "y blocks narrower than 2 (overlap + local_pml) with three or more blocks");
  }
}

GlobalAxes build_global_axes(const stf_params& p) {
  GlobalAxes g;
  g.sx.assign(p.nx, cd(1, 0));
  g.sxh.assign(p.nx + 1, cd(1, 0));
  g.sy.assign(p.ny, cd(1, 0));
  g.syh.assign(p.ny + 1, cd(1, 0));
  if (p.pml[0] > 0) pml_low(g.sx, g.sxh, p.pml[0], p.pml[0], p.pml_order, p.pml_R, p.k0, p.dx);
  if (p.pml[1] > 0)
    pml_high(g.sx, g.sxh, p.nx - p.pml[1], p.pml[1], p.pml_order, p.pml_R, p.k0, p.dx);
  if (p.pml[2] > 0) pml_low(g.sy, g.syh, p.pml[2], p.pml[2], p.pml_order, p.pml_R, p.k0, p.dy);
  if (p.pml[3] > 0)
    pml_high(g.sy, g.syh, p.ny - p.pml[3], p.pml[3], p.pml_order, p.pml_R, p.k0, p.dy);
  g.cx = coef_from(g.sx, g.sxh, p.dx);
  g.cy = coef_from(g.sy, g.syh, p.dy);
  return g;
}

std::vector<SubDesc> build_partition(const stf_params& p, const GlobalAxes& g) {
  int e = p.overlap + p.local_pml;
  auto xr = split_axis(p.nx, p.pml[0], p.pml[1], p.px);
  auto yr = split_axis(p.ny, p.pml[2], p.pml[3], p.py);
  // Local stretch along one axis: the global values, overridden on an extended
  // side by a local PML whose interface half point lies `overlap` cells past I_k.
  auto local_axis = [&](const std::vector<cd>& s, const std::vector<cd>& sh, int o0, int o1,
                        int i0, int i1, double d) {
    std::vector<cd> ls(s.begin() + o0, s.begin() + o1);
    std::vector<cd> lsh(sh.begin() + o0, sh.begin() + o1 + 1);
    if (o0 < i0)
      pml_low(ls, lsh, i0 - p.overlap - o0, p.local_pml, p.local_pml_order, p.local_pml_R, p.k0,
              d);
    if (o1 > i1)
      pml_high(ls, lsh, i1 + p.overlap - o0, p.local_pml, p.local_pml_order, p.local_pml_R, p.k0,
               d);
    return coef_from(ls, lsh, d);
  };
  std::vector<SubDesc> subs;
  for (int ky = 0; ky < p.py; ++ky)
    for (int kx = 0; kx < p.px; ++kx) {
      SubDesc s{};
      s.kx = kx;
      s.ky = ky;
      s.ix0 = xr[kx].first;
      s.ix1 = xr[kx].second;
      s.iy0 = yr[ky].first;
      s.iy1 = yr[ky].second;
      int ox0 = s.ix0 - (kx > 0 ? e : 0), ox1 = s.ix1 + (kx < p.px - 1 ? e : 0);
      int oy0 = s.iy0 - (ky > 0 ? e : 0), oy1 = s.iy1 + (ky < p.py - 1 ? e : 0);
      s.ox0 = ox0;
      s.oy0 = oy0;
      s.nxl = ox1 - ox0;
      s.nyl = oy1 - oy0;
      s.cx = local_axis(g.sx, g.sxh, ox0, ox1, s.ix0, s.ix1, p.dx);
      s.cy = local_axis(g.sy, g.syh, oy0, oy1, s.iy0, s.iy1, p.dy);
      s.shape = -1;
      subs.push_back(std::move(s));
    }
  return subs;
}

// Geometric nested dissection of an nxl x nyl grid: a box is split by the
// middle line across its longer side (the separator, eliminated last) until
// its area is at most `leaf`.  Each tree node becomes a dense front holding
// its separator followed by the box's halo (the nodes just outside the box,
// all on ancestor separators), which is exactly the front's update set.
std::shared_ptr<SymShape> build_symbolic(int nxl, int nyl, int leaf) {
  auto sh = std::make_shared<SymShape>();
  sh->nxl = nxl;
  sh->nyl = nyl;
  sh->leaf = leaf;
  struct Box { int x0, x1, y0, y1; };
  std::vector<Box> boxes;
  std::vector<std::vector<int>> kids;
  std::vector<int> pos(nxl * nyl, -1);

  std::function<int(Box, int, int)> rec = [&](Box b, int parent, int depth) -> int {
    int idx = (int)sh->fronts.size();
    sh->fronts.push_back(SymFront{});
    boxes.push_back(b);
    kids.emplace_back();
    SymFront& f0 = sh->fronts[idx];
    f0.parent = parent;
    f0.depth = depth;
    int w = b.x1 - b.x0, h = b.y1 - b.y0;
    std::vector<int> sep;
    std::vector<Box> sub;
    int sx0 = b.x0, sy0 = b.y0, sw = w;        // the separator's box (row by row)
    if (w * h <= leaf || (w <= 2 && h <= 2)) {
      for (int y = b.y0; y < b.y1; ++y)
        for (int x = b.x0; x < b.x1; ++x) sep.push_back(x + y * nxl);
    } else if (w >= h) {
      int xs = b.x0 + w / 2;
      for (int y = b.y0; y < b.y1; ++y) sep.push_back(xs + y * nxl);
      sx0 = xs;
      sw = 1;
      sub.push_back({b.x0, xs, b.y0, b.y1});
      sub.push_back({xs + 1, b.x1, b.y0, b.y1});
    } else {
      int ys = b.y0 + h / 2;
      for (int x = b.x0; x < b.x1; ++x) sep.push_back(x + ys * nxl);
      sy0 = ys;
      sub.push_back({b.x0, b.x1, b.y0, ys});
      sub.push_back({b.x0, b.x1, ys + 1, b.y1});
    }
    for (size_t i = 0; i < sep.size(); ++i)
      STF_REQUIRE(sep[i] == sx0 + (int)i % sw + (sy0 + (int)i / sw) * nxl,
                  "internal: separator not a row-by-row box");
    std::vector<int> halo;
    if (b.x0 > 0)
      for (int y = b.y0; y < b.y1; ++y) halo.push_back(b.x0 - 1 + y * nxl);
    if (b.x1 < nxl)
      for (int y = b.y0; y < b.y1; ++y) halo.push_back(b.x1 + y * nxl);
    if (b.y0 > 0)
      for (int x = b.x0; x < b.x1; ++x) halo.push_back(x + (b.y0 - 1) * nxl);
    if (b.y1 < nyl)
      for (int x = b.x0; x < b.x1; ++x) halo.push_back(x + b.y1 * nxl);
    {
      SymFront& f = sh->fronts[idx];
      f.sx0 = sx0;
      f.sy0 = sy0;
      f.sw = sw;
      f.p = (int)sep.size();
      f.q = (int)halo.size();
      f.var_off = (int)sh->vars.size();
      sh->vars.insert(sh->vars.end(), sep.begin(), sep.end());
      sh->vars.insert(sh->vars.end(), halo.begin(), halo.end());
    }
    for (const Box& c : sub)
      if (c.x1 > c.x0 && c.y1 > c.y0) {
        int ci = rec(c, idx, depth + 1);
        kids[idx].push_back(ci);
      }
    return idx;
  };
  rec(Box{0, nxl, 0, nyl}, -1, 0);

  // Children lists, child maps and original entries.
  const int dxs[5] = {0, -1, 1, 0, 0}, dys[5] = {0, 0, 0, -1, 1};
  const int opp[5] = {0, 2, 1, 4, 3};
  for (size_t i = 0; i < sh->fronts.size(); ++i) {
    SymFront& f = sh->fronts[i];
    f.child_off = (int)sh->children.size();
    f.nchild = (int)kids[i].size();
    sh->children.insert(sh->children.end(), kids[i].begin(), kids[i].end());
    int m = f.p + f.q;
    if (m > 32767) throw Error(STF_EINVAL, "front order exceeds 32767");
    for (int a = 0; a < m; ++a) pos[sh->vars[f.var_off + a]] = a;
    f.ent_off = (int)sh->ents.size();
    for (int a = 0; a < f.p; ++a) {
      int v = sh->vars[f.var_off + a];
      int vx = v % nxl, vy = v / nxl;
      sh->ents.push_back({a | (a << 16), v * 8 + 0});
      for (int d = 1; d <= 4; ++d) {
        int wx = vx + dxs[d], wy = vy + dys[d];
        if (wx < 0 || wx >= nxl || wy < 0 || wy >= nyl) continue;
        int wv = wx + wy * nxl;
        int b = pos[wv];
        if (b < 0) continue;                 // eliminated in a descendant front
        sh->ents.push_back({a | (b << 16), v * 8 + d});
        if (b >= f.p) sh->ents.push_back({b | (a << 16), wv * 8 + opp[d]});
      }
    }
    f.ent_cnt = (int)sh->ents.size() - f.ent_off;
    // Child maps: position of each child's update var in this front.
    for (int c : kids[i]) {
      SymFront& cf = sh->fronts[c];
      cf.cmap_off = (int)sh->cmap.size();
      for (int t = 0; t < cf.q; ++t) {
        int v = sh->vars[cf.var_off + cf.p + t];
        int b = pos[v];
        if (b < 0) throw Error(STF_EINVAL, "internal: child update var missing from parent front");
        sh->cmap.push_back(b);
      }
    }
    for (int a = 0; a < m; ++a) pos[sh->vars[f.var_off + a]] = -1;
  }
  for (const SymFront& f : sh->fronts) {
    int64_t m = f.p + f.q;
    // Front kernels index a front's entries (and a child's Schur complement)
    // with 32-bit products m*m.
    STF_REQUIRE(m <= 46340, "front order above 46340: subdomain too large");
    sh->max_depth = std::max(sh->max_depth, f.depth);
    sh->max_front = std::max<int>(sh->max_front, (int)m);
    sh->factor_entries += (int64_t)f.p * f.p + 2 * (int64_t)f.p * f.q;
    sh->front_entries += m * m;
    sh->vec_entries += m;
    for (int k = 1; k <= f.p; ++k) sh->lu_flops += 8.0 * (double)(m - k) * (double)(m - k);
  }
  return sh;
}

void build_cover(const stf_params& p, const std::vector<SubDesc>& subs, std::vector<int4>& cx,
                 std::vector<int4>& cy) {
  cx.assign(p.nx, make_int4(-1, 0, -1, 0));
  cy.assign(p.ny, make_int4(-1, 0, -1, 0));
  for (int kx = 0; kx < p.px; ++kx) {
    const SubDesc& s = subs[kx];
    for (int t = 0; t < s.nxl; ++t) {
      int4& c = cx[s.ox0 + t];
      if (c.x < 0) { c.x = kx; c.y = t; }
      else if (c.z < 0) { c.z = kx; c.w = t; }
      else throw Error(STF_EINVAL, "node covered by more than two x blocks");
    }
  }
  for (int ky = 0; ky < p.py; ++ky) {
    const SubDesc& s = subs[ky * p.px];
    for (int u = 0; u < s.nyl; ++u) {
      int4& c = cy[s.oy0 + u];
      if (c.x < 0) { c.x = ky; c.y = u; }
      else if (c.z < 0) { c.z = ky; c.w = u; }
      else throw Error(STF_EINVAL, "node covered by more than two y blocks");
    }
  }
}

Plan build_plan(const stf_params& p0,
                std::map<std::tuple<int, int, int>, std::shared_ptr<const SymShape>>* cache) {
  Plan pl;
  validate_params(p0);
  pl.prm = normalized(p0);
  const stf_params& p = pl.prm;
  pl.g = build_global_axes(p);
  pl.subs = build_partition(p, pl.g);
  std::map<std::tuple<int, int, int>, int> local;
  for (SubDesc& s : pl.subs) {
    auto key = std::make_tuple(s.nxl, s.nyl, p.leaf_size);
    auto it = local.find(key);
    if (it == local.end()) {
      std::shared_ptr<const SymShape> shp;
      if (cache) {
        auto c = cache->find(key);
        if (c != cache->end()) shp = c->second;
      }
      if (!shp) {
        shp = build_symbolic(s.nxl, s.nyl, p.leaf_size);
        if (cache) (*cache)[key] = shp;
      }
      it = local.emplace(key, (int)pl.shapes.size()).first;
      pl.shapes.push_back(shp);
    }
    s.shape = it->second;
  }
  build_cover(p, pl.subs, pl.cover_x, pl.cover_y);
  return pl;
}

stf_plan_info plan_info(const Plan& pl) {
  stf_plan_info r{};
  r.ndof = (int64_t)pl.prm.nx * pl.prm.ny;
  r.nsub = (int32_t)pl.subs.size();
  r.nshapes = (int32_t)pl.shapes.size();
  for (const SubDesc& s : pl.subs) {
    const SymShape& sh = *pl.shapes[s.shape];
    r.local_dof += (int64_t)s.nxl * s.nyl;
    r.nfronts += (int64_t)sh.fronts.size();
    r.max_front = std::max(r.max_front, sh.max_front);
    r.max_depth = std::max(r.max_depth, sh.max_depth);
    r.factor_entries += sh.factor_entries;
    r.front_entries += sh.front_entries;
    r.lu_flops += sh.lu_flops;
  }
  return r;
}

}  // namespace stf
