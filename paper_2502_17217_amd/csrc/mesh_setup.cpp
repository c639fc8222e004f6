// Host preprocessing of a polyhedral mesh (once per mesh):
//   * validation of the OpenFOAM-style description;
//   * geometry of Section 2.3 in FP64: face area vectors Gamma_f and
//     centroids x_f by fan triangulation about the mean vertex, cell volumes
//     and centroids by face pyramids about the mean face centroid;
//   * bandwidth-reducing renumbering (reverse Cuthill-McKee, kept only when
//     it beats the input order);
//   * packed arrays for the kernels: internal-face records {Gamma, w_f} in
//     owner orientation (w_f of Eq. stressInterp), boundary-face records,
//     and a sliced-ELL cell -> face slot map (64 cells per slice);
//   * the compact-stencil approximate Jacobian of Section 3.1 (scalar
//     coefficients alpha_pc K_bar |Delta||Gamma|/|d|; blocks are scalar
//     times identity) for the preconditioners.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace jfnk {

Material make_material(const jfnk_material& m) {
  JFNK_REQUIRE(m.law == JFNK_LINEAR_ELASTIC || m.law == JFNK_NEO_HOOKEAN || m.law == JFNK_ST_VENANT_KIRCHHOFF,
               JFNK_E_ARG, "material: unknown law");
  JFNK_REQUIRE(m.E > 0 && std::isfinite(m.E), JFNK_E_ARG, "material: E must be positive");
  JFNK_REQUIRE(m.nu > -1.0 && m.nu < 0.5, JFNK_E_ARG, "material: nu must lie in (-1, 0.5)");
  JFNK_REQUIRE(m.alpha_rc >= 0 && m.alpha_pc > 0, JFNK_E_ARG,
               "material: alpha_rc >= 0 and alpha_pc > 0 required");
  Material r;
  r.law = m.law;
  r.E = m.E;
  r.nu = m.nu;
  r.alpha_rc = m.alpha_rc;
  r.alpha_pc = m.alpha_pc;
  JFNK_REQUIRE(m.rho >= 0 && std::isfinite(m.rho), JFNK_E_ARG, "material: rho must be >= 0");
  r.rho = m.rho;
  r.mu = m.E / (2.0 * (1.0 + m.nu));
  r.lam = m.E * m.nu / ((1.0 + m.nu) * (1.0 - 2.0 * m.nu));
  r.kappa = m.E / (3.0 * (1.0 - 2.0 * m.nu));
  r.Kbar = 2.0 * r.mu + r.lam;
  return r;
}

namespace {

// Faces per host-thread work item in the geometry passes.
constexpr int64_t kGeomChunk = 4096;

struct V3 {
  double x = 0, y = 0, z = 0;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

std::string s_face(int64_t f) { return "face " + std::to_string(f); }
std::string s_cell(int64_t c) { return "cell " + std::to_string(c); }

// Breadth-first search over the cell graph from `start`, visiting neighbours
// in order of increasing degree (Cuthill-McKee); marks visited cells with
// `stamp`.  Returns the visit order and the index where the last level starts.
void bfs(int32_t start, const std::vector<int64_t>& aptr, const std::vector<int32_t>& adj,
         const std::vector<int32_t>& deg, std::vector<int32_t>& mark, int32_t stamp,
         std::vector<int32_t>& out, size_t& last_level_begin, int& n_levels) {
  out.clear();
  out.push_back(start);
  mark[start] = stamp;
  size_t level_begin = 0;
  n_levels = 0;
  std::vector<int32_t> nb;
  while (level_begin < out.size()) {
    size_t level_end = out.size();
    last_level_begin = level_begin;
    ++n_levels;
    for (size_t i = level_begin; i < level_end; ++i) {
      int32_t c = out[i];
      nb.clear();
      for (int64_t k = aptr[c]; k < aptr[c + 1]; ++k)
        if (mark[adj[k]] != stamp) {
          mark[adj[k]] = stamp;
          nb.push_back(adj[k]);
        }
      std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
        return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
      });
      out.insert(out.end(), nb.begin(), nb.end());
    }
    level_begin = level_end;
  }
}

// Reverse Cuthill-McKee order (old index of each new position); each
// connected component starts from a pseudo-peripheral cell.
std::vector<int32_t> rcm(int64_t nc, const std::vector<int64_t>& aptr,
                         const std::vector<int32_t>& adj) {
  std::vector<int32_t> deg(nc), mark(nc, 0), done(nc, 0), order, comp;
  order.reserve(nc);
  for (int64_t c = 0; c < nc; ++c) deg[c] = int32_t(aptr[c + 1] - aptr[c]);
  int32_t stamp = 0;
  for (int64_t s0 = 0; s0 < nc; ++s0) {
    if (done[s0]) continue;
    int32_t start = int32_t(s0);
    size_t last = 0;
    int levels = 0;
    bfs(start, aptr, adj, deg, mark, ++stamp, comp, last, levels);
    for (int iter = 0; iter < 8; ++iter) {
      int32_t cand = comp[last];
      for (size_t i = last; i < comp.size(); ++i)
        if (deg[comp[i]] < deg[cand]) cand = comp[i];
      size_t last2 = 0;
      int levels2 = 0;
      std::vector<int32_t> comp2;
      bfs(cand, aptr, adj, deg, mark, ++stamp, comp2, last2, levels2);
      if (levels2 <= levels) break;
      start = cand;
      levels = levels2;
      last = last2;
      comp.swap(comp2);
    }
    for (int32_t c : comp) done[c] = 1;
    order.insert(order.end(), comp.begin(), comp.end());
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// Tile order (old index of each new position): recursive coordinate
// bisection of the cell centroids into tiles of kFvBlock cells, so that the
// cells one workgroup handles form a compact block and most of their face
// neighbours lie in the same tile.  Each axis is measured in typical cell
// lengths along it (median |d_a| over the internal faces whose unit normal
// has |n_a| >= 0.9), so that stretched cells still give blocks that are
// compact in cell counts.  Inside a tile the input order is kept.
std::vector<int32_t> tile_order(int dim, const std::vector<V3>& xc, const std::vector<V3>& Gam,
                                const int32_t* owner, const int32_t* nbr, int64_t ni) {
  const int64_t nc = int64_t(xc.size());
  double scale[3] = {1.0, 1.0, 1.0};
  {
    std::vector<double> len[3];
    for (int64_t f = 0; f < ni; ++f) {
      const V3 g = Gam[f];
      const double mg = std::sqrt(dot(g, g));
      const V3 dd = xc[nbr[f]] - xc[owner[f]];
      const double n[3] = {g.x / mg, g.y / mg, g.z / mg}, dv[3] = {dd.x, dd.y, dd.z};
      for (int a = 0; a < dim; ++a)
        if (std::fabs(n[a]) >= 0.9) len[a].push_back(std::fabs(dv[a]));
    }
    double found = 0;
    int nfound = 0;
    for (int a = 0; a < dim; ++a) {
      if (len[a].empty()) {
        scale[a] = 0;
        continue;
      }
      auto mid = len[a].begin() + len[a].size() / 2;
      std::nth_element(len[a].begin(), mid, len[a].end());
      scale[a] = *mid > 0 ? *mid : 0;
      if (scale[a] > 0) {
        found += std::log(scale[a]);
        ++nfound;
      }
    }
    const double fallback = nfound ? std::exp(found / nfound) : 1.0;
    for (int a = 0; a < dim; ++a)
      if (!(scale[a] > 0)) scale[a] = fallback;
  }
  auto coord = [&](int32_t c, int a) {
    const V3& x = xc[c];
    return (a == 0 ? x.x : a == 1 ? x.y : x.z) / scale[a];
  };
  std::vector<int32_t> idx(nc);
  std::iota(idx.begin(), idx.end(), 0);
  // One bisection of idx[lo, hi): the range is split along its longest axis
  // into the first (tiles / 2) tiles' worth of cells and the rest, and the
  // split point is returned; a range of at most one tile has its cells put
  // back in input order and returns hi.
  auto bisect = [&](int64_t lo, int64_t hi) -> int64_t {
    const int64_t n = hi - lo;
    if (n <= kFvBlock) {
      std::sort(idx.begin() + lo, idx.begin() + hi);
      return hi;
    }
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = lo; i < hi; ++i)
      for (int a = 0; a < dim; ++a) {
        const double v = coord(idx[i], a);
        mn[a] = std::min(mn[a], v);
        mx[a] = std::max(mx[a], v);
      }
    int axis = 0;
    for (int a = 1; a < dim; ++a)
      if (mx[a] - mn[a] > mx[axis] - mn[axis]) axis = a;
    const int64_t tiles = (n + kFvBlock - 1) / kFvBlock;
    const int64_t left = (tiles / 2) * kFvBlock;
    std::nth_element(idx.begin() + lo, idx.begin() + lo + left, idx.begin() + hi,
                     [&](int32_t a, int32_t b) {
                       const double ca = coord(a, axis), cb = coord(b, axis);
                       return ca < cb || (ca == cb && a < b);
                     });
    return lo + left;
  };
  // The bisections form a binary tree whose leaves (the tiles) hold the same
  // cells in whatever order its nodes are processed: the nodes of one level
  // go to host threads together, and once a level has enough nodes each
  // node's subtree is finished by one thread.
  std::vector<std::pair<int64_t, int64_t>> level{{0, nc}};
  while (!level.empty() && level.size() < 64) {
    std::vector<int64_t> cut(level.size());
    parallel_for(int64_t(level.size()), [&](int64_t r, int) { cut[r] = bisect(level[r].first, level[r].second); });
    std::vector<std::pair<int64_t, int64_t>> next;
    for (size_t r = 0; r < level.size(); ++r)
      if (cut[r] < level[r].second) {
        next.push_back({level[r].first, cut[r]});
        next.push_back({cut[r], level[r].second});
      }
    level.swap(next);
  }
  parallel_for(int64_t(level.size()), [&](int64_t r, int) {
    std::vector<std::pair<int64_t, int64_t>> stack{level[r]};
    while (!stack.empty()) {
      const auto [lo, hi] = stack.back();
      stack.pop_back();
      const int64_t cut = bisect(lo, hi);
      if (cut < hi) {
        stack.push_back({cut, hi});
        stack.push_back({lo, cut});
      }
    }
  });
  return idx;
}

// Largest number of distinct cells outside a tile of kFvBlock cells that
// share an internal face with a cell of the tile (cell numbers: new_of_old).
// The outside neighbours are bucketed by tile and each tile's bucket is
// counted on a host thread.
int64_t max_tile_halo(const std::vector<int32_t>& new_of_old, const int32_t* owner, const int32_t* nbr,
                      int64_t ni) {
  const int64_t nt = (int64_t(new_of_old.size()) + kFvBlock - 1) / kFvBlock;
  std::vector<int64_t> tptr(static_cast<size_t>(nt) + 1, 0);
  for (int64_t f = 0; f < ni; ++f) {
    const int64_t a = new_of_old[owner[f]], b = new_of_old[nbr[f]];
    if (a / kFvBlock == b / kFvBlock) continue;
    tptr[a / kFvBlock + 1]++;
    tptr[b / kFvBlock + 1]++;
  }
  for (int64_t t = 0; t < nt; ++t) tptr[t + 1] += tptr[t];
  std::vector<int32_t> outside(static_cast<size_t>(tptr[nt]));
  {
    std::vector<int64_t> pos(tptr.begin(), tptr.end() - 1);
    for (int64_t f = 0; f < ni; ++f) {
      const int32_t a = new_of_old[owner[f]], b = new_of_old[nbr[f]];
      if (a / kFvBlock == b / kFvBlock) continue;
      outside[pos[a / kFvBlock]++] = b;
      outside[pos[b / kFvBlock]++] = a;
    }
  }
  constexpr int64_t kTilesPerItem = 64;
  const int64_t items = (nt + kTilesPerItem - 1) / kTilesPerItem;
  std::vector<int64_t> best(static_cast<size_t>(items), 0);
  parallel_for(items, [&](int64_t it, int) {
    for (int64_t t = it * kTilesPerItem; t < std::min(nt, (it + 1) * kTilesPerItem); ++t) {
      auto first = outside.begin() + tptr[t], last = outside.begin() + tptr[t + 1];
      std::sort(first, last);
      best[it] = std::max<int64_t>(best[it], std::unique(first, last) - first);
    }
  });
  int64_t most = 0;
  for (int64_t v : best) most = std::max(most, v);
  return most;
}

}  // namespace

void build_host_mesh(const jfnk_mesh_desc& d, const Material& mat, HostMesh& hm) {
  const int dim = d.dim;
  JFNK_REQUIRE(dim == 2 || dim == 3, JFNK_E_ARG, "mesh: dim must be 2 or 3");
  JFNK_REQUIRE(d.points && d.face_ptr && d.face_pts && d.owner, JFNK_E_ARG, "mesh: null array");
  JFNK_REQUIRE(d.n_cells > 0 && d.n_cells < (int64_t(1) << 31) - 64, JFNK_E_ARG,
               "mesh: n_cells out of range");
  JFNK_REQUIRE(d.n_internal >= 0 && d.n_internal <= d.n_faces && d.n_faces < (int64_t(1) << 31),
               JFNK_E_ARG, "mesh: inconsistent face counts");
  JFNK_REQUIRE(d.n_internal == 0 || d.neighbour, JFNK_E_ARG, "mesh: null neighbour array");
  const int64_t nc = d.n_cells, nf = d.n_faces, ni = d.n_internal, nb = nf - ni;
  JFNK_REQUIRE(d.face_ptr[0] == 0, JFNK_E_MESH, "mesh: face_ptr[0] must be 0");
  for (int64_t f = 0; f < nf; ++f) {
    int64_t k = d.face_ptr[f + 1] - d.face_ptr[f];
    JFNK_REQUIRE(dim == 2 ? k == 2 : k >= 3, JFNK_E_MESH,
                 "mesh: " + s_face(f) + " has a wrong number of vertices");
    for (int64_t i = d.face_ptr[f]; i < d.face_ptr[f + 1]; ++i)
      JFNK_REQUIRE(d.face_pts[i] >= 0 && d.face_pts[i] < d.n_points, JFNK_E_MESH,
                   "mesh: " + s_face(f) + " has a vertex index out of range");
    JFNK_REQUIRE(d.owner[f] >= 0 && d.owner[f] < nc, JFNK_E_MESH,
                 "mesh: owner of " + s_face(f) + " out of range");
    if (f < ni)
      JFNK_REQUIRE(d.neighbour[f] >= 0 && d.neighbour[f] < nc && d.neighbour[f] != d.owner[f],
                   JFNK_E_MESH, "mesh: neighbour of " + s_face(f) + " invalid");
  }

  // ---- boundary classification from the patches ----
  std::vector<int8_t> btype(nb, 0);
  std::vector<double> bval(nb * 3, 0.0);
  JFNK_REQUIRE(d.n_patches >= 0 && (d.n_patches == 0 || d.patches), JFNK_E_ARG,
               "mesh: null patch array");
  for (int32_t p = 0; p < d.n_patches; ++p) {
    const jfnk_patch& pt = d.patches[p];
    JFNK_REQUIRE(pt.type >= 1 && pt.type <= 4, JFNK_E_ARG,
                 "mesh: patch " + std::to_string(p) + " has an unknown type");
    JFNK_REQUIRE(pt.start >= ni && pt.size >= 0 && pt.start + pt.size <= nf, JFNK_E_ARG,
                 "mesh: patch " + std::to_string(p) + " face range outside the boundary faces");
    for (int64_t i = 0; i < pt.size; ++i) {
      int64_t b = pt.start - ni + i;
      JFNK_REQUIRE(btype[b] == 0, JFNK_E_ARG,
                   "mesh: boundary " + s_face(pt.start + i) + " is in two patches");
      btype[b] = int8_t(pt.type);
      for (int k = 0; k < dim; ++k)
        bval[b * 3 + k] = pt.per_face ? pt.per_face[i * dim + k] : pt.value[k];
      if (pt.type == JFNK_BC_PRESSURE) bval[b * 3] = pt.per_face ? pt.per_face[i * dim] : pt.value[0];
    }
  }
  for (int64_t b = 0; b < nb; ++b)
    JFNK_REQUIRE(btype[b] != 0, JFNK_E_ARG, "mesh: boundary " + s_face(ni + b) + " is in no patch");

  // ---- face geometry (input order) ----
  auto P = [&](int32_t i) {
    V3 r;
    r.x = d.points[int64_t(i) * dim];
    r.y = d.points[int64_t(i) * dim + 1];
    if (dim == 3) r.z = d.points[int64_t(i) * dim + 2];
    return r;
  };
  // faces are independent: chunks of them go to host threads, and the error
  // reported is that of the first bad face, as in one pass
  std::vector<V3> Gam(nf), xf(nf);
  parallel_for((nf + kGeomChunk - 1) / kGeomChunk, [&](int64_t chunk, int) {
    std::vector<V3> tri_a, tri_c;
    for (int64_t f = chunk * kGeomChunk; f < std::min(nf, (chunk + 1) * kGeomChunk); ++f) {
      const int64_t a = d.face_ptr[f], k = d.face_ptr[f + 1] - a;
      if (dim == 2) {
        V3 p0 = P(d.face_pts[a]), p1 = P(d.face_pts[a + 1]);
        Gam[f] = {p1.y - p0.y, -(p1.x - p0.x), 0.0};
        xf[f] = 0.5 * (p0 + p1);
      } else {
        V3 xbar;
        for (int64_t i = 0; i < k; ++i) xbar = xbar + P(d.face_pts[a + i]);
        xbar = (1.0 / double(k)) * xbar;
        V3 g;
        tri_a.resize(size_t(k));
        tri_c.resize(size_t(k));
        for (int64_t i = 0; i < k; ++i) {
          V3 pi = P(d.face_pts[a + i]), pj = P(d.face_pts[a + (i + 1) % k]);
          tri_a[i] = 0.5 * cross(pi - xbar, pj - xbar);
          tri_c[i] = (1.0 / 3.0) * (pi + pj + xbar);
          g = g + tri_a[i];
        }
        double mg = std::sqrt(dot(g, g));
        JFNK_REQUIRE(mg > 0, JFNK_E_MESH, "mesh: " + s_face(f) + " has zero area");
        V3 n = (1.0 / mg) * g, c;
        double wsum = 0;
        for (int64_t i = 0; i < k; ++i) {
          double w = dot(tri_a[i], n);
          wsum += w;
          c = c + w * tri_c[i];
        }
        Gam[f] = g;
        xf[f] = (1.0 / wsum) * c;
      }
      JFNK_REQUIRE(dot(Gam[f], Gam[f]) > 0, JFNK_E_MESH, "mesh: " + s_face(f) + " has zero area");
    }
  });

  // ---- cell geometry (input order) ----
  std::vector<int32_t> nfc(nc, 0);
  std::vector<V3> xbar(nc);
  for (int64_t f = 0; f < nf; ++f) {
    nfc[d.owner[f]]++;
    xbar[d.owner[f]] = xbar[d.owner[f]] + xf[f];
    if (f < ni) {
      nfc[d.neighbour[f]]++;
      xbar[d.neighbour[f]] = xbar[d.neighbour[f]] + xf[f];
    }
  }
  for (int64_t c = 0; c < nc; ++c) {
    JFNK_REQUIRE(nfc[c] >= dim + 1, JFNK_E_MESH, "mesh: " + s_cell(c) + " has too few faces");
    xbar[c] = (1.0 / double(nfc[c])) * xbar[c];
  }
  std::vector<double> vol(nc, 0.0);
  std::vector<V3> mom(nc);
  const double cfrac = dim == 3 ? 0.75 : 2.0 / 3.0, vfrac = dim == 3 ? 1.0 / 3.0 : 0.5;
  auto add_pyr = [&](int32_t c, V3 g_out, V3 x) {
    V3 r = x - xbar[c];
    double v = vfrac * dot(g_out, r);
    vol[c] += v;
    mom[c] = mom[c] + v * (xbar[c] + cfrac * r);
  };
  for (int64_t f = 0; f < nf; ++f) {
    add_pyr(d.owner[f], Gam[f], xf[f]);
    if (f < ni) add_pyr(d.neighbour[f], -1.0 * Gam[f], xf[f]);
  }
  std::vector<V3> xc0(nc);
  for (int64_t c = 0; c < nc; ++c) {
    JFNK_REQUIRE(vol[c] > 0 && std::isfinite(vol[c]), JFNK_E_MESH,
                 "mesh: " + s_cell(c) + " has a non-positive volume");
    xc0[c] = (1.0 / vol[c]) * mom[c];
  }

  // ---- renumbering ----
  std::vector<int64_t> aptr(nc + 1, 0);
  for (int64_t f = 0; f < ni; ++f) {
    aptr[d.owner[f] + 1]++;
    aptr[d.neighbour[f] + 1]++;
  }
  for (int64_t c = 0; c < nc; ++c) aptr[c + 1] += aptr[c];
  std::vector<int32_t> adj(aptr[nc]);
  {
    std::vector<int64_t> pos(aptr.begin(), aptr.end() - 1);
    for (int64_t f = 0; f < ni; ++f) {
      adj[pos[d.owner[f]]++] = d.neighbour[f];
      adj[pos[d.neighbour[f]]++] = d.owner[f];
    }
  }
  auto bandwidth_of = [&](const std::vector<int32_t>& nofo) {
    int64_t bw = 0;
    for (int64_t f = 0; f < ni; ++f)
      bw = std::max<int64_t>(bw, std::llabs(int64_t(nofo[d.owner[f]]) - nofo[d.neighbour[f]]));
    return bw;
  };
  std::vector<int32_t> ident(nc);
  std::iota(ident.begin(), ident.end(), 0);
  std::vector<int32_t> order, nofo(nc);
  // Preferred order: compact tiles whose neighbour halos fit the LDS budget
  // of the tiled kernels; otherwise RCM when it narrows the bandwidth.
#ifndef JFNK_ORDER_MODE
#define JFNK_ORDER_MODE 0   // 0: tiles if their halos fit, else RCM/input; 1: input; 2: RCM; 3: tiles
#endif
  hm.tiled = false;
  if (JFNK_ORDER_MODE == 0 || JFNK_ORDER_MODE == 3) {
    order = tile_order(dim, xc0, Gam, d.owner, d.neighbour, ni);
    for (int64_t i = 0; i < nc; ++i) nofo[order[i]] = int32_t(i);
    const int64_t hmax = max_tile_halo(nofo, d.owner, d.neighbour, ni);
    hm.tiled = hmax <= tile_halo_limit(dim);
    hm.tile_halo_max = hm.tiled ? hmax : 0;
    if (!hm.tiled && JFNK_ORDER_MODE == 0) order.clear();
  }
  if (order.empty()) {
    const int64_t bw_in = bandwidth_of(ident);
    order = (JFNK_ORDER_MODE == 1) ? ident : rcm(nc, aptr, adj);
    for (int64_t i = 0; i < nc; ++i) nofo[order[i]] = int32_t(i);
    if (JFNK_ORDER_MODE == 0 && bandwidth_of(nofo) >= bw_in) {
      order = ident;
      nofo = ident;
    }
  }
  hm.bandwidth = bandwidth_of(nofo);
  hm.old_of_new = order;
  hm.new_of_old = nofo;
  hm.dim = dim;
  hm.n_cells = nc;
  hm.n_int = ni;
  hm.n_bnd = nb;
  hm.xc.assign(nc * dim, 0.0);
  hm.vol.assign(nc, 0.0);
  for (int64_t i = 0; i < nc; ++i) {
    int32_t o = order[i];
    hm.vol[i] = vol[o];
    hm.xc[i * dim] = xc0[o].x;
    hm.xc[i * dim + 1] = xc0[o].y;
    if (dim == 3) hm.xc[i * dim + 2] = xc0[o].z;
  }
  auto XC = [&](int32_t c) {
    V3 r;
    r.x = hm.xc[int64_t(c) * dim];
    r.y = hm.xc[int64_t(c) * dim + 1];
    if (dim == 3) r.z = hm.xc[int64_t(c) * dim + 2];
    return r;
  };

  // ---- internal faces in the new numbering, owner < neighbour ----
  std::vector<int64_t> fperm(ni);
  std::vector<int32_t> o2(ni), n2(ni);
  std::vector<int8_t> flip(ni);
  for (int64_t f = 0; f < ni; ++f) {
    int32_t a = nofo[d.owner[f]], b = nofo[d.neighbour[f]];
    flip[f] = a > b;
    o2[f] = std::min(a, b);
    n2[f] = std::max(a, b);
  }
  // Face numbering for coalesced access: faces are grouped by the 64-cell
  // slice of their owner, then by their rank among the owner's faces (in
  // order of neighbour, equal neighbours in input order), then by the owner's
  // lane, so that the k-th owned face of 64 consecutive cells occupies
  // consecutive records.
  {
    std::vector<int64_t> optr(nc + 1, 0);
    for (int64_t f = 0; f < ni; ++f) optr[o2[f] + 1]++;
    for (int64_t c = 0; c < nc; ++c) optr[c + 1] += optr[c];
    std::vector<int64_t> owned(ni);
    {
      std::vector<int64_t> pos(optr.begin(), optr.end() - 1);
      for (int64_t f = 0; f < ni; ++f) owned[pos[o2[f]]++] = f;
    }
    for (int64_t c = 0; c < nc; ++c) {
      auto first = owned.begin() + optr[c], last = owned.begin() + optr[c + 1];
      if (last - first > 32) {
        std::stable_sort(first, last, [&](int64_t x, int64_t y) { return n2[x] < n2[y]; });
        continue;
      }
      for (auto it = first + (first != last); it < last; ++it) {  // insertion sort, stable
        const int64_t f = *it;
        auto j = it;
        for (; j > first && n2[*(j - 1)] > n2[f]; --j) *j = *(j - 1);
        *j = f;
      }
    }
    int64_t q = 0;
    for (int64_t s0 = 0; s0 < nc; s0 += kSlice) {
      const int64_t s1 = std::min<int64_t>(nc, s0 + kSlice);
      int64_t most = 0;
      for (int64_t c = s0; c < s1; ++c) most = std::max(most, optr[c + 1] - optr[c]);
      for (int64_t r = 0; r < most; ++r)
        for (int64_t c = s0; c < s1; ++c)
          if (optr[c] + r < optr[c + 1]) fperm[q++] = owned[optr[c] + r];
    }
  }
  // Face records are independent and filled by host threads (the error
  // reported is that of the first bad face); the diagonal of the approximate
  // Jacobian sums over each cell's faces further down, in face order.
  const double aKp = mat.alpha_pc * mat.Kbar;
  hm.face.assign(ni * kFaceRec, 0.0);
  hm.magG.assign(ni, 0.0);
  hm.fown.resize(ni);
  hm.fnb.resize(ni);
  hm.pc_off.resize(ni);
  parallel_for((ni + kGeomChunk - 1) / kGeomChunk, [&](int64_t chunk, int) {
    for (int64_t j = chunk * kGeomChunk; j < std::min(ni, (chunk + 1) * kGeomChunk); ++j) {
      int64_t f = fperm[j];
      int32_t A = o2[f], B = n2[f];
      V3 g = flip[f] ? -1.0 * Gam[f] : Gam[f];
      double mg = std::sqrt(dot(g, g));
      V3 n = (1.0 / mg) * g;
      V3 dAB = XC(B) - XC(A);
      double dn = dot(dAB, n);
      JFNK_REQUIRE(dn > 0, JFNK_E_MESH,
                   "mesh: " + s_face(f) + " has d.n <= 0 (cell centroids on the wrong side)");
      double w = dot(n, XC(B) - xf[f]) / dn;
      double* r = &hm.face[j * kFaceRec];
      if (dim == 3) {
        r[0] = g.x; r[1] = g.y; r[2] = g.z; r[3] = w;
      } else {
        r[0] = g.x; r[1] = g.y; r[2] = w; r[3] = 0.0;
      }
      hm.magG[j] = mg;
      hm.fown[j] = A;
      hm.fnb[j] = B;
      hm.pc_off[j] = aKp * mg / dn;  // alpha K_bar |Delta| |Gamma| / |d| = alpha K_bar |Gamma| / (d.n)
    }
  });

  // ---- boundary faces sorted by new owner ----
  std::vector<int64_t> bperm(nb);
  std::iota(bperm.begin(), bperm.end(), 0);
  std::stable_sort(bperm.begin(), bperm.end(), [&](int64_t x, int64_t y) {
    return nofo[d.owner[ni + x]] < nofo[d.owner[ni + y]];
  });
  hm.bface.assign(nb * kBfaceRec, 0.0);
  hm.bown.resize(nb);
  std::vector<double> bdiag(nb, 0.0);  // a displacement face's diagonal term
  std::vector<char> bsym(nb, 0);       // symmetry face (its diagonal block is aKp |Gamma| / h n n)
  parallel_for((nb + kGeomChunk - 1) / kGeomChunk, [&](int64_t chunk, int) {
    for (int64_t j = chunk * kGeomChunk; j < std::min(nb, (chunk + 1) * kGeomChunk); ++j) {
      int64_t b = bperm[j], f = ni + b;
      int32_t c = nofo[d.owner[f]];
      V3 g = Gam[f];
      V3 db = xf[f] - XC(c);
      double mg = std::sqrt(dot(g, g));
      double* r = &hm.bface[j * kBfaceRec];
      r[0] = g.x; r[1] = g.y; r[2] = g.z;
      r[3] = db.x; r[4] = db.y; r[5] = db.z;
      const double* v = &bval[b * 3];
      if (btype[b] == JFNK_BC_DISPLACEMENT) {
        double dbn = dot(db, g) / mg;
        JFNK_REQUIRE(dbn > 0, JFNK_E_MESH, "mesh: displacement " + s_face(f) + " has d.n <= 0");
        r[6] = v[0]; r[7] = v[1]; r[8] = v[2];
        r[9] = kBcDisp;
        bdiag[j] = aKp * mg / dbn;
      } else if (btype[b] == JFNK_BC_TRACTION) {
        r[6] = mg * v[0]; r[7] = mg * v[1]; r[8] = mg * v[2];   // |Gamma| T_bar
        r[9] = kBcTrac;
      } else if (btype[b] == JFNK_BC_SYMMETRY) {
        // the cell's mirror image lies at x_P + 2 h n, h = d_b . n
        double h = dot(db, g) / mg;
        JFNK_REQUIRE(h > 0, JFNK_E_MESH, "mesh: symmetry " + s_face(f) + " has d.n <= 0");
        r[6] = g.x / mg; r[7] = g.y / mg; r[8] = g.z / mg;        // unit normal
        r[9] = kBcSymm;
        bdiag[j] = aKp * mg / h;
        bsym[j] = 1;
      } else {
        r[6] = -v[0] * g.x; r[7] = -v[0] * g.y; r[8] = -v[0] * g.z;  // -p Gamma
        r[9] = kBcPres;
      }
      if (dim == 2) { r[2] = r[5] = r[8] = 0.0; }
      hm.bown[j] = c;
    }
  });

  // ---- per-cell face lists: internal faces ascending, then boundary faces ----
  std::vector<int32_t> cnt(nc + 1, 0);
  for (int64_t j = 0; j < ni; ++j) {
    cnt[hm.fown[j] + 1]++;
    cnt[hm.fnb[j] + 1]++;
  }
  for (int64_t j = 0; j < nb; ++j) cnt[hm.bown[j] + 1]++;
  for (int64_t c = 0; c < nc; ++c) cnt[c + 1] += cnt[c];
  std::vector<int32_t> snb(cnt[nc]), sfc(cnt[nc]);
  {
    std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t j = 0; j < ni; ++j) {  // faces ascend, so each cell's list is sorted by face
      int32_t A = hm.fown[j], B = hm.fnb[j];
      snb[pos[A]] = B;
      sfc[pos[A]++] = int32_t(j);
      snb[pos[B]] = A;
      sfc[pos[B]++] = ~int32_t(j);
    }
    for (int64_t j = 0; j < nb; ++j) {
      int32_t c = hm.bown[j];
      snb[pos[c]] = kSlotBoundary;
      sfc[pos[c]++] = int32_t(j);
    }
  }
  const int64_t cell_chunks = (nc + kGeomChunk - 1) / kGeomChunk;

  // ---- approximate-Jacobian diagonal: minus the cell's face coefficients ----
  // A symmetry face's block, the derivative of the compact term's symmetry
  // sum, -2 aKp |Delta_s| |Gamma| / |d_s| n n = -aKp |Gamma| / h n n, keeps
  // its diagonal per component (exact for planes normal to an axis).
  hm.pc_diag.assign(nc, 0.0);
  const bool any_sym = std::find(bsym.begin(), bsym.end(), 1) != bsym.end();
  if (any_sym) hm.pc_sym.assign(size_t(nc) * dim, 0.0);
  parallel_for(cell_chunks, [&](int64_t chunk, int) {
    for (int64_t c = chunk * kGeomChunk; c < std::min(nc, (chunk + 1) * kGeomChunk); ++c) {
      double s = 0.0;
      for (int32_t k = cnt[c]; k < cnt[c + 1]; ++k) {
        const int32_t fc = sfc[k];
        if (snb[k] == kSlotBoundary && bsym[fc]) {
          const double* r = &hm.bface[size_t(fc) * kBfaceRec];
          for (int q = 0; q < dim; ++q) hm.pc_sym[size_t(c) * dim + q] -= bdiag[fc] * r[6 + q] * r[6 + q];
          continue;
        }
        s -= snb[k] == kSlotBoundary ? bdiag[fc] : hm.pc_off[fc >= 0 ? fc : ~fc];
      }
      hm.pc_diag[c] = s;
    }
  });

  // ---- least-squares matrix check (the kernels rebuild G_P on the fly) ----
  parallel_for(cell_chunks, [&](int64_t chunk, int) {
    for (int64_t c = chunk * kGeomChunk; c < std::min(nc, (chunk + 1) * kGeomChunk); ++c) {
      double g[6] = {0, 0, 0, 0, 0, 0};
      for (int32_t k = cnt[c]; k < cnt[c + 1]; ++k) {
        if (snb[k] == kSlotBoundary) {
          if (!bsym[sfc[k]]) continue;
          // the mirror image: |Gamma| n n
          const double* r = &hm.bface[size_t(sfc[k]) * kBfaceRec];
          const double mgs = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
          const double e[6] = {r[6] * r[6], r[6] * r[7], r[6] * r[8], r[7] * r[7], r[7] * r[8], r[8] * r[8]};
          for (int q = 0; q < 6; ++q) g[q] += mgs * e[q];
          continue;
        }
        const int64_t j = sfc[k] >= 0 ? sfc[k] : ~sfc[k];
        const double* r = &hm.face[j * kFaceRec];
        V3 gf = dim == 3 ? V3{r[0], r[1], r[2]} : V3{r[0], r[1], 0.0};
        double mg = std::sqrt(dot(gf, gf));
        V3 dd = XC(hm.fnb[j]) - XC(hm.fown[j]);
        double wt = mg / dot(dd, dd);
        double e[6] = {dd.x * dd.x, dd.x * dd.y, dd.x * dd.z, dd.y * dd.y, dd.y * dd.z, dd.z * dd.z};
        for (int q = 0; q < 6; ++q) g[q] += wt * e[q];
      }
      double det, scale;
      if (dim == 3) {
        det = g[0] * (g[3] * g[5] - g[4] * g[4]) - g[1] * (g[1] * g[5] - g[4] * g[2]) +
              g[2] * (g[1] * g[4] - g[3] * g[2]);
        scale = std::pow((g[0] + g[3] + g[5]) / 3.0, 3);
      } else {
        det = g[0] * g[3] - g[1] * g[1];
        scale = std::pow((g[0] + g[3]) / 2.0, 2);
      }
      JFNK_REQUIRE(det > 1e-10 * scale && scale > 0, JFNK_E_MESH,
                   "mesh: input " + s_cell(order[c]) +
                       " has a singular least-squares matrix (too few internal-face directions)");
    }
  });

  // ---- sliced-ELL slot map ----
  const int64_t n_slices = (nc + kSlice - 1) / kSlice;
  hm.slice_ptr.assign(n_slices + 1, 0);
  for (int64_t s = 0; s < n_slices; ++s) {
    int32_t w = 0;
    for (int64_t c = s * kSlice; c < std::min<int64_t>(nc, (s + 1) * kSlice); ++c)
      w = std::max(w, cnt[c + 1] - cnt[c]);
    JFNK_REQUIRE(int64_t(hm.slice_ptr[s]) + int64_t(w) * kSlice < (int64_t(1) << 31), JFNK_E_ARG,
                 "mesh: too many face slots");
    hm.slice_ptr[s + 1] = hm.slice_ptr[s] + w * kSlice;
  }
  hm.slot_nb.assign(hm.slice_ptr[n_slices], kSlotPad);
  hm.slot_fc.assign(hm.slice_ptr[n_slices], 0);
  parallel_for(cell_chunks, [&](int64_t chunk, int) {
    for (int64_t c = chunk * kGeomChunk; c < std::min(nc, (chunk + 1) * kGeomChunk); ++c) {
      int64_t s = c / kSlice, lane = c % kSlice;
      for (int32_t k = 0; k < cnt[c + 1] - cnt[c]; ++k) {
        int64_t idx = hm.slice_ptr[s] + int64_t(k) * kSlice + lane;
        hm.slot_nb[idx] = snb[cnt[c] + k];
        hm.slot_fc[idx] = sfc[cnt[c] + k];
      }
    }
  });
}

}  // namespace jfnk

namespace jfnk {

// Concatenate the segments of a batch into one padded union numbering.
// Segment s occupies union cells [cell_off_s, cell_off_s + n_s); cell_off_s
// is a multiple of kSegAlign so that each workgroup of the cell passes lies
// in one segment.  Cells in the alignment gaps are padding: they own no face
// slots, carry zeros in every vector, and have a unit diagonal in the
// approximate Jacobian.
void build_union(jfnk_mesh& m, UnionArrays& ua) {
  const int S = m.n_seg();
  JFNK_REQUIRE(S >= 1, JFNK_E_ARG, "batch: no segments");
  const int dim = m.segs[0].host.dim;
  int64_t cell = 0, face = 0, bface = 0, ext = 0;
  for (int s = 0; s < S; ++s) {
    Segment& g = m.segs[s];
    JFNK_REQUIRE(g.host.dim == dim, JFNK_E_ARG, "batch: all meshes of a batch must have the same dim");
    if (s > 0) cell = (cell + kSegAlign - 1) / kSegAlign * kSegAlign;
    g.cell_off = cell;
    g.face_off = face;
    g.bface_off = bface;
    g.ext_off = ext;
    cell += g.host.n_cells;
    face += g.host.n_int;
    bface += g.host.n_bnd;
    ext += g.host.n_cells;
  }
  JFNK_REQUIRE(cell < (int64_t(1) << 31) - kSegAlign && face < (int64_t(1) << 31), JFNK_E_ARG,
               "batch: too many cells or faces");
  const int64_t N = cell;
  m.n_ext_cells = ext;
  HostMesh& U = m.host;
  U = HostMesh();
  U.dim = dim;
  U.n_cells = N;
  U.n_int = face;
  U.n_bnd = bface;
  U.fown.resize(face);
  U.fnb.resize(face);
  U.pc_off.resize(face);
  U.pc_diag.assign(N, -1.0);
  bool any_sym = false;
  for (int s = 0; s < S; ++s) any_sym = any_sym || !m.segs[s].host.pc_sym.empty();
  if (any_sym) U.pc_sym.assign(size_t(N) * dim, 0.0);
  U.bandwidth = 0;
  ua.xc.resize(size_t(N) * dim);   // segments write their cells and zero their padding
  ua.vol.assign(N, 0.0);
  ua.face.resize(size_t(face) * kFaceRec);
  ua.magG.resize(face);
  ua.bface.resize(size_t(bface) * kBfaceRec);
  ua.ext.assign(N, -1);
  const int64_t n_slices = (N + kSlice - 1) / kSlice;
  ua.slice_ptr.assign(n_slices + 1, 0);
  const int64_t n_blocks = (N + kFvBlock - 1) / kFvBlock;
  ua.seg_of_block.assign(n_blocks, 0);
  m.block_first.assign(S + 1, 0);
  ua.seg.resize(S);
  // slice widths first
  std::vector<int32_t> width(n_slices, 0);
  for (int s = 0; s < S; ++s) {
    const Segment& g = m.segs[s];
    const int64_t s0 = g.cell_off / kSlice;
    for (size_t k = 0; k + 1 < g.host.slice_ptr.size(); ++k)
      width[s0 + k] = (g.host.slice_ptr[k + 1] - g.host.slice_ptr[k]) / kSlice;
  }
  for (int64_t k = 0; k < n_slices; ++k) ua.slice_ptr[k + 1] = ua.slice_ptr[k] + width[k] * kSlice;
  ua.slot_nb.assign(ua.slice_ptr[n_slices], kSlotPad);
  ua.slot_fc.assign(ua.slice_ptr[n_slices], 0);
  // segments fill disjoint ranges: one host thread each
  parallel_for(S, [&](int64_t s, int) {
    const Segment& g = m.segs[s];
    const HostMesh& h = g.host;
    const int64_t co = g.cell_off, fo = g.face_off, bo = g.bface_off;
    const int64_t next = s + 1 < S ? m.segs[s + 1].cell_off : N;
    std::fill(ua.xc.begin() + (co + h.n_cells) * dim, ua.xc.begin() + next * dim, 0.0);  // padding
    for (int64_t c = 0; c < h.n_cells; ++c) {
      for (int k = 0; k < dim; ++k) ua.xc[(co + c) * dim + k] = h.xc[c * dim + k];
      ua.vol[co + c] = h.vol[c];
      U.pc_diag[co + c] = h.pc_diag[c];
      if (!h.pc_sym.empty())
        for (int k = 0; k < dim; ++k) U.pc_sym[(co + c) * dim + k] = h.pc_sym[c * dim + k];
      ua.ext[co + c] = int32_t(g.ext_off + h.old_of_new[c]);
    }
    for (int64_t j = 0; j < h.n_int; ++j) {
      U.fown[fo + j] = int32_t(h.fown[j] + co);
      U.fnb[fo + j] = int32_t(h.fnb[j] + co);
      U.pc_off[fo + j] = h.pc_off[j];
      ua.magG[fo + j] = h.magG[j];
      for (int k = 0; k < kFaceRec; ++k) ua.face[(fo + j) * kFaceRec + k] = h.face[j * kFaceRec + k];
    }
    for (int64_t j = 0; j < h.n_bnd * kBfaceRec; ++j) ua.bface[bo * kBfaceRec + j] = h.bface[j];
    const int64_t s0 = co / kSlice;
    for (size_t k = 0; k + 1 < h.slice_ptr.size(); ++k) {
      const int64_t src = h.slice_ptr[k], dst = ua.slice_ptr[s0 + k];
      for (int64_t q = 0; q < h.slice_ptr[k + 1] - src; ++q) {
        const int32_t nb = h.slot_nb[src + q], fc = h.slot_fc[src + q];
        if (nb >= 0) {
          ua.slot_nb[dst + q] = int32_t(nb + co);
          ua.slot_fc[dst + q] = fc >= 0 ? int32_t(fc + fo) : ~int32_t(~fc + fo);
        } else if (nb == kSlotBoundary) {
          ua.slot_nb[dst + q] = kSlotBoundary;
          ua.slot_fc[dst + q] = int32_t(fc + bo);
        }
      }
    }
  });
  for (int s = 0; s < S; ++s) {
    const Segment& g = m.segs[s];
    const HostMesh& h = g.host;
    const int64_t co = g.cell_off;
    U.bandwidth = std::max(U.bandwidth, h.bandwidth);
    SegInfo& si = ua.seg[s];
    si.mu = g.mat.mu;
    si.lam = g.mat.lam;
    si.kappa = g.mat.kappa;
    si.aK = g.mat.alpha_rc * g.mat.Kbar;
    si.law = g.mat.law;
    si.rho = g.mat.rho;
    si.cell_off = int32_t(co);
    si.n_cells = int32_t(h.n_cells);
    si.pad_ = 0;
    const int64_t b0 = co / kFvBlock;
    const int64_t b1 = (s + 1 < S) ? m.segs[s + 1].cell_off / kFvBlock : n_blocks;
    m.block_first[s] = int32_t(b0);
    for (int64_t b = b0; b < b1; ++b) ua.seg_of_block[b] = s;
  }
  m.block_first[S] = int32_t(n_blocks);
  // Tiles for the LDS-staged kernels (tiles never cross segments, since
  // segments start on multiples of kFvBlock).
  U.tiled = true;
  for (const Segment& g : m.segs) U.tiled = U.tiled && g.host.tiled;
  ua.halo_max = 0;
  ua.halo_ptr.assign(n_blocks + 1, 0);
  ua.halo_cells.clear();
  ua.slot_loc.clear();
  if (U.tiled) {
    ua.slot_loc.assign(ua.slot_nb.size(), kSlotPad);
    ua.slot_code.assign(ua.slot_nb.size(), -1);
    ua.bnd_ptr.assign(n_blocks + 1, 0);
    ua.bnd_face.clear();
    ua.bnd_loc.clear();
    ua.bnd_max = 0;
    ua.ent_max = 0;
    ua.fbeg.assign(n_blocks + 1, 0);
    ua.face_loc.assign(size_t(U.n_int), 0);
    ua.in_ptr.assign(n_blocks + 1, 0);
    ua.in_face.clear();
    ua.in_loc.clear();
    ua.faces_max = 0;
    ua.h2_ptr.assign(n_blocks + 1, 0);
    ua.h2_cells.clear();
    ua.h2_max = 0;
    ua.h1_width = 0;
    for (int64_t k = 0; k + 1 < int64_t(ua.slice_ptr.size()); ++k)
      ua.h1_width = std::max<int64_t>(ua.h1_width, (ua.slice_ptr[k + 1] - ua.slice_ptr[k]) / kSlice);
    ua.h1_loc.clear();
    ua.h1_mg.clear();
    ua.h1_fc.clear();
    ua.slot_mg.assign(ua.slot_nb.size(), 0.0);
    const int64_t n_slots = int64_t(ua.slot_nb.size());
    parallel_for((n_slots + 16 * kGeomChunk - 1) / (16 * kGeomChunk), [&](int64_t chunk, int) {
      const int64_t q0 = chunk * 16 * kGeomChunk, q1 = std::min(n_slots, q0 + 16 * kGeomChunk);
      for (int64_t q = q0; q < q1; ++q)
        if (ua.slot_nb[q] >= 0) {
          const int32_t fc = ua.slot_fc[q];
          ua.slot_mg[q] = ua.magG[fc >= 0 ? fc : ~fc];
        }
    });
    {
      // owned faces of tile t: owners ascend with the face number (slice order)
      int64_t f = 0;
      for (int64_t t = 0; t <= n_blocks; ++t) {
        while (f < U.n_int && U.fown[f] / kFvBlock < t) ++f;
        ua.fbeg[t] = int32_t(f);
      }
      for (int64_t j = 1; j < U.n_int; ++j)
        JFNK_REQUIRE(U.fown[j] / kFvBlock >= U.fown[j - 1] / kFvBlock, JFNK_E_MESH,
                     "mesh: internal faces not grouped by owner tile");
    }
    // Per tile: its lists into a buffer of its own (tiles on parallel host
    // threads; each tile writes only its own slots and owned faces in the
    // shared arrays), then the buffers are appended in tile order.
    struct TileLists {
      std::vector<int32_t> halo, ring2, in_face, in_loc, bnd_face, bnd_loc;
      std::vector<int16_t> h1_loc;
      std::vector<double> h1_mg;
      std::vector<int32_t> h1_fc;
      int32_t n_ent = 0;
    };
    std::vector<TileLists> tl(static_cast<size_t>(n_blocks));
    auto slots_of = [&](int32_t cell, auto&& fn) {
      const int64_t sl = cell / kSlice, lane = cell % kSlice;
      const int32_t w = (ua.slice_ptr[sl + 1] - ua.slice_ptr[sl]) / kSlice;
      for (int32_t k = 0; k < w; ++k) fn(k, ua.slice_ptr[sl] + k * kSlice + int32_t(lane));
    };
    auto one_tile = [&](int64_t t) {
      TileLists& o = tl[size_t(t)];
      std::vector<int32_t>& halo = o.halo;
      const int64_t c0 = t * kFvBlock, c1 = std::min<int64_t>(N, c0 + kFvBlock);
      const int64_t sl0 = c0 / kSlice, sl1 = (c1 - 1) / kSlice;
      for (int64_t sl = sl0; sl <= sl1; ++sl)
        for (int32_t q = ua.slice_ptr[sl]; q < ua.slice_ptr[sl + 1]; ++q) {
          const int32_t nb = ua.slot_nb[q];
          if (nb >= 0 && nb / kFvBlock != t) halo.push_back(nb);
        }
      std::sort(halo.begin(), halo.end());
      halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
      for (int64_t sl = sl0; sl <= sl1; ++sl)
        for (int32_t q = ua.slice_ptr[sl]; q < ua.slice_ptr[sl + 1]; ++q) {
          const int32_t nb = ua.slot_nb[q];
          if (nb < 0)
            ua.slot_loc[q] = nb;
          else if (nb / kFvBlock == t)
            ua.slot_loc[q] = int32_t(nb - c0);
          else
            ua.slot_loc[q] =
                kFvBlock + int32_t(std::lower_bound(halo.begin(), halo.end(), nb) - halo.begin());
        }
      // second ring: outside cells adjacent to the halo, not in tile or halo
      std::vector<int32_t>& ring2 = o.ring2;
      for (int32_t h : halo)
        slots_of(h, [&](int32_t, int32_t q) {
          const int32_t nb = ua.slot_nb[q];
          if (nb >= 0 && nb / kFvBlock != t && !std::binary_search(halo.begin(), halo.end(), nb))
            ring2.push_back(nb);
        });
      std::sort(ring2.begin(), ring2.end());
      ring2.erase(std::unique(ring2.begin(), ring2.end()), ring2.end());
      // halo cells' slots in the tile's local numbering, slot-major
      {
        const int64_t nh = int64_t(halo.size()), W = ua.h1_width;
        o.h1_loc.assign(size_t(nh * W), int16_t(kSlotPad));
        o.h1_mg.assign(size_t(nh * W), 0.0);
        o.h1_fc.assign(size_t(nh * W), 0);
        const int32_t nh32 = int32_t(nh);
        auto local = [&](int32_t cell) -> int32_t {
          if (cell / kFvBlock == t) return int32_t(cell - c0);
          auto it = std::lower_bound(halo.begin(), halo.end(), cell);
          if (it != halo.end() && *it == cell) return kFvBlock + int32_t(it - halo.begin());
          auto jt = std::lower_bound(ring2.begin(), ring2.end(), cell);
          return kFvBlock + nh32 + int32_t(jt - ring2.begin());
        };
        for (int64_t i = 0; i < nh; ++i)
          slots_of(halo[i], [&](int32_t k, int32_t q) {
            const int32_t nb = ua.slot_nb[q], fc = ua.slot_fc[q];
            const size_t e = size_t(k) * size_t(nh) + size_t(i);
            if (nb >= 0) {
              o.h1_loc[e] = int16_t(local(nb));
              o.h1_mg[e] = ua.magG[fc >= 0 ? fc : ~fc];
            } else {
              o.h1_loc[e] = int16_t(nb);
              if (nb == kSlotBoundary) o.h1_fc[e] = fc;
            }
          });
      }
      // face list: owned faces (entries 0 .. n_own-1), then incoming faces
      auto loc_of = [&](int32_t cell) {
        return cell / kFvBlock == t
                   ? int32_t(cell - c0)
                   : kFvBlock + int32_t(std::lower_bound(halo.begin(), halo.end(), cell) - halo.begin());
      };
      const int32_t f0 = ua.fbeg[t], n_own = ua.fbeg[t + 1] - f0;
      for (int32_t f = f0; f < f0 + n_own; ++f)
        ua.face_loc[f] = loc_of(U.fown[f]) | (loc_of(U.fnb[f]) << 16);
      int32_t n_in = 0;
      for (int64_t sl = sl0; sl <= sl1; ++sl)
        for (int32_t q = ua.slice_ptr[sl]; q < ua.slice_ptr[sl + 1]; ++q) {
          const int32_t nb = ua.slot_nb[q], fc = ua.slot_fc[q];
          if (nb < 0) continue;
          if (fc >= 0) {
            ua.slot_code[q] = 2 * (fc - f0);
          } else if (nb / kFvBlock == t) {
            ua.slot_code[q] = 2 * (~fc - f0) + 1;   // owner in this tile
          } else {
            o.in_face.push_back(~fc);
            o.in_loc.push_back(loc_of(U.fown[~fc]) | (loc_of(U.fnb[~fc]) << 16));
            ua.slot_code[q] = 2 * (n_own + n_in++) + 1;
          }
        }
      // boundary faces after the internal ones
      const int32_t n_ent = n_own + n_in;
      o.n_ent = n_ent;
      int32_t n_b = 0;
      for (int64_t sl = sl0; sl <= sl1; ++sl)
        for (int32_t q = ua.slice_ptr[sl]; q < ua.slice_ptr[sl + 1]; ++q) {
          if (ua.slot_nb[q] != kSlotBoundary) continue;
          const int32_t cell = int32_t(sl * kSlice + (q - ua.slice_ptr[sl]) % kSlice);
          o.bnd_face.push_back(ua.slot_fc[q]);
          o.bnd_loc.push_back(int32_t(cell - c0));
          ua.slot_code[q] = 2 * (n_ent + n_b++);
        }
    };
    parallel_for(n_blocks, [&](int64_t t, int) { one_tile(t); });
    // append in tile order
    for (int64_t t = 0; t < n_blocks; ++t) {
      TileLists& o = tl[size_t(t)];
      ua.halo_cells.insert(ua.halo_cells.end(), o.halo.begin(), o.halo.end());
      ua.halo_ptr[t + 1] = int32_t(ua.halo_cells.size());
      ua.halo_max = std::max<int64_t>(ua.halo_max, int64_t(o.halo.size()));
      ua.h2_cells.insert(ua.h2_cells.end(), o.ring2.begin(), o.ring2.end());
      ua.h2_ptr[t + 1] = int32_t(ua.h2_cells.size());
      ua.h2_max = std::max<int64_t>(ua.h2_max, int64_t(o.ring2.size()));
      ua.h1_loc.insert(ua.h1_loc.end(), o.h1_loc.begin(), o.h1_loc.end());
      ua.h1_mg.insert(ua.h1_mg.end(), o.h1_mg.begin(), o.h1_mg.end());
      ua.h1_fc.insert(ua.h1_fc.end(), o.h1_fc.begin(), o.h1_fc.end());
      ua.in_face.insert(ua.in_face.end(), o.in_face.begin(), o.in_face.end());
      ua.in_loc.insert(ua.in_loc.end(), o.in_loc.begin(), o.in_loc.end());
      ua.in_ptr[t + 1] = int32_t(ua.in_face.size());
      ua.bnd_face.insert(ua.bnd_face.end(), o.bnd_face.begin(), o.bnd_face.end());
      ua.bnd_loc.insert(ua.bnd_loc.end(), o.bnd_loc.begin(), o.bnd_loc.end());
      ua.bnd_ptr[t + 1] = int32_t(ua.bnd_face.size());
      ua.faces_max = std::max<int64_t>(ua.faces_max, o.n_ent);
      ua.bnd_max = std::max<int64_t>(ua.bnd_max, int64_t(o.bnd_face.size()));
      ua.ent_max = std::max<int64_t>(ua.ent_max, int64_t(o.n_ent) + int64_t(o.bnd_face.size()));
      o = TileLists();
    }
    JFNK_REQUIRE(ua.halo_max <= tile_halo_limit(dim), JFNK_E_MESH, "mesh: tile halo exceeds the LDS budget");
    JFNK_REQUIRE(ua.ent_max < 32768, JFNK_E_MESH, "mesh: too many faces inside a tile");
  }
  ua.pc_dinv = jacobi_inverse(U.pc_diag, U.pc_sym, dim);
}

std::vector<double> jacobi_inverse(const std::vector<double>& diag, const std::vector<double>& sym, int dim) {
  const size_t n = diag.size();
  if (sym.empty()) {
    std::vector<double> out(n);
    for (size_t c = 0; c < n; ++c) out[c] = 1.0 / diag[c];
    return out;
  }
  std::vector<double> out(n * dim);
  for (int q = 0; q < dim; ++q)
    for (size_t c = 0; c < n; ++c) out[q * n + c] = 1.0 / (diag[c] + sym[c * dim + q]);
  return out;
}

}  // namespace jfnk
