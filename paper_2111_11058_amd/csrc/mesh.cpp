// Mesh ingest: validation, canonical RWG tables, near-pair list, cell
// ordering and upload of the per-triangle geometry (paper Sec. II-B basis
// expansion, Sec. III-A cell division).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "internal.h"

namespace cbfm {

static thread_local std::string g_last_error = "no error";

void set_error(const std::string& msg) { g_last_error = msg; }

// 7-point degree-5 rule, barycentric coordinates (Radon; Strang & Fix).
static void quad_rule(double bary[7][3]) {
  const double s15 = std::sqrt(15.0);
  const double a = (6.0 - s15) / 21.0, b = (6.0 + s15) / 21.0;
  const double B[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {1 - 2 * a, a, a}, {a, 1 - 2 * a, a},
                          {a, a, 1 - 2 * a},           {1 - 2 * b, b, b}, {b, 1 - 2 * b, b},
                          {b, b, 1 - 2 * b}};
  std::memcpy(bary, B, sizeof(B));
}

static void build_tables(MeshHost& h) {
  const int64_t nt = h.nt;
  // local function a of triangle t: edge opposite vertex a, directed
  // v[a+1] -> v[a+2] in the triangle's counter-clockwise cycle.
  std::vector<std::array<int64_t, 3>> keys(nt * 3);  // (lo, hi, slot)
  for (int64_t t = 0; t < nt; ++t)
    for (int a = 0; a < 3; ++a) {
      int32_t u = h.T[t * 3 + (a + 1) % 3], v = h.T[t * 3 + (a + 2) % 3];
      keys[t * 3 + a] = {std::min(u, v), std::max(u, v), t * 3 + a};
    }
  std::sort(keys.begin(), keys.end());
  h.tri_edge.assign(nt * 3, -1);
  h.tri_sign.assign(nt * 3, 0);
  h.edges.clear();
  h.tplus.clear();
  h.tminus.clear();
  h.aplus.clear();
  h.aminus.clear();
  for (size_t i = 0; i < keys.size();) {
    size_t j = i;
    while (j < keys.size() && keys[j][0] == keys[i][0] && keys[j][1] == keys[i][1]) ++j;
    CBFM_REQUIRE(j - i == 2, CBFM_E_MESH,
                 "edge (" + std::to_string(keys[i][0]) + "," + std::to_string(keys[i][1]) +
                     ") is used by " + std::to_string(j - i) + " triangles (need 2)");
    const int32_t e = (int32_t)(h.edges.size() / 2);
    h.edges.push_back((int32_t)keys[i][0]);
    h.edges.push_back((int32_t)keys[i][1]);
    int32_t tp = -1, tm = -1, ap = -1, am = -1;
    for (size_t k = i; k < j; ++k) {
      const int64_t slot = keys[k][2], t = slot / 3;
      const int a = (int)(slot % 3);
      const int32_t from = h.T[t * 3 + (a + 1) % 3];
      const bool fwd = (from == (int32_t)keys[k][0]);
      if (fwd) {
        CBFM_REQUIRE(tp < 0, CBFM_E_MESH, "inconsistent triangle orientation");
        tp = (int32_t)t;
        ap = a;
      } else {
        CBFM_REQUIRE(tm < 0, CBFM_E_MESH, "inconsistent triangle orientation");
        tm = (int32_t)t;
        am = a;
      }
      h.tri_edge[slot] = e;
      h.tri_sign[slot] = fwd ? 1 : -1;
    }
    CBFM_REQUIRE(tp >= 0 && tm >= 0, CBFM_E_MESH, "inconsistent triangle orientation");
    h.tplus.push_back(tp);
    h.tminus.push_back(tm);
    h.aplus.push_back(ap);
    h.aminus.push_back(am);
    i = j;
  }
  h.ne = (int64_t)h.tplus.size();
  // geometry
  h.area.resize(nt);
  h.normal.resize(nt * 3);
  h.centroid.resize(nt * 3);
  double vol = 0;
  for (int64_t t = 0; t < nt; ++t) {
    const double* p0 = &h.V[3 * h.T[t * 3 + 0]];
    const double* p1 = &h.V[3 * h.T[t * 3 + 1]];
    const double* p2 = &h.V[3 * h.T[t * 3 + 2]];
    double e1[3], e2[3], cr[3];
    for (int i = 0; i < 3; ++i) {
      e1[i] = p1[i] - p0[i];
      e2[i] = p2[i] - p0[i];
    }
    cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double dbl = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    double scale = 0;
    for (int i = 0; i < 3; ++i) scale = std::max(scale, std::fabs(e1[i]) + std::fabs(e2[i]));
    CBFM_REQUIRE(dbl > 1e-14 * scale * scale && std::isfinite(dbl), CBFM_E_MESH,
                 "degenerate triangle " + std::to_string(t));
    h.area[t] = dbl / 2;
    for (int i = 0; i < 3; ++i) {
      h.normal[t * 3 + i] = cr[i] / dbl;
      h.centroid[t * 3 + i] = ((p0[i] + p1[i]) + p2[i]) / 3.0;
    }
    vol += p0[0] * (p1[1] * p2[2] - p1[2] * p2[1]) + p0[1] * (p1[2] * p2[0] - p1[0] * p2[2]) +
           p0[2] * (p1[0] * p2[1] - p1[1] * p2[0]);
  }
  CBFM_REQUIRE(vol > 0, CBFM_E_MESH, "enclosed volume is not positive (triangles must be "
                                     "counter-clockwise seen from outside)");
  h.length.resize(h.ne);
  for (int64_t e = 0; e < h.ne; ++e) {
    const double* a = &h.V[3 * h.edges[2 * e]];
    const double* b = &h.V[3 * h.edges[2 * e + 1]];
    const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    h.length[e] = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  }
}

// Near pairs: P == Q, a shared vertex, or |c_P - c_Q|^2 < 1.5^2 max(hP^2, hQ^2)
// with h the longest edge.  Candidates come from a uniform grid of cell size
// 1.5 max h, so no pair that passes the test is missed.
static void build_near(MeshHost& h) {
  const int64_t nt = h.nt;
  std::vector<double> h2(nt);
  double hmax = 0;
  for (int64_t t = 0; t < nt; ++t) {
    double m = 0;
    for (int a = 0; a < 3; ++a) {
      const double* u = &h.V[3 * h.T[t * 3 + a]];
      const double* v = &h.V[3 * h.T[t * 3 + (a + 1) % 3]];
      const double d0 = v[0] - u[0], d1 = v[1] - u[1], d2 = v[2] - u[2];
      m = std::max(m, (d0 * d0 + d1 * d1) + d2 * d2);
    }
    h2[t] = m;
    hmax = std::max(hmax, std::sqrt(m));
  }
  const double cell = 1.5 * hmax * (1 + 1e-9);
  double lo[3] = {1e300, 1e300, 1e300};
  for (int64_t t = 0; t < nt; ++t)
    for (int i = 0; i < 3; ++i) lo[i] = std::min(lo[i], h.centroid[t * 3 + i]);
  auto key = [&](int64_t x, int64_t y, int64_t z) { return (x * 1000003 + y) * 1000033 + z; };
  std::unordered_map<int64_t, std::vector<int32_t>> grid;
  std::vector<std::array<int64_t, 3>> gc(nt);
  for (int64_t t = 0; t < nt; ++t) {
    for (int i = 0; i < 3; ++i) gc[t][i] = (int64_t)std::floor((h.centroid[t * 3 + i] - lo[i]) / cell);
    grid[key(gc[t][0], gc[t][1], gc[t][2])].push_back((int32_t)t);
  }
  // vertex -> triangles
  std::vector<std::vector<int32_t>> vt(h.nv);
  for (int64_t t = 0; t < nt; ++t)
    for (int a = 0; a < 3; ++a) vt[h.T[t * 3 + a]].push_back((int32_t)t);
  h.near.clear();
  std::vector<int32_t> cand;
  for (int64_t p = 0; p < nt; ++p) {
    cand.clear();
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          auto it = grid.find(key(gc[p][0] + dx, gc[p][1] + dy, gc[p][2] + dz));
          if (it == grid.end()) continue;
          for (int32_t q : it->second) {
            const double d0 = h.centroid[q * 3 + 0] - h.centroid[p * 3 + 0];
            const double d1 = h.centroid[q * 3 + 1] - h.centroid[p * 3 + 1];
            const double d2 = h.centroid[q * 3 + 2] - h.centroid[p * 3 + 2];
            const double d2s = (d0 * d0 + d1 * d1) + d2 * d2;
            if (d2s < 2.25 * std::max(h2[p], h2[q])) cand.push_back(q);
          }
        }
    for (int a = 0; a < 3; ++a)
      for (int32_t q : vt[h.T[p * 3 + a]]) cand.push_back(q);
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    for (int32_t q : cand) {
      NearPair np{(int32_t)p, q, (int32_t)p, q, 0, 0};
      // coplanar: parallel normals and Q's centroid in P's plane
      const double* n1 = &h.normal[p * 3];
      const double* n2 = &h.normal[q * 3];
      const double c0 = n1[1] * n2[2] - n1[2] * n2[1];
      const double c1 = n1[2] * n2[0] - n1[0] * n2[2];
      const double c2 = n1[0] * n2[1] - n1[1] * n2[0];
      if ((c0 * c0 + c1 * c1) + c2 * c2 <= 1e-20) {
        double dc = 0;
        for (int i = 0; i < 3; ++i) dc += n1[i] * (h.centroid[q * 3 + i] - h.centroid[p * 3 + i]);
        if (std::fabs(dc) <= 1e-10 * std::sqrt(h.area[p])) np.coplanar = 1;
      }
      if (p == q) np.coplanar = 1;
      h.near.push_back(np);
    }
  }
}

}  // namespace cbfm

using namespace cbfm;

cbfm::TriTab<double> cbfm_mesh_s::tab64() const {
  TriTab<double> t;
  const int64_t nt = h.nt;
  for (int i = 0; i < 3; ++i) {
    t.q[i] = q64.as<double>() + i * 7 * nt;
    t.v[i] = v64.as<double>() + i * 3 * nt;
    t.cen[i] = cen.as<double>() + i * nt;
  }
  t.c = c64.as<double>();
  t.nt = nt;
  return t;
}

cbfm::TriTab<float> cbfm_mesh_s::tab32() const {
  TriTab<float> t;
  const int64_t nt = h.nt;
  for (int i = 0; i < 3; ++i) {
    t.q[i] = q32.as<float>() + i * 7 * nt;
    t.v[i] = v32.as<float>() + i * 3 * nt;
    t.cen[i] = cen.as<double>() + i * nt;
  }
  t.c = c32.as<float>();
  t.nt = nt;
  return t;
}

static void analyze_host(MeshHost& h, const double* xyz, int64_t nv, const int32_t* tri, int64_t nt,
                         const int32_t* edge_block, int32_t nblocks) {
  CBFM_REQUIRE(xyz && tri && nv >= 4 && nt >= 4, CBFM_E_ARG, "need nv >= 4, nt >= 4 and non-null arrays");
  CBFM_REQUIRE(nt < (int64_t)1 << 30 && nv < (int64_t)1 << 30, CBFM_E_ARG, "mesh too large");
  h.nv = nv;
  h.nt = nt;
  h.V.assign(xyz, xyz + nv * 3);
  h.T.assign(tri, tri + nt * 3);
  for (int64_t i = 0; i < nv * 3; ++i)
    CBFM_REQUIRE(std::isfinite(h.V[i]), CBFM_E_MESH, "non-finite vertex coordinate");
  for (int64_t i = 0; i < nt * 3; ++i)
    CBFM_REQUIRE(h.T[i] >= 0 && h.T[i] < nv, CBFM_E_MESH, "triangle vertex index out of range");
  for (int64_t t = 0; t < nt; ++t)
    CBFM_REQUIRE(h.T[t * 3] != h.T[t * 3 + 1] && h.T[t * 3] != h.T[t * 3 + 2] &&
                     h.T[t * 3 + 1] != h.T[t * 3 + 2],
                 CBFM_E_MESH, "triangle with repeated vertex");
  build_tables(h);
  // cells
  if (edge_block == nullptr) {
    h.nblocks = 1;
    h.edge_block.assign(h.ne, 0);
  } else {
    CBFM_REQUIRE(nblocks >= 1, CBFM_E_ARG, "nblocks must be >= 1");
    h.nblocks = nblocks;
    h.edge_block.assign(edge_block, edge_block + h.ne);
    for (int32_t b : h.edge_block)
      CBFM_REQUIRE(b >= 0 && b < nblocks, CBFM_E_ARG, "edge_block value out of range");
  }
  h.perm.resize(h.ne);
  std::iota(h.perm.begin(), h.perm.end(), 0);
  std::stable_sort(h.perm.begin(), h.perm.end(),
                   [&](int32_t a, int32_t b) { return h.edge_block[a] < h.edge_block[b]; });
  h.iperm.resize(h.ne);
  for (int64_t i = 0; i < h.ne; ++i) h.iperm[h.perm[i]] = (int32_t)i;
  h.cell_off.assign(h.nblocks + 1, 0);
  for (int32_t b : h.edge_block) h.cell_off[b + 1]++;
  for (int b = 0; b < h.nblocks; ++b) {
    CBFM_REQUIRE(h.cell_off[b + 1] > 0, CBFM_E_MESH, "cell " + std::to_string(b) + " is empty");
    h.cell_off[b + 1] += h.cell_off[b];
  }
  build_near(h);
}

static void upload(cbfm_mesh_s* m) {
  const MeshHost& h = m->h;
  const int64_t nt = h.nt;
  double bary[7][3];
  quad_rule(bary);
  std::vector<double> q64(3 * 7 * nt), v64(3 * 3 * nt), c64(3 * nt), cen(3 * nt), xyz9(9 * nt);
  std::vector<float> q32(q64.size()), v32(v64.size()), c32(c64.size());
  for (int64_t t = 0; t < nt; ++t) {
    const double* P[3] = {&h.V[3 * h.T[t * 3]], &h.V[3 * h.T[t * 3 + 1]], &h.V[3 * h.T[t * 3 + 2]]};
    const double* c = &h.centroid[3 * t];
    for (int i = 0; i < 3; ++i) {
      cen[i * nt + t] = c[i];
      for (int k = 0; k < 7; ++k) {
        const double x = bary[k][0] * P[0][i] + bary[k][1] * P[1][i] + bary[k][2] * P[2][i];
        q64[(i * 7 + k) * nt + t] = x - c[i];
      }
      for (int a = 0; a < 3; ++a) {
        v64[(i * 3 + a) * nt + t] = P[a][i] - c[i];
        xyz9[t * 9 + a * 3 + i] = P[a][i];
      }
    }
    for (int a = 0; a < 3; ++a)
      c64[a * nt + t] = h.tri_sign[t * 3 + a] * h.length[h.tri_edge[t * 3 + a]];
  }
  for (size_t i = 0; i < q64.size(); ++i) q32[i] = (float)q64[i];
  for (size_t i = 0; i < v64.size(); ++i) v32[i] = (float)v64[i];
  for (size_t i = 0; i < c64.size(); ++i) c32[i] = (float)c64[i];
  m->q64.upload(q64);
  m->v64.upload(v64);
  m->c64.upload(c64);
  m->q32.upload(q32);
  m->v32.upload(v32);
  m->c32.upload(c32);
  m->cen.upload(cen);
  m->tri_xyz.upload(xyz9);
  m->tri_edge.upload(h.tri_edge);
  m->tri_sign.upload(h.tri_sign);
  m->tplus.upload(h.tplus);
  m->tminus.upload(h.tminus);
  m->aplus.upload(h.aplus);
  m->aminus.upload(h.aminus);
  m->length.upload(h.length);
  m->area.upload(h.area);
  m->perm.upload(h.perm);
  m->iperm.upload(h.iperm);
}

extern "C" {

const char* cbfm_last_error(void) { return cbfm::g_last_error.c_str(); }

int32_t cbfm_version(void) { return 7; }

// Whether every cell is cell 0 moved by one vector: equal RWG counts, and
// RWG i of cell b (cell order) lies on triangles whose vertices, in their
// stored order, are those of RWG i of cell 0 plus the shift, with the same
// free vertices; and no triangle carries RWGs of two cells.  Coordinates
// must agree within 1e-9 of the mesh extent.
static void find_translates(cbfm_mesh_s* m) {
  const MeshHost& h = m->h;
  const int nb = h.nblocks;
  m->translated = false;
  if (nb < 2 || h.ne == 0) return;
  const int64_t N0 = h.cell_off[1] - h.cell_off[0];
  for (int b = 1; b < nb; ++b)
    if (h.cell_off[b + 1] - h.cell_off[b] != N0) return;
  std::vector<int32_t> tcell(h.nt, -1);
  for (int b = 0; b < nb; ++b)
    for (int64_t i = h.cell_off[b]; i < h.cell_off[b + 1]; ++i) {
      const int e = h.perm[i];
      for (const int32_t t : {h.tplus[e], h.tminus[e]}) {
        if (tcell[t] >= 0 && tcell[t] != b) return;
        tcell[t] = b;
      }
    }
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < h.nv; ++v)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], h.V[v * 3 + c]);
      hi[c] = std::max(hi[c], h.V[v * 3 + c]);
    }
  const double tol = 1e-9 * std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
  const double* V = h.V.data();
  auto vtx = [&](int32_t t, int a) { return V + 3 * (int64_t)h.T[3 * (int64_t)t + a]; };
  std::vector<double> shift((size_t)nb * 3, 0.0);
  const int e00 = h.perm[h.cell_off[0]];
  for (int b = 1; b < nb; ++b) {
    const int eb0 = h.perm[h.cell_off[b]];
    double* d = &shift[(size_t)b * 3];
    for (int c = 0; c < 3; ++c) d[c] = vtx(h.tplus[eb0], 0)[c] - vtx(h.tplus[e00], 0)[c];
    for (int64_t i = 0; i < N0; ++i) {
      const int e0 = h.perm[h.cell_off[0] + i], eb = h.perm[h.cell_off[b] + i];
      if (h.aplus[e0] != h.aplus[eb] || h.aminus[e0] != h.aminus[eb]) return;
      for (const auto& tt : {std::make_pair(h.tplus[e0], h.tplus[eb]), std::make_pair(h.tminus[e0], h.tminus[eb])})
        for (int a = 0; a < 3; ++a)
          for (int c = 0; c < 3; ++c)
            if (std::abs(vtx(tt.second, a)[c] - vtx(tt.first, a)[c] - d[c]) > tol) return;
    }
  }
  m->translated = true;
  m->shift = std::move(shift);
  m->tcell = std::move(tcell);
}

cbfm_status cbfm_mesh_load(const double* xyz, int64_t nv, const int32_t* tri, int64_t nt,
                           const int32_t* edge_block, int32_t nblocks, cbfm_mesh* out) {
  return guarded([&] {
    CBFM_REQUIRE(out != nullptr, CBFM_E_ARG, "out is NULL");
    *out = nullptr;
    auto* m = new cbfm_mesh_s();
    try {
      MeshHost& h = m->h;
      analyze_host(h, xyz, nv, tri, nt, edge_block, nblocks);
      find_translates(m);
      upload(m);
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
  });
}


cbfm_status cbfm_mesh_info(cbfm_mesh m, int64_t* ne, int64_t* nt, int32_t* nblocks, int64_t* n_near) {
  return guarded([&] {
    CBFM_REQUIRE(m != nullptr, CBFM_E_ARG, "mesh is NULL");
    if (ne) *ne = m->h.ne;
    if (nt) *nt = m->h.nt;
    if (nblocks) *nblocks = m->h.nblocks;
    if (n_near) *n_near = (int64_t)m->h.near.size();
  });
}

cbfm_status cbfm_mesh_edges(cbfm_mesh m, int32_t* ev, int32_t* eb) {
  return guarded([&] {
    CBFM_REQUIRE(m != nullptr, CBFM_E_ARG, "mesh is NULL");
    if (ev) std::memcpy(ev, m->h.edges.data(), m->h.edges.size() * sizeof(int32_t));
    if (eb) std::memcpy(eb, m->h.edge_block.data(), m->h.edge_block.size() * sizeof(int32_t));
  });
}

void cbfm_mesh_free(cbfm_mesh m) { delete m; }

}  // extern "C"

extern "C" cbfm_status cbfm_mesh_analyze(const double* xyz, int64_t nv, const int32_t* tri, int64_t nt,
                                         const int32_t* edge_block, int32_t nblocks, int64_t* ne,
                                         int32_t* edges_host, int32_t* tri_edge_host, int32_t* tri_sign_host,
                                         int64_t* n_near, int32_t* near_host, int64_t near_cap) {
  return guarded([&] {
    MeshHost h;
    analyze_host(h, xyz, nv, tri, nt, edge_block, nblocks);
    if (ne) *ne = h.ne;
    if (edges_host) std::memcpy(edges_host, h.edges.data(), h.edges.size() * sizeof(int32_t));
    if (tri_edge_host) std::memcpy(tri_edge_host, h.tri_edge.data(), h.tri_edge.size() * sizeof(int32_t));
    if (tri_sign_host) std::memcpy(tri_sign_host, h.tri_sign.data(), h.tri_sign.size() * sizeof(int32_t));
    if (n_near) *n_near = (int64_t)h.near.size();
    if (near_host) {
      CBFM_REQUIRE(near_cap >= (int64_t)h.near.size(), CBFM_E_ARG, "near_host capacity too small");
      for (size_t i = 0; i < h.near.size(); ++i) {
        near_host[3 * i] = h.near[i].p;
        near_host[3 * i + 1] = h.near[i].q;
        near_host[3 * i + 2] = h.near[i].coplanar;
      }
    }
  });
}
