// Host-side collision geometry: quickhull in FP64, coplanar-facet merging,
// feature edges and space-filling-curve serialization.
//
// A convex piece's SDF is the smooth intersection of its facet half-spaces
// (Sec. III-A.3); its mesh is its hull vertices and the edges between facets
// on different planes.  Vertices and edges are reordered along a Z-order or
// Hilbert curve so neighbouring indices are close in space (Sec. IV-C.3).
#include "geom.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <unordered_map>

namespace cm {

namespace {

struct P3 { double x, y, z; };
inline P3 sub(P3 a, P3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot3(P3 a, P3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline P3 cross3(P3 a, P3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm3(P3 a) { return std::sqrt(dot3(a, a)); }

struct Face {
  int v[3];        // counter-clockwise seen from outside
  int nb[3];       // neighbour across edge (v[i], v[(i+1)%3])
  P3 n;            // unit outward normal
  double d;        // plane: n.x + d = 0
  std::vector<int> outside;  // points strictly above the plane
  int far = -1;    // furthest outside point
  double far_d = 0;
  bool alive = true;
  int mark = 0;
};

class QuickHull {
 public:
  QuickHull(const double* xyz, int64_t n) : n_(int(n)) {
    pts_.resize(size_t(n));
    double s = 0;
    for (int i = 0; i < n_; ++i) {
      pts_[size_t(i)] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
      s = std::max({s, std::fabs(xyz[3 * i]), std::fabs(xyz[3 * i + 1]), std::fabs(xyz[3 * i + 2])});
    }
    scale_ = std::max(s, 1e-300);
    eps_ = 1e-11 * scale_;
  }

  int run() {
    if (n_ < 4) return -3;
    if (!initial_simplex()) return -3;
    std::vector<int> stack;
    for (int f = 0; f < int(faces_.size()); ++f) if (!faces_[size_t(f)].outside.empty()) stack.push_back(f);
    int iter = 0;
    while (!stack.empty()) {
      int f = stack.back();
      stack.pop_back();
      Face& F = faces_[size_t(f)];
      if (!F.alive || F.outside.empty()) continue;
      if (++iter > 8 * n_ + 64) return -3;  // safety: cannot happen on valid input
      add_point(f, F.far, stack);
    }
    return 0;
  }

  const std::vector<Face>& faces() const { return faces_; }
  const std::vector<P3>& pts() const { return pts_; }
  double scale() const { return scale_; }

 private:
  double dist(const Face& f, int p) const { return dot3(f.n, pts_[size_t(p)]) + f.d; }

  bool make_plane(Face& f) {
    P3 a = pts_[size_t(f.v[0])], b = pts_[size_t(f.v[1])], c = pts_[size_t(f.v[2])];
    P3 n = cross3(sub(b, a), sub(c, a));
    double l = norm3(n);
    if (!(l > 0)) return false;
    f.n = {n.x / l, n.y / l, n.z / l};
    // offset through the centroid of the three vertices (less rounding bias)
    P3 g = {(a.x + b.x + c.x) / 3, (a.y + b.y + c.y) / 3, (a.z + b.z + c.z) / 3};
    f.d = -dot3(f.n, g);
    return true;
  }

  bool initial_simplex() {
    // extremes along the axes; the farthest pair among them
    int ext[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < n_; ++i) {
      const P3& p = pts_[size_t(i)];
      if (p.x < pts_[size_t(ext[0])].x) ext[0] = i;
      if (p.x > pts_[size_t(ext[1])].x) ext[1] = i;
      if (p.y < pts_[size_t(ext[2])].y) ext[2] = i;
      if (p.y > pts_[size_t(ext[3])].y) ext[3] = i;
      if (p.z < pts_[size_t(ext[4])].z) ext[4] = i;
      if (p.z > pts_[size_t(ext[5])].z) ext[5] = i;
    }
    int i0 = 0, i1 = 0;
    double best = -1;
    for (int a = 0; a < 6; ++a)
      for (int b = a + 1; b < 6; ++b) {
        double d = norm3(sub(pts_[size_t(ext[a])], pts_[size_t(ext[b])]));
        if (d > best) { best = d; i0 = ext[a]; i1 = ext[b]; }
      }
    if (best <= eps_) return false;
    // farthest from the line i0-i1
    P3 u = sub(pts_[size_t(i1)], pts_[size_t(i0)]);
    int i2 = -1;
    best = eps_;
    for (int i = 0; i < n_; ++i) {
      double d = norm3(cross3(u, sub(pts_[size_t(i)], pts_[size_t(i0)]))) / norm3(u);
      if (d > best) { best = d; i2 = i; }
    }
    if (i2 < 0) return false;
    // farthest from the plane
    P3 pn = cross3(u, sub(pts_[size_t(i2)], pts_[size_t(i0)]));
    double pl = norm3(pn);
    int i3 = -1;
    best = eps_;
    for (int i = 0; i < n_; ++i) {
      double d = std::fabs(dot3(pn, sub(pts_[size_t(i)], pts_[size_t(i0)]))) / pl;
      if (d > best) { best = d; i3 = i; }
    }
    if (i3 < 0) return false;
    int V[4] = {i0, i1, i2, i3};
    P3 c = {0, 0, 0};
    for (int k = 0; k < 4; ++k) {
      c.x += pts_[size_t(V[k])].x / 4; c.y += pts_[size_t(V[k])].y / 4; c.z += pts_[size_t(V[k])].z / 4;
    }
    // faces opposite each vertex, oriented outward
    const int tri[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
    faces_.resize(4);
    for (int f = 0; f < 4; ++f) {
      Face& F = faces_[size_t(f)];
      F.v[0] = V[tri[f][0]]; F.v[1] = V[tri[f][1]]; F.v[2] = V[tri[f][2]];
      make_plane(F);
      if (dot3(F.n, c) + F.d > 0) {  // flip to point away from the centroid
        std::swap(F.v[1], F.v[2]);
        make_plane(F);
      }
    }
    // neighbours by matching directed edges
    for (int f = 0; f < 4; ++f)
      for (int e = 0; e < 3; ++e) {
        int a = faces_[size_t(f)].v[e], b = faces_[size_t(f)].v[(e + 1) % 3];
        faces_[size_t(f)].nb[e] = -1;
        for (int g = 0; g < 4; ++g) {
          if (g == f) continue;
          for (int k = 0; k < 3; ++k)
            if (faces_[size_t(g)].v[k] == b && faces_[size_t(g)].v[(k + 1) % 3] == a) faces_[size_t(f)].nb[e] = g;
        }
      }
    // conflict lists
    for (int i = 0; i < n_; ++i) {
      if (i == i0 || i == i1 || i == i2 || i == i3) continue;
      assign(i, 0, 4);
    }
    return true;
  }

  // Puts point p into the outside set of the first face in [f0, f1) that sees it.
  void assign(int p, int f0, int f1, const std::vector<int>* cand = nullptr) {
    if (cand) {
      for (int f : *cand) {
        Face& F = faces_[size_t(f)];
        double d = dist(F, p);
        if (d > eps_) { F.outside.push_back(p); if (d > F.far_d) { F.far_d = d; F.far = p; } return; }
      }
      return;
    }
    for (int f = f0; f < f1; ++f) {
      Face& F = faces_[size_t(f)];
      double d = dist(F, p);
      if (d > eps_) { F.outside.push_back(p); if (d > F.far_d) { F.far_d = d; F.far = p; } return; }
    }
  }

  void add_point(int f0, int eye, std::vector<int>& stack) {
    ++stamp_;
    // visible faces: flood fill from f0
    std::vector<int> visible, todo{f0};
    faces_[size_t(f0)].mark = stamp_;
    while (!todo.empty()) {
      int f = todo.back(); todo.pop_back();
      visible.push_back(f);
      for (int e = 0; e < 3; ++e) {
        int g = faces_[size_t(f)].nb[e];
        if (g < 0 || faces_[size_t(g)].mark == stamp_) continue;
        if (dist(faces_[size_t(g)], eye) > eps_) { faces_[size_t(g)].mark = stamp_; todo.push_back(g); }
      }
    }
    // horizon edges (a, b) of visible faces whose neighbour is not visible
    struct HE { int a, b, nbr; };
    std::vector<HE> horizon;
    for (int f : visible)
      for (int e = 0; e < 3; ++e) {
        int g = faces_[size_t(f)].nb[e];
        if (faces_[size_t(g)].mark != stamp_)
          horizon.push_back({faces_[size_t(f)].v[e], faces_[size_t(f)].v[(e + 1) % 3], g});
      }
    // new faces (a, b, eye), same winding as the visible face they replace
    std::unordered_map<int, int> by_start, by_end;
    std::vector<int> created;
    for (const HE& h : horizon) {
      Face F;
      F.v[0] = h.a; F.v[1] = h.b; F.v[2] = eye;
      make_plane(F);
      F.nb[0] = h.nbr;
      int id = int(faces_.size());
      faces_.push_back(F);
      created.push_back(id);
      by_start[h.a] = id;
      by_end[h.b] = id;
      // fix the outside neighbour's back pointer for edge (b, a)
      Face& N = faces_[size_t(h.nbr)];
      for (int k = 0; k < 3; ++k)
        if (N.v[k] == h.b && N.v[(k + 1) % 3] == h.a) N.nb[k] = id;
    }
    for (int id : created) {
      Face& F = faces_[size_t(id)];
      F.nb[1] = by_start[F.v[1]];  // edge (b, eye) borders the face starting at b
      F.nb[2] = by_end[F.v[0]];    // edge (eye, a) borders the face ending at a
    }
    // reassign orphaned points
    for (int f : visible) {
      Face& F = faces_[size_t(f)];
      F.alive = false;
      for (int p : F.outside) if (p != eye) assign(p, 0, 0, &created);
      F.outside.clear();
      F.outside.shrink_to_fit();
    }
    for (int id : created) if (!faces_[size_t(id)].outside.empty()) stack.push_back(id);
  }

  int n_;
  std::vector<P3> pts_;
  std::vector<Face> faces_;
  double scale_, eps_;
  int stamp_ = 0;
};

int find_root(std::vector<int>& par, int a) {
  while (par[size_t(a)] != a) { par[size_t(a)] = par[size_t(par[size_t(a)])]; a = par[size_t(a)]; }
  return a;
}

}  // namespace

int build_hull_piece(const double* xyz, int64_t n, PieceGeom* out) {
  QuickHull qh(xyz, n);
  int st = qh.run();
  if (st != 0) return st;
  const auto& faces = qh.faces();
  const auto& pts = qh.pts();
  std::vector<int> alive;
  std::vector<int> idx(faces.size(), -1);
  for (int f = 0; f < int(faces.size()); ++f)
    if (faces[size_t(f)].alive) { idx[size_t(f)] = int(alive.size()); alive.push_back(f); }
  const int F = int(alive.size());
  // merge adjacent facets on the same plane
  std::vector<int> par(static_cast<size_t>(F));
  std::iota(par.begin(), par.end(), 0);
  const double tol = 1e-9;
  for (int i = 0; i < F; ++i) {
    const Face& A = faces[size_t(alive[size_t(i)])];
    for (int e = 0; e < 3; ++e) {
      const int j = idx[size_t(A.nb[e])];
      const Face& B = faces[size_t(A.nb[e])];
      double dn = std::sqrt((A.n.x - B.n.x) * (A.n.x - B.n.x) + (A.n.y - B.n.y) * (A.n.y - B.n.y) +
                            (A.n.z - B.n.z) * (A.n.z - B.n.z));
      if (dn < tol && std::fabs(A.d - B.d) < tol * qh.scale()) {
        int ra = find_root(par, i), rb = find_root(par, j);
        if (ra != rb) par[size_t(std::max(ra, rb))] = std::min(ra, rb);
      }
    }
  }
  // one plane per group: normalised mean normal, offset through the outermost vertex
  std::vector<int> gid(size_t(F), -1);
  std::vector<int> roots;
  for (int i = 0; i < F; ++i) {
    int r = find_root(par, i);
    if (gid[size_t(r)] < 0) { gid[size_t(r)] = int(roots.size()); roots.push_back(r); }
    gid[size_t(i)] = gid[size_t(r)];
  }
  const int G = int(roots.size());
  std::vector<P3> gn(size_t(G), P3{0, 0, 0});
  for (int i = 0; i < F; ++i) {
    const Face& A = faces[size_t(alive[size_t(i)])];
    P3& s = gn[size_t(gid[size_t(i)])];
    s.x += A.n.x; s.y += A.n.y; s.z += A.n.z;
  }
  std::vector<double> gh(size_t(G), -1e300);
  for (int g = 0; g < G; ++g) {
    double l = norm3(gn[size_t(g)]);
    gn[size_t(g)] = {gn[size_t(g)].x / l, gn[size_t(g)].y / l, gn[size_t(g)].z / l};
  }
  for (int i = 0; i < F; ++i) {
    const Face& A = faces[size_t(alive[size_t(i)])];
    int g = gid[size_t(i)];
    for (int k = 0; k < 3; ++k) gh[size_t(g)] = std::max(gh[size_t(g)], dot3(gn[size_t(g)], pts[size_t(A.v[k])]));
  }
  // vertices used by the hull, in input order
  std::vector<int> used(pts.size(), -1);
  for (int i = 0; i < F; ++i)
    for (int k = 0; k < 3; ++k) used[size_t(faces[size_t(alive[size_t(i)])].v[k])] = 1;
  out->verts.clear();
  int nv = 0;
  for (size_t p = 0; p < pts.size(); ++p)
    if (used[p] > 0) {
      used[p] = nv++;
      out->verts.push_back(pts[p].x); out->verts.push_back(pts[p].y); out->verts.push_back(pts[p].z);
    }
  // feature edges: between facets of different planes
  std::vector<std::pair<int, int>> edges;
  for (int i = 0; i < F; ++i) {
    const Face& A = faces[size_t(alive[size_t(i)])];
    for (int e = 0; e < 3; ++e) {
      int j = idx[size_t(A.nb[e])];
      if (gid[size_t(i)] == gid[size_t(j)]) continue;
      int a = used[size_t(A.v[e])], b = used[size_t(A.v[(e + 1) % 3])];
      if (a < b) edges.push_back({a, b});  // each edge is seen twice; keep one direction
    }
  }
  std::sort(edges.begin(), edges.end());
  edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
  out->edges.clear();
  for (auto& e : edges) { out->edges.push_back(e.first); out->edges.push_back(e.second); }
  out->planes.clear();
  for (int g = 0; g < G; ++g) {
    out->planes.push_back(gn[size_t(g)].x); out->planes.push_back(gn[size_t(g)].y);
    out->planes.push_back(gn[size_t(g)].z); out->planes.push_back(-gh[size_t(g)]);
  }
  return 0;
}

uint32_t morton_key(uint32_t x, uint32_t y, uint32_t z) {
  auto spread = [](uint32_t v) {
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000ff;
    v = (v | (v << 8)) & 0x0300f00f;
    v = (v | (v << 4)) & 0x030c30c3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
  };
  return (spread(x) << 2) | (spread(y) << 1) | spread(z);
}

// Hilbert index of a 3-D point with 10-bit coordinates, after J. Skilling,
// "Programming the Hilbert curve", AIP Conf. Proc. 707 (2004): convert the
// axes to the "transposed" Hilbert index, then interleave its bits.
uint32_t hilbert_key(uint32_t x, uint32_t y, uint32_t z) {
  const int bits = 10;
  uint32_t X[3] = {x & 0x3ff, y & 0x3ff, z & 0x3ff};
  const uint32_t M = 1u << (bits - 1);
  // inverse undo of excess work
  for (uint32_t Q = M; Q > 1; Q >>= 1) {
    uint32_t P = Q - 1;
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        uint32_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  // Gray encode
  for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];
  uint32_t t = 0;
  for (uint32_t Q = M; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  for (int i = 0; i < 3; ++i) X[i] ^= t;
  // interleave: most significant bit of X[0] first
  uint32_t key = 0;
  for (int b = bits - 1; b >= 0; --b)
    for (int i = 0; i < 3; ++i) key = (key << 1) | ((X[i] >> b) & 1u);
  return key;
}

void serialize_piece(PieceGeom* g, int curve) {
  if (curve == 0) return;
  const size_t V = g->n_verts(), E = g->n_edges();
  if (V == 0) return;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (size_t i = 0; i < V; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], g->verts[3 * i + size_t(a)]);
      hi[a] = std::max(hi[a], g->verts[3 * i + size_t(a)]);
    }
  auto key = [&](const double* p) {
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
      double ext = hi[a] - lo[a];
      double u = ext > 0 ? (p[a] - lo[a]) / ext : 0.0;
      q[a] = uint32_t(std::min(1023.0, std::max(0.0, std::floor(u * 1024.0))));
    }
    return curve == 1 ? morton_key(q[0], q[1], q[2]) : hilbert_key(q[0], q[1], q[2]);
  };
  std::vector<uint32_t> vk(V);
  for (size_t i = 0; i < V; ++i) vk[i] = key(&g->verts[3 * i]);
  std::vector<int> order(V);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return vk[size_t(a)] < vk[size_t(b)]; });
  std::vector<int> inv(V);
  std::vector<double> nv(3 * V);
  for (size_t k = 0; k < V; ++k) {
    inv[size_t(order[k])] = int(k);
    for (int a = 0; a < 3; ++a) nv[3 * k + size_t(a)] = g->verts[3 * size_t(order[k]) + size_t(a)];
  }
  g->verts.swap(nv);
  std::vector<uint32_t> ek(E);
  for (size_t e = 0; e < E; ++e) {
    int a = inv[size_t(g->edges[2 * e])], b = inv[size_t(g->edges[2 * e + 1])];
    g->edges[2 * e] = std::min(a, b);
    g->edges[2 * e + 1] = std::max(a, b);
    double m[3];
    for (int c = 0; c < 3; ++c)
      m[c] = 0.5 * (g->verts[3 * size_t(a) + size_t(c)] + g->verts[3 * size_t(b) + size_t(c)]);
    ek[e] = key(m);
  }
  std::vector<int> eo(E);
  std::iota(eo.begin(), eo.end(), 0);
  std::stable_sort(eo.begin(), eo.end(), [&](int a, int b) { return ek[size_t(a)] < ek[size_t(b)]; });
  std::vector<int32_t> ne(2 * E);
  for (size_t k = 0; k < E; ++k) {
    ne[2 * k] = g->edges[2 * size_t(eo[k])];
    ne[2 * k + 1] = g->edges[2 * size_t(eo[k]) + 1];
  }
  g->edges.swap(ne);
}

}  // namespace cm
