// Host runtime and C ABI of the contact-manifold library (see include/cm.h).
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>

namespace cm {

constexpr double kLog2eD = 1.4426950408889634;

cm_status fail(cm_context* ctx, cm_status st, const std::string& msg) {
  if (ctx) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->err = msg;
  }
  return st;
}

cm_status hip_fail(cm_context* ctx, hipError_t e, const char* where) {
  return fail(ctx, CM_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

namespace {


#define CM_HIP(ctx, call)                                  \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

bool valid_params(const cm_params& p, std::string* why) {
  const float pos[] = {p.tau_cap, p.tau_cup, p.tau_st, p.tau_clip, p.tau_blend, p.eps_t, p.eps_n};
  for (float v : pos)
    if (!(v > 0.f) || !std::isfinite(v)) { *why = "temperatures, eps_t and eps_n must be positive"; return false; }
  if (!(p.d_max >= 0.f)) { *why = "d_max must be >= 0"; return false; }
  if (p.st_iters < 0 || p.st_iters > 64) { *why = "st_iters must be in [0, 64]"; return false; }
  if (p.grid_res < 1 || p.grid_res > 128) { *why = "grid_res must be in [1, 128]"; return false; }
  if (p.curve < 0 || p.curve > 2) { *why = "curve must be 0, 1 or 2"; return false; }
  if (!(p.grid_margin >= 0.f) || !(p.grid_margin_rel >= 0.f)) { *why = "grid margins must be >= 0"; return false; }
  if (p.prune_pieces < 0 || p.prune_pieces > 1) { *why = "prune_pieces must be 0 or 1"; return false; }
  if (p.sdf_kind < 0 || p.sdf_kind > 2) { *why = "sdf_kind must be 0 (planes), 1 (spline) or 2 (primitives)"; return false; }
  if (p.sdf_kind == 2 && (!(p.tau_t > 0.f) || !(p.tau_disc > 0.f) || !std::isfinite(p.tau_t) || !std::isfinite(p.tau_disc))) {
    *why = "tau_t and tau_disc must be positive";
    return false;
  }
  if (p.edge_assign < 0 || p.edge_assign > 1) { *why = "edge_assign must be 0 or 1"; return false; }
  return true;
}

}  // namespace

DevParams make_dev_params(const cm_params& p) {
  DevParams d{};
  d.kcap = float(kLog2eD / p.tau_cap);
  d.icap = float(p.tau_cap / kLog2eD);
  d.kcup = float(kLog2eD / p.tau_cup);
  d.icup = float(p.tau_cup / kLog2eD);
  d.inv_tau_st = 1.f / p.tau_st;
  d.tau_clip = p.tau_clip;
  d.inv_tau_clip = 1.f / p.tau_clip;
  d.inv_tau_blend = 1.f / p.tau_blend;
  d.tau_blend = p.tau_blend;
  d.d_max = p.d_max;
  d.inv_eps_t = 1.f / p.eps_t;
  d.eps_n2 = p.eps_n * p.eps_n;
  d.st_iters = p.st_iters;
  d.broad_phase = p.broad_phase;
  d.edge_bound = p.edge_bound;
  d.prune = p.prune_pieces;
  d.prune_margin = kPruneTau * p.tau_cup;
  d.tau_t = p.tau_t;
  d.inv_tau_t = p.tau_t > 0.f ? 1.f / p.tau_t : 0.f;
  d.tau_disc = p.tau_disc;
  d.inv_tau_disc = p.tau_disc > 0.f ? 1.f / p.tau_disc : 0.f;
  return d;
}

Arena::~Arena() {
  for (auto& c : chunks_)
    if (c.base) (void)hipFree(c.base);
}

void* Arena::alloc(size_t bytes, int* chunk_id) {
  bytes = align_up(bytes, 256);
  for (size_t i = 0; i < chunks_.size(); ++i) {
    Chunk& c = chunks_[i];
    if (c.base && c.size - c.used >= bytes) {
      void* p = c.base + c.used;
      c.used += bytes;
      c.live++;
      in_use_ += bytes;
      *chunk_id = int(i);
      return p;
    }
  }
  Chunk c;
  c.size = std::max(chunk_, bytes);
  if (hipMalloc(&c.base, c.size) != hipSuccess) return nullptr;
  c.used = bytes;
  c.live = 1;
  in_use_ += bytes;
  // reuse an empty slot
  for (size_t i = 0; i < chunks_.size(); ++i)
    if (!chunks_[i].base) { chunks_[i] = c; *chunk_id = int(i); return c.base; }
  chunks_.push_back(c);
  *chunk_id = int(chunks_.size() - 1);
  return c.base;
}

void Arena::release(int chunk_id) {
  Chunk& c = chunks_[size_t(chunk_id)];
  if (--c.live == 0) {
    in_use_ -= c.used;
    (void)hipFree(c.base);
    c = Chunk{};
  }
}

// Host packing of one object: device layout and descriptor offsets.
struct Packed {
  std::vector<char> bytes;
  size_t off_planes, off_sub, off_pieces, off_vx, off_vy, off_vz, off_edges, off_grid;
  size_t off_coef;  // spline coefficients (spline objects)
  int32_t K, P, V, E;
  float gorg[3], gh[3], ginv[3], gr;
  double gorg64[3], gh64[3];  // the grid box in FP64 (the spline fit's corners)
  int32_t gn;
  int32_t rep;
};

// Order of a piece's planes in which each run of kGrp consecutive planes has
// nearby normals: recursive halving of the normal set along the coordinate of
// largest spread, the first half a whole number of groups, so that only the
// piece's last group can be partial.
static void group_order(const std::vector<double>& planes, std::vector<int32_t>& idx, size_t b, size_t e) {
  const size_t n = e - b;
  if (n <= size_t(kGrp)) return;
  double lo[3] = {2, 2, 2}, hi[3] = {-2, -2, -2};
  for (size_t i = b; i < e; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], planes[4 * size_t(idx[i]) + size_t(a)]);
      hi[a] = std::max(hi[a], planes[4 * size_t(idx[i]) + size_t(a)]);
    }
  int ax = 0;
  for (int a = 1; a < 3; ++a)
    if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
  const size_t half = size_t(kGrp) * (((n + size_t(kGrp) - 1) / size_t(kGrp)) / 2);
  std::nth_element(idx.begin() + std::ptrdiff_t(b), idx.begin() + std::ptrdiff_t(b + half),
                   idx.begin() + std::ptrdiff_t(e), [&](int32_t u, int32_t v) {
                     const double pu = planes[4 * size_t(u) + size_t(ax)], pv = planes[4 * size_t(v) + size_t(ax)];
                     return pu < pv || (pu == pv && u < v);
                   });
  group_order(planes, idx, b, b + half);
  group_order(planes, idx, b + half, e);
}

// Cone record of the scaled planes q[0 .. n-1] of one group: axis a, the
// largest offset e, and the cone's half-angle (at most 90 degrees) as (cos,
// kappa cos, kappa sin), rounded outwards, so that for every plane of the group
// kappa n.v + kappa h <= kappa (cos (a.v) + sin |v|) + e.
static void group_cone(const std::vector<double>& planes, const int32_t* idx, size_t n, double kap,
                       const double* hl, F4* rec) {
  double a[3] = {0, 0, 0};
  for (size_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) a[c] += planes[4 * size_t(idx[i]) + size_t(c)];
  double an = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  if (!(an > 1e-12)) {  // normals that cancel: the whole sphere
    a[0] = 1; a[1] = 0; a[2] = 0; an = 1;
  }
  for (int c = 0; c < 3; ++c) a[c] /= an;
  double cmin = 1, emax = -1e300;
  for (size_t i = 0; i < n; ++i) {
    const double* q = &planes[4 * size_t(idx[i])];
    cmin = std::min(cmin, a[0] * q[0] + a[1] * q[1] + a[2] * q[2]);
    emax = std::max(emax, kap * hl[i]);
  }
  cmin = std::max(0.0, cmin - 1e-6);  // (a half-angle above 90 degrees counts as 90: the bound still holds)
  const double smax = std::min(1.0, std::sqrt(std::max(0.0, 1 - cmin * cmin)) + 1e-6);
  rec[0] = F4{float(a[0]), float(a[1]), float(a[2]), float(emax + 1e-6 * std::fabs(emax) + 1e-6)};
  rec[1] = F4{float(cmin), float(kap * cmin), float(kap * smax), 0.f};
}

static void pack_object(const ObjHost& o, const cm_params& prm, Packed* pk) {
  const double kap = kLog2eD / double(prm.tau_cap);
  pk->K = int32_t(o.pieces.size());
  // every piece's planes fill whole groups of kGrp: the last group is padded
  // with inert planes (n = 0, h = -1e30: value -1e30, weight 0, never the max)
  size_t n_grp = 0;  // plane groups of all pieces
  for (const PieceGeom& g : o.pieces) n_grp += (g.n_planes() + size_t(kGrp) - 1) / size_t(kGrp);
  pk->P = int32_t(n_grp * size_t(kGrp));
  pk->V = int32_t(o.n_verts);
  pk->E = int32_t(o.n_edges);
  const int gn = prm.grid_res;
  size_t off = 0;
  auto take = [&](size_t b) { size_t r = off; off = align_up(off + b, 256); return r; };
  pk->off_planes = take(16 * size_t(pk->P));
  pk->off_sub = take(16 * size_t(kSub) * size_t(pk->K) + 32 * n_grp);
  pk->off_pieces = take(sizeof(PieceDesc) * size_t(pk->K));
  pk->off_vx = take(4 * size_t(pk->V));
  pk->off_vy = take(4 * size_t(pk->V));
  pk->off_vz = take(4 * size_t(pk->V));
  pk->off_edges = take(8 * size_t(pk->E));
  pk->off_grid = take(4 * size_t(gn) * gn * gn);
  pk->rep = prm.sdf_kind == 1 ? kRepSpline : (prm.sdf_kind == 2 ? kRepPrims : kRepPlanes);
  pk->off_coef = pk->rep == kRepSpline ? take(16 * size_t(gn + 3) * (gn + 3) * (gn + 3)) : 0;
  pk->bytes.assign(off, 0);
  F4* planes = reinterpret_cast<F4*>(pk->bytes.data() + pk->off_planes);
  F4* sub = reinterpret_cast<F4*>(pk->bytes.data() + pk->off_sub);
  PieceDesc* pieces = reinterpret_cast<PieceDesc*>(pk->bytes.data() + pk->off_pieces);
  float* vx = reinterpret_cast<float*>(pk->bytes.data() + pk->off_vx);
  float* vy = reinterpret_cast<float*>(pk->bytes.data() + pk->off_vy);
  float* vz = reinterpret_cast<float*>(pk->bytes.data() + pk->off_vz);
  I2* edges = reinterpret_cast<I2*>(pk->bytes.data() + pk->off_edges);
  F4* grp = sub + size_t(kSub) * size_t(pk->K);
  int32_t pb = 0, vb = 0, eb = 0, gb = 0;
  std::vector<int32_t> vbase(size_t(pk->K) + 1, 0);  // object-level first vertex of each piece
  for (int32_t k = 0; k < pk->K; ++k) vbase[size_t(k) + 1] = vbase[size_t(k)] + int32_t(o.pieces[size_t(k)].n_verts());
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int32_t k = 0; k < pk->K; ++k) {
    const PieceGeom& g = o.pieces[size_t(k)];
    const double* c = &o.centres[3 * size_t(k)];
    PieceDesc& d = pieces[k];
    d = PieceDesc{};
    d.cx = float(c[0]); d.cy = float(c[1]); d.cz = float(c[2]);
    d.plane_begin = pb; d.plane_count = int32_t(g.n_planes());
    d.vert_begin = vb; d.vert_count = int32_t(g.n_verts());
    const std::vector<int32_t>& xe = o.xedges[size_t(k)];
    d.edge_begin = eb; d.edge_count = int32_t(g.n_edges() + xe.size() / 2);
    // the centre as stored in FP32 is the one the kernels subtract
    const double cf[3] = {double(d.cx), double(d.cy), double(d.cz)};
    double rin = 1e300;
    // planes in groups of kGrp with nearby normals, each with its cone record
    std::vector<int32_t> idx(g.n_planes());
    for (size_t j = 0; j < idx.size(); ++j) idx[j] = int32_t(j);
    group_order(g.planes, idx, 0, idx.size());
    std::vector<double> hls(idx.size());
    for (size_t j = 0; j < idx.size(); ++j) {
      const double* q = &g.planes[4 * size_t(idx[j])];
      const double hl = q[3] + q[0] * cf[0] + q[1] * cf[1] + q[2] * cf[2];
      planes[pb + int32_t(j)] = F4{float(kap * q[0]), float(kap * q[1]), float(kap * q[2]), float(kap * hl)};
      hls[j] = hl;
      rin = std::min(rin, -hl);
    }
    d.grp_begin = gb;
    for (size_t j = 0; j < idx.size(); j += size_t(kGrp), ++gb) {
      const size_t n = std::min(size_t(kGrp), idx.size() - j);
      group_cone(g.planes, &idx[j], n, kap, &hls[j], grp + 2 * size_t(gb));
    }
    const size_t padded = size_t(kGrp) * ((idx.size() + size_t(kGrp) - 1) / size_t(kGrp));
    for (size_t j = idx.size(); j < padded; ++j) planes[pb + int32_t(j)] = F4{0.f, 0.f, 0.f, -1e30f};
    // upper bound of the piece SDF: phi_k(x) <= |x - c| - rin + tau_cap ln P
    d.ub_off = float(double(prm.tau_cap) * std::log(double(g.n_planes())) - rin);
    // support subset: farthest-point sampling of the normals; the max plane
    // value over any subset is a lower bound of the piece's SDF
    {
      const size_t P = g.n_planes();
      std::vector<double> best(P, -2.0);
      size_t j = 0;
      for (int m = 0; m < kSub && m < int(P); ++m) {
        const double* a = &g.planes[4 * j];
        const double hl = a[3] + a[0] * cf[0] + a[1] * cf[1] + a[2] * cf[2];
        sub[size_t(kSub) * size_t(k) + size_t(m)] =
            F4{float(kap * a[0]), float(kap * a[1]), float(kap * a[2]), float(kap * hl)};
        size_t nxt = 0;
        double lo = 3.0;
        for (size_t i = 0; i < P; ++i) {
          const double* b = &g.planes[4 * i];
          best[i] = std::max(best[i], a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
          if (best[i] < lo) { lo = best[i]; nxt = i; }
        }
        j = nxt;
      }
      // a piece of fewer planes repeats its first one (the max is unchanged)
      for (int m = int(std::min<size_t>(P, size_t(kSub))); m < kSub && P > 0; ++m)
        sub[size_t(kSub) * size_t(k) + size_t(m)] = sub[size_t(kSub) * size_t(k)];
    }
    for (size_t i = 0; i < g.n_verts(); ++i) {
      vx[vb + int32_t(i)] = float(g.verts[3 * i]);
      vy[vb + int32_t(i)] = float(g.verts[3 * i + 1]);
      vz[vb + int32_t(i)] = float(g.verts[3 * i + 2]);
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], g.verts[3 * i + size_t(a)]);
        hi[a] = std::max(hi[a], g.verts[3 * i + size_t(a)]);
      }
    }
    for (size_t e = 0; e < g.n_edges(); ++e)
      edges[eb + int32_t(e)] = I2{vb + g.edges[2 * e], vb + g.edges[2 * e + 1]};
    // crossing edges of other pieces (Sec. IV-D.1), after the piece's own
    for (size_t x = 0; x < xe.size() / 2; ++x) {
      const PieceGeom& gk = o.pieces[size_t(xe[2 * x])];
      const size_t e = size_t(xe[2 * x + 1]);
      const int32_t vk = vbase[size_t(xe[2 * x])];
      edges[eb + int32_t(g.n_edges() + x)] = I2{vk + gk.edges[2 * e], vk + gk.edges[2 * e + 1]};
    }
    pb += int32_t(kGrp) * ((d.plane_count + int32_t(kGrp) - 1) / int32_t(kGrp));
    vb += d.vert_count; eb += d.edge_count;
  }
  // voxel grid over the vertex AABB grown by margin + margin_rel * radius
  const double margin = double(prm.grid_margin) + double(prm.grid_margin_rel) * o.radius;
  double r2 = 0;
  for (int a = 0; a < 3; ++a) {
    const double org = lo[a] - margin;
    const double h = (hi[a] - lo[a] + 2 * margin) / gn;
    pk->gorg[a] = float(org);
    pk->gh[a] = float(h);
    pk->gorg64[a] = org;
    pk->gh64[a] = h;
    pk->ginv[a] = float(1.0 / h);
    r2 += h * h;
  }
  pk->gr = float(0.5 * std::sqrt(r2));
  pk->gn = gn;
}

static ObjDesc make_desc(const Packed& pk, char* base) {
  ObjDesc d{};
  d.planes = reinterpret_cast<const F4*>(base + pk.off_planes);
  d.sub = reinterpret_cast<const F4*>(base + pk.off_sub);
  d.pieces = reinterpret_cast<const PieceDesc*>(base + pk.off_pieces);
  d.vx = reinterpret_cast<const float*>(base + pk.off_vx);
  d.vy = reinterpret_cast<const float*>(base + pk.off_vy);
  d.vz = reinterpret_cast<const float*>(base + pk.off_vz);
  d.edges = reinterpret_cast<const I2*>(base + pk.off_edges);
  d.grid = reinterpret_cast<const float*>(base + pk.off_grid);
  d.n_pieces = pk.K; d.n_planes = pk.P; d.n_verts = pk.V; d.n_edges = pk.E;
  for (int a = 0; a < 3; ++a) { d.gorg[a] = pk.gorg[a]; d.gh[a] = pk.gh[a]; d.ginv[a] = pk.ginv[a]; }
  d.gr = pk.gr;
  d.gn = pk.gn;
  d.rep = pk.rep;
  if (pk.rep == kRepSpline) d.sub = reinterpret_cast<const F4*>(base + pk.off_coef);
  if (pk.rep == kRepPrims) { d.sub = nullptr; d.gn = 0; }  // until cm_object_set_prims
  return d;
}

// Edge assignment (Sec. IV-D.1): an edge belongs to every convex piece it
// intersects.  Besides its own piece, edge e of piece k joins piece j when the
// segment, clipped by j's half-spaces (parameter interval [t_in, t_out] of
// a + t (b - a)), keeps a part longer than 1e-9 of the object's scale.
static void cross_edges(ObjHost& o) {
  double scale = 1e-300;
  for (const PieceGeom& g : o.pieces)
    for (double v : g.verts) scale = std::max(scale, std::fabs(v));
  const double tol = 1e-9 * scale;
  o.xedges.assign(o.pieces.size(), {});
  for (size_t j = 0; j < o.pieces.size(); ++j) {
    const PieceGeom& pj = o.pieces[j];
    for (size_t k = 0; k < o.pieces.size(); ++k) {
      if (k == j) continue;
      const PieceGeom& pk = o.pieces[k];
      for (size_t e = 0; e < pk.n_edges(); ++e) {
        const double* a = &pk.verts[3 * size_t(pk.edges[2 * e])];
        const double* b = &pk.verts[3 * size_t(pk.edges[2 * e + 1])];
        double t_in = 0.0, t_out = 1.0;
        bool miss = false;
        for (size_t i = 0; i < pj.n_planes() && !miss; ++i) {
          const double* q = &pj.planes[4 * i];
          const double fa = q[0] * a[0] + q[1] * a[1] + q[2] * a[2] + q[3];
          const double fb = q[0] * b[0] + q[1] * b[1] + q[2] * b[2] + q[3];
          if (fa > 0 && fb > 0) miss = true;
          else if (fa > 0) t_in = std::max(t_in, fa / (fa - fb));
          else if (fb > 0) t_out = std::min(t_out, fa / (fa - fb));
        }
        if (miss) continue;
        const double L = std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) +
                                   (b[2] - a[2]) * (b[2] - a[2]));
        if ((t_out - t_in) * L > tol) {
          o.xedges[j].push_back(int32_t(k));
          o.xedges[j].push_back(int32_t(e));
        }
      }
    }
  }
}

// Fills the derived host data of an object whose pieces are set.
static void finish_host(ObjHost& o, bool assign_crossing) {
  if (assign_crossing) cross_edges(o);
  else o.xedges.assign(o.pieces.size(), {});
  o.n_planes = o.n_verts = o.n_edges = o.n_words = 0;
  o.radius = 0;
  o.centres.assign(3 * o.pieces.size(), 0.0);
  o.counts.assign(2 * o.pieces.size(), 0);
  for (size_t k = 0; k < o.pieces.size(); ++k) {
    const PieceGeom& g = o.pieces[k];
    const int32_t nx = int32_t(o.xedges[k].size() / 2);
    o.counts[2 * k] = int32_t(g.n_verts());
    o.counts[2 * k + 1] = int32_t(g.n_edges()) + nx;
    o.n_planes += int64_t(g.n_planes());
    o.n_verts += int64_t(g.n_verts());
    o.n_edges += int64_t(g.n_edges()) + nx;
    o.n_words += (o.counts[2 * k] + kWave - 1) / kWave + (o.counts[2 * k + 1] + kWave - 1) / kWave;
    double c[3] = {0, 0, 0};
    for (size_t i = 0; i < g.n_verts(); ++i) {
      for (int a = 0; a < 3; ++a) c[a] += g.verts[3 * i + size_t(a)];
      o.radius = std::max(o.radius, std::sqrt(g.verts[3 * i] * g.verts[3 * i] + g.verts[3 * i + 1] * g.verts[3 * i + 1] +
                                              g.verts[3 * i + 2] * g.verts[3 * i + 2]));
    }
    for (int a = 0; a < 3; ++a) o.centres[3 * k + size_t(a)] = g.n_verts() ? c[a] / double(g.n_verts()) : 0.0;
  }
}

// Spline fits of freshly registered objects (Sec. III-B), on the device in
// chunks: their FP64 collision geometry (planes, feature edges as segments) is
// uploaded to scratch, the fit writes the coefficients and cell bounds into each
// object's memory, and the scratch is freed.
static cm_status fit_splines(cm_context* ctx, const std::vector<Packed>& packs, const std::vector<int32_t>& ids) {
  const int n = ctx->prm.grid_res, m = n + 3;
  const int64_t stride = 4 * int64_t(m) * m * m;
  const size_t chunk = 64;
  for (size_t c0 = 0; c0 < ids.size(); c0 += chunk) {
    const size_t cn = std::min(chunk, ids.size() - c0);
    std::vector<double> planes, segs;
    std::vector<int32_t> pieces;  // int4 per piece
    std::vector<size_t> pl_off(cn), pc_off(cn), sg_off(cn);
    for (size_t i = 0; i < cn; ++i) {
      const ObjHost& o = ctx->objs[size_t(ids[c0 + i])];
      pl_off[i] = planes.size();
      pc_off[i] = pieces.size();
      sg_off[i] = segs.size();
      int32_t pb = 0, eb = 0;
      for (const PieceGeom& g : o.pieces) {
        planes.insert(planes.end(), g.planes.begin(), g.planes.end());
        for (size_t e = 0; e < g.n_edges(); ++e)
          for (int k = 0; k < 2; ++k)
            for (int a = 0; a < 3; ++a) segs.push_back(g.verts[3 * size_t(g.edges[2 * e + size_t(k)]) + size_t(a)]);
        pieces.insert(pieces.end(), {pb, int32_t(g.n_planes()), eb, int32_t(g.n_edges())});
        pb += int32_t(g.n_planes());
        eb += int32_t(g.n_edges());
      }
    }
    const size_t b_pl = align_up(8 * planes.size(), 256), b_sg = align_up(8 * segs.size(), 256);
    const size_t b_pc = align_up(4 * pieces.size(), 256), b_job = align_up(sizeof(SplJob) * cn, 256);
    const size_t b_work = 8 * size_t(stride) * cn;
    char* d = nullptr;
    if (hipMalloc(&d, b_pl + b_sg + b_pc + b_job + 2 * b_work) != hipSuccess)
      return fail(ctx, CM_E_OOM, "spline fit scratch allocation failed");
    double* d_pl = reinterpret_cast<double*>(d);
    double* d_sg = reinterpret_cast<double*>(d + b_pl);
    int32_t* d_pc = reinterpret_cast<int32_t*>(d + b_pl + b_sg);
    SplJob* d_job = reinterpret_cast<SplJob*>(d + b_pl + b_sg + b_pc);
    double* wa = reinterpret_cast<double*>(d + b_pl + b_sg + b_pc + b_job);
    double* wb = wa + stride * int64_t(cn);
    std::vector<SplJob> jobs(cn);
    for (size_t i = 0; i < cn; ++i) {
      const ObjHost& o = ctx->objs[size_t(ids[c0 + i])];
      const Packed& pk = packs[c0 + i];
      SplJob& j = jobs[i];
      j.planes = d_pl + pl_off[i];
      j.pieces = reinterpret_cast<const int4*>(d_pc + pc_off[i]);
      j.segs = d_sg + sg_off[i];
      j.n_pieces = int32_t(o.pieces.size());
      j.pad = 0;
      for (int a = 0; a < 3; ++a) { j.org[a] = pk.gorg64[a]; j.h[a] = pk.gh64[a]; }
      j.coef = const_cast<F4*>(o.desc.sub);
      j.grid = const_cast<float*>(o.desc.grid);
    }
    hipError_t e = hipMemcpyAsync(d_pl, planes.data(), 8 * planes.size(), hipMemcpyHostToDevice, ctx->build_stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_sg, segs.data(), 8 * segs.size(), hipMemcpyHostToDevice, ctx->build_stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_pc, pieces.data(), 4 * pieces.size(), hipMemcpyHostToDevice, ctx->build_stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_job, jobs.data(), sizeof(SplJob) * cn, hipMemcpyHostToDevice, ctx->build_stream);
    if (e == hipSuccess) e = launch_spline_build(d_job, int(cn), n, wa, wb, stride, ctx->build_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->build_stream);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(ctx, e, "spline fit");
  }
  return CM_OK;
}

// Uploads host-built objects, refreshes the device table and builds their grids.
static cm_status register_objects(cm_context* ctx, std::vector<ObjHost>& built, cm_object* out) {
  const size_t n = built.size();
  std::vector<Packed> packs(n);
  {
    const int nt = int(std::min<size_t>(n, std::max(1u, std::min(16u, std::thread::hardware_concurrency()))));
    std::vector<std::thread> th;
    std::atomic<size_t> next{0};
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&]() {
        for (size_t i = next++; i < n; i = next++) pack_object(built[i], ctx->prm, &packs[i]);
      });
    for (auto& t : th) t.join();
  }
  if (ctx->device < 0) {
    std::unique_lock<std::shared_mutex> lk(ctx->reg_mu);
    for (size_t i = 0; i < n; ++i) {
      built[i].alive = true;
      out[i] = cm_object(ctx->objs.size());
      ctx->objs.push_back(std::move(built[i]));
    }
    return CM_OK;
  }
  std::vector<int32_t> ids(n);
  {
    std::unique_lock<std::shared_mutex> lk(ctx->reg_mu);
    for (size_t i = 0; i < n; ++i) {
      ObjHost& o = built[i];
      o.dmem = ctx->arena->alloc(packs[i].bytes.size(), &o.chunk);
      if (!o.dmem) {
        for (size_t k = 0; k < i; ++k) ctx->arena->release(built[k].chunk);
        return fail(ctx, CM_E_OOM, "device allocation of object geometry failed");
      }
      o.desc = make_desc(packs[i], static_cast<char*>(o.dmem));
      o.alive = true;
    }
    for (size_t i = 0; i < n; ++i) {
      hipError_t e = hipMemcpyAsync(built[i].dmem, packs[i].bytes.data(), packs[i].bytes.size(),
                                    hipMemcpyHostToDevice, ctx->build_stream);
      if (e != hipSuccess) return hip_fail(ctx, e, "object upload");
    }
    for (size_t i = 0; i < n; ++i) {
      ids[i] = int32_t(ctx->objs.size());
      out[i] = cm_object(ids[i]);
      ctx->objs.push_back(std::move(built[i]));
    }
    // device table
    const size_t need = ctx->objs.size();
    if (need > ctx->d_objs_cap) {
      size_t cap = std::max<size_t>(need, 2 * ctx->d_objs_cap + 64);
      ObjDesc* nd = nullptr;
      if (hipMalloc(&nd, cap * sizeof(ObjDesc)) != hipSuccess) return fail(ctx, CM_E_OOM, "object table allocation failed");
      // the old table is kept until shutdown: kernels in flight, captured
      // graphs and a serving batch being launched may still hold its address
      // (its descriptors stay valid for the objects it lists)
      if (ctx->d_objs) ctx->old_tables.push_back(ctx->d_objs);
      ctx->d_objs = nd;
      ctx->d_objs_cap = cap;
      std::vector<ObjDesc> all(need);
      for (size_t i = 0; i < need; ++i) all[i] = ctx->objs[i].desc;
      hipError_t e = hipMemcpyAsync(ctx->d_objs, all.data(), need * sizeof(ObjDesc), hipMemcpyHostToDevice,
                                    ctx->build_stream);
      if (e != hipSuccess) return hip_fail(ctx, e, "object table upload");
      (void)hipStreamSynchronize(ctx->build_stream);
    } else {
      std::vector<ObjDesc> fresh(n);
      for (size_t i = 0; i < n; ++i) fresh[i] = ctx->objs[size_t(ids[i])].desc;
      hipError_t e = hipMemcpyAsync(ctx->d_objs + ids[0], fresh.data(), n * sizeof(ObjDesc), hipMemcpyHostToDevice,
                                    ctx->build_stream);
      if (e != hipSuccess) return hip_fail(ctx, e, "object table upload");
      (void)hipStreamSynchronize(ctx->build_stream);
    }
  }
  // voxel grids (Sec. IV-C.2), one launch for the batch
  int32_t* d_ids = nullptr;
  CM_HIP(ctx, hipMalloc(&d_ids, n * sizeof(int32_t)));
  CM_HIP(ctx, hipMemcpyAsync(d_ids, ids.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, ctx->build_stream));
  const size_t per_launch = 4096;
  for (size_t i = 0; i < n; i += per_launch) {
    const int32_t cnt = int32_t(std::min(per_launch, n - i));
    hipError_t e = launch_grid_build(ctx->d_objs, d_ids + i, cnt, ctx->prm.grid_res, ctx->dp, ctx->build_stream);
    if (e != hipSuccess) { (void)hipFree(d_ids); return hip_fail(ctx, e, "grid build"); }
  }
  hipError_t e = hipStreamSynchronize(ctx->build_stream);
  (void)hipFree(d_ids);
  if (e != hipSuccess) return hip_fail(ctx, e, "grid build");
  if (ctx->prm.sdf_kind == 1) return fit_splines(ctx, packs, ids);
  return CM_OK;
}

ObjHost* get_obj(cm_context* ctx, cm_object h) {
  if (h >= ctx->objs.size() || !ctx->objs[h].alive) return nullptr;
  return &ctx->objs[h];
}

}  // namespace cm

using namespace cm;

extern "C" {

cm_status cm_default_params(float L_ref, cm_params* out) {
  if (!out || !(L_ref > 0.f)) return CM_E_INVALID;
  cm_params p{};
  p.tau_cap = p.tau_cup = p.tau_st = p.tau_clip = 0.01f * L_ref;
  p.tau_blend = 0.02f * L_ref;
  p.d_max = 0.05f * L_ref;
  p.eps_t = 0.025f * L_ref;
  p.eps_n = 1e-6f;
  p.grid_margin = 0.1f * L_ref;
  p.grid_margin_rel = 1.0f;
  p.st_iters = 3;
  p.grid_res = 32;
  p.curve = 2;
  p.broad_phase = 1;
  p.edge_bound = 0;
  p.prune_pieces = 1;
  p.tau_t = 0.01f;
  p.tau_disc = 1e-3f;
  *out = p;
  return CM_OK;
}

cm_status cm_init(int32_t device, const cm_params* params, size_t mem_budget_bytes, cm_context** out) {
  if (!out || !params) return CM_E_INVALID;
  *out = nullptr;
  std::string why;
  if (!valid_params(*params, &why)) return CM_E_INVALID;
  auto* ctx = new cm_context;
  ctx->device = device;
  ctx->prm = *params;
  ctx->dp = make_dev_params(*params);
  ctx->budget = mem_budget_bytes ? mem_budget_bytes : (size_t(32) << 30);
  if (device >= 0) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device >= n) { delete ctx; return CM_E_INVALID; }
    if (hipSetDevice(device) != hipSuccess) { delete ctx; return CM_E_HIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete ctx; return CM_E_HIP; }
    ctx->n_cu = prop.multiProcessorCount;
    warm_narrow_occupancy();
    // device address of the fixed launch scratch of cm_contacts_fwd_noalloc
    if (static_scratch_setup(device) != hipSuccess) { delete ctx; return CM_E_HIP; }
    if (hipStreamCreateWithFlags(&ctx->build_stream, hipStreamNonBlocking) != hipSuccess) { delete ctx; return CM_E_HIP; }
    ctx->arena.reset(new Arena(size_t(256) << 20));
  }
  *out = ctx;
  return CM_OK;
}

const char* cm_last_error(cm_context* ctx) {
  if (!ctx) return "null context";
  std::lock_guard<std::mutex> lk(ctx->mu);
  return ctx->err.c_str();
}

cm_status cm_build_objects(cm_context* ctx, int32_t n_objects, const int64_t* obj_off, const int64_t* piece_off,
                           const double* xyz, cm_object* out) {
  if (!ctx || n_objects < 0 || !obj_off || !piece_off || !xyz || !out) return fail(ctx, CM_E_INVALID, "null argument");
  if (n_objects == 0) return CM_OK;
  for (int32_t i = 0; i < n_objects; ++i) {
    const int64_t k0 = obj_off[i], k1 = obj_off[i + 1];
    if (k1 <= k0 || k1 - k0 > kMaxPieces) return fail(ctx, CM_E_INVALID, "object needs 1..4096 pieces");
    for (int64_t k = k0; k < k1; ++k)
      if (piece_off[k + 1] - piece_off[k] < 4) return fail(ctx, CM_E_DEGENERATE, "a piece has fewer than 4 points");
  }
  std::vector<ObjHost> built(static_cast<size_t>(n_objects));
  std::atomic<int> status{0};
  {
    const int nt = std::max(1, std::min<int>(n_objects, int(std::min(16u, std::max(1u, std::thread::hardware_concurrency())))));
    std::vector<std::thread> th;
    std::atomic<int32_t> next{0};
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&]() {
        for (int32_t i = next++; i < n_objects; i = next++) {
          ObjHost& o = built[size_t(i)];
          const int64_t k0 = obj_off[i], k1 = obj_off[i + 1];
          o.pieces.resize(size_t(k1 - k0));
          for (int64_t k = k0; k < k1; ++k) {
            PieceGeom& g = o.pieces[size_t(k - k0)];
            int st = build_hull_piece(xyz + 3 * piece_off[k], piece_off[k + 1] - piece_off[k], &g);
            if (st != 0) { status = st; break; }
            serialize_piece(&g, ctx->prm.curve);
          }
          finish_host(o, ctx->prm.edge_assign != 0);
        }
      });
    for (auto& t : th) t.join();
  }
  if (status != 0) return fail(ctx, CM_E_DEGENERATE, "a piece has fewer than 4 non-coplanar points");
  return register_objects(ctx, built, out);
}

cm_status cm_build_pieces(cm_context* ctx, int32_t n_pieces, const int64_t* offsets, const double* xyz, cm_object* out) {
  if (!ctx || n_pieces <= 0 || !offsets) return fail(ctx, CM_E_INVALID, "bad arguments");
  const int64_t oo[2] = {0, n_pieces};
  return cm_build_objects(ctx, 1, oo, offsets, xyz, out);
}

cm_status cm_build_pieces_raw(cm_context* ctx, int32_t n_pieces, const int64_t* plane_off, const double* planes,
                              const int64_t* vert_off, const double* verts, const int64_t* edge_off,
                              const int32_t* edges, cm_object* out) {
  if (!ctx || n_pieces <= 0 || n_pieces > kMaxPieces || !plane_off || !planes || !vert_off || !verts || !edge_off ||
      !out)
    return fail(ctx, CM_E_INVALID, "bad arguments");
  std::vector<ObjHost> built(1);
  ObjHost& o = built[0];
  o.pieces.resize(size_t(n_pieces));
  for (int32_t k = 0; k < n_pieces; ++k) {
    PieceGeom& g = o.pieces[size_t(k)];
    const int64_t P = plane_off[k + 1] - plane_off[k], V = vert_off[k + 1] - vert_off[k],
                  E = edge_off[k + 1] - edge_off[k];
    if (P < 1 || V < 1 || E < 0) return fail(ctx, CM_E_INVALID, "each piece needs >= 1 plane and >= 1 vertex");
    for (int64_t j = 0; j < P; ++j) {
      const double* q = planes + 4 * (plane_off[k] + j);
      const double l = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
      if (!(l > 0)) return fail(ctx, CM_E_INVALID, "zero plane normal");
      g.planes.insert(g.planes.end(), {q[0] / l, q[1] / l, q[2] / l, q[3] / l});
    }
    g.verts.assign(verts + 3 * vert_off[k], verts + 3 * vert_off[k + 1]);
    for (int64_t e = 0; e < E; ++e) {
      const int32_t a = edges[2 * (edge_off[k] + e)], b = edges[2 * (edge_off[k] + e) + 1];
      if (a < 0 || b < 0 || a >= V || b >= V || a == b) return fail(ctx, CM_E_INVALID, "edge index out of range");
      g.edges.push_back(std::min(a, b));
      g.edges.push_back(std::max(a, b));
    }
    serialize_piece(&g, ctx->prm.curve);
  }
  finish_host(o, ctx->prm.edge_assign != 0);
  return register_objects(ctx, built, out);
}

cm_status cm_release_object(cm_context* ctx, cm_object obj) {
  if (!ctx) return CM_E_INVALID;
  std::unique_lock<std::shared_mutex> lk(ctx->reg_mu);
  ObjHost* o = get_obj(ctx, obj);
  if (!o) return fail(ctx, CM_E_NOTFOUND, "unknown object");
  if (o->dmem) {
    (void)hipDeviceSynchronize();
    ctx->arena->release(o->chunk);
  }
  if (o->dprims) (void)hipFree(o->dprims);
  *o = ObjHost{};
  return CM_OK;
}

cm_status cm_object_info(cm_context* ctx, cm_object obj, int32_t* n_pieces, int64_t* n_planes, int64_t* n_verts,
                         int64_t* n_edges) {
  if (!ctx) return CM_E_INVALID;
  std::shared_lock<std::shared_mutex> lk(ctx->reg_mu);
  ObjHost* o = get_obj(ctx, obj);
  if (!o) return fail(ctx, CM_E_NOTFOUND, "unknown object");
  if (n_pieces) *n_pieces = int32_t(o->pieces.size());
  if (n_planes) *n_planes = o->n_planes;
  if (n_verts) *n_verts = o->n_verts;
  if (n_edges) *n_edges = o->n_edges;
  return CM_OK;
}

cm_status cm_object_export(cm_context* ctx, cm_object obj, int64_t* plane_off, double* planes, int64_t* vert_off,
                           double* verts, int64_t* edge_off, int32_t* edges) {
  if (!ctx) return CM_E_INVALID;
  std::shared_lock<std::shared_mutex> lk(ctx->reg_mu);
  ObjHost* o = get_obj(ctx, obj);
  if (!o) return fail(ctx, CM_E_NOTFOUND, "unknown object");
  int64_t pb = 0, vb = 0, eb = 0;
  for (size_t k = 0; k < o->pieces.size(); ++k) {
    const PieceGeom& g = o->pieces[k];
    if (plane_off) plane_off[k] = pb;
    if (vert_off) vert_off[k] = vb;
    if (edge_off) edge_off[k] = eb;
    if (planes) std::copy(g.planes.begin(), g.planes.end(), planes + 4 * pb);
    if (verts) std::copy(g.verts.begin(), g.verts.end(), verts + 3 * vb);
    if (edges) std::copy(g.edges.begin(), g.edges.end(), edges + 2 * eb);
    pb += int64_t(g.n_planes()); vb += int64_t(g.n_verts()); eb += int64_t(g.n_edges());
  }
  const size_t K = o->pieces.size();
  if (plane_off) plane_off[K] = pb;
  if (vert_off) vert_off[K] = vb;
  if (edge_off) edge_off[K] = eb;
  return CM_OK;
}

cm_status cm_object_spline(cm_context* ctx, cm_object obj, float* coef, float* meta) {
  if (!ctx || !meta) return fail(ctx, CM_E_INVALID, "null argument");
  ObjHost* o;
  {
    std::shared_lock<std::shared_mutex> lk(ctx->reg_mu);
    o = get_obj(ctx, obj);
    if (!o) return fail(ctx, CM_E_NOTFOUND, "unknown object");
  }
  if (ctx->prm.sdf_kind != 1 || ctx->device < 0) return fail(ctx, CM_E_INVALID, "not a spline object on a device");
  const int n = o->desc.gn;
  meta[0] = float(n);
  for (int a = 0; a < 3; ++a) { meta[1 + a] = o->desc.gorg[a]; meta[4 + a] = o->desc.gh[a]; }
  if (coef) {
    const size_t m = size_t(n) + 3;
    CM_HIP(ctx, hipMemcpy(coef, o->desc.sub, 16 * m * m * m, hipMemcpyDeviceToHost));
  }
  return CM_OK;
}

cm_status cm_object_set_prims(cm_context* ctx, cm_object obj, int32_t n, const double* rec, const int64_t* plane_off,
                              const double* planes) {
  if (!ctx || n <= 0 || n > kMaxPieces || !rec || !plane_off || (plane_off[n] > 0 && !planes))
    return fail(ctx, CM_E_INVALID, "bad arguments");
  if (ctx->prm.sdf_kind != 2 || ctx->device < 0) return fail(ctx, CM_E_INVALID, "not a primitive context on a device");
  if (plane_off[0] != 0) return fail(ctx, CM_E_INVALID, "plane_off[0] must be 0");
  std::vector<PrimDev> pd(static_cast<size_t>(n));
  for (int32_t i = 0; i < n; ++i) {
    const double* r = rec + 32 * i;
    PrimDev& q = pd[size_t(i)];
    q = PrimDev{};
    q.kind = int32_t(r[0]);
    q.op = int32_t(r[1]);
    if ((q.kind != 0 && q.kind != 1) || q.op < 0 || q.op > 2 || plane_off[i + 1] < plane_off[i])
      return fail(ctx, CM_E_INVALID, "primitive kind must be 0 or 1, op 0..2, plane offsets ascending");
    q.plane_begin = int32_t(plane_off[i]);
    q.plane_count = int32_t(plane_off[i + 1] - plane_off[i]);
    for (int k = 0; k < 3; ++k) {
      q.c[k] = float(r[2 + k]); q.p2[k] = float(r[5 + k]); q.p3[k] = float(r[8 + k]);
      q.a0[k] = float(r[15 + k]); q.a1[k] = float(r[20 + k]);
      if (!(r[15 + k] > 0.0) || !(r[20 + k] > 0.0)) return fail(ctx, CM_E_INVALID, "superquadric scales must be positive");
    }
    q.e0a = float(r[18]); q.e0b = float(r[19]); q.e1a = float(r[23]); q.e1b = float(r[24]);
    if (!(r[18] > 0.0) || !(r[19] > 0.0) || !(r[23] > 0.0) || !(r[24] > 0.0))
      return fail(ctx, CM_E_INVALID, "superquadric exponents must be positive");
    // PSQ rotation from its quaternion, in FP64, rounded once
    const double qn = std::sqrt(r[11] * r[11] + r[12] * r[12] + r[13] * r[13] + r[14] * r[14]);
    if (!(qn > 1e-12)) return fail(ctx, CM_E_INVALID, "degenerate quaternion");
    const double w = r[11] / qn, x = r[12] / qn, y = r[13] / qn, z = r[14] / qn;
    const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                         2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                         2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) q.Rt[3 * a + b] = float(R[3 * b + a]);
    if (q.kind == 1) {  // XPSQ spline constants in FP64
      double A[3], B[3];
      for (int k = 0; k < 3; ++k) { A[k] = r[2 + k] - 2 * r[5 + k] + r[8 + k]; B[k] = 2 * (r[5 + k] - r[2 + k]); }
      const double AA = A[0] * A[0] + A[1] * A[1] + A[2] * A[2], AB = A[0] * B[0] + A[1] * B[1] + A[2] * B[2];
      const double bn[3] = {B[1] * A[2] - B[2] * A[1], B[2] * A[0] - B[0] * A[2], B[0] * A[1] - B[1] * A[0]};
      const double bl = std::sqrt(bn[0] * bn[0] + bn[1] * bn[1] + bn[2] * bn[2]);
      const double BBd = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
      if (!(bl > 1e-9 * std::max(AA, BBd))) return fail(ctx, CM_E_INVALID, "an XPSQ spline must be curved (p2 off the line p1 p3)");
      q.a2 = float(1.5 * AB / AA);
      q.inv2AA = float(1.0 / (2.0 * AA));
      q.BB = float(BBd);
      for (int k = 0; k < 3; ++k) { q.A[k] = float(A[k]); q.B[k] = float(B[k]); q.bn[k] = float(bn[k] / bl); }
    }
  }
  const int64_t P = plane_off[n];
  std::vector<F4> pl(static_cast<size_t>(P));
  for (int64_t j = 0; j < P; ++j) {
    const double* v = planes + 4 * j;
    const double l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (!(l > 0)) return fail(ctx, CM_E_INVALID, "zero plane normal");
    pl[size_t(j)] = F4{float(v[0] / l), float(v[1] / l), float(v[2] / l), float(v[3] / l)};
  }
  const size_t bytes = sizeof(PrimDev) * size_t(n) + sizeof(F4) * size_t(P);
  void* mem = nullptr;
  CM_HIP(ctx, hipMalloc(&mem, bytes));
  hipError_t e = hipMemcpy(mem, pd.data(), sizeof(PrimDev) * size_t(n), hipMemcpyHostToDevice);
  if (e == hipSuccess && P)
    e = hipMemcpy(static_cast<char*>(mem) + sizeof(PrimDev) * size_t(n), pl.data(), sizeof(F4) * size_t(P),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) { (void)hipFree(mem); return hip_fail(ctx, e, "primitive upload"); }
  std::unique_lock<std::shared_mutex> lk(ctx->reg_mu);
  ObjHost* o = get_obj(ctx, obj);
  if (!o) { (void)hipFree(mem); return fail(ctx, CM_E_NOTFOUND, "unknown object"); }
  (void)hipDeviceSynchronize();  // (kernels in flight may read the old block)
  if (o->dprims) (void)hipFree(o->dprims);
  o->dprims = mem;
  o->n_prims = n;
  o->desc.sub = static_cast<const F4*>(mem);
  o->desc.gn = n;
  e = hipMemcpy(ctx->d_objs + obj, &o->desc, sizeof(ObjDesc), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "object table update");
  return CM_OK;
}

cm_status cm_object_grid(cm_context* ctx, cm_object obj, float* G, float* meta) {
  if (!ctx) return CM_E_INVALID;
  ObjDesc d;
  {
    std::shared_lock<std::shared_mutex> lk(ctx->reg_mu);
    ObjHost* o = get_obj(ctx, obj);
    if (!o) return fail(ctx, CM_E_NOTFOUND, "unknown object");
    if (ctx->device < 0) return fail(ctx, CM_E_INVALID, "host-only context has no grid");
    if (ctx->prm.sdf_kind == 2) return fail(ctx, CM_E_INVALID, "primitive objects have no voxel grid");
    d = o->desc;
  }
  if (meta) {
    for (int a = 0; a < 3; ++a) { meta[a] = d.gorg[a]; meta[3 + a] = d.gh[a]; }
    meta[6] = d.gr;
    meta[7] = float(d.gn);
  }
  if (G) CM_HIP(ctx, hipMemcpy(G, d.grid, sizeof(float) * size_t(d.gn) * d.gn * d.gn, hipMemcpyDeviceToHost));
  return CM_OK;
}

// ------------------------------------------------------------------ plans --
}  // extern "C"

namespace cm {

// Terms of one SDF evaluation against an object: its planes, or the 64
// coefficients of a spline evaluation.
static double sdf_terms(const cm_context* ctx, const ObjHost& o) {
  if (ctx->prm.sdf_kind == 2) return 64.0 * double(std::max(o.n_prims, 1));  // (a jet evaluation per primitive)
  return ctx->prm.sdf_kind == 1 ? 64.0 : double(o.n_planes);
}

// Sizes of the plan of a batch, from the objects' counts alone (no tables).
cm_status plan_sizes(cm_context* ctx, const cm_query* hq, int32_t n, PlanSizes* z) {
  *z = PlanSizes{};
  z->n = n;
  {
    std::shared_lock<std::shared_mutex> lk(ctx->reg_mu);
    for (int32_t i = 0; i < n; ++i) {
      const ObjHost* A = get_obj(ctx, hq[i].a);
      const ObjHost* B = get_obj(ctx, hq[i].b);
      if (!A || !B) return fail(ctx, CM_E_NOTFOUND, "query names an unknown object");
      z->G += int64_t(A->pieces.size() + B->pieces.size());
      z->C += A->n_verts + A->n_edges + B->n_verts + B->n_edges;
      z->W += A->n_words + B->n_words;
    }
  }
  z->E = 2 * z->G;
  z->R = 4 * int64_t(n);
  z->nb = (std::max(z->E, z->R) + 1023) / 1024;
  return CM_OK;
}

// Host tables of a plan (entries sorted by estimated cost, group -> entries)
// and the size of its device scratch.  Reads the object registry under a
// shared lock: batches are planned concurrently.
cm_status plan_host(cm_context* ctx, const cm_query* hq, int32_t n, cm_plan* pl, size_t* dev_bytes) {
  pl->ctx = ctx;
  pl->n = n;
  pl->W = 0;
  pl->group_off.assign(size_t(n) + 1, 0);
  pl->contact_off.assign(size_t(n) + 1, 0);
  pl->qa.resize(size_t(n));
  pl->qb.resize(size_t(n));
  // scratch kept across calls on this thread: planning a batch of tens of
  // thousands of queries touches tens of MB, and fresh allocations would take
  // a page fault on every page again (the serving thread plans every batch)
  thread_local std::vector<Entry> gen;  // entries in generation order
  thread_local std::vector<double> cost, rcost;
  thread_local std::vector<int64_t> rstart, rmem, rorder, fill;
  gen.clear();
  cost.clear();
  const int K2 = 2 * ctx->prm.st_iters + 1;
  {
    std::shared_lock<std::shared_mutex> lk(ctx->reg_mu);
    size_t n_ent = 0;  // 2 entries (vertices, edges) per piece of either side
    for (int32_t i = 0; i < n; ++i) {
      const ObjHost* A = get_obj(ctx, hq[i].a);
      const ObjHost* B = get_obj(ctx, hq[i].b);
      if (A && B) n_ent += 2 * (A->pieces.size() + B->pieces.size());
    }
    gen.reserve(n_ent);
    cost.reserve(n_ent);
    for (int32_t i = 0; i < n; ++i) {
      const ObjHost* A = get_obj(ctx, hq[i].a);
      const ObjHost* B = get_obj(ctx, hq[i].b);
      if (!A || !B) return fail(ctx, CM_E_NOTFOUND, "query names an unknown object");
      if (ctx->prm.sdf_kind == 2 && (A->n_prims <= 0 || B->n_prims <= 0))
        return fail(ctx, CM_E_INVALID, "an object of a primitive context has no primitives (cm_object_set_prims)");
      pl->qa[size_t(i)] = int32_t(hq[i].a);
      pl->qb[size_t(i)] = int32_t(hq[i].b);
      const int64_t ga = int64_t(A->pieces.size()), gb = int64_t(B->pieces.size());
      pl->group_off[size_t(i) + 1] = pl->group_off[size_t(i)] + ga + gb;
      pl->contact_off[size_t(i) + 1] =
          pl->contact_off[size_t(i)] + A->n_verts + A->n_edges + B->n_verts + B->n_edges;
      int64_t cbase = pl->contact_off[size_t(i)];
      for (int dir = 0; dir < 2; ++dir) {
        const ObjHost* Mo = dir ? B : A;
        const ObjHost* So = dir ? A : B;
        const size_t Km = Mo->pieces.size();
        const int32_t* cnt = Mo->counts.data();
        for (size_t k = 0; k < Km; ++k) {
          const int64_t group = pl->group_off[size_t(i)] + (dir ? ga : 0) + int64_t(k);
          for (int kind = 0; kind < 2; ++kind) {
            Entry e{};
            e.query = i;
            e.group = int32_t(group);
            e.piece = int32_t(k);
            e.count = cnt[2 * k + size_t(kind)];
            e.word_off = pl->W;
            e.contact_base = cbase;
            e.dir = dir;
            e.kind = kind;
            e.mesh_obj = int32_t(dir ? hq[i].b : hq[i].a);
            e.sdf_obj = int32_t(dir ? hq[i].a : hq[i].b);
            pl->W += (e.count + kWave - 1) / kWave;
            cbase += e.count;
            gen.push_back(e);
            cost.push_back(double(e.count) * sdf_terms(ctx, *So) * (kind ? K2 : 1));
          }
        }
      }
    }
  }
  pl->G = pl->group_off[size_t(n)];
  pl->C = pl->contact_off[size_t(n)];
  if (pl->G >= (int64_t(1) << 31)) return fail(ctx, CM_E_INVALID, "too many groups");
  // runs: the entries of one (query, direction, kind), i.e. every piece of the
  // mesh side, whose survivors share tiles; costliest runs first, so their tiles
  // head the work queue, pieces in order within a run
  const int64_t R = 4 * int64_t(n);
  const size_t E0 = gen.size();
  rcost.assign(static_cast<size_t>(R), 0.0);
  // members of each run by a counting pass (in generation order within a run)
  rstart.assign(static_cast<size_t>(R) + 1, 0);
  rmem.resize(E0);
  auto run_of = [](const Entry& e) { return 4 * int64_t(e.query) + 2 * e.dir + e.kind; };
  for (size_t i = 0; i < E0; ++i) {
    const int64_t r = run_of(gen[i]);
    rcost[size_t(r)] += cost[i];
    rstart[size_t(r) + 1]++;
  }
  for (int64_t r = 0; r < R; ++r) rstart[size_t(r) + 1] += rstart[size_t(r)];
  fill.assign(rstart.begin(), rstart.end() - 1);
  for (size_t i = 0; i < E0; ++i) rmem[size_t(fill[size_t(run_of(gen[i]))]++)] = int64_t(i);
  rorder.resize(static_cast<size_t>(R));
  std::iota(rorder.begin(), rorder.end(), 0);
  std::stable_sort(rorder.begin(), rorder.end(), [&](int64_t a, int64_t b) { return rcost[size_t(a)] > rcost[size_t(b)]; });
  pl->ents.resize(E0);
  pl->run_off.assign(size_t(R) + 1, 0);
  pl->q_runs.assign(size_t(R), 0);
  pl->ent_run.assign(E0, 0);
  pl->gent.assign(size_t(pl->G), I2{0, 0});
  size_t pos = 0;
  for (int64_t k = 0; k < R; ++k) {
    const int64_t r = rorder[size_t(k)];
    pl->q_runs[size_t(r)] = int32_t(k);
    for (int64_t m = rstart[size_t(r)]; m < rstart[size_t(r) + 1]; ++m, ++pos) {
      const Entry& e = gen[size_t(rmem[size_t(m)])];
      I2& ge = pl->gent[size_t(e.group)];
      if (e.kind == 0) ge.x = int32_t(pos); else ge.y = int32_t(pos);
      pl->ents[pos] = e;
      pl->ent_run[pos] = int32_t(k);
    }
    pl->run_off[size_t(k) + 1] = int64_t(pos);
  }
  // keep the scratch for batches of the serving size only (a plan of millions
  // of entries would otherwise hold hundreds of MB on this thread until exit)
  if (gen.capacity() > (size_t(1) << 21)) {
    std::vector<Entry>().swap(gen);
    std::vector<double>().swap(cost);
    std::vector<double>().swap(rcost);
    std::vector<int64_t>().swap(rstart);
    std::vector<int64_t>().swap(rmem);
    std::vector<int64_t>().swap(rorder);
    std::vector<int64_t>().swap(fill);
  }
  pl->E = int64_t(pl->ents.size());
  pl->R = R;
  pl->nb = (std::max(pl->E, pl->R) + 1023) / 1024;
  *dev_bytes = plan_layout(pl, nullptr);
  return CM_OK;
}

PlanSizes layout_sizes(const cm_plan* pl) {
  if (pl->reserved) return pl->cap;
  PlanSizes z;
  z.n = pl->n; z.G = pl->G; z.C = pl->C; z.E = pl->E; z.W = pl->W; z.nb = pl->nb; z.R = pl->R;
  return z;
}

// Carves the plan's device scratch out of `base` (nullptr: only sizes it),
// for the batch's sizes or, reserved, for the capacity.
size_t plan_layout(cm_plan* pl, char* b) {
  const PlanSizes z = layout_sizes(pl);
  const int64_t W = std::max<int64_t>(z.W, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t r = off; off = align_up(off + bytes, 256); return r; };
  const size_t o_ents = take(sizeof(Entry) * size_t(z.E));
  const size_t o_gent = take(sizeof(I2) * size_t(z.G));
  const size_t o_bits = take(8 * size_t(W));
  const size_t o_nsurv = take(4 * size_t(z.E));
  const size_t o_wpre = take(4 * size_t(W));
  const size_t o_soff = take(8 * size_t(z.E + 1));
  const size_t o_roff = take(8 * size_t(z.R + 1));
  const size_t o_erun = take(4 * size_t(z.E));
  const size_t o_qrun = take(4 * size_t(z.R));
  const size_t o_ntr = take(4 * size_t(z.R));
  const size_t o_npart = take(4 * size_t(z.E));
  const size_t o_poff = take(8 * size_t(z.E + 1));
  const size_t o_filt = take(16 * size_t(z.E));
  const size_t o_toff = take(8 * size_t(z.R + 1));
  const size_t o_bsum = take(8 * size_t(z.nb + 1));
  const size_t o_cnt = take(256);
  // blend partials: one per (entry, tile its survivors reach): at most W + E
  const size_t o_part = take(4 * size_t(kStride) * size_t(W + z.E));
  const size_t o_gs = take(4 * size_t(kGStride) * size_t(z.G));
  const size_t o_bp = take(4 * size_t(kStride) * size_t(W));
  const size_t o_goff = take(8 * size_t(z.n + 1));
  const size_t o_gt = take(4 * 12 * size_t(z.n));
  // the adjoint tape (dual values), for a quarter of the bitmask words as tiles
  // plus the partly filled last tile of each run: the broad phase leaves far
  // fewer tiles than words (a few per cent of the contacts survive), and sizing
  // for every word would make each request reserve ten times the memory it
  // uses; at most a quarter of the memory budget.  Tiles past the tape are
  // recomputed by the adjoint.
  const int st = pl->ctx->prm.st_iters;
  const int64_t tape_slot_bytes = int64_t(std::max(pl->tape_kind, 1) * 4 * tape_values(st));
  const int64_t budget_tiles = int64_t(pl->ctx->budget / 4) / (tape_slot_bytes * kWave);
  const int64_t want_tiles = std::min<int64_t>(W, W / 4 + z.R);
  // (spline SDFs keep no tape: an evaluation is 64 gathers, cheap to repeat)
  pl->tape_tiles = (st <= kMaxTraceAdj && pl->tape_kind > 0 && pl->ctx->prm.sdf_kind == 0)
                       ? std::min<int64_t>(want_tiles, budget_tiles) : 0;
  const size_t o_tape = take(size_t(tape_slot_bytes) * kWave * size_t(pl->tape_tiles));
  if (b) {
    pl->d_ents = reinterpret_cast<Entry*>(b + o_ents);
    pl->d_gent = reinterpret_cast<I2*>(b + o_gent);
    pl->d_bits = reinterpret_cast<uint64_t*>(b + o_bits);
    pl->d_nsurv = reinterpret_cast<int32_t*>(b + o_nsurv);
    pl->d_wpre = reinterpret_cast<int32_t*>(b + o_wpre);
    pl->d_surv_off = reinterpret_cast<int64_t*>(b + o_soff);
    pl->d_run_off = reinterpret_cast<int64_t*>(b + o_roff);
    pl->d_ent_run = reinterpret_cast<int32_t*>(b + o_erun);
    pl->d_q_runs = reinterpret_cast<int32_t*>(b + o_qrun);
    pl->d_ntr = reinterpret_cast<int32_t*>(b + o_ntr);
    pl->d_npart = reinterpret_cast<int32_t*>(b + o_npart);
    pl->d_part_off = reinterpret_cast<int64_t*>(b + o_poff);
    pl->d_filt = reinterpret_cast<F4*>(b + o_filt);
    pl->d_tile_off = reinterpret_cast<int64_t*>(b + o_toff);
    pl->d_bsum = reinterpret_cast<int64_t*>(b + o_bsum);
    pl->d_counter = reinterpret_cast<uint32_t*>(b + o_cnt);  // [kQueues]
    pl->d_work = reinterpret_cast<unsigned long long*>(b + o_cnt + 32);
    pl->d_dc = reinterpret_cast<DevCounts*>(b + o_cnt + 64);
    static_assert(4 * kQueues <= 32, "queue counters overlap the work counters");
    pl->d_partials = reinterpret_cast<float*>(b + o_part);
    pl->d_gscratch = reinterpret_cast<float*>(b + o_gs);
    pl->d_bpartials = reinterpret_cast<float*>(b + o_bp);
    pl->d_group_off = reinterpret_cast<int64_t*>(b + o_goff);
    pl->d_gradtmp = reinterpret_cast<float*>(b + o_gt);
    pl->d_tape = pl->tape_tiles ? reinterpret_cast<float*>(b + o_tape) : nullptr;
  }
  return off;
}

// Binds device scratch and uploads the plan's tables (asynchronously on `s`
// when given; the host tables live in the plan until it is destroyed).
cm_status plan_bind(cm_plan* pl, void* dmem, hipStream_t s) {
  plan_layout(pl, static_cast<char*>(dmem));
  pl->h_dc = DevCounts{};
  pl->h_dc.E = pl->E;
  pl->h_dc.R = pl->R;
  pl->h_dc.G = pl->G;
  pl->h_dc.n = pl->n;
  {
    std::shared_lock<std::shared_mutex> lk(pl->ctx->reg_mu);  // the table may be replaced by a concurrent build
    pl->h_dc.objs = pl->ctx->d_objs;
  }
  if (hipMemcpyAsync(pl->d_dc, &pl->h_dc, sizeof(DevCounts), hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(pl->ctx, CM_E_HIP, "plan upload failed");
  // (an empty batch of a reserved plan uploads its counts and offsets only)
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  hipError_t e1 = up(pl->d_ents, pl->ents.data(), sizeof(Entry) * size_t(pl->E));
  hipError_t e2 = up(pl->d_gent, pl->gent.data(), sizeof(I2) * size_t(pl->G));
  hipError_t e3 = up(pl->d_group_off, pl->group_off.data(), 8 * size_t(pl->n + 1));
  hipError_t e4 = pl->R ? up(pl->d_run_off, pl->run_off.data(), 8 * size_t(pl->R + 1)) : hipSuccess;
  hipError_t e5 = up(pl->d_ent_run, pl->ent_run.data(), 4 * size_t(pl->E));
  hipError_t e6 = up(pl->d_q_runs, pl->q_runs.data(), 4 * size_t(pl->R));
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess || e5 != hipSuccess ||
      e6 != hipSuccess)
    return fail(pl->ctx, CM_E_HIP, "plan upload failed");
  return CM_OK;
}

}  // namespace cm

extern "C" {

cm_status cm_plan_create(cm_context* ctx, const cm_query* hq, int32_t n, cm_plan** out) {
  if (!ctx || !out || n <= 0 || !hq) return fail(ctx, CM_E_INVALID, "bad arguments");
  *out = nullptr;
  if (ctx->device < 0) return fail(ctx, CM_E_INVALID, "host-only context cannot run queries");
  auto* pl = new cm_plan;
  size_t bytes = 0;
  cm_status st = plan_host(ctx, hq, n, pl, &bytes);
  if (st != CM_OK) { delete pl; return st; }
  if (hipMalloc(&pl->dmem, bytes) != hipSuccess) { delete pl; return fail(ctx, CM_E_OOM, "plan scratch allocation failed"); }
  pl->owns_mem = true;
  st = plan_bind(pl, pl->dmem, nullptr);
  if (st == CM_OK && hipDeviceSynchronize() != hipSuccess) st = fail(ctx, CM_E_HIP, "plan upload failed");
  if (st != CM_OK) {
    (void)hipFree(pl->dmem);
    delete pl;
    return st;
  }
  *out = pl;
  return CM_OK;
}

cm_status cm_plan_reserve(cm_context* ctx, int32_t max_queries, int64_t max_groups, int64_t max_contacts,
                          cm_plan** out) {
  if (!ctx || !out || max_queries <= 0 || max_groups <= 0 || max_contacts < 0)
    return fail(ctx, CM_E_INVALID, "bad arguments");
  *out = nullptr;
  if (ctx->device < 0) return fail(ctx, CM_E_INVALID, "host-only context cannot run queries");
  if (max_groups > (int64_t(1) << 30) || max_contacts > (int64_t(1) << 40))
    return fail(ctx, CM_E_INVALID, "capacity beyond the entry index range");
  auto* pl = new cm_plan;
  pl->ctx = ctx;
  pl->reserved = true;
  PlanSizes& c = pl->cap;
  c.n = max_queries;
  c.G = max_groups;
  c.C = max_contacts;
  c.E = 2 * max_groups;                     // a vertex and an edge entry per group
  c.R = 4 * int64_t(max_queries);           // (direction, kind) runs per query
  c.W = (max_contacts + kWave - 1) / kWave + c.E;  // an entry's words: at most count / 64 + 1
  c.nb = (std::max(c.E, c.R) + 1023) / 1024;
  pl->group_off.assign(1, 0);  // the empty batch
  pl->contact_off.assign(1, 0);
  const size_t bytes = plan_layout(pl, nullptr);
  if (hipMalloc(&pl->dmem, bytes) != hipSuccess) { delete pl; return fail(ctx, CM_E_OOM, "plan allocation failed"); }
  pl->owns_mem = true;
  cm_status st = plan_bind(pl, pl->dmem, nullptr);  // an empty batch
  if (st == CM_OK && (hipDeviceSynchronize() != hipSuccess || hipEventCreateWithFlags(&pl->uploaded, hipEventDisableTiming) != hipSuccess))
    st = fail(ctx, CM_E_HIP, "plan set-up failed");
  if (st != CM_OK) {
    (void)hipFree(pl->dmem);
    delete pl;
    return st;
  }
  *out = pl;
  return CM_OK;
}

cm_status cm_plan_refill(cm_context* ctx, cm_plan* pl, const cm_query* hq, int32_t n, void* stream) {
  if (!ctx || !pl || pl->ctx != ctx || n < 0 || (n > 0 && !hq)) return fail(ctx, CM_E_INVALID, "bad arguments");
  if (!pl->reserved) return fail(ctx, CM_E_INVALID, "cm_plan_refill needs a plan made by cm_plan_reserve");
  // the previous refill's uploads read the host tables about to be replaced
  if (hipEventSynchronize(pl->uploaded) != hipSuccess) return fail(ctx, CM_E_HIP, "waiting for the last refill");
  cm_plan tmp;
  tmp.tape_kind = pl->tape_kind;
  if (n > 0) {
    size_t bytes = 0;
    const cm_status st = plan_host(ctx, hq, n, &tmp, &bytes);
    if (st != CM_OK) return st;
  } else {
    tmp.ctx = ctx;
    tmp.group_off.assign(1, 0);
    tmp.contact_off.assign(1, 0);
  }
  const PlanSizes& c = pl->cap;
  if (tmp.n > c.n || tmp.G > c.G || tmp.C > c.C)
    return fail(ctx, CM_E_INVALID,
                "batch of " + std::to_string(tmp.n) + " queries, " + std::to_string(tmp.G) + " groups, " +
                    std::to_string(tmp.C) + " contacts exceeds the plan's capacity (" + std::to_string(c.n) + ", " +
                    std::to_string(c.G) + ", " + std::to_string(c.C) + ")");
  pl->n = tmp.n; pl->G = tmp.G; pl->C = tmp.C; pl->E = tmp.E; pl->W = tmp.W; pl->R = tmp.R; pl->nb = tmp.nb;
  pl->group_off.swap(tmp.group_off);
  pl->contact_off.swap(tmp.contact_off);
  pl->ents.swap(tmp.ents);
  pl->run_off.swap(tmp.run_off);
  pl->ent_run.swap(tmp.ent_run);
  pl->q_runs.swap(tmp.q_runs);
  pl->gent.swap(tmp.gent);
  pl->qa.swap(tmp.qa);
  pl->qb.swap(tmp.qb);
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const cm_status st = plan_bind(pl, pl->dmem, s);
  if (st != CM_OK) return st;
  if (hipEventRecord(pl->uploaded, s) != hipSuccess) return fail(ctx, CM_E_HIP, "refill event");
  return CM_OK;
}

cm_status cm_plan_capacity(const cm_plan* pl, int32_t* max_queries, int64_t* max_groups, int64_t* max_contacts) {
  if (!pl) return CM_E_INVALID;
  const PlanSizes z = layout_sizes(pl);
  if (max_queries) *max_queries = z.n;
  if (max_groups) *max_groups = z.G;
  if (max_contacts) *max_contacts = z.C;
  return CM_OK;
}

cm_status cm_plan_destroy(cm_plan* pl) {
  if (!pl) return CM_E_INVALID;
  if (pl->dmem && pl->owns_mem) {
    (void)hipDeviceSynchronize();
    (void)hipFree(pl->dmem);
  }
  if (pl->uploaded) (void)hipEventDestroy(pl->uploaded);
  for (auto& e : pl->ev)
    if (e) (void)hipEventDestroy(e);
  delete pl;
  return CM_OK;
}

cm_status cm_plan_set_timing(cm_plan* pl, int32_t enable) {
  if (!pl) return CM_E_INVALID;
  if (enable && !pl->ev[0])
    for (auto& e : pl->ev)
      if (hipEventCreate(&e) != hipSuccess) return fail(pl->ctx, CM_E_HIP, "hipEventCreate failed");
  pl->timing = enable != 0;
  return CM_OK;
}

cm_status cm_plan_timing(const cm_plan* pl, float* ms) {
  if (!pl || !ms) return CM_E_INVALID;
  for (int k = 0; k < kTimed; ++k) {
    ms[k] = -1.f;
    if (!pl->ev[0] || !(pl->timed_mask & (1u << k))) continue;
    float t = 0.f;
    if (hipEventSynchronize(pl->ev[2 * k + 1]) == hipSuccess &&
        hipEventElapsedTime(&t, pl->ev[2 * k], pl->ev[2 * k + 1]) == hipSuccess)
      ms[k] = t;
  }
  // slots the last pass did not record fail their query; that must not be
  // reported by the next launch
  (void)hipGetLastError();
  return CM_OK;
}

cm_status cm_plan_info(const cm_plan* pl, int64_t* n_groups, int64_t* n_contacts, int32_t* n_queries) {
  if (!pl) return CM_E_INVALID;
  if (n_groups) *n_groups = pl->G;
  if (n_contacts) *n_contacts = pl->C;
  if (n_queries) *n_queries = pl->n;
  return CM_OK;
}

cm_status cm_plan_offsets(const cm_plan* pl, int64_t* group_off, int64_t* contact_off) {
  if (!pl) return CM_E_INVALID;
  if (group_off) std::copy(pl->group_off.begin(), pl->group_off.end(), group_off);
  if (contact_off) std::copy(pl->contact_off.begin(), pl->contact_off.end(), contact_off);
  return CM_OK;
}

cm_status cm_plan_work(const cm_plan* pl, int64_t* performed) {
  if (!pl || !performed) return CM_E_INVALID;
  unsigned long long w[2] = {0, 0};
  CM_HIP(pl->ctx, hipDeviceSynchronize());
  CM_HIP(pl->ctx, hipMemcpy(w, pl->d_work, 16, hipMemcpyDeviceToHost));
  performed[0] = int64_t(w[0]);
  performed[1] = int64_t(w[1]);
  return CM_OK;
}

cm_status cm_plan_stats(const cm_plan* pl, int64_t* st) {  // 8 entries
  if (!pl || !st) return CM_E_INVALID;
  std::vector<int32_t> ns(size_t(pl->E));
  CM_HIP(pl->ctx, hipDeviceSynchronize());
  CM_HIP(pl->ctx, hipMemcpy(ns.data(), pl->d_nsurv, 4 * size_t(pl->E), hipMemcpyDeviceToHost));
  int64_t sv = 0, se = 0, tiles = 0, nv = 0, ne = 0;
  double pairs = 0, vpairs = 0, epairs = 0;
  const int K2 = 2 * pl->ctx->prm.st_iters + 1;
  for (int64_t r = 0; r < pl->R; ++r) {
    int64_t s = 0;
    for (int64_t e = pl->run_off[size_t(r)]; e < pl->run_off[size_t(r) + 1]; ++e) s += ns[size_t(e)];
    tiles += (s + kWave - 1) / kWave;
  }
  for (size_t i = 0; i < ns.size(); ++i) {
    const Entry& e = pl->ents[i];
    const double P = sdf_terms(pl->ctx, pl->ctx->objs[size_t(e.sdf_obj)]);
    if (e.kind == 0) { sv += ns[i]; nv += e.count; pairs += double(ns[i]) * P; vpairs += double(ns[i]) * P; }
    else { se += ns[i]; ne += e.count; pairs += double(ns[i]) * P * K2; epairs += double(ns[i]) * P; }
  }
  st[0] = sv; st[1] = se; st[2] = tiles; st[3] = nv; st[4] = ne; st[5] = int64_t(pairs);
  st[6] = int64_t(vpairs); st[7] = int64_t(epairs);
  return CM_OK;
}

}  // extern "C"

namespace cm {
FwdArgs fwd_args(cm_context* ctx, cm_plan* pl, const cm_query* q, const cm_groups& out, float* dbg) {
  FwdArgs a{};
  const PlanSizes z = layout_sizes(pl);  // grids and record strides: the capacity
  a.dc = pl->d_dc;
  a.ents = pl->d_ents;
  a.n_ent = z.E;
  a.Q = reinterpret_cast<const QueryDev*>(q);
  {
    std::shared_lock<std::shared_mutex> lk(ctx->reg_mu);  // the table may be replaced by a concurrent build
    a.objs = ctx->d_objs;
  }
  a.P = ctx->dp;
  a.bits = pl->d_bits;
  a.nsurv = pl->d_nsurv;
  a.wpre = pl->d_wpre;
  a.surv_off = pl->d_surv_off;
  a.run_off = pl->d_run_off;
  a.ent_run = pl->d_ent_run;
  a.q_runs = pl->d_q_runs;
  a.ntr = pl->d_ntr;
  a.npart = pl->d_npart;
  a.part_off = pl->d_part_off;
  a.n_run = z.R;
  a.filt = pl->d_filt;
  a.bsum = pl->d_bsum;
  a.tile_off = pl->d_tile_off;
  a.counter = pl->d_counter;
  a.partials = pl->d_partials;
  a.gent = pl->d_gent;
  a.G = z.G;
  a.out = OutPtrs{out.p, out.n, out.d, out.q, out.W, out.logZ};
  a.dbg = dbg;
  a.C = pl->C;
  a.n_cu = ctx->n_cu;
  a.blocks_per_cu = pl->blocks_per_cu;
  a.blocks_per_cu_dual = pl->blocks_per_cu_dual;
  a.wg_waves = pl->wg_waves;
  a.wg_waves_dual = pl->wg_waves_dual;
  a.gscratch = pl->d_gscratch;
  a.bpartials = pl->d_bpartials;
  a.group_off = pl->d_group_off;
  a.n = z.n;
  a.ev = pl->timing ? pl->ev : nullptr;
  a.work = pl->d_work;
  a.tape = pl->d_tape;
  a.tape_tiles = pl->d_tape ? pl->tape_tiles : 0;
  a.tape_nv = tape_values(ctx->prm.st_iters);
  a.rep = ctx->prm.sdf_kind == 1 ? kRepSpline : (ctx->prm.sdf_kind == 2 ? kRepPrims : kRepPlanes);
  return a;
}
}  // namespace cm

extern "C" {

cm_status cm_contacts_fwd(cm_context* ctx, cm_plan* pl, const cm_query* q, cm_groups out, float* dbg, void* stream) {
  if (!ctx || !pl || pl->ctx != ctx || !q) return fail(ctx, CM_E_INVALID, "bad arguments");
  if (!out.p || !out.n || !out.d || !out.q || !out.W || !out.logZ) return fail(ctx, CM_E_INVALID, "null output");
  FwdArgs a = fwd_args(ctx, pl, q, out, dbg);
  pl->timed_mask = (1u << kTBroad) | (1u << kTNarrowFwd);
  hipError_t e = launch_forward(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "forward launch");
  return CM_OK;
}

static bool valid_groups(const cm_groups& g) { return g.p && g.n && g.d && g.q && g.W && g.logZ; }

cm_status cm_contacts_bwd(cm_context* ctx, cm_plan* pl, const cm_query* q, cm_groups cot, float* grad, void* stream) {
  if (!ctx || !pl || pl->ctx != ctx || !q || !grad || !valid_groups(cot))
    return fail(ctx, CM_E_INVALID, "bad arguments");
  if (ctx->prm.st_iters > 4) return fail(ctx, CM_E_INVALID, "the adjoint supports st_iters <= 4");
  FwdArgs a = fwd_args(ctx, pl, q, cm_groups{}, nullptr);
  a.cot = OutPtrs{cot.p, cot.n, cot.d, cot.q, cot.W, cot.logZ};
  a.grad = grad;
  a.hv = nullptr;
  a.dir = nullptr;
  pl->timed_mask = (1u << kTBroad) | (1u << kTNarrowFwd) | (1u << kTNarrowAdj);
  hipError_t e = launch_backward(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "backward launch");
  return CM_OK;
}

cm_status cm_hvp(cm_context* ctx, cm_plan* pl, const cm_query* q, cm_groups cot, const float* dir, float* hv,
                 float* grad, void* stream) {
  if (!ctx || !pl || pl->ctx != ctx || !q || !dir || !hv || !valid_groups(cot))
    return fail(ctx, CM_E_INVALID, "bad arguments");
  if (ctx->prm.st_iters > 4) return fail(ctx, CM_E_INVALID, "the adjoint supports st_iters <= 4");
  FwdArgs a = fwd_args(ctx, pl, q, cm_groups{}, nullptr);
  a.cot = OutPtrs{cot.p, cot.n, cot.d, cot.q, cot.W, cot.logZ};
  a.grad = grad ? grad : pl->d_gradtmp;
  a.hv = hv;
  a.dir = dir;
  if (pl->tape_kind < 2) { a.tape = nullptr; a.tape_tiles = 0; }  // a float tape: recompute
  pl->timed_mask = (1u << kTBroad) | (1u << kTNarrowTan) | (1u << kTNarrowDualAdj);
  hipError_t e = launch_hvp(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "hvp launch");
  return CM_OK;
}

cm_status cm_contacts_jvp(cm_context* ctx, cm_plan* pl, const cm_query* q, cm_groups out, cm_groups out_t,
                          const float* dir, void* stream) {
  if (!ctx || !pl || pl->ctx != ctx || !q || !dir || !valid_groups(out) || !valid_groups(out_t))
    return fail(ctx, CM_E_INVALID, "bad arguments");
  FwdArgs a = fwd_args(ctx, pl, q, out, nullptr);
  a.out_t = OutPtrs{out_t.p, out_t.n, out_t.d, out_t.q, out_t.W, out_t.logZ};
  a.dir = dir;
  pl->timed_mask = (1u << kTBroad) | (1u << kTNarrowTan);
  hipError_t e = launch_jvp(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "jvp launch");
  return CM_OK;
}

cm_status cm_project_points(cm_context* ctx, cm_plan* pl, const cm_query* q, const float* p_in, float* p_out,
                            void* stream) {
  if (!ctx || !pl || pl->ctx != ctx || !q || !p_in || !p_out) return fail(ctx, CM_E_INVALID, "bad arguments");
  const ObjDesc* objs;
  {
    std::shared_lock<std::shared_mutex> lk(ctx->reg_mu);
    objs = ctx->d_objs;
  }
  hipError_t e = launch_project(reinterpret_cast<const QueryDev*>(q), objs, pl->d_group_off, pl->n, ctx->dp, p_in,
                                p_out, pl->G, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "projection launch");
  return CM_OK;
}

cm_status cm_contacts_step(cm_context* ctx, cm_plan* pl, const cm_query* q, cm_groups out, cm_groups cot,
                           float* grad, const float* dir, float* hv, void* stream) {
  if (!ctx || !pl || pl->ctx != ctx || !q || !grad || !valid_groups(cot) || (dir != nullptr) != (hv != nullptr))
    return fail(ctx, CM_E_INVALID, "bad arguments");
  const bool records = out.p || out.n || out.d || out.q || out.W || out.logZ;
  if (records && !valid_groups(out)) return fail(ctx, CM_E_INVALID, "partial output records");
  if (ctx->prm.st_iters > 4) return fail(ctx, CM_E_INVALID, "the adjoint supports st_iters <= 4");
  FwdArgs a = fwd_args(ctx, pl, q, out, nullptr);
  a.cot = OutPtrs{cot.p, cot.n, cot.d, cot.q, cot.W, cot.logZ};
  a.grad = grad;
  a.hv = hv;
  a.dir = dir;
  if (dir && pl->tape_kind < 2) { a.tape = nullptr; a.tape_tiles = 0; }  // a float tape: recompute
  hipError_t e;
  if (dir) {
    pl->timed_mask = (1u << kTBroad) | (1u << kTNarrowTan) | (1u << kTNarrowDualAdj);
    e = launch_hvp(a, static_cast<hipStream_t>(stream), records);
  } else {
    pl->timed_mask = (1u << kTBroad) | (1u << kTNarrowFwd) | (1u << kTNarrowAdj);
    e = launch_backward(a, static_cast<hipStream_t>(stream), records);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "step launch");
  return CM_OK;
}

cm_status cm_shutdown(cm_context* ctx) {
  if (!ctx) return CM_E_INVALID;
  serving_stop(ctx);
  if (ctx->device >= 0) (void)hipDeviceSynchronize();
  ctx->arena.reset();
  for (const cm::ObjHost& o : ctx->objs)
    if (o.dprims) (void)hipFree(o.dprims);
  if (ctx->d_objs) (void)hipFree(ctx->d_objs);
  for (cm::ObjDesc* t : ctx->old_tables) (void)hipFree(t);
  if (ctx->build_stream) (void)hipStreamDestroy(ctx->build_stream);
  delete ctx;
  return CM_OK;
}

}  // extern "C"
