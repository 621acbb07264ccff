// FP64 CPU oracle for the differentiable contact-manifold hot path.
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// CPU-baseline leg of the benchmark may load this library.  It shares no code,
// header, table or helper with the HIP path: it is an independent, plain,
// slow and obviously-correct restatement of the paper's definitions.
//
// Paper: Beker, Geist, Paulus, Martius, "Novel Algorithms for Smoothly
// Differentiable and Efficiently Vectorizable Contact Manifold Construction".
//
// Every routine is templated on the scalar type so the same code runs in
// double (values) and in forward-mode dual numbers (exact first and second
// derivatives with respect to the two 6-DoF poses).  Discrete decisions (the
// stabilising shifts of log-sum-exp, voxel indices, broad-phase filtering and
// the branches of the transition function) use the real part only.
//
// Steps (section of the paper in brackets):
//   O2  piece SDF: smooth intersection of facet half-spaces   [Sec. III-A.2/3, eq. smooth-intersection]
//   O3  object SDF: smooth union of its pieces                  [Sec. III-A.2, eq. soft_union]
//       normal n = grad / sqrt(|grad|^2 + eps_n^2)              (reading of the paper, see DESIGN)
//   O4  voxel grid of phi at voxel centres, vertex/edge filter  [Sec. IV-C.2]
//   O5  vertex-SDF contacts                                     [Sec. IV-B]
//   O6  edge-SDF contacts by sphere tracing + softclip          [Sec. IV-B.2, Fig. e_s]
//   O7  mollification with a C2 transition f_t                  [Sec. IV-C.1]
//   O8  softmax blending per convex piece                       [Sec. IV-D.1-3]
//   O9  both directions (SDF and mesh roles swapped)            [Sec. III, first paragraph]
//   O10 derivatives w.r.t. world-frame pose perturbations       (project addition)
//   S1  spline SDF: ground-truth SDF and normal of the pieces at the corners
//       of a voxel grid, cubic-spline coefficients by 1-D solves along each
//       axis, 64-term evaluation, a separate spline for the normal    [Sec. III-B.1/2]
//   S2  voxel lower bounds of a spline SDF (B-spline convex hull)   (reading, see DESIGN)
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <mutex>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

// ---------------------------------------------------------------- scalars --
inline double val(double x) { return x; }

// Forward-mode dual number with N tangent slots; T may itself be a Dual,
// which gives second derivatives (hyper-dual numbers).
template <class T, int N>
struct Dual {
  T v;
  T d[N];
  Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = T(0.0); }
  Dual(double c) : v(c) { for (int i = 0; i < N; ++i) d[i] = T(0.0); }
  explicit Dual(const T& c, int) : v(c) { for (int i = 0; i < N; ++i) d[i] = T(0.0); }
};
template <class T, int N> inline double val(const Dual<T, N>& x) { return val(x.v); }

#define ORC_DUAL template <class T, int N>
ORC_DUAL inline Dual<T, N> operator+(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
ORC_DUAL inline Dual<T, N> operator-(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
ORC_DUAL inline Dual<T, N> operator-(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
ORC_DUAL inline Dual<T, N> operator*(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.v * b.d[i] + a.d[i] * b.v; return r; }
ORC_DUAL inline Dual<T, N> operator/(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; T inv = T(1.0) / b.v; r.v = a.v * inv;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
  return r; }
ORC_DUAL inline Dual<T, N> operator+(const Dual<T, N>& a, double b) { Dual<T, N> r = a; r.v = r.v + b; return r; }
ORC_DUAL inline Dual<T, N> operator+(double b, const Dual<T, N>& a) { return a + b; }
ORC_DUAL inline Dual<T, N> operator-(const Dual<T, N>& a, double b) { Dual<T, N> r = a; r.v = r.v - b; return r; }
ORC_DUAL inline Dual<T, N> operator-(double b, const Dual<T, N>& a) { return (-a) + b; }
ORC_DUAL inline Dual<T, N> operator*(const Dual<T, N>& a, double b) {
  Dual<T, N> r; r.v = a.v * b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r; }
ORC_DUAL inline Dual<T, N> operator*(double b, const Dual<T, N>& a) { return a * b; }
ORC_DUAL inline Dual<T, N> operator/(const Dual<T, N>& a, double b) { return a * (1.0 / b); }
ORC_DUAL inline Dual<T, N> operator/(double a, const Dual<T, N>& b) { return Dual<T, N>(a) / b; }
ORC_DUAL inline Dual<T, N>& operator+=(Dual<T, N>& a, const Dual<T, N>& b) { a = a + b; return a; }
ORC_DUAL inline Dual<T, N>& operator-=(Dual<T, N>& a, const Dual<T, N>& b) { a = a - b; return a; }

using std::exp; using std::log; using std::log1p; using std::sqrt;
// f(x) = f(v) + f'(v) dx
ORC_DUAL inline Dual<T, N> exp(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = exp(a.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * r.v; return r; }
ORC_DUAL inline Dual<T, N> log(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = log(a.v); T inv = T(1.0) / a.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * inv; return r; }
ORC_DUAL inline Dual<T, N> log1p(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = log1p(a.v); T inv = T(1.0) / (a.v + 1.0); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * inv; return r; }
ORC_DUAL inline Dual<T, N> sqrt(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = sqrt(a.v); T inv = T(0.5) / r.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * inv; return r; }
using std::cbrt; using std::cos; using std::sin; using std::atan2;
// cbrt'(v) = 1 / (3 cbrt(v)^2); cos' = -sin; sin' = cos
ORC_DUAL inline Dual<T, N> cbrt(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = cbrt(a.v); T inv = T(1.0) / (r.v * r.v * 3.0); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * inv; return r; }
ORC_DUAL inline Dual<T, N> cos(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = cos(a.v); T m = -sin(a.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * m; return r; }
ORC_DUAL inline Dual<T, N> sin(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = sin(a.v); T m = cos(a.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * m; return r; }
// atan2(y, x): d = (x dy - y dx) / (x^2 + y^2)
ORC_DUAL inline Dual<T, N> atan2(const Dual<T, N>& y, const Dual<T, N>& x) {
  Dual<T, N> r; r.v = atan2(y.v, x.v); T inv = T(1.0) / (x.v * x.v + y.v * y.v);
  for (int i = 0; i < N; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) * inv;
  return r; }
// x^e = exp(e log x) (x > 0)
template <class T, class E> inline T powr(const T& x, const E& e) { return exp(e * log(x)); }

// ----------------------------------------------------------------- vectors --
template <class T> struct V3 { T x, y, z; };
template <class T> inline V3<T> mk(T x, T y, T z) { return V3<T>{x, y, z}; }
template <class T> inline V3<T> operator+(const V3<T>& a, const V3<T>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> inline V3<T> operator-(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T, class S> inline V3<T> operator*(const V3<T>& a, const S& s) { return {a.x * s, a.y * s, a.z * s}; }
template <class T> inline T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> inline V3<T> cvt(const double* p) { return {T(p[0]), T(p[1]), T(p[2])}; }
template <class T> inline V3<double> vval(const V3<T>& a) { return {val(a.x), val(a.y), val(a.z)}; }

// 3x3 matrix, row-major.
template <class T> struct M3 { T m[3][3]; };
template <class T> inline V3<T> mul(const M3<T>& R, const V3<T>& v) {
  return {R.m[0][0] * v.x + R.m[0][1] * v.y + R.m[0][2] * v.z,
          R.m[1][0] * v.x + R.m[1][1] * v.y + R.m[1][2] * v.z,
          R.m[2][0] * v.x + R.m[2][1] * v.y + R.m[2][2] * v.z}; }
template <class T> inline V3<T> mulT(const M3<T>& R, const V3<T>& v) {
  return {R.m[0][0] * v.x + R.m[1][0] * v.y + R.m[2][0] * v.z,
          R.m[0][1] * v.x + R.m[1][1] * v.y + R.m[2][1] * v.z,
          R.m[0][2] * v.x + R.m[1][2] * v.y + R.m[2][2] * v.z}; }
template <class T> inline M3<T> matmul(const M3<T>& A, const M3<T>& B) {
  M3<T> C; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
    T s = A.m[i][0] * B.m[0][j]; s = s + A.m[i][1] * B.m[1][j]; s = s + A.m[i][2] * B.m[2][j]; C.m[i][j] = s; }
  return C; }

// Rotation matrix of a quaternion (w, x, y, z), normalised first.
inline M3<double> quat_to_R(const double* q) {
  double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
  M3<double> R;
  R.m[0][0] = 1 - 2 * (y * y + z * z); R.m[0][1] = 2 * (x * y - w * z);     R.m[0][2] = 2 * (x * z + w * y);
  R.m[1][0] = 2 * (x * y + w * z);     R.m[1][1] = 1 - 2 * (x * x + z * z); R.m[1][2] = 2 * (y * z - w * x);
  R.m[2][0] = 2 * (x * z - w * y);     R.m[2][1] = 2 * (y * z + w * x);     R.m[2][2] = 1 - 2 * (x * x + y * y);
  return R;
}

// ------------------------------------------------------------- parameters --
struct Params {
  double tau_cap, tau_cup, tau_st, tau_clip, tau_blend, d_max, eps_t, eps_n;
  double grid_margin, grid_margin_rel;  // grid = vertex AABB grown by margin + margin_rel * radius
  int32_t st_iters, grid_res, broad_phase, edge_bound;  // edge_bound: 0 paper's min form, 1 tight form
  double jitter;        // FP32 conditioning probe: relative size of the injected perturbations (0: off)
  int32_t jitter_seed;  // its seed
  int32_t pad_;
  // primitive SDFs: temperature of the soft clip of the spline parameter t to
  // (0, 1), and of the softplus / sigmoid of the cubic's discriminant (both
  // dimensionless)
  double tau_t, tau_disc;
};

// ------------------------------------------------ FP32 conditioning probe --
// Not part of the method.  With Params::jitter = 2^-24 it perturbs every
// intermediate an FP32 evaluation has to round (positions in the SDF frame,
// plane values, piece and object phi and gradient, trace iterates, the edge
// point) by an independent uniform amount of that relative size: the value
// relative to the query's scene scale L_s (lengths) or to 1 (unit vectors),
// each derivative component relative to its own magnitude.  Comparing the perturbed result with the unperturbed one measures how
// far rounding alone moves the exact result of this query: its conditioning.
// Draws are a counter-based hash of (seed, query index, call index).
struct Probe {
  double rel = 0, len = 0;
  uint64_t key = 0, ctr = 0;
};
thread_local Probe g_probe;
inline uint64_t mix64(uint64_t z) {  // SplitMix64 finaliser
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline double probe_u() {  // uniform in [-1, 1)
  const uint64_t h = mix64(g_probe.key ^ mix64(g_probe.ctr++));
  return double(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}
// Real part: absolute perturbation of size rel * scale; every derivative
// component: relative to its own magnitude (an FP32 kernel rounds those too).
inline void perturb(double& x, double scale) { x += probe_u() * g_probe.rel * (scale > 0 ? scale : std::abs(x)); }
template <class T, int N> inline void perturb(Dual<T, N>& x, double scale) {
  perturb(x.v, scale);
  for (int i = 0; i < N; ++i) perturb(x.d[i], 0.0);
}
template <class T> inline void probe(T& x, bool length) {
  if (g_probe.rel == 0) return;
  perturb(x, length ? g_probe.len : 1.0);
}
template <class T> inline void probe3(V3<T>& v, bool length) { probe(v.x, length); probe(v.y, length); probe(v.z, length); }

// --------------------------------------------------------------- geometry --
struct Piece {
  std::vector<double> planes;  // 4 per plane: (n_x, n_y, n_z, h); inside where n.x + h <= 0
  std::vector<double> verts;   // 3 per vertex, object frame
  std::vector<int32_t> edges;  // 2 per edge, piece-local vertex indices
  std::vector<double> tris;    // 9 per boundary triangle (only for the spline's ground truth)
  std::vector<double> xedges;  // 6 per edge of another piece that crosses this one (both
                               // endpoints, object frame), in its group too (Sec. IV-D.1)
  size_t n_xedges() const { return xedges.size() / 6; }
  size_t n_planes() const { return planes.size() / 4; }
  size_t n_verts() const { return verts.size() / 3; }
  size_t n_edges() const { return edges.size() / 2; }
};
struct Grid {
  int n = 0;
  double origin[3] = {0, 0, 0}, h[3] = {0, 0, 0}, r = 0;
  std::vector<double> G;  // phi at voxel centres, index (i * n + j) * n + k (spline: its lower bound there)
  bool spline = false;    // the grid of a spline SDF (S2)
};
// Cubic-spline SDF of an object (Sec. III-B): n intervals per axis over the
// box [a, a + n h]; coefficients c[f] of phi (f = 0) and of the normal's three
// components (f = 1..3) at (n + 3)^3 basis functions, index (i (n+3) + j) (n+3) + k.
struct Spline {
  int n = 0;
  double a[3] = {0, 0, 0}, h[3] = {0, 0, 0};
  std::vector<double> c[4];
};
// A primitive of the primitive-based SDF representation (Sec. III-A.1, 3-5).
struct Prim {
  int kind = 0;  // 0: PSQ at a fixed pose; 1: XPSQ (a PSQ swept along a quadratic spline)
  int op = 0;    // how it joins the primitives before it: 0 union, 1 subtraction, 2 intersection
  double c[3] = {0, 0, 0}, R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};  // PSQ: centre, rotation (PSQ -> object)
  double p[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};                      // XPSQ: control points p1, p2, p3
  double a0[3] = {1, 1, 1}, a1[3] = {1, 1, 1};  // SQ scales at t = 0 and t = 1 (PSQ: a0)
  double e0[2] = {1, 1}, e1[2] = {1, 1};        // SQ exponents (eps1, eps2) at t = 0 and t = 1
  std::vector<double> planes;                   // 4 per half-space (n, h) in the PSQ frame
};
struct Object {
  std::vector<Piece> pieces;
  Grid grid;
  bool has_spline = false;
  Spline spl;
  bool has_prims = false;  // SDF side: the primitives (the pieces stay the mesh side)
  std::vector<Prim> prims;
};

std::mutex g_mu;
std::vector<Object*> g_objects;

inline const Object& obj(int h) { return *g_objects.at(size_t(h)); }

// Bounding radius: largest vertex norm in the object frame.
inline double radius_of(const Object& o) {
  double r2 = 0;
  for (const Piece& pc : o.pieces)
    for (size_t i = 0; i < pc.n_verts(); ++i) {
      const double* v = &pc.verts[3 * i];
      r2 = std::max(r2, v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    }
  return std::sqrt(r2);
}

// Arms the conditioning probe for query i (no-op when prm.jitter == 0).
inline void probe_begin(const Params& prm, int64_t i, const Object& A, const Object& B) {
  g_probe.rel = prm.jitter;
  g_probe.len = radius_of(A) + radius_of(B);
  g_probe.key = mix64(uint64_t(int64_t(prm.jitter_seed)) * 0x100000001B3ull ^ uint64_t(i));
  g_probe.ctr = 0;
}
inline void probe_end() { g_probe.rel = 0; }

// ---------------------------------------------------------------- O2 / O3 --
// Smooth intersection of the piece's half-spaces, phi_k = LSE_j(n_j.x + h_j) with
// temperature tau (Sec. II LSE; Sec. III-A.2 smooth intersection; Sec. III-A.3
// half-space SDF).  Also returns grad phi_k = sum_j softmax_j n_j.
template <class T>
void piece_sdf(const Piece& pc, const V3<T>& x, double tau, T& phi, V3<T>& grad) {
  const size_t P = pc.n_planes();
  double m = -std::numeric_limits<double>::infinity();
  for (size_t j = 0; j < P; ++j) {
    const double* p = &pc.planes[4 * j];
    m = std::max(m, val(x.x * p[0] + x.y * p[1] + x.z * p[2] + p[3]));
  }
  T s(0.0);
  V3<T> G{T(0.0), T(0.0), T(0.0)};
  for (size_t j = 0; j < P; ++j) {
    const double* p = &pc.planes[4 * j];
    T a = x.x * p[0] + x.y * p[1] + x.z * p[2] + p[3];
    probe(a, true);
    T w = exp((a - m) / tau);
    s += w;
    G.x += w * p[0]; G.y += w * p[1]; G.z += w * p[2];
  }
  phi = m + tau * log(s);
  grad = G * (1.0 / s);
  probe(phi, true);
  probe3(grad, false);
}

// Smooth union of the object's pieces, phi = -LSE_k(-phi_k) (eq. soft_union).
template <class T>
void object_sdf(const Object& o, const V3<T>& x, const Params& prm, T& phi, V3<T>& grad) {
  const size_t K = o.pieces.size();
  std::vector<T> pk(K);
  std::vector<V3<T>> gk(K);
  double M = std::numeric_limits<double>::infinity();
  for (size_t k = 0; k < K; ++k) {
    piece_sdf(o.pieces[k], x, prm.tau_cap, pk[k], gk[k]);
    M = std::min(M, val(pk[k]));
  }
  T S(0.0);
  V3<T> G{T(0.0), T(0.0), T(0.0)};
  for (size_t k = 0; k < K; ++k) {
    T u = exp((M - pk[k]) / prm.tau_cup);
    S += u;
    G.x += u * gk[k].x; G.y += u * gk[k].y; G.z += u * gk[k].z;
  }
  phi = M - prm.tau_cup * log(S);
  grad = G * (1.0 / S);
  probe(phi, true);
  probe3(grad, false);
}

template <class T>
V3<T> normal_of(const V3<T>& g, const Params& prm) {
  T s = sqrt(dot(g, g) + prm.eps_n * prm.eps_n);
  return g * (1.0 / s);
}

// ---------------------------------------------------------- smooth helpers --
// Sec. II: sigma(x) = 1 / (1 + exp(-x)), evaluated without overflow.
template <class T> T sigmoid(const T& z) {
  if (val(z) >= 0) return 1.0 / (1.0 + exp(-z));
  T e = exp(z);
  return e / (1.0 + e);
}
// Sec. II: s_+(x) = tau log(1 + exp(x / tau)), written as max(x,0) + tau log1p(exp(-|x|/tau)).
template <class T> T softplus(const T& x, double tau) {
  if (val(x) >= 0) return x + tau * log1p(exp(-x / tau));
  return tau * log1p(exp(x / tau));
}
// Sec. II: s_clip(x, a, b) = a + s_+(x - a) - s_+(x - b).
template <class T> T softclip(const T& x, const T& a, const T& b, double tau) {
  return a + softplus(x - a, tau) - softplus(x - b, tau);
}

// ------------------------------------------------------ primitive SDFs --
// Regulariser of the superquadric's powers: every squared coordinate q^2 enters
// as q^2 + delta^2 (q relative to its scale), so that each power is smooth on the
// coordinate planes; the radius as sqrt(|x|^2 + (delta a_min)^2).
constexpr double kSqDelta = 1e-3;

// Superquadric (Sec. III-A.1): f(x) = ((x/a_x)^(2/e2) + (y/a_y)^(2/e2))^(e2/e1)
// + (z/a_z)^(2/e1), e1 = eps1, e2 = eps2.  Its SDF read as the radial distance
// |x| (1 - f(x)^(-e1/2)): the point's distance to where the ray from the centre
// through it crosses f = 1 (f is homogeneous of degree 2/e1 along rays); exact
// for a sphere.
template <class T> T sq_sdf(const V3<T>& x, const T a[3], const T e[2]) {
  const double d2 = kSqDelta * kSqDelta;
  const T X = x.x / a[0], Y = x.y / a[1], Z = x.z / a[2];
  const T fxy = powr(X * X + d2, 1.0 / e[1]) + powr(Y * Y + d2, 1.0 / e[1]);
  const T f = powr(fxy, e[1] / e[0]) + powr(Z * Z + d2, 1.0 / e[0]);
  T amin = a[0];
  if (val(a[1]) < val(amin)) amin = a[1];
  if (val(a[2]) < val(amin)) amin = a[2];
  const T r = sqrt(dot(x, x) + amin * amin * d2);
  return r * (1.0 - powr(f, e[0] * -0.5));
}

// LSE of values with temperature tau (Sec. II): the smooth maximum.
template <class T> T lse(const std::vector<T>& v, double tau) {
  double m = -std::numeric_limits<double>::infinity();
  for (const T& x : v) m = std::max(m, val(x));
  T s(0.0);
  for (const T& x : v) s += exp((x - m) / tau);
  return m + tau * log(s);
}

// PSQ (Sec. III-A.3): smooth intersection of the SQ and the half-spaces, in
// the PSQ frame.
template <class T> T psq_sdf(const Prim& pr, const V3<T>& xs, const T a[3], const T e[2], const Params& prm) {
  std::vector<T> v;
  v.push_back(sq_sdf(xs, a, e));
  for (size_t j = 0; j + 3 < pr.planes.size(); j += 4) {
    const double* q = &pr.planes[j];
    v.push_back(xs.x * q[0] + xs.y * q[1] + xs.z * q[2] + q[3]);
  }
  return v.size() == 1 ? v[0] : lse(v, prm.tau_cap);
}

// The three spline parameters t* of a point's projection onto the XPSQ's
// quadratic spline p(t) = (1-t)^2 p1 + 2t(1-t) p2 + t^2 p3 (Sec. III-A.5):
// d/dt |x - p(t)|^2 / 2 = (p(t) - x) . p'(t) is the cubic
// 2|A|^2 t^3 + 3 A.B t^2 + (|B|^2 + 2 A.(p1 - x)) t + B.(p1 - x), A = p1 - 2 p2 + p3,
// B = 2 (p2 - p1); divided by 2|A|^2 and shifted t = s - a2/3 it reads
// s^3 + P s + Q = 0 with discriminant Delta = -(4 P^3 + 27 Q^2).  Both of
// Cardano's branches are always taken: one real root from Delta^- = -s_+(-Delta),
// s = cbrt(-Q/2 + sqrt(-Delta^-/108)) + cbrt(-Q/2 - sqrt(-Delta^-/108)); three from
// Delta^+ = s_+(Delta) through the cube roots of -Q/2 +- i sqrt(Delta^+/108),
// s_k = 2 r^(1/3) cos((theta + 2 pi k) / 3), r = sqrt(Q^2/4 + Delta^+/108),
// theta = atan2(sqrt(Delta^+/108), -Q/2).  Every root is soft-clipped to (0, 1)
// and t*_k = [Delta < 0] t^- + [Delta > 0] t^+_k with sigmoid brackets.
template <class T> void xpsq_roots(const Prim& pr, const V3<T>& x, const Params& prm, T t[3]) {
  const V3<double> P1{pr.p[0], pr.p[1], pr.p[2]}, P2{pr.p[3], pr.p[4], pr.p[5]}, P3{pr.p[6], pr.p[7], pr.p[8]};
  const V3<double> A = P1 - P2 * 2.0 + P3, B = (P2 - P1) * 2.0;
  const V3<T> C0{T(P1.x) - x.x, T(P1.y) - x.y, T(P1.z) - x.z};
  const double AA = dot(A, A);
  const double a2 = 1.5 * dot(A, B) / AA;
  const T a1 = (dot(B, B) + 2.0 * (C0.x * A.x + C0.y * A.y + C0.z * A.z)) / (2.0 * AA);
  const T a0 = (C0.x * B.x + C0.y * B.y + C0.z * B.z) / (2.0 * AA);
  const T P = a1 - a2 * a2 / 3.0;
  const T Q = a0 - a1 * (a2 / 3.0) + 2.0 * a2 * a2 * a2 / 27.0;
  const T Delta = -(4.0 * P * P * P + 27.0 * Q * Q);
  const double tau = prm.tau_disc, tiny = 1e-20;  // (keeps sqrt differentiable where s_+ underflows)
  const T u = Q * -0.5;
  const T Dm = softplus(-Delta, tau) / 108.0, Dp = softplus(Delta, tau) / 108.0;
  const T sm = sqrt(Dm + tiny);
  const T s_one = cbrt(u + sm) + cbrt(u - sm);
  const T r = sqrt(u * u + Dp), th = atan2(sqrt(Dp + tiny), u), rr = cbrt(r);
  const T w_one = sigmoid(-Delta / tau), w_three = sigmoid(Delta / tau);
  const T zero(0.0), one(1.0);
  const T t_one = softclip(s_one - a2 / 3.0, zero, one, prm.tau_t);
  for (int k = 0; k < 3; ++k) {
    const T sk = 2.0 * rr * cos((th + 2.0 * M_PI * k) / 3.0);
    t[k] = w_one * t_one + w_three * softclip(sk - a2 / 3.0, zero, one, prm.tau_t);
  }
}

// XPSQ (Sec. III-A.4/5): the PSQ placed at each of the three projection
// parameters -- centre p(t), frame R(t) = [N(t), b, T(t)] (the Frenet frame of
// the planar spline: unit tangent T = p'/|p'|, binormal b along B x A, constant
// for a quadratic, N = b x T; the SQ's z-axis runs along the spline), scales and
// exponents linear in t, half-spaces fixed in the PSQ frame -- and the smooth
// minimum of the three PSQ SDFs.
template <class T> T xpsq_sdf(const Prim& pr, const V3<T>& x, const Params& prm) {
  T t[3];
  xpsq_roots(pr, x, prm, t);
  const V3<double> P1{pr.p[0], pr.p[1], pr.p[2]}, P2{pr.p[3], pr.p[4], pr.p[5]}, P3{pr.p[6], pr.p[7], pr.p[8]};
  const V3<double> A = P1 - P2 * 2.0 + P3, B = (P2 - P1) * 2.0;
  V3<double> bn{B.y * A.z - B.z * A.y, B.z * A.x - B.x * A.z, B.x * A.y - B.y * A.x};
  bn = bn * (1.0 / std::sqrt(dot(bn, bn)));
  std::vector<T> neg(3);
  for (int k = 0; k < 3; ++k) {
    const T& tk = t[k];
    const T w0 = (1.0 - tk) * (1.0 - tk), w1 = 2.0 * tk * (1.0 - tk), w2 = tk * tk;
    const V3<T> pt{w0 * P1.x + w1 * P2.x + w2 * P3.x, w0 * P1.y + w1 * P2.y + w2 * P3.y,
                   w0 * P1.z + w1 * P2.z + w2 * P3.z};
    const V3<T> dp{2.0 * tk * A.x + B.x, 2.0 * tk * A.y + B.y, 2.0 * tk * A.z + B.z};
    const T il = 1.0 / sqrt(dot(dp, dp));
    const V3<T> Tn = dp * il;
    const V3<T> Nn{Tn.z * bn.y - Tn.y * bn.z, Tn.x * bn.z - Tn.z * bn.x, Tn.y * bn.x - Tn.x * bn.y};  // b x T
    const V3<T> d = x - pt;
    const V3<T> xs{dot(Nn, d), d.x * bn.x + d.y * bn.y + d.z * bn.z, dot(Tn, d)};
    T a[3], e[2];
    for (int i = 0; i < 3; ++i) a[i] = pr.a0[i] + tk * (pr.a1[i] - pr.a0[i]);
    for (int i = 0; i < 2; ++i) e[i] = pr.e0[i] + tk * (pr.e1[i] - pr.e0[i]);
    neg[size_t(k)] = -psq_sdf(pr, xs, a, e, prm);
  }
  return -lse(neg, prm.tau_cup);
}

template <class T> T prim_sdf(const Prim& pr, const V3<T>& x, const Params& prm) {
  if (pr.kind == 1) return xpsq_sdf(pr, x, prm);
  const V3<T> d{x.x - pr.c[0], x.y - pr.c[1], x.z - pr.c[2]};
  const V3<T> xs{pr.R[0] * d.x + pr.R[3] * d.y + pr.R[6] * d.z, pr.R[1] * d.x + pr.R[4] * d.y + pr.R[7] * d.z,
                 pr.R[2] * d.x + pr.R[5] * d.y + pr.R[8] * d.z};  // R^T d
  const T a[3] = {T(pr.a0[0]), T(pr.a0[1]), T(pr.a0[2])}, e[2] = {T(pr.e0[0]), T(pr.e0[1])};
  return psq_sdf(pr, xs, a, e, prm);
}

// The object's SDF from its primitives (Sec. III-A.2): folded in order, each
// joining the result so far by smooth union (-LSE(-phi, -phi_i), tau_cup),
// subtraction (LSE(phi, -phi_i), tau_cap) or intersection (LSE(phi, phi_i), tau_cap).
template <class T> T prims_sdf(const Object& o, const V3<T>& x, const Params& prm) {
  T phi = prim_sdf(o.prims[0], x, prm);
  for (size_t i = 1; i < o.prims.size(); ++i) {
    const T v = prim_sdf(o.prims[i], x, prm);
    const int op = o.prims[i].op;
    if (op == 0) phi = -lse(std::vector<T>{-phi, -v}, prm.tau_cup);
    else if (op == 1) phi = lse(std::vector<T>{phi, -v}, prm.tau_cap);
    else phi = lse(std::vector<T>{phi, v}, prm.tau_cap);
  }
  return phi;
}


// --------------------------------------------------- edge assignment --
// Sec. IV-D.1: a vertex belongs to the convex piece it lies in (here: its own
// piece), an edge to every piece it intersects.  Besides its own piece, an edge
// of piece k joins piece j != k when the segment keeps a part of positive length
// (> 1e-9 of the object's scale) inside j's hull: the segment a + t (b - a),
// t in [0, 1], clipped by each half-space n.x + h <= 0 of j.
inline bool segment_crosses_piece(const Piece& pj, const double* a, const double* b, double tol) {
  double t0 = 0.0, t1 = 1.0;
  for (size_t i = 0; i < pj.n_planes(); ++i) {
    const double* q = &pj.planes[4 * i];
    const double ca = q[0] * a[0] + q[1] * a[1] + q[2] * a[2] + q[3];
    const double cb = q[0] * b[0] + q[1] * b[1] + q[2] * b[2] + q[3];
    if (ca > 0 && cb > 0) return false;
    if (ca > 0) t0 = std::max(t0, ca / (ca - cb));
    if (cb > 0) t1 = std::min(t1, ca / (ca - cb));
  }
  const double L = std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) + (b[2] - a[2]) * (b[2] - a[2]));
  return (t1 - t0) * L > tol;
}
void assign_edges(Object& o) {
  double scale = 1e-300;
  for (const Piece& pc : o.pieces)
    for (double v : pc.verts) scale = std::max(scale, std::fabs(v));
  for (size_t j = 0; j < o.pieces.size(); ++j) {
    Piece& pj = o.pieces[j];
    pj.xedges.clear();
    for (size_t k = 0; k < o.pieces.size(); ++k) {
      if (k == j) continue;
      const Piece& pk = o.pieces[k];
      for (size_t e = 0; e < pk.n_edges(); ++e) {
        const double* a = &pk.verts[3 * size_t(pk.edges[2 * e])];
        const double* b = &pk.verts[3 * size_t(pk.edges[2 * e + 1])];
        if (segment_crosses_piece(pj, a, b, 1e-9 * scale)) {
          pj.xedges.insert(pj.xedges.end(), a, a + 3);
          pj.xedges.insert(pj.xedges.end(), b, b + 3);
        }
      }
    }
  }
}

// ------------------------------------------------------ S1 spline SDF --
// The ground truth of Sec. III-B.2 needs the closest point of the piece's
// surface: inside a convex piece it lies on the nearest facet plane, outside
// on one of its boundary triangles.
inline V3<double> closest_on_segment(const V3<double>& x, const V3<double>& a, const V3<double>& b) {
  const V3<double> d = b - a;
  const double dd = dot(d, d);
  double t = dd > 0 ? dot(x - a, d) / dd : 0.0;
  t = std::min(1.0, std::max(0.0, t));
  return a + d * t;
}
// Closest point of the triangle t[0..8] to x: the projection onto its plane when
// that lies inside (barycentric coordinates >= 0), else the closest of the three
// sides' closest points.
inline V3<double> closest_on_triangle(const V3<double>& x, const double* t) {
  const V3<double> p0{t[0], t[1], t[2]}, p1{t[3], t[4], t[5]}, p2{t[6], t[7], t[8]};
  const V3<double> e1 = p1 - p0, e2 = p2 - p0, r = x - p0;
  const double a11 = dot(e1, e1), a12 = dot(e1, e2), a22 = dot(e2, e2);
  const double b1 = dot(r, e1), b2 = dot(r, e2);
  const double det = a11 * a22 - a12 * a12;
  if (det > 0) {
    const double u = (b1 * a22 - b2 * a12) / det, v = (a11 * b2 - a12 * b1) / det;
    if (u >= 0 && v >= 0 && u + v <= 1) return p0 + e1 * u + e2 * v;
  }
  const V3<double> c[3] = {closest_on_segment(x, p0, p1), closest_on_segment(x, p1, p2),
                           closest_on_segment(x, p2, p0)};
  int best = 0;
  double bd = 1e300;
  for (int k = 0; k < 3; ++k) {
    const V3<double> d = x - c[k];
    if (dot(d, d) < bd) { bd = dot(d, d); best = k; }
  }
  return c[best];
}

// Exact SDF of a convex piece at x and the vector x - proj(x) from the closest
// surface point: inside, the largest plane value a_j* (<= 0) and a_j* n_j*;
// outside, the distance to the closest point over the boundary triangles.
inline double piece_exact(const Piece& pc, const V3<double>& x, V3<double>& diff) {
  double m = -1e300;
  size_t jm = 0;
  for (size_t j = 0; j < pc.n_planes(); ++j) {
    const double* p = &pc.planes[4 * j];
    const double a = x.x * p[0] + x.y * p[1] + x.z * p[2] + p[3];
    if (a > m) { m = a; jm = j; }
  }
  if (m <= 0) {
    const double* p = &pc.planes[4 * jm];
    diff = V3<double>{p[0], p[1], p[2]} * m;
    return m;
  }
  double best = 1e300;
  for (size_t t = 0; t < pc.tris.size() / 9; ++t) {
    const V3<double> d = x - closest_on_triangle(x, &pc.tris[9 * t]);
    if (dot(d, d) < best) { best = dot(d, d); diff = d; }
  }
  return std::sqrt(best);
}

// Ground-truth SDF and normal of the object (Sec. III-B.2), the union of its
// pieces: phi = min_k phi_k and, from the minimising piece, the unit direction
// sign(phi) (x - proj(x)) / |x - proj(x)|: outside (x - proj) / phi, inside and
// on the surface the outward normal of the nearest facet (the limit of the
// paper's (x - proj) / (|x - proj| + eps) as eps -> 0, defined on the surface too).
inline void ground_truth(const Object& o, const V3<double>& x, double* out4) {
  double phi = 1e300;
  V3<double> diff{0, 0, 0}, nin{0, 0, 0};
  for (const Piece& pc : o.pieces) {
    V3<double> d{0, 0, 0};
    const double p = piece_exact(pc, x, d);
    if (p < phi) {
      phi = p;
      diff = d;
      if (p <= 0) {  // inside: the nearest facet's normal, found again by its value
        double m = -1e300;
        for (size_t j = 0; j < pc.n_planes(); ++j) {
          const double* q = &pc.planes[4 * j];
          const double a = x.x * q[0] + x.y * q[1] + x.z * q[2] + q[3];
          if (a > m) { m = a; nin = V3<double>{q[0], q[1], q[2]}; }
        }
      }
    }
  }
  const V3<double> n = phi > 0 ? diff * (1.0 / std::sqrt(dot(diff, diff))) : nin;
  out4[0] = phi; out4[1] = n.x; out4[2] = n.y; out4[3] = n.z;
}

// 1-D interpolation operator (Sec. III-B.1): coefficients c_0..c_{n+2} of
// s(t) = sum_m c_m u(t - m + 1), t in node units, from the values f_0..f_n at
// the nodes, c = M f.  The square system is s(t_i) = c_i + 4 c_{i+1} + c_{i+2}
// = f_i (i = 0..n) and the natural end conditions s''(t_0) = s''(t_n) = 0,
// i.e. c_0 - 2 c_1 + c_2 = 0 and c_n - 2 c_{n+1} + c_{n+2} = 0; M is the first
// n + 1 columns of its inverse (Gauss-Jordan with partial pivoting).
inline std::vector<double> spline_operator(int n) {
  const int m = n + 3;
  std::vector<double> A(size_t(m) * m, 0.0), I(size_t(m) * m, 0.0);
  auto at = [m](std::vector<double>& X, int r, int c) -> double& { return X[size_t(r) * m + c]; };
  for (int i = 0; i <= n; ++i) { at(A, i, i) = 1; at(A, i, i + 1) = 4; at(A, i, i + 2) = 1; }
  at(A, n + 1, 0) = 1; at(A, n + 1, 1) = -2; at(A, n + 1, 2) = 1;
  at(A, n + 2, n) = 1; at(A, n + 2, n + 1) = -2; at(A, n + 2, n + 2) = 1;
  for (int i = 0; i < m; ++i) at(I, i, i) = 1;
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int r = col + 1; r < m; ++r)
      if (std::fabs(at(A, r, col)) > std::fabs(at(A, piv, col))) piv = r;
    for (int k = 0; k < m; ++k) { std::swap(at(A, col, k), at(A, piv, k)); std::swap(at(I, col, k), at(I, piv, k)); }
    const double d = at(A, col, col);
    for (int k = 0; k < m; ++k) { at(A, col, k) /= d; at(I, col, k) /= d; }
    for (int r = 0; r < m; ++r) {
      const double f = at(A, r, col);
      if (r == col || f == 0) continue;
      for (int k = 0; k < m; ++k) { at(A, r, k) -= f * at(A, col, k); at(I, r, k) -= f * at(I, col, k); }
    }
  }
  std::vector<double> M(size_t(m) * (n + 1));
  for (int r = 0; r < m; ++r)
    for (int k = 0; k <= n; ++k) M[size_t(r) * (n + 1) + k] = at(I, r, k);
  return M;
}

// The box of an object's voxel grid and spline: the vertex AABB grown by
// grid_margin + grid_margin_rel * (bounding radius), n = grid_res cells per axis.
inline void object_box(const Object& o, const Params& prm, double* origin, double* h) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  double rad = 0;
  for (const Piece& pc : o.pieces)
    for (size_t i = 0; i < pc.n_verts(); ++i) {
      const double* v = &pc.verts[3 * i];
      for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], v[a]); hi[a] = std::max(hi[a], v[a]); }
      rad = std::max(rad, std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
    }
  const double margin = prm.grid_margin + prm.grid_margin_rel * rad;
  for (int a = 0; a < 3; ++a) {
    origin[a] = lo[a] - margin;
    h[a] = (hi[a] - lo[a] + 2 * margin) / prm.grid_res;
  }
}

// S1: the ground truth at the (n + 1)^3 corners of the box, then the
// coefficients of the four splines by the 1-D operator along z, y and x in
// turn (the tensor-product interpolant; Sec. III-B.1).
// Coefficients of the four splines from values [4][(n+1)^3] at the corners
// (index (i (n+1) + j) (n+1) + k).
void fit_spline(Spline& sp, const std::vector<double>& f) {
  const int n = sp.n, n1 = n + 1, m = n + 3;
  const std::vector<double> M = spline_operator(n);
  for (int c = 0; c < 4; ++c) {
    const double* F = &f[size_t(c) * n1 * n1 * n1];
    std::vector<double> z(size_t(n1) * n1 * m), y(size_t(n1) * m * m);
    sp.c[c].assign(size_t(m) * m * m, 0.0);
    for (int i = 0; i < n1; ++i)
      for (int j = 0; j < n1; ++j)
        for (int r = 0; r < m; ++r) {
          double s = 0;
          for (int k = 0; k < n1; ++k) s += M[size_t(r) * n1 + k] * F[(size_t(i) * n1 + j) * n1 + k];
          z[(size_t(i) * n1 + j) * m + r] = s;
        }
    for (int i = 0; i < n1; ++i)
      for (int r = 0; r < m; ++r)
        for (int q = 0; q < m; ++q) {
          double s = 0;
          for (int j = 0; j < n1; ++j) s += M[size_t(r) * n1 + j] * z[(size_t(i) * n1 + j) * m + q];
          y[(size_t(i) * m + r) * m + q] = s;
        }
    for (int r = 0; r < m; ++r)
      for (int q = 0; q < m; ++q)
        for (int p = 0; p < m; ++p) {
          double s = 0;
          for (int i = 0; i < n1; ++i) s += M[size_t(r) * n1 + i] * y[(size_t(i) * m + q) * m + p];
          sp.c[c][(size_t(r) * m + q) * m + p] = s;
        }
  }
}

void build_spline(Object& o, const Params& prm) {
  Spline& sp = o.spl;
  const int n = prm.grid_res;
  sp.n = n;
  object_box(o, prm, sp.a, sp.h);
  const int n1 = n + 1;
  std::vector<double> f(size_t(4) * n1 * n1 * n1);
#ifdef _OPENMP
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
#endif
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j)
      for (int k = 0; k < n1; ++k) {
        const V3<double> x{sp.a[0] + i * sp.h[0], sp.a[1] + j * sp.h[1], sp.a[2] + k * sp.h[2]};
        double g[4];
        ground_truth(o, x, g);
        for (int c = 0; c < 4; ++c) f[((size_t(c) * n1 + i) * n1 + j) * n1 + k] = g[c];
      }
  fit_spline(sp, f);
  o.has_spline = true;
}

template <class T> T clamp_to(const T& x, double lo, double hi) {
  if (val(x) < lo) return T(lo);
  if (val(x) > hi) return T(hi);
  return x;
}
// The four basis functions that are nonzero in a cell, at the offset w in
// [0, 1] into it: u(w + 1), u(w), u(w - 1), u(w - 2) of Sec. III-B.1.
template <class T> void cell_weights(const T& w, T* b) {
  const T v = 1.0 - w;
  b[0] = v * v * v;
  b[1] = 4.0 - 6.0 * w * w + 3.0 * w * w * w;
  b[2] = 4.0 - 6.0 * v * v + 3.0 * v * v * v;
  b[3] = w * w * w;
}
// S1 evaluation at x (object frame): the 64 nonzero terms of each spline.
// Outside the box phi continues as s_phi(pi(x)) + |x - pi(x)| and the normal as
// s_n(pi(x)), pi(x) the closest point of the box (reading, see DESIGN).
template <class T> void spline_eval(const Spline& sp, const V3<T>& x, T& phi, V3<T>& nrm) {
  const T xs[3] = {x.x, x.y, x.z};
  T w[3][4];
  int i0[3];
  T out2(0.0);
  bool outside = false;
  for (int a = 0; a < 3; ++a) {
    const double lo = sp.a[a], hi = sp.a[a] + sp.n * sp.h[a];
    const T pa = clamp_to(xs[a], lo, hi);
    if (val(xs[a]) < lo || val(xs[a]) > hi) {
      const T d = xs[a] - pa;
      out2 = out2 + d * d;
      outside = true;
    }
    const T t = (pa - lo) * (1.0 / sp.h[a]);
    const int i = std::min(std::max(int(std::floor(val(t))), 0), sp.n - 1);
    i0[a] = i;
    cell_weights(t - double(i), w[a]);
  }
  const size_t m = size_t(sp.n) + 3;
  T acc[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q)
      for (int r = 0; r < 4; ++r) {
        const T wt = w[0][p] * w[1][q] * w[2][r];
        const size_t idx = (size_t(i0[0] + p) * m + size_t(i0[1] + q)) * m + size_t(i0[2] + r);
        for (int c = 0; c < 4; ++c) acc[c] += wt * sp.c[c][idx];
      }
  phi = outside ? acc[0] + sqrt(out2) : acc[0];
  nrm = V3<T>{acc[1], acc[2], acc[3]};
}

// The SDF side of a contact, for either representation: phi alone, and phi
// with the contact normal (planes: the normalised gradient; spline: the
// separately fitted normal spline, Sec. III-B.2).
template <class T> T object_phi(const Object& o, const V3<T>& x, const Params& prm) {
  T phi;
  if (o.has_prims) {
    phi = prims_sdf(o, x, prm);
    probe(phi, true);
  } else if (o.has_spline) {
    V3<T> n;
    spline_eval(o.spl, x, phi, n);
    probe(phi, true);
  } else {
    V3<T> g;
    object_sdf(o, x, prm, phi, g);
  }
  return phi;
}
template <class T> void object_phi_normal(const Object& o, const V3<T>& x, const Params& prm, T& phi, V3<T>& n) {
  if (o.has_prims) {
    // (primitives: the normalised gradient, by forward differentiation in x)
    using G = Dual<T, 3>;
    const V3<G> xg{G(x.x, 0), G(x.y, 0), G(x.z, 0)};
    V3<G> xs = xg;
    xs.x.d[0] = T(1.0); xs.y.d[1] = T(1.0); xs.z.d[2] = T(1.0);
    const G r = prims_sdf(o, xs, prm);
    phi = r.v;
    V3<T> g{r.d[0], r.d[1], r.d[2]};
    probe(phi, true);
    probe3(g, false);
    n = normal_of(g, prm);
  } else if (o.has_spline) {
    spline_eval(o.spl, x, phi, n);
    probe(phi, true);
    probe3(n, false);
  } else {
    V3<T> g;
    object_sdf(o, x, prm, phi, g);
    n = normal_of(g, prm);
  }
}

// ------------------------------------------------------------------ O4 grid --
void build_grid(Object& o, const Params& prm) {
  Grid& g = o.grid;
  g.n = prm.grid_res;
  object_box(o, prm, g.origin, g.h);
  double r2 = 0;
  for (int a = 0; a < 3; ++a) r2 += g.h[a] * g.h[a];
  g.r = 0.5 * std::sqrt(r2);  // circumradius of a voxel
  g.G.assign(size_t(g.n) * g.n * g.n, 0.0);
  // S2: a spline SDF is not a true distance (no 1-Lipschitz bound), so its
  // voxels (the spline's own cells) store a lower bound of the spline over the
  // cell instead: the three 1-D bases of a cell are >= 0 and each sums to 6, so
  // s is 216 times a convex combination of the 64 coefficients the cell
  // reaches, and s >= 216 min of them.
  g.spline = o.has_spline;
#ifdef _OPENMP
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
#endif
  for (int i = 0; i < g.n; ++i)
    for (int j = 0; j < g.n; ++j)
      for (int k = 0; k < g.n; ++k) {
        V3<double> c{g.origin[0] + (i + 0.5) * g.h[0], g.origin[1] + (j + 0.5) * g.h[1],
                     g.origin[2] + (k + 0.5) * g.h[2]};
        const size_t v = (size_t(i) * g.n + j) * g.n + k;
        if (o.has_spline) {
          const size_t m = size_t(g.n) + 3;
          double lo = 1e300;
          for (int p = 0; p < 4; ++p)
            for (int q = 0; q < 4; ++q)
              for (int r = 0; r < 4; ++r)
                lo = std::min(lo, o.spl.c[0][(size_t(i + p) * m + size_t(j + q)) * m + size_t(k + r)]);
          g.G[v] = 216.0 * lo;
        } else {
          double phi; V3<double> gr;
          object_sdf(o, c, prm, phi, gr);
          g.G[v] = phi;
        }
      }
}

// Lower bound of phi at x (SDF-object frame): phi(p_c) minus the distance bound,
// max(r, |x - p_c|), which is the circumradius inside the grid and the
// 1-Lipschitz extension for points clamped from outside it (Sec. IV-C.2, Fig. broadphase1).
inline double lower_bound(const Grid& g, const V3<double>& x, double* face_dist = nullptr) {
  const double xs[3] = {x.x, x.y, x.z};
  int idx[3];
  double d2 = 0;
  double fd = 1e300;
  for (int a = 0; a < 3; ++a) {
    double u = (xs[a] - g.origin[a]) / g.h[a];
    fd = std::min(fd, std::fabs(u - std::round(u)) * g.h[a]);  // distance to the nearest voxel face
    int i = int(std::floor(u));
    i = std::min(std::max(i, 0), g.n - 1);
    idx[a] = i;
    double c = g.origin[a] + (i + 0.5) * g.h[a];
    d2 += (xs[a] - c) * (xs[a] - c);
  }
  double Gc = g.G[(size_t(idx[0]) * g.n + idx[1]) * g.n + idx[2]];
  if (face_dist) *face_dist = fd;
  if (g.spline) {
    // S2: the cell's bound holds at pi(x), the closest point of the box (whose
    // cell is the clamped one), and outside the box phi = s(pi(x)) + |x - pi(x)|
    double o2 = 0;
    for (int a = 0; a < 3; ++a) {
      const double lo = g.origin[a], hi = g.origin[a] + g.n * g.h[a];
      const double d = xs[a] < lo ? lo - xs[a] : (xs[a] > hi ? xs[a] - hi : 0.0);
      o2 += d * d;
    }
    return Gc + std::sqrt(o2);
  }
  return Gc - std::max(g.r, std::sqrt(d2));
}

// S2 for an edge x1 -> x2 against a spline SDF: every point of the segment lies
// in its bounding box, whose closest points of the grid box lie in the cells
// of the clamped index range, so phi >= (least cell bound over that range) +
// (distance from the bounding box to the grid box).
inline double spline_edge_bound(const Grid& g, const V3<double>& x1, const V3<double>& x2) {
  const double a[3] = {x1.x, x1.y, x1.z}, b[3] = {x2.x, x2.y, x2.z};
  int lo[3], hi[3];
  double gap2 = 0;
  for (int k = 0; k < 3; ++k) {
    const double mn = std::min(a[k], b[k]), mx = std::max(a[k], b[k]);
    lo[k] = std::min(std::max(int(std::floor((mn - g.origin[k]) / g.h[k])), 0), g.n - 1);
    hi[k] = std::min(std::max(int(std::floor((mx - g.origin[k]) / g.h[k])), 0), g.n - 1);
    const double blo = g.origin[k], bhi = g.origin[k] + g.n * g.h[k];
    const double d = mx < blo ? blo - mx : (mn > bhi ? mn - bhi : 0.0);
    gap2 += d * d;
  }
  double m = 1e300;
  for (int i = lo[0]; i <= hi[0]; ++i)
    for (int j = lo[1]; j <= hi[1]; ++j)
      for (int k = lo[2]; k <= hi[2]; ++k) m = std::min(m, g.G[(size_t(i) * g.n + j) * g.n + k]);
  return m + std::sqrt(gap2);
}

// ------------------------------------------------------------- O6 E-SDF --
// Sphere trace both corners towards each other with the soft-gated step
// sigma(phi/tau_s) * phi (Sec. IV-B.2; Fig. e_s), K iterations, then softclip
// both arc lengths to [0, L] and return the midpoint (SDF-object frame).
template <class T, class Sdf>
V3<T> edge_point(const Sdf& sdf, const V3<T>& xI, const V3<T>& xII, const Params& prm,
                 T* alpha_out = nullptr, T* beta_out = nullptr) {
  V3<T> dvec = xII - xI;
  T L = sqrt(dot(dvec, dvec));
  V3<T> e = dvec * (1.0 / L);
  T alpha(0.0), beta(0.0);
  for (int k = 0; k < prm.st_iters; ++k) {
    T pa = sdf(xI + e * alpha);
    T pb = sdf(xII - e * beta);
    alpha = alpha + sigmoid(pa * (1.0 / prm.tau_st)) * pa;
    beta = beta + sigmoid(pb * (1.0 / prm.tau_st)) * pb;
    probe(alpha, true);
    probe(beta, true);
  }
  T zero(0.0);
  T ac = softclip(alpha, zero, L, prm.tau_clip);
  T bc = softclip(beta, zero, L, prm.tau_clip);
  if (alpha_out) *alpha_out = ac;
  if (beta_out) *beta_out = bc;
  return (xI + e * ac + xII - e * bc) * 0.5;
}

// ----------------------------------------------------------- O7 mollify --
// C2 transition: quintic smoothstep of s = (d_max - phi)/eps_t clamped to [0,1];
// non-increasing in phi, 0 for phi >= d_max, 1 for phi <= d_max - eps_t (Sec. IV-C.1).
template <class T> T transition(const T& phi, const Params& prm) {
  T s = (prm.d_max - phi) * (1.0 / prm.eps_t);
  if (val(s) <= 0) return T(0.0);
  if (val(s) >= 1) return T(1.0);
  return s * s * s * (10.0 - 15.0 * s + 6.0 * s * s);
}

template <class T> struct Contact {
  T d, f;            // mollified depth d_c and transition value f
  V3<T> pc, nc, fp;  // mollified point, mollified world normal, f * raw point
  double raw_phi;    // unmollified phi (NaN when filtered)
  int mask;          // 1 = survived the broad phase
  int kind;          // 0 vertex, 1 edge
  double bound = std::numeric_limits<double>::quiet_NaN();      // broad-phase lower bound
  double face_dist = std::numeric_limits<double>::quiet_NaN();  // distance to the nearest voxel face
};

template <class T>
Contact<T> mollify(const T& phi, const V3<T>& Nw, const V3<T>& p, const V3<T>& p_rest, const Params& prm) {
  Contact<T> c;
  T f = transition(phi, prm);
  c.f = f;
  c.d = f * phi + (1.0 - f) * prm.d_max;
  c.nc = Nw * f;
  c.pc = p * f + p_rest * (1.0 - f);
  c.fp = p * f;
  c.raw_phi = val(phi);
  c.mask = 1;
  return c;
}

template <class T>
Contact<T> filtered(const V3<T>& p_rest, const Params& prm) {
  Contact<T> c;
  c.f = T(0.0);
  c.d = T(prm.d_max);
  c.nc = V3<T>{T(0.0), T(0.0), T(0.0)};
  c.pc = p_rest;
  c.fp = V3<T>{T(0.0), T(0.0), T(0.0)};
  c.raw_phi = std::numeric_limits<double>::quiet_NaN();
  c.mask = 0;
  return c;
}

// ------------------------------------------------------------- O8 blend --
template <class T> struct GroupOut {
  V3<T> p, n; T d; V3<T> q; T W, logZ;
};

// Softmax over l_i = -d_c,i / tau_b (deeper contacts weigh more), then blend
// depth, normal (renormalised), point and the Jacobian moments q = sum w f p,
// W = sum w f (Sec. IV-D.2-3).
template <class T>
GroupOut<T> blend(const std::vector<Contact<T>>& cs, const Params& prm, std::vector<double>* w_out) {
  double Lam = -std::numeric_limits<double>::infinity();
  std::vector<T> l(cs.size());
  for (size_t i = 0; i < cs.size(); ++i) { l[i] = cs[i].d * (-1.0 / prm.tau_blend); Lam = std::max(Lam, val(l[i])); }
  T Z(0.0);
  std::vector<T> e(cs.size());
  for (size_t i = 0; i < cs.size(); ++i) { e[i] = exp(l[i] - Lam); Z += e[i]; }
  GroupOut<T> g;
  T zero(0.0);
  g.p = g.n = g.q = V3<T>{zero, zero, zero};
  g.d = g.W = zero;
  V3<T> m{zero, zero, zero};
  for (size_t i = 0; i < cs.size(); ++i) {
    T w = e[i] / Z;
    if (w_out) w_out->push_back(val(w));
    g.d += w * cs[i].d;
    m = m + cs[i].nc * w;
    g.p = g.p + cs[i].pc * w;
    g.q = g.q + cs[i].fp * w;
    g.W += w * cs[i].f;
  }
  g.n = normal_of(m, prm);
  g.logZ = Lam + log(Z);
  return g;
}

// ---------------------------------------------------------- O5-O9 query --
template <class T> struct Pose { M3<T> R; V3<T> t; };

template <class T> struct SdfFn {
  const Object* o; const Params* prm;
  T operator()(const V3<T>& x) const { return object_phi(*o, x, *prm); }
};

// One direction: vertices and edges of `mesh` against the SDF of `sdf`.
template <class T>
void direction(const Object& mesh, const Object& sdf, const Pose<T>& PM, const Pose<T>& PS,
               const Params& prm, std::vector<GroupOut<T>>& out, std::vector<double>* dbg) {
  const bool bp = prm.broad_phase != 0 && sdf.grid.n > 0;
  SdfFn<T> fn{&sdf, &prm};
  for (const Piece& pc : mesh.pieces) {
    std::vector<Contact<T>> cs;
    const size_t V = pc.n_verts();
    std::vector<V3<T>> Pw(V), xs(V);
    for (size_t i = 0; i < V; ++i) {
      Pw[i] = mul(PM.R, cvt<T>(&pc.verts[3 * i])) + PM.t;  // world position of the vertex
      xs[i] = mulT(PS.R, Pw[i] - PS.t);                       // in the SDF object's frame
      probe3(xs[i], true);
    }
    // O5: vertex-SDF contacts (Sec. IV-B).
    for (size_t i = 0; i < V; ++i) {
      double bound = 0, fd = 0;
      if (bp) bound = lower_bound(sdf.grid, vval(xs[i]), &fd);
      if (bp && bound >= prm.d_max) {
        cs.push_back(filtered(Pw[i], prm));
      } else {
        T phi; V3<T> nS;
        object_phi_normal(sdf, xs[i], prm, phi, nS);
        V3<T> Nw = mul(PS.R, nS);
        cs.push_back(mollify(phi, Nw, Pw[i], Pw[i], prm));
      }
      cs.back().kind = 0;
      if (bp) { cs.back().bound = bound; cs.back().face_dist = fd; }
    }
    // O6: edge-SDF contacts (Sec. IV-B.2).
    for (size_t k = 0; k < pc.n_edges(); ++k) {
      const int i0 = pc.edges[2 * k], i1 = pc.edges[2 * k + 1];
      V3<T> rest = (Pw[i0] + Pw[i1]) * 0.5;
      double ebound = 0, efd = 0;
      if (bp) {
        V3<double> a = vval(xs[i0]), b = vval(xs[i1]);
        V3<double> dv = b - a;
        double L = std::sqrt(dot(dv, dv));
        double fa = 0, fb = 0;
        double la = lower_bound(sdf.grid, a, &fa), lbb = lower_bound(sdf.grid, b, &fb);
        efd = std::min(fa, fb);
        // Any edge point is within s of one end and L - s of the other, so
        // phi >= min(la, lb) - L (the paper's form) and, tighter,
        // phi >= max(max(la, lb) - L, (la + lb - L) / 2).
        double lb = prm.edge_bound == 0 ? std::min(la, lbb) - L
                                        : std::max(std::max(la, lbb) - L, 0.5 * (la + lbb - L));
        if (sdf.grid.spline) lb = spline_edge_bound(sdf.grid, a, b);
        ebound = lb;
        if (lb >= prm.d_max) {
          cs.push_back(filtered(rest, prm));
          cs.back().kind = 1; cs.back().bound = ebound; cs.back().face_dist = efd;
          continue;
        }
      }
      V3<T> pe = edge_point(fn, xs[i0], xs[i1], prm);
      probe3(pe, true);
      T phi; V3<T> nS;
      object_phi_normal(sdf, pe, prm, phi, nS);
      V3<T> Nw = mul(PS.R, nS);
      V3<T> pw = mul(PS.R, pe) + PS.t;
      cs.push_back(mollify(phi, Nw, pw, rest, prm)); cs.back().kind = 1;
      if (bp) { cs.back().bound = ebound; cs.back().face_dist = efd; }
    }
    // edges of other pieces that cross this one (Sec. IV-D.1), the same E-SDF
    for (size_t k = 0; k < pc.n_xedges(); ++k) {
      V3<T> W0 = mul(PM.R, cvt<T>(&pc.xedges[6 * k])) + PM.t, W1 = mul(PM.R, cvt<T>(&pc.xedges[6 * k + 3])) + PM.t;
      V3<T> x0 = mulT(PS.R, W0 - PS.t), x1 = mulT(PS.R, W1 - PS.t);
      probe3(x0, true);
      probe3(x1, true);
      V3<T> rest = (W0 + W1) * 0.5;
      if (bp) {
        V3<double> a = vval(x0), b = vval(x1);
        V3<double> dv = b - a;
        double L = std::sqrt(dot(dv, dv));
        double la = lower_bound(sdf.grid, a), lbb = lower_bound(sdf.grid, b);
        double lb = prm.edge_bound == 0 ? std::min(la, lbb) - L
                                        : std::max(std::max(la, lbb) - L, 0.5 * (la + lbb - L));
        if (sdf.grid.spline) lb = spline_edge_bound(sdf.grid, a, b);
        if (lb >= prm.d_max) {
          cs.push_back(filtered(rest, prm));
          cs.back().kind = 1;
          continue;
        }
      }
      V3<T> pe = edge_point(fn, x0, x1, prm);
      probe3(pe, true);
      T phi; V3<T> nS;
      object_phi_normal(sdf, pe, prm, phi, nS);
      V3<T> Nw = mul(PS.R, nS);
      V3<T> pw = mul(PS.R, pe) + PS.t;
      cs.push_back(mollify(phi, Nw, pw, rest, prm));
      cs.back().kind = 1;
    }
    std::vector<double> w;
    out.push_back(blend(cs, prm, dbg ? &w : nullptr));
    if (dbg) {
      for (size_t i = 0; i < cs.size(); ++i) {
        const Contact<T>& c = cs[i];
        double rec[14] = {double(c.mask), val(c.d), val(c.f), w[i],
                          val(c.pc.x), val(c.pc.y), val(c.pc.z),
                          val(c.nc.x), val(c.nc.y), val(c.nc.z), c.raw_phi, double(c.kind), c.bound, c.face_dist};
        dbg->insert(dbg->end(), rec, rec + 14);
      }
    }
  }
}

template <class T>
void query(const Object& A, const Object& B, const Pose<T>& PA, const Pose<T>& PB, const Params& prm,
           std::vector<GroupOut<T>>& out, std::vector<double>* dbg) {
  direction(A, B, PA, PB, prm, out, dbg);  // A's mesh against B's SDF
  direction(B, A, PB, PA, prm, out, dbg);  // roles swapped (Sec. III)
}

template <class T> inline void put(const GroupOut<T>& g, double* o) {
  const T* v[12] = {&g.p.x, &g.p.y, &g.p.z, &g.n.x, &g.n.y, &g.n.z, &g.d, &g.q.x, &g.q.y, &g.q.z, &g.W, &g.logZ};
  for (int i = 0; i < 12; ++i) o[i] = val(*v[i]);
}
template <class T> inline const T& comp(const GroupOut<T>& g, int i) {
  const T* v[12] = {&g.p.x, &g.p.y, &g.p.z, &g.n.x, &g.n.y, &g.n.z, &g.d, &g.q.x, &g.q.y, &g.q.z, &g.W, &g.logZ};
  return *v[i];
}

// ----------------------------------------------------- O10 perturbed pose --
// T_X(xi) = (exp([w_X]x) R_X, t_X + v_X).  `second_order` uses I + W + W^2/2,
// whose first and second derivatives at xi = 0 equal those of the exponential;
// otherwise Rodrigues' formula (used for finite differences at +-h).
template <class T>
Pose<T> perturbed(const M3<double>& R0, const double* t0, const T* w, const T* v, bool second_order) {
  M3<T> E;
  T zero(0.0), one(1.0);
  if (second_order) {
    // W = [w]x
    M3<T> W;
    W.m[0][0] = zero; W.m[0][1] = -w[2]; W.m[0][2] = w[1];
    W.m[1][0] = w[2]; W.m[1][1] = zero; W.m[1][2] = -w[0];
    W.m[2][0] = -w[1]; W.m[2][1] = w[0]; W.m[2][2] = zero;
    M3<T> W2 = matmul(W, W);
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j)
      E.m[i][j] = (i == j ? one : zero) + W.m[i][j] + W2.m[i][j] * 0.5;
  } else {
    double wx = val(w[0]), wy = val(w[1]), wz = val(w[2]);
    double th = std::sqrt(wx * wx + wy * wy + wz * wz);
    double K[3][3] = {{0, -wz, wy}, {wz, 0, -wx}, {-wy, wx, 0}};
    double K2[3][3];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
      K2[i][j] = 0; for (int l = 0; l < 3; ++l) K2[i][j] += K[i][l] * K[l][j]; }
    double a = th > 1e-300 ? std::sin(th) / th : 1.0;
    double b = th > 1e-300 ? (1 - std::cos(th)) / (th * th) : 0.5;
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j)
      E.m[i][j] = T((i == j ? 1.0 : 0.0) + a * K[i][j] + b * K2[i][j]);
  }
  M3<T> R0T;
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) R0T.m[i][j] = T(R0.m[i][j]);
  Pose<T> P;
  P.R = matmul(E, R0T);
  P.t = V3<T>{T(t0[0]) + v[0], T(t0[1]) + v[1], T(t0[2]) + v[2]};
  return P;
}

size_t n_groups(const Object& A, const Object& B) { return A.pieces.size() + B.pieces.size(); }
size_t n_contacts(const Object& o) {
  size_t c = 0;
  for (const Piece& p : o.pieces) c += p.n_verts() + p.n_edges() + p.n_xedges();
  return c;
}

}  // namespace orc

using namespace orc;

extern "C" {

// Registers an object given explicitly as pieces; returns its handle.
int orc_object_create(int32_t n_pieces, const int64_t* plane_off, const double* planes,
                      const int64_t* vert_off, const double* verts,
                      const int64_t* edge_off, const int32_t* edges) {
  Object* o = new Object;
  o->pieces.resize(size_t(n_pieces));
  for (int k = 0; k < n_pieces; ++k) {
    Piece& p = o->pieces[size_t(k)];
    p.planes.assign(planes + 4 * plane_off[k], planes + 4 * plane_off[k + 1]);
    p.verts.assign(verts + 3 * vert_off[k], verts + 3 * vert_off[k + 1]);
    p.edges.assign(edges + 2 * edge_off[k], edges + 2 * edge_off[k + 1]);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_objects.push_back(o);
  return int(g_objects.size() - 1);
}

void orc_object_free(int32_t h) {
  std::lock_guard<std::mutex> lk(g_mu);
  delete g_objects.at(size_t(h));
  g_objects[size_t(h)] = nullptr;
}

void orc_build_grid(int32_t h, const Params* prm) { build_grid(*g_objects.at(size_t(h)), *prm); }

// Sec. IV-D.1 edge assignment: each piece also collects the edges of the other
// pieces that cross it; returns the number collected per piece (counts[n_pieces]).
void orc_assign_edges(int32_t h, int64_t* counts) {
  Object& o = *g_objects.at(size_t(h));
  assign_edges(o);
  for (size_t k = 0; k < o.pieces.size(); ++k) counts[k] = int64_t(o.pieces[k].n_xedges());
}

// Boundary triangles of each piece (9 doubles each, tri_off[n_pieces + 1]),
// used only by the spline's ground truth.
void orc_object_set_tris(int32_t h, const int64_t* tri_off, const double* tris) {
  Object& o = *g_objects.at(size_t(h));
  for (size_t k = 0; k < o.pieces.size(); ++k)
    o.pieces[k].tris.assign(tris + 9 * tri_off[k], tris + 9 * tri_off[k + 1]);
}

// S1: fits the object's spline SDF (then its voxel grid follows the spline).
void orc_build_spline(int32_t h, const Params* prm) { build_spline(*g_objects.at(size_t(h)), *prm); }

// The object's SDF side becomes its primitives (Sec. III-A), n records of 32
// doubles: [0] kind (0 PSQ, 1 XPSQ), [1] op (0 union, 1 subtraction,
// 2 intersection with the primitives before it), [2..4] PSQ centre / XPSQ p1,
// [5..7] p2, [8..10] p3, [11..14] PSQ rotation as a unit quaternion (w, x, y, z),
// [15..17] scales a at t = 0, [18..19] exponents (eps1, eps2) at t = 0,
// [20..22] a at t = 1, [23..24] exponents at t = 1; half-spaces planes[4 plane_off[i]
// .. 4 plane_off[i + 1]) in the PSQ frame.  Its pieces remain the mesh side.
void orc_object_set_prims(int32_t h, int32_t n, const double* rec, const int64_t* plane_off, const double* planes) {
  Object& o = *g_objects.at(size_t(h));
  o.prims.assign(size_t(n), Prim{});
  for (int32_t i = 0; i < n; ++i) {
    const double* r = rec + 32 * i;
    Prim& q = o.prims[size_t(i)];
    q.kind = int(r[0]);
    q.op = int(r[1]);
    for (int k = 0; k < 3; ++k) q.c[k] = r[2 + k];
    for (int k = 0; k < 9; ++k) q.p[k] = r[2 + k];
    const M3<double> R = quat_to_R(r + 11);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) q.R[3 * a + b] = R.m[a][b];
    for (int k = 0; k < 3; ++k) { q.a0[k] = r[15 + k]; q.a1[k] = r[20 + k]; }
    for (int k = 0; k < 2; ++k) { q.e0[k] = r[18 + k]; q.e1[k] = r[23 + k]; }
    q.planes.assign(planes + 4 * plane_off[i], planes + 4 * plane_off[i + 1]);
  }
  o.has_prims = n > 0;
}

// The primitive SDF phi and its gradient (n x 3) at n object-frame points.
void orc_prims_eval(int32_t h, const Params* prm, int64_t n, const double* x, double* phi, double* grad) {
  const Object& o = obj(h);
  typedef Dual<double, 3> D3;
  for (int64_t i = 0; i < n; ++i) {
    V3<D3> xd{D3(x[3 * i]), D3(x[3 * i + 1]), D3(x[3 * i + 2])};
    xd.x.d[0] = 1; xd.y.d[1] = 1; xd.z.d[2] = 1;
    const D3 r = prims_sdf(o, xd, *prm);
    phi[i] = r.v;
    if (grad)
      for (int a = 0; a < 3; ++a) grad[3 * i + a] = r.d[a];
  }
}

// The three projection parameters t* (Sec. III-A.5) of primitive `k` (an XPSQ)
// at n object-frame points (n x 3).
void orc_xpsq_roots(int32_t h, int32_t k, const Params* prm, int64_t n, const double* x, double* t) {
  const Prim& pr = obj(h).prims.at(size_t(k));
  for (int64_t i = 0; i < n; ++i) xpsq_roots(pr, cvt<double>(x + 3 * i), *prm, t + 3 * i);
}

// meta: n, origin (3), spacing (3); coeffs [4][(n+3)^3] may be null.
void orc_spline(int32_t h, double* meta, double* coeffs) {
  const Spline& sp = obj(h).spl;
  meta[0] = sp.n;
  for (int a = 0; a < 3; ++a) { meta[1 + a] = sp.a[a]; meta[4 + a] = sp.h[a]; }
  if (coeffs)
    for (int c = 0; c < 4; ++c) std::copy(sp.c[c].begin(), sp.c[c].end(), coeffs + size_t(c) * sp.c[c].size());
}

// S2 edge bound of the segment x1 -> x2 against the object's spline grid.
double orc_spline_edge_bound(int32_t h, const double* x1, const double* x2) {
  return spline_edge_bound(obj(h).grid, cvt<double>(x1), cvt<double>(x2));
}

// The spline's phi, normal (n x 3), gradient of phi (n x 3) and Jacobian of the
// normal (n x 9, row a = d n_a / dx) at n points.
void orc_spline_eval(int32_t h, int64_t n, const double* x, double* phi, double* nrm, double* grad, double* jac) {
  const Spline& sp = obj(h).spl;
  typedef Dual<double, 3> D3;
  for (int64_t i = 0; i < n; ++i) {
    V3<D3> xd{D3(x[3 * i]), D3(x[3 * i + 1]), D3(x[3 * i + 2])};
    xd.x.d[0] = 1; xd.y.d[1] = 1; xd.z.d[2] = 1;
    D3 p; V3<D3> nn;
    spline_eval(sp, xd, p, nn);
    phi[i] = p.v;
    const D3* c[3] = {&nn.x, &nn.y, &nn.z};
    for (int a = 0; a < 3; ++a) {
      if (nrm) nrm[3 * i + a] = c[a]->v;
      if (grad) grad[3 * i + a] = p.d[a];
      if (jac) for (int b = 0; b < 3; ++b) jac[9 * i + 3 * a + b] = c[a]->d[b];
    }
  }
}

// Ground truth (phi, n) of Sec. III-B.2 at n points (n x 4).
void orc_ground_truth(int32_t h, int64_t n, const double* x, double* out4) {
  for (int64_t i = 0; i < n; ++i) ground_truth(obj(h), cvt<double>(x + 3 * i), out4 + 4 * i);
}

// The spline fitted to values [4][(n+1)^3] given at the corners of the box
// [a, a + n h] (no object), evaluated at n_pts points: phi, normal spline,
// gradient of phi.
void orc_spline_from_values(int32_t n, const double* a, const double* h, const double* values, int64_t n_pts,
                            const double* x, double* phi, double* nrm, double* grad) {
  Spline sp;
  sp.n = n;
  for (int k = 0; k < 3; ++k) { sp.a[k] = a[k]; sp.h[k] = h[k]; }
  fit_spline(sp, std::vector<double>(values, values + size_t(4) * (n + 1) * (n + 1) * (n + 1)));
  typedef Dual<double, 3> D3;
  for (int64_t i = 0; i < n_pts; ++i) {
    V3<D3> xd{D3(x[3 * i]), D3(x[3 * i + 1]), D3(x[3 * i + 2])};
    xd.x.d[0] = 1; xd.y.d[1] = 1; xd.z.d[2] = 1;
    D3 p; V3<D3> nn;
    spline_eval(sp, xd, p, nn);
    phi[i] = p.v;
    if (nrm) { nrm[3 * i] = nn.x.v; nrm[3 * i + 1] = nn.y.v; nrm[3 * i + 2] = nn.z.v; }
    if (grad) for (int k = 0; k < 3; ++k) grad[3 * i + k] = p.d[k];
  }
}

// The 1-D interpolation operator M [(n+3) x (n+1)].
void orc_spline_operator(int32_t n, double* M) {
  const std::vector<double> m = spline_operator(n);
  std::copy(m.begin(), m.end(), M);
}

// meta: origin[3], h[3], r, n.  G may be null.
void orc_grid(int32_t h, double* G, double* meta) {
  const Grid& g = obj(h).grid;
  for (int a = 0; a < 3; ++a) { meta[a] = g.origin[a]; meta[3 + a] = g.h[a]; }
  meta[6] = g.r; meta[7] = g.n;
  if (G) std::copy(g.G.begin(), g.G.end(), G);
}

double orc_lower_bound(int32_t h, const double* x) { return lower_bound(obj(h).grid, V3<double>{x[0], x[1], x[2]}); }

// phi, grad (n x 3) and Hessian (n x 9) of the object SDF at n points.
void orc_sdf(int32_t h, const Params* prm, int64_t n, const double* x, double* phi, double* grad, double* hess) {
  const Object& o = obj(h);
  for (int64_t i = 0; i < n; ++i) {
    typedef Dual<double, 3> D3;
    V3<D3> xd{D3(x[3 * i]), D3(x[3 * i + 1]), D3(x[3 * i + 2])};
    xd.x.d[0] = 1; xd.y.d[1] = 1; xd.z.d[2] = 1;
    D3 p; V3<D3> g;
    object_sdf(o, xd, *prm, p, g);
    phi[i] = p.v;
    if (grad) { grad[3 * i] = g.x.v; grad[3 * i + 1] = g.y.v; grad[3 * i + 2] = g.z.v; }
    if (hess) {
      const D3* gg[3] = {&g.x, &g.y, &g.z};
      for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) hess[9 * i + 3 * a + b] = gg[a]->d[b];
    }
  }
}

// E-SDF of an edge against the sphere SDF |x - c| - R (generic-SDF check of O6).
void orc_edge_point_sphere(const Params* prm, const double* c, double R, const double* xI, const double* xII,
                           double* pe, double* alpha, double* beta) {
  struct Sphere { V3<double> c; double R;
    double operator()(const V3<double>& x) const { V3<double> d = x - c; return std::sqrt(dot(d, d)) - R; } };
  Sphere s{V3<double>{c[0], c[1], c[2]}, R};
  double a, b;
  V3<double> p = edge_point(s, cvt<double>(xI), cvt<double>(xII), *prm, &a, &b);
  pe[0] = p.x; pe[1] = p.y; pe[2] = p.z; *alpha = a; *beta = b;
}

// E-SDF point of an edge against an object's SDF (object frame); ab
// (nullable) receives the softclipped arc lengths (alpha', beta').
void orc_edge_point(int32_t h, const Params* prm, const double* xI, const double* xII, double* pe, double* ab) {
  SdfFn<double> fn{&obj(h), prm};
  double a = 0, b = 0;
  V3<double> p = edge_point(fn, cvt<double>(xI), cvt<double>(xII), *prm, &a, &b);
  pe[0] = p.x; pe[1] = p.y; pe[2] = p.z;
  if (ab) { ab[0] = a; ab[1] = b; }
}

// Transition f_t and its first two derivatives at phi (hyper-dual).
void orc_transition(const Params* prm, double phi, double* out3) {
  typedef Dual<double, 1> In; typedef Dual<In, 1> HD;
  HD x(0.0); x.v = In(phi); x.v.d[0] = 1.0; x.d[0] = In(1.0);
  HD f = transition(x, *prm);
  out3[0] = f.v.v; out3[1] = f.d[0].v; out3[2] = f.d[0].d[0];
}
// Softclip s_clip(x, a, b) with temperature tau and its derivative in x.
void orc_softclip(double x, double a, double b, double tau, double* out2) {
  typedef Dual<double, 1> D;
  D xd(x); xd.d[0] = 1.0;
  D r = softclip(xd, D(a), D(b), tau);
  out2[0] = r.v; out2[1] = r.d[0];
}

int64_t orc_n_groups(int32_t a, int32_t b) { return int64_t(n_groups(obj(a), obj(b))); }
int64_t orc_n_contacts(int32_t a, int32_t b) { return int64_t(n_contacts(obj(a)) + n_contacts(obj(b))); }

// Forward pass for n pair-queries.  poses: n x 14 = qa(w,x,y,z) ta qb tb.
// groups: [sum groups][12] = p(3) n(3) d q(3) W logZ, queries in order, A's
// pieces first.  contacts (nullable): [sum contacts][13] = mask d_c f w p_c(3)
// n_c(3) phi kind pad, in the same order (A's mesh first; per piece vertices
// then edges).
void orc_contacts(const Params* prm, int64_t n, const int32_t* qa, const int32_t* qb, const double* poses,
                  const int64_t* group_off, const int64_t* contact_off,
                  double* groups, double* contacts, int32_t n_threads) {
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t i = 0; i < n; ++i) {
    const double* ps = poses + 14 * i;
    Pose<double> PA{quat_to_R(ps), V3<double>{ps[4], ps[5], ps[6]}};
    Pose<double> PB{quat_to_R(ps + 7), V3<double>{ps[11], ps[12], ps[13]}};
    std::vector<GroupOut<double>> out;
    std::vector<double> dbg;
    probe_begin(*prm, i, obj(qa[i]), obj(qb[i]));
    query(obj(qa[i]), obj(qb[i]), PA, PB, *prm, out, contacts ? &dbg : nullptr);
    probe_end();
    for (size_t g = 0; g < out.size(); ++g) put(out[g], groups + 12 * (group_off[i] + int64_t(g)));
    if (contacts) std::copy(dbg.begin(), dbg.end(), contacts + 14 * contact_off[i]);
  }
}

// Group outputs of one query at the perturbed pose T(xi) (Rodrigues), for
// finite differences.
void orc_groups_at_xi(const Params* prm, int32_t a, int32_t b, const double* pose, const double* xi, double* groups) {
  M3<double> RA = quat_to_R(pose), RB = quat_to_R(pose + 7);
  Pose<double> PA = perturbed<double>(RA, pose + 4, xi, xi + 3, false);
  Pose<double> PB = perturbed<double>(RB, pose + 11, xi + 6, xi + 9, false);
  std::vector<GroupOut<double>> out;
  query(obj(a), obj(b), PA, PB, *prm, out, nullptr);
  for (size_t g = 0; g < out.size(); ++g) put(out[g], groups + 12 * g);
}

// Jacobian-vector product of the group records: y and dy/dxi . dir at xi = 0
// (one tangent slot seeded with dir; first derivatives of I + W + W^2/2 at
// zero are those of the exponential).  groups, tangents: [sum groups][12].
void orc_jvp(const Params* prm, int64_t n, const int32_t* qa, const int32_t* qb, const double* poses,
             const int64_t* group_off, const double* dir, double* groups, double* tangents, int32_t n_threads) {
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t i = 0; i < n; ++i) {
    const double* ps = poses + 14 * i;
    M3<double> RA = quat_to_R(ps), RB = quat_to_R(ps + 7);
    typedef Dual<double, 1> D;
    D xi[12];
    for (int k = 0; k < 12; ++k) { xi[k] = D(0.0); xi[k].d[0] = dir[12 * i + k]; }
    Pose<D> PA = perturbed<D>(RA, ps + 4, xi, xi + 3, true);
    Pose<D> PB = perturbed<D>(RB, ps + 11, xi + 6, xi + 9, true);
    std::vector<GroupOut<D>> out;
    probe_begin(*prm, i, obj(qa[i]), obj(qb[i]));
    query(obj(qa[i]), obj(qb[i]), PA, PB, *prm, out, nullptr);
    probe_end();
    for (size_t g = 0; g < out.size(); ++g)
      for (int k = 0; k < 12; ++k) {
        const D& c = comp(out[g], k);
        groups[12 * (group_off[i] + int64_t(g)) + k] = c.v;
        tangents[12 * (group_off[i] + int64_t(g)) + k] = c.d[0];
      }
  }
}

// Isosurface projection (Sec. IV-A, last paragraph): each group's point
// p_in[g] (world) moved onto the zero level set of the SDF it was evaluated
// against, proj(p) = p - phi(p) n(p) in that object's frame (A's groups
// against B's SDF, B's against A's).  points: [sum groups][3].
void orc_project(const Params* prm, int64_t n, const int32_t* qa, const int32_t* qb, const double* poses,
                 const int64_t* group_off, const double* p_in, double* p_out, int32_t n_threads) {
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t i = 0; i < n; ++i) {
    const double* ps = poses + 14 * i;
    const Object& A = obj(qa[i]);
    const Object& B = obj(qb[i]);
    for (int64_t g = group_off[i]; g < group_off[i + 1]; ++g) {
      const bool a_side = g - group_off[i] < int64_t(A.pieces.size());
      const Object& S = a_side ? B : A;
      const double* qs = a_side ? ps + 7 : ps;
      const M3<double> R = quat_to_R(qs);
      const V3<double> t{qs[4], qs[5], qs[6]};
      const V3<double> x = mulT(R, cvt<double>(p_in + 3 * g) - t);
      double phi;
      V3<double> nS;
      object_phi_normal(S, x, *prm, phi, nS);
      const V3<double> pw = mul(R, x - nS * phi) + t;
      p_out[3 * g] = pw.x; p_out[3 * g + 1] = pw.y; p_out[3 * g + 2] = pw.z;
    }
  }
}

// Gradient of L = <c, y> w.r.t. xi = (w_A, v_A, w_B, v_B) at xi = 0 and,
// when dir != null, the Hessian-vector product H dir, by hyper-dual numbers.
void orc_grad_hvp(const Params* prm, int64_t n, const int32_t* qa, const int32_t* qb, const double* poses,
                  const int64_t* group_off, const double* cot, const double* dir,
                  double* grad, double* hv, int32_t n_threads) {
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t i = 0; i < n; ++i) {
    const double* ps = poses + 14 * i;
    M3<double> RA = quat_to_R(ps), RB = quat_to_R(ps + 7);
    const double* c = cot + 12 * group_off[i];
    if (dir) {
      typedef Dual<double, 1> In;
      typedef Dual<In, 12> HD;
      HD xi[12];
      for (int k = 0; k < 12; ++k) {
        xi[k] = HD(0.0);
        xi[k].v.d[0] = dir[12 * i + k];
        xi[k].d[k] = In(1.0);
      }
      Pose<HD> PA = perturbed<HD>(RA, ps + 4, xi, xi + 3, true);
      Pose<HD> PB = perturbed<HD>(RB, ps + 11, xi + 6, xi + 9, true);
      std::vector<GroupOut<HD>> out;
      probe_begin(*prm, i, obj(qa[i]), obj(qb[i]));
      query(obj(qa[i]), obj(qb[i]), PA, PB, *prm, out, nullptr);
      probe_end();
      HD L(0.0);
      for (size_t g = 0; g < out.size(); ++g)
        for (int k = 0; k < 12; ++k) L += comp(out[g], k) * c[12 * g + k];
      for (int k = 0; k < 12; ++k) {
        grad[12 * i + k] = L.d[k].v;
        hv[12 * i + k] = L.d[k].d[0];
      }
    } else {
      typedef Dual<double, 12> D;
      D xi[12];
      for (int k = 0; k < 12; ++k) { xi[k] = D(0.0); xi[k].d[k] = 1.0; }
      Pose<D> PA = perturbed<D>(RA, ps + 4, xi, xi + 3, true);
      Pose<D> PB = perturbed<D>(RB, ps + 11, xi + 6, xi + 9, true);
      std::vector<GroupOut<D>> out;
      probe_begin(*prm, i, obj(qa[i]), obj(qb[i]));
      query(obj(qa[i]), obj(qb[i]), PA, PB, *prm, out, nullptr);
      probe_end();
      D L(0.0);
      for (size_t g = 0; g < out.size(); ++g)
        for (int k = 0; k < 12; ++k) L += comp(out[g], k) * c[12 * g + k];
      for (int k = 0; k < 12; ++k) grad[12 * i + k] = L.d[k];
    }
  }
}

}  // extern "C"
