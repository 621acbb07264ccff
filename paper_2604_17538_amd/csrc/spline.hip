// Fit of the cubic-spline SDF representation (Sec. III-B) on gfx950, in FP64:
//   k_spline_gt     ground-truth SDF and normal of the object (the union of
//                   its convex pieces) at the (n + 1)^3 corners of its grid box
//   k_spline_solve  natural cubic-spline coefficients along one axis (three
//                   passes, z then y then x: the tensor-product interpolant)
//   k_spline_pack   float4 coefficients (phi, n_x, n_y, n_z) into the object,
//                   and per cell the B-spline convex-hull bound of phi
// Runs once per object at registration; queries then only gather coefficients.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cm {

// Exact SDF of a convex piece at x and the unit direction of the closest
// surface point (inside: the nearest facet's outward normal; outside:
// (x - proj(x)) / |x - proj(x)|).  Outside, the closest point of a convex
// polytope lies inside a facet (the orthogonal projection onto that facet's
// plane, which then satisfies every other plane) or on a feature edge, so the
// distance is the least over the valid facet projections and the edge segments.
__device__ static double piece_exact64(const SplJob& jb, int k, const double x[3], double nrm[3]) {
  const int4 pd = jb.pieces[k];  // plane begin, plane count, edge begin, edge count
  const double* pl = jb.planes + 4 * int64_t(pd.x);
  double m = -1e300;
  int jm = 0;
  for (int j = 0; j < pd.y; ++j) {
    const double a = pl[4 * j] * x[0] + pl[4 * j + 1] * x[1] + pl[4 * j + 2] * x[2] + pl[4 * j + 3];
    if (a > m) { m = a; jm = j; }
  }
  if (m <= 0.0) {
    for (int c = 0; c < 3; ++c) nrm[c] = pl[4 * jm + c];
    return m;
  }
  double best = 1e300;
  const double* sg = jb.segs + 6 * int64_t(pd.z);
  for (int e = 0; e < pd.w; ++e) {
    const double* s = sg + 6 * e;
    const double d[3] = {s[3] - s[0], s[4] - s[1], s[5] - s[2]};
    const double r[3] = {x[0] - s[0], x[1] - s[1], x[2] - s[2]};
    const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double t = dd > 0.0 ? (r[0] * d[0] + r[1] * d[1] + r[2] * d[2]) / dd : 0.0;
    t = fmin(1.0, fmax(0.0, t));
    const double q[3] = {r[0] - t * d[0], r[1] - t * d[1], r[2] - t * d[2]};
    const double dist = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    if (dist < best) {
      best = dist;
      for (int c = 0; c < 3; ++c) nrm[c] = q[c] / dist;
    }
  }
  for (int j = 0; j < pd.y; ++j) {
    const double a = pl[4 * j] * x[0] + pl[4 * j + 1] * x[1] + pl[4 * j + 2] * x[2] + pl[4 * j + 3];
    if (!(a > 0.0) || !(a < best)) continue;
    const double y[3] = {x[0] - a * pl[4 * j], x[1] - a * pl[4 * j + 1], x[2] - a * pl[4 * j + 2]};
    // (the facet's own plane passes through y; the others without tolerance: a
    // projection just outside the facet is left to the edges, whose closest
    // points are exact, since accepting it would tilt the normal of a point
    // near the surface by (excess) / (distance))
    bool inside = true;
    for (int i = 0; i < pd.y && inside; ++i)
      inside = i == j || pl[4 * i] * y[0] + pl[4 * i + 1] * y[1] + pl[4 * i + 2] * y[2] + pl[4 * i + 3] <= 0.0;
    if (inside) {
      best = a;
      for (int c = 0; c < 3; ++c) nrm[c] = pl[4 * j + c];
    }
  }
  return best;
}

// Ground truth (Sec. III-B.2) at the corners: phi = min over pieces, the
// normal of the minimising piece.  out: [4][n + 1]^3 (phi, n_x, n_y, n_z).
__global__ __launch_bounds__(256) void k_spline_gt(const SplJob* __restrict__ jobs, int n, double* __restrict__ work,
                                                   int64_t work_stride) {
  const SplJob jb = jobs[blockIdx.y];
  const int n1 = n + 1;
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nc = int64_t(n1) * n1 * n1;
  if (c >= nc) return;
  const int i = int(c / (int64_t(n1) * n1)), j = int((c / n1) % n1), k = int(c % n1);
  const double x[3] = {jb.org[0] + i * jb.h[0], jb.org[1] + j * jb.h[1], jb.org[2] + k * jb.h[2]};
  double phi = 1e300, nrm[3] = {0.0, 0.0, 0.0};
  for (int p = 0; p < jb.n_pieces; ++p) {
    double nk[3];
    const double v = piece_exact64(jb, p, x, nk);
    if (v < phi) {
      phi = v;
      nrm[0] = nk[0]; nrm[1] = nk[1]; nrm[2] = nk[2];
    }
  }
  double* out = work + int64_t(blockIdx.y) * work_stride;
  out[c] = phi;
  out[nc + c] = nrm[0];
  out[2 * nc + c] = nrm[1];
  out[3 * nc + c] = nrm[2];
}

// One axis of the fit: every line of n + 1 values becomes n + 3 coefficients of
// s(t) = sum_m c_m u(t - m + 1) (u of Sec. III-B.1; t in cells) with natural end
// conditions.  Interpolation at node i reads c_i + 4 c_{i+1} + c_{i+2} = f_i, and
// s'' = 0 at both ends reads c_0 - 2 c_1 + c_2 = 0 = c_n - 2 c_{n+1} + c_{n+2}, so
// c_1 = f_0 / 6, c_{n+1} = f_n / 6, the inner c_2..c_n solve a (1, 4, 1)
// tridiagonal system (Thomas algorithm) and the end coefficients follow.
// Pass 0 (z): [4][n1][n1][n1] -> [4][n1][n1][m]; pass 1 (y): -> [4][n1][m][m];
// pass 2 (x): -> [4][m][m][m], with n1 = n + 1 and m = n + 3.
__global__ __launch_bounds__(256) void k_spline_solve(int pass, int n, const double* __restrict__ in_all,
                                                      double* __restrict__ out_all, int64_t work_stride) {
  __shared__ double cp[130];
  const int n1 = n + 1, m = n + 3, K = n - 1;
  if (threadIdx.x == 0) {
    double prev = 0.0;
    for (int i = 0; i < K; ++i) { prev = 1.0 / (4.0 - prev); cp[i] = prev; }
  }
  __syncthreads();
  // lines per field: pass 0: n1 * n1, pass 1: n1 * m, pass 2: m * m
  const int64_t per = pass == 0 ? int64_t(n1) * n1 : (pass == 1 ? int64_t(n1) * m : int64_t(m) * m);
  const int64_t l = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (l >= 4 * per) return;
  const int c = int(l / per);
  const int64_t r = l % per;
  const double* in = in_all + int64_t(blockIdx.y) * work_stride;
  double* out = out_all + int64_t(blockIdx.y) * work_stride;
  int64_t ib, is, ob, os;
  if (pass == 0) {  // line (i, j) along k
    ib = (int64_t(c) * n1 * n1 + r) * n1; is = 1;
    ob = (int64_t(c) * n1 * n1 + r) * m;  os = 1;
  } else if (pass == 1) {  // line (i, r) along j
    const int64_t i = r / m, q = r % m;
    ib = (int64_t(c) * n1 + i) * n1 * m + q; is = m;
    ob = (int64_t(c) * n1 + i) * m * m + q;  os = m;
  } else {  // line (q, r) along i
    ib = int64_t(c) * n1 * m * m + r; is = int64_t(m) * m;
    ob = int64_t(c) * m * m * m + r;  os = int64_t(m) * m;
  }
  auto f = [&](int t) { return in[ib + is * t]; };
  auto C = [&](int t) -> double& { return out[ob + os * t]; };
  const double c1 = f(0) / 6.0, cn1 = f(n) / 6.0;
  C(1) = c1;
  C(n + 1) = cn1;
  // forward elimination into C(2..n), then back substitution
  double dprev = 0.0;
  for (int i = 0; i < K; ++i) {
    double rhs = f(i + 1);
    if (i == 0) rhs -= c1;
    if (i == K - 1) rhs -= cn1;
    dprev = (rhs - dprev) * cp[i];
    C(i + 2) = dprev;
  }
  for (int i = K - 2; i >= 0; --i) C(i + 2) = C(i + 2) - cp[i] * C(i + 3);
  C(0) = 2.0 * c1 - C(2);
  C(n + 2) = 2.0 * cn1 - C(n);
}

// float4 coefficients into the object, and per cell 216 times the least phi
// coefficient the cell reaches (the three 1-D bases of a cell are >= 0 and
// each sums to 6: the spline is 216 times a convex combination of them).
__global__ __launch_bounds__(256) void k_spline_pack(const SplJob* __restrict__ jobs, int n,
                                                     const double* __restrict__ coef_all, int64_t work_stride) {
  const SplJob jb = jobs[blockIdx.y];
  const int m = n + 3;
  const int64_t m3 = int64_t(m) * m * m, n3 = int64_t(n) * n * n;
  const double* C = coef_all + int64_t(blockIdx.y) * work_stride;
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < m3) jb.coef[v] = F4{float(C[v]), float(C[m3 + v]), float(C[2 * m3 + v]), float(C[3 * m3 + v])};
  if (v < n3) {
    const int i = int(v / (int64_t(n) * n)), j = int((v / n) % n), k = int(v % n);
    double lo = 1e300;
    for (int p = 0; p < 4; ++p)
      for (int q = 0; q < 4; ++q)
        for (int r = 0; r < 4; ++r) lo = fmin(lo, C[(int64_t(i + p) * m + (j + q)) * m + (k + r)]);
    jb.grid[v] = float(216.0 * lo);
  }
}

hipError_t launch_spline_build(const SplJob* d_jobs, int n_jobs, int n, double* work_a, double* work_b,
                               int64_t work_stride, hipStream_t s) {
  const int n1 = n + 1, m = n + 3;
  const int64_t nc = int64_t(n1) * n1 * n1;
  hipLaunchKernelGGL(k_spline_gt, dim3(unsigned((nc + 255) / 256), unsigned(n_jobs)), dim3(256), 0, s, d_jobs, n,
                     work_a, work_stride);
  const int64_t lines[3] = {4 * int64_t(n1) * n1, 4 * int64_t(n1) * m, 4 * int64_t(m) * m};
  double* in = work_a;
  double* out = work_b;
  for (int pass = 0; pass < 3; ++pass) {
    hipLaunchKernelGGL(k_spline_solve, dim3(unsigned((lines[pass] + 255) / 256), unsigned(n_jobs)), dim3(256), 0, s,
                       pass, n, in, out, work_stride);
    double* t = in; in = out; out = t;
  }
  const int64_t m3 = int64_t(m) * m * m;
  hipLaunchKernelGGL(k_spline_pack, dim3(unsigned((m3 + 255) / 256), unsigned(n_jobs)), dim3(256), 0, s, d_jobs, n,
                     in, work_stride);
  return hipGetLastError();
}

}  // namespace cm
