// Device math for the gfx950 kernels: scalars (float and forward-mode dual
// floats), 3-vectors, symmetric 3x3 matrices, rotations, the smooth operators of
// Sec. II and the SDF of a union of convex pieces (Sec. III-A.2/3).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace cm {

#define CM_DEV __device__ __forceinline__

constexpr float kLn2 = 0.69314718055994530942f;
constexpr float kLog2e = 1.44269504088896340736f;

// ------------------------------------------------------------------ scalars --
// Dual float: value and one directional derivative.
struct df {
  float v, t;
};
CM_DEV float val(float x) { return x; }
CM_DEV float val(df x) { return x.v; }
CM_DEV float tan_(float) { return 0.f; }
CM_DEV float tan_(df x) { return x.t; }
template <class T> CM_DEV T cst(float c);
template <> CM_DEV float cst<float>(float c) { return c; }
template <> CM_DEV df cst<df>(float c) { return df{c, 0.f}; }
CM_DEV df mkd(float v, float t) { return df{v, t}; }

CM_DEV df operator+(df a, df b) { return {a.v + b.v, a.t + b.t}; }
CM_DEV df operator-(df a, df b) { return {a.v - b.v, a.t - b.t}; }
CM_DEV df operator-(df a) { return {-a.v, -a.t}; }
CM_DEV df operator*(df a, df b) { return {a.v * b.v, fmaf(a.v, b.t, a.t * b.v)}; }
CM_DEV df operator+(df a, float b) { return {a.v + b, a.t}; }
CM_DEV df operator+(float b, df a) { return {a.v + b, a.t}; }
CM_DEV df operator-(df a, float b) { return {a.v - b, a.t}; }
CM_DEV df operator-(float b, df a) { return {b - a.v, -a.t}; }
CM_DEV df operator*(df a, float b) { return {a.v * b, a.t * b}; }
CM_DEV df operator*(float b, df a) { return {a.v * b, a.t * b}; }
CM_DEV df operator/(df a, df b) {
  float r = 1.f / b.v;
  float q = a.v * r;
  return {q, (a.t - q * b.t) * r};
}
CM_DEV df operator/(df a, float b) { float r = 1.f / b; return {a.v * r, a.t * r}; }
CM_DEV df operator/(float a, df b) { float r = 1.f / b.v; float q = a * r; return {q, -q * b.t * r}; }
CM_DEV df& operator+=(df& a, df b) { a = a + b; return a; }
CM_DEV df& operator-=(df& a, df b) { a = a - b; return a; }
CM_DEV df fmaT(df a, df b, df c) { return {fmaf(a.v, b.v, c.v), fmaf(a.v, b.t, fmaf(a.t, b.v, c.t))}; }
CM_DEV float fmaT(float a, float b, float c) { return fmaf(a, b, c); }
CM_DEV df fmaT(float a, df b, df c) { return {fmaf(a, b.v, c.v), fmaf(a, b.t, c.t)}; }

// Hardware base-2 exponential / logarithm (v_exp_f32, v_log_f32).
CM_DEV float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
CM_DEV float lg2(float x) { return __builtin_amdgcn_logf(x); }
CM_DEV df ex2(df a) { float e = ex2(a.v); return {e, e * a.t * kLn2}; }
CM_DEV df lg2(df a) { return {lg2(a.v), a.t / (a.v * kLn2)}; }
CM_DEV float sqrtT(float x) { return sqrtf(x); }
CM_DEV df sqrtT(df a) { float s = sqrtf(a.v); return {s, 0.5f * a.t / s}; }
CM_DEV float expT(float x) { return expf(x); }
CM_DEV df expT(df a) { float e = expf(a.v); return {e, e * a.t}; }
CM_DEV float log1pT(float x) { return log1pf(x); }
CM_DEV df log1pT(df a) { return {log1pf(a.v), a.t / (1.f + a.v)}; }
CM_DEV float logT(float x) { return logf(x); }
CM_DEV df logT(df a) { return {logf(a.v), a.t / a.v}; }

// ------------------------------------------------------------------ vectors --
template <class T> struct V3 { T x, y, z; };
template <class T> CM_DEV V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> CM_DEV V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T, class S> CM_DEV V3<T> operator*(V3<T> a, S s) { return {a.x * s, a.y * s, a.z * s}; }
template <class T> CM_DEV T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> CM_DEV V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
template <class T> CM_DEV V3<T> zero3() { return {cst<T>(0.f), cst<T>(0.f), cst<T>(0.f)}; }
template <class T> CM_DEV V3<T> lift3(V3<float> a) { return {cst<T>(a.x), cst<T>(a.y), cst<T>(a.z)}; }
template <class T> CM_DEV V3<float> val3(V3<T> a) { return {val(a.x), val(a.y), val(a.z)}; }
// mixed: dual vector with constant vector
CM_DEV V3<df> operator+(V3<df> a, V3<float> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
CM_DEV V3<df> operator-(V3<df> a, V3<float> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }

// Symmetric 3x3: xx, yy, zz, xy, xz, yz.
template <class T> struct Sym { T xx, yy, zz, xy, xz, yz; };
template <class T> CM_DEV Sym<T> zsym() { T z = cst<T>(0.f); return {z, z, z, z, z, z}; }
template <class T> CM_DEV V3<T> mulS(const Sym<T>& S, V3<T> v) {
  return {S.xx * v.x + S.xy * v.y + S.xz * v.z, S.xy * v.x + S.yy * v.y + S.yz * v.z,
          S.xz * v.x + S.yz * v.y + S.zz * v.z}; }

// Rotation matrix (row-major) of a quaternion (w, x, y, z), normalised first.
template <class T> struct M3 { T m[9]; };
template <class T> CM_DEV V3<T> mulM(const M3<T>& R, V3<T> v) {
  return {R.m[0] * v.x + R.m[1] * v.y + R.m[2] * v.z, R.m[3] * v.x + R.m[4] * v.y + R.m[5] * v.z,
          R.m[6] * v.x + R.m[7] * v.y + R.m[8] * v.z}; }
template <class T> CM_DEV V3<T> mulMT(const M3<T>& R, V3<T> v) {
  return {R.m[0] * v.x + R.m[3] * v.y + R.m[6] * v.z, R.m[1] * v.x + R.m[4] * v.y + R.m[7] * v.z,
          R.m[2] * v.x + R.m[5] * v.y + R.m[8] * v.z}; }
template <class T> CM_DEV M3<T> mulMTM(const M3<T>& A, const M3<T>& B) {  // A^T B
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.m[3 * i + j] = A.m[i] * B.m[j] + A.m[3 + i] * B.m[3 + j] + A.m[6 + i] * B.m[6 + j];
  return C;
}
CM_DEV M3<float> quat_R(const float* q) {
  float n = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  float w = q[0] * n, x = q[1] * n, y = q[2] * n, z = q[3] * n;
  M3<float> R;
  R.m[0] = 1.f - 2.f * (y * y + z * z); R.m[1] = 2.f * (x * y - w * z); R.m[2] = 2.f * (x * z + w * y);
  R.m[3] = 2.f * (x * y + w * z); R.m[4] = 1.f - 2.f * (x * x + z * z); R.m[5] = 2.f * (y * z - w * x);
  R.m[6] = 2.f * (x * z - w * y); R.m[7] = 2.f * (y * z + w * x); R.m[8] = 1.f - 2.f * (x * x + y * y);
  return R;
}

// Both bodies' rotations and the mesh -> SDF-frame transform of one direction
// of a query, formed in FP64 and rounded once to FP32: R_M, R_S, R_rel =
// R_S^T R_M and t_rel = R_S^T (t_M - t_S).  In FP32 each entry would be rounded
// several times (normalisation, products, the composition), and position
// errors reach the second derivatives amplified by 1 / tau.
struct Frame32 {
  float RM[9], RS[9], Rrel[9], tM[3], tS[3], trel[3];
};
CM_DEV void quat_R64(const float* q, double* R) {
  const double w0 = q[0], x0 = q[1], y0 = q[2], z0 = q[3];
  const double n = 1.0 / sqrt(w0 * w0 + x0 * x0 + y0 * y0 + z0 * z0);
  const double w = w0 * n, x = x0 * n, y = y0 * n, z = z0 * n;
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}
CM_DEV Frame32 frame32(const float* qM, const float* tM, const float* qS, const float* tS) {
  double RM[9], RS[9];
  quat_R64(qM, RM);
  quat_R64(qS, RS);
  Frame32 f;
  for (int i = 0; i < 9; ++i) { f.RM[i] = float(RM[i]); f.RS[i] = float(RS[i]); }
  const double d[3] = {double(tM[0]) - double(tS[0]), double(tM[1]) - double(tS[1]), double(tM[2]) - double(tS[2])};
  for (int i = 0; i < 3; ++i) {
    f.tM[i] = tM[i];
    f.tS[i] = tS[i];
    f.trel[i] = float(RS[i] * d[0] + RS[3 + i] * d[1] + RS[6 + i] * d[2]);
    for (int j = 0; j < 3; ++j)
      f.Rrel[3 * i + j] = float(RS[i] * RM[j] + RS[3 + i] * RM[3 + j] + RS[6 + i] * RM[6 + j]);
  }
  return f;
}

// --------------------------------------------------------- smooth operators --
// sigma(z) = 1 / (1 + exp(-z))  (Sec. II)
template <class T> CM_DEV T sigmoidT(T z) {
  T e = expT(-z);
  return cst<T>(1.f) / (e + 1.f);
}
CM_DEV float sigmoidT(float z) { return 1.f / (1.f + expf(-z)); }
// dual: sigma' = sigma (1 - sigma) (no overflow of exp(-z) into the tangent)
CM_DEV df sigmoidT(df z) {
  const float s = sigmoidT(z.v);
  return {s, s * (1.f - s) * z.t};
}
// s_+(x) = tau log(1 + exp(x / tau)) = max(x, 0) + tau log1p(exp(-|x| / tau))  (Sec. II)
template <class T> CM_DEV T softplusT(T x, float tau, float inv_tau) {
  if (val(x) >= 0.f) return x + tau * log1pT(expT(-x * inv_tau));
  return tau * log1pT(expT(x * inv_tau));
}
// s_clip(x, 0, L) = s_+(x) - s_+(x - L)  (Sec. II)
template <class T> CM_DEV T softclip0T(T x, T L, float tau, float inv_tau) {
  return softplusT(x, tau, inv_tau) - softplusT(x - L, tau, inv_tau);
}
// C2 transition f_t: quintic smoothstep of s = clamp((d_max - phi)/eps_t, 0, 1)  (Sec. IV-C.1)
template <class T> CM_DEV T transitionT(T phi, const DevParams& P) {
  T s = (P.d_max - phi) * P.inv_eps_t;
  if (val(s) <= 0.f) return cst<T>(0.f);
  if (val(s) >= 1.f) return cst<T>(1.f);
  return s * s * s * (10.f - 15.f * s + 6.f * s * s);
}

// ----------------------------------------------------------------- loads --
// Plane data is read with wave-uniform addresses; going through the constant
// address space lets the compiler use scalar (SMEM) loads into SGPRs.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(4))) const v4i* cv4p;
template <class T> CM_DEV T ldc(const T* p) {
  static_assert(sizeof(T) % 16 == 0, "ldc needs a multiple of 16 bytes");
  T r;
  cv4p s = (cv4p)p;
#pragma unroll
  for (int i = 0; i < int(sizeof(T) / 16); ++i) {
    const v4i w = s[i];
    __builtin_memcpy(reinterpret_cast<char*>(&r) + 16 * i, &w, 16);
  }
  return r;
}

// --------------------------------------------------------------- the SDF --
// Result of an SDF evaluation: phi, grad phi and (MODE 2) the Hessian.
template <class T> struct SdfRes {
  T phi;
  V3<T> g;
  Sym<T> H;
};

template <class T> struct IsDual { static constexpr bool value = false; };
template <> struct IsDual<df> { static constexpr bool value = true; };

// dot of a scaled plane (kappa n, kappa h) with a point relative to the piece centre
CM_DEV float pdot(const F4& q, V3<float> x) { return fmaf(q.x, x.x, fmaf(q.y, x.y, fmaf(q.z, x.z, q.w))); }
CM_DEV df pdot(const F4& q, V3<df> x) {
  return {fmaf(q.x, x.x.v, fmaf(q.y, x.y.v, fmaf(q.z, x.z.v, q.w))), fmaf(q.x, x.x.t, fmaf(q.y, x.y.t, q.z * x.z.t))};
}

// The same dots for a block of 4 consecutive planes at every lane's point, on
// the matrix cores (v_mfma_f32_4x4x1_16b_f32: 16 blocks of 4 lanes, result i
// of lane l = A(lane 4 (l / 4) + i) B(l) + C_i).  Lane l supplies plane l & 3
// of the block as A and its own point as B, so result i is plane i at the
// lane's point.  Accumulated in the order w, z, y, x, one rounding per step,
// the values are those of pdot bit for bit (up to the sign of a zero).  The
// operands are read across lanes: every lane of the wave executes these.
typedef float f4v __attribute__((ext_vector_type(4)));
CM_DEV f4v mdot(const F4& ql, V3<float> x) {
  f4v a = {0.f, 0.f, 0.f, 0.f};
  a = __builtin_amdgcn_mfma_f32_4x4x1f32(ql.w, 1.f, a, 0, 0, 0);
  a = __builtin_amdgcn_mfma_f32_4x4x1f32(ql.z, x.z, a, 0, 0, 0);
  a = __builtin_amdgcn_mfma_f32_4x4x1f32(ql.y, x.y, a, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_4x4x1f32(ql.x, x.x, a, 0, 0, 0);
}
// kappa n . t for a tangent t (the dual part of pdot)
CM_DEV f4v mdot_n(const F4& ql, V3<float> t) {
  f4v a = {0.f, 0.f, 0.f, 0.f};
  a = __builtin_amdgcn_mfma_f32_4x4x1f32(ql.z, t.z, a, 0, 0, 0);
  a = __builtin_amdgcn_mfma_f32_4x4x1f32(ql.y, t.y, a, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_4x4x1f32(ql.x, t.x, a, 0, 0, 0);
}
// this lane's plane of the block q[j .. j + 3] (the last plane repeated past n),
// read through the global address space (plane data lives in device memory)
typedef __attribute__((address_space(1))) const v4i* gv4p;
CM_DEV F4 blk_plane(const F4* q, int j, int n) {
  const v4i w = ((gv4p)q)[min(j + (int(threadIdx.x) & 3), n - 1)];
  F4 r;
  __builtin_memcpy(&r, &w, 16);
  return r;
}
// this lane's plane of the block q[j .. j + 3] of a piece stored in whole groups
CM_DEV F4 grp_plane(const F4* q, int j) {
  const v4i w = ((gv4p)q)[j + (int(threadIdx.x) & 3)];
  F4 r;
  __builtin_memcpy(&r, &w, 16);
  return r;
}
// plane values of a block at NP points: value and (dual scalars) tangent
template <int NP, class T>
CM_DEV void blk_vals(const F4& ql, const V3<T>* xl, f4v* av, f4v* at) {
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    av[p] = mdot(ql, val3(xl[p]));
    if (IsDual<T>::value) at[p] = mdot_n(ql, V3<float>{tan_(xl[p].x), tan_(xl[p].y), tan_(xl[p].z)});
  }
}
// the same dots with a per-point constant c added first (c = -shift: the
// exponent a - m comes out of the chain, accumulated as (h + c) + z + y + x)
CM_DEV f4v mdot_c(const F4& ql, V3<float> x, const f4v& c) {
  f4v a = __builtin_amdgcn_mfma_f32_4x4x1f32(ql.w, 1.f, c, 0, 0, 0);
  a = __builtin_amdgcn_mfma_f32_4x4x1f32(ql.z, x.z, a, 0, 0, 0);
  a = __builtin_amdgcn_mfma_f32_4x4x1f32(ql.y, x.y, a, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_4x4x1f32(ql.x, x.x, a, 0, 0, 0);
}
// plane values of a block at NP points; with dual numbers already shifted,
// a - m (nm: -m per point in all 4 slots), and their tangents (xt: ln 2 times
// the points' tangents, so that the tangent of 2^(a - m) is 2^(a - m) times the
// block's dot directly)
template <int NP, bool DUAL>
CM_DEV void blk_vals_t(const F4& ql, const V3<float>* x0, const f4v* nm, const V3<float>* xt, f4v* av,
                       f4v* at) {
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    if (DUAL) {
      av[p] = mdot_c(ql, x0[p], nm[p]);
      at[p] = mdot_n(ql, xt[p]);
    } else {
      av[p] = mdot(ql, x0[p]);  // float sweeps: shift on the VALU (fewer registers)
    }
  }
}
// Order-preserving bits of a float (as unsigned: a < b iff bits(a) < bits(b)
// for non-NaN a, b); never all ones for a float.
CM_DEV uint32_t ord_bits(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
// Least value over the wave (every lane active): within rows of 16 lanes by
// DPP exchanges (quad swaps, half-row and row mirrors), then over the 4 rows.
CM_DEV uint32_t dpp_min(uint32_t v, int ctrl) {
  switch (ctrl) {  // (the DPP control must be a constant)
    case 0: return min(v, uint32_t(__builtin_amdgcn_mov_dpp(int(v), 0xB1, 0xf, 0xf, false)));   // quad [1,0,3,2]
    case 1: return min(v, uint32_t(__builtin_amdgcn_mov_dpp(int(v), 0x4E, 0xf, 0xf, false)));   // quad [2,3,0,1]
    case 2: return min(v, uint32_t(__builtin_amdgcn_mov_dpp(int(v), 0x141, 0xf, 0xf, false)));  // row half mirror
    default: return min(v, uint32_t(__builtin_amdgcn_mov_dpp(int(v), 0x140, 0xf, 0xf, false))); // row mirror
  }
}
CM_DEV uint32_t wave_umin(uint32_t v) {
  v = dpp_min(v, 0);
  v = dpp_min(v, 1);
  v = dpp_min(v, 2);
  v = dpp_min(v, 3);
  const uint32_t a = uint32_t(__builtin_amdgcn_readlane(int(v), 0));
  const uint32_t b = uint32_t(__builtin_amdgcn_readlane(int(v), 16));
  const uint32_t c = uint32_t(__builtin_amdgcn_readlane(int(v), 32));
  const uint32_t d = uint32_t(__builtin_amdgcn_readlane(int(v), 48));
  return min(min(a, b), min(c, d));
}

template <class T> CM_DEV T mkT(float v, float t);
template <> CM_DEV float mkT<float>(float v, float) { return v; }
template <> CM_DEV df mkT<df>(float v, float t) { return df{v, t}; }

// SDF of a union of convex pieces at NP points per lane (Sec. III-A.2/3):
//   phi_k = tau_cap LSE_j (n_kj . x + h_kj)          smooth intersection
//   phi   = -tau_cup LSE_k (-phi_k)                  smooth union
// Per piece, one pass finds the max plane value (the LSE shift), a second pass
// accumulates sum exp2 and the weighted normal sums.  Pieces are combined
// online with a running minimum.  MODE 0: phi; 1: + gradient; 2: + Hessian.
//
// Pieces that cannot matter at any of the wave's points are skipped (when
// P.prune): a piece's SDF is at least the max over its support subset of
// planes, and the union's minimum is at most min_k (|x - c_k| + ub_off_k) and at
// most the least piece SDF evaluated so far (the running minimum M).  A piece
// whose lower bound exceeds the smaller of the two by prune_margin = 20 tau_cup
// has union weight below e^-20 < 2^-28 relative to the sum, under FP32
// resolution.
//
// The Hessian is (1/tau_cap) sum_k u_k Cov_k(n) - (1/tau_cup) Cov_u(g_k), two
// weighted covariances.  Expanded as E[n n^T] - g g^T they cancel terms of size
// 1/tau down to results that can be many times smaller (a point in the face
// region of a piece), which costs FP32 most of its digits; the same happens to
// the tangent of the gradient with dual scalars.  Whenever second-order
// quantities are formed (MODE 2, or dual scalars), the covariances are therefore
// accumulated without that cancellation: the normals of a piece relative to
// the normal of its max plane, and the piece gradients with a weighted Welford
// update of their running mean.
template <class T, class S> CM_DEV Sym<T> operator*(const Sym<T>& a, S s) {
  return {a.xx * s, a.yy * s, a.zz * s, a.xy * s, a.xz * s, a.yz * s}; }
template <class T> CM_DEV Sym<T> operator+(const Sym<T>& a, const Sym<T>& b) {
  return {a.xx + b.xx, a.yy + b.yy, a.zz + b.zz, a.xy + b.xy, a.xz + b.xz, a.yz + b.yz}; }
template <class T> CM_DEV Sym<T> operator-(const Sym<T>& a, const Sym<T>& b) {
  return {a.xx - b.xx, a.yy - b.yy, a.zz - b.zz, a.xy - b.xy, a.xz - b.xz, a.yz - b.yz}; }
template <class T> CM_DEV Sym<T> outer(V3<T> a) {
  return {a.x * a.x, a.y * a.y, a.z * a.z, a.x * a.y, a.x * a.z, a.y * a.z}; }

template <int NP, int MODE, class T>
CM_DEV void sdf_eval(const ObjDesc& o, const DevParams& P, const V3<T>* x, SdfRes<T>* r, uint64_t* work = nullptr) {
  constexpr bool PREC = MODE == 2 || (MODE == 1 && IsDual<T>::value);
  float M[NP];
  T S[NP];
  V3<T> Ug[NP];           // sum u_k g_k (kappa folded out); PREC: running weighted mean of g_k
  Sym<T> C[NP], M2[NP];   // MODE 2: sum u_k kappa^2 Cov_k(n), sum u_k (g_k - mean)(g_k - mean)^T
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    M[p] = __builtin_inff();
    S[p] = cst<T>(0.f);
    if (MODE >= 1) Ug[p] = zero3<T>();
    if (MODE >= 2) { C[p] = zsym<T>(); M2[p] = zsym<T>(); }
  }
  const int K = min(o.n_pieces, kMaxPieces);
  float mub[NP];  // upper bound of the union's minimum
#pragma unroll
  for (int p = 0; p < NP; ++p) mub[p] = __builtin_inff();
  // With pruning, the first 64 pieces are visited in increasing order of their
  // least upper bound over the wave's points (|x - c_k| + ub_off_k), so that the
  // running minimum M is tight early; the others follow in index order.  Lane k
  // of `key` holds piece k's bound as order-preserving bits, all ones once the
  // piece is taken (or for no piece).
  const int lane = int(threadIdx.x) & (kWave - 1);
  uint32_t key = ~0u;
  if (P.prune) {
    for (int k = 0; k < K; ++k) {
      const PieceDesc pd = ldc(o.pieces + k);
      float umin = __builtin_inff();
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const V3<float> d = val3(x[p]) - V3<float>{pd.cx, pd.cy, pd.cz};
        const float u = sqrtf(dot(d, d)) + pd.ub_off;
        mub[p] = fminf(mub[p], u);
        umin = fminf(umin, u);
      }
      if (k < kWave) {
        const uint32_t w = wave_umin(ord_bits(umin));
        key = lane == k ? w : key;
      }
    }
  }
  const int K64 = P.prune ? min(K, kWave) : 0;
  for (int kk = 0; kk < K; ++kk) {
    int k = kk;
    if (kk < K64) {  // the untaken piece of least bound (lowest index on ties)
      const uint32_t w = wave_umin(key);
      k = int(__builtin_ctzll(__ballot(key == w)));
      key = lane == k ? ~0u : key;
    }
    const PieceDesc pd = ldc(o.pieces + k);
    const int pb = min(max(pd.plane_begin, 0), o.n_planes);
    const F4* pl = o.planes + pb;
    const int np = min(max(pd.plane_count, 0), o.n_planes - pb);  // never past the object's planes
    const F4* sp = o.sub + int64_t(kSub) * k;
    V3<T> xl[NP];
    float m[NP];
    // PREC: the max plane, as an index into the piece's planes (>= 0) or its
    // support subset (-1 - j); its kappa n is read once the passes are done
    int jm[NP];
    V3<float> xl0[NP];  // their values
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      xl[p] = x[p] - V3<float>{pd.cx, pd.cy, pd.cz};
      xl0[p] = val3(xl[p]);
      m[p] = -__builtin_inff();
      jm[p] = -1;
    }
    // the support subset: a lower bound of the piece SDF, and for a piece of
    // at most kSub planes (the subset is all of them) already the LSE shift
    // a piece matters at a lane while its lower bound m / kappa (the largest
    // plane value found so far) is below lim = min(mub, M) + prune_margin
    float lim[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) lim[p] = fminf(mub[p], M[p]) + P.prune_margin;
    auto needed = [&]() {
      bool need = false;
#pragma unroll
      for (int p = 0; p < NP; ++p) need = need || m[p] * P.icap < lim[p];
      return __any(need);
    };
    if (P.prune || np <= kSub) {
      if (work && P.prune) *work += uint64_t(kSub * NP);  // the bound
      // the kSub planes of the subset (a piece of fewer planes repeats its
      // first, and repeats never raise the max: equal values)
      if (np > 0) {
        F4 qv[kSub / 4];  // every block's lane plane is loaded first
#pragma unroll
        for (int b = 0; b < kSub / 4; ++b) qv[b] = grp_plane(sp, 4 * b);
#pragma unroll
        for (int b = 0; b < kSub / 4; ++b) {
          f4v av[NP], at[NP];
          blk_vals<NP, float>(qv[b], xl0, av, at);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
              const float a = av[p][i];
              if (PREC) {
                const bool up = a > m[p];
                m[p] = up ? a : m[p];
                jm[p] = up ? -1 - (4 * b + i) : jm[p];
              } else {
                m[p] = fmaxf(m[p], a);
              }
            }
          }
        }
      }
      if (P.prune && !needed()) continue;  // no lane of the wave needs this piece
    }
    // Plane groups (kGrp consecutive planes whose normals lie in a cone of axis
    // a and half-angle th <= 90 degrees; a piece's planes are stored padded to
    // whole groups with inert planes): at v = x - c every plane of the group has
    //   a_j = kappa (n_j . v + h_j) <= kappa (cos th (a . v) + sin th |v|) + e,
    // e the group's largest scaled offset (the max of n . v over the cone is
    // |v| cos(max(phi - th, 0)), phi = angle(a, v), which the right side bounds
    // for every phi when th <= 90 degrees: no square root or select per test).
    // With P.prune, a group whose bound lies more than gmarg below the running
    // max at every point of the wave is skipped: gmarg = 20 log2 e + log2(np),
    // so the skipped planes together weigh less than e^-20 < 2^-28 of the max
    // plane's term.  Groups are visited in index order through a 64-bit mask
    // per 64 groups.
    const int ng = min((np + kGrp - 1) / kGrp, (o.n_planes - pb) / kGrp);  // (never past the array)
    const F4* gr = o.sub + int64_t(kSub) * o.n_pieces + 2 * int64_t(pd.grp_begin);
    const float gmarg = kPruneTau * kLog2e + lg2(float(max(np, 1)));
    // (best: when given, the kept group of the highest bound at lane 0's first point)
    auto gmask = [&](int c0, int* best) -> uint64_t {
      const int c1 = min(ng, c0 + 64);
      if (best) *best = -1;
      if (!P.prune) return c1 - c0 >= 64 ? ~0ull : (1ull << (c1 - c0)) - 1ull;
      uint32_t bu = 0u;
      float vr[NP], thr[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        vr[p] = sqrtf(dot(xl0[p], xl0[p]));
        thr[p] = m[p] - gmarg;
      }
      uint64_t mk = 0;
      for (int g = c0; g < c1; ++g) {
        const F4 A = ldc(gr + 2 * g), B = ldc(gr + 2 * g + 1);
        bool nd = false;
        float ub0 = 0.f;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const float t = fmaf(A.x, xl0[p].x, fmaf(A.y, xl0[p].y, A.z * xl0[p].z));
          const float ub = fmaf(B.y, t, fmaf(B.z, vr[p], A.w));
          nd = nd || ub >= thr[p];
          if (p == 0) ub0 = ub;
        }
        if (__any(nd)) {
          mk |= 1ull << (g - c0);
          if (best) {
            const uint32_t u = uint32_t(__builtin_amdgcn_readfirstlane(int(ord_bits(ub0))));
            if (*best < 0 || u > bu) { bu = u; *best = g; }
          }
        }
      }
      return mk;
    };
    // the lowest kept group of the chunk at c0 (its bit cleared), -1 if none
    auto take = [&](uint64_t& mk, int c0) -> int {
      if (mk == 0) return -1;
      const int g = c0 + int(__builtin_ctzll(mk));
      mk &= mk - 1ull;
      return g;
    };
    // pass 1: shift = max_j a_j (value only; LSE is shift-invariant)
    if (np > kSub) {
      // the 4 blocks of each kept group, the lane plane in 4 buffers each
      // refilled with the next kept group's block as soon as it is used;
      // padding planes never raise the max
      auto blk = [&](const F4& ql, int j0) {
        f4v av[NP], at[NP];
        blk_vals<NP, float>(ql, xl0, av, at);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            const float a = av[p][i];
            if (PREC) {
              const bool up = a > m[p];
              m[p] = up ? a : m[p];
              jm[p] = up ? j0 + i : jm[p];
            } else {
              m[p] = fmaxf(m[p], a);
            }
          }
        }
      };
      // with pruning, the largest plane value found so far is a tighter lower
      // bound of the piece SDF than the subset's: the pass stops, and the piece
      // is skipped, once it shows that no lane needs the piece
      bool skip = false;
      for (int c0 = 0; c0 < ng && !skip; c0 += 64) {
        // the group most likely to hold the max first, then the others in order
        int g = -1;
        uint64_t mk = gmask(c0, &g);
        if (g >= 0) mk &= ~(1ull << (g - c0)); else g = take(mk, c0);  // (no best without pruning)
        const int j1 = max(g, 0) * kGrp;
        F4 q0 = grp_plane(pl, j1), q1 = grp_plane(pl, j1 + 4), q2 = grp_plane(pl, j1 + 8), q3 = grp_plane(pl, j1 + 12);
        while (g >= 0) {
          const int gn = take(mk, c0);
          const int j = g * kGrp, jn = (gn >= 0 ? gn : g) * kGrp;
          blk(q0, j);
          q0 = grp_plane(pl, jn);
          blk(q1, j + 4);
          q1 = grp_plane(pl, jn + 4);
          blk(q2, j + 8);
          q2 = grp_plane(pl, jn + 8);
          blk(q3, j + 12);
          q3 = grp_plane(pl, jn + 12);
          g = gn;
          if (P.prune && !needed()) { skip = true; break; }
        }
      }
      if (skip) continue;
    }
    V3<float> ref[NP];  // PREC: kappa n of the max plane (first of equal ones)
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      ref[p] = {0.f, 0.f, 0.f};
      if (PREC && np > 0) {
        const F4 q = jm[p] >= 0 ? pl[min(jm[p], np - 1)] : sp[min(-1 - jm[p], kSub - 1)];
        ref[p] = {q.x, q.y, q.z};
      }
    }
    // pass 2: sums (PREC: of kappa (n - n_ref) and its outer products)
    T s[NP];
    V3<T> G[NP];
    Sym<T> N[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      s[p] = cst<T>(0.f);
      if (MODE >= 1) G[p] = zero3<T>();
      if (MODE >= 2) N[p] = zsym<T>();
    }
    // plane j + i of a block (q: its wave-uniform copy) at the NP points
    constexpr bool DUAL = IsDual<T>::value;
    V3<float> xt[NP];  // dual: ln 2 times the tangents of the points
    f4v nm[NP];        // -m, the shift of the exponents
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      xt[p] = V3<float>{tan_(xl[p].x), tan_(xl[p].y), tan_(xl[p].z)} * kLn2;
      if (DUAL) nm[p] = f4v{-m[p], -m[p], -m[p], -m[p]};
    }
    auto term = [&](const F4& q, const f4v* av, const f4v* at, int i) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const float ev = ex2(DUAL ? av[p][i] : av[p][i] - m[p]);  // (dual: the chain subtracted m)
        const T e = mkT<T>(ev, DUAL ? ev * at[p][i] : 0.f);  // 2^a and its tangent ln 2 a' 2^a
        s[p] += e;
        if (MODE >= 1) {
          const float dx = PREC ? q.x - ref[p].x : q.x;
          const float dy = PREC ? q.y - ref[p].y : q.y;
          const float dz = PREC ? q.z - ref[p].z : q.z;
          G[p].x = fmaT(dx, e, G[p].x);
          G[p].y = fmaT(dy, e, G[p].y);
          G[p].z = fmaT(dz, e, G[p].z);
          if (MODE >= 2) {
            N[p].xx = fmaT(dx * dx, e, N[p].xx); N[p].yy = fmaT(dy * dy, e, N[p].yy);
            N[p].zz = fmaT(dz * dz, e, N[p].zz); N[p].xy = fmaT(dx * dy, e, N[p].xy);
            N[p].xz = fmaT(dx * dz, e, N[p].xz); N[p].yz = fmaT(dy * dz, e, N[p].yz);
          }
        }
      }
    };
    if (np > 0) {
      // The 4 blocks of each kept group: the lane's plane (matrix-core operand,
      // vector load) in 4 buffers, each refilled with the next kept group's
      // block as soon as it is used (a whole group ahead), and the block's
      // planes (SGPRs, scalar loads) in a ping-pong pair refilled two blocks
      // ahead: no buffer is copied across the loop, so every load has blocks of
      // work to complete behind it.  Padding planes add exact zeros.
      int n2 = 0;  // planes of the piece evaluated
      auto blk = [&](const F4& ql, const F4* sq) {
        f4v av[NP], at[NP];
        blk_vals_t<NP, DUAL>(ql, xl0, nm, xt, av, at);
#pragma unroll
        for (int i = 0; i < 4; ++i) term(sq[i], av, at, i);
      };
      auto sfill = [&](F4* sq, int j0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) sq[i] = ldc(pl + j0 + i);
      };
      static_assert(kGrp == 16, "four lane-plane buffers: one group");
      for (int c0 = 0; c0 < ng; c0 += 64) {
        uint64_t mk = gmask(c0, nullptr);
        int g = take(mk, c0);
        const int j1 = max(g, 0) * kGrp;
        F4 q0 = grp_plane(pl, j1), q1 = grp_plane(pl, j1 + 4), q2 = grp_plane(pl, j1 + 8), q3 = grp_plane(pl, j1 + 12);
        F4 sa[4], sb[4];
        sfill(sa, j1);
        sfill(sb, j1 + 4);
        while (g >= 0) {
          const int gn = take(mk, c0);
          const int j = g * kGrp, jn = (gn >= 0 ? gn : g) * kGrp;
          n2 += min(kGrp, np - j);
          blk(q0, sa);
          q0 = grp_plane(pl, jn);
          sfill(sa, j + 8);
          blk(q1, sb);
          q1 = grp_plane(pl, jn + 4);
          sfill(sb, j + 12);
          blk(q2, sa);
          q2 = grp_plane(pl, jn + 8);
          sfill(sa, jn);
          blk(q3, sb);
          q3 = grp_plane(pl, jn + 12);
          sfill(sb, jn + 4);
          g = gn;
        }
      }
      // point-plane evaluations performed by the wave (per lane)
      if (work) *work += uint64_t(n2 * NP);
    }
    // combine the piece into the running smooth union
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const T phik = (lg2(s[p]) + m[p]) * P.icap;
      const float Mn = fminf(M[p], val(phik));
      const float sc = ex2((Mn - M[p]) * P.kcup);  // rescale of the old terms (0 when M = +inf)
      const T u = ex2((cst<T>(Mn) - phik) * P.kcup);
      if (!PREC) {
        S[p] = S[p] * sc + u;
        if (MODE >= 1) Ug[p] = Ug[p] * sc + G[p] * (u * P.icap / s[p]);
      } else {
        const T is = cst<T>(1.f) / s[p];
        const V3<T> dg = G[p] * is;                          // kappa (g_k - n_ref)
        const V3<T> gk = (dg + ref[p]) * P.icap;             // g_k
        const bool first = M[p] == __builtin_inff();
        const T w_old = S[p] * sc;
        S[p] = w_old + u;
        const T t = first ? cst<T>(1.f) : u / S[p];
        const V3<T> dl = gk - Ug[p];
        Ug[p] = first ? gk : Ug[p] + dl * t;
        if (MODE >= 2) {
          M2[p] = first ? zsym<T>() : M2[p] * sc + outer(dl) * (w_old * t);
          C[p] = C[p] * sc + (N[p] * is - outer(dg)) * u;
        }
      }
      M[p] = Mn;
    }
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    r[p].phi = cst<T>(M[p]) - lg2(S[p]) * P.icup;
    if (MODE >= 1) {
      const T iS = cst<T>(1.f) / S[p];
      r[p].g = PREC ? Ug[p] : Ug[p] * iS;
      if (MODE >= 2) {
        // (1/tau_cap) / kappa^2 = ln2 / kappa;  1/tau_cup = ln2 kappa_cup
        r[p].H = C[p] * (iS * (kLn2 * P.icap)) - M2[p] * (iS * (kLn2 * P.kcup));
      }
    }
  }
}

// ------------------------------------------------------- spline SDF --
// Cubic-spline SDF of an object (Sec. III-B.1/2): over the box of its voxel grid
// (origin gorg, n = gn cells of size gh per axis) the spline of phi and the
// separately fitted spline of the normal share (n + 3)^3 basis functions, whose
// coefficients (phi, n_x, n_y, n_z) are one float4 each (`sub` of a spline
// object), index (i (n + 3) + j) (n + 3) + k.  At a point, 4 basis functions
// per axis are nonzero: 64 gathers of 16 bytes, the 4 z-neighbours contiguous.
// Outside the box phi continues as s(pi(x)) + |x - pi(x)| and the normal as
// s_n(pi(x)), pi the closest point of the box.
template <class T> struct SplRes {
  T phi;
  V3<T> g;   // grad phi (GRAD)
  V3<T> n;   // normal spline (NRM)
  M3<T> J;   // its Jacobian, row a = d n_a / dx (JAC)
};
// The 4 basis functions nonzero in a cell at offset w in [0, 1] (u(w + 1),
// u(w), u(w - 1), u(w - 2) with u of Sec. III-B.1) and their derivatives in w.
template <class T> CM_DEV void cell_basis(T w, T* b, T* db) {
  const T v = cst<T>(1.f) - w;
  const T w2 = w * w, v2 = v * v;
  b[0] = v2 * v;
  b[1] = w2 * (3.f * w - 6.f) + 4.f;
  b[2] = v2 * (3.f * v - 6.f) + 4.f;
  b[3] = w2 * w;
  db[0] = v2 * -3.f;
  db[1] = w * (9.f * w - 12.f);
  db[2] = v * (12.f - 9.f * v);
  db[3] = w2 * 3.f;
}
template <bool GRAD, bool NRM, bool JAC, class T>
CM_DEV void spline_eval(const ObjDesc& o, const V3<T>& x, SplRes<T>& r) {
  const int n = o.gn, m = n + 3;
  const T xs[3] = {x.x, x.y, x.z};
  T b[3][4], db[3][4];
  int i0[3];
  T out2 = cst<T>(0.f);
  T dd[3] = {cst<T>(0.f), cst<T>(0.f), cst<T>(0.f)};  // x - pi(x)
  float dsc[3];  // d t / d x, 0 for a clamped axis (s(pi(x)) does not move with it)
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T t = (xs[a] - o.gorg[a]) * o.ginv[a];
    dsc[a] = o.ginv[a];
    const float tv = val(t);
    if (!(tv >= 0.f) || tv > float(n)) {
      const float lim = tv > float(n) ? float(n) : 0.f;
      const T d = xs[a] - (o.gorg[a] + lim * o.gh[a]);
      out2 = out2 + d * d;
      dd[a] = d;
      t = cst<T>(lim);
      dsc[a] = 0.f;
    }
    const int i = min(max(int(floorf(val(t))), 0), n - 1);
    i0[a] = i;
    cell_basis(t - float(i), b[a], db[a]);
  }
  T phi = cst<T>(0.f);
  V3<T> g = zero3<T>(), nr = zero3<T>();
  M3<T> J;
  if (JAC)
#pragma unroll
    for (int i = 0; i < 9; ++i) J.m[i] = cst<T>(0.f);
  const F4* cf = o.sub;
  // one x-slab of 16 coefficients per iteration (the x weights picked by the
  // uniform counter), so that at most 16 gathers are in flight per lane
#pragma unroll 1
  for (int p = 0; p < 4; ++p) {
    const T bx = p == 0 ? b[0][0] : (p == 1 ? b[0][1] : (p == 2 ? b[0][2] : b[0][3]));
    const T dbx = p == 0 ? db[0][0] : (p == 1 ? db[0][1] : (p == 2 ? db[0][2] : db[0][3]));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T wpq = bx * b[1][q];
      const T wdx = dbx * b[1][q], wdy = bx * db[1][q];
      const F4* row = cf + (int64_t(i0[0] + p) * m + (i0[1] + q)) * m + i0[2];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const F4 c = row[k];
        const T w = wpq * b[2][k];
        phi = fmaT(c.x, w, phi);
        if (NRM) { nr.x = fmaT(c.y, w, nr.x); nr.y = fmaT(c.z, w, nr.y); nr.z = fmaT(c.w, w, nr.z); }
        if (GRAD || JAC) {
          const T wx = wdx * b[2][k], wy = wdy * b[2][k], wz = wpq * db[2][k];
          if (GRAD) { g.x = fmaT(c.x, wx, g.x); g.y = fmaT(c.x, wy, g.y); g.z = fmaT(c.x, wz, g.z); }
          if (JAC) {
            J.m[0] = fmaT(c.y, wx, J.m[0]); J.m[1] = fmaT(c.y, wy, J.m[1]); J.m[2] = fmaT(c.y, wz, J.m[2]);
            J.m[3] = fmaT(c.z, wx, J.m[3]); J.m[4] = fmaT(c.z, wy, J.m[4]); J.m[5] = fmaT(c.z, wz, J.m[5]);
            J.m[6] = fmaT(c.w, wx, J.m[6]); J.m[7] = fmaT(c.w, wy, J.m[7]); J.m[8] = fmaT(c.w, wz, J.m[8]);
          }
        }
      }
    }
  }
  const bool outside = val(out2) > 0.f;
  const T dl = outside ? sqrtT(out2) : cst<T>(0.f);
  r.phi = phi + dl;
  if (GRAD) {
    r.g = {g.x * dsc[0], g.y * dsc[1], g.z * dsc[2]};
    if (outside) r.g = r.g + V3<T>{dd[0], dd[1], dd[2]} * (cst<T>(1.f) / dl);
  }
  if (NRM) r.n = nr;
  if (JAC)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) r.J.m[3 * a + c] = J.m[3 * a + c] * dsc[c];
}

// Spline broad phase (B-spline convex hull): the grid of a spline object
// stores, per cell, 216 times the least coefficient of phi the cell reaches, a
// lower bound of the spline over the cell; a point's bound is its clamped
// cell's plus its distance outside the box.
CM_DEV float spline_lb(const ObjDesc& o, V3<float> x) {
  const int n = o.gn;
  const float xs[3] = {x.x, x.y, x.z};
  int id[3];
  float o2 = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lo = o.gorg[a], hi = o.gorg[a] + float(n) * o.gh[a];
    const float d = xs[a] < lo ? lo - xs[a] : (xs[a] > hi ? xs[a] - hi : 0.f);
    o2 = fmaf(d, d, o2);
    id[a] = min(max(int(floorf((xs[a] - lo) * o.ginv[a])), 0), n - 1);
  }
  return o.grid[(id[0] * n + id[1]) * n + id[2]] + sqrtf(o2);
}
// The same bound over a segment: the least cell bound over the clamped cell
// range of its bounding box plus the box's distance outside the grid box.
CM_DEV float spline_edge_lb(const ObjDesc& o, V3<float> x1, V3<float> x2) {
  const int n = o.gn;
  const float a1[3] = {x1.x, x1.y, x1.z}, a2[3] = {x2.x, x2.y, x2.z};
  int lo[3], hi[3];
  float o2 = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float mn = fminf(a1[a], a2[a]), mx = fmaxf(a1[a], a2[a]);
    const float blo = o.gorg[a], bhi = o.gorg[a] + float(n) * o.gh[a];
    const float d = mx < blo ? blo - mx : (mn > bhi ? mn - bhi : 0.f);
    o2 = fmaf(d, d, o2);
    lo[a] = min(max(int(floorf((mn - blo) * o.ginv[a])), 0), n - 1);
    hi[a] = min(max(int(floorf((mx - blo) * o.ginv[a])), 0), n - 1);
  }
  float m = __builtin_inff();
  for (int i = lo[0]; i <= hi[0]; ++i)
    for (int j = lo[1]; j <= hi[1]; ++j)
      for (int k = lo[2]; k <= hi[2]; ++k) m = fminf(m, o.grid[(i * n + j) * n + k]);
  return m + sqrtf(o2);
}

// Lower bound of phi from the voxel grid (Sec. IV-C.2): the stored phi at the
// centre of the voxel the point falls into (clamped to the grid) minus
// max(circumradius, distance to that centre).
CM_DEV float grid_lb(const ObjDesc& o, V3<float> x) {
  const int n = o.gn;
  float u0 = (x.x - o.gorg[0]) * o.ginv[0], u1 = (x.y - o.gorg[1]) * o.ginv[1], u2 = (x.z - o.gorg[2]) * o.ginv[2];
  int i = min(max(int(floorf(u0)), 0), n - 1);
  int j = min(max(int(floorf(u1)), 0), n - 1);
  int k = min(max(int(floorf(u2)), 0), n - 1);
  float c0 = o.gorg[0] + (float(i) + 0.5f) * o.gh[0];
  float c1 = o.gorg[1] + (float(j) + 0.5f) * o.gh[1];
  float c2 = o.gorg[2] + (float(k) + 0.5f) * o.gh[2];
  float d = sqrtf((x.x - c0) * (x.x - c0) + (x.y - c1) * (x.y - c1) + (x.z - c2) * (x.z - c2));
  return o.grid[(i * n + j) * n + k] - fmaxf(o.gr, d);
}

}  // namespace cm
