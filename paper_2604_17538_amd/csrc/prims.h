// Primitive-based SDFs (Sec. III-A) on gfx950: superquadric (SQ), plane-SQ
// intersection (PSQ), PSQ swept along a quadratic spline (XPSQ), folded into
// one object SDF by smooth union / subtraction / intersection.
//
// Every quantity is a second-order forward jet in the point x: value, gradient
// and (ORD 2) Hessian, over scalars T (float, or dual floats for H v).  The
// contact path needs phi (trace steps), phi and grad (normals) and the Hessian
// (the adjoint of the normal); the jets give all three from one evaluation.
#pragma once
#include "devmath.h"

namespace cm {

// ------------------------------------------------------- scalar functions --
CM_DEV float cbrtT(float x) { return cbrtf(x); }
CM_DEV df cbrtT(df a) { const float c = cbrtf(a.v); return {c, a.t / (3.f * c * c)}; }
CM_DEV float cosT(float x) { return cosf(x); }
CM_DEV df cosT(df a) { return {cosf(a.v), -sinf(a.v) * a.t}; }
CM_DEV float sinT(float x) { return sinf(x); }
CM_DEV df sinT(df a) { return {sinf(a.v), cosf(a.v) * a.t}; }
CM_DEV float atan2T(float y, float x) { return atan2f(y, x); }
CM_DEV df atan2T(df y, df x) {
  const float r2 = x.v * x.v + y.v * y.v;
  return {atan2f(y.v, x.v), (x.v * y.t - y.v * x.t) / r2};
}

// ------------------------------------------------------------------- jets --
// Hessian slots: xx, yy, zz, xy, xz, yz.
CM_DEV constexpr int hI(int k) { return k < 3 ? k : (k == 5 ? 1 : 0); }
CM_DEV constexpr int hJ(int k) { return k < 3 ? k : (k == 3 ? 1 : 2); }

template <class T, int ORD> struct Jt {
  T v;
  T g[3];
  T h[6];
};

template <class T, int O> CM_DEV Jt<T, O> jc(T c) {
  Jt<T, O> r;
  r.v = c;
#pragma unroll
  for (int i = 0; i < 3; ++i) r.g[i] = cst<T>(0.f);
#pragma unroll
  for (int k = 0; k < 6; ++k) r.h[k] = cst<T>(0.f);
  return r;
}
template <class T, int O> CM_DEV Jt<T, O> operator+(const Jt<T, O>& a, const Jt<T, O>& b) {
  Jt<T, O> r;
  r.v = a.v + b.v;
  if constexpr (O >= 1) {
#pragma unroll
    for (int i = 0; i < 3; ++i) r.g[i] = a.g[i] + b.g[i];
  }
  if constexpr (O >= 2) {
#pragma unroll
    for (int k = 0; k < 6; ++k) r.h[k] = a.h[k] + b.h[k];
  }
  return r;
}
template <class T, int O> CM_DEV Jt<T, O> operator-(const Jt<T, O>& a) {
  Jt<T, O> r;
  r.v = -a.v;
  if constexpr (O >= 1) {
#pragma unroll
    for (int i = 0; i < 3; ++i) r.g[i] = -a.g[i];
  }
  if constexpr (O >= 2) {
#pragma unroll
    for (int k = 0; k < 6; ++k) r.h[k] = -a.h[k];
  }
  return r;
}
template <class T, int O> CM_DEV Jt<T, O> operator-(const Jt<T, O>& a, const Jt<T, O>& b) { return a + (-b); }
// scalar (no x-dependence) on either side
template <class T, int O, class S> CM_DEV Jt<T, O> operator+(const Jt<T, O>& a, S c) {
  Jt<T, O> r = a;
  r.v = a.v + c;
  return r;
}
template <class T, int O, class S> CM_DEV Jt<T, O> operator-(const Jt<T, O>& a, S c) {
  Jt<T, O> r = a;
  r.v = a.v - c;
  return r;
}
template <class T, int O, class S> CM_DEV Jt<T, O> operator*(const Jt<T, O>& a, S c) {
  Jt<T, O> r;
  r.v = a.v * c;
  if constexpr (O >= 1) {
#pragma unroll
    for (int i = 0; i < 3; ++i) r.g[i] = a.g[i] * c;
  }
  if constexpr (O >= 2) {
#pragma unroll
    for (int k = 0; k < 6; ++k) r.h[k] = a.h[k] * c;
  }
  return r;
}
template <class T, int O> CM_DEV Jt<T, O> operator*(const Jt<T, O>& a, const Jt<T, O>& b) {
  Jt<T, O> r;
  r.v = a.v * b.v;
  if constexpr (O >= 1) {
#pragma unroll
    for (int i = 0; i < 3; ++i) r.g[i] = a.v * b.g[i] + b.v * a.g[i];
  }
  if constexpr (O >= 2) {
#pragma unroll
    for (int k = 0; k < 6; ++k)
      r.h[k] = a.v * b.h[k] + b.v * a.h[k] + a.g[hI(k)] * b.g[hJ(k)] + a.g[hJ(k)] * b.g[hI(k)];
  }
  return r;
}
// f(a) from f(v), f'(v), f''(v)
template <class T, int O> CM_DEV Jt<T, O> chain(const Jt<T, O>& a, T f0, T f1, T f2) {
  Jt<T, O> r;
  r.v = f0;
  if constexpr (O >= 1) {
#pragma unroll
    for (int i = 0; i < 3; ++i) r.g[i] = f1 * a.g[i];
  }
  if constexpr (O >= 2) {
#pragma unroll
    for (int k = 0; k < 6; ++k) r.h[k] = f1 * a.h[k] + f2 * (a.g[hI(k)] * a.g[hJ(k)]);
  }
  return r;
}
template <class T, int O> CM_DEV Jt<T, O> jexp(const Jt<T, O>& a) {
  const T e = expT(a.v);
  return chain(a, e, e, e);
}
template <class T, int O> CM_DEV Jt<T, O> jlog(const Jt<T, O>& a) {
  const T i = cst<T>(1.f) / a.v;
  return chain(a, logT(a.v), i, -(i * i));
}
template <class T, int O> CM_DEV Jt<T, O> jrcp(const Jt<T, O>& a) {
  const T i = cst<T>(1.f) / a.v;
  return chain(a, i, -(i * i), (i * i) * i * 2.f);
}
template <class T, int O> CM_DEV Jt<T, O> operator/(const Jt<T, O>& a, const Jt<T, O>& b) { return a * jrcp(b); }
template <class T, int O> CM_DEV Jt<T, O> jsqrt(const Jt<T, O>& a) {
  const T s = sqrtT(a.v);
  const T i = cst<T>(1.f) / s;
  return chain(a, s, i * 0.5f, -(i * i) * i * 0.25f);
}
template <class T, int O> CM_DEV Jt<T, O> jcbrt(const Jt<T, O>& a) {
  const T c = cbrtT(a.v);
  const T i2 = cst<T>(1.f) / (c * c);
  return chain(a, c, i2 * (1.f / 3.f), -(i2 * i2) / c * (2.f / 9.f));
}
template <class T, int O> CM_DEV Jt<T, O> jcos(const Jt<T, O>& a) {
  const T c = cosT(a.v);
  return chain(a, c, -sinT(a.v), -c);
}
// sigma(a) (Sec. II)
template <class T, int O> CM_DEV Jt<T, O> jsigmoid(const Jt<T, O>& a) {
  const T s = sigmoidT(a.v);
  const T d = s * (cst<T>(1.f) - s);
  return chain(a, s, d, d * (cst<T>(1.f) - s * 2.f));
}
// s_+(a) = tau log(1 + exp(a / tau)) (Sec. II)
template <class T, int O> CM_DEV Jt<T, O> jsoftplus(const Jt<T, O>& a, float tau, float inv_tau) {
  const T s = sigmoidT(a.v * inv_tau);
  return chain(a, softplusT(a.v, tau, inv_tau), s, s * (cst<T>(1.f) - s) * inv_tau);
}
// s_clip(a, 0, 1) (Sec. II)
template <class T, int O> CM_DEV Jt<T, O> jsoftclip01(const Jt<T, O>& a, float tau, float inv_tau) {
  return jsoftplus(a, tau, inv_tau) - jsoftplus(a - 1.f, tau, inv_tau);
}
// atan2(y, x)
template <class T, int O> CM_DEV Jt<T, O> jatan2(const Jt<T, O>& y, const Jt<T, O>& x) {
  Jt<T, O> r;
  r.v = atan2T(y.v, x.v);
  const T i2 = cst<T>(1.f) / (x.v * x.v + y.v * y.v);
  const T fy = x.v * i2, fx = -(y.v * i2);
  if constexpr (O >= 1) {
#pragma unroll
    for (int i = 0; i < 3; ++i) r.g[i] = fy * y.g[i] + fx * x.g[i];
  }
  if constexpr (O >= 2) {
    const T i4 = i2 * i2;
    const T fyy = -(x.v * y.v * i4 * 2.f), fxx = x.v * y.v * i4 * 2.f, fxy = (y.v * y.v - x.v * x.v) * i4;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int I = hI(k), J = hJ(k);
      r.h[k] = fy * y.h[k] + fx * x.h[k] + fyy * (y.g[I] * y.g[J]) + fxx * (x.g[I] * x.g[J]) +
               fxy * (y.g[I] * x.g[J] + x.g[I] * y.g[J]);
    }
  }
  return r;
}
// log(exp(a) + exp(b)), shifted by the larger value
template <class T, int O> CM_DEV Jt<T, O> jlse2(const Jt<T, O>& a, const Jt<T, O>& b) {
  const float m = fmaxf(val(a.v), val(b.v));
  return jlog(jexp(a - m) + jexp(b - m)) + m;
}

template <class T, int O> struct JV3 { Jt<T, O> x, y, z; };
template <class T, int O> CM_DEV Jt<T, O> jdot(const JV3<T, O>& a, const JV3<T, O>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}

// ----------------------------------------------------- primitive records --
// The object's primitive block (ObjDesc::sub of an object of kRepPrims):
// ObjDesc::gn records, then their half-spaces (F4 (n, h) in the PSQ frame).
CM_DEV const PrimDev* prim_records(const ObjDesc& o) { return reinterpret_cast<const PrimDev*>(o.sub); }
CM_DEV const F4* prim_planes(const ObjDesc& o) {
  return reinterpret_cast<const F4*>(reinterpret_cast<const PrimDev*>(o.sub) + o.gn);
}

// Superquadric (Sec. III-A.1) read as its radial distance |x| (1 - f^(-e1/2)),
// every squared coordinate q^2 as q^2 + 1e-6 and the radius as
// sqrt(|x|^2 + 1e-6 a_min^2); f in the log domain (its powers reach e^50).
template <class T, int O>
CM_DEV Jt<T, O> sq_sdf(const JV3<T, O>& x, const Jt<T, O> a[3], const Jt<T, O> e[2]) {
  constexpr float d2 = 1e-6f;
  const Jt<T, O> ie1 = jrcp(e[0]), ie2 = jrcp(e[1]);
  const Jt<T, O> X = x.x / a[0], Y = x.y / a[1], Z = x.z / a[2];
  const Jt<T, O> lx = jlog(X * X + d2) * ie2, ly = jlog(Y * Y + d2) * ie2;
  const Jt<T, O> l1 = jlse2(lx, ly) * (e[1] * ie1);
  const Jt<T, O> lz = jlog(Z * Z + d2) * ie1;
  const Jt<T, O> lf = jlse2(l1, lz);
  int k = val(a[1].v) < val(a[0].v) ? 1 : 0;
  if (val(a[2].v) < val(a[k].v)) k = 2;
  const Jt<T, O> r = jsqrt(jdot(x, x) + a[k] * a[k] * d2);
  return r * (jc<T, O>(cst<T>(1.f)) - jexp(lf * (e[0] * -0.5f)));
}

// PSQ (Sec. III-A.3): tau_cap LSE of the SQ and the half-spaces (PSQ frame).
template <class T, int O>
CM_DEV Jt<T, O> psq_sdf(const PrimDev& pr, const F4* planes, const JV3<T, O>& xs, const Jt<T, O> a[3],
                        const Jt<T, O> e[2], const DevParams& P) {
  const Jt<T, O> s = sq_sdf(xs, a, e);
  if (pr.plane_count <= 0) return s;
  float m = val(s.v);
  for (int j = 0; j < pr.plane_count; ++j) {
    const F4 q = planes[pr.plane_begin + j];
    m = fmaxf(m, val(xs.x.v) * q.x + val(xs.y.v) * q.y + val(xs.z.v) * q.z + q.w);
  }
  const float ic = P.kcap * kLn2;  // 1 / tau_cap
  Jt<T, O> acc = jexp((s - m) * ic);
  for (int j = 0; j < pr.plane_count; ++j) {
    const F4 q = planes[pr.plane_begin + j];
    const Jt<T, O> v = xs.x * q.x + xs.y * q.y + xs.z * q.z + q.w;
    acc = acc + jexp((v - m) * ic);
  }
  return jlog(acc) * (P.icap * kLog2e) + m;  // tau_cap = icap log2(e)
}

// The three projection parameters of x onto the XPSQ's spline (Sec. III-A.5):
// the stationarity cubic t^3 + a2 t^2 + a1 t + a0 (divided by 2|A|^2), shifted
// to s^3 + P s + Q, both of Cardano's branches from the softplus-projected
// discriminant, soft-clipped to (0, 1) and blended by sigmoid brackets.
template <class T, int O>
CM_DEV void xpsq_roots(const PrimDev& pr, const JV3<T, O>& x, const DevParams& P, Jt<T, O> t[3]) {
  const Jt<T, O> cx = x.x * -1.f + pr.c[0], cy = x.y * -1.f + pr.c[1], cz = x.z * -1.f + pr.c[2];  // p1 - x
  const float i2A = pr.inv2AA;  // 1 / (2 |A|^2)
  const Jt<T, O> a1 = ((cx * pr.A[0] + cy * pr.A[1] + cz * pr.A[2]) * 2.f + pr.BB) * i2A;
  const Jt<T, O> a0 = (cx * pr.B[0] + cy * pr.B[1] + cz * pr.B[2]) * i2A;
  const float a2 = pr.a2;
  const Jt<T, O> Pq = a1 - a2 * a2 * (1.f / 3.f);
  const Jt<T, O> Q = a0 - a1 * (a2 * (1.f / 3.f)) + 2.f * a2 * a2 * a2 * (1.f / 27.f);
  const Jt<T, O> Delta = -((Pq * Pq * Pq) * 4.f + (Q * Q) * 27.f);
  const float td = P.tau_disc, itd = P.inv_tau_disc;
  const Jt<T, O> u = Q * -0.5f;
  const Jt<T, O> Dm = jsoftplus(-Delta, td, itd) * (1.f / 108.f), Dp = jsoftplus(Delta, td, itd) * (1.f / 108.f);
  constexpr float tiny = 1e-20f;  // keeps sqrt differentiable where s_+ underflows
  const Jt<T, O> sm = jsqrt(Dm + tiny);
  // cbrt(u + sm) + cbrt(u - sm), the root of the larger magnitude first: the
  // other cube root's argument, u - sgn(u) sm, cancels in FP32 when |P| is small
  // (it can round to 0, where cbrt has no derivative), and equals
  // (u^2 - sm^2) / (u + sgn(u) sm) with u^2 - sm^2 = -P^3/27 - Dp - tiny exactly
  // (s_+(-Delta) = -Delta + s_+(Delta) and -Delta/108 = u^2 + P^3/27)
  const Jt<T, O> c1 = jcbrt(val(u.v) >= 0.f ? u + sm : u - sm);
  const Jt<T, O> c2 = jcbrt(-(Pq * Pq * Pq) * (1.f / 27.f) - Dp - tiny) / c1;
  const Jt<T, O> s_one = c1 + c2;
  const Jt<T, O> r = jsqrt(u * u + Dp), th = jatan2(jsqrt(Dp + tiny), u), rr = jcbrt(r);
  const Jt<T, O> w_one = jsigmoid(Delta * -itd), w_three = jsigmoid(Delta * itd);
  const Jt<T, O> t_one = jsoftclip01(s_one - a2 * (1.f / 3.f), P.tau_t, P.inv_tau_t);
  constexpr float kTwoPi = 6.28318530717958647693f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const Jt<T, O> sk = jcos((th + kTwoPi * float(k)) * (1.f / 3.f)) * rr * 2.f;
    t[k] = w_one * t_one + w_three * jsoftclip01(sk - a2 * (1.f / 3.f), P.tau_t, P.inv_tau_t);
  }
}

// XPSQ (Sec. III-A.4/5): the PSQ at each projection parameter (centre p(t),
// Frenet frame [N, b, T] of the planar spline, scales and exponents linear in
// t, half-spaces fixed in the PSQ frame), smooth minimum of the three.
template <class T, int O>
CM_DEV Jt<T, O> xpsq_sdf(const PrimDev& pr, const F4* planes, const JV3<T, O>& x, const DevParams& P) {
  Jt<T, O> t[3];
  xpsq_roots(pr, x, P, t);
  Jt<T, O> ph[3];
#pragma unroll 1
  for (int k = 0; k < 3; ++k) {
    const Jt<T, O>& tk = t[k];
    const Jt<T, O> omt = tk * -1.f + 1.f;
    const Jt<T, O> w0 = omt * omt, w1 = tk * omt * 2.f, w2 = tk * tk;
    JV3<T, O> d;
    d.x = x.x - (w0 * pr.c[0] + w1 * pr.p2[0] + w2 * pr.p3[0]);
    d.y = x.y - (w0 * pr.c[1] + w1 * pr.p2[1] + w2 * pr.p3[1]);
    d.z = x.z - (w0 * pr.c[2] + w1 * pr.p2[2] + w2 * pr.p3[2]);
    JV3<T, O> dp;  // p'(t) = 2 A t + B
    dp.x = tk * (2.f * pr.A[0]) + pr.B[0];
    dp.y = tk * (2.f * pr.A[1]) + pr.B[1];
    dp.z = tk * (2.f * pr.A[2]) + pr.B[2];
    const Jt<T, O> il = jrcp(jsqrt(jdot(dp, dp)));
    const JV3<T, O> Tn{dp.x * il, dp.y * il, dp.z * il};
    const float bx = pr.bn[0], by = pr.bn[1], bz = pr.bn[2];
    const JV3<T, O> Nn{Tn.z * by - Tn.y * bz, Tn.x * bz - Tn.z * bx, Tn.y * bx - Tn.x * by};  // b x T
    JV3<T, O> xs;
    xs.x = jdot(Nn, d);
    xs.y = d.x * bx + d.y * by + d.z * bz;
    xs.z = jdot(Tn, d);
    Jt<T, O> a[3], e[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) a[i] = tk * (pr.a1[i] - pr.a0[i]) + pr.a0[i];
    e[0] = tk * (pr.e1a - pr.e0a) + pr.e0a;
    e[1] = tk * (pr.e1b - pr.e0b) + pr.e0b;
    ph[k] = psq_sdf(pr, planes, xs, a, e, P);
  }
  // -tau_cup LSE(-phi_k / tau_cup)
  const float m = fminf(val(ph[0].v), fminf(val(ph[1].v), val(ph[2].v)));
  const float ic = P.kcup * kLn2;  // 1 / tau_cup
  const Jt<T, O> s = jexp((ph[0] - m) * -ic) + jexp((ph[1] - m) * -ic) + jexp((ph[2] - m) * -ic);
  return jlog(s) * -(P.icup * kLog2e) + m;
}

template <class T, int O>
CM_DEV Jt<T, O> prim_sdf(const PrimDev& pr, const F4* planes, const JV3<T, O>& x, const DevParams& P) {
  if (pr.kind == 1) return xpsq_sdf(pr, planes, x, P);
  const JV3<T, O> d{x.x - pr.c[0], x.y - pr.c[1], x.z - pr.c[2]};
  JV3<T, O> xs;  // R^T (x - c)
  xs.x = d.x * pr.Rt[0] + d.y * pr.Rt[1] + d.z * pr.Rt[2];
  xs.y = d.x * pr.Rt[3] + d.y * pr.Rt[4] + d.z * pr.Rt[5];
  xs.z = d.x * pr.Rt[6] + d.y * pr.Rt[7] + d.z * pr.Rt[8];
  const Jt<T, O> a[3] = {jc<T, O>(cst<T>(pr.a0[0])), jc<T, O>(cst<T>(pr.a0[1])), jc<T, O>(cst<T>(pr.a0[2]))};
  const Jt<T, O> e[2] = {jc<T, O>(cst<T>(pr.e0a)), jc<T, O>(cst<T>(pr.e0b))};
  return psq_sdf(pr, planes, xs, a, e, P);
}

// The object's SDF (Sec. III-A.2): its primitives folded in order by smooth
// union (tau_cup), subtraction or intersection (tau_cap).
template <class T, int O> CM_DEV Jt<T, O> prims_eval(const ObjDesc& o, const V3<T>& x, const DevParams& P) {
  JV3<T, O> xj;
  xj.x = jc<T, O>(x.x);
  xj.y = jc<T, O>(x.y);
  xj.z = jc<T, O>(x.z);
  if constexpr (O >= 1) {
    xj.x.g[0] = cst<T>(1.f);
    xj.y.g[1] = cst<T>(1.f);
    xj.z.g[2] = cst<T>(1.f);
  }
  const PrimDev* pr = prim_records(o);
  const F4* planes = prim_planes(o);
  Jt<T, O> phi = prim_sdf(pr[0], planes, xj, P);
  for (int i = 1; i < o.gn; ++i) {
    const Jt<T, O> v = prim_sdf(pr[i], planes, xj, P);
    const int op = pr[i].op;
    if (op == 0) {
      const float m = fminf(val(phi.v), val(v.v)), ic = P.kcup * kLn2;
      phi = jlog(jexp((phi - m) * -ic) + jexp((v - m) * -ic)) * -(P.icup * kLog2e) + m;
    } else {
      const Jt<T, O> w = op == 1 ? -v : v;
      const float m = fmaxf(val(phi.v), val(w.v)), ic = P.kcap * kLn2;
      phi = jlog(jexp((phi - m) * ic) + jexp((w - m) * ic)) * (P.icap * kLog2e) + m;
    }
  }
  return phi;
}

}  // namespace cm
