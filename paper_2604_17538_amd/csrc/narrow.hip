// Narrow phase, blending and its adjoint on gfx950, written once over a scalar
// type T (float, or the dual float `df` for forward-mode tangents):
//   k_narrow<float, false>  forward contacts -> per-tile blend partials
//   k_narrow<df,    false>  the same with tangents along a pose direction
//   k_finalize<T, 0/1>      fixed-order per-piece merge -> outputs, or the
//                           per-piece adjoint seeds of L = sum_g <c_g, y_g>
//   k_narrow<T, true>       per-contact adjoint -> per-tile pose gradients
//   k_reduce<T>             fixed-order per-query sum (+ filtered closed forms)
// The Hessian-vector product is this hand-written adjoint evaluated in dual
// numbers (forward over reverse).  Before an adjoint, the forward sweep keeps
// what needed passes over the planes (phi, gradient and Hessian at the contact
// point and at the sphere-trace iterates) on a tape for the tiles the plan's
// memory holds; the adjoint rebuilds the rest of each contact with a few
// arithmetic operations.  Tiles past the tape recompute their forward pass.
#include <atomic>

#include "devmath.h"
#include "kernels.h"
#include "prims.h"
#include "wave.h"

namespace cm {

CM_DEV void putT(float* o, float x) { o[0] = x; }
CM_DEV void putT(float* o, df x) { o[0] = x.v; o[1] = x.t; }
template <class T> CM_DEV T getT(const float* o);
template <> CM_DEV float getT<float>(const float* o) { return o[0]; }
template <> CM_DEV df getT<df>(const float* o) { return df{o[0], o[1]}; }
template <class T> constexpr int nT() { return int(sizeof(T) / sizeof(float)); }

// Tape access (layout in kernels.h): float values in rows v, duals in rows 2v
// (value) and 2v + 1 (tangent); `rs` is the row stride (taped slots).
CM_DEV void tput(float* tp, int64_t rs, int v, int64_t slot, float x) { tp[int64_t(v) * rs + slot] = x; }
CM_DEV void tput(float* tp, int64_t rs, int v, int64_t slot, df x) {
  tp[int64_t(2 * v) * rs + slot] = x.v;
  tp[int64_t(2 * v + 1) * rs + slot] = x.t;
}
template <class T> CM_DEV T tget(const float* tp, int64_t rs, int v, int64_t slot);
template <> CM_DEV float tget<float>(const float* tp, int64_t rs, int v, int64_t slot) {
  return tp[int64_t(v) * rs + slot];
}
template <> CM_DEV df tget<df>(const float* tp, int64_t rs, int v, int64_t slot) {
  return df{tp[int64_t(2 * v) * rs + slot], tp[int64_t(2 * v + 1) * rs + slot]};
}
template <class T> CM_DEV void tput3(float* tp, int64_t rs, int v, int64_t slot, const V3<T>& x) {
  tput(tp, rs, v, slot, x.x); tput(tp, rs, v + 1, slot, x.y); tput(tp, rs, v + 2, slot, x.z);
}
template <class T> CM_DEV V3<T> tget3(const float* tp, int64_t rs, int v, int64_t slot) {
  return {tget<T>(tp, rs, v, slot), tget<T>(tp, rs, v + 1, slot), tget<T>(tp, rs, v + 2, slot)};
}

template <class T> CM_DEV V3<T> mulMc(const M3<T>& R, V3<float> v) {
  return {R.m[0] * v.x + R.m[1] * v.y + R.m[2] * v.z, R.m[3] * v.x + R.m[4] * v.y + R.m[5] * v.z,
          R.m[6] * v.x + R.m[7] * v.y + R.m[8] * v.z};
}
template <class T> CM_DEV V3<T> neg3(V3<T> a) { return {-a.x, -a.y, -a.z}; }

// ------------------------------------------------------------------ poses --
template <class T> struct FrameT {
  M3<T> RM, RS, Rrel;
  V3<T> tM, tS, trel;
};
// Body pose; with duals, the tangent of the world-frame perturbation
// (exp([w]x) R, t + v) along d6 = (w, v): R' = [w]x R, t' = v.
CM_DEV void body_pose(const float* q, const float* t, const float*, M3<float>* R, V3<float>* tt) {
  *R = quat_R(q);
  *tt = {t[0], t[1], t[2]};
}
CM_DEV void body_pose(const float* q, const float* t, const float* d6, M3<df>* R, V3<df>* tt) {
  const M3<float> R0 = quat_R(q);
  for (int j = 0; j < 3; ++j) {
    const float r0 = R0.m[j], r1 = R0.m[3 + j], r2 = R0.m[6 + j];
    R->m[j] = {r0, d6[1] * r2 - d6[2] * r1};
    R->m[3 + j] = {r1, d6[2] * r0 - d6[0] * r2};
    R->m[6 + j] = {r2, d6[0] * r1 - d6[1] * r0};
  }
  *tt = {df{t[0], d6[3]}, df{t[1], d6[4]}, df{t[2], d6[5]}};
}
CM_DEV void setv(float& a, float v) { a = v; }
CM_DEV void setv(df& a, float v) { a.v = v; }
template <class T> CM_DEV FrameT<T> frame_t(const QueryDev& q, int dir, const float* d12) {
  M3<T> RA, RB;
  V3<T> tA, tB;
  body_pose(q.qa, q.ta, d12, &RA, &tA);
  body_pose(q.qb, q.tb, d12 ? d12 + 6 : nullptr, &RB, &tB);
  FrameT<T> F;
  F.RM = dir ? RB : RA;
  F.RS = dir ? RA : RB;
  F.tM = dir ? tB : tA;
  F.tS = dir ? tA : tB;
  // the value parts once rounded from FP64 (tangents: products of FP32 values)
  const Frame32 f = dir ? frame32(q.qb, q.tb, q.qa, q.ta) : frame32(q.qa, q.ta, q.qb, q.tb);
  for (int i = 0; i < 9; ++i) { setv(F.RM.m[i], f.RM[i]); setv(F.RS.m[i], f.RS[i]); }
  F.Rrel = mulMTM(F.RS, F.RM);
  F.trel = mulMT(F.RS, F.tM - F.tS);
  for (int i = 0; i < 9; ++i) setv(F.Rrel.m[i], f.Rrel[i]);
  setv(F.trel.x, f.trel[0]); setv(F.trel.y, f.trel[1]); setv(F.trel.z, f.trel[2]);
  return F;
}

// ------------------------------------------------------- contact forward --
template <class T> struct CF {
  T phi;
  V3<T> g;      // grad phi at the contact point (SDF frame)
  Sym<T> H;     // Hessian of phi there (adjoint only; plane SDFs)
  M3<T> J;      // Jacobian of the normal spline there (adjoint only; spline SDFs)
  T sg;         // sqrt(|g|^2 + eps_n^2) (plane SDFs)
  V3<T> nS;     // normal, SDF frame
  V3<T> N;      // normal, world
  V3<T> p;      // contact point, world
  V3<T> prest;  // point a filtered contact would carry (vertex / edge midpoint)
  T f, fd;      // transition f_t(phi) and its derivative
  T d;          // mollified depth
};

// The contact normal: for plane SDFs the normalised gradient (set here), for
// spline SDFs the normal spline's value (set by the evaluation, Sec. III-B.2).
template <class T, int REP> CM_DEV void finish_contact(CF<T>& c, const FrameT<T>& F, const DevParams& P) {
  if (REP != kRepSpline) {
    c.sg = sqrtT(dot(c.g, c.g) + P.eps_n2);
    c.nS = c.g * (cst<T>(1.f) / c.sg);
  }
  c.N = mulM(F.RS, c.nS);
  // C2 transition (Sec. IV-C.1): quintic smoothstep and its derivative
  const T s = (P.d_max - c.phi) * P.inv_eps_t;
  if (val(s) <= 0.f) {
    c.f = cst<T>(0.f); c.fd = cst<T>(0.f);
  } else if (val(s) >= 1.f) {
    c.f = cst<T>(1.f); c.fd = cst<T>(0.f);
  } else {
    const T s2 = s * s, om = cst<T>(1.f) - s;
    c.f = s2 * s * (10.f - 15.f * s + 6.f * s2);
    c.fd = s2 * om * om * (-30.f * P.inv_eps_t);
  }
  c.d = c.f * c.phi + (cst<T>(1.f) - c.f) * P.d_max;
}

// SDF evaluations for either representation.  Trace points: phi at NP points
// (GRAD: and its gradient, for the adjoint).  Spline evaluations count 64
// terms of work each.
template <int REP, int NP, bool GRAD, class T>
CM_DEV void sdf_points(const ObjDesc& S, const DevParams& P, const V3<T>* x, SdfRes<T>* r, uint64_t* work) {
  if constexpr (REP == kRepPlanes) {
    sdf_eval<NP, GRAD ? 1 : 0, T>(S, P, x, r, work);
  } else if constexpr (REP == kRepPrims) {
    for (int p = 0; p < NP; ++p) {
      const Jt<T, GRAD ? 1 : 0> j = prims_eval<T, GRAD ? 1 : 0>(S, x[p], P);
      r[p].phi = j.v;
      if (GRAD) r[p].g = V3<T>{j.g[0], j.g[1], j.g[2]};
    }
    if (work) *work += uint64_t(64 * NP * S.gn);
  } else {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      SplRes<T> q;
      spline_eval<GRAD, false, false, T>(S, x[p], q);
      r[p].phi = q.phi;
      if (GRAD) r[p].g = q.g;
    }
    if (work) *work += uint64_t(64 * NP);
  }
}
// The contact point: phi and what the normal needs (plane SDFs: the gradient;
// spline SDFs: the normal spline); HIST: also what the adjoint needs (the
// Hessian of phi, or the gradient of phi and the normal spline's Jacobian).
template <int REP, bool HIST, class T>
CM_DEV void sdf_contact(const ObjDesc& S, const DevParams& P, const V3<T>& x, CF<T>& c, uint64_t* work) {
  if constexpr (REP == kRepPlanes) {
    SdfRes<T> r;
    sdf_eval<1, HIST ? 2 : 1, T>(S, P, &x, &r, work);
    c.phi = r.phi;
    c.g = r.g;
    if (HIST) c.H = r.H;
  } else if constexpr (REP == kRepPrims) {
    const Jt<T, HIST ? 2 : 1> j = prims_eval<T, HIST ? 2 : 1>(S, x, P);
    c.phi = j.v;
    c.g = V3<T>{j.g[0], j.g[1], j.g[2]};
    if (HIST) c.H = Sym<T>{j.h[0], j.h[1], j.h[2], j.h[3], j.h[4], j.h[5]};
    if (work) *work += uint64_t(64 * S.gn);
  } else {
    SplRes<T> q;
    spline_eval<HIST, true, HIST, T>(S, x, q);
    c.phi = q.phi;
    if (HIST) { c.g = q.g; c.J = q.J; }
    c.nS = q.n;
    if (work) *work += 64;
  }
}

// Vertex-SDF contact (Sec. IV-B): the vertex itself is the contact point.
// HIST: also what the adjoint needs.
template <class T, bool HIST, int REP>
CM_DEV void vertex_fwd(const ObjDesc& M, const ObjDesc& S, const FrameT<T>& F, int vi, const DevParams& P,
                       CF<T>& c, uint64_t* work) {
  const V3<float> v = vert(M, vi);
  V3<T> x = mulMc(F.Rrel, v) + F.trel;
  sdf_contact<REP, HIST, T>(S, P, x, c, work);
  c.p = mulMc(F.RM, v) + F.tM;
  c.prest = c.p;
  finish_contact<T, REP>(c, F, P);
}

// The same contact rebuilt from its tape record (phi, gradient, Hessian).
template <class T>
CM_DEV void vertex_load(const ObjDesc& M, const FrameT<T>& F, int vi, const DevParams& P, const float* tp,
                        int64_t rs, int64_t slot, CF<T>& c) {
  const V3<float> v = vert(M, vi);
  c.phi = tget<T>(tp, rs, 0, slot);
  c.g = tget3<T>(tp, rs, 1, slot);
  c.H = {tget<T>(tp, rs, 4, slot), tget<T>(tp, rs, 5, slot), tget<T>(tp, rs, 6, slot),
         tget<T>(tp, rs, 7, slot), tget<T>(tp, rs, 8, slot), tget<T>(tp, rs, 9, slot)};
  c.p = mulMc(F.RM, v) + F.tM;
  c.prest = c.p;
  finish_contact<T, kRepPlanes>(c, F, P);
}

// Sphere-trace history kept for the adjoint.
template <class T> struct Trace {
  V3<float> v0, v1;
  V3<T> x0, x1, e, pe;
  T L, aK, bK, ac, bc;
  T al[kMaxTraceAdj], be[kMaxTraceAdj], pa[kMaxTraceAdj], pb[kMaxTraceAdj];
  V3<T> ga[kMaxTraceAdj], gb[kMaxTraceAdj];
};

// Edge geometry in the SDF frame: corners, length, direction.
template <class T>
CM_DEV void edge_setup(const ObjDesc& M, const FrameT<T>& F, int ei, Trace<T>& tr) {
  const I2 ed = M.edges[ei];
  tr.v0 = vert(M, ed.x);
  tr.v1 = vert(M, ed.y);
  tr.x0 = mulMc(F.Rrel, tr.v0) + F.trel;
  tr.x1 = mulMc(F.Rrel, tr.v1) + F.trel;
  const V3<T> dv = tr.x1 - tr.x0;
  tr.L = sqrtT(dot(dv, dv));
  tr.e = dv * (cst<T>(1.f) / tr.L);
}

// Softclipped arc lengths and the edge point from the traced ones.
template <class T>
CM_DEV void edge_point(Trace<T>& tr, T al, T be, const DevParams& P) {
  tr.aK = al;
  tr.bK = be;
  tr.ac = softclip0T(al, tr.L, P.tau_clip, P.inv_tau_clip);
  tr.bc = softclip0T(be, tr.L, P.tau_clip, P.inv_tau_clip);
  tr.pe = (tr.x0 + tr.e * tr.ac + tr.x1 - tr.e * tr.bc) * 0.5f;
}

template <class T, int REP>
CM_DEV void edge_contact(const ObjDesc& M, const FrameT<T>& F, const DevParams& P, const Trace<T>& tr, CF<T>& c) {
  c.p = mulM(F.RS, tr.pe) + F.tS;
  c.prest = mulMc(F.RM, (tr.v0 + tr.v1) * 0.5f) + F.tM;
  finish_contact<T, REP>(c, F, P);
}

// Edge-SDF contact (Sec. IV-B.2, Fig. e_s): trace both corners towards each
// other with the gated step sigma(phi / tau_s) phi, K steps (both ends share
// each pass over the planes), softclip the arc lengths to [0, L] and take the
// midpoint of the two points.  HIST: keep the trace and the Hessian; with a
// tape (tp != nullptr) the trace steps go to the tape as they are computed
// instead of being kept.
template <class T, bool HIST, int REP>
CM_DEV void edge_fwd(const ObjDesc& M, const ObjDesc& S, const FrameT<T>& F, int ei, const DevParams& P, CF<T>& c,
                     Trace<T>& tr, uint64_t* work, float* tp = nullptr, int64_t rs = 0, int64_t slot = 0) {
  edge_setup(M, F, ei, tr);
  T al = cst<T>(0.f), be = cst<T>(0.f);
  if (HIST) {
#pragma unroll
    for (int k = 0; k < kMaxTraceAdj; ++k) {
      if (k < P.st_iters) {
        V3<T> xs[2] = {tr.x0 + tr.e * al, tr.x1 - tr.e * be};
        SdfRes<T> r[2];
        sdf_points<REP, 2, true, T>(S, P, xs, r, work);
        if (tp != nullptr) {
          const int v = kTapeFixed + kTapeStep * k;
          tput(tp, rs, v, slot, r[0].phi);
          tput(tp, rs, v + 1, slot, r[1].phi);
          tput3(tp, rs, v + 2, slot, r[0].g);
          tput3(tp, rs, v + 5, slot, r[1].g);
        } else {
          tr.al[k] = al; tr.be[k] = be;
          tr.pa[k] = r[0].phi; tr.pb[k] = r[1].phi;
          tr.ga[k] = r[0].g; tr.gb[k] = r[1].g;
        }
        al = al + sigmoidT(r[0].phi * P.inv_tau_st) * r[0].phi;
        be = be + sigmoidT(r[1].phi * P.inv_tau_st) * r[1].phi;
      }
    }
  } else {
    for (int k = 0; k < P.st_iters; ++k) {
      V3<T> xs[2] = {tr.x0 + tr.e * al, tr.x1 - tr.e * be};
      SdfRes<T> r[2];
      sdf_points<REP, 2, false, T>(S, P, xs, r, work);
      al = al + sigmoidT(r[0].phi * P.inv_tau_st) * r[0].phi;
      be = be + sigmoidT(r[1].phi * P.inv_tau_st) * r[1].phi;
    }
  }
  edge_point(tr, al, be, P);
  sdf_contact<REP, HIST, T>(S, P, tr.pe, c, work);
  edge_contact<T, REP>(M, F, P, tr, c);
}

// The same contact rebuilt from its tape record: the trace steps replayed from
// the stored phi values, the rest from the stored phi, gradient and Hessian.
template <class T>
CM_DEV void edge_load(const ObjDesc& M, const FrameT<T>& F, int ei, const DevParams& P, const float* tp, int64_t rs,
                      int64_t slot, CF<T>& c, Trace<T>& tr) {
  edge_setup(M, F, ei, tr);
  T al = cst<T>(0.f), be = cst<T>(0.f);
#pragma unroll
  for (int k = 0; k < kMaxTraceAdj; ++k) {
    if (k < P.st_iters) {
      const int v = kTapeFixed + kTapeStep * k;
      tr.al[k] = al; tr.be[k] = be;
      tr.pa[k] = tget<T>(tp, rs, v, slot);
      tr.pb[k] = tget<T>(tp, rs, v + 1, slot);
      tr.ga[k] = tget3<T>(tp, rs, v + 2, slot);
      tr.gb[k] = tget3<T>(tp, rs, v + 5, slot);
      al = al + sigmoidT(tr.pa[k] * P.inv_tau_st) * tr.pa[k];
      be = be + sigmoidT(tr.pb[k] * P.inv_tau_st) * tr.pb[k];
    }
  }
  edge_point(tr, al, be, P);
  c.phi = tget<T>(tp, rs, 0, slot);
  c.g = tget3<T>(tp, rs, 1, slot);
  c.H = {tget<T>(tp, rs, 4, slot), tget<T>(tp, rs, 5, slot), tget<T>(tp, rs, 6, slot),
         tget<T>(tp, rs, 7, slot), tget<T>(tp, rs, 8, slot), tget<T>(tp, rs, 9, slot)};
  edge_contact<T, kRepPlanes>(M, F, P, tr, c);
}

// Writes the contact-point part of a tape record (the trace steps of an edge
// were written by edge_fwd).
template <class T>
CM_DEV void tape_store(const CF<T>& c, float* tp, int64_t rs, int64_t slot) {
  tput(tp, rs, 0, slot, c.phi);
  tput3(tp, rs, 1, slot, c.g);
  tput(tp, rs, 4, slot, c.H.xx); tput(tp, rs, 5, slot, c.H.yy); tput(tp, rs, 6, slot, c.H.zz);
  tput(tp, rs, 7, slot, c.H.xy); tput(tp, rs, 8, slot, c.H.xz); tput(tp, rs, 9, slot, c.H.yz);
}

// ------------------------------------------------------- contact adjoint --
// Adjoint seeds of one piece's blend for L = <c, y>: u_bar = (c_d, c_p, m_bar,
// c_q, c_W) pairs with the contact values u_i = (d, p_c, n_c, f p, f); the
// blended values (d, p, m, q, W) of the piece, i.e. sum_i w_i u_i; c_logZ; logZ.
template <class T> struct GAdj {
  T cd;
  V3<T> cp, mb, cq;
  T cW, clz, logZ;
  T yd;
  V3<T> yp, ym, yq;
  T yW;
};
template <class T> CM_DEV V3<T> getV3(const float* o, int i) {
  constexpr int s = nT<T>();
  return {getT<T>(o + i * s), getT<T>(o + (i + 1) * s), getT<T>(o + (i + 2) * s)};
}
template <class T> CM_DEV void putV3(float* o, int i, const V3<T>& v) {
  constexpr int s = nT<T>();
  putT(o + i * s, v.x); putT(o + (i + 1) * s, v.y); putT(o + (i + 2) * s, v.z);
}
template <class T> CM_DEV GAdj<T> load_gadj(const float* o) {
  constexpr int s = nT<T>();
  GAdj<T> a;
  a.cd = getT<T>(o);
  a.cp = getV3<T>(o, 1);
  a.mb = getV3<T>(o, 4);
  a.cq = getV3<T>(o, 7);
  a.cW = getT<T>(o + 10 * s);
  a.clz = getT<T>(o + 11 * s);
  a.logZ = getT<T>(o + 12 * s);
  a.yd = getT<T>(o + 13 * s);
  a.yp = getV3<T>(o, 14);
  a.ym = getV3<T>(o, 17);
  a.yq = getV3<T>(o, 20);
  a.yW = getT<T>(o + 23 * s);
  return a;
}

template <class T> struct PoseGrad {
  V3<T> wM, vM, wS, vS;
};

// Through the blend softmax (Sec. IV-D.2) and the mollification (Sec. IV-C.1):
// adjoints of phi, of the world normal N, of the world point p and of p_rest.
template <class T>
CM_DEV void blend_moll_adj(const CF<T>& c, const GAdj<T>& a, const DevParams& P, T& phib, V3<T>& Nb, V3<T>& pb,
                           V3<T>& prb) {
  const T omf = cst<T>(1.f) - c.f;
  const V3<T> nc = c.N * c.f, pc = c.p * c.f + c.prest * omf, fp = c.p * c.f;
  const T w = expT(c.d * (-P.inv_tau_blend) - a.logZ);
  // d L / d l_i = w_i (<u_bar, u_i - y> + c_logZ), with the differences formed
  // before the products: contacts close to the blend would otherwise cancel
  // terms of the size of the outputs down to their much smaller difference
  const T du = a.cd * (c.d - a.yd) + dot(a.cp, pc - a.yp) + dot(a.mb, nc - a.ym) + dot(a.cq, fp - a.yq) +
               a.cW * (c.f - a.yW);
  const T lb = w * (du + a.clz);
  const T db = w * a.cd - lb * P.inv_tau_blend;    // d L / d d_c
  const V3<T> pcb = a.cp * w, ncb = a.mb * w, fpb = a.cq * w;
  const T fb = w * a.cW + db * (c.phi - P.d_max) + dot(ncb, c.N) + dot(pcb, c.p - c.prest) + dot(fpb, c.p);
  phib = db * c.f + fb * c.fd;
  Nb = ncb * c.f;
  pb = (pcb + fpb) * c.f;
  prb = pcb * omf;
}

// Through N = R_S n_S and phi: adjoint of the contact point in the SDF frame.
// Plane SDFs, n_S = g / sqrt(|g|^2 + eps^2): x_bar = phi_bar grad phi + H g_bar.
// Spline SDFs, n_S the normal spline: x_bar = phi_bar grad phi + J^T n_S_bar.
template <class T, int REP>
CM_DEV V3<T> point_adj(const CF<T>& c, const FrameT<T>& F, T phib, V3<T> Nb, PoseGrad<T>& G) {
  G.wS = G.wS + cross(c.N, Nb);
  const V3<T> nSb = mulMT(F.RS, Nb);
  if (REP == kRepSpline) return c.g * phib + mulMT(c.J, nSb);
  const V3<T> gb = (nSb - c.nS * dot(c.nS, nSb)) * (cst<T>(1.f) / c.sg);
  return c.g * phib + mulS(c.H, gb);
}

template <class T, int REP>
CM_DEV void vertex_adj(const CF<T>& c, const FrameT<T>& F, const GAdj<T>& a, const DevParams& P, PoseGrad<T>& G) {
  T phib;
  V3<T> Nb, pb, prb;
  blend_moll_adj(c, a, P, phib, Nb, pb, prb);
  const V3<T> xb = point_adj<T, REP>(c, F, phib, Nb, G);
  const V3<T> xbw = mulM(F.RS, xb);
  const V3<T> Pb = pb + prb + xbw;  // p = p_rest = R_M v + t_M; x = R_S^T (p - t_S)
  G.wM = G.wM + cross(c.p - F.tM, Pb);
  G.vM = G.vM + Pb;
  G.wS = G.wS - cross(c.p - F.tS, xbw);
  G.vS = G.vS - xbw;
}

// Adjoint of the sphere trace: given the adjoint of p^e (SDF frame), the
// adjoints of the two corners in the SDF frame.
template <class T>
CM_DEV void trace_adj(const Trace<T>& tr, V3<T> peb, const DevParams& P, V3<T>& x0b, V3<T>& x1b) {
  x0b = peb * 0.5f;
  x1b = peb * 0.5f;
  const T pee = dot(peb, tr.e);
  const T acb = pee * 0.5f, bcb = pee * (-0.5f);
  V3<T> eb = peb * ((tr.ac - tr.bc) * 0.5f);
  // s_clip(x, 0, L) = s_+(x) - s_+(x - L): d/dx = sig(x/tau) - sig((x-L)/tau), d/dL = sig((x-L)/tau)
  const T sa0 = sigmoidT(tr.aK * P.inv_tau_clip), sa1 = sigmoidT((tr.aK - tr.L) * P.inv_tau_clip);
  const T sb0 = sigmoidT(tr.bK * P.inv_tau_clip), sb1 = sigmoidT((tr.bK - tr.L) * P.inv_tau_clip);
  const T Lb = acb * sa1 + bcb * sb1;
  T ab = acb * (sa0 - sa1), bb = bcb * (sb0 - sb1);
#pragma unroll
  for (int kk = kMaxTraceAdj - 1; kk >= 0; --kk) {
    if (kk < P.st_iters) {
      // alpha_{k+1} = alpha_k + G(phi(x0 + alpha_k e)), G(phi) = sigma(phi / tau_s) phi
      const T sa = sigmoidT(tr.pa[kk] * P.inv_tau_st);
      const T Ga = sa + tr.pa[kk] * P.inv_tau_st * sa * (cst<T>(1.f) - sa);
      const T c1 = ab * Ga;
      x0b = x0b + tr.ga[kk] * c1;
      eb = eb + tr.ga[kk] * (c1 * tr.al[kk]);
      ab = ab + c1 * dot(tr.ga[kk], tr.e);
      // beta_{k+1} = beta_k + G(phi(x1 - beta_k e))
      const T sb = sigmoidT(tr.pb[kk] * P.inv_tau_st);
      const T Gb = sb + tr.pb[kk] * P.inv_tau_st * sb * (cst<T>(1.f) - sb);
      const T c2 = bb * Gb;
      x1b = x1b + tr.gb[kk] * c2;
      eb = eb - tr.gb[kk] * (c2 * tr.be[kk]);
      bb = bb - c2 * dot(tr.gb[kk], tr.e);
    }
  }
  // e = d / |d|, L = |d|, d = x1 - x0
  const V3<T> db = (eb - tr.e * dot(tr.e, eb)) * (cst<T>(1.f) / tr.L) + tr.e * Lb;
  x1b = x1b + db;
  x0b = x0b - db;
}

template <class T, int REP>
CM_DEV void edge_adj(const CF<T>& c, const Trace<T>& tr, const FrameT<T>& F, const GAdj<T>& a, const DevParams& P,
                     PoseGrad<T>& G) {
  T phib;
  V3<T> Nb, pb, prb;
  blend_moll_adj(c, a, P, phib, Nb, pb, prb);
  const V3<T> xb = point_adj<T, REP>(c, F, phib, Nb, G);
  // p = R_S p^e + t_S
  G.wS = G.wS + cross(c.p - F.tS, pb);
  G.vS = G.vS + pb;
  const V3<T> peb = mulMT(F.RS, pb) + xb;
  V3<T> x0b, x1b;
  trace_adj(tr, peb, P, x0b, x1b);
  const V3<T> P0 = mulMc(F.RM, tr.v0) + F.tM, P1 = mulMc(F.RM, tr.v1) + F.tM;
  const V3<T> x0w = mulM(F.RS, x0b), x1w = mulM(F.RS, x1b);
  G.wS = G.wS - cross(P0 - F.tS, x0w) - cross(P1 - F.tS, x1w);
  G.vS = G.vS - x0w - x1w;
  const V3<T> P0b = x0w + prb * 0.5f, P1b = x1w + prb * 0.5f;
  G.wM = G.wM + cross(P0 - F.tM, P0b) + cross(P1 - F.tM, P1b);
  G.vM = G.vM + P0b + P1b;
}

// ------------------------------------------------------------ narrow kernel --
// One persistent launch; waves pop tiles (one entry's <= 64 surviving
// contacts) from a counter.
//   ADJ = false, TAPE = false  forward: tile blend partials
//   ADJ = false, TAPE = true   forward before an adjoint: partials, and the
//                              tape records of tiles [0, tape_tiles)
//   ADJ = true,  TAPE = true   adjoint of tiles [0, tape_tiles) from the tape
//   ADJ = true,  TAPE = false  adjoint of tiles [t_begin, total), recomputing
// Waves per SIMD the compiler must leave room for: 4 for the forward plane
// sweep in floats (records only), 3 for the float forward sweep keeping the
// tape (gradient without H v), no constraint for the others.
template <class T, bool ADJ, bool TAPE, int REP> struct NarrowWaves {
  static constexpr int value = (nT<T>() == 1 && !ADJ && REP == kRepPlanes) ? (TAPE ? 3 : 4) : 1;
};
template <class T, bool ADJ, bool TAPE, int REP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NarrowWaves<T, ADJ, TAPE, REP>::value))) void
k_narrow(NarrowArgs a) {
  static_assert(REP == kRepPlanes || !TAPE, "spline and primitive SDFs recompute instead of taping");
  const int l = lane();
  const int64_t n_run = a.dc->R;
  const ObjDesc* __restrict__ objs = a.dc->objs;
  const int64_t total = a.tile_off[n_run];
  const int64_t t_end = (ADJ && TAPE) ? min(total, a.tape_tiles) : total;
  const int64_t t_begin = (ADJ && !TAPE) ? a.t_begin : 0;
  const int64_t rs = a.tape_tiles * kWave;
  const DevParams& P = a.P;
  constexpr bool HIST = ADJ || TAPE;  // Hessian and trace history
  uint64_t work[2] = {0, 0};          // point-plane evaluations per lane by contact kind (wave-uniform)
  // One queue per XCD (workgroups are dispatched to the XCDs in turn): the
  // sweep's tiles, in queue order, form chunks of kChunk consecutive tiles
  // dealt to the queues in turn, so the tiles of a run (one query direction,
  // one SDF object) are mostly taken by waves of one XCD and its L2 serves the
  // object's planes to all of them.  Queue xq holds chunks xq, xq + kQueues, ...
  const int xq = int(blockIdx.x) & (kQueues - 1);
  const int64_t n_t = t_end > t_begin ? t_end - t_begin : 0;
  const int64_t n_ch = (n_t + kChunk - 1) / kChunk;
  const int64_t n_pop = n_ch > xq ? ((n_ch - 1 - xq) / kQueues + 1) * kChunk : 0;
  // each pop returns a distinct index of the queue, so a wave pops at most n_pop + 1 times
  for (int64_t it = 0; it <= n_pop; ++it) {
    uint32_t i0 = 0;
    if (l == 0) i0 = atomicAdd(a.counter + xq, 1u);
    const int64_t i = int64_t(uint32_t(uni(int(i0))));
    if (i >= n_pop) break;
    const int64_t t = t_begin + ((i / kChunk) * kQueues + xq) * kChunk + (i % kChunk);
    if (t >= t_end) continue;  // past the last tile (in the sweep's last chunk)
    // the tile: 64 consecutive survivors of a run (one query, direction, kind)
    const int64_t r = last_le(a.tile_off, 0, n_run, t);
    const int64_t j = t - a.tile_off[r];
    const int64_t eb = a.run_off[r], ee = a.run_off[r + 1];
    const int64_t sb = a.surv_off[eb];
    const int64_t rank = j * kWave + l;
    const bool valid = rank < a.surv_off[ee] - sb;
    const int64_t rk = valid ? rank : j * kWave;  // lane 0 always holds a survivor
    // this lane's entry (piece of the mesh side) and survivor within it
    const int64_t e = last_le(a.surv_off, eb, ee, sb + rk);
    const Entry E = a.ents[e];
    const int c = entry_survivor(a.bits, a.wpre, E, int(sb + rk - a.surv_off[e]));
    const Entry E0 = ldc(a.ents + eb);  // query, direction, kind, objects: uniform over the run
    const QueryDev q = ldc(a.Q + E0.query);
    const ObjDesc M = ldc(objs + E0.mesh_obj);
    const ObjDesc S = ldc(objs + E0.sdf_obj);
    const PieceDesc& pd = M.pieces[E.piece];
    const int ci = E0.kind == 0 ? pd.vert_begin + c : pd.edge_begin + c;
    const float* d12 = (nT<T>() == 2) ? a.dir + 12 * int64_t(E0.query) : nullptr;
    const FrameT<T> F = frame_t<T>(q, E0.dir, d12);
    CF<T> ct;
    Trace<T> tr;
    const int64_t slot = t * kWave + l;
    if constexpr (ADJ && TAPE) {
      if (E0.kind == 0) vertex_load<T>(M, F, ci, P, a.tape, rs, slot, ct);
      else edge_load<T>(M, F, ci, P, a.tape, rs, slot, ct, tr);
    } else {
      // the store sweep writes the records of taped tiles
      float* tp = (!ADJ && TAPE && t < a.tape_tiles) ? a.tape : nullptr;
      if (E0.kind == 0) vertex_fwd<T, HIST, REP>(M, S, F, ci, P, ct, &work[0]);
      else edge_fwd<T, HIST, REP>(M, S, F, ci, P, ct, tr, &work[1], tp, rs, slot);
      if constexpr (TAPE) {
        if (tp != nullptr) tape_store(ct, tp, rs, slot);
      }
    }
    if (!ADJ) {
      // online softmax over l_i = -d_c,i / tau_b, one partial per piece present
      // in the tile (its survivors are consecutive lanes)
      const T li = ct.d * (-P.inv_tau_blend);
      const T omf = cst<T>(1.f) - ct.f;
      const V3<T> nc = ct.N * ct.f, pc = ct.p * ct.f + ct.prest * omf, fp = ct.p * ct.f;
      const int e_first = uni(int(e));
      const int e_last = wmax_i(valid ? int(e) : e_first);
      for (int ex = e_first; ex <= e_last; ++ex) {
        const bool in = valid && int(e) == ex;
        if (!__any(in)) continue;
        const float Lam = wmax(in ? val(li) : -__builtin_inff());
        const T w = in ? expT(li - Lam) : cst<T>(0.f);
        T acc[13] = {w, w * ct.d, w * nc.x, w * nc.y, w * nc.z, w * pc.x, w * pc.y, w * pc.z,
                     w * fp.x, w * fp.y, w * fp.z, w * ct.f, cst<T>(in ? 1.f : 0.f)};
#pragma unroll
        for (int i = 0; i < 13; ++i) acc[i] = wsum(acc[i]);
        const int64_t k = j - (a.surv_off[ex] - sb) / kWave;  // the entry's k-th partial
        float* o = a.partials + (a.part_off[ex] + k) * kStride;
        if (l == 0) {
          o[0] = Lam;
#pragma unroll
          for (int i = 0; i < 13; ++i) putT(o + 1 + i * nT<T>(), acc[i]);
        }
      }
      if (nT<T>() == 1 && a.dbg != nullptr && valid) {
        const int64_t cidx = E.contact_base + c;
        const float rec[13] = {1.f, val(ct.d), val(ct.f), 0.f, val(pc.x), val(pc.y), val(pc.z), val(nc.x),
                               val(nc.y), val(nc.z), val(ct.phi), float(E0.kind), __int_as_float(E.group)};
#pragma unroll
        for (int rr = 0; rr < 13; ++rr) a.dbg[rr * a.C + cidx] = rec[rr];
      }
    } else {
      const GAdj<T> ga = load_gadj<T>(a.gscratch + int64_t(E.group) * kGStride);
      PoseGrad<T> G{zero3<T>(), zero3<T>(), zero3<T>(), zero3<T>()};
      if (E0.kind == 0) vertex_adj<T, REP>(ct, F, ga, P, G);
      else edge_adj<T, REP>(ct, tr, F, ga, P, G);
      // (w_A, v_A, w_B, v_B): all lanes of a tile belong to one query
      const V3<T> g4[4] = {E0.dir ? G.wS : G.wM, E0.dir ? G.vS : G.vM, E0.dir ? G.wM : G.wS,
                           E0.dir ? G.vM : G.vS};
      float* o = a.partials + t * kStride;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const T gx = wsum(valid ? g4[i].x : cst<T>(0.f));
        const T gy = wsum(valid ? g4[i].y : cst<T>(0.f));
        const T gz = wsum(valid ? g4[i].z : cst<T>(0.f));
        if (l == 0) {
          putT(o + (3 * i) * nT<T>(), gx);
          putT(o + (3 * i + 1) * nT<T>(), gy);
          putT(o + (3 * i + 2) * nT<T>(), gz);
        }
      }
    }
  }
  if (a.work != nullptr && l == 0) {
    if (work[0] != 0) atomicAdd(a.work, (unsigned long long)(work[0] * kWave));
    if (work[1] != 0) atomicAdd(a.work + 1, (unsigned long long)(work[1] * kWave));
  }
}

// ---------------------------------------------------------------- finalize --
template <class T> struct BlendT {
  float L;
  T Z, d, f;
  V3<T> n, p, q;
};
template <class T> CM_DEV void blend_merge(BlendT<T>& a, float L, const T& Z, const T& d, const V3<T>& n,
                                           const V3<T>& p, const V3<T>& q, const T& f) {
  if (!(val(Z) > 0.f)) return;
  const float Ln = fmaxf(a.L, L);
  const float sa = val(a.Z) > 0.f ? expf(a.L - Ln) : 0.f;
  const float sb = expf(L - Ln);
  a.L = Ln;
  a.Z = a.Z * sa + Z * sb;
  a.d = a.d * sa + d * sb;
  a.n = a.n * sa + n * sb;
  a.p = a.p * sa + p * sb;
  a.q = a.q * sa + q * sb;
  a.f = a.f * sa + f * sb;
}

// World-frame sum of the points of an entry's filtered contacts; with duals
// its tangent follows from the mesh body's perturbation: S' = w x (S - n t) + n v.
template <class T> CM_DEV V3<T> filt_sum(const F4& fl, const QueryDev& q, int dir, const float* d12);
template <> CM_DEV V3<float> filt_sum<float>(const F4& fl, const QueryDev&, int, const float*) {
  return {fl.y, fl.z, fl.w};
}
template <> CM_DEV V3<df> filt_sum<df>(const F4& fl, const QueryDev& q, int dir, const float* d12) {
  const float* d6 = d12 + (dir ? 6 : 0);
  const float* t = dir ? q.tb : q.ta;
  const V3<float> r{fl.y - fl.x * t[0], fl.z - fl.x * t[1], fl.w - fl.x * t[2]};
  const V3<float> w{d6[0], d6[1], d6[2]};
  const V3<float> tt = cross(w, r);
  return {df{fl.y, tt.x + fl.x * d6[3]}, df{fl.z, tt.y + fl.x * d6[4]}, df{fl.w, tt.z + fl.x * d6[5]}};
}

// Fixed-order merge of a piece's contacts: vertices (filtered closed form,
// then tiles) then edges (filtered, then tiles) (Sec. IV-D.2-3).
template <class T> CM_DEV BlendT<T> group_blend(const FinArgs& a, int64_t g) {
  BlendT<T> b;
  b.L = -__builtin_inff();
  b.Z = b.d = b.f = cst<T>(0.f);
  b.n = b.p = b.q = zero3<T>();
  const I2 ge = a.gent[g];
  const DevParams& P = a.P;
  for (int k = 0; k < 2; ++k) {
    const int e = k == 0 ? ge.x : ge.y;
    const F4 fl = a.filt[e];
    if (fl.x > 0.f) {
      const Entry E = ldc(a.ents + e);
      const QueryDev q = ldc(a.Q + E.query);
      const float* d12 = (nT<T>() == 2) ? a.dir + 12 * int64_t(E.query) : nullptr;
      const V3<T> S = filt_sum<T>(fl, q, E.dir, d12);
      blend_merge(b, -P.d_max * P.inv_tau_blend, cst<T>(fl.x), cst<T>(fl.x * P.d_max), zero3<T>(), S, zero3<T>(),
                  cst<T>(0.f));
    }
    for (int64_t t = a.part_off[e]; t < a.part_off[e + 1]; ++t) {
      const float* o = a.partials + t * kStride;
      constexpr int s = nT<T>();
      const T* dummy = nullptr;
      (void)dummy;
      blend_merge(b, o[0], getT<T>(o + 1), getT<T>(o + 1 + s),
                  V3<T>{getT<T>(o + 1 + 2 * s), getT<T>(o + 1 + 3 * s), getT<T>(o + 1 + 4 * s)},
                  V3<T>{getT<T>(o + 1 + 5 * s), getT<T>(o + 1 + 6 * s), getT<T>(o + 1 + 7 * s)},
                  V3<T>{getT<T>(o + 1 + 8 * s), getT<T>(o + 1 + 9 * s), getT<T>(o + 1 + 10 * s)},
                  getT<T>(o + 1 + 11 * s));
    }
  }
  return b;
}

// WHAT 0: write the group records.  WHAT 1: write the per-piece adjoint seeds
// for the cotangent `cot` (n_bar = cot_n, m_bar through the normalisation).
// WHAT 2: both (the records are the value parts).  WHAT 3 (dual numbers): the
// records and, to out_t, their tangents along the direction.
template <class T, int WHAT>
__global__ __launch_bounds__(256) void k_finalize(FinArgs a) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= a.dc->G) return;
  const BlendT<T> b = group_blend<T>(a, g);
  const T iz = cst<T>(1.f) / b.Z;
  const V3<T> m = b.n * iz;
  const T sg = sqrtT(dot(m, m) + a.P.eps_n2);
  const V3<T> n = m * (cst<T>(1.f) / sg);
  const V3<T> p = b.p * iz, q = b.q * iz;
  const T d = b.d * iz, W = b.f * iz;
  const T logZ = logT(b.Z) + b.L;
  const int64_t G = a.G;
  if (WHAT == 0 || WHAT == 2 || WHAT == 3) {
    a.out.p[g] = val(p.x); a.out.p[G + g] = val(p.y); a.out.p[2 * G + g] = val(p.z);
    a.out.n[g] = val(n.x); a.out.n[G + g] = val(n.y); a.out.n[2 * G + g] = val(n.z);
    a.out.q[g] = val(q.x); a.out.q[G + g] = val(q.y); a.out.q[2 * G + g] = val(q.z);
    a.out.d[g] = val(d);
    a.out.W[g] = val(W);
    a.out.logZ[g] = val(logZ);
  }
  if (WHAT == 3) {
    a.out_t.p[g] = tan_(p.x); a.out_t.p[G + g] = tan_(p.y); a.out_t.p[2 * G + g] = tan_(p.z);
    a.out_t.n[g] = tan_(n.x); a.out_t.n[G + g] = tan_(n.y); a.out_t.n[2 * G + g] = tan_(n.z);
    a.out_t.q[g] = tan_(q.x); a.out_t.q[G + g] = tan_(q.y); a.out_t.q[2 * G + g] = tan_(q.z);
    a.out_t.d[g] = tan_(d);
    a.out_t.W[g] = tan_(W);
    a.out_t.logZ[g] = tan_(logZ);
  }
  if (WHAT == 1 || WHAT == 2) {
    const V3<float> cp{a.cot.p[g], a.cot.p[G + g], a.cot.p[2 * G + g]};
    const V3<float> cn{a.cot.n[g], a.cot.n[G + g], a.cot.n[2 * G + g]};
    const V3<float> cq{a.cot.q[g], a.cot.q[G + g], a.cot.q[2 * G + g]};
    const float cd = a.cot.d[g], cW = a.cot.W[g], clz = a.cot.logZ[g];
    const V3<T> cnT = lift3<T>(cn);
    const V3<T> mb = (cnT - n * dot(n, cnT)) * (cst<T>(1.f) / sg);
    float* o = a.gscratch + g * kGStride;
    constexpr int s = nT<T>();
    putT(o, cst<T>(cd));
    putV3(o, 1, lift3<T>(cp));
    putV3(o, 4, mb);
    putV3(o, 7, lift3<T>(cq));
    putT(o + 10 * s, cst<T>(cW));
    putT(o + 11 * s, cst<T>(clz));
    putT(o + 12 * s, logZ);
    putT(o + 13 * s, d);
    putV3(o, 14, p);
    putV3(o, 17, m);
    putV3(o, 20, q);
    putT(o + 23 * s, W);
  }
}

// Per-contact blending weight w_i = exp(l_i - logZ_g) for the debug output.
__global__ void k_dbg_weights(float* __restrict__ dbg, int64_t C, const float* __restrict__ logZ, DevParams P) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int g = __float_as_int(dbg[12 * C + c]);
  dbg[3 * C + c] = expf(-dbg[C + c] * P.inv_tau_blend - logZ[g]);
}

// ----------------------------------------------------------------- reduce --
// Per query, in a fixed order: for each piece (group) its vertex then edge
// entry, the filtered contacts' closed form (their points move with the mesh
// body, with weight exp(-d_max / tau_b - logZ)); then the partials of the
// tiles of its runs.
// With duals, hv = d/de grad - (1/2) w_dir x grad_w per body: the second term
// converts the derivative of the world-frame gradient into the Hessian of
// L(exp([w]x) R, t + v) at zero.
template <class T>
__global__ __launch_bounds__(256) void k_reduce(FinArgs a, const float* __restrict__ bpartials,
                                                const int64_t* __restrict__ group_off,
                                                float* __restrict__ grad, float* __restrict__ hv) {
  const int64_t qi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (qi >= a.dc->n) return;
  T acc[12];
  for (int i = 0; i < 12; ++i) acc[i] = cst<T>(0.f);
  const DevParams& P = a.P;
  const float* d12 = (nT<T>() == 2) ? a.dir + 12 * qi : nullptr;
  for (int64_t g = group_off[qi]; g < group_off[qi + 1]; ++g) {
    const GAdj<T> ga = load_gadj<T>(a.gscratch + g * kGStride);
    const I2 ge = a.gent[g];
    for (int k = 0; k < 2; ++k) {
      const int e = k == 0 ? ge.x : ge.y;
      const F4 fl = a.filt[e];
      if (fl.x > 0.f) {
        const Entry E = ldc(a.ents + e);
        const QueryDev q = ldc(a.Q + E.query);
        const FrameT<T> F = frame_t<T>(q, E.dir, d12);
        const V3<T> S = filt_sum<T>(fl, q, E.dir, d12);
        const T wf = expT(ga.logZ * -1.f - P.d_max * P.inv_tau_blend);
        const V3<T> wM = cross(S - F.tM * fl.x, ga.cp) * wf;
        const V3<T> vM = ga.cp * (wf * fl.x);
        const int o = E.dir ? 6 : 0;
        acc[o + 0] += wM.x; acc[o + 1] += wM.y; acc[o + 2] += wM.z;
        acc[o + 3] += vM.x; acc[o + 4] += vM.y; acc[o + 5] += vM.z;
      }
    }
  }
  // the query's tiles: its four runs (direction, kind) in a fixed order
  for (int k = 0; k < 4; ++k) {
    const int64_t r = a.q_runs[4 * qi + k];
    for (int64_t t = a.tile_off[r]; t < a.tile_off[r + 1]; ++t) {
      const float* o = bpartials + t * kStride;
      for (int i = 0; i < 12; ++i) acc[i] += getT<T>(o + i * nT<T>());
    }
  }
  for (int i = 0; i < 12; ++i) grad[12 * qi + i] = val(acc[i]);
  if (nT<T>() == 2 && hv != nullptr) {
    for (int body = 0; body < 2; ++body) {
      const float* w = d12 + 6 * body;
      const float gw[3] = {val(acc[6 * body]), val(acc[6 * body + 1]), val(acc[6 * body + 2])};
      const float corr[3] = {w[1] * gw[2] - w[2] * gw[1], w[2] * gw[0] - w[0] * gw[2], w[0] * gw[1] - w[1] * gw[0]};
      for (int i = 0; i < 3; ++i) hv[12 * qi + 6 * body + i] = tan_(acc[6 * body + i]) - 0.5f * corr[i];
      for (int i = 3; i < 6; ++i) hv[12 * qi + 6 * body + i] = tan_(acc[6 * body + i]);
    }
  }
}

// ------------------------------------------------------------- launchers --
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Workgroups of `waves` waves of one narrow-phase kernel that a CU keeps
// resident (the occupancy query, cached per kernel and workgroup size; 0 if it
// fails).
template <class T, bool ADJ, bool TAPE, int REP> static int resident_per_cu(int waves) {
  static std::atomic<int> cache[5];  // by waves per workgroup, 1 .. 4; -1: the query failed
  int n = cache[waves].load(std::memory_order_relaxed);
  if (n == 0) {
    int r = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, reinterpret_cast<const void*>(&k_narrow<T, ADJ, TAPE, REP>),
                                                     kWave * waves, 0) != hipSuccess || r <= 0)
      r = -1;
    cache[waves].store(r, std::memory_order_relaxed);
    n = r;
  }
  return std::max(n, 0);
}

void warm_narrow_occupancy() {
  for (int w : {1, 2, 4}) {
    (void)resident_per_cu<float, false, false, kRepPlanes>(w);
    (void)resident_per_cu<float, false, true, kRepPlanes>(w);
    (void)resident_per_cu<float, true, true, kRepPlanes>(w);
    (void)resident_per_cu<float, true, false, kRepPlanes>(w);
    (void)resident_per_cu<df, false, false, kRepPlanes>(w);
    (void)resident_per_cu<df, false, true, kRepPlanes>(w);
    (void)resident_per_cu<df, true, true, kRepPlanes>(w);
    (void)resident_per_cu<df, true, false, kRepPlanes>(w);
    (void)resident_per_cu<float, false, false, kRepSpline>(w);
    (void)resident_per_cu<float, true, false, kRepSpline>(w);
    (void)resident_per_cu<df, false, false, kRepSpline>(w);
    (void)resident_per_cu<df, true, false, kRepSpline>(w);
    (void)resident_per_cu<float, false, false, kRepPrims>(w);
    (void)resident_per_cu<float, true, false, kRepPrims>(w);
    (void)resident_per_cu<df, false, false, kRepPrims>(w);
    (void)resident_per_cu<df, true, false, kRepPrims>(w);
  }
}

// Timing events bracket a group of launches: `first` records the start,
// `last` the stop.  A persistent sweep never launches fewer workgroups than
// the CUs keep resident: the launch shape is tuned on one sweep of a step and
// shared with sweeps that may fit more waves.
template <class T, bool ADJ, bool TAPE>
static void narrow_launch(const NarrowArgs& na, int n_cu, int per_cu, int waves, hipStream_t s, hipEvent_t* ev,
                          bool first = true, bool last = true) {
  waves = std::min(std::max(waves, 1), 4);  // (the kernels' bound: 256 threads)
  const dim3 block(unsigned(kWave * waves));
  const int res = na.rep == kRepSpline ? resident_per_cu<T, ADJ, false, kRepSpline>(waves)
                  : na.rep == kRepPrims ? resident_per_cu<T, ADJ, false, kRepPrims>(waves)
                                        : resident_per_cu<T, ADJ, TAPE, kRepPlanes>(waves);
  const int grid = n_cu * std::max(per_cu, res);
  launch_fill_u32(na.counter, 0u, kQueues, s);
  const int slot = nT<T>() == 1 ? (ADJ ? kTNarrowAdj : kTNarrowFwd) : (ADJ ? kTNarrowDualAdj : kTNarrowTan);
  if (ev && first) (void)hipEventRecord(ev[2 * slot], s);
  if (na.rep == kRepSpline) {
    if constexpr (!TAPE) hipLaunchKernelGGL((k_narrow<T, ADJ, false, kRepSpline>), dim3(unsigned(grid)), block, 0, s,
                                            na);
  } else if (na.rep == kRepPrims) {
    if constexpr (!TAPE) hipLaunchKernelGGL((k_narrow<T, ADJ, false, kRepPrims>), dim3(unsigned(grid)), block, 0, s,
                                            na);
  } else {
    hipLaunchKernelGGL((k_narrow<T, ADJ, TAPE, kRepPlanes>), dim3(unsigned(grid)), block, 0, s, na);
  }
  if (ev && last) (void)hipEventRecord(ev[2 * slot + 1], s);
}

static NarrowArgs narrow_args(const FwdArgs& a, float* partials, const float* dir, float* dbg) {
  NarrowArgs na{};
  na.dc = a.dc;
  na.ents = a.ents; na.n_ent = a.n_ent; na.tile_off = a.tile_off; na.bits = a.bits; na.Q = a.Q; na.objs = a.objs;
  na.run_off = a.run_off; na.surv_off = a.surv_off; na.part_off = a.part_off; na.wpre = a.wpre; na.n_run = a.n_run;
  na.P = a.P; na.counter = a.counter; na.partials = partials; na.gscratch = a.gscratch; na.dir = dir;
  na.dbg = dbg; na.C = a.C;
  na.tape = a.tape; na.tape_tiles = a.tape_tiles; na.tape_nv = a.tape_nv; na.t_begin = 0;
  na.work = a.work;
  na.rep = a.rep;
  return na;
}
static FinArgs fin_args(const FwdArgs& a, const float* partials, const float* dir) {
  FinArgs fa{};
  fa.dc = a.dc;
  fa.G = a.G; fa.gent = a.gent; fa.tile_off = a.tile_off; fa.filt = a.filt; fa.partials = partials;
  fa.part_off = a.part_off; fa.q_runs = a.q_runs;
  fa.ents = a.ents; fa.Q = a.Q; fa.P = a.P; fa.out = a.out; fa.out_t = a.out_t; fa.cot = a.cot;
  fa.gscratch = a.gscratch; fa.dir = dir;
  return fa;
}

// Each launcher reports the launch errors of its own kernels: a stale error
// left by an unrelated runtime call is cleared first.
hipError_t launch_forward(const FwdArgs& a, hipStream_t s) {
  (void)hipGetLastError();
  if (a.work) launch_fill_u32(reinterpret_cast<uint32_t*>(a.work), 0u, 4, s);
  launch_front(a, s);
  narrow_launch<float, false, false>(narrow_args(a, a.partials, nullptr, a.dbg), a.n_cu, a.blocks_per_cu, a.wg_waves, s,
                                     a.ev);
  hipLaunchKernelGGL((k_finalize<float, 0>), dim3(unsigned(cdiv(a.G, 256))), dim3(256), 0, s,
                     fin_args(a, a.partials, nullptr));
  if (a.dbg != nullptr)
    hipLaunchKernelGGL(k_dbg_weights, dim3(unsigned(cdiv(a.C, 256))), dim3(256), 0, s, a.dbg, a.C, a.out.logZ, a.P);
  return hipGetLastError();
}

// Forward sweep (taping), per-piece seeds (and, with records, the group
// records), adjoint from the tape and for tiles past it by recomputation,
// per-query reduction.  T = df adds the tangents along `dir` (H v).
template <class T> static hipError_t adjoint_impl(const FwdArgs& a, hipStream_t s, bool records) {
  (void)hipGetLastError();
  if (a.work) launch_fill_u32(reinterpret_cast<uint32_t*>(a.work), 0u, 4, s);
  launch_front(a, s);
  const int per_cu = nT<T>() == 2 ? a.blocks_per_cu_dual : a.blocks_per_cu;
  const int waves = nT<T>() == 2 ? a.wg_waves_dual : a.wg_waves;
  const float* dir = a.dir;
  const bool tape = a.tape != nullptr && a.tape_tiles > 0;
  if (tape) narrow_launch<T, false, true>(narrow_args(a, a.partials, dir, nullptr), a.n_cu, per_cu, waves, s, a.ev);
  else narrow_launch<T, false, false>(narrow_args(a, a.partials, dir, nullptr), a.n_cu, per_cu, waves, s, a.ev);
  if (records)
    hipLaunchKernelGGL((k_finalize<T, 2>), dim3(unsigned(cdiv(a.G, 256))), dim3(256), 0, s,
                       fin_args(a, a.partials, dir));
  else
    hipLaunchKernelGGL((k_finalize<T, 1>), dim3(unsigned(cdiv(a.G, 256))), dim3(256), 0, s,
                       fin_args(a, a.partials, dir));
  NarrowArgs nb = narrow_args(a, a.bpartials, dir, nullptr);
  if (tape) narrow_launch<T, true, true>(nb, a.n_cu, per_cu, waves, s, a.ev, true, false);
  nb.t_begin = tape ? a.tape_tiles : 0;  // tiles past the tape, if any
  narrow_launch<T, true, false>(nb, a.n_cu, per_cu, waves, s, a.ev, !tape, true);
  hipLaunchKernelGGL((k_reduce<T>), dim3(unsigned(cdiv(a.n, 256))), dim3(256), 0, s, fin_args(a, a.partials, dir),
                     a.bpartials, a.group_off, a.grad, a.hv);
  return hipGetLastError();
}

hipError_t launch_jvp(const FwdArgs& a, hipStream_t s) {
  (void)hipGetLastError();
  if (a.work) launch_fill_u32(reinterpret_cast<uint32_t*>(a.work), 0u, 4, s);
  launch_front(a, s);
  narrow_launch<df, false, false>(narrow_args(a, a.partials, a.dir, nullptr), a.n_cu, a.blocks_per_cu_dual,
                                  a.wg_waves_dual, s, a.ev);
  hipLaunchKernelGGL((k_finalize<df, 3>), dim3(unsigned(cdiv(a.G, 256))), dim3(256), 0, s,
                     fin_args(a, a.partials, a.dir));
  return hipGetLastError();
}

hipError_t launch_backward(const FwdArgs& a, hipStream_t s, bool records) { return adjoint_impl<float>(a, s, records); }
hipError_t launch_hvp(const FwdArgs& a, hipStream_t s, bool records) { return adjoint_impl<df>(a, s, records); }

}  // namespace cm
