// gfx950 kernels of the contact-manifold hot path: voxel-grid build, broad
// phase with survivor bitmasks, survivor-tile scan, the persistent narrow
// phase (vertex-SDF and edge-SDF contacts, mollification, per-tile blend
// partials) and the fixed-order per-piece finalize.
//
// One wavefront of 64 lanes handles one tile: up to 64 surviving contacts of
// one piece (vertices or edges).  Every lane evaluates the opposing object's
// SDF, streaming its planes through wave-uniform scalar loads.  Reductions are
// in a fixed order (xor butterflies within a wave, tiles in index order per
// piece) so a query's result does not depend on the rest of its batch.
#include "devmath.h"
#include "kernels.h"

namespace cm {

// ----------------------------------------------------------- wave helpers --
CM_DEV int lane() { return int(threadIdx.x) & (kWave - 1); }
CM_DEV float wsum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
CM_DEV float wmax(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}
CM_DEV int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }


// Index of the k-th set bit (k counted from 0) of a 64-bit word.
CM_DEV int kth_bit(uint64_t w, int k) {
  int pos = 0;
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    const uint64_t low = w & ((uint64_t(1) << s) - 1);
    const int c = __popcll(low);
    if (k >= c) { k -= c; w >>= s; pos += s; } else { w = low; }
  }
  return pos;
}

// Poses of one direction: mesh-side body (R_M, t_M), SDF-side body (R_S, t_S)
// and the mesh -> SDF-frame transform x = R_S^T (R_M v + t_M - t_S).
struct Frame {
  M3<float> RM, RS, Rrel;
  V3<float> tM, tS, trel;
};
CM_DEV Frame make_frame(const QueryDev& q, int dir) {
  Frame F;
  const M3<float> RA = quat_R(q.qa), RB = quat_R(q.qb);
  const V3<float> tA{q.ta[0], q.ta[1], q.ta[2]}, tB{q.tb[0], q.tb[1], q.tb[2]};
  F.RM = dir ? RB : RA;
  F.RS = dir ? RA : RB;
  F.tM = dir ? tB : tA;
  F.tS = dir ? tA : tB;
  F.Rrel = mulMTM(F.RS, F.RM);
  F.trel = mulMT(F.RS, F.tM - F.tS);
  return F;
}

CM_DEV V3<float> vert(const ObjDesc& o, int i) { return {o.vx[i], o.vy[i], o.vz[i]}; }

// --------------------------------------------------------------- grid build --
// phi of the object at every voxel centre (Sec. IV-C.2).
__global__ __launch_bounds__(256) void k_grid_build(const ObjDesc* __restrict__ objs, const int32_t* __restrict__ ids,
                                                    int32_t blocks_per_obj, DevParams P) {
  const int oi = uni(int(blockIdx.x) / blocks_per_obj);
  const int obj = uni(ids[oi]);
  const ObjDesc o = ldc(objs + obj);
  const int n = o.gn;
  const int n3 = n * n * n;
  const int v0 = (int(blockIdx.x) % blocks_per_obj) * 256 + int(threadIdx.x);
  const int v = min(v0, n3 - 1);
  const int i = v / (n * n), j = (v / n) % n, k = v % n;
  V3<float> c{o.gorg[0] + (float(i) + 0.5f) * o.gh[0], o.gorg[1] + (float(j) + 0.5f) * o.gh[1],
              o.gorg[2] + (float(k) + 0.5f) * o.gh[2]};
  SdfRes<float> r;
  sdf_eval<1, 0, float>(o, P, &c, &r);
  if (v0 < n3) const_cast<float*>(o.grid)[v] = r.phi;
}

// ------------------------------------------------------------- broad phase --
// One wave per entry: voxel-grid lower bound of every contact, a survivor
// bitmask word per 64 contacts (Sec. IV-C.2: a vertex is filtered when
// phi(p_c) - r >= d_max, an edge when min(lb_1, lb_2) - l >= d_max), and the
// count and world-frame point sum of filtered contacts, which enter the blend
// with (d_max, 0, 0) in closed form.
__global__ __launch_bounds__(256) void k_broad(const Entry* __restrict__ ents, int64_t n_ent,
                                               const QueryDev* __restrict__ Q, const ObjDesc* __restrict__ objs,
                                               DevParams P, uint64_t* __restrict__ bits, int32_t* __restrict__ nsurv,
                                               int32_t* __restrict__ ntiles, F4* __restrict__ filt,
                                               float* __restrict__ dbg, int64_t C) {
  const int l = lane();
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (int64_t(gridDim.x) * blockDim.x) >> 6;
  for (int64_t e = wave; e < n_ent; e += nwaves) {
    const Entry E = ldc(ents + e);
    const QueryDev q = ldc(Q + E.query);
    const ObjDesc M = ldc(objs + E.mesh_obj);
    const ObjDesc S = ldc(objs + E.sdf_obj);
    const PieceDesc pd = ldc(M.pieces + E.piece);
    const Frame F = make_frame(q, E.dir);
    int ns = 0;
    float fc = 0.f;
    V3<float> fp{0.f, 0.f, 0.f};
    for (int base = 0; base < E.count; base += kWave) {
      const int c = base + l;
      const bool valid = c < E.count;
      const int cc = valid ? c : 0;
      bool surv;
      V3<float> prest;
      if (E.kind == 0) {
        const V3<float> v = vert(M, pd.vert_begin + cc);
        const V3<float> x = mulM(F.Rrel, v) + F.trel;
        surv = !P.broad_phase || grid_lb(S, x) < P.d_max;
        prest = mulM(F.RM, v) + F.tM;
      } else {
        const I2 ed = M.edges[pd.edge_begin + cc];
        const V3<float> v0 = vert(M, ed.x), v1 = vert(M, ed.y);
        const V3<float> x0 = mulM(F.Rrel, v0) + F.trel, x1 = mulM(F.Rrel, v1) + F.trel;
        if (P.broad_phase) {
          const V3<float> dv = x1 - x0;
          const float L = sqrtf(dot(dv, dv));
          const float la = grid_lb(S, x0), lb = grid_lb(S, x1);
          const float bound = P.edge_bound == 0 ? fminf(la, lb) - L : fmaxf(fmaxf(la, lb) - L, 0.5f * (la + lb - L));
          surv = bound < P.d_max;
        } else {
          surv = true;
        }
        prest = mulM(F.RM, (v0 + v1) * 0.5f) + F.tM;
      }
      const uint64_t word = __ballot(valid && surv);
      if (l == 0) bits[E.word_off + base / kWave] = word;
      ns += __popcll(word);
      if (valid && !surv) { fc += 1.f; fp = fp + prest; }
      if (dbg != nullptr && valid && !surv) {
        const int64_t ci = E.contact_base + c;
        const float nan = __builtin_nanf("");
        const float rec[13] = {0.f, P.d_max, 0.f, 0.f, prest.x, prest.y, prest.z, 0.f, 0.f, 0.f, nan,
                               float(E.kind), __int_as_float(E.group)};
#pragma unroll
        for (int r = 0; r < 13; ++r) dbg[r * C + ci] = rec[r];
      }
    }
    fc = wsum(fc); fp.x = wsum(fp.x); fp.y = wsum(fp.y); fp.z = wsum(fp.z);
    if (l == 0) {
      nsurv[e] = ns;
      ntiles[e] = (ns + kWave - 1) / kWave;
      filt[e] = F4{fc, fp.x, fp.y, fp.z};
    }
  }
}

// ------------------------------------------------------------------ scan --
// Exclusive scan of per-entry tile counts into tile offsets (three passes:
// per-block sums, a single-block scan of the sums, per-block application).
constexpr int kScanItems = 4;
constexpr int kScanBlock = 256 * kScanItems;

CM_DEV int64_t block_excl_scan(int64_t v, int64_t* sm /*[4]*/, int64_t* total) {
  // inclusive wave scan
  int64_t x = v;
  const int l = lane();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t y = __shfl_up(x, o, kWave);
    if (l >= o) x += y;
  }
  const int w = int(threadIdx.x) >> 6;
  if (l == kWave - 1) sm[w] = x;
  __syncthreads();
  int64_t off = 0, tot = 0;
  for (int i = 0; i < int(blockDim.x) / kWave; ++i) {
    if (i < w) off += sm[i];
    tot += sm[i];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ __launch_bounds__(256) void k_scan_blocks(const int32_t* __restrict__ in, int64_t n,
                                                     int64_t* __restrict__ bsum) {
  __shared__ int64_t sm[4];
  const int64_t base = int64_t(blockIdx.x) * kScanBlock + int64_t(threadIdx.x) * kScanItems;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) s += (base + i < n) ? in[base + i] : 0;
  int64_t tot;
  block_excl_scan(s, sm, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_top(int64_t* __restrict__ bsum, int64_t nb, int64_t* __restrict__ out,
                                                  int64_t n) {
  __shared__ int64_t sm[4];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += blockDim.x) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < nb ? bsum[i] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan(v, sm, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) out[n] = carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t* __restrict__ in, int64_t n,
                                                    const int64_t* __restrict__ boff, int64_t* __restrict__ out) {
  __shared__ int64_t sm[4];
  const int64_t base = int64_t(blockIdx.x) * kScanBlock + int64_t(threadIdx.x) * kScanItems;
  int64_t v[kScanItems], s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) { v[i] = (base + i < n) ? in[base + i] : 0; s += v[i]; }
  int64_t tot;
  int64_t off = block_excl_scan(s, sm, &tot) + boff[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = off;
    off += v[i];
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------ narrow phase --
// Contact of one survivor, in the world frame (Sec. IV-B, IV-C.1).
struct Contact {
  float d, f, phi;
  V3<float> pc, nc, fp;
};

CM_DEV Contact mollify(float phi, V3<float> Nw, V3<float> p, V3<float> prest, const DevParams& P) {
  Contact c;
  const float f = transitionT(phi, P);
  c.f = f;
  c.phi = phi;
  c.d = f * phi + (1.f - f) * P.d_max;
  c.nc = Nw * f;
  c.pc = p * f + prest * (1.f - f);
  c.fp = p * f;
  return c;
}

// Vertex-SDF contact (Sec. IV-B): the vertex is the contact point.
CM_DEV Contact vertex_contact(const ObjDesc& M, const ObjDesc& S, const Frame& F, int vi, const DevParams& P) {
  const V3<float> v = vert(M, vi);
  V3<float> x = mulM(F.Rrel, v) + F.trel;
  SdfRes<float> r;
  sdf_eval<1, 1, float>(S, P, &x, &r);
  const float inv = rsqrtf(dot(r.g, r.g) + P.eps_n2);
  const V3<float> Nw = mulM(F.RS, r.g * inv);
  const V3<float> p = mulM(F.RM, v) + F.tM;
  return mollify(r.phi, Nw, p, p, P);
}

// Edge-SDF contact (Sec. IV-B.2, Fig. e_s): sphere-trace both corners towards
// each other with the gated step sigma(phi / tau_s) phi for K steps (the two
// ends share each pass over the planes), softclip the arc lengths to [0, L]
// and take the midpoint of the two points as the contact.
CM_DEV Contact edge_contact(const ObjDesc& M, const ObjDesc& S, const Frame& F, int ei, const DevParams& P) {
  const I2 ed = M.edges[ei];
  const V3<float> v0 = vert(M, ed.x), v1 = vert(M, ed.y);
  const V3<float> x0 = mulM(F.Rrel, v0) + F.trel, x1 = mulM(F.Rrel, v1) + F.trel;
  const V3<float> dv = x1 - x0;
  const float L = sqrtf(dot(dv, dv));
  const V3<float> e = dv * (1.f / L);
  float al = 0.f, be = 0.f;
  for (int k = 0; k < P.st_iters; ++k) {
    V3<float> xs[2] = {x0 + e * al, x1 - e * be};
    SdfRes<float> r[2];
    sdf_eval<2, 0, float>(S, P, xs, r);
    al += sigmoidT(r[0].phi * P.inv_tau_st) * r[0].phi;
    be += sigmoidT(r[1].phi * P.inv_tau_st) * r[1].phi;
  }
  const float ac = softclip0T(al, L, P.tau_clip, P.inv_tau_clip);
  const float bc = softclip0T(be, L, P.tau_clip, P.inv_tau_clip);
  V3<float> pe = (x0 + e * ac + x1 - e * bc) * 0.5f;
  SdfRes<float> r;
  sdf_eval<1, 1, float>(S, P, &pe, &r);
  const float inv = rsqrtf(dot(r.g, r.g) + P.eps_n2);
  const V3<float> Nw = mulM(F.RS, r.g * inv);
  const V3<float> p = mulM(F.RS, pe) + F.tS;
  const V3<float> prest = mulM(F.RM, (v0 + v1) * 0.5f) + F.tM;
  return mollify(r.phi, Nw, p, prest, P);
}

// Finds the piece-local contact index of this lane's survivor in a tile, or
// -1 past the last survivor.
CM_DEV int tile_contact(const uint64_t* __restrict__ bits, const Entry& E, int j) {
  const int r0 = j * kWave, r = r0 + lane();
  const int nw = (E.count + kWave - 1) / kWave;
  const uint64_t* wp = bits + E.word_off;
  int pre = 0, c = -1;
  for (int w = 0; w < nw && pre < r0 + kWave; ++w) {
    const uint64_t word = wp[w];
    const int pc = __popcll(word);
    if (pre + pc > r0 && r >= pre && r < pre + pc) c = w * kWave + kth_bit(word, r - pre);
    pre += pc;
  }
  return c;
}

// Decodes tile t: entry index (largest e with tile_off[e] <= t) and tile j.
CM_DEV int64_t find_entry(const int64_t* __restrict__ tile_off, int64_t n_ent, int64_t t) {
  int64_t lo = 0, hi = n_ent;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (tile_off[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// Persistent narrow phase: waves pop survivor tiles from a queue; each tile
// writes the online-softmax state of its contacts (max logit, sum of weights
// and weighted sums of d, n_c, p_c, f p, f) to its own slot.
__global__ __launch_bounds__(256) void k_narrow_fwd(const Entry* __restrict__ ents, int64_t n_ent,
                                                    const int64_t* __restrict__ tile_off,
                                                    const uint64_t* __restrict__ bits,
                                                    const QueryDev* __restrict__ Q, const ObjDesc* __restrict__ objs,
                                                    DevParams P, uint32_t* __restrict__ counter,
                                                    float* __restrict__ partials, float* __restrict__ dbg,
                                                    int64_t C) {
  const int l = lane();
  const int64_t total = tile_off[n_ent];
  for (;;) {
    uint32_t t0 = 0;
    if (l == 0) t0 = atomicAdd(counter, 1u);
    const int64_t t = int64_t(uint32_t(uni(int(t0))));
    if (t >= total) break;
    const int64_t e = find_entry(tile_off, n_ent, t);
    const int j = int(t - tile_off[e]);
    const Entry E = ldc(ents + e);
    const QueryDev q = ldc(Q + E.query);
    const ObjDesc M = ldc(objs + E.mesh_obj);
    const ObjDesc S = ldc(objs + E.sdf_obj);
    const PieceDesc pd = ldc(M.pieces + E.piece);
    const Frame F = make_frame(q, E.dir);
    int c = tile_contact(bits, E, j);
    const bool valid = c >= 0;
    const int c0 = uni(c);  // lane 0 always holds a survivor
    if (!valid) c = c0;
    Contact ct = E.kind == 0 ? vertex_contact(M, S, F, pd.vert_begin + c, P)
                             : edge_contact(M, S, F, pd.edge_begin + c, P);
    // online softmax over the tile's logits l_i = -d_c,i / tau_b
    const float li = valid ? -ct.d * P.inv_tau_blend : -__builtin_inff();
    const float Lam = wmax(li);
    const float w = valid ? expf(li - Lam) : 0.f;
    float acc[13] = {w, w * ct.d, w * ct.nc.x, w * ct.nc.y, w * ct.nc.z, w * ct.pc.x, w * ct.pc.y, w * ct.pc.z,
                     w * ct.fp.x, w * ct.fp.y, w * ct.fp.z, w * ct.f, valid ? 1.f : 0.f};
#pragma unroll
    for (int i = 0; i < 13; ++i) acc[i] = wsum(acc[i]);
    if (l == 0) {
      float* o = partials + t * kPartial;
      o[0] = Lam;
#pragma unroll
      for (int i = 0; i < 13; ++i) o[1 + i] = acc[i];
      o[14] = 0.f;
      o[15] = 0.f;
    }
    if (dbg != nullptr && valid) {
      const int64_t ci = E.contact_base + c;
      const float rec[13] = {1.f, ct.d, ct.f, 0.f, ct.pc.x, ct.pc.y, ct.pc.z, ct.nc.x, ct.nc.y, ct.nc.z, ct.phi,
                             float(E.kind), __int_as_float(E.group)};
#pragma unroll
      for (int r = 0; r < 13; ++r) dbg[r * C + ci] = rec[r];
    }
  }
}

// ---------------------------------------------------------------- finalize --
struct Blend {
  float L, Z, d, n[3], p[3], q[3], f;
};
CM_DEV void blend_merge(Blend& a, float L, float Z, float d, const float* n, const float* p, const float* q, float f) {
  if (!(Z > 0.f)) return;
  const float Ln = fmaxf(a.L, L);
  const float sa = a.Z > 0.f ? expf(a.L - Ln) : 0.f;
  const float sb = expf(L - Ln);
  a.L = Ln;
  a.Z = a.Z * sa + Z * sb;
  a.d = a.d * sa + d * sb;
  for (int i = 0; i < 3; ++i) {
    a.n[i] = a.n[i] * sa + n[i] * sb;
    a.p[i] = a.p[i] * sa + p[i] * sb;
    a.q[i] = a.q[i] * sa + q[i] * sb;
  }
  a.f = a.f * sa + f * sb;
}

// Merges, in a fixed order, a group's filtered-contact closed forms and its
// tile partials: vertices (filtered, then tiles) then edges (filtered, then
// tiles); writes p, n (renormalised), d, q, W, logZ (Sec. IV-D.2-3).
CM_DEV Blend group_blend(int64_t g, const I2* __restrict__ gent, const int64_t* __restrict__ tile_off,
                         const F4* __restrict__ filt, const float* __restrict__ partials, const DevParams& P) {
  Blend b;
  b.L = -__builtin_inff(); b.Z = 0.f; b.d = 0.f; b.f = 0.f;
  for (int i = 0; i < 3; ++i) { b.n[i] = 0.f; b.p[i] = 0.f; b.q[i] = 0.f; }
  const I2 ge = gent[g];
  const float zero3[3] = {0.f, 0.f, 0.f};
  for (int k = 0; k < 2; ++k) {
    const int e = k == 0 ? ge.x : ge.y;
    const F4 fl = filt[e];
    const float fps[3] = {fl.y, fl.z, fl.w};
    blend_merge(b, -P.d_max * P.inv_tau_blend, fl.x, fl.x * P.d_max, zero3, fps, zero3, 0.f);
    for (int64_t t = tile_off[e]; t < tile_off[e + 1]; ++t) {
      const float* o = partials + t * kPartial;
      blend_merge(b, o[0], o[1], o[2], o + 3, o + 6, o + 9, o[12]);
    }
  }
  return b;
}

__global__ __launch_bounds__(256) void k_finalize_fwd(int64_t G, const I2* __restrict__ gent,
                                                      const int64_t* __restrict__ tile_off,
                                                      const F4* __restrict__ filt, const float* __restrict__ partials,
                                                      DevParams P, OutPtrs out) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const Blend b = group_blend(g, gent, tile_off, filt, partials, P);
  const float iz = 1.f / b.Z;
  const float m[3] = {b.n[0] * iz, b.n[1] * iz, b.n[2] * iz};
  const float inv = rsqrtf(m[0] * m[0] + m[1] * m[1] + m[2] * m[2] + P.eps_n2);
  for (int i = 0; i < 3; ++i) {
    out.p[i * G + g] = b.p[i] * iz;
    out.n[i * G + g] = m[i] * inv;
    out.q[i * G + g] = b.q[i] * iz;
  }
  out.d[g] = b.d * iz;
  out.W[g] = b.f * iz;
  out.logZ[g] = b.L + logf(b.Z);
}

// Per-contact blending weight w_i = exp(l_i - logZ_g) for the debug output.
__global__ void k_dbg_weights(float* __restrict__ dbg, int64_t C, const float* __restrict__ logZ, DevParams P) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int g = __float_as_int(dbg[12 * C + c]);
  dbg[3 * C + c] = expf(-dbg[C + c] * P.inv_tau_blend - logZ[g]);
}

// ------------------------------------------------------------- launchers --
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

hipError_t launch_grid_build(const ObjDesc* objs, const int32_t* ids, int32_t n_ids, int32_t grid_res,
                             const DevParams& P, hipStream_t s) {
  const int n3 = grid_res * grid_res * grid_res;
  const int per = int(cdiv(n3, 256));
  hipLaunchKernelGGL(k_grid_build, dim3(unsigned(per * n_ids)), dim3(256), 0, s, objs, ids, per, P);
  return hipGetLastError();
}

hipError_t launch_forward(const FwdArgs& a, hipStream_t s) {
  const int64_t nb_broad = std::min<int64_t>(cdiv(a.n_ent, 4), int64_t(a.n_cu) * 16);
  hipLaunchKernelGGL(k_broad, dim3(unsigned(std::max<int64_t>(nb_broad, 1))), dim3(256), 0, s, a.ents, a.n_ent, a.Q,
                     a.objs, a.P, a.bits, a.nsurv, a.ntiles, a.filt, a.dbg, a.C);
  const int64_t nb = cdiv(a.n_ent, kScanBlock);
  hipLaunchKernelGGL(k_scan_blocks, dim3(unsigned(nb)), dim3(256), 0, s, a.ntiles, a.n_ent, a.bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, a.bsum, nb, a.tile_off, a.n_ent);
  hipLaunchKernelGGL(k_scan_apply, dim3(unsigned(nb)), dim3(256), 0, s, a.ntiles, a.n_ent, a.bsum, a.tile_off);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, a.counter, 0u, int64_t(1));
  hipLaunchKernelGGL(k_narrow_fwd, dim3(unsigned(a.n_cu * a.blocks_per_cu)), dim3(256), 0, s, a.ents, a.n_ent,
                     a.tile_off, a.bits, a.Q, a.objs, a.P, a.counter, a.partials, a.dbg, a.C);
  hipLaunchKernelGGL(k_finalize_fwd, dim3(unsigned(cdiv(a.G, 256))), dim3(256), 0, s, a.G, a.gent, a.tile_off,
                     a.filt, a.partials, a.P, a.out);
  if (a.dbg != nullptr)
    hipLaunchKernelGGL(k_dbg_weights, dim3(unsigned(cdiv(a.C, 256))), dim3(256), 0, s, a.dbg, a.C, a.out.logZ, a.P);
  return hipGetLastError();
}

}  // namespace cm
