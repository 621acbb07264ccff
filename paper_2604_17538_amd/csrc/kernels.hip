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
#include "prims.h"
#include "wave.h"

namespace cm {

// Poses of one direction: mesh-side body (R_M, t_M), SDF-side body (R_S, t_S)
// and the mesh -> SDF-frame transform x = R_S^T (R_M v + t_M - t_S).
struct Frame {
  M3<float> RM, RS, Rrel;
  V3<float> tM, tS, trel;
};
CM_DEV Frame make_frame(const QueryDev& q, int dir) {
  const Frame32 f = dir ? frame32(q.qb, q.tb, q.qa, q.ta) : frame32(q.qa, q.ta, q.qb, q.tb);
  Frame F;
  for (int i = 0; i < 9; ++i) { F.RM.m[i] = f.RM[i]; F.RS.m[i] = f.RS[i]; F.Rrel.m[i] = f.Rrel[i]; }
  F.tM = {f.tM[0], f.tM[1], f.tM[2]};
  F.tS = {f.tS[0], f.tS[1], f.tS[2]};
  F.trel = {f.trel[0], f.trel[1], f.trel[2]};
  return F;
}


// --------------------------------------------------------------- grid build --
// phi of the object at every voxel centre (Sec. IV-C.2).
__global__ __launch_bounds__(256) void k_grid_build(const ObjDesc* __restrict__ objs, const int32_t* __restrict__ ids,
                                                    int32_t blocks_per_obj, DevParams P) {
  const int oi = uni(int(blockIdx.x) / blocks_per_obj);
  const int obj = uni(ids[oi]);
  const ObjDesc o = ldc(objs + obj);
  if (o.rep != kRepPlanes) return;  // a spline object's cell bounds come with its fit
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
__global__ __launch_bounds__(256) void k_broad(const DevCounts* __restrict__ dc, const Entry* __restrict__ ents,
                                               const QueryDev* __restrict__ Q, DevParams P,
                                               uint64_t* __restrict__ bits, int32_t* __restrict__ nsurv,
                                               int32_t* __restrict__ wpre, F4* __restrict__ filt,
                                               float* __restrict__ dbg, int64_t C) {
  const int l = lane();
  const int64_t n_ent = dc->E;
  const ObjDesc* __restrict__ objs = dc->objs;
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
        // (primitive SDFs carry no bound: every contact survives)
        surv = !P.broad_phase || S.rep == kRepPrims ||
               (S.rep == kRepSpline ? spline_lb(S, x) : grid_lb(S, x)) < P.d_max;
        prest = mulM(F.RM, v) + F.tM;
      } else {
        const I2 ed = M.edges[pd.edge_begin + cc];
        const V3<float> v0 = vert(M, ed.x), v1 = vert(M, ed.y);
        const V3<float> x0 = mulM(F.Rrel, v0) + F.trel, x1 = mulM(F.Rrel, v1) + F.trel;
        if (S.rep == kRepPrims) {
          surv = true;
        } else if (P.broad_phase && S.rep == kRepSpline) {
          surv = spline_edge_lb(S, x0, x1) < P.d_max;
        } else if (P.broad_phase) {
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
      if (l == 0) {
        bits[E.word_off + base / kWave] = word;
        wpre[E.word_off + base / kWave] = ns;
      }
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
      filt[e] = F4{fc, fp.x, fp.y, fp.z};
    }
  }
}

// ------------------------------------------------------------------ scan --
// Exclusive scans of per-entry and per-run counts into offsets (three passes:
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

__global__ __launch_bounds__(256) void k_scan_blocks(const int32_t* __restrict__ in, const int64_t* __restrict__ np,
                                                     int64_t* __restrict__ bsum) {
  __shared__ int64_t sm[4];
  const int64_t n = *np;
  const int64_t base = int64_t(blockIdx.x) * kScanBlock + int64_t(threadIdx.x) * kScanItems;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) s += (base + i < n) ? in[base + i] : 0;
  int64_t tot;
  block_excl_scan(s, sm, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_top(int64_t* __restrict__ bsum, int64_t nb, int64_t* __restrict__ out,
                                                  const int64_t* __restrict__ np) {
  __shared__ int64_t sm[4];
  const int64_t n = *np;
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

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t* __restrict__ in, const int64_t* __restrict__ np,
                                                    const int64_t* __restrict__ boff, int64_t* __restrict__ out) {
  __shared__ int64_t sm[4];
  const int64_t n = *np;
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

// ------------------------------------------------------------- run tiles --
// A run is the entries of one (query, direction, kind): every piece of the
// mesh side.  Its survivors, in entry order, fill consecutive tiles of 64.
__global__ void k_run_tiles(const int64_t* __restrict__ run_off, const int64_t* __restrict__ surv_off,
                            const DevCounts* __restrict__ dc, int32_t* __restrict__ ntr) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= dc->R) return;
  const int64_t n = surv_off[run_off[r + 1]] - surv_off[run_off[r]];
  ntr[r] = int32_t((n + kWave - 1) / kWave);
}

// Blend partials of an entry: one per tile its survivors reach.
__global__ void k_entry_parts(const int64_t* __restrict__ run_off, const int32_t* __restrict__ ent_run,
                              const int64_t* __restrict__ surv_off, const DevCounts* __restrict__ dc,
                              int32_t* __restrict__ npart) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= dc->E) return;
  const int64_t rs = surv_off[run_off[ent_run[e]]];
  const int64_t a = surv_off[e] - rs, b = surv_off[e + 1] - rs;
  npart[e] = b > a ? int32_t((b - 1) / kWave - a / kWave + 1) : 0;
}

// ------------------------------------------------------ isosurface projection --
// Sec. IV-A, last paragraph: contact points found on the collision mesh are
// moved onto the SDF's zero level set, proj(p) = p - phi(p) n(p), in the frame of
// the SDF each group was evaluated against (A's groups: B's SDF; B's groups:
// A's).  One wave per (query, direction); its lanes take that direction's
// groups (every lane runs the SDF evaluation, whose piece loop is wave-uniform).
__global__ __launch_bounds__(256) void k_project(const QueryDev* __restrict__ Q, const ObjDesc* __restrict__ objs,
                                                 const int64_t* __restrict__ group_off, int32_t n, DevParams P,
                                                 const float* __restrict__ pin, float* __restrict__ pout, int64_t G) {
  const int l = lane();
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (wave >= 2 * int64_t(n)) return;
  const int qi = int(wave >> 1), dir = int(wave & 1);
  const QueryDev q = ldc(Q + qi);
  const ObjDesc A = ldc(objs + q.a);
  const ObjDesc S = ldc(objs + (dir ? q.a : q.b));
  const int64_t gq = group_off[qi], gn = group_off[qi + 1] - gq;
  const int64_t g0 = gq + (dir ? A.n_pieces : 0);
  const int64_t ng = dir ? gn - A.n_pieces : int64_t(A.n_pieces);
  const Frame32 f = dir ? frame32(q.qb, q.tb, q.qa, q.ta) : frame32(q.qa, q.ta, q.qb, q.tb);
  for (int64_t base = 0; base < ng; base += kWave) {
    const bool valid = base + l < ng;
    const int64_t g = g0 + (valid ? base + l : 0);
    const V3<float> d{pin[g] - f.tS[0], pin[G + g] - f.tS[1], pin[2 * G + g] - f.tS[2]};
    const V3<float> x{f.RS[0] * d.x + f.RS[3] * d.y + f.RS[6] * d.z, f.RS[1] * d.x + f.RS[4] * d.y + f.RS[7] * d.z,
                      f.RS[2] * d.x + f.RS[5] * d.y + f.RS[8] * d.z};
    float phi;
    V3<float> nS;
    if (S.rep == kRepSpline) {
      SplRes<float> r;
      spline_eval<false, true, false, float>(S, x, r);
      phi = r.phi;
      nS = r.n;
    } else if (S.rep == kRepPrims) {
      const Jt<float, 1> j = prims_eval<float, 1>(S, x, P);
      phi = j.v;
      const V3<float> g{j.g[0], j.g[1], j.g[2]};
      nS = g * (1.f / sqrtf(dot(g, g) + P.eps_n2));
    } else {
      SdfRes<float> r;
      sdf_eval<1, 1, float>(S, P, &x, &r);
      phi = r.phi;
      nS = r.g * (1.f / sqrtf(dot(r.g, r.g) + P.eps_n2));
    }
    const V3<float> y = x - nS * phi;
    if (valid) {
      pout[g] = f.RS[0] * y.x + f.RS[1] * y.y + f.RS[2] * y.z + f.tS[0];
      pout[G + g] = f.RS[3] * y.x + f.RS[4] * y.y + f.RS[5] * y.z + f.tS[1];
      pout[2 * G + g] = f.RS[6] * y.x + f.RS[7] * y.y + f.RS[8] * y.z + f.tS[2];
    }
  }
}

hipError_t launch_project(const QueryDev* Q, const ObjDesc* objs, const int64_t* group_off, int32_t n,
                          const DevParams& P, const float* pin, float* pout, int64_t G, hipStream_t s) {
  (void)hipGetLastError();
  const int64_t threads = 2 * int64_t(n) * kWave;
  hipLaunchKernelGGL(k_project, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, Q, objs, group_off, n, P, pin,
                     pout, G);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
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

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(unsigned(std::max<int64_t>(cdiv(n, 256), 1))), dim3(256), 0, s, p, v, n);
}

// device address of count i of a DevCounts (0: E, 1: R, 2: G, 3: n)
static const int64_t* dc_count(const DevCounts* dc, int i) { return reinterpret_cast<const int64_t*>(dc) + i; }

// out[0..n) = exclusive scan of in, out[n] = total; n read on the device
// (*np), the grid sized for the capacity n_cap >= n.
static void launch_scan(const int32_t* in, int64_t n_cap, const int64_t* np, int64_t* out, int64_t* bsum,
                        hipStream_t s) {
  const int64_t nb = std::max<int64_t>(cdiv(n_cap, kScanBlock), 1);
  hipLaunchKernelGGL(k_scan_blocks, dim3(unsigned(nb)), dim3(256), 0, s, in, np, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, bsum, nb, out, np);
  hipLaunchKernelGGL(k_scan_apply, dim3(unsigned(nb)), dim3(256), 0, s, in, np, bsum, out);
}

void launch_front(const FwdArgs& a, hipStream_t s) {
  const int64_t nb_broad = std::min<int64_t>(cdiv(a.n_ent, 4), int64_t(a.n_cu) * 16);
  if (a.ev) (void)hipEventRecord(a.ev[2 * kTBroad], s);
  hipLaunchKernelGGL(k_broad, dim3(unsigned(std::max<int64_t>(nb_broad, 1))), dim3(256), 0, s, a.dc, a.ents, a.Q,
                     a.P, a.bits, a.nsurv, a.wpre, a.filt, a.dbg, a.C);
  if (a.ev) (void)hipEventRecord(a.ev[2 * kTBroad + 1], s);
  launch_scan(a.nsurv, a.n_ent, dc_count(a.dc, 0), a.surv_off, a.bsum, s);
  hipLaunchKernelGGL(k_run_tiles, dim3(unsigned(std::max<int64_t>(cdiv(a.n_run, 256), 1))), dim3(256), 0, s, a.run_off,
                     a.surv_off, a.dc, a.ntr);
  launch_scan(a.ntr, a.n_run, dc_count(a.dc, 1), a.tile_off, a.bsum, s);
  hipLaunchKernelGGL(k_entry_parts, dim3(unsigned(std::max<int64_t>(cdiv(a.n_ent, 256), 1))), dim3(256), 0, s,
                     a.run_off, a.ent_run, a.surv_off, a.dc, a.npart);
  launch_scan(a.npart, a.n_ent, dc_count(a.dc, 0), a.part_off, a.bsum, s);
}

}  // namespace cm
