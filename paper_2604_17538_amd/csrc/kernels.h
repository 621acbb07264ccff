// Launch interface between the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "common.h"

namespace cm {

// Device pointers of the SoA group records (see cm_groups).
struct OutPtrs {
  float *p, *n, *d, *q, *W, *logZ;
};

constexpr int kStride = 32;   // floats per tile partial
constexpr int kQueues = 8;    // narrow-phase work queues: one per XCD of the MI355X
constexpr int kChunk = 16;    // consecutive tiles dealt to one queue at a time
constexpr int kGStride = 64;  // floats per per-group adjoint record (24 values, dual: 48)
constexpr int kMaxTraceAdj = 4;  // sphere-trace steps supported by the adjoint

// Tape: what the sweep before an adjoint keeps of each contact so that the
// adjoint needs no pass over the planes.  SoA [value][slot], slot = tile * 64
// + lane; with duals the tangent plane of value v follows its value plane
// (rows 2v, 2v + 1).  Values: phi, grad phi (3) and the Hessian (6) at the
// contact point, then per sphere-trace step phi and grad phi at both iterates.
constexpr int kTapeFixed = 10;
constexpr int kTapeStep = 8;
inline int tape_values(int st_iters) { return kTapeFixed + kTapeStep * st_iters; }

// The batch a plan holds, read by every kernel of a pass from device memory:
// the counts bound the loops, the object table is the one the entries index.
// A pass captured into a graph therefore replays whatever batch the plan holds
// when it is launched (up to the plan's capacity); the counts passed by value
// beside it are capacities (grid sizes, and the row stride of the SoA records).
struct DevCounts {
  int64_t E, R, G, n;     // entries, runs, groups, pair-queries
  const ObjDesc* objs;
  int64_t pad[3];
};
static_assert(sizeof(DevCounts) == 64, "DevCounts layout");

struct FwdArgs {
  const DevCounts* dc;
  const Entry* ents;
  int64_t n_ent;
  const QueryDev* Q;
  const ObjDesc* objs;
  DevParams P;
  uint64_t* bits;
  int32_t* nsurv;
  int32_t* wpre;        // [W] survivors of an entry before each of its bitmask words
  int64_t* surv_off;    // [E + 1]
  const int64_t* run_off;   // [R + 1] entry ranges of the runs
  const int32_t* ent_run;   // [E]
  const int32_t* q_runs;    // [4n] run of (query, 2 dir + kind)
  int32_t* ntr;         // [R] tiles per run
  int32_t* npart;       // [E] blend partials per entry
  int64_t* part_off;    // [E + 1]
  int64_t n_run;
  F4* filt;
  int64_t* bsum;
  int64_t* tile_off;    // [R + 1] tile offsets of the runs
  uint32_t* counter;    // [kQueues] work-queue counters
  float* partials;
  const I2* gent;       // per group: (vertex entry, edge entry)
  int64_t G;
  OutPtrs out;
  OutPtrs out_t;        // tangents of the records along dir (Jacobian-vector product)
  float* dbg;           // nullable
  int64_t C;
  int32_t n_cu;
  int32_t blocks_per_cu;       // persistent workgroups per CU, float sweeps
  int32_t blocks_per_cu_dual;  // the same in dual numbers
  int32_t wg_waves;            // waves per workgroup of the narrow sweeps (1, 2 or 4), float
  int32_t wg_waves_dual;       // the same in dual numbers
  // adjoint / HVP
  OutPtrs cot;          // cotangent group records
  float* gscratch;      // [G][kGStride] per-piece adjoint seeds
  float* bpartials;     // [tiles][kStride] per-tile pose gradients
  const float* dir;     // [n][12] HVP direction (nullable)
  const int64_t* group_off;  // [n + 1]
  int32_t n;
  float* grad;          // [n][12]
  float* hv;            // [n][12] (nullable)
  hipEvent_t* ev;       // nullable: start/stop events per timed kernel (kTimed pairs)
  unsigned long long* work;  // nullable: see NarrowArgs
  float* tape;          // [2 * tape_nv][tape_tiles * 64] (nullable)
  int64_t tape_tiles;   // tiles [0, tape_tiles) are taped; the rest is recomputed
  int32_t tape_nv;
  int32_t rep;          // SDF representation of every SDF-side object (kRepPlanes / kRepSpline);
                        // spline SDFs keep no tape (tape == nullptr)
};

// Kernels timed with events when a plan has timing enabled.
enum { kTBroad = 0, kTNarrowFwd = 1, kTNarrowTan = 2, kTNarrowAdj = 3, kTNarrowDualAdj = 4, kTimed = 5 };

struct NarrowArgs {
  const DevCounts* dc;
  const Entry* ents;
  int64_t n_ent;
  const int64_t* tile_off;   // [R + 1]
  const int64_t* run_off;    // [R + 1]
  const int64_t* surv_off;   // [E + 1]
  const int64_t* part_off;   // [E + 1]
  const int32_t* wpre;       // [W]
  int64_t n_run;
  const uint64_t* bits;
  const QueryDev* Q;
  const ObjDesc* objs;
  DevParams P;
  uint32_t* counter;    // [kQueues] work-queue counters
  float* partials;        // output partials
  const float* gscratch;  // per-piece adjoint seeds (adjoint pass)
  const float* dir;       // HVP direction (dual passes)
  float* dbg;
  int64_t C;
  float* tape;            // see FwdArgs
  int64_t tape_tiles;
  int32_t tape_nv;
  int64_t t_begin;        // first tile of this launch (recomputing adjoint)
  unsigned long long* work;  // nullable: [2] += point-plane evaluations performed for vertex and
                             // edge contacts (64 lanes per wave); spline SDFs: 64 terms per evaluation
  int32_t rep;               // see FwdArgs
};

struct FinArgs {
  const DevCounts* dc;
  int64_t G;            // capacity: the row stride of the SoA records
  const I2* gent;
  const int64_t* tile_off;   // [R + 1] tiles of the runs
  const int64_t* part_off;   // [E + 1] blend partials of the entries
  const int32_t* q_runs;     // [4n]
  const F4* filt;
  const float* partials;
  const Entry* ents;
  const QueryDev* Q;
  DevParams P;
  OutPtrs out;
  OutPtrs out_t;
  OutPtrs cot;
  float* gscratch;
  const float* dir;
};

hipError_t launch_grid_build(const ObjDesc* objs, const int32_t* ids, int32_t n_ids, int32_t grid_res,
                             const DevParams& P, hipStream_t s);

// One object's spline fit (spline.hip): its collision geometry in FP64 and
// where the results go.
struct SplJob {
  const double* planes;   // [P][4] unit outward n, h (n.x + h <= 0 inside), object frame
  const int4* pieces;     // per piece: plane begin, plane count, segment begin, segment count
  const double* segs;     // [E][6] feature edges as segments (both endpoints)
  int32_t n_pieces;
  int32_t pad;
  double org[3], h[3];    // grid box: corners org + (i, j, k) h, i, j, k in [0, n]
  F4* coef;               // out: [(n + 3)^3] (phi, n_x, n_y, n_z) coefficients
  float* grid;            // out: [n^3] per cell lower bound of the spline
};
// GT at the corners, three solve passes, pack; work_a and work_b hold
// n_jobs * work_stride doubles each, work_stride >= 4 (n + 3)^3.
hipError_t launch_spline_build(const SplJob* d_jobs, int n_jobs, int n, double* work_a, double* work_b,
                               int64_t work_stride, hipStream_t s);
// isosurface projection of group points (p_in, p_out: SoA [3][G], world)
hipError_t launch_project(const QueryDev* Q, const ObjDesc* objs, const int64_t* group_off, int32_t n,
                          const DevParams& P, const float* pin, float* pout, int64_t G, hipStream_t s);
// broad phase + tile scan (shared by every pass)
void launch_front(const FwdArgs& a, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_forward(const FwdArgs& a, hipStream_t s);
// records: also write the group records a.out (from the same sweep)
hipError_t launch_backward(const FwdArgs& a, hipStream_t s, bool records = false);
hipError_t launch_hvp(const FwdArgs& a, hipStream_t s, bool records = false);
// records and their tangents along dir (one forward sweep in dual numbers)
hipError_t launch_jvp(const FwdArgs& a, hipStream_t s);
// Fills the resident-workgroup cache of every narrow-phase kernel (called once
// per context before any launch, so no occupancy query runs inside a graph
// capture).
void warm_narrow_occupancy();

}  // namespace cm
