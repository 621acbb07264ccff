// Host runtime of the contact-manifold library: context, device arena,
// resident-object registry, plans.  Internal; the public ABI is include/cm.h.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/cm.h"
#include "common.h"
#include "geom.h"
#include "kernels.h"

namespace cm {

DevParams make_dev_params(const cm_params& p);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over large device chunks; a chunk is returned to HIP once
// every allocation in it has been released.
class Arena {
 public:
  explicit Arena(size_t chunk) : chunk_(chunk) {}
  ~Arena();
  void* alloc(size_t bytes, int* chunk_id);
  void release(int chunk_id);
  size_t bytes_in_use() const { return in_use_; }

 private:
  struct Chunk { char* base = nullptr; size_t size = 0, used = 0; int live = 0; };
  std::vector<Chunk> chunks_;
  size_t chunk_;
  size_t in_use_ = 0;
};

struct ObjHost {
  bool alive = false;
  std::vector<PieceGeom> pieces;
  std::vector<double> centres;  // 3 per piece
  std::vector<int32_t> counts;  // per piece: vertices, edges incl. crossing edges (compact, for planning)
  // per piece: edges of other pieces that cross it, as (piece, edge) pairs
  // (edge assignment of Sec. IV-D.1; empty unless cm_params.edge_assign)
  std::vector<std::vector<int32_t>> xedges;
  int64_t n_planes = 0, n_verts = 0, n_edges = 0;
  int64_t n_words = 0;  // survivor bitmask words of its entries (per piece and kind: count / 64 rounded up)
  double radius = 0;
  void* dmem = nullptr;
  int chunk = -1;
  ObjDesc desc{};
  void* dprims = nullptr;  // primitive block (sdf_kind 2), its own allocation
  int32_t n_prims = 0;
};

struct Serving;
void serving_stop(cm_context* ctx);

}  // namespace cm

struct cm_context {
  int device = -1;
  cm_params prm{};
  cm::DevParams dp{};
  int n_cu = 0;
  size_t budget = 0;
  std::mutex mu;             // error string, serving start
  std::string err;
  // the object registry (objs, d_objs, d_objs_cap, old_tables): shared by
  // planners and launches, exclusive for registration and release; taken
  // before mu when both are held
  std::shared_mutex reg_mu;
  std::vector<cm::ObjHost> objs;
  cm::ObjDesc* d_objs = nullptr;  // device table
  size_t d_objs_cap = 0;
  std::vector<cm::ObjDesc*> old_tables;  // outgrown tables, freed at shutdown
  std::unique_ptr<cm::Arena> arena;
  hipStream_t build_stream = nullptr;
  cm::Serving* serving = nullptr;
};

namespace cm {
// Sizes a plan's device memory is laid out for: the batch's own, or the
// capacity of a reserved plan (cm_plan_reserve), whose batch can be replaced.
struct PlanSizes {
  int32_t n = 0;
  int64_t G = 0, C = 0, E = 0, W = 0, nb = 0, R = 0;
};
}  // namespace cm

struct cm_plan {
  cm_context* ctx = nullptr;
  int32_t n = 0;
  int64_t G = 0, C = 0, E = 0, W = 0, nb = 0, R = 0;
  bool reserved = false;             // laid out for `cap`; cm_plan_refill replaces the batch
  cm::PlanSizes cap;
  cm::DevCounts h_dc{};              // the batch's counts and object table, uploaded with the tables
  cm::DevCounts* d_dc = nullptr;
  hipEvent_t uploaded = nullptr;     // reserved plans: the last refill's uploads are done
  std::vector<int64_t> group_off, contact_off;
  std::vector<cm::Entry> ents;       // host copy (device order: runs in cost order)
  std::vector<int64_t> run_off;      // [R + 1] entry ranges of the runs (query, direction, kind)
  std::vector<int32_t> ent_run;      // [E] run of each entry
  std::vector<int32_t> q_runs;       // [4n] run of (query, 2 dir + kind)
  std::vector<cm::I2> gent;          // per group: (vertex entry, edge entry)
  bool owns_mem = false;
  std::vector<int32_t> qa, qb;
  void* dmem = nullptr;
  cm::Entry* d_ents = nullptr;
  cm::I2* d_gent = nullptr;
  uint64_t* d_bits = nullptr;
  int32_t* d_nsurv = nullptr;
  int32_t* d_wpre = nullptr;     // [W] survivors of an entry before each of its bitmask words
  int64_t* d_surv_off = nullptr; // [E + 1] survivor offsets (entries in run order)
  int64_t* d_run_off = nullptr;  // [R + 1]
  int32_t* d_ent_run = nullptr;  // [E]
  int32_t* d_q_runs = nullptr;   // [4n]
  int32_t* d_ntr = nullptr;      // [R] tiles per run
  int32_t* d_npart = nullptr;    // [E] partials per entry
  int64_t* d_part_off = nullptr; // [E + 1]
  cm::F4* d_filt = nullptr;
  int64_t* d_tile_off = nullptr; // [R + 1] tile offsets of the runs
  int64_t* d_bsum = nullptr;
  uint32_t* d_counter = nullptr;
  float* d_partials = nullptr;
  float* d_gscratch = nullptr;   // per-group forward results for the adjoint
  float* d_bpartials = nullptr;  // per-tile adjoint partials
  int64_t* d_group_off = nullptr;
  float* d_gradtmp = nullptr;    // [n][12] gradient when the caller passes none
  float* d_tape = nullptr;       // adjoint tape (see kernels.h)
  unsigned long long* d_work = nullptr;  // point-plane evaluations of the last pass
  int64_t tape_tiles = 0;
  // what the tape holds per row: 0 nothing (the plan never runs an adjoint),
  // 1 float values (float adjoints only), 2 dual values (any adjoint)
  int32_t tape_kind = 2;
  int32_t blocks_per_cu = 8;       // persistent workgroups per CU, float sweeps (cm_plan_autotune)
  int32_t blocks_per_cu_dual = 8;  // the same for the sweeps in dual numbers
  int32_t wg_waves = 4;            // waves per workgroup of the narrow sweeps, float
  int32_t wg_waves_dual = 4;       // the same in dual numbers
  bool timing = false;
  uint32_t timed_mask = 0;  // timing slots launched by the last pass
  hipEvent_t ev[2 * cm::kTimed] = {};
};

namespace cm {
cm_status fail(cm_context* ctx, cm_status st, const std::string& msg);
cm_status hip_fail(cm_context* ctx, hipError_t e, const char* where);
ObjHost* get_obj(cm_context* ctx, cm_object h);
cm_status plan_host(cm_context* ctx, const cm_query* hq, int32_t n, cm_plan* pl, size_t* dev_bytes);
cm_status plan_sizes(cm_context* ctx, const cm_query* hq, int32_t n, PlanSizes* z);
size_t plan_layout(cm_plan* pl, char* base);
PlanSizes layout_sizes(const cm_plan* pl);
cm_status plan_bind(cm_plan* pl, void* dmem, hipStream_t s);
FwdArgs fwd_args(cm_context* ctx, cm_plan* pl, const cm_query* q, const cm_groups& out, float* dbg);
hipError_t static_scratch_setup(int device);  // noalloc.hip
}  // namespace cm
