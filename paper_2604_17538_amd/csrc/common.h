// Structures shared by the host runtime and the gfx950 kernels.
#pragma once
#include <cstdint>

namespace cm {

struct alignas(16) F4 { float x, y, z, w; };
struct alignas(8) I2 { int32_t x, y; };

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kPartial = 16;       // floats per tile partial (forward blend state)
constexpr int kMaxPieces = 4096;   // pieces per object (index fits 16 bits)
constexpr int kSub = 16;           // support planes per piece (lower bound of its SDF)
constexpr int kGrp = 16;           // planes per plane group (a cone of normals bounds their values)
static_assert(kGrp % 8 == 0, "plane groups are whole pairs of blocks of 4");
constexpr float kPruneTau = 20.f;  // a piece this many tau_cup above the union's minimum has weight < 2^-28

// SDF representations of an object (Sec. III): the smooth union of smooth
// intersections of half-spaces (one convex piece each), a cubic spline fitted
// to the ground-truth SDF with a separately fitted normal spline, or primitives
// (PSQ / XPSQ, Sec. III-A) folded by smooth union, subtraction and intersection.
constexpr int32_t kRepPlanes = 0;
constexpr int32_t kRepSpline = 1;
constexpr int32_t kRepPrims = 2;

// One primitive of the primitive representation (Sec. III-A), FP32; the
// derived XPSQ constants formed in FP64 and rounded once.
struct PrimDev {
  int32_t kind;         // 0 PSQ at a fixed pose, 1 XPSQ (PSQ swept along a quadratic spline)
  int32_t op;           // joins the primitives before it by 0 union, 1 subtraction, 2 intersection
  int32_t plane_begin;  // its half-spaces in the object's primitive planes
  int32_t plane_count;
  float c[3], pad0;     // PSQ centre; XPSQ p1
  float p2[3], pad1;    // XPSQ p2, p3
  float p3[3], pad2;
  float Rt[9], pad3[3]; // PSQ: R^T row-major (object frame -> PSQ frame)
  float a0[3], e0a;     // SQ scales and eps1 at t = 0 (PSQ: the SQ)
  float a1[3], e1a;     // the same at t = 1
  float e0b, e1b;       // eps2 at t = 0, t = 1
  float a2, inv2AA;     // XPSQ cubic: a2 = 3 A.B / (2 |A|^2); 1 / (2 |A|^2)
  float A[3], BB;       // A = p1 - 2 p2 + p3; |B|^2
  float B[3], pad4;     // B = 2 (p2 - p1)
  float bn[3], pad5;    // unit binormal along B x A
};
static_assert(sizeof(PrimDev) == 208, "PrimDev layout");

// Per piece of a resident object (device).  Planes of the piece are stored
// relative to `centre` and pre-scaled by kappa = log2(e) / tau_cap, so the
// piece's log-sum-exp runs in base 2 with the temperature folded in.
struct PieceDesc {
  float cx, cy, cz;       // centre (mean of the piece's vertices), object frame
  int32_t plane_begin;    // object-level plane index (a multiple of kGrp)
  int32_t plane_count;    // planes of the piece; the array holds them padded to whole groups
  int32_t vert_begin;     // object-level vertex index
  int32_t vert_count;
  int32_t edge_begin;     // object-level edge index
  int32_t edge_count;
  float ub_off;           // tau_cap ln(plane_count) - (distance from the centre to the nearest plane)
  int32_t grp_begin;      // object-level index of the piece's first plane group
  int32_t pad;
};
static_assert(sizeof(PieceDesc) == 48, "PieceDesc layout");

// A resident object (device).  All arrays are SoA in one allocation.
struct ObjDesc {
  const F4* planes;       // [P] (kappa n, kappa h_local), h_local relative to the piece centre;
                          // each piece padded to whole groups of kGrp with (0, 0, 0, -1e30)
  const PieceDesc* pieces;
  const float* vx;        // [V] object frame
  const float* vy;
  const float* vz;
  const I2* edges;        // [E] object-level vertex indices
  const float* grid;      // [n^3] phi at voxel centres
  int32_t n_pieces, n_planes, n_verts, n_edges;
  float gorg[3];          // grid origin
  float gh[3];            // voxel size
  float ginv[3];          // 1 / voxel size
  float gr;               // voxel circumradius
  int32_t gn;             // voxels per axis
  int32_t rep;            // SDF representation: kRepPlanes, kRepSpline or kRepPrims
  // kRepPlanes: [n_pieces][kSub] support planes (scaled like planes), min(kSub,
  // plane_count) used, then two float4 per plane group (groups of kGrp
  // consecutive planes of a piece, the last one of a piece possibly partial):
  // (axis, largest scaled offset), (cos, kappa cos, kappa sin of the cone's
  // half-angle).  kRepSpline: the spline coefficients, (gn + 3)^3 float4
  // (phi, n_x, n_y, n_z) over the grid's box (its cells are the grid's voxels).
  // kRepPrims: gn PrimDev records, then their half-spaces (float4 (n, h) in each
  // PSQ frame); such an object has no voxel grid
  const F4* sub;
};
static_assert(sizeof(ObjDesc) == 128, "ObjDesc layout");

// Query as laid out in cm_query (64 bytes).
struct QueryDev {
  uint32_t a, b;
  float qa[4], ta[3];
  float qb[4], tb[3];
};
static_assert(sizeof(QueryDev) == 64, "cm_query layout");

// One broad-phase entry: the vertices (kind 0) or edges (kind 1) of one piece
// of the mesh-side object of one direction of one query.
struct Entry {
  int32_t query;
  int32_t group;          // global group index of (query, dir, piece)
  int32_t piece;          // piece of the mesh-side object
  int32_t count;          // contacts in this entry
  int64_t word_off;       // first 64-bit survivor word
  int64_t contact_base;   // index of the first contact in the debug layout
  int32_t dir;            // 0: A's mesh vs B's SDF, 1: B's mesh vs A's SDF
  int32_t kind;           // 0 vertices, 1 edges
  int32_t mesh_obj;       // object whose vertices / edges are the contacts
  int32_t sdf_obj;        // object whose SDF they are evaluated against
};
static_assert(sizeof(Entry) == 48, "Entry layout");

// Method constants in the form the kernels use.
struct DevParams {
  float kcap;        // log2(e) / tau_cap
  float icap;        // 1 / kcap
  float kcup;        // log2(e) / tau_cup
  float icup;        // 1 / kcup
  float inv_tau_st;  // 1 / tau_st
  float tau_clip;
  float inv_tau_clip;
  float inv_tau_blend;
  float tau_blend;
  float d_max;
  float inv_eps_t;
  float eps_n2;      // eps_n^2
  int32_t st_iters;
  int32_t broad_phase;
  int32_t edge_bound;
  int32_t prune;       // skip pieces that cannot matter (see sdf_eval)
  float prune_margin;  // kPruneTau * tau_cup
  float tau_t, inv_tau_t;        // primitives: soft clip of the spline parameter to (0, 1)
  float tau_disc, inv_tau_disc;  // primitives: softplus / sigmoid of the cubic's discriminant
  int32_t pad;
};

}  // namespace cm
