/* cm.h -- C ABI of the MI355X (gfx950) contact-manifold library.
 *
 * Implements the data-parallel hot path of Beker, Geist, Paulus, Martius,
 * "Novel Algorithms for Smoothly Differentiable and Efficiently Vectorizable
 * Contact Manifold Construction":
 *   - each object is a union of convex pieces; a piece's SDF is the smooth
 *     intersection (log-sum-exp) of its hull facet half-spaces (Sec. III-A.2,
 *     eq. smooth-intersection; Sec. III-A.3) and the object's SDF is the smooth
 *     union of its pieces (eq. soft_union);
 *   - the mesh of one object (hull vertices and feature edges of its pieces)
 *     collides with the SDF of the other, and then the roles are swapped
 *     (Sec. III, opening paragraph);
 *   - voxel-grid broad phase (Sec. IV-C.2), vertex-SDF and edge-SDF narrow
 *     phase with sphere tracing (Sec. IV-B), C2 mollification (Sec. IV-C.1) and
 *     softmax blending per convex piece (Sec. IV-D).
 * Gradients w.r.t. both 6-DoF poses and Hessian-vector products are project
 * additions (the paper's goal is twice-differentiability, abstract).
 *
 * Conventions
 *   - Functions never throw across the ABI.  They return a cm_status; on error
 *     cm_last_error(ctx) holds a message (thread-local to the context).
 *   - Lengths are metres, quaternions are (w, x, y, z) and are normalised on
 *     input; a quaternion with norm < 1e-12 is CM_E_INVALID.
 *   - Outputs are in the world frame.  A pair-query (A, B) yields one group
 *     per piece of A (A's mesh against B's SDF) followed by one group per piece
 *     of B (B's mesh against A's SDF).
 *   - A group record is 12 floats: p (3), n (3), d, q (3), W, logZ, where p is
 *     the blended contact point, n the blended normal (renormalised), d the
 *     blended penetration value (negative = penetrating, saturating at d_max),
 *     q = sum_i w_i f_i p_i and W = sum_i w_i f_i the moments of the blended
 *     contact Jacobian J = [[q]x, W I] (Sec. IV-D.3 with J_c = f J), and logZ
 *     the log-partition of the blending softmax over -d_c / tau_blend.
 *   - The context owns all geometry and scratch memory.  Query, output,
 *     cotangent and gradient buffers belong to the caller.
 *   - Device entry points are asynchronous on the given stream (a hipStream_t
 *     passed as void*; NULL = the default stream).
 */
#ifndef CM_H
#define CM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cm_status;
enum {
  CM_OK = 0,
  CM_E_INVALID = -1,     /* bad argument, handle or size */
  CM_E_OOM = -2,         /* device or host allocation failed / over budget */
  CM_E_DEGENERATE = -3,  /* a piece has fewer than 4 non-coplanar points */
  CM_E_HIP = -4,         /* a HIP runtime call failed */
  CM_E_BUSY = -5,        /* serving queue full */
  CM_E_NOTFOUND = -6     /* unknown object or ticket */
};

typedef struct cm_context cm_context;
typedef struct cm_plan cm_plan;
typedef uint32_t cm_object;
typedef uint64_t cm_ticket;

/* Method constants; the paper leaves all of them open (Sec. II uses one
 * temperature tau everywhere, Sec. IV-C.1 names d_max and eps, Sec. IV-B.2
 * the number of sphere-trace steps). */
typedef struct {
  float tau_cap;     /* temperature of the smooth intersection of half-spaces */
  float tau_cup;     /* temperature of the smooth union of pieces */
  float tau_st;      /* sigmoid gate of the sphere-trace step */
  float tau_clip;    /* softclip temperature */
  float tau_blend;   /* blending softmax temperature */
  float d_max;       /* contact distance threshold */
  float eps_t;       /* transition bandwidth */
  float eps_n;       /* normal normalisation epsilon */
  float grid_margin;      /* voxel grid = vertex AABB grown by grid_margin + */
  float grid_margin_rel;  /*   grid_margin_rel * (object bounding radius)    */
  int32_t st_iters;  /* sphere-trace steps K */
  int32_t grid_res;  /* voxels per axis (1..128) */
  int32_t curve;     /* vertex/edge serialization: 0 none, 1 Morton, 2 Hilbert */
  int32_t broad_phase;  /* 0 off, 1 on */
  int32_t edge_bound;   /* 0: min(lb1, lb2) - l (the paper's); 1: tight form */
  int32_t prune_pieces; /* 1: skip, per wave, pieces whose union weight is provably
                           below 2^-28 at all its points (results equal within
                           FP32 rounding); 0: every piece at every point */
  int32_t sdf_kind;     /* SDF representation of every object of the context (the
                           paper's two alternatives, Sec. III):
                           0: smooth union of smooth intersections of the pieces'
                              hull half-spaces (Sec. III-A.2/3);
                           2: primitives (Sec. III-A), set per object by
                              cm_object_set_prims (its pieces stay the mesh side):
                              PSQs and XPSQs folded by smooth union, subtraction and
                              intersection.  No broad-phase bound (every contact is
                              evaluated) and no adjoint tape;
                           1: cubic spline (Sec. III-B): the ground-truth SDF and
                              normal of the pieces (closest point on their hulls,
                              phi = min over pieces) sampled at the (grid_res + 1)^3
                              corners of the grid box, natural cubic-spline
                              coefficients by 1-D solves along each axis, and a
                              separately fitted normal spline; the contact normal is
                              the normal spline's value.  Outside the box phi
                              continues as s(pi(x)) + |x - pi(x)|.  The broad phase
                              bounds the spline over each cell by 216 times its
                              least coefficient there (B-spline convex hull); the
                              grid margins set the box (grid_margin_rel = 0 keeps it
                              tight).  No adjoint tape: the adjoint recomputes. */
  int32_t edge_assign;  /* edge assignment for blending (Sec. IV-D.1): 0: an edge
                           counts in its own piece's group only; 1: also in the group
                           of every other piece of its object it crosses (a part of
                           positive length, > 1e-9 of the object's scale, inside that
                           piece's hull), after the piece's own edges.  Vertices stay
                           with their own piece.  cm_object_export lists own edges. */
  float tau_t;          /* primitives: soft clip of the spline parameter t to (0, 1) */
  float tau_disc;       /* primitives: softplus and sigmoid of the projection cubic's
                           discriminant (both dimensionless) */
} cm_params;

/* A pair-query: objects and poses (body -> world). 64 bytes. */
typedef struct {
  cm_object a, b;
  float qa[4], ta[3];
  float qb[4], tb[3];
} cm_query;

/* Device SoA group records: p, n, q are [3][G] (x row, y row, z row), d, W,
 * logZ are [G], G = total groups of the plan. */
typedef struct {
  float *p, *n, *d, *q, *W, *logZ;
} cm_groups;

/* Constants scaled with a length L_ref (metres): tau = 0.01 L_ref (all four
 * smoothing temperatures), tau_blend = 0.02 L_ref, d_max = 0.05 L_ref,
 * eps_t = 0.025 L_ref, eps_n = 1e-6, K = 3, 32^3 grid with margin
 * 0.1 L_ref + 1.0 * radius, Hilbert serialization, broad phase on, edge_bound 0,
 * tau_t = 0.01, tau_disc = 1e-3. */
cm_status cm_default_params(float L_ref, cm_params* out);

/* Creates a context on HIP device `device` (-1: host-only context that builds
 * and exports geometry but cannot run queries).  mem_budget_bytes bounds the
 * device memory the serving loop may keep in flight (0 = 32 GiB). */
cm_status cm_init(int32_t device, const cm_params* params, size_t mem_budget_bytes, cm_context** out);
/* Stops the serving loop, waits for device work and frees everything. */
cm_status cm_shutdown(cm_context* ctx);
/* Message of the last error on this context (never NULL). */
const char* cm_last_error(cm_context* ctx);

/* Builds one object from n_pieces point clouds (object frame, FP64, host).
 * offsets[n_pieces + 1] index xyz triplets.  Per piece: convex hull, merge of
 * coplanar facets (|dn| < 1e-9, |dh| < 1e-9 * scale), unit outward planes
 * (n, h) with n.x + h <= 0 inside (Sec. III-A.3), hull vertices and feature
 * edges (edges between facets on different planes), serialization along the
 * space-filling curve of params.curve within the piece (Sec. IV-C.3).  Then the
 * object's voxel grid of phi at voxel centres is built on the device
 * (Sec. IV-C.2).  CM_E_DEGENERATE if a piece has < 4 non-coplanar points. */
cm_status cm_build_pieces(cm_context* ctx, int32_t n_pieces, const int64_t* offsets, const double* xyz,
                          cm_object* out);
/* Builds n_objects objects at once (host threads + one device upload).
 * obj_off[n_objects + 1] indexes pieces, piece_off[total pieces + 1] indexes
 * xyz triplets.  out[n_objects]. */
cm_status cm_build_objects(cm_context* ctx, int32_t n_objects, const int64_t* obj_off, const int64_t* piece_off,
                           const double* xyz, cm_object* out);
/* Builds an object from explicit pieces: planes (n, h) [P][4], vertices [V][3],
 * edges [E][2] of piece-local vertex indices; *_off[n_pieces + 1] index them.
 * Normals need not be unit (they are normalised); no hull is computed. */
cm_status cm_build_pieces_raw(cm_context* ctx, int32_t n_pieces, const int64_t* plane_off, const double* planes,
                              const int64_t* vert_off, const double* verts, const int64_t* edge_off,
                              const int32_t* edges, cm_object* out);
/* Frees the object's device memory.  Plans that use it become invalid. */
cm_status cm_release_object(cm_context* ctx, cm_object obj);
cm_status cm_object_info(cm_context* ctx, cm_object obj, int32_t* n_pieces, int64_t* n_planes, int64_t* n_verts,
                         int64_t* n_edges);
/* Host copies of the collision geometry in the device order: plane_off,
 * vert_off, edge_off [n_pieces + 1]; planes [P][4] (unit n, h); verts [V][3];
 * edges [E][2] piece-local.  Any pointer may be NULL. */
cm_status cm_object_export(cm_context* ctx, cm_object obj, int64_t* plane_off, double* planes, int64_t* vert_off,
                           double* verts, int64_t* edge_off, int32_t* edges);
/* Copies the object's voxel grid to the host (synchronous): G [n^3] (index
 * (i * n + j) * n + k) and meta = origin (3), spacing (3), circumradius, n. */
cm_status cm_object_grid(cm_context* ctx, cm_object obj, float* G, float* meta);
/* Copies a spline object's coefficients to the host (synchronous; contexts
 * with sdf_kind = 1): coef [(n+3)^3][4] (phi, n_x, n_y, n_z; index
 * (i (n+3) + j) (n+3) + k; may be NULL) and meta = n, box origin (3), cell
 * size (3).  Its grid (cm_object_grid) holds the per-cell lower bounds. */
cm_status cm_object_spline(cm_context* ctx, cm_object obj, float* coef, float* meta);

/* The SDF side of an object of a primitive context (sdf_kind 2) as n
 * primitives (Sec. III-A), records of 32 doubles (host):
 *   [0] kind: 0 PSQ (a superquadric intersected with half-spaces, at a fixed
 *       pose), 1 XPSQ (a PSQ swept along the quadratic spline
 *       p(t) = (1-t)^2 p1 + 2t(1-t) p2 + t^2 p3, t in [0, 1]);
 *   [1] op: how it joins the primitives before it: 0 smooth union (tau_cup),
 *       1 smooth subtraction, 2 smooth intersection (tau_cap); ignored for the
 *       first;
 *   [2..4] PSQ centre / XPSQ p1, [5..7] p2, [8..10] p3 (object frame);
 *   [11..14] PSQ rotation (unit quaternion w, x, y, z: PSQ frame -> object);
 *   [15..17] superquadric scales a, [18..19] exponents (eps1, eps2), at t = 0
 *       (PSQ: the superquadric); [20..22], [23..24] the same at t = 1 (XPSQ,
 *       linear in t); [25..31] unused.
 * The superquadric's SDF is its radial distance |x| (1 - f(x)^(-eps1/2)) (f the
 * inside-outside function of Sec. III-A.1; exact for a sphere).  An XPSQ's PSQ
 * frame is the spline's Frenet frame: x along the in-plane normal, y along
 * the binormal (B x A, A = p1 - 2 p2 + p3, B = 2 (p2 - p1)), z along the
 * tangent; its spline must be curved.  Half-spaces planes[4 plane_off[i] ..
 * 4 plane_off[i + 1]) (n, h; n.x + h <= 0 inside; normalised here) in each PSQ
 * frame, plane_off[0] = 0.  Replaces the object's earlier primitives
 * (synchronous).  CM_E_INVALID for a bad record or a context of another
 * sdf_kind; CM_E_NOTFOUND for an unknown object. */
cm_status cm_object_set_prims(cm_context* ctx, cm_object obj, int32_t n, const double* rec, const int64_t* plane_off,
                              const double* planes);

/* A plan fixes the objects of a batch of n pair-queries (poses are read at run
 * time from the device query array) and owns the scratch of the batched
 * persistent launch: broad-phase survivor bitmasks, the work queue of survivor
 * tiles (64 contacts of one piece, vertices or edges), per-tile partials. */
/* n >= 1 (an empty batch is CM_E_INVALID); the context must own a device. */
cm_status cm_plan_create(cm_context* ctx, const cm_query* host_queries, int32_t n, cm_plan** out);
cm_status cm_plan_destroy(cm_plan* plan);
/* A plan of fixed capacity whose batch can be replaced (batching of the
 * persistent launch over changing sets of pair-queries, Sec. IV-C): device
 * memory laid out for up to max_queries pair-queries, max_groups groups (sum
 * over queries of both objects' piece counts) and max_contacts contacts (sum of
 * both objects' vertices and edges), holding an empty batch until
 * cm_plan_refill.  Every kernel of a pass reads the batch's counts and the
 * object table from the plan's device memory, so a graph captured on such a
 * plan (cm_graph_create) replays whatever batch the plan holds when it is
 * launched.  Records and cotangents of a reserved plan are SoA rows of stride
 * max_groups (cm_groups rows of a [12][max_groups] array), gradients and
 * directions [max_queries][12]; the first G (n) of each row are the batch's.
 * CM_E_INVALID for non-positive capacities; CM_E_OOM if the memory is not there. */
cm_status cm_plan_reserve(cm_context* ctx, int32_t max_queries, int64_t max_groups, int64_t max_contacts,
                          cm_plan** out);
/* Plans the batch host_queries[0..n) (n may be 0) into a reserved plan and
 * enqueues the upload of its tables on `stream`: passes enqueued on the same
 * stream before this call see the previous batch, those after it this one.
 * Waits (host) only for the previous refill's uploads.  CM_E_INVALID if the
 * plan was not reserved or the batch exceeds a capacity (the plan keeps its
 * previous batch); CM_E_NOTFOUND for an unknown object. */
cm_status cm_plan_refill(cm_context* ctx, cm_plan* plan, const cm_query* host_queries, int32_t n, void* stream);
/* Capacities of a reserved plan; for other plans the batch's own sizes. */
cm_status cm_plan_capacity(const cm_plan* plan, int32_t* max_queries, int64_t* max_groups, int64_t* max_contacts);
/* Totals of the batch the plan holds: groups G, contacts C (vertices + edges
 * of both sides), queries n. */
cm_status cm_plan_info(const cm_plan* plan, int64_t* n_groups, int64_t* n_contacts, int32_t* n_queries);
/* group_off[n + 1], contact_off[n + 1] (host).  Either may be NULL. */
cm_status cm_plan_offsets(const cm_plan* plan, int64_t* group_off, int64_t* contact_off);
/* Work statistics of the last launch on this plan (synchronous):
 * [0] surviving vertices, [1] surviving edges, [2] tiles, [3] vertices,
 * [4] edges, [5] point-plane evaluations of a forward pass (vertices once,
 * edges 2 K + 1 times), [6] surviving-vertex x opposing-plane pairs,
 * [7] surviving-edge x opposing-plane pairs. */
cm_status cm_plan_stats(const cm_plan* plan, int64_t* stats8);

/* Point-plane evaluations the narrow-phase kernels of the plan's last pass
 * performed (synchronous), counted per wave lane including lanes of partly
 * filled tiles and the support-plane bounds, after piece pruning:
 * performed2[0] for vertex contacts, performed2[1] for edge contacts (all
 * trace steps); compare with cm_plan_stats [6] and (2 K + 1) x [7] (times the
 * evaluation passes). */
cm_status cm_plan_work(const cm_plan* plan, int64_t* performed2);

/* Kernel timing with HIP events recorded on the launch stream around the
 * broad phase and each narrow-phase kernel of the plan's launches (off by
 * default).  cm_plan_timing (synchronous) returns the last durations in ms:
 * [0] broad phase, [1] forward narrow phase, [2] forward narrow phase with
 * tangents (HVP), [3] adjoint narrow phase, [4] dual adjoint narrow phase
 * (HVP); -1 for a kernel the plan's last pass did not launch. */
cm_status cm_plan_set_timing(cm_plan* plan, int32_t enable);
cm_status cm_plan_timing(const cm_plan* plan, float* ms5);

/* Forward pass over the plan's batch.  q_dev: device cm_query[n] (objects
 * must match the plan).  out: device group records.  contact_dbg (nullable):
 * device float [13][C] SoA per contact: mask (1 = survived the broad phase),
 * d_c, f, w, p_c (3), n_c (3), phi (NaN when filtered), kind (0 vertex,
 * 1 edge), group index (bit pattern of an int32).  Contact order per query:
 * A's pieces then B's; per piece its vertices then its edges, in the order of
 * cm_object_export. */
cm_status cm_contacts_fwd(cm_context* ctx, cm_plan* plan, const cm_query* q_dev, cm_groups out, float* contact_dbg,
                          void* stream);
/* For callers that cannot allocate device memory at call time (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward pass of cm_contacts_fwd (same kernels, same records, bitwise, at the
 * plan's launch shape) with all launch scratch -- survivor bitmasks, counts and
 * offsets, filtered sums, the tile counter, blend partials -- in one fixed
 * 64 MiB device array of the library (one per GPU, held until the process
 * ends) instead of the plan's memory.  The call allocates nothing; the plan
 * (created beforehand) supplies its uploaded tables, the caller the queries
 * and output records as for cm_contacts_fwd.  CM_E_INVALID, with nothing
 * launched, when the batch needs more than 64 MiB of launch scratch (about
 * (W + E) * 128 bytes for W survivor words and E entries: split the batch
 * into smaller plans).  Every call on a GPU shares that GPU's array: calls that
 * overlap in time on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  No debug output, timing or work counters. */
cm_status cm_contacts_fwd_noalloc(cm_context* ctx, cm_plan* plan, const cm_query* q_dev, cm_groups out,
                                  void* stream);
/* Gradient of L = sum_g <cot_g, y_g> w.r.t. xi = (w_A, v_A, w_B, v_B), the
 * world-frame perturbation T_X <- (exp([w_X]x) R_X, t_X + v_X) at xi = 0.
 * cot: device group records (same layout as out).  grad: device float [n][12].
 * Runs the forward sweep again (nothing is kept from an earlier
 * cm_contacts_fwd); that sweep writes, for the survivor tiles the plan's tape
 * holds (a quarter of the context's memory budget at most), the values the
 * adjoint needs (phi, gradient and Hessian at the contact point and at the
 * sphere-trace iterates), and the adjoint recomputes them for tiles past the
 * tape.  The adjoint keeps the trace steps in registers: st_iters <= 4
 * (CM_E_INVALID otherwise; the forward entry points take up to 64). */
cm_status cm_contacts_bwd(cm_context* ctx, cm_plan* plan, const cm_query* q_dev, cm_groups cot, float* grad,
                          void* stream);
/* Hessian-vector product H dir of the same L (dir: device float [n][12]),
 * written to hv [n][12]; grad (nullable) receives the gradient. */
cm_status cm_hvp(cm_context* ctx, cm_plan* plan, const cm_query* q_dev, cm_groups cot, const float* dir, float* hv,
                 float* grad, void* stream);
/* Jacobian-vector product of the group records (Sec. IV-D outputs) along the
 * pose direction dir (device float [n][12], the xi of cm_contacts_bwd): out
 * receives the records, out_tangent (same layout) their derivatives
 * d y_g / d xi . dir, from one forward sweep in dual numbers.  Twelve calls
 * with the unit directions give the blended Jacobian of every record.  All
 * buffers are caller-owned device memory; CM_E_INVALID on a null argument. */
cm_status cm_contacts_jvp(cm_context* ctx, cm_plan* plan, const cm_query* q_dev, cm_groups out,
                          cm_groups out_tangent, const float* dir, void* stream);

/* Isosurface projection of contact points (Sec. IV-A, last paragraph): the
 * collision mesh and the SDF's zero level set differ slightly, and a contact
 * point p found on the mesh is moved onto the level set by
 * proj(p) = p - phi(p) n(p), with phi and n those of the SDF the point's group
 * was evaluated against (groups of A: B's SDF; groups of B: A's), in that
 * body's frame.  p_in, p_out: device float [3][G] (SoA rows x, y, z; world
 * frame; typically the records' p), one point per group of the plan; may
 * alias.  Forward only (no derivatives).  Asynchronous on `stream`. */
cm_status cm_project_points(cm_context* ctx, cm_plan* plan, const cm_query* q_dev, const float* p_in, float* p_out,
                            void* stream);

/* ---------------------------------------------------------------- serving --
 * A background scheduler admits requests while the device memory they need
 * stays within the context's budget, packs the queries of all admitted
 * requests into one batch, runs it on one of several streams while the next
 * batch is formed, and completes tickets when their batch finishes.
 * Inputs are copied at submit; outputs are written into the request's host
 * buffers and are valid once cm_poll reports done.  Thread-safe.  Each
 * result is independent of what else shares its batch. */
typedef struct {
  const cm_query* q;        /* host cm_query[n] */
  int32_t n;
  int32_t want_grad;        /* 0: forward only; 1: forward + gradient */
  const float* cotangent;   /* host [G][12] AoS group cotangents (want_grad) */
  float* out_groups;        /* host [G][12] AoS group records */
  float* out_grad;          /* host [n][12] (want_grad) */
} cm_request;
/* CM_E_OOM if the request alone exceeds the budget; CM_E_BUSY if the queue is
 * full.  The group count G of a request is sum over its queries of the two
 * objects' piece counts. */
cm_status cm_submit(cm_context* ctx, const cm_request* req, cm_ticket* ticket);
/* done = 1 once finished; *result is the ticket's status.  A finished ticket
 * is forgotten after the poll that reports it. */
cm_status cm_poll(cm_context* ctx, cm_ticket ticket, int32_t* done, cm_status* result);
/* Blocks until the ticket finishes (or timeout_ms elapses: CM_E_BUSY). */
cm_status cm_wait(cm_context* ctx, cm_ticket ticket, int32_t timeout_ms, cm_status* result);
/* Latencies (seconds, from cm_submit to results written) of completed
 * requests in completion order since the last call; copies at most cap and
 * removes them from the record; *n = number copied. */
cm_status cm_serve_latencies(cm_context* ctx, double* out, int64_t cap, int64_t* n);
/* One pass of the whole path for the plan's batch: the group records (out;
 * all members null to skip them), the gradient of L = <cot, y> w.r.t. both
 * poses (grad, [n][12]) and, when dir is given, H dir (hv, [n][12]; dir and
 * hv both null or both set).  One broad phase, one forward sweep that keeps
 * the adjoint tape (in dual numbers when dir is given), one adjoint: the work
 * of cm_contacts_fwd + cm_contacts_bwd (+ cm_hvp) without repeating the
 * forward.  The records and the gradient equal theirs up to rounding (with
 * dir they are the value parts of the dual evaluation).  Device pointers,
 * enqueued on `stream`; CM_E_INVALID as for cm_hvp. */
cm_status cm_contacts_step(cm_context* ctx, cm_plan* plan, const cm_query* q_dev, cm_groups out, cm_groups cot,
                           float* grad, const float* dir, float* hv, void* stream);

/* HIP graph of a plan's step: cm_graph_create records the launches of
 * cm_contacts_step with these device buffers (same arguments and rules) into
 * a graph; cm_graph_launch replays it on `stream`.  The kernels read every
 * count on the device, so a replay computes the step for whatever poses the
 * query buffer holds at that time, and, on a reserved plan, for whatever batch
 * the last cm_plan_refill enqueued before it; buffers and plan must outlive the graph,
 * and replays of one plan must not overlap.  Timing events are not recorded
 * into the graph.  For callers whose step launch overhead matters (small
 * batches, serving loops). */
typedef struct cm_graph cm_graph;
cm_status cm_graph_create(cm_context* ctx, cm_plan* plan, const cm_query* q_dev, cm_groups out, cm_groups cot,
                          float* grad, const float* dir, float* hv, cm_graph** graph);
cm_status cm_graph_launch(cm_graph* graph, void* stream);
cm_status cm_graph_destroy(cm_graph* graph);

/* Launch-shape autotuner (batching of the persistent launch): times
 * cm_contacts_step (records not written) on `stream` (synchronous) with 2, 4,
 * 6, 8, 12 and 16 persistent workgroups of 4 waves per CU, then at the fastest
 * count of resident waves per CU with workgroups of 2 and of 1 wave, and keeps
 * the fastest (workgroups per CU, waves per workgroup) for the plan's later
 * launches of the same kind: with dir the sweeps in dual numbers (H v),
 * without dir the float sweeps (forward, gradient); *best (nullable) receives
 * the workgroups per CU (cm_plan_wg_waves the workgroup size).  A tile is one
 * wave's 64 contacts; results do not depend on the shape. */
cm_status cm_plan_autotune(cm_context* ctx, cm_plan* plan, const cm_query* q_dev, cm_groups cot, float* grad,
                           const float* dir, float* hv, void* stream, int32_t* best);

/* Launch shape of a plan: persistent workgroups per CU for the float sweeps
 * (forward, gradient) and for the sweeps in dual numbers (H v).  The setter
 * takes values in [1, 64] (else CM_E_INVALID, shape unchanged) and lets a shape
 * tuned on a representative sub-batch (cm_plan_autotune on a smaller plan of
 * the same workload) be applied to a large plan; results do not depend on it.
 * The getter's outputs are nullable. */
cm_status cm_plan_set_launch_shape(cm_plan* plan, int32_t float_per_cu, int32_t dual_per_cu);
cm_status cm_plan_launch_shape(const cm_plan* plan, int32_t* float_per_cu, int32_t* dual_per_cu);
/* Waves per workgroup of the narrow-phase sweeps (float, dual): 1, 2 or 4
 * (default 4; else CM_E_INVALID, unchanged); results do not depend on it.
 * The getter's outputs are nullable. */
cm_status cm_plan_set_wg_waves(cm_plan* plan, int32_t float_waves, int32_t dual_waves);
cm_status cm_plan_wg_waves(const cm_plan* plan, int32_t* float_waves, int32_t* dual_waves);

/* Serving statistics: [0] submitted, [1] completed, [2] batches, [3] queued,
 * [4] in flight, [5] peak device bytes held by the serving slots' buffers (the
 * admission keeps it within the budget), [6] queries completed. */
cm_status cm_serve_stats(cm_context* ctx, int64_t* stats7);

#ifdef __cplusplus
}
#endif
#endif /* CM_H */
