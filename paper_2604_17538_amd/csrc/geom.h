// Host-side collision geometry of convex pieces (FP64).
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace cm {

// Collision geometry of one convex piece.
struct PieceGeom {
  std::vector<double> planes;  // 4 per plane: unit outward n, h (n.x + h <= 0 inside)
  std::vector<double> verts;   // 3 per vertex
  std::vector<int32_t> edges;  // 2 per edge, piece-local vertex indices (a < b)
  size_t n_planes() const { return planes.size() / 4; }
  size_t n_verts() const { return verts.size() / 3; }
  size_t n_edges() const { return edges.size() / 2; }
};

// Convex hull of n points, merge of coplanar facets, feature edges.
// Returns 0 on success, -3 (CM_E_DEGENERATE) if the points span < 3 dimensions.
int build_hull_piece(const double* xyz, int64_t n, PieceGeom* out);

// Reorders vertices and edges along a space-filling curve over the piece's
// bounding box: 0 none, 1 Morton (Z-order), 2 Hilbert.
void serialize_piece(PieceGeom* g, int curve);

// 3-D curve keys of 10-bit integer coordinates (30-bit keys).
uint32_t morton_key(uint32_t x, uint32_t y, uint32_t z);
uint32_t hilbert_key(uint32_t x, uint32_t y, uint32_t z);

}  // namespace cm
