// Host-side PDDSparse discretisation of a grid-aligned rectangle (Sec. 3.1):
// knots on the grid lines, the patch of each knot (eqs. 13-15), the four
// patch sides (eq. 14) with their type and clamp range, the segment stencils
// (eq. 17) and the CSR sparsity pattern of G (support of eq. 24).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "pdd.h"

namespace pdd {

// Side order used everywhere: E, N, W, S.
enum Side { SIDE_E = 0, SIDE_N = 1, SIDE_W = 2, SIDE_S = 3 };

struct SideInfo {
  int32_t at;        // lattice coordinate of the side's grid line
  int32_t lo, hi;    // side range along the line (lattice units)
  int32_t clo, chi;  // clamp range along the line (lo - ext, hi + ext, clipped)
  bool boundary;     // the side lies on the domain boundary
  bool vertical;     // line x = const (E, W) or y = const (N, S)
};

struct Geometry {
  double x0 = 0, x1 = 0, y0 = 0, y1 = 0;
  int32_t H = 0, m = 0, ext = 0, L = 0;  // L = H m lattice intervals per direction
  double dx = 0, dy = 0;
  int64_t n = 0, nnz = 0;
  std::vector<int32_t> ix, iy;          // knot lattice coordinates, canonical order
  std::vector<int32_t> index;           // (L+1)^2 lattice -> knot index or -1, [iy * (L+1) + ix]
  std::vector<int32_t> box;             // 4 per knot: xlo, xhi, ylo, yhi (lattice)
  std::vector<int32_t> row_ptr, col_idx;
  int32_t slot_len = 0;                 // max clamp-range length over interface sides (+1)

  SideInfo side(int64_t k, int o) const;
  int32_t knot_at(int32_t lx, int32_t ly) const { return index[(int64_t)ly * (L + 1) + lx]; }
};

// Validates the partition/knots and fills g.  Returns PDD_OK or PDD_EINVAL
// with a message in err.  When with_pattern is false only the knots and
// patches are built.
pdd_status build_geometry(const pdd_partition& part, const pdd_knots& kn, Geometry& g,
                          std::string& err, bool with_pattern = true);

// Number of knots without building anything: 2 (H-1)(H m - 1) - (H-1)^2.
int64_t knot_count(int32_t H, int32_t m);

}  // namespace pdd
