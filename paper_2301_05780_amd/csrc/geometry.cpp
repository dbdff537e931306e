// Host discretisation: knots, patches, sides, stencils and the CSR pattern.
//
// Knots are the lattice points strictly inside the domain that lie on a grid
// line (Sec. 3.1); lattice points on the boundary carry the Dirichlet datum
// and are not unknowns.  A knot between two crossings belongs to two squares
// and its slab is the 2-square rectangle across its line; a crossing belongs
// to four squares (eq. 13).  The grid is aligned with the domain, so every
// slab lies in the closed domain and the patch equals the slab (eq. 15).
#include "geometry.h"

#include <algorithm>
#include <cmath>

namespace pdd {

int64_t knot_count(int32_t H, int32_t m) {
  const int64_t h = H, L = (int64_t)H * m;
  return 2 * (h - 1) * (L - 1) - (h - 1) * (h - 1);
}

SideInfo Geometry::side(int64_t k, int o) const {
  const int32_t xlo = box[4 * k + 0], xhi = box[4 * k + 1];
  const int32_t ylo = box[4 * k + 2], yhi = box[4 * k + 3];
  SideInfo s;
  switch (o) {
    case SIDE_E: s.at = xhi; s.lo = ylo; s.hi = yhi; s.vertical = true; break;
    case SIDE_W: s.at = xlo; s.lo = ylo; s.hi = yhi; s.vertical = true; break;
    case SIDE_N: s.at = yhi; s.lo = xlo; s.hi = xhi; s.vertical = false; break;
    default:     s.at = ylo; s.lo = xlo; s.hi = xhi; s.vertical = false; break;
  }
  s.boundary = (s.at == 0 || s.at == L);
  if (s.boundary) {
    s.clo = 0;
    s.chi = L;
  } else {
    s.clo = std::max(0, s.lo - ext);
    s.chi = std::min(L, s.hi + ext);
  }
  return s;
}

pdd_status build_geometry(const pdd_partition& part, const pdd_knots& kn, Geometry& g,
                          std::string& err, bool with_pattern) {
  if (!(part.x1 > part.x0) || !(part.y1 > part.y0) || !std::isfinite(part.x0) ||
      !std::isfinite(part.x1) || !std::isfinite(part.y0) || !std::isfinite(part.y1)) {
    err = "partition: need finite x0 < x1 and y0 < y1";
    return PDD_EINVAL;
  }
  if (part.H < 2) { err = "partition: need H >= 2 subdomains per direction"; return PDD_EINVAL; }
  if (kn.m < 1 || kn.ext < 0) { err = "knots: need m >= 1 and ext >= 0"; return PDD_EINVAL; }
  const int64_t L64 = (int64_t)part.H * kn.m;
  if (L64 > 8192) { err = "knots: H * m must not exceed 8192"; return PDD_EINVAL; }

  g = Geometry();
  g.x0 = part.x0; g.x1 = part.x1; g.y0 = part.y0; g.y1 = part.y1;
  g.H = part.H; g.m = kn.m; g.ext = kn.ext; g.L = (int32_t)L64;
  g.dx = (g.x1 - g.x0) / (double)g.L;
  g.dy = (g.y1 - g.y0) / (double)g.L;
  const int32_t L = g.L, m = g.m;

  g.index.assign((size_t)(L + 1) * (L + 1), -1);
  for (int32_t y = 1; y < L; ++y)
    for (int32_t x = 1; x < L; ++x)
      if (x % m == 0 || y % m == 0) {
        g.index[(size_t)y * (L + 1) + x] = (int32_t)g.ix.size();
        g.ix.push_back(x);
        g.iy.push_back(y);
      }
  g.n = (int64_t)g.ix.size();

  g.box.resize(4 * g.n);
  for (int64_t k = 0; k < g.n; ++k) {
    const int32_t x = g.ix[k], y = g.iy[k];
    const bool on_v = (x % m == 0), on_h = (y % m == 0);
    g.box[4 * k + 0] = on_v ? x - m : (x / m) * m;
    g.box[4 * k + 1] = on_v ? x + m : (x / m) * m + m;
    g.box[4 * k + 2] = on_h ? y - m : (y / m) * m;
    g.box[4 * k + 3] = on_h ? y + m : (y / m) * m + m;
  }

  int32_t slot = 1;
  for (int64_t k = 0; k < g.n; ++k)
    for (int o = 0; o < 4; ++o) {
      SideInfo s = g.side(k, o);
      if (!s.boundary) slot = std::max(slot, s.chi - s.clo + 1);
    }
  g.slot_len = slot;

  if (!with_pattern) return PDD_OK;

  g.row_ptr.assign(g.n + 1, 0);
  std::vector<int32_t> cols;
  cols.reserve(4 * (size_t)slot + 1);
  std::vector<int32_t> all;
  all.reserve((size_t)g.n * 16);
  for (int64_t k = 0; k < g.n; ++k) {
    cols.clear();
    cols.push_back((int32_t)k);
    for (int o = 0; o < 4; ++o) {
      SideInfo s = g.side(k, o);
      if (s.boundary) continue;
      for (int32_t q = std::max(1, s.clo); q <= std::min(L - 1, s.chi); ++q)
        cols.push_back(s.vertical ? g.knot_at(s.at, q) : g.knot_at(q, s.at));
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    if ((int64_t)all.size() + (int64_t)cols.size() > INT32_MAX) {
      err = "pattern: more than 2^31 - 1 structural nonzeros";
      return PDD_EINVAL;
    }
    all.insert(all.end(), cols.begin(), cols.end());
    g.row_ptr[k + 1] = (int32_t)all.size();
  }
  g.col_idx.swap(all);
  g.nnz = (int64_t)g.col_idx.size();
  return PDD_OK;
}

}  // namespace pdd
