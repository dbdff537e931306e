// Work decomposition of a single-instance assembly (host only): tickets, the
// order in which waves claim them, and the split of that order over the
// eight XCDs.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "geometry.h"
#include "kernels.h"

namespace pdd {

struct TicketPlan {
  std::vector<Ticket> tickets;     // knot, path range [p0, p1), instance
  std::vector<int32_t> begin;      // first ticket of each knot, n + 1 entries
  std::vector<int32_t> order;      // claim order (a permutation of the tickets)
  std::vector<double> cum_cost;    // spatial order: expected cost summed along the order (size + 1)
};

// Knot k's N_k paths are cut into ceil(N_k / per_ticket) near-equal
// contiguous ranges.  The claim order is, with `spatial`, the tickets sorted
// by the Morton (Z) index of their knot's subdomain (stable: knot order and
// path ranges within), else longest expected first (expected cost = patch
// area x paths, the mean exit time scaling with the area, eq. 26, divided
// by the knot's time step when per-knot steps h_knot (host, nullable) are
// given; stable).
pdd_status plan_tickets(const Geometry& g, const std::vector<int32_t>& npk, int64_t per_ticket, bool spatial,
                        uint32_t instance, TicketPlan& out, std::string& err, const double* h_knot = nullptr);

// Split of a spatial order over the XCDs for a grid of `grid` workgroups
// (grid >= 8; workgroup b runs on XCD b mod 8): XCD x, which holds
// ceil((grid - x) / 8) workgroups, takes tickets [xb[x], xb[x+1]) of the
// order, the share of the expected cost matching its share of workgroups.
void xcd_split(const std::vector<double>& cum_cost, int64_t n_tickets, int64_t grid, int32_t xb[9]);

}  // namespace pdd
