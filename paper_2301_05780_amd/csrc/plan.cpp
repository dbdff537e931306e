// Work decomposition of a single-instance assembly (host only).
#include "plan.h"

#include <algorithm>
#include <climits>

namespace pdd {

namespace {

// interleave the low 16 bits of v with zeros (Morton code helper)
uint32_t spread_bits(uint32_t v) {
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

}  // namespace

pdd_status plan_tickets(const Geometry& g, const std::vector<int32_t>& npk, int64_t per_ticket, bool spatial,
                        uint32_t instance, TicketPlan& out, std::string& err, const double* h_knot) {
  if (per_ticket < 1) {
    err = "plan_tickets: paths per ticket must be >= 1";
    return PDD_EINVAL;
  }
  if ((int64_t)npk.size() != g.n) {
    err = "plan_tickets: one path count per knot";
    return PDD_EINVAL;
  }
  out = TicketPlan();
  out.begin.assign(g.n + 1, 0);
  std::vector<double> cost;
  for (int64_t k = 0; k < g.n; ++k) {
    const int64_t N = npk[k];
    if (N < 1) {
      err = "plan_tickets: path counts must be >= 1";
      return PDD_EINVAL;
    }
    const int64_t c = (N + per_ticket - 1) / per_ticket;
    // expected steps per path: the mean exit time (which scales with the
    // patch area, eq. 26) over the knot's time step
    double area = (double)(g.box[4 * k + 1] - g.box[4 * k + 0]) * (double)(g.box[4 * k + 3] - g.box[4 * k + 2]);
    if (h_knot) area /= h_knot[k];
    for (int64_t i = 0; i < c; ++i) {
      Ticket t;
      t.knot = (int32_t)k;
      t.p0 = (int32_t)(N * i / c);
      t.p1 = (int32_t)(N * (i + 1) / c);
      t.inst = instance;
      out.tickets.push_back(t);
      cost.push_back(area * (double)(t.p1 - t.p0));
    }
    if ((int64_t)out.tickets.size() > INT32_MAX) {
      err = "too many tickets";
      return PDD_EUNSUPPORTED;
    }
    out.begin[k + 1] = (int32_t)out.tickets.size();
  }
  const size_t T = out.tickets.size();
  out.order.resize(T);
  for (size_t i = 0; i < T; ++i) out.order[i] = (int32_t)i;
  if (spatial) {
    std::vector<uint32_t> key(T);
    for (size_t i = 0; i < T; ++i) {
      const int32_t k = out.tickets[i].knot;
      const uint32_t sx = (uint32_t)(g.ix[k] / g.m), sy = (uint32_t)(g.iy[k] / g.m);
      key[i] = spread_bits(sx) | (spread_bits(sy) << 1);
    }
    std::stable_sort(out.order.begin(), out.order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    out.cum_cost.resize(T + 1);
    out.cum_cost[0] = 0.0;
    for (size_t i = 0; i < T; ++i) out.cum_cost[i + 1] = out.cum_cost[i] + cost[out.order[i]];
  } else {
    std::stable_sort(out.order.begin(), out.order.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
  }
  return PDD_OK;
}

void xcd_split(const std::vector<double>& cum_cost, int64_t n_tickets, int64_t grid, int32_t xb[9]) {
  xb[0] = 0;
  const double total_cost = cum_cost.back();
  int64_t blocks_before = 0;
  for (int x = 0; x < 8; ++x) {
    blocks_before += (grid - x + 7) / 8;
    const double target = total_cost * (double)blocks_before / (double)grid;
    const auto it = std::lower_bound(cum_cost.begin(), cum_cost.end(), target);
    xb[x + 1] = (x == 7) ? (int32_t)n_tickets
                         : std::max(xb[x], (int32_t)std::min<int64_t>(it - cum_cost.begin(), n_tickets));
  }
}

}  // namespace pdd
