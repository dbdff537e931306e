// Persistent lane-per-path Monte Carlo assembly of the PDDSparse rows
// (eqs. 9 and 20-25) for gfx950.
//
// Work decomposition.  The host cuts every knot's N_k paths into tickets
// (knot, path range).  Each wave of the persistent grid takes tickets in a
// fixed stride (wave w: tickets w, w + W, w + 2W, ...) and owns two LDS tally
// rows.  Every lane integrates one path at a time; when its path exits, the
// lane is refilled with the next path of the wave's current ticket, ranked
// among the idle lanes by a ballot (no atomics).  When the current ticket has
// handed out all its paths, the next ticket is opened in the other row while
// the stragglers of the previous one drain, so lanes never wait for the
// slowest path of a ticket.  A drained row is written once to the ticket's
// partial row in HBM; a second kernel sums a knot's partial rows in ticket
// order into the CSR values and b (deterministic for a fixed launch shape).
//
// Per lane and per Philox draw (one call feeds two Euler steps), both steps
// run with all lanes of the wave at the same draw parity, so the Philox call
// is never divergent.
//
// Tallies: G slots are float64 LDS atomics (two per interface exit); b, the
// score moments, the step count and the exit-side counts accumulate in lane
// registers and are spilled into the row only when the lane moves to another
// row or the row is flushed.
#include <type_traits>

#include "device_common.h"

namespace pdd {

namespace {

struct WaveBuf {
  KnotDesc d;
  double ebox[4];      // strict exit thresholds: x > e[0], y > e[1], x < e[2], y < e[3]
  int32_t ticket, p0, p1;
  uint32_t inst;
};
static_assert(sizeof(WaveBuf) % 16 == 0, "WaveBuf alignment");

__device__ __forceinline__ int lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

template <typename R>
__device__ __forceinline__ R next_down(R v) {
  return nextafter(v, -INFINITY);
}
template <typename R>
__device__ __forceinline__ R next_up(R v) {
  return nextafter(v, INFINITY);
}

// One Euler-Maruyama step of eq. (9) with coefficients frozen at the left point.
template <int KIND, typename R>
__device__ __forceinline__ void em_step(const AsmParams& P, R z0, R z1, R& x, R& y, R& Y, R& Z) {
  Coef<R> c;
  coef_at<KIND>(P.coef, x, y, c);
  if constexpr (std::is_same<R, double>::value) {
#pragma clang fp contract(off)
    const double sq = P.sqrt_h, h = P.h;
    const double dWx = sq * z0, dWy = sq * z1;
    const double nx = x + c.dx * h + (c.sxx * dWx + c.sxy * dWy);
    const double ny = y + c.dy * h + (c.sxy * dWx + c.syy * dWy);
    const double nZ = Z - c.f * Y * h;
    Y = Y * (1.0 + c.c * h);
    x = nx; y = ny; Z = nZ;
  } else {
    const float sq = (float)P.sqrt_h, h = (float)P.h;
    const float dWx = sq * z0, dWy = sq * z1;
    const float nx = x + c.dx * h + (c.sxx * dWx + c.sxy * dWy);
    const float ny = y + c.dy * h + (c.sxy * dWx + c.syy * dWy);
    const float nZ = Z - c.f * Y * h;
    Y = Y * (1.0f + c.c * h);
    x = nx; y = ny; Z = nZ;
  }
}

// Exit threshold of side o for the knot in `d` (NAIVE: the side line; GM: the
// line shifted inwards by c_GM sqrt(a_nn) sqrt(h), a_nn = N^T A N evaluated on
// the side at the knot's along-line coordinate; for every analytic family a_nn
// of a vertical side depends on x only and of a horizontal side on y only).
// Returned as the strict threshold of the test that flags side o.
template <int KIND, typename R>
__device__ R exit_threshold(const AsmParams& P, const KnotDesc& d, int o) {
  const double line = d.line[o];
  if (P.exit_rule == PDD_EXIT_NAIVE) return (R)line;
  const bool vert = (o == 0 || o == 2);
  Coef<R> c;
  const R px = vert ? (R)line : (R)d.sx;
  const R py = vert ? (R)d.sy : (R)line;
  coef_at<KIND>(P.coef, px, py, c);
  R thr;
  {
#pragma clang fp contract(off)
    const R ann = vert ? (c.sxx * c.sxx + c.sxy * c.sxy) : (c.sxy * c.sxy + c.syy * c.syy);
    const R delta = (R)kGM * sqrt(ann) * (R)P.sqrt_h;
    thr = (o < 2) ? (R)line - delta : (R)line + delta;
  }
  // x >= thr  <=>  x > next_down(thr);  x <= thr  <=>  x < next_up(thr)
  return (o < 2) ? next_down(thr) : next_up(thr);
}

template <int KIND, bool F64>
__global__ __launch_bounds__(256) void k_assemble(AsmParams P) {
  using R = typename std::conditional<F64, double, float>::type;
  extern __shared__ double smem[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int waves_per_block = blockDim.x >> 6;
  const int RL = P.row_len, SL = P.slot_len;
  const size_t wave_doubles = (2 * sizeof(WaveBuf)) / sizeof(double) + 2 * (size_t)RL;
  double* wbase = smem + (size_t)wid * wave_doubles;
  WaveBuf* B = reinterpret_cast<WaveBuf*>(wbase);
  double* rows = wbase + (2 * sizeof(WaveBuf)) / sizeof(double);
  const uint32_t nw = gridDim.x * waves_per_block;
  uint32_t next_ticket = blockIdx.x * waves_per_block + wid;

  // wave-uniform ticket state of the two rows
  int tk0 = -1, tk1 = -1;
  int nx0 = 0, en0 = 0, nx1 = 0, en1 = 0;
  int cur = 0;

  // lane state
  bool active = false;
  int buf = 0;
  uint32_t p = 0, kn = 0, inst = 0, j = 0;
  R x = 0, y = 0, Y = 0, Z = 0, Xi = 0;
  R ehx = 0, ehy = 0, elx = 0, ely = 0;
  int abuf = -1;
  double acc_b = 0, acc_s = 0, acc_s2 = 0;
  uint32_t acc_k = 0, acc_en = 0, acc_ws = 0;   // side counts packed 16 + 16 bits

  auto spill = [&](int b) {
    double* ex = rows + (size_t)b * RL + 4 * SL;
    lds_add(ex + EX_B, acc_b);
    lds_add(ex + EX_S, acc_s);
    lds_add(ex + EX_S2, acc_s2);
    lds_add(ex + EX_K, (double)acc_k);
    lds_add(ex + EX_E, (double)(acc_en & 0xFFFFu));
    lds_add(ex + EX_N, (double)(acc_en >> 16));
    lds_add(ex + EX_W, (double)(acc_ws & 0xFFFFu));
    lds_add(ex + EX_S_SIDE, (double)(acc_ws >> 16));
    acc_b = acc_s = acc_s2 = 0.0;
    acc_k = acc_en = acc_ws = 0;
  };

  auto acquire = [&](int b) {
    const uint32_t t = next_ticket;
    next_ticket += nw;
    const Ticket T = P.tickets[t];
    WaveBuf& W = B[b];
    const double* src = reinterpret_cast<const double*>(P.desc + T.knot);
    if (lane < (int)(sizeof(KnotDesc) / sizeof(double)))
      reinterpret_cast<double*>(&W.d)[lane] = src[lane];
    if (lane == 0) { W.ticket = (int32_t)t; W.p0 = T.p0; W.p1 = T.p1; W.inst = T.inst; }
    double* row = rows + (size_t)b * RL;
    for (int i = lane; i < RL; i += 64) row[i] = 0.0;
    wave_sync();
    if (lane < 4) W.ebox[lane] = (double)exit_threshold<KIND, R>(P, W.d, lane);
    wave_sync();
    if (b) { tk1 = (int)t; nx1 = T.p0; en1 = T.p1; } else { tk0 = (int)t; nx0 = T.p0; en0 = T.p1; }
  };

  auto flush = [&](int b) {
    if (abuf == b) { spill(b); abuf = -1; }
    wave_sync();
    const int t = b ? tk1 : tk0;
    const double* row = rows + (size_t)b * RL;
    double* dst = P.partial + (size_t)t * RL;
    for (int i = lane; i < RL; i += 64) dst[i] = row[i];
    wave_sync();
    if (b) tk1 = -1; else tk0 = -1;
  };

  while (true) {
    // ---- refill idle lanes -------------------------------------------------
    while (true) {
      const uint64_t idle = __ballot(!active);
      if (idle == 0) break;
      const int nx = cur ? nx1 : nx0, en = cur ? en1 : en0;
      if (nx >= en) {
        const int old = cur ^ 1;
        int tgt = -1;
        if ((old ? tk1 : tk0) < 0) tgt = old;
        else if ((cur ? tk1 : tk0) < 0) tgt = cur;
        if (tgt < 0 || next_ticket >= (uint32_t)P.n_tickets) break;
        acquire(tgt);
        cur = tgt;
        continue;
      }
      const int take = min(__popcll(idle), en - nx);
      const int rank = lane_rank(idle);
      if (!active && rank < take) {
        if (abuf >= 0 && abuf != cur) spill(abuf);
        abuf = cur;
        const WaveBuf& W = B[cur];
        p = (uint32_t)(nx + rank);
        kn = (uint32_t)W.d.knot;
        inst = W.inst;
        j = 0;
        x = (R)W.d.sx; y = (R)W.d.sy;
        Y = (R)1; Z = (R)0; Xi = (R)0;
        ehx = (R)W.ebox[0]; ehy = (R)W.ebox[1]; elx = (R)W.ebox[2]; ely = (R)W.ebox[3];
        active = true;
        buf = cur;
      }
      if (cur) nx1 = nx + take; else nx0 = nx + take;
    }
    if (__ballot(active) == 0) break;

    // ---- one Philox draw, up to two Euler steps -------------------------------
    bool ex = false;
    bool forced = false;
    uint32_t K = 0;
    if (active) {
      const U4 r = philox10(j, p, kn, inst, P.key0, P.key1);
      R z0, z1;
      if constexpr (F64) box_muller(uniform64(r.a), uniform64(r.b), z0, z1);
      else box_muller(uniform32(r.a), uniform32(r.b), z0, z1);
      em_step<KIND, R>(P, z0, z1, x, y, Y, Z);
      K = 2 * j + 1;
      ex = (x > ehx) | (y > ehy) | (x < elx) | (y < ely);
      if (!ex) {
        if constexpr (F64) box_muller(uniform64(r.c), uniform64(r.d), z0, z1);
        else box_muller(uniform32(r.c), uniform32(r.d), z0, z1);
        em_step<KIND, R>(P, z0, z1, x, y, Y, Z);
        K = 2 * j + 2;
        ex = (x > ehx) | (y > ehy) | (x < elx) | (y < ely);
      }
      ++j;
      if (!ex && 2 * j >= P.max_steps) { ex = true; forced = true; }
    }

    // ---- exits: side, projection, interpolation, tallies -----------------------
    if (__ballot(ex) != 0 && ex) {
      const WaveBuf& W = B[buf];
      const KnotDesc& d = W.d;
      bool fE = x > ehx, fN = y > ehy, fW = x < elx, fS = y < ely;
      if (forced) fE = fN = fW = fS = true;
      const R lE = (R)d.line[0], lN = (R)d.line[1], lW = (R)d.line[2], lS = (R)d.line[3];
      int o = -1;
      R best = 0;
      if (fE) { o = 0; best = fabs(x - lE); }
      if (fN) { const R v = fabs(y - lN); if (o < 0 || v < best) { o = 1; best = v; } }
      if (fW) { const R v = fabs(x - lW); if (o < 0 || v < best) { o = 2; best = v; } }
      if (fS) { const R v = fabs(y - lS); if (o < 0 || v < best) { o = 3; best = v; } }
      const bool vert = (o == 0 || o == 2);
      const R along = vert ? y : x;
      const R lpos = (R)d.line[o];
      R bp, uref = 0, trec;
      if ((d.bmask >> o) & 1) {
        const R a0 = vert ? (R)P.y0 : (R)P.x0, a1 = vert ? (R)P.y1 : (R)P.x1;
        const R pa = fmin(fmax(along, a0), a1);
        const R gv = vert ? g_at<KIND>(lpos, pa) : g_at<KIND>(pa, lpos);
        {
#pragma clang fp contract(off)
          bp = Z + Xi + Y * gv;
        }
        trec = pa;
      } else {
        const R a0 = vert ? (R)P.y0 : (R)P.x0;
        const R da = vert ? (R)P.dy : (R)P.dx;
        const int clo = d.clo[o], chi = d.chi[o];
        R t;
        if constexpr (F64) {
          t = (along - a0) / da;
        } else {
          t = (along - a0) * ((R)1 / da);
        }
        t = fmin(fmax(t, (R)clo), (R)chi);
        const R i0 = fmin(floor(t), (R)(chi - 1));
        const R w = t - i0;
        const int q0 = (int)i0;
        trec = t;
        bp = Z + Xi;
        double* row = rows + (size_t)buf * RL + o * SL;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int q = q0 + e;
          R c;
          {
#pragma clang fp contract(off)
            c = Y * (e == 0 ? (R)1 - w : w);
          }
          if (q == 0 || q == P.L) {
            const R qc = vert ? (R)P.y0 + (R)q * (R)P.dy : (R)P.x0 + (R)q * (R)P.dx;
            const R gv = vert ? g_at<KIND>(lpos, qc) : g_at<KIND>(qc, lpos);
            {
#pragma clang fp contract(off)
              bp = bp + c * gv;
            }
          } else {
            lds_add(row + (q - clo), (double)c);
            if (P.u_ref) {
              const int at = d.at[o];
              const int lx = vert ? at : q, ly = vert ? q : at;
              const int col = P.lattice[(size_t)ly * (P.L + 1) + lx];
              {
#pragma clang fp contract(off)
                uref = uref + c * (R)P.u_ref[col];
              }
            }
          }
        }
      }
      const double s = (double)bp + (double)uref;
      acc_b += (double)bp;
      acc_s += s;
      acc_s2 += s * s;
      acc_k += K;
      if (o == 0) acc_en += 1u;
      else if (o == 1) acc_en += 1u << 16;
      else if (o == 2) acc_ws += 1u;
      else acc_ws += 1u << 16;
      if (P.dump && (int)p < P.dump_paths) {
        double* rec = P.dump + ((size_t)kn * P.dump_paths + p) * PDD_DUMP_WIDTH;
        rec[0] = (double)K; rec[1] = (double)x; rec[2] = (double)y; rec[3] = (double)Y;
        rec[4] = (double)Z; rec[5] = (double)Xi; rec[6] = (double)o; rec[7] = (double)trec;
      }
      active = false;
      // 16-bit side counters: spill before they can wrap
      if (((acc_en | acc_ws) & 0x80008000u) != 0) spill(buf);
    }

    // ---- flush rows whose ticket is handed out and drained ---------------------
    if (tk0 >= 0 && nx0 >= en0 && __ballot(active && buf == 0) == 0) flush(0);
    if (tk1 >= 0 && nx1 >= en1 && __ballot(active && buf == 1) == 0) flush(1);
  }
}

// Sum a knot's partial rows (ticket order, then side order) into its CSR row,
// b entry and diagnostics.  One wave per knot.
__global__ __launch_bounds__(256) void k_finalize(FinalizeParams F) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (k >= F.n) return;
  const KnotDesc d = F.desc[k];
  const int tb = F.ticket_begin[k], te = F.ticket_begin[k + 1];
  const double N = (double)F.n_paths[k];
  const int RL = F.row_len, SL = F.slot_len;
  for (int pos = F.row_ptr[k] + lane; pos < F.row_ptr[k + 1]; pos += 64) {
    const int col = F.col_idx[pos];
    if (col == (int)k) { F.val[pos] = 1.0; continue; }
    const int cx = F.knot_ij[2 * col], cy = F.knot_ij[2 * col + 1];
    double s = 0.0;
    for (int o = 0; o < 4; ++o) {
      if ((d.bmask >> o) & 1) continue;
      const bool vert = (o == 0 || o == 2);
      const int on = vert ? cx : cy, q = vert ? cy : cx;
      if (on != d.at[o] || q < d.clo[o] || q > d.chi[o]) continue;
      const int slot = o * SL + (q - d.clo[o]);
      double so = 0.0;
      for (int t = tb; t < te; ++t) so += F.partial[(size_t)t * RL + slot];
      s += so;
    }
    F.val[pos] = -s / N;
  }
  if (lane < EX_COUNT) {
    double e = 0.0;
    for (int t = tb; t < te; ++t) e += F.partial[(size_t)t * RL + 4 * SL + lane];
    if (lane == EX_B) F.b[k] = e / N;
    if (F.diag) {
      // diag layout: sum K, N, exits E, N, W, S, sum s, sum s^2
      int where = -1;
      switch (lane) {
        case EX_S: where = 6; break;
        case EX_S2: where = 7; break;
        case EX_K: where = 0; break;
        case EX_E: where = 2; break;
        case EX_N: where = 3; break;
        case EX_W: where = 4; break;
        case EX_S_SIDE: where = 5; break;
        default: break;
      }
      if (where >= 0) F.diag[k * PDD_DIAG_WIDTH + where] = e;
      if (lane == 0) F.diag[k * PDD_DIAG_WIDTH + 1] = N;
    }
  }
}

template <int KIND, bool F64>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&k_assemble<KIND, F64>);
}

template <bool F64>
const void* pick(int kind) {
  switch (kind) {
    case PDD_COEF_POISSON: return kernel_ptr<PDD_COEF_POISSON, F64>();
    case PDD_COEF_VARCOEF: return kernel_ptr<PDD_COEF_VARCOEF, F64>();
    case PDD_COEF_AMPLITUDE: return kernel_ptr<PDD_COEF_AMPLITUDE, F64>();
    case PDD_COEF_LUT: return kernel_ptr<PDD_COEF_LUT, F64>();
    case PDD_COEF_CONSTSOL: return kernel_ptr<PDD_COEF_CONSTSOL, F64>();
    case PDD_COEF_EXITTIME: return kernel_ptr<PDD_COEF_EXITTIME, F64>();
    default: return nullptr;
  }
}

const void* assemble_kernel(int precision, int kind) {
  return precision == PDD_FP64_SAME_STREAM ? pick<true>(kind) : pick<false>(kind);
}

}  // namespace

size_t assemble_lds_bytes(int row_len, int block) {
  const size_t waves = (size_t)block / 64;
  return waves * (2 * sizeof(WaveBuf) + 2 * (size_t)row_len * sizeof(double));
}

hipError_t assemble_occupancy(int precision, int kind, int block, size_t lds_bytes, int* blocks_per_cu) {
  const void* f = assemble_kernel(precision, kind);
  if (!f) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, block, lds_bytes);
}

hipError_t launch_assemble(const AsmParams& p, int precision, int grid, int block, size_t lds_bytes,
                           hipStream_t stream) {
  const void* f = assemble_kernel(precision, p.coef.kind);
  if (!f) return hipErrorInvalidValue;
  AsmParams arg = p;
  void* args[] = {&arg};
  return hipLaunchKernel(f, dim3(grid), dim3(block), args, lds_bytes, stream);
}

hipError_t launch_finalize(const FinalizeParams& p, hipStream_t stream) {
  const int block = 256;
  const int64_t grid = (p.n + 3) / 4;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)grid), dim3(block), 0, stream, p);
  return hipGetLastError();
}

}  // namespace pdd
