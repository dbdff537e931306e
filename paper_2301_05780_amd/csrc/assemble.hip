// Persistent lane-per-path Monte Carlo assembly of the PDDSparse rows
// (eqs. 9 and 20-25) for gfx950.
//
// Work decomposition.  The host cuts every knot's N_k paths into tickets
// (knot, path range).  Each wave of the persistent grid takes tickets in a
// fixed stride (wave w: tickets w, w + W, w + 2W, ...; or from a device
// counter) and holds up to two LDS tally rows, taken from a pool shared by
// the waves of its workgroup (two per wave unless the launch asks for fewer,
// which trades waiting for occupancy).  Every lane integrates one path at a
// time; when its path exits, the lane is refilled with the next path of the
// wave's current ticket, ranked among the idle lanes by a ballot (no
// atomics), at once or, with a refill threshold, once enough lanes are idle.
// When the current ticket has handed out all its paths, the next ticket opens
// in the other row while the stragglers of the previous one drain, so lanes
// wait for the slowest path of a ticket only when a whole ticket is handed
// out before its predecessor drains.  A drained row is written once to the ticket's
// partial row in HBM; a second kernel sums a knot's partial rows in ticket
// order into the CSR values and b (deterministic for a fixed launch shape).
//
// Hot loop.  One Philox draw feeds two Euler steps; every path starts at an
// even step, so all lanes of a wave draw together and the generator is never
// divergent.  An exiting lane only appends its exit state (X_K, Y_K,
// Z_K + Xi_K, K) to a per-wave LDS queue and is refilled; the exit work (side
// choice, projection, hat weights, tallies) runs over 64 queued exits at a
// time with every lane busy, instead of in a branch with a handful of lanes
// active.
//
// Tallies: G slots, b, the score moments and the step count are float64 LDS
// atomics; exit-side counts are ballot popcounts added by one lane.
#include <type_traits>

#include "device_common.h"
#include "net_grad.h"

namespace pdd {

namespace {

constexpr int QCAP = 128;          // exit records per wave (processed at >= 64)
constexpr uint32_t MAX_STEPS = (1u << 24) - 2;

// Per-buffer header: the ticket's knot, the instance parameters (batched
// launches only), the strict exit thresholds x > e[0], y > e[1], x < e[2],
// y < e[3] in the path precision, the values a refilled lane starts from
// (start point, step, its square root, family parameter; path precision),
// the pool row holding the buffer's tallies and the instance word.  Refill
// reads the header from LDS rather than keeping copies in scalar registers.
template <typename R, bool BATCH>
struct WaveBuf {
  KnotDesc d;
  R ebox[4];
  R start[8];          // sx, sy, h, sqrt h, a
  int32_t row, pad0, pad1;
  uint32_t inst;
};
template <typename R>
struct WaveBuf<R, true> {
  KnotDesc d;
  InstDesc I;
  R ebox[4];
  R start[8];
  int32_t row, pad0, pad1;
  uint32_t inst;
};
static_assert(sizeof(WaveBuf<float, false>) % 16 == 0 && sizeof(WaveBuf<double, false>) % 16 == 0 &&
                  sizeof(WaveBuf<float, true>) % 16 == 0 && sizeof(WaveBuf<double, true>) % 16 == 0,
              "WaveBuf alignment");

template <typename R>
struct ExitRec {
  R x, y, Y, bp;       // exit iterate, Y_K, Z_K + Xi_K
};

// block-level LDS for the control-variate network (staged once per workgroup)
template <bool F64, int CV>
constexpr size_t net_lds_bytes() {
  if constexpr (CV != PDD_CV_NETWORK) return 0;
  else if constexpr (F64) return ((MLP_PARAMS * sizeof(float) + 15) / 16) * 16;
  else return ((sizeof(NetLds) + 15) / 16) * 16;
}

// Per-wave LDS of the cooperative table read (float32 LUT kernels): each
// lane's cell and weights, and the 8 interpolated fields of each lane.
struct CoopLds {
  uint32_t cell[64];
  float tx[64], ty[64];
  float res[64 * 8];
};
static_assert(sizeof(CoopLds) % 16 == 0, "CoopLds alignment");

// The table block of a wave's LDS: none, the cooperative-read block, or the
// eight constant-field values of the lane-per-path kernel.
enum { TB_NONE = 0, TB_COOP = 1, TB_LANE = 2 };
template <int TB>
constexpr size_t table_block_bytes() {
  return TB == TB_COOP ? sizeof(CoopLds) : (TB == TB_LANE ? 8 * sizeof(float) : 0);
}

// per-wave LDS bytes: two row headers, the exit queue (records + meta words)
// and the table block; the tally rows follow all waves' blocks as the
// workgroup's pool (a 16-byte free mask, then the rows)
template <typename R, int TB, bool BATCH>
constexpr size_t wave_lds_bytes() {
  return 2 * sizeof(WaveBuf<R, BATCH>) + QCAP * sizeof(ExitRec<R>) + QCAP * sizeof(uint32_t) + table_block_bytes<TB>();
}
constexpr size_t POOL_HEAD = 16;

__device__ __forceinline__ int lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// One DPP step of a float64 wave reduction: each lane adds the value of
// the lane the control selects (0 where the source lies outside the row or
// the row is masked off).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, true);
  return v + __hiloint2double(hi, lo);
}

// Sum of v over each row of 16 lanes, left in the row's last lane (lanes 15,
// 31, 47, 63): shifts by 1, 2, 4 and 8 within the row.  A fixed order.
__device__ __forceinline__ double row_total_dpp(double v) {
  v = dpp_add_f64<0x111, 0xf>(v);    // row_shr:1
  v = dpp_add_f64<0x112, 0xf>(v);    // row_shr:2
  v = dpp_add_f64<0x114, 0xf>(v);    // row_shr:4
  v = dpp_add_f64<0x118, 0xf>(v);    // row_shr:8
  return v;
}

// Sum of v over the 64 lanes, returned to every lane: shifts by 1, 2, 4
// and 8 within each row of 16 lanes leave the row's sum in its lane 15; the
// row broadcasts of lanes 15 and 31 then carry the four row sums into lane
// 63, which is read out.  A fixed order, no LDS traffic.
__device__ __forceinline__ double wave_total_dpp(double v) {
  v = dpp_add_f64<0x111, 0xf>(v);    // row_shr:1
  v = dpp_add_f64<0x112, 0xf>(v);    // row_shr:2
  v = dpp_add_f64<0x114, 0xf>(v);    // row_shr:4
  v = dpp_add_f64<0x118, 0xf>(v);    // row_shr:8
  v = dpp_add_f64<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
  v = dpp_add_f64<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
  return readlane_f64(v, 63);
}

__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ uint32_t to_uniform_u(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Bilinear coefficients of the whole wave's points from the cell-major table.
// A lookup needs 112 bytes of one 128-byte cell; with one lane per path, a
// wave's eight 16-byte loads would each touch 64 scattered lines.  Instead,
// round r has the 8 lanes of group g load the 8 float4 of the cell of path
// 8 r + g (one line per group, eight lines per instruction) and interpolate
// one field each; the fields go back to their path's lane through LDS.  The
// interpolation is the per-lane read's (same cell, weights and formula).
__device__ __forceinline__ void lut_fetch_coop(const CoefParams& cp, float x, float y, CoopLds* C, int lane,
                                               Coef<float>& o) {
  const int n = cp.lut_n;
  float fx = (x - cp.x0f) * cp.lut_sx;
  float fy = (y - cp.y0f) * cp.lut_sy;
  fx = clamp_node(fx, (float)(n - 1));
  fy = clamp_node(fy, (float)(n - 1));
  const int i = min((int)fx, n - 2);
  const int j = min((int)fy, n - 2);
  wave_sync();
  C->cell[lane] = __umul24((uint32_t)j, (uint32_t)(n - 1)) + (uint32_t)i;     // j, n - 1 < 2^24
  C->tx[lane] = fx - (float)i;
  C->ty[lane] = fy - (float)j;
  wave_sync();
  const int q = lane & 7, g = lane >> 3;
  // 32-bit byte offsets from the table's base (the host keeps (n-1)^2 cells
  // of 128 B below 4 GiB), so each load takes the base from scalar registers
  const char* cb = reinterpret_cast<const char*>(cp.cells);
  float4 v[8];                                // all eight loads in flight
#pragma unroll
  for (int r = 0; r < 8; ++r)
    v[r] = *reinterpret_cast<const float4*>(cb + (C->cell[8 * r + g] * 128u + (uint32_t)q * 16u));
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int pth = 8 * r + g;
    const float tx = C->tx[pth], ty = C->ty[pth];
    // the cell holds the field's bilinear form (a, b, c, d): a + tx b + ty (c + tx d)
    C->res[pth * 8 + q] = __builtin_fmaf(ty, __builtin_fmaf(tx, v[r].w, v[r].z), __builtin_fmaf(tx, v[r].y, v[r].x));
  }
  wave_sync();
  const float4 a = reinterpret_cast<const float4*>(C->res)[2 * lane];
  const float4 b = reinterpret_cast<const float4*>(C->res)[2 * lane + 1];
  o.sxx = a.x; o.sxy = a.y; o.syy = a.z; o.dx = a.w;
  o.dy = b.x; o.c = b.y; o.f = b.z;
}

// Bilinear coefficients from the lane-read layout, one lane per path: the
// stored forms at the lane's own cell, the other fields constant.  Cell,
// weights and formula are the cooperative read's, and a constant field's
// form (v, 0, 0, 0) evaluates to v + 0 there, the value kept for it, so both
// reads give the same bits.
__device__ __forceinline__ void lut_fetch_lane(const CoefParams& cp, uint32_t lay, const float* kc_lds, float x, float y,
                                               Coef<float>& o) {
  // the layout word (see CoefParams::lut_info), decoded at every call: the
  // empty asm keeps the decoded fields and the field masks from being
  // hoisted out of the path loop, where they would only occupy registers
  __asm__ volatile("" : "+s"(lay));
  const int k1 = (int)(lay & 15u), k2 = (int)((lay >> 4) & 15u);
  const uint32_t stride = ((lay >> 8) & 15u) == 2u ? 32u : 16u;
  const int n = cp.lut_n;
  float fx = (x - cp.x0f) * cp.lut_sx;
  float fy = (y - cp.y0f) * cp.lut_sy;
  fx = clamp_node(fx, (float)(n - 1));
  fy = clamp_node(fy, (float)(n - 1));
  const int i = min((int)fx, n - 2);
  const int j = min((int)fy, n - 2);
  const float tx = fx - (float)i, ty = fy - (float)j;
  const uint32_t off = (__umul24((uint32_t)j, (uint32_t)(n - 1)) + (uint32_t)i) * stride;   // j, n - 1 < 2^24
  const char* cb = reinterpret_cast<const char*>(cp.cells);
  const float4 a = *reinterpret_cast<const float4*>(cb + off);
  float v2 = 0.0f;
  if (k2 < 7) {
    const float4 b = *reinterpret_cast<const float4*>(cb + (off + 16u));
    v2 = __builtin_fmaf(ty, __builtin_fmaf(tx, b.w, b.z), __builtin_fmaf(tx, b.y, b.x));
  }
  const float v1 = __builtin_fmaf(ty, __builtin_fmaf(tx, a.w, a.z), __builtin_fmaf(tx, a.y, a.x));
  // the constant fields' values, kept in the wave's LDS; the second stored
  // field's selects only when there is one (a uniform branch)
  typedef float v4f __attribute__((ext_vector_type(4)));
  const v4f c0 = reinterpret_cast<const v4f*>(kc_lds)[0];
  const v4f c1 = reinterpret_cast<const v4f*>(kc_lds)[1];
  __asm__("" ::"v"(c0), "v"(c1));      // two whole 16-byte LDS reads at immediate offsets
  if (k1 == 6 && k2 >= 7) {
    // only the source term varies (a uniform branch without the selects)
    o.sxx = c0.x; o.sxy = c0.y; o.syy = c0.z; o.dx = c0.w;
    o.dy = c1.x; o.c = c1.y; o.f = v1;
    return;
  }
  float f[7] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z};
#pragma unroll
  for (int q = 0; q < 7; ++q) f[q] = q == k1 ? v1 : f[q];
  if (k2 < 7) {
#pragma unroll
    for (int q = 0; q < 7; ++q) f[q] = q == k2 ? v2 : f[q];
  }
  o.sxx = f[0]; o.sxy = f[1]; o.syy = f[2]; o.dx = f[3];
  o.dy = f[4]; o.c = f[5]; o.f = f[6];
}

// The full layout (all seven forms of the cell) read by one lane per path:
// the lane-per-path kernel's fallback when the layout word says the copy is
// full, the same cell, weights and formula as the cooperative read.
__device__ __forceinline__ void lut_fetch_cell(const CoefParams& cp, float x, float y, Coef<float>& o) {
  const int n = cp.lut_n;
  float fx = (x - cp.x0f) * cp.lut_sx;
  float fy = (y - cp.y0f) * cp.lut_sy;
  fx = clamp_node(fx, (float)(n - 1));
  fy = clamp_node(fy, (float)(n - 1));
  const int i = min((int)fx, n - 2);
  const int j = min((int)fy, n - 2);
  const float tx = fx - (float)i, ty = fy - (float)j;
  const char* cb = reinterpret_cast<const char*>(cp.cells) + (__umul24((uint32_t)j, (uint32_t)(n - 1)) + (uint32_t)i) * 128u;
  float v[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const float4 a = reinterpret_cast<const float4*>(cb)[q];
    v[q] = __builtin_fmaf(ty, __builtin_fmaf(tx, a.w, a.z), __builtin_fmaf(tx, a.y, a.x));
  }
  o.sxx = v[0]; o.sxy = v[1]; o.syy = v[2]; o.dx = v[3];
  o.dy = v[4]; o.c = v[5]; o.f = v[6];
}

// Exact Gobet-Menozzi threshold of side o for a table whose sigma fields are
// constant (scan word bits 0-2 clear; the values at lut_info[8..10]): a_nn is
// then the same at every projection, so the threshold is fixed per knot as
// for the closed-form families, and the exact test at the projection that
// the general table needs would decide every point the same way (its
// bilinear reads of a constant field give the constant, and its arithmetic
// is this one).
template <typename R>
__device__ __forceinline__ R lut_const_threshold(const uint32_t* info, double sqrt_h, const KnotDesc& d, int o) {
  const double line = d.line[o];
  const bool vert = (o == 0 || o == 2);
  const R sxx = (R)__uint_as_float(info[8]), sxy = (R)__uint_as_float(info[9]), syy = (R)__uint_as_float(info[10]);
  R thr;
  {
#pragma clang fp contract(off)
    const R ann = vert ? (sxx * sxx + sxy * sxy) : (sxy * sxy + syy * syy);
    const R delta = (R)kGM * sqrt(ann) * (R)sqrt_h;
    thr = (o < 2) ? (R)line - delta : (R)line + delta;
  }
  return (o < 2) ? nextafter(thr, (R)-INFINITY) : nextafter(thr, (R)INFINITY);
}

// Geometry used when resolving exits (the launch's, or a batched instance's).
template <typename R>
struct GeoView {
  R x0, x1, y0, y1;
  double dx, dy;
  float inv_dx, inv_dy;
  int L;
};

template <int KIND, bool F64, int CV, bool BATCH, bool RBF = false, bool HK = false, bool LANEK = false>
__device__ __forceinline__ void assemble_body(const AsmParams& P) {
  using R = typename std::conditional<F64, double, float>::type;
  constexpr bool CVON = CV != PDD_CV_NONE;
  // float32 table reads go through the cooperative read (except beside the
  // network, whose registers leave no room for it), or, in the lane-per-path
  // kernel (LANEK), through the per-lane read of the varying fields; the
  // cooperative read and the network gradient are wave-wide operations,
  // evaluated with every lane before each half step, and the lane kernel
  // keeps the same loop
  static_assert(!LANEK || (KIND == PDD_COEF_LUT && !F64 && CV != PDD_CV_NETWORK && !BATCH), "lane kernel");
  constexpr bool LANE = LANEK;
  constexpr bool COOP = KIND == PDD_COEF_LUT && !F64 && CV != PDD_CV_NETWORK && !LANE;
  constexpr bool WAVEWIDE = !F64 && (CV == PDD_CV_NETWORK || COOP || LANE);
  constexpr int TB = COOP ? TB_COOP : (LANE ? TB_LANE : TB_NONE);
  // row extras (sum b, sum s^2, sum K): per-lane float64 sums flushed once
  // per ticket (LACC), or summed per 16-lane row before the LDS atomics
  // (ROWRED), or one atomic per exit (see process_queue)
  constexpr bool LACC = (LANE && CV == PDD_CV_NONE) || BATCH;
  constexpr bool ROWRED = !LACC && KIND == PDD_COEF_LUT;
  extern __shared__ double smem[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int waves_per_block = blockDim.x >> 6;
  const int RL = P.row_len, SL = P.slot_len;
  unsigned char* lds0 = reinterpret_cast<unsigned char*>(smem);
  NetLds* NL = reinterpret_cast<NetLds*>(lds0);            // network, CV == NETWORK (float32)
  float* TH = reinterpret_cast<float*>(lds0);              // network, CV == NETWORK (float64 mode)
  if constexpr (CV == PDD_CV_NETWORK) {
    if constexpr (F64) {
      for (int i = threadIdx.x; i < MLP_PARAMS; i += blockDim.x) TH[i] = P.cv_params[i];
    } else {
      net_stage(NL, P.cv_params);
    }
    __syncthreads();
  }
  using WB = WaveBuf<R, BATCH>;
  unsigned char* gbase = lds0 + net_lds_bytes<F64, CV>();
  unsigned char* wbase = gbase + (size_t)wid * wave_lds_bytes<R, TB, BATCH>();
  WB* B = reinterpret_cast<WB*>(wbase);
  ExitRec<R>* Q = reinterpret_cast<ExitRec<R>*>(wbase + 2 * sizeof(WB));
  uint32_t* Qm = reinterpret_cast<uint32_t*>(wbase + 2 * sizeof(WB) + QCAP * sizeof(ExitRec<R>));
  CoopLds* CW = reinterpret_cast<CoopLds*>(wbase + wave_lds_bytes<R, TB_NONE, BATCH>());   // COOP only
  float* KCW = reinterpret_cast<float*>(wbase + wave_lds_bytes<R, TB_NONE, BATCH>());       // LANE only
  // the workgroup's pool of tally rows and its free mask (bit r: row r free)
  unsigned char* pbase = gbase + (size_t)waves_per_block * wave_lds_bytes<R, TB, BATCH>();
  uint32_t* pool = reinterpret_cast<uint32_t*>(pbase);
  double* rows = reinterpret_cast<double*>(pbase + POOL_HEAD);
  // Batched launches and the table family share the rows through the pool;
  // elsewhere wave w keeps rows 2w and 2w + 1 (no mask, no extra registers)
  constexpr bool POOL = BATCH || KIND == PDD_COEF_LUT;
  if constexpr (POOL) {
    const int n_rows = P.pool_rows > 0 ? P.pool_rows : 2 * waves_per_block;
    if (threadIdx.x == 0) *pool = n_rows >= 32 ? ~0u : (1u << n_rows) - 1u;
    __syncthreads();
  }
  // the row of buffer b (header W), counted from `wrows`: the pool's first
  // row, or this wave's own first row
  double* wrows = POOL ? rows : rows + (size_t)2 * wid * RL;
  auto row_of = [&](int b, const WaveBuf<R, BATCH>& W) __attribute__((always_inline)) -> int {
    if constexpr (POOL) return W.row;
    else return b;
  };
  // offset of that row in the LDS rows (pool rows < 64 and RL < 2^16: 24-bit multiply)
  auto row_off = [&](int b, const WaveBuf<R, BATCH>& W) __attribute__((always_inline)) -> uint32_t {
    return __umul24((uint32_t)row_of(b, W), (uint32_t)RL);
  };
  // a free row of the pool (wave-uniform), or -1 when every row is taken
  auto pool_take = [&]() __attribute__((always_inline)) -> int {
    int r = -1;
    if (lane == 0) {
      uint32_t m = atomicOr(pool, 0u);
      while (m != 0u) {                 // each pass takes a row or drops a taken bit from m
        const int b = __builtin_ctz(m);
        const uint32_t old = atomicAnd(pool, ~(1u << b));
        if (old & (1u << b)) { r = b; break; }
        m = old & ~(1u << b);
      }
    }
    return __builtin_amdgcn_readfirstlane(r);
  };
  // next ticket this wave takes: fixed stride over the whole order (static
  // schedule, reproducible sums), fixed stride over its XCD's share of the
  // order (static, spatially ordered tickets: the workgroups of one XCD, which
  // share an L2, work on neighbouring knots), or claimed from a device counter
  // (dynamic schedule, balanced)
  uint32_t t_stride = gridDim.x * waves_per_block, t_end = (uint32_t)P.n_tickets, t_base = 0;
  uint32_t next_ticket = blockIdx.x * waves_per_block + wid;
  uint32_t* counter = P.ticket_counter;
  if (P.xcd_begin) {
    const uint32_t x = blockIdx.x & 7u;
    const uint32_t blocks_x = (gridDim.x - x + 7u) >> 3;
    t_stride = blocks_x * waves_per_block;
    t_base = (uint32_t)P.xcd_begin[x];
    next_ticket = t_base + (blockIdx.x >> 3) * waves_per_block + wid;
    t_end = (uint32_t)P.xcd_begin[x + 1];
    if (counter) counter += x;        // dynamic: one counter per XCD share
  }
  auto claim = [&](uint32_t prev) __attribute__((always_inline)) -> uint32_t {
    if (counter) {
      uint32_t v = 0;
      if (lane == 0) v = atomicAdd(counter, 1u);
      return t_base + (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
    }
    return prev + t_stride;
  };
  if (P.ticket_counter) next_ticket = claim(0);

  // wave-uniform ticket state of the two buffers
  int tk0 = -1, tk1 = -1;
  int nx0 = 0, en0 = 0, nx1 = 0, en1 = 0;
  int cur = 0;
  int qn = 0;                    // queued exit records
  // LACC: this lane's sums of b, s^2 and K over the exits it processed, per buffer
  double ab0 = 0.0, aq0 = 0.0, ak0 = 0.0, ab1 = 0.0, aq1 = 0.0, ak1 = 0.0;

  // lane state
  bool active = false;
  int buf = 0;
  uint32_t p = 0, kn = 0, inst = 0, j = 0;
  R x = 0, y = 0, Y = 0, Z = 0, Xi = 0;
  R ehx = 0, ehy = 0, elx = 0, ely = 0;
  R lh = (R)P.h, lsq = (R)P.sqrt_h, la = (R)P.coef.a;   // per lane in batched launches
  // network control variate: unit coordinates of the domain (x - x0) / (x1 - x0)
  const R ux0 = (R)P.x0, uy0 = (R)P.y0;
  const R usx = (R)(1.0 / (P.x1 - P.x0)), usy = (R)(1.0 / (P.y1 - P.y0));
  // float32 table: the layout of its cell copy; for the lane-per-path read,
  // the constant fields go to the wave's LDS (the cooperative block, unused
  // then, or the lane kernel's own)
  uint32_t lut_lay = 0u;
  float* KC = COOP ? CW->res : KCW;
  // GM exits on a table with constant sigma: exact thresholds, no refinement
  // (kept as bit 16 of lut_lay, a bit the layout word leaves clear)
  constexpr uint32_t SIG_EXACT = 1u << 16;
  if constexpr (COOP || LANE) {
    lut_lay = to_uniform_u(P.coef.lut_info[1]);
    if (P.exit_rule == PDD_EXIT_GM && (to_uniform_u(P.coef.lut_info[0]) & 7u) == 0u) lut_lay |= SIG_EXACT;
    if (lut_lay & LUT_LANE_READ) {
      if (lane < 8) KC[lane] = __uint_as_float(P.coef.lut_info[8 + lane]);
      wave_sync();
    }
  }

  auto geo = [&](const WB& W) __attribute__((always_inline)) -> GeoView<R> {
    GeoView<R> G;
    if constexpr (BATCH) {
      G.x0 = (R)W.I.x0; G.x1 = (R)W.I.x1; G.y0 = (R)W.I.y0; G.y1 = (R)W.I.y1;
      G.dx = W.I.dx; G.dy = W.I.dy; G.inv_dx = W.I.inv_dx; G.inv_dy = W.I.inv_dy; G.L = W.I.L;
    } else {
      G.x0 = (R)P.x0; G.x1 = (R)P.x1; G.y0 = (R)P.y0; G.y1 = (R)P.y1;
      G.dx = P.dx; G.dy = P.dy; G.inv_dx = P.inv_dx; G.inv_dy = P.inv_dy; G.L = P.L;
    }
    return G;
  };

  // ---- exit test at the new iterate --------------------------------------------
  // The negation of "strictly inside the thresholds", so a NaN iterate exits
  // (and is tallied as NaN) instead of running to the step cap.  For the LUT
  // family under GM the thresholds are candidate ones (unless sigma is
  // constant: then they are exact, and the exit processing flags the sides
  // from them as for the closed-form families): a candidate hit is decided
  // exactly at the projection, and the flagged sides travel with the exit
  // record.
  auto exit_test = [&](uint32_t& fl) __attribute__((always_inline)) -> bool {
    const bool inside = (x <= ehx) & (y <= ehy) & (x >= elx) & (y >= ely);
    if constexpr (KIND == PDD_COEF_LUT) {
      if (!inside && P.exit_rule == PDD_EXIT_GM && !(lut_lay & SIG_EXACT)) {
        const uint32_t cand = (uint32_t)(x > ehx) | ((uint32_t)(y > ehy) << 1) | ((uint32_t)(x < elx) << 2) |
                              ((uint32_t)(y < ely) << 3);
        if (cand == 0) { fl = 0; return true; }
        fl = lut_gm_refine<R>(P.coef, lsq, B[buf].d.line, x, y, cand);
        return fl != 0;
      }
    }
    return !inside;
  };

  // ---- exit processing over the queue (all lanes) ----------------------------
  auto process_queue = [&]() __attribute__((always_inline)) {
    for (int base = 0; base < qn; base += 64) {
      const int i = base + lane;
      const bool valid = i < qn;
      int rb = 0, o = 0;
      double vb = 0.0, vs = 0.0, vk = 0.0;
      int rkey = -1;                 // RBF: 4 buffer + side of an interface exit (-1: none)
      double rtd = 0.0, rY = 0.0;    // RBF: exit point along the line (domain units from its origin), Y
      if (valid) {
        ExitRec<R> r = Q[i];
        const uint32_t meta = Qm[i];
        // an iterate that went NaN (NaN coefficients) poisons its row instead
        // of landing on a clamped side point
        if (isnan(r.x) || isnan(r.y)) { r.Y = (R)NAN; r.bp = (R)NAN; }
        rb = (int)((meta >> 24) & 1u);
        const bool forced = (meta >> 25) & 1u;
        const WB& W = B[rb];
        const KnotDesc& d = W.d;
        const GeoView<R> G = geo(W);
        bool fE, fN, fW, fS;
        if (KIND == PDD_COEF_LUT && P.exit_rule == PDD_EXIT_GM && !(lut_lay & SIG_EXACT)) {
          fE = (meta >> 26) & 1u; fN = (meta >> 27) & 1u; fW = (meta >> 28) & 1u; fS = (meta >> 29) & 1u;
        } else {
          fE = r.x > (R)W.ebox[0]; fN = r.y > (R)W.ebox[1];
          fW = r.x < (R)W.ebox[2]; fS = r.y < (R)W.ebox[3];
        }
        // the step cap, or a NaN iterate (no side flagged): every side is a candidate
        if (forced || !(fE | fN | fW | fS)) fE = fN = fW = fS = true;
        o = choose_side<R>(r.x, r.y, fE, fN, fW, fS, d.line);
        const bool vert = (o == 0 || o == 2);
        const R along = vert ? r.y : r.x;
        const R lpos = (R)d.line[o];
        R bp = r.bp, uref = 0;
        if ((d.bmask >> o) & 1) {
          // boundary side: Y g(P), P the projection clamped to the domain
          const R a0 = vert ? G.y0 : G.x0, a1 = vert ? G.y1 : G.x1;
          const R pa = fmin(fmax(along, a0), a1);
          const R gv = vert ? g_at<KIND>(lpos, pa) : g_at<KIND>(pa, lpos);
          {
#pragma clang fp contract(off)
            bp = bp + r.Y * gv;
          }
        } else if constexpr (RBF) {
          // interface side, RBF: the exit's lattice coordinate on the line,
          // clamped to the stencil; its contributions are summed below, one
          // group of exits sharing a row side at a time
          const double a0 = vert ? (double)G.y0 : (double)G.x0;
          const double da = vert ? G.dy : G.dx;
          const double t = fmin(fmax(((double)along - a0) / da, (double)d.clo[o]), (double)d.chi[o]);
          rtd = t * da;
          rY = (double)r.Y;
          rkey = 4 * rb + o;
        } else {
          // interface side: hat weights on the line lattice, clamped to the stencil range
          const int clo = d.clo[o], chi = d.chi[o];
          int q0;
          R w;
          hat_weights<R, F64>(along, vert ? G.y0 : G.x0, vert ? G.dy : G.dx, vert ? G.inv_dy : G.inv_dx,
                              clo, chi, q0, w);
          double* row = wrows + row_off(rb, W) + __umul24((uint32_t)o, (uint32_t)SL);
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int q = q0 + e;
            R c;
            {
#pragma clang fp contract(off)
              c = r.Y * (e == 0 ? (R)1 - w : w);
            }
            if (q == 0 || q == G.L) {
              const R qc = vert ? G.y0 + (R)q * (R)G.dy : G.x0 + (R)q * (R)G.dx;
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
        vb = (double)bp;
        vs = vb + (double)uref;
        vk = (double)(meta & 0xFFFFFFu);
      }
      if constexpr (RBF) {
        // RBF cardinal interpolation, one group of exits with the same row
        // and side at a time, lanes across the side's stencil points: lane q
        // sums Y phi_c(|z - z_q|) over the group's exits and adds the sum to
        // the row's slot once (the weights Phi^{-1} phi are applied at the
        // row flush).  float64 throughout: the interpolation matrix is
        // ill-conditioned by design.  The stencil's boundary lattice points
        // (q = 0, q = L) take each exit's cardinal weight H_q(z) =
        // (Phi^{-1} phi(z))_q, a sum across the lanes, times g into b.
        constexpr int RU = 2;          // exits per pass of the group loop
        double hb = 0.0;               // this lane's exit: sum over the boundary points q of H_q(z) g(z_q)
        uint64_t todo = __ballot(rkey >= 0);
        while (todo) {
          const int key = __builtin_amdgcn_readlane(rkey, __builtin_ctzll(todo));
          const uint64_t grp = __ballot(rkey == key);
          todo &= ~grp;
          const int gb = key >> 2, go = key & 3;
          const WB& W = B[gb];
          const KnotDesc& d = W.d;
          const GeoView<R> Gg = geo(W);
          const bool vert = (go == 0 || go == 2);
          const int clo = d.clo[go], chi = d.chi[go], S = chi - clo + 1;
          const double da = vert ? Gg.dy : Gg.dx;
          const bool b0 = clo == 0, bL = chi == Gg.L;
          const double* Mi = P.rbf_inv + (vert ? P.rbf_half : 0) + rbf_block_offset(S);
          double* row = wrows + row_off(gb, W) + __umul24((uint32_t)go, (uint32_t)SL);
          // g at the stencil's boundary points (q = 0, q = L)
          const R lpos = (R)d.line[go];
          auto g_end = [&](int q) __attribute__((always_inline)) -> double {
            const R qc = vert ? Gg.y0 + (R)q * (R)Gg.dy : Gg.x0 + (R)q * (R)Gg.dx;
            return (double)(vert ? g_at<KIND>(lpos, qc) : g_at<KIND>(qc, lpos));
          };
          const double g0 = b0 ? g_end(clo) : 0.0, gL = bL ? g_end(chi) : 0.0;
          for (int c0 = 0; c0 < S; c0 += 64) {
            const int si = c0 + lane;
            const bool in = si < S;
            const double qd = (double)(clo + si) * da;     // the stencil point, in domain units from the line's origin
            // rows 0 and S-1 of Phi^{-1} weighted by the boundary data
            double wb = 0.0;
            if (b0 && in) wb = Mi[si] * g0;
            if (bL && in) wb = fma(Mi[(size_t)(S - 1) * S + si], gL, wb);
            double acc = 0.0;
            uint64_t m = grp;
            // two exits per pass (independent chains; a missing one takes
            // Y = 0 and the first one's coordinate), added in exit order
            while (m) {
              int e[RU];
              bool has[RU];
              e[0] = __builtin_ctzll(m);
              has[0] = true;
              m &= m - 1;
#pragma unroll
              for (int u = 1; u < RU; ++u) {
                has[u] = m != 0;
                e[u] = has[u] ? __builtin_ctzll(m) : e[0];
                m &= m - 1;
              }
              double ph[RU];
#pragma unroll
              for (int u = 0; u < RU; ++u) {
                const double rr = readlane_f64(rtd, e[u]) - qd;
                ph[u] = rsqrt_f64(fma(rr, rr, P.rbf_c2));
              }
#pragma unroll
              for (int u = 0; u < RU; ++u) acc = fma(has[u] ? readlane_f64(rY, e[u]) : 0.0, ph[u], acc);
              if (b0 || bL) {
                double t[RU];
#pragma unroll
                for (int u = 0; u < RU; ++u) t[u] = wave_total_dpp(wb * ph[u]);
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                  if (has[u] && lane == e[u]) hb += t[u];
                }
              }
            }
            if (in) lds_add(row + si, acc);
          }
        }
        if (rkey >= 0) {
          // Y times the boundary points' cardinal weights and data, into b
          {
#pragma clang fp contract(off)
            vb = vb + rY * hb;
          }
          vs = vb;
        }
      }
      // row extras b, sum s, sum s^2 and sum K: every exit of a buffer adds
      // to the same four words, and the LDS pipe serialises same-address
      // atomics (up to 64 per word per batch, a cost shared by the CU's
      // waves).  Where paths are short (many exits per step: the table
      // family, batched launches) the plain lane-per-path table kernel and
      // batched launches keep per-lane float64 sums in registers, summed
      // over the wave when the ticket is flushed; the other table kernels
      // (cooperative read, or the control variate's registers) first sum
      // each 16-lane row of the wave (DPP) and the row's last lane adds the
      // row sum; the register-capped closed-form kernels keep one atomic per
      // exit.  Without u_ref, s = b and sum s is copied
      // from b at the flush (with u_ref, LACC adds s per exit).
      // Exit-side counts through ballots.
      if constexpr (LACC) {
        if (valid) {
          if (P.u_ref) lds_add(wrows + row_off(rb, B[rb]) + 4 * SL + EX_S, vs);
          // both buffers' sums take an addend (0 for the other buffer): a
          // branch here lets the compiler index the sums through memory
          const double q = vs * vs;
          ab0 += rb ? 0.0 : vb; aq0 += rb ? 0.0 : q; ak0 += rb ? 0.0 : vk;
          ab1 += rb ? vb : 0.0; aq1 += rb ? q : 0.0; ak1 += rb ? vk : 0.0;
        }
      } else if constexpr (!ROWRED) {
        if (valid) {
          double* ex = wrows + row_off(rb, B[rb]) + 4 * SL;
          lds_add(ex + EX_B, vb);
          if (P.u_ref) lds_add(ex + EX_S, vs);
          lds_add(ex + EX_S2, vs * vs);
          lds_add(ex + EX_K, vk);
        }
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const bool mine = valid && rb == b;
        const uint64_t mm = ROWRED ? __ballot(mine) : 0ull;
        if (mm != 0) {
          double tb = mine ? vb : 0.0, ts = mine ? vs : 0.0, tk = mine ? vk : 0.0;
          double t2 = ts * ts;
          tb = row_total_dpp(tb);
          t2 = row_total_dpp(t2);
          tk = row_total_dpp(tk);
          if (P.u_ref) ts = row_total_dpp(ts);
          if ((lane & 15) == 15 && ((mm >> (lane & 48)) & 0xFFFFull) != 0) {
            double* ex = wrows + row_off(b, B[b]) + 4 * SL;
            lds_add(ex + EX_B, tb);
            if (P.u_ref) lds_add(ex + EX_S, ts);
            lds_add(ex + EX_S2, t2);
            lds_add(ex + EX_K, tk);
          }
        }
      }
      // one integer code per lane (buffer and side), so that each count is a
      // single compare into a lane mask (booleans joined from the branches
      // above would each pass through a vector register first)
      const int scode = valid ? 4 * rb + o : -1;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int cE = __popcll(__ballot(scode == 4 * b + 0));
        const int cN = __popcll(__ballot(scode == 4 * b + 1));
        const int cW = __popcll(__ballot(scode == 4 * b + 2));
        const int cS = __popcll(__ballot(scode == 4 * b + 3));
        if (lane == 0 && (cE | cN | cW | cS) != 0) {
          double* ex = wrows + row_off(b, B[b]) + 4 * SL;
          ex[EX_E] += (double)cE;
          ex[EX_N] += (double)cN;
          ex[EX_W] += (double)cW;
          ex[EX_S_SIDE] += (double)cS;
        }
      }
    }
    wave_sync();
    qn = 0;
  };

  auto acquire = [&](int b, int prow) __attribute__((always_inline)) {
    const uint32_t slot = next_ticket;
    next_ticket = claim(slot);
    const uint32_t t = (uint32_t)P.order[slot];
    const Ticket T = P.tickets[t];
    WB& W = B[b];
    const double* src = reinterpret_cast<const double*>(P.desc + T.knot);
    if (lane < (int)(sizeof(KnotDesc) / sizeof(double)))
      reinterpret_cast<double*>(&W.d)[lane] = src[lane];
    if constexpr (BATCH) {
      const double* isrc = reinterpret_cast<const double*>(P.insts + T.inst);
      if (lane < (int)(sizeof(InstDesc) / sizeof(double)))
        reinterpret_cast<double*>(&W.I)[lane] = isrc[lane];
    }
    if (lane == 0) {
      if constexpr (POOL) W.row = prow;
      W.inst = BATCH ? P.insts[T.inst].inst_id : T.inst;
    }
    double* row = wrows + (size_t)prow * RL;
    for (int i = lane; i < RL; i += 64) row[i] = 0.0;
    wave_sync();
    // the ticket's time step: the instance's, the knot's own (h_i of
    // eq. 40), or the launch's
    double hk = P.h, sqk = P.sqrt_h;
    if constexpr (HK) {
      if (P.h_knot) {
        hk = P.h_knot[T.knot];
        sqk = sqrt(hk);
      }
    }
    if (lane < 4) {
      CoefParams cp = P.coef;
      double sqh = sqk;
      if constexpr (BATCH) { cp.a = W.I.a; sqh = W.I.sqrt_h; }
      W.ebox[lane] = (lut_lay & SIG_EXACT) ? lut_const_threshold<R>(P.coef.lut_info, sqh, W.d, lane)
                                           : exit_threshold<KIND, R>(cp, P.exit_rule, sqh, W.d, lane);
    }
    if (lane == 0) {
      W.start[0] = (R)W.d.sx;
      W.start[1] = (R)W.d.sy;
      if constexpr (BATCH) {
        W.start[2] = (R)W.I.h;
        W.start[3] = (R)W.I.sqrt_h;
        W.start[4] = (R)W.I.a;
      } else {
        W.start[2] = (R)hk;
        W.start[3] = (R)sqk;
      }
    }
    wave_sync();
    if (b) { tk1 = (int)t; nx1 = T.p0; en1 = T.p1; }
    else { tk0 = (int)t; nx0 = T.p0; en0 = T.p1; }
  };

  auto flush = [&](int b) __attribute__((always_inline)) {
    if (qn > 0) process_queue();
    const int t = b ? tk1 : tk0;
    const int prow = row_of(b, B[b]);
    double* row = wrows + (size_t)prow * RL;
    if constexpr (LACC) {
      // the lanes' sums of this buffer, summed over the wave (a fixed order)
      const double tb = wave_sum(b ? ab1 : ab0), tq = wave_sum(b ? aq1 : aq0), tk = wave_sum(b ? ak1 : ak0);
      if (lane == 0) {
        row[4 * SL + EX_B] += tb;
        row[4 * SL + EX_S2] += tq;
        row[4 * SL + EX_K] += tk;
      }
      if (b) { ab1 = 0.0; aq1 = 0.0; ak1 = 0.0; }
      else { ab0 = 0.0; aq0 = 0.0; ak0 = 0.0; }
    }
    // without u_ref every score equals its b contribution: sum s = sum b
    if (!P.u_ref && lane == 0) row[4 * SL + EX_S] = row[4 * SL + EX_B];
    wave_sync();
    double* dst = P.partial + (size_t)t * RL;
    for (int i = lane; i < RL; i += 64) dst[i] = row[i];
    wave_sync();
    // the row goes back to the pool after the wave's reads of it
    if constexpr (POOL) {
      if (lane == 0) atomicOr(pool, 1u << prow);
    }
    if (b) tk1 = -1; else tk0 = -1;
  };

  while (true) {
    // ---- refill idle lanes -------------------------------------------------
    while (true) {
      const uint64_t idle = __ballot(!active);
      if (idle == 0) break;
      // deferred refill: while some lanes still run, wait for enough idle ones
      if (P.refill_min > 1 && idle != ~0ull && __popcll(idle) < P.refill_min) break;
      const int nx = cur ? nx1 : nx0, en = cur ? en1 : en0;
      if (nx >= en) {
        const int old = cur ^ 1;
        int tgt = -1;
        if ((old ? tk1 : tk0) < 0) tgt = old;
        else if ((cur ? tk1 : tk0) < 0) tgt = cur;
        if (tgt < 0 || next_ticket >= t_end) break;
        const int r = POOL ? pool_take() : tgt;
        if (POOL && r < 0) {
          // every row of the pool is taken: step the running lanes and try
          // again; with every lane idle this wave holds no row (its drained
          // tickets were flushed), so the rows are held by other waves of
          // the workgroup, which free them as their tickets drain
          if (idle != ~0ull) break;
          __builtin_amdgcn_s_sleep(2);
          continue;
        }
        acquire(tgt, r);
        cur = tgt;
        continue;
      }
      const int take = min((int)__popcll(idle), en - nx);   // int min (mixed types pick the double overload)
      const int rank = lane_rank(idle);
      if (!active && rank < take) {
        const WB& U = B[cur];
        p = (uint32_t)(nx + rank);
        kn = (uint32_t)U.d.knot;
        inst = U.inst;
        j = 0;
        x = U.start[0];
        y = U.start[1];
        Y = (R)1; Z = (R)0; Xi = (R)0;
        ehx = U.ebox[0];
        ehy = U.ebox[1];
        elx = U.ebox[2];
        ely = U.ebox[3];
        if constexpr (BATCH || HK) {
          lh = U.start[2];
          lsq = U.start[3];
        }
        if constexpr (BATCH) la = U.start[4];
        active = true;
        buf = cur;
      }
      if (cur) nx1 = nx + take; else nx0 = nx + take;
    }
    if (__ballot(active) == 0) break;

    // ---- one Philox draw, up to two Euler steps -------------------------------
    bool ex = false;
    bool forced = false;
    uint32_t K = 0, fl = 0;
    CoefParams cpl = P.coef;
    if constexpr (BATCH) cpl.a = (double)la;
    if constexpr (WAVEWIDE) {
      // the network gradient (a wave-wide MFMA product) and the cooperative
      // table read run with every lane, at each lane's left point, before
      // each half step; the step itself is per lane
      U4 r{};
      R gx = 0, gy = 0;
      Coef<R> cc;
      auto prep = [&]() __attribute__((always_inline)) {
        if constexpr (CV == PDD_CV_NETWORK) {
          // the network's input is the point in the domain's unit coordinates
          net_grad_mfma(NL, (x - ux0) * usx, (y - uy0) * usy, gx, gy);
          gx *= usx;
          gy *= usy;
        }
        if constexpr (COOP) {
          if (lut_lay & LUT_LANE_READ) lut_fetch_lane(cpl, lut_lay, KC, x, y, cc);
          else lut_fetch_coop(cpl, x, y, CW, lane, cc);
        }
        if constexpr (LANE) {
          // only lanes that step read (the others' loads would be wasted)
          if (active && !ex) {
            if (lut_lay & LUT_LANE_READ) lut_fetch_lane(cpl, lut_lay, KC, x, y, cc);
            else lut_fetch_cell(cpl, x, y, cc);
          }
        }
      };
      auto step = [&](R z0, R z1) __attribute__((always_inline)) {
        if constexpr (CV == PDD_CV_GRAD_LUT) grad_lut(P, x, y, gx, gy);
        if constexpr (COOP || LANE) em_step_c<KIND, R, CVON>(cc, lh, lsq, z0, z1, x, y, Y, Z, gx, gy, &Xi);
        else em_step<KIND, R, CVON>(cpl, lh, lsq, z0, z1, x, y, Y, Z, gx, gy, &Xi);
      };
      prep();
      if (active) {
        r = philox10(j, p, kn, inst, P.key0, P.key1);
        R z0, z1;
        box_muller(uniform32(r.a), uniform32(r.b), z0, z1);
        step(z0, z1);
        K = 2 * j + 1;
        ex = exit_test(fl);
      }
      prep();
      if (active) {
        if (!ex) {
          R z0, z1;
          box_muller(uniform32(r.c), uniform32(r.d), z0, z1);
          step(z0, z1);
          K = 2 * j + 2;
          ex = exit_test(fl);
        }
        ++j;
        if (!ex && 2 * j >= MAX_STEPS) { ex = true; forced = true; }
      }
    } else if (active) {
      // grad v at the current (left) point for the per-lane control variates
      auto cv_grad = [&](R& gx, R& gy) __attribute__((always_inline)) {
        if constexpr (CV == PDD_CV_GRAD_LUT) grad_lut(P, x, y, gx, gy);
        else if constexpr (CV == PDD_CV_NETWORK) {
          net_grad_f64(TH, (x - ux0) * usx, (y - uy0) * usy, gx, gy);
          gx *= usx;
          gy *= usy;
        }
        else { gx = 0; gy = 0; }
      };
      const U4 r = philox10(j, p, kn, inst, P.key0, P.key1);
      R z0, z1, gx, gy;
      if constexpr (F64) box_muller(uniform64(r.a), uniform64(r.b), z0, z1);
      else box_muller(uniform32(r.a), uniform32(r.b), z0, z1);
      cv_grad(gx, gy);
      em_step<KIND, R, CVON>(cpl, lh, lsq, z0, z1, x, y, Y, Z, gx, gy, &Xi);
      K = 2 * j + 1;
      ex = exit_test(fl);
      if (!ex) {
        if constexpr (F64) box_muller(uniform64(r.c), uniform64(r.d), z0, z1);
        else box_muller(uniform32(r.c), uniform32(r.d), z0, z1);
        cv_grad(gx, gy);
        em_step<KIND, R, CVON>(cpl, lh, lsq, z0, z1, x, y, Y, Z, gx, gy, &Xi);
        K = 2 * j + 2;
        ex = exit_test(fl);
      }
      ++j;
      if (!ex && 2 * j >= MAX_STEPS) { ex = true; forced = true; }
    }

    // ---- queue the exits ------------------------------------------------------
    const uint64_t em = __ballot(ex);
    if (em != 0) {
      if (ex) {
        const int i = qn + lane_rank(em);
        ExitRec<R> rec;
        rec.x = x; rec.y = y; rec.Y = Y;
        {
#pragma clang fp contract(off)
          rec.bp = Z + Xi;
        }
        Q[i] = rec;
        Qm[i] = K | ((uint32_t)buf << 24) | ((uint32_t)forced << 25) | (fl << 26);
        if (P.dump && (int)p < P.dump_paths) {
          double* d = P.dump + ((size_t)kn * P.dump_paths + p) * PDD_DUMP_WIDTH;
          d[0] = (double)K; d[1] = (double)x; d[2] = (double)y; d[3] = (double)Y;
          d[4] = (double)Z; d[5] = (double)Xi; d[6] = (double)kn; d[7] = (double)p;
        }
        active = false;
      }
      qn += __popcll(em);
      wave_sync();
      if (qn >= 64) process_queue();
    }

    // ---- flush rows whose ticket is handed out and drained ---------------------
    if (tk0 >= 0 && nx0 >= en0 && __ballot(active && buf == 0) == 0) flush(0);
    if (tk1 >= 0 && nx1 >= en1 && __ballot(active && buf == 1) == 0) flush(1);
  }
}

// single launches take per-knot time steps when P.h_knot is set
template <int KIND, bool F64, int CV, bool BATCH>
__global__ __launch_bounds__(256) void k_assemble(AsmParams P) {
  assemble_body<KIND, F64, CV, BATCH, false, !BATCH>(P);
}

// float32 closed-form families without a control variate: capped at 80
// VGPRs, i.e. 6 waves per SIMD (measured 4-12 % faster than the uncapped 5
// waves; with the gradient-table control variate the extra spills cost more
// than the occupancy gains)
// RBF cardinal interpolation at the exits (single launches)
template <int KIND, bool F64, int CV>
__global__ __launch_bounds__(256) void k_assemble_rbf(AsmParams P) {
  assemble_body<KIND, F64, CV, false, true, true>(P);
}

template <int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_assemble_w6(AsmParams P) {
  assemble_body<KIND, false, PDD_CV_NONE, false>(P);
}

// float32 table family, plain or with the gradient-table control variate:
// capped at 128 VGPRs, i.e. 4 waves per SIMD, which fits the LDS when the
// workgroup shares fewer tally rows (the path is latency-bound on its table
// reads and gains with every resident wave)
template <int KIND, int CV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_assemble_w4(AsmParams P) {
  assemble_body<KIND, false, CV, false>(P);
}

// float32 table family whose copy holds only the varying fields (at most two
// of the seven): one lane per path reads them, with no cooperative block in
// LDS.  Five waves per SIMD (at most 96 VGPRs): the fifth wave hides more
// latency than the few spilled words cost.  With the gradient-table control
// variate the exit tallies are row-summed rather than kept per lane, which
// frees the twelve registers that would spill there.
template <int CV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_assemble_lane(AsmParams P) {
  assemble_body<PDD_COEF_LUT, false, CV, false, false, false, true>(P);
}

// Sum a knot's partial rows (ticket order, then side order) into its CSR row,
// b entry and diagnostics.  One wave per knot.
__global__ __launch_bounds__(256) void k_finalize(FinalizeParams F) {
  extern __shared__ double fsum[];
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (F.ticket_counter && blockIdx.x == 0 && threadIdx.x < 8) F.ticket_counter[threadIdx.x] = 0u;
  if (k >= F.n) return;
  const int RL = F.row_len, SL = F.slot_len;
  double* row = fsum + (size_t)(threadIdx.x >> 6) * (F.rbf_inv ? 2 * RL : RL);
  const int tb = F.ticket_begin[k], te = F.ticket_begin[k + 1];
  // the knot's partial rows summed slot by slot in ticket order (coalesced reads)
  for (int i = lane; i < RL; i += 64) {
    double sacc = 0.0;
#pragma unroll 8
    for (int t = tb; t < te; ++t) sacc += F.partial[(size_t)t * RL + i];
    row[i] = sacc;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const KnotDesc d = F.desc[k];
  const double N = (double)F.n_paths[k];
  // RBF: the slots of side o hold sums of Y phi_c(|z - z_q|); its weights
  // are Phi^{-1} times them (Phi^{-1} symmetric: lane i reads column i)
  const double* src = row;
  if (F.rbf_inv) {
    double* wv = row + RL;
    for (int o = 0; o < 4; ++o) {
      if ((d.bmask >> o) & 1) continue;
      const int S = d.chi[o] - d.clo[o] + 1;
      const double* Mi = F.rbf_inv + ((o == 0 || o == 2) ? F.rbf_half : 0) + rbf_block_offset(S);
      for (int i = lane; i < S; i += 64) {
        double acc = 0.0;
        for (int j = 0; j < S; ++j) acc = fma(Mi[(size_t)j * S + i], row[o * SL + j], acc);
        wv[o * SL + i] = acc;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    src = wv;
  }
  for (int pos = F.row_ptr[k] + lane; pos < F.row_ptr[k + 1]; pos += 64) {
    const int col = F.col_idx[pos];
    if (col == (int)k) { F.val[pos] = 1.0; continue; }
    const int cx = F.knot_ij[2 * col], cy = F.knot_ij[2 * col + 1];
    double sv = 0.0;
    for (int o = 0; o < 4; ++o) {
      if ((d.bmask >> o) & 1) continue;
      const bool vert = (o == 0 || o == 2);
      const int on = vert ? cx : cy, q = vert ? cy : cx;
      if (on != d.at[o] || q < d.clo[o] || q > d.chi[o]) continue;
      sv += src[o * SL + (q - d.clo[o])];
    }
    F.val[pos] = -sv / N;
  }
  if (lane < EX_COUNT) {
    const double e = row[4 * SL + lane];
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

// hk: per-knot time steps (the capped kernels take the launch's h only)
template <int KIND, bool F64, int CV, bool BATCH = false>
const void* kernel_ptr(bool hk = false) {
  if constexpr (!F64 && CV == PDD_CV_NONE && !BATCH && KIND != PDD_COEF_LUT) {
    if (!hk) return reinterpret_cast<const void*>(&k_assemble_w6<KIND>);
  } else if constexpr (!F64 && (CV == PDD_CV_NONE || CV == PDD_CV_GRAD_LUT) && !BATCH && KIND == PDD_COEF_LUT) {
    if (!hk) return reinterpret_cast<const void*>(&k_assemble_w4<KIND, CV>);
  }
  return reinterpret_cast<const void*>(&k_assemble<KIND, F64, CV, BATCH>);
}

template <bool F64, int CV>
const void* pick_batch_kind(int kind) {
  switch (kind) {
    case PDD_COEF_POISSON: return kernel_ptr<PDD_COEF_POISSON, F64, CV, true>();
    case PDD_COEF_VARCOEF: return kernel_ptr<PDD_COEF_VARCOEF, F64, CV, true>();
    case PDD_COEF_AMPLITUDE: return kernel_ptr<PDD_COEF_AMPLITUDE, F64, CV, true>();
    default: return nullptr;
  }
}

// batched launches: no control variate, the gradient table, or (float32
// only) the network
template <bool F64>
const void* pick_batch(int kind, int cv) {
  switch (cv) {
    case PDD_CV_NONE: return pick_batch_kind<F64, PDD_CV_NONE>(kind);
    case PDD_CV_GRAD_LUT: return pick_batch_kind<F64, PDD_CV_GRAD_LUT>(kind);
    case PDD_CV_NETWORK:
      if constexpr (!F64) return pick_batch_kind<false, PDD_CV_NETWORK>(kind);
      else return nullptr;
    default: return nullptr;
  }
}

template <bool F64, int CV>
const void* pick_kind(int kind, bool hk) {
  switch (kind) {
    case PDD_COEF_POISSON: return kernel_ptr<PDD_COEF_POISSON, F64, CV>(hk);
    case PDD_COEF_VARCOEF: return kernel_ptr<PDD_COEF_VARCOEF, F64, CV>(hk);
    case PDD_COEF_AMPLITUDE: return kernel_ptr<PDD_COEF_AMPLITUDE, F64, CV>(hk);
    case PDD_COEF_LUT: return kernel_ptr<PDD_COEF_LUT, F64, CV>(hk);
    case PDD_COEF_EQ43: return kernel_ptr<PDD_COEF_EQ43, F64, CV>(hk);
    default: break;
  }
  if constexpr (CV == PDD_CV_NONE) {
    if (kind == PDD_COEF_CONSTSOL) return kernel_ptr<PDD_COEF_CONSTSOL, F64, CV>(hk);
    if (kind == PDD_COEF_EXITTIME) return kernel_ptr<PDD_COEF_EXITTIME, F64, CV>(hk);
  }
  return nullptr;
}

template <bool F64>
const void* pick(int kind, int cv, bool hk) {
  switch (cv) {
    case PDD_CV_NONE: return pick_kind<F64, PDD_CV_NONE>(kind, hk);
    case PDD_CV_NETWORK: return pick_kind<F64, PDD_CV_NETWORK>(kind, hk);
    case PDD_CV_GRAD_LUT: return pick_kind<F64, PDD_CV_GRAD_LUT>(kind, hk);
    default: return nullptr;
  }
}

template <bool F64, int CV>
const void* pick_rbf_kind(int kind) {
  switch (kind) {
    case PDD_COEF_POISSON: return reinterpret_cast<const void*>(&k_assemble_rbf<PDD_COEF_POISSON, F64, CV>);
    case PDD_COEF_VARCOEF: return reinterpret_cast<const void*>(&k_assemble_rbf<PDD_COEF_VARCOEF, F64, CV>);
    case PDD_COEF_AMPLITUDE: return reinterpret_cast<const void*>(&k_assemble_rbf<PDD_COEF_AMPLITUDE, F64, CV>);
    case PDD_COEF_LUT: return reinterpret_cast<const void*>(&k_assemble_rbf<PDD_COEF_LUT, F64, CV>);
    case PDD_COEF_EQ43: return reinterpret_cast<const void*>(&k_assemble_rbf<PDD_COEF_EQ43, F64, CV>);
    default: break;
  }
  if constexpr (CV == PDD_CV_NONE) {
    if (kind == PDD_COEF_CONSTSOL) return reinterpret_cast<const void*>(&k_assemble_rbf<PDD_COEF_CONSTSOL, F64, CV>);
    if (kind == PDD_COEF_EXITTIME) return reinterpret_cast<const void*>(&k_assemble_rbf<PDD_COEF_EXITTIME, F64, CV>);
  }
  return nullptr;
}

// RBF interpolation: no control variate or the gradient table
template <bool F64>
const void* pick_rbf(int kind, int cv) {
  switch (cv) {
    case PDD_CV_NONE: return pick_rbf_kind<F64, PDD_CV_NONE>(kind);
    case PDD_CV_GRAD_LUT: return pick_rbf_kind<F64, PDD_CV_GRAD_LUT>(kind);
    default: return nullptr;
  }
}

const void* rbf_kernel(int precision, int kind, int cv) {
  return precision == PDD_FP64_SAME_STREAM ? pick_rbf<true>(kind, cv) : pick_rbf<false>(kind, cv);
}

// lane: the float32 table family with the lane-read layout (single launches
// with the launch's h, hat interpolation)
const void* assemble_kernel(int precision, int kind, int cv, bool batch, bool hk = false, bool lane = false) {
  if (lane && !batch && !hk && precision == PDD_FP32_PRODUCTION && kind == PDD_COEF_LUT) {
    if (cv == PDD_CV_NONE) return reinterpret_cast<const void*>(&k_assemble_lane<PDD_CV_NONE>);
    if (cv == PDD_CV_GRAD_LUT) return reinterpret_cast<const void*>(&k_assemble_lane<PDD_CV_GRAD_LUT>);
  }
  if (batch) return precision == PDD_FP64_SAME_STREAM ? pick_batch<true>(kind, cv) : pick_batch<false>(kind, cv);
  return precision == PDD_FP64_SAME_STREAM ? pick<true>(kind, cv, hk) : pick<false>(kind, cv, hk);
}

}  // namespace

size_t assemble_lds_bytes(int precision, int kind, int row_len, int block, int cv_mode, bool batch, int pool_rows,
                          bool lane) {
  const size_t waves = (size_t)block / 64;
  const size_t rows = POOL_HEAD + (size_t)(pool_rows > 0 ? pool_rows : 2 * (int)waves) * row_len * sizeof(double);
  if (precision == PDD_FP64_SAME_STREAM) {
    const size_t net = cv_mode == PDD_CV_NETWORK ? net_lds_bytes<true, PDD_CV_NETWORK>() : 0;
    return net + rows + waves * (batch ? wave_lds_bytes<double, TB_NONE, true>() : wave_lds_bytes<double, TB_NONE, false>());
  }
  const size_t net = cv_mode == PDD_CV_NETWORK ? net_lds_bytes<false, PDD_CV_NETWORK>() : 0;
  if (batch) return net + rows + waves * wave_lds_bytes<float, TB_NONE, true>();
  if (kind == PDD_COEF_LUT && cv_mode != PDD_CV_NETWORK)
    return net + rows + waves * (lane ? wave_lds_bytes<float, TB_LANE, false>() : wave_lds_bytes<float, TB_COOP, false>());
  return net + rows + waves * wave_lds_bytes<float, TB_NONE, false>();
}

hipError_t assemble_occupancy(int precision, int kind, int cv_mode, bool batch, int block, size_t lds_bytes,
                              int* blocks_per_cu, bool per_knot_h, bool lane) {
  const void* f = assemble_kernel(precision, kind, cv_mode, batch, per_knot_h, lane);
  if (!f) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, block, lds_bytes);
}

hipError_t launch_assemble(const AsmParams& p, int precision, int grid, int block, size_t lds_bytes,
                           hipStream_t stream) {
  const void* f = assemble_kernel(precision, p.coef.kind, p.cv_mode, p.insts != nullptr, p.h_knot != nullptr,
                                  p.table_lane != 0);
  if (!f) return hipErrorInvalidValue;
  AsmParams arg = p;
  void* args[] = {&arg};
  return hipLaunchKernel(f, dim3(grid), dim3(block), args, lds_bytes, stream);
}

hipError_t assemble_occupancy_rbf(int precision, int kind, int cv_mode, int block, size_t lds_bytes,
                                  int* blocks_per_cu) {
  const void* f = rbf_kernel(precision, kind, cv_mode);
  if (!f) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, block, lds_bytes);
}

hipError_t launch_assemble_rbf(const AsmParams& p, int precision, int grid, int block, size_t lds_bytes,
                               hipStream_t stream) {
  const void* f = rbf_kernel(precision, p.coef.kind, p.cv_mode);
  if (!f || !p.rbf_inv || p.insts) return hipErrorInvalidValue;
  AsmParams arg = p;
  void* args[] = {&arg};
  return hipLaunchKernel(f, dim3(grid), dim3(block), args, lds_bytes, stream);
}

hipError_t launch_finalize(const FinalizeParams& p, hipStream_t stream) {
  // one summed row per wave in LDS (and its RBF weights beside it), at most
  // 160 KiB per workgroup
  const size_t per_wave = (size_t)(p.rbf_inv ? 2 : 1) * p.row_len * sizeof(double);
  const int block = 4 * per_wave <= 163840 ? 256 : 64;
  const int64_t grid = (p.n + block / 64 - 1) / (block / 64);
  const size_t lds = (size_t)(block / 64) * per_wave;
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_finalize),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)grid), dim3(block), lds, stream, p);
  return hipGetLastError();
}

}  // namespace pdd
