// C ABI of the deposition step (include/depo.h): validation, workspace
// planning, uploads, the per-step launch sequence (optionally replayed from a
// captured HIP graph), tallies and checkpoints.  Host code only; the kernels
// live in k_particle.hip, k_coulomb.hip and k_cells.hip.
#include "depo.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "adjoint.hpp"
#include "common.hpp"
#include "launch.hpp"

using namespace depo;

constexpr int kSymTileMin = 256;       // smallest symmetric pair-kernel item (64 * ipl * waves targets)
constexpr int kP3mImages = 256;        // x images summed into the P3M Green's function
constexpr int64_t kMaxItems = 1 << 22; // largest symmetric item list a layout reserves room for (32 B each)
// FP32 defaults: the symmetric kernel, or the one-sided kernel where the layout has too many items
const CoulombConfig kDefaultSym{4, 2, 64, true, true};
const CoulombConfig kDefaultOneSided{1, 8, 32, true};

namespace {

constexpr uint32_t kKnownFlags = (1u << 10) - 1;
constexpr int kMaxN = 1 << 26;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

uint32_t crc32_update(uint32_t crc, const void *data, size_t n) {
  static uint32_t table[256];
  static bool init = false;
  if (!init) {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t c = i;
      for (int k = 0; k < 8; ++k) c = (c & 1) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
      table[i] = c;
    }
    init = true;
  }
  const uint8_t *p = (const uint8_t *)data;
  crc = ~crc;
  for (size_t i = 0; i < n; ++i) crc = table[(crc ^ p[i]) & 0xFF] ^ (crc >> 8);
  return ~crc;
}

struct BlobHeader {
  char magic[8];
  uint32_t version, real_bytes;
  int64_t n;
  int32_t s, nstep;
  uint64_t payload;
  uint32_t crc, pad;
};

}  // namespace

struct depo_ctx {
  depo_params p{};
  std::string err;
  // layout
  bool has_layout = false;
  int S = 0;
  int64_t N = 0;
  std::vector<int64_t> off;
  int nx = 0, ny = 0, nz = 0;
  int64_t cell_cap = 0;
  int scan_blocks = 0;
  int tile_cap = 0;
  // symmetric pair kernel (FP32): item capacity (for the smallest item size),
  // item counts, per-sample bounds for the fixed-point scale
  int64_t sym_cap = 0;
  int n_diag = 0, n_off = 0;
  // P3M electrostatics (configured before the layout; single-sample layouts)
  bool p3m_cfg = false, p3m_use = false, p3m_green = false;
  int p3m_nx = 0, p3m_nc = 0;
  double p3m_alpha_h = 0.0, p3m_rmax_alpha = 0.0;
  P3mDev pm{};
  double *p3m_qscale = nullptr;
  std::vector<double> sum_abs_qb, dmin;
  // workspace
  size_t ws_need = 0;
  char *ws = nullptr;
  bool bound = false, field_ready = false, seeded = false;
  // state
  int nstep = 0;
  int n_cells = 0;
  int n_tiles = 0;
  std::vector<SampleDev> samples;
  std::vector<depo_sample_params> sp;
  double dmax_all = 0.0;
  CoulombConfig ccfg = kDefaultSym;
  Phys ph{};
  State<float> sf{};
  State<double> sd{};
  OrderScratch<float> of{};
  OrderScratch<double> od{};
  int order_every = 0;        // steps between storage reorders (0: never)
  // captured step graph
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;
  hipStream_t cap_side = nullptr;               // the graph's short-range branch
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool use_graph = true;
  // state generation: every call that changes the particle state, the parameters, the field or the
  // kernel configuration advances it; a pending reverse sweep belongs to one generation
  uint64_t gen = 0;
  bool adj_pending = false;
  uint64_t adj_gen = 0;
  int adj_n = 0, adj_ce = 0;
  void *adj_ws = nullptr;
  size_t adj_bytes = 0;

  bool fp64() const { return p.real_bytes == 8; }
  depo_status fail(depo_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return st;
  }
  void drop_graph() {
    if (gexec) hipGraphExecDestroy(gexec);
    gexec = nullptr;
  }
};

#define HIP_TRY(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return ctx->fail(DEPO_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

template <class Real> OrderScratch<Real> &order_scratch(depo_ctx *ctx);
template <> OrderScratch<float> &order_scratch<float>(depo_ctx *ctx) { return ctx->of; }
template <> OrderScratch<double> &order_scratch<double>(depo_ctx *ctx) { return ctx->od; }

// Carve the workspace (base == nullptr: only size it).
template <class Real>
size_t carve(depo_ctx *ctx, char *base, State<Real> &st) {
  using Pos = typename Prec<Real>::Pos;
  const size_t N = (size_t)std::max<int64_t>(ctx->N, 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + o : nullptr;
    o = align_up(o + bytes);
    return p;
  };
  st.px = (Pos *)take(N * sizeof(Pos));
  st.py = (Pos *)take(N * sizeof(Pos));
  st.pz = (Pos *)take(N * sizeof(Pos));
  Real **reals[] = {&st.rx, &st.ry, &st.rz, &st.vx, &st.vy, &st.vz, &st.ax, &st.ay, &st.az, &st.ux, &st.uy,
                    &st.uz, &st.cx, &st.cy, &st.cz, &st.sx, &st.sy, &st.sz, &st.jr};
  for (Real **r : reals) *r = (Real *)take(N * sizeof(Real));
  st.d = (double *)take(N * sizeof(double));
  st.qb = (double *)take(N * sizeof(double));
  st.ell = (double *)take(N * sizeof(double));
  st.dep = (int32_t *)take(N * 4);
  st.sid = (int32_t *)take(N * 4);
  st.nbr = (int32_t *)take(N * 4);
  st.perm = (int32_t *)take(N * 4);
  st.cell_of = (int32_t *)take(N * 4);
  st.cell_idx = (int32_t *)take(N * 4);
  st.cell_count = (int32_t *)take((size_t)ctx->cell_cap * 4);
  st.cell_start = (int32_t *)take(((size_t)ctx->cell_cap + 1) * 4);
  st.scan_part = (int32_t *)take((size_t)std::max(ctx->scan_blocks, 1) * 4);
  st.js = (JSrc<Real> *)take(N * sizeof(JSrc<Real>));
  st.samples = (SampleDev *)take((size_t)ctx->S * sizeof(SampleDev));
  st.tiles = (TileDev *)take((size_t)std::max(ctx->tile_cap, 1) * sizeof(TileDev));
  const size_t nacc = sizeof(Real) == 4 ? N : 1;   // fixed-point accumulators: FP32 form only
  st.items = (SymItem *)take((size_t)std::max<int64_t>(ctx->sym_cap, 1) * sizeof(SymItem));
  st.fx_scale = (double *)take((size_t)ctx->S * sizeof(double));
  st.accx = (unsigned long long *)take(nacc * 8);
  st.accy = (unsigned long long *)take(nacc * 8);
  st.accz = (unsigned long long *)take(nacc * 8);
  if (ctx->p3m_cfg) {
    P3mDev &m = ctx->pm;
    const size_t total = (size_t)m.nx * m.P * m.P, ncell = (size_t)m.ncx * m.ncy * m.ncy;
    const size_t me = sizeof(Real) == 4 ? sizeof(float2) : sizeof(double2);   // mesh element
    for (int c = 0; c < 3; ++c) m.ghat[c] = take(total * me);
    m.rho = take(2 * total * me);   // rho, then work
    m.work = m.rho ? (void *)((char *)m.rho + total * me) : nullptr;
    m.qmesh = (unsigned long long *)take((size_t)m.nx * m.nc * m.nc * 8);
    m.slong = (double *)take(3 * N * sizeof(double));
    m.cell_of = (int32_t *)take(N * 4);
    m.counts = (int32_t *)take(ncell * 4);
    m.starts = (int32_t *)take((ncell + 1) * 4);
    m.fill = (int32_t *)take(ncell * 4);
    m.sorted = (int32_t *)take(N * 4);
    m.rec = take(N * 5 * sizeof(typename Prec<Real>::Pos));
    m.table = (float2 *)take(2049 * sizeof(float2));   // 2,048 intervals + the terminating (0, 0)
    ctx->p3m_qscale = (double *)take(64);
    m.q_scale = ctx->p3m_qscale;
  }
  {
    OrderScratch<Real> &sc = order_scratch<Real>(ctx);
    sc.px = (Pos *)take(N * sizeof(Pos));
    sc.py = (Pos *)take(N * sizeof(Pos));
    sc.pz = (Pos *)take(N * sizeof(Pos));
    Real **reals[] = {&sc.rx, &sc.ry, &sc.rz, &sc.vx, &sc.vy, &sc.vz, &sc.ax, &sc.ay, &sc.az,
                      &sc.ux, &sc.uy, &sc.uz, &sc.jr};
    for (Real **r : reals) *r = (Real *)take(N * sizeof(Real));
    sc.d = (double *)take(N * 8);
    sc.qb = (double *)take(N * 8);
    sc.ell = (double *)take(N * 8);
    sc.dep = (int32_t *)take(N * 4);
    sc.nbr = (int32_t *)take(N * 4);
    sc.perm = (int32_t *)take(N * 4);
  }
  st.field = (typename Prec<Real>::Vec4 *)take((size_t)ctx->nx * ctx->ny * ctx->nz * sizeof(typename Prec<Real>::Vec4));
  st.nstep = (int32_t *)take(64);
  st.err = (uint32_t *)take(64);
  st.tally = (double *)take((size_t)ctx->S * 8 * sizeof(double));
  return o;
}

template <class Real> State<Real> &state(depo_ctx *ctx);
template <> State<float> &state<float>(depo_ctx *ctx) { return ctx->sf; }
template <> State<double> &state<double>(depo_ctx *ctx) { return ctx->sd; }

// The Coulomb source records hold integer y and z only for the symmetric integer-record kernel.
void set_record_format(depo_ctx *ctx) {
  ctx->ph.flags &= ~F_INT_RECORDS;
  if (ctx->ccfg.int_rec && !ctx->fp64()) ctx->ph.flags |= F_INT_RECORDS;
}

void fill_phys(depo_ctx *ctx) {
  const depo_params &p = ctx->p;
  Phys &ph = ctx->ph;
  const int B = ctx->fp64() ? 64 : 32;
  ph.flags = p.flags;
  ph.R = p.R;
  ph.L = p.L;
  ph.ux = p.L * std::ldexp(1.0, -B);
  ph.ur = p.R * std::ldexp(1.0, -(B - 2));
  ph.inv_ux = 1.0 / ph.ux;
  ph.inv_ur = 1.0 / ph.ur;
  ph.dt = p.dt;
  ph.nu = p.nu;
  ph.rho_p = p.rho_p;
  ph.rho_f = p.rho_f;
  ph.tau_coef = p.rho_p / (18.0 * p.rho_f * p.nu);
  ph.mass_coef = p.rho_p * M_PI / 6.0;
  ph.k_e = 1.0 / (4.0 * M_PI * p.eps0);
  ph.q_ref = 1e-15;
  ph.yz_over_x = ph.ur / ph.ux;
  ph.delta_sat = (p.flags & DEPO_VDW_GU) ? p.delta_min * std::pow(p.kr_over_k, 0.25) : p.delta_min;
  const double tau_col = p.tau_col_steps * p.dt;
  const double le = std::log(p.e_pp);
  ph.col_K = (M_PI * M_PI + le * le) / (tau_col * tau_col);
  ph.col_H = -2.0 * le / tau_col;
  for (int k = 0; k < 3; ++k) ph.g_body[k] = p.g_body[k];
  ph.E_young = p.E_young;
  ph.delta_c = p.delta_c;
  ph.acont_coef = p.acont_coef;
  ph.soft_eps = p.soft_eps;
  ph.soft_rate = (p.soft_tau > 0.0) ? 1.0 / (p.soft_tau * p.dt) : 0.0;
  ph.N = (int32_t)ctx->N;
  ph.S = ctx->S;
  ph.nx = ctx->nx;
  ph.ny = ctx->ny;
  ph.nz = ctx->nz;
  set_record_format(ctx);
}

void build_tiles(depo_ctx *ctx, std::vector<TileDev> &tiles) {
  const int T = coulomb_tile_targets(ctx->ccfg);
  std::vector<int> order(ctx->S);
  for (int s = 0; s < ctx->S; ++s) order[s] = s;
  // longest samples first: their tiles cost the most (work ~ N_s per tile)
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return ctx->off[a + 1] - ctx->off[a] > ctx->off[b + 1] - ctx->off[b];
  });
  tiles.clear();
  for (int s : order) {
    const int64_t b = ctx->off[s], e = ctx->off[s + 1];
    for (int64_t i = b; i < e; i += T)
      tiles.push_back(TileDev{(int32_t)i, (int32_t)std::min<int64_t>(T, e - i), (int32_t)b, (int32_t)(e - b)});
  }
}

// Work items of the symmetric pair kernel for item size T: per sample, the n_t
// diagonal items, then the n_t (n_t - 1) / 2 items above the diagonal.
void build_items(const depo_ctx *ctx, int T, std::vector<SymItem> &items, int &n_diag, int &n_off) {
  std::vector<SymItem> diag, off;
  for (int s = 0; s < ctx->S; ++s) {
    const int64_t b = ctx->off[s], n = ctx->off[s + 1] - b;
    const int64_t nt = (n + T - 1) / T;
    auto cnt = [&](int64_t I) { return (int32_t)std::min<int64_t>(T, n - I * T); };
    for (int64_t I = 0; I < nt; ++I) {
      const int32_t i0 = (int32_t)(b + I * T);
      diag.push_back(SymItem{i0, cnt(I), i0, cnt(I), s, {0, 0, 0}});
      for (int64_t J = I + 1; J < nt; ++J)
        off.push_back(SymItem{i0, cnt(I), (int32_t)(b + J * T), cnt(J), s, {0, 0, 0}});
    }
  }
  // costliest items first
  auto by_cost = [](const SymItem &a, const SymItem &c) {
    return (int64_t)a.icount * a.jcount > (int64_t)c.icount * c.jcount;
  };
  std::stable_sort(diag.begin(), diag.end(), by_cost);
  std::stable_sort(off.begin(), off.end(), by_cost);
  n_diag = (int)diag.size();
  n_off = (int)off.size();
  items = diag;
  items.insert(items.end(), off.begin(), off.end());
}

// Upload the symmetric work items for the current configuration.
depo_status upload_items(depo_ctx *ctx) {
  std::vector<SymItem> items;
  build_items(ctx, coulomb_sym_tile(ctx->ccfg), items, ctx->n_diag, ctx->n_off);
  if ((int64_t)items.size() > ctx->sym_cap) return ctx->fail(DEPO_E_CAPACITY, "symmetric item list exceeds capacity");
  if (!items.empty()) HIP_TRY(hipMemcpy(ctx->sf.items, items.data(), items.size() * sizeof(SymItem), hipMemcpyHostToDevice));
  return DEPO_OK;
}

// Per-sample sum of |qbase| and smallest diameter (host copies of the seeded arrays).
void set_charge_bounds(depo_ctx *ctx, const double *h_d, const double *h_qb) {
  ctx->sum_abs_qb.assign(ctx->S, 0.0);
  ctx->dmin.assign(ctx->S, 0.0);
  for (int s = 0; s < ctx->S; ++s) {
    double sq = 0.0, dm = INFINITY;
    for (int64_t i = ctx->off[s]; i < ctx->off[s + 1]; ++i) {
      sq += std::fabs(h_qb[i]);
      dm = std::min(dm, h_d[i]);
    }
    ctx->sum_abs_qb[s] = sq;
    ctx->dmin[s] = std::isfinite(dm) ? dm : 1.0;
  }
}

// Fixed-point scale of the P3M charge mesh: every node holds at most sum_j |q~_j|.
depo_status upload_p3m_scale(depo_ctx *ctx, hipStream_t stream) {
  if (!ctx->p3m_cfg || ctx->S == 0) return DEPO_OK;
  const double bound = std::fabs(ctx->samples[0].charge_scale) * ctx->sum_abs_qb[0] / ctx->ph.q_ref;
  double sc = 1.0;
  if (bound > 0.0 && std::isfinite(bound)) sc = std::ldexp(1.0, 62 - (int)std::ceil(std::log2(bound)));
  HIP_TRY(hipMemcpyAsync(ctx->p3m_qscale, &sc, sizeof sc, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return DEPO_OK;
}

// Fixed-point scale of the symmetric pair sums: |pair sum| <= sum_j |q~_j| / (d_min/ux)^2 =: B
// for every particle of the sample (each term is at most |q~_j| / d_ij^2), so 2^62 / B (rounded
// down to a power of two) units per unit of sum cannot overflow 64 bits.
depo_status upload_fx_scale(depo_ctx *ctx, hipStream_t stream) {
  if (ctx->fp64() || ctx->S == 0) return DEPO_OK;
  std::vector<double> sc(ctx->S, 1.0);
  for (int s = 0; s < ctx->S; ++s) {
    const double dq = ctx->dmin[s] * ctx->ph.inv_ux;
    const double bound = std::fabs(ctx->samples[s].charge_scale) * ctx->sum_abs_qb[s] / ctx->ph.q_ref / (dq * dq);
    if (bound > 0.0 && std::isfinite(bound)) sc[s] = std::ldexp(1.0, 62 - (int)std::ceil(std::log2(bound)));
  }
  HIP_TRY(hipMemcpyAsync(ctx->sf.fx_scale, sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return DEPO_OK;
}

bool short_range_on(const depo_ctx *ctx) { return (ctx->p.flags & (DEPO_COLLIDE | DEPO_VDW)) != 0; }

// Items of the symmetric kernel for item size T: n_t (n_t + 1) / 2 per sample.
int64_t count_items(const std::vector<int64_t> &off, int64_t T) {
  int64_t total = 0;
  for (size_t s = 0; s + 1 < off.size(); ++s) {
    const int64_t nt = (off[s + 1] - off[s] + T - 1) / T;
    total += nt * (nt + 1) / 2;
  }
  return total;
}

// Returns the k_finish mode bit that the pair sums need: with defer_finish, the symmetric pair
// kernel leaves its fixed-point accumulators to k_finish (F_PAIR_SUMS), one pass fewer per step.
template <class Real> int enqueue_coulomb(depo_ctx *ctx, hipStream_t s, bool defer_finish = false) {
  if (!(ctx->p.flags & DEPO_COULOMB)) return 0;
  if (ctx->p3m_use) {
    launch_p3m<Real>(state<Real>(ctx), ctx->ph, ctx->pm, s);
    return 0;
  }
  if constexpr (std::is_same<Real, float>::value) {
    if (ctx->ccfg.symmetric) {
      launch_coulomb_sym(ctx->sf, ctx->ph, ctx->n_diag, ctx->n_off, ctx->ccfg, s, defer_finish);
      return defer_finish ? F_PAIR_SUMS : 0;
    }
  }
  launch_coulomb<Real>(state<Real>(ctx), ctx->ph, ctx->n_tiles, ctx->ccfg, s);
  return 0;
}

// Enqueue the force evaluation at the current positions (prepare has run).
template <class Real> void enqueue_forces(depo_ctx *ctx, hipStream_t s) {
  const State<Real> &st = state<Real>(ctx);
  if (short_range_on(ctx)) launch_cells<Real>(st, ctx->ph, ctx->n_cells, (ctx->n_cells + 1023) / 1024, s);
  enqueue_coulomb<Real>(ctx, s);
  if (short_range_on(ctx)) launch_short_range<Real>(st, ctx->ph, ctx->n_cells, s);
}

int prepare_mode(const depo_ctx *ctx) {
  int m = P_COULOMB;   // always refresh the source records (cheap, keeps them consistent)
  if (short_range_on(ctx)) m |= P_CELLS;
  return m;
}

// The storage reorder kernels of a step (they act only on the steps that follow a multiple of
// order_every steps).  Not in the smoothed-tally mode, whose adjoint stores states in one order,
// and only with a cell list, which the short-range forces build every step.
template <class Real> void enqueue_order(depo_ctx *ctx, hipStream_t s) {
  if (ctx->order_every <= 0 || !short_range_on(ctx) || (ctx->p.flags & DEPO_SOFT_TALLY) || ctx->N <= 0) return;
  launch_order<Real>(state<Real>(ctx), order_scratch<Real>(ctx), (int)ctx->N, ctx->n_cells, ctx->order_every, s);
}

template <class Real> void enqueue_step(depo_ctx *ctx, hipStream_t s) {
  const State<Real> &st = state<Real>(ctx);
  enqueue_order<Real>(ctx, s);
  launch_prepare<Real>(st, ctx->ph, prepare_mode(ctx) | P_KICK_DRIFT, s);
  if (short_range_on(ctx)) launch_cells<Real>(st, ctx->ph, ctx->n_cells, (ctx->n_cells + 1023) / 1024, s);
  const int pair_mode = enqueue_coulomb<Real>(ctx, s, true);
  if (short_range_on(ctx)) launch_short_range<Real>(st, ctx->ph, ctx->n_cells, s);
  launch_finish<Real>(st, ctx->ph, F_KICK | pair_mode, s);
}

// One step as a graph with two branches after prepare: the direct Coulomb sums, and the cell
// build + short-range forces (which touch disjoint buffers), joined before finish, so that the
// O(N) branch fills the pair kernel's tail.
template <class Real> hipError_t capture_forked_step(depo_ctx *ctx) {
  const State<Real> &st = state<Real>(ctx);
  hipStream_t a = ctx->cap_stream, b = ctx->cap_side;
  enqueue_order<Real>(ctx, a);
  launch_prepare<Real>(st, ctx->ph, prepare_mode(ctx) | P_KICK_DRIFT, a);
  hipError_t e = hipEventRecord(ctx->ev_fork, a);
  if (e == hipSuccess) e = hipStreamWaitEvent(b, ctx->ev_fork, 0);
  if (e != hipSuccess) return e;
  launch_cells<Real>(st, ctx->ph, ctx->n_cells, (ctx->n_cells + 1023) / 1024, b);
  launch_short_range<Real>(st, ctx->ph, ctx->n_cells, b);
  if ((e = hipEventRecord(ctx->ev_join, b)) != hipSuccess) return e;
  const int pair_mode = enqueue_coulomb<Real>(ctx, a, true);
  if ((e = hipStreamWaitEvent(a, ctx->ev_join, 0)) != hipSuccess) return e;
  launch_finish<Real>(st, ctx->ph, F_KICK | pair_mode, a);
  return hipGetLastError();
}

template <class Real> depo_status run_steps(depo_ctx *ctx, int n, hipStream_t s) {
  if (n == 0) return DEPO_OK;
  if (ctx->use_graph) {
    if (!ctx->gexec) {
      if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
      // the P3M pipeline has cell passes of its own: it stays on one branch
      const bool fork = short_range_on(ctx) && (ctx->p.flags & DEPO_COULOMB) && !ctx->p3m_use;
      if (fork && !ctx->cap_side) {
        HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_side, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
      }
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
      hipError_t e = hipSuccess;
      if (fork)
        e = capture_forked_step<Real>(ctx);
      else {
        enqueue_step<Real>(ctx, ctx->cap_stream);
        e = hipGetLastError();
      }
      hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return ctx->fail(DEPO_E_HIP, "step graph capture failed: %s",
                         hipGetErrorString(e != hipSuccess ? e : e2));
      }
      hipError_t e3 = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e3 != hipSuccess) {
        ctx->gexec = nullptr;
        return ctx->fail(DEPO_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e3));
      }
    }
    for (int k = 0; k < n; ++k) HIP_TRY(hipGraphLaunch(ctx->gexec, s));
  } else {
    for (int k = 0; k < n; ++k) enqueue_step<Real>(ctx, s);
    HIP_TRY(hipGetLastError());
  }
  ctx->nstep += n;
  return DEPO_OK;
}

template <class Real> depo_status run_steps_timed(depo_ctx *ctx, int n, hipStream_t s, double *ms) {
  // phase boundaries: prepare | cell build | Coulomb | short range | finish
  const State<Real> &st = state<Real>(ctx);
  std::vector<hipEvent_t> ev(6 * (size_t)n, nullptr);
  for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
  for (int k = 0; k < n; ++k) {
    hipEvent_t *E = &ev[6 * (size_t)k];
    HIP_TRY(hipEventRecord(E[0], s));
    // a storage reorder counts with the particle update before the forces
    enqueue_order<Real>(ctx, s);
    launch_prepare<Real>(st, ctx->ph, prepare_mode(ctx) | P_KICK_DRIFT, s);
    HIP_TRY(hipEventRecord(E[1], s));
    if (short_range_on(ctx)) launch_cells<Real>(st, ctx->ph, ctx->n_cells, (ctx->n_cells + 1023) / 1024, s);
    HIP_TRY(hipEventRecord(E[2], s));
    enqueue_coulomb<Real>(ctx, s);
    HIP_TRY(hipEventRecord(E[3], s));
    if (short_range_on(ctx)) launch_short_range<Real>(st, ctx->ph, ctx->n_cells, s);
    HIP_TRY(hipEventRecord(E[4], s));
    launch_finish<Real>(st, ctx->ph, F_KICK, s);
    HIP_TRY(hipEventRecord(E[5], s));
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  for (int q = 0; q < 5; ++q) ms[q] = 0.0;
  for (int k = 0; k < n; ++k)
    for (int q = 0; q < 5; ++q) {
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, ev[6 * (size_t)k + q], ev[6 * (size_t)k + q + 1]));
      ms[q] += t;
    }
  for (auto &e : ev) hipEventDestroy(e);
  ctx->nstep += n;
  return DEPO_OK;
}

template <class Real> depo_status do_init_field(depo_ctx *ctx, const double *h, hipStream_t s) {
  using V4 = typename Prec<Real>::Vec4;
  const size_t n = (size_t)ctx->nx * ctx->ny * ctx->nz;
  std::vector<V4> tmp(n);
  for (size_t k = 0; k < n; ++k) {
    const double a = h[3 * k], b = h[3 * k + 1], c = h[3 * k + 2];
    if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c))
      return ctx->fail(DEPO_E_INVALID, "field value %zu is not finite", k);
    tmp[k].x = (Real)a; tmp[k].y = (Real)b; tmp[k].z = (Real)c; tmp[k].w = (Real)0;
  }
  HIP_TRY(hipMemcpyAsync(state<Real>(ctx).field, tmp.data(), n * sizeof(V4), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return DEPO_OK;
}

depo_status build_samples(depo_ctx *ctx, const depo_sample_params *sp, const double *h_d) {
  const depo_params &p = ctx->p;
  ctx->samples.assign(ctx->S, SampleDev{});
  double dmax_all = 0.0;
  int64_t cells = 0;
  for (int s = 0; s < ctx->S; ++s) {
    SampleDev &sd = ctx->samples[s];
    const int64_t b = ctx->off[s], e = ctx->off[s + 1];
    sd.start = (int32_t)b;
    sd.count = (int32_t)(e - b);
    sd.charge_scale = sp[s].charge_scale;
    sd.hamaker = sp[s].hamaker;
    sd.temperature = sp[s].temperature;
    double dmax = 0.0;
    for (int64_t i = b; i < e; ++i) dmax = std::max(dmax, h_d[i]);
    dmax_all = std::max(dmax_all, dmax);
    const double reach = 1.25 * dmax;   // largest centre distance with a short-range force
    if (reach * 3.0 > p.L) return ctx->fail(DEPO_E_INVALID, "sample %d: particles too large for L", s);
    const double ns = (double)std::max<int64_t>(e - b, 1);
    double h = std::max(reach, std::cbrt(4.0 * p.R * p.R * p.L / ns));
    const int64_t cap = (e - b) + 64;
    int ncx, ncy;
    for (;;) {
      ncx = std::max(3, (int)std::floor(p.L / h));
      ncy = std::max(1, (int)std::floor(2.0 * p.R / h));
      if ((int64_t)ncx * ncy * ncy <= cap) break;
      h *= 1.05;
    }
    sd.ncx = ncx;
    sd.ncy = ncy;
    sd.ncz = ncy;
    sd.sr_tx = reach * (1.0 + 1e-5) * ncx / p.L;
    sd.sr_tr = reach * (1.0 + 1e-5) * ncy / (2.0 * p.R);
    sd.cell_base = (int32_t)cells;
    cells += (int64_t)ncx * ncy * ncy;
  }
  if (cells > ctx->cell_cap) return ctx->fail(DEPO_E_CAPACITY, "cell grid exceeds reserved capacity");
  ctx->n_cells = (int)cells;
  ctx->dmax_all = dmax_all;
  const double dq = dmax_all * ctx->ph.inv_ux;
  ctx->ph.near2 = dq * dq;
  return DEPO_OK;
}

// Everything on the device besides the particle state itself that a seeded or restored state
// needs: sample ids and table, neighbour counts, the tile and item lists of the pair kernels, the
// fixed-point scales and zeroed accumulators, the P3M charge mesh and histogram (zeroed) and its
// Green's function, a clear error flag.  build_samples and set_charge_bounds have run.  Synchronises.
template <class Real> depo_status upload_tables(depo_ctx *ctx, hipStream_t s) {
  State<Real> &st = state<Real>(ctx);
  const size_t N = (size_t)ctx->N;
  std::vector<int32_t> sid(N), zeros_i(N, 0);
  for (int k = 0; k < ctx->S; ++k)
    for (int64_t i = ctx->off[k]; i < ctx->off[k + 1]; ++i) sid[i] = k;
  std::vector<TileDev> tiles;
  build_tiles(ctx, tiles);
  ctx->n_tiles = (int)tiles.size();
  HIP_TRY(hipMemcpyAsync(st.sid, sid.data(), N * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(st.nbr, zeros_i.data(), N * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(st.samples, ctx->samples.data(), ctx->S * sizeof(SampleDev), hipMemcpyHostToDevice, s));
  if (!tiles.empty())
    HIP_TRY(hipMemcpyAsync(st.tiles, tiles.data(), tiles.size() * sizeof(TileDev), hipMemcpyHostToDevice, s));
  const int32_t zero[16] = {0};
  HIP_TRY(hipMemcpyAsync(st.err, zero, 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (!ctx->fp64()) {
    depo_status u = upload_fx_scale(ctx, s);
    if (u == DEPO_OK && ctx->ccfg.symmetric) u = upload_items(ctx);
    if (u != DEPO_OK) return u;
    launch_clear_int((int32_t *)ctx->sf.accx, 2 * N, s);
    launch_clear_int((int32_t *)ctx->sf.accy, 2 * N, s);
    launch_clear_int((int32_t *)ctx->sf.accz, 2 * N, s);
  }
  if (ctx->p3m_cfg) {
    if (depo_status u = upload_p3m_scale(ctx, s); u != DEPO_OK) return u;
    const P3mDev &m = ctx->pm;
    launch_clear_int((int32_t *)m.qmesh, 2 * (size_t)m.nx * m.nc * m.nc, s);
    launch_clear_int(m.counts, (size_t)m.ncx * m.ncy * m.ncy, s);
    if (!ctx->p3m_green) {
      p3m_setup_green(m, ctx->p.L, kP3mImages, sizeof(Real) == 4, s);
      ctx->p3m_green = true;
    }
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return DEPO_OK;
}

template <class Real>
depo_status do_seed(depo_ctx *ctx, const depo_sample_params *sp, const double *hx, const double *hv,
                    const double *hd, const double *hq, hipStream_t s) {
  using Pos = typename Prec<Real>::Pos;
  using SPos = typename Prec<Real>::SPos;
  const depo_params &p = ctx->p;
  const int64_t N = ctx->N;
  const int B = ctx->fp64() ? 64 : 32;
  for (int k = 0; k < ctx->S; ++k) {
    if (!std::isfinite(sp[k].charge_scale) || !std::isfinite(sp[k].hamaker) || sp[k].hamaker < 0.0 ||
        !std::isfinite(sp[k].temperature))
      return ctx->fail(DEPO_E_INVALID, "sample %d: parameters must be finite, hamaker >= 0", k);
  }
  std::vector<Pos> px(N), py(N), pz(N);
  std::vector<Real> rx(N), ry(N), rz(N);   // remainders of the positions beyond the fixed-point values
  std::vector<int32_t> zeros_i(N, 0);
  std::vector<double> zeros_d(N, 0.0);
  for (int64_t i = 0; i < N; ++i) {
    const double x = hx[3 * i], y = hx[3 * i + 1], z = hx[3 * i + 2];
    if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z))
      return ctx->fail(DEPO_E_INVALID, "particle %lld: position not finite", (long long)i);
    if (y * y + z * z >= p.R * p.R)
      return ctx->fail(DEPO_E_INVALID, "particle %lld: outside the pipe", (long long)i);
    if (!(hd[i] > 0.0) || !(hd[i] < 0.25 * p.R) || !std::isfinite(hq[i]))
      return ctx->fail(DEPO_E_INVALID, "particle %lld: diameter must be in (0, R/4), charge finite", (long long)i);
    double fx = std::fmod(x, p.L) / p.L;
    if (fx < 0.0) fx += 1.0;
    const double sc = std::ldexp(fx, B);
    const double lim = std::ldexp(1.0, B);
    if constexpr (sizeof(Pos) == 4) {
      const double k = std::nearbyint(sc);
      rx[i] = (Real)(sc - k);
      px[i] = (Pos)(uint64_t)(k >= lim ? 0.0 : k);
    } else {
      // FP64 form: 2^-64 L quanta; the remainder is below the double's resolution of x
      px[i] = sc >= lim ? (Pos)0 : (Pos)sc;
      rx[i] = 0;
    }
    const double qy = y * ctx->ph.inv_ur, qz = z * ctx->ph.inv_ur;
    const double ky = std::nearbyint(qy), kz = std::nearbyint(qz);
    py[i] = (Pos)(SPos)(int64_t)ky;
    pz[i] = (Pos)(SPos)(int64_t)kz;
    ry[i] = (Real)(qy - ky);
    rz[i] = (Real)(qz - kz);
    if (hv) {
      for (int c = 0; c < 3; ++c)
        if (!std::isfinite(hv[3 * i + c]))
          return ctx->fail(DEPO_E_INVALID, "particle %lld: velocity not finite", (long long)i);
    }
  }
  depo_status stt = build_samples(ctx, sp, hd);
  if (stt != DEPO_OK) return stt;
  ctx->sp.assign(sp, sp + ctx->S);
  ctx->ph.N = (int32_t)N;
  set_charge_bounds(ctx, hd, hq);
  State<Real> &st = state<Real>(ctx);
  const size_t nb = (size_t)N;
  HIP_TRY(hipMemcpyAsync(st.px, px.data(), nb * sizeof(Pos), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(st.py, py.data(), nb * sizeof(Pos), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(st.pz, pz.data(), nb * sizeof(Pos), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(st.rx, rx.data(), nb * sizeof(Real), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(st.ry, ry.data(), nb * sizeof(Real), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(st.rz, rz.data(), nb * sizeof(Real), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(st.d, hd, nb * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(st.qb, hq, nb * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(st.ell, zeros_d.data(), nb * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(st.dep, zeros_i.data(), nb * 4, hipMemcpyHostToDevice, s));
  {
    std::vector<int32_t> iota(nb);
    for (size_t i = 0; i < nb; ++i) iota[i] = (int32_t)i;
    HIP_TRY(hipMemcpyAsync(st.perm, iota.data(), nb * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  std::vector<Real> vbuf;
  if (hv) {
    vbuf.resize(nb);
    Real *dst[3] = {st.vx, st.vy, st.vz};
    for (int c = 0; c < 3; ++c) {
      for (size_t i = 0; i < nb; ++i) vbuf[i] = (Real)hv[3 * i + c];
      HIP_TRY(hipMemcpyAsync(dst[c], vbuf.data(), nb * sizeof(Real), hipMemcpyHostToDevice, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
  }
  const int32_t zero[16] = {0};
  HIP_TRY(hipMemcpyAsync(st.nstep, zero, 4, hipMemcpyHostToDevice, s));
  if (depo_status u = upload_tables<Real>(ctx, s); u != DEPO_OK) return u;
  // v^0 = u_f(x^0) when no velocity is given, before the initial force evaluation at x^0
  // (collision damping reads v^0 of the neighbours)
  if (!hv) launch_finish<Real>(st, ctx->ph, F_FLUID_ONLY, s);
  launch_prepare<Real>(st, ctx->ph, prepare_mode(ctx) | P_SEED, s);
  enqueue_forces<Real>(ctx, s);
  launch_finish<Real>(st, ctx->ph, hv ? 0 : F_V_FROM_FLUID, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  ctx->nstep = 0;
  ctx->seeded = true;
  ctx->drop_graph();
  return DEPO_OK;
}

template <class Real> depo_status check_err(depo_ctx *ctx, hipStream_t s) {
  uint32_t e = 0;
  HIP_TRY(hipMemcpyAsync(&e, state<Real>(ctx).err, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (e & ERR_NONFINITE) return ctx->fail(DEPO_E_NONFINITE, "a velocity or acceleration became non-finite");
  if (e & ERR_ORDER) return ctx->fail(DEPO_E_CORRUPT, "storage reorder met a cell list that does not match the state");
  return DEPO_OK;
}

template <class Real>
depo_status do_read(depo_ctx *ctx, double *hx, double *hv, double *ha, int32_t *hdep, int32_t *hnb, hipStream_t s) {
  using Pos = typename Prec<Real>::Pos;
  const State<Real> &st = state<Real>(ctx);
  const size_t N = (size_t)ctx->N;
  // slot k holds particle perm[k] of the caller's order
  std::vector<int32_t> perm(N);
  if (N) HIP_TRY(hipMemcpyAsync(perm.data(), st.perm, N * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (size_t k = 0; k < N; ++k)
    if (perm[k] < 0 || (size_t)perm[k] >= N) return ctx->fail(DEPO_E_CORRUPT, "particle permutation corrupted");
  if (hx) {
    std::vector<Pos> p(3 * N);
    std::vector<Real> r(3 * N);
    HIP_TRY(hipMemcpyAsync(p.data(), st.px, N * sizeof(Pos), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(p.data() + N, st.py, N * sizeof(Pos), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(p.data() + 2 * N, st.pz, N * sizeof(Pos), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(r.data(), st.rx, N * sizeof(Real), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(r.data() + N, st.ry, N * sizeof(Real), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(r.data() + 2 * N, st.rz, N * sizeof(Real), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (size_t i = 0; i < N; ++i) {
      double x = ((double)p[i] + (double)r[i]) * ctx->ph.ux;
      if (x < 0.0) x += ctx->p.L;
      if (x >= ctx->p.L) x -= ctx->p.L;
      double *o = hx + 3 * (size_t)perm[i];
      o[0] = x;
      if constexpr (sizeof(Pos) == 4) {
        o[1] = ((double)(int32_t)p[N + i] + (double)r[N + i]) * ctx->ph.ur;
        o[2] = ((double)(int32_t)p[2 * N + i] + (double)r[2 * N + i]) * ctx->ph.ur;
      } else {
        o[1] = ((double)(int64_t)p[N + i] + (double)r[N + i]) * ctx->ph.ur;
        o[2] = ((double)(int64_t)p[2 * N + i] + (double)r[2 * N + i]) * ctx->ph.ur;
      }
    }
  }
  auto vec3 = [&](double *h, Real *a, Real *b, Real *c) -> depo_status {
    std::vector<Real> t(3 * N);
    HIP_TRY(hipMemcpyAsync(t.data(), a, N * sizeof(Real), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(t.data() + N, b, N * sizeof(Real), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(t.data() + 2 * N, c, N * sizeof(Real), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (size_t i = 0; i < N; ++i)
      for (int k = 0; k < 3; ++k) h[3 * (size_t)perm[i] + k] = (double)t[k * N + i];
    return DEPO_OK;
  };
  auto ints = [&](int32_t *h, const int32_t *a) -> depo_status {
    std::vector<int32_t> t(N);
    if (N) HIP_TRY(hipMemcpyAsync(t.data(), a, N * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (size_t i = 0; i < N; ++i) h[perm[i]] = t[i];
    return DEPO_OK;
  };
  depo_status r;
  if (hv && (r = vec3(hv, st.vx, st.vy, st.vz)) != DEPO_OK) return r;
  if (ha && (r = vec3(ha, st.ax, st.ay, st.az)) != DEPO_OK) return r;
  if (hdep && (r = ints(hdep, st.dep)) != DEPO_OK) return r;
  if (hnb && (r = ints(hnb, st.nbr)) != DEPO_OK) return r;
  return check_err<Real>(ctx, s);
}

template <class Real> depo_status do_tally(depo_ctx *ctx, depo_tally *out, hipStream_t s) {
  const State<Real> &st = state<Real>(ctx);
  launch_tally<Real>(st, ctx->ph, ctx->nstep, s);
  HIP_TRY(hipGetLastError());
  std::vector<double> t((size_t)ctx->S * 8);
  HIP_TRY(hipMemcpyAsync(t.data(), st.tally, t.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double us = ctx->p.re_tau * ctx->p.nu / ctx->p.R;
  for (int k = 0; k < ctx->S; ++k) {
    const double *r = &t[(size_t)k * 8];
    depo_tally &o = out[k];
    o.m_dep = r[0];
    o.n_dep = (int64_t)std::llround(r[1]);
    o.m_alive_dt = r[2] * ctx->p.dt;
    o.t = ctx->nstep * ctx->p.dt;
    o.v_dep = o.m_alive_dt > 0.0 ? 0.5 * ctx->p.R * o.m_dep / o.m_alive_dt : 0.0;
    o.v_dep_plus = o.v_dep / us;
    o.v_dep_se = o.m_dep > 0.0 ? o.v_dep * std::sqrt(r[3]) / o.m_dep : 0.0;
    o.j_soft = r[4];
    o.n_alive = (int64_t)std::llround(r[5]);
    // capture efficiency, Eq. CE
    o.ce = ctx->p.u_bulk > 0.0 ? 4.0 * ctx->p.L / (2.0 * ctx->p.R) * (us / ctx->p.u_bulk) * o.v_dep_plus : 0.0;
  }
  return check_err<Real>(ctx, s);
}

// checkpoint payload: positions (fixed point, then remainders), velocities, accelerations,
// fluid velocities, d, qbase, ell, dep, per-sample parameters
// (all in storage order), then the storage permutation
constexpr uint32_t kBlobVersion = 3;
template <class Real> size_t blob_payload(const depo_ctx *ctx) {
  const size_t N = (size_t)ctx->N;
  return N * (3 * sizeof(typename Prec<Real>::Pos) + 12 * sizeof(Real) + 3 * 8 + 4 + 4) +
         (size_t)ctx->S * sizeof(depo_sample_params);
}

template <class Real> depo_status do_download(depo_ctx *ctx, void *blob, size_t bytes, hipStream_t s) {
  using Pos = typename Prec<Real>::Pos;
  const State<Real> &st = state<Real>(ctx);
  const size_t N = (size_t)ctx->N;
  const size_t pay = blob_payload<Real>(ctx);
  if (bytes != sizeof(BlobHeader) + pay) return ctx->fail(DEPO_E_INVALID, "blob size must be %zu", sizeof(BlobHeader) + pay);
  char *p = (char *)blob + sizeof(BlobHeader);
  auto get = [&](const void *src, size_t n) -> depo_status {
    HIP_TRY(hipMemcpyAsync(p, src, n, hipMemcpyDeviceToHost, s));
    p += n;
    return DEPO_OK;
  };
  depo_status r;
  for (const Pos *a : {st.px, st.py, st.pz})
    if ((r = get(a, N * sizeof(Pos))) != DEPO_OK) return r;
  for (const Real *a : {st.rx, st.ry, st.rz, st.vx, st.vy, st.vz, st.ax, st.ay, st.az, st.ux, st.uy, st.uz})
    if ((r = get(a, N * sizeof(Real))) != DEPO_OK) return r;
  for (const double *a : {st.d, st.qb, st.ell})
    if ((r = get(a, N * 8)) != DEPO_OK) return r;
  if ((r = get(st.dep, N * 4)) != DEPO_OK) return r;
  if ((r = get(st.perm, N * 4)) != DEPO_OK) return r;
  HIP_TRY(hipStreamSynchronize(s));
  std::memcpy(p, ctx->sp.data(), ctx->S * sizeof(depo_sample_params));
  BlobHeader h{};
  std::memcpy(h.magic, "DEPOCKPT", 8);
  h.version = kBlobVersion;
  h.real_bytes = (uint32_t)ctx->p.real_bytes;
  h.n = ctx->N;
  h.s = ctx->S;
  h.nstep = ctx->nstep;
  h.payload = pay;
  h.crc = crc32_update(0, (const char *)blob + sizeof(BlobHeader), pay);
  std::memcpy(blob, &h, sizeof h);
  return check_err<Real>(ctx, s);
}

template <class Real> depo_status do_upload(depo_ctx *ctx, const void *blob, size_t bytes, hipStream_t s) {
  using Pos = typename Prec<Real>::Pos;
  const State<Real> &st = state<Real>(ctx);
  const size_t N = (size_t)ctx->N;
  const size_t pay = blob_payload<Real>(ctx);
  if (bytes != sizeof(BlobHeader) + pay) return ctx->fail(DEPO_E_CORRUPT, "blob size mismatch");
  BlobHeader h;
  std::memcpy(&h, blob, sizeof h);
  if (std::memcmp(h.magic, "DEPOCKPT", 8) != 0 || h.version != kBlobVersion || h.real_bytes != (uint32_t)ctx->p.real_bytes ||
      h.n != ctx->N || h.s != ctx->S || h.payload != pay || h.nstep < 0)
    return ctx->fail(DEPO_E_CORRUPT, "blob header does not match this context");
  const char *p = (const char *)blob + sizeof(BlobHeader);
  if (crc32_update(0, p, pay) != h.crc) return ctx->fail(DEPO_E_CORRUPT, "blob CRC mismatch");
  {
    // the storage permutation must be one (it indexes the host arrays of depo_read_particles)
    std::vector<int32_t> perm(N);
    std::memcpy(perm.data(), p + N * (3 * sizeof(Pos) + 12 * sizeof(Real) + 3 * 8 + 4), N * 4);
    std::vector<char> seen(N, 0);
    for (size_t k = 0; k < N; ++k) {
      if (perm[k] < 0 || (size_t)perm[k] >= N || seen[perm[k]])
        return ctx->fail(DEPO_E_CORRUPT, "blob permutation invalid");
      seen[perm[k]] = 1;
    }
  }
  // per-sample parameters and diameters rebuild the sample table
  const char *q = p + N * (3 * sizeof(Pos) + 12 * sizeof(Real));
  std::vector<double> d(N);
  std::memcpy(d.data(), q, N * 8);
  std::vector<depo_sample_params> sp(ctx->S);
  std::memcpy(sp.data(), p + pay - ctx->S * sizeof(depo_sample_params), ctx->S * sizeof(depo_sample_params));
  depo_status r = build_samples(ctx, sp.data(), d.data());
  if (r != DEPO_OK) return r;
  ctx->sp = sp;
  ctx->ph.N = (int32_t)N;
  {
    std::vector<double> qb(N);
    std::memcpy(qb.data(), q + N * 8, N * 8);
    set_charge_bounds(ctx, d.data(), qb.data());
  }
  auto put = [&](void *dst, size_t n) -> depo_status {
    HIP_TRY(hipMemcpyAsync(dst, p, n, hipMemcpyHostToDevice, s));
    p += n;
    return DEPO_OK;
  };
  for (Pos *a : {st.px, st.py, st.pz})
    if ((r = put(a, N * sizeof(Pos))) != DEPO_OK) return r;
  for (Real *a : {st.rx, st.ry, st.rz, st.vx, st.vy, st.vz, st.ax, st.ay, st.az, st.ux, st.uy, st.uz})
    if ((r = put(a, N * sizeof(Real))) != DEPO_OK) return r;
  for (double *a : {st.d, st.qb, st.ell})
    if ((r = put(a, N * 8)) != DEPO_OK) return r;
  if ((r = put(st.dep, N * 4)) != DEPO_OK) return r;
  if ((r = put(st.perm, N * 4)) != DEPO_OK) return r;
  const int32_t ns = h.nstep;
  HIP_TRY(hipMemcpyAsync(st.nstep, &ns, 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  // the tables a context that was never seeded lacks (sample ids, pair-kernel work lists, ...)
  if ((r = upload_tables<Real>(ctx, s)) != DEPO_OK) return r;
  // refresh the Coulomb source radii and the cell list (a storage reorder reads it)
  launch_prepare<Real>(st, ctx->ph, P_SEED | P_COULOMB | (short_range_on(ctx) ? P_CELLS : 0), s);
  if (short_range_on(ctx)) launch_cells<Real>(st, ctx->ph, ctx->n_cells, (ctx->n_cells + 1023) / 1024, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  ctx->nstep = h.nstep;
  ctx->seeded = true;
  ctx->drop_graph();
  return DEPO_OK;
}

}  // namespace

// ---------------------------------------------------------------- adjoint

template <class Real> struct AdjPlan {
  std::vector<TapeEntry<Real>> ckpt, tape;
  TapeEntry<Real> fin{};
  AdjState<Real> ad{};
  // raw Coulomb sums [n_steps - n_ckpt][3][N] of the steps the reverse sweep recomputes (Coulomb
  // on): step c*seg_len + j of segment c, j < seg_len - 1, sits at entry c*(seg_len - 1) + j
  Real *ctape = nullptr;
};

template <class Real>
size_t carve_adjoint(const depo_ctx *ctx, char *base, int n_steps, int n_ckpt, int seg_len, AdjPlan<Real> &pl) {
  using Pos = typename Prec<Real>::Pos;
  const size_t N = (size_t)std::max<int64_t>(ctx->N, 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + o : nullptr;
    o = align_up(o + bytes);
    return p;
  };
  auto entry = [&](bool ell) {
    TapeEntry<Real> t{};
    t.px = (Pos *)take(N * sizeof(Pos)); t.py = (Pos *)take(N * sizeof(Pos)); t.pz = (Pos *)take(N * sizeof(Pos));
    Real **r[] = {&t.rx, &t.ry, &t.rz, &t.vx, &t.vy, &t.vz, &t.ax, &t.ay, &t.az, &t.ux, &t.uy, &t.uz, &t.cx, &t.cy, &t.cz};
    for (Real **q : r) *q = (Real *)take(N * sizeof(Real));
    t.ell = ell ? (double *)take(N * 8) : nullptr;
    return t;
  };
  pl.ckpt.clear();
  pl.tape.clear();
  for (int k = 0; k < n_ckpt; ++k) pl.ckpt.push_back(entry(false));
  // tape[k] holds S_{k+1} of a segment; its last state is the next checkpoint (or the final state)
  for (int k = 0; k < seg_len - 1; ++k) pl.tape.push_back(entry(false));
  pl.fin = entry(true);
  AdjState<Real> &a = pl.ad;
  a.lam_ell = (Real *)take(N * sizeof(Real));
  Real **arrs[] = {&a.xb[0], &a.xb[1], &a.xb[2], &a.vb[0], &a.vb[1], &a.vb[2], &a.ab[0], &a.ab[1], &a.ab[2],
                   &a.ub[0], &a.ub[1], &a.ub[2], &a.xp[0], &a.xp[1], &a.xp[2], &a.vpb[0], &a.vpb[1], &a.vpb[2],
                   &a.vp[0], &a.vp[1], &a.vp[2], &a.xc[0], &a.xc[1], &a.xc[2], &a.xs[0], &a.xs[1], &a.xs[2],
                   &a.vs[0], &a.vs[1], &a.vs[2]};
  for (Real **q : arrs) *q = (Real *)take(N * sizeof(Real));
  a.gs = (double *)take(N * 8);
  a.gA = (double *)take(N * 8);
  a.rec = (JAdj<Real> *)take(N * sizeof(JAdj<Real>));
  a.weights = (double *)take((size_t)ctx->S * 8);
  a.out = (double *)take((size_t)ctx->S * 2 * 8);
  const size_t n_sums = (size_t)(n_steps - n_ckpt);
  pl.ctape = (ctx->p.flags & DEPO_COULOMB) && n_sums ? (Real *)take(n_sums * 3 * N * sizeof(Real)) : nullptr;
  return o;
}

// Forward run of the adjoint: the n steps from the seeded state with checkpoints every ce steps and
// the Coulomb tape, into the caller's workspace; leaves the context at step n and records the
// pending reverse sweep.
template <class Real>
depo_status do_adjoint_forward(depo_ctx *ctx, int n, int ce, void *dws, size_t bytes, hipStream_t s) {
  AdjPlan<Real> pl;
  const int K = (n + ce - 1) / ce;
  const size_t need = carve_adjoint<Real>(ctx, nullptr, n, K, ce, pl);
  if (bytes < need) return ctx->fail(DEPO_E_CAPACITY, "adjoint workspace needs %zu bytes", need);
  carve_adjoint<Real>(ctx, (char *)dws, n, K, ce, pl);
  const State<Real> &st = state<Real>(ctx);
  const int N = (int)ctx->N;
  const bool coul = (ctx->p.flags & DEPO_COULOMB) != 0;
  const size_t nb = (size_t)N * sizeof(Real);
  // the raw Coulomb sums of a step to its Coulomb-tape entry
  auto sums_to_tape = [&](int k) -> hipError_t {
    Real *t = pl.ctape + (size_t)k * 3 * N;
    hipError_t e = hipMemcpyAsync(t, st.cx, nb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(t + N, st.cy, nb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(t + 2 * (size_t)N, st.cz, nb, hipMemcpyDeviceToDevice, s);
    return e;
  };
  // forward run with checkpoints every ce steps; the pair sums of every step that does not end
  // at a checkpoint (or at the final state) are kept, so that the per-segment recomputation
  // of the reverse sweep runs only the O(N) kernels
  for (int k = 0; k < n; ++k) {
    if (k % ce == 0) launch_tape_store<Real>(st, pl.ckpt[k / ce], N, false, s);
    // the same step as depo_step (the captured graph, when enabled); the step counter is set below
    if (depo_status r = run_steps<Real>(ctx, 1, s); r != DEPO_OK) return r;
    if (coul && k % ce != ce - 1 && k != n - 1) HIP_TRY(sums_to_tape((k / ce) * (ce - 1) + k % ce));
  }
  launch_tape_store<Real>(st, pl.fin, N, true, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  ctx->nstep = n;
  ctx->adj_pending = true;
  ctx->adj_gen = ctx->gen;
  ctx->adj_n = n;
  ctx->adj_ce = ce;
  ctx->adj_ws = dws;
  ctx->adj_bytes = bytes;
  return check_err<Real>(ctx, s);
}

// Reverse sweep over the workspace of the pending forward run; the context ends at the forward's
// final state.
template <class Real> depo_status do_adjoint_backward(depo_ctx *ctx, const double *hw, double *hg, hipStream_t s) {
  const int n = ctx->adj_n, ce = ctx->adj_ce;
  AdjPlan<Real> pl;
  const int K = (n + ce - 1) / ce;
  carve_adjoint<Real>(ctx, (char *)ctx->adj_ws, n, K, ce, pl);
  const State<Real> &st = state<Real>(ctx);
  const Phys &ph = ctx->ph;
  const int N = (int)ctx->N;
  const bool coul = (ctx->p.flags & DEPO_COULOMB) != 0, sr = short_range_on(ctx);
  double wmax = 0.0;
  for (int k = 0; k < ctx->S; ++k) wmax = std::max(wmax, std::fabs(hw[k]));
  const double mmax = ph.mass_coef * ctx->dmax_all * ctx->dmax_all * ctx->dmax_all;
  const double scale = (wmax > 0.0 && mmax > 0.0) ? 1.0 / (wmax * mmax) : 1.0;
  HIP_TRY(hipMemcpyAsync(pl.ad.weights, hw, ctx->S * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  const size_t nb = (size_t)N * sizeof(Real);
  // the raw Coulomb sums of a step back from its Coulomb-tape entry
  auto sums_from_tape = [&](int k) -> hipError_t {
    const Real *t = pl.ctape + (size_t)k * 3 * N;
    hipError_t e = hipMemcpyAsync(st.cx, t, nb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(st.cy, t + N, nb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(st.cz, t + 2 * (size_t)N, nb, hipMemcpyDeviceToDevice, s);
    return e;
  };
  launch_adj_init<Real>(st, ph, pl.ad, pl.ad.weights, scale, s);
  auto rebuild_cells = [&]() {
    if (sr) {
      launch_prepare<Real>(st, ph, P_CELLS, s);
      launch_cells<Real>(st, ph, ctx->n_cells, (ctx->n_cells + 1023) / 1024, s);
    }
  };
  for (int seg = K - 1; seg >= 0; --seg) {
    const int len = std::min(ce, n - seg * ce);
    // the segment's last state is the next checkpoint (or the final state): the forward is
    // bitwise deterministic, so only the len - 1 states before it are recomputed
    const TapeEntry<Real> &last = seg + 1 < K ? pl.ckpt[seg + 1] : pl.fin;
    if (len > 1) {
      launch_tape_load<Real>(st, pl.ckpt[seg], N, false, s);
      for (int k = 0; k < len - 1; ++k) {
        // the step with its pair sums read from the Coulomb tape (bitwise what the pair kernel gave)
        launch_prepare<Real>(st, ph, prepare_mode(ctx) | P_KICK_DRIFT, s);
        if (sr) launch_cells<Real>(st, ph, ctx->n_cells, (ctx->n_cells + 1023) / 1024, s);
        if (coul) HIP_TRY(sums_from_tape(seg * (ce - 1) + k));
        if (sr) launch_short_range<Real>(st, ph, ctx->n_cells, s);
        launch_finish<Real>(st, ph, F_KICK, s);
        launch_tape_store<Real>(st, pl.tape[k], N, false, s);
      }
    }
    for (int k = len - 1; k >= 0; --k) {
      const TapeEntry<Real> &s0 = k == 0 ? pl.ckpt[seg] : pl.tape[k - 1];
      const TapeEntry<Real> &s1 = k == len - 1 ? last : pl.tape[k];
      launch_tape_load<Real>(st, s1, N, false, s);
      rebuild_cells();
      launch_adj_post<Real>(st, ph, s0, s1, pl.ad, 0, s);
      if (coul) {
        if constexpr (std::is_same<Real, float>::value) {
          if (ctx->ccfg.symmetric)
            launch_coulomb_vjp_sym(ctx->sf, ph, pl.ad, ctx->n_diag, ctx->n_off, ctx->ccfg, s);
          else
            launch_coulomb_vjp<Real>(st, ph, pl.ad, ctx->n_tiles, s);
        } else {
          launch_coulomb_vjp<Real>(st, ph, pl.ad, ctx->n_tiles, s);
        }
      }
      if (sr) launch_short_range_vjp<Real>(st, ph, pl.ad, ctx->n_cells, 0, s);
      launch_adj_pre<Real>(st, ph, s0, pl.ad, coul, sr, s);
    }
  }
  // the seed's force evaluation a^0 = F(x^0, v^0; params)
  launch_tape_load<Real>(st, pl.ckpt[0], N, false, s);
  rebuild_cells();
  launch_adj_post<Real>(st, ph, pl.ckpt[0], pl.ckpt[0], pl.ad, ADJ_SEED, s);
  if (sr) launch_short_range_vjp<Real>(st, ph, pl.ad, ctx->n_cells, ADJ_SEED, s);
  launch_adj_reduce<Real>(st, ph, pl.ad, pl.ad.out, s);
  // back to the state after the forward run
  launch_tape_load<Real>(st, pl.fin, N, true, s);
  HIP_TRY(hipGetLastError());
  std::vector<double> out((size_t)ctx->S * 2);
  HIP_TRY(hipMemcpyAsync(out.data(), pl.ad.out, out.size() * 8, hipMemcpyDeviceToHost, s));
  const int32_t ns = n;
  HIP_TRY(hipMemcpyAsync(st.nstep, &ns, 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  ctx->nstep = n;
  for (int k = 0; k < ctx->S; ++k) {
    hg[3 * k + 0] = out[2 * k] / scale;
    hg[3 * k + 1] = out[2 * k + 1] / scale;
    hg[3 * k + 2] = 0.0;   // temperature enters only the rebound law, which the smoothed tally disables
  }
  return check_err<Real>(ctx, s);
}

// ---------------------------------------------------------------- allocation-free adjoint workspace
//
// depo_adjoint_noalloc keeps its adjoint workspace in this file-scope device array instead of
// caller memory.  Each GPU the library runs on holds its own copy until the process ends.  In host
// code the array's name is not a device address: the address is taken per device with
// hipGetSymbolAddress on the first call on that device and only that pointer is used afterwards.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};
}  // namespace

// Device address of this GPU's scratch array (the current device), taken once per device.
static depo_status scratch_address(depo_ctx *ctx, void **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return ctx->fail(DEPO_E_INVALID, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return ctx->fail(DEPO_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DEPO_OK;
}

#define DISPATCH(fn, ...) (ctx->fp64() ? fn<double>(__VA_ARGS__) : fn<float>(__VA_ARGS__))

extern "C" {

const char *depo_status_string(int status) {
  switch (status) {
    case DEPO_OK: return "DEPO_OK";
    case DEPO_E_INVALID: return "DEPO_E_INVALID";
    case DEPO_E_STATE: return "DEPO_E_STATE";
    case DEPO_E_HIP: return "DEPO_E_HIP";
    case DEPO_E_NONFINITE: return "DEPO_E_NONFINITE";
    case DEPO_E_CAPACITY: return "DEPO_E_CAPACITY";
    case DEPO_E_CORRUPT: return "DEPO_E_CORRUPT";
    default: return "DEPO_E_UNKNOWN";
  }
}

depo_status depo_create(const depo_params *p, depo_ctx **out) {
  if (!out) return DEPO_E_INVALID;
  *out = nullptr;
  if (!p) return DEPO_E_INVALID;
  const bool ok = finite_pos(p->R) && finite_pos(p->L) && finite_pos(p->nu) && finite_pos(p->rho_f) &&
                  finite_pos(p->rho_p) && finite_pos(p->dt) && finite_pos(p->re_tau) && finite_pos(p->e_pp) &&
                  p->e_pp <= 1.0 && p->tau_col_steps >= 1 && (p->real_bytes == 4 || p->real_bytes == 8) &&
                  finite_pos(p->delta_min) && finite_pos(p->kr_over_k) && finite_pos(p->eps0) &&
                  std::isfinite(p->g_body[0]) && std::isfinite(p->g_body[1]) && std::isfinite(p->g_body[2]) &&
                  finite_pos(p->E_young) && finite_pos(p->delta_c) && std::isfinite(p->acont_coef) &&
                  p->acont_coef >= 0.0 && (p->flags & ~kKnownFlags) == 0 && p->reserved == 0 &&
                  std::isfinite(p->u_bulk) && p->u_bulk >= 0.0 &&
                  (!(p->flags & DEPO_SOFT_TALLY) || (finite_pos(p->soft_eps) && finite_pos(p->soft_tau)));
  if (!ok) return DEPO_E_INVALID;
  depo_ctx *ctx = new depo_ctx();
  ctx->p = *p;
  if (ctx->fp64()) ctx->ccfg = CoulombConfig{1, 4, 16, false};
  fill_phys(ctx);
  *out = ctx;
  return DEPO_OK;
}

void depo_destroy(depo_ctx *ctx) {
  if (!ctx) return;
  ctx->drop_graph();
  if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
  if (ctx->cap_side) hipStreamDestroy(ctx->cap_side);
  if (ctx->ev_fork) hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) hipEventDestroy(ctx->ev_join);
  delete ctx;
}

const char *depo_last_error(const depo_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

depo_status depo_set_layout(depo_ctx *ctx, int32_t n_samples, const int64_t *offsets, int32_t nx, int32_t ny,
                            int32_t nz) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (n_samples < 1 || !offsets) return ctx->fail(DEPO_E_INVALID, "need n_samples >= 1 and offsets");
  if (offsets[0] != 0) return ctx->fail(DEPO_E_INVALID, "offsets[0] must be 0");
  for (int s = 0; s < n_samples; ++s)
    if (offsets[s + 1] < offsets[s]) return ctx->fail(DEPO_E_INVALID, "offsets must be non-decreasing");
  if (offsets[n_samples] > kMaxN) return ctx->fail(DEPO_E_INVALID, "at most 2^26 particles");
  for (int v : {nx, ny, nz})
    if (v < 4 || v > 4096) return ctx->fail(DEPO_E_INVALID, "field grid must be 4..4096 nodes per axis");
  ctx->drop_graph();
  ctx->has_layout = true;
  ctx->bound = ctx->field_ready = ctx->seeded = false;
  ctx->ws = nullptr;
  ctx->S = n_samples;
  ctx->off.assign(offsets, offsets + n_samples + 1);
  ctx->N = offsets[n_samples];
  ctx->nx = nx;
  ctx->ny = ny;
  ctx->nz = nz;
  ctx->cell_cap = ctx->N + 64LL * n_samples;
  ctx->scan_blocks = (int)((ctx->cell_cap + 1023) / 1024);
  int tiles = 0;
  for (int s = 0; s < n_samples; ++s) tiles += (int)((offsets[s + 1] - offsets[s] + 63) / 64);
  ctx->tile_cap = tiles;
  // symmetric pair kernel (FP32): room for the items of the smallest item size whose list stays
  // within kMaxItems; the FP32 default falls back to the one-sided kernel beyond that
  ctx->sym_cap = 0;
  if (!ctx->fp64()) {
    for (int64_t T = kSymTileMin; T <= 1024 && ctx->sym_cap == 0; T *= 2) {
      const int64_t k = count_items(ctx->off, T);
      if (k <= kMaxItems) ctx->sym_cap = k;
    }
    if (ctx->ccfg.symmetric && count_items(ctx->off, coulomb_sym_tile(ctx->ccfg)) > ctx->sym_cap)
      ctx->ccfg = kDefaultOneSided;
  }
  if (ctx->p3m_cfg) {
    if (n_samples != 1) {
      ctx->has_layout = false;
      return ctx->fail(DEPO_E_INVALID, "P3M electrostatics needs a single-sample layout");
    }
    P3mDev &m = ctx->pm;
    m = P3mDev{};
    m.nx = ctx->p3m_nx;
    m.nc = ctx->p3m_nc;
    m.P = 2 * m.nc;
    m.hx = ctx->p.L / m.nx;
    m.hy = 2.0 * ctx->p.R / (m.nc - 3);
    m.alpha = ctx->p3m_alpha_h / std::max(m.hx, m.hy);
    m.rmax = ctx->p3m_rmax_alpha / m.alpha;
    m.ncx = (int)std::floor(ctx->p.L / m.rmax);
    m.ncy = std::max(1, (int)std::floor(2.0 * ctx->p.R / m.rmax));
    if (m.ncx < 3 || (int64_t)m.ncx * m.ncy * m.ncy > (1 << 22)) {
      ctx->has_layout = false;
      return ctx->fail(DEPO_E_INVALID, "P3M cutoff %g m: need L >= 3 r_max and at most 2^22 short-range cells", m.rmax);
    }
    ctx->p3m_green = false;
  }
  fill_phys(ctx);
  ctx->ws_need = ctx->fp64() ? carve<double>(ctx, nullptr, ctx->sd) : carve<float>(ctx, nullptr, ctx->sf);
  return DEPO_OK;
}

depo_status depo_workspace_bytes(const depo_ctx *ctx, size_t *bytes) {
  if (!ctx || !bytes) return DEPO_E_INVALID;
  if (!ctx->has_layout) return DEPO_E_STATE;
  *bytes = ctx->ws_need;
  return DEPO_OK;
}

depo_status depo_bind(depo_ctx *ctx, void *d_work, size_t bytes) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (!ctx->has_layout) return ctx->fail(DEPO_E_STATE, "set the layout before binding");
  if (!d_work || ((uintptr_t)d_work % kAlign) != 0) return ctx->fail(DEPO_E_INVALID, "workspace must be 256-byte aligned");
  if (bytes < ctx->ws_need) return ctx->fail(DEPO_E_CAPACITY, "workspace needs %zu bytes", ctx->ws_need);
  ctx->drop_graph();
  ctx->ws = (char *)d_work;
  if (ctx->fp64()) carve<double>(ctx, ctx->ws, ctx->sd); else carve<float>(ctx, ctx->ws, ctx->sf);
  ctx->p3m_green = false;
  int32_t *counts = ctx->fp64() ? ctx->sd.cell_count : ctx->sf.cell_count;
  launch_clear_int(counts, (size_t)ctx->cell_cap, nullptr);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(nullptr));
  ctx->bound = true;
  ctx->field_ready = ctx->seeded = false;
  return DEPO_OK;
}

depo_status depo_init_field(depo_ctx *ctx, const double *h_uvw, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (!ctx->bound) return ctx->fail(DEPO_E_STATE, "bind a workspace first");
  if (!h_uvw) return ctx->fail(DEPO_E_INVALID, "null field");
  depo_status r = DISPATCH(do_init_field, ctx, h_uvw, (hipStream_t)stream);
  if (r == DEPO_OK) ctx->field_ready = true;
  return r;
}

depo_status depo_seed(depo_ctx *ctx, const depo_sample_params *sp, const double *h_x3, const double *h_v3,
                      const double *h_d, const double *h_qbase, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (!ctx->bound || !ctx->field_ready) return ctx->fail(DEPO_E_STATE, "bind a workspace and upload the field first");
  if (!sp || (ctx->N > 0 && (!h_x3 || !h_d || !h_qbase))) return ctx->fail(DEPO_E_INVALID, "null input array");
  ctx->seeded = false;
  return DISPATCH(do_seed, ctx, sp, h_x3, h_v3, h_d, h_qbase, (hipStream_t)stream);
}

depo_status depo_set_sample_params(depo_ctx *ctx, const depo_sample_params *sp, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (!ctx->seeded) return ctx->fail(DEPO_E_STATE, "seed first");
  if (!sp) return ctx->fail(DEPO_E_INVALID, "null sample parameters");
  for (int k = 0; k < ctx->S; ++k) {
    if (!std::isfinite(sp[k].charge_scale) || !std::isfinite(sp[k].hamaker) || sp[k].hamaker < 0.0 ||
        !std::isfinite(sp[k].temperature))
      return ctx->fail(DEPO_E_INVALID, "sample %d: parameters must be finite, hamaker >= 0", k);
  }
  for (int k = 0; k < ctx->S; ++k) {
    ctx->samples[k].charge_scale = sp[k].charge_scale;
    ctx->samples[k].hamaker = sp[k].hamaker;
    ctx->samples[k].temperature = sp[k].temperature;
  }
  ctx->sp.assign(sp, sp + ctx->S);
  if (depo_status u = upload_fx_scale(ctx, (hipStream_t)stream); u != DEPO_OK) return u;
  if (depo_status u = upload_p3m_scale(ctx, (hipStream_t)stream); u != DEPO_OK) return u;
  SampleDev *dst = ctx->fp64() ? ctx->sd.samples : ctx->sf.samples;
  HIP_TRY(hipMemcpyAsync(dst, ctx->samples.data(), ctx->S * sizeof(SampleDev), hipMemcpyHostToDevice,
                         (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return DEPO_OK;
}

depo_status depo_step(depo_ctx *ctx, int32_t n_steps, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (!ctx->seeded) return ctx->fail(DEPO_E_STATE, "seed first");
  if (n_steps < 0) return ctx->fail(DEPO_E_INVALID, "n_steps must be >= 0");
  if ((int64_t)ctx->nstep + n_steps > (int64_t)INT32_MAX - 1) return ctx->fail(DEPO_E_INVALID, "step counter overflow");
  return DISPATCH(run_steps, ctx, n_steps, (hipStream_t)stream);
}

depo_status depo_step_timed(depo_ctx *ctx, int32_t n_steps, depo_stream stream, double *h_phase_ms) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (!ctx->seeded) return ctx->fail(DEPO_E_STATE, "seed first");
  if (n_steps < 1 || n_steps > 100000 || !h_phase_ms) return ctx->fail(DEPO_E_INVALID, "need 1..100000 steps and an output array");
  if ((int64_t)ctx->nstep + n_steps > (int64_t)INT32_MAX - 1) return ctx->fail(DEPO_E_INVALID, "step counter overflow");
  return DISPATCH(run_steps_timed, ctx, n_steps, (hipStream_t)stream, h_phase_ms);
}

depo_status depo_set_kernel_config(depo_ctx *ctx, int32_t targets_per_lane, int32_t waves, int32_t block,
                                   int32_t mode, int32_t use_graph) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (mode == DEPO_PAIR_P3M) {
    if (!ctx->p3m_cfg) return ctx->fail(DEPO_E_INVALID, "P3M is not configured (depo_set_p3m before the layout)");
    ctx->p3m_use = true;
    ctx->use_graph = use_graph != 0;
    ctx->drop_graph();
    return DEPO_OK;
  }
  if (mode < DEPO_PAIR_PLAIN || mode > DEPO_PAIR_SYMMETRIC_INT || mode == DEPO_PAIR_P3M)
    return ctx->fail(DEPO_E_INVALID, "unknown pair-kernel mode %d", mode);
  const bool sym = mode == DEPO_PAIR_SYMMETRIC || mode == DEPO_PAIR_SYMMETRIC_INT;
  CoulombConfig c{targets_per_lane, waves, block, mode != DEPO_PAIR_PLAIN, sym, mode == DEPO_PAIR_SYMMETRIC_INT};
  if (c.int_rec && !(ctx->p.L >= 2.0 * ctx->p.R))
    return ctx->fail(DEPO_E_INVALID, "integer source records need L >= 2R (y and z within 2^31 x quanta)");
  if (c.symmetric) {
    if (ctx->fp64() || !coulomb_sym_supported(c))
      return ctx->fail(DEPO_E_INVALID, "unsupported symmetric pair-kernel configuration (%d, %d, %d)", targets_per_lane,
                       waves, block);
    if (coulomb_sym_tile(c) < kSymTileMin)
      return ctx->fail(DEPO_E_INVALID, "symmetric items must hold at least %d targets", kSymTileMin);
    if (ctx->has_layout && count_items(ctx->off, coulomb_sym_tile(c)) > ctx->sym_cap)
      return ctx->fail(DEPO_E_INVALID, "too many symmetric work items for this layout; use larger items");
  } else if (!coulomb_config_supported(ctx->p.real_bytes, c)) {
    return ctx->fail(DEPO_E_INVALID, "unsupported pair-kernel configuration (%d, %d, %d, %d)", targets_per_lane, waves,
                     block, mode);
  }
  ctx->ccfg = c;
  ctx->p3m_use = false;
  ctx->use_graph = use_graph != 0;
  ctx->drop_graph();
  set_record_format(ctx);
  if (ctx->seeded) {
    std::vector<TileDev> tiles;
    build_tiles(ctx, tiles);
    ctx->n_tiles = (int)tiles.size();
    TileDev *dst = ctx->fp64() ? ctx->sd.tiles : ctx->sf.tiles;
    HIP_TRY(hipMemcpy(dst, tiles.data(), tiles.size() * sizeof(TileDev), hipMemcpyHostToDevice));
    if (c.symmetric) return upload_items(ctx);
  }
  return DEPO_OK;
}

depo_status depo_eval_accel(depo_ctx *ctx, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (!ctx->seeded) return ctx->fail(DEPO_E_STATE, "seed first");
  hipStream_t s = (hipStream_t)stream;
  if (ctx->fp64()) {
    launch_prepare<double>(ctx->sd, ctx->ph, prepare_mode(ctx), s);
    enqueue_forces<double>(ctx, s);
    launch_finish<double>(ctx->sd, ctx->ph, 0, s);
  } else {
    launch_prepare<float>(ctx->sf, ctx->ph, prepare_mode(ctx), s);
    enqueue_forces<float>(ctx, s);
    launch_finish<float>(ctx->sf, ctx->ph, 0, s);
  }
  HIP_TRY(hipGetLastError());
  return DEPO_OK;
}

depo_status depo_read_particles(depo_ctx *ctx, double *h_x3, double *h_v3, double *h_a3, int32_t *h_dep_step,
                                int32_t *h_neighbours, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  if (!ctx->seeded) return ctx->fail(DEPO_E_STATE, "seed first");
  return DISPATCH(do_read, ctx, h_x3, h_v3, h_a3, h_dep_step, h_neighbours, (hipStream_t)stream);
}

depo_status depo_tally_read(depo_ctx *ctx, depo_tally *out, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  if (!ctx->seeded) return ctx->fail(DEPO_E_STATE, "seed first");
  if (!out) return ctx->fail(DEPO_E_INVALID, "null output");
  return DISPATCH(do_tally, ctx, out, (hipStream_t)stream);
}

depo_status depo_state_bytes(const depo_ctx *ctx, size_t *bytes) {
  if (!ctx || !bytes) return DEPO_E_INVALID;
  if (!ctx->has_layout) return DEPO_E_STATE;
  *bytes = sizeof(BlobHeader) + (ctx->fp64() ? blob_payload<double>(ctx) : blob_payload<float>(ctx));
  return DEPO_OK;
}

depo_status depo_state_download(depo_ctx *ctx, void *h_blob, size_t bytes, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  if (!ctx->seeded) return ctx->fail(DEPO_E_STATE, "seed first");
  if (!h_blob) return ctx->fail(DEPO_E_INVALID, "null blob");
  return DISPATCH(do_download, ctx, h_blob, bytes, (hipStream_t)stream);
}

depo_status depo_state_upload(depo_ctx *ctx, const void *h_blob, size_t bytes, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (!ctx->bound || !ctx->field_ready) return ctx->fail(DEPO_E_STATE, "bind a workspace and upload the field first");
  if (!h_blob) return ctx->fail(DEPO_E_INVALID, "null blob");
  return DISPATCH(do_upload, ctx, h_blob, bytes, (hipStream_t)stream);
}

depo_status depo_adjoint_workspace_bytes(const depo_ctx *ctx, int32_t n_steps, int32_t ckpt_every, size_t *bytes) {
  if (!ctx || !bytes) return DEPO_E_INVALID;
  if (!ctx->has_layout) return DEPO_E_STATE;
  if (n_steps < 1 || ckpt_every < 1 || ckpt_every > n_steps) return DEPO_E_INVALID;
  const int K = (n_steps + ckpt_every - 1) / ckpt_every;
  if (ctx->fp64()) {
    AdjPlan<double> pl;
    *bytes = carve_adjoint<double>(ctx, nullptr, n_steps, K, ckpt_every, pl);
  } else {
    AdjPlan<float> pl;
    *bytes = carve_adjoint<float>(ctx, nullptr, n_steps, K, ckpt_every, pl);
  }
  return DEPO_OK;
}

depo_status depo_adjoint_forward(depo_ctx *ctx, int32_t n_steps, int32_t ckpt_every, void *d_adj_work, size_t bytes,
                                 depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  if (!ctx->seeded) return ctx->fail(DEPO_E_STATE, "seed first");
  if (ctx->nstep != 0) return ctx->fail(DEPO_E_STATE, "the adjoint starts from the seeded state (step 0)");
  if (!(ctx->p.flags & DEPO_SOFT_TALLY)) return ctx->fail(DEPO_E_INVALID, "the adjoint needs DEPO_SOFT_TALLY");
  if (ctx->p3m_use) return ctx->fail(DEPO_E_INVALID, "the adjoint differentiates the direct Coulomb sum; select a direct mode");
  if (n_steps < 1 || ckpt_every < 1 || ckpt_every > n_steps) return ctx->fail(DEPO_E_INVALID, "need 1 <= ckpt_every <= n_steps");
  if (!d_adj_work || ((uintptr_t)d_adj_work % kAlign) != 0) return ctx->fail(DEPO_E_INVALID, "adjoint workspace must be 256-byte aligned");
  ctx->adj_pending = false;
  ++ctx->gen;
  return DISPATCH(do_adjoint_forward, ctx, n_steps, ckpt_every, d_adj_work, bytes, (hipStream_t)stream);
}

depo_status depo_adjoint_backward(depo_ctx *ctx, const double *h_weights, double *h_grad, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  if (!ctx->adj_pending || ctx->adj_gen != ctx->gen)
    return ctx->fail(DEPO_E_STATE, "no pending adjoint forward run (or the state changed since)");
  if (!h_weights || !h_grad) return ctx->fail(DEPO_E_INVALID, "null weights or gradient array");
  for (int k = 0; k < ctx->S; ++k)
    if (!std::isfinite(h_weights[k])) return ctx->fail(DEPO_E_INVALID, "weight %d not finite", k);
  ctx->adj_pending = false;
  return DISPATCH(do_adjoint_backward, ctx, h_weights, h_grad, (hipStream_t)stream);
}

depo_status depo_adjoint(depo_ctx *ctx, int32_t n_steps, int32_t ckpt_every, const double *h_weights,
                         double *h_grad, void *d_adj_work, size_t bytes, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  if (!h_weights || !h_grad) return ctx->fail(DEPO_E_INVALID, "null weights or gradient array");
  for (int k = 0; k < ctx->S; ++k)
    if (!std::isfinite(h_weights[k])) return ctx->fail(DEPO_E_INVALID, "weight %d not finite", k);
  depo_status r = depo_adjoint_forward(ctx, n_steps, ckpt_every, d_adj_work, bytes, stream);
  if (r != DEPO_OK) return r;
  return depo_adjoint_backward(ctx, h_weights, h_grad, stream);
}

depo_status depo_adjoint_noalloc(depo_ctx *ctx, int32_t n_steps, int32_t ckpt_every, const double *h_weights,
                                 double *h_grad, depo_stream stream) {
  if (!ctx) return DEPO_E_INVALID;
  if (!ctx->seeded) return ctx->fail(DEPO_E_STATE, "seed first");
  if (!h_weights || !h_grad) return ctx->fail(DEPO_E_INVALID, "null weights or gradient array");
  for (int k = 0; k < ctx->S; ++k)
    if (!std::isfinite(h_weights[k])) return ctx->fail(DEPO_E_INVALID, "weight %d not finite", k);
  size_t need = 0;
  if (depo_adjoint_workspace_bytes(ctx, n_steps, ckpt_every, &need) != DEPO_OK)
    return ctx->fail(DEPO_E_INVALID, "need 1 <= ckpt_every <= n_steps");
  if (need > kScratchBytes)
    return ctx->fail(DEPO_E_CAPACITY, "the adjoint needs %zu bytes of workspace; the static workspace holds %zu "
                                      "(use depo_adjoint with a caller workspace)", need, kScratchBytes);
  void *ws = nullptr;
  if (depo_status r = scratch_address(ctx, &ws); r != DEPO_OK) return r;
  // the forward runs the step kernels directly: capturing a step graph could allocate
  const bool graph = ctx->use_graph;
  ctx->use_graph = false;
  depo_status r = depo_adjoint_forward(ctx, n_steps, ckpt_every, ws, kScratchBytes, stream);
  ctx->use_graph = graph;
  if (r != DEPO_OK) return r;
  return depo_adjoint_backward(ctx, h_weights, h_grad, stream);
}

depo_status depo_set_reorder(depo_ctx *ctx, int32_t every) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (every < 0 || every > (1 << 20)) return ctx->fail(DEPO_E_INVALID, "reorder interval must be 0..2^20 steps");
  ctx->order_every = every;
  ctx->drop_graph();
  return DEPO_OK;
}

static bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

depo_status depo_set_p3m(depo_ctx *ctx, int32_t mesh_x, int32_t mesh_yz, double alpha_h, double rmax_alpha) {
  if (!ctx) return DEPO_E_INVALID;
  ++ctx->gen;   // a pending adjoint reverse sweep no longer applies
  if (ctx->has_layout) return ctx->fail(DEPO_E_STATE, "configure P3M before depo_set_layout");
  if (!pow2_in(mesh_x, 16, 1024) || !pow2_in(mesh_yz, 16, 512) || !(alpha_h > 0.0 && alpha_h <= 2.0) ||
      !(rmax_alpha >= 2.0 && rmax_alpha <= 6.0))
    return ctx->fail(DEPO_E_INVALID, "P3M needs power-of-two meshes (16..1024 along x, 16..512 across), "
                                     "0 < alpha h <= 2 and 2 <= alpha r_max <= 6");
  ctx->p3m_cfg = true;
  ctx->p3m_use = true;
  ctx->p3m_nx = mesh_x;
  ctx->p3m_nc = mesh_yz;
  ctx->p3m_alpha_h = alpha_h;
  ctx->p3m_rmax_alpha = rmax_alpha;
  return DEPO_OK;
}

depo_status depo_lf_solve(const depo_params *p, int64_t n, const double *d_diam, const double *d_charge,
                          const double *d_hamaker, int32_t n_wall, int32_t n_core, double *d_vdep_plus,
                          depo_stream stream) {
  if (!p || n < 0 || n_wall < 2 || n_core < 1) return DEPO_E_INVALID;
  if (!(finite_pos(p->R) && finite_pos(p->nu) && finite_pos(p->rho_f) && finite_pos(p->rho_p) &&
        finite_pos(p->re_tau) && finite_pos(p->eps0)))
    return DEPO_E_INVALID;
  if (n == 0) return DEPO_OK;
  if (!d_diam || !d_charge || !d_hamaker || !d_vdep_plus) return DEPO_E_INVALID;
  const LfConst c{p->R, p->nu, p->rho_f, p->rho_p, p->re_tau, p->eps0, n_wall, n_core};
  launch_lf(c, n, d_diam, d_charge, d_hamaker, d_vdep_plus, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? DEPO_OK : DEPO_E_HIP;
}

}  // extern "C"

