// Symmetric direct Coulomb sums (Eq. coulomb; F_i = sum_j F_ij n_ij, Appendix A.2.4),
// FP32 form: every unordered pair of a sample is evaluated once and its force
// is applied to both particles (F_ji = -F_ij, Newton's third law).
//
// The pair matrix of a sample is cut into T x T items (T = 64 IPL W).  An item
// (I, J), I < J, pairs the targets of tile I (IPL per lane, 64 IPL per wave)
// with the sources of tile J; a diagonal item (I, I) forms all ordered pairs of
// its tile on the target side only.  Per pair the body is the point-charge form
// r / (|r|^2 + 1)^(3/2) (one rsq); any round of sources that holds a pair
// closer than the largest diameter (wave-uniform ballot) is recomputed with the
// exact overlap clamp r / (|r| max(|r|, d_ij)^2).
//
// Ring schedule: the item's source tile is staged in LDS; a wave takes the
// sources 64 at a time (a round), one per lane, and in step t of a round lane l
// pairs its targets with source (l + t) mod 64, read from LDS (each round is
// stored twice in a row, so that entry l + t needs no wrap-around).  The reaction
// accumulated for a source travels with it: after each step the three
// accumulators move one lane down (DPP wave rotate), so after 64 steps every
// source's reaction from all 64 IPL targets of the wave is back in its own
// lane.  No cross-lane reduction tree; 3 VALU moves per step.
// * Target side: round sums are added to the running sum with Kahan
//   compensation.  Source side: each wave adds its reaction on the round's
//   sources as soon as the round ends.
// * Items are combined in 64-bit fixed point: each item adds its target and
//   source partials, rounded to multiples of 2^-62 of a per-sample bound on
//   |sum| (sum_j |q~_j| / d_min^2, so no total or intermediate sum can
//   overflow), to per-particle integer accumulators with atomic adds.
//   Integer addition is associative, so the result does not depend on the
//   order in which items finish: bitwise reproducible.  k_pair_finish converts
//   the totals back and clears the accumulators for the next evaluation.
#include "common.hpp"
#include "launch.hpp"

namespace depo {

namespace {

// every lane receives a value under a wave rotate, so the old-value operand is never used
template <int CTRL> __device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, 0xf, 0xf, false));
}
constexpr int kWaveRol1 = 0x134;   // lane l receives the value of lane (l + 1) mod 64

__device__ __forceinline__ void fx_add(unsigned long long *acc, int64_t i, double v, double scale) {
  atomicAdd(acc + i, (unsigned long long)__double2ll_rn(v * scale));
}

// y or z difference of two records: float records subtract; integer records (bit patterns of
// int32 x-quanta counts) subtract exactly and convert.
template <bool INTREC> __device__ __forceinline__ float rdiff(float a, float b) {
  if constexpr (INTREC) return (float)(__float_as_int(a) - __float_as_int(b));
  else return a - b;
}

template <int IPL, int W, bool REACT, bool INTREC>
__device__ __forceinline__ void ring_item(const SymItem &it, const JSrc<float> *__restrict__ js,
                                          const float *__restrict__ jr, double scale,
                                          unsigned long long *__restrict__ accx, unsigned long long *__restrict__ accy,
                                          unsigned long long *__restrict__ accz, float near2, JSrc<float> *src,
                                          float *srad) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // stage the source tile, each round of 64 twice in a row (entry 128 r + k holds source
  // 64 r + (k mod 64)); charge 0 beyond jcount: padding of the last round
  for (int e = threadIdx.x; e < 2 * 64 * IPL * W; e += 64 * W) {
    const int jj = (e >> 7) * 64 + (e & 63);
    const bool has = jj < it.jcount;
    JSrc<float> r = js[it.j0 + (has ? jj : 0)];
    if (!has) r.q = 0.0f;
    src[e] = r;
    srad[e] = jr[it.j0 + (has ? jj : 0)];
  }

  uint32_t xi[IPL];
  float yi[IPL], zi[IPL], qi[IPL], ri[IPL];
  bool valid[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    const int ii = w * 64 * IPL + lane + 64 * k;
    valid[k] = ii < it.icount;
    const int i = it.i0 + (valid[k] ? ii : 0);
    const JSrc<float> me = js[i];
    xi[k] = me.x; yi[k] = me.y; zi[k] = me.z;
    qi[k] = valid[k] ? me.q : 0.0f;   // absent targets exert no reaction
    ri[k] = jr[i];
  }
  float hx[IPL], hy[IPL], hz[IPL], cx[IPL], cy[IPL], cz[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) hx[k] = hy[k] = hz[k] = cx[k] = cy[k] = cz[k] = 0.0f;
  __syncthreads();

  for (int jb = 0; jb < it.jcount; jb += 64) {
    const JSrc<float> *rs = src + 2 * jb + lane;
    float sx[IPL], sy[IPL], sz[IPL];
    float rx = 0.0f, ry = 0.0f, rz = 0.0f;   // reaction of the source now in this lane
#pragma unroll
    for (int k = 0; k < IPL; ++k) sx[k] = sy[k] = sz[k] = 0.0f;
    uint64_t nearmask = 0;
    // one ring step; target kskip (if any) is skipped: in a diagonal item, step 0 of the round
    // that holds target chunk k pairs every lane with itself (zero force, but never "near")
    auto step = [&](int t, int kskip) {
      const JSrc<float> s = rs[t];
#pragma unroll
      for (int k = 0; k < IPL; ++k) {
        if (k == kskip) continue;
        const float dx = sdiff(xi[k], s.x);
        const float dy = rdiff<INTREC>(yi[k], s.y);
        const float dz = rdiff<INTREC>(zi[k], s.z);
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, 1.0f)));
        nearmask |= __builtin_amdgcn_ballot_w64(r2 < near2);
        const float inv = __builtin_amdgcn_rsqf(r2);
        const float i3 = (inv * inv) * inv;
        const float wt = s.q * i3;
        sx[k] = fmaf(wt, dx, sx[k]);
        sy[k] = fmaf(wt, dy, sy[k]);
        sz[k] = fmaf(wt, dz, sz[k]);
        if constexpr (REACT) {
          const float ws = qi[k] * i3;
          rx = fmaf(ws, dx, rx);
          ry = fmaf(ws, dy, ry);
          rz = fmaf(ws, dz, rz);
        }
      }
      if constexpr (REACT) {
        rx = dpp<kWaveRol1>(rx);
        ry = dpp<kWaveRol1>(ry);
        rz = dpp<kWaveRol1>(rz);
      }
    };
    if constexpr (REACT) {
#pragma unroll 4
      for (int t = 0; t < 64; ++t) step(t, -1);
    } else {
      const int kself = (jb - w * 64 * IPL) >> 6;   // wave-uniform; outside [0, IPL) when no self pair
      step(0, kself);
#pragma unroll 3
      for (int t = 1; t < 64; ++t) step(t, -1);
    }
    if (nearmask) {
      // exact overlap clamp for this round, both sides: r / (|r| max(|r|, d_ij)^2), zero at r = 0
#pragma unroll
      for (int k = 0; k < IPL; ++k) sx[k] = sy[k] = sz[k] = 0.0f;
      rx = ry = rz = 0.0f;
      for (int t = 0; t < 64; ++t) {
        const int e = 2 * jb + lane + t;
        const JSrc<float> s = src[e];
        const float rj = srad[e];
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          const float dx = sdiff(xi[k], s.x);
          const float dy = rdiff<INTREC>(yi[k], s.y);
          const float dz = rdiff<INTREC>(zi[k], s.z);
          const float r2 = dx * dx + dy * dy + dz * dz;
          const float dd = ri[k] + rj;
          const float rc2 = fmaxf(r2, dd * dd);
          const float f = r2 > 0.0f ? 1.0f / (sqrtf(r2) * rc2) : 0.0f;
          const float wt = s.q * f;
          sx[k] = fmaf(wt, dx, sx[k]);
          sy[k] = fmaf(wt, dy, sy[k]);
          sz[k] = fmaf(wt, dz, sz[k]);
          if constexpr (REACT) {
            const float ws = qi[k] * f;
            rx = fmaf(ws, dx, rx);
            ry = fmaf(ws, dy, ry);
            rz = fmaf(ws, dz, rz);
          }
        }
        if constexpr (REACT) {
          rx = dpp<kWaveRol1>(rx);
          ry = dpp<kWaveRol1>(ry);
          rz = dpp<kWaveRol1>(rz);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      float y, t;
      y = sx[k] - cx[k]; t = hx[k] + y; cx[k] = (t - hx[k]) - y; hx[k] = t;
      y = sy[k] - cy[k]; t = hy[k] + y; cy[k] = (t - hy[k]) - y; hy[k] = t;
      y = sz[k] - cz[k]; t = hz[k] + y; cz[k] = (t - hz[k]) - y; hz[k] = t;
    }
    if constexpr (REACT) {
      // after 64 rotations lane l holds the reaction of source jb + l on this wave's targets
      if (jb + lane < it.jcount) {
        const int64_t j = (int64_t)it.j0 + jb + lane;
        fx_add(accx, j, -(double)rx, scale);
        fx_add(accy, j, -(double)ry, scale);
        fx_add(accz, j, -(double)rz, scale);
      }
    }
  }

  // target side: this item's partial of each valid target
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    if (!valid[k]) continue;
    const int64_t i = it.i0 + w * 64 * IPL + lane + 64 * k;
    fx_add(accx, i, (double)hx[k] - (double)cx[k], scale);
    fx_add(accy, i, (double)hy[k] - (double)cy[k], scale);
    fx_add(accz, i, (double)hz[k] - (double)cz[k], scale);
  }
}

template <int IPL, int W, bool INTREC>
__global__ __launch_bounds__(64 * W) void k_coulomb_sym(const SymItem *__restrict__ items,
                                                        const JSrc<float> *__restrict__ js,
                                                        const float *__restrict__ jr,
                                                        const double *__restrict__ fx_scale,
                                                        unsigned long long *__restrict__ accx,
                                                        unsigned long long *__restrict__ accy,
                                                        unsigned long long *__restrict__ accz, float near2) {
  constexpr int T = 64 * IPL * W;
  __shared__ JSrc<float> src[2 * T];
  __shared__ float srad[2 * T];
  const SymItem it = items[blockIdx.x];
  const double scale = fx_scale[it.sample];
  if (it.j0 == it.i0)
    ring_item<IPL, W, false, INTREC>(it, js, jr, scale, accx, accy, accz, near2, src, srad);
  else
    ring_item<IPL, W, true, INTREC>(it, js, jr, scale, accx, accy, accz, near2, src, srad);
}

// Fixed-point totals back to pair sums; the accumulators are cleared for the next evaluation.
__global__ __launch_bounds__(256) void k_pair_finish(int32_t N, const int32_t *__restrict__ sid,
                                                     const double *__restrict__ fx_scale,
                                                     unsigned long long *__restrict__ accx,
                                                     unsigned long long *__restrict__ accy,
                                                     unsigned long long *__restrict__ accz, float *__restrict__ ox,
                                                     float *__restrict__ oy, float *__restrict__ oz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double inv = 1.0 / fx_scale[sid[i]];
  ox[i] = (float)((double)(long long)accx[i] * inv);
  oy[i] = (float)((double)(long long)accy[i] * inv);
  oz[i] = (float)((double)(long long)accz[i] * inv);
  accx[i] = 0ull;
  accy[i] = 0ull;
  accz[i] = 0ull;
}

}  // namespace

// (targets per lane, waves); T = 64 IPL W targets per item, rounds of 64 sources
#define DEPO_COULOMB_SYM_CASES(X) X(1, 4) X(1, 8) X(2, 2) X(2, 4) X(4, 1) X(4, 2) X(4, 4) X(8, 1)

int coulomb_sym_tile(const CoulombConfig &cfg) { return 64 * cfg.ipl * cfg.waves; }

bool coulomb_sym_supported(const CoulombConfig &cfg) {
  if (!cfg.symmetric || !cfg.compensated || cfg.block != 64) return false;
#define X(I, W) \
  if (cfg.ipl == I && cfg.waves == W) return true;
  DEPO_COULOMB_SYM_CASES(X)
#undef X
  return false;
}

void launch_coulomb_sym(const State<float> &st, const Phys &ph, int n_diag, int n_off, const CoulombConfig &cfg,
                        hipStream_t s, bool defer_finish) {
  const float near2 = (float)ph.near2;
  const int n_items = n_diag + n_off;
#define X(I, W)                                                                                              \
  if (n_items > 0 && cfg.ipl == I && cfg.waves == W) {                                                       \
    if (cfg.int_rec)                                                                                         \
      hipLaunchKernelGGL((k_coulomb_sym<I, W, true>), dim3(n_items), dim3(64 * W), 0, s, st.items, st.js,    \
                         st.jr, st.fx_scale, st.accx, st.accy, st.accz, near2);                              \
    else                                                                                                     \
      hipLaunchKernelGGL((k_coulomb_sym<I, W, false>), dim3(n_items), dim3(64 * W), 0, s, st.items, st.js,   \
                         st.jr, st.fx_scale, st.accx, st.accy, st.accz, near2);                              \
  }
  DEPO_COULOMB_SYM_CASES(X)
#undef X
  if (ph.N > 0 && !defer_finish)
    hipLaunchKernelGGL(k_pair_finish, dim3((ph.N + 255) / 256), dim3(256), 0, s, ph.N, st.sid, st.fx_scale, st.accx,
                       st.accy, st.accz, st.cx, st.cy, st.cz);
}

}  // namespace depo
