// Symmetric Coulomb pair adjoint, FP32 form: the reverse of the symmetric
// direct sums (Eq. coulomb, Appendix A.2.4) under the same item list.
//
// With b_i = c_i a_bar_i (c_i the factor that turns the raw pair sum of particle
// i into its acceleration) and r = r_i - r_j, the pair law's contribution to the
// position adjoints is
//     x_bar_i += (1/u_x) J(r) p_ij,   p_ij = q_j b_i - q_i b_j,
// with J(r) = I/|r|^3 - 3 r r^T/|r|^5 (or (I - r^ r^T)/(|r| d_ij^2) inside the
// overlap clamp).  J is even in r and p_ji = -p_ij, so particle j receives
// exactly the negative: each unordered pair is evaluated once and its term is
// added to i and subtracted from j, as in the forward kernel.
//
// Schedule (same as the forward): the source tile of an item is staged in LDS,
// each round of 64 twice in a row; in step t lane l pairs its IPL targets with
// source (l + t) mod 64 and the three reaction sums travel with the source (DPP
// wave rotate), so after 64 steps they are back in the source's own lane.
// Per pair the fast body uses the point-charge form with |r|^2 + 1 (one rsq);
// a round that holds a pair closer than the largest diameter is recomputed
// with the exact clamp.  Diagonal items form all ordered pairs of their tile on
// the target side; their self pairs (step 0 of one round per target chunk) are
// skipped, since they contribute nothing.
//
// Items are combined with FP64 atomic adds into per-particle accumulators
// (the near-overlap branch of J has no useful a priori bound, so the forward's
// fixed-point scheme does not apply); k_vjp_finish scales by 1/u_x, writes the
// FP32 result and clears the accumulators.  The order of the FP64 additions
// varies from run to run; the FP32 results differ only when an FP64 sum lies
// within its own rounding error of an FP32 rounding boundary.
#include "common.hpp"
#include "launch.hpp"
#include "adjoint.hpp"

namespace depo {

namespace {

template <int CTRL> __device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, 0xf, 0xf, false));
}
constexpr int kWaveRol1 = 0x134;   // lane l receives the value of lane (l + 1) mod 64

__device__ __forceinline__ void dadd(double *acc, int64_t i, double v) { unsafeAtomicAdd(acc + i, v); }

template <int IPL, int W, bool REACT>
__device__ __forceinline__ void vjp_item(const SymItem &it, const JAdj<float> *__restrict__ rec,
                                         const float *__restrict__ jr, double *__restrict__ ax,
                                         double *__restrict__ ay, double *__restrict__ az, float near2,
                                         JAdj<float> *src, float *srad) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // stage the source tile (entry 128 r + k holds source 64 r + (k mod 64)); padding of the
  // last round has q = 0 and b = 0, so p = 0 and it contributes nothing to either side
  for (int e = threadIdx.x; e < 2 * 64 * IPL * W; e += 64 * W) {
    const int jj = (e >> 7) * 64 + (e & 63);
    const bool has = jj < it.jcount;
    JAdj<float> r = rec[it.j0 + (has ? jj : 0)];
    if (!has) r.q = r.bx = r.by = r.bz = 0.0f;
    src[e] = r;
    srad[e] = jr[it.j0 + (has ? jj : 0)];
  }

  uint32_t xi[IPL];
  float yi[IPL], zi[IPL], qi[IPL], bx[IPL], by[IPL], bz[IPL], ri[IPL];
  bool valid[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    const int ii = w * 64 * IPL + lane + 64 * k;
    valid[k] = ii < it.icount;
    const int i = it.i0 + (valid[k] ? ii : 0);
    const JAdj<float> me = rec[i];
    xi[k] = me.x; yi[k] = me.y; zi[k] = me.z;
    // absent targets: p = q_j * 0 - 0 * b_j = 0, no reaction
    qi[k] = valid[k] ? me.q : 0.0f;
    bx[k] = valid[k] ? me.bx : 0.0f;
    by[k] = valid[k] ? me.by : 0.0f;
    bz[k] = valid[k] ? me.bz : 0.0f;
    ri[k] = jr[i];
  }
  double hx[IPL], hy[IPL], hz[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) hx[k] = hy[k] = hz[k] = 0.0;
  __syncthreads();

  for (int jb = 0; jb < it.jcount; jb += 64) {
    const JAdj<float> *rs = src + 2 * jb + lane;
    float sx[IPL], sy[IPL], sz[IPL];
    float rx = 0.0f, ry = 0.0f, rz = 0.0f;   // reaction of the source now in this lane
#pragma unroll
    for (int k = 0; k < IPL; ++k) sx[k] = sy[k] = sz[k] = 0.0f;
    uint64_t nearmask = 0;
    auto step = [&](int t, int kskip) {
      const JAdj<float> s = rs[t];
#pragma unroll
      for (int k = 0; k < IPL; ++k) {
        if (k == kskip) continue;
        const float dx = sdiff(xi[k], s.x);
        const float dy = yi[k] - s.y;
        const float dz = zi[k] - s.z;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, 1.0f)));
        nearmask |= __builtin_amdgcn_ballot_w64(r2 < near2);
        const float inv = __builtin_amdgcn_rsqf(r2);
        const float inv2 = inv * inv;
        const float inv3 = inv2 * inv;
        const float px = fmaf(s.q, bx[k], -qi[k] * s.bx);
        const float py = fmaf(s.q, by[k], -qi[k] * s.by);
        const float pz = fmaf(s.q, bz[k], -qi[k] * s.bz);
        const float t3 = -3.0f * (fmaf(dx, px, fmaf(dy, py, dz * pz)) * inv2);
        const float ux = fmaf(t3, dx, px), uy = fmaf(t3, dy, py), uz = fmaf(t3, dz, pz);
        sx[k] = fmaf(inv3, ux, sx[k]);
        sy[k] = fmaf(inv3, uy, sy[k]);
        sz[k] = fmaf(inv3, uz, sz[k]);
        if constexpr (REACT) {
          rx = fmaf(-inv3, ux, rx);
          ry = fmaf(-inv3, uy, ry);
          rz = fmaf(-inv3, uz, rz);
        }
      }
      if constexpr (REACT) {
        rx = dpp<kWaveRol1>(rx);
        ry = dpp<kWaveRol1>(ry);
        rz = dpp<kWaveRol1>(rz);
      }
    };
    const int kself = REACT ? -1 : (jb - w * 64 * IPL) >> 6;   // wave-uniform
    step(0, kself);
#pragma unroll 3
    for (int t = 1; t < 64; ++t) step(t, -1);
    if (nearmask) {
      // exact pair law for this round: J p = k0 p - k1 (r.p / r^2) r, zero at r = 0
#pragma unroll
      for (int k = 0; k < IPL; ++k) sx[k] = sy[k] = sz[k] = 0.0f;
      rx = ry = rz = 0.0f;
      for (int t = 0; t < 64; ++t) {
        const int e = 2 * jb + lane + t;
        const JAdj<float> s = src[e];
        const float rj = srad[e];
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          const float dx = sdiff(xi[k], s.x);
          const float dy = yi[k] - s.y;
          const float dz = zi[k] - s.z;
          const float r2 = dx * dx + dy * dy + dz * dz;
          float gx = 0.0f, gy = 0.0f, gz = 0.0f;
          if (r2 > 0.0f) {
            const float r = sqrtf(r2);
            const float dd = ri[k] + rj;
            const float px = s.q * bx[k] - qi[k] * s.bx;
            const float py = s.q * by[k] - qi[k] * s.by;
            const float pz = s.q * bz[k] - qi[k] * s.bz;
            const float rp = (dx * px + dy * py + dz * pz) / r2;
            float k0, k1;
            if (r >= dd) { k0 = 1.0f / (r2 * r); k1 = 3.0f * k0; }
            else { k0 = 1.0f / (r * dd * dd); k1 = k0; }
            gx = k0 * px - k1 * rp * dx;
            gy = k0 * py - k1 * rp * dy;
            gz = k0 * pz - k1 * rp * dz;
          }
          sx[k] += gx; sy[k] += gy; sz[k] += gz;
          if constexpr (REACT) { rx -= gx; ry -= gy; rz -= gz; }
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
      hx[k] += (double)sx[k];
      hy[k] += (double)sy[k];
      hz[k] += (double)sz[k];
    }
    if constexpr (REACT) {
      // after 64 rotations lane l holds the reaction of source jb + l on this wave's targets
      if (jb + lane < it.jcount) {
        const int64_t j = (int64_t)it.j0 + jb + lane;
        dadd(ax, j, (double)rx);
        dadd(ay, j, (double)ry);
        dadd(az, j, (double)rz);
      }
    }
  }

#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    if (!valid[k]) continue;
    const int64_t i = it.i0 + w * 64 * IPL + lane + 64 * k;
    dadd(ax, i, hx[k]);
    dadd(ay, i, hy[k]);
    dadd(az, i, hz[k]);
  }
}

template <int IPL, int W>
__global__ __launch_bounds__(64 * W) void k_coulomb_vjp_sym(const SymItem *__restrict__ items,
                                                            const JAdj<float> *__restrict__ rec,
                                                            const float *__restrict__ jr, double *__restrict__ ax,
                                                            double *__restrict__ ay, double *__restrict__ az,
                                                            float near2) {
  constexpr int T = 64 * IPL * W;
  __shared__ JAdj<float> src[2 * T];
  __shared__ float srad[2 * T];
  const SymItem it = items[blockIdx.x];
  if (it.j0 == it.i0)
    vjp_item<IPL, W, false>(it, rec, jr, ax, ay, az, near2, src, srad);
  else
    vjp_item<IPL, W, true>(it, rec, jr, ax, ay, az, near2, src, srad);
}

// Totals (in units of the x quantum) to x_bar contributions; the accumulators are cleared.
__global__ __launch_bounds__(256) void k_vjp_finish(int32_t N, float inv_ux, double *__restrict__ ax,
                                                    double *__restrict__ ay, double *__restrict__ az,
                                                    float *__restrict__ ox, float *__restrict__ oy,
                                                    float *__restrict__ oz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  ox[i] = (float)(ax[i] * (double)inv_ux);
  oy[i] = (float)(ay[i] * (double)inv_ux);
  oz[i] = (float)(az[i] * (double)inv_ux);
  ax[i] = 0.0;
  ay[i] = 0.0;
  az[i] = 0.0;
}

}  // namespace

#define DEPO_VJP_SYM_CASES(X) X(1, 4) X(1, 8) X(2, 2) X(2, 4) X(4, 1) X(4, 2) X(4, 4) X(8, 1)

void launch_coulomb_vjp_sym(const State<float> &st, const Phys &ph, const AdjState<float> &ad, int n_diag, int n_off,
                            const CoulombConfig &cfg, hipStream_t s) {
  // the forward's fixed-point accumulators are zero between evaluations; the same memory
  // holds the FP64 sums here and is zero again after k_vjp_finish
  double *ax = reinterpret_cast<double *>(st.accx);
  double *ay = reinterpret_cast<double *>(st.accy);
  double *az = reinterpret_cast<double *>(st.accz);
  const int n_items = n_diag + n_off;
#define X(I, W)                                                                                            \
  if (n_items > 0 && cfg.ipl == I && cfg.waves == W)                                                       \
    hipLaunchKernelGGL((k_coulomb_vjp_sym<I, W>), dim3(n_items), dim3(64 * W), 0, s, st.items, ad.rec,     \
                       st.jr, ax, ay, az, (float)ph.near2);
  DEPO_VJP_SYM_CASES(X)
#undef X
  if (ph.N > 0)
    hipLaunchKernelGGL(k_vjp_finish, dim3((ph.N + 255) / 256), dim3(256), 0, s, ph.N, (float)ph.inv_ux, ax, ay, az,
                       ad.xc[0], ad.xc[1], ad.xc[2]);
}

}  // namespace depo
