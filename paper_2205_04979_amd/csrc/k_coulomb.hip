// Direct O(N^2) Coulomb sums (Eq. coulomb; F_i = sum_j F_ij n_ij, Appendix A.2.4).
//
// For every alive target i of a sample the kernel forms
//     S_i = sum_{j in sample, j != i} q~_j r_ij / (|r_ij| max(|r_ij|, d_ij)^2)
// in units of the x quantum, with r_ij the minimum-image displacement (x is a
// fixed-point fraction of L, so the signed integer difference already is the
// minimum image) and q~ the scaled charge (0 for removed particles).  The
// acceleration k_e q_i q_ref S_i / (m_i ux^2) is applied by k_finish.
//
// Mapping to CDNA4:
// * a workgroup owns 64*IPL targets (IPL per lane, kept in VGPRs) and its
//   WAVES wavefronts split the source range;
// * the source records are wave-uniform, so they are fetched with scalar
//   loads into SGPRs and every VALU instruction of the pair body takes its
//   source operand straight from an SGPR: no LDS traffic, no shuffles;
// * the pair body is the point-charge form r / (|r|^2 + 1)^(3/2) (one rsq);
//   a wave-uniform ballot flags a block of BLK sources holding any pair
//   closer than the largest diameter, and only such blocks are recomputed
//   with the exact overlap clamp max(|r|, d_ij);
// * FP32: each block is summed plainly and then added to the running sum with
//   Kahan compensation; the per-wave partial sums are combined in FP64
//   through LDS in a fixed order, so results are bitwise reproducible.
#include "common.hpp"
#include "launch.hpp"

#include <type_traits>

namespace depo {

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

template <class Real, int IPL, int WAVES, int BLK, bool KAHAN, bool PIPE>
__global__ __launch_bounds__(64 * WAVES) void k_coulomb(const TileDev *__restrict__ tiles,
                                                        const JSrc<Real> *__restrict__ js,
                                                        const Real *__restrict__ jr, Real *__restrict__ ox,
                                                        Real *__restrict__ oy, Real *__restrict__ oz,
                                                        Real near2) {
  using Pos = typename Prec<Real>::Pos;
  __shared__ double red[WAVES][3][64 * IPL];
  const TileDev t = tiles[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  Pos xi[IPL];
  Real yi[IPL], zi[IPL], ri[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    const int ii = lane + 64 * k;
    const int i = t.i0 + (ii < t.icount ? ii : 0);
    const JSrc<Real> me = js[i];
    xi[k] = me.x; yi[k] = me.y; zi[k] = me.z;
    ri[k] = jr[i];
  }

  const int per = ((t.jcount + WAVES - 1) / WAVES + BLK - 1) / BLK * BLK;
  const int jb = t.j0 + w * per;
  const int je = min(t.j0 + t.jcount, jb + per);

  Real hx[IPL], hy[IPL], hz[IPL], cx[IPL], cy[IPL], cz[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) { hx[k] = hy[k] = hz[k] = cx[k] = cy[k] = cz[k] = Real(0); }

  Real sx[IPL], sy[IPL], sz[IPL];
  uint64_t nearmask = 0;

  auto body = [&](const JSrc<Real> &s) {
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const Real dx = sdiff(xi[k], s.x);
      const Real dy = yi[k] - s.y;
      const Real dz = zi[k] - s.z;
      const Real r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, Real(1))));
      nearmask |= __builtin_amdgcn_ballot_w64(r2 < near2);
      const Real inv = rsq(r2);
      const Real wq = s.q * (inv * inv) * inv;
      sx[k] = fma(wq, dx, sx[k]);
      sy[k] = fma(wq, dy, sy[k]);
      sz[k] = fma(wq, dz, sz[k]);
    }
  };
  auto open_block = [&]() {
#pragma unroll
    for (int k = 0; k < IPL; ++k) { sx[k] = sy[k] = sz[k] = Real(0); }
    nearmask = 0;
  };
  // close a block of n sources starting at j0: exact recompute if any pair was
  // closer than the largest diameter, then compensated accumulation
  auto close_block = [&](int j0, int n) {
    if (nearmask) {
      // exact overlap clamp for this block: r / (|r| max(|r|, d_ij)^2), zero at r = 0
#pragma unroll
      for (int k = 0; k < IPL; ++k) { sx[k] = sy[k] = sz[k] = Real(0); }
      for (int jj = 0; jj < n; ++jj) {
        const JSrc<Real> s = js[j0 + jj];
        const Real rj = jr[j0 + jj];
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
          const Real dx = sdiff(xi[k], s.x);
          const Real dy = yi[k] - s.y;
          const Real dz = zi[k] - s.z;
          const Real r2 = dx * dx + dy * dy + dz * dz;
          const Real dd = ri[k] + rj;
          const Real rc2 = fmax(r2, dd * dd);
          const Real wq = r2 > Real(0) ? s.q / (sqrt(r2) * rc2) : Real(0);
          sx[k] = fma(wq, dx, sx[k]);
          sy[k] = fma(wq, dy, sy[k]);
          sz[k] = fma(wq, dz, sz[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      if constexpr (KAHAN) {
        Real y, tt;
        y = sx[k] - cx[k]; tt = hx[k] + y; cx[k] = (tt - hx[k]) - y; hx[k] = tt;
        y = sy[k] - cy[k]; tt = hy[k] + y; cy[k] = (tt - hy[k]) - y; hy[k] = tt;
        y = sz[k] - cz[k]; tt = hz[k] + y; cz[k] = (tt - hz[k]) - y; hz[k] = tt;
      } else {
        hx[k] += sx[k]; hy[k] += sy[k]; hz[k] += sz[k];
      }
    }
  };

  int j0 = jb;
  if constexpr (PIPE) {
    // full blocks, source records prefetched one group of G ahead (across block
    // boundaries) so the scalar-load latency overlaps the arithmetic
    constexpr int G = 4;
    JSrc<Real> cur[G];
    if (j0 + BLK <= je) {
#pragma unroll
      for (int g = 0; g < G; ++g) cur[g] = js[j0 + g];
    }
    for (; j0 + BLK <= je; j0 += BLK) {
      open_block();
#pragma unroll 1
      for (int jj = 0; jj < BLK; jj += G) {
        const int jn = j0 + jj + G;
        JSrc<Real> nxt[G];
        const bool more = (jj + G < BLK) || (jn + BLK <= je);
        if (more) {
#pragma unroll
          for (int g = 0; g < G; ++g) nxt[g] = js[jn + g];
        }
#pragma unroll
        for (int g = 0; g < G; ++g) body(cur[g]);
        if (more) {
#pragma unroll
          for (int g = 0; g < G; ++g) cur[g] = nxt[g];
        }
      }
      close_block(j0, BLK);
    }
  } else {
    for (; j0 + BLK <= je; j0 += BLK) {
      open_block();
#pragma unroll 8
      for (int jj = 0; jj < BLK; ++jj) body(js[j0 + jj]);
      close_block(j0, BLK);
    }
  }
  if (j0 < je) {   // ragged tail block
    const int n = je - j0;
    open_block();
    for (int jj = 0; jj < n; ++jj) body(js[j0 + jj]);
    close_block(j0, n);
  }

#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    red[w][0][lane + 64 * k] = (double)hx[k] - (double)cx[k];
    red[w][1][lane + 64 * k] = (double)hy[k] - (double)cy[k];
    red[w][2][lane + 64 * k] = (double)hz[k] - (double)cz[k];
  }
  __syncthreads();
  for (int ii = threadIdx.x; ii < 64 * IPL; ii += 64 * WAVES) {
    if (ii >= t.icount) continue;
    double s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int q = 0; q < WAVES; ++q) { s0 += red[q][0][ii]; s1 += red[q][1][ii]; s2 += red[q][2][ii]; }
    const int i = t.i0 + ii;
    ox[i] = Real(s0); oy[i] = Real(s1); oz[i] = Real(s2);
  }
}

int coulomb_tile_targets(const CoulombConfig &cfg) { return 64 * cfg.ipl; }

// (type, targets per lane, waves, block, Kahan, prefetch); block 64 selects the prefetching variant
#define DEPO_COULOMB_CASES(X)                                                                              \
  X(float, 1, 4, 32, true, false) X(float, 1, 8, 32, true, false) X(float, 2, 4, 32, true, false)           \
  X(float, 2, 8, 32, true, false) X(float, 4, 4, 32, true, false) X(float, 4, 8, 32, true, false)           \
  X(float, 1, 16, 32, true, false) X(float, 2, 16, 32, true, false)                                         \
  X(float, 1, 8, 64, true, true) X(float, 1, 16, 64, true, true) X(float, 2, 8, 64, true, true)             \
  X(float, 2, 16, 64, true, true) X(float, 1, 4, 64, true, true)                                            \
  X(float, 1, 16, 32, false, false)                                                                         \
  X(double, 1, 4, 16, false, false) X(double, 1, 8, 16, false, false) X(double, 2, 4, 16, false, false)           \
  X(double, 1, 16, 16, false, false)

bool coulomb_config_supported(int real_bytes, const CoulombConfig &cfg) {
#define X(R, I, W, B, K, P) \
  if ((int)sizeof(R) == real_bytes && cfg.ipl == I && cfg.waves == W && cfg.block == B && cfg.compensated == K) \
    return true;
  DEPO_COULOMB_CASES(X)
#undef X
  return false;
}

template <class Real>
void launch_coulomb(const State<Real> &st, const Phys &ph, int n_tiles, const CoulombConfig &cfg, hipStream_t s) {
  if (n_tiles <= 0) return;
  const Real near2 = Real(ph.near2);
#define X(R, I, W, B, K, P)                                                                              \
  if constexpr (std::is_same<Real, R>::value) {                                                         \
    if (cfg.ipl == I && cfg.waves == W && cfg.block == B && cfg.compensated == K) {                     \
      hipLaunchKernelGGL((k_coulomb<R, I, W, B, K, P>), dim3(n_tiles), dim3(64 * W), 0, s, st.tiles, st.js, \
                         st.jr, st.cx, st.cy, st.cz, near2);                                             \
      return;                                                                                           \
    }                                                                                                   \
  }
  DEPO_COULOMB_CASES(X)
#undef X
}

template void launch_coulomb<float>(const State<float> &, const Phys &, int, const CoulombConfig &, hipStream_t);
template void launch_coulomb<double>(const State<double> &, const Phys &, int, const CoulombConfig &, hipStream_t);

}  // namespace depo
