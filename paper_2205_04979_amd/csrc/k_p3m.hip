// Particle-particle particle-mesh electrostatics (Appendix A.2.4, Eq. coulomb_force):
// the same raw Coulomb sums S_i as the direct kernels, for the lattice that is
// periodic in x (period L) and unbounded across the pipe section, in O(N log N).
//
// Split (Gaussian): 1/r = erfc(a r)/r + erf(a r)/r.  Long range: the erf part,
// on a mesh of nx x P x P nodes (x periodic, hx = L/nx; y and z: nc nodes across
// [-R, R] with one spare node on each side, hy = 2R/(nc - 3), zero-padded to
// P = 2 nc for the aperiodic convolution), with triangular-shaped-cloud (TSC)
// charge assignment and field interpolation and a Green's function that is the
// erf field of a unit charge summed over the x images and divided by the squared
// TSC transfer function.  Short range: Coulomb's law (with the overlap clamp of
// the direct sum) minus the erf field, over nearest-image pairs closer than
// r_max, found through a cell list with cells of at least r_max.
//
// Charge assignment adds 64-bit fixed-point weights with integer atomics (order
// independent), the FFTs are radix-2 Cooley-Tukey passes over mesh lines staged
// in LDS, and the short-range sum is a gather over cell-sorted neighbours in a
// fixed order, so results are bitwise reproducible.  The mesh holds complex
// values in the form's precision (FP32 form: float2, half the bytes of every
// mesh pass; FP64 form: double2); the Green's function is always built and
// transformed in FP64 and only then rounded to the mesh type.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace depo {

namespace {

constexpr int kFftLds = 2048;   // complex values per FFT workgroup (32 KB of LDS)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <class T> __device__ __forceinline__ T cplx(double re, double im);
template <> __device__ __forceinline__ double2 cplx<double2>(double re, double im) { return make_double2(re, im); }
template <> __device__ __forceinline__ float2 cplx<float2>(double re, double im) {
  return make_float2((float)re, (float)im);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// mesh element of a form
template <class Real> using MeshT = typename std::conditional<sizeof(Real) == 4, float2, double2>::type;

// Continuous mesh coordinates of particle i (x periodic in [0, nx); y, z in [1, nc - 2]).
template <class Real>
__device__ __forceinline__ void mesh_coords(const State<Real> &st, const Phys &ph, const P3mDev &m, int i, double &gx,
                                            double &gy, double &gz) {
  using SPos = typename std::make_signed<typename Prec<Real>::Pos>::type;
  const double x = ((double)st.px[i] + (double)st.rx[i]) * ph.ux;
  const double y = ((double)(SPos)st.py[i] + (double)st.ry[i]) * ph.ur;
  const double z = ((double)(SPos)st.pz[i] + (double)st.rz[i]) * ph.ur;
  gx = x / m.hx;
  if (gx >= m.nx) gx -= m.nx;
  if (gx < 0.0) gx += m.nx;
  gy = (y + ph.R) / m.hy + 1.0;
  gz = (z + ph.R) / m.hy + 1.0;
}

__device__ __forceinline__ void tsc(double g, int &i, double (&w)[3]) {
  const double c = floor(g + 0.5);
  const double dl = g - c;
  i = (int)c;
  w[0] = 0.5 * (0.5 - dl) * (0.5 - dl);
  w[1] = 0.75 - dl * dl;
  w[2] = 0.5 * (0.5 + dl) * (0.5 + dl);
}

// Erf field of a unit charge at displacement (dx, dy, dz), summed over the x images n = -M..M:
// all three components (comp < 0) or component comp alone into gx_.
__global__ void k_p3m_green(P3mDev m, double L, int images, int comp, double2 *__restrict__ gx_,
                            double2 *__restrict__ gy_, double2 *__restrict__ gz_) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)m.nx * m.P * m.P;
  if (e >= total) return;
  const int iz = (int)(e % m.P), iy = (int)((e / m.P) % m.P), ix = (int)(e / ((int64_t)m.P * m.P));
  double dx = ix * m.hx;
  if (dx >= 0.5 * L) dx -= L;
  const double dy = (iy < m.P / 2 ? iy : iy - m.P) * m.hy;
  const double dz = (iz < m.P / 2 ? iz : iz - m.P) * m.hy;
  const double a = m.alpha, c2 = 2.0 * m.alpha / sqrt(M_PI);
  double ex = 0.0, ey = 0.0, ez = 0.0;
  for (int n = -images; n <= images; ++n) {
    const double rx = dx + n * L;
    const double r2 = rx * rx + dy * dy + dz * dz;
    if (r2 <= 0.0) continue;
    const double r = sqrt(r2);
    const double mag = erf(a * r) / r2 - c2 * exp(-a * a * r2) / r;   // |E_l|
    const double f = mag / r;
    ex += f * rx;
    ey += f * dy;
    ez += f * dz;
  }
  if (comp < 0) {
    gx_[e] = make_double2(ex, 0.0);
    gy_[e] = make_double2(ey, 0.0);
    gz_[e] = make_double2(ez, 0.0);
  } else {
    gx_[e] = make_double2(comp == 0 ? ex : (comp == 1 ? ey : ez), 0.0);
  }
}

// Divide the transformed Green's functions by the squared TSC transfer sinc^3 per axis.
__device__ __forceinline__ double sinc_pi(double u) { return u == 0.0 ? 1.0 : sin(M_PI * u) / (M_PI * u); }

__device__ __forceinline__ double tsc_inv_transfer2(const P3mDev &m, int64_t e) {
  const int iz = (int)(e % m.P), iy = (int)((e / m.P) % m.P), ix = (int)(e / ((int64_t)m.P * m.P));
  auto freq = [](int i, int n) { return (double)(i < (n + 1) / 2 ? i : i - n) / n; };   // cycles per node
  const double sx = sinc_pi(freq(ix, m.nx)), sy = sinc_pi(freq(iy, m.P)), sz = sinc_pi(freq(iz, m.P));
  const double W = sx * sx * sx * sy * sy * sy * sz * sz * sz;
  return 1.0 / (W * W);
}

__global__ void k_p3m_deconv(P3mDev m, double2 *__restrict__ gx_, double2 *__restrict__ gy_,
                             double2 *__restrict__ gz_) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)m.nx * m.P * m.P;
  if (e >= total) return;
  const double inv = tsc_inv_transfer2(m, e);
  gx_[e] = make_double2(gx_[e].x * inv, gx_[e].y * inv);
  gy_[e] = make_double2(gy_[e].x * inv, gy_[e].y * inv);
  gz_[e] = make_double2(gz_[e].x * inv, gz_[e].y * inv);
}

// One transformed FP64 component, deconvolved and rounded to an FP32 mesh array.
__global__ void k_p3m_deconv_f32(P3mDev m, const double2 *__restrict__ g, float2 *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)m.nx * m.P * m.P;
  if (e >= total) return;
  const double inv = tsc_inv_transfer2(m, e);
  out[e] = make_float2((float)(g[e].x * inv), (float)(g[e].y * inv));
}

// Complex FFT of length n = 2^log2n along lines of the mesh: line l starts at
// (l >> log2inner) * outer_stride + (l & (2^log2inner - 1)) * inner_stride, points are
// point_stride apart.  A workgroup transforms kFftLds / n lines through LDS (bit-reversed load,
// in-place radix-2 butterflies, twiddles exp(sign 2 pi i k / n) from sincospi).  Every extent is
// a power of two, so all index arithmetic is shifts and masks.
constexpr int kFftLog2Lds = 11;
static_assert((1 << kFftLog2Lds) == kFftLds, "kFftLds is 2^kFftLog2Lds");
// Where a pass takes its input (its output always goes to data):
//  kData     data itself;
//  kCharge   the fixed-point TSC charge (line l = ix nc + iy of a z pass over iy < nc, point iz: the
//            node l nc + iz for iz < nc, zero beyond), which it clears for the next step;
//  kZeroPad  data for points p < nc and zero beyond (a y pass of the charge: iy >= nc is empty);
//  kMul2     a g1 + i a g2 at the same node: two real fields in one transform (the charge and
//            both Green's functions are real on the mesh, so the inverse transforms of a g1 and of
//            a g2 are real and that of a g1 + i a g2 is E1 + i E2);
//  kMul      a g1 at the same node.
enum FftLoad : int { kData, kCharge, kZeroPad, kMul2, kMul };

struct FftSrc {
  const void *a, *g1, *g2;          // kMul2 / kMul operands (mesh type)
  unsigned long long *qmesh;        // kCharge: fixed-point charge, nx x nc x nc
  const double *q_scale;            // kCharge: fixed-point units per unit of scaled charge
  int nc;                           // kCharge / kZeroPad: populated extent across the section
};

template <class T, int LOAD>
__global__ __launch_bounds__(256) void k_fft_lines(T *__restrict__ data, int log2n, int log2inner,
                                                   int64_t inner_stride, int64_t outer_stride, int64_t point_stride,
                                                   int sign, int points_contiguous, FftSrc src) {
  __shared__ T buf[kFftLds];
  __shared__ T tw[kFftLds / 2];
  const int n = 1 << log2n;
  const int log2lpw = kFftLog2Lds - log2n;   // lines per workgroup: 2^log2lpw
  const int64_t l0 = (int64_t)blockIdx.x << log2lpw;
  const int64_t inner_mask = ((int64_t)1 << log2inner) - 1;
  for (int k = threadIdx.x; k < n / 2; k += blockDim.x) {
    double s, c;
    sincospi(2.0 * k / n, &s, &c);
    tw[k] = cplx<T>(c, sign * s);   // in FP64, then rounded to the mesh type
  }
  auto addr = [&](int line, int p) {
    const int64_t l = l0 + line;
    return (l >> log2inner) * outer_stride + (l & inner_mask) * inner_stride + (int64_t)p * point_stride;
  };
  const int lmask = (1 << log2lpw) - 1, pmask = n - 1;
  for (int e = threadIdx.x; e < kFftLds; e += blockDim.x) {
    const int line = points_contiguous ? e >> log2n : e & lmask;
    const int p = points_contiguous ? e & pmask : e >> log2lpw;
    const int rev = (int)(__brev((unsigned)p) >> (32 - log2n));
    T v;
    if constexpr (LOAD == kData) {
      v = data[addr(line, p)];
    } else if constexpr (LOAD == kCharge) {
      v = cplx<T>(0.0, 0.0);
      if (p < src.nc) {
        const int64_t o = (l0 + line) * src.nc + p;
        v = cplx<T>((double)(long long)src.qmesh[o] / *src.q_scale, 0.0);
        src.qmesh[o] = 0ull;
      }
    } else if constexpr (LOAD == kZeroPad) {
      v = p < src.nc ? data[addr(line, p)] : cplx<T>(0.0, 0.0);
    } else {
      const int64_t o = addr(line, p);
      const T a = ((const T *)src.a)[o];
      const T pp = cmul(a, ((const T *)src.g1)[o]);
      if constexpr (LOAD == kMul2) {
        const T qq = cmul(a, ((const T *)src.g2)[o]);
        v = T{pp.x - qq.y, pp.y + qq.x};
      } else {
        v = pp;
      }
    }
    buf[(line << log2n) + rev] = v;
  }
  __syncthreads();
  // radix-2 stages lg and lg + 1 fused: each group of 4 points (i0, i0 + h, i0 + 2h, i0 + 3h),
  // h = 2^(lg-1), takes both stages' butterflies in registers -- the same operations in the
  // same order as two separate stages, with one LDS round trip and one barrier instead of two
  int lg = 1;
  for (; lg + 1 <= log2n; lg += 2) {
    const int half = 1 << (lg - 1);
    for (int b = threadIdx.x; b < kFftLds / 4; b += blockDim.x) {
      const int line = b >> (log2n - 2), k = b & ((n >> 2) - 1);
      const int pos = k & (half - 1);
      const int i0 = (line << log2n) + ((k >> (lg - 1)) << (lg + 1)) + pos;
      const T w1 = tw[pos << (log2n - lg)];
      const T w2a = tw[pos << (log2n - lg - 1)], w2b = tw[(pos + half) << (log2n - lg - 1)];
      const T a0 = buf[i0], a1 = buf[i0 + half], a2 = buf[i0 + 2 * half], a3 = buf[i0 + 3 * half];
      T v = cmul(w1, a1);
      const T b0 = cadd(a0, v), b1 = csub(a0, v);
      v = cmul(w1, a3);
      const T b2 = cadd(a2, v), b3 = csub(a2, v);
      v = cmul(w2a, b2);
      buf[i0] = cadd(b0, v);
      buf[i0 + 2 * half] = csub(b0, v);
      v = cmul(w2b, b3);
      buf[i0 + half] = cadd(b1, v);
      buf[i0 + 3 * half] = csub(b1, v);
    }
    __syncthreads();
  }
  if (lg == log2n) {   // odd log2n: the last radix-2 stage
    const int half = 1 << (lg - 1);
    for (int b = threadIdx.x; b < kFftLds / 2; b += blockDim.x) {
      const int line = b >> (log2n - 1), k = b & ((n >> 1) - 1);
      const int pos = k & (half - 1);
      const int i = (line << log2n) + ((k >> (lg - 1)) << lg) + pos;
      const T u = buf[i];
      const T v = cmul(tw[pos << (log2n - lg)], buf[i + half]);
      buf[i] = cadd(u, v);
      buf[i + half] = csub(u, v);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kFftLds; e += blockDim.x) {
    const int line = points_contiguous ? e >> log2n : e & lmask;
    const int p = points_contiguous ? e & pmask : e >> log2lpw;
    data[addr(line, p)] = buf[(line << log2n) + p];
  }
}

// TSC stencil of particle i: centre node (ix unwrapped in [0, nx], iy and iz clamped to
// [1, nc - 2]) and weights; false for a particle without charge.
template <class Real>
__device__ __forceinline__ bool tsc_stencil(const State<Real> &st, const Phys &ph, const P3mDev &m, int i, int &ix,
                                            int &iy, int &iz, double (&wx)[3], double (&wy)[3], double (&wz)[3]) {
  if (st.js[i].q == 0) return false;
  double gx, gy, gz;
  mesh_coords<Real>(st, ph, m, i, gx, gy, gz);
  tsc(gx, ix, wx);
  tsc(gy, iy, wy);
  tsc(gz, iz, wz);
  iy = min(max(iy, 1), m.nc - 2);   // suspended particles stay inside [-R, R]; the clamp only guards
  iz = min(max(iz, 1), m.nc - 2);
  return true;
}

// Fixed-point contribution of a particle to stencil node (a, b, c), units of the per-sample
// bound 2^-62 sum |q~|.
__device__ __forceinline__ unsigned long long tsc_part(double q, const double (&wx)[3], const double (&wy)[3],
                                                       const double (&wz)[3], int a, int b, int c, double qs) {
  return (unsigned long long)__double2ll_rn(q * wx[a] * wy[b] * wz[c] * qs);
}

constexpr int kAsgCap = 4096;   // mesh nodes of the per-cell accumulation box (32 KB of LDS)

// TSC charge assignment in 64-bit fixed point, one workgroup per short-range cell: the cell's
// particles add their 27 stencil contributions to an LDS box spanning the cell's stencils (LDS
// atomics), and the box is added to the mesh with one global atomic per touched node.  Integer
// additions commute, so the mesh is the same as with per-particle global atomics, which a cell
// whose box exceeds kAsgCap nodes uses instead.
template <class Real>
__global__ __launch_bounds__(256) void k_p3m_assign(State<Real> st, Phys ph, P3mDev m,
                                                    const int32_t *__restrict__ starts,
                                                    const int32_t *__restrict__ sorted,
                                                    unsigned long long *__restrict__ qmesh) {
  __shared__ unsigned long long box[kAsgCap];
  __shared__ int lo[3], hi[3];
  const int cell = blockIdx.x;
  const int b0 = starts[cell], n = starts[cell + 1] - b0;
  if (n == 0) return;   // uniform
  const double qs = *m.q_scale;
  if (threadIdx.x < 3) {
    lo[threadIdx.x] = INT_MAX;
    hi[threadIdx.x] = INT_MIN;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    int ix, iy, iz;
    double wx[3], wy[3], wz[3];
    if (!tsc_stencil<Real>(st, ph, m, sorted[b0 + k], ix, iy, iz, wx, wy, wz)) continue;
    atomicMin(&lo[0], ix); atomicMax(&hi[0], ix);
    atomicMin(&lo[1], iy); atomicMax(&hi[1], iy);
    atomicMin(&lo[2], iz); atomicMax(&hi[2], iz);
  }
  __syncthreads();
  if (lo[0] > hi[0]) return;   // uniform: no charged particle
  const int ex = hi[0] - lo[0] + 3, ey = hi[1] - lo[1] + 3, ez = hi[2] - lo[2] + 3;
  const int64_t vol = (int64_t)ex * ey * ez;
  if (vol > kAsgCap) {   // uniform: per-particle global atomics
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const int i = sorted[b0 + k];
      int ix, iy, iz;
      double wx[3], wy[3], wz[3];
      if (!tsc_stencil<Real>(st, ph, m, i, ix, iy, iz, wx, wy, wz)) continue;
      const double q = (double)st.js[i].q;
      for (int a = 0; a < 3; ++a) {
        int jx = ix + a - 1;
        jx = jx < 0 ? jx + m.nx : (jx >= m.nx ? jx - m.nx : jx);
        for (int b = 0; b < 3; ++b)
          for (int c = 0; c < 3; ++c)
            atomicAdd(qmesh + ((int64_t)jx * m.nc + (iy + b - 1)) * m.nc + (iz + c - 1),
                      tsc_part(q, wx, wy, wz, a, b, c, qs));
      }
    }
    return;
  }
  for (int e = threadIdx.x; e < vol; e += blockDim.x) box[e] = 0ull;
  __syncthreads();
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int i = sorted[b0 + k];
    int ix, iy, iz;
    double wx[3], wy[3], wz[3];
    if (!tsc_stencil<Real>(st, ph, m, i, ix, iy, iz, wx, wy, wz)) continue;
    const double q = (double)st.js[i].q;
    // box coordinates of the stencil's first node: (ix - 1 - (lo - 1), ...) = (ix - lo, ...)
    const int bx = ix - lo[0], by = iy - lo[1], bz = iz - lo[2];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c)
          atomicAdd(&box[((bx + a) * ey + (by + b)) * ez + (bz + c)], tsc_part(q, wx, wy, wz, a, b, c, qs));
  }
  __syncthreads();
  for (int e = threadIdx.x; e < vol; e += blockDim.x) {
    const unsigned long long v = box[e];
    if (v == 0ull) continue;
    const int c = e % ez, b = (e / ez) % ey, a = e / (ey * ez);
    int jx = lo[0] - 1 + a;
    jx = jx < 0 ? jx + m.nx : (jx >= m.nx ? jx - m.nx : jx);
    atomicAdd(qmesh + ((int64_t)jx * m.nc + (lo[1] - 1 + b)) * m.nc + (lo[2] - 1 + c), v);
  }
}

// TSC interpolation of the unnormalised inverse transform: its real part to out_re and, when
// out_im is given, its imaginary part (a second real field) to out_im.
template <class Real>
__global__ void k_p3m_interp(State<Real> st, Phys ph, P3mDev m, const int32_t *__restrict__ order,
                             const MeshT<Real> *__restrict__ E, double *__restrict__ out_re,
                             double *__restrict__ out_im) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;   // cell order, for locality of the mesh reads
  if (k >= ph.N) return;
  const int i = order[k];
  double gx, gy, gz, wx[3], wy[3], wz[3];
  int ix, iy, iz;
  mesh_coords<Real>(st, ph, m, i, gx, gy, gz);
  tsc(gx, ix, wx);
  tsc(gy, iy, wy);
  tsc(gz, iz, wz);
  iy = min(max(iy, 1), m.nc - 2);
  iz = min(max(iz, 1), m.nc - 2);
  double s = 0.0, t = 0.0;
  for (int a = 0; a < 3; ++a) {
    int jx = ix + a - 1;
    jx = jx < 0 ? jx + m.nx : (jx >= m.nx ? jx - m.nx : jx);
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        const double w = wx[a] * wy[b] * wz[c];
        const MeshT<Real> v = E[((int64_t)jx * m.P + (iy + b - 1)) * m.P + (iz + c - 1)];
        s += w * (double)v.x;
        t += w * (double)v.y;
      }
  }
  const double norm = 1.0 / ((double)m.nx * m.P * m.P);
  out_re[i] = s * norm;
  if (out_im) out_im[i] = t * norm;
}

// Short-range cell of a particle (cells of at least r_max; x periodic).
template <class Real>
__device__ __forceinline__ int3 sr_cell(const State<Real> &st, const Phys &ph, const P3mDev &m, int i) {
  using SPos = typename std::make_signed<typename Prec<Real>::Pos>::type;
  const double x = ((double)st.px[i] + (double)st.rx[i]) * ph.ux;
  const double y = ((double)(SPos)st.py[i] + (double)st.ry[i]) * ph.ur;
  const double z = ((double)(SPos)st.pz[i] + (double)st.rz[i]) * ph.ur;
  int cx = (int)(x / ph.L * m.ncx), cy = (int)((y + ph.R) / (2.0 * ph.R) * m.ncy),
      cz = (int)((z + ph.R) / (2.0 * ph.R) * m.ncy);
  cx = min(max(cx, 0), m.ncx - 1);
  cy = min(max(cy, 0), m.ncy - 1);
  cz = min(max(cz, 0), m.ncy - 1);
  return make_int3(cx, cy, cz);
}

// Adds 1 to ctr[key] for every active lane with one atomic per distinct key in the wave (the
// particles of a wave often share a cell: the storage follows the cells).  Returns the counter's
// value before the lane's own increment; the lanes of one key take consecutive values in lane
// order.  Lanes outside the execution mask take no part.
__device__ __forceinline__ int32_t wave_count_add(int32_t *__restrict__ ctr, int key, bool active) {
  const int lane = (int)(threadIdx.x & 63);
  uint64_t todo = __builtin_amdgcn_ballot_w64(active);
  int32_t mine = 0;
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const int lkey = __builtin_amdgcn_readlane(key, leader);
    const uint64_t grp = __builtin_amdgcn_ballot_w64(active && key == lkey) & todo;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(ctr + lkey, (int32_t)__builtin_popcountll(grp));
    base = __builtin_amdgcn_readlane(base, leader);
    if ((grp >> lane) & 1)
      mine = base + (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(grp >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)grp, 0u));
    todo &= ~grp;
  }
  return mine;
}

// Cell id and sub-cell key of the particle, packed as 64 id + key.  The key orders the 4 x 4 x 4
// sub-cells of a cell along a Morton curve (bits: the halves along x, y, z, then the quarters
// within them), so that consecutive particles of the cell-sorted order lie close together.
template <class Real>
__global__ void k_p3m_bin(State<Real> st, Phys ph, P3mDev m, int32_t *__restrict__ cell_of,
                          int32_t *__restrict__ counts) {
  using SPos = typename std::make_signed<typename Prec<Real>::Pos>::type;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  const int3 c = sr_cell<Real>(st, ph, m, i);
  const int id = (c.x * m.ncy + c.y) * m.ncy + c.z;
  const double x = ((double)st.px[i] + (double)st.rx[i]) * ph.ux;
  const double y = ((double)(SPos)st.py[i] + (double)st.ry[i]) * ph.ur;
  const double z = ((double)(SPos)st.pz[i] + (double)st.rz[i]) * ph.ur;
  auto quarter = [](double f) { return min(max((int)(4.0 * f), 0), 3); };
  const int qx = quarter(x / ph.L * m.ncx - c.x), qy = quarter((y + ph.R) / (2.0 * ph.R) * m.ncy - c.y),
            qz = quarter((z + ph.R) / (2.0 * ph.R) * m.ncy - c.z);
  const int key = ((qx >> 1) << 5) | ((qy >> 1) << 4) | ((qz >> 1) << 3) | ((qx & 1) << 2) | ((qy & 1) << 1) | (qz & 1);
  cell_of[i] = 64 * id + key;
  wave_count_add(counts, id, true);
}

// Exclusive scan of the cell counts by one workgroup; starts[ncell] = N; fill pointers copied.
__global__ __launch_bounds__(1024) void k_p3m_scan(int32_t ncell, const int32_t *__restrict__ counts,
                                                   int32_t *__restrict__ starts, int32_t *__restrict__ fill) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int per = (ncell + 1023) / 1024;
  const int b = t * per, e = min(ncell, b + per);
  int32_t s = 0;
  for (int k = b; k < e; ++k) s += counts[k];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = part[t] - s;
  for (int k = b; k < e; ++k) {
    starts[k] = run;
    fill[k] = run;
    run += counts[k];
  }
  if (t == 1023) starts[ncell] = part[1023];
}

__global__ void k_p3m_scatter(int32_t N, const int32_t *__restrict__ cell_of, int32_t *__restrict__ fill,
                              int32_t *__restrict__ sorted) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < N;
  const int slot = wave_count_add(fill, active ? cell_of[i] >> 6 : 0, active);
  if (active) sorted[slot] = i;
}

// Particles of each cell ordered by (sub-cell key, index): a fixed summation order in which
// consecutive targets of the short-range pass are close together.  The counts are cleared.  One
// workgroup per cell: the cell's keys (sub-cell key, index; distinct) are staged in LDS and each
// particle is written to its rank (the number of smaller keys).  A cell of more than kSortCap
// particles is sorted by one thread.
constexpr int kSortCap = 2048;
__global__ __launch_bounds__(256) void k_p3m_sort(int32_t ncell, const int32_t *__restrict__ starts,
                                                  int32_t *__restrict__ sorted, int32_t *__restrict__ counts,
                                                  const int32_t *__restrict__ cell_of) {
  __shared__ int64_t v[kSortCap];
  const int c = blockIdx.x;
  const int b = starts[c], n = starts[c + 1] - b;
  auto key = [&](int i) { return ((int64_t)(cell_of[i] & 63) << 32) | (int64_t)i; };
  if (threadIdx.x == 0) counts[c] = 0;
  if (n <= 1) return;   // uniform
  if (n > kSortCap) {
    if (threadIdx.x == 0) {
      for (int k = b + 1; k < b + n; ++k) {
        const int x = sorted[k];
        const int64_t kx = key(x);
        int j = k - 1;
        while (j >= b && key(sorted[j]) > kx) {
          sorted[j + 1] = sorted[j];
          --j;
        }
        sorted[j + 1] = x;
      }
    }
    return;
  }
  for (int e = threadIdx.x; e < n; e += blockDim.x) v[e] = key(sorted[b + e]);
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int64_t x = v[e];
    int rank = 0;
    for (int k = 0; k < n; ++k) rank += v[k] < x ? 1 : 0;
    sorted[b + rank] = (int32_t)(x & 0xffffffff);
  }
}

// Source record of the short-range pass in the FP64 form, in cell-sorted order.
struct __align__(8) SrRec64 {
  uint64_t x;        // fixed-point position: x as the unsigned fraction of L,
  int64_t y, z;      // y and z as signed multiples of the y/z quantum
  double q, d;       // scaled charge, diameter [m]
};

// Cell-sorted copy of the records the short-range pass reads (contiguous per cell).
// FP64 form: one SrRec64 per particle.  FP32 form: a 16-byte record (x bits; y and z as floats in
// y/z position quanta, so that the short-range body takes their differences with one subtraction;
// scaled charge) read by every pair with one LDS load, and the radius in y/z position quanta in an
// array of its own, read only for pairs that may overlap; both arrays share the record region
// (16 N bytes, then 4 N).
template <class Real>
__global__ void k_p3m_records(State<Real> st, Phys ph, const int32_t *__restrict__ sorted, void *rec) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ph.N) return;
  const int i = sorted[k];
  using SPos = typename std::make_signed<typename Prec<Real>::Pos>::type;
  if constexpr (sizeof(Real) == 4) {
    float4 r;
    r.x = __uint_as_float(st.px[i]);
    r.y = (float)((double)(SPos)st.py[i] + (double)st.ry[i]);
    r.z = (float)((double)(SPos)st.pz[i] + (double)st.rz[i]);
    r.w = st.js[i].q;
    ((float4 *)rec)[k] = r;
    ((float *)((float4 *)rec + ph.N))[k] = (float)(0.5 * st.d[i] * ph.inv_ur);
  } else {
    SrRec64 r;
    r.x = st.px[i];
    r.y = (SPos)st.py[i];
    r.z = (SPos)st.pz[i];
    r.q = st.js[i].q;
    r.d = st.d[i];
    ((SrRec64 *)rec)[k] = r;
  }
}

constexpr int kSrLds = 65536;    // bytes of LDS for staged neighbour records (FP64 form)
constexpr int kSrWaves = 8;      // waves per cell
constexpr int kSrLanes = 64 * kSrWaves;
constexpr int kSrMaxSlices = 32; // FP64 form: at most this many threads share one target
constexpr int kSrTable = 2048;   // intervals of the tabulated short-range profile (FP32 form)
// FP32 form: 28,000 B of staged records + 16.4 KB of table + 7 KB of source lists keep a workgroup
// within a third of the 160 KB LDS, so three workgroups (24 waves) share a CU
constexpr int kSrLdsF32 = 28000;
constexpr int kSrCluster = 8;                     // FP32 form: targets of one wave (a cluster)
constexpr int kSrSlices = 64 / kSrCluster;        // lanes per target
constexpr int kSrRounds = 64;                     // clusters per wave and staging pass
constexpr int kSrList = 448;                      // entries of a wave's source list

// Short-range force profile g(s) = erfc(s) + (2 s / sqrt(pi)) exp(-s^2), s = alpha r, so that the
// short-range force of a non-overlapping pair is q g(alpha r) r_vec / r^3; tabulated on
// [0, alpha r_max] in kSrTable intervals as (g at the interval start, increment over the
// interval) for linear interpolation in the table coordinate u = kSrTable r / r_max
// (interpolation error at most h^2 |g''| / 8 of the pair force with |g''| < 1.2 and the step
// h = alpha r_max / kSrTable: 4.4e-7 at alpha r_max = 3.5); entry kSrTable is (0, 0): pairs at or
// beyond r_max get nothing.
__global__ void k_p3m_table(P3mDev m, float2 *__restrict__ tab) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > kSrTable) return;
  if (k == kSrTable) { tab[k] = make_float2(0.0f, 0.0f); return; }
  const double hs = m.alpha * m.rmax / kSrTable;
  auto g = [](double x) { return erfc(x) + 2.0 / sqrt(M_PI) * x * exp(-x * x); };
  const double s0 = k * hs, g0 = g(s0), g1 = g(s0 + hs);
  tab[k] = make_float2((float)g0, (float)(g1 - g0));
}

// The 27 cells around cell c (periodic in x; none beyond the section) as ranges of the
// cell-sorted records: begin rb, count rn and offset roff in their concatenation (roff[27] is the
// total).  Called by every thread; returns after a barrier.
__device__ __forceinline__ void neighbour_ranges(const P3mDev &m, const int32_t *__restrict__ starts, int cx,
                                                 int cy, int cz, int32_t *rb, int32_t *rn, int32_t *roff) {
  if (threadIdx.x < 27) {
    const int ox = (int)threadIdx.x / 9 - 1, oy = ((int)threadIdx.x / 3) % 3 - 1, oz = (int)threadIdx.x % 3 - 1;
    int x = cx + ox;
    x = x < 0 ? x + m.ncx : (x >= m.ncx ? x - m.ncx : x);
    const int y = cy + oy, z = cz + oz;
    int b = 0, n = 0;
    if (y >= 0 && y < m.ncy && z >= 0 && z < m.ncy) {
      const int id = (x * m.ncy + y) * m.ncy + z;
      b = starts[id];
      n = starts[id + 1] - b;
    }
    rb[threadIdx.x] = b;
    rn[threadIdx.x] = n;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    roff[0] = 0;
    for (int k = 0; k < 27; ++k) roff[k + 1] = roff[k] + rn[k];
  }
  __syncthreads();
}

// Stage entries [cb, cb + n) of the concatenated 27 cell ranges into LDS, cell by cell (and,
// when rad is given, the radii beside them).
template <class Rec>
__device__ __forceinline__ void stage_sources(const Rec *__restrict__ rec, const float *__restrict__ rad,
                                              const int32_t *rb, const int32_t *roff, int cb, int n, Rec *src,
                                              float *srad) {
  __syncthreads();
  for (int k = 0; k < 27; ++k) {
    const int lo = max(roff[k], cb), hi = min(roff[k + 1], cb + n);
    for (int q = lo + (int)threadIdx.x; q < hi; q += blockDim.x) {
      src[q - cb] = rec[rb[k] + (q - roff[k])];
      if (rad) srad[q - cb] = rad[rb[k] + (q - roff[k])];
    }
  }
  __syncthreads();
}

// Short range (Coulomb with the overlap clamp minus the erf field) over nearest-image neighbours
// closer than r_max, added to the long-range part; result in units of the x quantum.
//
// FP64 form: the exact expressions, in metres.  One workgroup per cell: the records of the 27
// neighbouring cells are staged in LDS (in chunks when they exceed it); the cell's nb targets (up
// to 512 at a time) share the 512 threads, S = 512 / nb threads per target (at most 32), and
// thread g takes target g mod nb and every S-th staged source from slice g / nb on; the S partial
// sums of a target are combined in FP64 in slice order.
__global__ __launch_bounds__(kSrLanes) void k_p3m_short_f64(State<double> st, Phys ph, P3mDev m,
                                                            const int32_t *__restrict__ starts,
                                                            const int32_t *__restrict__ sorted,
                                                            const SrRec64 *__restrict__ rec,
                                                            const double *__restrict__ slong) {
  constexpr int CAP = kSrLds / sizeof(SrRec64);
  __shared__ SrRec64 src[CAP];
  __shared__ double part[3][kSrLanes];
  __shared__ int32_t rb[27], rn[27], roff[28];
  const int c = blockIdx.x;
  const int cz = c % m.ncy, cy = (c / m.ncy) % m.ncy, cx = c / (m.ncy * m.ncy);
  const int t0 = starts[c], nt = starts[c + 1] - t0;
  if (nt == 0) return;   // uniform: the whole workgroup leaves
  neighbour_ranges(m, starts, cx, cy, cz, rb, rn, roff);
  const int total = roff[27];
  const double ux = ph.ux, ur = ph.ur;
  const double a = m.alpha, c2 = 2.0 * m.alpha / sqrt(M_PI), rmax2 = m.rmax * m.rmax;
  const bool once = total <= CAP;   // all sources fit: staged once for every target block
  for (int tb = 0; tb < nt; tb += kSrLanes) {
    const int nb = min(kSrLanes, nt - tb);
    const int S = min(kSrLanes / nb, kSrMaxSlices);   // threads per target
    const int g = threadIdx.x;
    const bool has = g < nb * S;
    const int t = has ? g % nb : 0, slice = has ? g / nb : 0;
    const SrRec64 me = rec[t0 + tb + t];
    double sx = 0, sy = 0, sz = 0;
    for (int cb = 0; cb < total; cb += CAP) {
      const int n = min(CAP, total - cb);
      if (!once || tb == 0) stage_sources(rec, (const float *)nullptr, rb, roff, cb, n, src, (float *)nullptr);
      if (!has) continue;
      for (int e = slice; e < n; e += S) {
        const SrRec64 s = src[e];
        const double dx = double((int64_t)(me.x - s.x)) * ux;
        const double dy = double(me.y - s.y) * ur;
        const double dz = double(me.z - s.z) * ur;
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double dij = 0.5 * (me.d + s.d);
        double f = 0.0;
        if (r2 < rmax2 && r2 > 0.0) {
          const double r = sqrt(r2);
          const double gg = c2 * exp(-a * a * r2) / r;
          f = (r >= dij ? erfc(a * r) / r2 + gg : 1.0 / (dij * dij) - (erf(a * r) / r2 - gg)) * s.q / r;
        }
        sx += f * dx;
        sy += f * dy;
        sz += f * dz;
      }
    }
    part[0][g] = sx;
    part[1][g] = sy;
    part[2][g] = sz;
    __syncthreads();
    if (g < nb) {
      double ax = 0.0, ay = 0.0, az = 0.0;
      for (int q = 0; q < S; ++q) {
        ax += part[0][q * nb + g];
        ay += part[1][q * nb + g];
        az += part[2][q * nb + g];
      }
      const int i = sorted[t0 + tb + g];
      const double u2 = ph.ux * ph.ux;
      st.cx[i] = slong[i] * u2 + ax * u2;
      st.cy[i] = slong[ph.N + i] * u2 + ay * u2;
      st.cz[i] = slong[2 * (int64_t)ph.N + i] * u2 + az * u2;
    }
    __syncthreads();
  }
}

// FP32 form, in y/z position quanta, with per-wave source lists.  One workgroup per cell, whose
// targets (sorted by sub-cell key) are cut into clusters of kSrCluster consecutive targets; a wave
// takes one cluster at a time, lane l pairing target l mod 8 of it with every 8th source of the
// wave's list from l / 8 on.  The records of the 27 neighbouring cells are staged in LDS (in
// chunks when they exceed it); for each staged chunk a wave lists the sources within r_max of its
// cluster's bounding box (the distance from a point to a box is a lower bound of its distance to
// every target in the box), so sources that cannot reach any target of the cluster are never
// paired.  Every source left out would add an exact zero (it lies beyond r_max, where the profile
// table ends in (0, 0)), so the set of contributing pairs is that of the 27-cell walk.  Each lane
// sums its pairs of a chunk in FP32 in list order; the 8 lane sums of a target are added in FP64
// by a butterfly and then to the target's long-range part (in FP64, chunk by chunk; the last
// chunk writes the acceleration), a fixed order: the results are bitwise reproducible.  Pairs take
// the tabulated profile from a copy of the table in LDS; overlapping pairs, which are rare, take
// the exact clamp.  The list holds byte offsets of the staged records and is padded with a far,
// uncharged dummy record (it adds an exact zero), so that every lane of the wave runs the same
// iterations; the loop loads the next list entries and their records while it evaluates the
// current ones.
__global__ __launch_bounds__(kSrLanes) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_p3m_short_f32(State<float> st, Phys ph, P3mDev m,
                                                            const int32_t *__restrict__ starts,
                                                            const int32_t *__restrict__ sorted,
                                                            const float4 *__restrict__ rec,
                                                            const float *__restrict__ rad,
                                                            double *__restrict__ slong,
                                                            const float2 *__restrict__ tab) {
  constexpr int CAP = kSrLdsF32 / (sizeof(float4) + sizeof(float)) - 1;
  static_assert((CAP + 1) * sizeof(float4) <= 65536, "list entries are 16-bit byte offsets");
  __shared__ float4 src[CAP + 1];   // entry CAP: the dummy record
  __shared__ float srad[CAP + 1];
  __shared__ float2 stab[kSrTable + 1];
  __shared__ uint16_t list[kSrWaves][kSrList];
  __shared__ int32_t rb[27], rn[27], roff[28];
  const int c = blockIdx.x;
  const int cz = c % m.ncy, cy = (c / m.ncy) % m.ncy, cx = c / (m.ncy * m.ncy);
  const int t0 = starts[c], nt = starts[c + 1] - t0;
  if (nt == 0) return;   // uniform: the whole workgroup leaves
  for (int k = threadIdx.x; k <= kSrTable; k += kSrLanes) stab[k] = tab[k];   // read after the barriers below
  if (threadIdx.x == 0) {
    // far (r^2 ~ 1e36, finite) and uncharged: its pairs fall past the table's end and add 0
    src[CAP] = make_float4(0.0f, 1.0e18f, 1.0e18f, 0.0f);
    srad[CAP] = 0.0f;
  }
  neighbour_ranges(m, starts, cx, cy, cz, rb, rn, roff);
  const int total = roff[27];
  const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
  const int tl = lane & (kSrCluster - 1), sl = lane / kSrCluster;   // target in the cluster, slice
  uint16_t *wl = list[wave];
  // x differences scaled by u_x / u_r, alpha per quantum, table coordinate u = r * tq, the largest
  // contact distance squared (uniform: held in scalar registers)
  auto uniform = [](double v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int((float)v))); };
  const float kx = uniform(ph.ux / ph.ur), aq = uniform(m.alpha * ph.ur), c2q = uniform(2.0 * m.alpha * ph.ur / sqrt(M_PI));
  const float tq = uniform(kSrTable * ph.ur / m.rmax);
  const float near2q = uniform(ph.near2 * (ph.ux / ph.ur) * (ph.ux / ph.ur));
  // beyond this (r_max squared in quanta, plus 1e-4 for rounding) the table coordinate u is surely
  // past the last interval, so the pair adds an exact zero
  const float skip2q = uniform((m.rmax / ph.ur) * (m.rmax / ph.ur) * 1.0001);
  // With at least 4 cells along x, three neighbouring cells cannot reach around the period, so an
  // x offset taken relative to the cluster's first target is the pair's own minimum-image offset
  // up to a whole period that puts the pair beyond r_max; with 3 cells the x extent is not used.
  const bool use_x = m.ncx >= 4;
  const int ncl = (nt + kSrCluster - 1) / kSrCluster;
  const bool once = total <= CAP;   // all sources fit: staged once for the whole cell
  const double u2 = ph.ux * ph.ux;
  // the sums are in y/z quanta: 1 / u_r^2 takes them to the units of the long-range part
  const double us = 1.0 / (ph.ur * ph.ur);
  for (int pass = 0; pass < ncl; pass += kSrWaves * kSrRounds) {
    for (int cb = 0; cb < total; cb += CAP) {
      const int n = min(CAP, total - cb);
      const bool last = cb + n >= total;
      if (!once || pass == 0) stage_sources(rec, rad, rb, roff, cb, n, src, srad);
#pragma unroll 1
      for (int r = 0; r < kSrRounds; ++r) {
        const int q = pass + r * kSrWaves + wave;   // this wave's cluster (wave-uniform)
        if (q >= ncl) break;
        const int ti = min(q * kSrCluster + tl, nt - 1);   // a short cluster repeats its last target
        const float4 me = rec[t0 + ti];
        const uint32_t mx = __float_as_uint(me.x);
        const uint32_t xref = __float_as_uint(rec[t0 + q * kSrCluster].x);
        // the cluster's bounding box (x relative to its first target), reduced over the 8 targets
        float lo[3], hi[3];
        lo[0] = hi[0] = (float)(int32_t)(mx - xref) * kx;
        lo[1] = hi[1] = me.y;
        lo[2] = hi[2] = me.z;
#pragma unroll
        for (int k = 1; k < kSrCluster; k <<= 1)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], k));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], k));
          }
        // the box is the same in every lane: kept in scalar registers
        float bc[3], bh[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          bc[a] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(0.5f * (lo[a] + hi[a]))));
          bh[a] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(0.5f * (hi[a] - lo[a]))));
        }
        if (!use_x) bh[0] = 3.0e38f;
        float sx = 0.0f, sy = 0.0f, sz = 0.0f;
        int cnt = 0;   // entries in the wave's list (wave-uniform)
        for (int e0 = 0; e0 < n; e0 += 64) {
          const int e = e0 + lane;
          bool ok = false;
          if (e < n) {
            const float4 s = src[e];
            const float gx = fmaxf(fabsf((float)(int32_t)(__float_as_uint(s.x) - xref) * kx - bc[0]) - bh[0], 0.0f);
            const float gy = fmaxf(fabsf(s.y - bc[1]) - bh[1], 0.0f);
            const float gz = fmaxf(fabsf(s.z - bc[2]) - bh[2], 0.0f);
            ok = fmaf(gx, gx, fmaf(gy, gy, gz * gz)) < skip2q;
          }
          const uint64_t mask = __builtin_amdgcn_ballot_w64(ok);
          if (ok)
            wl[cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u))] =
                (uint16_t)(e * sizeof(float4));
          cnt += __builtin_popcountll(mask);
          if (cnt <= kSrList - 64 - 4 * kSrSlices && e0 + 64 < n) continue;
          // pair the cluster with the listed sources, then empty the list: iterations of 8 entries,
          // taken two at a time and loaded two iterations ahead, so the list is padded with 32
          // dummy entries (every entry read lies below cnt + 32)
          const int iters = (cnt + kSrSlices - 1) / kSrSlices;
          if (lane < 4 * kSrSlices) wl[cnt + lane] = (uint16_t)(CAP * sizeof(float4));
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          auto pair = [&](const float4 cur, uint32_t off) {
            // r2 carries 1e-20 (below the rounding of any r2 >= 1, i.e. of any two distinct
            // positions) so that r = 0 (the target itself) gives a finite f times dx = 0
            const float dx = (float)(int32_t)(mx - __float_as_uint(cur.x)) * kx;
            const float dy = me.y - cur.y;
            const float dz = me.z - cur.z;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, 1e-20f)));
            if (!__builtin_amdgcn_ballot_w64(r2 < skip2q)) return;   // no lane within r_max
            const float inv = __builtin_amdgcn_rsqf(r2);
            const float rr = r2 * inv;
            const float u = fminf(rr * tq, (float)kSrTable);   // u >= kSrTable: beyond r_max, entry (0, 0)
            const float2 tv = stab[(int)u];
            float f = cur.w * fmaf(__builtin_amdgcn_fractf(u), tv.y, tv.x) * ((inv * inv) * inv);
            if (__builtin_amdgcn_ballot_w64(r2 < near2q)) {
              // a pair of this source may overlap: clamped Coulomb minus the erf field, exactly
              const float dij = rad[t0 + ti] + srad[off / sizeof(float4)];
              if (r2 > 1e-20f && rr < dij) {
                // 1/r = inv and 1/r^2 = inv^2 (from the rsq above, 1 ulp)
                const float gg = c2q * expf(-aq * aq * r2) * inv;
                f = cur.w * (1.0f / (dij * dij) - (erff(aq * rr) * (inv * inv) - gg)) * inv;
              }
            }
            sx = fmaf(f, dx, sx);
            sy = fmaf(f, dy, sy);
            sz = fmaf(f, dz, sz);
          };
          auto rec_at = [&](uint32_t off) { return *(const float4 *)((const char *)src + off); };
          uint32_t oa = wl[sl], ob = wl[kSrSlices + sl];
          float4 sa = rec_at(oa), sb = rec_at(ob);
          for (int k = 0; k < iters; k += 2) {
            const uint32_t na = wl[(k + 2) * kSrSlices + sl], nb = wl[(k + 3) * kSrSlices + sl];
            const float4 ca = sa, cb4 = sb;
            const uint32_t pa = oa, pb = ob;
            sa = rec_at(na);
            sb = rec_at(nb);
            oa = na;
            ob = nb;
            pair(ca, pa);
            if (k + 1 < iters) pair(cb4, pb);
          }
          cnt = 0;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // the 8 slices of each target, added in FP64 by a butterfly; slice 0 adds them to the
        // long-range part, and after the last chunk writes the acceleration
        double v[3] = {(double)sx, (double)sy, (double)sz};
#pragma unroll
        for (int k = kSrCluster; k < 64; k <<= 1)
#pragma unroll
          for (int a = 0; a < 3; ++a) v[a] += __shfl_xor(v[a], k);
        if (sl == 0 && q * kSrCluster + tl < nt) {
          const int i = sorted[t0 + q * kSrCluster + tl];
          const double lx = slong[i] + v[0] * us, ly = slong[ph.N + i] + v[1] * us,
                       lz = slong[2 * (int64_t)ph.N + i] + v[2] * us;
          if (last) {
            st.cx[i] = (float)(lx * u2);
            st.cy[i] = (float)(ly * u2);
            st.cz[i] = (float)(lz * u2);
          } else {
            slong[i] = lx;
            slong[ph.N + i] = ly;
            slong[2 * (int64_t)ph.N + i] = lz;
          }
        }
      }
    }
  }
}

int ilog2(int n) {
  int k = 0;
  while ((1 << k) < n) ++k;
  return k;
}

// Which lines of a 3D transform are needed.  The charge occupies iy, iz < nc of the padded mesh,
// so its forward z pass reads the fixed-point charge directly (the lines iy >= nc are all zero and
// are not stored: the y pass takes them as zero); the fields are read back only at iy, iz < nc,
// so their inverse y pass needs the lines iz < nc and the x pass the lines iy, iz < nc, and their
// z pass forms the spectral product as it loads.  The Green's function set-up transforms every
// line of data in place.
enum class FftLines { kAll, kChargeForward, kFieldInverse };

// 3D transform of the padded mesh: lines along z, y, x.  first: the load mode of the z pass
// (kData, kCharge for the charge, kMul2 / kMul for the fields).
template <class T> void fft3d(const P3mDev &m, T *d, int sign, FftLines which, int first, const FftSrc &src,
                              hipStream_t s) {
  const int64_t P = m.P, nx = m.nx, nc = m.nc;
  const int lp = ilog2((int)P), lx = ilog2((int)nx), lc = ilog2((int)nc);
  auto grid = [](int64_t points) { return dim3((unsigned)(points / kFftLds)); };
  if (which == FftLines::kChargeForward)   // z: line (ix, iy < nc) at ix P^2 + iy P, points contiguous
    hipLaunchKernelGGL((k_fft_lines<T, kCharge>), grid(nx * nc * P), dim3(256), 0, s, d, lp, lc, P, P * P,
                       (int64_t)1, sign, 1, src);
  else if (first == kMul2)   // z: line l at l P, points contiguous
    hipLaunchKernelGGL((k_fft_lines<T, kMul2>), grid(nx * P * P), dim3(256), 0, s, d, lp, 0, (int64_t)0, P,
                       (int64_t)1, sign, 1, src);
  else if (first == kMul)
    hipLaunchKernelGGL((k_fft_lines<T, kMul>), grid(nx * P * P), dim3(256), 0, s, d, lp, 0, (int64_t)0, P,
                       (int64_t)1, sign, 1, src);
  else
    hipLaunchKernelGGL((k_fft_lines<T, kData>), grid(nx * P * P), dim3(256), 0, s, d, lp, 0, (int64_t)0, P,
                       (int64_t)1, sign, 1, src);
  if (which == FftLines::kFieldInverse)    // y: line (ix, iz < nc) at ix P^2 + iz, points P apart
    hipLaunchKernelGGL((k_fft_lines<T, kData>), grid(nx * nc * P), dim3(256), 0, s, d, lp, lc, (int64_t)1, P * P,
                       P, sign, 0, src);
  else if (which == FftLines::kChargeForward)   // y: line (ix, iz), points iy >= nc taken as zero
    hipLaunchKernelGGL((k_fft_lines<T, kZeroPad>), grid(nx * P * P), dim3(256), 0, s, d, lp, lp, (int64_t)1,
                       P * P, P, sign, 0, src);
  else   // y: line (ix, iz) at ix P^2 + iz, points P apart
    hipLaunchKernelGGL((k_fft_lines<T, kData>), grid(nx * P * P), dim3(256), 0, s, d, lp, lp, (int64_t)1, P * P,
                       P, sign, 0, src);
  if (which == FftLines::kFieldInverse)    // x: line (iy < nc, iz < nc) at iy P + iz, points P^2 apart
    hipLaunchKernelGGL((k_fft_lines<T, kData>), grid(nc * nc * nx), dim3(256), 0, s, d, lx, lc, (int64_t)1, P,
                       P * P, sign, 0, src);
  else   // x: line (iy, iz) at iy P + iz, points P^2 apart
    hipLaunchKernelGGL((k_fft_lines<T, kData>), grid(nx * P * P), dim3(256), 0, s, d, lx, 0, (int64_t)0,
                       (int64_t)1, P * P, sign, 0, src);
}

}  // namespace

void p3m_setup_green(const P3mDev &m, double L, int images, bool fp32_mesh, hipStream_t s) {
  const int64_t total = (int64_t)m.nx * m.P * m.P;
  const unsigned g = (unsigned)((total + 255) / 256);
  if (fp32_mesh) {
    // each component in FP64 in the rho + work region (one double2 mesh), then rounded
    double2 *tmp = (double2 *)m.rho;
    for (int c = 0; c < 3; ++c) {
      hipLaunchKernelGGL(k_p3m_green, dim3(g), dim3(256), 0, s, m, L, images, c, tmp, tmp, tmp);
      fft3d<double2>(m, tmp, -1, FftLines::kAll, kData, FftSrc{}, s);
      hipLaunchKernelGGL(k_p3m_deconv_f32, dim3(g), dim3(256), 0, s, m, tmp, (float2 *)m.ghat[c]);
    }
  } else {
    double2 *gh[3] = {(double2 *)m.ghat[0], (double2 *)m.ghat[1], (double2 *)m.ghat[2]};
    hipLaunchKernelGGL(k_p3m_green, dim3(g), dim3(256), 0, s, m, L, images, -1, gh[0], gh[1], gh[2]);
    for (int c = 0; c < 3; ++c) fft3d<double2>(m, gh[c], -1, FftLines::kAll, kData, FftSrc{}, s);
    hipLaunchKernelGGL(k_p3m_deconv, dim3(g), dim3(256), 0, s, m, gh[0], gh[1], gh[2]);
  }
  hipLaunchKernelGGL(k_p3m_table, dim3((kSrTable + 256) / 256), dim3(256), 0, s, m, m.table);
}

template <class Real> void launch_p3m(const State<Real> &st, const Phys &ph, const P3mDev &m, hipStream_t s) {
  if (ph.N <= 0) return;
  const unsigned gp = (unsigned)((ph.N + 255) / 256);
  // short-range cells first: the mesh passes also walk the particles in cell order
  const int ncell = m.ncx * m.ncy * m.ncy;
  hipLaunchKernelGGL((k_p3m_bin<Real>), dim3(gp), dim3(256), 0, s, st, ph, m, m.cell_of, m.counts);
  hipLaunchKernelGGL(k_p3m_scan, dim3(1), dim3(1024), 0, s, ncell, m.counts, m.starts, m.fill);
  hipLaunchKernelGGL(k_p3m_scatter, dim3(gp), dim3(256), 0, s, ph.N, m.cell_of, m.fill, m.sorted);
  hipLaunchKernelGGL(k_p3m_sort, dim3((unsigned)ncell), dim3(256), 0, s, ncell, m.starts, m.sorted, m.counts,
                     m.cell_of);
  hipLaunchKernelGGL((k_p3m_assign<Real>), dim3((unsigned)ncell), dim3(256), 0, s, st, ph, m, m.starts, m.sorted,
                     m.qmesh);
  using T = MeshT<Real>;
  T *rho = (T *)m.rho, *work = (T *)m.work;
  const T *g0 = (const T *)m.ghat[0], *g1 = (const T *)m.ghat[1], *g2 = (const T *)m.ghat[2];
  // forward transform of the charge, read from the fixed-point mesh by the first pass
  fft3d<T>(m, rho, -1, FftLines::kChargeForward, kCharge, FftSrc{nullptr, nullptr, nullptr, m.qmesh, m.q_scale, m.nc},
           s);
  // E_x + i E_y from one inverse transform, then E_z; the first pass forms the spectral product
  fft3d<T>(m, work, +1, FftLines::kFieldInverse, kMul2, FftSrc{rho, g0, g1, nullptr, nullptr, m.nc}, s);
  hipLaunchKernelGGL((k_p3m_interp<Real>), dim3(gp), dim3(256), 0, s, st, ph, m, m.sorted, work, m.slong,
                     m.slong + ph.N);
  fft3d<T>(m, work, +1, FftLines::kFieldInverse, kMul, FftSrc{rho, g2, nullptr, nullptr, nullptr, m.nc}, s);
  hipLaunchKernelGGL((k_p3m_interp<Real>), dim3(gp), dim3(256), 0, s, st, ph, m, m.sorted, work,
                     m.slong + 2 * (int64_t)ph.N, (double *)nullptr);
  hipLaunchKernelGGL((k_p3m_records<Real>), dim3(gp), dim3(256), 0, s, st, ph, m.sorted, m.rec);
  if constexpr (sizeof(Real) == 4) {
    const float4 *rec = (const float4 *)m.rec;
    hipLaunchKernelGGL(k_p3m_short_f32, dim3(ncell), dim3(kSrLanes), 0, s, st, ph, m, m.starts, m.sorted, rec,
                       (const float *)(rec + ph.N), m.slong, m.table);
  } else {
    hipLaunchKernelGGL(k_p3m_short_f64, dim3(ncell), dim3(kSrLanes), 0, s, st, ph, m, m.starts, m.sorted,
                       (const SrRec64 *)m.rec, m.slong);
  }
}

template void launch_p3m<float>(const State<float> &, const Phys &, const P3mDev &, hipStream_t);
template void launch_p3m<double>(const State<double> &, const Phys &, const P3mDev &, hipStream_t);

}  // namespace depo
