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
// Everything on the mesh is FP64: charge assignment adds 64-bit fixed-point
// weights with integer atomics (order independent), the FFTs are radix-2
// Cooley-Tukey passes over mesh lines staged in LDS, and the short-range sum is
// a gather over cell-sorted neighbours in a fixed order, so results are
// bitwise reproducible.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace depo {

namespace {

constexpr int kFftLds = 2048;   // complex values per FFT workgroup (32 KB of LDS)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Continuous mesh coordinates of particle i (x periodic in [0, nx); y, z in [1, nc - 2]).
template <class Real>
__device__ __forceinline__ void mesh_coords(const State<Real> &st, const Phys &ph, const P3mDev &m, int i, double &gx,
                                            double &gy, double &gz) {
  using SPos = typename std::make_signed<typename Prec<Real>::Pos>::type;
  const double x = (double)st.px[i] * ph.ux;
  const double y = (double)(SPos)st.py[i] * ph.ur;
  const double z = (double)(SPos)st.pz[i] * ph.ur;
  gx = x / m.hx;
  if (gx >= m.nx) gx -= m.nx;
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

// Erf field of a unit charge at displacement (dx, dy, dz), summed over the x images n = -M..M.
__global__ void k_p3m_green(P3mDev m, double L, int images, double2 *__restrict__ gx_, double2 *__restrict__ gy_,
                            double2 *__restrict__ gz_) {
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
  gx_[e] = make_double2(ex, 0.0);
  gy_[e] = make_double2(ey, 0.0);
  gz_[e] = make_double2(ez, 0.0);
}

// Divide the transformed Green's functions by the squared TSC transfer sinc^3 per axis.
__device__ __forceinline__ double sinc_pi(double u) { return u == 0.0 ? 1.0 : sin(M_PI * u) / (M_PI * u); }

__global__ void k_p3m_deconv(P3mDev m, double2 *__restrict__ gx_, double2 *__restrict__ gy_,
                             double2 *__restrict__ gz_) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)m.nx * m.P * m.P;
  if (e >= total) return;
  const int iz = (int)(e % m.P), iy = (int)((e / m.P) % m.P), ix = (int)(e / ((int64_t)m.P * m.P));
  auto freq = [](int i, int n) { return (double)(i < (n + 1) / 2 ? i : i - n) / n; };   // cycles per node
  const double sx = sinc_pi(freq(ix, m.nx)), sy = sinc_pi(freq(iy, m.P)), sz = sinc_pi(freq(iz, m.P));
  const double W = sx * sx * sx * sy * sy * sy * sz * sz * sz;
  const double inv = 1.0 / (W * W);
  gx_[e] = make_double2(gx_[e].x * inv, gx_[e].y * inv);
  gy_[e] = make_double2(gy_[e].x * inv, gy_[e].y * inv);
  gz_[e] = make_double2(gz_[e].x * inv, gz_[e].y * inv);
}

// Complex FFT of length n = 2^log2n along lines of the mesh: line l starts at
// (l / inner) * outer_stride + (l % inner) * inner_stride, points are point_stride apart.
// A workgroup transforms kFftLds / n lines through LDS (bit-reversed load, in-place
// radix-2 butterflies, twiddles exp(sign 2 pi i k / n) from sincospi).
__global__ __launch_bounds__(256) void k_fft_lines(double2 *__restrict__ data, int n, int log2n, int64_t inner,
                                                   int64_t inner_stride, int64_t outer_stride, int64_t point_stride,
                                                   int sign, int points_contiguous) {
  __shared__ double2 buf[kFftLds];
  __shared__ double2 tw[kFftLds / 2];
  const int lpw = kFftLds / n;   // lines per workgroup
  const int64_t l0 = (int64_t)blockIdx.x * lpw;
  for (int k = threadIdx.x; k < n / 2; k += blockDim.x) {
    double s, c;
    sincospi(2.0 * k / n, &s, &c);
    tw[k] = make_double2(c, sign * s);
  }
  auto addr = [&](int line, int p) {
    const int64_t l = l0 + line;
    return (l / inner) * outer_stride + (l % inner) * inner_stride + (int64_t)p * point_stride;
  };
  for (int e = threadIdx.x; e < kFftLds; e += blockDim.x) {
    const int line = points_contiguous ? e / n : e % lpw;
    const int p = points_contiguous ? e % n : e / lpw;
    const int rev = (int)(__brev((unsigned)p) >> (32 - log2n));
    buf[line * n + rev] = data[addr(line, p)];
  }
  __syncthreads();
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len >> 1, step = n / len;
    for (int b = threadIdx.x; b < kFftLds / 2; b += blockDim.x) {
      const int line = b / (n / 2), k = b % (n / 2);
      const int pos = k % half;
      const int i = line * n + (k / half) * len + pos;
      const double2 u = buf[i];
      const double2 v = cmul(tw[pos * step], buf[i + half]);
      buf[i] = make_double2(u.x + v.x, u.y + v.y);
      buf[i + half] = make_double2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kFftLds; e += blockDim.x) {
    const int line = points_contiguous ? e / n : e % lpw;
    const int p = points_contiguous ? e % n : e / lpw;
    data[addr(line, p)] = buf[line * n + p];
  }
}

// TSC charge assignment in 64-bit fixed point (units of the per-sample bound 2^-62 sum |q~|).
template <class Real>
__global__ void k_p3m_assign(State<Real> st, Phys ph, P3mDev m, unsigned long long *__restrict__ qmesh) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  const double q = (double)st.js[i].q;
  if (q == 0.0) return;
  const double qs = *m.q_scale;
  double gx, gy, gz, wx[3], wy[3], wz[3];
  int ix, iy, iz;
  mesh_coords<Real>(st, ph, m, i, gx, gy, gz);
  tsc(gx, ix, wx);
  tsc(gy, iy, wy);
  tsc(gz, iz, wz);
  iy = min(max(iy, 1), m.nc - 2);   // suspended particles stay inside [-R, R]; the clamp only guards
  iz = min(max(iz, 1), m.nc - 2);
  for (int a = 0; a < 3; ++a) {
    int jx = ix + a - 1;
    jx = jx < 0 ? jx + m.nx : (jx >= m.nx ? jx - m.nx : jx);
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        const int64_t o = ((int64_t)jx * m.nc + (iy + b - 1)) * m.nc + (iz + c - 1);
        atomicAdd(qmesh + o, (unsigned long long)__double2ll_rn(q * wx[a] * wy[b] * wz[c] * qs));
      }
  }
}

// Fixed-point charges into the zero-padded complex mesh (every node written); the charge mesh is cleared.
__global__ void k_p3m_load(P3mDev m, unsigned long long *__restrict__ qmesh, double2 *__restrict__ rho) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)m.nx * m.P * m.P;
  if (e >= total) return;
  const int iz = (int)(e % m.P), iy = (int)((e / m.P) % m.P), ix = (int)(e / ((int64_t)m.P * m.P));
  double v = 0.0;
  if (iy < m.nc && iz < m.nc) {
    const int64_t o = ((int64_t)ix * m.nc + iy) * m.nc + iz;
    v = (double)(long long)qmesh[o] / *m.q_scale;
    qmesh[o] = 0ull;
  }
  rho[e] = make_double2(v, 0.0);
}

__global__ void k_p3m_mul(P3mDev m, const double2 *__restrict__ a, const double2 *__restrict__ g,
                          double2 *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m.nx * m.P * m.P) return;
  out[e] = cmul(a[e], g[e]);
}

// TSC interpolation of one field component (real part of the unnormalised inverse transform).
template <class Real>
__global__ void k_p3m_interp(State<Real> st, Phys ph, P3mDev m, const double2 *__restrict__ E,
                             double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  double gx, gy, gz, wx[3], wy[3], wz[3];
  int ix, iy, iz;
  mesh_coords<Real>(st, ph, m, i, gx, gy, gz);
  tsc(gx, ix, wx);
  tsc(gy, iy, wy);
  tsc(gz, iz, wz);
  iy = min(max(iy, 1), m.nc - 2);
  iz = min(max(iz, 1), m.nc - 2);
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    int jx = ix + a - 1;
    jx = jx < 0 ? jx + m.nx : (jx >= m.nx ? jx - m.nx : jx);
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c)
        s += wx[a] * wy[b] * wz[c] * E[((int64_t)jx * m.P + (iy + b - 1)) * m.P + (iz + c - 1)].x;
  }
  out[i] = s / ((double)m.nx * m.P * m.P);
}

// Short-range cell of a particle (cells of at least r_max; x periodic).
template <class Real>
__device__ __forceinline__ int3 sr_cell(const State<Real> &st, const Phys &ph, const P3mDev &m, int i) {
  using SPos = typename std::make_signed<typename Prec<Real>::Pos>::type;
  const double x = (double)st.px[i] * ph.ux;
  const double y = (double)(SPos)st.py[i] * ph.ur;
  const double z = (double)(SPos)st.pz[i] * ph.ur;
  int cx = (int)(x / ph.L * m.ncx), cy = (int)((y + ph.R) / (2.0 * ph.R) * m.ncy),
      cz = (int)((z + ph.R) / (2.0 * ph.R) * m.ncy);
  cx = min(max(cx, 0), m.ncx - 1);
  cy = min(max(cy, 0), m.ncy - 1);
  cz = min(max(cz, 0), m.ncy - 1);
  return make_int3(cx, cy, cz);
}

template <class Real>
__global__ void k_p3m_bin(State<Real> st, Phys ph, P3mDev m, int32_t *__restrict__ cell_of,
                          int32_t *__restrict__ counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  const int3 c = sr_cell<Real>(st, ph, m, i);
  const int id = (c.x * m.ncy + c.y) * m.ncy + c.z;
  cell_of[i] = id;
  atomicAdd(counts + id, 1);
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
  if (i >= N) return;
  sorted[atomicAdd(fill + cell_of[i], 1)] = i;
}

// Particles of each cell in index order (a fixed summation order); the counts are cleared.
__global__ void k_p3m_sort(int32_t ncell, const int32_t *__restrict__ starts, int32_t *__restrict__ sorted,
                           int32_t *__restrict__ counts) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int b = starts[c], e = starts[c + 1];
  for (int k = b + 1; k < e; ++k) {
    const int v = sorted[k];
    int j = k - 1;
    while (j >= b && sorted[j] > v) {
      sorted[j + 1] = sorted[j];
      --j;
    }
    sorted[j + 1] = v;
  }
  counts[c] = 0;
}

// Short range (Coulomb with the overlap clamp minus the erf field) over nearest-image neighbours
// closer than r_max, added to the long-range part; result in units of the x quantum.
template <class Real>
__global__ void k_p3m_short(State<Real> st, Phys ph, P3mDev m, const int32_t *__restrict__ starts,
                            const int32_t *__restrict__ sorted, const double *__restrict__ slong) {
  using Pos = typename Prec<Real>::Pos;
  using SPos = typename std::make_signed<Pos>::type;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  const int3 c = sr_cell<Real>(st, ph, m, i);
  const Pos xi = st.px[i], yi = st.py[i], zi = st.pz[i];
  const double di = st.d[i];
  const double a = m.alpha, c2 = 2.0 * m.alpha / sqrt(M_PI), rmax2 = m.rmax * m.rmax;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int ox = -1; ox <= 1; ++ox) {   // ncx >= 3: the three x neighbours are distinct cells
    int cx = c.x + ox;
    cx = cx < 0 ? cx + m.ncx : (cx >= m.ncx ? cx - m.ncx : cx);
    for (int cy = max(c.y - 1, 0); cy <= min(c.y + 1, m.ncy - 1); ++cy)
      for (int cz = max(c.z - 1, 0); cz <= min(c.z + 1, m.ncy - 1); ++cz) {
        const int id = (cx * m.ncy + cy) * m.ncy + cz;
        for (int k = starts[id]; k < starts[id + 1]; ++k) {
          const int j = sorted[k];
          if (j == i) continue;
          const double q = (double)st.js[j].q;
          if (q == 0.0) continue;
          const double dx = (double)(SPos)(xi - st.px[j]) * ph.ux;
          const double dy = (double)((SPos)yi - (SPos)st.py[j]) * ph.ur;
          const double dz = (double)((SPos)zi - (SPos)st.pz[j]) * ph.ur;
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 >= rmax2 || r2 <= 0.0) continue;
          const double r = sqrt(r2);
          const double dij = 0.5 * (di + st.d[j]);
          const double rc = fmax(r, dij);
          const double full = 1.0 / (rc * rc);
          const double lng = erf(a * r) / r2 - c2 * exp(-a * a * r2) / r;
          const double f = q * (full - lng) / r;
          sx += f * dx;
          sy += f * dy;
          sz += f * dz;
        }
      }
  }
  // metres^-2 -> units of the x quantum (the direct kernels' convention)
  const double u2 = ph.ux * ph.ux;
  st.cx[i] = Real((slong[i] + sx) * u2);
  st.cy[i] = Real((slong[ph.N + i] + sy) * u2);
  st.cz[i] = Real((slong[2 * (int64_t)ph.N + i] + sz) * u2);
}

int ilog2(int n) {
  int k = 0;
  while ((1 << k) < n) ++k;
  return k;
}

// 3D transform of the padded mesh: lines along z, y, x.
void fft3d(const P3mDev &m, double2 *d, int sign, hipStream_t s) {
  const int64_t P = m.P, nx = m.nx;
  const int64_t total = nx * P * P;
  // z: points contiguous, line l at l * P
  hipLaunchKernelGGL(k_fft_lines, dim3((unsigned)(total / kFftLds)), dim3(256), 0, s, d, (int)P, ilog2((int)P),
                     (int64_t)1, (int64_t)0, P, (int64_t)1, sign, 1);
  // y: line (ix, iz) at ix P^2 + iz, points P apart
  hipLaunchKernelGGL(k_fft_lines, dim3((unsigned)(total / kFftLds)), dim3(256), 0, s, d, (int)P, ilog2((int)P), P,
                     (int64_t)1, P * P, P, sign, 0);
  // x: line (iy, iz) at iy P + iz, points P^2 apart
  hipLaunchKernelGGL(k_fft_lines, dim3((unsigned)(total / kFftLds)), dim3(256), 0, s, d, (int)nx, ilog2((int)nx),
                     (int64_t)1, (int64_t)0, (int64_t)1, P * P, sign, 0);
}

}  // namespace

void p3m_setup_green(const P3mDev &m, double L, int images, hipStream_t s) {
  const int64_t total = (int64_t)m.nx * m.P * m.P;
  const unsigned g = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL(k_p3m_green, dim3(g), dim3(256), 0, s, m, L, images, m.ghat[0], m.ghat[1], m.ghat[2]);
  for (int c = 0; c < 3; ++c) fft3d(m, m.ghat[c], -1, s);
  hipLaunchKernelGGL(k_p3m_deconv, dim3(g), dim3(256), 0, s, m, m.ghat[0], m.ghat[1], m.ghat[2]);
}

template <class Real> void launch_p3m(const State<Real> &st, const Phys &ph, const P3mDev &m, hipStream_t s) {
  if (ph.N <= 0) return;
  const int64_t total = (int64_t)m.nx * m.P * m.P;
  const unsigned gm = (unsigned)((total + 255) / 256), gp = (unsigned)((ph.N + 255) / 256);
  hipLaunchKernelGGL((k_p3m_assign<Real>), dim3(gp), dim3(256), 0, s, st, ph, m, m.qmesh);
  hipLaunchKernelGGL(k_p3m_load, dim3(gm), dim3(256), 0, s, m, m.qmesh, m.rho);
  fft3d(m, m.rho, -1, s);
  for (int c = 0; c < 3; ++c) {
    hipLaunchKernelGGL(k_p3m_mul, dim3(gm), dim3(256), 0, s, m, m.rho, m.ghat[c], m.work);
    fft3d(m, m.work, +1, s);
    hipLaunchKernelGGL((k_p3m_interp<Real>), dim3(gp), dim3(256), 0, s, st, ph, m, m.work,
                       m.slong + (int64_t)c * ph.N);
  }
  const int ncell = m.ncx * m.ncy * m.ncy;
  hipLaunchKernelGGL((k_p3m_bin<Real>), dim3(gp), dim3(256), 0, s, st, ph, m, m.cell_of, m.counts);
  hipLaunchKernelGGL(k_p3m_scan, dim3(1), dim3(1024), 0, s, ncell, m.counts, m.starts, m.fill);
  hipLaunchKernelGGL(k_p3m_scatter, dim3(gp), dim3(256), 0, s, ph.N, m.cell_of, m.fill, m.sorted);
  hipLaunchKernelGGL(k_p3m_sort, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, ncell, m.starts, m.sorted,
                     m.counts);
  hipLaunchKernelGGL((k_p3m_short<Real>), dim3(gp), dim3(256), 0, s, st, ph, m, m.starts, m.sorted, m.slong);
}

template void launch_p3m<float>(const State<float> &, const Phys &, const P3mDev &, hipStream_t);
template void launch_p3m<double>(const State<double> &, const Phys &, const P3mDev &, hipStream_t);

}  // namespace depo
