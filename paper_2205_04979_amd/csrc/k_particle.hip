// Per-particle kernels of the step: half kicks with exponential Schiller-Naumann
// drag, fixed-point drift, FP64 wall test with removal or rebound, assembly of
// the non-drag acceleration (Coulomb sums, short-range forces, wall terms),
// trilinear gather of the carrier velocity and the smoothed deposition tally.
//
// One thread per particle; every array access is a coalesced SoA row.
#include "common.hpp"
#include "launch.hpp"

namespace depo {

// Half kick of dv/dt = f (u - v) / tau_p + a over h with f, u and a frozen at the
// start (drag law Eq. part_source, Re_p = |u - v| d / nu): the exact solution
// v + (u + a tau - v)(1 - exp(-h / tau)), tau = tau_p / f.
template <class Real>
__device__ __forceinline__ void half_kick(Real v[3], const Real u[3], const Real a[3], Real d, Real taup,
                                          Real h, Real inv_nu, bool drag) {
  if (!drag) {
    v[0] += a[0] * h; v[1] += a[1] * h; v[2] += a[2] * h;
    return;
  }
  Real wx = u[0] - v[0], wy = u[1] - v[1], wz = u[2] - v[2];
  Real re = sqrt(wx * wx + wy * wy + wz * wz) * d * inv_nu;
  Real f = Real(1) + Real(0.15) * pow(re, Real(0.687));
  Real tau = taup / f;
  Real g = -expm1(-h / tau);
  v[0] += (wx + a[0] * tau) * g;
  v[1] += (wy + a[1] * tau) * g;
  v[2] += (wz + a[2] * tau) * g;
}

template <class Real>
__device__ __forceinline__ void gather(const typename Prec<Real>::Vec4 *__restrict__ F, int nx, int ny, int nz,
                                       typename Prec<Real>::Pos px, typename Prec<Real>::Pos py,
                                       typename Prec<Real>::Pos pz, Real u[3]) {
  double fx, fy, fz;
  int ix = frac_cell(px, nx, fx);
  int ix1 = ix + 1 == nx ? 0 : ix + 1;
  int iy = node_cell(as_signed(py), ny, fy);
  int iz = node_cell(as_signed(pz), nz, fz);
  const Real wx[2] = {Real(1.0 - fx), Real(fx)};
  const Real wy[2] = {Real(1.0 - fy), Real(fy)};
  const Real wz[2] = {Real(1.0 - fz), Real(fz)};
  const int xs[2] = {ix, ix1};
  Real s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const size_t base = ((size_t)xs[a] * ny + (iy + b)) * nz + iz;
      const auto c0 = F[base];
      const auto c1 = F[base + 1];
      const Real w = wx[a] * wy[b];
      s0 += w * (wz[0] * c0.x + wz[1] * c1.x);
      s1 += w * (wz[0] * c0.y + wz[1] * c1.y);
      s2 += w * (wz[0] * c0.z + wz[1] * c1.z);
    }
  u[0] = s0; u[1] = s1; u[2] = s2;
}

// First half of a step (mode P_KICK_DRIFT): half kick, drift, wall test.  Always
// (re)writes the Coulomb source record and, with P_CELLS, the cell id and the
// cell histogram of the short-range search.
template <class Real>
__global__ __launch_bounds__(256) void k_prepare(State<Real> st, Phys ph, int mode) {
  using Pos = typename Prec<Real>::Pos;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  const int step = *st.nstep + 1;
  bool alive = st.dep[i] == 0;
  Pos px = st.px[i], py = st.py[i], pz = st.pz[i];
  Real rx = st.rx[i], ry = st.ry[i], rz = st.rz[i];
  const double d = st.d[i];
  const int s = st.sid[i];
  if (mode & P_SEED) st.jr[i] = Real(0.5 * d * ph.inv_ux);
  if (alive && (mode & P_KICK_DRIFT)) {
    Real v[3] = {st.vx[i], st.vy[i], st.vz[i]};
    const Real u[3] = {st.ux[i], st.uy[i], st.uz[i]};
    const Real a[3] = {st.ax[i], st.ay[i], st.az[i]};
    const Real dr = Real(d);
    half_kick(v, u, a, dr, Real(ph.tau_coef * d * d), Real(0.5 * ph.dt), Real(1.0 / ph.nu),
              (ph.flags & F_DRAG) != 0);
    const Real qx = Real(ph.dt * ph.inv_ux), qr = Real(ph.dt * ph.inv_ur);
    // keep one step's displacement inside the signed range of the fixed-point type
    const Real lim = sizeof(Real) == 4 ? Real(1 << 30) : Real(0x1p62);
    // compensated drift: the displacement in quanta plus the carried remainder is split into the
    // integer step added to the fixed-point position and the new remainder (exact: q - rint(q)),
    // so rounding to the quantum does not accumulate from step to step
    const Real mx = fmin(fmax(fma(v[0], qx, rx), -lim), lim);
    const Real my = fmin(fmax(fma(v[1], qr, ry), -lim), lim);
    const Real mz = fmin(fmax(fma(v[2], qr, rz), -lim), lim);
    const auto kx = round_step(mx), ky = round_step(my), kz = round_step(mz);
    rx = mx - Real(kx); ry = my - Real(ky); rz = mz - Real(kz);
    px += (Pos)kx;
    py = (Pos)(as_signed(py) + ky);
    pz = (Pos)(as_signed(pz) + kz);
    if (!(ph.flags & F_SOFT)) {
      const double y = pos_m(py, ry, ph.ur), z = pos_m(pz, rz, ph.ur);
      const double rho = sqrt(y * y + z * z);
      if (rho + 0.5 * d >= ph.R) {
        bool stick = true;
        if ((ph.flags & F_REBOUND) && rho > 0.0) {
          // rebound law (Eq. CoR): V_n2^2 = min(V_n1^2, sigma_y^2/(rho_p E)) - 2 A_cont gamma_c / m
          const SampleDev sp = st.samples[s];
          const double ery = y / rho, erz = z / rho;
          const double vn1 = (double)v[1] * ery + (double)v[2] * erz;
          // yield stress floored at zero: theta = 0.225 (T - 1000) / 200 is defined on [0, 1]
          const double sig = fmax(200.0 - 0.225 * (sp.temperature - 1000.0), 0.0) * 1e6;
          const double gam = sp.hamaker / (24.0 * M_PI * ph.delta_c * ph.delta_c);
          const double acont = ph.acont_coef * M_PI * d * d * 0.25;
          const double m = ph.mass_coef * d * d * d;
          const double vn2sq = fmin(vn1 * vn1, sig * sig / (ph.rho_p * ph.E_young)) - 2.0 * acont * gam / m;
          if (vn2sq > 0.0) {
            stick = false;
            const double dv = vn1 + sqrt(vn2sq);
            v[1] = Real((double)v[1] - dv * ery);
            v[2] = Real((double)v[2] - dv * erz);
            const double pen = rho + 0.5 * d - ph.R;
            const double sc = (rho - 2.0 * pen) / rho;
            const double ny = y * sc * ph.inv_ur, nz = z * sc * ph.inv_ur;
            const auto jy = round_step(ny), jz = round_step(nz);
            py = (Pos)jy;
            pz = (Pos)jz;
            ry = Real(ny - (double)jy);
            rz = Real(nz - (double)jz);
          }
        }
        if (stick) {
          st.dep[i] = step;
          st.nbr[i] = 0;
          alive = false;
        }
      }
    }
    st.vx[i] = v[0]; st.vy[i] = v[1]; st.vz[i] = v[2];
    st.px[i] = px; st.py[i] = py; st.pz[i] = pz;
    st.rx[i] = rx; st.ry[i] = ry; st.rz[i] = rz;
  }
  if (mode & P_COULOMB) {
    JSrc<Real> js;
    js.x = px;
    const double yx = ((double)as_signed(py) + (double)ry) * ph.yz_over_x;
    const double zx = ((double)as_signed(pz) + (double)rz) * ph.yz_over_x;
    if constexpr (sizeof(Real) == 4) {
      if (ph.flags & F_INT_RECORDS) {
        // |y| < R: within +-2^31 x quanta for L >= 2R
        js.y = __int_as_float((int32_t)fmin(fmax(rint(yx), -2147483647.0), 2147483647.0));
        js.z = __int_as_float((int32_t)fmin(fmax(rint(zx), -2147483647.0), 2147483647.0));
      } else {
        js.y = Real(yx);
        js.z = Real(zx);
      }
    } else {
      js.y = Real(yx);
      js.z = Real(zx);
    }
    js.q = alive ? Real(st.samples[s].charge_scale * st.qb[i] / ph.q_ref) : Real(0);
    st.js[i] = js;
  }
  if (mode & P_CELLS) {
    int c = -1;
    if (alive) {
      const SampleDev sp = st.samples[s];
      const int cx = x_cell(px, sp.ncx);
      const int cy = box_cell(as_signed(py), sp.ncy);
      const int cz = box_cell(as_signed(pz), sp.ncz);
      c = sp.cell_base + (cx * sp.ncy + cy) * sp.ncz + cz;
      atomicAdd(&st.cell_count[c], 1);
    }
    st.cell_of[i] = c;
  }
}

// Second half of a step (F_KICK): assemble a^{n+1} = Coulomb + short-range + wall
// (+ body) at the new positions, gather u_f(x^{n+1}), half kick, smoothed tally.
// Without F_KICK it only evaluates the acceleration and the fluid velocity
// (seed / diagnostic force evaluation); with F_V_FROM_FLUID the velocity is set
// to the local fluid velocity.  F_FLUID_ONLY sets u and v = u_f(x) and nothing
// else: the seed runs it before the first force evaluation, whose collision
// damping reads the velocities of neighbours.
template <class Real>
__global__ __launch_bounds__(256) void k_finish(State<Real> st, Phys ph, int mode) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  // the step counter advances once per step; no thread of this kernel reads it
  if ((mode & F_KICK) && i == 0) *st.nstep += 1;
  if (i >= ph.N) return;
  Real cs[3];   // Coulomb pair sums of this particle
  if constexpr (sizeof(Real) == 4) {
    if (mode & F_PAIR_SUMS) {
      // fixed point -> FP32 and the accumulators cleared, for removed particles too (the pair kernel
      // adds to every target of its items)
      const double inv = 1.0 / st.fx_scale[st.sid[i]];
      cs[0] = (Real)((double)(long long)st.accx[i] * inv);
      cs[1] = (Real)((double)(long long)st.accy[i] * inv);
      cs[2] = (Real)((double)(long long)st.accz[i] * inv);
      st.accx[i] = 0ull;
      st.accy[i] = 0ull;
      st.accz[i] = 0ull;
      st.cx[i] = cs[0]; st.cy[i] = cs[1]; st.cz[i] = cs[2];
    }
  }
  if (st.dep[i] != 0) return;
  if (mode & F_FLUID_ONLY) {
    Real u[3];
    gather<Real>(st.field, ph.nx, ph.ny, ph.nz, st.px[i], st.py[i], st.pz[i], u);
    st.ux[i] = u[0]; st.uy[i] = u[1]; st.uz[i] = u[2];
    st.vx[i] = u[0]; st.vy[i] = u[1]; st.vz[i] = u[2];
    return;
  }
  const int s = st.sid[i];
  const SampleDev sp = st.samples[s];
  const double d = st.d[i];
  const double m = ph.mass_coef * d * d * d;
  const double q = sp.charge_scale * st.qb[i];
  Real a[3] = {0, 0, 0};
  if (ph.flags & F_COULOMB) {
    if (!(sizeof(Real) == 4 && (mode & F_PAIR_SUMS))) {
      cs[0] = st.cx[i]; cs[1] = st.cy[i]; cs[2] = st.cz[i];
    }
    const Real c = Real(ph.k_e * q * ph.q_ref / (m * ph.ux * ph.ux));
    a[0] += c * cs[0]; a[1] += c * cs[1]; a[2] += c * cs[2];
  }
  if (ph.flags & (F_COLLIDE | F_VDW)) {
    a[0] += st.sx[i]; a[1] += st.sy[i]; a[2] += st.sz[i];
  }
  const auto py = st.py[i], pz = st.pz[i];
  const double y = pos_m(py, st.ry[i], ph.ur), z = pos_m(pz, st.rz[i], ph.ur);
  if (ph.flags & (F_WALL_IMAGE | F_WALL_VDW)) {
    const double rho = sqrt(y * y + z * z);
    if (rho > 0.0) {
      const double h = fmax(ph.R - rho, 0.5 * d);    // centre-to-wall distance, never below contact
      const double g = ph.R - rho - 0.5 * d;          // surface gap
      double mag = 0.0;
      if (ph.flags & F_WALL_IMAGE) mag += ph.k_e * q * q / (4.0 * h * h) / m;
      if ((ph.flags & F_WALL_VDW) && g <= 0.25 * d) {
        const double gs = fmax(g, ph.delta_sat);
        mag += sp.hamaker * d / (12.0 * gs * gs) / m;
      }
      a[1] += Real(mag * y / rho);
      a[2] += Real(mag * z / rho);
    }
  }
  if (ph.flags & F_BODY) {
    a[0] += Real(ph.g_body[0]); a[1] += Real(ph.g_body[1]); a[2] += Real(ph.g_body[2]);
  }
  st.ax[i] = a[0]; st.ay[i] = a[1]; st.az[i] = a[2];
  Real u[3];
  gather<Real>(st.field, ph.nx, ph.ny, ph.nz, st.px[i], py, pz, u);
  st.ux[i] = u[0]; st.uy[i] = u[1]; st.uz[i] = u[2];
  Real v[3];
  if (mode & F_V_FROM_FLUID) {
    v[0] = u[0]; v[1] = u[1]; v[2] = u[2];
  } else {
    v[0] = st.vx[i]; v[1] = st.vy[i]; v[2] = st.vz[i];
  }
  if (mode & F_KICK) {
    half_kick(v, u, a, Real(d), Real(ph.tau_coef * d * d), Real(0.5 * ph.dt), Real(1.0 / ph.nu),
              (ph.flags & F_DRAG) != 0);
    if (ph.flags & F_SOFT) {
      const double g = ph.R - sqrt(y * y + z * z) - 0.5 * d;
      const double zz = -g / (ph.soft_eps * d);
      st.ell[i] += ph.soft_rate * ph.dt / (1.0 + exp(-zz));
    }
  }
  if (mode & (F_KICK | F_V_FROM_FLUID)) {
    st.vx[i] = v[0]; st.vy[i] = v[1]; st.vz[i] = v[2];
  }
  bool finite = isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]) && isfinite(a[0]) && isfinite(a[1]) &&
                isfinite(a[2]);
  if (!finite) atomicOr(st.err, ERR_NONFINITE);
}

// Per-sample tally (Eq. 2): deposited mass/count, the alive-mass time integral
// dt * sum_i m_i * (steps suspended), the Poisson error term and the smoothed
// deposited mass.  One block per sample; fixed-order strided loop and tree
// reduction, so the result is bitwise reproducible.
template <class Real>
__global__ __launch_bounds__(256) void k_tally(State<Real> st, Phys ph, int nstep) {
  __shared__ double red[7][256];
  const SampleDev sp = st.samples[blockIdx.x];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};   // m_dep, n_dep, m*steps, m^2 dep, j_soft, n_alive, -
  for (int i = sp.start + threadIdx.x; i < sp.start + sp.count; i += blockDim.x) {
    const double d = st.d[i];
    const double m = ph.mass_coef * d * d * d;
    const int dep = st.dep[i];
    if (dep > 0) {
      acc[0] += m; acc[1] += 1.0; acc[2] += m * (double)(dep - 1); acc[3] += m * m;
    } else {
      acc[2] += m * (double)nstep; acc[5] += 1.0;
    }
    acc[4] += m * -expm1(-st.ell[i]);
  }
  for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 7; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 7) st.tally[blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

template <class Real>
void launch_prepare(const State<Real> &st, const Phys &ph, int mode, hipStream_t s) {
  if (ph.N == 0) return;
  hipLaunchKernelGGL(k_prepare<Real>, dim3((ph.N + 255) / 256), dim3(256), 0, s, st, ph, mode);
}
template <class Real>
void launch_finish(const State<Real> &st, const Phys &ph, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_finish<Real>, dim3((ph.N + 255) / 256 > 0 ? (ph.N + 255) / 256 : 1), dim3(256), 0, s, st,
                     ph, mode);
}
template <class Real>
void launch_tally(const State<Real> &st, const Phys &ph, int nstep, hipStream_t s) {
  hipLaunchKernelGGL(k_tally<Real>, dim3(ph.S), dim3(256), 0, s, st, ph, nstep);
}

template void launch_prepare<float>(const State<float> &, const Phys &, int, hipStream_t);
template void launch_prepare<double>(const State<double> &, const Phys &, int, hipStream_t);
template void launch_finish<float>(const State<float> &, const Phys &, int, hipStream_t);
template void launch_finish<double>(const State<double> &, const Phys &, int, hipStream_t);
template void launch_tally<float>(const State<float> &, const Phys &, int, hipStream_t);
template void launch_tally<double>(const State<double> &, const Phys &, int, hipStream_t);

}  // namespace depo
