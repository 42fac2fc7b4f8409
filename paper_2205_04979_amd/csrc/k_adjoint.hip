// Reverse-mode (adjoint) kernels of the particle step under the smoothed
// deposition tally (no removal): gradients of J = sum_s w_s sum_i m_i (1 - exp(-l_i))
// with respect to each sample's charge scale and Hamaker constant.
//
// The forward step is kick / drift / forces / gather / kick / tally.  Its
// reverse, for one step n with the states S_n (start) and S_{n+1} (end) taken
// from the tape, is:
//   k_adj_post   smoothed-tally, second half-kick, gather and wall-term adjoints
//                at x^{n+1}; charge-scale and Hamaker partials of the Coulomb and
//                wall accelerations; writes the source records of the pair adjoint
//   k_coulomb_vjp    x_bar_i += (1/ux) sum_j J(r_ij) (q_j b_i - q_i b_j), with
//                J(r) the Jacobian of the pair law and b = c a_bar (O(N^2))
//   k_short_range_vjp  contact and cohesion adjoints over the cell-list pairs
//   k_adj_pre    drift and first half-kick adjoints -> adjoint state of S_n
// All adjoint quantities carry a common scale factor chosen on the host so that
// FP32 intermediates stay in range; the host divides it out.
#include "common.hpp"
#include "launch.hpp"
#include "adjoint.hpp"

#include <type_traits>

namespace depo {

// ---------------------------------------------------------------- tape copies

template <class Real>
__global__ __launch_bounds__(256) void k_tape_store(State<Real> st, TapeEntry<Real> t, int n, int with_ell) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  t.px[i] = st.px[i]; t.py[i] = st.py[i]; t.pz[i] = st.pz[i];
  t.rx[i] = st.rx[i]; t.ry[i] = st.ry[i]; t.rz[i] = st.rz[i];
  t.vx[i] = st.vx[i]; t.vy[i] = st.vy[i]; t.vz[i] = st.vz[i];
  t.ax[i] = st.ax[i]; t.ay[i] = st.ay[i]; t.az[i] = st.az[i];
  t.ux[i] = st.ux[i]; t.uy[i] = st.uy[i]; t.uz[i] = st.uz[i];
  t.cx[i] = st.cx[i]; t.cy[i] = st.cy[i]; t.cz[i] = st.cz[i];
  if (with_ell) t.ell[i] = st.ell[i];
}

template <class Real>
__global__ __launch_bounds__(256) void k_tape_load(State<Real> st, TapeEntry<Real> t, int n, int with_ell) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  st.px[i] = t.px[i]; st.py[i] = t.py[i]; st.pz[i] = t.pz[i];
  st.rx[i] = t.rx[i]; st.ry[i] = t.ry[i]; st.rz[i] = t.rz[i];
  st.vx[i] = t.vx[i]; st.vy[i] = t.vy[i]; st.vz[i] = t.vz[i];
  st.ax[i] = t.ax[i]; st.ay[i] = t.ay[i]; st.az[i] = t.az[i];
  st.ux[i] = t.ux[i]; st.uy[i] = t.uy[i]; st.uz[i] = t.uz[i];
  st.cx[i] = t.cx[i]; st.cy[i] = t.cy[i]; st.cz[i] = t.cz[i];
  if (with_ell) st.ell[i] = t.ell[i];
}

// ---------------------------------------------------------------- helpers

// Forward half kick (same arithmetic as the step) returning the intermediate
// quantities its adjoint needs.
template <class Real> struct KickCache {
  Real v[3], w[3], c[3], a[3];
  Real tau, g, E, dtau_dW, W;
};

template <class Real>
__device__ __forceinline__ void kick_fwd(const Real v0[3], const Real u[3], const Real a[3], Real d, Real taup, Real h,
                                         Real inv_nu, bool drag, KickCache<Real> &kc) {
  for (int k = 0; k < 3; ++k) { kc.a[k] = a[k]; kc.v[k] = v0[k]; }
  if (!drag) {
    for (int k = 0; k < 3; ++k) kc.v[k] = v0[k] + a[k] * h;
    kc.tau = 0; kc.g = 0; kc.E = 0; kc.dtau_dW = 0; kc.W = 0;
    return;
  }
  Real wx = u[0] - v0[0], wy = u[1] - v0[1], wz = u[2] - v0[2];
  const Real W = sqrt(wx * wx + wy * wy + wz * wz);
  const Real re = W * d * inv_nu;
  const Real pw = pow(re, Real(0.687));
  const Real f = Real(1) + Real(0.15) * pw;
  const Real tau = taup / f;
  const Real g = -expm1(-h / tau);
  kc.w[0] = wx; kc.w[1] = wy; kc.w[2] = wz;
  kc.c[0] = wx + a[0] * tau; kc.c[1] = wy + a[1] * tau; kc.c[2] = wz + a[2] * tau;
  kc.v[0] = v0[0] + kc.c[0] * g; kc.v[1] = v0[1] + kc.c[1] * g; kc.v[2] = v0[2] + kc.c[2] * g;
  kc.tau = tau; kc.g = g; kc.E = Real(1) - g; kc.W = W;
  // d tau / d W = -tau / f * df/dW, df/dW = 0.15 * 0.687 * re^(0.687 - 1) * d / nu
  kc.dtau_dW = re > Real(0) ? -tau / f * Real(0.15 * 0.687) * (pw / re) * d * inv_nu : Real(0);
}

// Adjoint of one half kick: given lam = v_out_bar, accumulate into v_in_bar,
// u_bar and a_bar.
template <class Real>
__device__ __forceinline__ void kick_adj(const KickCache<Real> &kc, const Real lam[3], Real h, bool drag,
                                         Real vin_bar[3], Real u_bar[3], Real a_bar[3]) {
  if (!drag) {
    for (int k = 0; k < 3; ++k) { vin_bar[k] += lam[k]; a_bar[k] += h * lam[k]; }
    return;
  }
  // v_out = v + c g,  c = w + a tau,  g = 1 - exp(-h/tau),  w = u - v,  tau = tau(|w|)
  const Real dg_dtau = -kc.E * h / (kc.tau * kc.tau);
  Real s_tau = 0;
  for (int k = 0; k < 3; ++k) s_tau += lam[k] * (kc.a[k] * kc.g + kc.c[k] * dg_dtau);
  const Real coef = kc.W > Real(0) ? s_tau * kc.dtau_dW / kc.W : Real(0);
  for (int k = 0; k < 3; ++k) {
    const Real lw = kc.g * lam[k] + coef * kc.w[k];
    u_bar[k] += lw;
    vin_bar[k] += lam[k] - lw;
    a_bar[k] += kc.tau * kc.g * lam[k];
  }
}

// Trilinear weights and their gradient: u = sum w F, du/dx_m = sum dw/dx_m F.
template <class Real>
__device__ __forceinline__ void gather_grad(const typename Prec<Real>::Vec4 *__restrict__ F, const Phys &ph,
                                            typename Prec<Real>::Pos px, typename Prec<Real>::Pos py,
                                            typename Prec<Real>::Pos pz, Real G[3][3]) {
  double fx, fy, fz;
  const int nx = ph.nx, ny = ph.ny, nz = ph.nz;
  int ix = frac_cell(px, nx, fx);
  int ix1 = ix + 1 == nx ? 0 : ix + 1;
  int iy = node_cell(as_signed(py), ny, fy);
  int iz = node_cell(as_signed(pz), nz, fz);
  // derivative of the fractions with respect to the coordinates in metres (0 where clamped)
  const double sy = (as_signed(py) * ph.ur + ph.R) * (ny - 1) / (2.0 * ph.R);
  const double sz = (as_signed(pz) * ph.ur + ph.R) * (nz - 1) / (2.0 * ph.R);
  const Real dfx = Real(nx / ph.L);
  const Real dfy = (sy > 0.0 && sy < ny - 1) ? Real((ny - 1) / (2.0 * ph.R)) : Real(0);
  const Real dfz = (sz > 0.0 && sz < nz - 1) ? Real((nz - 1) / (2.0 * ph.R)) : Real(0);
  const Real wx[2] = {Real(1.0 - fx), Real(fx)}, wy[2] = {Real(1.0 - fy), Real(fy)},
             wz[2] = {Real(1.0 - fz), Real(fz)};
  const Real sgn[2] = {Real(-1), Real(1)};
  const int xs[2] = {ix, ix1};
  for (int c = 0; c < 3; ++c)
    for (int m = 0; m < 3; ++m) G[c][m] = 0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 2; ++e) {
        const auto v = F[((size_t)xs[a] * ny + (iy + b)) * nz + iz + e];
        const Real dwx = sgn[a] * dfx * wy[b] * wz[e];
        const Real dwy = wx[a] * sgn[b] * dfy * wz[e];
        const Real dwz = wx[a] * wy[b] * sgn[e] * dfz;
        const Real val[3] = {(Real)v.x, (Real)v.y, (Real)v.z};
        for (int c = 0; c < 3; ++c) {
          G[c][0] += dwx * val[c];
          G[c][1] += dwy * val[c];
          G[c][2] += dwz * val[c];
        }
      }
}

// ---------------------------------------------------------------- k_adj_init

template <class Real>
__global__ __launch_bounds__(256) void k_adj_init(State<Real> st, Phys ph, AdjState<Real> ad, const double *w_s,
                                                  double scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  const double d = st.d[i];
  const double m = ph.mass_coef * d * d * d;
  ad.lam_ell[i] = Real(scale * w_s[st.sid[i]] * m * exp(-st.ell[i]));
  ad.xb[0][i] = ad.xb[1][i] = ad.xb[2][i] = 0;
  ad.vb[0][i] = ad.vb[1][i] = ad.vb[2][i] = 0;
  ad.ab[0][i] = ad.ab[1][i] = ad.ab[2][i] = 0;
  ad.ub[0][i] = ad.ub[1][i] = ad.ub[2][i] = 0;
  ad.gs[i] = 0.0;
  ad.gA[i] = 0.0;
}

// ---------------------------------------------------------------- k_adj_post
// Reverse of the end of step n (S_n -> S_{n+1}).  mode ADJ_SEED: only the
// parameter partials of the force evaluation at S_{n+1} (the seed).
template <class Real>
__global__ __launch_bounds__(256) void k_adj_post(State<Real> st, Phys ph, TapeEntry<Real> s0, TapeEntry<Real> s1,
                                                  AdjState<Real> ad, int mode) {
  using Pos = typename Prec<Real>::Pos;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  const SampleDev sp = st.samples[st.sid[i]];
  const double d = st.d[i];
  const double m = ph.mass_coef * d * d * d;
  const Real dr = Real(d);
  const Real taup = Real(ph.tau_coef * d * d);
  const Real h = Real(0.5 * ph.dt);
  const Real inv_nu = Real(1.0 / ph.nu);
  const bool drag = (ph.flags & F_DRAG) != 0;
  const Pos px = s1.px[i], py = s1.py[i], pz = s1.pz[i];
  Real xb[3] = {0, 0, 0}, vpb[3] = {0, 0, 0};
  Real ab[3] = {ad.ab[0][i], ad.ab[1][i], ad.ab[2][i]};
  Real ub[3] = {ad.ub[0][i], ad.ub[1][i], ad.ub[2][i]};
  const double y = pos_m(py, s1.ry[i], ph.ur), z = pos_m(pz, s1.rz[i], ph.ur);
  const double rho = sqrt(y * y + z * z);
  const double ery = rho > 0.0 ? y / rho : 0.0, erz = rho > 0.0 ? z / rho : 0.0;

  if (!(mode & ADJ_SEED)) {
    // recompute v' (first half kick of step n) from S_n
    KickCache<Real> k1, k2;
    const Real v0[3] = {s0.vx[i], s0.vy[i], s0.vz[i]};
    const Real u0[3] = {s0.ux[i], s0.uy[i], s0.uz[i]};
    const Real a0[3] = {s0.ax[i], s0.ay[i], s0.az[i]};
    kick_fwd(v0, u0, a0, dr, taup, h, inv_nu, drag, k1);
    ad.vp[0][i] = k1.v[0]; ad.vp[1][i] = k1.v[1]; ad.vp[2][i] = k1.v[2];
    // smoothed tally: l += sigma(-g / (eps d)) / soft_tau, g = R - rho - d/2
    {
      const double gg = ph.R - rho - 0.5 * d;
      const double sig = 1.0 / (1.0 + exp(gg / (ph.soft_eps * d)));
      const double dl_drho = sig * (1.0 - sig) / (ph.soft_eps * d) * ph.soft_rate * ph.dt;
      const Real c = Real((double)ad.lam_ell[i] * dl_drho);
      xb[1] += c * Real(ery);
      xb[2] += c * Real(erz);
    }
    // second half kick: v^{n+1} = K(v', u^{n+1}, a^{n+1})
    const Real u1[3] = {s1.ux[i], s1.uy[i], s1.uz[i]};
    const Real a1[3] = {s1.ax[i], s1.ay[i], s1.az[i]};
    kick_fwd(k1.v, u1, a1, dr, taup, h, inv_nu, drag, k2);
    const Real lam[3] = {ad.vb[0][i], ad.vb[1][i], ad.vb[2][i]};
    kick_adj(k2, lam, h, drag, vpb, ub, ab);
    // gather: u^{n+1} = U(x^{n+1})
    Real G[3][3];
    gather_grad<Real>(st.field, ph, px, py, pz, G);
    for (int mm = 0; mm < 3; ++mm) xb[mm] += ub[0] * G[0][mm] + ub[1] * G[1][mm] + ub[2] * G[2][mm];
  }

  // wall terms at x^{n+1}: a = mag(rho) e_r
  const double q = sp.charge_scale * st.qb[i];
  double gs_acc = 0.0, gA_acc = 0.0;
  if ((ph.flags & (F_WALL_IMAGE | F_WALL_VDW)) && rho > 0.0) {
    const double hh = ph.R - rho;
    const bool hclamp = hh < 0.5 * d;
    const double hc = hclamp ? 0.5 * d : hh;
    const double g = ph.R - rho - 0.5 * d;
    double mag = 0.0, dmag = 0.0;   // dmag = d mag / d rho
    if (ph.flags & F_WALL_IMAGE) {
      const double mi = ph.k_e * q * q / (4.0 * hc * hc) / m;
      mag += mi;
      if (!hclamp) dmag += 2.0 * mi / hc;                 // d/drho of 1/h^2 with h = R - rho
      gs_acc += ((double)ab[1] * ery + (double)ab[2] * erz) * 2.0 * sp.charge_scale * ph.k_e * st.qb[i] * st.qb[i] /
                (4.0 * hc * hc) / m;
    }
    if ((ph.flags & F_WALL_VDW) && g <= 0.25 * d) {
      const bool sat = g <= ph.delta_sat;
      const double gs = sat ? ph.delta_sat : g;
      const double base = d / (12.0 * gs * gs) / m;        // per unit Hamaker constant
      mag += sp.hamaker * base;
      if (!sat) dmag += 2.0 * sp.hamaker * base / gs;
      gA_acc += ((double)ab[1] * ery + (double)ab[2] * erz) * base;
    }
    if (!(mode & ADJ_SEED)) {
      // d a_y/dy = dmag ey^2 + mag/rho (1 - ey^2), d a_y/dz = (dmag - mag/rho) ey ez, ...
      const double mr = mag / rho;
      const double jyy = dmag * ery * ery + mr * (1.0 - ery * ery);
      const double jzz = dmag * erz * erz + mr * (1.0 - erz * erz);
      const double jyz = (dmag - mr) * ery * erz;
      xb[1] += Real(ab[1] * jyy + ab[2] * jyz);
      xb[2] += Real(ab[1] * jyz + ab[2] * jzz);
    }
  }
  // Coulomb: a_C = (k_e s qb q_ref / (m ux^2)) S with S = s * S'  ->  d a_C / d s = 2 a_C / s
  if (ph.flags & F_COULOMB) {
    const double c1 = ph.k_e * st.qb[i] * ph.q_ref / (m * ph.ux * ph.ux);
    const double cs = (double)ab[0] * s1.cx[i] + (double)ab[1] * s1.cy[i] + (double)ab[2] * s1.cz[i];
    gs_acc += 2.0 * c1 * cs;
    // source record of the pair adjoint: b = c a_bar with c = k_e q q_ref / (m ux^2)
    JAdj<Real> r;
    r.x = px;
    r.y = Real(y * ph.inv_ux);
    r.z = Real(z * ph.inv_ux);
    r.q = Real(q / ph.q_ref);
    const double c = ph.k_e * q * ph.q_ref / (m * ph.ux * ph.ux);
    r.bx = Real(c * ab[0]); r.by = Real(c * ab[1]); r.bz = Real(c * ab[2]);
    r.pad = 0;
    ad.rec[i] = r;
  }
  ad.gs[i] += gs_acc;
  ad.gA[i] += gA_acc;
  ad.xp[0][i] = xb[0]; ad.xp[1][i] = xb[1]; ad.xp[2][i] = xb[2];
  ad.vpb[0][i] = vpb[0]; ad.vpb[1][i] = vpb[1]; ad.vpb[2][i] = vpb[2];
  ad.ab[0][i] = ab[0]; ad.ab[1][i] = ab[1]; ad.ab[2][i] = ab[2];
}

// ---------------------------------------------------------------- Coulomb pair adjoint

__device__ __forceinline__ float rsqa(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqa(double x) { return 1.0 / sqrt(x); }

// x_bar_i += (1/ux) sum_j J(r_ij) (q_j b_i - q_i b_j), J(r) = I/r^3 - 3 r r^T / r^5
// (or (I - r^ r^T) / (r d^2) inside the overlap clamp).  Same mapping as the
// forward pair kernel: targets in lanes, source records from SGPRs, waves
// splitting the source range, blocks recomputed exactly when a source is
// closer than the largest diameter, FP64 combination of the per-wave partials.
template <class Real, int WAVES, int BLK>
__global__ __launch_bounds__(64 * WAVES) void k_coulomb_vjp(const TileDev *__restrict__ tiles,
                                                            const JAdj<Real> *__restrict__ rec,
                                                            const Real *__restrict__ jr, Real *__restrict__ ox,
                                                            Real *__restrict__ oy, Real *__restrict__ oz, Real near2,
                                                            Real inv_ux) {
  using Pos = typename Prec<Real>::Pos;
  __shared__ double red[WAVES][3][64];
  const TileDev t = tiles[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int per = ((t.jcount + WAVES - 1) / WAVES + BLK - 1) / BLK * BLK;
  const int jb = t.j0 + w * per;
  const int je = min(t.j0 + t.jcount, jb + per);
  // the tile may hold more than 64 targets (its width follows the forward pair
  // kernel's shape): walk it in chunks of one target per lane
  for (int c0 = 0; c0 < t.icount; c0 += 64) {
    const int ii = c0 + lane < t.icount ? c0 + lane : c0;
    const JAdj<Real> me = rec[t.i0 + ii];
    const Pos xi = me.x;
    const Real yi = me.y, zi = me.z, qi = me.q, bx = me.bx, by = me.by, bz = me.bz;
    const Real ri = jr[t.i0 + ii];
    double hx = 0, hy = 0, hz = 0;
    for (int j0 = jb; j0 < je; j0 += BLK) {
      const int n = min(BLK, je - j0);
      Real sx = 0, sy = 0, sz = 0;
      uint64_t nearmask = 0;
      for (int jj = 0; jj < n; ++jj) {
        const JAdj<Real> s = rec[j0 + jj];
        const Real dx = sdiff(xi, s.x), dy = yi - s.y, dz = zi - s.z;
        const Real r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, Real(1))));
        nearmask |= __builtin_amdgcn_ballot_w64(r2 < near2);
        const Real inv = rsqa(r2);
        const Real inv2 = inv * inv;
        const Real inv3 = inv2 * inv;
        const Real px_ = fma(s.q, bx, -qi * s.bx);
        const Real py_ = fma(s.q, by, -qi * s.by);
        const Real pz_ = fma(s.q, bz, -qi * s.bz);
        const Real t3 = Real(3) * (dx * px_ + dy * py_ + dz * pz_) * inv2;
        sx = fma(inv3, px_ - t3 * dx, sx);
        sy = fma(inv3, py_ - t3 * dy, sy);
        sz = fma(inv3, pz_ - t3 * dz, sz);
      }
      if (nearmask) {
        sx = sy = sz = 0;
        for (int jj = 0; jj < n; ++jj) {
          const JAdj<Real> s = rec[j0 + jj];
          const Real rj = jr[j0 + jj];
          const Real dx = sdiff(xi, s.x), dy = yi - s.y, dz = zi - s.z;
          const Real r2 = dx * dx + dy * dy + dz * dz;
          if (!(r2 > Real(0))) continue;
          const Real r = sqrt(r2);
          const Real dd = ri + rj;
          const Real px_ = s.q * bx - qi * s.bx, py_ = s.q * by - qi * s.by, pz_ = s.q * bz - qi * s.bz;
          const Real rp = (dx * px_ + dy * py_ + dz * pz_) / r2;
          Real k0, k1;   // J p = k0 p - k1 (r.p / r^2) r
          if (r >= dd) { k0 = Real(1) / (r2 * r); k1 = Real(3) * k0; }
          else { k0 = Real(1) / (r * dd * dd); k1 = k0; }
          sx += k0 * px_ - k1 * rp * dx;
          sy += k0 * py_ - k1 * rp * dy;
          sz += k0 * pz_ - k1 * rp * dz;
        }
      }
      hx += (double)sx; hy += (double)sy; hz += (double)sz;
    }
    red[w][0][lane] = hx; red[w][1][lane] = hy; red[w][2][lane] = hz;
    __syncthreads();
    if ((int)threadIdx.x < 64 && c0 + (int)threadIdx.x < t.icount) {
      double s0 = 0, s1 = 0, s2 = 0;
      for (int q = 0; q < WAVES; ++q) { s0 += red[q][0][threadIdx.x]; s1 += red[q][1][threadIdx.x]; s2 += red[q][2][threadIdx.x]; }
      const int i = t.i0 + c0 + threadIdx.x;
      ox[i] = Real(s0 * (double)inv_ux); oy[i] = Real(s1 * (double)inv_ux); oz[i] = Real(s2 * (double)inv_ux);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- short-range pair adjoint

// dF/dr of the cohesive force of vdw_force (product form), same units.
template <class Real>
__device__ __forceinline__ void vdw_force_and_slope(Real gs_m, Real di_m, Real dj_m, Real A, Real &F, Real &dF) {
  const Real u = Real(1e6);
  const Real r1 = Real(0.5) * di_m * u, r2 = Real(0.5) * dj_m * u, g = gs_m * u;
  const Real s = r1 + r2, t = r1 - r2;
  const Real r = s + g;
  const Real P = g * (g + Real(2) * s);
  const Real Q = (r - t) * (r + t);
  const Real PQ = P * Q;
  F = Real(32.0 / 3.0) * A * u * (r1 * r1 * r1) * (r2 * r2 * r2) * r / (PQ * PQ);
  // dF/dr = F (1/r - 4r/P - 4r/Q), r in micrometres -> per metre: * u
  dF = F * (Real(1) / r - Real(4) * r / P - Real(4) * r / Q) * u;
}

template <class Real>
__global__ __launch_bounds__(256) void k_short_range_vjp(State<Real> st, Phys ph, AdjState<Real> ad, int n_cells,
                                                         int mode) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= st.cell_start[n_cells]) return;
  const int i = st.cell_idx[t];
  const SampleDev sp = st.samples[st.sid[i]];
  const auto px = st.px[i], py = st.py[i], pz = st.pz[i];
  const double rxi = st.rx[i], ryi = st.ry[i], rzi = st.rz[i];
  int cx, cy, cz, mx, my, mz;
  short_range_cells(px, py, pz, sp, cx, cy, cz, mx, my, mz);
  const double di_d = st.d[i];
  const Real di = Real(di_d);
  const Real mi = Real(ph.mass_coef) * di * di * di;
  const Real A = Real(sp.hamaker);
  const Real dsat = Real(ph.delta_sat);
  const bool vdw = (ph.flags & F_VDW) != 0, col = (ph.flags & F_COLLIDE) != 0;
  const Real wi[3] = {ad.ab[0][i] / mi, ad.ab[1][i] / mi, ad.ab[2][i] / mi};
  const Real vi[3] = {ad.vp[0][i], ad.vp[1][i], ad.vp[2][i]};
  Real xb[3] = {0, 0, 0}, vb[3] = {0, 0, 0};
  double gA = 0.0;
  // only the neighbour cells whose shared face is closer than the reach can hold a partner
  for (int ox = -1; ox <= 1; ++ox) {
    if ((ox < 0 && !(mx & 1)) || (ox > 0 && !(mx & 2))) continue;
    int xx = cx + ox;
    xx = xx < 0 ? xx + sp.ncx : (xx >= sp.ncx ? xx - sp.ncx : xx);
    for (int oy = -1; oy <= 1; ++oy) {
      if ((oy < 0 && !(my & 1)) || (oy > 0 && !(my & 2))) continue;
      const int yy = cy + oy;
      if (yy < 0 || yy >= sp.ncy) continue;
      for (int oz = -1; oz <= 1; ++oz) {
        if ((oz < 0 && !(mz & 1)) || (oz > 0 && !(mz & 2))) continue;
        const int zz = cz + oz;
        if (zz < 0 || zz >= sp.ncz) continue;
        const int c = sp.cell_base + (xx * sp.ncy + yy) * sp.ncz + zz;
        const int e = st.cell_start[c + 1];
        for (int k = st.cell_start[c]; k < e; ++k) {
          const int j = st.cell_idx[k];
          if (j == i) continue;
          // the forward's pair geometry and range test (FP64 gap)
          const double dj_d = st.d[j];
          double gx, gy, gz, gd;
          const double gap_d = pair_gap(px, py, pz, st.px[j], st.py[j], st.pz[j], rxi - (double)st.rx[j],
                                        ryi - (double)st.ry[j], rzi - (double)st.rz[j], ph.ux, ph.ur,
                                        0.5 * (di_d + dj_d), gx, gy, gz, gd);
          if (gap_d > 0.25 * fmin(di_d, dj_d) || gd == 0.0) continue;
          const double inv_d = 1.0 / gd;
          const Real inv = Real(inv_d);
          const Real n[3] = {Real(gx * inv_d), Real(gy * inv_d), Real(gz * inv_d)};
          const Real dj = Real(dj_d);
          const Real gap = Real(gap_d);
          const Real mj = Real(ph.mass_coef) * dj * dj * dj;
          // pair force on i along n: Fs = -F_vdw(gs) + [gap<0] m_eff (K overlap - H v_n)
          Real Fs = 0, Fr = 0, Fv = 0;
          Real vrel[3] = {0, 0, 0}, vn = 0;
          if (vdw) {
            Real F1, dF1;
            const bool sat = gap <= dsat;
            vdw_force_and_slope(sat ? dsat : gap, di, dj, Real(1), F1, dF1);
            Fs -= A * F1;
            if (!sat) Fr -= A * dF1;
            gA -= (double)((wi[0] * n[0] + wi[1] * n[1] + wi[2] * n[2]) * F1);
          }
          if (col && gap < Real(0)) {
            const Real meff = mi * mj / (mi + mj);
            for (int q = 0; q < 3; ++q) vrel[q] = vi[q] - ad.vp[q][j];
            vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
            Fs += meff * (Real(ph.col_K) * (-gap) - Real(ph.col_H) * vn);
            Fr += meff * -Real(ph.col_K);
            Fv = meff * -Real(ph.col_H);
          }
          if (mode & ADJ_SEED) continue;
          // omega = a_bar_i/m_i - a_bar_j/m_j
          const Real om[3] = {wi[0] - ad.ab[0][j] / mj, wi[1] - ad.ab[1][j] / mj, wi[2] - ad.ab[2][j] / mj};
          const Real on = om[0] * n[0] + om[1] * n[1] + om[2] * n[2];
          for (int q = 0; q < 3; ++q) {
            xb[q] += Fr * n[q] * on + Fv * on * (vrel[q] - vn * n[q]) * inv + Fs * inv * (om[q] - n[q] * on);
            vb[q] += Fv * n[q] * on;
          }
        }
      }
    }
  }
  ad.gA[i] += gA;
  ad.xs[0][i] = xb[0]; ad.xs[1][i] = xb[1]; ad.xs[2][i] = xb[2];
  ad.vs[0][i] = vb[0]; ad.vs[1][i] = vb[1]; ad.vs[2][i] = vb[2];
}

// ---------------------------------------------------------------- k_adj_pre

template <class Real>
__global__ __launch_bounds__(256) void k_adj_pre(State<Real> st, Phys ph, TapeEntry<Real> s0, AdjState<Real> ad,
                                                 int have_coulomb, int have_sr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  const double d = st.d[i];
  const Real dr = Real(d);
  const Real taup = Real(ph.tau_coef * d * d);
  const Real h = Real(0.5 * ph.dt);
  const bool drag = (ph.flags & F_DRAG) != 0;
  Real xb[3] = {ad.xb[0][i] + ad.xp[0][i], ad.xb[1][i] + ad.xp[1][i], ad.xb[2][i] + ad.xp[2][i]};
  if (have_coulomb) { xb[0] += ad.xc[0][i]; xb[1] += ad.xc[1][i]; xb[2] += ad.xc[2][i]; }
  Real vpb[3] = {ad.vpb[0][i], ad.vpb[1][i], ad.vpb[2][i]};
  if (have_sr) {
    for (int q = 0; q < 3; ++q) { xb[q] += ad.xs[q][i]; vpb[q] += ad.vs[q][i]; }
  }
  const Real dt = Real(ph.dt);
  for (int q = 0; q < 3; ++q) vpb[q] += dt * xb[q];     // drift x^{n+1} = x^n + dt v'
  KickCache<Real> k1;
  const Real v0[3] = {s0.vx[i], s0.vy[i], s0.vz[i]};
  const Real u0[3] = {s0.ux[i], s0.uy[i], s0.uz[i]};
  const Real a0[3] = {s0.ax[i], s0.ay[i], s0.az[i]};
  kick_fwd(v0, u0, a0, dr, taup, h, Real(1.0 / ph.nu), drag, k1);
  Real vb[3] = {0, 0, 0}, ub[3] = {0, 0, 0}, ab[3] = {0, 0, 0};
  kick_adj(k1, vpb, h, drag, vb, ub, ab);
  for (int q = 0; q < 3; ++q) {
    ad.xb[q][i] = xb[q];
    ad.vb[q][i] = vb[q];
    ad.ub[q][i] = ub[q];
    ad.ab[q][i] = ab[q];
  }
}

// ---------------------------------------------------------------- per-sample reduction

template <class Real>
__global__ __launch_bounds__(256) void k_adj_reduce(State<Real> st, AdjState<Real> ad, double *out) {
  __shared__ double red[2][256];
  const SampleDev sp = st.samples[blockIdx.x];
  double a = 0, b = 0;
  for (int i = sp.start + threadIdx.x; i < sp.start + sp.count; i += blockDim.x) { a += ad.gs[i]; b += ad.gA[i]; }
  red[0][threadIdx.x] = a; red[1][threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) { red[0][threadIdx.x] += red[0][threadIdx.x + s]; red[1][threadIdx.x] += red[1][threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[2 * blockIdx.x] = red[0][0]; out[2 * blockIdx.x + 1] = red[1][0]; }
}

// ---------------------------------------------------------------- launchers

template <class Real> static dim3 grid_n(int n) { return dim3((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

template <class Real> void launch_tape_store(const State<Real> &st, const TapeEntry<Real> &t, int n, bool ell, hipStream_t s) {
  hipLaunchKernelGGL(k_tape_store<Real>, grid_n<Real>(n), dim3(256), 0, s, st, t, n, (int)ell);
}
template <class Real> void launch_tape_load(const State<Real> &st, const TapeEntry<Real> &t, int n, bool ell, hipStream_t s) {
  hipLaunchKernelGGL(k_tape_load<Real>, grid_n<Real>(n), dim3(256), 0, s, st, t, n, (int)ell);
}
template <class Real>
void launch_adj_init(const State<Real> &st, const Phys &ph, const AdjState<Real> &ad, const double *w, double scale,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_adj_init<Real>, grid_n<Real>(ph.N), dim3(256), 0, s, st, ph, ad, w, scale);
}
template <class Real>
void launch_adj_post(const State<Real> &st, const Phys &ph, const TapeEntry<Real> &s0, const TapeEntry<Real> &s1,
                     const AdjState<Real> &ad, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_post<Real>, grid_n<Real>(ph.N), dim3(256), 0, s, st, ph, s0, s1, ad, mode);
}
template <class Real>
void launch_coulomb_vjp(const State<Real> &st, const Phys &ph, const AdjState<Real> &ad, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return;
  constexpr int W = 16, B = sizeof(Real) == 4 ? 32 : 16;
  hipLaunchKernelGGL((k_coulomb_vjp<Real, W, B>), dim3(n_tiles), dim3(64 * W), 0, s, st.tiles, ad.rec, st.jr,
                     ad.xc[0], ad.xc[1], ad.xc[2], Real(ph.near2), Real(ph.inv_ux));
}
template <class Real>
void launch_short_range_vjp(const State<Real> &st, const Phys &ph, const AdjState<Real> &ad, int n_cells, int mode,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_short_range_vjp<Real>, grid_n<Real>(ph.N), dim3(256), 0, s, st, ph, ad, n_cells, mode);
}
template <class Real>
void launch_adj_pre(const State<Real> &st, const Phys &ph, const TapeEntry<Real> &s0, const AdjState<Real> &ad,
                    bool coulomb, bool sr, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_pre<Real>, grid_n<Real>(ph.N), dim3(256), 0, s, st, ph, s0, ad, (int)coulomb, (int)sr);
}
template <class Real>
void launch_adj_reduce(const State<Real> &st, const Phys &ph, const AdjState<Real> &ad, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_reduce<Real>, dim3(ph.S), dim3(256), 0, s, st, ad, out);
}

#define DEPO_ADJ_INST(R)                                                                                     \
  template void launch_tape_store<R>(const State<R> &, const TapeEntry<R> &, int, bool, hipStream_t);       \
  template void launch_tape_load<R>(const State<R> &, const TapeEntry<R> &, int, bool, hipStream_t);        \
  template void launch_adj_init<R>(const State<R> &, const Phys &, const AdjState<R> &, const double *,     \
                                   double, hipStream_t);                                                    \
  template void launch_adj_post<R>(const State<R> &, const Phys &, const TapeEntry<R> &, const TapeEntry<R> &, \
                                   const AdjState<R> &, int, hipStream_t);                                  \
  template void launch_coulomb_vjp<R>(const State<R> &, const Phys &, const AdjState<R> &, int, hipStream_t); \
  template void launch_short_range_vjp<R>(const State<R> &, const Phys &, const AdjState<R> &, int, int,    \
                                          hipStream_t);                                                     \
  template void launch_adj_pre<R>(const State<R> &, const Phys &, const TapeEntry<R> &, const AdjState<R> &, \
                                  bool, bool, hipStream_t);                                                 \
  template void launch_adj_reduce<R>(const State<R> &, const Phys &, const AdjState<R> &, double *, hipStream_t);
DEPO_ADJ_INST(float)
DEPO_ADJ_INST(double)

}  // namespace depo
