// One-dimensional Eulerian deposition model (Appendix B): particle momentum
// equation with turbophoresis, image-charge and wall-cohesion forces, and the
// constant-flux equation that gives V_dep+, for many particle classes at once.
//
// One lane solves one class (d, q, A).  The momentum equation is marched from
// the pipe centre (V = 0) to the wall with implicit drag; the flux equation
// J = D drho/dy + V rho, rho(centre) = 1, J = rho_w h_w, is carried along the
// SAME inward pass: over each cell the exact solution with V, D frozen at the
// cell means maps rho linearly, so rho(y) = alpha(y) + J beta(y) and only two
// scaled coefficients travel with the march (s = 1/alpha, b = beta/alpha; both
// stay bounded where alpha itself would overflow).  At the wall the kinetic
// wall condition closes J = h_w / (s_0 - h_w b_0).  No per-node storage.
//
// Closures (the paper defers them to other publications; these are stated
// substitutes): tau_1+ = tau_p+; V'_fy+ = 0.005 y^2 / (1 + 0.002923 y^2.128);
// Rr = 1 / (1 + tau_p+ / tau_L+), tau_L+ = 10; eps/nu = tau_L+ Rr V'_fy+^2;
// D_B/nu by Stokes-Einstein at 293 K; wall velocity variance
// Rr V'_fy+^2 + k_B T / (m u*^2); half-Maxwellian wall flux.
// Grid: gaps y+ - d+/2 geometric from 1e-12 m to 1 wall unit (n_wall nodes),
// then uniform to the centre (n_core more nodes).

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "launch.hpp"

namespace depo {

namespace {

constexpr double kBoltzmann = 1.380649e-23;
constexpr double kTempLF = 293.0;
constexpr double kTauLPlus = 10.0;
constexpr double kGapMin = 1e-12;

__device__ inline double rms_fluid_plus(double y) {
  return 0.005 * y * y / (1.0 + 0.002923 * pow(y, 2.128));
}

struct Node {
  double y, ym, gap, phi, dif;  // y+, y [m], gap [m], Rr V'^2, D+
};

__global__ void __launch_bounds__(256) k_lf(LfConst c, int64_t n, const double *__restrict__ d_diam,
                                            const double *__restrict__ d_q, const double *__restrict__ d_A,
                                            double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = d_diam[i], q = d_q[i], A = d_A[i];
  if (!(d > 0.0) || !isfinite(d) || !isfinite(q) || !isfinite(A)) {
    out[i] = NAN;
    return;
  }
  const double us = c.re_tau * c.nu / c.R;
  const double lw = c.nu / us;
  const double taup_plus = c.rho_p * d * d / (18.0 * c.rho_f * c.nu) * us * us / c.nu;
  const double m = c.rho_p * M_PI * d * d * d / 6.0;
  const double rr = 1.0 / (1.0 + taup_plus / kTauLPlus);
  const double db_plus = kBoltzmann * kTempLF / (3.0 * M_PI * c.rho_f * c.nu * c.nu * d);
  const double yw = 0.5 * d / lw, yc = c.R / lw;
  const double e_img = q * q / (16.0 * M_PI * c.eps0 * m);  // image force per mass times y^2
  const double c_vdw = A * d / (12.0 * m);                  // wall cohesion per mass times gap^2
  const double inv_us2 = 1.0 / (us * us);
  const int nw = c.n_wall, nn = c.n_wall + c.n_core;
  const double lg0 = log(kGapMin / lw);
  const double core_step = (yc - yw - 1.0) / c.n_core;

  auto node = [&](int k) {
    double g;
    if (k == 0) g = kGapMin / lw;
    else if (k < nw - 1) g = exp(lg0 * (1.0 - (double)k / (double)(nw - 1)));
    else if (k == nw - 1) g = 1.0;
    else if (k == nn - 1) g = yc - yw;
    else g = 1.0 + (double)(k - nw + 1) * core_step;
    Node o;
    o.y = yw + g;
    o.ym = o.y * lw;
    o.gap = g * lw;
    const double v = rms_fluid_plus(o.y);
    o.phi = rr * v * v;
    o.dif = db_plus + kTauLPlus * o.phi;
    return o;
  };

  Node up = node(nn - 1);
  double V = 0.0, K = 0.0;  // speed toward the wall and its kinetic energy at node `up`
  double s = 1.0, b = 0.0;  // flux coefficients at node `up`
  for (int k = nn - 1; k > 0; --k) {
    const Node lo = node(k - 1);
    const double h = up.y - lo.y;
    // momentum: K_lo = K_up + (Phi_up - Phi_lo) + work - h V_lo / tau_1, drag implicit
    const double work =
        (e_img * (1.0 / lo.ym - 1.0 / up.ym) + c_vdw * (1.0 / lo.gap - 1.0 / up.gap)) * inv_us2;
    const double rhs = K + (up.phi - lo.phi) + work;
    double v_lo = 0.0;
    if (rhs > 0.0) {
      const double a = h / taup_plus;
      v_lo = 2.0 * rhs / (a + sqrt(a * a + 2.0 * rhs));
    }
    // flux over the cell: rho_up = rho_lo e^-x + J (h / Dm) (1 - e^-x) / x, x = Vm h / Dm; inverted
    const double vm = 0.5 * (V + v_lo), dm = 0.5 * (up.dif + lo.dif);
    const double x = vm * h / dm;
    double e = 1.0, cf = h / dm;
    if (x > 0.0) {
      e = exp(-x);
      cf *= -expm1(-x) / x;
    }
    b -= cf * s;
    s *= e;
    V = v_lo;
    K = 0.5 * v_lo * v_lo;
    up = lo;
  }
  // kinetic wall condition: flux of a half-Maxwellian with mean V_w and rms vp
  const double vfw = rms_fluid_plus(up.y);
  const double vp = sqrt(rr * vfw * vfw + kBoltzmann * kTempLF / (m * us * us));
  const double M = V / (M_SQRT2 * vp);
  const double hw = vp * exp(-M * M) / sqrt(2.0 * M_PI) + V * (1.0 + erf(M)) * 0.5;
  out[i] = hw / (s - hw * b);
}

}  // namespace

void launch_lf(const LfConst &c, int64_t n, const double *d, const double *q, const double *A, double *out,
               hipStream_t s) {
  if (n <= 0) return;
  const int block = 256;
  const int64_t grid = (n + block - 1) / block;
  hipLaunchKernelGGL(k_lf, dim3((unsigned)grid), dim3(block), 0, s, c, n, d, q, A, out);
}

}  // namespace depo
