// Device-side data layout and shared helpers of the deposition step (gfx950).
//
// Particle state lives in HBM as structure-of-arrays so that every per-particle
// kernel reads and writes fully coalesced 64-lane rows.  Positions are stored
// as fixed-point integers: x as an unsigned B-bit fraction of the periodic
// length L (so the periodic wrap and the minimum-image displacement are plain
// integer wrap-around), y and z as signed B-bit multiples of R / 2^(B-2).
// B = 32 in the FP32 form and 64 in the FP64 form.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace depo {

template <class Real> struct Prec;
template <> struct Prec<float> {
  using Pos = uint32_t;
  using SPos = int32_t;
  using Vec4 = float4;
  static constexpr int B = 32;
};
template <> struct Prec<double> {
  using Pos = uint64_t;
  using SPos = int64_t;
  using Vec4 = double4;
  static constexpr int B = 64;
};

// Coulomb source record streamed through the scalar cache by the pair kernel:
// raw x bits, y and z in units of the x quantum, and the scaled charge (0 for
// a removed particle, so it drops out of every sum without compaction).  With
// F_INT_RECORDS (FP32) y and z are rounded to integers in x quanta and stored as
// int32 bit patterns, so that every coordinate difference of a pair is exact.
template <class Real> struct JSrc;
template <> struct __align__(16) JSrc<float> { uint32_t x; float y, z, q; };
template <> struct __align__(32) JSrc<double> { uint64_t x; double y, z, q; };

struct SampleDev {
  int32_t start, count;           // particle range
  int32_t ncx, ncy, ncz;          // cell grid
  int32_t cell_base;              // first global cell id of this sample
  double charge_scale, hamaker, temperature;
  // short-range reach (largest centre distance with a contact or cohesive force, plus a
  // relative margin of 1e-5 for rounding) in cell widths along x and along y/z
  double sr_tx, sr_tr;
};

// One work item of the pair kernel: targets [i0, i0+icount) of a sample whose
// sources are [j0, j0+jcount).
struct TileDev { int32_t i0, icount, j0, jcount; };

// One work item of the symmetric pair kernel: targets [i0, i0+icount) against
// sources [j0, j0+jcount) of sample `sample`.  A diagonal item (j0 == i0) forms
// all ordered pairs of its tile on the target side and applies no reaction.
struct __align__(32) SymItem {
  int32_t i0, icount, j0, jcount, sample, pad[3];
};

// Per-launch constants, all in double; kernels convert to the working type.
struct Phys {
  int32_t N, S, nx, ny, nz;
  uint32_t flags;
  double R, L, ux, ur;            // lengths [m]; fixed-point quanta of x and of y/z
  double inv_ux, inv_ur;
  double dt;
  double nu, rho_p, rho_f;
  double tau_coef;                // tau_p = tau_coef d^2
  double mass_coef;               // m = mass_coef d^3
  double k_e;                     // Coulomb constant
  double q_ref;                   // charge unit of the j-stream
  double yz_over_x;               // ur / ux
  double delta_sat;               // van der Waals saturation gap [m]
  double col_K, col_H;            // contact: a = m_j/(m_i+m_j) (col_K overlap - col_H v_n)
  double g_body[3];
  double E_young, delta_c, acont_coef;
  double soft_eps, soft_rate;     // eps_s = soft_eps d ; dl/dt = sigma(-g/eps_s) * soft_rate
  double near2;                   // (largest diameter / ux)^2: pair-kernel exact-path threshold
};

enum : uint32_t {
  F_DRAG = 1u << 0, F_COULOMB = 1u << 1, F_COLLIDE = 1u << 2, F_VDW = 1u << 3, F_VDW_GU = 1u << 4,
  F_WALL_IMAGE = 1u << 5, F_WALL_VDW = 1u << 6, F_REBOUND = 1u << 7, F_SOFT = 1u << 8, F_BODY = 1u << 9
};

// Internal switch (not a depo_params flag): the Coulomb source records hold y and z as 32-bit
// integers in x quanta (bit patterns in the float fields) for the symmetric integer-record kernel.
enum : uint32_t { F_INT_RECORDS = 1u << 16 };

enum : uint32_t { ERR_NONFINITE = 1u, ERR_ORDER = 2u };

template <class Real>
struct State {
  using Pos = typename Prec<Real>::Pos;
  Pos *px, *py, *pz;
  Real *rx, *ry, *rz;             // position remainder beyond the fixed-point value, in quanta (|r| <= 1/2)
  Real *vx, *vy, *vz;
  Real *ax, *ay, *az;             // stored non-drag acceleration a^n
  Real *ux, *uy, *uz;             // fluid velocity at the particle, u_f(x^n)
  Real *cx, *cy, *cz;             // raw Coulomb sums from the pair kernel
  Real *sx, *sy, *sz;             // short-range accelerations
  double *d, *qb, *ell;
  int32_t *dep, *sid, *nbr;
  int32_t *perm;                  // original index of the particle held in each slot (storage order)
  int32_t *cell_of, *cell_idx, *cell_count, *cell_start, *scan_part;
  JSrc<Real> *js;
  Real *jr;                       // radius in units of the x quantum
  SampleDev *samples;
  TileDev *tiles;
  SymItem *items;                 // symmetric pair-kernel work items (FP32 only)
  double *fx_scale;               // [S] fixed-point units per unit of pair sum, per sample
  unsigned long long *accx, *accy, *accz;  // [N] fixed-point pair-sum accumulators (zero between steps)
  typename Prec<Real>::Vec4 *field;
  int32_t *nstep;
  uint32_t *err;
  double *tally;                  // [S][8]
};

// Second copy of the per-particle state that the storage reorder gathers into (same types).
template <class Real> struct OrderScratch {
  typename Prec<Real>::Pos *px, *py, *pz;
  Real *rx, *ry, *rz, *vx, *vy, *vz, *ax, *ay, *az, *ux, *uy, *uz, *jr;
  double *d, *qb, *ell;
  int32_t *dep, *nbr, *perm;
};

// ---------------------------------------------------------------- fixed-point helpers

// Signed view of a y/z coordinate.
template <class Pos> __device__ __forceinline__ auto as_signed(Pos p) {
  if constexpr (sizeof(Pos) == 4) return (int32_t)p; else return (int64_t)p;
}

// floor(x * n / 2^B) and its fractional part for an unsigned B-bit fraction x.
__device__ __forceinline__ int frac_cell(uint32_t x, int n, double &f) {
  uint64_t t = (uint64_t)x * (uint64_t)n;
  f = (double)(uint32_t)t * 0x1p-32;
  return (int)(t >> 32);
}
__device__ __forceinline__ int frac_cell(uint64_t x, int n, double &f) {
  uint64_t hi = __umul64hi(x, (uint64_t)n);
  uint64_t lo = x * (uint64_t)n;
  f = (double)lo * 0x1p-64;
  return (int)hi;
}

// Cell index along y or z for a grid of n nodes spanning [-R, R]:
// s = (y + R) (n-1) / (2R); returns clamp(floor(s), 0, n-2) and the clamped
// fraction (used by the field gather).
__device__ __forceinline__ int node_cell(int32_t y, int n, double &f) {
  int64_t u = (int64_t)y + (1ll << 30);
  if (u <= 0) { f = 0.0; return 0; }
  int64_t t = u * (int64_t)(n - 1);
  int64_t c = t >> 31;
  if (c >= n - 1) { f = 1.0; return n - 2; }
  f = (double)(t & ((1ll << 31) - 1)) * 0x1p-31;
  return (int)c;
}
__device__ __forceinline__ int node_cell(int64_t y, int n, double &f) {
  // u = y + 2^62 in [0, 2^63] for |y| <= R; product with (n-1) needs 128 bits
  if (y <= -(1ll << 62)) { f = 0.0; return 0; }
  uint64_t u = (uint64_t)(y + (1ll << 62));
  uint64_t hi = __umul64hi(u, (uint64_t)(n - 1));
  uint64_t lo = u * (uint64_t)(n - 1);
  uint64_t c = (hi << 1) | (lo >> 63);
  if (c >= (uint64_t)(n - 1)) { f = 1.0; return n - 2; }
  f = (double)(lo & ((1ull << 63) - 1)) * 0x1p-63;
  return (int)c;
}

// Cell index along y or z for a grid of n cells covering [-R, R]: floor((y + R) n / 2R), clamped.
__device__ __forceinline__ int box_cell(int32_t y, int n) {
  int64_t u = (int64_t)y + (1ll << 30);
  int64_t c = u <= 0 ? 0 : (u * (int64_t)n) >> 31;
  return c >= n ? n - 1 : (int)c;
}
__device__ __forceinline__ int box_cell(int64_t y, int n) {
  if (y <= -(1ll << 62)) return 0;
  uint64_t u = (uint64_t)(y + (1ll << 62));
  uint64_t hi = __umul64hi(u, (uint64_t)n);
  uint64_t lo = u * (uint64_t)n;
  uint64_t c = (hi << 1) | (lo >> 63);
  return c >= (uint64_t)n ? n - 1 : (int)c;
}

// box_cell with the position's fraction of its cell width (0 for a clamped position).
__device__ __forceinline__ int box_cell_frac(int32_t y, int n, double &f) {
  int64_t u = (int64_t)y + (1ll << 30);
  if (u <= 0) { f = 0.0; return 0; }
  int64_t t = u * (int64_t)n;
  int64_t c = t >> 31;
  if (c >= n) { f = 0.0; return n - 1; }
  f = (double)(t & ((1ll << 31) - 1)) * 0x1p-31;
  return (int)c;
}
__device__ __forceinline__ int box_cell_frac(int64_t y, int n, double &f) {
  if (y <= -(1ll << 62)) { f = 0.0; return 0; }
  uint64_t u = (uint64_t)(y + (1ll << 62));
  uint64_t hi = __umul64hi(u, (uint64_t)n);
  uint64_t lo = u * (uint64_t)n;
  uint64_t c = (hi << 1) | (lo >> 63);
  if (c >= (uint64_t)n) { f = 0.0; return n - 1; }
  f = (double)(lo & ((1ull << 63) - 1)) * 0x1p-63;
  return (int)c;
}

// A partner within the reach lies in the neighbour cell below (above) along an axis only
// if the particle is closer than the reach to that face: bit 0 lower, bit 1 upper.
__device__ __forceinline__ int reach_sides(double f, double thr) {
  return (f < thr ? 1 : 0) | (1.0 - f < thr ? 2 : 0);
}

// Cell of a particle and the neighbour cells its short-range walk must visit.
template <class Pos>
__device__ __forceinline__ void short_range_cells(Pos px, Pos py, Pos pz, const SampleDev &sp, int &cx, int &cy,
                                                  int &cz, int &mx, int &my, int &mz) {
  double fx, fy, fz;
  cx = frac_cell(px, sp.ncx, fx);
  cy = box_cell_frac(as_signed(py), sp.ncy, fy);
  cz = box_cell_frac(as_signed(pz), sp.ncz, fz);
  mx = reach_sides(fx, sp.sr_tx);
  my = reach_sides(fy, sp.sr_tr);
  mz = reach_sides(fz, sp.sr_tr);
}

__device__ __forceinline__ int x_cell(uint32_t x, int n) { return (int)(((uint64_t)x * (uint64_t)n) >> 32); }
__device__ __forceinline__ int x_cell(uint64_t x, int n) { return (int)__umul64hi(x, (uint64_t)n); }

// Signed fixed-point difference a - b converted to the working type (minimum image in x).
__device__ __forceinline__ float sdiff(uint32_t a, uint32_t b) { return (float)(int32_t)(a - b); }
__device__ __forceinline__ double sdiff(uint64_t a, uint64_t b) { return (double)(int64_t)(a - b); }

// Centre displacement of particle i from particle j in metres (minimum image in x), its length,
// and the surface gap |r| - s for the contact distance s = (d_i + d_j)/2, all in FP64 from the
// exact integer differences of the fixed-point positions plus the difference of their
// remainders (dr*, in quanta).  The gap is formed as (|r|^2 - s^2) / (|r| + s): near contact it
// is a small fraction of |r|, and the plain difference |r| - s would lose most of its digits.
template <class Pos>
__device__ __forceinline__ double pair_gap(Pos xi, Pos yi, Pos zi, Pos xj, Pos yj, Pos zj, double drx, double dry,
                                           double drz, double ux, double ur, double s, double &dx, double &dy,
                                           double &dz, double &dist) {
  dx = ((double)as_signed(Pos(xi - xj)) + drx) * ux;
  dy = ((double)as_signed(Pos(yi - yj)) + dry) * ur;
  dz = ((double)as_signed(Pos(zi - zj)) + drz) * ur;
  const double r2 = dx * dx + dy * dy + dz * dz;
  dist = sqrt(r2);
  return (r2 - s * s) / (dist + s);
}

// Position along y or z in metres: fixed-point value plus remainder.
template <class Pos, class Real>
__device__ __forceinline__ double pos_m(Pos p, Real r, double ur) { return ((double)as_signed(p) + (double)r) * ur; }

// Round a displacement in quanta to the nearest integer step.
__device__ __forceinline__ int32_t round_step(float q) { return (int32_t)__builtin_rintf(q); }
__device__ __forceinline__ int64_t round_step(double q) { return (int64_t)__builtin_rint(q); }

}  // namespace depo
