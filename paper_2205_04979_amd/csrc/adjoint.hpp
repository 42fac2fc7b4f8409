// Data layout of the reverse pass: tape entries (one particle state per step),
// the adjoint state and the source records of the Coulomb pair adjoint.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace depo {

enum : int { ADJ_SEED = 1 };

// One stored particle state: positions (fixed point and remainder), velocity, non-drag acceleration, fluid
// velocity and raw Coulomb sums (those that formed the acceleration), plus the
// smoothed-tally accumulator when the entry is the final state.
template <class Real> struct TapeEntry {
  typename Prec<Real>::Pos *px, *py, *pz;
  Real *rx, *ry, *rz;
  Real *vx, *vy, *vz, *ax, *ay, *az, *ux, *uy, *uz, *cx, *cy, *cz;
  double *ell;
};

// Source record of the pair adjoint: position, scaled charge and b = c a_bar.
template <class Real> struct JAdj;
template <> struct __align__(32) JAdj<float> { uint32_t x; float y, z, q, bx, by, bz, pad; };
template <> struct __align__(64) JAdj<double> { uint64_t x; double y, z, q, bx, by, bz, pad; };

template <class Real> struct AdjState {
  Real *lam_ell;            // d J / d l_i (scaled)
  Real *xb[3], *vb[3];      // adjoints of x and v at the current step boundary
  Real *ab[3], *ub[3];      // adjoints of the stored acceleration and fluid velocity
  Real *xp[3], *vpb[3];     // partial adjoints from k_adj_post (x^{n+1}, v')
  Real *vp[3];              // recomputed half-step velocity v'
  Real *xc[3];              // Coulomb pair adjoint
  Real *xs[3], *vs[3];      // short-range pair adjoint
  double *gs, *gA;          // per-particle partials of the charge-scale and Hamaker gradients
  JAdj<Real> *rec;
  double *weights;          // [S]
  double *out;              // [S][2]
};

template <class Real>
void launch_tape_store(const State<Real> &st, const TapeEntry<Real> &t, int n, bool ell, hipStream_t s);
template <class Real>
void launch_tape_load(const State<Real> &st, const TapeEntry<Real> &t, int n, bool ell, hipStream_t s);
template <class Real>
void launch_adj_init(const State<Real> &st, const Phys &ph, const AdjState<Real> &ad, const double *w, double scale,
                     hipStream_t s);
template <class Real>
void launch_adj_post(const State<Real> &st, const Phys &ph, const TapeEntry<Real> &s0, const TapeEntry<Real> &s1,
                     const AdjState<Real> &ad, int mode, hipStream_t s);
template <class Real>
void launch_coulomb_vjp(const State<Real> &st, const Phys &ph, const AdjState<Real> &ad, int n_tiles, hipStream_t s);
// FP32 symmetric form over the forward's item list (ipl, waves of cfg); uses the
// state's pair accumulators as FP64 scratch and leaves them zero.
void launch_coulomb_vjp_sym(const State<float> &st, const Phys &ph, const AdjState<float> &ad, int n_diag, int n_off,
                            const CoulombConfig &cfg, hipStream_t s);
template <class Real>
void launch_short_range_vjp(const State<Real> &st, const Phys &ph, const AdjState<Real> &ad, int n_cells, int mode,
                            hipStream_t s);
template <class Real>
void launch_adj_pre(const State<Real> &st, const Phys &ph, const TapeEntry<Real> &s0, const AdjState<Real> &ad,
                    bool coulomb, bool sr, hipStream_t s);
template <class Real>
void launch_adj_reduce(const State<Real> &st, const Phys &ph, const AdjState<Real> &ad, double *out, hipStream_t s);

}  // namespace depo
