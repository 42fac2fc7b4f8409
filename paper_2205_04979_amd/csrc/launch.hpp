// Host-side launchers of the device kernels (one translation unit per kernel family).
#pragma once

#include "common.hpp"

namespace depo {

// k_prepare modes
enum : int { P_KICK_DRIFT = 1, P_COULOMB = 2, P_CELLS = 4, P_SEED = 8 };
// k_finish modes
// F_PAIR_SUMS (FP32): the symmetric pair kernel ran without its own finishing pass; k_finish turns
// the fixed-point accumulators into the FP32 Coulomb sums and clears them, every particle's
enum : int { F_KICK = 1, F_V_FROM_FLUID = 2, F_FLUID_ONLY = 4, F_PAIR_SUMS = 8 };

template <class Real> void launch_prepare(const State<Real> &st, const Phys &ph, int mode, hipStream_t s);
template <class Real> void launch_finish(const State<Real> &st, const Phys &ph, int mode, hipStream_t s);
template <class Real> void launch_tally(const State<Real> &st, const Phys &ph, int nstep, hipStream_t s);

// Storage order: at the start of a step that follows a multiple of `every` steps (decided on the
// device from the step counter), permute the per-particle state into the order of the last cell list.
template <class Real>
void launch_order(const State<Real> &st, const OrderScratch<Real> &sc, int n, int n_cells, int every, hipStream_t s);

// Cell list: scan of the histogram, scatter, in-cell ordering, short-range forces.
template <class Real>
void launch_cells(const State<Real> &st, const Phys &ph, int n_cells, int n_scan_blocks, hipStream_t s);
template <class Real> void launch_short_range(const State<Real> &st, const Phys &ph, int n_cells, hipStream_t s);
void launch_clear_int(int32_t *p, size_t n, hipStream_t s);

// Coulomb pair sums.
struct CoulombConfig {
  int ipl;     // targets per lane
  int waves;   // waves per workgroup (split the source range; symmetric: each owns 64*ipl targets)
  int block;   // sources per compensated block
  bool compensated;  // Kahan accumulation of the block sums (FP32); plain sums otherwise
  bool symmetric = false;  // FP32: each unordered pair once, reaction on the source (Newton's third law)
  bool int_rec = false;    // symmetric FP32: y and z of the source records as 32-bit integers in x quanta
};
template <class Real>
void launch_coulomb(const State<Real> &st, const Phys &ph, int n_tiles, const CoulombConfig &cfg, hipStream_t s);
int coulomb_tile_targets(const CoulombConfig &cfg);
bool coulomb_config_supported(int real_bytes, const CoulombConfig &cfg);

// Symmetric FP32 pair sums: diagonal items, off-diagonal items, then the fixed-order
// reduction of each particle's partial slots into cx/cy/cz.
int coulomb_sym_tile(const CoulombConfig &cfg);   // targets (= sources) per item
bool coulomb_sym_supported(const CoulombConfig &cfg);
// defer_finish: leave the fixed-point accumulators for k_finish (mode F_PAIR_SUMS) instead of
// converting them with k_pair_finish
void launch_coulomb_sym(const State<float> &st, const Phys &ph, int n_diag, int n_off, const CoulombConfig &cfg,
                        hipStream_t s, bool defer_finish = false);

// P3M electrostatics (single-sample layouts): mesh geometry, splitting and workspace.
struct P3mDev {
  int nx, nc, P;          // mesh nodes along x; across the section (with spares); padded P = 2 nc
  int ncx, ncy;           // short-range cells along x and across the section (cells >= r_max)
  double hx, hy;          // mesh spacings [m]
  double alpha, rmax;     // splitting parameter [1/m] and short-range cutoff [m]
  const double *q_scale;  // device: fixed-point units per unit of scaled charge
  // mesh arrays of nx x P x P complex values: float2 in the FP32 form, double2 in the FP64 form
  void *ghat[3];          // transformed, deconvolved Green's function per field component
  void *rho, *work;       // transformed charge; one field component (FP32 form: adjacent, so that
                          // together they hold one double2 mesh for the Green's function set-up)
  unsigned long long *qmesh;   // fixed-point TSC charge, nx x nc x nc (zero between steps)
  double *slong;          // [3][N] long-range part at the particles [1/m^2]
  int32_t *cell_of, *counts, *starts, *fill, *sorted;   // short-range cell list
  void *rec;              // cell-sorted source records of the short-range pass (N records)
  float2 *table;          // tabulated short-range profile (FP32 form), 2048 intervals + (0, 0)
};
void p3m_setup_green(const P3mDev &m, double L, int images, bool fp32_mesh, hipStream_t s);
template <class Real> void launch_p3m(const State<Real> &st, const Phys &ph, const P3mDev &m, hipStream_t s);

// One-dimensional Eulerian low-fidelity model, one lane per particle class.
struct LfConst {
  double R, nu, rho_f, rho_p, re_tau, eps0;
  int n_wall, n_core;
};
void launch_lf(const LfConst &c, int64_t n, const double *d, const double *q, const double *A, double *out,
               hipStream_t s);

}  // namespace depo
