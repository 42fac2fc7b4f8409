/*
 * depo.h - C ABI of the MI355X (gfx950) Lagrangian particle-deposition step.
 *
 * The library advances the particles of the high-fidelity model of
 * Yao, Huan & Capecelatro, "Multi-fidelity uncertainty quantification of
 * particle deposition in turbulent pipe flow" (arXiv 2205.04979) through a
 * frozen carrier-gas velocity field: fluid velocity at the particle
 * (Appendix A.2.1), Schiller-Naumann drag (Eq. part_source), pairwise
 * Coulomb forces (Eq. coulomb, Appendix A.2.4), soft-sphere contact
 * (Appendix A.2.2) with van der Waals cohesion (Eq. vdw, Appendix A.2.3),
 * wall image charge and wall cohesion (Section 2.2, Appendix B.2), time
 * integration of Newton's law (Eq. newtonlaw), removal of particles that
 * touch the wall (Appendix A) and the deposition tally that gives V_dep
 * (Eq. 2).  Several independent Monte Carlo samples with their own charge
 * scale, Hamaker constant and temperature (Sections 2.1, 3, 4.4) can share
 * one field and one launch.
 *
 * Conventions
 * -----------
 * - Units are SI; every host-side floating-point input is double.
 * - Memory: the library allocates no device memory.  The caller allocates
 *   one device workspace of depo_workspace_bytes() bytes (for instance a
 *   torch uint8 tensor) and hands it to depo_bind(); the workspace must stay
 *   alive and unmoved until depo_destroy() or the next depo_bind().  Host
 *   arrays are borrowed for the duration of the call only.
 * - Streams: every entry point that takes a depo_stream enqueues its device
 *   work on that HIP stream (NULL = the legacy default stream).  Calls that
 *   return data to the host synchronise that stream before returning.
 * - Errors: every entry point returns a depo_status.  Arguments are validated
 *   on the host before anything is enqueued; on an error nothing is enqueued
 *   and depo_last_error() describes the problem.  Device-side conditions
 *   (a non-finite velocity or acceleration) are recorded in a sticky flag and
 *   reported by the next call that synchronises (depo_tally_read,
 *   depo_read_particles, depo_state_download).  After DEPO_E_HIP the context
 *   should be destroyed.
 * - Threading: a context is used by one host thread at a time.
 * - Precision: params.real_bytes = 4 selects the FP32 form (positions stored
 *   as 32-bit fixed point, velocities/forces FP32, compensated summation of
 *   the Coulomb sums, FP64 wall test and tally); 8 selects FP64 throughout
 *   (positions as 64-bit fixed point).
 * - Layout of particle arrays on the host: [N][3] row-major for vectors,
 *   [N] for scalars; particles of sample s occupy rows
 *   offsets[s] .. offsets[s+1]-1.
 */
#ifndef DEPO_H
#define DEPO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct depo_ctx depo_ctx;   /* opaque, library-owned host object */
typedef void *depo_stream;          /* a hipStream_t; NULL = default stream */

typedef enum {
  DEPO_OK = 0,
  DEPO_E_INVALID = -1,    /* bad argument; nothing was enqueued                 */
  DEPO_E_STATE = -2,      /* call out of order (e.g. step before seed)          */
  DEPO_E_HIP = -3,        /* HIP runtime error; destroy the context            */
  DEPO_E_NONFINITE = -4,  /* a velocity or acceleration became NaN/Inf         */
  DEPO_E_CAPACITY = -5,   /* workspace too small for the requested layout      */
  DEPO_E_CORRUPT = -6     /* checkpoint blob failed its size/format/CRC checks */
} depo_status;

/* Force and behaviour switches (depo_params.flags). */
enum {
  DEPO_DRAG = 1u << 0,        /* Schiller-Naumann drag, Eq. part_source                       */
  DEPO_COULOMB = 1u << 1,     /* pairwise Coulomb force, Eq. coulomb (direct O(N^2) sum)      */
  DEPO_COLLIDE = 1u << 2,     /* soft-sphere normal contact, Appendix A.2.2                   */
  DEPO_VDW = 1u << 3,         /* pair van der Waals cohesion, Eq. vdw                         */
  DEPO_VDW_GU = 1u << 4,      /* soft-sphere saturation gap delta_min (k_r/k)^(1/4), A.2.3    */
  DEPO_WALL_IMAGE = 1u << 5,  /* image-charge attraction to the wall, Section 2.2 / App. B.2  */
  DEPO_WALL_VDW = 1u << 6,    /* sphere-plane cohesion with the wall, Section 2.2 / App. B.2  */
  DEPO_REBOUND_OSU = 1u << 7, /* temperature-dependent stick/rebound at the wall, Eq. CoR     */
  DEPO_SOFT_TALLY = 1u << 8,  /* no removal; smoothed deposition tally (differentiable)       */
  DEPO_BODY_FORCE = 1u << 9   /* constant body acceleration g_body (used by tests)            */
};

/* Physical and numerical parameters, SI.  Validated by depo_create(). */
typedef struct {
  double R;            /* pipe radius [m] (> 0)                                         */
  double L;            /* periodic pipe length [m] (>= 2R)                              */
  double nu;           /* kinematic viscosity of the gas [m^2/s]                        */
  double rho_f;        /* gas density [kg/m^3]                                          */
  double rho_p;        /* particle material density [kg/m^3]                            */
  double dt;           /* time step [s]                                                 */
  double re_tau;       /* friction Reynolds number u* R / nu (only scales V_dep+)       */
  double e_pp;         /* particle-particle restitution coefficient, 0 < e <= 1          */
  int32_t tau_col_steps; /* contact duration in time steps (paper: 15)                  */
  int32_t real_bytes;  /* 4 = FP32 form, 8 = FP64                                       */
  double delta_min;    /* van der Waals saturation gap [m] (paper: 1e-9)                */
  double kr_over_k;    /* real / simulated contact stiffness (paper: 700)               */
  double eps0;         /* vacuum permittivity [F/m]                                     */
  double g_body[3];    /* body acceleration [m/s^2], used with DEPO_BODY_FORCE          */
  double E_young;      /* particle Young's modulus [Pa] (rebound law)                   */
  double delta_c;      /* cohesion length of the rebound law [m]                        */
  double acont_coef;   /* wall contact area = acont_coef * pi d^2 / 4                   */
  double soft_eps;     /* smoothed tally width, fraction of d                           */
  double soft_tau;     /* smoothed tally time scale, in time steps                      */
  uint32_t flags;      /* DEPO_* switches                                               */
  uint32_t reserved;   /* must be 0                                                     */
  double u_bulk;       /* bulk (area-mean axial) gas velocity U_b [m/s], used only by the
                        * capture efficiency of the tally (Eq. CE); 0 = not reported      */
} depo_params;

/* Per-sample inputs of the uncertainty study (Sections 2.1 and 4.4):
 * particle charge q_i = charge_scale * qbase_i, Hamaker constant A [J],
 * particle temperature T [K] (enters only the rebound law). */
typedef struct {
  double charge_scale;
  double hamaker;
  double temperature;
} depo_sample_params;

/* Per-sample deposition tally (Eq. 2). */
typedef struct {
  double m_dep;       /* deposited mass [kg]                                           */
  int64_t n_dep;      /* deposited particle count                                      */
  double m_alive_dt;  /* time integral of the suspended mass [kg s]                    */
  double t;           /* simulated time [s]                                            */
  double v_dep;       /* deposition velocity (R/2) m_dep / m_alive_dt [m/s]            */
  double v_dep_plus;  /* V_dep / u*                                                    */
  double v_dep_se;    /* Poisson standard error of v_dep                               */
  double j_soft;      /* smoothed deposited mass sum_i m_i (1 - exp(-l_i)) [kg]        */
  int64_t n_alive;    /* particles still suspended                                     */
  double ce;          /* capture efficiency (4L/D)(u* / U_b) V_dep+ (Eq. CE, D = 2R); with
                       * DEPO_REBOUND_OSU only sticking impacts deposit, so V_dep+ is the
                       * paper's V_dep+|stick; 0 when u_bulk = 0                         */
} depo_tally;

/* Human-readable name of a status code.  Never NULL; static storage. */
const char *depo_status_string(int status);

/* Create a context from validated parameters.  Host only, touches no GPU.
 * The parameters are those of the particle-phase model of Appendix A.2: the gas
 * (viscosity and density, Eq. part_source), the particle material density, the
 * soft-sphere contact of Appendix A.2.2 (restitution e_pp, contact duration
 * tau_col_steps time steps, stiffness ratio kr_over_k = k_r/k), the van der Waals
 * saturation gap delta_min of Appendix A.2.3, the vacuum permittivity of Coulomb's
 * law (Eq. coulomb), the rebound law of Section 4.4 (Eq. CoR: E_young, delta_c,
 * acont_coef), and the pipe of Section 2.1 (radius R, periodic length L, Re_tau).
 * Returns DEPO_E_INVALID (with *out = NULL) for non-positive or non-finite
 * lengths, densities, viscosity or dt, e_pp outside (0, 1], tau_col_steps < 1,
 * real_bytes not 4 or 8, unknown flag bits, reserved != 0 or a negative or
 * non-finite u_bulk. */
depo_status depo_create(const depo_params *p, depo_ctx **out);

/* Destroy a context and its host-side objects (graphs, staging).  Never frees
 * the caller's workspace.  NULL is ignored. */
void depo_destroy(depo_ctx *ctx);

/* Message of the last failed call on ctx ("" if none); valid until the next call. */
const char *depo_last_error(const depo_ctx *ctx);

/* Declare the batch layout: n_samples >= 1 samples, offsets[n_samples+1]
 * non-decreasing from 0 with N = offsets[n_samples] <= 2^26 particles, and the
 * field grid nx, ny, nz (each 4..4096; nodes x_i = i L / nx periodic,
 * y_j = -R + 2R j/(ny-1), z_k = -R + 2R k/(nz-1)).  Host only.  Resets the
 * binding and the seeded state. */
depo_status depo_set_layout(depo_ctx *ctx, int32_t n_samples, const int64_t *offsets,
                            int32_t nx, int32_t ny, int32_t nz);

/* Device workspace size for the current layout.  Host only. */
depo_status depo_workspace_bytes(const depo_ctx *ctx, size_t *bytes);

/* Bind a caller-owned device workspace (256-byte aligned, at least
 * depo_workspace_bytes() bytes; DEPO_E_CAPACITY otherwise).  Clears the
 * library's counters on the default stream and waits for it. */
depo_status depo_bind(depo_ctx *ctx, void *d_work, size_t bytes);

/* Upload the carrier-gas velocity u_f on the node grid declared by
 * depo_set_layout: h_uvw[nx][ny][nz][3] (z fastest), copied and converted
 * to the working precision; it stays frozen while the particles move.  This is
 * the carrier flow of Section 2.1 and Appendix A.1 that the paper takes from its
 * DNS; any field on the grid is accepted (for instance a synthetic turbulent pipe
 * field: mean profile plus random Fourier modes, zero outside the pipe), and the
 * particles see it through the interpolation u_f[x_p] of Appendix A.2.1
 * (trilinear here).  DEPO_E_INVALID for a non-finite value (nothing is kept);
 * DEPO_E_STATE before depo_bind.  Synchronises the stream. */
depo_status depo_init_field(depo_ctx *ctx, const double *h_uvw, depo_stream stream);

/* Seed the particles (Section 2.1: particles distributed at random in the pipe,
 * each Monte Carlo sample with its own uncertain inputs): per-sample parameters
 * sp[n_samples] (charge scale xi, Hamaker constant A = zeta A_0, temperature T of
 * Sections 2.1 and 4.4); positions h_x3[N][3] with 0 <= x < L (x is wrapped) and
 * y^2 + z^2 < R^2; diameters h_d[N] in (0, R/4); base charges h_qbase[N], so that
 * particle i of sample s carries q_i = sp[s].charge_scale * h_qbase[i] (with
 * h_qbase = q_max(d) this is the charge xi q_max of Eq. 1).  h_v3[N][3] may be
 * NULL, in which case each particle starts at the local fluid velocity.  Positions
 * are stored as fixed point plus a remainder, so they are kept to the input's
 * precision.  Computes the initial acceleration (all forces at the seeded
 * positions) and resets the tally and the step counter.  DEPO_E_INVALID (nothing
 * changed) for a non-finite or out-of-range value; DEPO_E_STATE before the field
 * is uploaded.  Synchronises the stream. */
depo_status depo_seed(depo_ctx *ctx, const depo_sample_params *sp, const double *h_x3,
                      const double *h_v3, const double *h_d, const double *h_qbase,
                      depo_stream stream);

/* Replace the per-sample parameters without touching the particle state
 * (charges are rebuilt from the stored base charges).  Synchronises the stream. */
depo_status depo_set_sample_params(depo_ctx *ctx, const depo_sample_params *sp, depo_stream stream);

/* Advance all samples by n_steps >= 0 time steps (Appendix A.2: drag half
 * kick, drift, wall test, force evaluation, second half kick, tally).
 * Asynchronous: enqueues the step n_steps times on the stream and returns
 * without waiting.  With graphs enabled (the default) the step is captured
 * once and replayed; with direct pair sums and short-range forces both on,
 * the captured step runs the cell build and short-range forces beside the
 * pair kernel (disjoint buffers, same kernels: results equal the direct
 * launches bitwise).  Any call that changes the layout, the parameters, the
 * pair mode or the state (seed, upload) drops the captured step.
 * DEPO_E_STATE before depo_seed; DEPO_E_INVALID for n_steps < 0 or a step
 * counter that would pass 2^31 - 1. */
depo_status depo_step(depo_ctx *ctx, int32_t n_steps, depo_stream stream);

/* Same as depo_step without graph replay, with HIP events recorded on the
 * stream between the kernel families of every step; h_phase_ms[5] receives
 * the summed durations of (particle update before the forces, cell-list build,
 * Coulomb pair sums, short-range forces, force assembly and second half kick)
 * in milliseconds.  1 <= n_steps <= 100000.  Synchronises the stream. */
depo_status depo_step_timed(depo_ctx *ctx, int32_t n_steps, depo_stream stream, double *h_phase_ms);

/* Pair-kernel modes (depo_set_kernel_config). */
enum {
  DEPO_PAIR_PLAIN = 0,      /* one-sided sums, plain accumulation                          */
  DEPO_PAIR_KAHAN = 1,      /* one-sided sums, Kahan-compensated block accumulation        */
  DEPO_PAIR_SYMMETRIC = 2,  /* FP32 only: every unordered pair once, the reaction applied to
                             * the source (Newton's third law); Kahan on the target side,
                             * 64-bit fixed-point combination of per-item partials          */
  DEPO_PAIR_P3M = 3,        /* P3M electrostatics (configured with depo_set_p3m)           */
  DEPO_PAIR_SYMMETRIC_INT = 4 /* FP32 only: DEPO_PAIR_SYMMETRIC with the y and z coordinates of
                             * the source records held as 32-bit integers in x quanta
                             * (L/2^32) instead of floats, so that every coordinate difference
                             * of a pair is exact (the float records hold y and z to 64 quanta
                             * near the wall); needs L >= 2R; about 10 % slower           */
};

/* Choose the Coulomb pair-kernel shape (targets per lane, wavefronts per
 * workgroup, sources per block, mode DEPO_PAIR_*) and whether depo_step
 * replays a captured HIP graph (use_graph != 0, the default) or launches
 * kernels directly.  DEPO_E_INVALID for a shape that is not compiled in.
 * Defaults: (4, 2, 64, DEPO_PAIR_SYMMETRIC) in FP32 (or (1, 8, 32,
 * DEPO_PAIR_KAHAN) for a layout with more than 2^22 symmetric items),
 * (1, 4, 16, DEPO_PAIR_PLAIN) in FP64; block 64 selects the one-sided variant
 * that prefetches source records one group ahead.  The symmetric mode takes
 * block = 64 (sources are paired in rounds of 64) and items of
 * 64 * targets_per_lane * waves >= 256 targets, at most 2^22 of them per
 * layout (DEPO_E_INVALID beyond). */
depo_status depo_set_kernel_config(depo_ctx *ctx, int32_t targets_per_lane, int32_t waves, int32_t block,
                                   int32_t mode, int32_t use_graph);

/* Storage order of the particles: with short-range forces on (a cell list is built every step),
 * the per-particle state is permuted into the order of the last cell list at the start of every
 * step that follows a multiple of `every` steps (0: never, the default), so that the cell-ordered
 * walks and the field gather read contiguous memory.  Every sample keeps its slots (alive particles
 * in cell order, then the removed ones), and the permutation is deterministic.  The library keeps
 * the permutation: every host array it returns is in the caller's order, and checkpoint blobs carry
 * it.  Sums whose order follows the storage (one-sided pair sums, short-range sums, tallies) then
 * round differently from a run without reordering.  The reorder is part of the captured step and
 * decided on the device from the step counter.  The smoothed-tally mode never reorders (the
 * adjoint's stored states share one order).  Drops the captured step.  Host only; DEPO_E_INVALID
 * outside 0..2^20. */
depo_status depo_set_reorder(depo_ctx *ctx, int32_t every);

/* P3M electrostatics (Appendix A.2.4, Eq. coulomb_force): the Coulomb sums
 * from a Gaussian split into a short-range direct part and a long-range mesh
 * part solved with FFTs, O(N log N).  It computes the lattice sum over all x
 * images (period L) with free space across the pipe section, not the nearest
 * image of the direct modes.  Mesh: mesh_x nodes along x (power of two,
 * 16..1024) and mesh_yz across [-R, R] (power of two, 16..512, with one spare
 * node on each side), zero-padded to 2 mesh_yz; splitting parameter
 * alpha = alpha_h / h (h the larger spacing, 0 < alpha_h <= 2) and short-range
 * cutoff r_max = rmax_alpha / alpha (2 <= rmax_alpha <= 6).  Triangular-
 * shaped-cloud assignment and interpolation, image-summed Green's function
 * deconvolved by the squared TSC transfer (built in FP64), mesh and FFTs in
 * the form's precision (complex FP32 in the FP32 form, FP64 in the FP64
 * form), deterministic.  Must be called before depo_set_layout (it sizes the
 * workspace: about 40 B per mesh node in the FP32 form, 80 B in the FP64
 * form); needs a single-sample layout with L >= 3 r_max, and
 * selects P3M as the Coulomb solver (depo_set_kernel_config switches between
 * it, mode DEPO_PAIR_P3M, and the direct modes).  The adjoint rejects P3M.
 * DEPO_E_STATE after the layout is set, DEPO_E_INVALID for bad sizes. */
depo_status depo_set_p3m(depo_ctx *ctx, int32_t mesh_x, int32_t mesh_yz, double alpha_h, double rmax_alpha);

/* Recompute the non-drag acceleration of every alive particle at the
 * current positions and velocities (the force evaluation of a step without
 * moving anything), and the fluid velocity at each particle.  Async. */
depo_status depo_eval_accel(depo_ctx *ctx, depo_stream stream);

/* Copy the particle state to the host, converted to SI doubles: positions
 * [N][3] (x in [0, L)), velocities [N][3], non-drag accelerations [N][3],
 * the step at which each particle deposited (0 = suspended) and the number
 * of short-range neighbours of each particle found at the last force
 * evaluation.  Any pointer may be NULL.  Synchronises the stream. */
depo_status depo_read_particles(depo_ctx *ctx, double *h_x3, double *h_v3, double *h_a3,
                                int32_t *h_dep_step, int32_t *h_neighbours, depo_stream stream);

/* Per-sample tallies out[n_samples] (Eq. 2).  Reduces on the device in a
 * fixed order (bitwise reproducible) and synchronises the stream. */
depo_status depo_tally_read(depo_ctx *ctx, depo_tally *out, depo_stream stream);

/* Checkpoint blob size for the current layout and precision.  Host only. */
depo_status depo_state_bytes(const depo_ctx *ctx, size_t *bytes);

/* Write the full particle state and step counter into h_blob (exactly
 * depo_state_bytes() bytes, with a CRC32).  Synchronises the stream. */
depo_status depo_state_download(depo_ctx *ctx, void *h_blob, size_t bytes, depo_stream stream);

/* Restore a blob written by depo_state_download for the same layout and
 * precision; DEPO_E_CORRUPT on a size, format or CRC mismatch (nothing is
 * changed then).  Synchronises the stream. */
depo_status depo_state_upload(depo_ctx *ctx, const void *h_blob, size_t bytes, depo_stream stream);

/* Device bytes needed by depo_adjoint for n_steps and a checkpoint interval
 * (1 <= ckpt_every <= n_steps): ceil(n_steps / ckpt_every) stored states, the
 * ckpt_every - 1 per-step states of one segment (its last state is the next
 * checkpoint), the final state, the adjoint arrays and, with Coulomb on, the
 * raw pair sums (3 reals per particle) of the n_steps - ceil(n_steps /
 * ckpt_every) steps the reverse sweep recomputes, so that it does not rerun
 * the O(N^2) pair kernel.  Host only. */
depo_status depo_adjoint_workspace_bytes(const depo_ctx *ctx, int32_t n_steps, int32_t ckpt_every, size_t *bytes);

/* Gradient of J = sum_s w_s J_s, J_s = sum_{i in s} m_i (1 - exp(-l_i)) the
 * smoothed deposited mass after n_steps, with respect to each sample's
 * (charge_scale, hamaker, temperature) — the uncertain inputs of Sections 2.1
 * and 4.4.  Hand-written reverse mode of the whole step (drag, gather, Coulomb
 * pair sums, contact and cohesion, wall terms, smoothed tally) with
 * checkpoints every ckpt_every steps and recomputation of each segment.
 * Requires DEPO_SOFT_TALLY and a freshly seeded context (step 0): runs the
 * n_steps forward (the context ends at step n_steps, exactly as after
 * depo_step(n_steps)) and then the reverse sweep, including the dependence of
 * the seeded acceleration on the parameters.  h_weights[S] = w_s;
 * h_grad[S][3] receives dJ/d(charge_scale, hamaker, temperature); the
 * temperature column is exactly 0 (it enters only the rebound law, which the
 * smoothed tally turns off).  d_adj_work: caller-owned device memory of
 * depo_adjoint_workspace_bytes() bytes, 256-byte aligned.  Synchronises the
 * stream.  Pair adjoint: in FP32 with the symmetric pair mode, each unordered
 * pair is evaluated once and items are combined with FP64 atomic additions, so
 * repeated calls agree to the rounding of those additions (not bitwise); every
 * other configuration is bitwise reproducible.  DEPO_E_INVALID in the P3M mode. */
depo_status depo_adjoint(depo_ctx *ctx, int32_t n_steps, int32_t ckpt_every, const double *h_weights,
                         double *h_grad, void *d_adj_work, size_t bytes, depo_stream stream);

/* depo_adjoint in two halves, for callers that need J before they know the weights (an autograd
 * function: J in its forward pass, the weights = incoming gradient in its backward pass).
 *
 * depo_adjoint_forward: the forward run of depo_adjoint (same preconditions and errors, except the
 * weights): n_steps steps from the seeded state, storing checkpoints and the Coulomb tape in
 * d_adj_work (caller-owned, depo_adjoint_workspace_bytes() bytes, 256-byte aligned, kept alive and
 * unchanged until the backward call).  The context ends at step n_steps exactly as after
 * depo_step(n_steps), so the tally can be read; it records one pending reverse sweep.
 * Synchronises the stream.
 *
 * depo_adjoint_backward: the reverse sweep of the pending forward run for weights h_weights[S]
 * (finite), h_grad[S][3] as for depo_adjoint; the context is back at the forward's final state
 * afterwards.  Consumes the pending sweep.  DEPO_E_STATE when there is none, or when any call that
 * changes the state, the parameters, the field or the kernel configuration (seed, step, restore,
 * eval, set_*, bind, init_field, another adjoint forward) came in between.  Synchronises. */
depo_status depo_adjoint_forward(depo_ctx *ctx, int32_t n_steps, int32_t ckpt_every, void *d_adj_work,
                                 size_t bytes, depo_stream stream);
depo_status depo_adjoint_backward(depo_ctx *ctx, const double *h_weights, double *h_grad, depo_stream stream);

/* depo_adjoint without any device allocation, for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, results and errors as depo_adjoint,
 * but the adjoint workspace is a static device array of the library, 64 MiB on each GPU it runs on
 * (held until the process ends), instead of caller memory; the forward steps are launched directly
 * (results equal the captured graph's bitwise).  DEPO_E_CAPACITY, with nothing run, when
 * depo_adjoint_workspace_bytes() exceeds 64 MiB.  Calls no hipMalloc or hipFree.  Every call on one
 * GPU shares that GPU's array (it keeps the last call's contents, none of which a call reads before
 * writing): calls that overlap on one GPU, from several contexts or threads, race.  Synchronises. */
depo_status depo_adjoint_noalloc(depo_ctx *ctx, int32_t n_steps, int32_t ckpt_every, const double *h_weights,
                                 double *h_grad, depo_stream stream);

/* Low-fidelity model: the one-dimensional Eulerian deposition model of
 * Appendix B (particle momentum equation with turbophoresis, image-charge and
 * wall-cohesion forces, Eq. mom_modified with implicit drag; constant-flux
 * equation, Eq. continuity, with a kinetic wall condition) for n particle
 * classes, one V_dep+ per class, in FP64.  The paper leaves the closures to
 * other publications; this model uses stated substitutes: tau_1+ = tau_p+,
 * V'_fy+ = 0.005 y+^2 / (1 + 0.002923 y+^2.128), Rr = 1/(1 + tau_p+/10),
 * eps/nu = 10 Rr V'_fy+^2, Stokes-Einstein D_B at 293 K, wall velocity
 * variance Rr V'_fy+^2 + k_B T/(m u*^2), half-Maxwellian wall flux.
 *
 * p: only R, nu, rho_f, rho_p, re_tau and eps0 are used (each finite and
 *   positive, else DEPO_E_INVALID); no context is needed.
 * d_diam, d_charge, d_hamaker: DEVICE arrays of n doubles (diameter [m],
 *   charge [C], Hamaker constant [J]) per class; d_vdep_plus: DEVICE array of
 *   n doubles, written.  All caller-owned.  A class with a non-positive or
 *   non-finite diameter or a non-finite charge or Hamaker constant gets NaN.
 * n_wall >= 2 nodes span the gap from 1e-12 m to one wall unit geometrically;
 *   n_core >= 1 more nodes reach the pipe centre uniformly.
 * n = 0 is a no-op.  Asynchronous on `stream` (does not synchronise).  Errors
 * are reported through the status only (there is no context for
 * depo_last_error). */
depo_status depo_lf_solve(const depo_params *p, int64_t n, const double *d_diam, const double *d_charge,
                          const double *d_hamaker, int32_t n_wall, int32_t n_core, double *d_vdep_plus,
                          depo_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* DEPO_H */
