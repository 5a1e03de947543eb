/*
 * alch_nb.h - C ABI of the MI355X alchemical short-range nonbonded library.
 *
 * The library evaluates the lambda-dependent potential U(x, lambda) of the
 * paper's lambda-dynamics method (Linear Basis Function section, eq. 4):
 *   U = U_solv + U_solu + (lambda-scaled solute-solvent interactions),
 * restricted to its short-range nonbonded part, together with the atomic
 * forces -dU/dx and the generalized force dU/dlambda that drives lambda and
 * whose conditional mean is integrated for the free energy (eq. 2).
 *
 * Pair potential (Angstrom, kcal/mol, e):
 *   every unordered, non-excluded pair i<j with minimum-image distance
 *   r < cutoff is evaluated once, with Lorentz-Berthelot combination.
 *   Pairs inside the solvent or inside the solute:  LJ(r) S(r) + k_e q q D(r).
 *   Solute-solvent pairs, ALCH_NB_BEUTLER_DSF (default):
 *       lv 4 eps (x^2 - x) S(r) + le k_e q q D(r),
 *       x = 1/(sc_alpha (1 - lv) + (r/sigma)^6), lv = min(1, 2 lambda),
 *       le = max(0, 2 lambda - 1)  (the conventional soft core the paper
 *       contrasts with LBF; Linear Basis Function section).
 *   Solute-solvent pairs, ALCH_NB_LBF_DSF (the paper's eq. 4-10):
 *       hA(lambda) [LJ S + k_e q q D] + hB(lambda) eps u_cap(r/sigma) S.
 *   S(r) = 1 - S22((r - r_s)/w) on (r_s = cutoff - w, cutoff) (eq. 9 as the
 *   switch; Simulation Details section); D(r) is the damped shifted-force
 *   Coulomb kernel erfc(a r)/r - erfc(a rc)/rc + [erfc(a rc)/rc^2 +
 *   2a/sqrt(pi) exp(-a^2 rc^2)/rc](r - rc), a = dsf_alpha, k_e = 332.06371.
 *   dU/dlambda uses the left derivative at the Beutler kink lambda = 1/2.
 *
 * Conventions
 *   - All functions return alch_nb_status (0 = OK).  No exception crosses
 *     the ABI.  alch_nb_strerror() names each code.
 *   - "host" pointers are read during the call only; "device" pointers must
 *     point to device memory that stays valid until the bound stream has
 *     executed the enqueued work.  The library never allocates device
 *     memory: alch_nb_workspace_size() reports the bytes it needs and the
 *     caller hands a buffer of that size to alch_nb_bind().
 *   - Work is enqueued on the stream given to alch_nb_bind() (a hipStream_t
 *     passed as void*; NULL = the null stream) and the calls return without
 *     waiting.  Conditions detected on the device set sticky flag bits read
 *     with alch_nb_get_flags(), which synchronizes the stream.
 *   - One context is used by one host thread at a time.
 *   - Atom order: the concatenation of the systems passed to
 *     alch_nb_create(), each in its own order.  Positions and forces are
 *     float64 [N_total][3], row major.
 *   - Results are bit-identical from run to run for a fixed context,
 *     precision and variant (forces are summed in 64-bit fixed point).
 */
#ifndef ALCH_NB_H
#define ALCH_NB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t alch_nb_status;
enum {
  ALCH_NB_OK = 0,
  ALCH_NB_E_INVALID_ARG = 1,   /* a pointer, size, index or parameter is invalid */
  ALCH_NB_E_BOX_TOO_SMALL = 2, /* cutoff + skin exceeds half the shortest box edge */
  ALCH_NB_E_UNSUPPORTED = 3,   /* valid request that the library does not implement */
  ALCH_NB_E_CAPACITY = 4,      /* the neighbour list outgrew its workspace */
  ALCH_NB_E_HIP = 5,           /* a HIP runtime call failed (see alch_nb_last_hip_error) */
  ALCH_NB_E_NOT_BOUND = 6,     /* the context has no workspace/stream yet */
  ALCH_NB_E_NO_DEVICE = 7,     /* no usable GPU */
  ALCH_NB_E_SCRATCH_SIZE = 8   /* the workspace exceeds the library's static device scratch */
};

enum { ALCH_NB_BEUTLER_DSF = 0, ALCH_NB_LBF_DSF = 1 };     /* schedule */
enum { ALCH_NB_FP32_FIXED = 0, ALCH_NB_FP64 = 1 };         /* precision */

/* alch_nb_compute() flags */
enum { ALCH_NB_AUTO_REBUILD = 1u, ALCH_NB_FORCE_REBUILD = 2u };

/* sticky device flags */
enum {
  ALCH_NB_FLAG_FIXED_OVERFLOW = 1u, /* a force left the fixed-point range */
  ALCH_NB_FLAG_SKIN_EXCEEDED = 2u,  /* an atom moved > skin/2 since the list was built (no auto rebuild) */
  ALCH_NB_FLAG_NONFINITE = 4u,      /* a position was NaN or infinite */
  ALCH_NB_FLAG_LAMBDA_RANGE = 8u,   /* a lambda outside [0,1] was clamped */
  ALCH_NB_FLAG_CAPACITY = 16u,      /* the list did not fit its capacity; results of that call are invalid */
  ALCH_NB_FLAG_BARRIER_TIMEOUT = 32u,/* a list-build phase waited too long for the others; results invalid */
  ALCH_NB_FLAG_BAD_INDEX = 64u,      /* alch_nb_dihedrals or alch_nb_ld_step_dafed met an atom index outside [0, N); that CV was skipped */
  ALCH_NB_FLAG_LD_CAPACITY = 128u    /* alch_nb_ld_step(_dafed) could not store an OPES kernel (capacity); it was dropped */
};

/* energy-term slots of alch_nb_out.terms, per system */
enum {
  ALCH_NB_T_SOLV_SOLV = 0, /* solvent-solvent pair energy */
  ALCH_NB_T_SOLU_SOLU = 1, /* solute-solute (non-excluded) pair energy */
  ALCH_NB_T_SS_VDW = 2,    /* lambda-scaled solute-solvent van der Waals energy */
  ALCH_NB_T_SS_ELEC = 3,   /* lambda-scaled solute-solvent electrostatic energy */
  ALCH_NB_T_UA = 4,        /* LBF basis U_solu-solv (0 for Beutler) */
  ALCH_NB_T_UB = 5,        /* LBF basis U_softLJ (0 for Beutler) */
  ALCH_NB_T_DUDL_VDW = 6,  /* van der Waals part of dU/dlambda */
  ALCH_NB_T_DUDL_ELEC = 7, /* electrostatic part of dU/dlambda */
  ALCH_NB_T_TOTAL = 8,     /* total energy */
  ALCH_NB_T_DUDL = 9,      /* dU/dlambda */
  ALCH_NB_NTERMS = 10
};

typedef struct alch_nb_ctx alch_nb_ctx;

/* One periodic orthorhombic box (one replica).  All pointers are host. */
typedef struct {
  int32_t n_atoms;            /* >= 0 */
  const int32_t *type;        /* [n_atoms] in [0, n_types) */
  const uint8_t *is_solute;   /* [n_atoms] 1 = alchemically coupled group, 0 = environment */
  int32_t n_excl;             /* >= 0 */
  const int32_t *excl;        /* [n_excl][2] local indices, i < j, sorted by (i, j), no duplicates */
  double box[3];              /* edge lengths, Angstrom */
} alch_nb_system;

/* Parameters shared by all systems.  Pointers are host. */
typedef struct {
  int32_t n_types;
  const double *sigma;        /* [n_types] > 0, Angstrom */
  const double *epsilon;      /* [n_types] >= 0, kcal/mol */
  const double *charge;       /* [n_types] e */
  double cutoff;              /* r_c > 0 */
  double skin;                /* list buffer >= 0; cutoff + skin <= min(box)/2 */
  double switch_width;        /* LJ switch width in [0, cutoff); 0 = hard truncation */
  double dsf_alpha;           /* DSF damping a >= 0; FP32 path needs a * cutoff <= 4 */
  double sc_alpha;            /* Beutler soft-core alpha >= 0 (0.5) */
  int32_t schedule;           /* ALCH_NB_BEUTLER_DSF | ALCH_NB_LBF_DSF */
  int32_t precision;          /* ALCH_NB_FP32_FIXED | ALCH_NB_FP64 */
  int32_t variant;            /* launch variant index, -1 = default (see alch_nb_autotune) */
  double list_capacity_factor;/* scales the neighbour-list capacity estimate; <= 0 means 1 */
  /* Long-range electrostatics (appended; zero-initialised callers get DSF).
   * ALCH_NB_ELEC_PME: Ewald electrostatics by smooth particle-mesh Ewald,
   * as the paper's simulations use (Simulation Details): dsf_alpha is then
   * the Ewald splitting parameter a > 0, D(r) becomes erfc(a r)/r truncated
   * at the cutoff, and the reciprocal-space, self, excluded-pair and
   * neutralising-background parts are added per box, the solute-solvent
   * part of each scaled like the solute-solvent Coulomb pairs (see
   * alch_nb_compute). */
  int32_t electrostatics;     /* ALCH_NB_ELEC_DSF (0) | ALCH_NB_ELEC_PME */
  int32_t pme_order;          /* B-spline interpolation order, 4..6 (PME) */
  double pme_spacing;         /* largest grid spacing, Angstrom (PME): each box edge L gets the
                                 smallest n >= max(L / pme_spacing, 2 pme_order) of the form
                                 2^a 3^b 5^c; n > 512 gives ALCH_NB_E_UNSUPPORTED */
} alch_nb_params;

enum { ALCH_NB_ELEC_DSF = 0, ALCH_NB_ELEC_PME = 1 };  /* electrostatics */

/* Outputs of alch_nb_compute().  Device pointers; any may be NULL. */
typedef struct {
  double *terms;              /* [K][ALCH_NB_NTERMS] */
  double *forces;             /* [N_total][3]  -dU/dx, float64 for both precisions */
  double *dudl;               /* [K] dU/dlambda */
  int64_t *n_pairs;           /* [K] pairs with r < cutoff that were evaluated */
} alch_nb_out;

/* Gradients written by alch_nb_backward().  Device pointers; NULL skips. */
typedef struct {
  double *d_pos;              /* [N_total][3] accumulated: += g_k * dU_k/dx */
  double *d_lambda;           /* [K] written: g_k * dU_k/dlambda */
  double *d_sigma;            /* [n_types] written: sum_k g_k dU_k/dsigma_t */
  double *d_sqrt_epsilon;     /* [n_types] written: sum_k g_k dU_k/dsqrt(eps_t) (finite for every type) */
  double *d_charge;           /* [n_types] written: sum_k g_k dU_k/dq_t */
  double *d_epsilon;          /* [n_types] written: sum_k g_k dU_k/deps_t = d_sqrt_epsilon / (2 sqrt(eps_t));
                                 NaN where eps_t = 0 (the combination sqrt(eps_i eps_j) has no
                                 derivative there) */
} alch_nb_grad;

typedef struct {
  int64_t n_atoms, n_systems;
  int64_t n_superclusters, n_entries, n_units;   /* current list (valid after a sync) */
  int64_t entry_capacity, unit_capacity;
  int64_t n_rebuilds;                            /* list builds since bind */
  int64_t n_tiles;                               /* 64-pair tiles of the current list */
  int32_t variant;                               /* variant in use */
  int32_t entries_per_unit, blocks;              /* launch shape of the tile kernel */
  double tile_ms_total;                          /* summed tile-kernel time of timed calls */
  int64_t tile_launches_timed;
} alch_nb_stats;

/* Create a context for n_systems boxes (host-only work: validation and
 * planning; no HIP call).  *out receives the context or NULL on error. */
alch_nb_status alch_nb_create(const alch_nb_params *params, const alch_nb_system *systems, int32_t n_systems,
                              alch_nb_ctx **out);

/* PME grid of box k (ALCH_NB_ELEC_PME): dims[3] = grid points along x, y, z.
 * ALCH_NB_E_UNSUPPORTED for a DSF context. */
alch_nb_status alch_nb_pme_grid(const alch_nb_ctx *ctx, int32_t k, int32_t dims[3]);

/* Bytes of device workspace the context needs. */
alch_nb_status alch_nb_workspace_size(const alch_nb_ctx *ctx, size_t *bytes);

/* Bind a device workspace (>= workspace_size bytes, 256-byte aligned) and a
 * stream; uploads the static tables.  Rebinding is allowed. */
alch_nb_status alch_nb_bind(alch_nb_ctx *ctx, void *d_workspace, size_t bytes, void *stream);

/* Bind without allocating: for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Binds the context, on the current device, to a device array
 * the library owns (ALCH_NB_STATIC_SCRATCH_BYTES on each GPU it runs on,
 * held until the process ends) in place of a caller workspace, with the
 * stream as in alch_nb_bind(); calls no allocating routine.  The context is
 * then used as with alch_nb_bind().  Returns ALCH_NB_E_SCRATCH_SIZE when
 * alch_nb_workspace_size() exceeds the array (nothing is bound then).
 * One array per device serves one context at a time: binding takes it over
 * from the previous owner, whose later calls return ALCH_NB_E_NOT_BOUND, and
 * clears it.  Work of two contexts on one device that overlaps in time
 * races on the array: the previous owner's enqueued work must have finished
 * before another context is bound.  alch_nb_bind() or alch_nb_destroy()
 * releases the array. */
#define ALCH_NB_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
alch_nb_status alch_nb_bind_static(alch_nb_ctx *ctx, void *stream);

/* Build the neighbour list from device positions d_pos [N_total][3]:
 * every non-excluded pair i < j of a box whose minimum-image distance is
 * below cutoff + skin (canonical FP64 test: positions wrapped into the box,
 * displacement shifted by -+L beyond +-L/2, r^2 = (dx^2 + dy^2) + dz^2 without
 * fused multiply-adds), grouped into 8-atom clusters of 64-slot
 * super-clusters.  The list serves every later call until a rebuild.  It is
 * the pair set over which eq. 4's sums run, restricted to the short range
 * (the paper truncates nonbonded terms at a cutoff: Simulation Details).
 * A list larger than its capacity raises ALCH_NB_FLAG_CAPACITY (read with
 * alch_nb_get_flags) and later evaluations compute nothing until a larger
 * context is created. */
alch_nb_status alch_nb_build_list(alch_nb_ctx *ctx, const double *d_pos);

/* Evaluate energies, forces and dU/dlambda at device positions d_pos
 * [N_total][3] and device lambdas d_lambda [K] (lambda in [0, 1]; values
 * outside are clamped and raise ALCH_NB_FLAG_LAMBDA_RANGE).  This is the
 * potential U(x, lambda) of eq. 4 (the LBF schedule: U_solv + U_solu +
 * hA U_solu-solv + hB U_softLJ with eqs. 5-10; the Beutler schedule: the
 * conventional soft core in place of the last two terms), the forces
 * -dU/dx, and the generalized force dU/dlambda whose conditional mean eq. 2
 * integrates (LBF: hA' U_A + hB' U_B; Beutler: the left derivative at
 * lambda = 1/2).  With ALCH_NB_AUTO_REBUILD the list is rebuilt on the
 * device when an atom moved more than skin/2 since the last build (always
 * when skin = 0); ALCH_NB_FORCE_REBUILD rebuilds unconditionally.  Outputs
 * are written in full (forces in atom order; terms per box as listed under
 * ALCH_NB_T_*); any output pointer may be NULL.
 * With ALCH_NB_ELEC_PME the Coulomb energy is an Ewald sum (long-range
 * electrostatics by PME: Simulation Details; smooth PME of Essmann et al.
 * 1995): the short-range pairs use erfc(a r)/r, and per box the smooth-PME
 * reciprocal energy of two charge grids (solute S, solvent W; order-n
 * cardinal B-splines, FP64 complex FFTs, 64-bit fixed-point charge spreading
 * so that results stay bit-identical), the self part -k_e a/sqrt(pi) sum
 * q^2, the excluded pairs' -k_e q q erf(a r)/r and the background part
 * -k_e pi Q^2/(2 V a^2) are split into S-S, W-W and S-W parts.  S-S and
 * W-W join E_solu_solu and E_solv_solv; the S-W part X is scaled like the
 * solute-solvent Coulomb pairs (Beutler: le X in E_ss_elec, dle/dlambda X
 * in dU/dlambda; LBF: X joins U_A, hA X E_ss_elec, hA' X dU/dlambda), and
 * the forces are those of that energy. */
alch_nb_status alch_nb_compute(alch_nb_ctx *ctx, const double *d_pos, const double *d_lambda, uint32_t flags,
                               const alch_nb_out *out);

/* Gradients of L = sum_k g_k E_total,k for upstream device weights
 * d_grad_energy [K] (the reverse pass of eq. 4's potential: dU/dx and
 * dU/dlambda as in alch_nb_compute; the per-type derivatives of every pair
 * term of eqs. 4-10 through the combination rules sigma_ij = (sigma_i +
 * sigma_j)/2, eps_ij = sqrt(eps_i eps_j), q_i q_j), at the same
 * positions/lambdas as the last compute:
 * every gradient comes from that compute's state (forces, dU/dlambda, the
 * list and the slot coordinates it wrote), so d_pos and d_lambda must be the
 * inputs of that call.  The parameter gradients are per-atom 64-bit
 * fixed-point sums (the forces' scale; a value beyond 2^62 units raises
 * ALCH_NB_FLAG_FIXED_OVERFLOW) added per type in a fixed order, so repeated
 * calls give identical results.  They need n_types <= 256 and DSF
 * electrostatics (ALCH_NB_E_UNSUPPORTED otherwise; with PME the position
 * and lambda gradients are available, the per-type ones are not). */
alch_nb_status alch_nb_backward(alch_nb_ctx *ctx, const double *d_pos, const double *d_lambda,
                                const double *d_grad_energy, const alch_nb_grad *grad);

/* Dihedral collective variables xi_c in (-pi, pi] (atom quadruples d_idx
 * [n_cv][4], global indices; bond vectors by minimum image in the box of
 * the second atom; an index outside [0, N) skips that CV and raises
 * ALCH_NB_FLAG_BAD_INDEX) with their Cartesian gradients d_dxi [n_cv][4][3], and,
 * when d_mass_inv [N_total] is given, the sum_i m_i^-1 |dxi/dr_i|^2 of the
 * paper's eq. 16 into d_msum [n_cv].  With d_s and d_kappa [n_cv] the
 * d-AFED coupling (eq. 15) energy goes to d_u_dafed [1] and its force is
 * added to d_forces [N_total][3].  All device pointers; optional ones may be
 * NULL. */
alch_nb_status alch_nb_dihedrals(alch_nb_ctx *ctx, const double *d_pos, int32_t n_cv, const int32_t *d_idx,
                                 double *d_xi, double *d_dxi, const double *d_mass_inv, double *d_msum,
                                 const double *d_s, const double *d_kappa, double *d_u_dafed, double *d_forces);

/* Lambda/OPES for one box: the paper's mirror-periodic theta (eq. 3) and
 * the dual OPES bias U = U_Standard + U_Explore (eqs. 11-14) on theta, with
 * uncompressed Gaussian kernels of width sigma on the periodic [0, 2) line.
 * The state is one device array of alch_nb_opes_state_size(capacity)
 * doubles (layout from alch_nb_opes_layout(): header slots theta, lambda,
 * dlambda/dtheta, U_OPES, dU_OPES/dtheta, F_theta, kT, sigma, the two
 * barriers, kernel count, capacity and running sums; then the bias and its
 * derivative on 101 output grid nodes theta_g = 2g/101; then the kernel
 * centres and their Standard weights).  The caller may write theta (slot 0)
 * between calls, e.g. from an integrator.
 * alch_nb_opes_init: zeroes the state and sets the constants (kcal/mol).
 * alch_nb_opes_update: optionally deposits a kernel at the current theta
 * (Standard weight exp(U_total/kT), Explore weight 1; no deposit once the
 * capacity is reached), then writes lambda (eq. 3) to d_lambda_out [1], the
 * bias and F_theta = -(dlambda/dtheta) dU/dlambda - dU_OPES/dtheta with
 * dU/dlambda read from d_dudl [1] (NULL = 0).  The grid is refreshed on
 * deposition (a second launch, one block per node).  Device pointers;
 * FP64; the update itself is one thread block. */
#define ALCH_NB_OPES_GRID 101
#define ALCH_NB_OPES_HEADER 16
int64_t alch_nb_opes_state_size(int32_t capacity);
alch_nb_status alch_nb_opes_init(alch_nb_ctx *ctx, double *d_state, int32_t capacity, double kT, double sigma,
                                 double barrier_std, double barrier_expl, double theta0);
alch_nb_status alch_nb_opes_update(alch_nb_ctx *ctx, double *d_state, const double *d_dudl, double *d_lambda_out,
                                   int32_t deposit);
/* Offsets of the state sections (host query, no HIP call); n >= 18. */
alch_nb_status alch_nb_opes_layout(int32_t *offsets, int32_t n);

/* Lambda dynamics with dual OPES and TI, and d-AFED extended dynamics
 * (device, FP64), for the K boxes of the context.  The paper's extended
 * Hamiltonian gives lambda (through the periodic theta of eq. 3) and the
 * d-AFED variables s_k masses and thermostats of their own; OPES
 * (eqs. 11-14) biases theta with kernels deposited every `stride` steps and
 * compressed; dU/dlambda is binned along lambda for the free energy
 * (eq. 2); s_k couples to the dihedral xi_k through eq. 15.  Integration:
 * Langevin BAOAB (the paper names a regulated Nose-Hoover-Langevin
 * thermostat without giving it), one step per call, the normal deviates
 * taken from the caller's array.  Kernel compression: a new kernel within
 * `compress` widths of the nearest centre is merged into it (weight, mean
 * and variance conserved); rho_bar is the mean of rho_hat over the kernel
 * centres.  Units: kcal/mol, fs, radians.
 * alch_nb_ld_state_size: doubles of state for n_replicas (= K) boxes (-1 on
 *   invalid parameters).
 * alch_nb_ld_layout: offsets (doubles) into the state: [0] first replica
 *   record, [1] record stride, [2] theta, [3] p_theta, [4] lambda (next),
 *   [5] lambda (last step), [6] U_OPES, [7] dU_OPES/dtheta, [8] F_theta,
 *   [9] steps done, [10] Standard kernel count, [11] Explore kernel count,
 *   [12] Standard kernels (centres, weights, widths: capacity each),
 *   [13] Explore kernels, [14] TI sums then counts (ti_bins each), all
 *   within a record; [15] auxiliary section: s [n_cv] (for
 *   alch_nb_dihedrals' d_s), [16] p_s, [17] last force on s; n >= 18.
 * alch_nb_ld_init: clears d_state and sets theta0 [K] (device), and for
 *   d-AFED s0, mass_s, kappa [n_cv] (device; NULL when n_cv = 0).
 * alch_nb_ld_step: one step from d_dudl [K] (dU/dlambda at the current
 *   lambda, e.g. alch_nb_out.dudl) and d_xi [n_cv] (the CVs at the current
 *   positions; NULL when n_cv = 0), with the normal deviates of row
 *   (step mod noise_rows) of d_noise [noise_rows][K + n_cv]; writes the
 *   next lambda to d_lambda_out [K] (may be the array the next
 *   alch_nb_compute reads).  A full kernel store raises
 *   ALCH_NB_FLAG_LD_CAPACITY.
 * alch_nb_ld_free_energy: Delta G per box by the midpoint rule over the
 *   lambda bins (NaN while a bin has no sample) into d_out [K].
 * All device pointers; work on the bound stream; FP64. */
typedef struct {
  int32_t capacity;           /* OPES kernels per variant and box (>= 1) */
  int32_t stride;             /* deposition every stride steps (<= 0: no OPES) */
  int32_t ti_bins;            /* lambda bins in [0, 1] (>= 1) */
  int32_t n_cv;               /* d-AFED variables (0: lambda dynamics only) */
  double kT;                  /* k_B T of theta, kcal/mol */
  double mass;                /* theta mass, kcal/mol fs^2 (1 Da nm^2 = 239005.7) */
  double friction;            /* theta friction, 1/fs */
  double dt;                  /* time step, fs */
  double sigma;               /* OPES kernel width on theta */
  double barrier_std, barrier_expl; /* OPES barriers, kcal/mol (> kT) */
  double compress;            /* merge threshold in kernel widths (0: no merging) */
  double kT_s;                /* k_B T of the auxiliary variables, kcal/mol */
  double friction_s;          /* their friction, 1/fs */
} alch_nb_ld_params;
int64_t alch_nb_ld_state_size(const alch_nb_ld_params *params, int32_t n_replicas);
alch_nb_status alch_nb_ld_layout(const alch_nb_ld_params *params, int32_t n_replicas, int64_t *offsets, int32_t n);
alch_nb_status alch_nb_ld_init(alch_nb_ctx *ctx, const alch_nb_ld_params *params, double *d_state,
                               const double *d_theta0, const double *d_s0, const double *d_mass_s,
                               const double *d_kappa);
alch_nb_status alch_nb_ld_step(alch_nb_ctx *ctx, double *d_state, const double *d_dudl, const double *d_xi,
                               const double *d_noise, int32_t noise_rows, double *d_lambda_out);
alch_nb_status alch_nb_ld_free_energy(alch_nb_ctx *ctx, const double *d_state, double *d_out);

/* alch_nb_ld_step with the d-AFED coupling (eq. 15) evaluated in the same
 * launch: the state's n_cv > 0 dihedral CVs of d_idx [n_cv][4] (n_cv of
 * the state, global atom indices) at d_pos
 * (as alch_nb_dihedrals, with s and kappa read from the state), their
 * coupling energy into d_u_dafed [1] and force added to d_forces
 * [N_total][3], the CV values into d_xi [n_cv] (those three may be NULL),
 * then the step.  With valid indices the results are identical, bit for
 * bit, to alch_nb_dihedrals(d_s = the state's s, d_kappa = the state's
 * kappa) followed by alch_nb_ld_step; a CV with an index outside [0, N)
 * raises ALCH_NB_FLAG_BAD_INDEX, exerts no force and leaves its outputs
 * unwritten.  ALCH_NB_E_INVALID_ARG for a state without auxiliary
 * variables.  Device pointers; work on the bound stream. */
alch_nb_status alch_nb_ld_step_dafed(alch_nb_ctx *ctx, double *d_state, const double *d_dudl, const double *d_pos,
                                     const int32_t *d_idx, double *d_xi, double *d_u_dafed, double *d_forces,
                                     const double *d_noise, int32_t noise_rows, double *d_lambda_out);

/* Replica exchange between lambda states (LBF schedule only; the paper's
 * HREX reference protocol, Simulation Details): box r holds state
 * d_state_of[r] of the ascending d_lambda_states [K]; with the LBF potential
 * linear in its bases (eq. 4) the basis energies U_A, U_B of each box (the
 * terms of the last alch_nb_compute, d_terms [K][ALCH_NB_NTERMS]) give every
 * neighbour swap's D = [U_a(l_s+1) - U_a(l_s) + U_b(l_s) - U_b(l_s+1)]/kT;
 * the swap is accepted when D <= 0 or u < exp(-D).  Attempt n (counted in
 * d_stats[0]) pairs the states (s, s+1) with s of parity n mod 2 and takes
 * pair s's uniform deviate from row (n mod rows) of d_uniform [rows][K-1];
 * d_lambda [K] is rewritten with each box's new state's lambda (it may be
 * the array the next alch_nb_compute reads).  d_stats [2K-1] int64:
 * attempts so far, then attempts and accepts per pair (K-1 each).
 * alch_nb_hrex_init sets d_state_of to the identity and clears d_stats.
 * ALCH_NB_E_UNSUPPORTED for the Beutler schedule (its cross-state energies
 * need evaluations at the other lambdas) or K outside [2, 4096].  Device
 * pointers; work on the bound stream. */
alch_nb_status alch_nb_hrex_init(alch_nb_ctx *ctx, int32_t *d_state_of, int64_t *d_stats);
alch_nb_status alch_nb_hrex_exchange(alch_nb_ctx *ctx, const double *d_terms, const double *d_lambda_states,
                                     int32_t *d_state_of, double *d_lambda, const double *d_uniform, int32_t rows,
                                     double kT, int64_t *d_stats);

/* Record every call made between alch_nb_capture_begin() and
 * alch_nb_capture_end() on the bound stream (e.g. alch_nb_compute,
 * alch_nb_dihedrals, alch_nb_ld_step, alch_nb_ld_step_dafed,
 * alch_nb_hrex_exchange) as one HIP graph, replayed with
 * alch_nb_launch_step(); the pointers are captured.
 * Calls that synchronize (flags, statistics, pair export) are not allowed
 * in between. */
alch_nb_status alch_nb_capture_begin(alch_nb_ctx *ctx);
alch_nb_status alch_nb_capture_end(alch_nb_ctx *ctx);

/* Write the current list's pair set (i<j global indices, canonical FP64
 * test r^2 < (cutoff + skin)^2 at build time) to d_pairs [cap][2] in
 * unspecified order and its size to the host *n_out; syncs the stream.
 * Returns ALCH_NB_E_CAPACITY if cap is too small (*n_out still set). */
alch_nb_status alch_nb_export_pairs(alch_nb_ctx *ctx, int32_t *d_pairs, int64_t cap, int64_t *n_out);

/* Record one alch_nb_compute() with AUTO_REBUILD into a HIP graph and
 * replay it with alch_nb_launch_step().  The pointers are captured. */
alch_nb_status alch_nb_capture_step(alch_nb_ctx *ctx, const double *d_pos, const double *d_lambda,
                                    const alch_nb_out *out);
alch_nb_status alch_nb_launch_step(alch_nb_ctx *ctx);

/* Time every launch variant on the current list and select the fastest;
 * results are cached in the JSON file named by $ALCHNB_TUNE_CACHE (if set). */
alch_nb_status alch_nb_autotune(alch_nb_ctx *ctx, const double *d_pos, const double *d_lambda, int32_t reps);
alch_nb_status alch_nb_set_variant(alch_nb_ctx *ctx, int32_t variant);
int32_t alch_nb_num_variants(void);

/* How the list is built on a rebuild.  ALCH_NB_LIST_AUTO (the default):
 * one launch whose phases meet at bounded grid barriers, when every block
 * fits on the device at once; otherwise one kernel per phase.
 * ALCH_NB_LIST_PHASES: always one kernel per phase.  A fused build whose
 * barrier wait gives up raises ALCH_NB_FLAG_BARRIER_TIMEOUT and that call's
 * results are invalid: switch to ALCH_NB_LIST_PHASES and evaluate again with
 * ALCH_NB_FORCE_REBUILD.  alch_nb_get_list_mode() reports what a rebuild
 * launches now (ALCH_NB_LIST_FUSED_ACTIVE or ALCH_NB_LIST_PHASES; -1 for a
 * NULL context).  Setting the mode drops a captured step. */
enum { ALCH_NB_LIST_AUTO = 0, ALCH_NB_LIST_PHASES = 1, ALCH_NB_LIST_FUSED_ACTIVE = 2 };
alch_nb_status alch_nb_set_list_mode(alch_nb_ctx *ctx, int32_t mode);
int32_t alch_nb_get_list_mode(const alch_nb_ctx *ctx);

/* Tile-kernel timing with HIP events on the bound stream.  every = 0: off;
 * every = n >= 1: from now on the tile launch of every n-th call is
 * bracketed by two events (each pair costs a few microseconds of stream
 * time, so a sample of the calls keeps a timed run close to an untimed
 * one).  The summed time and the count of timed launches are read with
 * alch_nb_get_stats.  ALCH_NB_E_INVALID_ARG for every < 0. */
alch_nb_status alch_nb_set_timing(alch_nb_ctx *ctx, int32_t every);

/* Read and clear the sticky flags (synchronizes the stream). */
alch_nb_status alch_nb_get_flags(alch_nb_ctx *ctx, uint32_t *flags);
/* Statistics (synchronizes the stream). */
alch_nb_status alch_nb_get_stats(alch_nb_ctx *ctx, alch_nb_stats *stats);

void alch_nb_destroy(alch_nb_ctx *ctx);
const char *alch_nb_strerror(alch_nb_status status);
int32_t alch_nb_last_hip_error(const alch_nb_ctx *ctx);
/* Algorithmic floating-point operations charged per evaluated pair, by
 * kind: 0 = plain pair (90: the work of its defining formulas, switched LJ
 * and shifted-force electrostatics with their forces, erfc evaluated
 * through an exponential), 1 = solute-solvent pair (120: the soft core and
 * dU/dlambda add 30).  Used for roofline reports; independent of how a
 * kernel computes the pair. */
double alch_nb_flops_per_pair(int32_t kind);

#ifdef __cplusplus
}
#endif
#endif /* ALCH_NB_H */
