/*
 * dda.h -- C ABI of the MI355X (gfx950) discrete-dipole-approximation solver.
 *
 * The library solves A P = E for the dipole polarizations P of a target made
 * of polarizable points on a cubic lattice (DDSCAT 7.1 User Guide, section
 * "Choice of Iterative Algorithm", eq. AP=E), with the off-diagonal part of A
 * applied as a convolution by FFT on a doubled grid, a complex-symmetric
 * BiCGstab solver, and the cross-section and scattering-amplitude reductions;
 * around them, the phase-lag and backscattering efficiencies and moments of
 * the scattered intensity, and orientational averaging (orientation samples
 * and weights, efficiencies at other rotations Phi from polarization pairs).
 *
 * Conventions shared by every call
 *  - Units: lattice spacing d = 1; incident amplitude |E0| = 1; Gaussian
 *    units; time dependence exp(-i omega t).  Wavenumbers are k d.
 *  - Complex numbers are interleaved (re, im) doubles unless stated.
 *  - Per-site vectors (P, E) cross the ABI as [nrhs][N][3] complex128:
 *    right-hand side slowest, then site, then Cartesian component, with the
 *    sites in the order of increasing linear box index ix + n1 (iy + n2 iz)
 *    of the occupancy grid passed to dda_set_target / dda_add_target.  When
 *    the right-hand sides of one call use different targets, their rows are
 *    concatenated in call order, each with its own target's N.
 *  - Pointers are host pointers unless the call's flags contain
 *    DDA_DEVICE_PTRS, in which case they are device pointers valid on the
 *    context's device, ordered on the context's stream.
 *  - Inputs are borrowed for the duration of the call only; outputs are
 *    written into caller-owned buffers.  The context owns all device memory
 *    it allocates and frees it in dda_destroy.
 *  - Return value: 0 on success, a negative dda_status on error (outputs
 *    unspecified, context still usable unless it is DDA_ERR_HIP), a positive
 *    value for warnings that come with valid outputs.  The text of the last
 *    error or warning is available from dda_last_error.  No C++ exception
 *    crosses the ABI.
 *  - A context is used by one host thread at a time.
 */
#ifndef DDA_H
#define DDA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dda_status;

enum {
    DDA_OK = 0,
    DDA_ERR_INVALID_ARG = -1,
    DDA_ERR_OOM = -2,
    DDA_ERR_HIP = -3,
    DDA_ERR_STATE = -4,            /* call out of order (e.g. solve before set_target) */
    DDA_ERR_UNSUPPORTED_DIMS = -5, /* box size the FFT cannot factor into 2, 3, 5 */
    DDA_ERR_NO_DEVICE = -6,
    DDA_ERR_IO = -7,
    DDA_WARN_NOT_CONVERGED = 1,    /* some right-hand side hit max_iter */
    DDA_WARN_MKD_GE_1 = 2          /* |m| k d >= 1: outside the validity range of the DDA */
};

/* Polarizability prescriptions (guide, section "Dipole Polarizabilities"). */
enum {
    DDA_ALPHA_CM = 0,     /* Clausius-Mossotti (3/4pi)(eps-1)/(eps+2), no radiative reaction */
    DDA_ALPHA_CM_RR = 1,  /* Clausius-Mossotti with radiative reaction -(2/3) i k^3 in 1/alpha */
    DDA_ALPHA_LDR = 2     /* lattice dispersion relation of Draine & Goodman 1993 (LATTDR) */
};

/* Arithmetic precision of a matvec or of the Green's-tensor spectrum. */
enum { DDA_FP64 = 1, DDA_FP32 = 2 };

/* Solve precision modes. */
enum {
    DDA_SOLVE_FP64 = 0,         /* FP64 vectors, FP64 matvec, FP64 residual check */
    DDA_SOLVE_FP32_REFINE = 1   /* FP32 inner BiCGstab on FP32 matvec, FP64 residual + refinement */
};

/* Initial guess. */
enum {
    DDA_GUESS_ZERO = 0,   /* P0 = 0 (the guide's default) */
    DDA_GUESS_USER = 1,   /* P0 from the p0 argument */
    DDA_GUESS_PREV = 2,   /* P0 = this context's previous solution in the same rhs slot */
    DDA_GUESS_NN = 3,     /* P0 = alpha (E_sh + net(features)), attached learned-guess network */
    DDA_GUESS_PREV_SHIFT = 4, /* P0 = alpha_new E_sh: the previous local field carried to the new
                                 incidence direction, E_sh,j = (1/alpha_prev) P_prev,j
                                 exp(i k (khat - khat_prev) . r_j) */
    DDA_GUESS_PROJECT = 5     /* P0 = sum_e c_e v_e over the slot's history of solutions (see
                                 dda_solve_opts.history; the previous solution alone while the
                                 history is empty), v_e each carried to the new direction as for
                                 PREV_SHIFT, c minimising ||E - A P0||_2 (one FP32 matvec per
                                 basis vector) */
};

/* Flags. */
enum {
    DDA_DEVICE_PTRS = 1u << 0,  /* vector arguments are device pointers */
    DDA_NO_GRAPH = 1u << 1,     /* run the Krylov loop eagerly instead of replaying a HIP graph */
    DDA_NO_FALLBACK = 1u << 2   /* keep a supplied guess even if its residual exceeds ||E|| */
};

typedef struct dda_ctx dda_ctx;

/* One incident wave, target-frame components (guide, section "Target
 * Orientation": the lab axis x_LF is the incidence direction). */
typedef struct {
    double khat[3];   /* unit propagation direction (|khat| = 1 within 1e-6, else DDA_ERR_INVALID_ARG) */
    double e0[6];     /* polarization vector, (re, im) x 3, khat . e0 = 0, |e0| = 1 within 1e-6
                         (else DDA_ERR_INVALID_ARG: the efficiencies are per unit |E0|^2) */
    int32_t target;   /* id returned by dda_set_target (0) or dda_add_target */
    int32_t pad_;
} dda_wave;

typedef struct {
    double tol;           /* stop when ||E - A P||_2 / ||E||_2 <= tol (FP64); 1e-5 if <= 0 */
    int32_t max_iter;     /* BiCGstab iterations per right-hand side (all inner steps); 1000 if <= 0 */
    int32_t guess;        /* DDA_GUESS_* */
    int32_t prec;         /* DDA_SOLVE_* */
    uint32_t flags;       /* DDA_DEVICE_PTRS | DDA_NO_GRAPH | DDA_NO_FALLBACK */
    int32_t graph_iters;  /* BiCGstab iterations per graph replay; 0 = autotuned/default */
    int32_t history;      /* 0..4: keep the solutions of the last `history` solves of every slot
                             (for DDA_GUESS_PROJECT and the learned guess); 0 clears them */
    int32_t restart_every; /* test hook: force the breakdown restart of the inner Krylov solver
                              (BiCGstab: rhat = p = r after every restart_every-th iteration;
                              BiCGstab(2): rt = r0 at the next cycle once the BiCG step count is a
                              multiple of it); 0 = never (normal operation), < 0 is
                              DDA_ERR_INVALID_ARG */
    int32_t solver;        /* DDA_SOLVER_*: inner Krylov method */
} dda_solve_opts;

/* Inner Krylov methods (guide, section "Choice of Iterative Algorithm"). */
enum {
    DDA_SOLVER_BICGSTAB = 0,  /* BiCGstab (van der Vorst 1992), fused into the matvec passes */
    DDA_SOLVER_BICGSTAB2 = 1  /* BiCGstab(2) (Sleijpen & Fokkema 1993), the guide's PBCGS2:
                                 cycles of two BiCG steps and a degree-2 minimal-residual step;
                                 iteration counts are BiCG steps (two matvecs each), convergence is
                                 checked at the end of a cycle */
};

typedef struct {
    int32_t iters;        /* BiCGstab iterations taken */
    int32_t matvecs;      /* FFT matvecs (FP32 and FP64) */
    int32_t outer;        /* FP64 residual checks (from a zero guess the first is E itself, no matvec) */
    int32_t status;       /* 0 converged, DDA_WARN_NOT_CONVERGED otherwise */
    double rel_resid;     /* final ||E - A P|| / ||E|| with the FP64 matvec */
    double guess_resid;   /* ||E - A P0|| / ||E|| of the guess actually used */
} dda_solve_stats;

/* Library version string. */
const char* dda_version(void);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * order all work on, or NULL to create a private stream.  */
dda_status dda_create(dda_ctx** out, int32_t device, void* hip_stream);
dda_status dda_destroy(dda_ctx* ctx);
const char* dda_last_error(const dda_ctx* ctx);

/*
 * Define the target (replacing all previous targets; it gets id 0).
 *   dims[3]   box size (n1, n2, n3); each must factor into 2, 3 and 5 and be >= 2
 *   occ       n1*n2*n3 bytes, x fastest: 0 = vacuum, c >= 1 = composition c
 *             (guide, section "Target Generation", FROM_FILE: occupied sites
 *             and their composition)
 *   ncomp     number of compositions (max occupancy value)
 *   m         2*ncomp doubles: complex refractive index per composition
 *   kd        k d (wavenumber times lattice spacing)
 *   alpha_kind DDA_ALPHA_*
 *   origin    3 doubles, target-frame origin in lattice units relative to
 *             site (0,0,0), or NULL for the centroid of the occupied sites
 * Returns DDA_WARN_MKD_GE_1 when |m| k d >= 1 for some composition (guide,
 * section "Applicability of the DDA").
 */
dda_status dda_set_target(dda_ctx* ctx, const int32_t dims[3], const uint8_t* occ, int32_t ncomp,
                          const double* m, double kd, int32_t alpha_kind, const double* origin);
/* Append another target for batched solves; *id_out receives its id. */
dda_status dda_add_target(dda_ctx* ctx, const int32_t dims[3], const uint8_t* occ, int32_t ncomp,
                          const double* m, double kd, int32_t alpha_kind, const double* origin,
                          int32_t* id_out);
/* Number of occupied sites N and the effective radius a_eff = (3N/4pi)^(1/3)
 * (guide, section "Applicability of the DDA") of a target. */
dda_status dda_target_info(const dda_ctx* ctx, int32_t target, int64_t* n_sites, double* aeff);

/*
 * Make composition `comp` (1..ncomp) of a target anisotropic (guide, section
 * "Composite Targets with Anisotropic Constituents"): a dielectric tensor that
 * is diagonal in its Dielectric Frame, with principal refractive indices
 * m3[0..2] ((re, im) x 3, eps_j = m_j^2) along the frame's axes e_1, e_2,
 * e_3, the frame rotated from the target frame by angles[] = {Theta_DF,
 * Phi_DF, beta_DF} (radians; e_j in target-frame components as the guide
 * expands them).  Each site of the composition then has the symmetric
 * polarizability tensor sum_j alpha_j e_j e_j^T, alpha_j from the target's
 * prescription with eps_j (LDR with the wave's S, taken in the target frame),
 * in the diagonal term of A and in the absorption sum
 * C_abs = 4 pi k sum_j [Im(P_j . (1/alpha_j)^* P_j^*) - (2/3) k^3 |P_j|^2].
 * The composition's isotropic m from dda_set_target is no longer used.
 * Anisotropic targets are solved without the matvec passes' fused inner
 * products; the guesses PREV_SHIFT, PROJECT and NN and
 * dda_cross_sections_phi are refused for them (DDA_ERR_INVALID_ARG), and
 * dda_matvec takes their tensors for the wave khat = x, e0 = y (its ainv
 * entries of these compositions are not used).  Clears the context's solve
 * state (groups, previous solutions).  Returns DDA_WARN_MKD_GE_1 when
 * max_j |m_j| k d >= 1; DDA_ERR_INVALID_ARG for an unknown target or
 * composition, null pointers or non-finite values.
 */
dda_status dda_set_anisotropic(dda_ctx* ctx, int32_t target, int32_t comp, const double* m3, const double* angles);

/* Build the FFT of the Green's tensor on the doubled grid for every target
 * whose spectrum is missing or stale.  Always computed in FP64; `prec` selects
 * which copies are kept for the matvec (DDA_FP32 | DDA_FP64). */
dda_status dda_build_green_fft(dda_ctx* ctx, uint32_t prec);

/*
 * Solve A P = E_inc for nrhs incident waves.  E_inc,j = e0 exp(i k khat . r_j)
 * is generated on the device.  p0 ([nrhs][N][3] complex128) is read only for
 * DDA_GUESS_USER.  p_out ([nrhs][N][3] complex128) receives P; it may be NULL
 * to keep the solution on the device only (for cross sections, amplitudes or
 * DDA_GUESS_PREV).  stats (nrhs entries) may be NULL.  The waves of one call
 * may reference different targets (batched multi-target solve).
 * DDA_GUESS_PREV, _PREV_SHIFT, _PROJECT and _NN need a previous solve with
 * the same nrhs whose slots hold the same targets (DDA_ERR_STATE otherwise);
 * the waves themselves may change (the next orientation or direction of a
 * sweep).  Redefining a target clears the history of its slots.
 * Returns DDA_WARN_NOT_CONVERGED if any right-hand side missed tol: max_iter
 * reached, 40 refinement steps, or an inner breakdown that ended non-finite
 * (its P is then the last finite iterate).  DDA_ERR_INVALID_ARG for a
 * non-finite incident field.
 *
 * Environment: DDA_TRACE=path appends, per solve call, one line per FP64
 * residual check ("rhs outer iteration rel_resid fp64") and per inner
 * BiCGstab iteration ("... inner", the inner recursive residual times the
 * FP64 relative residual it started from, an estimate of ||E - A P|| / ||E||)
 * to that text file; DDA_ERR_IO if it cannot be opened.
 */
dda_status dda_solve(dda_ctx* ctx, int32_t nrhs, const dda_wave* waves, const dda_solve_opts* opts,
                     const void* p0, void* p_out, dda_solve_stats* stats);

/*
 * Solve A P = E_inc for nrhs caller-supplied incident fields (the linear
 * system of the guide's section "The DDA" for any right-hand side, not only
 * a plane wave).  e_inc is [nrhs][N][3] complex128 in the same site order and
 * concatenation as p0 and p_out (host memory, or device memory with
 * DDA_DEVICE_PTRS); it is read during the call only.  waves[i] still selects
 * the target of rhs i and, through khat and e0, its polarizability (LDR
 * depends on them; CM does not).  Everything else is as for dda_solve; the
 * guesses that carry a previous solution to a new incidence direction
 * (PREV_SHIFT, PROJECT, NN) assume plane waves.  dda_cross_sections after
 * this call uses e_inc as E in the same sums, still divided by pi a_eff^2
 * only: they are efficiencies per unit incident |E0|^2 only if the caller's
 * field has unit amplitude (scale them by 1/|E0|^2 otherwise).  Errors:
 * DDA_ERR_INVALID_ARG for a NULL or non-finite e_inc, otherwise those of
 * dda_solve.
 */
dda_status dda_solve_field(dda_ctx* ctx, int32_t nrhs, const dda_wave* waves, const dda_solve_opts* opts,
                           const void* e_inc, const void* p0, void* p_out, dda_solve_stats* stats);

/* y = A x for nrhs vectors on target `target`.  ainv holds 1/alpha per
 * (rhs, composition) as 2*nrhs*ncomp doubles, or is NULL to use the
 * polarizability of the target's prescription with the wave khat=(1,0,0),
 * e0=(0,1,0).  x, y: [nrhs][N][3] complex128. `prec` is DDA_FP32 or DDA_FP64. */
dda_status dda_matvec(dda_ctx* ctx, int32_t target, int32_t nrhs, const double* ainv,
                      const void* x, void* y, uint32_t prec, uint32_t flags);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = A x as
 * dda_matvec computes it, with every intermediate (the site-ordered vectors,
 * the spectrum slab, the FP32 copy of 1/alpha) in a fixed device array of
 * DDA_NOALLOC_SCRATCH_BYTES per GPU, held from the first dda_create on that
 * GPU until the process ends.  No hipMalloc, hipFree, allocating library call
 * or synchronization: the work is enqueued on the context's stream and the
 * call returns.
 *   ainv  device pointer, [nrhs][ncomp] complex128 1/alpha per (rhs, composition)
 *   x, y  device pointers, [nrhs][N][3] complex128 in the ABI site order
 *   prec  DDA_FP32 or DDA_FP64 (the matvec's arithmetic)
 * The target's spectrum for `prec` must exist (dda_build_green_fft or an
 * earlier solve or matvec of that precision), else DDA_ERR_STATE; a call whose
 * scratch need, nrhs x (spectrum slab + 2 vectors) in the precision of the
 * matvec plus the 1/alpha copy, exceeds DDA_NOALLOC_SCRATCH_BYTES returns
 * DDA_ERR_INVALID_ARG (64 MiB: e.g. 2 FP32 rhs of a 64^3 box, 13 of a 32^3
 * box).  Every call on a GPU shares that GPU's scratch and leaves its
 * contents behind: calls that overlap on one GPU (other contexts or streams)
 * race and must be ordered by the caller. */
#define DDA_NOALLOC_SCRATCH_BYTES (64u << 20)
dda_status dda_matvec_noalloc(dda_ctx* ctx, int32_t target, int32_t nrhs, const void* ainv, const void* x, void* y,
                              uint32_t prec);

/* 1/alpha of every composition of a target for a wave (host arithmetic);
 * out: 2*ncomp doubles. */
dda_status dda_inverse_polarizability(const dda_ctx* ctx, int32_t target, const dda_wave* wave,
                                      double* out);

/* Efficiencies of the last solve: q is nrhs x {Q_ext, Q_abs, Q_sca} with
 * C_ext = 4 pi k sum_j Im(E_j^* . P_j),
 * C_abs = 4 pi k sum_j [Im(P_j . (1/alpha_j)^* P_j^*) - (2/3) k^3 |P_j|^2],
 * Q_sca = Q_ext - Q_abs, Q = C / (pi a_eff^2) (guide, section "What Does It
 * Calculate?"; sums from Draine 1988).  FP64 reductions on the device. */
dda_status dda_cross_sections(dda_ctx* ctx, int32_t nrhs, double* q);

/* Phase-lag and backscattering efficiencies and the moments of the
 * scattered intensity of the last solve (guide, sections "What Does It
 * Calculate?", "Calculation of <cos theta>, Radiative Force, and Radiation
 * Torque" and "Averaging over Scattering Directions").  n_tf, w: ndir
 * target-frame scattering directions (3 doubles each) and solid-angle
 * weights, e.g. from dda_scattering_quadrature.  out: nrhs x DDA_NMOMENTS
 * doubles, per rhs
 *   [0] Q_pha = 2 pi k Re(sum_j E_j^* . P_j) / (pi a_eff^2) (the phase-shift
 *       cross section of Draine 1988 over pi a_eff^2);
 *   [1] Q_bk = k^4 |sum_j (P_j - n (n . P_j)) exp(-i k n . r_j)|^2 / (pi a_eff^2)
 *       at n = -khat (differential backscattering cross section per sr);
 *   [2] Q_sca from the quadrature, sum_d w_d dC/dOmega(n_d) / (pi a_eff^2);
 *   [3..5] Q_sca g = sum_d w_d dC/dOmega n_d / (pi a_eff^2), target frame;
 *   [6] <cos theta> = g . khat and [7] <cos^2 theta>, both normalized by
 *       Q_sca = Q_ext - Q_abs;
 *   [8..10] Q_pr = Q_ext khat - Q_sca g, target frame.
 * FP64 device sums over the sites (the amplitude kernel), weighted sums over
 * the directions on the host.  DDA_ERR_STATE before a solve,
 * DDA_ERR_INVALID_ARG for nrhs other than the last solve's or ndir < 1. */
enum { DDA_NMOMENTS = 11 };
dda_status dda_scattering_moments(dda_ctx* ctx, int32_t nrhs, int32_t ndir, const double* n_tf, const double* w,
                                  double* out);

/* Efficiencies at other target rotations Phi about the incidence direction
 * without new solves (guide, section "Scattering by Finite Targets", the
 * IORTH remark: the solution for another Phi is a linear combination of the
 * solutions for two incident polarizations of one orientation).  Right-hand
 * sides 2p and 2p+1 of the last solve form pair p: one target, one incidence
 * direction, polarizations e_0, e_1.  coeffs: npairs x ncomb x 2 (output
 * state l) x 2 (basis a) complex128 (re, im) with E_l = sum_a c[l][a] E_a,
 * e.g. from dda_phi_coefficients; the solution is combined the same way.
 * q: npairs x ncomb x 2 x {Q_ext, Q_abs, Q_sca}, the sums of
 * dda_cross_sections on the combined field and solution (FP64 pair sums on
 * the device, 2 x 2 bilinear forms combined on the host).  Exact only when
 * 1/alpha does not depend on the polarization: DDA_ERR_INVALID_ARG for LDR
 * targets, for 2 * npairs != rhs count of the last solve, and for pairs that
 * span two targets or two incidence directions; DDA_ERR_STATE before a
 * solve. */
dda_status dda_cross_sections_phi(dda_ctx* ctx, int32_t npairs, int32_t ncomb, const double* coeffs, double* q);

/* Scattering amplitudes of the last solve:
 *   f[rhs][dir][m] = k^3 e_m . sum_j P_j exp(-i k n_dir . r_j),  m = 0, 1,
 * with n (ndir x 3 doubles) and the two scattered polarization vectors e_1,
 * e_2 (ndir x 6 doubles: e_1 then e_2) given in the target frame (guide,
 * section "Scattering by Finite Targets: The Mueller Matrix", eq. f_ml_def).
 * f: nrhs*ndir*2 complex128 (interleaved). */
dda_status dda_amplitudes(dda_ctx* ctx, int32_t nrhs, int32_t ndir, const double* n_tf,
                          const double* e_tf, double* f);
/* The same amplitudes with a direction set per right-hand side: rhs i of the
 * last solve takes the ndir directions n_tf[i][0..ndir-1] (n_tf: nrhs x ndir
 * x 3 doubles) with polarization vectors e_tf[i] (nrhs x ndir x 6 doubles),
 * e.g. the lab-frame scattering directions of each orientation of a sweep
 * expressed in the target frame.  f: nrhs*ndir*2 complex128, as above.
 * DDA_ERR_INVALID_ARG for nrhs other than the last solve's or ndir <= 0;
 * DDA_ERR_STATE before a solve. */
dda_status dda_amplitudes_per_rhs(dda_ctx* ctx, int32_t nrhs, int32_t ndir, const double* n_tf, const double* e_tf,
                                  double* f);

/* Total E and B at npts points in or near the targets of the last solve
 * (guide, "Postprocessing: Calculating E and B In or Near the Target"): the
 * incident plane wave (B_inc = khat x E_inc) plus the retarded field of
 * every dipole, E = exp(ikR)[k^2/R (p - n(n.p)) + (1/R^3 - ik/R^2)(3n(n.p) - p)]
 * and B = exp(ikR)(k^2/R + ik/R^2)(n x p) for a dipole p at R = R n from the
 * point (Gaussian units, exp(-i omega t)).  A point on an occupied site takes
 * no contribution from that site, so there E is the site's local field
 * (1/alpha) P.  The guide's smoothing of contributions from dipoles closer
 * than d (a factor from a paper it cites but does not print) is not applied:
 * the bare dipole sum is evaluated everywhere.  pts: npts x 3 doubles, target
 * frame, units of d, from the same origin as the sites (dda_set_target's
 * origin, by default the centroid); every rhs of the last solve is evaluated
 * in its own target's frame.  E: nrhs x npts x 3 complex128 (interleaved);
 * B: the same, or NULL.  FP64 on the device, O(npts x N) per rhs.  Errors:
 * DDA_ERR_STATE before a solve, DDA_ERR_INVALID_ARG for nrhs other than the
 * last solve's, npts <= 0 or NULL pts or E. */
dda_status dda_near_field(dda_ctx* ctx, int32_t nrhs, int32_t npts, const double* pts, double* E, double* B);

/* Amplitude matrix S_1..S_4 and the 4x4 Mueller matrix from the amplitudes
 * of two orthogonal incident polarizations (guide, eqs. S_1_relto_f21andf22
 * and the bilinears of "Relation Between Stokes Parameters of Incident and
 * Scattered Radiation").  f: ndir x 2 (m) x 2 (l) complex128 ordered
 * [dir][m][l]; phi: ndir scattering-plane angles; e01, e02: lab-frame
 * incident polarization vectors (6 doubles each).  S: ndir x 4 complex128
 * (may be NULL); mueller: ndir x 16 doubles row-major (may be NULL). */
dda_status dda_mueller(int32_t ndir, const double* f, const double* phi, const double* e01,
                       const double* e02, double* S, double* mueller);

/* Polarized differential scattering cross sections and the degree of linear
 * polarization from the Mueller matrix (guide, "Polarization Properties of
 * the Scattered Radiation": an ideal linear polarizer parallel or
 * perpendicular to the scattering plane applied to the scattered Stokes
 * vector; "Relation Between Mueller Matrix and Scattering Cross Sections":
 * I_s r^2 = (dC_sca/dOmega) I_i).  mu: ndir x 16 Mueller elements S_ij,
 * row-major as dda_mueller writes them; k: wavenumber in units of 1/d;
 * stokes_in: the incident Stokes vector (I, Q, U, V) with I > 0 (results
 * are per unit incident intensity).  out: ndir x 4 doubles = dC_sca/dOmega
 * of the scattered light polarized parallel to the scattering plane,
 * perpendicular to it, in total, and P = (S21^2 + S31^2)^(1/2) / S11, the
 * linear polarization for unpolarized incidence (0 where S11 = 0).  Host
 * only.  DDA_ERR_INVALID_ARG for ndir <= 0, NULL pointers, k <= 0 or I <= 0. */
dda_status dda_polarization(int32_t ndir, const double* mu, double k, const double* stokes_in, double* out);

/* Lab-frame axes in the target frame for target orientation (beta, Theta,
 * Phi) in radians and target axes a1, a2 (target frame; NULL for x and y)
 * (guide, section "Orientation of the Target in the Lab Frame").
 * out: 9 doubles, rows x_LF, y_LF, z_LF. */
dda_status dda_lab_frame(double beta, double theta, double phi, const double* a1, const double* a2,
                         double* out);

/* The two incident waves of orientation (beta, Theta, Phi): khat = x_LF, and
 * the polarizations e01 (lab frame, 6 doubles, normalized here) and
 * e02 = x_LF x conj(e01) (guide, sections "Target Orientation" and "Incident
 * Polarization State"), all expressed in the target frame.  a1, a2: target
 * axes in the target frame (NULL: x, y).  e01 NULL means y_LF.  out[0..1]
 * receive the waves with target = `target`. */
dda_status dda_orientation_waves(double beta, double theta, double phi, const double* a1, const double* a2,
                                 const double* e01, int32_t target, dda_wave* out);

/* The scattering directions and solid-angle weights that average over
 * directions (guide, section "Averaging over Scattering Directions"):
 * theta_j at equal steps of s(theta) = theta + theta / (theta + theta0),
 * theta0 = 2 pi / (1 + x), from 0 to pi, N_theta from eta (rounded to the
 * nearest integer, at least 3); one phi at theta = 0 and pi, else
 * N_phi(j) = max{3, nint[4 pi sin(theta_j) / (theta_{j+1} - theta_{j-1})]}
 * values phi = 2 pi k / N_phi(j), k = 0.., about x_LF from y_LF; weights
 * Omega_jk of the guide's formulas.  lab_axes: 9 doubles (dda_lab_frame).
 * ndir receives the number of directions; with n_tf or w NULL only the count
 * is returned, else n_tf (ndir x 3, target frame) and w (ndir) are filled when
 * cap >= ndir (DDA_ERR_INVALID_ARG otherwise).  Host arithmetic. */
dda_status dda_scattering_quadrature(double x, double eta, const double* lab_axes, int32_t cap, int32_t* ndir,
                                     double* n_tf, double* w);

/* Orientation samples and weights for orientational averages (guide,
 * sections "Sampling in Theta, Phi, and beta" and "Orientational
 * Averaging").  lims: {BETAMI, BETAMX, THETMI, THETMX, PHIMIN, PHIMAX} in
 * radians; counts: {NBETA, NTHETA, NPHI}, each >= 1.  beta (NBETA) and phi
 * (NPHI) are the midpoints of equal intervals of their ranges; theta
 * (NTHETA) is uniform in cos(Theta): for odd NTHETA from THETMI to THETMX
 * inclusive with Simpson weights (1, 4, 2, ..., 4, 1) / (3 (NTHETA - 1)), for
 * even NTHETA the midpoints of NTHETA equal intervals of cos(Theta) with
 * weight 1/NTHETA (the guide prints the odd-NTHETA weights over NTHETA,
 * which does not sum to one; the normalized Simpson form is used), for
 * NTHETA = 1 THETMI alone.  weight: NBETA x NTHETA x NPHI (beta slowest),
 * the product of the beta, Theta and Phi weights; it sums to one.  Host
 * arithmetic; DDA_ERR_INVALID_ARG for NULL pointers or counts < 1. */
dda_status dda_orientation_samples(const double* lims, const int32_t* counts, double* beta, double* theta,
                                   double* phi, double* weight);

/* Combination coefficients for other rotations Phi of one (beta, Theta): for
 * each phi[k], c[k][l][a] (complex128, (re, im)) with e_l(beta, Theta, phi[k])
 * = sum_a c[k][l][a] e_a(beta, Theta, phi_ref), the target-frame incident
 * polarizations of dda_orientation_waves (same a1, a2, e01 arguments).  The
 * incidence direction does not depend on Phi, so the fields combine the same
 * way.  coeffs: nphi x 2 x 2 complex128.  Host arithmetic. */
dda_status dda_phi_coefficients(double beta, double theta, double phi_ref, int32_t nphi, const double* phi,
                                const double* a1, const double* a2, const double* e01, double* coeffs);

/* Target-frame scattering directions and polarization basis for lab-frame
 * scattering angles: n = x cos(theta) + y sin(theta) cos(phi) + z sin(theta)
 * sin(phi) (guide, section "Scattering Directions", LFRAME), e_1 = theta_hat
 * (parallel to the scattering plane) and e_2 = phi_hat (guide, section
 * "Scattering by Finite Targets: The Mueller Matrix").  lab_axes: 9 doubles
 * from dda_lab_frame.  n_tf: ndir x 3, e_tf: ndir x 6 (e_1 then e_2). */
dda_status dda_scattering_frame(int32_t ndir, const double* theta, const double* phi, const double* lab_axes,
                                double* n_tf, double* e_tf);

/* Choose FFT tile shapes and graph depth for every target by timing
 * candidates on the device; results are cached in the JSON file named by
 * `cache_path` (NULL: the DDA_TUNE_CACHE environment variable, else no
 * file).  `nrhs_hint` is the batch size to tune for. */
dda_status dda_autotune(dda_ctx* ctx, int32_t nrhs_hint, const char* cache_path);

/* Milliseconds the last solve spent producing an initial guess from the
 * previous solution (phase shift, plus the network for DDA_GUESS_NN). */
dda_status dda_last_guess_ms(const dda_ctx* ctx, double* ms);

/* Launch shape of a target's matvec passes for precision DDA_FP32 or
 * DDA_FP64, as 8 integers: {planes in LDS, plane threads, z threads, z tile
 * columns, fallback lines per block, fallback threads, specialised kernels
 * bitmask (1 plane passes, 2 z pass, 4 two-factor inverse plane pass for
 * n = 64, 8 class-grouped spectrum slab for n = 64 with z pass variant 3: the
 * z pass combines the four quadrants that each output parity class of the
 * inverse plane pass needs), z pass variant (0 one rhs per block, 1 up to 8 rhs per block with
 * the spectrum in registers, 2 two-factor 8 x 8 pass for n = 64, 3 the same
 * with the two frequency parities in the two halves of a block)}.
 * dda_set_shape rejects shapes that do
 * not fit the kernels' LDS or thread limits. */
dda_status dda_get_shape(const dda_ctx* ctx, int32_t target, uint32_t prec, int32_t* out8);
dda_status dda_set_shape(dda_ctx* ctx, int32_t target, uint32_t prec, const int32_t* in8);

/* Timing of the last solve: milliseconds in FP32 matvecs, FP64 matvecs,
 * and the whole call (device events).  Any pointer may be NULL. */
dda_status dda_last_timing(const dda_ctx* ctx, double* ms_mv32, double* ms_mv64, double* ms_total);

/* Per-pass kernel timing of `reps` FP32 or FP64 matvecs of nrhs vectors on
 * target `target` with the current tiles: fills ms[3] with the mean duration
 * of the xy-forward pass, the z pass and the xy-inverse pass (HIP events on
 * the context stream), and bytes[3] with the algorithmic bytes moved by each
 * pass per launch.  Either pointer may be NULL. */
dda_status dda_profile_matvec(dda_ctx* ctx, int32_t target, int32_t nrhs, uint32_t prec, int32_t reps,
                              double* ms, double* bytes);

/* ---- Learned initial guess ----
 * For a sweep over orientations (or incidence directions) of one target, a 3D
 * convolutional network on the target's cubic box (side divisible by 16)
 * corrects the DDA_GUESS_PROJECT guess P_b.  With E_b = (1/alpha) P_b its
 * local field, R = E_inc - A P_b its residual field (both FP32, R from the
 * products the projection already formed) and sigma the rms of R, the local
 * field is E_loc = E_b + sigma net(features) at the occupied sites and the
 * guess is P0 = E_loc / (1/alpha): a learned approximate inverse of A applied
 * once to R / sigma.  Features per voxel: occupancy, R / sigma, E_b,
 * (eps-1)/(eps+2), k d (16 channels).  Train and use the network with the
 * same history setting.
 * 3x3x3 convolutions with dilations 1, 2, 4, 8, ReLU; BF16 operands on MFMA
 * with FP32 accumulation; FP32 master weights trained with Adam on solutions
 * of DDA_GUESS_PROJECT solves (dda_nn_record).  The network of zeros reproduces
 * DDA_GUESS_PROJECT.  A guess is used only if its FP64 residual is below
 * ||E|| (else P0 = 0). */
typedef struct dda_nn dda_nn;

typedef struct {
    int32_t width;      /* hidden channels: 16, 32 or 64 (width 64, depth 10: 940k parameters) */
    int32_t depth;      /* number of convolution layers, >= 2 */
    int32_t seed;       /* weight initialisation seed */
    int32_t reserved;
} dda_nn_config;

typedef struct {
    int32_t epochs;
    int32_t batch;      /* samples per Adam step (<= 8) */
    double lr;          /* Adam learning rate */
    double weight_decay;
    int32_t reserved[4];
} dda_nn_train_opts;

dda_status dda_nn_create(dda_ctx* ctx, const dda_nn_config* cfg, dda_nn** out);
dda_status dda_nn_destroy(dda_nn* nn);
int64_t dda_nn_num_params(const dda_nn* nn);
int32_t dda_nn_num_samples(const dda_nn* nn);
/* Layer shapes: depth x {cin, cout, dilation}. */
dda_status dda_nn_layer_info(const dda_nn* nn, int32_t* out3);
/* Flat FP32 parameters: per layer W[27][cin][cout] (offset index
 * (dz+1)*9 + (dy+1)*3 + (dx+1)) then b[cout]. */
dda_status dda_nn_get_params(const dda_nn* nn, float* out);
dda_status dda_nn_set_params(dda_nn* nn, const float* in);
/* Attach a network as the DDA_GUESS_NN model of the context (NULL detaches). */
dda_status dda_set_guess_model(dda_ctx* ctx, dda_nn* nn);
/* Record every solution of the last solve as a training sample (target
 * (E_loc - E_b) / sigma).  The last solve must have used DDA_GUESS_PROJECT or
 * DDA_GUESS_NN, so that E_b and R exist (DDA_ERR_STATE otherwise). */
dda_status dda_nn_record(dda_ctx* ctx, dda_nn* nn);
/* Train on the recorded samples; mean loss of the last epoch in *loss. */
dda_status dda_nn_train(dda_ctx* ctx, dda_nn* nn, const dda_nn_train_opts* opts, double* loss);
dda_status dda_nn_save(const dda_nn* nn, const char* path);
dda_status dda_nn_load(dda_nn* nn, const char* path);
/* Timing hook: forward passes and parameter-gradient passes of the network
 * on ns (1..8) samples of a D^3 box (D a multiple of 16) of device-resident
 * pseudo-random BF16 features and output gradients, reps times each (HIP
 * events on the null stream).  Mean milliseconds per forward (*ms_fwd) and
 * per backward (*ms_bwd) pass over the ns samples, and the forward pass's
 * dense GFLOP (2 x 27 cin cout D^3 ns summed over layers, *gflop_fwd); any
 * pointer may be NULL.  Overwrites the network's activation buffers. */
dda_status dda_nn_profile(dda_nn* nn, int32_t D, int32_t ns, int32_t reps, double* ms_fwd, double* ms_bwd,
                          double* gflop_fwd);
/* Test hook on dense host arrays over a D^3 box (D >= 16): x_in [ns][D^3][16],
 * target [ns][D^3][16], mask [ns][D^3]; runs the forward pass (out, [ns][D^3][16],
 * may be NULL) and, when target, mask and grads are given, the masked mean
 * squared error over the first nout channels normalised per sample by the
 * target's squared norm, averaged over samples, and its parameter gradients
 * (flat, as dda_nn_get_params). */
dda_status dda_nn_forward_backward(dda_nn* nn, int32_t ns, int32_t D, const float* x_in, const float* target,
                                   const uint8_t* mask, int32_t nout, float* out, float* grads, double* loss);

#ifdef __cplusplus
}
#endif
#endif /* DDA_H */
