/*
 * hubbard_chfsi.h - C ABI of the MI355X (gfx950) library for the hot path of
 * real-space Hubbard-corrected DFT (arXiv:2507.23612): Chebyshev-filtered
 * subspace iteration of the operator
 *
 *   H[D] = -1/2 Delta_h + V_loc + sum_I chi_I Gamma_I chi_I^H dV
 *          + sum_{I in U} Phi_I U_I (1/2 - D_I) Phi_I^H dV
 *
 * on a uniform periodic grid (Sec. II.B), with the Dudarev energy
 * E_U = sum_{sigma I} U_I/2 Tr(D - D^2) (Sec. II.A, Eq. E_U), occupation
 * matrices D (Eq. orbital_occup_ext) and the Hubbard potential derived from
 * them (Sec. II.A potential section, Eq. DerED).
 *
 * Conventions
 *   - grid node (i,j,k) is at (i h1, j h2, k h3), 0-based, h_a = L_a / n_a;
 *     linear index i + n1*(j + n2*k) (x fastest); quadrature weight
 *     dV = h1 h2 h3 (trapezoidal rule, Sec. II.B);
 *   - a block of ncol states is column-major nd x ncol with leading
 *     dimension ld >= nd: state j starts at element j*ld.  Real blocks hold
 *     double (FP64 mode) or float (mixed mode); blocks at k != 0 hold
 *     interleaved complex values of the same precision;
 *   - orbitals are normalised as dV sum |psi|^2 = 1 (bohr^-3/2); energies are
 *     in hartree; lengths in bohr; k-points are Cartesian, bohr^-1;
 *   - occupation matrices are passed as [nspin][n_hubbard_atoms][5][5]
 *     row-major doubles (real: every k-point set used here is closed under
 *     k -> -k, which makes D real).
 *
 * Ownership and threading
 *   - every host array passed to a call is read during the call only and
 *     copied where it must persist; the caller keeps ownership;
 *   - device memory comes from the caller: hcu_workspace_size() tells how many
 *     bytes the context needs, hcu_bind() hands over one device buffer and
 *     the HIP stream all work is queued on.  The library does not free it;
 *   - device pointers passed to compute calls must be valid on the bound
 *     device and stream; calls return once the work is queued unless stated;
 *   - a context is not thread-safe; distinct contexts are independent.
 *
 * Errors
 *   - every call returns an hcu_status; HCU_OK = 0.  Arguments are validated
 *     on the host before any device work is queued; on error nothing is
 *     queued and hcu_last_error(ctx) describes the problem.  No C++
 *     exception crosses this interface.
 */
#ifndef HUBBARD_CHFSI_H
#define HUBBARD_CHFSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hcu_status {
  HCU_OK = 0,
  HCU_INVALID_ARG = 1,    /* a size, pointer or option is invalid          */
  HCU_OOM = 2,            /* bound workspace too small                     */
  HCU_NOT_SPD = 3,        /* Gram matrix of the filtered block not SPD     */
  HCU_NOT_CONVERGED = 4,  /* SCF reached max_iter (state stays usable)     */
  HCU_NAN = 5,            /* non-finite value in inputs or results         */
  HCU_DEVICE = 6,         /* HIP / rocSOLVER reported an error             */
  HCU_NOT_BOUND = 7       /* compute call before hcu_bind()                */
} hcu_status;

typedef enum hcu_precision {
  HCU_FP64 = 0,   /* every step in double                                     */
  HCU_MIXED = 1   /* filter stencil and blocks in FP32; projector and RR
                     contractions on FP32 MFMA with FP32 accumulation;
                     Cholesky, subspace eigensolve, occupations, D, E_U in FP64 */
} hcu_precision;

#define HCU_MAX_KB 4

/* One species (Sec. II.B: atom-centred functions = real Y_lm x radial, cut
 * where the radial value drops below `threshold` and not stored beyond). */
typedef struct hcu_species {
  double vloc_depth;            /* V_loc = -depth exp(-r^2/(2 width^2)), Ha  */
  double vloc_width;            /* bohr                                      */
  int    n_kb;                  /* number of KB channels (<= HCU_MAX_KB)     */
  int    kb_l[HCU_MAX_KB];      /* channel angular momentum, 0 or 1          */
  double kb_gamma[HCU_MAX_KB];  /* channel energy, Ha                        */
  double kb_width;              /* radial N r^l exp(-r^2/(2 w^2)), bohr      */
  int    hub_l;                 /* Hubbard manifold l (0..2), -1 = none      */
  double hub_U;                 /* effective U, Ha                           */
  int    hub_power;             /* Hubbard radial N r^p exp(-alpha r)        */
  double hub_alpha;             /* bohr^-1                                   */
  double threshold;             /* truncation value, bohr^-3/2 (> 0)         */
} hcu_species;

/* The problem statement (Sec. II.B grid and stencil; Sec. II.A atoms,
 * orbitals, U, spins and k-points). */
typedef struct hcu_problem {
  double L[3];                  /* orthorhombic cell lengths, bohr           */
  int    n[3];                  /* grid points per axis (each >= 2; a stencil
                                   wider than the cell wraps several times)  */
  int    n0;                    /* half stencil order: FD order is 2*n0      */
  int    nspin;                 /* 1 (unpolarised) or 2                      */
  int    nk;                    /* number of k-points                        */
  const double* kpts;           /* [nk][3], Cartesian bohr^-1                */
  const double* kw;             /* [nk], weights summing to 1                */
  int    natom;
  const int*    atom_species;   /* [natom] index into species                */
  const double* pos;            /* [natom][3], bohr                          */
  int    nspecies;
  const hcu_species* species;   /* [nspecies]                                */
  int    ns;                    /* states per (spin, k)                      */
  double nelec;                 /* electrons in the cell                     */
  double kT;                    /* Fermi-Dirac smearing, Ha (> 0)            */
  int    degree;                /* Chebyshev filter degree (>= 1)            */
  int    precision;             /* hcu_precision                             */
  int    lowdin;                /* 1: Loewdin-orthonormalise Hubbard orbitals
                                   per atom (O^-1/2, O = Phi^H Phi dV)       */
  int    hxc;                   /* 1: density-dependent Hamiltonian (Sec.
                                   II.B): V = V_loc + V_H[rho] + V_x[rho],
                                   the SCF mixes the density and D together
                                   (nspin = 1 only); 0: fixed V_loc          */
} hcu_problem;

typedef struct hcu_scf_opts {
  int    max_iter;              /* SCF iterations (>= 1)                     */
  int    first_passes;          /* filter + Rayleigh-Ritz passes, 1st iter   */
  int    lanczos_steps;         /* steps of the spectral upper bound         */
  int    pulay_history;         /* Pulay mixing history (>= 1)               */
  double pulay_beta;            /* mixing parameter                          */
  double tol_d;                 /* stop when |D_out - D_in|_F < tol_d ...    */
  double tol_f;                 /* ... and |F_n - F_{n-1}| / natom < tol_f   */
  int    fixed_iterations;      /* > 0: run exactly this many, no test       */
  int    verbose;               /* 1: one line per iteration on stderr       */
  double kerker_k0;             /* hxc: Kerker wave number k0 (bohr^-1, >= 0)
                                   of the density preconditioner             */
  double tol_rho;               /* hxc: ... and sqrt(dV sum (rho_out -
                                   rho_in)^2) / N_e < tol_rho (> 0)          */
} hcu_scf_opts;

typedef struct hcu_scf_report {
  int    iterations;
  int    converged;
  double F;                     /* Mermin free energy of the model, Ha       */
  double E_U;                   /* Hubbard energy, both spin channels        */
  double e_band;
  double residual;              /* last |D_out - D_in|_F                     */
  double seconds;               /* wall time of the SCF loop                 */
  double filter_seconds;        /* of which: filters + H Y of Rayleigh-Ritz  */
  double hx_columns;            /* number of single-column H applications    */
  double residual_rho;          /* hxc: last density residual (else 0)       */
} hcu_scf_report;

typedef struct hcu_energies {
  double F;                     /* e_band - dc + E_U - kT S (+ e_hxc)        */
  double e_band;                /* g_s sum_k w_k sum_j f_j lambda_j          */
  double dc;                    /* sum Tr(M(D_in) D_out) over spins, atoms   */
  double E_U;                   /* sum_sigma sum_I U/2 Tr(D - D^2)           */
  double ts;                    /* kT S                                      */
  double mu;                    /* Fermi level                               */
  double E_H;                   /* hxc: Hartree energy of rho_out (else 0)   */
  double E_x;                   /* hxc: LDA exchange energy of rho_out       */
  double e_hxc;                 /* hxc: -int rho_out (V_H + V_x)[rho_in] +
                                   E_H + E_x, included in F                  */
} hcu_energies;

/* Accumulated device time per kernel family, recorded only while profiling
 * is on: from the begin/end timestamps of the family's own kernel dispatches
 * (the eigensolve and the rotation, which call the vendor libraries, from
 * events around them).  Rayleigh-
 * Ritz steps of several blocks run side by side, so their times can add up
 * to more than the wall time.  For real and complex FP32 blocks the
 * projections of a Chebyshev step's output are computed in the scatter pass
 * of that step and counted under scatter; project then holds the first
 * step's projections. */
typedef struct hcu_kernel_times {
  double stencil_ms;  long long stencil_launches;  /* stencil + V + Chebyshev step       */
  double project_ms;  long long project_launches;  /* projections onto atom functions    */
  double gram_ms;     long long gram_launches;     /* S, Hs contractions + reduction     */
  double eig_ms;      long long eig_launches;      /* generalized eigensolve (one-workgroup
                                                      tridiagonalization + rocSOLVER)   */
  double rotate_ms;   long long rotate_launches;   /* X = Y C (rocBLAS GEMM)             */
  double scatter_ms;  long long scatter_launches;  /* projector scatter (KB + Hubbard)   */
  double fused_ms;    long long fused_launches;    /* of scatter: the fused scatter +
                                                      projection kernel alone           */
  double hxc_ms;      long long hxc_launches;      /* hxc: density, Hartree and exchange
                                                      energies, density mixing step
                                                      (stream time, host solve included) */
} hcu_kernel_times;

typedef struct hcu_ctx hcu_ctx;

/* Create a context from the problem statement: validates it, builds the
 * per-atom support lists (grid nodes within the truncation radius of any
 * periodic image) and sizes the device workspace.  Host arrays are copied.
 * Errors: HCU_INVALID_ARG (bad sizes, species, l > 2, n0 outside 1..6, ...). */
hcu_status hcu_create(const hcu_problem* p, hcu_ctx** out);

/* Free the context (not the bound device buffer). NULL is ignored. */
void hcu_destroy(hcu_ctx* ctx);

/* Text of the last error on this context (valid until the next call). */
const char* hcu_last_error(const hcu_ctx* ctx);

/* Device bytes the context needs (orbital blocks for every spin and k-point,
 * three filter/Rayleigh-Ritz work blocks, tables, small dense buffers). */
hcu_status hcu_workspace_size(const hcu_ctx* ctx, size_t* bytes);

/* Bind `bytes` of device memory at `dev_ptr` (256-byte aligned) and the HIP
 * stream `stream` (NULL = default stream); evaluates V_loc and every atom-
 * centred function on the grid (Sec. II.B) on the device.  The context also
 * takes a few bytes of pinned host memory (eigensolve status copies) and,
 * when it leads a pass over several blocks (several (spin, k) blocks, or a
 * batch), up to four side streams of its own for the blocks' Rayleigh-Ritz
 * steps and the members' projections and scatters; their work is ordered
 * after and before the bound stream's by events, so to the caller
 * everything stays ordered on `stream`.  Errors: HCU_OOM if bytes < hcu_workspace_size(), HCU_DEVICE on
 * a HIP error. */
hcu_status hcu_bind(hcu_ctx* ctx, void* dev_ptr, size_t bytes, void* stream);

/* Move the atoms of a bound context (ab initio molecular dynamics, Sec.
 * II.B): pos is host [natom][3] bohr.  The supports, the atom-centred
 * function tables and V_loc are rebuilt on the device for the new geometry;
 * the orbitals are kept (the start of the next SCF) and the next hcu_scf /
 * hcu_scf_begin recomputes the spectral bounds.  If the context holds
 * converged results (after hcu_scf or hcu_update_occupations), their
 * positions and occupation matrices D_out first join a history of the last
 * three geometries.  extrapolate = 1 then sets the input occupation
 * matrices by the second-order extrapolation the paper uses for D in AIMD:
 * D split into the isolated-atom part and a residual, the residual carried
 * forward as
 *   D(t+dt) = D(t) + a (D(t) - D(t-dt)) + b (D(t-dt) - D(t-2dt)),
 * with a, b the least-squares fit of the atomic trajectory
 *   R(t+dt) - R(t) ~ a (R(t) - R(t-dt)) + b (R(t-dt) - R(t-2dt))
 * (minimum-norm solution when the two steps are parallel; with one or two
 * recorded geometries b = 0, and a = 0 with one).  The isolated-atom part
 * does not depend on the positions, so it cancels from the differences.
 * extrapolate = 0 leaves D_in unchanged.  coeffs (optional, host double[3])
 * receives {a, b, order}.  Errors: HCU_NOT_BOUND, HCU_INVALID_ARG, HCU_NAN
 * (non-finite position), HCU_OOM when the moved supports need more than the
 * bound workspace (nothing changes; bind a larger buffer - the binding may
 * be larger than hcu_workspace_size() - and retry). */
hcu_status hcu_move_atoms(hcu_ctx* ctx, const double* pos, int extrapolate, double* coeffs);

/* Hubbard occupation matrices D_in (host, [nspin][nhub][5][5] row-major;
 * rows/cols beyond 2l+1 ignored for l < 2) defining H[D] (Sec. II.A). */
hcu_status hcu_set_hubbard_occupation(hcu_ctx* ctx, const double* D);

/* Number of atoms carrying a Hubbard manifold (in atom order). */
int hcu_num_hubbard_atoms(const hcu_ctx* ctx);

/* Sizes of the discretised problem (valid after hcu_create). */
typedef struct hcu_sizes {
  int64_t nd;               /* grid points                                   */
  int     nproj;            /* atom-centred functions (KB + Hubbard)         */
  int     nblocks;          /* projector blocks (per atom: KB, Hubbard)      */
  int64_t support_points;   /* sum of block support sizes                    */
  int64_t table_nnz;        /* (point, function) pairs of the per-point table */
  size_t  workspace_bytes;
  int     max_brick_functions;  /* most functions touching one 256-point brick */
  int64_t brick_slots;      /* sum over 256-point bricks of their function counts */
} hcu_sizes;
hcu_status hcu_get_sizes(const hcu_ctx* ctx, hcu_sizes* out);

/* Copy a start block X0 (device, nd x ns, ld = nd, the context precision)
 * and a Lanczos start vector v0 (device, nd, same precision) for spin
 * `spin`, k-point `ik`.  These are the random draws of the method; the
 * caller supplies them so runs are reproducible. */
hcu_status hcu_set_start(hcu_ctx* ctx, int spin, int ik, const void* X0, const void* v0);

/* Y = H[D] X for ncol states (device pointers, column-major, leading
 * dimension ld >= nd, context precision; X and Y must not overlap).
 * Includes kinetic stencil of order 2 n0 with Bloch wrap, V_loc (with hxc:
 * V_loc + V_H + V_x of the current input density), KB and Hubbard terms
 * (Sec. II.A potential; Sec. II.B implementation).
 * Errors: HCU_INVALID_ARG (spin/ik out of range, ncol < 1 or > ns, ld < nd). */
hcu_status hcu_apply_h(hcu_ctx* ctx, int spin, int ik, const void* X, void* Y,
                       int ncol, int64_t ld);

/* Scaled degree-m Chebyshev filter Y = p_m(H) X on [a, b] normalised at aL
 * (the filter of Chebyshev-filtered subspace iteration, Sec. II.B).  Uses the
 * context's work blocks, so ncol <= ns.  Errors as hcu_apply_h, plus
 * HCU_INVALID_ARG unless aL < a < b and m >= 1. */
hcu_status hcu_cheb_filter(hcu_ctx* ctx, int spin, int ik, const void* X, void* Y,
                           int ncol, int64_t ld, int m, double a, double b, double aL);

/* One filter + Rayleigh-Ritz pass on the context's orbitals of (spin, ik)
 * with the context's current bounds (set by hcu_lanczos_bounds or a previous
 * pass): X <- Y C with S = Y^H Y dV, Hs = Y^H H Y dV, Hs C = S C diag(lam).
 * Errors: HCU_NOT_SPD when S is not positive definite. */
hcu_status hcu_chfsi_pass(hcu_ctx* ctx, int spin, int ik);

/* k-step Lanczos on the start vector: sets the bounds of (spin, ik) to
 * b = theta_max + |beta_k|, aL = theta_min, a = aL + (b - aL)/10. */
hcu_status hcu_lanczos_bounds(hcu_ctx* ctx, int spin, int ik, int steps,
                              double* theta_min, double* upper);

/* Rayleigh-Ritz contractions alone (the matrices of the projected problem):
 * S = Y^H Y dV and Hs = Y^H HY dV for ncol <= ns states (device blocks,
 * leading dimension ld >= nd); results to host, ncol x ncol column-major
 * doubles (complex: interleaved).  Diagonal tiles are symmetrised. */
hcu_status hcu_gram(hcu_ctx* ctx, const void* Y, const void* HY, int ncol, int64_t ld, double* S, double* Hs);

/* Subspace rotation X = Y C (device blocks, ld >= nd; C host, ncol x ncol
 * column-major doubles, complex interleaved at k != 0).  A plain GEMM: run
 * by the vendor library (rocBLAS) on the context's stream. */
hcu_status hcu_rotate(hcu_ctx* ctx, const void* Y, const double* C, void* X, int ncol, int64_t ld);

/* Full SCF loop (Sec. II.B): per iteration, filter + Rayleigh-Ritz for every
 * (spin, k) (first iteration: first_passes), Fermi level, occupations, D_out,
 * E_U, free energy, Pulay mixing of D.
 * With hxc the Hamiltonian depends on the input density rho_in as well:
 *   -Delta_h V_H = 4 pi (rho_in - <rho_in>) with the kinetic term's
 *   finite-difference Laplacian (solved exactly by FFT with the stencil's
 *   symbol), V_x = -(3 rho_in / pi)^(1/3) (LDA exchange);
 *   F = e_band - dc + E_U - kT S - int rho_out (V_H + V_x)[rho_in]
 *       + E_H[rho_out] + E_x[rho_out];
 * the mixing is one Pulay step on the density (history pulay_history <= 8)
 * whose coefficients, fitted to the density residuals, mix D as well; the
 * density's residual step is preconditioned with the Kerker operator
 * (-Delta_h)(-Delta_h + k0^2)^-1 and the new density keeps N_e electrons.
 * rho_in is uniform (N_e / Omega) after hcu_bind and carries over from one
 * SCF to the next (and across hcu_move_atoms), like D_in.  Convergence then
 * also needs the density residual below tol_rho.  The FFT plans are created
 * in hcu_bind and allocate their own work areas.
 * Errors: HCU_NOT_CONVERGED when max_iter is reached without meeting the
 * tolerances (results stay valid), HCU_NOT_SPD, HCU_NAN, HCU_INVALID_ARG
 * (bad options; with hxc also pulay_history > 8, kerker_k0 < 0, tol_rho <= 0). */
hcu_status hcu_scf(hcu_ctx* ctx, const hcu_scf_opts* opts, hcu_scf_report* rep);

/* Step-wise SCF for callers that drive the loop themselves.  hcu_scf_begin
 * stores the options, computes the Lanczos bounds of every (spin, k) and
 * resets the mixing history; each hcu_scf_step runs one SCF iteration (first
 * one: first_passes filter + Rayleigh-Ritz passes per (spin, k)), updates
 * occupations, D_out and energies, tests convergence and, unless converged,
 * Pulay-mixes D and installs the new D_in.  hcu_scf = begin + steps. */
typedef struct hcu_scf_step_info {
  int    iteration;
  int    converged;
  double F;
  double E_U;
  double residual;             /* |D_out - D_in|_F of this iteration        */
  double dF;                   /* |F - F_prev| / natom (inf on the first)   */
  double residual_rho;         /* hxc: density residual (else 0)            */
} hcu_scf_step_info;
hcu_status hcu_scf_begin(hcu_ctx* ctx, const hcu_scf_opts* opts);
hcu_status hcu_scf_step(hcu_ctx* ctx, hcu_scf_step_info* info);

/* Occupations, energies and D_out of the current orbitals (used by hcu_scf;
 * callable after hcu_chfsi_pass on every (spin, k)). */
hcu_status hcu_update_occupations(hcu_ctx* ctx);

/* ------------------------------------------------- Hubbard forces, stress
 * Hellmann-Feynman Hubbard atomic forces (Sec. II.A force section: Eq.
 * Force1, Eq. DerR and the final force expression) and Hubbard stress tensor
 * (Sec. II.A stress section: Eq. StressDef and the final stress expression,
 * orthorhombic cell, S = I) of the context's current orbitals (after
 * hcu_scf, hcu_chfsi_pass or hcu_set_start) with occupations `occ` (host
 * [nspin][nk][ns] doubles; NULL = the occupations of the last
 * hcu_update_occupations / SCF iteration).  The derivative is moved to the
 * Kohn-Sham orbitals and taken with the paper's centred finite-difference
 * gradient (Sec. II.B weights, Bloch wrap):
 *   f^J_a = g sum_k w_k Re sum_mm' U (2 D_m'm - delta_mm') sum_j f_j P_mj conj(G^a_m'j)
 *   sigma_ab = g/|Omega| sum_J sum_mm' U/2 (delta_mm' - 2 D_m'm)
 *              [-2 sum_k w_k Re sum_j f_j Q^ab_mj conj(P_m'j) - delta_ab D_mm']
 * with P = <phi|psi> dV, G^a = <phi|d_a psi> dV, Q^ab = <phi^b|d_a psi> dV,
 * phi^b = sum_T phi(x-R-T) (x-R-T)_b e^{ik.T} (Loewdin coefficients of the
 * orbitals, when used, held fixed: the orbital moves rigidly), g = 2 for
 * nspin = 1 and 1 otherwise, and D the occupation matrix of these orbitals
 * and occupations (complex in general).  The printed expressions carry
 * D_mm' in the first factor; that equals D_m'm whenever D is real (Gamma,
 * k-sets closed under k -> -k) and D_m'm is the exact derivative for complex
 * D.  forces: host [natom][3] doubles, Ha/bohr, zero for atoms without a
 * Hubbard manifold; stress: host [3][3] row-major (a = gradient direction,
 * b = moment direction), Ha/bohr^3.  The context's three filter work blocks
 * of each (spin, k) are overwritten (the next filter recomputes them).
 * Errors: HCU_NOT_BOUND, HCU_INVALID_ARG (NULL output, no occupations yet),
 * HCU_NAN (non-finite occupations or results), HCU_DEVICE. */
hcu_status hcu_hubbard_forces(hcu_ctx* ctx, const double* occ, double* forces);
hcu_status hcu_hubbard_stress(hcu_ctx* ctx, const double* occ, double* stress);

/* Stencil tile shape: tile_x threads along x (== n1: the x halo is taken
 * from the tile itself), tile_yt thread rows of ry points, tile_z planes
 * streamed per workgroup; stencil_ms = measured time of one full-block
 * launch (autotune output). */
typedef struct hcu_tuning {
  int tile_x, tile_yt, ry, tile_z;
  int halo_ring;   /* 1: the y/x halo of a plane is read together with the
                      tile's own queue head, R planes before the plane is
                      computed, and held in an LDS ring of R planes (order-12
                      stencil, at most 4 halo values per thread and 512
                      threads, LDS within 160 KB) */
  double stencil_ms;
} hcu_tuning;
/* Time every admissible tile shape (with and without the halo ring) on the
 * full orbital block of (spin 0, k 0) (contents are not changed) and keep
 * the fastest; shapes the device cannot launch are skipped.  tile_x = 0 in
 * hcu_set_tuning restores the built-in choice.  Errors: HCU_INVALID_ARG for
 * a shape the grid does not admit, HCU_DEVICE if no shape launches. */
hcu_status hcu_autotune(hcu_ctx* ctx, hcu_tuning* best);
hcu_status hcu_set_tuning(hcu_ctx* ctx, const hcu_tuning* t);

/* Turn per-kernel event timing on (1) or off (0); resets the accumulators. */
hcu_status hcu_set_profiling(hcu_ctx* ctx, int on);
/* Accumulated kernel times since profiling was turned on (synchronises). */
hcu_status hcu_get_kernel_times(hcu_ctx* ctx, hcu_kernel_times* t);

/* Results (host outputs, caller-owned buffers). */
hcu_status hcu_get_eigenvalues(const hcu_ctx* ctx, double* eig);    /* [nspin][nk][ns] */
hcu_status hcu_get_occupations(const hcu_ctx* ctx, double* occ);    /* [nspin][nk][ns] */
hcu_status hcu_get_hubbard_occupation(const hcu_ctx* ctx, double* D);   /* D_out */
hcu_status hcu_get_energies(const hcu_ctx* ctx, hcu_energies* e);
/* Orbitals of (spin, ik) into dst (device if on_device, else host), nd x ns
 * column-major in the context precision (complex interleaved at k != 0). */
hcu_status hcu_get_orbitals(hcu_ctx* ctx, int spin, int ik, void* dst, int on_device);
/* Density rho[sigma][nd] (host, double): total for nspin = 1, spin densities
 * for nspin = 2; rho = (2/nspin) sum_k w_k sum_j f_j |x_j|^2. */
hcu_status hcu_get_density(hcu_ctx* ctx, double* rho);
/* The local potential the next H application uses, host double [nd]:
 * V_loc, or with hxc V_loc + V_H[rho_in] + V_x[rho_in] of the current input
 * density rho_in (written to rho_in, host double [nd], when rho_in is not
 * NULL).  Errors: HCU_NOT_BOUND, HCU_INVALID_ARG (NULL V; rho_in without
 * hxc). */
hcu_status hcu_get_potential(hcu_ctx* ctx, double* V, double* rho_in);

/* ------------------------------------------------------------ save / resume
 * Snapshot of the SCF state in a caller-owned host buffer: input occupation
 * matrices and the Pulay history (Sec. II.B mixing), iteration counter and
 * convergence bookkeeping, filter bounds per (spin, k), last eigenvalues,
 * occupations and energies, the orbital blocks and their projections onto
 * the atom-centred functions (left by the last Rayleigh-Ritz rotation, where
 * the next filter starts); with hxc also the input density and the density
 * mixing window.  A context of the same
 * problem (same shape, precision, real/complex type and hxc flag) that loads it
 * continues with hcu_scf_step exactly as the saved one would have.
 * Errors: HCU_NOT_BOUND, HCU_INVALID_ARG (buffer too small, foreign or
 * corrupt state, shape mismatch). */
hcu_status hcu_state_size(const hcu_ctx* ctx, size_t* bytes);
hcu_status hcu_save_state(hcu_ctx* ctx, void* host, size_t bytes);
hcu_status hcu_load_state(hcu_ctx* ctx, const void* host, size_t bytes);

/* ---------------------------------------------------------------- batches
 * Independent problems (cells of different size, each with its spins and
 * k-points) advanced together: in every Chebyshev step the stencil of every
 * (cell, spin, k) block runs as ONE persistent launch that drains a work list
 * of (block, tile, z-chunk, state) items; projections, scatters and the
 * Rayleigh-Ritz steps run per block.  Members must be bound to the same
 * stream and share the block element type (precision, real/complex), the
 * filter degree and n0.  A batch does not own its contexts. */
typedef struct hcu_batch hcu_batch;
hcu_status hcu_batch_create(hcu_ctx* const* ctxs, int n, hcu_batch** out);
void hcu_batch_destroy(hcu_batch* b);
const char* hcu_batch_last_error(const hcu_batch* b);
/* One filter + Rayleigh-Ritz pass on every (member, spin, k) (bounds must be
 * set, e.g. by hcu_lanczos_bounds). */
hcu_status hcu_batch_chfsi_pass(hcu_batch* b);
/* SCF of every member in lockstep (same options; a converged member stops
 * taking part); reps[i] is member i's report.  HCU_NOT_CONVERGED if any
 * member reached max_iter. */
hcu_status hcu_batch_scf(hcu_batch* b, const hcu_scf_opts* opts, hcu_scf_report* reps);

/* ------------------------------------------------------------ learned guess
 * A start for the Hubbard occupation matrices predicted from each site's
 * environment, in place of the isolated-atom average occupation with which
 * the paper begins the SCF (Sec. II.B, initial guess of the occupation
 * matrices).
 *
 * Site descriptor of Hubbard atom I (32 entries per species, table order):
 *   G[32 S + k] = sum over atoms J of species S and lattice images with
 *   0 < r < 6.5 bohr of exp(-(r - mu_k)^2 / (2 * 0.25^2)) * (cos(pi r/6.5)+1)/2,
 *   mu_k = 1 + 5.5 k / 31 bohr, r = |R_J + T - R_I|.
 * Site frame flag: 1 when the site's apical neighbours without a Hubbard
 * manifold (r < 4.5 bohr, |dz| < 1 bohr) lie along (1, -1, 0), i.e. the
 * rutile sublattice rotated by 90 degrees about z; such a site's occupation
 * matrix is learned in the rotated frame D_loc = M D M^T, M the signed
 * permutation of the real d orbitals (xy, yz, z^2, xz, x^2-y^2) under
 * (x, y, z) -> (y, -x, z).
 * Density shells: c_k = sum_x rho(x) g_k(x) / sum_x g_k(x), g_k(x) = sum over
 * images of exp(-(|x - R_I - T| - r_k)^2 / (2 * 0.25^2)), r_k = 0.5 + 3.5 k/14
 * (k = 0..14), rho summed over spins. */

/* desc: device float [nhub][32 * nspecies]; frame: host int [nhub]. */
hcu_status hcu_descriptor(hcu_ctx* ctx, float* desc, int* frame);
/* Shell averages of the density of the current orbitals and occupations
 * (after an SCF or hcu_update_occupations): host double [nhub][15]. */
hcu_status hcu_shell_density(hcu_ctx* ctx, double* out);

/* Training targets of ctx's Hubbard sites after an SCF: host float
 * [nhub][30], the 15 upper-triangle entries (row-major) of the spin-averaged
 * occupation matrix in the site frame, then the 15 density shells. */
hcu_status hcu_site_targets(hcu_ctx* ctx, float* out);

/* MLP dims[0] -> dims[1] -> ... -> dims[nlayers], SiLU (z / (1 + e^-z))
 * after every layer but the last.  Parameters: FP32, flat, per layer the
 * weight W [dims[l+1]][dims[l]] (row-major) followed by the bias.  Inputs
 * and targets are standardised with per-column means and deviations held by
 * the object.  Training: loss = mean over rows and outputs of
 * (y - t_standardised)^2, gradients by the backward pass, Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected).  Rows of X / T are selected by a
 * device index array (NULL = rows 0..batch-1); X [rows][dims[0]] and T
 * [rows][dims[L]] are device FP32.  Inference in FP32, or with BF16 weights
 * and activations and FP32 accumulation (bf16 = 1).  An object is bound to
 * a caller-provided workspace and stream like a context. */
typedef struct hcu_mlp hcu_mlp;
hcu_status hcu_mlp_create(const int* dims, int nlayers, int max_batch, hcu_mlp** out);
void hcu_mlp_destroy(hcu_mlp* m);
const char* hcu_mlp_last_error(const hcu_mlp* m);
hcu_status hcu_mlp_param_count(const hcu_mlp* m, int64_t* n);
hcu_status hcu_mlp_workspace_size(hcu_mlp* m, size_t* bytes);
hcu_status hcu_mlp_bind(hcu_mlp* m, void* dev, size_t bytes, void* hip_stream);
/* host float [param_count]; resets the Adam moments */
hcu_status hcu_mlp_set_params(hcu_mlp* m, const float* params);
hcu_status hcu_mlp_get_params(hcu_mlp* m, float* params);
/* host float vectors of lengths dims[0], dims[0], dims[L], dims[L] */
hcu_status hcu_mlp_set_scaling(hcu_mlp* m, const float* in_mean, const float* in_sd, const float* out_mean,
                               const float* out_sd);
hcu_status hcu_mlp_get_scaling(hcu_mlp* m, float* in_mean, float* in_sd, float* out_mean, float* out_sd);
/* scaling from the column statistics of `rows` device rows (deviations
 * below 1e-6 are replaced by 1) */
hcu_status hcu_mlp_fit_scaling(hcu_mlp* m, const float* X, const float* T, int rows);
/* Y (device float [batch][dims[L]]) = de-standardised network output */
hcu_status hcu_mlp_forward(hcu_mlp* m, const float* X, int batch, float* Y, int bf16);
/* loss (host) and its gradient (host float [param_count]) at the current
 * parameters, without an update */
hcu_status hcu_mlp_gradient(hcu_mlp* m, const float* X, const float* T, const int* idx, int batch, float* grad,
                            double* loss);
/* one Adam step; *loss (if non-NULL) is the loss before the step */
hcu_status hcu_mlp_train_step(hcu_mlp* m, const float* X, const float* T, const int* idx, int batch, float lr,
                              double* loss);
/* Descriptors of ctx's Hubbard sites -> network -> occupation matrices
 * (first 15 outputs: upper triangle of D_loc, row-major), rotated back,
 * symmetrised, spectrum clipped to [0, 1], set as the context's D for every
 * spin.  outputs (optional, host float [nhub][dims[L]]) receives the raw
 * physical outputs (entries 15..29: predicted density shells). */
hcu_status hcu_mlp_guess(hcu_ctx* ctx, hcu_mlp* m, int bf16, float* outputs);

/* ------------------------------------------------------- no allocation
 * For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the contractions of hcu_gram without a context,
 *   S = Y^H Y dv,  Hs = Y^H HY dv   (ncol x ncol, column-major doubles,
 *   complex interleaved; diagonal 64 x 64 (complex: 32 x 32) tiles
 *   symmetrised, the rest mirrored, as hcu_gram),
 * with the same kernels and summation order as hcu_gram.  Y and HY are
 * device blocks of ncol states, nd grid values each, leading dimension
 * ld >= nd, element type double (precision HCU_FP64) or float (HCU_MIXED),
 * complex interleaved when is_complex.  S and Hs are caller-owned device
 * buffers.  The work is queued on `stream` (NULL = default stream) and the
 * call returns without waiting; nothing is allocated or freed.
 * Scratch: split-K partial sums and the tile list live in a fixed 80 MiB
 * device array that the library holds on each GPU it runs on until the
 * process ends; every call on one GPU uses the same array, so calls that
 * overlap on one GPU race (serialise them).  Each call rewrites all the
 * scratch it reads.  The first call on a device looks up the array's
 * device address (hipGetSymbolAddress).
 * Errors (nothing is queued): HCU_INVALID_ARG (null pointer, ncol < 1,
 * nd < 1, ld < nd, dv <= 0, unknown precision); HCU_OOM when the
 * contraction's partial sums exceed the 80 MiB (about ncol > 3200 real or
 * > 2200 complex on any grid); HCU_DEVICE for a HIP error. */
hcu_status hcu_gram_noalloc(const void* Y, const void* HY, int ncol, int64_t nd, int64_t ld, int precision,
                            int is_complex, double dv, double* S, double* Hs, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HUBBARD_CHFSI_H */
