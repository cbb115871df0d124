/*
 * qhp.h -- C ABI of the MI355X ring-polymer MD / adaptive quantum thermal bath library.
 *
 * Method: Ple, Mauger, Adjoua, Jaffrelot-Inizan, Lagardere, Huppert & Piquemal,
 * "Routine Molecular Dynamics Simulations Including Nuclear Quantum Effects: from Force
 * Fields to Machine Learning Potentials" (2022).
 *
 * A ring polymer of P replicas ("beads") of an N-atom system of flexible 3-site waters.
 * Bead positions x_i (i = 0..P-1) are propagated in scaled normal modes (Sec. "Ring-Polymer
 * Molecular Dynamics": eqs. isomorphism_RPMD, matrix_free_RP, beads_positions,
 * force_normal_modes) with the BAOAB splitting of the TRPMD equations of motion
 * (Sec. "Integration Scheme", eq. RPMD_EOM). For P = 1 the coloured-noise adaptive quantum
 * thermal bath may replace the white noise (Secs. "Adaptive Quantum Thermal Bath", "adQTB":
 * eqs. eq_langevin, Cff_qtb, QTB_spectra; SIMPLE adaptation and the gamma_min clamp).
 *
 * Units are the caller's, as long as they are consistent; the library is written for
 * Angstrom, fs, e, kcal/mol, with masses in kcal/mol * fs^2 / Angstrom^2.
 *
 * Layouts at the boundary (row-major, FP64):
 *   positions, velocities, forces  [P][N][3]
 *   per-bead energies              [P][QHP_NTERMS]
 * Molecules are three consecutive atoms O, H, H (atom 3w is the oxygen of water w).
 *
 * Ownership: the caller owns every pointer it passes. The library copies what it needs
 * before returning from qhp_create and keeps no caller pointer afterwards. Arrays passed
 * to the other calls are read or written during the call only; `mem_kind` says whether
 * they are host memory (QHP_MEM_HOST) or device memory on the context's GPU
 * (QHP_MEM_DEVICE). All GPU work is queued on the context's stream; calls that return
 * data to host memory synchronise that stream, calls writing device memory do not
 * (use qhp_sync).
 *
 * Errors: every call returns QHP_OK (0) or a negative code; qhp_last_error(ctx) gives a
 * message for the last failure on that context. No C++ exception crosses this ABI.
 * A context must be used from one host thread at a time.
 */
#ifndef QHP_H
#define QHP_H

#include <stdint.h>

#if defined(__GNUC__)
#define QHP_API __attribute__((visibility("default")))
#else
#define QHP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define QHP_OK            0
#define QHP_EINVAL       -1   /* bad argument (null pointer, sizes, cutoff >= L/2, ...)   */
#define QHP_ENOMEM       -2   /* device allocation failed or a capacity was exceeded      */
#define QHP_EDEVICE      -3   /* HIP runtime error; the HIP message is in qhp_last_error  */
#define QHP_ENONFINITE   -4   /* non-finite input or state                                */
#define QHP_EUNSUPPORTED -5   /* valid request the library does not implement            */

/* memory kinds */
#define QHP_MEM_HOST   0
#define QHP_MEM_DEVICE 1

/* precision of the real-space pair interactions (everything else is FP64) */
#define QHP_FP64        0
#define QHP_FP32_PAIRS  1   /* pair forces in FP32 from FP64 displacements; FP64 sums */

/* execution layout */
#define QHP_BATCHED 0   /* all beads of a step in one launch per kernel, bead innermost */
#define QHP_PLAIN   1   /* one launch per bead and kernel, as a per-replica MD code   */

/* thermostat */
#define QHP_TRPMD 0     /* white-noise Langevin on every normal mode                 */
#define QHP_ADQTB 1     /* adaptive quantum thermal bath (requires P = 1)             */

/* free ring-polymer step of the splitting (Sec. "Integration Scheme") */
#define QHP_BAOAB 0     /* exact rotation of each internal mode                      */
#define QHP_BCOCB 1     /* its Cayley form (implicit midpoint rule): stable for any
                           omega_n dt, after Korol, Bou-Rabee and Miller              */

/* adQTB adaptation (Sec. "Computation of the adQTB Spectra and Adaptation Procedure") */
#define QHP_QTB_SIMPLE 0 /* gamma <- gamma - A_gamma Delta_FDT                        */
#define QHP_QTB_RATIO  1 /* gamma <- Re<C_vF> / (m <C_vv>), running means over tau    */

/* per-bead energy terms */
#define QHP_E_BOND       0
#define QHP_E_ANGLE      1
#define QHP_E_COUL_REAL  2
#define QHP_E_LJ         3
#define QHP_E_COUL_EXCL  4
#define QHP_E_COUL_SELF  5
#define QHP_E_COUL_RECIP 6
#define QHP_NTERMS       7

/* Parameters of a run. Host pointers; copied by qhp_create. */
typedef struct qhp_params {
  int32_t n_atoms;          /* N, a multiple of 3                                         */
  int32_t n_beads;          /* P in 1..64 (eq. isomorphism_RPMD); a count that is not a
                               power of two runs in the lanes of the next one, whose extra
                               "phantom" beads carry no mode and are never reported     */
  double box[3];            /* orthorhombic box edges                                     */
  int32_t n_types;          /* atom types (1..8)                                          */
  const int32_t* type;      /* [N] type of each atom                                      */
  const double* mass;       /* [N] mass; must be equal within a type                      */
  const double* charge;     /* [N]                                                        */
  const double* lj_sigma;   /* [n_types]; pair sigma = (s_i + s_j) / 2                    */
  const double* lj_epsilon; /* [n_types]; pair epsilon = sqrt(e_i e_j)                    */
  double bond_r0, bond_k;          /* E = k/2 (r - r0)^2 for both O-H bonds              */
  double angle_theta0, angle_k;    /* E = k/2 (theta - theta0)^2 for H-O-H (radians)     */
  double coulomb;           /* Coulomb constant C in E = C q_i q_j / r                    */
  double ewald_alpha;       /* Ewald splitting parameter alpha                            */
  double cutoff;            /* real-space cutoff rc (< half the smallest box edge)        */
  double skin;              /* neighbour-list skin: r_list = rc + skin                    */
  int32_t pme_grid[3];      /* SPME grid, each in 8..128 and >= 2*pme_order: powers of
                               two (the tuned kernels), or multiples of 8 with prime
                               factors 2, 3, 5, 7 (a plainer, slower transform path)   */
  int32_t pme_order;        /* B-spline order n: 4, 5, 6 or 8 (3 and 7: EUNSUPPORTED)    */
  int32_t precision;        /* QHP_FP64 | QHP_FP32_PAIRS                                  */
  int32_t exec;             /* QHP_BATCHED | QHP_PLAIN                                    */
  int32_t thermostat;       /* QHP_TRPMD | QHP_ADQTB                                      */
  double dt;                /* time step                                                  */
  double kT;                /* k_B T                                                      */
  double hbar;              /* reduced Planck constant                                    */
  double gamma_centroid;    /* TRPMD: centroid friction gamma_0                          */
  double trpmd_c;           /* TRPMD: internal-mode friction max(gamma_0, c * omega_n)   */
  uint64_t seed;            /* Philox-4x64-10 key word 0                                  */
  double qtb_gamma0;        /* adQTB: friction gamma_0                                   */
  int32_t qtb_nseg;         /* adQTB: segment length N_seg: 16..1024, a multiple of 8
                               whose prime factors are 2, 3, 5, 7 (powers of two take
                               the fastest transforms)                                  */
  double qtb_adapt_rate;    /* adQTB: SIMPLE rate A_gamma (same for every type)          */
  double qtb_gamma_min_frac;/* adQTB: gamma_min = frac * gamma_0 (paper default 0.01)    */
  int32_t qtb_classical;    /* adQTB test switch: Theta(omega) = kT (white-noise limit)  */
  int32_t nbr_capacity;     /* initial neighbours per atom a row holds; 0 = sized from
                               the density. Rows grow by themselves when a build finds
                               more (qhp_eval, qhp_step, ...); see qhp_nlist_stats      */
  int32_t use_graph;        /* 1: replay each step as one captured HIP graph; 0: launch   */
  /* Multiple time stepping with ring-polymer contraction (Sec. "Multi-timestep Methods",
   * paragraphs "Ring-polymer Contractions" and "Path-integral RESPA integrator"):
   * V = V_f + V_s with V_f = O-H bonds + H-O-H angles on the P beads and V_s = every other
   * term on P~ contracted beads x~_j = Q_0 + sqrt(P~) sum_{0<n<P~} T~_jn Q_n, T~ the
   * transfer matrix of P~ beads (eq. beads_positions with P~ in place of P: the P~ lowest
   * modes, each with unit weight). BAOAB-RESPA: one outer step is Bs(n dt/2) [Bf(dt/2)
   * A(dt/2) O(dt) A(dt/2) Bf(dt/2)]^n Bs(n dt/2) with n = respa_nalt. Both need exec =
   * QHP_BATCHED and thermostat = QHP_TRPMD (else QHP_EUNSUPPORTED). */
  int32_t rpc_beads;        /* P~ in 1..P (any count; 0 = P, no contraction)             */
  int32_t respa_nalt;       /* n: inner steps per outer step, 1..64; 0 = 1               */
  int32_t integrator;       /* QHP_BAOAB | QHP_BCOCB                                      */
  int32_t qtb_adapt_scheme; /* QHP_QTB_SIMPLE | QHP_QTB_RATIO (every type; see below)     */
  double qtb_tau;           /* RATIO: running-mean time tau (every type; see below), > 0.
                               The means start from zero; where <C_vv> <= 0 gamma keeps
                               its value; the gamma_min clamp follows either scheme.    */
  /* Alchemical coupling of a solute (Sec. "Hydration free energies": the solute is
   * decoupled from the solvent by scaling its charges down, then its van der Waals
   * interactions through a soft-core potential). The solute is the set of atoms whose type
   * has type_soft = 1. Every solute charge is multiplied by lambda_elec in all
   * electrostatic terms (so solute-solvent terms scale with lambda_elec and the solute's
   * internal ones with its square). The LJ term of a pair with exactly one solute atom
   * takes Beutler's soft-core form lambda_vdw 4 eps [1/D^2 - 1/D], D = sc_alpha
   * (1 - lambda_vdw) + (r/sigma)^6; solute-solute and solvent-solvent pairs keep the plain
   * form. type_soft = NULL: no solute, and the three numbers below are ignored.         */
  const int32_t* type_soft; /* [n_types] 0/1, or NULL                                   */
  double lambda_elec;       /* in [0, 1]; 1 = fully coupled                               */
  double lambda_vdw;        /* in [0, 1]; 1 = fully coupled                               */
  double sc_alpha;          /* soft-core alpha >= 0 (0.5 in the free-energy workload)    */
  /* Test-only harmonic tether (statistical checks against the closed-form P-bead
   * harmonic oscillator of Sec. "Path Integrals and Ring Polymer Molecular Dynamics"):
   * V += (k_h / 2) |x_b - a|^2 for every atom at every bead b, a = the atom's anchor;
   * its energy is added to the bond term and its force to grad V. 0 = off. Not
   * available with RESPA / contraction, parameter gradients or Hessian-vector products
   * (QHP_EUNSUPPORTED). */
  double tether_k;          /* k_h >= 0, kcal/mol/A^2                                     */
  const double* tether_anchor; /* [N][3] anchors (host, copied at creation) when k_h > 0  */
  /* adQTB adaptation per atom type (Sec. "Computation of the adQTB Spectra and Adaptation
   * Procedure": every type z has its own running-mean time tau_z, and the two schemes may
   * be combined, e.g. SIMPLE for a solute's types and RATIO for the solvent's). A type's
   * update reads only its own spectra. NULL: every type takes qtb_adapt_scheme and
   * qtb_tau. Host arrays, read at creation. Bad entries: QHP_EINVAL.                    */
  const int32_t* qtb_scheme_of; /* [n_types] QHP_QTB_SIMPLE | QHP_QTB_RATIO, or NULL    */
  const double* qtb_tau_of;     /* [n_types] tau_z, > 0 for RATIO types, or NULL        */
} qhp_params;

typedef struct qhp_ctx qhp_ctx;

/* Create a context on the current HIP device (the set-up of Secs. "Ring-Polymer Molecular
 * Dynamics" and "Integration Scheme": transfer matrix of eq. matrix_free_RP, mode
 * frequencies, per-mode BAOAB coefficients; the SPME influence function of the Ewald sum
 * the force field uses). `stream` is a hipStream_t; all work of the
 * context is queued on it (NULL: the library creates a private non-blocking stream).
 * Validates `p` (QHP_EINVAL; QHP_EUNSUPPORTED for valid settings the library does not run:
 * B-spline order 3 or 7), allocates device state
 * (QHP_ENOMEM) and precomputes the normal-mode transfer matrix, mode frequencies,
 * thermostat and A-block coefficients and the SPME influence function.
 * The state is undefined until qhp_set_state. */
QHP_API int qhp_create(const qhp_params* p, void* stream, qhp_ctx** out);
/* Wait for the context's queued work, free its device memory and the context. */
QHP_API int qhp_destroy(qhp_ctx* ctx);

/* Stateless evaluation of V on every bead (eq. PI_potential summands): `pos` [P][N][3]
 * in the orthorhombic box `box` [3] -> `energy` [P][QHP_NTERMS] (nullable) and `forces` =
 * -grad V [P][N][3] (nullable). The box is fixed per context (cell grid, SPME influence
 * function and tables depend on it): `box` must equal the context's edges to 1e-12
 * relative, else QHP_EINVAL; NULL means the context's box. Builds the centroid neighbour
 * list of these positions (Sec. "Massively Parallel Implementation": neighbours are found
 * on ring-polymer centroids and shared by all beads), growing its rows if they are too
 * short. The full potential on all P beads, whatever rpc_beads and respa_nalt are. Does
 * not change the propagated state (a later step rebuilds the list if it must).
 * Synchronises the stream for either memory kind (the list and state flags are read). */
QHP_API int qhp_eval(qhp_ctx* ctx, const double* pos, const double box[3], double* energy,
                     double* forces, int mem_kind);

/* Gradients of the summed bead energies E = sum_b V(x_b) (eq. PI_potential without the
 * 1/P) at `pos` [P][N][3] with respect to the force-field parameters: `dq` [N] per-atom
 * charges (real-space, exclusion, self and reciprocal terms; the reciprocal part is the
 * SPME-interpolated potential at the atom), `deps` [n_types] and `dsig` [n_types] per-type
 * LJ epsilon and sigma (Lorentz-Berthelot combination; the epsilon derivative of a type
 * with epsilon = 0 is unbounded and returned as 0). Pair terms: with precision =
 * QHP_FP32_PAIRS, r, 1/r, erfc(alpha r) and exp(-alpha^2 r^2) are FP32 values computed
 * from the FP64 displacement and every product and sum is FP64; else all FP64. Builds
 * the list of these positions like qhp_eval and leaves the
 * propagated state alone. QHP_EUNSUPPORTED for exec = QHP_PLAIN. */
QHP_API int qhp_param_grad(qhp_ctx* ctx, const double* pos, double* dq, double* deps,
                           double* dsig, int mem_kind);

/* Hessian-vector product of every bead's potential at `pos` [P][N][3] along `dir`
 * [P][N][3]: out[b] = (d^2 V / dx^2)(x_b) dir_b, [P][N][3]. Exact analytic second
 * derivatives (all terms: bonds, angle and exclusion by forward differentiation of their
 * gradient; real-space pairs by the pair Hessian blocks; the SPME sum by spreading the
 * tangent charge density, one more convolution and a gather with second-derivative
 * B-splines), pair terms at `precision` as for qhp_param_grad, on the list of these
 * positions.
 * The potential is the truncated one: pairs crossing the cutoff contribute no delta
 * terms. With `dq` [N], `deps` [n_types], `dsig` [n_types] (all three or none), also the
 * mixed derivatives d(dir . grad E)/d(q, epsilon, sigma) of the summed bead energies
 * (as qhp_param_grad differentiates E): the parameter gradient of a loss on forces.
 * Leaves the propagated state alone; the first call allocates a second SPME grid and an
 * output buffer that the context keeps. QHP_EUNSUPPORTED for exec = QHP_PLAIN. */
QHP_API int qhp_hvp(qhp_ctx* ctx, const double* pos, const double* dir, double* out,
                    double* dq, double* deps, double* dsig, int mem_kind);

/* Set the propagated state from bead positions and bead velocities [P][N][3] and the
 * step counter (which indexes the noise streams). Computes the normal modes
 * Q = T^T x / sqrt(P), P_n = m T^T v / sqrt(P) and the forces of this state (under
 * RESPA / contraction: V_f on the beads and V_s on the contracted beads); for adQTB
 * `step` must be a multiple of N_seg, gamma is reset to gamma_0 and the coloured noise
 * of the current segment is generated. */
QHP_API int qhp_set_state(qhp_ctx* ctx, const double* pos, const double* vel, int64_t step, int mem_kind);

/* Read the state back as bead positions x = sqrt(P) T Q (eq. beads_positions) and bead
 * velocities v = sqrt(P) T P_n / m [P][N][3] (either nullable), with the momenta after
 * the step's final half kick. */
QHP_API int qhp_get_state(qhp_ctx* ctx, double* pos, double* vel, int64_t* step, int mem_kind);

/* Advance `nsteps` BAOAB steps (Sec. "Integration Scheme": B(dt/2) A(dt/2) O(dt) A(dt/2)
 * B(dt/2), one force evaluation each). For adQTB the spectra, SIMPLE (or RATIO)
 * adaptation, clamp and the next noise segment are computed after the last step of every
 * segment (Secs. "Colored Noise Generation", "Computation of the adQTB Spectra and
 * Adaptation Procedure"). `energy` (nullable) receives the per-bead energies of the final
 * state [P][QHP_NTERMS]. The centroid list is rebuilt on the device whenever the skin rule
 * asks; if a build finds more neighbours than a row holds, the call restarts from the
 * state it began with (kept on the device), with longer rows, so its result never depends
 * on the row length. Returns QHP_ENONFINITE if the state became non-finite and
 * QHP_ENOMEM only if the rows cannot grow (device memory).
 * Synchronises the stream at the end (the list and state flags are read).
 * With respa_nalt = n > 1 or rpc_beads = P~ < P, `nsteps` counts outer steps of n inner
 * steps each; the step counter (qhp_get_state, noise counter) counts inner steps. The
 * energies are then: bond and angle columns on the P beads, the other columns on rows
 * 0..P~-1 (the contracted beads) and zero below, so that the estimator of the contraction
 * equation is sum(bond, angle)/P + sum(others)/P~. */
QHP_API int qhp_step(qhp_ctx* ctx, int32_t nsteps, double* energy, int mem_kind);

/* Kinetic energy sum_n P_n^2 / 2m and free ring-polymer spring energy
 * sum_n m omega_n^2 Q_n^2 / 2 of the current state (the two quadratic terms of the
 * ring-polymer Hamiltonian in normal modes, Sec. "Ring-Polymer Molecular Dynamics";
 * host outputs). */
QHP_API int qhp_mode_energies(qhp_ctx* ctx, double* kinetic, double* spring);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): qhp_mode_energies with the two sums written to device
 * memory `out` [2] (kinetic, spring) on the context's stream, without synchronising and
 * without allocating. The per-block partial sums go to a 1 MiB file-scope device array
 * that every call on a GPU shares (at most 65,536 blocks of 256 / P atoms, i.e. N P up to
 * 16.7 million bead-atoms; beyond that QHP_ENOMEM); they are added in a fixed order, so the
 * result does not depend on block scheduling. Calls that overlap on one GPU (two streams,
 * or two host threads) race on that array and must be serialised by the caller. */
QHP_API int qhp_mode_energies_noalloc(qhp_ctx* ctx, double* out);

/* The centroid pair list of the last build (Sec. "Massively Parallel Implementation":
 * pairs whose centroid distance is below rc + skin), canonical form: pairs (i, j), i < j,
 * different molecules, sorted by i then j, written to `pairs` [*npairs][2] (host).
 * If `capacity` (in pairs) is too small, *npairs is set and QHP_ENOMEM returned. */
QHP_API int qhp_nlist_export(qhp_ctx* ctx, int32_t* pairs, int64_t capacity, int64_t* npairs);

/* Neighbour-list bookkeeping of the centroid list (Sec. "Massively Parallel
 * Implementation"): number of list builds since qhp_create, the largest neighbour count
 * of the last build and the current row length (host outputs). */
QHP_API int qhp_nlist_stats(qhp_ctx* ctx, int64_t* builds, int32_t* max_count, int32_t* capacity);

/* Gaussian noise as the kernels draw it (the O step's white noise, Sec. "Integration
 * Scheme"; the adQTB white noise, Sec. "Colored Noise Generation"; Philox-4x64-10 of
 * Salmon et al. 2011, key (seed, stream), Box-Muller):
 * stream 5 = TRPMD O-step noise of step `step`, out [P][N][3] indexed [mode][atom][xyz];
 * stream 6 = adQTB white noise of global step `step`, out [N][3]. Device computation,
 * host output. */
QHP_API int qhp_noise_export(qhp_ctx* ctx, int32_t stream, int64_t step, double* out);

/* Alchemical runs (type_soft set): change the couplings of the propagated system
 * (both in [0, 1]; the solute charges are rescaled from the ones given at creation).
 * QHP_EINVAL without a solute. Takes effect for the next step or evaluation. */
QHP_API int qhp_set_lambda(qhp_ctx* ctx, double lambda_elec, double lambda_vdw);

/* qhp_eval at other couplings, for the energy differences of free-energy estimators
 * (Sec. "Hydration free energies": each window's samples are evaluated in the neighbouring
 * states): `pos` [P][N][3] -> `energy` [P][QHP_NTERMS] (nullable) and `forces`
 * (nullable) of the system at (lambda_elec, lambda_vdw). The propagated state and its
 * couplings are left alone. QHP_EINVAL without a solute. */
QHP_API int qhp_eval_lambda(qhp_ctx* ctx, const double* pos, double lambda_elec,
                            double lambda_vdw, double* energy, double* forces, int mem_kind);

/* Bennett acceptance ratio (Sec. "Hydration free energies", eqs. PIBAR1-PIBAR2): with
 * du_a[k] = U_B - U_A at the n_a configurations sampled in state A and du_b[k] =
 * U_B - U_A at the n_b configurations of state B (host arrays), solves the self-consistent
 *   dF = C + (1/beta) ln( <f(-du + C)>_B / <f(du - C)>_A ),  C = dF + (1/beta) ln(n_b/n_a),
 * f(x) = 1/(1 + exp(beta x)). The pair holds exactly when sum_B f(C - du) = sum_A f(du - C),
 * a monotone equation in C with one root, found by safeguarded Newton steps to 1e-13
 * relative (at most 500). *dF = Delta F_AB = (1/beta) ln(Z_A/Z_B), the paper's sign. PI-BAR takes U = the bead average of V
 * (eq. PI_potential); the single-bead estimator V at one bead. Host code only: needs no
 * device. QHP_EINVAL for null pointers, n_a or n_b < 1, beta <= 0; QHP_ENONFINITE for
 * non-finite input or no convergence. `iterations` is nullable. */
QHP_API int qhp_bar(const double* du_a, int64_t n_a, const double* du_b, int64_t n_b,
                    double beta, double* dF, int32_t* iterations);

/* A group of contexts stepped together (batched uneven instances: free-energy windows of
 * different sizes and bead counts). qhp_group_step advances every member by `nsteps`
 * steps; each step of all members is one captured HIP graph, launched once, in which each
 * member's kernels form an independent branch (on its own stream, which must differ from
 * the other members' for the branches to overlap). The group keeps pointers to the
 * members, which the caller keeps alive and does not step otherwise while the group is in
 * use; members need use_graph = 1 and a state (qhp_set_state) before the first group
 * step. qhp_group_create copies the member list; QHP_EINVAL for n < 1, a null member or a
 * member twice. A member's qhp_set_lambda or qhp_set_state is picked up by recapturing at
 * the next group step. Work is queued on the first member's stream. */
typedef struct qhp_group qhp_group;
QHP_API int qhp_group_create(qhp_ctx* const* members, int32_t n, qhp_group** out);
QHP_API int qhp_group_step(qhp_group* group, int32_t nsteps);
QHP_API int qhp_group_destroy(qhp_group* group);
QHP_API const char* qhp_group_last_error(qhp_group* group);

/* Launch-shape autotuner: times the context's force kernels on its current beads (`reps`
 * launches per candidate, HIP events on the context's stream; the propagated state is not
 * changed). First the SPME spreading block: 1, 2, 4, 8 or 16 beads per block (up to the
 * beads the pass covers) times 1, 2, 4 or 8 grid tiles of 8^3 points along z; with two or
 * more complex grid slots the spreading fused with the x transform uses these as its slots
 * per block (beads / 2, at least 1) and the z extent of its rectangle of grid lines. Then,
 * for square 32^2 or 64^2 y-z planes, the plane kernel of the y and z transforms with 1, 2,
 * 4 or 8 complex grid slots per block (at most 2 at 64^2) against three one-axis passes
 * (reported as -1). Then, where the FP32 pair kernel applies (precision = QHP_FP32_PAIRS
 * and 2 (cutoff + skin) below the shortest box edge), 2, 4 or 8 atoms per block of that
 * kernel (one wavefront per atom). Keeps the fastest of each for the context's later
 * launches and returns them in `spread_beads`, `spread_ztiles`, `fft_slots` and
 * `pair_atoms` (all nullable; 0 = no choice applies). Needs a state (qhp_set_state).
 * Results do not depend on the choice beyond the order of floating-point additions in the
 * SPME sums; the pair kernel's results do not depend on it at all. */
QHP_API int qhp_autotune(qhp_ctx* ctx, int32_t reps, int32_t* spread_beads,
                         int32_t* spread_ztiles, int32_t* fft_slots, int32_t* pair_atoms);

/* Set the same launch shapes by hand (the autotuner's search space): spreading beads per
 * block (0 = min(P, 8), else a power of two <= 16, capped at the beads of the pass),
 * spreading 8^3 tiles along z (0 = 1, else a power of two <= 8, capped so that beads x
 * tiles <= 16 and at the grid's tiles), y-z plane kernel slots per block (0 = default,
 * -1 = one-axis passes, else a power of two <= 8, capped at 2 for 64^2 planes and at the
 * grid's slots; ignored where no plane kernel applies), FP32 pair kernel atoms per block
 * (0 = 4, else 2, 4 or 8). QHP_EINVAL otherwise. */
QHP_API int qhp_set_launch(qhp_ctx* ctx, int32_t spread_beads, int32_t spread_ztiles,
                           int32_t fft_slots, int32_t pair_atoms);

/* adQTB (Sec. "adQTB": the adapted friction gamma_z(omega) of each atom type):
 * gamma_z(omega_k), omega_k = pi k / (N_seg dt), k = 0..N_seg, for every type:
 * [n_types][N_seg + 1] (host). qhp_qtb_set_gamma replaces it and regenerates the current
 * segment's coloured noise from it. */
QHP_API int qhp_qtb_get_gamma(qhp_ctx* ctx, double* gamma);
QHP_API int qhp_qtb_set_gamma(qhp_ctx* ctx, const double* gamma);
/* adQTB: the coloured noise of the current segment [N_seg][N][3] (Sec. "Colored Noise
 * Generation") and the type-averaged Delta_FDT of the last completed segment
 * [n_types][N_seg + 1] (eq. QTB_spectra; host outputs). */
QHP_API int qhp_qtb_get_noise(qhp_ctx* ctx, double* noise);
QHP_API int qhp_qtb_get_delta(qhp_ctx* ctx, double* delta);

/* Per-kernel timing (measurement of the step's phases, not part of the method): HIP
 * events recorded on the context's stream around every launch of the selected kernel
 * class (0 = off); steps are then launched kernel by kernel on one stream.
 * qhp_profile_read returns the summed milliseconds and the number of launches since
 * enabling. */
#define QHP_PROF_OFF    0
#define QHP_PROF_PAIR   1
#define QHP_PROF_SPREAD 2
#define QHP_PROF_FFT    3
#define QHP_PROF_GATHER 4
#define QHP_PROF_NM     5
QHP_API int qhp_profile(qhp_ctx* ctx, int which);
QHP_API int qhp_profile_read(qhp_ctx* ctx, double* ms, int64_t* launches);

/* Wait for the context's queued work (results written to device memory are then valid). */
QHP_API int qhp_sync(qhp_ctx* ctx);
/* Message of the last failure on the context (valid until its next call). */
QHP_API const char* qhp_last_error(qhp_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* QHP_H */
