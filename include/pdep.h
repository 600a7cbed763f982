/*
 * pdep.h -- C ABI of the MI355X PDEP chi0 library (libpdep.so).
 *
 * The library applies the static independent-particle response chi0bar of a
 * Kohn-Sham system to blocks of trial potentials through density-functional
 * perturbation theory, and finds the PDEP eigenpairs of chi0bar by block Davidson
 * (Govoni & Galli, "Large scale GW calculations", Sec. 2.3: the Sternheimer equation
 * Eq. stern, the density response Eq. deltani and the projected polarizability
 * Eq. chiisamatrixinpdep; the spectral form of Eq. eigendecompzerofreq).
 *
 * Model and conventions (all calls):
 *  - Hartree atomic units, e^2 = 1.  The paper writes Rydberg units; dielectric
 *    eigenvalues are dimensionless and do not depend on the choice.
 *  - Orthorhombic cell with edges L[3] (bohr), FFT grid n[3], volume Omega.
 *    Grid points r = (ix Lx/nx, iy Ly/ny, iz Lz/nz); real-space arrays are C order
 *    (ix slowest, iz fastest), length N_g = nx*ny*nz.
 *  - Wavefunction basis S: all G = 2 pi (mx/Lx, my/Ly, mz/Lz) with
 *    1/2 |G|^2 <= ecut (the plane-wave expansion and cutoff of Sec. 2.1), listed
 *    lexicographically in (mx, my, mz), mz fastest.  N_pw = |S|.
 *    S' = S without G = 0 (N_pw' = N_pw - 1) is the space of the PDEP potentials.
 *  - Transforms: Inv(c)(r) = sum_{G in S} c_G exp(iG.r);
 *                Fwd(f)(G) = N_g^-1 sum_r f(r) exp(-iG.r).
 *  - Hamiltonian: H = 1/2|G|^2 + Fwd(V_loc * Inv(.)) restricted to S (a local
 *    potential only; products alias on the grid exactly as the transforms make them).
 *  - Occupied orbitals: the N_v lowest eigenvectors c_v of H, normalised to
 *    sum_G |c_vG|^2 = 1, doubly occupied (two spins, Gamma point only).
 *  - chi0bar phi for phi on S' (Hermitian-symmetric: phi(-G) = conj phi(G), so the
 *    potential is real in r):  phi~ = sqrt(4 pi)/|G| phi, dV = Re Inv(phi~),
 *    solve P_c (H - e_v) P_c dc_v = -P_c Fwd(dV u_v) for every v (u_v = Inv(c_v)),
 *    dn = (4/Omega) Re sum_v conj(u_v) Inv(dc_v), result sqrt(4 pi)/|G| Fwd(dn) on S'.
 *  - Complex arrays are interleaved (re, im) doubles, row-major; "a x b complex"
 *    means 2*a*b doubles.
 *
 * Memory and ownership: inputs are read during the call and stay owned by the
 * caller; outputs are written into caller-allocated buffers.  By default every
 * array argument is host memory; with PDEP_DEVICE_PTRS in pdep_opts.flags the
 * array arguments of chi0_apply / chi0_apply_raw / pdep_eigs are device memory
 * on the context's device instead.  The context owns all device-resident state
 * (tables, potential, orbitals, u_v grids, solver work space), allocated through
 * pdep_opts.alloc when given, else hipMalloc.  All device work is queued on
 * pdep_opts.stream (NULL: the default stream); calls return after it finished.
 *
 * Errors: every call returns a pdep_status; on error pdep_last_error() gives a
 * message for the calling thread.  PDEP_ENOTCONV still fills outputs and stats.
 * A context must not be used by two threads at once.
 *
 * Launch shapes: the first application with at least 1024 Sternheimer systems times the
 * candidate shapes of the transform chain (rows per launch) and of the BF16x3
 * coefficient GEMMs (split-K target, column tiles) on its own data and keeps the
 * fastest for the context; results do not depend on them beyond rounding.  With the
 * environment variable PDEP_TUNE_CACHE=<file>, the chosen shapes are also written to
 * that JSON file (one object per grid, N_pw, N_v and precision) and read back by later
 * contexts of the same problem, which then skip the timing runs.  PDEP_FFT_CHUNK=<fp32
 * rows>[:<fp64 rows>] fixes the chain shape.
 */
#ifndef PDEP_H
#define PDEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PDEP_OK = 0,
    PDEP_EINVAL = -1,     /* bad argument (sizes, NaN/Inf in inputs, bad options) */
    PDEP_ENOMEM = -2,     /* device allocation failed or the HBM budget is exceeded */
    PDEP_ENOTCONV = -3,   /* an iterative solver hit its iteration cap */
    PDEP_EGAP = -4,       /* HOMO-LUMO gap below opts.gap_min: chi0 is undefined */
    PDEP_EDEVICE = -5,    /* HIP runtime or device library error */
    PDEP_EBUSY = -6,      /* server queue full */
    PDEP_ENOTFOUND = -7   /* unknown ticket */
} pdep_status;

typedef enum {
    PDEP_FP64 = 0,        /* every step in FP64 */
    PDEP_MIXED_FP32 = 1,  /* FP32 inner CG (transforms, H, P_c) with FP64 residual
                             refinement; FP64 right-hand sides, density, projection */
    PDEP_MIXED_BF16X3 = 2 /* as PDEP_MIXED_FP32, but the inner P_c GEMMs split each FP32
                             operand into two bfloat16 parts and sum three bf16 products
                             with FP32 accumulation (about 16 significant bits); the FP64
                             refinement restores the requested tolerance.  If an inner
                             solve diverges with these products (its residual grows
                             100-fold), its result is dropped and the remaining
                             refinement steps of the block use FP32 products */
} pdep_precision;

#define PDEP_DEVICE_PTRS 1u
#define PDEP_CG_GRAPHS 2u     /* replay the batched inner CG iterations as HIP graphs: every
                                 block of iterations between two reads of the active-row count
                                 is captured once per row count and relaunched (eager when the
                                 kernel profiler is on); results are identical to eager mode */

typedef struct {
    void* (*alloc)(size_t bytes, void* ctx);
    void (*free)(void* ptr, void* ctx);
    void* ctx;
} pdep_allocator;

typedef struct {
    double L[3];          /* cell edges (bohr), each > 0 */
    int n[3];             /* FFT grid, each a product of 2s and 3s, 4 <= n <= 128 */
    double ecut;          /* wavefunction cutoff (Ha); the sphere must fit the grid */
} pdep_cell;

typedef struct {
    int n_v;              /* number of doubly occupied bands, >= 1 */
    int precision;        /* pdep_precision */
    double cg_tol;        /* Sternheimer stop: ||P_c(b - A x)|| <= cg_tol ||b|| (FP64 residual) */
    int cg_maxit;         /* iteration cap of each CG solve */
    double inner_tol;     /* mixed: relative reduction asked of each FP32 inner solve */
    int refine_maxit;     /* mixed: cap on FP64 refinement steps */
    int precond;          /* 1: diagonal kinetic preconditioner 1/max(1/2|G|^2 - e_v, 0.1 Ha)
                             followed by P_c (the CG of Sec. 2.3 is "preconditioned" without a
                             named preconditioner; it changes iteration counts only), 0: none */
    double gap_min;       /* setup fails with PDEP_EGAP below this HOMO-LUMO gap (Ha) */
    double gs_tol;        /* ground state: residual norm target ||H c - e c|| */
    int gs_maxit;         /* ground state: Davidson iteration cap */
    size_t hbm_budget;    /* bytes of solver work space per call; 0 = size to the problem */
    int rhs_tile;         /* Sternheimer systems per batched CG tile; 0 = automatic */
    void* stream;         /* hipStream_t; NULL = default stream */
    pdep_allocator alloc; /* device allocator; alloc == NULL: hipMalloc / hipFree */
    uint32_t flags;       /* PDEP_DEVICE_PTRS | PDEP_CG_GRAPHS */
} pdep_opts;

/* Fill *o with defaults: FP64, cg_tol 1e-10, cg_maxit 2000, inner_tol 1e-5,
 * refine_maxit 8, precond 1, gap_min 1e-3, gs_tol 1e-10, gs_maxit 400, no budget,
 * automatic tiles, default stream, hipMalloc, host pointers. */
void pdep_default_opts(pdep_opts* o);

typedef struct {
    int n_pw;             /* |S| */
    int n_v;
    int n_grid;
    double gap;           /* e_{N_v+1} - e_{N_v} (Ha); 0 when orbitals were supplied */
    double volume;
    int gs_iterations;    /* ground-state Davidson iterations (0 if supplied) */
    double gs_residual;   /* max_v ||H c_v - e_v c_v|| of the orbitals in use */
} pdep_info;

typedef struct {
    int n_rhs;                    /* Sternheimer systems solved (n_pert * n_v) */
    int cg_iter_max;              /* largest CG iteration count of any system (sum over refinement steps) */
    long long cg_iter_total;      /* sum of CG iterations over systems */
    long long op_applications;    /* batched operator applications (launch count of the CG operator) */
    int refine_steps;             /* FP64 refinement steps taken (mixed) */
    int n_notconv;                /* systems that missed cg_tol */
    double max_rel_residual;      /* max over systems of the final FP64 relative residual */
    double ms;                    /* wall time of the call on the device stream */
    int fft_chunk;                /* rows per launch of the transform chain of the inner solves
                                     (chosen by timing on the first large application) */
    int n_fp32_fallback_rows;     /* PDEP_MIXED_BF16X3: systems that ran an inner solve with FP32
                                     projection products after a BF16x3 inner solve diverged
                                     (0 when the BF16x3 products held throughout) */
    long long graph_launches;     /* PDEP_CG_GRAPHS: CG iteration blocks replayed as graphs */
    long long graph_captures;     /* PDEP_CG_GRAPHS: graphs captured (one per row count and phase) */
    long long graph_updates;      /* PDEP_CG_GRAPHS: captures applied to an executable graph in place */
} pdep_apply_stats;

typedef struct {
    double tol;           /* converged when every wanted residual ||A x - l x|| <= tol */
    int maxit;            /* Davidson iteration cap */
    int max_subspace;     /* restart size (columns); 0 = 4 * n_pdep; else >= 2 (n_pdep + n_buffer) */
    int n_buffer;         /* extra unreported vectors carried for faster convergence */
    int reducible;        /* 0: A = chi0bar (Fig. pdepscheme, left panel); 1: A = the reducible
                             chibar, each application made self-consistent with the Hartree
                             response as in chibar_apply (right panel) */
    double scr_tol;       /* reducible: self-consistency tolerance of each application
                             (0: tol / 10) */
    int scr_maxit;        /* reducible: cap on self-consistency passes (0: 200) */
} pdep_eig_opts;

typedef struct {
    int iterations;
    int chi0_columns;             /* chi0bar applications performed */
    double max_residual;          /* of the reported pairs */
    long long cg_iter_total;
    double ms;
    int n_notconv;                /* Sternheimer systems that missed cg_tol, summed over every
                                     chi0bar application, plus (reducible) columns whose
                                     self-consistency missed scr_tol; > 0 makes pdep_eigs
                                     return PDEP_ENOTCONV (outputs still filled) */
    int scr_passes;               /* reducible: self-consistency passes, summed */
} pdep_eig_stats;

typedef struct {
    int passes;                   /* self-consistency passes (chi0bar applications to the block) */
    long long chi0_columns;       /* chi0bar columns computed */
    int n_notconv;                /* columns that missed tol within maxit passes */
    double max_rel_residual;      /* max over columns of ||phi - (1 - chi0bar) y|| / ||phi|| */
    long long cg_iter_total;      /* Sternheimer CG iterations, summed */
    int cg_notconv;               /* Sternheimer systems that missed cg_tol */
    double ms;
} pdep_chibar_stats;

typedef struct pdep_ctx pdep_ctx;

/* Build the basis tables, upload V_loc and obtain the occupied orbitals: the N_v
 * lowest solutions of the Kohn-Sham equation of Sec. 2 with a local potential only,
 * H = 1/2|G|^2 + V_loc on the plane-wave sphere of Sec. 2.1 (the ground-state input of
 * the G0W0 scheme, Fig. scheme_overview).  The gap test follows the integer occupations
 * of Sec. 2.1 (chi0 exists only for a positive HOMO-LUMO gap).
 * vloc: N_g doubles (host), real potential in Ha.  psi_in: NULL, or N_v x N_pw
 * complex (host) orthonormal occupied coefficients in S order with eps_in their
 * N_v energies; when NULL the library finds the N_v lowest eigenpairs of H with an
 * FP64 block Davidson to opts.gs_tol and checks the gap (PDEP_EGAP below
 * opts.gap_min).  Either way the orbitals are then replaced by an orthonormal basis
 * of the same subspace made of functions real in r (c_{-G} = conj c_G), each a Ritz
 * vector of H, with the Ritz values as energies (H is real in r, so a complete
 * occupied eigenspace has such a basis); caller orbitals whose span is not closed
 * under complex conjugation in r give PDEP_EINVAL.  *out receives the new context
 * (NULL on error). */
int pdep_setup(const pdep_cell* cell, const double* vloc, const pdep_opts* opts,
               const double* psi_in, const double* eps_in, pdep_ctx** out);

/* Sizes and ground-state figures of the context (host struct, caller-owned). */
int pdep_get_info(pdep_ctx* ctx, pdep_info* info);

/* The plane-wave basis S of Sec. 2.1 (1/2|G|^2 <= ecut): *n_pw (may be NULL) receives
 * N_pw; miller (may be NULL: size query) receives 3 * N_pw int32 Miller indices (host),
 * lexicographic (mx, my, mz), mz fastest.  PDEP_EINVAL if both are NULL. */
int pdep_get_gvectors(pdep_ctx* ctx, int* n_pw, int32_t* miller);

/* The occupied Kohn-Sham states in use (Sec. 2; the psi_v and e_v of Eq. stern):
 * energies (N_v doubles) and coefficients (N_v x N_pw complex, real in r: the basis
 * pdep_setup keeps), host, caller-allocated.  Either pointer may be NULL. */
int pdep_get_orbitals(pdep_ctx* ctx, double* eps, double* psi);

/* chi0bar applied to n_pert potentials (Eq. chiisamatrixinpdep with V_pert = phi~):
 * phi: n_pert x N_pw' complex on S' (Hermitian-symmetric rows); out: same shape.
 * The n_pert * N_v Sternheimer systems are solved as one batched CG (tiled under
 * opts.hbm_budget / opts.rhs_tile).  st may be NULL. */
int chi0_apply(pdep_ctx* ctx, int n_pert, const double* phi, double* out, pdep_apply_stats* st);

/* Test hook: density response dn (n_pert x N_g doubles) to real potentials
 * dv_r (n_pert x N_g doubles) given directly on the grid, no Coulomb scaling. */
int chi0_apply_raw(pdep_ctx* ctx, int n_pert, const double* dv_r, double* dn_r, pdep_apply_stats* st);

/* chi0_apply for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not allocate, harnesses that forbid it).  Same
 * arguments, results, statistics and errors as chi0_apply, but the work space comes
 * from a fixed 256 MiB array in the library's device code (each device the library
 * runs on holds its own copy until the process ends) instead of pdep_opts.alloc, no
 * routine that allocates device memory is called (the FP64 projection update runs on
 * the library's own matrix-core kernel), no events are created (st->ms is host wall
 * time; pdep_profile_* does not time these calls) and the transform-chain block is not
 * tuned here (a block tuned by an earlier chi0_apply is used).  The perturbations run in
 * as many passes as the array needs; PDEP_ENOMEM if the work space of one perturbation
 * (about N_v x (11 N_pw x 16 + 2 N_sticks n_z x 16) bytes) exceeds it.  All calls on a
 * device share that device's array and its last contents (the library initialises
 * what it reads); two such calls that overlapped on one device would race, so the
 * library serialises them within the process. */
int chi0_apply_noalloc(pdep_ctx* ctx, int n_pert, const double* phi, double* out, pdep_apply_stats* st);

/* The reducible symmetrised polarizability chibar = (1 - chi0bar)^-1 chi0bar of the RPA
 * (Eq. linearalgebrachichi0) applied to n_pert potentials phi (n_pert x N_pw' complex,
 * Hermitian-symmetric rows on S'; out: same shape), without a PDEP basis: the
 * Sternheimer perturbation of each column is phi~ plus the Hartree potential of the
 * density response it induces (Eq. LF with the Hartree term only, Eq. LFHartree,
 * dV_H(G) = 4 pi dn(G)/|G|^2 on S'), made self-consistent (Fig. pdepscheme, right
 * panel) by conjugate gradients on (1 - chi0bar) y = phi, chibar phi = y - phi, until
 * ||phi - (1 - chi0bar) y|| <= tol ||phi|| (tol > 0; every pass is one chi0bar
 * application to the unconverged columns, with the context's precision and cg_tol,
 * which should lie well below tol).  The inverse dielectric matrix is
 * eps^-1 = 1 + chibar (Eq. epsilonandchi).  PDEP_ENOTCONV if a column misses tol within
 * maxit passes or a Sternheimer solve misses cg_tol (outputs and stats still filled).
 * st may be NULL. */
int chibar_apply(pdep_ctx* ctx, int n_pert, const double* phi, double* out, double tol, int maxit,
                 pdep_chibar_stats* st);

typedef struct {
    int chains;                   /* Lanczos chains run (one per basis potential and band, zero
                                     start vectors excluded) */
    int max_length;               /* longest chain (n_lanczos unless a chain closed earlier) */
    long long h_applications;     /* batched applications of the deflated Hamiltonian */
    double ms;
} pdep_lanczos_stats;

/* The body of chi0bar at imaginary frequencies in the basis phi (n_pert x N_pw' complex,
 * Hermitian-symmetric rows on S', e.g. the PDEP eigenvectors):
 *   body[f][i][j] = -(4/Omega) sum_v Re <w_iv| A_v (A_v^2 + u_f^2)^-1 |w_jv>,
 * w_jv = P_c Fwd(V_j u_v), V_j = Re Inv(sqrt(4 pi)/|G| phi_j), A_v = P_c (H - e_v) P_c:
 * the Adler-Wiser form (Eq. AdlerWiser) of the body at omega = i u_f (Eq. finalB), equal to
 * the static <phi_i| chi0bar phi_j> at u = 0.  Computed without empty states by one
 * Lanczos chain of the deflated Hamiltonian P_c H P_c per (j, v), started at
 * w_jv / ||w_jv|| and n_lanczos long (Sec. 2.4, Eqs. MCdef and MCfinal; the paper uses
 * 40), so that every frequency costs only sums over the chains.  freq: n_freq values
 * u_f >= 0 (Ha, host); body: n_freq x n_pert x n_pert doubles (host, caller-allocated),
 * row i, column j (column j comes from the chains of phi_j).  Device memory: about
 * 5 n_pert N_v rows of N_pw complex doubles plus n_lanczos N_v n_pert^2 complex doubles.
 * phi follows PDEP_DEVICE_PTRS; freq and body are host arrays.  st may be NULL. */
int pdep_body_lanczos(pdep_ctx* ctx, int n_pert, const double* phi, int n_lanczos, int n_freq, const double* freq,
                      double* body, pdep_lanczos_stats* st);

/* Head, wings and body of chi0bar at q -> 0 (Table limitqchi0) at the imaginary
 * frequencies freq, in the basis phi (as pdep_body_lanczos), and the reducible
 * quantities of Eq. Bfinal.  The dipole vectors xi^a_v = P_c r_a psi_v solve
 * (H - e_v) xi = P_c [H, r_a] psi_v (Eq. commu; for the local potential here the
 * commutator is -d/dr_a) with the context's precision and cg_tol; they join the
 * Lanczos chains of pdep_body_lanczos as three more start vectors, so that, with
 * f(A) = A (A^2 + u^2)^-1:
 *   F[f][a][b]   = -(16 pi / Omega) sum_v <xi^a_v| f(A_v) |xi^b_v>                (Eq. finalF)
 *   U[f][a][j]   = -(4 / Omega) sqrt(4 pi) sum_v <xi^a_v| f(A_v) |w_jv>          (Eq. finalU1)
 *   B[f][i][j]   as pdep_body_lanczos                                             (Eq. finalB)
 *   Lambda[f]    = (1 - B)^-1 B + (1/k) (1 - B)^-1 mu (1 - B)^-1,
 *   Xi[f]        = (1 - k)/k * int_BZ d^3q / (2 pi)^3 4 pi / q^2                 (Eq. Bfinal)
 * with k = 1 - Tr F / 3 - Tr[mu (1 - B)^-1], mu_ij = 1/3 sum_a U_ia U_aj (U_ia from the
 * chains of the dipole vectors, Eq. finalU2) and the integral over the Brillouin zone of
 * the Gamma-only cell, |q_a| <= pi / L_a.  All outputs are host arrays (caller-allocated,
 * real); any of F, U, B, Lambda, Xi may be NULL.  PDEP_ENOTCONV if a dipole solve missed
 * cg_tol (outputs still filled).  st may be NULL. */
int pdep_head_wings(pdep_ctx* ctx, int n_pert, const double* phi, int n_lanczos, int n_freq, const double* freq,
                    double* F, double* U, double* B, double* Lambda, double* Xi, pdep_lanczos_stats* st);

/* ------------------------------------------------------ G0W0 quasiparticle energies ---
 * Options of pdep_qp_energies; a zero field takes the default in brackets. */
typedef struct {
    int n_lanczos;        /* chain length (Sec. 2.4) [40] */
    int n_freq;           /* Gauss-Legendre nodes of the imaginary-axis integral [64] */
    double omega0;        /* scale (Ha) of the node map u = omega0 t / (1 - t), t in (0, 1) [0.5] */
    double eta;           /* broadening (Ha) of W_p at the real frequencies of the residues [1e-3] */
    double e_fermi;       /* Fermi level (Ha); 0: midgap, which needs the context's own ground
                           * state (caller orbitals leave the gap unknown: then it is required) */
    double secant_tol;    /* stop when |E_k+1 - E_k| <= secant_tol (Ha) [1e-8] */
    int secant_maxit;     /* [40] */
    double dE;            /* step (Ha) of the central difference for Z [1e-3] */
} pdep_qp_opts;

/* Per state.  Energies in Ha. */
typedef struct {
    double eps_ks;        /* e_n */
    double sigma_x;       /* <n|Sigma_X|n> */
    double sigma_c_ks[2]; /* Re, Im <n|Sigma_C(e_n)|n> */
    double z;             /* renormalisation 1 / (1 - d Re Sigma_C / dE) at e_n */
    double e_lin;         /* linearised root (Eq. QPconZ) */
    double e_qp;          /* secant root of Eq. QPenergies with Re Sigma_C */
    double sigma_c_qp[2]; /* Re, Im <n|Sigma_C(e_qp)|n> */
    int iterations;       /* secant iterations */
    int converged;        /* 1 if |E_k+1 - E_k| reached secant_tol */
} pdep_qp_result;

typedef struct {
    int chains;              /* Lanczos chains run */
    int max_length;
    long long h_applications;
    int secant_iterations;   /* sum over states */
    int residue_points;      /* real frequencies at which W_p was evaluated */
    double ms;
} pdep_qp_stats;

/* G0W0 quasiparticle energies of the occupied states `states` (band indices 0 .. N_v - 1,
 * n_states of them) with W_p in the basis phi (n_pdep x N_pw' complex, Hermitian-symmetric,
 * orthonormal rows on S': normally the PDEP eigenvectors of pdep_eigs):
 *   W_p(w) = Xi(w) + (1/Omega) sum_ij V_i Lambda_ij(w) V_j                     (Eq. Wchihb)
 * with Lambda, Xi from the head, wings and body of pdep_head_wings (Eq. Bfinal), and
 *   Sigma_X = -sum_{m occ} [I_BZ delta_mn + (4 pi / Omega) sum_{G in S'} |rho_mn(G)|^2 / |G|^2]
 *   Sigma_C(E) = -(1/2 pi) int dw <n| G_KS(E + i w) W_p(i w) |n>
 *                + sum_m f_m <n m| W_p(e_m - E) |m n>                 (Eqs. contourdeformationfinal, fcontour)
 *   E_qp = e_n + Sigma_X + Re Sigma_C(E_qp) - vxc_n                                (Eq. QPenergies)
 * rho_mn = Fwd(conj(u_m) u_n); I_BZ is the integral of 4 pi / q^2 over the Brillouin zone
 * of the Gamma-only cell (as Xi uses).  G_KS is split by P_v and P_c (Eq. Glehmann): the
 * occupied part is the explicit sum over the N_v orbitals (Eq. MVfinal), the empty part
 * comes from the Lanczos chains of the deflated Hamiltonian started at P_c V_j u_n, which
 * are the body's chains of band n (Eq. MCfinal; each chain's tridiagonal matrix is
 * diagonalised).  The imaginary-axis integral is taken pole by pole: the Lorentzian of
 * each pole with W_p(0) exactly, the rest on n_freq Gauss-Legendre nodes of
 * u = omega0 t / (1 - t).  W_p at the residues' real frequencies carries the broadening
 * eta (Eq. AdlerWiser), so Sigma_C is complex there.  The QP equation starts from the
 * linearised root (Eq. QPconZ, Z by a central difference of step dE) and is solved by the
 * secant method through e_n and e_lin.  vxc: n_states values <n|V_xc|n> (NULL: zero; the
 * model Hamiltonian here has no exchange-correlation potential of its own).  Empty-state
 * residues come from the chains' Ritz values when a QP energy rises above e_fermi.
 * out: n_states results (host).  energies / sigma_c_e (both NULL or both set): n_e energies
 * per state (host [n_states][n_e]) at which <n|Sigma_C(E)|n> is also returned (host
 * [n_states][n_e][2], Re and Im).  phi follows PDEP_DEVICE_PTRS.  PDEP_ENOTCONV if a
 * dipole solve missed cg_tol or a secant iteration did not converge (outputs still
 * filled); PDEP_EINVAL for bad states or options.  opts and st may be NULL. */
int pdep_qp_energies(pdep_ctx* ctx, int n_pdep, const double* phi, int n_states, const int* states,
                     const double* vxc, const pdep_qp_opts* opts, pdep_qp_result* out, int n_e,
                     const double* energies, double* sigma_c_e, pdep_qp_stats* st);

/* PDEP eigenpairs: the n_pdep lowest (most screened) eigenvalues lambda_i of
 * chi0bar by block Davidson in FP64 (Sec. 2.3, Davidson iteration from a random
 * orthonormal start).  phi0: NULL (start drawn from `seed` by the library's own
 * SplitMix64 + Box-Muller generator) or n_pdep x N_pw' complex Hermitian-symmetric
 * start vectors.  eps_out: n_pdep dielectric eigenvalues 1 - lambda_i, descending.
 * basis_out: NULL or n_pdep x N_pw' complex eigenvectors in the same order.
 * eo may be NULL (tol 1e-9, maxit 60, restart 4 n_pdep, no buffer, chi0bar).
 * With eo->reducible the iteration diagonalises chibar instead (Fig. pdepscheme, right
 * panel); it has the same eigenvectors, eigenvalues mu_i = lambda_i / (1 - lambda_i)
 * (Eq. linearalgebrachichi0), and eps_out receives the same dielectric eigenvalues,
 * 1 / (1 + mu_i); the eigenvalues of eps^-1 are 1 / eps_i. */
int pdep_eigs(pdep_ctx* ctx, int n_pdep, uint64_t seed, const double* phi0,
              const pdep_eig_opts* eo, double* eps_out, double* basis_out, pdep_eig_stats* st);

int pdep_destroy(pdep_ctx* ctx);

/* Message of the last error on the calling thread ("" if none). */
const char* pdep_last_error(void);

/* ------------------------------------------------------------------ serving ------
 * A server runs PDEP jobs (setup + pdep_eigs) submitted from any thread.  Jobs are
 * admitted in submission order while the sum of the HBM estimates of running jobs stays
 * within the server budget and fewer than max_running jobs run; each running job has
 * its own HIP stream and stream-ordered device memory, so jobs admitted while others
 * run overlap on the device.  Results stay in the server until polled; a job's
 * failure (any pdep_status) does not affect the others. */
typedef struct pdep_server pdep_server;

#define PDEP_SERVER_FAKE 1u   /* test hook: no GPU work; each job sleeps for
                                 fake_ms_per_gb * (HBM estimate in GB) and returns
                                 eps_i = 1 + (seed % 97 + 1) / (i + 1); a resident
                                 system is not set up, and a chi0 batch sleeps
                                 fake_ms_per_gb ms plus 1 ms per perturbation and
                                 returns out = -phi / 2 */

typedef struct {
    int max_running;          /* jobs on the GPU at once (>= 1) */
    size_t hbm_budget;        /* bytes for running jobs; 0 = 80 % of free device memory */
    int queue_capacity;       /* queued jobs beyond this -> PDEP_EBUSY (0 = 1024) */
    uint32_t flags;           /* PDEP_SERVER_FAKE */
    double fake_ms_per_gb;    /* fake executor run time per GB of estimate */
} pdep_server_opts;

typedef struct {
    pdep_cell cell;
    const double* vloc;       /* N_g doubles, host; copied by pdep_submit */
    pdep_opts opts;           /* stream, alloc and flags are set by the server */
    int n_pdep;
    uint64_t seed;            /* start block of pdep_eigs (library generator) */
    pdep_eig_opts eig;
} pdep_job;

enum { PDEP_JOB_QUEUED = 0, PDEP_JOB_RUNNING = 1, PDEP_JOB_DONE = 2, PDEP_JOB_FAILED = 3 };

typedef struct {
    int status;               /* pdep_status of the finished job (PDEP_OK when DONE) */
    int n_pdep;
    int eig_iterations;
    double gap;               /* HOMO-LUMO gap of the job's ground state (Ha) */
    double queue_ms;          /* submit -> start */
    double run_ms;            /* start -> finish */
    double latency_ms;        /* submit -> finish */
    size_t hbm_estimate;      /* bytes reserved by admission */
} pdep_job_result;

typedef struct {
    int queued, running, done, failed;
    size_t committed_bytes;       /* HBM estimates of the running jobs */
    size_t peak_committed_bytes;  /* maximum of committed_bytes so far */
    int peak_running;
} pdep_server_stats;

int pdep_server_create(const pdep_server_opts* o, pdep_server** out);
/* Queue a job; *ticket identifies it.  PDEP_EINVAL for a bad job (checked here),
 * PDEP_ENOMEM if its estimate exceeds the whole budget, PDEP_EBUSY if the queue is full. */
int pdep_submit(pdep_server* s, const pdep_job* job, uint64_t* ticket);
/* Non-blocking.  *state is PDEP_JOB_*; when DONE, res and up to eps_cap dielectric
 * eigenvalues (descending) are filled; when FAILED, res->status holds the error and
 * pdep_last_error() its message.  PDEP_ENOTFOUND for an unknown ticket.  res / eps_out
 * may be NULL. */
int pdep_poll(pdep_server* s, uint64_t ticket, int* state, pdep_job_result* res, double* eps_out, int eps_cap);
/* Block until the job is DONE or FAILED or timeout_ms passes (< 0: no limit). */
int pdep_server_wait(pdep_server* s, uint64_t ticket, double timeout_ms, int* state);
int pdep_server_stats_get(pdep_server* s, pdep_server_stats* st);
/* Stop admitting, drop queued jobs and chi0 requests, wait for running ones and
 * running batches, remove every resident system, free everything. */
int pdep_server_destroy(pdep_server* s);

/* Resident systems and batched chi0 requests.
 * A server can keep Kohn-Sham systems resident on the device (orbitals, grids and the
 * chi0 work space of pdep_setup, set up once) and apply chi0bar to blocks of trial
 * potentials on them as requests (Sec. 2.3, Eqs. stern, deltani, chiisamatrixinpdep:
 * the operation of chi0_apply).  Every system has one batcher thread with its own HIP
 * stream: it takes the requests queued on the system in submission order, up to
 * max_batch_pert perturbations (at least one whole request), concatenates their
 * perturbations and runs them as ONE chi0_apply, so the Sternheimer systems of all
 * requests of the batch go through one batched CG; the result rows go back to their
 * requests.  Requests that arrive while a batch runs join the next one (continuous
 * batching); batches of different systems run concurrently.  Each row of chi0bar phi
 * depends only on its own perturbation, so a result is the same alone and in a batch
 * up to the rounding of the transforms that pair rows (within cg_tol of the system).
 * The system's HBM estimate (job_hbm_estimate of its cell, options and
 * max_batch_pert) is committed against the server budget while it is resident. */
int pdep_server_add_system(pdep_server* s, const pdep_cell* cell, const double* vloc, const pdep_opts* opts,
                           int max_batch_pert, uint64_t* system_id);
/* Sizes and ground-state figures of a resident system (as pdep_get_info of its context;
 * n_pw fixes the row length N_pw - 1 of its requests; in the fake mode only the sizes and
 * the volume are set).  PDEP_ENOTFOUND for an unknown id. */
int pdep_server_system_info(pdep_server* s, uint64_t system_id, pdep_info* info);
/* Fail the system's queued requests (PDEP_EINVAL), wait for its running batch, free it.
 * PDEP_ENOTFOUND for an unknown id. */
int pdep_server_remove_system(pdep_server* s, uint64_t system_id);
/* Queue chi0bar applied to phi (n_pert x N_pw' complex on S', host, copied here) on a
 * resident system; the ticket is also accepted by pdep_server_wait. */
int pdep_submit_chi0(pdep_server* s, uint64_t system_id, int n_pert, const double* phi, uint64_t* ticket);

/* Queue a PDEP Davidson on a resident system (pdep_eigs of n_pdep eigenvalues with the
 * library's seeded start and options eo, Sec. 2.3): it reuses the system's orbitals
 * instead of a new ground state, runs on the system's batcher in submission order with
 * its chi0 batches (never merged into one), and is polled with pdep_poll_eigs; the
 * ticket is also accepted by pdep_server_wait.  PDEP_EINVAL for bad options,
 * PDEP_ENOTFOUND for an unknown system. */
int pdep_submit_eigs(pdep_server* s, uint64_t system_id, int n_pdep, uint64_t seed, const pdep_eig_opts* eo,
                     uint64_t* ticket);
/* As pdep_poll for a job: res->gap is the system's, res->hbm_estimate the system's
 * estimate; up to eps_cap eigenvalues (descending) when DONE.  PDEP_ENOTFOUND for a
 * ticket that is not such a request. */
int pdep_poll_eigs(pdep_server* s, uint64_t ticket, int* state, pdep_job_result* res, double* eps_out, int eps_cap);

typedef struct {
    int status;               /* pdep_status of the batch (PDEP_OK when DONE) */
    int n_pert;
    int batch_requests;       /* requests in the batch this request ran in */
    int batch_pert;           /* perturbations of that batch */
    double queue_ms;          /* submit -> batch start */
    double run_ms;            /* batch start -> finish */
    double latency_ms;        /* submit -> finish */
    pdep_apply_stats stats;   /* statistics of the whole batch */
} pdep_chi0_result;

/* Non-blocking.  When DONE and out_cap_pert >= n_pert, out (n_pert x N_pw' complex)
 * receives the result, which the server then releases: a later poll with out set fails
 * with PDEP_EINVAL (state and res stay available).  res may be NULL.  PDEP_ENOTFOUND
 * for a ticket that is not a chi0 request. */
int pdep_poll_chi0(pdep_server* s, uint64_t ticket, int* state, pdep_chi0_result* res, double* out,
                   int out_cap_pert);

/* Kernel timing (instrumentation, process-wide).  While enabled, every kernel launch
 * of the library is bracketed by two HIP events recorded on its launch stream.
 * pdep_profile_read returns, per kernel class k < max_kernels, the summed device time
 * (ms), launch count, algorithmic HBM bytes and algorithmic flops since the last reset
 * (any output pointer may be NULL); classes are named by pdep_profile_kernel_name(k)
 * ("" past the last class).  Call after the timed work finished. */
int pdep_profile_enable(int on);
/* Restrict timing to the kernel classes whose bit (1 << k) is set in mask (default: all);
 * the other launches then run without events. */
int pdep_profile_set_classes(unsigned mask);
int pdep_profile_read(int reset, double* total_ms, long long* launches, double* bytes, double* flops,
                      int max_kernels);
const char* pdep_profile_kernel_name(int k);

#ifdef __cplusplus
}
#endif

#endif /* PDEP_H */
