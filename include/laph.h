/*
 * laph.h -- C ABI of the MI355X (gfx950) LapH perambulator library.
 *
 * What it computes (paper: Sec. "Current state-of-the-art", Sec. "LapH",
 * Sec. "QUDA", Sec. "Eigenvector Projection", Sec. "Batched Linear Solves"):
 * quark propagators X = D(m0)^-1 b from spin-diluted LapH sources b, and the
 * perambulators tau = V^dagger D(m0)^-1 V obtained by projecting every solution
 * onto the LapH vectors V of every sink timeslice.  The paper names the Dirac
 * matrix but not its form; this library implements the Wilson-clover matrix
 *
 *   D = A - 1/2 H,   (H psi)(x) = sum_mu [ eta+ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                        + eta- (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *   A = (4 + m0) + c_sw (i/2) sum_{mu<nu} sigma_munu F_munu   (two 6x6 Hermitian chiral blocks)
 *
 * in the DeGrand-Rossi chiral gamma basis, F_munu the traceless anti-Hermitian
 * four-leaf clover, periodic links, and fermion hops across the time boundary
 * multiplied by -1 when the context is created with t_antiperiodic = 1.
 *
 * Conventions shared by every call
 *  - Every pointer argument is a DEVICE pointer unless its name ends in _host.
 *  - The library never allocates device memory: the caller provides the
 *    context state buffer (laph_attach_state) and a per-call workspace for the
 *    solver entry points.  Buffers are owned by the caller and must stay alive
 *    until the call's work on the context stream has finished.
 *  - All work is enqueued on the stream given to laph_create.  laph_solve and
 *    laph_perambulator synchronise that stream before returning (they return
 *    host statistics); every other call is asynchronous.
 *  - Inputs are never modified.  No call aborts or throws: each returns a
 *    laph_status and, on failure, a message readable with laph_last_error();
 *    C++ exceptions inside the library (e.g. host allocation failures) are
 *    caught at the boundary and returned as LAPH_ERR_HOST (size queries then
 *    return 0).
 *  - Canonical (boundary) layouts, C order, complex128 as interleaved (re, im):
 *      gauge   U  [Lt][Lz][Ly][Lx][mu=4][3][3]
 *      spinor  psi[nrhs][Lt][Lz][Ly][Lx][spin=4][colour=3]
 *      LapH    V  [Lt][nev][Lz][Ly][Lx][3]        (V[t][l] = l-th vector of timeslice t)
 *      tau        [Lt][nev][nev][4][4]            (tau[t][l][k][beta][alpha], sink t, l, beta;
 *                                                 source k, alpha; RHS index r = 4k + alpha)
 *  - Internal layouts (used by laph_apply_dslash / laph_apply_clover) are
 *    even-odd structure-of-arrays per right-hand side; laph_field_bytes gives
 *    their size and laph_pack_spinor / laph_unpack_spinor convert.
 */
#ifndef LAPH_H
#define LAPH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct laph_ctx_s *laph_ctx;

typedef enum {
    LAPH_OK = 0,
    LAPH_ERR_INVALID = 1,    /* bad argument, shape, pointer or gauge field */
    LAPH_ERR_HIP = 2,        /* HIP runtime error (message holds the HIP error string) */
    LAPH_ERR_WORKSPACE = 3,  /* state or workspace missing or too small */
    LAPH_ERR_NOCONV = 4,     /* some RHS missed the tolerance within maxiter (X, stats still written) */
    LAPH_ERR_BREAKDOWN = 5,  /* BiCGStab broke down more often than the restart budget allows */
    LAPH_ERR_NONFINITE = 6,  /* a source or an iterate became NaN/Inf (that RHS only) */
    LAPH_ERR_HOST = 7        /* host-side failure inside the library (out of host memory or an
                                internal C++ exception); outputs of that call are undefined */
} laph_status;

/* Storage precision of internal fields and of the solver's inner iterations. */
typedef enum {
    LAPH_F64 = 0,   /* FP64 storage, FP64 arithmetic */
    LAPH_F32 = 1,   /* FP32 storage, FP32 arithmetic */
    LAPH_F16N = 2   /* IEEE binary16 storage scaled by one FP32 norm per site and RHS
                       (n = max |v| over the 24 reals, codes = fp16(v * (1/n))),
                       FP32 arithmetic; gauge links in binary16 */
} laph_prec;

/* Per-RHS solver outcome (laph_rhs_stats.status). */
enum { LAPH_RHS_ACTIVE = 0, LAPH_RHS_CONVERGED = 1, LAPH_RHS_NOCONV = 2,
       LAPH_RHS_BREAKDOWN = 3, LAPH_RHS_NONFINITE = 4 };

typedef struct {
    int inner_prec;    /* laph_prec of the Krylov iterations (FP64 reliable updates always) */
    int batched;       /* 1: all RHS in one solver invocation; 0: one RHS after another */
    double delta;      /* reliable update when |r_inner| < delta * |r| at the last update;
                          <= 0 picks 0.005 (F16N), 0.001 (F32), 0 (F64: update only at the end) */
    int maxiter;       /* per RHS; <= 0 picks 10000 */
    int graph_iters;   /* iterations per captured HIP graph between host polls; <= 0 picks 8 */
    int use_graph;     /* 1: replay captured HIP graphs; 0: plain launches */
    int dagger;        /* 1: solve D^dagger x = b (= gamma5 D gamma5 x = b) */
    int use_x0;        /* 1: start from the contents of X instead of zero */
    int rhs_tile;      /* RHS sharing one load of the links: register tiles 1, 2, 4;
                          LDS-staged links 4, 8, 16; <= 0: chosen by the library */
    int chunk;         /* laph_perambulator: RHS per solver batch; <= 0: largest that fits */
    int stencil;       /* inner stencil form: 1 register RHS tiles (one thread, several RHS),
                          2 links staged in LDS (one wave per RHS); 0: chosen by the library */
    int traversal;     /* stencil workgroup order: 1 the tiles of one site block together,
                          2 each tile sweeps the lattice; 0: chosen by the library */
    int stencil64;     /* form of the FP64 reliable-update stages when inner_prec is not FP64
                          (1 register tiles, 2 LDS-staged links, 0: chosen by the library) */
    int rhs_tile64;    /* their RHS per link load (as rhs_tile; <= 0: chosen by the library) */
} laph_solve_params;

typedef struct {
    int status;        /* LAPH_RHS_* */
    int iters;         /* Krylov iterations */
    int updates;       /* FP64 reliable updates */
    int restarts;      /* breakdown restarts */
    double true_res;   /* ||b - D x|| / ||b|| on the full lattice, FP64, at exit */
} laph_rhs_stats;

/* Fill *p with the defaults described above. */
void laph_default_params(laph_solve_params *p);

/* Create a context for an Lx x Ly x Lz x Lt lattice (dims[0..3]); every extent
 * must be even and >= 4.  n_mass_max bounds the number of masses laph_set_clover
 * may hold.  hip_stream is a hipStream_t (NULL = the default stream).  The
 * context owns no device memory until laph_attach_state. */
laph_status laph_create(laph_ctx *out, const int dims[4], int t_antiperiodic,
                        int n_mass_max, void *hip_stream);
laph_status laph_destroy(laph_ctx ctx);

/* Message of the last failure on the calling thread (valid until the next failing
 * call on that thread; a fixed buffer owned by the library, never freed). */
const char *laph_last_error(void);

/* Device bytes for the context state (gauge copies in FP64 / FP32 / FP16 and
 * the clover term and its inverses for n_mass_max masses), and attach a
 * caller-owned buffer of at least that size (256-byte aligned). */
size_t laph_state_bytes(laph_ctx ctx);
laph_status laph_attach_state(laph_ctx ctx, void *dev, size_t bytes);

/* Load the gauge field (canonical layout, device).  Fails with INVALID if any
 * link is further than 1e-10 from SU(3) (|U U^+ - 1| or |det U - 1|). */
laph_status laph_load_gauge(laph_ctx ctx, const double *U);

/* Build the clover term from the loaded links and, for each of the n_mass
 * masses m0_host[i], the FP64 and FP32 inverses of its two chiral blocks per
 * site.  INVALID if a block is not positive definite (e.g. 4 + m0 too small). */
laph_status laph_set_clover(laph_ctx ctx, double csw, int n_mass, const double *m0_host);

/* Bytes of an internal spinor field of nrhs right-hand sides, one parity
 * (parity_only = 1) or both. */
size_t laph_field_bytes(laph_ctx ctx, int prec, int nrhs, int parity_only);

/* Canonical complex128 <-> internal layout.  parity = 0 or 1 converts that
 * parity (internal field parity-only), parity = -1 both (internal full field). */
laph_status laph_pack_spinor(laph_ctx ctx, void *out, const double *in, int prec, int nrhs, int parity);
laph_status laph_unpack_spinor(laph_ctx ctx, double *out, const void *in, int prec, int nrhs, int parity);

/* out = H_{p, 1-p} in on internal parity-only fields (p = out_parity): the bare
 * hopping sum without the -1/2 and without the clover term; dagger = 1 applies
 * gamma5 H gamma5.  Single-application accuracy: FP64 ~1e-15, FP32 ~1e-7 relative. */
laph_status laph_apply_dslash(laph_ctx ctx, void *out, const void *in, int out_parity,
                              int prec, int nrhs, int dagger);

/* out = A (inverse = 0) or A^-1 (inverse = 1) on internal parity-only fields of
 * the given parity, with the mass laph_set_clover stored at mass_idx. */
laph_status laph_apply_clover(laph_ctx ctx, void *out, const void *in, int parity, int mass_idx,
                              int inverse, int prec, int nrhs);

/* out = D in (dagger = 0) or D^dagger in, FP64, canonical layout, full lattice.
 * work must hold laph_field_bytes(ctx, LAPH_F64, 2, 0) bytes. */
laph_status laph_apply_D(laph_ctx ctx, double *out, const double *in, int mass_idx, int nrhs,
                         int dagger, void *work, size_t work_bytes);

/* Workspace for laph_solve with nrhs right-hand sides. */
size_t laph_solve_workspace_bytes(laph_ctx ctx, int nrhs, const laph_solve_params *p);

/* Solve D(m0[mass_idx_host[r]]) X_r = B_r for r < nrhs (canonical layouts) by
 * even-odd preconditioned BiCGStab with inner iterations in p->inner_prec,
 * FP64 reliable updates and FP64 inner products, until the FP64 full-lattice
 * residual ||B_r - D X_r|| <= tol ||B_r||.  stats_host (nrhs entries, may be
 * NULL) receives the per-RHS outcome.  Returns NOCONV / BREAKDOWN / NONFINITE
 * if any RHS ended that way; X is written in every case. */
laph_status laph_solve(laph_ctx ctx, double *X, const double *B, int nrhs,
                       const int *mass_idx_host, double tol, const laph_solve_params *p,
                       laph_rhs_stats *stats_host, void *work, size_t work_bytes);

/* Workspace for laph_perambulator with nev LapH vectors per timeslice. */
size_t laph_perambulator_workspace_bytes(laph_ctx ctx, int nev, const laph_solve_params *p);

/* tau[t][l][k][beta][alpha] = sum_{x,a} conj(V_l(x,t)_a) X^(4k+alpha)(x,t)_(beta,a)
 * for every sink timeslice t, with X^(4k+alpha) = D(m0[mass_idx])^-1 b^(4k+alpha)
 * and b^(4k+alpha)(x,t)_(s,a) = delta_{t,t0} delta_{s,alpha} V_k(x,t0)_a.  The
 * 4*nev solves run in batches of p->chunk RHS; solutions are projected with an
 * FP64 matrix-core GEMM and never stored whole.  stats_host: 4*nev entries. */
laph_status laph_perambulator(laph_ctx ctx, double *tau, const double *V, int nev, int t0,
                              int mass_idx, double tol, const laph_solve_params *p,
                              laph_rhs_stats *stats_host, void *work, size_t work_bytes);

/* Stochastic LapH (the noise-diluted variant of LapH the paper's earlier CPU work
 * used, Sec. "Current state-of-the-art"): the caller's noise rho = c128 [4][nev] on
 * the device (rho[alpha][k] for spin alpha and LapH index k of the source time t0;
 * e.g. Z4 values) is diluted fully in time and spin and into n_dil interlaced LapH
 * groups {k : k mod n_dil = j}, 1 <= n_dil <= nev.  Source r = 4j + alpha:
 *   b^(4j+alpha)(x,t)_(s,a) = delta_{t,t0} delta_{s,alpha} sum_{k = j mod n_dil} rho[alpha][k] V_k(x,t0)_a
 * laph_stochastic_perambulator solves the 4*n_dil sources like laph_perambulator and
 * writes phi = c128 [Lt][nev][n_dil][4][4] = [t][l][j][beta][alpha] (the projection of
 * the solutions onto the LapH vectors of every sink time); its workspace is
 * laph_perambulator_workspace_bytes(ctx, nev, p); stats_host: 4*n_dil entries.
 * With n_dil = nev and rho = 1, phi = tau.  laph_make_noise_sources writes the
 * sources alone: B canonical, 4*n_dil RHS. */
laph_status laph_stochastic_perambulator(laph_ctx ctx, double *phi, const double *V, int nev, int t0,
                                         int mass_idx, const double *rho, int n_dil, double tol,
                                         const laph_solve_params *p, laph_rhs_stats *stats_host,
                                         void *work, size_t work_bytes);
laph_status laph_make_noise_sources(laph_ctx ctx, double *B, const double *V, int nev, int t0,
                                    const double *rho, int n_dil);

/* Spin basis of tau (the paper's driver adds a Dirac spin basis of its own, Sec.
 * "Quda_laph", without defining it): for a change of basis psi' = S psi with S a
 * unitary 4 x 4 matrix (S_host: c128 [4][4] row-major, host), every trailing 4 x 4
 * block of tau (sink spin beta, source spin alpha) becomes S tau S^dagger:
 *   out[b][beta'][alpha'] = sum S[beta'][beta] tau[b][beta][alpha] conj(S[alpha'][alpha])
 * tau, out: c128 [n_blocks][4][4] on the device (out may be tau).  For a
 * perambulator n_blocks = Lt * nev * nev (or Lt * nev * n_dil for phi).
 * Asynchronous on the context stream. */
laph_status laph_spin_rotate(laph_ctx ctx, double *out, const double *tau, long n_blocks, const double *S_host);

/* Building blocks of the perambulator, exposed for the differentiable wrapper:
 *  laph_make_sources: B (canonical, 4*nev RHS) = spin-diluted sources at t0;
 *  laph_project:      tau (as above) from solutions X (canonical, 4*nev_src RHS);
 *  laph_project_adjoint: G_X (canonical, 4*nev_src RHS) = sum_l V_l(x,t) Gtau[t][l][k][beta][alpha]
 *                     at every t (the adjoint of laph_project).
 * work for laph_project / laph_project_adjoint: laph_project_workspace_bytes. */
laph_status laph_make_sources(laph_ctx ctx, double *B, const double *V, int nev, int t0);
size_t laph_project_workspace_bytes(laph_ctx ctx, int nev, int nev_src);
laph_status laph_project(laph_ctx ctx, double *tau, const double *X, const double *V, int nev,
                         int nev_src, void *work, size_t work_bytes);
laph_status laph_project_adjoint(laph_ctx ctx, double *GX, const double *Gtau, const double *V,
                                 int nev, int nev_src);

/* LapH vectors on the GPU (Sec. "LapH", "QUDA": the LapH subspace of each time
 * slice is spanned by the lowest eigenvectors of the gauge-covariant 3-D
 * Laplacian).  -Delta acts on colour fields of one timeslice,
 *   (-Delta f)(x) = sum_{k=x,y,z} [2 f(x) - U_k(x) f(x+k) - U_k(x-k)^dagger f(x-k)],
 * periodic, with the loaded gauge field's spatial links.
 *  laph_apply_laplacian: out[t][j] = (-Delta) in[t][j] for every timeslice t and
 *    j < nvec; in, out: c128 [Lt][nvec][Lz][Ly][Lx][3] device arrays (no aliasing).
 *  laph_laplacian_eigvecs: the nev lowest eigenpairs of -Delta on every timeslice
 *    (1 <= nev <= 64) by Chebyshev-filtered subspace iteration on the device:
 *    V = c128 [Lt][nev][Lz][Ly][Lx][3] (device; the layout laph_perambulator
 *    takes), each vector of unit norm with its largest-modulus component real
 *    positive (the lowest index among those within 1e-12 of the largest);
 *    lambda_host = [Lt][nev] ascending.  It stops when every returned pair has
 *    ||(-Delta) v - lambda v|| <= tol (absolute; the spectrum lies in [0, 12]) or
 *    after max_iter iterations (then LAPH_ERR_NOCONV; V is not written).  degree:
 *    largest Chebyshev filter degree per iteration (<= 1: 96); the degree is also
 *    kept low enough that the filter grows the lowest Ritz direction by at most
 *    about 1e6 over the damped interval.  iters_host and
 *    residual_host (may be null) receive the iterations used and the largest
 *    residual norm.  work: laph_laplacian_workspace_bytes(ctx, nev) bytes of device
 *    memory (about 4 Lt (nev + nev/2) 3 Lx Ly Lz complex doubles).  The block is
 *    orthonormalised by Cholesky factors of its Gram matrix; a timeslice with a
 *    pivot below 1e-12 of the largest diagonal entry uses the Gram matrix's
 *    eigendecomposition instead.  The environment variable LAPH_EIG_CHOL_TINY, read
 *    at each call, replaces that threshold (a value >= 1 takes the eigendecomposition
 *    on every timeslice). */
size_t laph_laplacian_workspace_bytes(laph_ctx ctx, int nev);
laph_status laph_apply_laplacian(laph_ctx ctx, double *out, const double *in, int nvec);
laph_status laph_laplacian_eigvecs(laph_ctx ctx, double *V, double *lambda_host, int nev, double tol, int max_iter,
                                   int degree, void *work, size_t work_bytes, int *iters_host,
                                   double *residual_host);

/* Meson doublets and baryon triplets of the LapH vectors (Sec. "QUDA": the LapH
 * vectors also form the quark-antiquark doublets and three-quark triplets used in
 * the Wick contractions of meson and baryon correlators).  For each momentum
 * p = 2 pi (nx / Lx, ny / Ly, nz / Lz) given as integers mom_host[3 q .. 3 q + 2]
 * (any sign; host array of 3 n_mom ints) and every timeslice t:
 *   Phi[q][t][l][m]    = sum_x e^{-i p.x} sum_a conj(V_l(x,t)_a) V_m(x,t)_a
 *   B[q][t][l][m][n]   = sum_x e^{-i p.x} eps_abc V_l(x,t)_a V_m(x,t)_b V_n(x,t)_c
 * x runs over the sites of the timeslice (x, y, z integer coordinates).
 *  V:   c128 [Lt][nev][Lz][Ly][Lx][3] on the device (the laph_laplacian_eigvecs
 *       layout), 1 <= nev <= 64 (triplets: nev >= 3); not modified.
 *  phi: c128 [n_mom][Lt][nev][nev] on the device, every entry written.
 *  B:   c128 [n_mom][Lt][nev][nev][nev] on the device, every entry written (the
 *       tensor is antisymmetric: entries with a repeated index are exactly 0).
 *  work: laph_contract_workspace_bytes(ctx, kind, nev, n_mom) bytes of device
 *       memory (kind 0 doublets, 1 triplets); LAPH_ERR_WORKSPACE if smaller.
 * Needs only the context's geometry (no gauge field, clover or state).  FP64
 * throughout; asynchronous on the context stream. */
size_t laph_contract_workspace_bytes(laph_ctx ctx, int kind, int nev, int n_mom);
laph_status laph_meson_doublets(laph_ctx ctx, double *phi, const double *V, int nev, int n_mom,
                                const int *mom_host, void *work, size_t work_bytes);
laph_status laph_baryon_triplets(laph_ctx ctx, double *B, const double *V, int nev, int n_mom,
                                 const int *mom_host, void *work, size_t work_bytes);

/* Milliseconds of the last laph_solve / laph_perambulator split as
 * [0] total, [1] solve, [2] projection (HIP events on the context stream). */
laph_status laph_last_timings(laph_ctx ctx, double *ms_host3);

/* Measurement of the solver's two fused stencil kernels on synthetic fields:
 * launches the inner-iteration stages of M_hat exactly as the batched solver
 * does for nrhs right-hand sides of one mass (mass_idx) in the stencil form
 * `stencil` (1 register tiles, 2 LDS-staged links) with tiles of rhs_tile and
 * workgroup order `traversal` (1 or 2, as in laph_solve_params) --
 * stage 1: t_o = A_oo^-1 H_oe p_e;  stage 2: v_e = p_e - 1/4 A_ee^-1 H_eo t_o with
 * the fused <r^, v> partial sums -- each reps times, and returns the average
 * duration of one launch in ms_host2[0] (stage 1) and ms_host2[1] (stage 2),
 * measured with HIP events on the context stream.  The fields hold a fixed
 * byte pattern; work must hold laph_time_stages_workspace_bytes bytes. */
size_t laph_time_stages_workspace_bytes(laph_ctx ctx, int prec, int nrhs, int rhs_tile);
laph_status laph_time_stages(laph_ctx ctx, int prec, int nrhs, int stencil, int rhs_tile, int traversal,
                             int mass_idx, int reps, void *work, size_t work_bytes, double *ms_host2);

/* Autotuner (the paper tunes launch parameters per machine, Sec. "QUDA"):
 * time every stencil form / RHS-per-link-load candidate for nrhs RHS of
 * mass_idx as laph_time_stages does, keep the fastest for this context and
 * (precision, nrhs), and return it (stencil 1 or 2, rhs_tile, traversal).
 * laph_solve / laph_perambulator with stencil = 0 and rhs_tile <= 0 use the
 * tuned choice for their inner precision and batch size, and with
 * stencil64 = 0 and rhs_tile64 <= 0 the LAPH_F64 choice for the FP64
 * reliable-update stages, tuning on first use on their own workspace.  If the environment variable LAPH_TUNE_CACHE names a file,
 * choices are appended there and read back by later contexts of the same
 * lattice.  work: laph_time_stages_workspace_bytes(ctx, prec, nrhs, 16). */
laph_status laph_autotune(laph_ctx ctx, int prec, int nrhs, int mass_idx, void *work, size_t work_bytes,
                          int *stencil_out, int *rhs_tile_out, int *traversal_out, double *ms_host);

/* The autotuner's stored choice for (prec, nrhs) in this context, without timing
 * anything: *found = 1 and the shape (stencil 1 or 2, rhs_tile, traversal 1 or 2)
 * if the context tuned that key or read it from the LAPH_TUNE_CACHE file at
 * creation, else *found = 0.  Cache entries are keyed by the lattice extents,
 * the device architecture (e.g. gfx950) and a digest of the stencil sources the
 * library was built from; entries of another architecture or build are ignored. */
laph_status laph_tuned_choice(laph_ctx ctx, int prec, int nrhs, int *found, int *stencil_out, int *rhs_tile_out,
                              int *traversal_out);

/* One fused stage of the batched solver's even-odd operator
 *   M_hat = 1 - 1/4 A_ee^-1 H_eo A_oo^-1 H_oe
 * (the symmetric Schur complement of D = A - 1/2 H), run with exactly the kernels
 * and launch shape laph_solve uses for its inner iterations (and, with
 * prec = LAPH_F64, for its reliable updates), on internal parity-only fields of
 * nrhs right-hand sides of the mass stored at mass_idx:
 *   which = 1:  out_o = A_oo^-1 H_oe in_e                      (stage 1; y, w unused)
 *   which = 2:  out_e = y_e - 1/4 A_ee^-1 H_eo in_o            (stage 2 of v = M_hat p)
 *               dots_host[3 r + 0, 1] = <w_r, out_r>  (re, im)
 *   which = 3:  out_e = y_e - 1/4 A_ee^-1 H_eo in_o            (stage 2 of t = M_hat s)
 *               dots_host[3 r + 0, 1] = <out_r, y_r>, dots_host[3 r + 2] = |out_r|^2
 * with <a, b> = sum conj(a) b over the sites and spin-colour components of one
 * parity.  The inner products are those the solver's BiCGStab takes its scalars
 * from: accumulated from the stage's arithmetic-precision results before they are
 * stored, per site block in FP64 and over blocks in a fixed order.  dagger = 1
 * replaces H by gamma5 H gamma5.  stencil (1 register RHS tiles, 2 LDS-staged
 * links), rhs_tile (1, 2, 4 for register tiles; 4, 8, 16 for LDS links) and
 * traversal (1 the tiles of one site block together, 2 each tile sweeps the
 * lattice) select the launch shape as in laph_solve_params.
 *   in, out, y, w: laph_field_bytes(ctx, prec, nrhs, 1)-byte internal fields
 *       (RHS r at offset r * laph_field_bytes(ctx, prec, 1, 1)); out must not
 *       alias in, y or w.
 *   dots_host: 3 * nrhs doubles on the host (which 2, 3; may be NULL for which 1).
 *   work: laph_apply_stage_workspace_bytes(ctx, nrhs) bytes of device memory.
 * Synchronises the context stream when it returns dots (which 2, 3). */
size_t laph_apply_stage_workspace_bytes(laph_ctx ctx, int nrhs);
laph_status laph_apply_stage(laph_ctx ctx, int which, void *out, const void *in, const void *y, const void *w,
                             int prec, int nrhs, int mass_idx, int dagger, int stencil, int rhs_tile, int traversal,
                             double *dots_host, void *work, size_t work_bytes);

/* laph_apply_stage without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operation, arguments, layouts and results as
 * laph_apply_stage; the tile table, per-block partials and per-RHS sums live in
 * one fixed 16 MiB device array of the library per GPU (taken at load time and
 * held until the process ends; its address is looked up once per device in
 * laph_create).  The call itself allocates nothing, on the device or the host.
 * Fails with LAPH_ERR_WORKSPACE when laph_apply_stage_workspace_bytes(ctx, nrhs)
 * exceeds 16 MiB (at 32^3 x 64: above about 40 RHS) and with LAPH_ERR_HIP when
 * no device was current at laph_create.  Every call on one GPU uses the same
 * array: calls that overlap on that GPU (other streams, other contexts, other
 * threads) race and must be serialised by the caller.  Synchronises the
 * context stream when it returns dots (which 2, 3). */
laph_status laph_apply_stage_noalloc(laph_ctx ctx, int which, void *out, const void *in, const void *y,
                                     const void *w, int prec, int nrhs, int mass_idx, int dagger, int stencil,
                                     int rhs_tile, int traversal, double *dots_host);

/* Mass gradient of the differentiable solve.  For X = D(m0)^-1 B (nrhs RHS,
 * canonical complex128 layout) and a real loss L(X), dD/dm0 = 1 gives
 * dX/dm0 = -D^-1 X, so with the adjoint solutions Z = D^-dagger G (G = dL/dRe X
 * + i dL/dIm X, solved by laph_solve with dagger = 1)
 *   *g_host = dL/dm0 = -sum_r Re <Z_r, X_r>
 * summed in FP64 in a fixed order (per thread, per block, then over blocks).
 * Z, X: device arrays of nrhs full-lattice spinors; work:
 * laph_mass_gradient_workspace_bytes(ctx) bytes of device memory (a fixed size).
 * Synchronises the context stream. */
size_t laph_mass_gradient_workspace_bytes(laph_ctx ctx);
laph_status laph_mass_gradient(laph_ctx ctx, double *g_host, const double *Z, const double *X, int nrhs,
                               void *work, size_t work_bytes);

/* Measurement: copy `bytes` (a multiple of 16) from src to dst on the device with
 * the library's streaming kernel (one 16-byte word per thread, one pass of the
 * grid over the buffer), once to warm up and then reps times; *ms_host = average ms per copy (HIP events
 * on the context stream).  Read + written bytes / time is the HBM rate a
 * bandwidth-bound kernel of the library can reach.  dst and src must not overlap. */
laph_status laph_stream_copy(laph_ctx ctx, void *dst, const void *src, size_t bytes, int reps, double *ms_host);

/* ---- Two-level aggregation multigrid -------------------------------------------
 * The paper's production solver is an adaptive geometric multigrid (Sec. "QUDA";
 * Sec. "Performance Measurement Method" names a mixed-precision multigrid solve the
 * kernel of the computation; Sec. "Batched Linear Solves" batches it because coarse
 * grids have little parallelism).  This is its two-level aggregation form:
 *   - near-null vectors: the caller's nvec start fields relaxed by null_passes
 *     inverse-iteration solves x <- D^-1 x (the library's batched FP32-inner solver
 *     to relative residual null_tol; a pass that misses null_tol still counts);
 *   - prolongator P: on every aggregate (a block[0] x .. x block[3] block of sites)
 *     and chirality (spins 0,1 and 2,3, gamma5 = diag(1,1,-1,-1)) the restricted
 *     halves of the vectors, Gram-Schmidt orthonormalised in vector order;
 *   - coarse matrix D_c = P^dagger D P (nearest-neighbour stencil of 2 nvec x 2 nvec
 *     complex blocks on the coarse lattice), built on the device in FP64;
 *   - solve: flexible GCR(restart) on the full system with x, r, b in FP64 and one
 *     multigrid cycle per iteration in FP32 (pre-smoother, coarse correction by
 *     coarse_iters BiCGStab iterations to coarse_tol, post-smoother; the smoother is
 *     smooth_iters minimal-residual steps on the even-odd Schur system); every
 *     restart recomputes the residual in FP64 (a reliable update).
 * The multigrid belongs to one mass (mass_idx of laph_set_clover) and is detached by
 * laph_load_gauge, laph_set_clover and any failed laph_mg_setup.
 * Coarse vectors: complex128 [n][Tc][Zc][Yc][Xc][2][nvec] (coarse extents L/block, then
 * chirality, then vector); coarse matrix: complex128 [nc][9][2 nvec][2 nvec] with the
 * coarse site index ((tc Zc + zc) Yc + yc) Xc + xc, direction 0 = the aggregate itself,
 * 1 + 2 mu / 2 + 2 mu = the neighbour aggregate in +mu / -mu, row / column index
 * chirality * nvec + vector. */
typedef struct {
    int nvec;            /* near-null vectors, 1..16 (2 nvec coarse components per aggregate) */
    int block[4];        /* aggregate extents in x, y, z, t; each divides the lattice extent,
                            their product is at most 256 */
    int null_passes;     /* inverse-iteration passes (0: the start vectors are used as given) */
    double null_tol;     /* relative residual of each pass's solve, in (0, 1) */
    int smooth_iters;    /* minimal-residual steps per smoother application, >= 1 */
    int coarse_iters;    /* coarse BiCGStab iterations per cycle at most, >= 1 */
    double coarse_tol;   /* relative residual at which a coarse solve stops, in (0, 1) */
    int restart;         /* GCR directions between FP64 residual recomputations, 1..16 */
    int maxiter;         /* outer iterations at most, >= 1 */
} laph_mg_params;

/* Defaults: nvec 12, block 4 x 4 x 4 x 4, null_passes 4, null_tol 1e-2, smooth_iters 4,
 * coarse_iters 16, coarse_tol 0.1, restart 8, maxiter 500. */
void laph_mg_default_params(laph_mg_params *p);
/* Bytes of the caller's multigrid buffer (basis: nvec full FP64 fields; coarse matrix)
 * and of the setup workspace (the inverse-iteration solves, then an aggregate-major copy
 * of the basis for the coarse-matrix build: at least nvec full FP64 fields); 0 for
 * invalid parameters. */
size_t laph_mg_state_bytes(laph_ctx ctx, const laph_mg_params *p);
size_t laph_mg_setup_workspace_bytes(laph_ctx ctx, const laph_mg_params *p);
/* Build the multigrid of mass mass_idx from V0 (device, nvec canonical complex128 spinor
 * fields, not modified) into state (device, laph_mg_state_bytes; must stay allocated
 * while the multigrid is used).  Fails with LAPH_ERR_INVALID for a bad shape or when a
 * vector is linearly dependent on an aggregate.  Synchronises the context stream. */
laph_status laph_mg_setup(laph_ctx ctx, int mass_idx, const laph_mg_params *p, const double *V0, void *state,
                          size_t state_bytes, void *work, size_t work_bytes);
/* The basis (P's columns) as nvec canonical spinor fields; the coarse matrix (layouts above). */
laph_status laph_mg_basis(laph_ctx ctx, double *out);
laph_status laph_mg_coarse_matrix(laph_ctx ctx, double *out);
/* c = P^dagger f and f = P c on n canonical spinor fields / coarse vectors; work:
 * laph_mg_field_workspace_bytes(ctx, n) bytes of device memory. */
size_t laph_mg_field_workspace_bytes(laph_ctx ctx, int n);
laph_status laph_mg_restrict(laph_ctx ctx, double *c_out, const double *f, int n, void *work, size_t work_bytes);
laph_status laph_mg_prolong(laph_ctx ctx, double *f_out, const double *c, int n, void *work, size_t work_bytes);
/* out = D_c in on n coarse vectors (out must not alias in). */
laph_status laph_mg_coarse_apply(laph_ctx ctx, double *out, const double *in, int n);
/* One building block of the multigrid cycle on n inputs (for tests), with the cycle
 * parameters of p (NULL: the setup's): what 0: out = D in computed in FP32; 1: the
 * smoother (smooth_iters MR steps on the even-odd system, odd half reconstructed);
 * 2: one whole cycle; 4: out = D in computed in FP64 (the reliable update's operator);
 * these on n canonical spinor fields; 3: the coarse BiCGStab (coarse_iters iterations,
 * stopping at coarse_tol) on n coarse vectors; 5 and 6: the normalised GCR directions
 * z_k (5) or w_k = D z_k (6), k < restart, after maxiter iterations of the solve of
 * D x = in, as restart x n canonical fields ([k][r]).
 * work: laph_mg_solve_workspace_bytes(ctx, n, p) bytes.  Synchronises the stream. */
laph_status laph_mg_component(laph_ctx ctx, int what, double *out, const double *in, int n,
                              const laph_mg_params *p, void *work, size_t work_bytes);
/* X = D^-1 B for nrhs canonical complex128 fields, all in one batch, to the per-RHS
 * full-lattice FP64 relative residual tol.  p (may be NULL: the setup's values) gives
 * the cycle parameters of this call (smooth_iters, coarse_iters, coarse_tol, restart,
 * maxiter; its other fields are ignored).  stats_host (may be NULL): iters = GCR
 * iterations, updates = FP64 residual recomputations, true_res at exit.  Returns
 * LAPH_ERR_NOCONV if an RHS misses tol within maxiter (X and stats still written).
 * work: laph_mg_solve_workspace_bytes(ctx, nrhs, p) bytes.  Synchronises the stream. */
size_t laph_mg_solve_workspace_bytes(laph_ctx ctx, int nrhs, const laph_mg_params *p);
laph_status laph_mg_solve(laph_ctx ctx, double *X, const double *B, int nrhs, double tol,
                          const laph_mg_params *p, laph_rhs_stats *stats_host, void *work, size_t work_bytes);

#ifdef __cplusplus
}
#endif
#endif /* LAPH_H */
