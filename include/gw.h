/* gw.h - C-ABI of libgw: the contour-deformation G0W0 hot path on one
 * MI355X (gfx950) GPU.
 *
 * Method: Mejia-Rodriguez, Kunitsa, Apra, Govind, "Scalable Molecular GW
 * Calculations: Valence and Core Spectra" (JCTC 2021).  Sections cited:
 *   [CD-theory]  Theory - Contour Deformation (Sigma = R - I, the residue
 *                term R and the imaginary-axis term I)
 *   [CD-impl]    Implementation - Contour Deformation (W in the fitted
 *                auxiliary basis, Pi_PQ(omega), the dielectric matrix 1 - Pi,
 *                the imaginary-axis integral I_nn on a modified Gauss-Legendre
 *                grid, the residue term R_nn solved with MINRES and the
 *                explicit-build fallback)
 *   [Alg1]       Algorithm 1 (CD-GW)
 *   [QP]         Implementation - Solution of the Quasiparticle Equations
 *                (QP equation, Z, the step-selection tree figure)
 *   [SD-theory]  Theory - Spectral Decomposition (Casida equations, W and
 *                Sigma_nn as sums over the excitations Omega_s)
 *   [SD-impl]    Implementation - Spectral Decomposition (the Hermitian form
 *                of the Casida problem, A + B in the fitted basis, w^s_mn)
 *   [RVF]        Implementation - Variational Fitting Approximation (the
 *                orthonormalised three-index integrals (P|pq))
 *
 * Conventions (all entry points):
 *   - Hartree atomic units, closed shell.  Orbitals 0..n_occ-1 are occupied,
 *     n_occ..n_mo-1 virtual; eps must be strictly ascending.
 *   - Every pointer argument is a HOST pointer unless stated otherwise.  The
 *     caller owns all input and output arrays; inputs are copied to device
 *     memory before the call returns and are not retained.
 *   - Arrays are row-major float64 unless stated otherwise.
 *   - Return value: 0 on success, a negative GW_E* code on a hard error (the
 *     context is left unchanged where possible; gw_last_error() describes it).
 *   - A context is not thread-safe; distinct contexts may be used from
 *     different threads.  All device work of a context runs on its stream.
 *   - Every entry point computes on the GPU; there is no host fallback.
 */
#ifndef GW_H
#define GW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hard errors */
#define GW_OK 0
#define GW_EINVAL (-1)   /* bad sizes, unsorted/non-finite eps, unknown state, bad grid */
#define GW_ENOMEM (-2)   /* device allocation failed or the memory budget is exceeded */
#define GW_EDEVICE (-3)  /* a HIP runtime call or kernel launch failed */
#define GW_ENOTSPD (-4)  /* 1 - Pi(i xi) was not positive definite (cannot happen for real B) */

/* per-state soft status bits returned by gw_qp */
#define GW_ST_MAXITER 1   /* the QP iteration limit was reached */
#define GW_ST_SMALL_Z 2   /* Z < 0.1 at the returned point */
#define GW_ST_FALLBACK 4  /* at least one residue used the dense fallback */

/* precision of the Pi(i xi) build (gw_opts.pi_prec) and, optionally, of the
 * W^c contraction (gw_opts.wc_prec: FP64 or BF16X3 only); Cholesky, MINRES
 * and the QP step are always float64 */
#define GW_PI_FP64 0
#define GW_PI_FP32 1    /* FP32 operands, FP32 MFMA accumulation, FP64 split-K sum */
#define GW_PI_BF16X3 2  /* bf16 hi/lo split, 3 MFMA products, FP32 accumulation */

typedef struct gw_ctx gw_ctx;

/* Options; a zero-initialised struct means the defaults. */
typedef struct gw_opts {
  int pi_prec;              /* GW_PI_*                                   (0: FP64)  */
  int minres_max_iter;      /* MINRES iteration cap before the fallback  (0: 200)   */
  double minres_rtol;       /* MINRES relative residual target           (0: 1e-12) */
  double qp_tol;            /* |f| < qp_tol ends the QP iteration, Ha    (0: 1e-10) */
  int qp_max_iter;          /* QP iteration cap                          (0: 100)   */
  const double* dsig_x;     /* optional [n_mo]: Sigma^x_nn - V^xc_nn; NULL means 0.
                               Copied at setup. */
  void* stream;             /* hipStream_t to run on; NULL: the context creates one */
  size_t mem_budget_bytes;  /* cap on device memory of this context (0: no cap) */
  size_t work_budget_bytes; /* cap on the stage-A workspace (0: 16 GiB); grid points
                               are factored in chunks that fit */
  int minres_batch;         /* residue systems per MINRES batch, >= 64 (0: 384); bounds
                               the MINRES workspace */
  int no_graphs;            /* nonzero: launch every MINRES iteration eagerly instead of
                               replaying it from a captured HIP graph (0: graphs; they
                               are also skipped on a stream that cannot be captured) */
  int no_precond;           /* nonzero: plain MINRES.  0: residue systems with |omega|
                               below 0.9 of the lowest transition energy run MINRES
                               preconditioned by M = 1 - Pi(0) (SPD), factored as one more
                               grid point (xi = 0) of the W^c build; their residual target
                               is then relative in the M^-1 norm */
  double cluster_width;     /* > 0: the cluster initial-guess layer of [QP] in gw_qp and
                               every gw_evgw cycle (0: off).  The requested states,
                               sorted by their energy in G, form clusters wherever
                               neighbours lie within cluster_width Ha; each cluster's
                               median member is solved first, the others start the step
                               tree at eps_n plus its QP shift (at eps_n if it hit the
                               iteration cap).  States of different clusters advance
                               together; a member joins the batched rounds once its
                               representative is done. */
  int wc_prec;              /* precision of the W^c contraction of the table build
                               (W_{mn,mn}(i xi) in [CD-impl]; 0: GW_PI_FP64).
                               GW_PI_BF16X3 forms W^c = 2 b^T y + |y|^2 with
                               y = (L^-1 - I) b in BF16x3 products with FP32
                               accumulation (L the Cholesky factor of 1 - Pi), so
                               that its error is relative to W^c rather than to
                               |b|^2; adds 4 Np^2 bytes of workspace per grid point
                               of a chunk and 4 Rp Np bytes per context.  Other
                               values: GW_EINVAL. */
} gw_opts;

/* Imaginary-frequency quadrature: nodes xi[n] > 0 and d-xi weights w[n]
 * (no 1/pi), so that sum_g w_g h(xi_g) approximates int_0^inf h(xi) d xi. */
typedef struct gw_grid {
  int n;
  const double* xi;
  const double* w;
} gw_grid;

/* Modified Gauss-Legendre grid [CD-impl]: Gauss-Legendre nodes t_g, weights
 * u_g on [-1, 1] mapped by xi = x0 (1 + t)/(1 - t), w = u 2 x0/(1 - t)^2.
 * xi, w: caller arrays of length n.  Returns GW_EINVAL for n < 1 or
 * x0 <= 0.  (Host arithmetic only; no device needed.) */
int gw_grid_gauss_legendre(int n, double x0, double* xi, double* w);

/* Create a context holding one molecule on the current HIP device.
 *   n_mo, n_occ, n_aux: sizes (0 < n_occ < n_mo, n_aux >= 1)
 *   eps    [n_mo]                        Kohn-Sham levels, strictly ascending
 *   B_ov   [n_aux][n_occ*(n_mo-n_occ)]   (P|ia), column ia = i*n_virt + a   [RVF]
 *   row_ids[n_rows]                      states n whose rows are supplied (distinct)
 *   B_rows [n_rows][n_mo][n_aux]         (P|nm) for n = row_ids[r], every m
 *   opts   may be NULL (defaults)
 * On success *ctx owns device copies of everything it needs.
 * Errors: GW_EINVAL (sizes, ordering, non-finite values, duplicate rows),
 * GW_ENOMEM, GW_EDEVICE. */
int gw_setup(gw_ctx** ctx, int n_mo, int n_occ, int n_aux, const double* eps,
             const double* B_ov, int n_rows, const int* row_ids, const double* B_rows,
             const gw_opts* opts);

/* Setup from the full symmetric tensor B [n_aux][n_mo][n_mo], B[P][p][q] =
 * (P|pq) [RVF] (the orthonormalised three-index integrals that [Alg1]'s
 * initialisation produces).  The same as gw_setup with
 * B_ov[P][i*n_virt + a] = B[P][i][n_occ + a], row_ids = 0..n_mo-1 and
 * B_rows[n][m][P] = B[P][n][m], so that every state may be requested; the
 * rows of all states stay resident (n_mo * n_mo * n_aux doubles of device
 * memory).  B is read as given (rows from B[P][n][m]); it must be symmetric
 * in p, q.  Errors: as gw_setup. */
int gw_setup_full(gw_ctx** ctx, int n_mo, int n_occ, int n_aux, const double* eps,
                  const double* B, const gw_opts* opts);

/* Open-shell context [CD-impl] (Pi_PQ(omega) with its explicit sum over the
 * spin sigma; W_{mn sigma, mn sigma} and I_{nn sigma} per spin):
 * Pi(i xi) = -2 sum_s (P|ia s) D_s/(D_s^2 + xi^2) (ia s|Q), and a state of
 * spin s sees only the levels and occupation of spin s in its residue set,
 * residue frequencies and quadrature.
 *   n_occ [2]                  occupied levels of spin up, spin down
 *   eps   [2][n_mo]            levels of each spin, each row strictly ascending
 *   B_ov_up   [n_aux][n_occ[0]*(n_mo-n_occ[0])]   (P|ia up), column i*n_virt + a
 *   B_ov_down [n_aux][n_occ[1]*(n_mo-n_occ[1])]   (P|ia down)
 *   row_ids[n_rows]            spin-orbitals sigma*n_mo + n whose rows are supplied
 *   B_rows [n_rows][n_mo][n_aux]  (P|nm sigma) over the orbitals m of the row's spin
 *   opts   as for gw_setup; opts->dsig_x, if given, has 2*n_mo entries
 * Every other entry point then names states by spin-orbital index.  Both
 * spins' transitions share one Pi build, Cholesky, W^c table and MINRES
 * operator.  gw_footprint and the server cover closed-shell contexts only.
 * Errors: as gw_setup. */
int gw_setup_uhf(gw_ctx** ctx, int n_mo, const int* n_occ, int n_aux, const double* eps,
                 const double* B_ov_up, const double* B_ov_down, int n_rows, const int* row_ids,
                 const double* B_rows, const gw_opts* opts);

/* G0W0 quasiparticle energies [QP], [Alg1] with maxeviter = 0:
 * for each state n solves eps_QP = eps_n + dsig_x_n + Re Sigma^c_nn(eps_QP)
 * with Sigma^c = R - I [CD-theory]: the imaginary-axis term from the W^c
 * table on `grid` (Pi build -> Cholesky of 1 - Pi -> W^c, computed once per
 * grid and cached in the context) and the residue term from batched MINRES
 * at real frequencies, using the step-selection tree of [QP].
 *   states[n_states]: each must be one of the setup's row_ids
 *   outputs (caller arrays of length n_states): E_qp, sigma_c = Re Sigma^c at
 *   E_qp, Z = 1/(1 - dRe Sigma^c/d omega) at E_qp; status may be NULL.
 * Errors: GW_EINVAL, GW_ENOMEM, GW_EDEVICE, GW_ENOTSPD. */
int gw_qp(gw_ctx* ctx, int n_states, const int* states, const gw_grid* grid, double* E_qp,
          double* sigma_c, double* Z, int* status);

/* Eigenvalue self-consistent GW [Alg1] (its outer loop over maxeviter) in
 * the two flavours the Introduction names: evGW0 updates the energies in G
 * only, evGW in G and W.
 *   mode: GW_EVGW0 or GW_EVGW.  Cycle 1 solves the QP equations of `states`
 *   as gw_qp does; after every cycle the states' QP energies replace their
 *   eigenvalues in G (the residue set, the residue frequencies and the
 *   imaginary-axis term) and, for GW_EVGW, in the transition energies of Pi,
 *   so that the next cycle rebuilds W^c; the next cycle then solves again,
 *   starting from those energies.  The QP equation keeps gw_setup's eps_n as
 *   its constant term; states not requested keep their eigenvalues.
 *   The imaginary-axis term integrates the static part exactly: W^c is also
 *   built at xi = 0 (one more grid point), the quadrature takes
 *   W^c(i xi) - W^c(0) only and -(1/2) sum_m sgn(omega - eps_m) W^c_nm(0) is
 *   added, which stays accurate when omega sits next to a state's own moved
 *   pole (plain quadrature cannot resolve a/(a^2 + xi^2) there).  Cycle 1
 *   therefore differs from gw_qp by the quadrature error of the static part.
 *   Cycles stop after n_cycles (>= 1), or earlier once the largest change of
 *   a QP energy from the previous cycle is below ev_tol (>= 0; 0: never).
 *   Outputs (caller arrays of length n_states) as gw_qp's, from the last
 *   cycle; E_cycles (nullable) [n_cycles][n_states]: the QP energies of each
 *   cycle run (later rows untouched); cycles_done (nullable): cycles run.
 * On return, also on error, the context holds gw_setup's energies again; a
 * W^c table built from moved energies is dropped from its cache.
 * Closed-shell contexts only (GW_EINVAL for a gw_setup_uhf context).
 * Errors: as gw_qp; GW_ENOTSPD also when GW_EVGW's updated energies put an
 * occupied level at or above a virtual one. */
#define GW_EVGW0 0
#define GW_EVGW 1
int gw_evgw(gw_ctx* ctx, int mode, int n_cycles, double ev_tol, int n_states, const int* states,
            const gw_grid* grid, double* E_qp, double* sigma_c, double* Z, int* status,
            double* E_cycles, int* cycles_done);

/* G0W0 by the spectral-decomposition route [SD-impl], [SD-theory]: the
 * Hermitian Casida problem (A-B)^1/2 (A+B) (A-B)^1/2 T = Omega^2 T with
 * A - B = diag(D) and A + B = diag(D) + 4 B_ov^T B_ov (closed shell; an
 * open-shell context uses its spin-block form) is built and diagonalised on
 * the GPU (two-sided block Jacobi), the pole strengths w^s_nm of every
 * supplied row are formed, and the QP equations of `states` are solved with
 * the step tree of [QP] on the pole form
 *   Re Sigma^c_nn(omega) = sum_{i,s} (w^s_in)^2/(omega - eps_i + Omega_s)
 *                        + sum_{a,s} (w^s_an)^2/(omega - eps_a - Omega_s).
 * No frequency grid and no residue solves are involved.  The decomposition
 * is kept in the context until gw_reset_cache; it needs two N_ov x N_ov
 * FP64 matrices, and N_ov above 16384 is refused (GW_EINVAL): the route is
 * meant for small systems.  Outputs as gw_qp's.
 * Errors: GW_EINVAL, GW_ENOMEM, GW_EDEVICE (no Jacobi convergence). */
int gw_qp_sd(gw_ctx* ctx, int n_states, const int* states, double* E_qp, double* sigma_c,
             double* Z, int* status);

/* The RPA excitation energies Omega_s [SD-impl] of the context, ascending:
 * Omega [N_ov], N_ov = n_occ * n_virt (open shell: the sum over spins). */
int gw_rpa_excitations(gw_ctx* ctx, double* Omega);

/* Release the context and all of its device memory.  NULL is ignored. */
void gw_free(gw_ctx* ctx);

/* Text describing the last nonzero return of this thread ("" if none). */
const char* gw_last_error(void);

/* Select the precision of subsequent Pi builds (GW_PI_*); invalidates the
 * cached W^c table.  GW_EINVAL for an unknown value. */
int gw_set_pi_prec(gw_ctx* ctx, int pi_prec);

/* Device memory (bytes requested from the allocator) that a context of
 * these sizes uses over gw_setup plus gw_qp of up to n_states states on a
 * grid of grid_n points with these options (NULL: defaults).  Setting
 * opts->mem_budget_bytes to this value never makes such a context fail
 * with GW_ENOMEM.  Returns 0 for invalid sizes. */
size_t gw_footprint(int n_mo, int n_occ, int n_aux, int n_rows, int n_states, int grid_n,
                    const gw_opts* opts);

/* Drop the cached W^c table: the next gw_qp / gw_sigma / gw_wtable call
 * rebuilds it (Pi build, Cholesky, reduction) from the resident inputs. */
int gw_reset_cache(gw_ctx* ctx);

/* ---- stage entry points (the same kernels gw_qp runs; for parity checks
 *      and tooling) ------------------------------------------------------- */

/* The dielectric matrices 1 - Pi(i xi_g) [CD-impl], Pi = -4 sum_ia
 * (P|ia) D_ia/(D_ia^2 + xi^2) (ia|Q) (closed-shell spin sum, eta -> 0+), in
 * the context's Pi precision.  out: [n_xi][n_aux][n_aux], lower triangle
 * written (the strict upper triangle is set to 0). */
int gw_dielectric(gw_ctx* ctx, int n_xi, const double* xi, double* out);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): gw_dielectric without any
 * allocation, asynchronous on the context's stream.  d_xi: [n_xi] device
 * array; d_out: caller's device buffer, matrix g at d_out + g * out_stride
 * with rows of ld_out doubles (ld_out >= N_aux padded to 128, even;
 * out_stride >= that padded N_aux times ld_out); the lower triangle of the
 * padded matrix 1 - Pi(i xi_g) is written (rows and columns past N_aux are
 * the identity's), the strict upper triangle is left as it was.  The scale
 * vectors go into a 32 MiB device array of the library, one per GPU, held
 * until the process ends: n_xi * Kp * 8 bytes (12 for the FP32 and BF16x3
 * builds, Kp = n_occ n_virt padded to 128) must fit, else GW_EINVAL names
 * the limit.  The FP32 / BF16x3 builds need the context's split copies of
 * B_ov, made by a first gw_dielectric, gw_wtable or gw_qp (GW_EINVAL
 * otherwise).  Calls on one GPU share that array, so calls that overlap in
 * time on one GPU (different streams) race; serialise them. */
int gw_dielectric_noalloc(gw_ctx* ctx, int n_xi, const double* d_xi, double* d_out,
                          long ld_out, long out_stride);

/* Cholesky factors L_g of 1 - Pi(i xi_g): out [n_xi][n_aux][n_aux] lower
 * triangular (upper set to 0). */
int gw_cholesky(gw_ctx* ctx, int n_xi, const double* xi, double* out);

/* The screened-interaction table W^c_nm(i xi_g) = b^T[(1 - Pi)^-1 - 1]b,
 * b = (P|nm) [CD-impl], [Alg1], for every supplied row n and every m:
 * out [n_rows][n_mo][grid->n].  Also fills the context's cache. */
int gw_wtable(gw_ctx* ctx, const gw_grid* grid, double* out);

/* Re Sigma^c_nn(omega) and its omega-derivative at fixed real frequencies
 * (one omega per entry; states may repeat) [CD-theory], [Alg1]:
 *   sigma, dsigma: [n] outputs; n_res (nullable): residues used per entry.
 * The residue term uses batched MINRES (with the dense fallback). */
int gw_sigma(gw_ctx* ctx, int n, const int* states, const double* omega, const gw_grid* grid,
             double* sigma, double* dsigma, int* n_res);

/* Batched residue solves [CD-impl]: for j < k, x_j solves
 * (1 - Pi(w_j)) x_j = b_j with b_j = (P|n_j m_j), Pi(w) = -4 sum_ia (P|ia)
 * D/(D^2 - w^2) (ia|Q).  Outputs (nullable each):
 *   x [k][n_aux], wc [k] = b^T x - b^T b, dwc [k] = x^T (dPi/dw) x,
 *   iters [k] = MINRES iterations (negative: did not converge; the dense
 *   fallback was used when use_fallback != 0). */
int gw_residues(gw_ctx* ctx, int k, const int* states, const int* m, const double* w,
                int use_fallback, double* x, double* wc, double* dwc, int* iters);

/* Per-context timing of the last gw_qp / gw_evgw / gw_wtable call,
 * milliseconds, measured with HIP events on the context stream (stage times
 * summed over the W^c builds of the call). */
typedef struct gw_timing {
  double pi_ms, chol_ms, wtab_ms, quad_ms, minres_ms, fallback_ms, total_ms;
  int qp_rounds, minres_iters, minres_systems, fallback_systems, wtab_cached;
  double sd_ms;     /* spectral-decomposition build (Casida matrix, Jacobi, pole strengths) */
  int sd_sweeps;    /* block-Jacobi sweeps of that build */
  /* the Pi-build kernel and the W^c kernel (FP64 GEMM or BF16x3 contraction)
   * alone, summed over their launches, and the number of launches of each
   * (one per stage-A chunk) */
  double pi_kernel_ms, wc_kernel_ms;
  int pi_launches, wc_launches;
} gw_timing;
int gw_get_timing(gw_ctx* ctx, gw_timing* out);

/* ---- serving ------------------------------------------------------------
 * A request server for molecules of uneven size arriving over time (not in
 * the paper, whose runs are one molecule per job).  gw_server_submit copies
 * the request and returns at once.  Requests are admitted first come, first
 * served when a pipeline slot is free and their device-memory footprint
 * (gw_footprint) fits in the remaining budget; each admitted request keeps
 * its inputs, W^c table and workspaces resident until it completes, and its
 * context may not allocate past its reserved footprint.  Up to n_streams
 * pipelines run at once, each on its own HIP stream, so the work of requests
 * admitted while others are on the GPU overlaps with theirs.
 * Small requests (N_aux up to batch_max_aux) are batched: when one is
 * admitted, every pending request of the same padded shape (N_aux, n_occ n_virt
 * and n_rows n_mo, each padded to 128) joins it, up to a batch size the
 * shape's workspace allows, and when that makes two or more, their stage A
 * (the Pi build, Cholesky and W^c table on every grid point) runs as one set
 * of launches over all their grid points, replayed from a graph captured for
 * that shape and batch size.  Each
 * request's quasiparticle stage then runs on whichever pipeline is free.
 * Results are those of gw_qp on the request alone, bit for bit.  Device and
 * pinned host blocks are kept by the server and reused across requests, so a
 * stream of recurring shapes runs without hipMalloc / hipFree once warm.  The
 * server is internally synchronised. */
typedef struct gw_server gw_server;

typedef struct gw_server_opts {
  int pi_prec, minres_max_iter, qp_max_iter;  /* as in gw_opts (0: defaults) */
  double minres_rtol, qp_tol;                 /* as in gw_opts (0: defaults) */
  int grid_n;                                 /* imaginary grid shared by all requests */
  const double* grid_xi;                      /* [grid_n], copied */
  const double* grid_w;                       /* [grid_n], copied */
  size_t mem_budget_bytes;  /* admission budget; 0: 80% of free device memory */
  int n_streams;            /* concurrent request pipelines, 1..4 (0: 2) */
  size_t work_budget_bytes; /* stage-A workspace cap per request (0: 2 GiB) */
  int wc_prec;              /* as in gw_opts (0: FP64) */
  int batch_max_aux;        /* requests whose N_aux, padded to 128, is at most this
                               run stage A batched with others of their padded shape
                               (0: 768; negative: never batched) */
} gw_server_opts;

typedef struct gw_request {
  int n_mo, n_occ, n_aux;
  const double* eps;      /* [n_mo] */
  const double* B_ov;     /* [n_aux][n_occ*n_virt] */
  int n_rows;
  const int* row_ids;     /* [n_rows] */
  const double* B_rows;   /* [n_rows][n_mo][n_aux] */
  int n_states;
  const int* states;      /* [n_states], each among row_ids */
  const double* dsig_x;   /* [n_mo] or NULL */
} gw_request;

typedef struct gw_request_info {
  int rc;                 /* 0, or the GW_E* code the request failed with */
  size_t footprint_bytes; /* reserved device memory while resident */
  double t_submit, t_admit, t_done;  /* seconds on the server clock */
  int slot;               /* pipeline (stream) that ran it */
} gw_request_info;

typedef struct gw_server_stats {
  unsigned long long submitted, completed, failed;
  size_t budget_bytes, reserved_bytes, peak_reserved_bytes;
  int active, peak_active;
  long batches;             /* grouped stage-A launches (graph replays or captures) */
  long batched_requests;    /* requests whose stage A ran in such a batch */
  long graph_replays;       /* batches that replayed an already captured graph */
  long device_mallocs;      /* device and pinned blocks the server obtained from the
                               runtime (each later reuse of a block is a cache hit) */
  long cache_hits;
  long device_frees;        /* cached device blocks given back to the runtime to make
                               room (each such hipFree waits for the whole device) */
  size_t cached_bytes;      /* device bytes held in the cache, not in use */
} gw_server_stats;

/* GW_EINVAL for bad options, GW_EDEVICE if no device or stream is usable. */
int gw_server_create(gw_server** s, const gw_server_opts* opts);
/* Checks the request's inputs as gw_setup does, then copies them (into
 * pinned host memory from a pool the server reuses, while it stays within
 * 64 GiB; pageable memory beyond) on the calling thread; *ticket identifies
 * the request.  GW_EINVAL for a malformed request, GW_ENOMEM if its footprint
 * exceeds the whole budget. */
int gw_server_submit(gw_server* s, const gw_request* r, unsigned long long* ticket);
/* 1 while pending or running; 0 when done: E_qp, sigma_c, Z, status
 * ([n_states] each, each nullable) and info (nullable) are filled and the
 * ticket is released.  A request that failed returns 0 with info->rc < 0. */
int gw_server_poll(gw_server* s, unsigned long long ticket, double* E_qp, double* sigma_c,
                   double* Z, int* status, gw_request_info* info);
/* Blocks until every submitted request has finished. */
int gw_server_drain(gw_server* s);
int gw_server_get_stats(gw_server* s, gw_server_stats* out);
/* Seconds since the server was created (the clock of gw_request_info). */
double gw_server_clock(gw_server* s);
/* Drains, stops the pipelines and frees everything. */
void gw_server_destroy(gw_server* s);

#ifdef __cplusplus
}
#endif
#endif /* GW_H */
