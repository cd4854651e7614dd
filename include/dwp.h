/*
 * dwp.h -- C ABI of the MI355X dry/wet generalized-Poisson library (libdwp.so).
 *
 * The library solves the generalized Poisson problem of the paper's continuum
 * solvent model, div(eps grad phi) = -4 pi rho (Eq. 3), on a periodic 3-D grid,
 * with the paper's split of the cell into a solvent-free ("dry") part handled
 * by a periodic FFT Poisson solve (Eq. 15) and a solvated ("wet") slab handled
 * by multigrid with boundary data from the dry solution (Sec. II.F); the two
 * are iterated to self-consistency on the full box.  It also returns the
 * Hartree energy E = 1/2 int phi rho (Sec. II.C, equal to Eq. 4 at the
 * solution), its derivative with respect to the permittivity (first term of
 * Eq. 11) and the atomic forces dE/dR (Eq. 11, derived in Appendix B).
 *
 * Conventions shared by every entry point:
 *   - lengths in Angstrom, charges in e, energies in e^2/Angstrom
 *     (multiply by 14.399645 for eV);
 *   - grids are float64 arrays laid out [nz][ny][nx] with x fastest; node
 *     (i, j, k) sits at (i hx, j hy, k hz), h_d = L_d / n_d, all directions
 *     periodic;
 *   - "_dev" pointers are device (HBM) pointers on the context's device,
 *     owned by the caller, 8-byte aligned, dense; "_host" pointers are host
 *     memory, owned by the caller and only read or written during the call;
 *   - all device work is enqueued on the context's stream; entry points that
 *     return host values (energy, forces, info) synchronise that stream;
 *   - every function returns a dwp_status; nothing throws across the ABI.  On
 *     error the context stays usable and dwp_last_error() describes the
 *     failure.  Arguments are validated before any device work is issued.
 *   - a context is not thread-safe; use one context per stream.
 *
 * Discretisation (the paper's Eq. 3 written in conservative form):
 *   (A phi)_n = sum_d [eps_{n+e_d/2} (phi_{n+e_d} - phi_n)
 *                      - eps_{n-e_d/2} (phi_n - phi_{n-e_d})] / h_d^2,
 *   eps_{n+e_d/2} = (eps_n + eps_{n+e_d}) / 2.
 * The solution is the unique zero-mean phi with A phi = -4 pi (rho - mean rho):
 * a uniform neutralising background, the G = 0 convention of Eq. 15.
 */
#ifndef DWP_H
#define DWP_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dwp_ctx dwp_ctx; /* opaque, library-owned */

typedef enum {
    DWP_OK = 0,
    DWP_EINVAL = -1,     /* an argument is out of range or inconsistent        */
    DWP_ESTATE = -2,     /* called before set_grid / set_epsilon / solve       */
    DWP_ENOCONV = -3,    /* tolerance not reached; best iterate returned       */
    DWP_EHIP = -4,       /* the HIP runtime reported an error                  */
    DWP_ENOMEM = -5,     /* device allocation failed                          */
    DWP_ENONFINITE = -6  /* NaN or Inf found in an input or a residual        */
} dwp_status;

typedef enum { DWP_FP64 = 0, DWP_MIXED = 1 } dwp_precision;

/* Solver options.  dwp_default_opts() fills every field. */
typedef struct {
    int precision;         /* DWP_FP64, or DWP_MIXED: the multigrid hierarchy
                              (smoothing, inner residuals, transfers, coarse
                              solve) in float32 inside the float64 Krylov
                              coupling; the full-box residual, the wet-slab
                              residual, the FFT dry update, the coupling update
                              and the energy stay float64                      */
    double z_wet_lo;       /* wet slab W = [z_wet_lo, z_wet_hi) (Angstrom);    */
    double z_wet_hi;       /* z_wet_hi may exceed Lz: W then wraps through 0.  */
                           /* The first wet plane is ceil(z_wet_lo / hz), the  */
                           /* plane past the last one ceil(z_wet_hi / hz); the */
                           /* library may move the first plane down by a few   */
                           /* planes so that W coarsens well (info reports it) */
    int pre, post;         /* red-black Gauss-Seidel sweeps per V-cycle level  */
    int coarse_sweeps;     /* sweeps on the coarsest level                     */
    int max_levels;        /* upper bound on multigrid levels (>= 1)           */
    int cycles;            /* V-cycles per application of the split (0..64;    */
                           /* 0: no wet correction, the split is the FFT dry   */
                           /* update alone; many: the wet solve converges and  */
                           /* one application is the paper's one-pass scheme)  */
    int scaled_dry;        /* 1: dry update s * L^-1 (s * r), s = eps^-1/2     */
    double tol;            /* stop at ||b - A phi||_2 <= tol ||b||_2           */
    int max_outer;         /* cap on preconditioned Krylov iterations          */
    int restart;           /* FGMRES restart length m (1..63)                  */
    int warm_start;        /* 1: phi_dev holds the initial guess on entry      */
    int profile;           /* 1: time every kernel group with HIP events on    */
                           /* the context stream (see dwp_profile); 2: only    */
                           /* the fine-level smoother (least overhead); 0 off  */
    int smoother;          /* red-black Gauss-Seidel on the large levels:      */
                           /* 1 = one fused pass per sweep (out of place), on  */
                           /* blocks of whole grid rows where that shape fits  */
                           /* (nx a multiple of the vector width, at most 1024 */
                           /* threads, an even band height dividing ny), else  */
                           /* on 32 x 16 tiles; 2 = the fused pass on tiles    */
                           /* always; 0 = one launch per colour (in place);    */
                           /* all give the same sweep up to rounding           */
    int fft_fp32;          /* 1 (mixed precision only): the FFT dry update     */
                           /* runs its spectrum and transforms in float32; the */
                           /* real input and output stay float64.  0: float64  */
    int order;             /* operator: 2 = the conservative 7-point form      */
                           /* (default); 6 = the paper's sixth-order           */
                           /* non-conservative form (Eqs. 16-18):              */
                           /* A6 phi = sum_d (D1_d eps)(D1_d phi) + eps D2_d phi */
                           /* with seven-point central D1, D2.  A6 is not      */
                           /* symmetric and its range misses the constants by  */
                           /* O(h^6): the solve returns the zero-mean phi with */
                           /* A6 phi = b - c for a constant c (info.background)*/
                           /* and the residual is measured after removing its  */
                           /* mean.  The dry update then uses the symbol of    */
                           /* Eq. 18 (exact for eps = 1); the wet multigrid    */
                           /* keeps the 7-point operator (a preconditioner).   */
                           /* Gradients and forces solve the adjoint problem   */
                           /* once per solve.  Needs eps resolved by the grid. */
                           /* The 7-point wet V-cycle is a poor approximation  */
                           /* of A6 near the switch functions: on the slab     */
                           /* workloads cycles = 0 (the FFT dry update alone)  */
                           /* with scaled_dry = 0 converges fastest, and with  */
                           /* the exclusion rule of Eq. 19 every cycles >= 1   */
                           /* setting stalls (DWP_ENOCONV at max_outer).       */
    int smooth6;           /* order 6 only: 1 = the finest wet level smooths   */
                           /* (weighted Jacobi, weight 2/3) and forms the      */
                           /* residual it restricts with the sixth-order       */
                           /* operator itself, zero Dirichlet data on the      */
                           /* three planes beyond W; the coarser levels keep   */
                           /* the 7-point operator (so does the adjoint solve  */
                           /* of dwp_eps_gradient / dwp_forces).  0 = 7-point  */
                           /* everywhere                                       */
    int krylov_fp32;       /* mixed precision, restart <= 16 (order 6: with    */
                           /* cycles = 0 only): 1 =                            */
                           /* the Krylov bases V and Z are stored in float32   */
                           /* (every dot product, the Hessenberg matrix, the   */
                           /* operator's arithmetic and the iterate stay       */
                           /* float64; every restart recomputes the true       */
                           /* residual in float64).  0 = float64 bases         */
    int krylov_fp16;       /* with krylov_fp32 = 1 and the second-order        */
                           /* operator: 1 = the Arnoldi basis V of a restart   */
                           /* cycle is stored in float16 (Z stays float32, the */
                           /* current vector is kept in float32 too for the    */
                           /* preconditioner; the arithmetic is as above, the  */
                           /* true residual is still recomputed in float64 at  */
                           /* every restart, so the tolerance still holds for  */
                           /* the float64 residual), except any cycle after    */
                           /* one that reduced the residual more than 100-fold */
                           /* and the first cycle of a solve unless the first  */
                           /* cycle of the context's previous solve reduced it */
                           /* less: there a float16 basis would limit the      */
                           /* cycle, which runs on the float32 basis.          */
                           /* 0 = as krylov_fp32 says                          */
    double semi_ratio;     /* multigrid coarsening: a level halves z too only  */
                           /* once hz <= semi_ratio * max(hx, hy) (before,     */
                           /* only x and y: semi-coarsening for anisotropic    */
                           /* spacing); 1..64, default sqrt(2).  A larger      */
                           /* value coarsens z sooner: cheaper cycles, weaker  */
                           /* where the wet solve limits the iteration count   */
} dwp_opts;

/* Per-solve report. */
typedef struct {
    int outer_iters;         /* Krylov iterations = applications of the split  */
                             /* (whole restart cycles: a cycle runs all its    */
                             /* steps before the residual is checked)          */
    int vcycles;             /* V-cycles run                                   */
    int restarts;            /* FGMRES cycles                                  */
    int k_w0, k_w1;          /* wet planes actually used: [k_w0, k_w1) mod nz  */
    int n_levels;            /* multigrid levels on W                          */
    double rel_res;          /* final ||b - A phi||_2 / ||b||_2 (true residual)*/
    double energy;           /* E = 1/2 h^3 sum rho phi                        */
    double energy_eps_form;  /* (h^3 / 8 pi) sum_faces eps_f (D_f phi)^2       */
    double mean_rho_removed; /* mean of rho that was projected out            */
    double t_total_ms;       /* wall time of the solve                         */
    double background;       /* order 6: c = mean(b - A6 phi); order 2: 0      */
    /* Device time of the solve's phases, from HIP events recorded on the   */
    /* context stream at the phase boundaries of every Krylov step:         */
    double t_fft_ms;         /* the FFT dry updates (Eq. 15 on the grid)       */
    double t_mg_ms;          /* wet residual, V-cycles and the combination     */
    double t_krylov_ms;      /* operator applications, Gram-Schmidt, restarts  */
                             /* (together: the solve from its first residual   */
                             /* to its last update, setup and energy excluded) */
} dwp_info;

/* Permittivity built from the atoms (dwp_build_epsilon), two models.
 *
 * model 0 (product of switches):
 *   eps_n = 1 + (eps_inf - 1) * prod_i s_i(d_in) * H(z_n),
 *   s_i(d) = 1/2 [1 + erf((d - r_i) / delta)], d_in the minimum-image distance,
 * a product of smooth switches that plays the role of the paper's
 * atom-defined dielectric (Eqs. 9-10).  s_i is taken as exactly 0 below
 * r_i - 6 delta and exactly 1 beyond r_i + 6 delta.  With exclusion = 1 every
 * atom with z_i <= z_lim ("buried") adds the height factor
 *   h_i(z) = 1/2 [1 + erf((z - z_i) / delta_z)],  H(z) = prod_buried h_i(z),
 * with z the node height in [0, Lz): the smooth counterpart of Eq. 19, which
 * drives eps to 1 underneath the buried atoms so that the region below the
 * exposed face is really dry (Sec. II.F).  exclusion = 0 gives H = 1.
 *
 * model 1 (the paper's own form, Sec. II.E): the dummy density of Eq. 9 fed
 * into Eq. 10,
 *   gamma_n = sum_i exp(-s_in (d_in - R_i) / a),
 *   eps_n = 1 + (eps_inf - 1) / (1 + gamma_n^(2 beta)),
 * with R_i = radius_host[i] the van der Waals radius, a = decay the length
 * unit of the exponent (1 bohr = 0.529177 Angstrom in the paper's atomic
 * units), d_in the minimum-image distance (one term per atom) and s_in = 1,
 * except that with exclusion = 1 a buried atom (z_i <= z_lim) has
 * s_in = -1 at the nodes below it (z_n < z_i, heights in [0, Lz)): the solvent
 * exclusion of Eq. 19, which saturates eps to 1 under the buried atoms.  Its
 * force term is the derivative of this eps (the sign of the printed Eq. 12 is
 * reversed); where a buried atom's z crosses a grid plane eps jumps, and the
 * force is the derivative of the smooth pieces.  delta and delta_z are not
 * used.  Needs 0.5 < beta <= 100, decay > 0, at most 4096 atoms, and the
 * half-diagonal of the cell below 600 decay lengths (no overflow). */
typedef struct {
    double eps_inf;  /* bulk solvent permittivity (> 1)            */
    double delta;    /* switch width (Angstrom, > 0; model 0)      */
    int exclusion;   /* 0 or 1                                     */
    double z_lim;    /* buried atoms: z_i <= z_lim                 */
    double delta_z;  /* width of the height factor (Angstrom, > 0; model 0) */
    int model;       /* 0: product of switches; 1: Eqs. 9, 10, 19  */
    double beta;     /* exponent of Eq. 10 (model 1)               */
    double decay;    /* length unit of Eq. 9 (Angstrom; model 1)   */
} dwp_eps_params;

/* Defaults: FP64, W = [0.35 Lz, Lz), V(2,2), 64 coarse sweeps, 1 cycle,
 * unscaled dry update, tol 1e-10, 600 iterations, restart 10, cold start,
 * profiling off, fused sweeps. */
void dwp_default_opts(dwp_opts *opts);

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t (or
 * NULL for the null stream), typically torch's current stream. */
int dwp_create(dwp_ctx **ctx, int device, void *hip_stream);
int dwp_destroy(dwp_ctx *ctx);
/* Change the stream later calls enqueue on. */
int dwp_set_stream(dwp_ctx *ctx, void *hip_stream);

/* Fix the grid and plan the solver (Sec. II.F: FFT plan for the whole cell,
 * multigrid hierarchy for the wet slab).  Each n_d must be even, at least 8,
 * with no prime factor other than 2 and 3 and at most 4096; L_d > 0; W must
 * leave at least one dry plane and hold at least 3 planes.  Allocates all
 * device memory the solver needs (about (2 restart + 14) N doubles).
 * Invalidates epsilon and the last solution. */
int dwp_set_grid(dwp_ctx *ctx, int nx, int ny, int nz, double Lx, double Ly, double Lz,
                 const dwp_opts *opts);
/* Replace the options of the current grid (the wet slab may change). */
int dwp_set_opts(dwp_ctx *ctx, const dwp_opts *opts);

/* Use a caller-supplied node permittivity grid (copied; >= 1 and finite,
 * else DWP_EINVAL / DWP_ENONFINITE). */
int dwp_set_epsilon(dwp_ctx *ctx, const double *eps_dev);

/* Build eps from n atoms (xyz_host: n x 3, radius_host: n), see
 * dwp_eps_params.  The result stays in the context; dwp_get_epsilon copies it
 * out. */
int dwp_build_epsilon(dwp_ctx *ctx, int n, const double *xyz_host, const double *radius_host,
                      const dwp_eps_params *params);
int dwp_get_epsilon(dwp_ctx *ctx, double *eps_dev);

/* Density-dependent permittivity (Secs. II.C-II.D): eps_n = eps(rho_n) by Eq. 7,
 *   eps(rho) = 1 + (eps_inf - 1)/2 (1 + (1 - (rho/rho0)^(2 beta)) / (1 + (rho/rho0)^(2 beta))),
 * from an electron-density grid rho_dev (N doubles on the device, the grid's
 * x-fastest layout; read only during the call; negative values are read as
 * zero density).  Also stores d eps/d rho (Eq. 8) in the context for
 * dwp_v_eps.  eps_inf >= 1, rho0 > 0 and 0.5 < beta <= 1000 (2 beta > 1 keeps
 * Eq. 8 finite at zero density), else DWP_EINVAL; a non-finite density gives
 * DWP_ENONFINITE.  Replaces any earlier eps; dwp_forces then takes no
 * permittivity term (params must be NULL, or DWP_ESTATE). */
int dwp_build_epsilon_density(dwp_ctx *ctx, const double *rho_dev, double eps_inf, double rho0,
                              double beta);

/* V_eps of Eq. 6 for the last solution, on the grid: the derivative of the
 * discrete energy with respect to the density that enters eps, per unit
 * volume,
 *   V_eps,n = (dE/d eps_n / h^3) (d eps/d rho)_n
 *           = -(1/8 pi) sum_d 1/2 [(D+_d phi)_n^2 + (D-_d phi)_n^2] (d eps/d rho)_n,
 * written to out_dev (N doubles, device).  add_phi = 1 adds phi_n: the
 * density derivative of E per unit volume when the same density is the
 * source and the argument of eps (Eq. 5).  DWP_ESTATE unless eps came from
 * dwp_build_epsilon_density and dwp_solve has run since. */
int dwp_v_eps(dwp_ctx *ctx, int add_phi, double *out_dev);

/* Gaussian charges (the smeared ionic densities of Sec. II.C, here with
 * sigma_i a standard deviation): rho_n = sum_i q_i (2 pi sigma_i^2)^(-3/2)
 * exp(-d_in^2 / (2 sigma_i^2)), minimum image, cut off at 9 sigma_i
 * (sigma_i must be below min(L)/18).  Writes N doubles to rho_dev. */
int dwp_build_rho(dwp_ctx *ctx, int n, const double *xyz_host, const double *q_host,
                  const double *sigma_host, double *rho_dev);

/* Solve A phi = -4 pi (rho - mean rho) to the tolerance of the options.
 * phi_dev (N doubles) receives the zero-mean solution; with warm_start it
 * also supplies the initial guess.  *energy_host (nullable) receives
 * E = 1/2 h^3 sum rho phi, *info (nullable) the report.  Returns DWP_ENOCONV
 * with the best iterate in phi_dev if max_outer is reached. */
int dwp_solve(dwp_ctx *ctx, const double *rho_dev, double *phi_dev, double *energy_host,
              dwp_info *info);

/* Vector-Jacobian product of the map (rho, eps) -> (phi, E) of dwp_solve at
 * its solution, for the symmetric second-order operator (order 2; order 6
 * gives DWP_EINVAL): given the cotangents g_E of E and g_phi of phi,
 *   grad_rho = g_E h^3 phi - 4 pi lambda,
 *   grad_eps_n = sum_d 1/2 [(D+_d u)_n (D+_d phi)_n + (D-_d u)_n (D-_d phi)_n],
 *   u = lambda - g_E (h^3 / 8 pi) phi,
 * where lambda is the zero-mean solution of A lambda = g_phi - mean(g_phi)
 * (the adjoint problem of Eq. 3; A is symmetric), solved by the same coupled
 * FFT/multigrid iteration with the current options, from zero.  The g_E
 * terms are dE/d rho (Sec. II.C) and dE/d eps (first term of Eq. 11); the
 * lambda terms the derivative of a loss through phi.  phi_dev must be the
 * solution of the current eps (the caller keeps it; the library reads it),
 * g_phi_dev may be NULL (lambda = 0), grad_rho_dev and grad_eps_dev receive
 * N doubles each.  Does not change the state dwp_eps_gradient, dwp_forces
 * and dwp_v_eps read (the last solution), only scratch buffers.  *info
 * (nullable) reports the adjoint solve; DWP_ENOCONV if it misses the
 * tolerance (outputs written from the best iterate). */
int dwp_backward(dwp_ctx *ctx, const double *phi_dev, double g_E, const double *g_phi_dev,
                 double *grad_rho_dev, double *grad_eps_dev, dwp_info *info);

/* dE/d eps_n = -(h^3 / 8 pi) sum_d 1/2 [(D+_d phi)_n^2 + (D-_d phi)_n^2] for
 * the last solution (the discrete first term of Eq. 11).  N doubles.  With
 * order 6: dE/d eps_n = sum_d D1_d(lambda D1_d phi)_n - lambda_n (sum_d D2_d
 * phi)_n with lambda the zero-mean solution of Q A6^T lambda = h^3/2 Q rho
 * (Q removes the mean), solved on the first call after a solve. */
int dwp_eps_gradient(dwp_ctx *ctx, double *dEdeps_dev);

/* out_n = scale * sum_d 1/2 [(D+_d a)_n (D+_d b)_n + (D-_d a)_n (D-_d b)_n]:
 * -d(a.A b)/d eps_n times scale (no h^3 factor), for two grids a, b (N
 * doubles each).  With a = b = phi and scale = -h^3/(8 pi) it is
 * dwp_eps_gradient; with a = lambda (an adjoint solution) it gives the
 * permittivity gradient of a loss that depends on phi itself.  It is the
 * derivative of the second-order operator (order 2) whatever the options. */
int dwp_eps_pair_gradient(dwp_ctx *ctx, const double *a_dev, const double *b_dev, double scale,
                          double *out_dev);

/* dE/dR (n x 3, host) for the last solution: sum_n (dE/d eps_n) d eps_n/dR_I
 * + h^3 sum_n phi_n d rho_n / dR_I (Eq. 11).  The atoms and parameters must
 * be those eps and rho were built from: the switch term reuses the switch
 * product stored by dwp_build_epsilon, and positions, radii or parameters
 * that differ from that build give DWP_ESTATE.  params == NULL means eps does
 * not depend on the atoms (caller-supplied eps): only the charge term is
 * returned.  Forces are F = -dE/dR. */
int dwp_forces(dwp_ctx *ctx, int n, const double *xyz_host, const double *radius_host,
               const double *q_host, const double *sigma_host, const dwp_eps_params *params,
               double *dEdR_host);

/* dwp_forces for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, result and kernels as dwp_forces, but the packed atoms (8 n
 * doubles), the force partial sums and the device copy of dE/dR (3 n doubles)
 * live in a static device array of 2^21 doubles (16 MiB) that every GPU the
 * library runs on holds until the process ends; the call makes no device
 * allocation of any kind (dwp_forces grows context buffers to fit n).  Inputs
 * that need more scratch than that give DWP_EINVAL before any device work:
 * about 8 n + 3 max(n, 8192) + 3 n + nz doubles with the switch model or a
 * caller eps (up to ~1.4e5 atoms), plus 6144 n with model 1 (up to ~330
 * atoms).  Second-order operator only (order 6 gives DWP_EINVAL).  Every call
 * on one GPU, from any context, shares that GPU's array and leaves its
 * contents behind; each call writes every slot before reading it, so nothing
 * needs clearing, but calls that overlap on one GPU (two streams or two host
 * threads) race and must be serialised by the caller. */
int dwp_forces_noalloc(dwp_ctx *ctx, int n, const double *xyz_host, const double *radius_host,
                       const double *q_host, const double *sigma_host, const dwp_eps_params *params,
                       double *dEdR_host);

/* Building blocks, exposed for checking and for callers that compose them.
 * dwp_apply_operator applies the operator of the options (order 6: A6, without
 * the removal of the mean); dwp_vacuum_solve inverts the vacuum operator of
 * that order (the 7-point or the Eq. 18 symbol). */
/* out = A phi on the full periodic box with the current eps. */
int dwp_apply_operator(dwp_ctx *ctx, const double *phi_dev, double *out_dev);
/* out = zero-mean psi with L psi = r - mean r, L the vacuum operator (the
 * 7-point Laplacian, or sum_d D2_d of Eq. 18 with order 6),
 * by the library's 3-D FFT and discrete Green's function (Eq. 15 on the
 * grid), with the spectrum in float32 when opts.fft_fp32 is set (as inside
 * the split; input and output stay float64), else in float64. */
int dwp_vacuum_solve(dwp_ctx *ctx, const double *r_dev, double *out_dev);
/* out = one application of the dry/wet split to r (the preconditioner of the
 * coupled iteration). */
int dwp_apply_split(dwp_ctx *ctx, const double *r_dev, double *out_dev);
/* E = 1/2 h^3 sum rho phi (compensated, deterministic). */
int dwp_energy(dwp_ctx *ctx, const double *rho_dev, const double *phi_dev, double *energy_host);

/* Kernel-group timings gathered while opts.profile = 1 (HIP events recorded
 * around each launch on the context stream).  Group g in [0, dwp_profile_count()):
 * *name receives a static string, *ms the summed launch durations, *launches
 * the number of launches, *bytes the algorithmic HBM bytes those launches
 * must move (the minimum traffic of the operation, not a counter reading).
 * dwp_profile_reset() clears the sums. */
int dwp_profile_count(void);
int dwp_profile_get(dwp_ctx *ctx, int group, const char **name, double *ms, long *launches, double *bytes);
int dwp_profile_reset(dwp_ctx *ctx);

/* Validate a grid and options on the host and report the solver plan without
 * touching a device: out[0] = first wet plane k_w0 (in [0, nz)), out[1] =
 * k_w1 (W = planes [k_w0, k_w1) mod nz), out[2] = number of multigrid levels
 * nl, then (nx, ny, nw) of each level.  out_len must be >= 3 + 3 nl (100 is
 * always enough).  Errors are described by dwp_last_error(NULL). */
int dwp_plan(int nx, int ny, int nz, double Lx, double Ly, double Lz, const dwp_opts *opts, int *out,
             int out_len);

/* Message of the last failure on this context (ctx-owned, valid until the
 * next call).  Also accepts NULL (then describes the last dwp_create error). */
const char *dwp_last_error(const dwp_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* DWP_H */
