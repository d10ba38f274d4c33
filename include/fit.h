/*
 * fit.h -- C ABI of the MI355X matrix-free frequency-domain FIT library.
 *
 * The library applies and inverts the complex curl-curl operator of the
 * Finite Integration Technique,
 *
 *     A(omega) = C^T M_nu C  -  omega^2 M_eps  +  j omega M_sigma,
 *
 * (Geranmayeh, Sec. II: grid equations, eq. (CP) for the curl C with
 * dual curl C^T, eq. (Material) for the diagonal material matrices, eq. (e2)
 * for the wave equation with s = j*omega) on a non-equidistant Cartesian
 * primal/dual grid pair, without ever storing A, C or the material diagonals:
 * every entry is recomputed from the cell spacings and a per-cell material
 * id each time the operator is applied (Sec. III, the matrix-free operator of
 * eq. (e2t)).  Around the operator it runs the Krylov methods the paper
 * compares (Sec. IV: BiCGStab, restarted GMRES, flexible GMRES) to a
 * relative residual tolerance.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Time factor e^{+j omega t}; the right-hand side of eq. (e2) is
 *    b = -j omega j, where j is the impressed current per edge [A].  The
 *    unknown e is the edge voltage [V].
 *  - Unknown ordering is the paper's cell-by-cell interleaving (Sec. II,
 *    eq. (e12Nxyz)): with Nx = ncx+1, Ny = ncy+1, Nz = ncz+1 primal nodes,
 *    edge (w, i, j, k), w = 0/1/2 for x/y/z, is element
 *        3 * (i + Nx * (j + Ny * k)) + w
 *    of an n_e = 3 Nx Ny Nz vector.  Edges that do not exist (ghost edges at
 *    the upper end of an axis), edges tangential to an electric wall and
 *    edges touching a PEC cell are "masked": they carry no unknown.
 *  - Complex vectors are interleaved (re, im): complex128 = 2 doubles,
 *    complex64 = 2 floats per element.  Device buffers are owned by the
 *    caller, live on the grid's device, are contiguous and at least 16-byte
 *    aligned (8-byte for complex64).
 *  - Streams are hipStream_t passed as void*; NULL means the null stream.
 *  - Every call returns a fit_status; nothing throws or aborts across the
 *    ABI.  fit_last_error() returns a thread-local description of the most
 *    recent failure on the calling thread.
 */
#ifndef FIT_H
#define FIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FIT_OK = 0,
  FIT_E_INVALID = 1,       /* bad argument; nothing was written */
  FIT_E_NOMEM = 2,         /* device or host allocation failed */
  FIT_E_DEVICE = 3,        /* a HIP runtime call failed */
  FIT_E_NOT_CONVERGED = 4, /* iteration cap reached; best iterate returned */
  FIT_E_BREAKDOWN = 5,     /* Krylov breakdown not cured by restarts */
  FIT_E_NAN = 6,           /* NaN/Inf met in the iteration */
  FIT_E_UNSUPPORTED = 7
} fit_status;

typedef enum { FIT_C128 = 0, FIT_C64 = 1 } fit_dtype;

/* Tile-table key of the block shape that batched (fit_sweep) launches use in
 * complex128; fit_tile_set and fit_tile_get accept it in place of a dtype.
 * Without an entry under this key the batched launches use the FIT_C128
 * shape. */
#define FIT_TILE_BATCHED_C128 2

/* FIT_SCALE_NONE: y = A(omega) x, the operator of eq. (e2) with losses.
 * FIT_SCALE_SYM:  y = S A(omega) S x with S = diag(M_eps,c^{-1/2}),
 *   M_eps,c = M_eps - j M_sigma / omega: the symmetrically scaled operator of
 *   eqs. (e2s)/(e2t), S C^T M_nu C S - omega^2 I.  Requires omega > 0.
 * FIT_SCALE_FACT: the same scaled operator in the factorized order of
 *   eq. (e2tt), y = calA^T (calA x) - omega^2 x with
 *   calA = M_mu^{-1/2} C S (the reluctance split as sqrt(M_nu) on both
 *   factors).  fit_matvec only (fit_matvec_batched, fit_solve and fit_sweep
 *   take NONE or SYM).  Requires omega > 0. */
typedef enum { FIT_SCALE_NONE = 0, FIT_SCALE_SYM = 1, FIT_SCALE_FACT = 2 } fit_scaling;

/* FIT_COCG is the paper's conjugate-gradient method (Sec. IV, "cg") in the
 * form that is valid for the complex symmetric (A = A^T, not Hermitian)
 * operator: CG recurrences with the unconjugated bilinear form x^T y
 * (conjugate orthogonal CG).  One operator application per iteration.
 * FIT_COCR is the paper's conjugate residual method (Sec. IV, "cr") in the
 * same complex symmetric form (CR recurrences with x^T y), one operator
 * application per iteration; FIT_TFQMR is the transpose-free QMR method of
 * the same comparison (Freund), two operator applications per iteration,
 * stopping on its residual bound tau sqrt(m + 1) before the true residual is
 * checked; FIT_CGS is conjugate gradients squared (Sonneveld), also two
 * operator applications per iteration.  TFQMR and CGS use the dense shadow
 * vector of BiCGStab.  All three run on the internal operator (S A S with
 * FIT_SCALE_SYM). */
typedef enum {
  FIT_BICGSTAB = 0,
  FIT_GMRES = 1,
  FIT_FGMRES = 2,
  FIT_COCG = 3,
  FIT_COCR = 4,
  FIT_TFQMR = 5,
  FIT_CGS = 6
} fit_solver;

/* FIT_PREC_FP64:  complex128 operator and Krylov vectors throughout.
 * FIT_PREC_MIXED: complex64 operator and inner Krylov iterations, complex128
 *   outer residual r = b - A x, solution update and stopping test
 *   (iterative refinement). */
typedef enum { FIT_PREC_FP64 = 0, FIT_PREC_MIXED = 1 } fit_precision;

/* Diagonal preconditioner of FIT_COCG, m = diag(M)^{-1} applied as z = m .* r
 * (a complex symmetric diagonal, so COCG stays valid).
 * FIT_DIAG_AUTO:   the symmetric scaling of eq. (e2t) when scaling is
 *   FIT_SCALE_SYM (m = 1/M_eps,c recomputed inside the fused operator and
 *   update kernels, nothing stored), none with FIT_SCALE_NONE.
 * FIT_DIAG_MASS:   the same m = 1/M_eps,c, kept as a stored vector (unfused;
 *   the same iterates up to rounding).
 * FIT_DIAG_PAPER:  the paper's diagonal preconditioner of the factorized form
 *   (Sec. III, eq. (Precond)): the squared column norms of
 *   calA = M_mu^{-1/2} C M_eps^{-1/2}, P_ee = K_ee / M_eps,e with
 *   K = C^T M_nu C; on the unscaled system this is m = 1/K_ee.
 * FIT_DIAG_JACOBI: m = 1/diag(A(omega)) = 1/(K_ee + d_e).
 * The stored forms cost one more vector and three more passes per iteration
 * than FIT_DIAG_AUTO. */
typedef enum { FIT_DIAG_AUTO = 0, FIT_DIAG_MASS = 1, FIT_DIAG_PAPER = 2, FIT_DIAG_JACOBI = 3 } fit_diag;

/* One material (Sec. II, eq. (Material); complex permittivity for dielectric
 * losses eps0 eps_r (1 - j tan_delta); conductivity sigma [S/m]). */
typedef struct {
  double eps_r;
  double mu_r;
  double sigma;
  double tan_delta;
  int32_t is_pec; /* nonzero: perfect electric conductor cell */
  int32_t reserved;
} fit_material;

/* Lumped port (Sec. IV): the z-edges (i, j, k) with k0 <= k < k1.  The port
 * drives equal currents through its edges and loads them with an internal
 * impedance z0 [Ohm] split evenly over the k1-k0 edges (each edge gets a
 * conductance (k1-k0)/z0). */
typedef struct {
  int32_t i, j, k0, k1;
  double z0;
} fit_port;

/* Grid description; all pointers are host pointers and are copied by
 * fit_grid_create (the caller may free them afterwards). */
typedef struct {
  int32_t ncx, ncy, ncz;    /* cells per axis, each >= 1 */
  int32_t nmat;             /* 1 <= nmat <= 254 */
  const double *dx;         /* ncx cell widths [m], > 0 */
  const double *dy;         /* ncy */
  const double *dz;         /* ncz */
  const uint8_t *cell_mat;  /* ncx*ncy*ncz ids < nmat; cell (a,b,c) at a + ncx*(b + ncy*c) */
  const fit_material *mats; /* nmat entries */
  int32_t nports;           /* 0 <= nports <= 64 */
  uint32_t pec_walls;       /* electric walls, bits -x,+x,-y,+y,-z,+z (0x3F: closed box) */
  const fit_port *ports;    /* nports entries; at most one port per (i, j) column */
} fit_grid_desc;

struct fit_grid;
struct fit_precond;

typedef struct {
  int32_t solver;      /* fit_solver */
  int32_t restart;     /* GMRES/FGMRES restart length m, 1..64 (0 -> 30) */
  int32_t max_iters;   /* cap on Krylov iterations (BiCGStab: iterations of two
                          operator applications; GMRES: Arnoldi steps); 0 -> 100000 */
  int32_t check_every; /* host polls the device convergence flag every this many
                          iterations (0 -> automatic) */
  int32_t precision;   /* fit_precision */
  int32_t scaling;     /* fit_scaling the Krylov iteration works in internally;
                          the stopping test always uses the unscaled system */
  double inner_tol;    /* FIT_PREC_MIXED: relative tolerance of each inner solve
                          (0 -> 1e-4) */
  struct fit_precond *precond; /* FIT_FGMRES: learned right preconditioner, or NULL.
                                  With one, a run whose restart residual has not
                                  halved within 10 cycles falls back to the
                                  mass-preconditioned FIT_COCG from the current
                                  iterate (info.fell_back = 1) */
  void *stream;        /* hipStream_t for all work of the call */
  double *resid_history; /* optional host array: recursive residual estimate
                            (relative) after each iteration */
  int32_t resid_history_len;
  int32_t use_graph;   /* nonzero: replay captured hipGraphs of check_every
                          iterations instead of eager launches */
  int32_t diag;        /* fit_diag: FIT_COCG's diagonal preconditioner; any value
                          but FIT_DIAG_AUTO with another solver is
                          FIT_E_UNSUPPORTED (fit_sweep ignores it) */
  int32_t reserved;
} fit_solve_opts;

typedef struct {
  int32_t status;       /* fit_status of the call */
  int32_t iterations;   /* Krylov iterations performed (inner ones for MIXED) */
  int32_t refinements;  /* outer refinement steps (MIXED) or true-residual restarts */
  int32_t fell_back;    /* preconditioner or precision fallback taken */
  int32_t matvecs;      /* operator applications (all precisions) */
  int32_t reserved;
  double true_relres;   /* ||b - A x||_2 / ||b||_2, unscaled, complex128 */
  double time_ms;       /* wall time of the call */
  double bytes_moved;   /* algorithmic HBM bytes of the kernels launched */
} fit_solve_info;

/* Validate a grid description and upload it to device `device`.
 * Errors: FIT_E_INVALID (sizes < 1, non-positive or non-finite spacing,
 * material id >= nmat, nmat outside 1..254, port outside the grid or two ports
 * on one column), FIT_E_DEVICE, FIT_E_NOMEM.  On success *out owns device
 * copies of the geometry; release with fit_grid_destroy. */
fit_status fit_grid_create(const fit_grid_desc *desc, int device, struct fit_grid **out);

/* Release a grid (NULL-safe).  Waits for nothing: the caller must have
 * synchronised work that uses it. */
void fit_grid_destroy(struct fit_grid *g);

/* n_e = 3 Nx Ny Nz, or -1 for NULL. */
int64_t fit_num_edges(const struct fit_grid *g);

/* Boundary condition of Sec. II: write 1 for every edge that carries an
 * unknown (exists, not tangential to an electric wall, touches no PEC cell)
 * and 0 otherwise into the n_e-byte device buffer mask_dev.  Asynchronous on
 * `stream`. */
fit_status fit_edge_mask(const struct fit_grid *g, uint8_t *mask_dev, void *stream);

/* Material diagonals as recomputed on the fly by the operator (debug/test):
 *   kind 0: M_eps per edge (complex: eps averaged over the dual facet / length)
 *   kind 1: M_sigma per edge including port conductances (real part only)
 *   kind 2: M_nu = M_mu^{-1} per primal facet (facet (w,i,j,k) at the edge
 *           index formula), real part only
 *   kind 3: the curl-curl diagonal K_ee = sum of M_nu over the four facets
 *           that contain edge e (real part only), from which the paper's
 *           diagonal preconditioner follows (Sec. III, eq. (Precond):
 *           P_ee = K_ee / M_eps,e)
 * Written as complex128 into out_dev (n_e elements), for every index
 * including masked and ghost ones.  Asynchronous on `stream`. */
fit_status fit_material_diag(const struct fit_grid *g, int kind, double *out_dev, void *stream);

/* y = A(omega) x (or S A S x for FIT_SCALE_SYM) in the given precision.
 * x_dev, y_dev: n_e complex elements of dtype; they must not overlap.
 * y is 0 on masked edges and x is ignored there.  Asynchronous on `stream`.
 * Errors: FIT_E_INVALID (NULL pointers, omega < 0, SYM with omega == 0). */
fit_status fit_matvec(const struct fit_grid *g, double omega, int dtype, int scaling,
                      const void *x_dev, void *y_dev, void *stream);

/* Batched operator (Sec. II: one system per frequency): for b in
 * [0, nbatch), y_b = A(omegas[b]) x_b (or S_b A S_b x_b), with the nbatch
 * vectors stored back to back (x_dev + b*n_e complex elements, same for
 * y_dev).  omegas is a host array read before return.  Up to 16 systems
 * share one launch, so small grids still fill the GPU.  The x and y ranges
 * must not overlap.  Asynchronous on `stream`; 1 <= nbatch <= 64.
 * Errors: FIT_E_INVALID (NULL, nbatch out of range, omega < 0 or not finite,
 * SYM with omega == 0, overlap, unknown dtype or scaling). */
fit_status fit_matvec_batched(const struct fit_grid *g, int nbatch, const double *omegas,
                              int dtype, int scaling, const void *x_dev, void *y_dev,
                              void *stream);

/* Solve A(omega) e = -j omega j for e (Sec. II eq. (e2), Sec. IV) with the
 * Krylov method in opts, from e = 0, until the unscaled complex128 relative
 * residual ||b - A e|| / ||b|| <= tol.
 * source_dev: impressed current j, n_e complex128 on the device; must be zero
 *   on masked edges (else FIT_E_INVALID).
 * x_dev: output e, n_e complex128 (0 on masked edges).
 * info: optional, filled on every return except FIT_E_INVALID.
 * FIT_E_NOT_CONVERGED / FIT_E_BREAKDOWN / FIT_E_NAN still return the best
 * iterate.  Synchronous: returns after the stream has drained. */
fit_status fit_solve(struct fit_grid *g, double omega, const void *source_dev, double tol,
                     const fit_solve_opts *opts, void *x_dev, fit_solve_info *info);

/* Frequency and right-hand-side sweep over several grids (Sec. II: each
 * frequency and excitation is an independent system; Sec. IV: multi-port
 * excitation).  For every grid g, omega index f and right-hand side r, solves
 * A_g(omegas[f]) e = -j omegas[f] j_{g,r} to the true relative residual tol.
 * Systems are advanced together in batches (up to 64 per batch, within half
 * of the free device memory): each iteration of a batch is one operator
 * launch over all its systems' tiles, one streaming update launch and two
 * small finish launches, replayed from a captured hipGraph; converged
 * systems drop out at once.  The systems of a launch share the largest
 * grid's block shape (complex128: its FIT_TILE_BATCHED_C128 entry if there
 * is one, see fit_autotune_sweep) with their own z-chunks; the batch size is
 * fit_sweep_set_batch's.  The method is the mass-preconditioned COCG of
 * fit_solve (opts->solver must be FIT_COCG, else FIT_E_UNSUPPORTED);
 * opts->precision FIT_PREC_FP64 iterates in complex128, FIT_PREC_MIXED in
 * complex64 with complex128 refinement and a complex128 finish for systems
 * whose complex64 refinement stalls.  opts->max_iters, check_every,
 * inner_tol, use_graph and stream are honoured; scaling, restart, precond
 * and the residual history are ignored.
 *   omegas:         nomega host values, each finite and > 0.
 *   sources_dev[g]: nrhs * n_e(g) complex128 device buffer (rhs r at r*n_e);
 *                   zero on masked edges (else FIT_E_INVALID, nothing solved).
 *   port_v_host:    NULL or [g][f][r][p] complex128 (2 doubles) port voltages,
 *                   the sum of edge voltages over port p of grid g (Sec. IV
 *                   probes); p runs over that grid's nports, so the block of
 *                   grid g has nomega*nrhs*nports(g) entries, grids back to
 *                   back.
 *   x_dev_opt:      NULL, or per grid a nomega*nrhs*n_e complex128 buffer for
 *                   the fields (system (f, r) at (f*nrhs + r)*n_e).
 *   infos:          NULL or ngrids*nomega*nrhs entries in the same order;
 *                   time_ms is the whole sweep's wall time.
 * All grids must live on one device.  Synchronous.  Returns FIT_OK only if
 * every system met tol, else the first failing system's status (every
 * system still gets its best iterate and its info). */
fit_status fit_sweep(struct fit_grid *const *grids, int ngrids, const double *omegas, int nomega,
                     const void *const *sources_dev, int nrhs, double tol,
                     const fit_solve_opts *opts, double *port_v_host, void *const *x_dev_opt,
                     fit_solve_info *infos);

/* Sum of edge voltages over each port of g for `nvec` complex128 fields
 * stored back to back on the device; writes nvec*nports complex128 values
 * (2 doubles each) to the host array out_host.  Synchronous. */
fit_status fit_port_voltages(const struct fit_grid *g, const void *x_dev, int nvec,
                             double *out_host, void *stream);

/* fit_port_voltages for callers that cannot allocate device memory (code
 * inside a tight serving loop, or a harness that forbids hipMalloc): the same
 * kernel and the same result, bit for bit, but the port sums are staged in a
 * static device array of 65536 complex128 values (1 MiB) that every GPU the
 * library runs on keeps until the process ends, instead of a buffer
 * allocated per call.  Calls no allocating routine.  FIT_E_INVALID (nothing
 * written) for the bad arguments of fit_port_voltages and for
 * nvec * nports > 65536.  Calls that overlap on one GPU share the array and
 * race: serialise them (one stream, or host-side ordering).  Synchronous. */
fit_status fit_port_voltages_noalloc(const struct fit_grid *g, const void *x_dev, int nvec,
                                     double *out_host, void *stream);

/* Network parameters of the ports (Sec. IV port model: each lumped port is a
 * 1 A source in parallel with its internal impedance z0, which the port's
 * edges carry as conductance).  Host-only and synchronous.
 *   zl:    host, nports x nports complex128 (2 doubles each), row-major: the
 *          loaded impedance zl[p][q] = -u_p for a unit current at port q
 *          with every port loaded by z0 (u = fit_port_voltages of that
 *          solve; the minus sign because an edge voltage integrates E from
 *          the ground end up).
 *   z_out: NULL or host nports x nports complex128: the network's own
 *          impedance matrix with the loads removed, Z = (zl^-1 - I/z0)^-1.
 *   s_out: NULL or host nports x nports complex128: the scattering matrix
 *          for reference impedance z0, S = (Z - z0 I)(Z + z0 I)^-1, which
 *          equals 2 zl / z0 - I.
 * FIT_E_INVALID (nothing written) for nports outside [1, 64], z0 <= 0, a NULL
 * or non-finite zl, or, when z_out is asked for, a singular zl or
 * zl^-1 - I/z0. */
fit_status fit_port_network(int nports, double z0, const double *zl, double *z_out, double *s_out);

/* ---- stencil launch shapes and the autotuner ------------------------------
 * A workgroup of tx x ty threads covers tx x ty node columns -- the
 * (tx-2) x (ty-2) columns it outputs plus a one-node halo ring -- and marches
 * up zc z-planes, 1 <= zc <= 128.  Compiled shapes: (tx, ty) in {(64,8),
 * (48,8), (32,8), (32,16)}.  The table is process-wide and keyed by the
 * grid's node dimensions and dtype. */

/* Force a tile shape for grids of g's node dimensions in `dtype` (or under
 * FIT_TILE_BATCHED_C128).  FIT_E_INVALID for a shape that is not compiled or
 * zc outside [1, 128]. */
fit_status fit_tile_set(const struct fit_grid *g, int dtype, int tx, int ty, int zc);

/* The tile shape that launches on g in `dtype` (or, with
 * FIT_TILE_BATCHED_C128, batched complex128 launches) use now: the table's
 * entry for its node dimensions, else the default shape (for the batched
 * key: the FIT_C128 shape).  FIT_E_INVALID for a NULL grid or output
 * pointer, or a bad dtype. */
fit_status fit_tile_get(const struct fit_grid *g, int dtype, int32_t *tx, int32_t *ty, int32_t *zc);

/* Time every compiled (TX, TY) with a range of ZC on g (operator in `dtype`
 * and `scaling` at omega, `reps` timed launches each, HIP events on `stream`),
 * record the fastest in the table and report it.  Candidates are timed in a
 * fixed order ((64,8), (48,8), (32,8), (32,16), each with ascending zc) and a
 * later one replaces the best so far only if it is more than 2 % faster, so
 * near-ties resolve the same way from run to run.  best_us: mean kernel time
 * of the winner.  Synchronous; allocates two scratch vectors. */
fit_status fit_autotune(const struct fit_grid *g, int dtype, int scaling, double omega, int reps,
                        void *stream, int32_t *tx, int32_t *ty, int32_t *zc, double *best_us);

/* Time every compiled (TX, TY) with a range of ZC on the solver's own
 * iteration instead of the plain operator: the complex128 COCG with the
 * symmetric scaling (fused operator step and update kernel, captured graphs)
 * at omega, from the difference of two solves capped at iters and 2 iters
 * iterations (which removes set-up and graph capture), with a source of 1 A
 * on every free edge; record the fastest for complex128 and report it with
 * its time per iteration.  Same candidate order and 2 % rule as fit_autotune.
 * Synchronous; allocates three work vectors. */
fit_status fit_autotune_solver(struct fit_grid *g, double omega, int iters, void *stream,
                               int32_t *tx, int32_t *ty, int32_t *zc, double *best_us_per_iter);

/* Systems that fit_sweep advances together in one batch (one operator launch
 * over all of them per iteration), process-wide; 1..64 (default 64).  The
 * per-system results do not depend on it. */
fit_status fit_sweep_set_batch(int systems);

/* Choose fit_sweep's launch shape for grids like g: time `iters` COCG
 * iterations (difference of runs of iters and 2 iters) of batched sweeps
 * (frequencies taken from omegas, at most nomega; one source of 1 A on every
 * free edge).  First the complex128 block shape: every compiled shape with
 * z-chunks of 4 and 8 planes on batches of up to 16 systems; the one with
 * the most system-iterations per second (a later one must win by more than
 * 2 %) is stored under FIT_TILE_BATCHED_C128 for g's node dimensions (the
 * shape of single solves is left alone).  Then the systems per batch: 64,
 * 32, 16, 8 and 4,
 * from the largest down (a smaller batch must win by more than 2 %: fewer
 * batches leave fewer serial tails).  Sets the process-wide batch size;
 * reports it and its rate.  Synchronous. */
fit_status fit_autotune_sweep(struct fit_grid *g, const double *omegas, int nomega, int iters,
                              void *stream, int32_t *best_batch, double *best_rate);

/* Write / read the tile table as JSON ({"entries": [{"nx":..,"ny":..,"nz":..,
 * "dtype":..,"tx":..,"ty":..,"zc":..,"us":..}, ...], "arch": "gfx950"}). */
fit_status fit_tune_save(const char *path);
fit_status fit_tune_load(const char *path);

/* ---- launch profiler ------------------------------------------------------
 * While on, every operator launch and every fused Krylov update launch is
 * bracketed by a HIP event pair on its own stream; fit_profile_stop waits for
 * the recorded events and returns the summed durations per kernel family
 * (names such as "cocg_step1", "bicgstab_step1", "matvec"). */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
} fit_kernel_stat;

fit_status fit_profile_start(void);
/* out may be NULL; *n receives the number of families (all of them, even if
 * more than max). */
fit_status fit_profile_stop(fit_kernel_stat *out, int max, int *n);

/* ---- learned right preconditioner (3-level 3D U-Net, BF16 MFMA) ---------- *
 *
 * A nonlinear right preconditioner z = M(v) for FIT_FGMRES (Sec. IV: flexible
 * GMRES stores the preconditioned directions, so M may change from one
 * application to the next and need not be linear).  M(v) = s U(v/s) with
 * s = rms(v) over the free edges and U a 3-level 3D U-Net over the node grid
 * (base channels c, 2c, 4c; two 3x3x3 convolutions per level, 2x2x2 stride-2
 * down and transposed up convolutions, skip concatenations, a 1x1x1 head,
 * ReLU).  Input per node: Re/Im of its three edge values of v/s, eps_r/12 and
 * (log10(sigma + 1e-3) + 3)/11 of the cell it owns, log10(f/GHz)/1.6 and
 * log10(h/100 um) of that cell's three widths; output:
 * Re/Im of its three edge values of z/s; masked edges give 0.  All
 * convolutions run as BF16 MFMA implicit GEMMs with fp32 accumulation; bf16
 * activations and weights, fp32 biases, master weights and head output.
 * With FIT_SCALE_SYM the solver works on S A S and the adapter applies
 * S^-1 M(S^-1 v).
 *
 * Blob format (fit_precond_save / _load): uint64 magic 0x3154454E55544946
 * ("FITUNET1" little-endian), int32 c, int32 0, int64 nparams, then nparams
 * fp32 parameters: for each layer in the order enc1a, enc1b, down1, enc2a,
 * enc2b, down2, bot_a, bot_b, up2, dec2a, dec2b, up1, dec1a, dec1b, head, its
 * weights w[tap][ci][co] (3x3x3 tap = (dz+1)*9 + (dy+1)*3 + (dx+1), 2x2x2
 * tap = dz*4 + dy*2 + dx) and then its biases b[co].  Layer channel counts
 * (cin -> cout): 12->c, c->c, c->2c, 2c->2c, 2c->2c, 2c->4c, 4c->4c, 4c->4c,
 * 4c->2c, 4c->2c, 2c->2c, 2c->c, 2c->c, c->c, c->6. */

/* Configuration for fit_precond_create / fit_precond_train (0 = default). */
typedef struct {
  int32_t base_channels; /* c, one of 8, 16, 24, 32 (16) */
  int32_t steps;         /* optimiser steps (2000) */
  int32_t batch;         /* residual->error pairs per step (4) */
  int32_t crop;          /* crop edge in nodes, multiple of 4 (32) */
  int32_t pairs_per_system; /* > 0: solver-generated pairs per (grid, omega); 0: noise pairs */
  int32_t seed;          /* initial weights and sampling */
  double lr;             /* Adam learning rate (1e-3) */
  double weight_decay;   /* added to the gradient as weight_decay * w (0) */
  void *stream;
} fit_precond_cfg;

/* Train a new preconditioner with Adam on residual->error pairs r = A(omega) e.
 * With cfg->pairs_per_system = P > 0 the pairs are generated by the solver
 * (fit_precond_harvest): for every training grid and every omega of `omegas`,
 * P pairs e = x* - x_k, r = A e from COCG iterates x_k of the grid's port
 * excitation (port index = (grid index + omega index) mod nports; every
 * training grid needs a port), harvested once before the first step.  With
 * P = 0, e is seeded complex noise on the free edges smoothed 2, 4, 8 or 16
 * times by averaging each edge value with the same component at the
 * neighbouring nodes.  One pair per sample, on a random crop of `crop` nodes
 * per axis (at a random omega of `omegas` for noise pairs).  Loss: the mean
 * over the crop's free edges of |U(r/s_r) - e/s_e|^2 with s_r, s_e the rms of
 * r and e there.  Synchronous; *out receives the trained object.  The mean
 * loss of every optimiser step is kept for fit_precond_train_history. */
fit_status fit_precond_train(struct fit_grid *const *train, int ntrain, const double *omegas,
                             int nomega, const fit_precond_cfg *cfg, struct fit_precond **out);
/* The solver-generated training pairs (the paper's excitation, Sec. IV: 1 A
 * on every edge of a lumped port): on grid g at omega with the source j = 1 A
 * on every edge of port `port`, COCG (complex128, symmetric scaling) runs to
 * the true relative residual tol, giving x*; a second identical run keeps its
 * iterate x_k every iterations/(npairs+1) iterations; then e_k = x* - x_k and
 * r_k = A(omega) e_k (= b - A x_k up to rounding).
 *   e_dev, r_dev: npairs * n_e complex128 each on the grid's device (pair k at
 *                 k * n_e); *made receives the number of pairs written (fewer
 *                 than npairs when the solve ends early); *iterations (may be
 *                 NULL) the first solve's COCG iterations.
 * FIT_E_INVALID for NULL pointers, npairs < 1, a port index outside the grid's
 * ports, omega <= 0 or tol outside (0, 1); the solve's own status if it does
 * not converge.  Allocates three work vectors.  Synchronous. */
fit_status fit_precond_harvest(struct fit_grid *g, double omega, int port, int npairs, double tol,
                               void *e_dev, void *r_dev, int *made, int *iterations);
/* Per-step mean training loss of this thread's last fit_precond_train:
 * copies min(max, steps) values to out (may be NULL); *n = steps. */
fit_status fit_precond_train_history(double *out, int max, int *n);
/* Create an untrained preconditioner (seeded He-uniform weights, zero
 * biases) on `device`. */
fit_status fit_precond_create(const fit_precond_cfg *cfg, int device, struct fit_precond **out);
/* Serialise to the blob format above (blob NULL: only report the size in *n;
 * *n smaller than needed: FIT_E_INVALID and *n = size) / deserialise. */
fit_status fit_precond_save(const struct fit_precond *p, void *blob, size_t *n);
fit_status fit_precond_load(const void *blob, size_t n, int device, struct fit_precond **out);
/* z = M(v) for one complex128 edge vector on grid g at omega (the unscaled
 * form).  v_dev, z_dev: n_e complex128 on the grid's device.  Synchronous.
 * The first preconditioner call on a grid computes its edge mask (n_e bytes)
 * and keeps it with the grid until fit_grid_destroy; the activations of the
 * last padded grid size are kept with the preconditioner (reallocated when
 * the size changes). */
fit_status fit_precond_apply(struct fit_precond *p, const struct fit_grid *g, double omega,
                             const void *v_dev, void *z_dev, void *stream);
/* Training objective of one pair over the whole grid (padded to multiples of
 * 4 nodes): *loss = mean over free edges of |U(r/s_r) - e/s_e|^2 and its
 * gradient with respect to the parameters, in blob order, as fp32 into the
 * host array grad_host (nparams entries; may be NULL).  r_dev, e_dev: n_e
 * complex128 on the device.  Synchronous. */
fit_status fit_precond_loss_grad(struct fit_precond *p, const struct fit_grid *g, double omega,
                                 const void *r_dev, const void *e_dev, double *loss,
                                 float *grad_host, void *stream);
void fit_precond_destroy(struct fit_precond *p);

/* Thread-local message for the last failing call on this thread ("" if none). */
const char *fit_last_error(void);

/* Library version string. */
const char *fit_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FIT_H */
