/*
 * vie.h -- C interface of the MI355X (gfx950) volume-integral-equation solver.
 *
 * The library solves the well-conditioned second-kind volume integral
 * equations of Imbert-Gerard, Vico, Greengard and Ferrando, "Integral equation
 * methods for electrostatics, acoustics and electromagnetics in smoothly
 * varying, anisotropic media" (arXiv:1805.04791):
 *
 *   anisotropic Laplace   (Section 2, eq. intLap):   J - 2 H T_0 J = 2 H grad phi_inc,
 *                         H = (eps + I)^{-1} (eps - I)  (eq. rhodef),
 *   anisotropic Helmholtz (Section 3, eqs. contractionK / intH):
 *                         J - 2 H T_w J = 2 H grad phi_inc,  H = (eps^{-1} + I)^{-1} (eps^{-1} - I),
 *                         (the sign follows the derivation; the printed summary
 *                         equation carries "+"),
 *   anisotropic Maxwell   (Section 4, eq. intM, and eq. contraction_Maxwell_reduced for mu = I):
 *                         J - H_eps (J + 2 U_J + 2 i w W_M) = 2 H_eps E_inc,
 *                         M - H_mu  (M + 2 U_M - 2 i w W_J) = 2 H_mu  H_inc,
 * with T J = J/2 + grad div V J, U = grad div V J (Laplace, Helmholtz) or
 * (grad div + w^2) V J (Maxwell), W = curl V J, and V the volume potential of
 * eq. Vo / eq. Vw.  The integral operators are discretised on a uniform n^3
 * grid with the truncated-kernel FFT method described at the start of
 * Section 5, and the linear systems are solved with GMRES (or Bi-CGStab, the
 * solver of Section 5) without preconditioner.
 *
 * Discretisation (the readings of Section 5 used here):
 *   grid      x_i = origin + (i + 1/2) h, i in [0, n)^3;
 *   kernel    cut off at R = sqrt(3) n h, its transform sampled at
 *             s = 2 pi k / (4 n h), |k_a| <= 2n, cube cut-off at pi/h with the
 *             Nyquist plane averaged over +-pi/h; the windowed real-space
 *             kernel (displacements |m_a| < n) is convolved on a 2n grid.
 *
 * Layout of every density / field / incident array: interleaved complex128
 * (re, im) [nrhs][c][n][n][n], C order, x the fastest axis; c = 3 (Laplace,
 * Helmholtz, Maxwell with mu = I) or c = 6 (Maxwell with mu: [J; M], [E; H]).
 * Tensor fields (coef, mu): complex128 [9][n][n][n], entry (a, b) at 3a + b.
 *
 * Memory: unless stated otherwise the vector arguments of vie_apply,
 * vie_solve, vie_rhs and vie_field are DEVICE pointers (hipMalloc or a torch
 * tensor's data_ptr()) on the plan's device, owned by the caller.  The plan
 * owns its own device memory (contrast, kernel tables, workspaces, Krylov
 * basis) until vie_destroy.  Calls are queued on the given HIP stream (NULL:
 * the default stream); vie_solve synchronises that stream for its
 * convergence tests.  A plan must not be used from two streams or threads at
 * the same time.
 *
 * Errors: functions return VIE_OK (0), a negative VIE_E_* code, or the
 * positive warning VIE_W_NOCONV.  vie_last_error(plan) returns a message for
 * the last failure on that plan; vie_status_string() names a code.
 */
#ifndef VIE_H
#define VIE_H

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define VIE_OK 0
#define VIE_E_ARG (-1)       /* null pointer, bad enum, n/h/omega/nrhs out of range */
#define VIE_E_SIZE (-2)      /* n with no compiled FFT length for 2n (or 4n) */
#define VIE_E_MEDIUM (-3)    /* a + I singular or non-finite at a grid point; or ||H||_2 >= 1 in strict mode */
#define VIE_E_NOMEM (-4)     /* device allocation failed */
#define VIE_E_DEVICE (-5)    /* a HIP call failed (message in vie_last_error) */
#define VIE_E_STATE (-6)     /* call not valid for this plan (e.g. mu-dependent call on a 3-component plan) */
#define VIE_W_NOCONV 1       /* vie_solve: some right-hand side did not reach tol within max_iters */

typedef enum { VIE_LAPLACE = 0, VIE_HELMHOLTZ = 1, VIE_MAXWELL = 2 } vie_kind;

typedef enum {
  VIE_PREC_FP64 = 0,  /* FP64 FFT apply everywhere */
  VIE_PREC_MIXED = 1  /* FP32-complex FFT apply inside GMRES; FP64 Arnoldi, least squares,
                         true residuals (iterative refinement) and kernel precompute */
} vie_precision;

/* vie_problem.flags */
#define VIE_PTR_HOST 0x1u        /* coef / mu are host pointers (default: device pointers) */
#define VIE_STRICT_MEDIUM 0x2u   /* fail with VIE_E_MEDIUM when max ||H(x)||_2 >= 1 (Lemma 1) */
#define VIE_NO_GRAPHS 0x4u       /* never replay solver applies from captured hipGraphs.  Capture
                                    (on by default) forbids, in every thread of the process, HIP
                                    calls that allocate, free or synchronise the device; hosts whose
                                    other threads make such calls while a plan solves set this flag. */
/* Unknowns of the solver.  By default they are the support rows of H (in
 * each (z, y) row of the bounding box of supp(H), the x-interval from the
 * first to the last point where H != 0; the integral equation gives J = 0
 * wherever H = 0) and its x and y transforms have the shortest compiled
 * length >= 2 max(bx, by).  These flags widen that, for comparisons; the
 * discrete operator is the same. */
#define VIE_WHOLE_GRID 0x8u      /* the solver works on the whole n^3 grid with 2n-point transforms */
#define VIE_DENSE_BOX 0x10u      /* unknowns: every point of the bounding box (no support rows) */
#define VIE_FULL_LENGTH 0x20u    /* the solver's x and y transforms have length 2n */
#define VIE_GRID_TABLES 0x40u    /* build the whole grid's kernel tables at plan creation (otherwise
                                    at the first vie_apply / vie_field when the solver's transform
                                    is shorter than 2n); vie_apply_noalloc needs them */

/*
 * The problem statement of the paper (Introduction and Section 5): a grid,
 * samples of the coefficient tensor(s), and the frequency.
 *   kind=LAPLACE:   coef = eps(x)            (eq. Laplace0), omega ignored (0)
 *   kind=HELMHOLTZ: coef = eps^{-1}(x)       (eq. Helmholtz0), omega > 0
 *   kind=MAXWELL:   coef = eps(x), mu = mu(x) or NULL for mu = I (eq. Maxwell0), omega > 0
 * n: points per axis; supported n = 8, 12, 16, 24, 32, 48, 64, 96, 128, 160.
 * h > 0 grid spacing; origin only positions the grid (the operator is
 * translation invariant).  max_rhs >= 1 sizes the apply workspace (larger
 * batches are processed in chunks).  The coefficient arrays are copied.
 */
typedef struct {
  int kind;             /* vie_kind */
  int n;
  double h;
  double origin[3];
  double omega;
  const double *coef;   /* complex128 [9][n][n][n] */
  const double *mu;     /* complex128 [9][n][n][n] or NULL */
  int precision;        /* vie_precision: the default apply precision of vie_solve */
  int max_rhs;
  unsigned flags;
} vie_problem;

struct vie_plan;
typedef struct vie_plan vie_plan;

/* solver selection (vie_solve_opts.solver) */
#define VIE_SOLVER_GMRES 0
#define VIE_SOLVER_BICGSTAB 1

/* vie_solve_opts.flags */
#define VIE_SOLVE_X0 0x1u        /* density holds the initial guess (resume) instead of 0 */
#define VIE_SOLVE_FP64 0x2u      /* plain FP64 solve regardless of the plan precision */

typedef struct {
  double tol;          /* stop when ||b - A x||_2 / ||b||_2 <= tol (true residual, FP64) */
  int max_iters;       /* total matvec budget per right-hand side (FP32 + FP64) */
  int restart;         /* GMRES basis size m (inner cycle length) */
  double inner_tol;    /* mixed: relative reduction asked of each FP32 inner cycle (0: 1e-5) */
  int solver;          /* VIE_SOLVER_* */
  unsigned flags;      /* VIE_SOLVE_* */
} vie_solve_opts;

typedef struct {
  int status;          /* VIE_OK or VIE_W_NOCONV */
  int iters;           /* Krylov iterations */
  int matvecs_fp32;
  int matvecs_fp64;
  int refinements;     /* outer true-residual steps */
  double rel_residual; /* final true ||b - A x|| / ||b|| (FP64) */
  double seconds;      /* wall time of the batch this right-hand side was solved in */
} vie_solve_stats;

/* Plan: validates the problem, computes the contrast H (FP64 and FP32) and the
 * kernel-transform tables (FP64 precompute, FP32 copy), and allocates the
 * apply workspace.  hip_stream may be NULL.  On success *out owns all device
 * memory of the plan.  Errors: VIE_E_ARG, VIE_E_SIZE, VIE_E_MEDIUM,
 * VIE_E_NOMEM, VIE_E_DEVICE (*out is NULL on error). */
int vie_plan_create(const vie_problem *p, void *hip_stream, vie_plan **out);

/* vie_apply flags */
#define VIE_APPLY_FP64 0x1u      /* FP64 FFTs (default: the plan precision) */
#define VIE_APPLY_FP32 0x2u      /* FP32 FFTs */
#define VIE_APPLY_CONV 0x4u      /* return the raw convolution U (Z for full Maxwell) instead of A x */
#define VIE_APPLY_C64 0x8u       /* x and y are complex64 (float pairs); FP32 matvec only */

/* y = A x for nrhs densities (device pointers, complex128 [nrhs][c][n^3], or
 * complex64 with VIE_APPLY_C64; x and y are passed as double* either way).
 * The discrete operator of the integral equation (see the header comment).
 * x and y must not overlap. */
int vie_apply(vie_plan *pl, const double *x, double *y, int nrhs, unsigned flags, void *hip_stream);

/* Size of the device scratch of vie_apply_noalloc, per device (MiB). */
#define VIE_NOALLOC_SCRATCH_MIB 128

/* vie_apply without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, flags, layouts and results as
 * vie_apply; the apply workspace is the library's static device scratch of
 * VIE_NOALLOC_SCRATCH_MIB MiB per device (held from the first plan creation
 * on a device until the process ends) instead of the plan's.  Nothing is
 * allocated, freed or synchronised: no hipMalloc, no event, no tile
 * measurement (tiles measured earlier by vie_apply for this batch size are
 * reused, else fixed defaults).  The whole grid's kernel tables must exist:
 * create the plan with VIE_GRID_TABLES, or call vie_apply once before
 * (VIE_E_STATE otherwise).  Right-hand sides are processed in chunks of at
 * most min(max_rhs, scratch / workspace per right-hand side); VIE_E_SIZE when
 * one right-hand side alone needs more workspace than the scratch holds
 * (C * n^2 * 2n + C * n * (2n)^2 complex values of the apply precision: e.g.
 * n <= 64 in FP64 or n <= 96 in FP32 with c = 3).  Every call on one device
 * shares its scratch, which keeps the last call's contents: calls that
 * overlap in time on one device (other streams or threads) race and must be
 * serialised by the caller. */
int vie_apply_noalloc(vie_plan *pl, const double *x, double *y, int nrhs, unsigned flags, void *hip_stream);

/* b = 2 H g (the right-hand side of the integral equation; for full Maxwell
 * [2 H_eps E_inc; 2 H_mu H_inc]).  Device pointers, [nrhs][c][n^3]. */
int vie_rhs(vie_plan *pl, const double *inc, double *b, int nrhs, void *hip_stream);

/* Total field from a density: grad phi_tot = g + grad div V J (Sections 2-3),
 * E_tot = E_inc + U_J + i w W_M, H_tot = H_inc + U_M - i w W_J (eqs.
 * represent_Maxwell / represent_Maxwell_reduced; reduced: E only).
 * Computed with FP64 FFTs.  Device pointers. */
int vie_field(vie_plan *pl, const double *density, const double *inc, double *field, int nrhs, void *hip_stream);

/* Solve for nrhs incident fields (device pointers).  inc: g = grad phi_inc
 * (Laplace, Helmholtz) or [E_inc; H_inc] (Maxwell); density: J (and M);
 * field may be NULL, else receives the total field.  opts may be NULL
 * (tol 1e-10, restart 40, max_iters 2000, GMRES).  stats may be NULL, else an
 * array of nrhs entries.  Right-hand sides are solved together in fused
 * launches; each keeps its own convergence test, so its result does not
 * depend on the others in the batch.  The unknowns are the support rows of
 * H (vie_plan_info): the integral equation forces J = 0 where H = 0, and
 * density is written as exactly 0 outside them; with VIE_SOLVE_X0 only the
 * initial density on them is used.  Returns
 * VIE_OK, VIE_W_NOCONV (the best iterate is written) or an error. */
int vie_solve(vie_plan *pl, const double *inc, double *density, double *field, int nrhs,
              const vie_solve_opts *opts, vie_solve_stats *stats, void *hip_stream);

/* Continuous batching: the solve of vie_solve (the integral equations in
 * the header comment, GMRES or Bi-CGStab with FP64 true-residual refinement)
 * run step by step on a batch of `capacity` slots (1..256) of one plan, so
 * that right-hand sides can join while others are being solved and leave as
 * soon as they are done.  One batch per plan; vie_solve returns VIE_E_STATE
 * while it is open.  Each slot's arithmetic is independent of the other
 * slots, of its position and of when it joined: a right-hand side gets
 * bitwise the result vie_solve gives it alone with the same options (within
 * one process: the pencil splits of a shape are measured once per process).
 * Slots are filled lowest first, and the launches of a step cover the slots
 * up to the highest one in use.
 *
 * vie_batch_open:  opens the batch with the options of vie_solve (opts may be
 *                  NULL: its defaults); sizes the Krylov workspace for it.
 * vie_batch_add:   nrhs incident fields (device, [nrhs][c][n^3] as in
 *                  vie_solve; x0 NULL or initial densities of the same
 *                  layout) take free slots, written to slots[0..nrhs-1]; they
 *                  start iterating at the next vie_batch_step.  The inputs are
 *                  read before the call returns (it synchronises the stream).
 *                  VIE_E_ARG if fewer than nrhs slots are free.
 * vie_batch_step:  one outer cycle (an inner GMRES cycle of `restart`
 *                  iterations or a Bi-CGStab run, then the FP64 true
 *                  residual) for every slot still iterating; *nactive =
 *                  slots still iterating after it.  Synchronises the stream.
 * vie_batch_done:  host arrays: the finished slots not yet taken (up to
 *                  max_slots of them in slots, their count in *ndone) and the
 *                  free slots (*nfree).
 * vie_batch_take:  writes a finished slot's density (device, [c][n^3], zero
 *                  outside the support rows) and, if field is not NULL, the
 *                  total field (then inc is its incident field [c][n^3]),
 *                  fills *stats (seconds: from its vie_batch_add to the step
 *                  that finished it; may be NULL) and frees the slot.
 *                  Returns VIE_OK or VIE_W_NOCONV (the slot's status).
 * vie_batch_close: frees the batch (slots still holding right-hand sides are
 *                  dropped); the plan stays valid. */
int vie_batch_open(vie_plan *pl, int capacity, const vie_solve_opts *opts, void *hip_stream);
int vie_batch_add(vie_plan *pl, const double *inc, const double *x0, int nrhs, int *slots, void *hip_stream);
int vie_batch_step(vie_plan *pl, int *nactive, void *hip_stream);
int vie_batch_done(vie_plan *pl, int *slots, int max_slots, int *ndone, int *nfree);
int vie_batch_take(vie_plan *pl, int slot, double *density, double *field, const double *inc,
                   vie_solve_stats *stats, void *hip_stream);
int vie_batch_close(vie_plan *pl);

/* Waits for the work of the plan's latest call (an event recorded after it on
 * its stream, not later work of other callers on that stream), then frees
 * the plan.  Work on other streams that uses the plan must have completed.
 * Its device blocks (and small pinned host buffers) go to a process-wide
 * cache from which later plans take their memory (blocks above 64 MiB come
 * in size classes 2^(1/4) apart, so plans of nearby sizes share them; up to
 * 96 GiB kept while 32 GiB of the device stay free; a hipFree would wait for
 * the whole device); an allocation that cannot be met frees the cache of its
 * device and retries.
 * vie_destroy(NULL) is a no-op. */
int vie_destroy(vie_plan *pl);

/* Frees the library's cache of released device blocks and pinned host
 * buffers (e.g. before handing the memory to another allocator).  Returns the
 * device bytes that were cached.  Thread-safe; plans in use are unaffected. */
long vie_release_cached_memory(void);

/* Introspection (host pointers).
 * vie_plan_info: out[0] = n, out[1] = components c, out[2] = P (= 2n),
 * out[3] = oversampled grid M (= 4n), out[4] = max ||H(x)||_2 (Lemma 1),
 * out[5] = table entries, out[6] = device bytes held by the plan,
 * out[7] = applies replayed from captured hipGraphs so far,
 * out[8..10] = corner (x0, y0, z0) and out[11..13] = extent (bx, by, bz) of
 * the box the solver works on: the bounding box of the points where H (or
 * H_mu) is non-zero, outside which the density vanishes (a single point if
 * H = 0 everywhere; the whole grid with the plan flag VIE_WHOLE_GRID),
 * out[14] = the solver's unknown points per component: in each (z, y) row
 * of the box, the x-interval from the first to the last point where H (or
 * H_mu) is non-zero (the whole box with VIE_DENSE_BOX, the whole grid with
 * VIE_WHOLE_GRID), out[15] = the periodic transform length along x and y of
 * the solver's applies: the shortest compiled length >= 2 max(bx, by) and
 * <= 2n (2n with VIE_FULL_LENGTH or VIE_WHOLE_GRID); its kernel tables are
 * the transform of the kernel windowed to |m_a| <= length_a/2 - 1;
 * out[16], out[17] = right-hand sides the FP32 and
 * FP64 apply workspaces hold now (each grows on demand, up to max_rhs, by
 * c (n^2 2n + n 2n w) elements of 8 or 16 bytes per right-hand side, w = 2n
 * rounded up to a multiple of 16),
 * out[18] = solver slots the Krylov workspace holds now, out[19] = the
 * periodic transform length along z of the solver's applies: 64 or 256 when
 * it is >= 2 bz and >= out[15] and < 2n (their square pencil splits keep the
 * fused z pass's lanes busy), else 2n (always 2n with VIE_FULL_LENGTH or
 * VIE_WHOLE_GRID).  Entries beyond nout are not written. */
int vie_plan_info(const vie_plan *pl, double *out, int nout);

/* Copies the FP64 kernel-transform tables into host memory:
 * complex128 [n+1][n+1][nxp][ne] (z, y, x-octant index padded to nxp, entry),
 * the transform of the windowed kernel on the 2n grid at frequencies
 * q in [0, n]^3, scaled by (2n)^-3 (curl entries also by i omega).
 * host_bytes must be at least the size reported in *needed. */
int vie_copy_tables(const vie_plan *pl, double *host, long host_bytes, long *needed, int *nxp, int *ne);

/* Copies the FP64 contrast H (and H_mu if present) into host memory as
 * complex128 [9][n^3] (followed by [9][n^3] for H_mu). */
int vie_copy_contrast(const vie_plan *pl, double *host, long host_bytes);

const char *vie_status_string(int status);
/* Message of the last failure on pl; with pl == NULL, of the last failed
 * vie_plan_create on the calling thread. */
const char *vie_last_error(const vie_plan *pl);

/* Whether n is a supported grid size (1/0). */
int vie_supported_n(int n);

/* Scattered potential phi_scat = div V_omega J on the grid (Laplace and
 * Helmholtz; the summary of Section 3: F = V_omega J solves the vector
 * problem and div F the anisotropic scalar one).  density: complex128
 * [nrhs][3][n^3], phi: complex128 [nrhs][n^3], device pointers.  The symbol
 * i s G^ is windowed and transformed like the operator's (built at the first
 * call); FP64.  VIE_E_STATE for Maxwell plans. */
int vie_potential(vie_plan *pl, const double *density, double *phi, int nrhs, void *hip_stream);

/* Maxwell with mu = I: H_tot = H_inc - i omega curl V_omega J on the grid
 * (eq. represent_Maxwell_reduced; vie_field gives E).  h_inc may be NULL
 * (then the scattered field).  Device pointers, complex128 [nrhs][3][n^3];
 * FP64.  VIE_E_STATE for other plans (full Maxwell: vie_field gives E and H). */
int vie_field_h(vie_plan *pl, const double *density, const double *h_inc, double *h, int nrhs, void *hip_stream);

/* Scattered fields at user points away from the density, by direct sums over
 * the grid points y of the free-space kernel G = e^{i omega r}/(4 pi r) with
 * weights h^3 (the representations of Sections 3 and 4, eqs. Vw,
 * represent_Maxwell):
 *   Laplace, Helmholtz: (phi, d_x phi, d_y phi, d_z phi), phi = div V J;
 *   Maxwell: (E_x, E_y, E_z, H_x, H_y, H_z) of eq. represent_Maxwell (M = 0
 *   for mu = I).
 * density: device complex128 [nrhs][c][n^3]; points: HOST double [npts][3]
 * (grid coordinates, origin as in vie_problem); out: device complex128
 * [nrhs][npts][4 or 6].  Every point must lie outside the support box grown
 * by 2h (VIE_E_ARG otherwise), where the sums are spectrally accurate for
 * smooth densities.  Only the density inside the support box is read (a
 * solution of vie_solve is zero outside it).  FP64. */
int vie_fields_at(vie_plan *pl, const double *density, int nrhs, const double *points, int npts, double *out,
                  void *hip_stream);

/* Far-field patterns f(r d) = e^{i omega r}/r f_inf(d) + O(1/r^2) in unit
 * directions d (HOST double [ndirs][3]), from J^(d) = sum h^3 e^{-i omega d.y} J(y):
 *   Helmholtz: phi_inf = (i omega / 4 pi) d . J^  (1 value);
 *   Maxwell: E_inf = (omega^2 / 4 pi)[(I - d d^T) J^ - d x M^],
 *            H_inf = (omega^2 / 4 pi)[(I - d d^T) M^ + d x J^]  (6 values).
 * out: device complex128 [nrhs][ndirs][1 or 6].  VIE_E_STATE for Laplace;
 * VIE_E_ARG for a direction that is not a unit vector.  Only the density
 * inside the support box is read.  FP64. */
int vie_far_field(vie_plan *pl, const double *density, int nrhs, const double *dirs, int ndirs, double *out,
                  void *hip_stream);

/* Upper estimate of the device bytes a plan of this size holds at its peak
 * (the larger of: the kernel-table precompute, or the plan plus apply
 * workspaces and a Krylov basis of `restart` vectors for batches of
 * nrhs_batch right-hand sides).  Host-only; -1 on bad arguments.  Used for
 * admission control by callers that share one GPU among many plans. */
long vie_footprint_bytes(int kind, int n, int full, int nrhs_batch, int restart);

/* Kernel timing.  vie_profile(pl, 1) starts recording a HIP event pair on the
 * launch stream around every kernel of the apply passes and of the Krylov
 * operations (and resets the totals); vie_profile(pl, 0) stops.
 * vie_profile_read waits for the recorded events and writes, per kernel
 * family, the summed duration in milliseconds, the launch count, the
 * summed algorithmic bytes (every operand of a launch read or written once)
 * and the summed nominal flops (5 L log2 L per transformed pencil of length
 * L, 66 per frequency point for the 3x3 multiply and 216 for the 6x6 Maxwell
 * block, 72 per point and 3-component half for the combine, 8 per complex
 * multiply-add of the Krylov operations); host arrays of nfam entries, flops
 * may be NULL.  It returns the number of families.
 * vie_profile_family(i) names family i. */
int vie_profile(vie_plan *pl, int enable);
int vie_profile_read(vie_plan *pl, double *ms, long *counts, double *bytes, double *flops, int nfam);
const char *vie_profile_family(int fam);

#ifdef __cplusplus
}
#endif

#endif /* VIE_H */
