/*
 * sbd.h - C ABI of the MI355X Sparse Bessel Decomposition (SBD) matvec.
 *
 * Computes the discrete convolution of the paper's Introduction (eq.
 * "discreteConv"), q_k = sum_{l != k} G(z_k - z_l) f_l, for points z in R^2,
 * with the algorithm of Section 1 (M. Averseng, "Fast discrete convolution in
 * R^2 using Sparse Bessel Decomposition"):
 *
 *   off-line (sbd_plan):  sparse spectrum sampling (SBD fit of Sections 3-4,
 *                         circular quadrature of Section 5), fixed-radius
 *                         neighbour search and close-correction matrix D
 *                         (Section 1, eq. "defD");
 *   on-line  (sbd_apply): q_far = NUFFT_+(omega_hat * NUFFT_-(f))
 *                         (eq. "far convolution", Section 6.2 steps (i)-(iii)),
 *                         q_close = D f, q = q_far + q_close.
 *
 * Kernels: SBD_LAPLACE G(x) = -(1/2 pi) log|x|; SBD_HELMHOLTZ
 * G(x) = (i/4) H0^(1)(k|x|) (Section 4.2); SBD_GENERAL a log-plus-trigonometric
 * radial kernel (Section 4.3, see sbd_kernel).  The self term l = k is omitted.
 * For Helmholtz the Y0 part is fitted through the next zero kappa' of Y0 when
 * kappa = k delta_max is at or above the first zero of Y0, and below it in the
 * Dini basis of the Robin condition u' + H u = 0, H = -kappa Y0'(kappa)/Y0(kappa)
 * (Section 2.3; the small-k case of Section 4.2), which needs no rescaling.
 *
 * Accuracy: eps bounds the L-infinity error of the unit-scaled radial fit
 * (eps/2) plus the circular quadrature (eps/2), so that for every k
 * |q_k - exact_k| <= c_G * eps * sum_l |f_l| up to the NUFFT tolerance
 * (Section 1, "Output"), with c_G = 1/(2 pi) for Laplace and 1/4 for
 * Helmholtz.
 *
 * Memory: every pointer argument documented "device" is HIP device memory on
 * the current device; "host" pointers are ordinary host memory.  The caller
 * owns all buffers it passes; the plan copies what it needs and owns all of
 * its internal allocations until sbd_free.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default
 * stream).  sbd_plan synchronises the stream (it reads back sizes);
 * sbd_apply only enqueues work and never synchronises.
 *
 * Errors: every function returns an sbd_status and never aborts.
 * sbd_last_error() returns a thread-local description of the last failure.
 * Asynchronous device faults surface as SBD_EHIP on a later call.
 */
#ifndef SBD_H_
#define SBD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbd_plan_s* sbd_plan_t;

typedef enum {
  SBD_OK = 0,
  SBD_EINVAL = -1,        /* bad argument (N < 2, eps <= 0, NaN coordinates, ...) */
  SBD_ENOMEM = -2,        /* device allocation failed or byte_cap exceeded */
  SBD_EDUP = -3,          /* two distinct points coincide */
  SBD_EFLOOR = -4,        /* eps below what the SBD fit can reach (Section 4.1 remark) */
  SBD_EHIP = -5,          /* HIP runtime error */
  SBD_EUNSUPPORTED = -6,  /* option combination not implemented */
  SBD_ENOCONV = -7        /* iterative solve stopped above its tolerance (x holds the last iterate) */
} sbd_status;

typedef enum { SBD_LAPLACE = 0, SBD_HELMHOLTZ = 1, SBD_GENERAL = 2 } sbd_kernel_kind;

/* SBD_GENERAL (Section 4.3, general kernel with the multi-Dirichlet condition
 * enforced): the real radial kernel
 *   G(r) = c_log log r + sum_j r^m_j (a_j sin(w_j r) + b_j cos(w_j r)),
 * term j given as terms[4 j .. 4 j + 3] = {m_j, w_j, a_j, b_j} (host memory,
 * read during sbd_plan only), m_j an integer in [0, 8], w_j >= 0, at most 8
 * terms.  The fit subtracts K(r) = sum_{t<=enforce} mu_t J0(omega_t r), with
 * omega_t the roots of J1 nearest the square root of the mean ratio of
 * successive iterates (-Delta)^s G at r = delta_max and mu solving
 * sum_t mu_t omega_t^(2s) J0(omega_t) = (-Delta)^s G(delta_max), s = 1..enforce
 * (0 <= enforce <= 4; 0 fits G itself), and adds K back as extra circles.
 * The error bound of the header's Accuracy paragraph holds with c_G = 1.  f
 * and q are real (SBD_F64 or SBD_F32).  The fit depends on delta_max, so it is
 * never shared between plans (fit_reuse and force_order do not apply), and
 * sbd_info.P counts its fitted circles plus the enforce ones. */
typedef struct {
  int kind;               /* sbd_kernel_kind */
  double wavenumber;      /* k > 0 for SBD_HELMHOLTZ, ignored otherwise */
  double c_log;           /* SBD_GENERAL: coefficient of log r */
  int nterms;             /* SBD_GENERAL: number of trigonometric terms (0..8) */
  const double* terms;    /* SBD_GENERAL: host, [nterms][4] = {m, w, a, b} */
  int enforce;            /* SBD_GENERAL: multi-Dirichlet order n (0..4) */
} sbd_kernel;

/* Element type of f and q in sbd_apply (layout [nrhs][N], row-major). */
typedef enum { SBD_F64 = 0, SBD_F32 = 1, SBD_C128 = 2, SBD_C64 = 3 } sbd_dtype;

/* Which parts of q sbd_apply computes. */
enum { SBD_PART_FAR = 1, SBD_PART_NEAR = 2, SBD_PART_ALL = 3 };

/* Flag for the parts argument of sbd_apply_parts: f is read and q written in the plan's
 * sorted order instead of the caller's: entry i of f belongs to source perm[i], entry k of
 * q to target tperm[k] (SBD_ARR_PERM / SBD_ARR_TPERM; tperm = perm for one point set).
 * Callers that apply the operator many times (iterative solvers) permute once and avoid
 * the scattered reads of f and writes of q that user order costs for unordered points. */
enum { SBD_IO_SORTED = 4 };

typedef struct {
  double delta_min;       /* near/far radius; <= 0 selects the curve rule of
                             Theorem 1 with alpha = 0: a = |ln eps|^(2/3) / N^(2/3) */
  int precision;          /* 0: far field in FP32 (complex64 grids),
                             1: far field in FP64 (complex128 grids) */
  int max_rhs;            /* largest nrhs sbd_apply will be called with (>= 1) */
  double nufft_tol;       /* worst-case plane-wave reconstruction error of the spreading
                             kernel; <= 0 selects eps (floored at 2e-8 FP32, 1e-14 FP64) */
  double sigma;           /* x-grid oversampling; <= 0 selects 1.25 */
  int force_order;        /* > 0 forces the number P of Bessel terms */
  int tile;               /* grid tile edge (cells); 0 selects 32 */
  int timing;             /* 1: record a HIP event after every kernel sbd_apply launches
                             (read with sbd_launch_times) */
  size_t byte_cap;        /* 0: no cap; else SBD_ENOMEM if plan + workspace exceed it */
  int fit_reuse;          /* 1: share SBD fits between plans of this process.  The fit is
                             made on [a', 1] with a' = 2^(-k/8) the largest such value
                             <= a = delta_min / delta_max (a fit on a larger annulus keeps
                             the eps bound of Section 1 on [a, 1]; P grows by at most ~9%)
                             and cached by (kernel, eps, a', k delta_max, force_order).
                             0: fit exactly on [a, 1]. */
  int near_fp32;          /* FP32 far-field plans only (precision 0): 0 keeps the close-
                             correction entries D_kl in FP64 and sums each row of D f in FP64
                             (the FP64 entries of Section 1, eq. "defD", where G and its Bessel
                             series cancel); 1 stores D rounded to FP32 (relative rounding
                             6e-8 per entry, 4 bytes instead of 8 per entry) and sums rows in
                             FP32.  Ignored by FP64 plans, which always keep FP64 entries. */
  int deterministic;      /* 1: every sbd_apply of the same f returns bit-identical q: the
                             FP64 spread accumulates in 64-bit fixed point and the close
                             correction sums each row in one fixed order (no float atomics
                             anywhere).  0: the FP64 spread and the close-correction row
                             partial sums use FP64 LDS atomics, whose order varies between
                             runs (differences in the last bits of q).  The FP32 spread is
                             fixed-point, hence reproducible, in both modes. */
  int near_assembly;      /* how the entries D_kl (Section 1, eq. "defD") are computed.
                             0: G(r) minus the radial Bessel series sum_p alpha_p J0(rho_p r)
                             (the limit of the circle quadrature), from FP64 Chebyshev tables
                             in r^2 inside the neighbour-search kernel.
                             1: G(y) minus the plane-wave sum over every circle node at each
                             pair difference y = z_k - z_l (targets minus sources for
                             sbd_plan_targets), evaluated as a type-3 NUFFT in FP64 (Section 1;
                             Section 6.1, eq. "Complex:assemble") with tolerance
                             pd_tol = max(1e-13, min(1e-8, 1e-3 nufft_tol)) relative to the
                             l1 norm of the weights.  The two differ by the quadrature error
                             and the NUFFT tolerance.  SBD_LAPLACE and SBD_HELMHOLTZ only; the
                             frequency grid (about 2 (2 S delta_min / pi + w / 2) cells per
                             axis, S the largest circle radius) is limited to 48 cells per axis.
                             SBD_EUNSUPPORTED beyond either limit, SBD_EINVAL for other values.
                             Only the real part of D is stored: for Helmholtz the imaginary
                             parts of G and of the sum cancel up to the same errors. */
} sbd_options;

/* Summary of a plan (all host values). */
typedef struct {
  int64_t n;              /* number of points */
  int kind;               /* sbd_kernel_kind */
  int precision;
  int P;                  /* number of Bessel terms */
  int64_t n_xi;           /* number of frequencies (all circles, plus xi = 0 for Laplace) */
  int64_t nnz;            /* non-zeros of D (diagonal included) */
  double eps, delta_min, delta_max, center_x, center_y;
  double fit_error;       /* max check-grid error of the radial fit (unit-scaled shape) */
  double h;               /* x-grid spacing */
  int w;                  /* spreading kernel width (cells) */
  double beta;            /* exponential-of-semicircle shape parameter */
  double sigma;
  int64_t nx, ny;         /* spread-grid size (cells) */
  int64_t Mx, My;         /* FFT sizes */
  int tile;               /* tile edge (cells) */
  int64_t ntx, nty;       /* tiles per axis */
  /* binning parameters (fine near-field cells, see sbd_plan_export) */
  double x0, y0, inv_c;   /* fine cell fx = clamp(floor((x - x0) * inv_c), 0, ncx - 1) */
  int64_t ncx, ncy;
  int nsub;               /* fine cells per tile edge */
  double d2max;           /* delta_min * delta_min used by the pair predicate */
  double plan_seconds;    /* wall time of sbd_plan */
  double fit_seconds;     /* host SBD fit part of it */
  size_t plan_bytes;      /* resident device bytes */
  int64_t n_targets;      /* number of targets (= n for a plan made by sbd_plan) */
  int bipartite;          /* 1: plan made by sbd_plan_targets */
  int near_fp32;          /* 1: close-correction entries stored in FP32 (see sbd_options) */
  int deterministic;      /* 1: bit-reproducible applies (see sbd_options) */
  int colconv;            /* 1: the column transforms run as one compiled whole-column
                             convolution of length My (0: generic column passes) */
  int near_assembly;      /* sbd_options.near_assembly of the plan */
  int pd_grid;            /* near_assembly = 1: frequency-grid cells per axis (else 0) */
  double pd_tol;          /* near_assembly = 1: tolerance of the pair-difference NUFFT */
  double near_seconds;    /* wall time of the neighbour search and the series entries */
  double assembly_seconds;/* wall time of the pair-difference NUFFT (0 unless near_assembly) */
  double bin_seconds;     /* wall time of the binning (keys, counting sort, sorted copies) */
  double symbol_seconds;  /* wall time of the Toeplitz symbol (node spreading, FFTs) */
  int row_pairs;          /* 1: real-data applies store the row spectra interleaved in row
                             pairs (compiled row and column transforms; the layout moves
                             data only: results match natural rows, bit for bit in FP32 and
                             to rounding in FP64); SBD_ROW_PAIRS=0 in the environment at plan
                             time keeps natural rows */
} sbd_info;

/* Arrays sbd_plan_export can copy out. */
typedef enum {
  SBD_ARR_PERM = 0,       /* int32 [N]: sorted position -> input index */
  SBD_ARR_ROWPTR = 1,     /* int64 [N+1]: CSR row pointer of D (rows in sorted order) */
  SBD_ARR_COL = 2,        /* int32 [nnz]: CSR columns (sorted positions, ascending) */
  SBD_ARR_VAL = 3,        /* double [nnz]: real part of D (Helmholtz: D is real off the
                             diagonal; the diagonal's imaginary part is -1/4) */
  SBD_ARR_COEF = 4,       /* double [P]: coefficient of J0(r_p s) in the fitted shape */
  SBD_ARR_RADII = 5,      /* double [P]: unit-scaled circle radii r_p */
  SBD_ARR_M = 6,          /* int64 [P]: nodes per circle M_p */
  SBD_ARR_KEYS = 7,       /* int64 [N]: sort key of each sorted point (source) */
  SBD_ARR_TPERM = 8,      /* int32 [M]: sorted target position -> target index (= PERM for sbd_plan) */
  SBD_ARR_TKEYS = 9       /* int64 [M]: sort key of each sorted target */
} sbd_array;

/* Fill opt with the defaults described in sbd_options. */
void sbd_default_options(sbd_options* opt);

/*
 * Off-line part (Section 1).  points: device, [n][2] FP64, x then y.
 * kernel: host pointer.  eps > 0.  opt: host pointer or NULL for defaults.
 * On success *out receives the plan; on failure *out is NULL.
 */
sbd_status sbd_plan(const double* points, int64_t n, const sbd_kernel* kernel, double eps,
                    const sbd_options* opt, void* stream, sbd_plan_t* out);

/*
 * Off-line part for separate targets and sources (the two-set form of the
 * paper's numerical experiments, Section 7):
 *
 *   q_k = sum_l G(x_k - y_l) f_l,  k < m (targets x), l < n (sources y),
 *
 * with no term omitted.  targets: device [m][2] FP64; sources: device [n][2]
 * FP64.  The bounding box and delta_max cover both sets; the default
 * delta_min rule uses n.  D has one row per target and its columns are sorted
 * source positions.  sbd_apply then reads f as [nrhs][n] and writes q as
 * [nrhs][m].  A target that coincides with a source returns SBD_EDUP.
 */
sbd_status sbd_plan_targets(const double* targets, int64_t m, const double* sources, int64_t n,
                            const sbd_kernel* kernel, double eps, const sbd_options* opt, void* stream,
                            sbd_plan_t* out);

/*
 * Sparse spectrum sampling alone (Section 1, off-line part; the fit of Section 2):
 * computes the SBD fit of kernel for tolerance eps on the annulus ratio
 * a = delta_min / delta_max and stores it in the process-wide fit cache that plans
 * made with sbd_options.fit_reuse = 1 share, under the same key such a plan uses
 * (kernel kind, eps, a' = 2^(-k/8) the largest such value <= a, wavenumber * delta_max
 * for SBD_HELMHOLTZ, force_order).  Host computation only (no device memory, no
 * stream); a server calls it at start-up for the annulus ratios its requests will
 * need.  delta_max only matters for SBD_HELMHOLTZ.  *out_P (may be NULL) receives the
 * number of Bessel terms.  SBD_EUNSUPPORTED for SBD_GENERAL (fitted per plan),
 * SBD_EINVAL for eps or a outside (0, 1), SBD_EFLOOR when eps is below what the fit
 * reaches.  Thread-safe.
 */
sbd_status sbd_prefit(const sbd_kernel* kernel, double eps, double a, double delta_max, int force_order,
                      int* out_P);

/*
 * Device memory cache for a process that makes and frees many plans (a server).  While
 * the limit is positive, every block of 32 MiB or more that sbd_plan, sbd_plan_targets,
 * sbd_apply (internal workspace) or sbd_gmres allocates comes from hipMalloc in size
 * classes 2^(k/4) bytes (rounded up to 2 MiB), and when released it is kept for a later
 * request of the same class on the same device instead of being freed: plan temporaries
 * at the end of sbd_plan (stream-ordered: the next user waits on an event recorded on the
 * releasing stream), a plan's arrays at sbd_free (the plan must then be idle, see
 * sbd_free).  Reuse avoids the device driver's cost of supplying freshly allocated
 * memory, which grows with the volume allocated.  At most `bytes` are kept (largest
 * classes freed first).  While the limit is positive every release is stream-ordered
 * (hipFreeAsync) and none waits for the whole device, so freeing plans on one thread
 * never disturbs a stream that another thread is capturing into a graph (sbd_gmres
 * does).  0, the default, disables the cache and frees what it holds.  Thread-safe; one
 * cache for all devices of the process.  Always SBD_OK.
 */
sbd_status sbd_set_cache_limit(size_t bytes);

/* Device bytes the cache of sbd_set_cache_limit holds (free blocks only). */
size_t sbd_cache_bytes(void);

/* Bytes of device workspace sbd_apply needs for nrhs right-hand sides. */
size_t sbd_workspace_bytes(sbd_plan_t plan, int nrhs);

/* Resident device bytes held by the plan (for admission control). */
size_t sbd_plan_bytes(sbd_plan_t plan);

/*
 * On-line part (Section 1): q = q_far + q_close for nrhs right-hand sides.
 * f: device, [nrhs][N] of dtype; q: device, [nrhs][M] of dtype (overwritten),
 * with M = N except for plans made by sbd_plan_targets.
 * Laplace accepts SBD_F64, SBD_F32 (real f, real q) and SBD_C128, SBD_C64;
 * Helmholtz accepts SBD_C128 and SBD_C64.  workspace: device buffer of at
 * least sbd_workspace_bytes(plan, nrhs) bytes, or NULL to use a workspace the
 * plan allocates on first use (then calls on one plan must not overlap).
 * 1 <= nrhs <= opt.max_rhs.  Asynchronous on `stream`.
 * Non-finite f: f is not checked.  A NaN or infinite value makes q NaN or
 * infinite at every point, because the far field mixes every source (the
 * fixed-point spread of FP32 plans and of deterministic FP64 plans, which has
 * no scale for such a value, writes its tile as NaN; the FP64 floating-point
 * spread carries the value into the grid).
 */
sbd_status sbd_apply(sbd_plan_t plan, const void* f, void* q, int nrhs, int dtype,
                     void* workspace, size_t workspace_bytes, void* stream);

/*
 * As sbd_apply, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * workspace is a static device array of SBD_NOALLOC_SCRATCH_BYTES (64 MiB) in
 * the library, one per device, held until the process ends; its device address
 * is looked up once per device on the first call there.  The call allocates and
 * frees nothing and records no timing events (sbd_options.timing is ignored).
 * f, q: device, as for sbd_apply (the caller still owns them).  Returns
 * SBD_ENOMEM, before any launch, when sbd_workspace_bytes(plan, nrhs) exceeds
 * SBD_NOALLOC_SCRATCH_BYTES.  Every call on one device shares that device's
 * array, which keeps the last call's contents (the apply needs no cleared
 * memory: every workspace value is written before it is read).  Calls that
 * overlap on one device, on different streams or from different threads,
 * race on the array: serialise them.  Asynchronous on `stream`.
 */
#define SBD_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
sbd_status sbd_apply_noalloc(sbd_plan_t plan, const void* f, void* q, int nrhs, int dtype, void* stream);

/* As sbd_apply, restricted to the parts in `parts` (SBD_PART_FAR / SBD_PART_NEAR), with
 * f and q in the plan's sorted order when SBD_IO_SORTED is set too. */
sbd_status sbd_apply_parts(sbd_plan_t plan, const void* f, void* q, int nrhs, int dtype,
                           int parts, void* workspace, size_t workspace_bytes, void* stream);

/* Copy the plan summary into *out (host). */
sbd_status sbd_plan_info(sbd_plan_t plan, sbd_info* out);

/* Copy an internal array into a host buffer of `bytes` bytes (synchronous). */
sbd_status sbd_plan_export(sbd_plan_t plan, int which, void* host_dst, size_t bytes);

/* Release the plan and everything it owns.  NULL is a no-op.  With the device cache off
 * (sbd_set_cache_limit(0), the default) the release waits for the device as hipFree does,
 * so work still queued with the plan is safe.  With the cache on, the plan must be idle:
 * every stream that used it synchronised; nothing then waits for the whole device. */
void sbd_free(sbd_plan_t plan);

/* Switch per-launch event timing on or off for later sbd_apply calls (0 ok, -1 NULL plan). */
int sbd_set_timing(sbd_plan_t plan, int enable);

/*
 * Per-kernel timing of the sbd_apply calls made while timing was on, since
 * the last call.  Synchronises on the recorded events.  Writes up to
 * max_entries kernel labels into `names` (host, newline-separated,
 * NUL-terminated, names_bytes bytes), into ms[i] (host) the milliseconds per
 * sbd_apply call between the events before and after the launches with label
 * i (summed over launches with the same label), and into bytes[i] (host, may
 * be NULL) the algorithmic bytes those launches move per call (each element
 * of their input read once, each output written once).  Returns the number of
 * entries, or -1 for a NULL plan.  Resets the accumulated values.
 */
int sbd_launch_times(sbd_plan_t plan, char* names, size_t names_bytes, double* ms, double* bytes, int max_entries);

/*
 * Restarted GMRES on the SBD operator, for integral equations whose dense
 * matrix is the kernel times quadrature weights (the use of the fast matvec
 * that the Introduction motivates):
 *
 *   (A v)_k = sum_{l != k} G(z_k - z_l) w_l v_l + d_k v_k,
 *
 * i.e. sbd_apply of (w o v) plus a diagonal, solved for A x = b.  Real
 * kernels only: SBD_LAPLACE and SBD_GENERAL plans (real FP64 vectors).  Arnoldi with classical Gram-Schmidt
 * applied twice, Givens rotations on the host (one small device-to-host read
 * and one stream synchronisation per iteration).
 */
typedef struct {
  int restart;            /* Krylov dimension m per cycle, 1..64; 0 selects 30 */
  int max_restarts;       /* cap on cycles; 0 selects 100 */
  double rtol;            /* stop when ||b - A x||_2 <= rtol ||b||_2; <= 0 selects 1e-6 */
  int zero_guess;         /* 1: start from x = 0 (x is not read); 0: x holds the initial guess */
} sbd_gmres_options;

/* Device bytes of workspace sbd_gmres needs for restart m (0: 30); 0 on bad arguments. */
size_t sbd_gmres_workspace_bytes(sbd_plan_t plan, int restart);

/*
 * weights, diag: device FP64 [N] or NULL (all ones / all zeros).  b: device
 * FP64 [N].  x: device FP64 [N], initial guess on entry (unless zero_guess),
 * solution on exit.  All in the user's point order.  opt: host pointer or
 * NULL for defaults.  workspace: device buffer of at least
 * sbd_gmres_workspace_bytes bytes, or NULL to allocate and free one inside
 * the call.  iterations (host, may be NULL): Arnoldi steps taken (operator
 * applications minus residual checks).  relres (host, may be NULL): the true
 * relative residual ||b - A x|| / ||b|| of the returned x, recomputed with
 * the operator.  Synchronises `stream`.  Returns SBD_ENOCONV when the cycle
 * cap is reached above rtol, SBD_EUNSUPPORTED for Helmholtz plans.
 */
sbd_status sbd_gmres(sbd_plan_t plan, const double* weights, const double* diag, const double* b, double* x,
                     const sbd_gmres_options* opt, void* workspace, size_t workspace_bytes, void* stream,
                     int* iterations, double* relres);

/* Static description of a status code. */
const char* sbd_strerror(sbd_status status);

/* Thread-local description of the last error (empty if none). */
const char* sbd_last_error(void);

/*
 * 2-D complex FFT of the library (the transform inside NUFFT_-/NUFFT_+ of
 * Section 1), exposed for testing: data is device memory [ny][nx] complex
 * (dtype SBD_C128 or SBD_C64), transformed in place along both axes
 * (dir = -1: exp(-2 pi i ...), +1: exp(+2 pi i ...), unnormalised).  ny and nx
 * must have no prime factor above 7.  Synchronous.
 */
sbd_status sbd_fft2(void* data, int64_t ny, int64_t nx, int dtype, int dir, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SBD_H_ */
