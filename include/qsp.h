/*
 * qsp.h -- C ABI of libqsp, an MI355X (gfx950) implementation of the
 * quasi-static particle-in-cell per-slice loop of HiPACE++
 * (S. Diederichs et al., arXiv:2109.10277).
 *
 * One context holds one simulation box: a transverse node grid, one slice of
 * plasma electrons with their Adams-Bashforth history, the few field slices
 * the loop needs and the drive beam.  The box is computed slice by slice
 * from its head (zeta_hi) to its tail, each slice following the 2D slice
 * routine of Sec. II (push, plasma deposit, beam deposit, psi / Ez / Bz
 * solves, Bx/By predictor-corrector).  All work runs in hand-written HIP
 * kernels on the stream given at creation.
 *
 * Conventions (every entry point):
 *  - Return value: QSP_OK (0) or an error code; no exception crosses the ABI.
 *    Argument and state errors are found before any device work starts and
 *    leave the context and all outputs untouched.  A device error is sticky:
 *    every later call on the context returns QSP_ERR_DEVICE.
 *    qsp_last_error() gives a message for the last failure.
 *  - Ownership: the context owns all of its device memory.  Pointers passed in
 *    are borrowed for the duration of the call only.  "device" pointers must
 *    point to device memory of the context's GPU, "host" pointers to host
 *    memory.  Device outputs are written asynchronously on the context's
 *    stream; host outputs are complete when the call returns (those calls
 *    synchronise the stream and say so).
 *  - Grid layout of every node array passed across the ABI: row-major
 *    [ny+1][nx+1], element [j][i] is node (x_lo + i*hx, y_lo + j*hy).
 *    Boundary rows and columns (i or j equal to 0 or n) are zero for fields.
 *  - Field arrays are float (QSP_FP32 contexts) or double (QSP_FP64);
 *    charge/current deposits are always double.
 *  - Threads: a context may be used by one host thread at a time.
 */
#ifndef QSP_H
#define QSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QSP_ABI_VERSION 1

typedef enum {
  QSP_OK = 0,
  QSP_ERR_INVALID_ARG = 1,   /* bad argument or configuration             */
  QSP_ERR_BAD_STATE = 2,     /* call out of order (see state machine)     */
  QSP_ERR_OUT_OF_MEMORY = 3, /* device allocation failed or over mem cap  */
  QSP_ERR_DEVICE = 4,        /* HIP error; sticky until qsp_destroy       */
  QSP_ERR_NONFINITE = 5      /* NaN/Inf met in a field norm or residual   */
} qsp_status;

enum { QSP_FP32 = 0, QSP_FP64 = 1 };

/* Bx/By field solver (Sec. III.B offers two). */
enum { QSP_BXBY_PC = 0, QSP_BXBY_EXPLICIT = 1 };

/* Quantities a slice produces, in the order used by every output array
 * below.  The first seven are fields (precision of the context), the last
 * five are deposits of slice k including ions and beam (always double). */
enum {
  QSP_PSI = 0,     /* wake potential psi,                eq. (psi)            */
  QSP_EXMBY = 1,   /* Ex - By = -d_x psi,                eq. (exmby)          */
  QSP_EYPBX = 2,   /* Ey + Bx = -d_y psi,                eq. (exmby)          */
  QSP_EZ = 3,      /* Ez,                                eq. (ez)             */
  QSP_BX = 4,      /* Bx after the predictor-corrector,  eq. (bxby)           */
  QSP_BY = 5,      /* By after the predictor-corrector,  eq. (bxby)           */
  QSP_BZ = 6,      /* Bz,                                eq. (bz)             */
  QSP_RHO_MJZ = 7, /* rho - Jz                                                */
  QSP_JX = 8,
  QSP_JY = 9,
  QSP_JZ = 10,
  QSP_RHO = 11,
  QSP_NQ = 12
};

/* Box description.  Normalised units (Sec. VI): lengths in k_p^-1,
 * densities in n0, fields in E0.
 *   nodes    x_i = x_lo + i*(x_hi-x_lo)/nx, i = 0..nx (same for y); zero
 *            Dirichlet values on i or j in {0, n}.  nx, ny: powers of two,
 *            16 <= n <= 2048.
 *   slices   zeta_k = zeta_hi - k*dzeta, k = 0..nzeta-1 (head first).
 *   plasma   electrons start at rest on (nx*ppc_x) x (ny*ppc_y) lattice sites,
 *            site (I, J) at (x_lo + (I+1/2)*hx/ppc_x, y_lo + (J+1/2)*hy/ppc_y),
 *            particle index I + J*nx*ppc_x; immobile ions of density n0.
 *   solver   Bx/By predictor-corrector: at most pc_max_iter iterations, stop
 *            when the relative change of (Bx, By) drops below pc_tol
 *            (pc_tol <= 0: always pc_max_iter).  pc_shift < 0 selects the
 *            default screening shift (1901/1440)*n0.  psi_floor is the
 *            floor applied to 1 + Psi of a plasma particle (0 < floor < 1).
 *   deposit_mode: 0 (default) accumulates each workgroup's particles in FP64
 *            LDS histograms before the global FP64 atomics, 1 sends every
 *            particle contribution straight to global FP64 atomics (same
 *            result up to summation order; kept for differential testing).
 *   mem_cap_bytes: 0 = no cap, else creation fails with
 *            QSP_ERR_OUT_OF_MEMORY if the context would hold more.
 *   shape_order: transverse particle shape of plasma and beam deposit and
 *            gather (Sec. III.B: orders 0-3 transversely, zeroth order in
 *            zeta), the centred B-spline of that degree: 0 nearest node,
 *            1 linear (CIC, the usual choice), 2 quadratic, 3 cubic.  A
 *            zero-initialised config selects 0.  The ions are the
 *            electrons' rest lattice deposited with the same shape, so the
 *            unperturbed plasma is neutral at every node.
 *   bxby_solver: QSP_BXBY_PC (the predictor-corrector above) or
 *            QSP_BXBY_EXPLICIT: d_zeta J_perp integrated analytically along
 *            the plasma orbits, which turns eq. (bxby) into
 *            (lap - chi) B = R with chi = sum w S / (1 + Psi) per node; it is
 *            solved by conjugate gradients preconditioned with the sine
 *            transform of (lap - c0), c0 = pc_shift (< 0: n0).  For this
 *            solver pc_max_iter bounds the conjugate-gradient iterations and
 *            pc_tol is their relative residual target; it needs
 *            shape_order >= 1 and has no adjoint. */
typedef struct {
  int32_t nx, ny;
  double x_lo, x_hi, y_lo, y_hi;
  int32_t nzeta;
  int32_t precision; /* QSP_FP32 or QSP_FP64 */
  double zeta_hi, dzeta;
  int32_t ppc_x, ppc_y;
  double n0;
  int32_t pc_max_iter;
  int32_t deposit_mode; /* 0: LDS-tiled FP64 histograms, 1: direct global atomics */
  double pc_tol;
  double pc_shift;
  double psi_floor;
  int64_t mem_cap_bytes;
  int32_t shape_order; /* 0..3 */
  int32_t bxby_solver; /* QSP_BXBY_PC or QSP_BXBY_EXPLICIT */
} qsp_config;

/* Per-slice outputs of qsp_advance_slice: one device pointer per quantity
 * (NULL = not wanted), each a [ny+1][nx+1] node array of slice k. */
typedef struct {
  void* q[QSP_NQ];
} qsp_slice_out;

/* Per-box outputs of qsp_run_box (device pointers, NULL = not wanted).
 *   stack[q]    [n_stack][ny+1][nx+1] node arrays of slices
 *               k = k0, k0+stack_every, ... (k0 = first slice of the run,
 *               n_stack = ceil((nzeta-k0)/stack_every)); stack_every >= 1.
 *   lineout[q]  [nzeta-k0][nx+1]: row j = ny/2 of every slice.
 *   axis[q]     [nzeta-k0]: node (nx/2, ny/2) of every slice.
 *   pc_iters    int32  [nzeta-k0]: predictor-corrector iterations per slice.
 *   pc_resid    double [nzeta-k0]: last relative change of (Bx, By). */
typedef struct {
  void* stack[QSP_NQ];
  int32_t stack_every;
  int32_t reserved0;
  void* lineout[QSP_NQ];
  void* axis[QSP_NQ];
  int32_t* pc_iters;
  double* pc_resid;
} qsp_box_out;

/* Counters since qsp_init_plasma (host struct, filled synchronously). */
typedef struct {
  int64_t slices;             /* slices computed                              */
  int64_t particle_pushes;    /* real plasma pushes (particles x slices)       */
  int64_t pc_iterations;      /* predictor-corrector iterations, all slices    */
  int64_t pc_not_converged;   /* slices that hit pc_max_iter with pc_tol > 0   */
  int64_t n_clamped;          /* real pushes in which 1 + Psi was floored      */
  int64_t n_absorbed;         /* plasma particles absorbed at the box edge     */
  int64_t n_deposit_global;   /* particle deposits outside their LDS tile      */
  int64_t dst_solves;         /* scalar 2D Dirichlet solves                    */
  double max_pc_residual;     /* largest final residual of a slice             */
  double elapsed_ms;          /* device time of the last qsp_run_box           */
  int64_t device_bytes;       /* device memory held by the context             */
  int64_t box_reruns;         /* boxes run a second time: a box replayed with  */
                              /* the speculative predictor-corrector launch    */
                              /* budgets left a slice unconverged below        */
                              /* pc_max_iter, and was rerun with every         */
                              /* iteration launched (results are those of the  */
                              /* second run)                                   */
} qsp_stats;

/* Full state at the start of slice k (host arrays, double precision, in
 * the particle order defined by qsp_config).  Used to resume a box and to
 * import an externally computed state.
 *   x, y        absolute particle positions [np]
 *   ux, uy, psi transverse momentum and Psi of the pusher [np]
 *   w           macro weight per cell area n0/(ppc_x*ppc_y); 0 = absorbed [np]
 *   hist        [4][5][np]: hist[m] is the right-hand side f_{k-1-m} of
 *               (x, y, ux, uy, Psi), m = 0..3 (zeros before slice 0)
 *   jx_prev, jy_prev          [ny+1][nx+1] J_perp of slice k-1
 *   bx_prev1, by_prev1        [ny+1][nx+1] Bx, By of slice k-1
 *   bx_prev2, by_prev2        [ny+1][nx+1] Bx, By of slice k-2 */
typedef struct {
  int32_t k;
  int32_t reserved0;
  int64_t np;
  double *x, *y, *ux, *uy, *psi, *w;
  double* hist;
  double *jx_prev, *jy_prev;
  double *bx_prev1, *by_prev1, *bx_prev2, *by_prev2;
} qsp_slice_state;

/* Opaque context handle. */
typedef struct qsp_ctx_s* qsp_ctx;

/* Checks a configuration without touching any GPU.  On failure writes a
 * NUL-terminated reason into msg (if msg != NULL and msg_len > 0).
 * Returns QSP_OK or QSP_ERR_INVALID_ARG. */
qsp_status qsp_validate_config(const qsp_config* cfg, char* msg, size_t msg_len);

/* Creates a context on HIP device `device`; all later work of the context is
 * enqueued on `hip_stream` (a hipStream_t; NULL = the null stream).  Allocates
 * every device buffer the box needs (the size does not depend on nzeta).
 * On success *out holds the new context; on failure *out is NULL. */
qsp_status qsp_create(const qsp_config* cfg, int device, void* hip_stream,
                      qsp_ctx* out);

/* Releases the context and its device memory (synchronises its stream).
 * NULL is accepted and ignored. */
qsp_status qsp_destroy(qsp_ctx ctx);

/* Puts the unperturbed plasma ahead of the box (Sec. II): electrons at rest
 * on the lattice, Psi = 0, zero Adams-Bashforth history, zero J_perp and
 * Bx/By of the (virtual) previous slices; moves the slice cursor to 0 and
 * clears the counters.  The beams are kept. */
qsp_status qsp_init_plasma(qsp_ctx ctx);

/* Rigid, ultra-relativistic electron drive beam with a Gaussian transverse
 * profile, sampled at the nodes of each slice (zeroth order in zeta):
 * n_b(x, y, zeta_k) = amp[k] * exp(-(x-x0)^2/(2 sx^2) - (y-y0)^2/(2 sy^2)),
 * giving rho_b = Jz_b = -n_b and J_perp,b = 0 (Sec. II step 3).
 * amp: host array [nzeta] (copied).  Replaces any previous Gaussian beam.
 * Errors: non-finite amp, sx <= 0 or sy <= 0 -> QSP_ERR_INVALID_ARG. */
qsp_status qsp_set_beam_gaussian(qsp_ctx ctx, const double* amp, double sx,
                                 double sy, double x0, double y0);

/* Macro-particle electron beam (Sec. III.A: beam particles sorted per slice
 * and deposited inside the slice loop).  soa: device array [7][n] of float,
 * rows x, y, zeta, ux, uy, uz, w (w = physical electrons per macro-particle,
 * in n0 k_p^-3).  The context copies the particles, stably sorted by their
 * nearest slice (NGP in zeta); particles outside the box in zeta are kept,
 * sorted last, and neither deposit nor move.  Each
 * slice deposits its beam particles (with the configured transverse shape) before the field
 * solves and, once the slice's fields are final, advances them by one
 * time step dt (drift-kick-drift, Boris kick; dt = 0: no push).  n = 0
 * removes the particle beam.  Replaces any previous particle beam.  A beam
 * pushed during a box is sorted again by qsp_init_plasma.  Synchronises.
 * Errors: n outside [0, 2^31), null soa with n > 0, non-finite dt, or a
 * particle beam in a box of nzeta >= 16384 slices -> QSP_ERR_INVALID_ARG. */
qsp_status qsp_set_beam_particles(qsp_ctx ctx, int64_t n, const float* soa,
                                  double dt);

/* Explicit drive-beam current of slice k (Sec. II step 3, the beam as a
 * given source): an ultra-relativistic beam with rho_b = Jz_b = jz and
 * J_perp,b = 0, added to the plasma deposit of slice k together with any
 * Gaussian or macro-particle beam.  jz: device array [ny+1][nx+1] of double
 * in node layout (copied; boundary entries ignored), or NULL to remove the
 * current of slice k; k = -1 with jz = NULL removes every slice's current.
 * Each stored slice holds nx*ny doubles of device memory (mem_cap_bytes
 * applies).  Errors: k outside [0, nzeta) (other than the -1 form) ->
 * QSP_ERR_INVALID_ARG. */
qsp_status qsp_set_beam_current(qsp_ctx ctx, int32_t k, const double* jz);

/* Copies the particle beam back (device array [7][n] of float in the sorted
 * order; n must equal the stored count, see qsp_get_beam_count).
 * Synchronises. */
qsp_status qsp_get_beam_particles(qsp_ctx ctx, int64_t n, float* soa);
qsp_status qsp_get_beam_count(qsp_ctx ctx, int64_t* n);

/* Computes slice k (the cursor) and advances the plasma to slice k+1:
 * deposit, beam source, psi/Ez/Bz solves, Bx/By predictor-corrector, real
 * push with deposit at k+1.  Writes the requested quantities of slice k.
 * Errors: cursor == nzeta or plasma not initialised -> QSP_ERR_BAD_STATE. */
qsp_status qsp_advance_slice(qsp_ctx ctx, const qsp_slice_out* out);

/* Runs every remaining slice (cursor .. nzeta-1) and writes the requested
 * outputs.  If stats != NULL it synchronises and fills *stats.
 * Returns QSP_ERR_NONFINITE if a field norm or P-C residual was not finite. */
qsp_status qsp_run_box(qsp_ctx ctx, const qsp_box_out* out, qsp_stats* stats);

/* Counters since qsp_init_plasma (synchronises). */
qsp_status qsp_get_stats(qsp_ctx ctx, qsp_stats* stats);

/* Copies the state at the start of the cursor slice into host arrays
 * (synchronises).  dst->np must equal the particle count; every pointer
 * must be non-NULL. */
qsp_status qsp_get_slice_state(qsp_ctx ctx, qsp_slice_state* dst);

/* Replaces the state at the start of slice src->k (0 <= k < nzeta) and moves
 * the cursor there (synchronises).  Positions must lie inside the box for
 * particles with w > 0.  Like qsp_init_plasma it sorts a pushed
 * macro-particle beam by slice again. */
qsp_status qsp_set_slice_state(qsp_ctx ctx, const qsp_slice_state* src);

/* Batched 2D Dirichlet solve with the context's transforms (Sec. III.B fast
 * Poisson solver): for b < nbatch solves (lap_h - shift) u_b = src_b on the
 * interior nodes, u_b = 0 on the boundary, lap_h the 5-point Laplacian.
 * src, dst: device arrays [nbatch][ny+1][nx+1] in the context's precision
 * (boundary entries of src are ignored); 1 <= nbatch <= 4; shift >= 0.
 * Asynchronous on the context's stream; uses the context's scratch, so it
 * must not overlap other calls on the same context. */
qsp_status qsp_solve_poisson(qsp_ctx ctx, int32_t nbatch, const void* src, void* dst,
                             double shift);

/* The batched 2D Dirichlet solve of qsp_solve_poisson without a context and
 * without allocating device memory, for callers that cannot allocate (code
 * under stream capture, tight serving loops).  Only the grid fields of cfg
 * are read: nx, ny (powers of two in [16, 2048]), x_lo, x_hi, y_lo, y_hi and
 * precision.  Solves (lap_h - shift) u_b = src_b for b < nbatch on
 * `device`, enqueued on `hip_stream` (a hipStream_t; NULL = the null
 * stream); src, dst: device arrays [nbatch][ny+1][nx+1] in the given
 * precision (boundary entries of src ignored, of dst written as 0);
 * 1 <= nbatch <= 4; shift >= 0.  Intermediate planes and transform tables
 * live in one static device array per GPU of 16 MiB + 256 KiB (held from
 * the library's first use on that GPU until the process ends):
 * nbatch * nx * ny values above 16 MiB -> QSP_ERR_INVALID_ARG.  Every call
 * on one GPU uses that GPU's array, so calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller.
 * Asynchronous; argument errors leave dst untouched.  HIP errors ->
 * QSP_ERR_DEVICE (no context, nothing sticky).  qsp_last_error(NULL) gives
 * the message. */
qsp_status qsp_solve_poisson_noalloc(const qsp_config* cfg, int device, void* hip_stream,
                                     int32_t nbatch, const void* src, void* dst,
                                     double shift);

/* Cotangent weights of a recorded run for qsp_run_box_adjoint: the loss is
 *   L = sum_{k = k_lo}^{n-1} sum_F < w_F[k - k_lo], F_k >
 * over the interior nodes, F in psi, Ex-By, Ey+Bx, Ez, Bx, By, Bz of slice
 * k (n = slices of the record).
 *   w[q]  q = QSP_PSI .. QSP_BZ: device array [n - k_lo][ny+1][nx+1] in the
 *         context precision, or NULL for a zero weight.  Boundary nodes
 *         are ignored. */
typedef struct {
  int32_t k_lo;
  int32_t reserved0;
  const void* w[7];
} qsp_box_cotangent;

/* Checkpointed forward pass for the adjoint.  Runs slices 0 .. n_slices-1
 * of the slice loop (Sec. II, with the Sec. III.B predictor-corrector)
 * from the state left by qsp_init_plasma, writes the requested outputs like
 * qsp_run_box (relative slice index = k), keeps the full slice state
 * (particles, Adams-Bashforth history, J_perp of the previous slice, Bx/By
 * of the two previous slices) every ckpt_every slices in device memory and
 * the per-slice record of the last chunk of slices.  Device memory grows by
 * about ceil(n_slices/ckpt_every) slice states plus ckpt_every records;
 * mem_cap_bytes applies.  Requires the cursor at 0, a Gaussian beam, and no
 * macro-particle beam that moves (dt != 0) -> else QSP_ERR_BAD_STATE;
 * 1 <= n_slices <= nzeta, ckpt_every >= 1, shape_order >= 1 (the
 * nearest-node shape has no derivative) and the predictor-corrector
 * Bx/By solver -> else QSP_ERR_INVALID_ARG.
 * Synchronises. */
qsp_status qsp_run_box_record(qsp_ctx ctx, int32_t n_slices, int32_t ckpt_every,
                              const qsp_box_out* out, qsp_stats* stats);

/* Reverse pass of the last qsp_run_box_record: the gradient of the loss of
 * `cot` with respect to the Gaussian beam's per-slice amplitudes and its
 * transverse sizes.  Each chunk of slices is recomputed from its checkpoint
 * (the predictor-corrector takes the iteration counts of that recompute)
 * and then transposed slice by slice in reverse order.  Outputs (device,
 * FP64, overwritten): grad_amp [nzeta] (zero for slices >= n_slices),
 * grad_sigma [2] (d/d sx, d/d sy), loss [1] or NULL (L evaluated on the
 * recomputed fields).  The record is consumed: afterwards the plasma state
 * is an intermediate one and qsp_init_plasma is required before the next
 * run.  Errors: no valid record -> QSP_ERR_BAD_STATE; k_lo outside
 * [0, n_slices) or NULL outputs -> QSP_ERR_INVALID_ARG.  Synchronises. */
qsp_status qsp_run_box_adjoint(qsp_ctx ctx, const qsp_box_cotangent* cot, double* grad_amp,
                               double* grad_sigma, double* loss);

/* Kernel classes of the per-kernel device timers. */
enum {
  QSP_K_PUSH = 0,        /* real gather + push + deposit (one per slice)      */
  QSP_K_TRIAL = 1,       /* predictor-corrector trial push + Jx, Jy deposit   */
  QSP_K_ROW_FWD = 2,     /* source assembly + forward DST along x             */
  QSP_K_COL = 3,         /* DST along y, eigenvalue division, inverse along y */
  QSP_K_ROW_INV = 4,     /* inverse DST along x with its epilogue             */
  QSP_K_OTHER = 5,       /* clears, initial guess, outputs, bookkeeping       */
  QSP_NK = 6
};

typedef struct {
  double ms[QSP_NK];        /* summed device time of the timed launches */
  int64_t launches[QSP_NK]; /* number of timed launches                 */
} qsp_kernel_times;

/* Enables per-kernel timing: with every > 0, each kernel launched while
 * computing a slice k with k % every == 0 is bracketed by HIP events on the
 * context's stream; every = 0 turns timing off.  Clears the accumulators. */
qsp_status qsp_set_timing(qsp_ctx ctx, int32_t every);

/* Accumulated kernel times since qsp_set_timing (synchronises). */
qsp_status qsp_get_kernel_times(qsp_ctx ctx, qsp_kernel_times* out);

/* Number of plasma particles and slice cursor of the context. */
qsp_status qsp_get_info(qsp_ctx ctx, int64_t* n_particles, int32_t* cursor);

/* Static description of a status code. */
const char* qsp_status_string(qsp_status s);

/* Message of the last failed call on ctx (or of the last failed
 * qsp_create / qsp_validate_config in this thread if ctx is NULL). */
const char* qsp_last_error(qsp_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif
