/*
 * pipe_poisson.h -- C ABI of libpipe: Poisson's equation in an open-ended
 * rectangular pipe by zero-padded FFT mixed convolution/correlation, on
 * AMD MI355X (gfx950).
 *
 * Method: R. D. Ryne, "On FFT-based convolutions and correlations, with
 * application to solving Poisson's equation in an open rectangular pipe"
 * (arXiv:1111.4971).  The potential on the mesh is
 *
 *   phi[i,j,k] = hx hy hz sum_{i',j',k'} rho[i',j',k']
 *                 { R(X_i-X_i', Y_j-Y_j', w) - R(X_i-X_i', Y_j+Y_j', w)
 *                 - R(X_i+X_i', Y_j-Y_j', w) + R(X_i+X_i', Y_j+Y_j', w) },
 *   w = (k-k') hz,
 *
 * (the Eq. 4 discretisation of Eq. 1 with the four-term Green function of
 * Eq. 8), with R from Eq. 9 (PIPE_GREEN_POINT) or its z-integrated form
 * R_int from Eq. 14-16 (PIPE_GREEN_IGF_Z), the mode sums truncated at
 * m <= mx, n <= my.  It is computed as in Eq. 10: one forward transform of
 * the zero-padded charge, a pointwise product against Green spectra computed
 * once per plan, and one backward transform; the four terms' mixed FFT
 * directions become index reflections of the charge spectrum (Appendix, A.9).
 *
 * Conventions shared by every entry point:
 *  - Mesh node i (0-based) sits at X_i = (i+1) hx, node j at Y_j = (j+1) hy;
 *    z is translation invariant (only k - k' enters).  The pipe walls are at
 *    x in {0, a}, y in {0, b}; nodes must satisfy nx hx <= a, ny hy <= b.
 *  - R carries the prefactor 1/(2 pi a b) printed in Eq. 9 (Eq. 7 as printed
 *    is a quarter of Eq. 8 with that R).  Multiply by 4 pi^2 for G -> 1/r in
 *    the free-space limit.
 *  - Arrays rho and phi are device pointers to C-contiguous (nx, ny, nz)
 *    arrays, z fastest, of double (PIPE_PREC_FP64 plans) or float
 *    (PIPE_PREC_FP32 plans).  The Green function is always evaluated and
 *    transformed in FP64; FP32 plans store its spectra rounded to FP32.
 *  - Every function returns a status and never throws or aborts.  Arguments
 *    are validated before any HIP call.  pipe_last_error() returns a
 *    thread-local message about the most recent failure on this thread.
 *  - Solve calls are asynchronous on the given hipStream_t (NULL = default
 *    stream); they read rho, write phi and use the caller's workspace, and
 *    allocate nothing.  Concurrent solves on one plan need distinct
 *    workspaces.
 */
#ifndef PIPE_POISSON_H
#define PIPE_POISSON_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pipe_plan_s* pipe_plan_t;
typedef struct pipe_batch_s* pipe_batch_t;

typedef enum pipe_status {
    PIPE_OK = 0,
    PIPE_ERR_INVALID_ARG = 1,      /* bad size, spacing, geometry, handle or pointer        */
    PIPE_ERR_UNSUPPORTED_SIZE = 2, /* padded length not available (see pipe_green_plan_ex)  */
    PIPE_ERR_OUT_OF_MEMORY = 3,    /* device allocation failed                               */
    PIPE_ERR_NO_DEVICE = 4,        /* no HIP device visible                                  */
    PIPE_ERR_HIP = 5,              /* a HIP runtime call failed (message has the HIP error)  */
    PIPE_ERR_ALIASING = 6          /* rho and phi overlap                                    */
} pipe_status_t;

/* kind flags: low nibble = Green function, bits 4..7 = FFT/product precision */
enum {
    PIPE_GREEN_POINT = 0,   /* R of Eq. 9: z-factor e^{-kappa|w|}                         */
    PIPE_GREEN_IGF_Z = 1,   /* R_int of Eq. 16: z-factor g_z(w) of Eq. 15 (hat basis)     */
    PIPE_GREEN_FREE = 2,    /* free space, G = 1/r of Eq. 3 (plans from pipe_free_plan)   */
    PIPE_PREC_FP64 = 0x00,  /* transforms, products, rho and phi in double                */
    PIPE_PREC_FP32 = 0x10,  /* transforms, products, rho and phi in float                 */
    PIPE_KEEP_GREEN = 0x100,/* keep the on-mesh Green table for pipe_plan_green_table     */
    PIPE_AUTOTUNE = 0x200,  /* time the candidate padded lengths, keep the fastest        */
    PIPE_AUTOTUNE_BATCH = 0x400, /* as PIPE_AUTOTUNE, timing 16 concurrent solves (batches) */
    PIPE_BAND_FASTEST = 0x800    /* pipe_green_plan_banded: return the 3-D plan if it is faster */
};

typedef struct pipe_plan_info {
    int nx, ny, nz;          /* physical mesh                                               */
    int lx, ly, lz;          /* padded transform lengths (each >= 2n - 1; lz even)          */
    int mx, my;              /* mode truncation m <= mx, n <= my                            */
    int kind;                /* as passed                                                   */
    int real_bytes;          /* 8 (FP64) or 4 (FP32)                                        */
    double hx, hy, hz, a, b;
    double x0, y0;           /* mesh offset (pipe_green_plan_region; 0 otherwise)           */
    double norm;             /* the R prefactor 1/(2 pi a b); 1 for free-space plans         */
    size_t workspace_bytes;  /* device bytes a solve needs as scratch                       */
    size_t spectra_bytes;    /* device bytes held by the plan's Green spectra               */
    double model_bytes;      /* algorithmic HBM bytes of one solve (all passes)             */
    double pass_bytes[5];    /* the same per pass: z-forward, y-forward, x+product,         */
                             /* y-inverse, z-inverse                                        */
    double build_ms;         /* wall time of the plan build (Green evaluation + spectra)    */
    double tune_ms;          /* PIPE_AUTOTUNE: the chosen lengths' measured ms per solve  */
                             /* (0 = taken from the cache; -1 = not tuned)                */
    int band;                /* pipe_green_plan_banded: planes kept each side (N of Eq. 18);*/
                             /* -1 for the full 3-D plans                                 */
    double band_speedup;     /* pipe_green_plan_banded: measured time of the mesh's 3-D     */
                             /* solve over the banded solve's (> 1: banded is faster);      */
                             /* also on a 3-D plan returned for PIPE_BAND_FASTEST; else 0  */
    int xtile;               /* launch schedule (3-D plans; banded plans report only xtile, */
    int apad;                /* for N = 0): kz (packed-column) tile of the x pass, unused   */
    int zblocks;             /* slots per row of the y-transformed array, block cap of the  */
                             /* z passes; none of them changes a result                    */
    int xnt;                 /* schedule: 1 if the x pass writes with non-temporal stores  */
    int a1pad;               /* schedule: slots per row of the z-transformed array = lz/2 + a1pad */
} pipe_plan_info_t;

/*
 * pipe_green_plan -- evaluate the Green function on the mesh and cache its
 * spectra: the one-time tabulation and transformation that Sec. 2 (after
 * Eq. 10) describes and Sec. 5 argues is amortised over many solves.
 *
 * nx, ny, nz >= 1 nodes; hx, hy, hz > 0 spacings; a, b > 0 pipe widths with
 * nx*hx <= a and ny*hy <= b (1e-12 relative slack, so a node may sit on a
 * wall).  kind = PIPE_GREEN_* | PIPE_PREC_*.  Modes default to mx = 2nx,
 * my = 2ny and padded lengths as pipe_green_plan_ex describes.
 * Blocks until the plan is built.  *out receives an opaque handle owned by
 * the caller (free with pipe_plan_destroy).
 * Errors: INVALID_ARG, UNSUPPORTED_SIZE, NO_DEVICE, OUT_OF_MEMORY, HIP.
 */
pipe_status_t pipe_green_plan(int nx, int ny, int nz, double hx, double hy, double hz,
                              double a, double b, int kind, pipe_plan_t* out);

/*
 * pipe_green_plan_ex -- as pipe_green_plan with explicit mode counts
 * (mx, my >= 1) and padded lengths (0 = default).  Each padded length must be
 * at least 2n - 1 (Appendix: N >= M = J + K - 1, else INVALID_ARG); lx and ly
 * must be of the form 2^p 3^q in [8, 1024] (odd ones included), and lz must be
 * even with lz/2 of that form (z is transformed real-to-complex as lz/2 packed
 * pairs), i.e. lz in [16, 2048]; otherwise UNSUPPORTED_SIZE.  The default
 * (length 0) is, per dimension, the supported length >= 2n (lz: lz/2 >= nz)
 * with the lowest modelled pass time among those within 20 % of the smallest
 * one: a table of the HBM-peak fraction each length's passes reached on
 * MI355X, so a slow factorisation (432 = 27 * 16) gives way to a fast one
 * (512) when that is quicker overall; below 64 it is the smallest length.
 * The physical result does
 * not depend on the padded lengths.  hip_stream (a hipStream_t, may be NULL) orders the plan build's GPU
 * work; the call still returns only when the build has finished.
 * Every 3-D plan (here, pipe_green_plan_region, pipe_free_plan) also picks a
 * launch schedule by timing the solve on scratch buffers during the build:
 * the kz tile of the x pass (its widest or half of it), the row pitch of the
 * y-transformed array (lz/2 plus 0, 16 or 32), the block cap of the z
 * passes (1024, 2048 or 4096) and whether the x pass writes with non-temporal
 * stores; the row pitch of the z-transformed array is lz/2 plus 16 where lz/2
 * is a power of two and a row spans at least 8 KB, else lz/2.  None
 * of these changes any result; the choice is cached for the process (and in
 * PIPE_TUNE_CACHE, "pipe-sched-v3" lines) and reported in pipe_plan_info
 * (xtile, apad, zblocks, xnt, a1pad).  The environment variable
 * PIPE_SCHEDULE=fixed skips the timing (widest tile, no pad on the
 * y-transformed array, 2048 blocks, plain stores, the z-transformed array's
 * pitch by the rule above); PIPE_SCHEDULE=T,pad,cap[,nt[,a1pad]] forces a
 * schedule, a1pad being the slots added to the z-transformed array's pitch
 * (INVALID_ARG if T is neither the widest tile nor half of it, pad is outside
 * [0, 256], nt is not 0 or 1, or a1pad is not even in [0, 256]; non-temporal
 * stores are an FP64 option only).
 * With PIPE_AUTOTUNE in kind and all lengths 0, the plan times the five
 * passes for each candidate factorisation per dimension (the default above,
 * the smallest supported length >= 2n, the smallest even one, the smallest
 * power of two, the smallest 3 * 2^k)
 * on scratch buffers and keeps the fastest: one solve at a time (latency)
 * with PIPE_AUTOTUNE, one grouped launch of 16 concurrent solves (throughput,
 * the batched form) with PIPE_AUTOTUNE_BATCH.  The choice is cached for the
 * process per (device architecture, mesh, precision, values per spectra
 * orbit, mode) and appended to the file named by the environment variable
 * PIPE_TUNE_CACHE, if set, which later processes read (one line per entry:
 * "pipe-tune-v2 arch nx ny nz real_bytes nval members lx ly lz"; nval is 9 for
 * pipe plans and 1 for free-space plans, members 1 or 16).  An entry whose
 * lengths this mesh cannot use (see the rules above) is ignored and the
 * lengths are tuned again; malformed lines are skipped.
 */
pipe_status_t pipe_green_plan_ex(int nx, int ny, int nz, double hx, double hy, double hz,
                                 double a, double b, int kind, int mx, int my,
                                 int lx, int ly, int lz, void* hip_stream, pipe_plan_t* out);

/*
 * pipe_green_plan_region -- as pipe_green_plan_ex for a mesh covering only a
 * sub-region of the pipe cross-section (Sec. 5: a thin beam needs only the
 * area around it meshed): node i at x0 + (i+1) hx, node j at y0 + (j+1) hy,
 * with x0, y0 >= 0, x0 + nx hx <= a and y0 + ny hy <= b.  The Green function
 * is still that of the whole pipe; only the distances X_i + X_i' of the image
 * terms change (to 2 x0 + (i+i'+2) hx).  Errors as pipe_green_plan_ex.
 */
pipe_status_t pipe_green_plan_region(int nx, int ny, int nz, double hx, double hy, double hz,
                                     double a, double b, double x0, double y0, int kind, int mx, int my,
                                     int lx, int ly, int lz, void* hip_stream, pipe_plan_t* out);

/*
 * pipe_green_plan_banded -- a plan that keeps only the z distances |k - k'| <= N
 * of the sum (Eq. 18; N = 0 is the set of independent 2-D problems of Eq. 17),
 * for long bunches whose Green function falls off within a few planes (Sec. 4,
 * end).  The z transform disappears: each plane is transformed in x and y
 * only (padded lengths lx, ly as in pipe_green_plan_ex, except that lx must be
 * one of 8, 12, 16, 24, 32, 36, 48, 64, 72, 96, 108, 128, 144, 192, 216, 256,
 * 288, 384, 432, 512, 576, 768, 864, 1024 -- the banded x pass splits each
 * line's orbits evenly over its threads -- else UNSUPPORTED_SIZE; the default
 * is the smallest of these >= 2 nx; lz is reported as 0),
 * each output plane sums 2N + 1 transverse spectral products, and the plan
 * holds N + 1 two-dimensional Green spectra.  Solving is otherwise the same
 * call (pipe_poisson_solve / pipe_poisson_adjoint with info.workspace_bytes
 * of workspace); phi then equals the full solve with R set to zero beyond N
 * planes.  nband >= 0 sets N (values above nz - 1 are reduced to nz - 1, which
 * gives the full z sum); nband < 0 chooses the smallest N with
 *   B(d) <= tol * B(0) for every plane distance N < d < nz,
 * B(d) = sum over the kept modes (m, n) of |the mode's z factor at d hz|
 * times the Eq. 9 prefactor, an upper bound on |R| over the cross-section at
 * that distance.  tol must then be in (0, 1).  The build times one banded
 * solve against one solve of the 3-D plan the mesh would get from
 * pipe_green_plan_region (on scratch buffers) and reports the ratio in
 * info.band_speedup (below 1: the banded plan is the slower one, which happens
 * once 2N + 1 plane products cost more than the z transforms they replace).
 * With PIPE_BAND_FASTEST in kind, the call then returns the 3-D plan (exact,
 * info.band = -1) whenever it is the faster.  Other arguments, ownership and
 * errors as pipe_green_plan_region; PIPE_AUTOTUNE flags are ignored.  In a
 * batch (pipe_batch_create) a banded plan runs its own three passes inside the
 * captured graph rather than in grouped launches.
 */
pipe_status_t pipe_green_plan_banded(int nx, int ny, int nz, double hx, double hy, double hz,
                                     double a, double b, double x0, double y0, int kind, int mx, int my,
                                     int lx, int ly, int nband, double tol, void* hip_stream,
                                     pipe_plan_t* out);

/*
 * pipe_free_plan -- the isolated (free-space) problem by Hockney's method,
 * Sec. 1, Eq. 3-5: phi[i,j,k] = hx hy hz sum rho[i',j',k'] G((i-i') hx,
 * (j-j') hy, (k-k') hz) with G = 1/sqrt(u^2 + v^2 + w^2) (the 4 pi dropped, as
 * in Eq. 3), computed as one zero-padded convolution (Eq. 5).  G is singular
 * at zero separation and the paper leaves that grid value open: g0 (finite)
 * is used there.  kind = PIPE_PREC_* optionally | PIPE_AUTOTUNE* (a Green
 * kind in its low nibble is INVALID_ARG; PIPE_KEEP_GREEN is INVALID_ARG).
 * Padded lengths as pipe_green_plan_ex.  The plan reports kind
 * PIPE_GREEN_FREE, a = b = 0, norm = 1, and solves, adjoints (the operator
 * is symmetric), batches and timing hooks work on it unchanged.
 * Errors: INVALID_ARG, UNSUPPORTED_SIZE, NO_DEVICE, OUT_OF_MEMORY, HIP.
 */
pipe_status_t pipe_free_plan(int nx, int ny, int nz, double hx, double hy, double hz, double g0, int kind,
                             int lx, int ly, int lz, void* hip_stream, pipe_plan_t* out);

/* pipe_plan_info -- sizes and constants of a plan.  Errors: INVALID_ARG. */
pipe_status_t pipe_plan_info(pipe_plan_t plan, pipe_plan_info_t* out);

/*
 * pipe_default_lengths -- the padded lengths a 3-D plan of an nx x ny x nz
 * mesh gets when it leaves them at 0 (pipe_green_plan, pipe_green_plan_ex,
 * pipe_green_plan_region, pipe_free_plan without PIPE_AUTOTUNE): per dimension
 * the supported length >= 2n (lz: lz/2 >= nz) with the lowest modelled pass
 * time among those within 20 % of the smallest such length (any padded
 * length >= 2n - 1 gives the same potential: Appendix, after Eq. A.3).  kind:
 * PIPE_PREC_FP32 or PIPE_PREC_FP64 (the model has one table per precision),
 * optionally with a PIPE_GREEN_* kind, which does not change the result.
 * *lx, *ly, *lz receive the lengths.  Host only: no GPU, no HIP call.
 * Errors: INVALID_ARG (n < 1, other kind bits, a null output),
 * UNSUPPORTED_SIZE (no supported length is long enough).
 */
pipe_status_t pipe_default_lengths(int nx, int ny, int nz, int kind, int* lx, int* ly, int* lz);

/*
 * pipe_poisson_solve -- phi = A rho for the plan's mesh (Eq. 10, all four
 * terms summed).  rho, phi: device arrays as described above; workspace: a
 * device buffer of at least info.workspace_bytes, 256-byte aligned.
 * rho is read-only and must not overlap phi (ALIASING).  Asynchronous on
 * hip_stream.  Errors: INVALID_ARG, ALIASING, HIP.
 */
pipe_status_t pipe_poisson_solve(pipe_plan_t plan, const void* rho, void* phi,
                                 void* workspace, void* hip_stream);

/*
 * pipe_poisson_adjoint -- drho = A^T dphi: the transposed gather of the
 * spectral product, sum_ab sigma_ab conj(T_ab(S_ab k)) g(S_ab k), on the same
 * cached spectra, between the same transforms.  A is symmetric (the Green
 * function of Eq. 7 is symmetric in (x,y,z) <-> (x',y',z')), so this equals
 * pipe_poisson_solve up to rounding.  Same arguments and errors.
 */
pipe_status_t pipe_poisson_adjoint(pipe_plan_t plan, const void* dphi, void* drho,
                                   void* workspace, void* hip_stream);

/*
 * pipe_poisson_solve_noalloc -- pipe_poisson_solve without a workspace
 * argument, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * workspace is a fixed scratch array of 256 MiB inside the library, one per
 * device, held from the first plan built on that device until the process
 * ends; the call itself allocates nothing and creates no HIP objects.  Every
 * call on one device shares that device's scratch, so calls that overlap in
 * time on one device (concurrent streams, or host threads) race and give
 * wrong results: order them.  Nothing in the scratch needs to start at zero
 * (each pass writes what the next reads), and it keeps the last call's
 * contents.  pipe_plan_destroy does not wait for solves made through this
 * entry point: finish them before destroying the plan.  A plan whose
 * info.workspace_bytes exceeds 256 MiB (e.g. 128 x 128 x 512 in FP64) gets
 * UNSUPPORTED_SIZE.  Otherwise arguments, results and errors as
 * pipe_poisson_solve.
 */
pipe_status_t pipe_poisson_solve_noalloc(pipe_plan_t plan, const void* rho, void* phi, void* hip_stream);

/*
 * pipe_batch_create -- group count >= 1 plans (any sizes, one precision) for
 * repeated batched solves: the per-plan pass launches are captured once into
 * a HIP graph and replayed by pipe_batch_solve.  The plans must outlive the
 * batch.  The workspace a batched solve needs is reported by
 * pipe_batch_workspace.  Errors: INVALID_ARG, OUT_OF_MEMORY, HIP.
 */
pipe_status_t pipe_batch_create(const pipe_plan_t* plans, int count, pipe_batch_t* out);

/* pipe_batch_workspace -- bytes of device workspace pipe_batch_solve needs. */
pipe_status_t pipe_batch_workspace(pipe_batch_t batch, size_t* bytes);

/*
 * pipe_batch_solve -- phi[s] = A_s rho[s] for every member s.  rho and phi
 * are host arrays of count device pointers.  The grouped kernels read their
 * per-member pointers from a device descriptor array: when the pointers or the
 * workspace differ from the previous call, the new descriptors are copied on
 * hip_stream (ordered after the previous replay, on whatever stream it ran)
 * and the captured graph is replayed unchanged.  The graph is captured again
 * only on the first call, when a banded member's pointers or the workspace of
 * a batch holding banded members change, or when the 2-element alignment of a
 * shape group's rho or phi pointers changes.  Asynchronous on hip_stream.
 * Replays on different streams are ordered by the library (each waits for the
 * descriptor copy it needs).  Errors: INVALID_ARG, ALIASING, HIP.
 */
pipe_status_t pipe_batch_solve(pipe_batch_t batch, const void* const* rho, void* const* phi,
                               void* workspace, void* hip_stream);

/* Destroy a plan or batch.  A handle that is not live (e.g. destroyed twice)
 * is rejected with INVALID_ARG.  Before freeing, waits for the work this
 * handle queued itself: every solve queued on a plan (one event per stream it
 * was used on, recorded after the solve's last kernel; solves queued while
 * their stream was being captured into a graph are the caller's to order), or
 * a batch's last replay and descriptor copy.  Other work on the device is not
 * waited for (the HIP runtime's free itself may still synchronise). */
pipe_status_t pipe_plan_destroy(pipe_plan_t plan);
pipe_status_t pipe_batch_destroy(pipe_batch_t batch);

const char* pipe_status_string(pipe_status_t status);
const char* pipe_last_error(void);

/* ------------------------------------------------------------------------ */
/* Inspection and measurement hooks (tests and benchmarks).                 */
/* ------------------------------------------------------------------------ */

/*
 * pipe_plan_green_table -- copy the on-mesh Green table the plan evaluated
 * (Eq. 9 or Eq. 16 at the distances the four terms need) to out_device:
 * FP64 array [3nx-1][3ny-1][nz], element [p][q][r] = R(u_p, v_q, r hz) with
 * u_p = p hx for p < nx (differences X_i - X_i') and u_p = 2 x0 + (p - nx + 2) hx
 * for nx <= p < 3nx - 1 (sums X_i + X_i'); v_q likewise in y.
 * Returns INVALID_ARG unless the plan was built with PIPE_KEEP_GREEN in kind.
 */
pipe_status_t pipe_plan_green_table(pipe_plan_t plan, void* out_device, void* hip_stream);

/*
 * pipe_plan_spectra -- copy the plan's compressed Green spectra to out_device
 * (plan precision): 9 planes of (lx/2+1)(ly/2+1)(lz/2) values followed by 9
 * planes of (lx/2+1)(ly/2+1) values for kz = lz/2.  For orbit
 * (kx, ky, kz), kx <= lx/2, ky <= ly/2, with T_ab the unscaled forward 3-D DFT
 * of term ab's zero-padded Green array (Appendix A.3, A.9 layouts):
 *   plane 0 = Re T_cc(kx,ky,kz); planes 1,2 = T_cr(kx,ky,kz);
 *   planes 3,4 = T_rc(kx,ky,kz); planes 5,6 = T_rr(kx,ky,kz);
 *   planes 7,8 = T_rr(lx-kx,ky,kz)   (re, im pairs).
 * A free-space plan (pipe_free_plan) has only plane 0 (T_cc of G = 1/r);
 * planes 1..8 of its copy are zero.
 * For a banded plan (pipe_green_plan_banded) the copy is the plan's own
 * coefficient table: with T_ab now the 2-D DFT of the four terms' slices at
 * plane distance d, ten values K0..K9 of (ky, d, kx) at
 * ((ky (N+1) + d) 10 + k)(lx/2+1) + kx:
 *   K0 = Re(T_cc + T_rr)   K1 = Im T_rr           K2 = Re(T_cc - T_rr)
 *   K3 = -Re(T_cr + T_rc)  K4 = Im(T_rc - T_cr)   K5 = -Im(T_cr + T_rc)
 *   K6 = Re(T_cr - T_rc)   K7 = Re(T_cc + T_rr')  K8 = Im T_rr'   K9 = Re(T_cc - T_rr'),
 * T_rr' = T_rr(lx-kx, ky): the symmetric 4 x 4 real matrix the solve applies
 * to the real and imaginary parts of a plane's spectrum at (kx,ky), (-kx,ky).
 */
pipe_status_t pipe_plan_spectra(pipe_plan_t plan, void* out_device, void* hip_stream);

/*
 * pipe_poisson_solve_timed -- pipe_poisson_solve preceded and followed by
 * HIP events around each of its five kernels on hip_stream; pass_ms[5]
 * receives the elapsed time of each kernel of this call (blocks until done).
 */
pipe_status_t pipe_poisson_solve_timed(pipe_plan_t plan, const void* rho, void* phi,
                                       void* workspace, void* hip_stream, float* pass_ms);

/*
 * pipe_plan_timing -- per-kernel timing of ordinary solves on this plan.
 * max_solves > 0 starts recording: each of the next max_solves calls of
 * pipe_poisson_solve / pipe_poisson_adjoint on this plan records a HIP event
 * on its own stream before, between and after its five kernels (no host
 * synchronisation).  max_solves = 0 stops recording, waits for the last
 * recorded solve and writes the mean elapsed time of each kernel over the
 * recorded solves to pass_ms_mean[5] and their number to *count (either may
 * be NULL).  Not thread-safe with concurrent solves on the same plan.
 */
pipe_status_t pipe_plan_timing(pipe_plan_t plan, int max_solves, float* pass_ms_mean, int* count);

/*
 * pipe_fft_lines -- the library's batched 1-D complex DFT, exposed for tests:
 * for each of howmany lines (line l at in + l*n_in, out + l*len, complex
 * interleaved, real_bytes 4 or 8), out = sum_{e<n_in} in[e] W^{+-ek} for
 * k < len, W = e^{-2 pi i/len}, sign -1 (forward, dir = -1) or +1 (dir = +1),
 * unscaled.  len must be a supported length; 1 <= n_in <= len.
 */
pipe_status_t pipe_fft_lines(int real_bytes, int len, int n_in, int howmany, int dir,
                             const void* in_device, void* out_device, void* hip_stream);

/*
 * pipe_fft3d -- unscaled 3-D complex DFT with the direction chosen per
 * dimension (Sec. 5: the method needs, and other uses such as split-operator
 * Vlasov solvers want, per-dimension direction control that multidimensional
 * FFT packages rarely offer; Eq. 6 is an example).  in, out: device arrays of
 * n0 x n1 x n2 complex values (interleaved re, im; real_bytes 4 or 8), C order,
 * last index fastest; out may equal in (in place) but must not otherwise
 * overlap it (ALIASING).  dirs: three characters, one per dimension in order,
 * 'f' = sum_n a_n W^{nk}, 'b' = sum_n a_n W^{-nk}, W = e^{-2 pi i/N}
 * (Eq. A.4's conventions; e.g. "fbf" is F^{fbf} of Eq. 6).  Each n must be a
 * supported length (2^p 3^q in [8, 1024], odd ones included).  Asynchronous on hip_stream.
 * Errors: INVALID_ARG, UNSUPPORTED_SIZE, ALIASING, NO_DEVICE, HIP.
 */
pipe_status_t pipe_fft3d(int real_bytes, int n0, int n1, int n2, const char* dirs, const void* in_device,
                         void* out_device, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PIPE_POISSON_H */
