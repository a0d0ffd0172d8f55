/*
 * lgf.h -- Fourier-accelerated steepest-descent Landau gauge fixing of 4D
 * SU(3) lattice gauge fields on an AMD MI355X (gfx950), C ABI.
 *
 * The method (Cardoso, Silva, Oliveira, Bicudo, "Landau gauge fixing on the
 * lattice using GPU's", arXiv:1301.3460):
 *
 *   Landau gauge maximises, on each gauge orbit, the functional of the
 *   paper's display equation
 *       F_U[g] = 1/(Nd Nc V) sum_x sum_mu Re Tr[ g(x) U_mu(x) g(x+mu)^dagger ],
 *   Nd = 4, Nc = 3, V = Lx Ly Lz Lt.  It is maximised by steepest descent with
 *   Fourier acceleration (the text following the display equation), with the
 *   step parameter alpha = 0.08 and the stopping criterion theta < 1e-15 of
 *   the paper's 32^4 comparison runs.
 *
 * The paper does not print the iteration formulae; this library uses the
 * reading of the cited method documented with the sources:
 *   Delta(x) = A - Tr(A)/3,  A = X - X^dagger,  X = sum_mu [U_mu(x-mu) - U_mu(x)]
 *   theta    = 1/(Nc V) sum_x Tr[Delta(x) Delta(x)^dagger]
 *   g(x)     = reunit(1 + (alpha/2) IFFT[ p2max/p2(p) * FFT[Delta] ](x)),
 *              p2(p) = sum_mu 4 sin^2(pi p_mu/L_mu), zero mode dropped,
 *              reunit = Gram-Schmidt of rows 0,1 and row 2 = conj(row0 x row1)
 *   U_mu(x) <- g(x) U_mu(x) g(x+mu)^dagger  (all links at once)
 *
 * Conventions shared by every entry point
 *   Lattice      L[4] = {Lx, Ly, Lz, Lt}; each extent a product 2^a 3^b
 *                with 2 <= L_mu <= 256 (2 3 4 6 8 9 12 16 18 24 27 32 36 48
 *                54 64 72 81 96 108 128 144 162 192 216 243 256: the
 *                extents of the hand-written mixed-radix transform), fewer
 *                than 2^31 sites.  Periodic boundaries.
 *                Site index s = x + Lx*(y + Ly*(z + Lz*t)).
 *   Links U      DEVICE pointer to complex128 data (interleaved re, im)
 *                laid out [4][Lt][Lz][Ly][Lx][3][3] (mu = x, y, z, t), i.e. a
 *                contiguous torch.complex128 tensor of shape (4,Lt,Lz,Ly,Lx,3,3).
 *                Only rows 0 and 1 of every link are read: the library stores
 *                links as 12 reals and rebuilds row 2 = conj(row0 x row1),
 *                which is exact for SU(3).  Links written back are full 3x3.
 *   Site fields  DEVICE pointers; g: complex128 [Lt][Lz][Ly][Lx][3][3];
 *                omega, dF/domega: float64 [Lt][Lz][Ly][Lx][8];
 *                eps, dtheta/deps: float64 [4][Lt][Lz][Ly][Lx][8].
 *                Generators T^a = lambda_a/2 (Gell-Mann matrices lambda_1..8).
 *   Ownership    The caller owns every pointer it passes.  The context owns
 *                its device scratch (working links, Fourier fields, partial
 *                sums), allocated in lgf_create and freed in lgf_destroy.
 *   Ordering     All device work is enqueued on the context's stream.  Calls
 *                that return host scalars synchronise that stream first.
 *   Errors       Every call returns an lgf_status value; no C++ exception
 *                crosses the ABI.  lgf_last_error() gives a message.  On
 *                LGF_ERR_ARG no device memory is touched.  Solver statuses
 *                LGF_NOT_CONVERGED / LGF_ERR_NONFINITE / LGF_DIVERGING still
 *                fill the result and write back the last completed iterate.
 *   Threads      A context may be used by one host thread at a time.
 */
#ifndef LGF_H
#define LGF_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lgf_ctx lgf_ctx;

typedef enum {
    LGF_OK = 0,
    LGF_ERR_ARG = 1,          /* invalid argument (pointer, extent, alpha, tol) */
    LGF_ERR_DEVICE = 2,       /* a HIP call failed */
    LGF_ERR_OOM = 3,          /* device allocation failed */
    LGF_NOT_CONVERGED = 4,    /* max_iter updates applied, theta >= tol */
    LGF_ERR_NONFINITE = 5,    /* theta became NaN or Inf */
    LGF_DIVERGING = 6         /* theta rose 8 sweeps in a row to over 100x its minimum */
} lgf_status;

typedef enum {
    LGF_FP64 = 0,   /* every sweep in double precision */
    LGF_MIXED = 1   /* FP32 sweeps until theta < theta_switch, then FP64 */
} lgf_precision;

typedef struct {
    int iterations;       /* gauge updates applied by the call (all phases) */
    int fp32_iterations;  /* of which in the FP32 phase (LGF_MIXED only) */
    int status;           /* lgf_status of the solve */
    double F;             /* F_U[1] of the returned links */
    double theta;         /* theta of the returned links */
    double seconds;       /* wall time of the call, device work included */
} lgf_result;

/* Create a context for lattice L (see conventions) and precision mode.
 * The lattice is the periodic 4D lattice of V = Lx Ly Lz Lt sites on which
 * the paper's display equation defines F_U[g]; its comparison runs use 32^4.
 * precision: LGF_FP64 (the paper's double precision) or LGF_MIXED.
 * stream: a hipStream_t to enqueue on (NULL: the null stream).  The current
 * HIP device at creation is the context's device.  *out receives the context
 * (NULL on failure).  Allocates the context's device scratch (about 1 GiB at
 * 32^4 FP64).  LGF_ERR_ARG for a NULL pointer, an unsupported extent or
 * precision, or a lattice whose transform passes would exceed the LDS or grid
 * limits of one kernel launch; LGF_ERR_OOM if the scratch does not fit;
 * LGF_ERR_DEVICE if no HIP device is current.  lgf_last_error(NULL) explains a
 * failure. */
int lgf_create(lgf_ctx **out, const int L[4], int precision, void *stream);

/* As lgf_create for the gauge group SU(nc), nc = 3 or 2 (the paper's
 * functional is written for a general N_c: F = 1/(Nd Nc V) sum Re Tr[...],
 * theta = 1/(Nc V) sum Tr[Delta Delta^+]).  lgf_create(...) is
 * lgf_create_group(..., 3, ...).  SU(2) contexts take links of shape
 * [4][Lt][Lz][Ly][Lx][2][2] complex128, store row 0 of each link (an SU(2)
 * matrix is [[a, b], [-conj(b), conj(a)]]) and run lgf_fix, lgf_iterate,
 * lgf_theta, lgf_functional (g == NULL), lgf_profile and the step options, in
 * both precisions; the other entry points return LGF_ERR_ARG for them. */
int lgf_create_group(lgf_ctx **out, const int L[4], int nc, int precision, void *stream);

/* Free the context's device scratch; NULL is ignored. */
void lgf_destroy(lgf_ctx *ctx);

/* Threshold at which LGF_MIXED hands over from FP32 to FP64 (default 1e-8). */
int lgf_set_theta_switch(lgf_ctx *ctx, double theta_switch);

/* on != 0 (default): Fourier-accelerated steepest descent.  on == 0: plain
 * steepest descent, g = reunit(1 + (alpha/2) Delta) with no transform -- the
 * method the paper accelerates, which slows down on large lattices (the
 * paragraph after the display equation). */
int lgf_set_acceleration(lgf_ctx *ctx, int on);

/* exact == 0 (default): the gauge transformation of a sweep is the first-
 * order step 1 + (alpha/2) L Delta made unitary by Gram-Schmidt.  exact != 0:
 * g = exp((alpha/2) L Delta), evaluated exactly (Cayley-Hamilton form of the
 * exponential series).  Both are readings of the steepest-descent step of the
 * method (the paragraph after the display equation); they share the fixed
 * points and differ at second order in alpha along the way.  Applies to
 * lgf_fix and lgf_iterate, in both precisions. */
int lgf_set_exponential(lgf_ctx *ctx, int exact);

/* bits = 64 (default) or 32: the precision in which FP64 sweeps (those of
 * LGF_FP64 contexts and the FP64 phase of LGF_MIXED) keep the Fourier field,
 * i.e. Delta and the transformed L Delta between the update and the
 * transforms.  Links, g(x), the update and the reductions stay FP64, and g is
 * exactly unitary either way, so an FP32 field only perturbs the step
 * direction (relative 1e-7): the fixed point and the stopping test are those
 * of the FP64 method, while the sweep moves 1024 instead of 1280 bytes per
 * site.  A reading of the method, not the paper's double-precision code.
 * LGF_ERR_ARG for other values. */
int lgf_set_field_precision(lgf_ctx *ctx, int bits);

/* Storage of the working links during lgf_fix / lgf_iterate (the paper's
 * GPU paragraph picks its 12-real form for speed; the alternatives trade
 * bytes against arithmetic): nreal = 12 (default; the paper's "12 real number
 * representation": rows 0 and 1, row 2 rebuilt as conj(row0 x row1) on every
 * load), 18 (all three rows stored, no rebuild, 50% more link traffic) or 8
 * (the minimal form: a link is brought to a frame whose stored entries leave
 * every reconstruction step well conditioned -- no singular set -- and
 * rebuilt from 6 matrix entries, two phases held as tan(phi/4) and 3
 * permutation bits in the lowest mantissa bits of one stored entry; one
 * third less link traffic, more arithmetic, about 1e-15 per store in FP64).
 * The caller's links are always full 3x3 complex128 (rows 0,1 read for 12
 * and 8); the other entry points always use 12.  Changing the format
 * reallocates the context's link buffers (synchronises the stream).
 * LGF_ERR_ARG for another nreal; LGF_ERR_OOM if the new buffers do not fit (the
 * context then holds 12-real buffers again, or none, which later calls
 * report). */
int lgf_set_link_format(lgf_ctx *ctx, int nreal);

/* Exactly n_iter updates of the links U (in place), n_iter >= 0.  One update
 * is one steepest-descent step with Fourier acceleration (the paragraph
 * following the display equation; plain steepest descent after
 * lgf_set_acceleration(ctx, 0)), with the step size alpha > 0 (the paper's
 * runs use alpha = 0.08).  There is no stopping test: neither theta < tol nor
 * a rising or stalling theta ends the run.  Only a non-finite theta or F
 * stops it early, with LGF_ERR_NONFINITE and res->iterations < n_iter.  res
 * (may be NULL) gets the updates applied and F and theta of the returned
 * links.  An LGF_MIXED context runs the sweeps in FP32, accumulating the
 * applied transformation, and applies it to U in FP64 at the end. */
int lgf_iterate(lgf_ctx *ctx, double *U, double alpha, int n_iter, lgf_result *res);

/* Gauge fixing by Fourier-accelerated steepest descent (the paragraph
 * following the display equation), with the parameters of the paper's
 * comparison runs (alpha = 0.08, stopping criterion theta < 1e-15; the
 * paragraph on those runs).  Updates U in place until theta < theta_tol
 * (tested before each update, so an already-fixed input takes 0 updates) or
 * max_iter updates.  alpha > 0, theta_tol > 0, max_iter >= 0, else
 * LGF_ERR_ARG with U untouched.  Returns LGF_OK (converged),
 * LGF_NOT_CONVERGED (max_iter reached), LGF_ERR_NONFINITE or LGF_DIVERGING
 * (theta rose for 8 sweeps in a row to over 100x its minimum, e.g. for alpha
 * above 2/p2max); these still fill res and write back the last iterate.
 * LGF_MIXED: FP32 sweeps until theta < the hand-over threshold
 * (lgf_set_theta_switch), then FP64 sweeps to theta_tol. */
int lgf_fix(lgf_ctx *ctx, double *U, double alpha, double theta_tol, int max_iter,
            lgf_result *res);

/* F_U[g] of the display equation (g == NULL: identity) into *F (host). */
int lgf_functional(lgf_ctx *ctx, const double *U, const double *g, double *F);

/* theta of the links U into *theta (host): the quantity the paper's
 * comparison runs bring below 1e-15.  The paper does not print its formula;
 * this is the reading theta = 1/(Nc V) sum_x Tr[Delta(x) Delta(x)^dagger] with
 * Delta as above (no factor 1/2), equal to 384 V |dF/domega|^2 at omega = 0.
 * Synchronises the context's stream. */
int lgf_theta(lgf_ctx *ctx, const double *U, double *theta);

/* Average plaquette 1/(6 Nc V) sum_x sum_{mu<nu} Re Tr U_mu(x) U_nu(x+mu)
 * U_mu(x+nu)^dagger U_nu(x)^dagger into *P (host): a gauge-invariant check. */
int lgf_plaquette(lgf_ctx *ctx, const double *U, double *P);

/* Per-step entry points, for step-by-step checking of the sweep.
 * lgf_divergence: Delta(x) of U as complex128 [Lt][Lz][Ly][Lx][3][3].
 * lgf_fourier_accelerate: LD = IFFT[p2max/p2 * FFT[D]] of an anti-hermitian
 *   traceless site field D (same layout, only its independent entries read).
 * lgf_fft4d: unnormalised 4D DFT, in place, of 4 complex128 fields laid out
 *   [4][Lt][Lz][Ly][Lx]; sign = -1 forward exp(-2 pi i n.x/L), +1 inverse. */
int lgf_divergence(lgf_ctx *ctx, const double *U, double *Delta);
int lgf_fourier_accelerate(lgf_ctx *ctx, const double *D, double *LD);
int lgf_fft4d(lgf_ctx *ctx, double *fields, int sign);

/* Differentiation (FP64).  g(x) = exp(i omega^a(x) T^a), exactly.
 * lgf_functional_omega: *F = F_U[g].
 * lgf_functional_omega_grad: *F and dF/domega^a(x) into dF (device). */
int lgf_functional_omega(lgf_ctx *ctx, const double *U, const double *omega, double *F);
int lgf_functional_omega_grad(lgf_ctx *ctx, const double *U, const double *omega,
                              double *F, double *dF);

/* theta of the links U'_mu(x) = exp(i eps^a_mu(x) T^a) U_mu(x) (eps == NULL:
 * zero) and its derivative dtheta/deps^a_mu(x) (device, may be NULL). */
int lgf_theta_grad(lgf_ctx *ctx, const double *U, const double *eps, double *theta,
                   double *dtheta);

/* Per-iteration history of the last lgf_fix/lgf_iterate: F_n and theta_n for
 * n = 0..iterations (FP32 phase first in LGF_MIXED).  Copies at most cap
 * entries into host arrays; *count receives the number of entries. */
int lgf_history(lgf_ctx *ctx, double *F, double *theta, int cap, int *count);

/* Per-kernel timing of n_iter sweeps (n_iter >= 1) of the context's precision
 * (LGF_MIXED: the FP32 sweep with transformation accumulation), run on the
 * context's working copy of U (U itself is not modified).  HIP events are
 * recorded between the launches of every sweep, all sweeps are enqueued
 * before one synchronisation, and kernel_ms[k] receives the mean duration in
 * milliseconds of: 0 (x,y) forward FFT, 1 (z,t) FFT + scaling + inverse,
 * 2 (x,y) inverse FFT, 3 update + next divergence, 4 finalize. */
int lgf_profile(lgf_ctx *ctx, const double *U, double alpha, int n_iter, double *kernel_ms);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): F_U[1] and
 * theta of the SU(3) links U without a context -- the values lgf_functional
 * (g == NULL) and lgf_theta return, from the same arithmetic in the same
 * summation order.  L: as for lgf_create, with V <= LGF_NOALLOC_MAX_SITES.
 * U: DEVICE complex128 links (rows 0,1 of each link read).  out: DEVICE
 * pointer to 2 doubles that receive {F, theta}.  The work is enqueued on
 * `stream` (a hipStream_t, NULL: the null stream) of the current HIP device
 * and the call returns without synchronising.  It allocates nothing: the
 * per-block partial sums live in a fixed device array of the library
 * (LGF_NOALLOC_MAX_SITES/256 pairs of doubles, 2 MiB, on each device it is
 * used on, held until the process ends), looked up on the first call on a
 * device.  Every call on a device shares that array, so calls that overlap in
 * time on one device race: serialise them (e.g. one stream).  LGF_ERR_ARG
 * (nothing enqueued) for a NULL pointer, an unsupported extent or a larger
 * lattice; LGF_ERR_DEVICE if the array cannot be looked up or the launch
 * fails.  Messages via lgf_last_error(NULL). */
#define LGF_NOALLOC_MAX_SITES (1L << 25)
int lgf_measure_noalloc(const int L[4], const double *U, double *out, void *stream);

/* Message for the last failure on ctx (ctx == NULL: last failure of
 * lgf_create or lgf_measure_noalloc on this thread).  Never NULL. */
const char *lgf_last_error(const lgf_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LGF_H */
